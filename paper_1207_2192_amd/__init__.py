"""lib_llgdisk for AMD Instinct MI355X: the thin-film LLG disk hot path
(Wysin & Figueiredo 2012) as hand-written HIP kernels behind a C ABI
(include/llgdisk.h), with this thin Python binding on top."""
from .api import (Disk, LLGParams, batch_create, build_kernels, demag_field, energy, heun_step,  # noqa: F401
                  llg_rhs, params_from_si, power_spectrum, rk4_step, vortex_core_position)
