"""FP64 CPU oracle for the thin-film LLG disk method (Wysin & Figueiredo, 2012).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP library is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library's product path never does.  It shares no code with the HIP path.

Everything here is float64 and follows the paper's equations in the order the
paper states them, using library primitives (torch FFTs, numpy integer
arithmetic) as single steps, without blocking or fusion:

* ``units``       - dimensionless parameters (Sec. II.A, Sec. III.A-B).
* ``geometry``    - the disk mask and padded FFT size (Sec. II.B).
* ``greens``      - the thin-film Green's kernels and their self terms (Sec. II.B).
* ``demag``       - demagnetisation field: direct real-space sum (the plain
                    definition) and zero-padded FFT convolution (Sec. II.B).
* ``dynamics``    - effective induction, LLG right-hand side, RK4, Heun
                    (eq. Bi, damped torque equation, Sec. III.A-C).
* ``philox``      - Philox4x32-10 counter-based generator + Box-Muller.
* ``observables`` - energy (eq. Hmm), <m>, vorticity centre and the
                    m_z^2-weighted core position (Sec. IV).
* ``relax``       - Lagrange-constrained alignment relaxation, k_F fit and
                    the Thiele frequency (Sec. IV, Sec. IV.B, eqs. wG, OG, Ux).

Parity status of each function is stated in its own docstring; functions
without an independent pin say "parity unpinned".
"""
from .units import Material, Params, dimensionless  # noqa: F401
from .geometry import Disk  # noqa: F401
