"""Python binding of lib_llgdisk: same entry points as include/llgdisk.h.

Only argument marshalling happens here (tensor checks, pointers, the current
HIP stream); every step of the hot path runs in the library's kernels.  Torch
supplies device memory and streams.  Arrays are float32 tensors on the
handle's GPU laid out [3][D][D] per disk and packed back to back for batches.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import LLGParamsC, check


@dataclass
class LLGParams:
    """Dimensionless parameters (see llg_params in include/llgdisk.h), including the
    time-dependent field h_ext(tau) = hext + hac sin(2 pi freq tau + phase)
    + hpulse exp(-(tau - tpulse)^2 / (2 wpulse^2)) and the start time tau0."""
    alpha: float = 0.0
    c: float = 0.0
    hext: tuple = (0.0, 0.0, 0.0)
    temp: float = 0.0
    dtau: float = 0.04
    renorm: bool = False
    fd_factor: bool = False
    hac: tuple = (0.0, 0.0, 0.0)
    freq: float = 0.0
    phase: float = 0.0
    hpulse: tuple = (0.0, 0.0, 0.0)
    tpulse: float = 0.0
    wpulse: float = 1.0
    tau0: float = 0.0

    def to_c(self) -> LLGParamsC:
        p = LLGParamsC()
        p.alpha, p.c, p.temp, p.dtau = self.alpha, self.c, self.temp, self.dtau
        for i in range(3):
            p.hext[i] = float(self.hext[i])
            p.hac[i] = float(self.hac[i])
            p.hpulse[i] = float(self.hpulse[i])
        p.renorm, p.fd_factor = int(bool(self.renorm)), int(bool(self.fd_factor))
        p.freq, p.phase, p.tpulse, p.wpulse, p.tau0 = (float(self.freq), float(self.phase), float(self.tpulse),
                                                       float(self.wpulse), float(self.tau0))
        return p


def params_from_si(A: float, Ms: float, gamma: float, a_nm: float, L_nm: float, dt_ps: float,
                   T_K: float = 0.0, alpha: float = 0.0):
    """(LLGParams, lambda_ex_nm) from SI material data via llg_params_from_si."""
    lib = _lib.load()
    p = LLGParamsC()
    lam = ctypes.c_double()
    check(lib.llg_params_from_si(A, Ms, gamma, a_nm, L_nm, dt_ps, T_K, alpha, ctypes.byref(p),
                                 ctypes.byref(lam)), "llg_params_from_si")
    return LLGParams(alpha=p.alpha, c=p.c, hext=tuple(p.hext), temp=p.temp, dtau=p.dtau), lam.value


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Disk:
    """A disk (or a batch of disks) built by llg_build_kernels / llg_batch_create."""

    def __init__(self, handle, device: torch.device):
        self._h = handle
        self.device = device
        lib = _lib.load()
        self.n = lib.llg_disk_count(self._h)
        self.D, self.P, self.n_cells, self.offsets, self.workgroups = [], [], [], [], []
        for k in range(self.n):
            D, P, N = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            check(lib.llg_disk_info(self._h, k, ctypes.byref(D), ctypes.byref(P), ctypes.byref(N)), "llg_disk_info")
            self.D.append(D.value)
            self.P.append(P.value)
            self.n_cells.append(N.value)
            self.offsets.append(lib.llg_disk_offset(self._h, k))
            self.workgroups.append(lib.llg_disk_workgroups(self._h, k))
        self.state_size = lib.llg_state_size(self._h)

    # ---------------------------------------------------------------- creation
    @classmethod
    def build(cls, R_nm: float, L_nm: float, a_nm: float = 2.0, P: int = 0) -> "Disk":
        lib = _lib.load()
        h = ctypes.c_void_p()
        dev = torch.device("cuda", torch.cuda.current_device())
        check(lib.llg_build_kernels(R_nm, L_nm, a_nm, P, ctypes.byref(h)), "llg_build_kernels")
        return cls(h, dev)

    @classmethod
    def batch(cls, R_nm, L_nm, a_nm: float = 2.0, wg_per_disk=None) -> "Disk":
        lib = _lib.load()
        n = len(R_nm)
        R = (ctypes.c_double * n)(*[float(r) for r in R_nm])
        L = (ctypes.c_double * n)(*[float(x) for x in L_nm])
        W = None if wg_per_disk is None else (ctypes.c_int * n)(*[int(w) for w in wg_per_disk])
        h = ctypes.c_void_p()
        dev = torch.device("cuda", torch.cuda.current_device())
        check(lib.llg_batch_create(n, R, L, a_nm, W, ctypes.byref(h)), "llg_batch_create")
        return cls(h, dev)

    def tune(self, unit_groups: int, wg_per_disk=None, radix_policy: int = 0):
        """Re-plan the persistent launch (llg_tune)."""
        lib = _lib.load()
        W = None if wg_per_disk is None else (ctypes.c_int * self.n)(*[int(w) for w in wg_per_disk])
        check(lib.llg_tune(self._h, int(unit_groups), int(radix_policy), W), "llg_tune")
        self.workgroups = [lib.llg_disk_workgroups(self._h, k) for k in range(self.n)]

    def autotune(self, m: torch.Tensor, params, integrator: str = "rk4", probe_steps: int = 200) -> float:
        """Time candidate launch plans on a copy of m and keep the fastest (llg_autotune);
        returns microseconds per step of the chosen plan."""
        m = self._state(m)
        best = ctypes.c_double()
        check(_lib.load().llg_autotune(self._h, _ptr(m), self._params(params), 0 if integrator == "rk4" else 1,
                                       int(probe_steps), _stream(), ctypes.byref(best)), "llg_autotune")
        lib = _lib.load()
        self.workgroups = [lib.llg_disk_workgroups(self._h, k) for k in range(self.n)]
        return best.value

    def set_on_chip(self, max_P: int):
        """Disks with FFT size P <= max_P (64 or 128; 0 = none) run on one workgroup
        each with their spectra in LDS (llg_set_on_chip); re-plans the launch."""
        lib = _lib.load()
        check(lib.llg_set_on_chip(self._h, int(max_P)), "llg_set_on_chip")
        self.workgroups = [lib.llg_disk_workgroups(self._h, k) for k in range(self.n)]

    def timing(self, enable: bool = True):
        """Opt-in timing of the persistent launches (llg_timing)."""
        check(_lib.load().llg_timing(self._h, int(bool(enable))), "llg_timing")

    LAUNCH_MODES = {"field": 0, "rhs": 1, "energy": 2, "rk4": 3, "heun": 4, "rk4_vjp": 5, "relax": 6, "heun_vjp": 7}

    def last_launch_ms(self, kind: str) -> float:
        """Duration in ms of the last timed launch of one kind (llg_last_launch_ms):
        'field', 'rhs', 'energy', 'rk4', 'heun', 'rk4_vjp', 'relax' or 'heun_vjp'."""
        ms = ctypes.c_float()
        check(_lib.load().llg_last_launch_ms(self._h, self.LAUNCH_MODES[kind], ctypes.byref(ms)), "llg_last_launch_ms")
        return ms.value

    def debug_spin_limit(self, polls: int):
        """Failure-path test hook (llg_debug_spin_limit): group-barrier waits of later
        launches give up after `polls` polls; 0 restores the default."""
        check(_lib.load().llg_debug_spin_limit(self._h, int(polls)), "llg_debug_spin_limit")

    @property
    def on_chip(self) -> int:
        """The max_P of the on-chip spectra plan (0: none)."""
        return _lib.load().llg_get_on_chip(self._h)

    def launch_shape(self):
        """(unit groups, workgroups, threads per workgroup, transform policy)."""
        ug, nwg, nt, rs = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(_lib.load().llg_launch_shape(self._h, ctypes.byref(ug), ctypes.byref(nwg), ctypes.byref(nt),
                                           ctypes.byref(rs)), "llg_launch_shape")
        return ug.value, nwg.value, nt.value, rs.value

    def close(self):
        if self._h:
            _lib.load().llg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- helpers
    def _state(self, m: torch.Tensor, name="m") -> torch.Tensor:
        if not isinstance(m, torch.Tensor) or m.device.type != "cuda" or m.dtype != torch.float32:
            raise TypeError(f"{name} must be a float32 CUDA tensor")
        if not m.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if m.numel() != self.state_size:
            raise ValueError(f"{name} has {m.numel()} elements, the handle expects {self.state_size}")
        return m

    def _params(self, params):
        if isinstance(params, LLGParams):
            params = [params] * self.n
        if len(params) != self.n:
            raise ValueError(f"need {self.n} parameter sets")
        arr = (LLGParamsC * self.n)(*[p.to_c() for p in params])
        return arr

    def unpack(self, flat: torch.Tensor, k: int) -> torch.Tensor:
        D = self.D[k]
        o = self.offsets[k]
        return flat[o:o + 3 * D * D].view(3, D, D)

    def pack(self, states) -> torch.Tensor:
        return torch.cat([s.reshape(-1) for s in states]).contiguous()

    # ---------------------------------------------------------------- entry points
    def demag_field(self, m: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        m = self._state(m)
        H = torch.empty_like(m) if out is None else self._state(out, "out")
        check(_lib.load().llg_demag_field(self._h, _ptr(m), _ptr(H), _stream()), "llg_demag_field")
        return H

    def rhs(self, m: torch.Tensor, params, out: torch.Tensor | None = None) -> torch.Tensor:
        m = self._state(m)
        f = torch.empty_like(m) if out is None else self._state(out, "out")
        check(_lib.load().llg_rhs(self._h, _ptr(m), _ptr(f), self._params(params), _stream()), "llg_rhs")
        return f

    def rk4_step(self, m: torch.Tensor, nsteps: int, params) -> torch.Tensor:
        m = self._state(m)
        check(_lib.load().llg_rk4_step(self._h, _ptr(m), int(nsteps), self._params(params), _stream()), "llg_rk4_step")
        return m

    def heun_step(self, m: torch.Tensor, nsteps: int, params, *, seed: int, step0=0,
                  replica: int = 0) -> torch.Tensor:
        """step0=None: continue from the handle's device step counter (and advance it)."""
        m = self._state(m)
        s0 = _lib.STEP_COUNTER if step0 is None else int(step0)
        check(_lib.load().llg_heun_step(self._h, _ptr(m), int(nsteps), int(seed), s0, int(replica),
                                        self._params(params), _stream()), "llg_heun_step")
        return m

    def rk4_series(self, m: torch.Tensor, nsteps: int, params, sample_every: int) -> torch.Tensor:
        """RK4 steps in place with the observable series (llg_rk4_series): returns
        [ceil(nsteps / sample_every), n, 4] float64 (<m_x>, <m_y>, <m_z>, E) of the state
        at the start of every sample_every-th step."""
        m = self._state(m)
        ns = -(-int(nsteps) // int(sample_every))
        out = torch.empty(max(ns, 1), self.n, 4, dtype=torch.float64, device=self.device)
        check(_lib.load().llg_rk4_series(self._h, _ptr(m), int(nsteps), self._params(params), int(sample_every),
                                         _ptr(out), _stream()), "llg_rk4_series")
        return out[:ns]

    def heun_series(self, m: torch.Tensor, nsteps: int, params, sample_every: int, *, seed: int, step0=0,
                    replica: int = 0) -> torch.Tensor:
        """Heun steps in place with the observable series (llg_heun_series); step0=None
        continues the handle's step counter."""
        m = self._state(m)
        ns = -(-int(nsteps) // int(sample_every))
        out = torch.empty(max(ns, 1), self.n, 4, dtype=torch.float64, device=self.device)
        s0 = _lib.STEP_COUNTER if step0 is None else int(step0)
        check(_lib.load().llg_heun_series(self._h, _ptr(m), int(nsteps), int(seed), s0, int(replica),
                                          self._params(params), int(sample_every), _ptr(out), _stream()),
              "llg_heun_series")
        return out[:ns]

    def set_step(self, step: int):
        check(_lib.load().llg_step_counter_set(self._h, int(step), _stream()), "llg_step_counter_set")

    def get_step(self) -> int:
        v = ctypes.c_ulonglong(0)
        check(_lib.load().llg_step_counter_get(self._h, ctypes.byref(v), _stream()), "llg_step_counter_get")
        return int(v.value)

    def graph(self, integrator: str, m: torch.Tensor, nsteps: int, params, *, seed: int = 0,
              replica: int = 0) -> "Graph":
        """An executable hipGraph of nsteps RK4 or Heun steps on m (Heun continues the
        device step counter on every replay)."""
        m = self._state(m)
        g = ctypes.c_void_p()
        check(_lib.load().llg_graph_create(self._h, {"rk4": 0, "heun": 1}[integrator], _ptr(m), int(nsteps),
                                           self._params(params), int(seed), int(replica), ctypes.byref(g)),
              "llg_graph_create")
        return Graph(g, self, m)

    def relax(self, m: torch.Tensor, X_nm, params, *, kappa: float = 2.0, tol: float = 2e-6,
              max_sweeps: int = 100000, cutoff_nm: float = 0.0) -> torch.Tensor:
        """Constrained relaxation in place; returns [n, 8] float64 (lambda_x, lambda_y,
        sweeps, residual, C_x, C_y, 0, 0).  X_nm: one (x, y) per disk.  cutoff_nm:
        constraint over the cells within this distance of X (0 = the whole disk)."""
        m = self._state(m)
        flat = [float(v) for xy in X_nm for v in xy]
        if len(flat) != 2 * self.n:
            raise ValueError("need one (x, y) target per disk")
        X = (ctypes.c_double * (2 * self.n))(*flat)
        out = torch.zeros(self.n, 8, dtype=torch.float64, device=self.device)
        check(_lib.load().llg_relax(self._h, _ptr(m), X, float(cutoff_nm), float(kappa), float(tol), int(max_sweeps),
                                    self._params(params), _ptr(out), _stream()), "llg_relax")
        return out

    def rk4_record(self, m: torch.Tensor, nsteps: int, params, rec: torch.Tensor) -> torch.Tensor:
        m = self._state(m)
        if rec.dtype != torch.float32 or rec.device.type != "cuda" or rec.numel() < 8 * nsteps * self.state_size:
            raise ValueError("rec must be a float32 CUDA tensor of 8 * nsteps * state_size elements")
        check(_lib.load().llg_rk4_record(self._h, _ptr(m), int(nsteps), self._params(params), _ptr(rec), _stream()),
              "llg_rk4_record")
        return m

    def rk4_vjp(self, rec: torch.Tensor, nsteps: int, ybar: torch.Tensor, pgrad: torch.Tensor, params):
        ybar = self._state(ybar, "ybar")
        if pgrad.dtype != torch.float64 or pgrad.numel() != 2 * self.n or pgrad.device.type != "cuda":
            raise ValueError("pgrad must be a float64 CUDA tensor with 2 entries per disk")
        check(_lib.load().llg_rk4_vjp(self._h, _ptr(rec), int(nsteps), _ptr(ybar), _ptr(pgrad),
                                      self._params(params), _stream()), "llg_rk4_vjp")
        return ybar

    def heun_record(self, m: torch.Tensor, nsteps: int, params, rec: torch.Tensor, *, seed: int, step0: int,
                    replica: int = 0) -> torch.Tensor:
        m = self._state(m)
        if rec.numel() < 4 * nsteps * self.state_size or rec.dtype != torch.float32 or not rec.is_contiguous():
            raise ValueError("rec needs 4 * nsteps * state_size contiguous float32")
        check(_lib.load().llg_heun_record(self._h, _ptr(m), int(nsteps), int(seed), int(step0), int(replica),
                                          self._params(params), _ptr(rec), _stream()), "llg_heun_record")
        return m

    def heun_vjp(self, rec: torch.Tensor, nsteps: int, ybar: torch.Tensor, pgrad: torch.Tensor, params, *,
                 seed: int, step0: int, replica: int = 0):
        ybar = self._state(ybar, "ybar")
        if pgrad.dtype != torch.float64 or pgrad.numel() != 2 * self.n:
            raise ValueError("pgrad: 2 float64 per disk")
        check(_lib.load().llg_heun_vjp(self._h, _ptr(rec), int(nsteps), int(seed), int(step0), int(replica),
                                       _ptr(ybar), _ptr(pgrad), self._params(params), _stream()), "llg_heun_vjp")
        return ybar

    def core_position_vjp(self, m: torch.Tensor, lambda_ex_nm: float, core: torch.Tensor, rbar: torch.Tensor,
                          mbar: torch.Tensor):
        m = self._state(m)
        mbar = self._state(mbar, "mbar")
        check(_lib.load().llg_core_position_vjp(self._h, _ptr(m), float(lambda_ex_nm), _ptr(core.contiguous()),
                                                _ptr(rbar.contiguous()), _ptr(mbar), _stream()),
              "llg_core_position_vjp")
        return mbar

    def noise(self, seed: int, step: int, replica: int = 0) -> torch.Tensor:
        w = torch.empty(self.state_size, dtype=torch.float32, device=self.device)
        check(_lib.load().llg_noise(self._h, int(seed), int(step), int(replica), _ptr(w), _stream()), "llg_noise")
        return w

    def energy(self, m: torch.Tensor, params) -> torch.Tensor:
        m = self._state(m)
        out = torch.empty(self.n, 4, dtype=torch.float64, device=self.device)
        check(_lib.load().llg_energy(self._h, _ptr(m), self._params(params), _ptr(out), _stream()), "llg_energy")
        return out

    def vortex_core_position(self, m: torch.Tensor, lambda_ex_nm: float, hint_nm=None) -> torch.Tensor:
        m = self._state(m)
        out = torch.empty(self.n, 5, dtype=torch.float64, device=self.device)
        hint = None
        if hint_nm is not None:
            flat = [float(v) for xy in hint_nm for v in xy] if self.n > 1 or hasattr(hint_nm[0], "__len__") \
                else [float(hint_nm[0]), float(hint_nm[1])]
            hint = (ctypes.c_double * (2 * self.n))(*flat)
        check(_lib.load().llg_vortex_core_position(self._h, _ptr(m), float(lambda_ex_nm), hint, _ptr(out),
                                                   _stream()), "llg_vortex_core_position")
        return out

    def mean_m(self, m: torch.Tensor) -> torch.Tensor:
        m = self._state(m)
        out = torch.empty(self.n, 3, dtype=torch.float64, device=self.device)
        check(_lib.load().llg_mean_m(self._h, _ptr(m), _ptr(out), _stream()), "llg_mean_m")
        return out

    def check(self):
        """Synchronise and raise if a device-side failure was recorded."""
        check(_lib.load().llg_check(self._h, _stream()), "llg_check")


# ---------------------------------------------------------------- C-ABI-named functions
class Graph:
    """Executable graph from Disk.graph; launch() enqueues one replay on the current stream."""

    def __init__(self, handle, disk: Disk, m: torch.Tensor):
        self._g = handle
        self._disk = disk      # the handle and the state must outlive the graph
        self._m = m

    def launch(self):
        check(_lib.load().llg_graph_launch(self._g, _stream()), "llg_graph_launch")

    def close(self):
        if self._g:
            _lib.load().llg_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def power_spectrum(x: torch.Tensor, remove_mean: bool = True, window: str = "none") -> torch.Tensor:
    """llg_power_spectrum of the rows of x ([n_seq, len] or [len], float64 on the GPU,
    len a power of two): |X_k|^2 / len for k = 0 .. len/2."""
    if x.dtype != torch.float64 or x.device.type != "cuda":
        raise TypeError("x must be a float64 CUDA tensor")
    x2 = x.reshape(-1, x.shape[-1])
    n_seq, n = x2.shape
    out = torch.empty(n_seq, n // 2 + 1, dtype=torch.float64, device=x.device)
    work = torch.empty(4 * n * n_seq, dtype=torch.float64, device=x.device)
    check(_lib.load().llg_power_spectrum(_ptr(x2), int(n_seq), int(x2.stride(0)), int(n), int(x2.stride(1)),
                                         int(bool(remove_mean)), {"none": 0, "hann": 1}[window], _ptr(work),
                                         _ptr(out), _stream()), "llg_power_spectrum")
    return out.reshape(*x.shape[:-1], n // 2 + 1)


def build_kernels(R_nm: float, L_nm: float, a_nm: float = 2.0, P: int = 0) -> Disk:
    return Disk.build(R_nm, L_nm, a_nm, P)


def batch_create(R_nm, L_nm, a_nm: float = 2.0, wg_per_disk=None) -> Disk:
    return Disk.batch(R_nm, L_nm, a_nm, wg_per_disk)


def demag_field(disk: Disk, m, out=None):
    return disk.demag_field(m, out)


def llg_rhs(disk: Disk, m, params, out=None):
    return disk.rhs(m, params, out)


def rk4_step(disk: Disk, m, nsteps, params):
    return disk.rk4_step(m, nsteps, params)


def heun_step(disk: Disk, m, nsteps, params, *, seed, step0=0, replica=0):
    return disk.heun_step(m, nsteps, params, seed=seed, step0=step0, replica=replica)


def vortex_core_position(disk: Disk, m, lambda_ex_nm, hint_nm=None):
    return disk.vortex_core_position(m, lambda_ex_nm, hint_nm)


def energy(disk: Disk, m, params):
    return disk.energy(m, params)
