"""The C-ABI library loads and exports every entry point the header declares
(no device work: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "llgdisk.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(llg_[a-z0-9_]+)\s*\(", txt)))


def lib():
    from paper_1207_2192_amd import _lib
    return _lib.load()


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("llg_build_kernels", "llg_demag_field", "llg_rhs", "llg_rk4_step", "llg_heun_step",
              "llg_vortex_core_position", "llg_energy", "llg_batch_create", "llg_destroy", "llg_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = lib()
    for n in declared():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L._name], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (llg_[a-z0-9_]+)", out))
    assert set(declared()) <= exported


def test_binding_covers_every_symbol():
    from paper_1207_2192_amd import _lib
    assert set(declared()) == set(_lib.SIGNATURES)


def test_params_from_si_matches_oracle_units():
    from oracle import Material, dimensionless
    from paper_1207_2192_amd import params_from_si
    p, lam = params_from_si(13e-12, 860e3, 1.76e11, 2.0, 20.0, 0.02, 300.0, 0.1)
    ref = dimensionless(Material(), 2.0, 20.0, dt_ps=0.02, T_K=300.0)
    assert abs(lam - ref["lambda_ex_nm"]) < 1e-12
    assert abs(p.c - ref["c"]) < 1e-15 and abs(p.temp - ref["temp"]) < 1e-15
    assert abs(p.dtau - ref["dtau"]) < 1e-12 and p.alpha == 0.1


def test_host_argument_errors_are_reported():
    L = lib()
    from paper_1207_2192_amd._lib import LLGParamsC
    rc = L.llg_params_from_si(-1.0, 860e3, 1.76e11, 2.0, 20.0, 0.02, 300.0, 0.1, ctypes.byref(LLGParamsC()), None)
    assert rc == -1 and b"positive" in L.llg_last_error()
    assert L.llg_disk_count(None) == -1
