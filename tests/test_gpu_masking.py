"""The integrators read the caller's state only inside the disk (Sec. II: the
magnetisation lives on the disk cells; cells of the box outside the disk carry
none).  The kernels apply the disk test only where a caller's state is read
(the first stage of a launch); every later stage reads states the kernel wrote
itself, which are zero outside the disk.  So a start state with NaN outside
the disk must give bitwise the same result as the same state with zeros there,
and every returned state is zero outside the disk.

Ragged batch over the FFT sizes 64, 128 and 256; RK4 and Heun, with and
without the observable series, and RK4 with the small disks' spectra on chip;
the series of the two runs must agree bitwise as well (their first sample
reads the caller's state)."""
import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle

pytestmark = pytest.mark.gpu
C_PY = 0.14298555


def _batch():
    from paper_1207_2192_amd import Disk
    Rs, Ls = [30.0, 45.0, 80.0], [10.0, 6.0, 8.0]
    disk = Disk.batch(Rs, Ls)
    masks = [oracle.Disk(R, L).mask.numpy() for R, L in zip(Rs, Ls)]
    return disk, masks


def _states(disk, masks):
    clean, junk = [], []
    for k, (D, mk) in enumerate(zip(disk.D, masks)):
        s = li.vortex_ansatz(D, 2.0 + k, -1.5).astype(np.float32)
        s[:, ~mk] = 0.0
        j = s.copy()
        j[:, ~mk] = np.nan
        clean.append(s.reshape(-1))
        junk.append(j.reshape(-1))
    dev = lambda parts: torch.tensor(np.concatenate(parts), dtype=torch.float32, device="cuda")
    return dev(clean), dev(junk)


@pytest.mark.parametrize("kind", ["rk4", "heun", "rk4_series", "heun_series", "rk4_on_chip"])
def test_state_outside_the_disk_is_never_read(kind):
    from paper_1207_2192_amd import LLGParams
    disk, masks = _batch()
    print(f"masking: {kind}, D = {disk.D}, P = {disk.P}", flush=True)
    thermal = kind.startswith("heun")
    ps = [LLGParams(alpha=0.05, c=C_PY, dtau=0.04, hext=(0.01, 0.0, 0.0), temp=0.05 if thermal else 0.0,
                    renorm=thermal)] * disk.n
    a, b = _states(disk, masks)
    if kind == "rk4_on_chip":   # the P <= 128 disks keep their spectra in LDS
        disk.tune(1, None, 0)
        disk.set_on_chip(128)
    if kind.startswith("rk4") and not kind.endswith("series"):
        disk.rk4_step(a, 5, ps)
        disk.rk4_step(b, 5, ps)
    elif kind == "heun":
        disk.heun_step(a, 5, ps, seed=11, step0=3)
        disk.heun_step(b, 5, ps, seed=11, step0=3)
    elif kind == "rk4_series":
        sa = disk.rk4_series(a, 6, ps, 2)
        sb = disk.rk4_series(b, 6, ps, 2)
        assert torch.equal(sa, sb)
        assert bool(torch.isfinite(sa).all())
    else:
        sa = disk.heun_series(a, 6, ps, 2, seed=11, step0=3)
        sb = disk.heun_series(b, 6, ps, 2, seed=11, step0=3)
        assert torch.equal(sa, sb)
        assert bool(torch.isfinite(sa).all())
    disk.check()
    assert torch.equal(a, b)
    for k, mk in enumerate(masks):
        out = disk.unpack(a, k).cpu().numpy().reshape(3, *mk.shape)
        assert np.all(out[:, ~mk] == 0.0)
        assert np.all(np.isfinite(out))
    disk.close()
