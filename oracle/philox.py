"""Counter-based thermal noise: Philox4x64-10 and Box-Muller.

The paper draws its stochastic fields from a sequential generator (Sec. III.C);
a sequential stream cannot give independent streams per cell and replica, so
this method uses the counter-based Philox4x64 generator with 10 rounds
(Salmon, Moraes, Dror, Shaw, SC'11), implemented here from its definition:
each round multiplies counter words 0 and 2 by two fixed 64-bit constants,
takes the high and low halves of the 128-bit products, and mixes them with
the other two words and the key; the key is bumped by two Weyl constants
between rounds.

Noise layout (shared with the HIP library): the two cells (2p, ix) and
(2p+1, ix) of row pair p and column ix draw from one block.  For time step
``step`` and replica ``replica`` the block counter is (step, p*D + ix,
replica, 0) and the key is (seed, 0).  Each 64-bit output x_k gives two
uniforms, from its top 24 bits and from bits 8..31:
  hi(x) = ((x >> 40) + 0.5) * 2^-24,  lo(x) = (((x >> 8) mod 2^24) + 0.5) * 2^-24
(both exact in FP32), and U = (hi x0, lo x0, hi x1, lo x1, hi x2, lo x2)
gives six standard normals by Box-Muller,
  n_{2k} = sqrt(-2 ln U_{2k}) cos(2 pi U_{2k+1}),
  n_{2k+1} = sqrt(-2 ln U_{2k}) sin(2 pi U_{2k+1}),   k = 0, 1, 2;
cell (2p, ix) takes (n0, n1, n2) and cell (2p+1, ix) takes (n3, n4, n5).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO = np.uint64(0xFFFFFFFF)
_32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: np.uint64):
    """High and low 64-bit halves of the 128-bit product a*b (elementwise)."""
    a_lo, a_hi = a & _LO, a >> _32
    b_lo, b_hi = b & _LO, b >> _32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _32) + (lh & _LO) + (hl & _LO)
    hi = hh + (lh >> _32) + (hl >> _32) + (mid >> _32)
    lo = (mid << _32) | (ll & _LO)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64-10 block function.

    ctr: four uint64 arrays (broadcastable), key: two uint64 arrays.
    Returns four uint64 arrays.
    """
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
        k0, k1 = (np.asarray(k, dtype=np.uint64) for k in key)
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniforms24(x: np.ndarray) -> np.ndarray:
    """Top 24 bits of a uint64 as a uniform in (0, 1), in float64."""
    return ((x >> np.uint64(40)).astype(np.float64) + 0.5) * 2.0 ** -24


def uniforms24_low(x: np.ndarray) -> np.ndarray:
    """Bits 8..31 of a uint64 as a uniform in (0, 1), in float64."""
    return (((x >> np.uint64(8)) & np.uint64(0xFFFFFF)).astype(np.float64) + 0.5) * 2.0 ** -24


def gaussian_field(seed: int, step: int, replica, D: int) -> np.ndarray:
    """Standard-normal noise of every box cell.

    replica: an int (returns [3, D, D]) or a 1-D array of replica indices
    (returns [B, 3, D, D]); all float64.
    """
    scalar = np.ndim(replica) == 0
    reps = np.atleast_1d(np.asarray(replica, dtype=np.uint64))[:, None]
    n_pairs = (D + 1) // 2
    q = np.arange(n_pairs * D, dtype=np.uint64)[None, :]          # q = p*D + ix
    x0, x1, x2, _ = philox4x64_10((np.uint64(step), q, reps, np.uint64(0)),
                                  (np.uint64(seed), np.uint64(0)))
    U = [f(x) for x in (x0, x1, x2) for f in (uniforms24, uniforms24_low)]
    n = []
    for k in range(3):
        r = np.sqrt(-2.0 * np.log(U[2 * k]))
        n += [r * np.cos(2 * np.pi * U[2 * k + 1]), r * np.sin(2 * np.pi * U[2 * k + 1])]
    even = np.stack(n[:3], axis=1).reshape(-1, 3, n_pairs, D)    # cells (2p, ix)
    odd = np.stack(n[3:], axis=1).reshape(-1, 3, n_pairs, D)     # cells (2p+1, ix)
    w = np.stack([even, odd], axis=3).reshape(-1, 3, 2 * n_pairs, D)[:, :, :D]
    return w[0] if scalar else w
