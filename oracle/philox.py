"""Counter-based thermal noise: Philox4x32-10 and Box-Muller.

The paper draws its stochastic fields from a sequential generator (Sec. III.C);
a sequential stream cannot give independent streams per cell and replica, so
this method uses the counter-based Philox4x32 generator with 10 rounds
(Salmon, Moraes, Dror, Shaw, SC'11), implemented here from its definition:
each round multiplies counter words 0 and 2 by two fixed 32-bit constants,
takes the high and low halves of the 64-bit products, and mixes them with the
other two words and the key; the key is bumped by two Weyl constants between
rounds.

Noise layout (shared with the HIP library): the two cells (2p, ix) and
(2p+1, ix) of row pair p draw from two blocks with counters
(s mod 2^32, s div 2^32, 2q + h, replica), h = 0, 1, q = p*D + ix, and key
(seed mod 2^32, seed div 2^32) for time step s.  Each 32-bit output x gives a
uniform u = ((x >> 8) + 0.5) * 2^-24 (exact in FP32); the first six of the
eight uniforms U0..U7 (block h = 0, then h = 1) give three Box-Muller pairs
  n_2k = sqrt(-2 ln U_2k) cos(2 pi U_2k+1),  n_2k+1 = sqrt(-2 ln U_2k) sin(2 pi U_2k+1),
and cell (2p, ix) takes (n0, n1, n2), cell (2p+1, ix) takes (n3, n4, n5).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)
_32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function.

    ctr: four arrays of 32-bit values, key: two (broadcastable; any integer
    dtype).  Returns four uint64 arrays holding 32-bit values.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _LO for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & _LO for k in key)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & _LO
            k1 = (k1 + W1) & _LO
        p0 = M0 * c0            # exact: both factors < 2^32
        p1 = M1 * c2
        c0, c1, c2, c3 = (p1 >> _32) ^ c1 ^ k0, p1 & _LO, (p0 >> _32) ^ c3 ^ k1, p0 & _LO
    return c0, c1, c2, c3


def uniforms24(x: np.ndarray) -> np.ndarray:
    """Top 24 bits of a 32-bit word as a uniform in (0, 1), in float64."""
    return (((np.asarray(x, dtype=np.uint64) & _LO) >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24


def gaussian_field(seed: int, step: int, replica, D: int) -> np.ndarray:
    """Standard-normal noise of every box cell.

    replica: an int (returns [3, D, D]) or a 1-D array of replica indices
    (returns [B, 3, D, D]); all float64.
    """
    scalar = np.ndim(replica) == 0
    reps = np.atleast_1d(np.asarray(replica, dtype=np.uint64))[:, None]
    n_pairs = (D + 1) // 2
    q = np.arange(n_pairs * D, dtype=np.uint64)[None, :]          # q = p*D + ix
    s_lo, s_hi = np.uint64(step & 0xFFFFFFFF), np.uint64(step >> 32)
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64(seed >> 32))
    U = []
    for h in (0, 1):
        U += [uniforms24(x) for x in philox4x32_10((s_lo, s_hi, 2 * q + np.uint64(h), reps), key)]
    n = []
    for k in range(3):
        r = np.sqrt(-2.0 * np.log(U[2 * k]))
        n += [r * np.cos(2 * np.pi * U[2 * k + 1]), r * np.sin(2 * np.pi * U[2 * k + 1])]
    even = np.stack(n[:3], axis=1).reshape(-1, 3, n_pairs, D)    # cells (2p, ix)
    odd = np.stack(n[3:], axis=1).reshape(-1, 3, n_pairs, D)     # cells (2p+1, ix)
    w = np.stack([even, odd], axis=3).reshape(-1, 3, 2 * n_pairs, D)[:, :, :D]
    return w[0] if scalar else w
