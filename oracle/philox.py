"""Gaussian test matrices from a counter-based generator (oracle side).

The paper only asks for randn: every entry of the range test matrix
Omega_r (Sect. 3, Alg. 1-2, Alg. 9) and of the co-range test matrix Omega_c
(Sect. 6.2, Alg. 7) is an independent standard Gaussian.  A counter-based
generator lets every entry be recomputed from its coordinates, so the GPU
library and this oracle can draw the *same* matrices without ever exchanging
them.  Each side implements the generator independently from its published
definition:

* Philox4x32-10, Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11: a 4x32-bit counter and a 2x32-bit key, ten rounds
  of two 32x32->64-bit multiplications and xors, key bumped by the golden-ratio
  and sqrt(3)-1 Weyl constants between rounds.
* Box & Muller (1958): two uniforms (u0, u1) in (0, 1) give two independent
  N(0, 1) values sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1).

Coordinate convention (shared by contract, not by code, with the GPU side):
an entry has a *long* index i (the index along the matrix's long side), a
*short* index j, a batch index b and a tag t naming the matrix.  Its counter is
(i >> 2, j, b, t), its key is (seed mod 2^32, seed >> 32), and output word
i & 3 of the Philox block is used.  Words (0, 1) form one Box-Muller pair (cos,
sin) and words (2, 3) the other.  A word x becomes the uniform (x + 1/2) 2^-32.

Pinned by: the Random123 known-answer vectors (tests/golden/philox_kat.txt),
sample moments and a Kolmogorov-Smirnov test of the Gaussians.
"""

import numpy as np

# Round multipliers and Weyl key increments of Philox4x32 (SC'11, Sect. 4).
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_SH = np.uint64(32)

TAG_OMEGA = 1      # range test matrix Omega_r (n x s); long = row, short = column
TAG_PSI = 2        # co-range test matrix Omega_c^T (s_w x m); long = column, short = row
TAG_PHI = 3        # optional core test matrix Phi (s_c x m)
TAG_PHI2 = 4       # optional core test matrix Phi' (s_c x n)


def philox4x32_10(ctr, key):
    """Ten Philox4x32 rounds.

    ctr: uint array of shape (4, N) (values < 2^32); key: pair of ints.
    Returns a uint64 array of shape (4, N) holding 32-bit words.
    """
    c0, c1, c2, c3 = (np.asarray(w, dtype=np.uint64) & _MASK for w in ctr)
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0          # exact: both factors < 2^32
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _SH, p0 & _MASK
        hi1, lo1 = p1 >> _SH, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3])


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def gaussian(seed, tag, batch, long_idx, short_idx):
    """Canonical FP64 N(0,1) values at the given (long, short) coordinates.

    long_idx and short_idx are broadcast against each other.
    """
    li, sj = np.broadcast_arrays(np.asarray(long_idx, dtype=np.int64),
                                 np.asarray(short_idx, dtype=np.int64))
    shape = li.shape
    li = li.ravel()
    sj = sj.ravel()
    n = li.size
    ctr = (li >> 2, sj, np.full(n, int(batch)), np.full(n, int(tag)))
    words = philox4x32_10(ctr, seed_key(seed))           # (4, n)
    u = (words.astype(np.float64) + 0.5) * 2.0 ** -32     # uniforms in (0, 1)
    lane = (li & 3).astype(np.int64)
    first = lane & 2                                      # 0 -> pair (0,1), 2 -> pair (2,3)
    cols = np.arange(n)
    ua = u[first, cols]
    ub = u[first + 1, cols]
    radius = np.sqrt(-2.0 * np.log(ua))
    angle = 2.0 * np.pi * ub
    z = np.where((lane & 1) == 0, radius * np.cos(angle), radius * np.sin(angle))
    return z.reshape(shape)


def omega(seed, n, s, batch=0):
    """Range test matrix Omega (n x s): entry (i, j) has long i, short j."""
    return gaussian(seed, TAG_OMEGA, batch, np.arange(n)[:, None], np.arange(s)[None, :])


def psi(seed, s_w, m, batch=0):
    """Co-range test matrix Psi = Omega_c^T (s_w x m): entry (r, i) has long i, short r."""
    return gaussian(seed, TAG_PSI, batch, np.arange(m)[None, :], np.arange(s_w)[:, None])


def phi(seed, s_c, length, tag, batch=0):
    """Core-sketch test matrix (s_c x length) with the given tag (TAG_PHI/TAG_PHI2)."""
    return gaussian(seed, tag, batch, np.arange(length)[None, :], np.arange(s_c)[:, None])
