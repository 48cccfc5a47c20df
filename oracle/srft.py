"""Subsampled randomized trigonometric test matrices (the SRFTs of Sect. 6.7).

TEST INFRASTRUCTURE ONLY (see the package header).

For one side of length L (L = m for Phi_r, L = n for Phi_c) the paper's SRFT is
Phi = D F P (L x s): D a diagonal of independent random signs, F a discrete
cosine transform matrix (A is real), and P the s columns of the identity at s
positions drawn without replacement.  Readings taken here:

* F is the transpose of the orthonormal DCT-II matrix C,
  C[f, j] = a_f cos(pi (2j + 1) f / (2L)) with a_0 = sqrt(1/L) and
  a_f = sqrt(2/L) otherwise, so that Phi^T x = P^T C D x: flip the signs of
  x, take its orthonormal DCT-II and keep the sampled frequencies.  The
  sketch Z = Phi_r^T A Phi_c is then the sampled two-dimensional DCT-II of
  D_r A D_c.
* Signs and samples come from the same counter-based generator as the
  Gaussian test matrices (``philox``): entry j of a side uses counter
  (j >> 2, 0, 0, tag) and output word j & 3.  The sign is - when the top bit
  of the word under the side's sign tag is set.  The sample holds the s
  positions with the smallest (word under the side's key tag, position)
  pairs, i.e. a uniformly random s-subset, listed in increasing position
  (the extended sketch does not depend on the order of the columns of Phi).

Pinned by: Phi^T x against scipy's orthonormal DCT-II (also at a length of
65536, where an unreduced angle would be off by about 1e-11), orthonormal
columns, distinct in-range sample positions, and the sample against a
brute-force sort of the generator words.
"""

import numpy as np

from . import philox

ROWS = (6, 7)      # (sign tag, sample tag) of Phi_r (length m)
COLS = (8, 9)      # (sign tag, sample tag) of Phi_c (length n)


def words(seed, tag, length):
    """Generator word of every position j = 0..length-1 under ``tag``."""
    j = np.arange(length, dtype=np.int64)
    ctr = (j >> 2, np.zeros(length, dtype=np.int64), np.zeros(length, dtype=np.int64),
           np.full(length, int(tag), dtype=np.int64))
    w = philox.philox4x32_10(ctr, philox.seed_key(seed))
    return w[j & 3, np.arange(length)].astype(np.uint64)


def signs(seed, length, side):
    """The diagonal of D: +1 or -1 for every position."""
    w = words(seed, side[0], length)
    return np.where((w >> np.uint64(31)) & np.uint64(1), -1.0, 1.0)


def sample(seed, length, s, side):
    """P: the s sampled positions, in increasing order."""
    if not 0 <= s <= length:
        raise ValueError("need 0 <= s <= length")
    w = words(seed, side[1], length)
    order = np.lexsort((np.arange(length), w))        # by word, then by position
    return np.sort(order[:s])


def _cos_angles(j, f, length):
    """cos(pi (2j + 1) f / (2 length)) for integer arrays j, f.  The cosine has
    period 4 length in the integer (2j + 1) f, which is reduced exactly before
    the one rounding of t / (2 length): the angle then carries an absolute
    error of about 2^-53 pi instead of one proportional to its size (up to
    pi length)."""
    t = np.mod((2 * np.asarray(j, dtype=np.int64) + 1) * np.asarray(f, dtype=np.int64), 4 * length)
    return np.cos(np.pi * (t.astype(np.float64) / (2.0 * length)))


def dct2_matrix(length):
    """The orthonormal DCT-II matrix C (length x length), from its definition."""
    f = np.arange(length, dtype=np.int64)[:, None]
    j = np.arange(length, dtype=np.int64)[None, :]
    c = _cos_angles(j, f, length)
    scale = np.full(length, np.sqrt(2.0 / length))
    scale[0] = np.sqrt(1.0 / length)
    return c * scale[:, None]


def matrix(seed, length, s, side):
    """Phi = D C^T P (length x s): column c is sign-flipped row P[c] of C."""
    d = signs(seed, length, side)
    pos = sample(seed, length, s, side)
    j = np.arange(length, dtype=np.int64)[:, None]
    scale = np.where(pos == 0, np.sqrt(1.0 / length), np.sqrt(2.0 / length))[None, :]
    return d[:, None] * scale * _cos_angles(j, pos[None, :], length)
