"""Pins of the oracle's Gaussian test matrices (the paper's randn, Sect. 2)."""

import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(row):
    ctr = np.array(row[0:4], dtype=np.uint64)[:, None]
    out = philox.philox4x32_10(ctr, (row[4], row[5]))[:, 0]
    assert [int(x) for x in out] == row[6:10]


def test_gaussian_moments_and_ks():
    z = philox.gaussian(12345, philox.TAG_OMEGA, 0, np.arange(1 << 20), 7)
    assert abs(z.mean()) < 5e-3
    assert abs(z.var() - 1.0) < 5e-3
    assert abs(stats.skew(z)) < 1e-2
    assert abs(stats.kurtosis(z)) < 2e-2
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_box_muller_pairs_share_radius():
    # words (0,1) and (2,3) of one Philox block form two Box-Muller pairs:
    # z_a^2 + z_b^2 = -2 ln u_a for each pair (closed form of the transform).
    seed, tag, j = 99, philox.TAG_PSI, 3
    i = np.arange(64)
    z = philox.gaussian(seed, tag, 0, i, j).reshape(16, 4)
    words = philox.philox4x32_10((np.arange(16), np.full(16, j), np.zeros(16), np.full(16, tag)),
                                 philox.seed_key(seed))
    u = (words.astype(np.float64) + 0.5) * 2.0 ** -32
    np.testing.assert_allclose(z[:, 0] ** 2 + z[:, 1] ** 2, -2 * np.log(u[0]), rtol=1e-12)
    np.testing.assert_allclose(z[:, 2] ** 2 + z[:, 3] ** 2, -2 * np.log(u[2]), rtol=1e-12)
    np.testing.assert_allclose(np.arctan2(z[:, 1], z[:, 0]) % (2 * np.pi), 2 * np.pi * u[1],
                               rtol=1e-9, atol=1e-9)


def test_matrix_coordinates_and_independence():
    om = philox.omega(7, 37, 5)
    assert om.shape == (37, 5)
    assert om[13, 2] == philox.gaussian(7, philox.TAG_OMEGA, 0, 13, 2)
    ps = philox.psi(7, 5, 37)
    assert ps[2, 13] == philox.gaussian(7, philox.TAG_PSI, 0, 13, 2)
    # different tags, seeds and batch indices give unrelated streams
    assert not np.allclose(om, ps.T)
    assert not np.allclose(om, philox.omega(8, 37, 5))
    assert not np.allclose(om, philox.omega(7, 37, 5, batch=1))
    # the high half of the 64-bit seed reaches the key
    assert not np.allclose(om, philox.omega(7 + (1 << 32), 37, 5))
    # column j of a wider matrix is column j of a narrower one (prefix property)
    np.testing.assert_array_equal(philox.omega(7, 37, 9)[:, :5], om)
