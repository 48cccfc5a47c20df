"""Truncated eigendecompositions of the normal matrix J^T J (Sect. 4.2).

TEST INFRASTRUCTURE ONLY (see the package header).

J is m x n (the paper's n_r x n_c); every method returns V (n x k, the
approximate leading eigenvectors of J^T J, i.e. right singular vectors of J)
and the k leading approximate eigenvalues lam2 (descending).  Each column of
V is sign-fixed so that its entry of largest magnitude is positive.

* ``nystrom``   -- Alg. 4, the prolonged (Nystrom) sketch with v >= 2 views.
* ``pinched``   -- Alg. 5, the pinched sketch with v >= 2 views.
* ``subspace_rule`` -- Alg. 2 used for J^T J the way Sect. 4.2.1 recommends:
  on J for even v and on J^T for odd v (the side whose basis the final small
  SVD expands is then the more accurate one).

Pinned by: exact recovery of an exactly rank-k J; the dense eigendecomposition
of J^T J when s = n; the equivalences of Sect. 4.2.3 (Alg. 4 with v views
equals Alg. 2 applied to J for even v and to J^T for odd v, up to the shift
nu; Alg. 5 with v views equals Alg. 2 applied to J^T for even v and to J for
odd v); and Nystrom at least as accurate as pinched on average.
"""

from dataclasses import dataclass

import numpy as np
import scipy.linalg

from . import linalg, philox, rsvd


@dataclass
class NormalResult:
    V: np.ndarray          # n x k
    lam2: np.ndarray       # k eigenvalues of J^T J, descending
    Qr: np.ndarray = None  # the co-range basis the approximation is built on
    nu: float = 0.0


def _signs(v):
    return linalg.canonical_signs(v, v)[0]


def _co_range_basis(j, k, p, views, seed, on_transpose):
    """Alg. 3 on J (even ``views``) or on J^T (odd ``views``): an n x s basis."""
    src = rsvd.Transposed(j) if on_transpose else j
    return rsvd.alg3_qr_or_qc(src, k, p, views, seed)


def nystrom(j, k, p, v, seed):
    """Alg. 4: Q_r from v - 2 views (Alg. 3 on J for even v, on J^T for odd v;
    orth(Omega) for v = 2), then two views Y_r = J^T (J Q_r), the shift
    nu = 2.2e-16 ||Y_r||_2, Y_r += nu Q_r, B = Q_r^T Y_r,
    C_L = chol((B + B^T)/2, lower), F = C_L^-1 Y_r^T, [~, Lam^, V] = tsvd(F, k)
    and Lam^2 = Lam^^2 - nu with negative entries set to 0."""
    m, n, s = rsvd._check_sizes(j, k, p)
    if v < 2:
        raise ValueError("Alg. 4 needs v >= 2 views")
    if v == 2:
        q_r = linalg.orth(philox.omega(seed, n, s))
    else:
        q_r = _co_range_basis(j, k, p, v - 2, seed, on_transpose=(v % 2 == 1))
    y_r = rsvd.times_t(j, rsvd.times(j, q_r))
    nu = 2.2e-16 * np.linalg.norm(y_r, 2)
    y_r = y_r + nu * q_r
    b = q_r.T @ y_r
    c_l = np.linalg.cholesky((b + b.T) / 2.0)
    f = scipy.linalg.solve_triangular(c_l, y_r.T, lower=True)
    _, lam_hat, vk = linalg.tsvd(f, k)
    lam2 = np.maximum(lam_hat ** 2 - nu, 0.0)
    return NormalResult(_signs(vk), lam2, q_r, nu)


def pinched(j, k, p, v, seed):
    """Alg. 5: Q_r from v - 1 views (Alg. 3 on J^T for even v, on J for odd v),
    one more view B_c = J Q_r, [Lam^2, V^] = tevd(B_c^T B_c, k), V = Q_r V^."""
    m, n, s = rsvd._check_sizes(j, k, p)
    if v < 2:
        raise ValueError("Alg. 5 needs v >= 2 views")
    q_r = _co_range_basis(j, k, p, v - 1, seed, on_transpose=(v % 2 == 0))
    b_c = rsvd.times(j, q_r)
    evals, evecs = np.linalg.eigh(b_c.T @ b_c)
    order = np.argsort(evals)[::-1][:k]
    return NormalResult(_signs(q_r @ evecs[:, order]), evals[order].copy(), q_r)


def subspace_rule(j, k, p, v, seed):
    """Alg. 2 for J^T J per Sect. 4.2.1: on J for even v (V = its right factor),
    on J^T for odd v (V = the left factor of J^T); eigenvalues sigma^2."""
    if v % 2 == 0:
        res = rsvd.alg2_gensubit(j, k, p, v, seed)
        return NormalResult(_signs(res.V), res.S ** 2, res.Qr)
    res = rsvd.alg2_gensubit(rsvd.Transposed(j), k, p, v, seed)
    return NormalResult(_signs(res.U), res.S ** 2, res.Qc)
