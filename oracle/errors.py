"""Accuracy measures of Sect. 8.2 and the projection errors of Thm. 3.1/4.1.

TEST INFRASTRUCTURE ONLY.
"""

import numpy as np

from .rsvd import dense, times, times_t


def optimal_tail_frob(sigma_all, k):
    """||A - [[A]]_k||_F from the full singular spectrum."""
    s = np.asarray(sigma_all, dtype=np.float64)
    return float(np.sqrt(np.sum(s[k:] ** 2)))


def approx_frob_error(a, u, s, v):
    """||A - U diag(s) V^T||_F for orthonormal U, V, via
    ||A||_F^2 - 2 tr(diag(s) U^T A V) + ||s||^2 (one product with A)."""
    av = times(a, v)
    cross = float(np.sum(s * np.einsum("ij,ij->j", u, av)))
    m = a.shape[0]
    fro2 = 0.0
    for r0 in range(0, m, 8192):
        blk = dense_rows(a, r0, min(m, r0 + 8192))
        fro2 += float(np.sum(blk * blk))
    val = fro2 - 2.0 * cross + float(np.sum(s * s))
    return float(np.sqrt(max(val, 0.0)))


def dense_rows(a, r0, r1):
    if hasattr(a, "rows_f64"):
        return a.rows_f64(r0, r1)
    return np.asarray(a[r0:r1], dtype=np.float64)


def relative_frobenius_error(a, u, s, v, sigma_all):
    """eq. relfroberr: ||A - A_out||_F / ||A - [[A]]_k||_F - 1."""
    k = len(s)
    return approx_frob_error(a, u, s, v) / optimal_tail_frob(sigma_all, k) - 1.0


def relative_spectral_error(a, u, s, v, sigma_all):
    """eq. relspecerr: ||A - A_out||_2 / ||A - [[A]]_k||_2 - 1 (dense; small A)."""
    k = len(s)
    ad = dense(a)
    err = np.linalg.norm(ad - (u * s[None, :]) @ v.T, 2)
    return err / float(np.asarray(sigma_all)[k]) - 1.0


def range_projection_error(a, qc):
    """||A - Q_c Q_c^T A||_2 (dense; small A)."""
    ad = dense(a)
    return float(np.linalg.norm(ad - qc @ (qc.T @ ad), 2))


def corange_projection_error(a, qr_):
    """||A - A Q_r Q_r^T||_2 (dense; small A)."""
    ad = dense(a)
    return float(np.linalg.norm(ad - (ad @ qr_) @ qr_.T, 2))


def expected_error_bound(sigma_all, k, p, exponent):
    """The bound of Thm. 3.1 / Thm. 4.1 with the exponent e that applies
    (e = v - 1 for the basis Alg. 2 returns after v views):
    [(1 + sqrt(k/(p-1))) sigma_{k+1}^e + (e_N sqrt(k+p)/p) (sum_{j>k} sigma_j^{2e})^{1/2}]^{1/e}
    where e_N is Euler's number."""
    sig = np.asarray(sigma_all, dtype=np.float64)
    e = float(exponent)
    tail = sig[k:]
    term1 = (1.0 + np.sqrt(k / (p - 1.0))) * tail[0] ** e
    term2 = np.e * np.sqrt(k + p) / p * np.sqrt(np.sum(tail ** (2 * e)))
    return float((term1 + term2) ** (1.0 / e))


__all__ = ["optimal_tail_frob", "approx_frob_error", "relative_frobenius_error",
           "relative_spectral_error", "range_projection_error", "corange_projection_error",
           "expected_error_bound", "times", "times_t"]
