"""The paper's primitives (Sect. 2), in FP64, by LAPACK through numpy.

* qr(A)      -- thin QR, A = Q R with Q orthonormal (n_r x n_c) and R upper
                triangular (n_c x n_c).  Householder (LAPACK geqrf/orgqr);
                signs fixed so that diag(R) >= 0, which makes the factorization
                unique for full-rank A.
* orth(A)    -- an orthonormal basis of range(A): the Q factor of qr(A).
* tsvd(A, k) -- the SVD of the optimal rank-k approximation [[A]]_k, i.e. the
                k leading singular triplets, singular values descending.
"""

import numpy as np


def qr(a):
    a = np.asarray(a, dtype=np.float64)
    q, r = np.linalg.qr(a, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :], r * d[:, None]


def orth(a):
    return qr(a)[0]


def tsvd(a, k):
    """Return (U_k, sigma_k, V_k) with A ~ U_k diag(sigma_k) V_k^T."""
    u, s, vt = np.linalg.svd(np.asarray(a, dtype=np.float64), full_matrices=False)
    return u[:, :k], s[:k], vt[:k, :].T


def canonical_signs(u, v):
    """Fix the sign of each singular pair (u_i, v_i) jointly so that the entry of
    largest magnitude in u_i is positive (ties go to the lowest index).  The
    factorization U diag(sigma) V^T is unchanged."""
    u = np.array(u, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    for i in range(u.shape[1]):
        idx = int(np.argmax(np.abs(u[:, i])))   # numpy's argmax returns the first maximum
        if u[idx, i] < 0:
            u[:, i] = -u[:, i]
            v[:, i] = -v[:, i]
    return u, v
