"""One-view sketches of a matrix presented as a stream of linear updates
(Sect. 6.1, eq. streammat and eq. streammatmult).

TEST INFRASTRUCTURE ONLY (see the package header).

A = sum_i H_i is never formed: each innovation H_i updates the range sketch
Y = A Omega_r (m x s) and the co-range sketch W = Psi A (s_w x n) by
Y += H_i Omega_r and W += Psi H_i, and is then discarded.  An update is either
a dense block (H_i zero outside rows r0.., columns c0..) or a list of
(row, column, value) entries, the "sparse matrix containing a few elements of
A" of Sect. 6.1; repeated coordinates add up.

After the stream, the sketches feed the one-view post-processing of Alg. 7 or
Alg. 8 exactly as the one-read sketches would (``finish``).

Pinned by: linearity against the sketches of the summed matrix (eq.
streammatmult) and, after ``finish``, equality with ``rsvd.alg7_one_view`` /
``rsvd.alg8_woolfe`` on the summed matrix.
"""

import numpy as np

from . import linalg, philox, rsvd


class Sketch:
    def __init__(self, m, n, k, p, seed, s_w=None):
        s = k + p
        if k < 1 or p < 0 or s > min(m, n):
            raise ValueError("need k >= 1, p >= 0 and k + p <= min(m, n)")
        self.m, self.n, self.k, self.p, self.s = m, n, k, p, s
        self.s_w = 2 * s + 1 if s_w is None else s_w
        self.seed = seed
        self.omega = philox.omega(seed, n, s)                  # Omega_r (n x s)
        self.psi = philox.psi(seed, self.s_w, m)               # Psi = Omega_c^T (s_w x m)
        self.y = np.zeros((m, s))
        self.w = np.zeros((self.s_w, n))

    def add_dense(self, r0, c0, block):
        """H_i = block placed at rows r0.., columns c0..: Y[rows] += H Omega[cols],
        W[:, cols] += Psi[:, rows] H."""
        h = np.asarray(block, dtype=np.float64)
        r1, c1 = r0 + h.shape[0], c0 + h.shape[1]
        if r0 < 0 or c0 < 0 or r1 > self.m or c1 > self.n:
            raise ValueError("block outside A")
        self.y[r0:r1] += h @ self.omega[c0:c1]
        self.w[:, c0:c1] += self.psi[:, r0:r1] @ h

    def add_entries(self, rows, cols, vals):
        """H_i = sum_e vals[e] e_{rows[e]} e_{cols[e]}^T: Y[r] += v Omega[c],
        W[:, c] += v Psi[:, r] for every entry, one entry at a time."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        vals = np.asarray(vals, dtype=np.float64)
        if rows.size and (rows.min() < 0 or rows.max() >= self.m or cols.min() < 0 or cols.max() >= self.n):
            raise ValueError("entry outside A")
        for r, c, v in zip(rows, cols, vals):
            self.y[r] += v * self.omega[c]
            self.w[:, c] += v * self.psi[:, r]

    def finish(self, method="tropp", lc=None):
        """Alg. 7 (method="tropp") or Alg. 8 (method="woolfe") on the streamed
        sketches; lc as in ``rsvd.alg7_one_view``."""
        k, s = self.k, self.s
        spectra = lambda: _spectra(self.y, self.w, self.psi, k)   # noqa: E731
        lc = rsvd._one_view_lc(k, s, self.s_w, lc, spectra)
        qc = rsvd.leading_basis(self.y, k + lc)
        qhat, rhat = linalg.qr(self.psi @ qc)
        if method == "tropp":
            x = np.linalg.solve(rhat, qhat.T @ self.w)
            uh, lam, vt = np.linalg.svd(x, full_matrices=False)
            u, v = linalg.canonical_signs(qc @ uh[:, :k], vt[:k, :].T)
            return rsvd.Result(u, lam[:k].copy(), v, qc, None, "Qc [[X]]_k", {"lc": lc})
        if method != "woolfe":
            raise ValueError("method must be 'tropp' or 'woolfe'")
        qr_ = rsvd.leading_basis(self.w.T, k + lc)
        xh = np.linalg.solve(rhat, qhat.T @ (self.w @ qr_))
        uh, lam, vh = linalg.tsvd(xh, k)
        u, v = linalg.canonical_signs(qc @ uh, qr_ @ vh)
        return rsvd.Result(u, lam.copy(), v, qc, qr_, "Qc [[X^]]_k Qr^T", {"lc": lc})


def _spectra(y, w, psi, k):
    s = y.shape[1]
    out = []
    for lc in range(0, s - k + 1):
        qc = rsvd.leading_basis(y, k + lc)
        qhat, rhat = linalg.qr(psi @ qc)
        x = np.linalg.solve(rhat, qhat.T @ w)
        out.append(np.linalg.svd(x, compute_uv=False)[:k])
    return out
