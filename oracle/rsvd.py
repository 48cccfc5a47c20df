"""Plain FP64 implementations of the paper's randomized SVD algorithms.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each function follows the steps of the cited algorithm in the paper's order,
with numpy/LAPACK for the primitives (products, qr, svd).  Letters: target
rank k (paper: p), oversampling p (paper: l), sketch width s = k + p
(paper: p + l).  A is an m x n matrix (paper: n_r x n_c).

A may be given as a numpy array of any real dtype or as an object with
``shape`` and ``rows_f64(r0, r1)`` (exact FP64 values of rows r0..r1-1; used
for BF16/FP8 storage and for matrices too large to upcast whole).  Products
with A are taken one block of rows at a time; for A^T Y the block
contributions are summed, which only reorders the sum inside the matmul.

Every result carries U (m x k), S (k, descending), V (n x k) with the joint
sign convention of ``linalg.canonical_signs``, plus the final bases Qc, Qr.
"""

from dataclasses import dataclass, field

import numpy as np

from . import linalg, philox

BLOCK_ROWS = 8192


# --------------------------------------------------------------------------
# access to A
# --------------------------------------------------------------------------

def _shape(a):
    return tuple(a.shape)


def _rows(a, r0, r1):
    if hasattr(a, "rows_f64"):
        return a.rows_f64(r0, r1)
    return np.asarray(a[r0:r1], dtype=np.float64)


def times(a, x):
    """A X (the paper's 'A times a thin matrix'), FP64."""
    m, _ = _shape(a)
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((m, x.shape[1]))
    for r0 in range(0, m, BLOCK_ROWS):
        r1 = min(m, r0 + BLOCK_ROWS)
        out[r0:r1] = _rows(a, r0, r1) @ x
    return out


def times_t(a, y):
    """A^T Y (the paper's 'A^* times a thin matrix'), FP64."""
    m, n = _shape(a)
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros((n, y.shape[1]))
    for r0 in range(0, m, BLOCK_ROWS):
        r1 = min(m, r0 + BLOCK_ROWS)
        out += _rows(a, r0, r1).T @ y[r0:r1]
    return out


def dense(a):
    m, _ = _shape(a)
    return _rows(a, 0, m)


class Transposed:
    """A^T of a stored matrix, for running an algorithm on the transpose."""

    def __init__(self, a):
        self.a = a
        m, n = _shape(a)
        self.shape = (n, m)

    def rows_f64(self, r0, r1):
        m, _ = _shape(self.a)
        return _rows(self.a, 0, m)[:, r0:r1].T


@dataclass
class Result:
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    Qc: np.ndarray = None
    Qr: np.ndarray = None
    approx: str = ""           # "QcQc^T A" or "A QrQr^T": which approximation the basis gives
    extra: dict = field(default_factory=dict)


def _finish(uh_full, lam, vh_full, qc, qr, k, approx, **extra):
    u = qc @ uh_full[:, :k]
    v = qr @ vh_full[:, :k]
    u, v = linalg.canonical_signs(u, v)
    return Result(u, lam[:k].copy(), v, qc, qr, approx, dict(extra))


def _check_sizes(a, k, p):
    m, n = _shape(a)
    if k < 1 or p < 0 or k + p > min(m, n):
        raise ValueError("need k >= 1, p >= 0 and k + p <= min(m, n)")
    return m, n, k + p


# --------------------------------------------------------------------------
# Alg. 1: standard subspace iteration, 2(q+1) views
# --------------------------------------------------------------------------

def alg1_subit(a, k, p, q, seed):
    """Alg. 1 (Sect. 3): QR after every product with A or A^T, q iterations.

    Pinned by: equality with Alg. 2 at v = 2(q+1) (the claim after Alg. 2),
    exact recovery, and the dense-SVD special case.
    """
    m, n, s = _check_sizes(a, k, p)
    omega_r = philox.omega(seed, n, s)                       # Omega_r = randn(n_c, p+l)
    qc, _ = linalg.qr(times(a, omega_r))                     # [Q_c, ~] = qr(A Omega_r)
    for _ in range(q):
        qr_, _ = linalg.qr(times_t(a, qc))                   # [Q_r, ~] = qr(A^* Q_c)
        qc, _ = linalg.qr(times(a, qr_))                     # [Q_c, ~] = qr(A Q_r)
    qr_, rr = linalg.qr(times_t(a, qc))                      # [Q_r, R_r] = qr(A^* Q_c)
    vh, lam, uh_t = np.linalg.svd(rr)                        # R_r = V^ Lam U^^T
    return _finish(uh_t.T, lam, vh, qc, qr_, k, "QcQc^T A")


# --------------------------------------------------------------------------
# Alg. 2 / Alg. 3: generalized subspace iteration, any v >= 2
# --------------------------------------------------------------------------

def alg3_qr_or_qc(a, k, p, v, seed):
    """Alg. 3 (constructQrOrQc): Q_c for odd v, Q_r for even v (v >= 1)."""
    m, n, s = _check_sizes(a, k, p)
    qr_ = philox.omega(seed, n, s)
    qc = None
    for j in range(1, v + 1):
        if j % 2 == 1:
            qc, _ = linalg.qr(times(a, qr_))
        else:
            qr_, _ = linalg.qr(times_t(a, qc))
    return qr_ if v % 2 == 0 else qc


def alg2_gensubit(a, k, p, v, seed):
    """Alg. 2 (Sect. 4): generalized randomized subspace iteration.

    Q_r starts as the Gaussian Omega (n x s), not orthonormalized.  Views
    alternate qr(A Q_r) (odd j) and qr(A^T Q_c) (even j).  For even v the
    approximation is Q_c Q_c^T A and the small SVD is of R_r
    (A^T Q_c = Q_r R_r, so Q_c^T A = R_r^T Q_r^T); for odd v it is A Q_r Q_r^T
    and the small SVD is of R_c (A Q_r = Q_c R_c).

    Pinned by: exact recovery of a rank-r matrix (r <= k), the dense SVD when
    s = min(m, n), a closed-form re-derivation through explicit powers
    (A A^T)^q A Omega on tiny inputs, Alg. 1 at v = 2q+2, the Ritz interlacing
    bound and the expected-error bounds of Thm. 3.1/4.1 averaged over seeds.
    """
    if v < 2:
        raise ValueError("Alg. 2 needs v >= 2 views")
    m, n, s = _check_sizes(a, k, p)
    qr_ = philox.omega(seed, n, s)
    qc = rc = rr = None
    for j in range(1, v + 1):
        if j % 2 == 1:
            qc, rc = linalg.qr(times(a, qr_))
        else:
            qr_, rr = linalg.qr(times_t(a, qc))
    if v % 2 == 0:
        vh, lam, uh_t = np.linalg.svd(rr)                    # tsvd(R_r) = V^ Lam U^^T
        return _finish(uh_t.T, lam, vh, qc, qr_, k, "QcQc^T A")
    uh, lam, vh_t = np.linalg.svd(rc)                        # tsvd(R_c) = U^ Lam V^^T
    return _finish(uh, lam, vh_t.T, qc, qr_, k, "A QrQr^T")


# --------------------------------------------------------------------------
# Alg. 7: one view (Tropp variant with l_c)
# --------------------------------------------------------------------------

def decay_oversampling(k, budget):
    """The moderate-decay oversampling rule (eq. overmed, Sect. 6.3) for a sketch
    budget T = 2k + l1 + l2: l1 = max(2, floor((T-1)/3) - k), l2 = T - 2k - l1."""
    l1 = max(2, (budget - 1) // 3 - k)
    return l1, budget - 2 * k - l1


def flat_oversampling(k, budget):
    """eq. overflat (Sect. 6.3)."""
    t = budget
    frac = (np.sqrt(k * (t - k - 2) * (1 - 2 / (t - 1))) - (k - 1)) / (t - 2 * k - 1)
    l1 = max(2, int(np.floor((t - 1) * frac)) - k)
    return l1, t - 2 * k - l1


def rapid_oversampling(k, budget):
    """eq. overrapid (Sect. 6.3)."""
    l1 = (budget - 2) // 2 - k
    return l1, budget - 2 * k - l1


def alg7_one_view(a, k, p, seed, s_w=None, lc=None):
    """Alg. 7 (Sect. 6.5): the 1-view method, Tropp variant.

    Range sketch Y_c = A Omega_r with s = k+p columns (l1 = p); co-range sketch
    W = Psi A = Y_r^T with Psi = Omega_c^T of s_w rows (default 2s+1, i.e.
    k + l2 rows with l2 = s + p + 1).  The optional orthonormalization of the
    test matrices is not applied (as in the paper's experiments).  With
    l_c = l1 (the default) Q_c is an orthonormal basis of Y_c; with l_c < l1
    it is the k+l_c leading left singular vectors of Y_c.  Then
    [Q^, R^] = qr(Psi Q_c), X = R^^-1 Q^^T W, [U^, Lam, V] = tsvd(X, k) and
    U = Q_c U^.

    Pinned by: exact recovery (X = Q_c^T A when A = Q_c Q_c^T A), and the
    least-squares definition X = (Psi Q_c)^+ W solved by an unrelated library
    routine.
    """
    m, n, s = _check_sizes(a, k, p)
    if s_w is None:
        s_w = 2 * s + 1
    if s_w < s or s_w > m:
        raise ValueError("need s <= s_w <= m")
    l1 = p
    if lc is None:
        lc = l1
    omega_r = philox.omega(seed, n, s)                       # a) Omega_r
    psi = philox.psi(seed, s_w, m)                           # b) Omega_c^T
    yc = times(a, omega_r)                                   # a) Y_c = A Omega_r
    w = times_t(a, psi.T).T                                  # b) Y_r^T = Omega_c^T A
    if lc < l1:
        qc, rc = linalg.qr(yc)
        qhat_c = linalg.tsvd(rc, k + lc)[0]
        qc = qc @ qhat_c
    else:
        qc, _ = linalg.qr(yc)
    qhat, rhat = linalg.qr(psi @ qc)                         # [Q^, R^] = qr(Omega_c^* Q_c)
    x = np.linalg.solve(rhat, qhat.T @ w)                    # X = R^^-1 Q^^* Y_r^*
    uh, lam, vt = np.linalg.svd(x, full_matrices=False)      # tsvd(X, k)
    u = qc @ uh[:, :k]
    u, v = linalg.canonical_signs(u, vt[:k, :].T)
    return Result(u, lam[:k].copy(), v, qc, None, "Qc [[X]]_k", {"X": x, "W": w, "Yc": yc})


def extended_one_view(a, k, p, seed, s_c):
    """Sect. 6.7: the extended 1-view sketch with the improved reconstruction
    (eq. bwzimproved), with Gaussian core test matrices in place of SRFTs.

    The range and co-range sketches have the same width s = k + p (l1 = l2):
    Y_c = A Omega_r and Y_r = A^T Omega_c, with Omega_c^T = Psi (s x m); the
    core sketch is Z = Phi_r^T A Phi_c (s_c x s_c), with Phi_r^T = Phi (s_c x m)
    and Phi_c^T = Phi' (s_c x n), s_c >= s.  Then
    Q_c R_c = Y_c, Q_r R_r = Y_r, U_c T_c = Phi_r^T Q_c, U_r T_r = Phi_c^T Q_r,
    C = T_c^+ U_c^T Z U_r (T_r^T)^+, and A ~ Q_c [[C]]_k Q_r^T, so that
    U = Q_c U^_k, V = Q_r V^_k with [U^, Lam, V^] = tsvd(C, k).

    Pinned by: exact recovery of an exactly rank-k A (every sketch then holds
    the whole range), and the core C = (Phi Q_c)^+ Z (Q_r^T Phi'^T)^+ formed
    with pseudo-inverses from an unrelated library routine.
    """
    m, n, s = _check_sizes(a, k, p)
    if s_c < s or s_c > min(m, n):
        raise ValueError("need s <= s_c <= min(m, n)")
    omega_r = philox.omega(seed, n, s)                       # Omega_r (n x s)
    psi = philox.psi(seed, s, m)                             # Omega_c^T (s x m)
    phi_r = philox.phi(seed, s_c, m, philox.TAG_PHI)         # Phi_r^T (s_c x m)
    phi_c = philox.phi(seed, s_c, n, philox.TAG_PHI2)        # Phi_c^T (s_c x n)
    yc = times(a, omega_r)                                   # Y_c = A Omega_r
    yr = times_t(a, psi.T)                                   # Y_r = A^T Omega_c
    z = phi_r @ times(a, phi_c.T)                            # Z = Phi_r^T A Phi_c
    qc, _ = linalg.qr(yc)
    qr_, _ = linalg.qr(yr)
    uc, tc = linalg.qr(phi_r @ qc)                           # U_c T_c = Phi_r^T Q_c
    ur, tr = linalg.qr(phi_c @ qr_)                          # U_r T_r = Phi_c^T Q_r
    core = np.linalg.solve(tc, uc.T @ z @ ur)                # T_c^+ U_c^T Z U_r
    core = np.linalg.solve(tr, core.T).T                     # ... (T_r^T)^+
    uh, lam, vh = linalg.tsvd(core, k)
    u, v = linalg.canonical_signs(qc @ uh, qr_ @ vh)
    return Result(u, lam.copy(), v, qc, qr_, "Qc [[C]]_k Qr^T", {"C": core, "Z": z})


# --------------------------------------------------------------------------
# Alg. 9: generalized block Krylov, any v >= 2
# --------------------------------------------------------------------------

def alg9_block_krylov(a, k, p, v, seed):
    """Alg. 9 (Sect. 7.2), as printed: the loop runs v-1 views, QR'ing every
    block except the last; the blocks of one parity are stacked into K_c (even
    v) or K_r (odd v), orthonormalized, and one final view forms the small
    matrix whose SVD is taken.

    Pinned by: equality with Alg. 2 for v < 4 (stated after Alg. 9), exact
    recovery, and a closed-form re-derivation through explicit Krylov powers
    on tiny inputs.
    """
    if v < 2:
        raise ValueError("Alg. 9 needs v >= 2 views")
    m, n, s = _check_sizes(a, k, p)
    blocks_c, blocks_r = {}, {0: philox.omega(seed, n, s)}
    for j in range(1, v):
        if j % 2 == 1:
            prod = times(a, blocks_r[j - 1])
            blocks_c[j] = linalg.qr(prod)[0] if j < v - 1 else prod
        else:
            prod = times_t(a, blocks_c[j - 1])
            blocks_r[j] = linalg.qr(prod)[0] if j < v - 1 else prod
    if v % 2 == 0:
        kc = np.hstack([blocks_c[j] for j in range(1, v, 2)])
        qc, _ = linalg.qr(kc)
        qr_, rr = linalg.qr(times_t(a, qc))
        vh, lam, uh_t = np.linalg.svd(rr)
        return _finish(uh_t.T, lam, vh, qc, qr_, k, "QcQc^T A")
    kr = np.hstack([blocks_r[j] for j in range(2, v, 2)])
    qr_, _ = linalg.qr(kr)
    qc, rc = linalg.qr(times(a, qr_))
    uh, lam, vh_t = np.linalg.svd(rc)
    return _finish(uh, lam, vh_t.T, qc, qr_, k, "A QrQr^T")


# --------------------------------------------------------------------------
# Sect. 7.3: block Krylov for matrices read one block of rows at a time
# --------------------------------------------------------------------------

def default_tau(precision):
    """Relative cut for the pseudo-inverse of R_K (the TSVD remedy of Sect. 6.8)."""
    return 2.0 ** -40 if precision == "f64" else 2.0 ** -20


def row_sweep_krylov(a, k, p, v, seed, tau=2.0 ** -40, block_rows=None):
    """Accuracy-enhanced block Krylov for row-wise access (Sect. 7.3 with the
    single-sweep products of Sect. 6.8).  The paper gives prose, not
    pseudocode; this is the reading used throughout the library.

    One sweep over the row blocks A_b of A evaluates both Y = A X
    (Y[b] = A_b X) and Z = A^T Y (Z += A_b^T Y[b]), i.e. A^T A X in a single
    view.  With v sweeps:
      X_0 = orth(Omega); for j = 1..v: Y_j = A X_{j-1}, Z_j = A^T Y_j, and for
      j < v: X_j = orth of Z_j projected twice off span[X_0..X_{j-1}].
    K = [Y_1 .. Y_v] = A [X_0 .. X_{v-1}] spans the range block Krylov space
    of Alg. 9 with 2v views, and [Z_1 .. Z_v] = A^T K.
    [Q_K, R_K] = qr(K), R_K = P S W^T, keep r = #{S_i >= tau S_1};
    Q_c = Q_K P_r and B^T = A^T Q_c = [Z_1..Z_v] W_r S_r^-1 (no extra view).
    [Q_r, R_r] = qr(B^T), R_r = V^ Lam U^^T, U = Q_c U^_k, V = Q_r V^_k.

    Pinned by: v = 1 equals Alg. 2 with two views (Sect. 6.8), v sweeps equal
    Alg. 9 with 2v views on well-conditioned inputs, exact recovery, the
    interlacing bound, and independence of the row-block size.
    """
    m, n, s = _check_sizes(a, k, p)
    if v < 1:
        raise ValueError("the row sweep needs v >= 1 sweeps")
    if v * s > min(m, n):
        raise ValueError("need v * (k + p) <= min(m, n)")
    rows = block_rows or m
    xs = [linalg.orth(philox.omega(seed, n, s))]
    ys, zs = [], []
    for j in range(1, v + 1):
        x = xs[-1]
        y = np.empty((m, s))
        z = np.zeros((n, s))
        for r0 in range(0, m, rows):                        # one sweep over row blocks
            r1 = min(m, r0 + rows)
            ab = _rows(a, r0, r1)
            y[r0:r1] = ab @ x
            z += ab.T @ y[r0:r1]
        ys.append(y)
        zs.append(z)
        if j < v:
            basis = np.hstack(xs)
            w = z - basis @ (basis.T @ z)
            w = w - basis @ (basis.T @ w)
            xs.append(linalg.orth(w))
    kmat = np.hstack(ys)
    zmat = np.hstack(zs)
    qk, rk = linalg.qr(kmat)
    pmat, sv, wt = np.linalg.svd(rk)
    r = int(np.count_nonzero(sv >= tau * sv[0])) if sv[0] > 0 else 0
    qc = qk @ pmat[:, :r]
    bt = (zmat @ wt[:r, :].T) / sv[:r][None, :]
    qr_, rr = linalg.qr(bt)
    vh, lam, uh_t = np.linalg.svd(rr)
    if r < k:
        raise ValueError("numerical rank of the Krylov basis fell below k")
    return _finish(uh_t.T, lam, vh, qc, qr_, k, "QcQc^T A", r=r)


def col_sweep_krylov(a, k, p, v, seed, tau=2.0 ** -40):
    """The same procedure on A^T (column-wise access, end of Sect. 6.8):
    U and V trade places."""
    res = row_sweep_krylov(Transposed(a), k, p, v, seed, tau)
    u, v_ = linalg.canonical_signs(res.V, res.U)
    return Result(u, res.S, v_, res.Qr, res.Qc, "A QrQr^T", res.extra)
