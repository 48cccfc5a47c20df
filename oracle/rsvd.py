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

from . import linalg, philox, srft

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
# Sect. 4: views that alternate between A and A^T (Alg. 2 and Alg. 3)
# --------------------------------------------------------------------------

def alternating_views(a, start, views):
    """The sequence of views behind Alg. 2 and Alg. 3 (Sect. 4).

    ``start`` is an n x s block on the co-range side (Omega for the methods
    here).  A view applies A to the newest co-range block or A^T to the
    newest range block, whichever side the previous view did not produce,
    and orthonormalizes the product.  After j views the newest block spans
    range((A A^T)^((j-1)/2) A Omega) (odd j: a range basis Q_c, A Q_r = Q_c R)
    or range((A^T A)^(j/2) Omega) (even j: a co-range basis Q_r,
    A^T Q_c = Q_r R): the Krylov-type subspaces of Sect. 4.1.

    Yields (j, Q_c, Q_r, R) after every view j = 1..views, where Q_c and Q_r
    are the newest bases on each side (Q_r is ``start`` until the second
    view) and R is the triangular factor of view j.
    """
    q_c, q_r = None, start
    for j in range(1, views + 1):
        if j % 2 == 1:
            q_c, r = linalg.qr(times(a, q_r))
        else:
            q_r, r = linalg.qr(times_t(a, q_c))
        yield j, q_c, q_r, r


def _subspace_result(q_c, q_r, r, views, k):
    """The small SVD that closes Alg. 2 after ``views`` views.

    Even v: the approximation is Q_c Q_c^T A, and A^T Q_c = Q_r R_r gives
    Q_c^T A = R_r^T Q_r^T, so the SVD R_r = V^ Lam U^^T yields U = Q_c U^ and
    V = Q_r V^.  Odd v: the approximation is A Q_r Q_r^T = Q_c R_c Q_r^T and
    R_c = U^ Lam V^^T.
    """
    if views % 2 == 0:
        vh, lam, uh_t = np.linalg.svd(r)
        return _finish(uh_t.T, lam, vh, q_c, q_r, k, "QcQc^T A")
    uh, lam, vh_t = np.linalg.svd(r)
    return _finish(uh, lam, vh_t.T, q_c, q_r, k, "A QrQr^T")


def alg3_qr_or_qc(a, k, p, v, seed):
    """Alg. 3 (Sect. 4.2): the newest basis after v >= 1 alternating views of
    A started from Omega: a range basis Q_c (m x s) for odd v, a co-range basis
    Q_r (n x s) for even v.

    Pinned by: its span against explicit powers (A A^T)^q A Omega /
    (A^T A)^q Omega on tiny inputs, and by being the basis Alg. 2 ends with.
    """
    if v < 1:
        raise ValueError("Alg. 3 needs v >= 1 views")
    m, n, s = _check_sizes(a, k, p)
    last = None
    for _, q_c, q_r, _ in alternating_views(a, philox.omega(seed, n, s), v):
        last = q_c if v % 2 == 1 else q_r
    return last


def alg2_gensubit(a, k, p, v, seed):
    """Alg. 2 (Sect. 4): generalized randomized subspace iteration.

    Q_r starts as the Gaussian Omega (n x s), not orthonormalized; v views
    alternate as in ``alternating_views``; the small SVD of the last
    triangular factor gives the SVD of Q_c Q_c^T A (even v) or A Q_r Q_r^T
    (odd v).

    Pinned by: exact recovery of a rank-r matrix (r <= k), the dense SVD when
    s = min(m, n), a closed-form re-derivation through explicit powers
    (A A^T)^q A Omega on tiny inputs, Alg. 1 at v = 2q+2, the Ritz interlacing
    bound and the expected-error bounds of Thm. 3.1/4.1 averaged over seeds.
    """
    if v < 2:
        raise ValueError("Alg. 2 needs v >= 2 views")
    return alg2_every_view_count(a, k, p, v, seed)[v]


def alg2_every_view_count(a, k, p, vmax, seed):
    """Alg. 2 for every view budget v = 2..vmax at once: the first v views of a
    budget-vmax run are exactly the views of a budget-v run, so one sequence
    of views serves all budgets.  Returns {v: Result}."""
    if vmax < 2:
        raise ValueError("Alg. 2 needs v >= 2 views")
    m, n, s = _check_sizes(a, k, p)
    out = {}
    for j, q_c, q_r, r in alternating_views(a, philox.omega(seed, n, s), vmax):
        if j >= 2:
            out[j] = _subspace_result(q_c, q_r, r, j, k)
    return out


# --------------------------------------------------------------------------
# Sect. 6.3 and 6.6: oversampling rules of the one-view methods
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


def fixed_ratio_lc(l1, alpha):
    """eq. lcutfixedratio (Sect. 6.6.1): l_c = floor(alpha l1), 0 <= alpha <= 1."""
    if not 0.0 <= alpha <= 1.0:
        raise ValueError("need 0 <= alpha <= 1")
    return int(np.floor(alpha * l1))


def min_variance_lc(spectra):
    """eq. MinVar (Sect. 6.6.2).

    ``spectra[c]`` holds the k leading singular values lambda_1..lambda_k of
    X(l_c = c) for c = 0..l1 (l1 + 1 arrays).  For 0 < c < l1 the vector s(c)
    stacks lambda(c-1)/lambda(c), lambda(c)/lambda(c) and
    lambda(c+1)/lambda(c) (elementwise, 3k entries); for c = 0 it stacks the
    last two (2k entries).  Returns argmin over 0 <= c < l1 of Var[s(c)],
    the population variance (mean squared deviation from the mean); ties go
    to the smallest c.  With l1 = 0 there is no choice and 0 is returned.
    """
    lam = [np.asarray(x, dtype=np.float64) for x in spectra]
    l1 = len(lam) - 1
    if l1 <= 0:
        return 0
    best, best_var = 0, None
    for c in range(l1):
        parts = [lam[c] / lam[c], lam[c + 1] / lam[c]]
        if c > 0:
            parts.insert(0, lam[c - 1] / lam[c])
        var = float(np.var(np.concatenate(parts)))
        if best_var is None or var < best_var:
            best, best_var = c, var
    return best


# --------------------------------------------------------------------------
# Sect. 6: one-view methods (Alg. 7, Alg. 8)
# --------------------------------------------------------------------------

def one_view_sketches(a, s, s_w, seed):
    """Steps 1 and 3 of Alg. 7 / Alg. 8 (the optional orthonormalization of the
    test matrices is not applied, as in the paper's experiments):
    Omega_r (n x s), Psi = Omega_c^T (s_w x m), the range sketch
    Y_c = A Omega_r (m x s) and the co-range sketch W = Psi A = Y_r^T (s_w x n),
    both from one read of A (eq. streammatmult with a single term)."""
    m, n = _shape(a)
    omega_r = philox.omega(seed, n, s)
    psi = philox.psi(seed, s_w, m)
    return omega_r, psi, times(a, omega_r), times_t(a, psi.T).T


def leading_basis(y, width):
    """Sect. 6.5: an orthonormal basis of the sketch y (width = its column
    count), or its ``width`` leading left singular vectors, taken as the QR
    factor times the leading left singular vectors of the triangular factor
    (Alg. 7 and Alg. 8, the l_c < l1 branch)."""
    q, r = linalg.qr(y)
    if width >= y.shape[1]:
        return q
    return q @ linalg.tsvd(r, width)[0]


def _one_view_lc(k, s, s_w, lc, spectra_fn):
    """The l_c a one-view call uses: l1 (the default), an integer, ('ratio', alpha)
    for eq. lcutfixedratio, or 'minvar' for eq. MinVar."""
    l1 = s - k
    if lc is None:
        return l1
    if isinstance(lc, str) and lc == "minvar":
        return min_variance_lc(spectra_fn())
    if isinstance(lc, tuple) and lc[0] == "ratio":
        return fixed_ratio_lc(l1, lc[1])
    lc = int(lc)
    if not 0 <= lc <= l1:
        raise ValueError("need 0 <= l_c <= l1")
    return lc


def one_view_spectra(a, k, p, seed, s_w=None):
    """lambda(l_c) for l_c = 0..l1: the k leading singular values of
    X(l_c) = (Psi Q_c)^+ W of Alg. 7, with Q_c the k + l_c leading left
    singular vectors of Y_c, each formed as the algorithm forms it."""
    m, n, s = _check_sizes(a, k, p)
    s_w = 2 * s + 1 if s_w is None else s_w
    _, psi, yc, w = one_view_sketches(a, s, s_w, seed)
    out = []
    for lc in range(0, s - k + 1):
        qc = leading_basis(yc, k + lc)
        qhat, rhat = linalg.qr(psi @ qc)
        x = np.linalg.solve(rhat, qhat.T @ w)
        out.append(np.linalg.svd(x, compute_uv=False)[:k])
    return out


def alg7_one_view(a, k, p, seed, s_w=None, lc=None):
    """Alg. 7 (Sect. 6.5): the 1-view method, Tropp variant.

    Range sketch Y_c = A Omega_r with s = k+p columns (l1 = p); co-range sketch
    W = Psi A = Y_r^T with Psi = Omega_c^T of s_w rows (default 2s+1, i.e.
    k + l2 rows with l2 = s + p + 1).  Q_c is an orthonormal basis of Y_c
    (l_c = l1, the default) or its k + l_c leading left singular vectors
    (l_c < l1); lc may be an integer, ('ratio', alpha) (eq. lcutfixedratio) or
    'minvar' (eq. MinVar).  Then [Q^, R^] = qr(Psi Q_c), X = R^^-1 Q^^T W,
    [U^, Lam, V] = tsvd(X, k) and U = Q_c U^.

    Pinned by: exact recovery (X = Q_c^T A when A = Q_c Q_c^T A), the
    least-squares definition X = (Psi Q_c)^+ W solved by an unrelated library
    routine, and (l_c < l1) the leading-subspace form of Q_c checked against
    LAPACK's SVD of Y_c.
    """
    m, n, s = _check_sizes(a, k, p)
    s_w = 2 * s + 1 if s_w is None else s_w
    if s_w < s or s_w > m:
        raise ValueError("need s <= s_w <= m")
    lc = _one_view_lc(k, s, s_w, lc, lambda: one_view_spectra(a, k, p, seed, s_w))
    _, psi, yc, w = one_view_sketches(a, s, s_w, seed)
    qc = leading_basis(yc, k + lc)
    qhat, rhat = linalg.qr(psi @ qc)                         # [Q^, R^] = qr(Omega_c^* Q_c)
    x = np.linalg.solve(rhat, qhat.T @ w)                    # X = R^^-1 Q^^* Y_r^*
    uh, lam, vt = np.linalg.svd(x, full_matrices=False)      # tsvd(X, k)
    u = qc @ uh[:, :k]
    u, v = linalg.canonical_signs(u, vt[:k, :].T)
    return Result(u, lam[:k].copy(), v, qc, None, "Qc [[X]]_k",
                  {"X": x, "W": w, "Yc": yc, "lc": lc})


def alg8_woolfe(a, k, p, seed, s_w=None, lc=None):
    """Alg. 8 (Sect. 6.5): the 1-view method, Woolfe variant.

    The same sketches as Alg. 7; Q_c holds the k + l_c leading left singular
    vectors of Y_c and Q_r those of Y_r = W^T; X^ solves the least-squares
    problem (Psi Q_c) X^ = Y_r^T Q_r (eq. lstsqWoolfe); [U^, Lam, V^] =
    tsvd(X^, k), U = Q_c U^ and V = Q_r V^, so A ~ Q_c [[X^]]_k Q_r^T.
    lc as for ``alg7_one_view``.

    Pinned by: exact recovery, X^ checked against LAPACK's least-squares
    driver, and equality with Alg. 7 when l_c = l1 = l2 (Q_r then spans the
    whole row space of W, so X = X^ Q_r^T).
    """
    m, n, s = _check_sizes(a, k, p)
    s_w = 2 * s + 1 if s_w is None else s_w
    if s_w < s or s_w > min(m, n):
        raise ValueError("need s <= s_w <= min(m, n)")
    lc = _one_view_lc(k, s, s_w, lc, lambda: one_view_spectra(a, k, p, seed, s_w))
    _, psi, yc, w = one_view_sketches(a, s, s_w, seed)
    qc = leading_basis(yc, k + lc)
    qr_ = leading_basis(w.T, k + lc)
    qhat, rhat = linalg.qr(psi @ qc)
    xh = np.linalg.solve(rhat, qhat.T @ (w @ qr_))           # (Omega_c^* Q_c) X^ = Y_r^* Q_r
    uh, lam, vh = linalg.tsvd(xh, k)
    u, v = linalg.canonical_signs(qc @ uh, qr_ @ vh)
    return Result(u, lam.copy(), v, qc, qr_, "Qc [[X^]]_k Qr^T",
                  {"X": xh, "W": w, "Yc": yc, "lc": lc})


# --------------------------------------------------------------------------
# Sect. 6.7: the extended one-view sketch
# --------------------------------------------------------------------------

def extended_sizes(k, budget, m, n):
    """The sizing of the extended sketch the paper found best (Sect. 6.7):
    l1 = l2 = floor(0.8 floor(T/2 - k)) (eq. bwzafac8, rounded down to an
    integer), and s_c the largest core size with
    (2k + l1 + l2 + 1)(m + n) + s_c (s_c + 2) <= T (m + n), capped at
    min(m, n).  Returns (l1, s_c); ValueError when s_c < k + l1."""
    l1 = int(np.floor(0.8 * np.floor(budget / 2.0 - k)))
    room = (budget - 2 * k - 2 * l1 - 1) * (m + n)
    sc = int(np.floor(np.sqrt(1.0 + room))) - 1 if room >= 0 else -1
    while sc >= 0 and sc * (sc + 2) > room:
        sc -= 1
    while (sc + 1) * (sc + 3) <= room:
        sc += 1
    sc = min(sc, m, n)
    if l1 < 0 or sc < k + l1:
        raise ValueError("budget too small for the extended sketch")
    return l1, sc


def extended_one_view(a, k, p, seed, s_c, core="gaussian"):
    """Sect. 6.7: the extended 1-view sketch with the improved reconstruction
    (eq. bwzimproved).

    The range and co-range sketches have the same width s = k + p (l1 = l2):
    Y_c = A Omega_r and Y_r = A^T Omega_c, with Omega_c^T = Psi (s x m); the
    core sketch is Z = Phi_r^T A Phi_c (s_c x s_c) with core test matrices
    Phi_r (m x s_c) and Phi_c (n x s_c), s_c >= s: Gaussian (core="gaussian")
    or the paper's SRFTs D F P with a DCT (core="srft", see ``srft``).  Then
    Q_c R_c = Y_c, Q_r R_r = Y_r, U_c T_c = Phi_r^T Q_c, U_r T_r = Phi_c^T Q_r,
    C = T_c^+ U_c^T Z U_r (T_r^T)^+, and A ~ Q_c [[C]]_k Q_r^T, so that
    U = Q_c U^_k, V = Q_r V^_k with [U^, Lam, V^] = tsvd(C, k).

    Pinned by: exact recovery of an exactly rank-k A (every sketch then holds
    the whole range), and the core C = (Phi_r^T Q_c)^+ Z (Q_r^T Phi_c)^+
    formed with pseudo-inverses from an unrelated library routine; for SRFT
    cores Z is checked against a two-dimensional DCT from scipy.
    """
    m, n, s = _check_sizes(a, k, p)
    if s_c < s or s_c > min(m, n):
        raise ValueError("need s <= s_c <= min(m, n)")
    omega_r = philox.omega(seed, n, s)                       # Omega_r (n x s)
    psi = philox.psi(seed, s, m)                             # Omega_c^T (s x m)
    if core == "gaussian":
        phi_r = philox.phi(seed, s_c, m, philox.TAG_PHI)     # Phi_r^T (s_c x m)
        phi_c = philox.phi(seed, s_c, n, philox.TAG_PHI2)    # Phi_c^T (s_c x n)
    elif core == "srft":
        phi_r = srft.matrix(seed, m, s_c, srft.ROWS).T
        phi_c = srft.matrix(seed, n, s_c, srft.COLS).T
    else:
        raise ValueError("core must be 'gaussian' or 'srft'")
    yc = times(a, omega_r)                                   # Y_c = A Omega_r
    yr = times_t(a, psi.T)                                   # Y_r = A^T Omega_c
    z = phi_r @ times(a, phi_c.T)                            # Z = Phi_r^T A Phi_c
    qc, _ = linalg.qr(yc)
    qr_, _ = linalg.qr(yr)
    uc, tc = linalg.qr(phi_r @ qc)                           # U_c T_c = Phi_r^T Q_c
    ur, tr = linalg.qr(phi_c @ qr_)                          # U_r T_r = Phi_c^T Q_r
    core_m = np.linalg.solve(tc, uc.T @ z @ ur)              # T_c^+ U_c^T Z U_r
    core_m = np.linalg.solve(tr, core_m.T).T                 # ... (T_r^T)^+
    uh, lam, vh = linalg.tsvd(core_m, k)
    u, v = linalg.canonical_signs(qc @ uh, qr_ @ vh)
    return Result(u, lam.copy(), v, qc, qr_, "Qc [[C]]_k Qr^T", {"C": core_m, "Z": z})


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
