"""Pins of the oracle's one-view post-processing (Sect. 6.5-6.6: l_c, Alg. 8),
the normal-matrix methods (Sect. 4.2: Alg. 3, 4, 5), the streamed sketches
(Sect. 6.1) and the SRFT core sketch (Sect. 6.7), against hand-computed
values, unrelated library routines and the equivalences the paper states."""

import numpy as np
import pytest
import scipy.fft

import synth
from oracle import linalg, normal, philox, rsvd, srft, stream

SEED = synth.METHOD_SEED


def _decaying(m, n, power=1.0, seed=5):
    sigma = np.arange(1, min(m, n) + 1, dtype=np.float64) ** -power
    return synth.spectral_matrix(m, n, sigma, seed), sigma


def _rank_r(m, n, r, seed=3):
    sigma = np.arange(1, r + 1, dtype=np.float64) ** -2.0
    return synth.spectral_matrix(m, n, sigma, seed), sigma


def _span_dist(q1, q2):
    """max |sin| of the principal angles between two orthonormal bases."""
    return float(np.linalg.norm(q1 - q2 @ (q2.T @ q1), 2))


# ---------------------------------------------------------------- oversampling rules

def test_flat_oversampling_hand_values():
    # eq. overflat worked by hand: T = 50, k = 10: sqrt(10 * 38 * 47/49) = 19.092,
    # (19.092 - 9) / 29 = 0.3480, floor(49 * 0.3480) = 17, l1 = 17 - 10 = 7, l2 = 23;
    # T = 100, k = 20: (39.096 - 19) / 59 = 0.3406, floor(99 * 0.3406) = 33 -> (13, 47);
    # T = 30, k = 5: (10.347 - 4) / 19 = 0.3341, floor(29 * 0.3341) = 9 -> (4, 16).
    assert rsvd.flat_oversampling(10, 50) == (7, 23)
    assert rsvd.flat_oversampling(20, 100) == (13, 47)
    assert rsvd.flat_oversampling(5, 30) == (4, 16)


def test_fixed_ratio_lc_hand_values():
    # eq. lcutfixedratio: floor(alpha l1)
    assert rsvd.fixed_ratio_lc(20, 0.5) == 10
    assert rsvd.fixed_ratio_lc(20, 0.33) == 6
    assert rsvd.fixed_ratio_lc(21, 0.5) == 10
    assert rsvd.fixed_ratio_lc(7, 1.0) == 7
    assert rsvd.fixed_ratio_lc(7, 0.0) == 0
    with pytest.raises(ValueError):
        rsvd.fixed_ratio_lc(7, 1.5)


def test_extended_sizes_hand_values():
    # eq. bwzafac8: k = 10, T = 100, m = n = 1000: l1 = floor(0.8 * 40) = 32;
    # (100 - 20 - 64 - 1) * 2000 = 30000 >= s (s + 2): 172 * 174 = 29928, 173 * 175 = 30275.
    assert rsvd.extended_sizes(10, 100, 1000, 1000) == (32, 172)
    # k = 5, T = 40, 500 x 300: l1 = 12; 5 * 800 = 4000: 62 * 64 = 3968, 63 * 65 = 4095.
    assert rsvd.extended_sizes(5, 40, 500, 300) == (12, 62)
    assert rsvd.extended_sizes(5, 41, 500, 300)[0] == 12      # floor(20.5 - 5) = 15


# ---------------------------------------------------------------- eq. MinVar by hand

def test_min_variance_hand_example():
    # k = 2, l1 = 3.  s(0) = [1, 1, 2, 2]: var 0.25.  s(1) = [.5, .5, 1, 1, 1, 1]:
    # mean 5/6, var 1/18.  s(2) = [1, 1, 1, 1, 2, 2]: mean 4/3, var 2/9.  -> 1.
    lam = [np.array([1.0, 1.0]), np.array([2.0, 2.0]), np.array([2.0, 2.0]), np.array([4.0, 4.0])]
    assert rsvd.min_variance_lc(lam) == 1


def test_min_variance_uses_the_stated_ratios():
    # lambda(0) = 4, lambda(1) = lambda(2) = 1 (k = 2, l1 = 2).  s(0) = [1, 1, .25, .25]:
    # var 0.140625; s(1) = [4, 4, 1, 1, 1, 1]: var 2 -> 0.  Inverting the first ratio
    # (lambda(c)/lambda(c-1)) would give s(1) var 0.125 and pick 1.
    lam = [np.array([4.0, 4.0]), np.array([1.0, 1.0]), np.array([1.0, 1.0])]
    assert rsvd.min_variance_lc(lam) == 0
    # elementwise ratios: lambda(0) = [1, 2], lambda(1) = lambda(2) = [1, 1]:
    # s(0) = [1, 1, 1, .5]: var 0.046875; s(1) = [1, 2, 1, 1, 1, 1]: var 0.1389 -> 0
    lam = [np.array([1.0, 2.0]), np.array([1.0, 1.0]), np.array([1.0, 1.0])]
    assert rsvd.min_variance_lc(lam) == 0
    # all spectra equal: every variance is 0, the tie goes to the smallest l_c
    lam = [np.array([3.0, 1.0])] * 5
    assert rsvd.min_variance_lc(lam) == 0
    assert rsvd.min_variance_lc([np.array([1.0])]) == 0


# ---------------------------------------------------------------- Alg. 3

@pytest.mark.parametrize("v", [1, 2, 3, 4, 5])
def test_alg3_spans_the_explicit_powers(v):
    # Alg. 3 returns range((A A^T)^((v-1)/2) A Omega) (odd v) or
    # range((A^T A)^(v/2) Omega) (even v), formed here by explicit powers and an SVD basis.
    m, n, k, p = 70, 50, 5, 3
    a, _ = _decaying(m, n, 0.8, seed=61)
    om = philox.omega(SEED, n, k + p)
    x = om
    for j in range(1, v + 1):
        x = a @ x if j % 2 else a.T @ x
    ref = np.linalg.svd(x, full_matrices=False)[0]
    q = rsvd.alg3_qr_or_qc(a, k, p, v, SEED)
    assert q.shape == ((m, k + p) if v % 2 else (n, k + p))
    np.testing.assert_allclose(q.T @ q, np.eye(k + p), atol=1e-13)
    assert _span_dist(q, ref) < 1e-8
    if v >= 2:
        res = rsvd.alg2_gensubit(a, k, p, v, SEED)
        np.testing.assert_allclose(q, res.Qc if v % 2 else res.Qr, atol=1e-14)


def test_alg2_every_view_count_equals_single_budgets():
    a, _ = _decaying(120, 90, 1.0, seed=63)
    allv = rsvd.alg2_every_view_count(a, 8, 4, 5, SEED)
    for v in (2, 3, 4, 5):
        r = rsvd.alg2_gensubit(a, 8, 4, v, SEED)
        np.testing.assert_array_equal(allv[v].S, r.S)
        np.testing.assert_array_equal(allv[v].U, r.U)


# ---------------------------------------------------------------- Alg. 7 with l_c, Alg. 8

def test_leading_basis_is_lapack_leading_subspace():
    # Sect. 6.5: Q_c = the k + l_c leading left singular vectors of Y_c, checked
    # against LAPACK's SVD of Y_c itself.
    rng = np.random.default_rng(3)
    y = rng.standard_normal((200, 12)) * (0.5 ** np.arange(12))[None, :]
    for w in (3, 7, 12):
        q = rsvd.leading_basis(y, w)
        u = np.linalg.svd(y, full_matrices=False)[0][:, :w]
        np.testing.assert_allclose(q @ q.T, u @ u.T, atol=1e-12)


LC_CHOICES = [0, 2, "minvar", ("ratio", 0.5), None]


@pytest.mark.parametrize("lc", LC_CHOICES, ids=str)
@pytest.mark.parametrize("alg", ["alg7", "alg8"])
def test_one_view_exact_recovery_any_lc(alg, lc):
    m, n, k, p = 300, 200, 10, 6
    a, _ = _rank_r(m, n, k)
    fn = rsvd.alg7_one_view if alg == "alg7" else rsvd.alg8_woolfe
    res = fn(a, k, p, SEED, lc=lc)
    recon = (res.U * res.S[None, :]) @ res.V.T
    assert np.linalg.norm(a - recon) <= 1e3 * np.finfo(float).eps * np.linalg.norm(a)
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    np.testing.assert_allclose(res.S, s[:k], rtol=1e-11)


def test_alg8_solves_the_stated_least_squares_problem():
    # eq. lstsqWoolfe solved by LAPACK's least-squares driver
    m, n, k, p = 160, 120, 6, 6
    a, _ = _decaying(m, n, 1.0, seed=67)
    res = rsvd.alg8_woolfe(a, k, p, SEED, lc=3)
    s_w = 2 * (k + p) + 1
    psi = philox.psi(SEED, s_w, m)
    qc, qr_ = res.Qc, res.Qr
    assert qc.shape[1] == k + 3 and qr_.shape[1] == k + 3
    xh = np.linalg.lstsq(psi @ qc, (psi @ a) @ qr_, rcond=None)[0]
    np.testing.assert_allclose(res.extra["X"], xh, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(res.S, np.linalg.svd(xh, compute_uv=False)[:k], rtol=1e-10)
    # Q_r: the leading left singular vectors of Y_r = (Psi A)^T
    ur = np.linalg.svd((psi @ a).T, full_matrices=False)[0][:, :k + 3]
    np.testing.assert_allclose(qr_ @ qr_.T, ur @ ur.T, atol=1e-10)


def test_alg8_equals_alg7_when_l2_equals_l1():
    # With l_c = l1 = l2, Q_r spans the whole row space of W and X = X^ Q_r^T.
    m, n, k, p = 150, 110, 6, 5
    a, _ = _decaying(m, n, 1.0, seed=71)
    s = k + p
    r7 = rsvd.alg7_one_view(a, k, p, SEED, s_w=s)
    r8 = rsvd.alg8_woolfe(a, k, p, SEED, s_w=s)
    np.testing.assert_allclose(r8.S, r7.S, rtol=1e-9)
    np.testing.assert_allclose(np.abs(np.sum(r8.U * r7.U, axis=0)), 1.0, atol=1e-8)
    np.testing.assert_allclose(np.abs(np.sum(r8.V * r7.V, axis=0)), 1.0, atol=1e-8)


def test_trial_spectra_through_the_co_range_factor():
    # The GPU forms lambda(l_c) as the singular values of R^^-1 Q^^T R_W^T, with
    # W^T = Q_W R_W, since X = R^^-1 Q^^T W = (R^^-1 Q^^T R_W^T) Q_W^T and Q_W^T
    # has orthonormal rows: the identity is checked here against the definition.
    m, n, k, p = 140, 100, 5, 6
    a, _ = _decaying(m, n, 1.2, seed=73)
    spectra = rsvd.one_view_spectra(a, k, p, SEED)
    s, s_w = k + p, 2 * (k + p) + 1
    _, psi, yc, w = rsvd.one_view_sketches(a, s, s_w, SEED)
    _, rw = linalg.qr(w.T)
    for lc in range(p + 1):
        qc = rsvd.leading_basis(yc, k + lc)
        qh, rh = linalg.qr(psi @ qc)
        lam = np.linalg.svd(np.linalg.solve(rh, qh.T @ rw.T), compute_uv=False)[:k]
        np.testing.assert_allclose(lam, spectra[lc], rtol=1e-10)


def test_min_variance_choice_runs_the_chosen_lc():
    m, n, k, p = 200, 150, 6, 8
    a, _ = _decaying(m, n, 1.5, seed=79)
    spectra = rsvd.one_view_spectra(a, k, p, SEED)
    lc = rsvd.min_variance_lc(spectra)
    res = rsvd.alg7_one_view(a, k, p, SEED, lc="minvar")
    assert res.extra["lc"] == lc and 0 <= lc < p
    fixed = rsvd.alg7_one_view(a, k, p, SEED, lc=lc)
    np.testing.assert_array_equal(res.S, fixed.S)
    np.testing.assert_allclose(res.S, spectra[lc], rtol=1e-12)


# ---------------------------------------------------------------- Sect. 4.2: J^T J

def _evd(j, k):
    evals, evecs = np.linalg.eigh(j.T @ j)
    order = np.argsort(evals)[::-1][:k]
    return evals[order], linalg.canonical_signs(evecs[:, order], evecs[:, order])[0]


@pytest.mark.parametrize("method", ["nystrom", "pinched", "subspace_rule"])
@pytest.mark.parametrize("v", [2, 3, 4])
def test_normal_exact_recovery(method, v):
    m, n, k, p = 260, 180, 8, 5
    j, sigma = _rank_r(m, n, k, seed=83)
    res = getattr(normal, method)(j, k, p, v, SEED)
    np.testing.assert_allclose(res.lam2, sigma[:k] ** 2, rtol=1e-10)
    lam, vec = _evd(j, k)
    np.testing.assert_allclose(np.abs(np.sum(res.V * vec, axis=0)), 1.0, atol=1e-9)


@pytest.mark.parametrize("method", ["nystrom", "pinched"])
def test_normal_full_width_is_the_dense_evd(method):
    # s = n: Q_r spans R^n, so the result is the eigendecomposition of J^T J itself
    m, n, k, p = 50, 12, 5, 7
    j, _ = _decaying(m, n, 0.6, seed=89)
    res = getattr(normal, method)(j, k, p, 3, SEED)
    lam, vec = _evd(j, k)
    np.testing.assert_allclose(res.lam2, lam, rtol=1e-10)
    np.testing.assert_allclose(np.abs(np.sum(res.V * vec, axis=0)), 1.0, atol=1e-9)


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_nystrom_equals_subspace_in_the_recommended_way(v):
    # Sect. 4.2.3: Alg. 4 with v views is Alg. 2 with v views on J (even v) or J^T
    # (odd v), up to the shift nu = 2.2e-16 ||Y_r||.
    j, _ = _decaying(160, 120, 1.0, seed=97)
    k, p = 8, 4
    ny = normal.nystrom(j, k, p, v, SEED)
    if v % 2 == 0:
        r = rsvd.alg2_gensubit(j, k, p, v, SEED)
        vec = r.V
    else:
        r = rsvd.alg2_gensubit(rsvd.Transposed(j), k, p, v, SEED)
        vec = r.U
    np.testing.assert_allclose(ny.lam2, r.S ** 2, rtol=1e-9)
    np.testing.assert_allclose(np.abs(np.sum(ny.V * vec, axis=0)), 1.0, atol=1e-8)
    sub = normal.subspace_rule(j, k, p, v, SEED)
    np.testing.assert_allclose(sub.lam2, r.S ** 2, rtol=1e-14)


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_pinched_equals_subspace_the_other_way(v):
    # Sect. 4.2.3: Alg. 5 with v views is Alg. 2 with v views on J^T (even v) or J
    # (odd v), the side Sect. 4.2.1 does not recommend.
    j, _ = _decaying(160, 120, 1.0, seed=101)
    k, p = 8, 4
    pi = normal.pinched(j, k, p, v, SEED)
    if v % 2 == 0:
        r = rsvd.alg2_gensubit(rsvd.Transposed(j), k, p, v, SEED)
        vec = r.U
    else:
        r = rsvd.alg2_gensubit(j, k, p, v, SEED)
        vec = r.V
    np.testing.assert_allclose(pi.lam2, r.S ** 2, rtol=1e-9)
    np.testing.assert_allclose(np.abs(np.sum(pi.V * vec, axis=0)), 1.0, atol=1e-8)


def test_nystrom_at_least_as_accurate_as_pinched_on_average():
    # Sect. 4.2.3 and the results of Sect. 8: the prolonged sketch is one view ahead.
    j, sigma = _decaying(200, 150, 0.5, seed=103)
    k, p, v = 10, 5, 3
    jtj = j.T @ j
    errs = {"nystrom": [], "pinched": []}
    for t in range(8):
        for name in errs:
            r = getattr(normal, name)(j, k, p, v, SEED + t)
            approx = (r.V * r.lam2[None, :]) @ r.V.T
            errs[name].append(np.linalg.norm(jtj - approx, 2))
    assert np.mean(errs["nystrom"]) <= np.mean(errs["pinched"])


# ---------------------------------------------------------------- Sect. 6.1: streams

def test_streamed_sketches_are_the_sketches_of_the_sum():
    # eq. streammatmult: Y = sum_i H_i Omega_r, W = sum_i Psi H_i, with H_i dense
    # blocks and single entries (repeated coordinates add); A = sum_i H_i formed
    # separately.
    m, n, k, p = 90, 70, 5, 3
    rng = np.random.default_rng(5)
    sk = stream.Sketch(m, n, k, p, SEED)
    a = np.zeros((m, n))
    for _ in range(6):
        r0, c0 = rng.integers(0, m - 10), rng.integers(0, n - 10)
        h = rng.standard_normal((rng.integers(1, 11), rng.integers(1, 11)))
        sk.add_dense(int(r0), int(c0), h)
        a[r0:r0 + h.shape[0], c0:c0 + h.shape[1]] += h
    rows = rng.integers(0, m, 300)
    cols = rng.integers(0, n, 300)
    vals = rng.standard_normal(300)
    rows[1] = rows[0]
    cols[1] = cols[0]
    sk.add_entries(rows, cols, vals)
    np.add.at(a, (rows, cols), vals)
    s = k + p
    _, _, yc, w = rsvd.one_view_sketches(a, s, 2 * s + 1, SEED)
    np.testing.assert_allclose(sk.y, yc, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sk.w, w, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("method, lc", [("tropp", None), ("tropp", 1), ("woolfe", None), ("woolfe", "minvar")])
def test_streamed_one_view_equals_the_one_read_method(method, lc):
    m, n, k, p = 120, 90, 6, 4
    a, _ = _decaying(m, n, 1.0, seed=107)
    sk = stream.Sketch(m, n, k, p, SEED)
    for r0 in range(0, m, 25):                   # row blocks, then half of a column block twice
        sk.add_dense(r0, 0, a[r0:r0 + 25, :45])
    sk.add_dense(0, 45, 0.5 * a[:, 45:])
    sk.add_dense(0, 45, 0.5 * a[:, 45:])
    res = sk.finish(method, lc)
    ref = (rsvd.alg7_one_view if method == "tropp" else rsvd.alg8_woolfe)(a, k, p, SEED, lc=lc)
    np.testing.assert_allclose(res.S, ref.S, rtol=1e-10)
    np.testing.assert_allclose(res.U, ref.U, atol=1e-9)
    np.testing.assert_allclose(res.V, ref.V, atol=1e-9)


# ---------------------------------------------------------------- Sect. 6.7: SRFT

@pytest.mark.parametrize("length, s", [(64, 10), (257, 40), (1000, 1), (65536, 24)])
def test_srft_applies_a_sampled_dct(length, s):
    # Phi^T x = P^T C D x: scipy's orthonormal DCT-II of the sign-flipped vector,
    # at the sampled positions.
    phi = srft.matrix(SEED, length, s, srft.COLS)
    d = srft.signs(SEED, length, srft.COLS)
    pos = srft.sample(SEED, length, s, srft.COLS)
    x = np.random.default_rng(length).standard_normal((length, 3))
    ref = scipy.fft.dct(d[:, None] * x, type=2, norm="ortho", axis=0)[pos]
    np.testing.assert_allclose(phi.T @ x, ref, atol=1e-12)
    np.testing.assert_allclose(phi.T @ phi, np.eye(s), atol=1e-12)


def test_srft_sample_and_signs():
    length, s = 500, 37
    pos = srft.sample(SEED, length, s, srft.ROWS)
    assert len(set(pos.tolist())) == s and pos.min() >= 0 and pos.max() < length
    assert np.all(np.diff(pos) > 0)
    w = srft.words(SEED, srft.ROWS[1], length)
    brute = sorted(range(length), key=lambda j: (int(w[j]), j))[:s]
    assert sorted(brute) == pos.tolist()
    d = srft.signs(SEED, 4000, srft.ROWS)
    assert set(np.unique(d).tolist()) == {-1.0, 1.0} and abs(d.mean()) < 0.06
    # the two sides draw from different tags
    assert not np.array_equal(srft.sample(SEED, length, s, srft.COLS), pos)


def test_extended_srft_core_and_recovery():
    m, n, k, p = 180, 140, 6, 4
    s, s_c = k + p, 2 * (k + p) + 1
    a, _ = _decaying(m, n, 1.0, seed=109)
    res = rsvd.extended_one_view(a, k, p, SEED, s_c, core="srft")
    dr = srft.signs(SEED, m, srft.ROWS)
    dc = srft.signs(SEED, n, srft.COLS)
    pr = srft.sample(SEED, m, s_c, srft.ROWS)
    pc = srft.sample(SEED, n, s_c, srft.COLS)
    z2 = scipy.fft.dctn(dr[:, None] * a * dc[None, :], type=2, norm="ortho")
    np.testing.assert_allclose(res.extra["Z"], z2[np.ix_(pr, pc)], atol=1e-12)
    phi_r = srft.matrix(SEED, m, s_c, srft.ROWS)
    phi_c = srft.matrix(SEED, n, s_c, srft.COLS)
    core = np.linalg.pinv(phi_r.T @ res.Qc) @ res.extra["Z"] @ np.linalg.pinv((phi_c.T @ res.Qr).T)
    np.testing.assert_allclose(res.extra["C"], core, rtol=1e-9, atol=1e-11)
    ar, _ = _rank_r(m, n, k, seed=113)
    rr = rsvd.extended_one_view(ar, k, p, SEED, s_c, core="srft")
    recon = (rr.U * rr.S[None, :]) @ rr.V.T
    assert np.linalg.norm(ar - recon) <= 1e3 * np.finfo(float).eps * np.linalg.norm(ar)
    del s
