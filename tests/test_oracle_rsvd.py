"""Pins of the oracle's randomized SVD algorithms against what the paper and
the mathematics fix (exact recovery, the dense SVD, closed forms, stated
equivalences, interlacing, the expected-error theorems)."""

import numpy as np
import pytest

import synth
from oracle import errors, formats, linalg, philox, rsvd

SEED = synth.METHOD_SEED


def _rank_r(m, n, r, seed=3):
    sigma = np.arange(1, r + 1, dtype=np.float64) ** -2.0
    return synth.spectral_matrix(m, n, sigma, seed), sigma


def _decaying(m, n, power=1.0, seed=5):
    sigma = np.arange(1, min(m, n) + 1, dtype=np.float64) ** -power
    return synth.spectral_matrix(m, n, sigma, seed), sigma


def _assert_factors_match(res, u, s, v, k, rtol=1e-12, vec_tol=1e-9):
    np.testing.assert_allclose(res.S, s[:k], rtol=rtol, atol=rtol * s[0])
    # singular vectors up to sign (signs are canonicalized on both sides)
    uu, vv = linalg.canonical_signs(u[:, :k], v[:, :k])
    assert np.max(np.abs(np.abs(np.sum(res.U * uu, axis=0)) - 1.0)) < vec_tol
    assert np.max(np.abs(np.abs(np.sum(res.V * vv, axis=0)) - 1.0)) < vec_tol
    np.testing.assert_allclose(res.U, uu, atol=1e-6)
    np.testing.assert_allclose(res.V, vv, atol=1e-6)


def _exact_svd(a, k):
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    return u, s, vt.T


# ---------------------------------------------------------------- P1: exact recovery

ALGOS = {
    "alg2_v2": lambda a, k, p: rsvd.alg2_gensubit(a, k, p, 2, SEED),
    "alg2_v3": lambda a, k, p: rsvd.alg2_gensubit(a, k, p, 3, SEED),
    "alg2_v4": lambda a, k, p: rsvd.alg2_gensubit(a, k, p, 4, SEED),
    "alg2_v5": lambda a, k, p: rsvd.alg2_gensubit(a, k, p, 5, SEED),
    "alg1_q1": lambda a, k, p: rsvd.alg1_subit(a, k, p, 1, SEED),
    "alg7": lambda a, k, p: rsvd.alg7_one_view(a, k, p, SEED),
    "alg7_lc": lambda a, k, p: rsvd.alg7_one_view(a, k, p, SEED, lc=p // 2),
    "ext1v": lambda a, k, p: rsvd.extended_one_view(a, k, p, SEED, 2 * (k + p) + 1),
    "alg9_v2": lambda a, k, p: rsvd.alg9_block_krylov(a, k, p, 2, SEED),
    "alg9_v4": lambda a, k, p: rsvd.alg9_block_krylov(a, k, p, 4, SEED),
    "alg9_v5": lambda a, k, p: rsvd.alg9_block_krylov(a, k, p, 5, SEED),
    "row1": lambda a, k, p: rsvd.row_sweep_krylov(a, k, p, 1, SEED),
    "row3": lambda a, k, p: rsvd.row_sweep_krylov(a, k, p, 3, SEED, block_rows=128),
    "col2": lambda a, k, p: rsvd.col_sweep_krylov(a, k, p, 2, SEED),
}


@pytest.mark.parametrize("name", sorted(ALGOS))
def test_exact_recovery_of_rank_r(name):
    # A of exact rank r = k: every algorithm must return its SVD to rounding.
    m, n, k, p = 300, 200, 12, 6
    a, sigma = _rank_r(m, n, k)
    res = ALGOS[name](a, k, p)
    u, s, v = _exact_svd(a, k)
    _assert_factors_match(res, u, s, v, k, rtol=1e-11, vec_tol=1e-9)
    recon = (res.U * res.S[None, :]) @ res.V.T
    assert np.linalg.norm(a - recon) <= 1e3 * np.finfo(float).eps * np.linalg.norm(a)


# ---------------------------------------------------------------- P2: dense SVD

@pytest.mark.parametrize("name", ["alg2_v2", "alg2_v3", "alg2_v4", "alg7", "alg9_v2", "row1", "col2"])
def test_full_width_sketch_is_the_dense_svd(name):
    # s = min(m, n): the sketch spans the whole co-range, so the answer is the
    # truncated LAPACK SVD of A itself.
    m, n, k, p = 40, 12, 6, 6
    if name == "col2":
        m, n, k, p = 40, 24, 6, 6           # two column sweeps: 2s = n
    a, sigma = _decaying(m, n, 0.5, seed=11)
    res = ALGOS[name](a, k, p)
    u, s, v = _exact_svd(a, k)
    _assert_factors_match(res, u, s, v, k, rtol=1e-12, vec_tol=1e-10)


# ---------------------------------------------------------------- closed forms

def _svd_orth(x):
    u, s, _ = np.linalg.svd(x, full_matrices=False)
    return u


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_alg2_matches_explicit_powers(v):
    # Sect. 4.1: even v gives Q_c = orth((A A^T)^((v-2)/2) A Omega) and the
    # TSVD of Q_c Q_c^T A; odd v gives Q_r = orth((A^T A)^((v-1)/2) Omega) and
    # the TSVD of A Q_r Q_r^T.  Computed here through explicit powers and an
    # SVD-based orth (a different route to the same matrices).
    m, n, k, p = 60, 45, 5, 4
    a, _ = _decaying(m, n, 0.7, seed=21)
    om = philox.omega(SEED, n, k + p)
    if v % 2 == 0:
        x = a @ om
        for _ in range((v - 2) // 2):
            x = a @ (a.T @ x)
        qc = _svd_orth(x)
        approx = qc @ (qc.T @ a)
    else:
        x = om
        for _ in range((v - 1) // 2):
            x = a.T @ (a @ x)
        qr_ = _svd_orth(x)
        approx = (a @ qr_) @ qr_.T
    u, s, vt = np.linalg.svd(approx, full_matrices=False)
    res = rsvd.alg2_gensubit(a, k, p, v, SEED)
    _assert_factors_match(res, u, s, vt.T, k, rtol=1e-9, vec_tol=1e-8)


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_alg9_matches_explicit_krylov(v):
    # Sect. 7.2: even v: Q_c spans [A Om, (AA^T) A Om, ..., (AA^T)^((v-2)/2) A Om];
    # odd v: Q_r spans [(A^T A) Om, ..., (A^T A)^((v-1)/2) Om].
    m, n, k, p = 80, 60, 4, 3
    a, _ = _decaying(m, n, 0.5, seed=23)
    om = philox.omega(SEED, n, k + p)
    if v % 2 == 0:
        blocks, x = [], a @ om
        for _ in range(v // 2):
            blocks.append(x)
            x = a @ (a.T @ x)
        qc = _svd_orth(np.hstack(blocks))
        approx = qc @ (qc.T @ a)
    else:
        blocks, x = [], om
        for _ in range((v - 1) // 2):
            x = a.T @ (a @ x)
            blocks.append(x)
        qr_ = _svd_orth(np.hstack(blocks))
        approx = (a @ qr_) @ qr_.T
    u, s, vt = np.linalg.svd(approx, full_matrices=False)
    res = rsvd.alg9_block_krylov(a, k, p, v, SEED)
    _assert_factors_match(res, u, s, vt.T, k, rtol=1e-8, vec_tol=1e-7)


def test_alg7_solves_the_stated_least_squares_problem():
    # Sect. 6.2, step 4: X = (Omega_c^* Q_c)^+ Y_r^*; here solved by LAPACK's
    # least-squares driver instead of the QR route the algorithm prints.
    m, n, k, p = 120, 90, 6, 4
    a, _ = _decaying(m, n, 1.0, seed=31)
    res = rsvd.alg7_one_view(a, k, p, SEED)
    s = k + p
    psi = philox.psi(SEED, 2 * s + 1, m)
    qc = res.Qc
    np.testing.assert_allclose(qc.T @ qc, np.eye(s), atol=1e-13)
    np.testing.assert_allclose(res.extra["Yc"], a @ philox.omega(SEED, n, s), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(res.extra["W"], psi @ a, rtol=1e-12, atol=1e-14)
    x_ls = np.linalg.lstsq(psi @ qc, psi @ a, rcond=None)[0]
    np.testing.assert_allclose(res.extra["X"], x_ls, rtol=1e-9, atol=1e-12)
    u, lam, vt = np.linalg.svd(x_ls, full_matrices=False)
    np.testing.assert_allclose(res.S, lam[:k], rtol=1e-10)


def test_extended_core_is_the_pseudo_inverse_product():
    # Sect. 6.7, eq. bwzimproved: C = T_c^+ U_c^T Z U_r (T_r^T)^+ equals
    # (Phi_r^T Q_c)^+ Z (Q_r^T Phi_c)^+, formed here with LAPACK's pseudo-inverse
    # instead of the two QR factorizations the method takes; Z is checked
    # against the plain product Phi_r^T A Phi_c.
    m, n, k, p = 150, 110, 6, 4
    s, s_c = k + p, 2 * (k + p) + 1
    a, _ = _decaying(m, n, 1.0, seed=37)
    res = rsvd.extended_one_view(a, k, p, SEED, s_c)
    phi_r = philox.phi(SEED, s_c, m, philox.TAG_PHI)
    phi_c = philox.phi(SEED, s_c, n, philox.TAG_PHI2)
    np.testing.assert_allclose(res.extra["Z"], phi_r @ a @ phi_c.T, rtol=1e-12, atol=1e-13)
    qc, qr_ = res.Qc, res.Qr
    np.testing.assert_allclose(qc.T @ qc, np.eye(s), atol=1e-13)
    np.testing.assert_allclose(qr_.T @ qr_, np.eye(s), atol=1e-13)
    np.testing.assert_allclose(qr_ @ (qr_.T @ a.T @ philox.psi(SEED, s, m).T), a.T @ philox.psi(SEED, s, m).T,
                               rtol=1e-10, atol=1e-12)
    core = np.linalg.pinv(phi_r @ qc) @ res.extra["Z"] @ np.linalg.pinv((phi_c @ qr_).T)
    np.testing.assert_allclose(res.extra["C"], core, rtol=1e-9, atol=1e-12)
    lam = np.linalg.svd(core, compute_uv=False)
    np.testing.assert_allclose(res.S, lam[:k], rtol=1e-10)


def test_extended_exact_at_the_smallest_core():
    # With s_c = s the core test matrices are square on the sketched subspaces and
    # the reconstruction stays exact for an exact rank-k A (a special case of the
    # exact-recovery property at the smallest admissible core).
    m, n, k, p = 200, 150, 8, 4
    a, _ = _rank_r(m, n, k)
    res = rsvd.extended_one_view(a, k, p, SEED, k + p)
    recon = (res.U * res.S[None, :]) @ res.V.T
    assert np.linalg.norm(a - recon) <= 1e3 * np.finfo(float).eps * np.linalg.norm(a)


def test_alg7_oversampling_rules():
    # eq. overmed with T = 3s+1 gives l1 = p and k + l2 = 2s + 1 rows for Psi.
    for k, p in [(100, 20), (20, 10), (64, 16), (5, 5)]:
        s = k + p
        l1, l2 = rsvd.decay_oversampling(k, 3 * s + 1)
        assert l1 == p and k + l2 == 2 * s + 1
    l1, l2 = rsvd.rapid_oversampling(10, 50)
    assert (l1, l2) == (14, 16)
    l1, l2 = rsvd.flat_oversampling(10, 50)
    assert l1 >= 2 and l1 + l2 == 30


# ---------------------------------------------------------------- equivalences

@pytest.mark.parametrize("q", [0, 1, 2])
def test_alg1_equals_alg2_even_views(q):
    a, _ = _decaying(150, 100, 1.0, seed=41)
    r1 = rsvd.alg1_subit(a, 8, 5, q, SEED)
    r2 = rsvd.alg2_gensubit(a, 8, 5, 2 * q + 2, SEED)
    np.testing.assert_allclose(r1.S, r2.S, rtol=1e-13)
    np.testing.assert_allclose(r1.U, r2.U, atol=1e-11)
    np.testing.assert_allclose(r1.V, r2.V, atol=1e-11)


@pytest.mark.parametrize("v", [2, 3])
def test_alg9_equals_alg2_below_four_views(v):
    a, _ = _decaying(150, 100, 1.0, seed=43)
    r9 = rsvd.alg9_block_krylov(a, 8, 5, v, SEED)
    r2 = rsvd.alg2_gensubit(a, 8, 5, v, SEED)
    np.testing.assert_allclose(r9.S, r2.S, rtol=1e-12)
    np.testing.assert_allclose(r9.U, r2.U, atol=1e-10)
    np.testing.assert_allclose(r9.V, r2.V, atol=1e-10)


def test_row_sweep_one_pass_equals_two_view_subspace():
    # Sect. 6.8: Y = A Om and A^T Y in one sweep give the basic 2-view method.
    a, _ = _decaying(200, 120, 1.0, seed=47)
    rs = rsvd.row_sweep_krylov(a, 10, 5, 1, SEED, block_rows=64)
    r2 = rsvd.alg2_gensubit(a, 10, 5, 2, SEED)
    np.testing.assert_allclose(rs.S, r2.S, rtol=1e-11)
    np.testing.assert_allclose(rs.U, r2.U, atol=1e-9)
    np.testing.assert_allclose(rs.V, r2.V, atol=1e-9)


@pytest.mark.parametrize("v", [2, 3])
def test_row_sweep_equals_alg9_with_twice_the_views(v):
    # Sect. 7.3: one sweep gives A^T A X, so v sweeps span Alg. 9's K_c for 2v views.
    a, _ = _decaying(240, 160, 0.5, seed=53)
    rs = rsvd.row_sweep_krylov(a, 6, 4, v, SEED)
    r9 = rsvd.alg9_block_krylov(a, 6, 4, 2 * v, SEED)
    np.testing.assert_allclose(rs.S, r9.S, rtol=1e-9)
    np.testing.assert_allclose(rs.U, r9.U, atol=1e-7)
    np.testing.assert_allclose(rs.V, r9.V, atol=1e-7)


def test_row_sweep_independent_of_block_rows():
    a, _ = _decaying(256, 100, 1.0, seed=59)
    base = rsvd.row_sweep_krylov(a, 8, 4, 2, SEED)
    for rows in (1, 17, 64, 255):
        r = rsvd.row_sweep_krylov(a, 8, 4, 2, SEED, block_rows=rows)
        np.testing.assert_allclose(r.S, base.S, rtol=1e-12)
        np.testing.assert_allclose(r.U, base.U, atol=1e-10)


def test_col_sweep_is_row_sweep_of_transpose():
    a, _ = _decaying(120, 200, 1.0, seed=61)
    c = rsvd.col_sweep_krylov(a, 8, 4, 2, SEED)
    r = rsvd.row_sweep_krylov(np.ascontiguousarray(a.T), 8, 4, 2, SEED)
    np.testing.assert_allclose(c.S, r.S, rtol=1e-12)
    np.testing.assert_allclose(np.abs(c.U), np.abs(r.V), atol=1e-10)


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("name", ["alg2_v2", "alg2_v3", "alg2_v4", "alg9_v4", "alg9_v5", "row3"])
def test_interlacing_and_orthonormality(name):
    # sigma_i(Q^T A) <= sigma_i(A) for any orthonormal Q (Ritz values).
    a, sigma = _decaying(300, 200, 1.0, seed=67)
    k, p = 10, 5
    res = ALGOS[name](a, k, p)
    assert np.all(res.S <= sigma[:k] * (1 + 1e-12))
    for q in (res.Qc, res.Qr):
        if q is not None:
            assert np.max(np.abs(q.T @ q - np.eye(q.shape[1]))) < 1e-13
    for f in (res.U, res.V):
        assert np.max(np.abs(f.T @ f - np.eye(k))) < 1e-12
    assert np.all(np.diff(res.S) <= 0)


def test_sketches_are_linear():
    # eq. streammatmult: sketches of a sum of updates are sums of sketches.
    rng = np.random.default_rng(0)
    a1 = rng.standard_normal((70, 50))
    a2 = rng.standard_normal((70, 50))
    om = philox.omega(SEED, 50, 9)
    ps = philox.psi(SEED, 19, 70)
    np.testing.assert_allclose(rsvd.times(a1 + a2, om), rsvd.times(a1, om) + rsvd.times(a2, om),
                               rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(rsvd.times_t(a1 + a2, ps.T),
                               rsvd.times_t(a1, ps.T) + rsvd.times_t(a2, ps.T), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- expected error (Thm 3.1/4.1)

def test_error_decays_with_views_within_theorem_bounds():
    # Sect. 4.2.2: after v views the returned basis (Q_c for even v, Q_r for
    # odd v) has expected spectral error at most the Thm. 3.1/4.1 bound with
    # exponent v-1; errors fall with v (Sect. 8.3).  Mean over 20 seeds.
    m, n, k, p = 240, 160, 10, 5
    sigma = np.arange(1, n + 1, dtype=np.float64) ** -1.0
    a = synth.spectral_matrix(m, n, sigma, seed=71)
    means = []
    for v in range(2, 7):
        errs = []
        for t in range(20):
            res = rsvd.alg2_gensubit(a, k, p, v, SEED + t)
            if v % 2 == 0:
                errs.append(errors.range_projection_error(a, res.Qc))
            else:
                errs.append(errors.corange_projection_error(a, res.Qr))
        mean = float(np.mean(errs))
        bound = errors.expected_error_bound(sigma, k, p, v - 1)
        # a rank-(k+p) projection cannot beat sigma_{k+p+1} (Eckart-Young)
        assert sigma[k + p] <= mean <= bound, (v, mean, bound)
        means.append(mean)
    assert all(b < a_ for a_, b in zip(means, means[1:]))


def test_theorem_bound_values_for_c1():
    # B(v)/sigma_{k+1} for sigma_j = j^-2 (j <= 1000), k = 20, p = 10.
    sigma = np.arange(1, 1001, dtype=np.float64) ** -2.0
    got = [errors.expected_error_bound(sigma, 20, 10, v - 1) / sigma[20] for v in range(2, 7)]
    np.testing.assert_allclose(got, [6.57, 2.30, 1.69, 1.46, 1.35], atol=0.006)


def test_relative_errors_of_the_optimal_approximation_vanish():
    a, sigma = _decaying(90, 60, 1.0, seed=73)
    u, s, v = _exact_svd(a, 7)
    assert abs(errors.relative_frobenius_error(a, u[:, :7], s[:7], v[:, :7], sigma)) < 1e-10
    assert abs(errors.relative_spectral_error(a, u[:, :7], s[:7], v[:, :7], sigma)) < 1e-10


# ---------------------------------------------------------------- storage formats

def test_format_decoders():
    assert formats.bf16_bits_to_f64(np.array([0x3F80, 0xC000, 0x0000])).tolist() == [1.0, -2.0, 0.0]
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "e4m3_values.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        byte, val = line.split()
        assert formats.e4m3_value(int(byte, 16)) == float(val)
    assert np.isnan(formats.e4m3_value(0x7F)) and np.isnan(formats.e4m3_value(0xFF))
    # every finite code decodes to a distinct value, monotone in the code
    pos = np.array([formats.e4m3_value(b) for b in range(0x7F)])
    assert np.all(np.diff(pos) > 0)


def test_quantizers_round_to_nearest_even():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((64, 33)) * 10.0 ** rng.uniform(-3, 3, (64, 1))
    bits, scale = synth.to_fp8_rows(a)
    deq = formats.fp8_rows_to_f64(bits, scale)
    # nearest: no representable value is closer than the chosen one
    table = np.array([formats.e4m3_value(b) for b in range(0x7F)])
    x = np.abs(a / scale.astype(np.float64)[:, None])
    best = np.min(np.abs(table[None, None, :] - x[..., None]), axis=-1)
    assert np.all(np.abs(np.abs(deq / scale.astype(np.float64)[:, None]) - x) <= best + 1e-12)
    b16 = synth.to_bf16_bits(a.astype(np.float32))
    back = formats.bf16_bits_to_f64(b16)
    assert np.all(np.abs(back - a.astype(np.float32)) <= 2.0 ** -8 * np.abs(a.astype(np.float32)))
