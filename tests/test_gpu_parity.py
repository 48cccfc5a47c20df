"""GPU parity: the HIP library against the FP64 CPU oracle on the same seeded
inputs.  Tolerances (relative, singular values): 1e-10 on the FP64 path,
1e-4 on the FP32 path."""

import sys

import numpy as np
import pytest

import synth
from oracle import linalg as olinalg
from oracle import philox as ophilox
from oracle import rsvd as orsvd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1804_07531_amd as rs  # noqa: E402

DEV = torch.device("cuda:0")
SEED = synth.METHOD_SEED


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _decaying(m, n, power, seed, rank=None):
    r = min(m, n) if rank is None else rank
    sigma = np.arange(1, r + 1, dtype=np.float64) ** -power
    return synth.spectral_matrix(m, n, sigma, seed), sigma


def _compare(res_gpu, ref, k, s_tol, vec_tol, nvec=None):
    U, S, V = (x.double().cpu().numpy() for x in res_gpu)
    rel = np.abs(S - ref.S) / np.abs(ref.S)
    assert np.max(rel) <= s_tol, f"sigma rel err {np.max(rel):.3e} > {s_tol:.1e} (at {int(np.argmax(rel))})"
    nv = k if nvec is None else nvec
    du = np.max(np.abs(np.abs(np.sum(U[:, :nv] * ref.U[:, :nv], axis=0)) - 1.0))
    dv = np.max(np.abs(np.abs(np.sum(V[:, :nv] * ref.V[:, :nv], axis=0)) - 1.0))
    assert du <= vec_tol and dv <= vec_tol, f"vector misalignment U {du:.3e} V {dv:.3e}"
    return np.max(rel), du, dv


# ----------------------------------------------------------------- generator

def test_philox_words_bitwise():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 1 << 32, size=(4, 4099), dtype=np.int64)
    key = (0x12345678, 0x9ABCDEF0)
    got = rs.philox_words(torch.from_numpy(ctr).to(DEV), *key).cpu().numpy()
    ref = ophilox.philox4x32_10(ctr.astype(np.uint64), key).astype(np.int64)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("long_is_row", [1, 0])
def test_gaussian_matches_oracle(long_is_row):
    seed, tag = 0xDEADBEEF12345, 1
    rows, cols = (1031, 7) if long_is_row else (7, 1031)
    g64 = rs.gaussian(seed, tag, rows, cols, long_is_row).cpu().numpy()
    if long_is_row:
        ref = ophilox.gaussian(seed, tag, 0, np.arange(rows)[:, None], np.arange(cols)[None, :])
    else:
        ref = ophilox.gaussian(seed, tag, 0, np.arange(cols)[None, :], np.arange(rows)[:, None])
    np.testing.assert_allclose(g64, ref, rtol=1e-14, atol=1e-14)
    g32 = rs.gaussian(seed, tag, rows, cols, long_is_row, dtype=torch.float32).cpu().numpy()
    assert np.max(np.abs(g32 - ref.astype(np.float32))) <= 1e-6 * np.max(np.abs(ref))


# ----------------------------------------------------------------- the views

VIEW_SHAPES = [(16, 16, 16), (1, 1, 1), (37, 53, 5), (300, 17, 30), (17, 300, 30), (1000, 700, 120),
               (2048, 4096, 64), (4099, 33, 129), (65, 20000, 20), (20000, 65, 20), (64, 64, 256),
               # thin widths of 1, 2 and 6 blocks of 16 with one and two blocks of A per wave
               (9000, 520, 80), (520, 9000, 96), (8200, 256, 24), (256, 8200, 9),
               # co-range views with two column blocks per wave and 12 or 16 thin blocks
               (600, 9000, 241), (300, 8200, 180),
               # range views with four row blocks per wave (ragged last workgroup) and 4, 6 or 8 thin blocks,
               # and wide co-range views with a ragged last workgroup
               (33000, 600, 120), (40000, 64, 50), (36000, 200, 90), (700, 16500, 120), (300, 20000, 70)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", VIEW_SHAPES)
@pytest.mark.parametrize("trans", [False, True])
def test_views_match_products(dtype, shape, trans):
    m, n, s = shape
    say(f"view {dtype} m={m} n={n} s={s} trans={trans}")
    rng = np.random.default_rng(m * 7 + n + s)
    a = rng.standard_normal((m, n))
    x = rng.standard_normal((s, n))
    y = rng.standard_normal((s, m))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    stored = a.T if trans else a
    A = _t(stored, tdt)
    a_used = (A.double().cpu().numpy().T if trans else A.double().cpu().numpy())
    X = _t(x, tdt)
    Y = _t(y, tdt)
    yt = rs.view_range(A, X, trans=trans).double().cpu().numpy()
    zt = rs.view_corange(A, Y, trans=trans).double().cpu().numpy()
    ref_y = (a_used @ X.double().cpu().numpy().T).T
    ref_z = (a_used.T @ Y.double().cpu().numpy().T).T
    tol = 1e-13 if dtype == "f64" else 3e-6
    scale_y = np.sqrt(n) * np.max(np.abs(a_used)) * np.max(np.abs(x))
    scale_z = np.sqrt(m) * np.max(np.abs(a_used)) * np.max(np.abs(y))
    assert np.max(np.abs(yt - ref_y)) <= tol * scale_y
    assert np.max(np.abs(zt - ref_z)) <= tol * scale_z


def test_views_are_linear_and_deterministic():
    # eq. streammatmult: sketch(A1 + A2) = sketch(A1) + sketch(A2); repeated
    # runs are bitwise identical (fixed-order reductions).
    rng = np.random.default_rng(9)
    a1, a2 = rng.standard_normal((2, 3000, 2500))
    X = _t(rng.standard_normal((40, 2500)))
    y1 = rs.view_range(_t(a1), X).cpu().numpy()
    y2 = rs.view_range(_t(a2), X).cpu().numpy()
    y12 = rs.view_range(_t(a1 + a2), X).cpu().numpy()
    np.testing.assert_allclose(y12, y1 + y2, rtol=0, atol=1e-11)
    again = rs.view_range(_t(a1), X).cpu().numpy()
    assert np.array_equal(again, y1)


# ----------------------------------------------------------------- Alg. 2

@pytest.mark.parametrize("v", [2, 3, 4, 5, 6])
def test_subspace_c1_fp64(v):
    # 2000 x 1000, sigma_j = j^-2, k = 20, p = 10: the FP64 parity workload.
    a, sigma = synth.workload_c1()
    say(f"subspace f64 2000x1000 k=20 p=10 v={v}")
    res = rs.subspace(_t(a), 20, 10, v, seed=SEED)
    ref = orsvd.alg2_gensubit(a, 20, 10, v, SEED)
    _compare(res, ref, 20, 1e-10, 1e-8)


@pytest.mark.parametrize("shape", [(777, 333, 9, 7, 3), (333, 777, 9, 7, 4), (130, 70, 30, 40, 2),
                                   (5000, 257, 40, 10, 5)])
def test_subspace_ragged_fp64(shape):
    m, n, k, p, v = shape
    a, _ = _decaying(m, n, 1.0, seed=m + n)
    say(f"subspace f64 {m}x{n} k={k} p={p} v={v}")
    res = rs.subspace(_t(a), k, p, v, seed=SEED + 1)
    ref = orsvd.alg2_gensubit(a, k, p, v, SEED + 1)
    _compare(res, ref, k, 1e-10, 1e-7)


@pytest.mark.parametrize("v", [2, 3])
def test_subspace_trans_storage(v):
    a, _ = _decaying(600, 400, 1.0, seed=17)
    res = rs.subspace(_t(np.ascontiguousarray(a.T)), 10, 6, v, trans=True, seed=SEED)
    ref = orsvd.alg2_gensubit(a, 10, 6, v, SEED)
    _compare(res, ref, 10, 1e-10, 1e-8)


@pytest.mark.parametrize("method", ["one_view", "extended", "row_sweep"])
def test_trans_storage_other_methods(method):
    # A held as A^T row-major (trans = 1): the one-view sweep then takes column
    # panels of the stored matrix, and the row sweep row blocks of A
    m, n, k, p = 900, 500, 12, 6
    a, _ = _decaying(m, n, 1.0, seed=19)
    At = _t(np.ascontiguousarray(a.T))
    say(f"trans storage {method} {m}x{n}")
    if method == "one_view":
        res = rs.single_pass(At, k, p, trans=True, seed=SEED, block_rows=256)
        ref = orsvd.alg7_one_view(a, k, p, SEED)
    elif method == "extended":
        res = rs.single_pass(At, k, p, trans=True, seed=SEED, core_rows=2 * (k + p) + 1, block_rows=256)
        ref = orsvd.extended_one_view(a, k, p, SEED, 2 * (k + p) + 1)
    else:
        res = rs.block_krylov(At, k, p, 3, mode="row", trans=True, seed=SEED, block_rows=256)
        ref = orsvd.row_sweep_krylov(a, k, p, 3, SEED, tau=2.0 ** -40)
    _compare(res, ref, k, 1e-10, 1e-7)


@pytest.mark.parametrize("v", [2, 3, 4])
def test_subspace_fp32(v):
    m, n, k, p = 6000, 3000, 60, 20
    a, _ = _decaying(m, n, 1.5, seed=29, rank=1500)
    a32 = a.astype(np.float32)
    say(f"subspace f32 {m}x{n} k={k} p={p} v={v}")
    res = rs.subspace(_t(a32, torch.float32), k, p, v, seed=SEED)
    ref = orsvd.alg2_gensubit(a32, k, p, v, SEED)
    _compare(res, ref, k, 1e-4, 1e-2, nvec=20)


# The FP32 Gram matrices of the orthonormalization run whole 16-wide steps with
# their loads four steps ahead of the products: panels of 16 to 100 rows or
# columns give 1 to 6 whole steps, with and without a ragged tail, in one split.
@pytest.mark.parametrize("m,n", [(16, 48), (64, 80), (100, 37), (52, 64)])
def test_subspace_fp32_short_panels(m, n):
    k, p, v = 6, 4, 3
    a, _ = _decaying(m, n, 1.5, seed=31, rank=min(m, n))
    a32 = a.astype(np.float32)
    say(f"subspace f32 short panels {m}x{n} k={k} p={p} v={v}")
    res = rs.subspace(_t(a32, torch.float32), k, p, v, seed=SEED)
    ref = orsvd.alg2_gensubit(a32, k, p, v, SEED)
    _compare(res, ref, k, 1e-4, 1e-2)


def test_subspace_exact_recovery_rank_deficient():
    # rank 12 < s = 18: every CholeskyQR meets an exactly singular Gram matrix.
    a, sigma = _decaying(500, 300, 2.0, seed=3, rank=12)
    for v in (2, 3):
        U, S, V = rs.subspace(_t(a), 12, 6, v, seed=SEED)
        s = S.cpu().numpy()
        np.testing.assert_allclose(s, sigma[:12], rtol=1e-10)
        recon = (U.cpu().numpy() * s) @ V.cpu().numpy().T
        assert np.linalg.norm(recon - a) <= 1e-10 * np.linalg.norm(a)


def test_zero_matrix():
    U, S, V = rs.subspace(_t(np.zeros((200, 100))), 5, 5, 2, seed=SEED)
    assert np.all(S.cpu().numpy() == 0)
    assert np.all(np.isfinite(U.cpu().numpy())) and np.all(np.isfinite(V.cpu().numpy()))


def test_seed_changes_result_and_is_reproducible():
    a, _ = _decaying(400, 300, 0.5, seed=7)
    A = _t(a)
    s1 = rs.subspace(A, 10, 5, 2, seed=1)[1].cpu().numpy()
    s1b = rs.subspace(A, 10, 5, 2, seed=1)[1].cpu().numpy()
    s2 = rs.subspace(A, 10, 5, 2, seed=2)[1].cpu().numpy()
    assert np.array_equal(s1, s1b)
    assert not np.array_equal(s1, s2)


# ----------------------------------------------------------------- Alg. 7

@pytest.mark.parametrize("shape", [(2000, 1000, 20, 10), (700, 333, 9, 5), (333, 700, 12, 4)])
def test_single_pass_fp64(shape):
    m, n, k, p = shape
    a, _ = _decaying(m, n, 2.0, seed=41)
    say(f"single pass f64 {m}x{n} k={k} p={p}")
    res = rs.single_pass(_t(a), k, p, seed=SEED)
    ref = orsvd.alg7_one_view(a, k, p, SEED)
    _compare(res, ref, k, 1e-10, 1e-7)


@pytest.mark.parametrize("rows", [256, 768, 1792, 4096])
def test_single_pass_panel_heights(rows):
    # the one-view sweep over row panels (several panels, a ragged last one,
    # or a single panel taller than A) computes the same Y and W
    m, n, k, p = 2000, 1000, 20, 10
    a, _ = _decaying(m, n, 2.0, seed=45)
    say(f"single pass f64 {m}x{n} panels of {rows} rows")
    res = rs.single_pass(_t(a), k, p, seed=SEED, block_rows=rows)
    ref = orsvd.alg7_one_view(a, k, p, SEED)
    _compare(res, ref, k, 1e-10, 1e-7)


def test_single_pass_fp32_and_psi_rows():
    m, n, k, p = 4000, 2000, 40, 10
    a, _ = _decaying(m, n, 2.0, seed=43, rank=800)
    a32 = a.astype(np.float32)
    res = rs.single_pass(_t(a32, torch.float32), k, p, seed=SEED)
    ref = orsvd.alg7_one_view(a32, k, p, SEED)
    _compare(res, ref, k, 1e-4, 1e-2, nvec=10)
    res = rs.single_pass(_t(a), 10, 5, seed=SEED, psi_rows=50)
    ref = orsvd.alg7_one_view(a, 10, 5, SEED, s_w=50)
    _compare(res, ref, 10, 1e-10, 1e-7)


@pytest.mark.parametrize("shape", [(2000, 1000, 20, 10, 61), (700, 333, 9, 5, 14), (333, 700, 12, 4, 40),
                                   (1500, 400, 30, 10, 300)])
def test_extended_one_view_fp64(shape):
    # Sect. 6.7, eq. bwzimproved with Gaussian core test matrices; the last case has
    # s + s_c = 340 thin rows in the sweep (several view slices, ragged)
    m, n, k, p, sc = shape
    a, _ = _decaying(m, n, 1.0, seed=71)
    say(f"extended one view f64 {m}x{n} k={k} p={p} s_c={sc}")
    res = rs.single_pass(_t(a), k, p, seed=SEED, core_rows=sc)
    ref = orsvd.extended_one_view(a, k, p, SEED, sc)
    _compare(res, ref, k, 1e-10, 1e-7)


def test_extended_one_view_fp32_and_panels():
    m, n, k, p = 4000, 2000, 40, 10
    sc = 2 * (k + p) + 1
    a, _ = _decaying(m, n, 1.5, seed=73, rank=800)
    a32 = a.astype(np.float32)
    ref = orsvd.extended_one_view(a32.astype(np.float64), k, p, SEED, sc)
    for rows in (1024, 768):   # default panels (one panel here), then ragged 768-row panels
        res = rs.single_pass(_t(a32, torch.float32), k, p, seed=SEED, core_rows=sc, block_rows=rows)
        _compare(res, ref, k, 1e-4, 1e-2, nvec=10)


def test_extended_one_view_rejects_bad_sizes():
    A = _t(np.random.default_rng(1).standard_normal((200, 100)))
    with pytest.raises(rs.RsvdError):
        rs.single_pass(A, 10, 5, seed=SEED, core_rows=14)            # s_c < k + p
    with pytest.raises(rs.RsvdError):
        rs.single_pass(A, 10, 5, seed=SEED, core_rows=101)           # s_c > min(m, n)
    with pytest.raises(rs.RsvdError):
        rs.single_pass(A, 10, 5, seed=SEED, core_rows=31, psi_rows=31)   # l1 != l2
    with pytest.raises(rs.RsvdError):
        rs.subspace(A, 10, 5, 2, seed=SEED, core_rows=31)            # core sketch only in the one-view method


# ----------------------------------------------------------------- Alg. 9 and the row sweep

@pytest.mark.parametrize("v", [2, 3, 4, 5, 6])
def test_block_krylov_alternating_fp64(v):
    a, _ = _decaying(1500, 900, 1.0, seed=47)
    say(f"krylov alternating f64 1500x900 v={v}")
    res = rs.block_krylov(_t(a), 16, 8, v, mode="alternating", seed=SEED)
    ref = orsvd.alg9_block_krylov(a, 16, 8, v, SEED)
    _compare(res, ref, 16, 1e-10, 1e-7)


@pytest.mark.parametrize("v,rows", [(1, 1024), (2, 1024), (3, 256), (2, 5000), (3, 77)])
def test_row_sweep_fp64(v, rows):
    a, _ = _decaying(3000, 800, 1.0, seed=53)
    say(f"krylov row sweep f64 3000x800 v={v} block_rows={rows}")
    res = rs.block_krylov(_t(a), 20, 10, v, mode="row", block_rows=rows, seed=SEED)
    ref = orsvd.row_sweep_krylov(a, 20, 10, v, SEED, tau=2.0 ** -40)
    _compare(res, ref, 20, 1e-10, 1e-7)


@pytest.mark.parametrize("v", [1, 2])
def test_col_sweep_fp64(v):
    a, _ = _decaying(700, 1600, 1.0, seed=59)
    res = rs.block_krylov(_t(a), 12, 8, v, mode="col", seed=SEED)
    ref = orsvd.col_sweep_krylov(a, 12, 8, v, SEED, tau=2.0 ** -40)
    _compare(res, ref, 12, 1e-10, 1e-7)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_row_sweep_truncated(dtype):
    # rank 40 below v s = 60: K is rank-deficient, so the TSVD of R_K cuts columns
    # (the path that takes the small SVD of R_K; full-rank cases skip it).  A
    # rank-deficient K also sends its CholeskyQR down the shifted path, whose
    # shift 11 (m sk + sk (sk + 1)) u tr(G) leaves a near-uniform relative error of
    # a few times the shift factor on sigma in FP64 (measured 2.2e-9): the FP64
    # bound here is 100 times that factor, not the 1e-10 of full-rank cases.
    m, n, k, p, v = 1500, 700, 12, 8, 3
    sk = v * (k + p)
    a, _ = _decaying(m, n, 1.0, seed=67, rank=40)
    tau = 2.0 ** -40 if dtype == "f64" else 2.0 ** -20
    if dtype == "f32":
        a = a.astype(np.float32).astype(np.float64)
    say(f"krylov row sweep {dtype} {m}x{n} rank 40, v s = 60")
    res = rs.block_krylov(_t(a, torch.float64 if dtype == "f64" else torch.float32), k, p, v, mode="row", seed=SEED)
    ref = orsvd.row_sweep_krylov(a, k, p, v, SEED, tau=tau)
    s_tol = 100 * 11 * (m * sk + sk * (sk + 1)) * 2.0 ** -53 if dtype == "f64" else 1e-4
    _compare(res, ref, k, s_tol, 1e-7 if dtype == "f64" else 1e-2, nvec=k // 2)


def test_row_sweep_fp32():
    m, n, k, p, v = 8192, 2048, 48, 16, 3
    a, _ = _decaying(m, n, 1.0, seed=61)
    a32 = a.astype(np.float32)
    say(f"krylov row sweep f32 {m}x{n} v={v}")
    res = rs.block_krylov(_t(a32, torch.float32), k, p, v, mode="row", seed=SEED)
    ref = orsvd.row_sweep_krylov(a32, k, p, v, SEED, tau=2.0 ** -20)
    _compare(res, ref, k, 1e-4, 1e-2, nvec=16)


def test_exact_recovery_all_methods():
    a, sigma = _decaying(600, 400, 2.0, seed=3, rank=10)
    A = _t(a)
    outs = [rs.single_pass(A, 10, 6, seed=SEED), rs.block_krylov(A, 10, 6, 4, seed=SEED),
            rs.block_krylov(A, 10, 6, 2, mode="row", seed=SEED)]
    for U, S, V in outs:
        s = S.cpu().numpy()
        np.testing.assert_allclose(s, sigma[:10], rtol=1e-9)
        recon = (U.cpu().numpy() * s) @ V.cpu().numpy().T
        assert np.linalg.norm(recon - a) <= 1e-9 * np.linalg.norm(a)


def test_outputs_are_orthonormal_and_sign_canonical():
    a, _ = _decaying(900, 500, 1.0, seed=67)
    U, S, V = (x.cpu().numpy() for x in rs.subspace(_t(a), 15, 5, 3, seed=SEED))
    assert np.max(np.abs(U.T @ U - np.eye(15))) < 1e-12
    assert np.max(np.abs(V.T @ V - np.eye(15))) < 1e-12
    u2, v2 = olinalg.canonical_signs(U, V)
    assert np.array_equal(u2, U) and np.array_equal(v2, V)
    assert np.all(np.diff(S) <= 0)


# ------------------------------------------------------- widths above 256

@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_row_sweep_width_320(dtype):
    """v * s = 320 (k = 64, p = 16, v = 4): the widths of the differentiation workload."""
    m, n, k, p, v = 2048, 1024, 64, 16, 4
    say(f"row sweep width 320 {dtype}")
    sigma = np.arange(1, 1025, dtype=np.float64) ** -1.0
    A = synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 5)
    if dtype == "f32":
        A = A.astype(np.float32).astype(np.float64)
    tau = 2.0 ** -40 if dtype == "f64" else 2.0 ** -20
    ref = orsvd.row_sweep_krylov(A, k, p, v, SEED, tau=tau, block_rows=1024)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    res = rs.block_krylov(_t(A, tdt), k, p, v, mode="row", seed=SEED)
    _compare(res, ref, k, 1e-10 if dtype == "f64" else 1e-4, 1e-8 if dtype == "f64" else 1e-2, nvec=k // 2)


def test_subspace_width_300_fp64():
    m, n, k, p, v = 1500, 900, 250, 50, 3
    say("subspace width 300 fp64")
    A, _ = _decaying(m, n, 1.0, synth.GEN_SEED + 6)
    ref = orsvd.alg2_gensubit(A, k, p, v, SEED)
    res = rs.subspace(_t(A), k, p, v, seed=SEED)
    _compare(res, ref, k, 1e-10, 1e-6, nvec=20)


@pytest.mark.parametrize("k,p", [(111, 10), (112, 10), (118, 10), (100, 30), (7, 2), (13, 3)])
def test_subspace_small_svd_widths_fp64(k, p):
    """Core widths s = k + p on both sides of the small SVD's LDS limit
    (s = 121 in LDS, 122 and above in global scratch) and ragged blocks."""
    m, n, v = 700, 450, 2
    say(f"subspace small-SVD width {k + p}")
    A, _ = _decaying(m, n, 1.5, synth.GEN_SEED + 7)
    ref = orsvd.alg2_gensubit(A, k, p, v, SEED)
    res = rs.subspace(_t(A), k, p, v, seed=SEED)
    _compare(res, ref, k, 1e-10, 1e-6, nvec=min(k, 20))
