"""GPU checks at the full FP32 benchmark size, in the launch configurations the
benchmark times: A is 65536 x 16384 FP32 (4 GiB), sigma_j = j^-1.5 on rank
2048 plus Gaussian noise of spectral norm about 1e-4 sigma_1 (sigma_1 = 1),
k = 100, p = 20.

The views (Sect. 2, the products with A) are checked element by element:
sampled rows of Y = A X and sampled columns of Z = A^T Y of the whole matrix,
and every output of the range and co-range views of one 4096-row panel as the
one-view sweep of Alg. 7 takes it, against the oracle's FP64 products.

Whole solves are checked against the FP64 oracle run on the same stored
values (the FP32 matrix upcast exactly, streamed in blocks of rows): Alg. 2
for every view budget v = 2..6 and Alg. 7 with s_w = 2s + 1 = 241, the step
the benchmark times.  All k = 100 singular values are held to the FP32
tolerance of 1e-4 relative, and every left and right singular vector to a
subspace angle of at most 2e-5 sigma_1 / gap_i, where gap_i is the oracle's
distance from sigma_i to its nearest neighbour among the k values (a
first-order perturbation bound for an FP32-sized error in the projected
matrix; it is vacuous once gap_i < 2e-5 sigma_1).

Properties that hold at any size are checked beside them:
- Alg. 2 returns the singular values of Q^T A, which interlace those of A, so
  each sigma_i is a lower bound (up to FP32 rounding) that tightens with the
  number of views;
- Weyl's inequality keeps sigma_i(A) within the noise norm of the prescribed
  sigma_i;
- orthonormal factors and small singular-triplet residuals;
- agreement between independent methods (Alg. 2 and Alg. 9).
The bounds come from the oracle run on an 8192 x 4096 matrix built the same
way (FP64): top-10 residuals 2e-5 at v = 3 and 2e-10 at v = 6; top-50
singular values of v = 2..5 views within 8e-2, 6e-3, 4e-4 and 3e-5 of v = 6;
Alg. 9 and Alg. 2 at v = 6 within 2e-6; Alg. 7 top 10 within 4.4e-3; the
extended one-view sketch of Sect. 6.7 (s_c = 241) top 10 within 8.2e-3.
"""

import sys
import time

import numpy as np
import pytest

import synth
from oracle import rsvd as orsvd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1804_07531_amd as rs  # noqa: E402

M, N, K, P, RANK = 65536, 16384, 100, 20, 2048
S_W = 2 * (K + P) + 1
PANEL = 4096
SEED = synth.METHOD_SEED
SIGMA = np.arange(1, RANK + 1, dtype=np.float64) ** -1.5
NOISE_NORM = 1.1e-4        # spectral norm of the noise, with a margin (about 1e-4 sigma_1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    say(f"full size: building {M}x{N} FP32 A (rank {RANK}, sigma_j = j^-1.5, noise 1e-4)")
    a = synth.spectral_matrix_torch(M, N, SIGMA, synth.GEN_SEED + 2, noise=1e-4, dtype=torch.float32,
                                    device="cuda")
    torch.cuda.synchronize()
    yield a
    del a
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def solves(A):
    out = {}
    for v in (2, 3, 4, 5, 6):
        say(f"full size: subspace v={v}")
        out[v] = [x.double().cpu().numpy() for x in rs.subspace(A, K, P, v, seed=SEED)]
    return out


def _panel(gen, rows, cols):
    return torch.randn(rows, cols, generator=gen, device="cuda", dtype=torch.float32)


def _bound(n, a, x):
    # same form as the small-size view tests: FP32 sums of n terms
    return 3e-6 * np.sqrt(n) * np.max(np.abs(a)) * np.max(np.abs(x))


def test_full_size_range_view_sampled_rows(A):
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    XT = _panel(g, K + P, N)
    say("full size: range view, s = 120")
    YT = rs.view_range(A, XT)
    rng = np.random.default_rng(12)
    idx = np.unique(np.concatenate([[0, 1, 63, 64, 127, 128, 4095, 4096, 32767, 32768, M - 1],
                                    rng.integers(0, M, 245)]))
    a_rows = A[torch.from_numpy(idx).cuda()].double().cpu().numpy()
    x = XT.double().cpu().numpy().T
    ref = orsvd.times(a_rows, x)
    got = YT[:, torch.from_numpy(idx).cuda()].double().cpu().numpy().T
    err = np.max(np.abs(got - ref))
    assert err <= _bound(N, a_rows, x), f"range view max err {err:.3e}"


def test_full_size_corange_view_sampled_columns(A):
    g = torch.Generator(device="cuda")
    g.manual_seed(13)
    YT = _panel(g, K + P, M)
    say("full size: co-range view, s = 120")
    ZT = rs.view_corange(A, YT)
    rng = np.random.default_rng(14)
    cols = np.unique(np.concatenate([[0, 1, 63, 64, 8191, 8192, N - 1], rng.integers(0, N, 121)]))
    a_cols = A[:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    y = YT.double().cpu().numpy().T
    ref = orsvd.times_t(a_cols, y)
    got = ZT[:, torch.from_numpy(cols).cuda()].double().cpu().numpy().T
    err = np.max(np.abs(got - ref))
    assert err <= _bound(M, a_cols, y), f"co-range view max err {err:.3e}"


@pytest.mark.parametrize("panel", [0, 7, M // PANEL - 1])
def test_full_size_one_view_panel_products(A, panel):
    # the products the one-view sweep takes on one 4096-row panel: Y_b = A_b Omega
    # (s = 120) and Psi_b A_b (s_w = 241), every output element
    r0 = panel * PANEL
    Ab = A[r0:r0 + PANEL]
    g = torch.Generator(device="cuda")
    g.manual_seed(15 + panel)
    XT = _panel(g, K + P, N)
    PsiT = _panel(g, S_W, PANEL)
    say(f"full size: one-view panel {panel} (rows {r0}..{r0 + PANEL - 1})")
    yt = rs.view_range(Ab, XT).double().cpu().numpy().T
    wt = rs.view_corange(Ab, PsiT).double().cpu().numpy().T
    a = Ab.double().cpu().numpy()
    x = XT.double().cpu().numpy().T
    psi = PsiT.double().cpu().numpy().T
    ey = np.max(np.abs(yt - orsvd.times(a, x)))
    ew = np.max(np.abs(wt - orsvd.times_t(a, psi)))
    assert ey <= _bound(N, a, x), f"panel range max err {ey:.3e}"
    assert ew <= _bound(PANEL, a, psi), f"panel co-range max err {ew:.3e}"


def _residuals(A, U, S, V, count):
    """max_i ||A v_i - s_i u_i|| and max_i ||A^T u_i - s_i v_i|| over the first count triplets (FP64)."""
    Ut = torch.from_numpy(U[:, :count]).cuda()
    Vt = torch.from_numpy(V[:, :count]).cuda()
    St = torch.from_numpy(S[:count]).cuda()
    av = torch.zeros(M, count, dtype=torch.float64, device="cuda")
    atu = torch.zeros(N, count, dtype=torch.float64, device="cuda")
    for r0 in range(0, M, 8192):
        blk = A[r0:r0 + 8192].double()
        av[r0:r0 + 8192] = blk @ Vt
        atu += blk.t() @ Ut[r0:r0 + 8192]
    ra = torch.linalg.norm(av - Ut * St, dim=0).max().item()
    rb = torch.linalg.norm(atu - Vt * St, dim=0).max().item()
    return ra, rb


def _orth_err(Q):
    return np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1])))


@pytest.mark.parametrize("v, bound", [(3, 2e-4), (6, 1e-5)])
def test_full_size_subspace_triplets(A, solves, v, bound):
    U, S, V = solves[v]
    assert np.all(np.diff(S) <= 0)
    assert _orth_err(U) <= 2e-5 and _orth_err(V) <= 2e-5
    ra, rb = _residuals(A, U, S, V, 10)
    say(f"full size: v={v} residuals {ra:.2e} {rb:.2e}")
    assert max(ra, rb) <= bound


def test_full_size_subspace_bounds_and_decay(solves):
    S6 = solves[6][1]
    # Weyl: sigma_i(A) is within the noise norm of the prescribed sigma_i; at six views
    # the top 50 have converged far below that
    assert np.max(np.abs(S6[:50] - SIGMA[:50])) <= NOISE_NORM
    errs = {}
    for v in (2, 3, 4, 5):
        Sv = solves[v][1]
        # Rayleigh-Ritz lower bounds: no estimate exceeds the converged one beyond FP32 rounding
        assert np.all(Sv[:K] <= S6[:K] * (1 + 2e-4) + 1e-7), f"v={v} exceeds the six-view values"
        errs[v] = np.max((S6[:50] - Sv[:50]) / S6[:50])
    say("full size: top-50 gaps to v=6:", {v: f"{e:.2e}" for v, e in errs.items()})
    assert errs[2] > errs[3] > errs[4]
    assert errs[2] <= 0.3 and errs[3] <= 3e-2 and errs[4] <= 2e-3 and errs[5] <= 3e-4


def test_full_size_krylov_and_one_view_agree(A, solves):
    S6 = solves[6][1]
    say("full size: block Krylov v=6")
    _, Sk, _ = rs.block_krylov(A, K, P, 6, seed=SEED)
    Sk = Sk.double().cpu().numpy()
    assert np.max(np.abs(Sk[:50] - S6[:50]) / S6[:50]) <= 2e-4
    say("full size: one view (Alg. 7)")
    U1, S1, V1 = (x.double().cpu().numpy() for x in rs.single_pass(A, K, P, seed=SEED))
    assert _orth_err(U1) <= 2e-5 and _orth_err(V1) <= 2e-5
    assert np.max(np.abs(S1[:10] - S6[:10]) / S6[:10]) <= 3e-2
    say("full size: extended one view (Sect. 6.7), s_c = 241")
    U2, S2, V2 = (x.double().cpu().numpy() for x in rs.single_pass(A, K, P, seed=SEED, core_rows=S_W))
    assert _orth_err(U2) <= 2e-5 and _orth_err(V2) <= 2e-5
    e2 = np.max(np.abs(S2[:10] - S6[:10]) / S6[:10])
    say(f"  extended one view: top-10 sigma within {e2:.2e} of six views")
    assert e2 <= 3e-2


# ------------------------------------------------------------ oracle parity

SIGMA_TOL = 1e-4          # FP32 path against the FP64 oracle, relative, every one of the k values
ANGLE_SCALE = 2e-5        # subspace-angle bound: ANGLE_SCALE * sigma_1 / gap_i


@pytest.fixture(scope="module")
def oracle_c2(A):
    say("full size: copying A to the host for the FP64 oracle")
    a_host = A.cpu().numpy()          # the stored FP32 values; the oracle upcasts one block of rows at a time
    t0 = time.time()
    sub = orsvd.alg2_every_view_count(a_host, K, P, 6, SEED)
    say(f"  oracle Alg. 2, v = 2..6: {time.time() - t0:.1f} s")
    t0 = time.time()
    one = orsvd.alg7_one_view(a_host, K, P, SEED, s_w=S_W)
    say(f"  oracle Alg. 7, s_w = {S_W}: {time.time() - t0:.1f} s")
    del a_host
    return sub, one


def _gaps(S):
    d = np.abs(np.diff(S))
    g = np.full(S.shape, np.inf)
    g[:-1] = np.minimum(g[:-1], d)
    g[1:] = np.minimum(g[1:], d)
    return g


def _angles(got, ref):
    """sin of the angle between matching columns (both unit vectors)."""
    c = np.abs(np.sum(got * ref, axis=0)) / (np.linalg.norm(got, axis=0) * np.linalg.norm(ref, axis=0))
    return np.sqrt(np.maximum(0.0, 1.0 - np.minimum(1.0, c) ** 2))


def _check_against_oracle(what, U, S, V, ref):
    rel = np.abs(S - ref.S) / ref.S
    bound = np.minimum(1.0, ANGLE_SCALE * ref.S[0] / _gaps(ref.S))
    au, av = _angles(U, ref.U), _angles(V, ref.V)
    say(f"  {what}: sigma rel err max {rel.max():.2e} (at i = {int(rel.argmax())}); "
        f"worst angle / bound: U {np.max(au / bound):.2e}, V {np.max(av / bound):.2e}; "
        f"top-10 angles U {au[:10].max():.2e} V {av[:10].max():.2e}")
    assert rel.max() <= SIGMA_TOL, f"{what}: sigma differs from the oracle by {rel.max():.3e}"
    assert np.all(au <= bound), f"{what}: left vectors off the oracle's (index {int(np.argmax(au / bound))})"
    assert np.all(av <= bound), f"{what}: right vectors off the oracle's (index {int(np.argmax(av / bound))})"


@pytest.mark.parametrize("v", [2, 3, 4, 5, 6])
def test_full_size_subspace_matches_oracle(solves, oracle_c2, v):
    U, S, V = solves[v]
    _check_against_oracle(f"Alg. 2, v = {v}", U, S, V, oracle_c2[0][v])


def test_full_size_one_view_matches_oracle(A, oracle_c2):
    say("full size: one view (Alg. 7), s_w = 241, against the oracle")
    U, S, V = (x.double().cpu().numpy() for x in rs.single_pass(A, K, P, seed=SEED))
    _check_against_oracle("Alg. 7", U, S, V, oracle_c2[1])
