"""GPU: the hand-written adjoint of the row-sweep block Krylov method.

Reference: oracle/grad.py (FP64 torch autograd on the CPU through a plain
implementation, itself pinned by finite differences of the numpy oracle).
Tolerances, relative Frobenius norm of the gradient: 1e-8 on the FP64 path,
1e-3 on the FP32 path; forward sigma and E: 1e-10 (FP64).  The GPU forward
is also checked by central differences of itself (FP64) along Philox
directions, independently of the adjoint.
"""

import sys

import numpy as np
import pytest

import synth
from oracle import grad as ograd
from oracle import philox as ophilox

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1804_07531_amd as rs  # noqa: E402
from paper_1804_07531_amd.autograd import row_sweep_svd  # noqa: E402

DEV = torch.device("cuda:0")
SEED = synth.METHOD_SEED


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _matrix(m, n, power, seed):
    r = min(m, n)
    sigma = np.arange(1, r + 1, dtype=np.float64) ** -power
    return synth.spectral_matrix(m, n, sigma, seed)


def _gpu_grad(A_np, k, p, v, dtype, dE=1.0, block_rows=1024):
    A = torch.from_numpy(A_np).to(DEV, dtype).requires_grad_(True)
    S, E, U, V = row_sweep_svd(A, k, p, v, SEED, block_rows)
    w = torch.from_numpy(ograd.loss_weights(k)).to(DEV)
    loss = (w * S).sum() + dE * E
    (G,) = torch.autograd.grad(loss, A)
    return G.double().cpu().numpy(), S.detach().cpu().numpy(), float(E.detach())


@pytest.mark.parametrize("shape", [(300, 200, 6, 4, 1), (300, 200, 6, 4, 2), (300, 200, 6, 4, 3),
                                   (1000, 700, 16, 8, 4), (700, 1000, 10, 6, 3), (2048, 1024, 64, 16, 4)])
@pytest.mark.parametrize("dE", [1.0, 0.0])
def test_gradient_fp64_matches_reference(shape, dE):
    m, n, k, p, v = shape
    say(f"grad fp64 {shape} dE={dE}")
    A = _matrix(m, n, 1.0, synth.GEN_SEED + 5)
    Gref, sref, eref = ograd.reference_gradient(A, k, p, v, SEED, de=dE)
    G, S, E = _gpu_grad(A, k, p, v, torch.float64, dE=dE, block_rows=256)
    rel = np.linalg.norm(G - Gref) / np.linalg.norm(Gref)
    say(f"  sigma {np.max(np.abs(S - sref) / sref):.2e} E {abs(E - eref) / abs(eref):.2e} grad {rel:.2e}")
    assert np.max(np.abs(S - sref) / sref) <= 1e-10
    assert abs(E - eref) <= 1e-10 * abs(eref)
    assert rel <= 1e-8


# (700, 1000, 10, 5, 3): panel row counts 10, 45, 45, 30 leave ragged steps of
# the register-fed FP32 assembly; (1001, 703, ...): rows not on 16-byte
# boundaries take the LDS-staged assembly
@pytest.mark.parametrize("shape", [(1000, 700, 16, 8, 4), (2048, 1024, 64, 16, 4), (700, 1000, 10, 5, 3),
                                   (1001, 703, 8, 4, 3)])
def test_gradient_fp32_matches_reference(shape):
    m, n, k, p, v = shape
    say(f"grad fp32 {shape}")
    A = _matrix(m, n, 1.0, synth.GEN_SEED + 5).astype(np.float32).astype(np.float64)
    Gref, sref, eref = ograd.reference_gradient(A, k, p, v, SEED)
    G, S, E = _gpu_grad(A, k, p, v, torch.float32)
    rel = np.linalg.norm(G - Gref) / np.linalg.norm(Gref)
    say(f"  sigma {np.max(np.abs(S - sref) / sref):.2e} E {abs(E - eref) / abs(eref):.2e} grad {rel:.2e}")
    assert rel <= 1e-3


def test_gpu_forward_finite_differences():
    """<G, D_t> against central differences of the GPU FP64 forward itself."""
    m, n, k, p, v = 400, 300, 8, 4, 3
    A = _matrix(m, n, 1.0, synth.GEN_SEED + 8)
    G, _, _ = _gpu_grad(A, k, p, v, torch.float64)
    w = torch.from_numpy(ograd.loss_weights(k)).to(DEV)
    # the GPU FP64 forward carries about 1e-13 relative rounding (Jacobi, CholeskyQR): with
    # h = 1e-5 ||A|| that is about 1e-7 in the quotient, the truncation error about 1e-10
    h = 1e-5 * np.linalg.norm(A)

    def loss(X):
        S, E, _, _ = row_sweep_svd(torch.from_numpy(X).to(DEV), k, p, v, SEED)
        return float((w * S).sum() + E)

    worst = 0.0
    for t in range(8):
        d = ophilox.gaussian(SEED, 19, t, np.arange(m)[:, None], np.arange(n)[None, :])
        d /= np.linalg.norm(d)
        fd = (loss(A + h * d) - loss(A - h * d)) / (2 * h)
        an = float(np.sum(G * d))
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    say(f"  worst FD mismatch {worst:.2e}")
    assert worst <= 1e-6


def test_forward_matches_block_krylov_row_sweep():
    m, n, k, p, v = 1000, 700, 16, 8, 3
    A = torch.from_numpy(_matrix(m, n, 1.0, synth.GEN_SEED + 5)).to(DEV)
    S1, E, U1, V1 = row_sweep_svd(A, k, p, v, SEED)
    U2, S2, V2 = rs.block_krylov(A, k, p, v, mode="row", seed=SEED)
    assert torch.allclose(S1, S2, rtol=1e-12, atol=0)
    assert torch.allclose(U1, U2, rtol=0, atol=1e-10) and torch.allclose(V1, V2, rtol=0, atol=1e-10)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(1000, 700, 16, 8, 4), (2048, 1024, 64, 16, 4)])
def test_kept_small_svds_equal_recomputed(shape, dtype):
    """The backward with the forward's small SVDs carried over (keep_mode 2 after
    a keep_mode 1 forward) equals the backward that recomputes them, bit for bit."""
    from paper_1804_07531_amd import autograd as ag
    m, n, k, p, v = shape
    say(f"kept small SVDs {shape} {dtype}")
    A = torch.from_numpy(_matrix(m, n, 1.0, synth.GEN_SEED + 6)).to(DEV, dtype)
    dS = torch.from_numpy(ograd.loss_weights(k)).to(DEV)
    _, _, _, _, G0 = ag._call(A, k, p, v, SEED, 1024, dS=dS, dE=1.0, want_grad=True)
    kept = ag.kept_record(k, p, v, DEV)
    S1, E1, _, _, _ = ag._call(A, k, p, v, SEED, 1024, kept=kept, keep_mode=1)
    _, _, _, _, G2 = ag._call(A, k, p, v, SEED, 1024, dS=dS, dE=1.0, want_grad=True, kept=kept, keep_mode=2)
    torch.cuda.synchronize()
    assert torch.equal(G0, G2)
    S0, E0, _, _, _ = ag._call(A, k, p, v, SEED, 1024)
    assert torch.equal(S0, S1) and torch.equal(E0, E1)
