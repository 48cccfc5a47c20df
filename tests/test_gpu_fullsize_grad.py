"""GPU checks of the differentiable row sweep at its full benchmark size: A is
32768 x 8192 FP32 with sigma_j = j^-1 and full Haar factors, k = 64, p = 16,
v = 4, 1024-row blocks; loss = sum_i w_i sigma_i + ||A - Q_c Q_c^T A||_F^2
with w_i = (k - i + 1) / k, Omega held fixed.

- The FP32 gradient, computed as the benchmark computes it, is compared with
  the oracle's FP64 reference gradient on the same stored values (relative
  Frobenius norm 1e-3), and the FP64 gradient with it at 1e-8.
- Central differences of the GPU FP64 forward along 64 Gaussian directions
  are compared with <G, D>. A random unit direction sees about
  ||G||_F / sqrt(mn) of the gradient, so the mismatch is measured in that
  unit (the forward's rounding, about 1e-14 of the loss, over the step h,
  is a few 1e-6 of it; the bound is 1e-3).
"""

import sys

import numpy as np
import pytest

import synth
from oracle import grad as ograd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1804_07531_amd.autograd import row_sweep_svd  # noqa: E402

M, N, K, P, V, ROWS = 32768, 8192, 64, 16, 4, 1024
SEED = synth.METHOD_SEED


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    say(f"full size grad: building {M}x{N} FP32 A (sigma_j = j^-1, full rank)")
    sigma = np.arange(1, N + 1, dtype=np.float64) ** -1.0
    a = synth.spectral_matrix_torch(M, N, sigma, synth.GEN_SEED + 5, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    yield a
    del a
    torch.cuda.empty_cache()


def _weights(dev):
    return torch.from_numpy(ograd.loss_weights(K)).to(dev)


def _grad(A):
    Ar = A.detach().requires_grad_(True)
    S, E, _, _ = row_sweep_svd(Ar, K, P, V, SEED, ROWS)
    (G,) = torch.autograd.grad((_weights(A.device) * S).sum() + E, Ar)
    return G


def test_full_size_gradient_matches_oracle(A):
    say("full size grad: FP32 and FP64 gradients on the GPU")
    G32 = _grad(A).double().cpu().numpy()
    G64 = _grad(A.double()).cpu().numpy()
    say("full size grad: oracle reference gradient (FP64, CPU)")
    Gref, _, _ = ograd.reference_gradient(A.double().cpu().numpy(), K, P, V, SEED)
    nref = np.linalg.norm(Gref)
    r32 = np.linalg.norm(G32 - Gref) / nref
    r64 = np.linalg.norm(G64 - Gref) / nref
    say(f"full size grad: relative Frobenius error FP32 {r32:.2e}, FP64 {r64:.2e}")
    assert r32 <= 1e-3
    assert r64 <= 1e-8


def test_full_size_forward_finite_differences(A):
    A64 = A.double()
    w = _weights(A64.device)
    G = _grad(A64)
    unit = (torch.linalg.norm(G) / np.sqrt(M * N)).item()
    h = 1e-5 * torch.linalg.norm(A64).item()

    def loss(X):
        S, E, _, _ = row_sweep_svd(X, K, P, V, SEED, ROWS)
        return float((w * S).sum() + E)

    gen = torch.Generator(device="cuda")
    gen.manual_seed(21)
    worst = 0.0
    for t in range(64):
        d = torch.randn(M, N, generator=gen, device="cuda", dtype=torch.float64)
        d /= torch.linalg.norm(d)
        fd = (loss(A64 + h * d) - loss(A64 - h * d)) / (2 * h)
        an = torch.sum(G * d).item()
        worst = max(worst, abs(fd - an) / unit)
        del d
    say(f"full size grad: worst FD mismatch over 64 directions {worst:.2e} (unit ||G||/sqrt(mn) = {unit:.2e})")
    assert worst <= 1e-3
