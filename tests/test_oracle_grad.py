"""Pins of the reference gradient (oracle/grad.py) from outside it: its
forward values equal the numpy oracle of the row sweep, and its directional
derivatives equal central finite differences of that numpy oracle along 64
Philox directions (||E_t||_F = 1, h = 1e-6 ||A||_F), FP64 throughout."""

import numpy as np
import pytest

import synth
from oracle import grad as ograd
from oracle import philox as ophilox
from oracle import rsvd as orsvd

torch = pytest.importorskip("torch")

SEED = synth.METHOD_SEED
TAG_FD = 19


def _loss_numpy(a, k, p, v, w):
    res = orsvd.row_sweep_krylov(a, k, p, v, SEED, tau=2.0 ** -40)
    qc = res.Qc
    b = qc.T @ a
    e = float(np.sum(a * a) - np.sum(b * b))
    return float(np.dot(w, res.S)) + e, res.S, e


def _direction(t, m, n):
    g = ophilox.gaussian(SEED, TAG_FD, t, np.arange(m)[:, None], np.arange(n)[None, :])
    return g / np.linalg.norm(g)


@pytest.mark.parametrize("v", [1, 2, 3])
def test_reference_forward_matches_numpy_oracle(v):
    m, n, k, p = 150, 100, 6, 4
    sigma = np.arange(1, 101, dtype=np.float64) ** -1.0
    a = synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 5)
    w = ograd.loss_weights(k)
    l_np, s_np, e_np = _loss_numpy(a, k, p, v, w)
    sig, e = ograd.row_sweep_outputs(torch.from_numpy(a), k, p, v, SEED)
    np.testing.assert_allclose(sig.numpy(), s_np, rtol=1e-12)
    assert abs(float(e) - e_np) <= 1e-10 * abs(e_np)


@pytest.mark.parametrize("v", [2, 3])
def test_reference_gradient_matches_finite_differences(v):
    m, n, k, p = 150, 100, 6, 4
    sigma = np.arange(1, 101, dtype=np.float64) ** -1.0
    a = synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 5)
    w = ograd.loss_weights(k)
    g, _, _ = ograd.reference_gradient(a, k, p, v, SEED)
    h = 1e-6 * np.linalg.norm(a)
    worst = 0.0
    for t in range(64):
        d = _direction(t, m, n)
        lp = _loss_numpy(a + h * d, k, p, v, w)[0]
        lm = _loss_numpy(a - h * d, k, p, v, w)[0]
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(g * d))
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    assert worst <= 1e-6, f"worst relative FD mismatch {worst:.2e}"


def test_reference_gradient_special_case_full_space():
    """s = min(m, n): Q_c spans the whole column space, so E = 0 and sigma are
    the exact singular values; the gradient of sum w_i sigma_i is then the
    classical sum w_i u_i v_i^T (distinct singular values)."""
    m, n, k, p = 40, 12, 6, 6
    sigma = np.linspace(3.0, 0.5, 12)
    a = synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 7)
    g, sig, e = ograd.reference_gradient(a, k, p, 1, SEED, de=0.0)
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    w = ograd.loss_weights(k)
    np.testing.assert_allclose(sig, s[:k], rtol=1e-12)
    assert abs(e) <= 1e-12 * np.sum(a * a)
    np.testing.assert_allclose(g, (u[:, :k] * w[None, :]) @ vt[:k], atol=1e-10)
