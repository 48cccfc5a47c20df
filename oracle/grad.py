"""Reference gradient of the row-sweep block Krylov method (Sect. 7.3), in
FP64 with PyTorch autograd on the CPU.

TEST INFRASTRUCTURE ONLY (see the package header).

The forward follows ``rsvd.row_sweep_krylov`` step by step, with the same
Philox test matrix held fixed, written in torch so that autograd can
differentiate it:

    X_0 = orth(Omega); for j = 1..v: Y_j = A X_{j-1}, Z_j = A^T Y_j and, for
    j < v, X_j = orth of Z_j projected twice off span[X_0 .. X_{j-1}];
    K = [Y_1 .. Y_v]; Q_c = an orthonormal basis of range(K); B = Q_c^T A.

The outputs are sigma = the k leading singular values of B (those the
method returns, since R_r's singular values are B's) and
E = ||A - Q_c Q_c^T A||_F^2 = ||A||_F^2 - ||B||_F^2.  Q_c is taken from the
QR of K directly: the TSVD of R_K in the method only rotates the basis (no
column is cut at full numerical rank), which changes neither sigma nor E.

The loss of the differentiation workload is L = sum_i w_i sigma_i + E with
w_i = (k - i + 1) / k (i = 1..k).

Pinned by: central finite differences of the numpy oracle
(``rsvd.row_sweep_krylov`` plus E) along Philox directions, and by the
forward values matching that oracle.
"""

import numpy as np
import torch

from . import philox


def _orth(x):
    q, r = torch.linalg.qr(x)
    d = torch.sign(torch.diagonal(r))
    d = torch.where(d == 0, torch.ones_like(d), d)
    return q * d[None, :]


def row_sweep_outputs(a, k, p, v, seed):
    """(sigma[:k], E) of the row-sweep method as differentiable functions of
    the FP64 CPU tensor a (m x n)."""
    m, n = a.shape
    s = k + p
    omega = torch.from_numpy(philox.omega(seed, n, s)).to(torch.float64)
    xs = [_orth(omega)]
    ys = []
    for j in range(1, v + 1):
        x = xs[-1]
        y = a @ x
        z = a.T @ y
        ys.append(y)
        if j < v:
            basis = torch.cat(xs, dim=1)
            w = z - basis @ (basis.T @ z)
            w = w - basis @ (basis.T @ w)
            xs.append(_orth(w))
    kmat = torch.cat(ys, dim=1)
    qc, _ = torch.linalg.qr(kmat)
    b = qc.T @ a
    sig = torch.linalg.svdvals(b)
    e = (a * a).sum() - (b * b).sum()
    return sig[:k], e


def loss_weights(k):
    """w_i = (k - i + 1) / k, i = 1..k."""
    return (k - np.arange(k)) / float(k)


def reference_gradient(a_np, k, p, v, seed, dsig=None, de=1.0):
    """Gradient of sum_i dsig_i sigma_i + de E with respect to A (FP64),
    with the forward values (sigma, E)."""
    a = torch.from_numpy(np.asarray(a_np, dtype=np.float64)).clone().requires_grad_(True)
    sig, e = row_sweep_outputs(a, k, p, v, seed)
    w = torch.from_numpy(loss_weights(k) if dsig is None else np.asarray(dsig, dtype=np.float64))
    loss = (w * sig).sum() + de * e
    loss.backward()
    return a.grad.numpy().copy(), sig.detach().numpy().copy(), float(e.detach())
