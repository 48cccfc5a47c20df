"""Differentiable row-sweep block Krylov SVD (Sect. 7.3) behind
torch.autograd.Function.

    S, E, U, V = RowSweepSVD.apply(A, k, p, v, seed, block_rows)

S (k,) are the leading singular values the method returns and
E = ||A - Q_c Q_c^T A||_F^2 with Q_c its range basis; both are
differentiable in A with the Gaussian test matrix held fixed by `seed`.
U and V are returned without gradients.  The backward calls the library's
hand-written adjoint (rsvd_block_krylov_grad_kept), which recomputes the
sketches on the GPU instead of storing them; only the two small SVDs of the
forward (2 (2 s_K^2 + s_K) FP64 values, s_K = v (k + p)) are carried from
the forward to the backward.  This module only marshals tensors.
"""

import ctypes

import torch

from . import _lib
from . import _mat, _opts, _stream, lib


def _call(A, k, p, v, seed, block_rows, dS=None, dE=0.0, want_grad=False, kept=None, keep_mode=0):
    mat = _mat(A)
    o = _opts(seed=seed, mode="row", block_rows=block_rows)
    L = lib()
    need = L.rsvd_grad_workspace_bytes(ctypes.byref(mat), k, p, v, ctypes.byref(o), int(want_grad))
    if need == 0:
        raise _lib.RsvdError(1, "rsvd_block_krylov_grad: invalid arguments")
    ws = torch.empty(need, dtype=torch.uint8, device=A.device)
    out_dtype = A.dtype
    m, n = A.shape
    U = torch.empty(m, k, dtype=out_dtype, device=A.device)
    V = torch.empty(n, k, dtype=out_dtype, device=A.device)
    S = torch.empty(k, dtype=torch.float64, device=A.device)
    E = torch.empty((), dtype=torch.float64, device=A.device)
    out = _lib.RsvdOut(U.data_ptr(), S.data_ptr(), V.data_ptr())
    G = torch.empty_like(A) if want_grad else None
    ds_ptr = None
    if dS is not None:
        dS = dS.to(device=A.device, dtype=torch.float64).contiguous()
        ds_ptr = dS.data_ptr()
    code = L.rsvd_block_krylov_grad_kept(ctypes.byref(mat), k, p, v, ctypes.byref(o), ctypes.byref(out),
                                         ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(ds_ptr), ctypes.c_double(dE),
                                         ctypes.c_void_p(G.data_ptr() if G is not None else None),
                                         ctypes.c_int64(n),
                                         ctypes.c_void_p(kept.data_ptr() if kept is not None else None),
                                         keep_mode, ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(need), _stream())
    _lib.check(code, "rsvd_block_krylov_grad_kept")
    # the adjoint assumes K at full numerical rank (a cut of R_K's TSVD sets FLAG_TRUNCATED), and a
    # non-finite value or a timed-out small-SVD barrier invalidates the result: raise on any of them
    flags = ctypes.c_uint32(0)
    status = L.rsvd_device_status(ctypes.c_void_p(ws.data_ptr()), _stream(), ctypes.byref(flags))
    bad = flags.value & (_lib.FLAG_NONFINITE | _lib.FLAG_TRUNCATED | _lib.FLAG_SYNC_TIMEOUT)
    if status != _lib.RSVD_OK or bad:
        raise _lib.RsvdError(status if status != _lib.RSVD_OK else _lib.RSVD_EBREAKDOWN,
                             "rsvd_block_krylov_grad_kept", flags.value)
    return S, E, U, V, G


def kept_record(k, p, v, device):
    """Device FP64 buffer for the small SVDs carried from forward to backward."""
    count = lib().rsvd_grad_kept_doubles(k, p, v)
    if count == 0:
        raise _lib.RsvdError(1, "rsvd_grad_kept_doubles: invalid sizes")
    return torch.empty(count, dtype=torch.float64, device=device)


class RowSweepSVD(torch.autograd.Function):
    """(S, E, U, V) of the row-sweep method; gradients flow through S and E."""

    @staticmethod
    def forward(ctx, A, k, p, v, seed=0, block_rows=1024):
        if A.dim() != 2 or A.stride(1) != 1:
            raise ValueError("A must be a 2-D tensor with unit stride along its rows")
        kept = kept_record(k, p, v, A.device)
        S, E, U, V, _ = _call(A, k, p, v, seed, block_rows, kept=kept, keep_mode=1)
        ctx.save_for_backward(A)
        ctx.kept = kept
        ctx.args = (k, p, v, seed, block_rows)
        ctx.mark_non_differentiable(U, V)
        return S, E, U, V

    @staticmethod
    def backward(ctx, dS, dE, dU, dV):
        (A,) = ctx.saved_tensors
        k, p, v, seed, block_rows = ctx.args
        de = float(dE) if dE is not None else 0.0
        _, _, _, _, G = _call(A, k, p, v, seed, block_rows, dS=dS, dE=de, want_grad=True, kept=ctx.kept,
                              keep_mode=2)
        ctx.kept = None
        return G, None, None, None, None, None


def row_sweep_svd(A, k, p, v, seed=0, block_rows=1024):
    return RowSweepSVD.apply(A, k, p, v, seed, block_rows)
