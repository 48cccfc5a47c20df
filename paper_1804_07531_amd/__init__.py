"""Pass-efficient randomized low-rank SVD on MI355X (gfx950).

Thin Python binding of the C ABI in include/rsvd.h: it only marshals torch
tensors (device memory) and the current HIP stream into the library's
arguments.  Every step of every algorithm runs in the library's HIP kernels;
there is no CPU or PyTorch fallback.

    U, S, V = subspace(A, k, p, v, seed=...)        # Alg. 2, any v >= 2 views
    U, S, V = single_pass(A, k, p, seed=...)        # Alg. 7, one view
    U, S, V = block_krylov(A, k, p, v, mode="row")  # Alg. 9 / row-sweep Krylov (Sect. 7)

A is a 2-D CUDA tensor with unit stride along its rows: float64, float32,
bfloat16, or float8_e4m3fn together with row_scale (one float32 per stored
row); trans=True passes A^T's storage (the result is still the SVD of the
logical A).  U (m x k) and V (n x k) come back in float64 for a float64 A and
float32 otherwise; S (k,) is float64, descending.

Options: seed, refine (BF16/FP8 A: the last view is FP32-accurate; default
on for those types), f32_mode (F32_MFMA or F32_BF16X6 for float32 A),
mode / block_rows / psi_rows / trunc_tau / core_rows as in include/rsvd.h.
single_pass also takes method ("tropp": Alg. 7, "woolfe": Alg. 8) and lc
(None: l_c = p; an integer; ("ratio", alpha); or "minvar"), and core_kind
("gaussian" or "srft") with core_rows.

Device-side failures (a non-finite singular value, a small-SVD barrier that
timed out) are recorded in the call's workspace.  check=True makes a call
wait for its stream and raise RsvdError when one was recorded; without it the
call returns at once and device_status(workspace) reads the word later.
"""

import ctypes

from . import _lib
from ._lib import (ALGO_BLOCK_KRYLOV, ALGO_SINGLE_PASS, ALGO_SUBSPACE, CORE_GAUSSIAN, CORE_SRFT, F32_BF16X6, F32_MFMA,
                   KRYLOV_ALTERNATING, KRYLOV_COL_SWEEP, KRYLOV_ROW_SWEEP, LC_FIXED, LC_FULL, LC_MINVAR, LC_RATIO,
                   ONE_VIEW_TROPP, ONE_VIEW_WOOLFE, RSVD_BF16, RSVD_F32, RSVD_F64, RSVD_FP8_E4M3, RSVD_OK, RsvdError,
                   RsvdMat, RsvdOpts, RsvdOut, RsvdViewTrace)

__all__ = ["subspace", "single_pass", "block_krylov", "gaussian", "view_range", "view_corange", "BatchPlan",
           "StreamSketch", "normal_tevd", "extended_sizes",
           "philox_words", "workspace_bytes", "device_status", "one_view_lc", "RsvdError", "RsvdViewTrace",
           "ViewTimer", "lib", "F32_MFMA", "F32_BF16X6"]


def lib():
    return _lib.load()


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return RSVD_F64
    if t.dtype == torch.float32:
        return RSVD_F32
    if t.dtype == torch.bfloat16:
        return RSVD_BF16
    if t.dtype == torch.float8_e4m3fn:
        return RSVD_FP8_E4M3
    raise TypeError(f"unsupported dtype {t.dtype}")


def _low_precision(A):
    return _dtype_code(A) in (RSVD_BF16, RSVD_FP8_E4M3)


def _mat(A, trans=False, row_scale=None):
    torch = _torch()
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D CUDA tensor")
    if A.stride(1) != 1:
        raise ValueError("A must have unit stride along its rows")
    rows, cols = A.shape
    m, n = (cols, rows) if trans else (rows, cols)
    scale_ptr = None
    if row_scale is not None:
        if row_scale.dtype != torch.float32 or not row_scale.is_cuda or row_scale.numel() != rows:
            raise ValueError("row_scale must be a float32 CUDA tensor with one entry per stored row")
        if not row_scale.is_contiguous():
            raise ValueError("row_scale must be contiguous")
        scale_ptr = row_scale.data_ptr()
    return RsvdMat(_dtype_code(A), m, n, A.stride(0), int(bool(trans)), A.data_ptr(), scale_ptr)


_MODES = {"alternating": KRYLOV_ALTERNATING, "row": KRYLOV_ROW_SWEEP, "col": KRYLOV_COL_SWEEP}


_METHODS = {"tropp": ONE_VIEW_TROPP, "woolfe": ONE_VIEW_WOOLFE}
_CORES = {"gaussian": CORE_GAUSSIAN, "srft": CORE_SRFT}


def _lc_fields(lc):
    """(lc_rule, lc, lc_alpha) of the one-view l_c choice: None (l_c = p), an
    integer, ("ratio", alpha) or "minvar"."""
    if lc is None:
        return LC_FULL, 0, 0.0
    if isinstance(lc, str):
        if lc != "minvar":
            raise ValueError("lc must be None, an integer, ('ratio', alpha) or 'minvar'")
        return LC_MINVAR, 0, 0.0
    if isinstance(lc, tuple):
        if len(lc) != 2 or lc[0] != "ratio":
            raise ValueError("lc must be None, an integer, ('ratio', alpha) or 'minvar'")
        return LC_RATIO, 0, float(lc[1])
    return LC_FIXED, int(lc), 0.0


def _opts(seed=0, mode="alternating", block_rows=1024, psi_rows=0, trunc_tau=0.0, trace=None, refine=0,
          f32_mode=F32_MFMA, core_rows=0, method="tropp", lc=None, core_kind="gaussian", sync_spins=0):
    o = RsvdOpts()
    lib().rsvd_default_opts(ctypes.byref(o))
    o.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    o.refine = int(refine)
    o.f32_mode = int(f32_mode)
    o.krylov_mode = _MODES[mode] if isinstance(mode, str) else int(mode)
    o.block_rows = int(block_rows)
    o.psi_rows = int(psi_rows)
    o.trunc_tau = float(trunc_tau)
    o.core_rows = int(core_rows)
    o.one_view_method = _METHODS[method] if isinstance(method, str) else int(method)
    o.lc_rule, o.lc, o.lc_alpha = _lc_fields(lc)
    o.core_kind = _CORES[core_kind] if isinstance(core_kind, str) else int(core_kind)
    o.sync_spins = int(sync_spins)
    if trace is not None:
        o.trace = ctypes.pointer(trace)
    return o


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _fill_refine(A, opts):
    if opts.get("refine") is None:
        opts["refine"] = 1 if _low_precision(A) else 0
    return opts


def workspace_bytes(A, k, p, v, algo, trans=False, row_scale=None, **opts):
    mat = _mat(A, trans, row_scale)
    o = _opts(**_fill_refine(A, opts))
    return lib().rsvd_workspace_bytes(ctypes.byref(mat), k, p, v, algo, ctypes.byref(o))


def _check_device(workspace, where):
    """Waits for the stream and raises RsvdError if the call recorded a device-side failure."""
    code, flags = device_status(workspace)
    if code != RSVD_OK:
        raise RsvdError(code, where, flags)


def _run(entry, algo, A, k, p, v, trans, workspace, opts):
    torch = _torch()
    row_scale = opts.pop("row_scale", None)
    check = bool(opts.pop("check", False))
    mat = _mat(A, trans, row_scale)
    o = _opts(**_fill_refine(A, opts))
    L = lib()
    need = L.rsvd_workspace_bytes(ctypes.byref(mat), k, p, v, algo, ctypes.byref(o))
    if need == 0:
        # let the entry point report the precise argument error
        need = 256
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
    out_dtype = torch.float64 if A.dtype == torch.float64 else torch.float32
    U = torch.empty(mat.m, k, dtype=out_dtype, device=A.device)
    V = torch.empty(mat.n, k, dtype=out_dtype, device=A.device)
    S = torch.empty(k, dtype=torch.float64, device=A.device)
    out = RsvdOut(U.data_ptr(), S.data_ptr(), V.data_ptr())
    code = getattr(L, entry)(ctypes.byref(mat), k, p, v, ctypes.byref(o), ctypes.byref(out),
                             ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()), _stream())
    _lib.check(code, entry)
    if check:
        _check_device(workspace, entry)
    return U, S, V, workspace


def subspace(A, k, p, v, trans=False, workspace=None, return_workspace=False, **opts):
    """Alg. 2: generalized randomized subspace iteration with v >= 2 views."""
    U, S, V, ws = _run("rsvd_subspace", ALGO_SUBSPACE, A, k, p, v, trans, workspace, opts)
    return (U, S, V, ws) if return_workspace else (U, S, V)


def single_pass(A, k, p, trans=False, workspace=None, return_workspace=False, **opts):
    """Alg. 7 (method='tropp') or Alg. 8 (method='woolfe'): one-view method
    (Psi has 2(k+p)+1 rows unless psi_rows is given), with l_c chosen by lc
    (Sect. 6.6).  With core_rows = s_c > 0: the extended one-view sketch of
    Sect. 6.7 with the improved reconstruction (Psi has k+p rows; core test
    matrices Gaussian or, with core_kind='srft', the paper's SRFTs)."""
    U, S, V, ws = _run("rsvd_single_pass", ALGO_SINGLE_PASS, A, k, p, 1, trans, workspace, opts)
    return (U, S, V, ws) if return_workspace else (U, S, V)


def block_krylov(A, k, p, v, mode="alternating", trans=False, workspace=None, return_workspace=False, **opts):
    """Alg. 9 (mode='alternating') or the row/column-sweep Krylov of Sect. 7.3."""
    opts["mode"] = mode
    U, S, V, ws = _run("rsvd_block_krylov", ALGO_BLOCK_KRYLOV, A, k, p, v, trans, workspace, opts)
    return (U, S, V, ws) if return_workspace else (U, S, V)


def device_status(workspace):
    """Synchronizes the current stream and returns the raw status word of the last call."""
    flags = ctypes.c_uint32(0)
    code = lib().rsvd_device_status(ctypes.c_void_p(workspace.data_ptr()), _stream(), ctypes.byref(flags))
    return code, flags.value


_NORMAL = {"nystrom": _lib.NORMAL_NYSTROM, "pinched": _lib.NORMAL_PINCHED, "subspace": _lib.NORMAL_SUBSPACE}


def normal_tevd(J, k, p, v, method="nystrom", trans=False, workspace=None, return_workspace=False, check=False,
                **opts):
    """Truncated eigendecomposition J^T J ~ V diag(lam2) V^T from v >= 2 views of
    J (Sect. 4.2): method 'nystrom' (Alg. 4), 'pinched' (Alg. 5) or 'subspace'
    (Alg. 2 on J or J^T by the rule of Sect. 4.2.1).  Returns (V, lam2)."""
    torch = _torch()
    mat = _mat(J, trans)
    o = _opts(**opts)
    code_m = _NORMAL[method] if isinstance(method, str) else int(method)
    L = lib()
    need = L.rsvd_normal_workspace_bytes(ctypes.byref(mat), k, p, v, code_m, ctypes.byref(o))
    if workspace is None or workspace.numel() < max(need, 256):
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=J.device)
    V = torch.empty(mat.n, k, dtype=torch.float64 if J.dtype == torch.float64 else torch.float32, device=J.device)
    lam2 = torch.empty(k, dtype=torch.float64, device=J.device)
    code = L.rsvd_normal_tevd(ctypes.byref(mat), k, p, v, code_m, ctypes.byref(o), ctypes.c_void_p(V.data_ptr()),
                              ctypes.c_void_p(lam2.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                              ctypes.c_size_t(workspace.numel()), _stream())
    _lib.check(code, "rsvd_normal_tevd")
    if check:
        _check_device(workspace, "rsvd_normal_tevd")
    return (V, lam2, workspace) if return_workspace else (V, lam2)


def extended_sizes(k, budget, m, n):
    """(l1, s_c) of the extended one-view sketch for a storage budget T (eq.
    bwzafac8, Sect. 6.7): call single_pass(A, k, l1, core_rows=s_c, ...)."""
    l1 = ctypes.c_int(0)
    sc = ctypes.c_int64(0)
    _lib.check(lib().rsvd_extended_sizes(int(k), int(budget), int(m), int(n), ctypes.byref(l1), ctypes.byref(sc)),
               "rsvd_extended_sizes")
    return l1.value, sc.value


def one_view_lc(workspace):
    """Synchronizes the current stream and returns the l_c the last one-view
    call with this workspace used (the minimum-variance choice included)."""
    lc = ctypes.c_int(0)
    _lib.check(lib().rsvd_one_view_lc(ctypes.c_void_p(workspace.data_ptr()), _stream(), ctypes.byref(lc)),
               "rsvd_one_view_lc")
    return lc.value


def gaussian(seed, tag, rows, cols, long_is_row, dtype=None, batch=0, device="cuda"):
    """Counter-based Gaussian test matrix (rows x cols) on the device."""
    torch = _torch()
    dtype = dtype or torch.float64
    out = torch.empty(rows, cols, dtype=dtype, device=device)
    code = lib().rsvd_gaussian(int(seed) & 0xFFFFFFFFFFFFFFFF, tag, batch, rows, cols, int(long_is_row),
                               _dtype_code(out), ctypes.c_void_p(out.data_ptr()), cols, _stream())
    _lib.check(code, "rsvd_gaussian")
    return out


def _view(entry, A, thin_panel, out_len, trans=False, row_scale=None, **opts):
    torch = _torch()
    mat = _mat(A, trans, row_scale)
    o = _opts(**opts)
    s = thin_panel.shape[0]
    need = lib().rsvd_view_workspace_bytes(ctypes.byref(mat), s, ctypes.byref(o))
    if need == 0:
        raise RsvdError(6, f"{entry}: no view kernel for these arguments")
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=A.device)
    out = torch.empty(s, out_len, dtype=thin_panel.dtype, device=A.device)
    code = getattr(lib(), entry)(ctypes.byref(mat), s, ctypes.c_void_p(thin_panel.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                                 ctypes.c_size_t(ws.numel()), _stream())
    _lib.check(code, entry)
    return out


def view_range(A, XT, trans=False, row_scale=None, **opts):
    """Y^T = (A X)^T for a panel X^T (s x n); opts: refine, f32_mode."""
    m = A.shape[1] if trans else A.shape[0]
    return _view("rsvd_view_range", A, XT.contiguous(), m, trans, row_scale, **opts)


def view_corange(A, YT, trans=False, row_scale=None, **opts):
    """Z^T = (A^T Y)^T for a panel Y^T (s x m); opts: refine, f32_mode."""
    n = A.shape[0] if trans else A.shape[1]
    return _view("rsvd_view_corange", A, YT.contiguous(), n, trans, row_scale, **opts)


def philox_words(ctr, key0, key1):
    """Raw Philox4x32-10 words for a (4, N) uint32-valued int64 CUDA tensor of counters."""
    torch = _torch()
    c = ctr.to(torch.int32).contiguous()
    out = torch.empty_like(c)
    code = lib().rsvd_philox_words(ctypes.c_void_p(c.data_ptr()), c.shape[1], key0 & 0xFFFFFFFF,
                                   key1 & 0xFFFFFFFF, ctypes.c_void_p(out.data_ptr()), _stream())
    _lib.check(code, "rsvd_philox_words")
    return out.to(torch.int64) & 0xFFFFFFFF


class ViewTimer:
    """Per-view kernel timing through the library's trace hook: HIP events
    recorded on the call's own stream around the kernels of every view (with
    inner=True: around each panel's or block's products inside the one-view
    and row-sweep passes instead of the passes as a whole)."""

    def __init__(self, capacity=64, inner=False):
        self._hip = ctypes.CDLL("libamdhip64.so")
        self.capacity = capacity
        self._events = (ctypes.c_void_p * (2 * capacity))()
        for i in range(2 * capacity):
            code = self._hip.hipEventCreate(ctypes.byref(self._events, i * ctypes.sizeof(ctypes.c_void_p)))
            if code != 0:
                raise RuntimeError(f"hipEventCreate failed ({code})")
        self._kind = (ctypes.c_int * capacity)()
        self.trace = RsvdViewTrace(ctypes.cast(self._events, ctypes.POINTER(ctypes.c_void_p)), capacity, 0,
                                   ctypes.cast(self._kind, ctypes.POINTER(ctypes.c_int)), int(bool(inner)))

    def results(self):
        """[(kind, milliseconds)] of the views of the last traced call (synchronizes on the events)."""
        out = []
        ms = ctypes.c_float(0.0)
        for u in range(self.trace.used):
            end = ctypes.c_void_p(self._events[2 * u + 1])
            self._hip.hipEventSynchronize(end)
            code = self._hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self._events[2 * u]), end)
            if code != 0:
                raise RuntimeError(f"hipEventElapsedTime failed ({code})")
            out.append((int(self._kind[u]), float(ms.value)))
        return out


class StreamSketch:
    """One-view sketches of A = sum_i H_i built from linear updates (Sect. 6.1;
    rsvd_stream_* in include/rsvd.h).

        sk = StreamSketch(m, n, k, p, dtype=torch.float64, seed=..., method="tropp", lc=None)
        sk.add_dense(r0, c0, H)            # H placed at rows r0.., columns c0..
        sk.add_entries(rows, cols, vals)   # sparse entries (repeats add up)
        U, S, V = sk.finish()              # Alg. 7 / Alg. 8 on the current sketches

    All work is enqueued on the current stream; the workspace is allocated here."""

    def __init__(self, m, n, k, p, dtype=None, seed=0, method="tropp", lc=None, psi_rows=0, device="cuda"):
        torch = _torch()
        self.dtype = dtype or torch.float64
        self.m, self.n, self.k = int(m), int(n), int(k)
        self.device = torch.device(device)
        code = RSVD_F64 if self.dtype == torch.float64 else RSVD_F32 if self.dtype == torch.float32 else None
        if code is None:
            raise TypeError("the sketches are float64 or float32")
        L = lib()
        o = _opts(seed=seed, method=method, lc=lc, psi_rows=psi_rows)
        self._h = ctypes.c_void_p()
        need = ctypes.c_size_t()
        _lib.check(L.rsvd_stream_create(self.m, self.n, self.k, int(p), code, ctypes.byref(o), ctypes.byref(self._h),
                                        ctypes.byref(need)), "rsvd_stream_create")
        self.workspace = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=self.device)
        _lib.check(L.rsvd_stream_bind(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                      ctypes.c_size_t(self.workspace.numel()), _stream()), "rsvd_stream_bind")

    def add_dense(self, r0, c0, H, trans=False):
        mat = _mat(H, trans)
        _lib.check(lib().rsvd_stream_add_dense(self._h, int(r0), int(c0), ctypes.byref(mat), _stream()),
                   "rsvd_stream_add_dense")

    def add_entries(self, rows, cols, vals):
        torch = _torch()
        rows = rows.to(device=self.device, dtype=torch.int64).contiguous()
        cols = cols.to(device=self.device, dtype=torch.int64).contiguous()
        vals = vals.to(device=self.device, dtype=self.dtype).contiguous()
        if not (rows.numel() == cols.numel() == vals.numel()):
            raise ValueError("rows, cols and vals must have one entry each")
        _lib.check(lib().rsvd_stream_add_entries(self._h, rows.numel(), ctypes.c_void_p(rows.data_ptr()),
                                                 ctypes.c_void_p(cols.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                                                 _stream()), "rsvd_stream_add_entries")
        self._keep = (rows, cols, vals)   # alive until the stream has consumed them

    def finish(self, check=False):
        torch = _torch()
        U = torch.empty(self.m, self.k, dtype=self.dtype, device=self.device)
        V = torch.empty(self.n, self.k, dtype=self.dtype, device=self.device)
        S = torch.empty(self.k, dtype=torch.float64, device=self.device)
        out = RsvdOut(U.data_ptr(), S.data_ptr(), V.data_ptr())
        _lib.check(lib().rsvd_stream_finish(self._h, ctypes.byref(out), _stream()), "rsvd_stream_finish")
        if check:
            _check_device(self.workspace, "rsvd_stream_finish")
        return U, S, V

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().rsvd_stream_destroy(h)
            self._h = None


class BatchPlan:
    """Alg. 2 on a batch of independent matrices in a few dozen grouped
    launches (rsvd_batch_plan_* in include/rsvd.h).

        plan = BatchPlan(mats, ks, p, v, seed=..., tuning=(plan_cus, view_mr))
        plan.run()                 # enqueue on the current stream (capturable)
        U, S, V = plan.outputs[b]

    mats are 2-D CUDA tensors (float32 or float64) with unit row stride; the
    outputs are allocated here and rewritten by every run."""

    def __init__(self, mats, ks, p, v, seed=0, tuning=None):
        torch = _torch()
        L = lib()
        self.mats = list(mats)
        nb = len(self.mats)
        self.outputs = []
        marr = (RsvdMat * nb)()
        oarr = (RsvdOut * nb)()
        karr = (ctypes.c_int * nb)(*[int(k) for k in ks])
        for b, A in enumerate(self.mats):
            marr[b] = _mat(A)
            m, n = A.shape
            k = int(ks[b])
            U = torch.empty(m, k, dtype=A.dtype, device=A.device)
            V = torch.empty(n, k, dtype=A.dtype, device=A.device)
            S = torch.empty(k, dtype=torch.float64, device=A.device)
            oarr[b] = RsvdOut(U.data_ptr(), S.data_ptr(), V.data_ptr())
            self.outputs.append((U, S, V))
        o = _opts(seed=seed)
        t = _lib.RsvdBatchTuning()
        L.rsvd_default_batch_tuning(ctypes.byref(t))
        if tuning is not None:
            t.plan_cus, t.view_mr = int(tuning[0]), int(tuning[1])
        self.tuning = (t.plan_cus, t.view_mr)
        self._plan = ctypes.c_void_p()
        need = ctypes.c_size_t()
        _lib.check(L.rsvd_batch_plan_create(nb, marr, karr, p, v, ctypes.byref(o), oarr, ctypes.byref(t),
                                            ctypes.byref(self._plan), ctypes.byref(need)), "rsvd_batch_plan_create")
        self.workspace = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=self.mats[0].device)
        _lib.check(L.rsvd_batch_plan_bind(self._plan, ctypes.c_void_p(self.workspace.data_ptr()),
                                          ctypes.c_size_t(self.workspace.numel()), _stream()), "rsvd_batch_plan_bind")
        self.launches = L.rsvd_batch_plan_launches(self._plan)

    def run(self):
        _lib.check(lib().rsvd_subspace_batched(self._plan, _stream()), "rsvd_subspace_batched")

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            lib().rsvd_batch_plan_destroy(plan)
            self._plan = None

