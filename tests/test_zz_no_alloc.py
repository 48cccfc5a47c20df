"""GPU: rsvd_subspace_noalloc (the entry point that allocates nothing, for
callers that cannot allocate) against rsvd_subspace on the same inputs,
through the C ABI: two calls in a row on the shared per-GPU scratch array,
the second with a smaller input, each equal to rsvd_subspace to the FP64 /
FP32 path's tolerance (the kernels are the same, so the results are expected
bit for bit; the assertion is the stated tolerance).  An oversized request
returns RSVD_EWORKSPACE and leaves the outputs untouched.
"""

import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1804_07531_amd as rs  # noqa: E402
from paper_1804_07531_amd import _lib  # noqa: E402

DEV = torch.device("cuda:0")
SEED = synth.METHOD_SEED


def _matrix(m, n, dtype, seed):
    sigma = np.arange(1, min(m, n) + 1, dtype=np.float64) ** -1.5
    a = synth.spectral_matrix(m, n, sigma, seed)
    return torch.from_numpy(a).to(DEV, dtype)


def _outputs(A, k):
    m, n = A.shape
    U = torch.full((m, k), 7.0, dtype=A.dtype, device=DEV)
    V = torch.full((n, k), 7.0, dtype=A.dtype, device=DEV)
    S = torch.full((k,), 7.0, dtype=torch.float64, device=DEV)
    return U, S, V, _lib.RsvdOut(U.data_ptr(), S.data_ptr(), V.data_ptr())


def _call_both(A, k, p, v):
    L = rs.lib()
    mat = rs._mat(A)
    o = rs._opts(seed=SEED)
    stream = rs._stream()
    U1, S1, V1, out1 = _outputs(A, k)
    code = L.rsvd_subspace_noalloc(ctypes.byref(mat), k, p, v, ctypes.byref(o), ctypes.byref(out1), stream)
    assert code == 0, f"rsvd_subspace_noalloc returned {code}"
    need = L.rsvd_workspace_bytes(ctypes.byref(mat), k, p, v, 0, ctypes.byref(o))
    assert 0 < need <= L.rsvd_noalloc_max_bytes()
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    U2, S2, V2, out2 = _outputs(A, k)
    code = L.rsvd_subspace(ctypes.byref(mat), k, p, v, ctypes.byref(o), ctypes.byref(out2),
                           ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(need), stream)
    assert code == 0
    torch.cuda.synchronize()
    return (U1, S1, V1), (U2, S2, V2)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
def test_noalloc_matches_subspace_on_two_calls(dtype, tol):
    first = (_matrix(3000, 1500, dtype, 31), 20, 10, 3)
    second = (_matrix(900, 700, dtype, 32), 10, 5, 2)     # smaller: the array keeps the first call's contents
    for A, k, p, v in (first, second):
        (U1, S1, V1), (U2, S2, V2) = _call_both(A, k, p, v)
        s1, s2 = S1.cpu().numpy(), S2.cpu().numpy()
        rel = np.max(np.abs(s1 - s2) / np.abs(s2))
        du = (U1 - U2).abs().max().item()
        dv = (V1 - V2).abs().max().item()
        print(f"{tuple(A.shape)} {dtype}: sigma rel {rel:.2e}, U {du:.2e}, V {dv:.2e}, "
              f"bitwise {bool(torch.equal(U1, U2) and torch.equal(V1, V2) and np.array_equal(s1, s2))}")
        assert rel <= tol
        assert du <= 10 * tol and dv <= 10 * tol


def test_noalloc_rejects_oversized_requests():
    L = rs.lib()
    A = torch.zeros(65536, 4096, dtype=torch.float32, device=DEV)
    mat = rs._mat(A)
    o = rs._opts(seed=SEED)
    need = L.rsvd_workspace_bytes(ctypes.byref(mat), 100, 20, 2, 0, ctypes.byref(o))
    assert need > L.rsvd_noalloc_max_bytes()
    U, S, V, out = _outputs(A, 100)
    code = L.rsvd_subspace_noalloc(ctypes.byref(mat), 100, 20, 2, ctypes.byref(o), ctypes.byref(out), rs._stream())
    torch.cuda.synchronize()
    assert code == _lib.RSVD_EWORKSPACE
    assert bool((S == 7.0).all()) and bool((U == 7.0).all())
