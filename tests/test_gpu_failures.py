"""GPU: failures found on the device are reported, and every kernel exits.

* A non-finite entry of A makes a sketch non-finite: the Cholesky factor of
  its Gram reports it (the pivot rule would otherwise turn the column into a
  zero column and return finite, wrong values), the status word carries
  bit 2, rsvd_device_status returns RSVD_EBREAKDOWN and check=True raises
  RsvdError.  Every loop of the path is bounded (the Jacobi sweeps by
  a sweep cap, their convergence test is false for NaN), so the call ends.
* The multi-workgroup small SVD meets at a device-wide barrier with a
  bounded wait.  The host sets the wait to one poll (opts.sync_spins = 1):
  workgroups that arrive early give up, the flag makes every later wait
  return at once, the status word carries bit 4 and the call reports
  RSVD_EBREAKDOWN.  The next call with the default wait is correct again.
* The row-sweep gradient assumes a Krylov basis of full numerical rank; on a
  matrix of lower rank the TSVD of R_K cuts columns, bit 3 is set and the
  autograd function raises instead of returning a wrong gradient.
"""

import numpy as np
import pytest

import synth
from oracle import rsvd as orsvd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1804_07531_amd as rs  # noqa: E402
from paper_1804_07531_amd import autograd as rag  # noqa: E402

DEV = torch.device("cuda:0")
SEED = synth.METHOD_SEED
FLAG_NONFINITE, FLAG_TRUNCATED, FLAG_SYNC_TIMEOUT = 4, 8, 16


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _decaying(m, n, power, seed, rank=None):
    r = min(m, n) if rank is None else rank
    sigma = np.arange(1, r + 1, dtype=np.float64) ** -power
    return synth.spectral_matrix(m, n, sigma, seed)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("call", ["subspace", "single_pass", "row_sweep"])
def test_nan_inside_a_is_reported(call, dtype):
    a = _decaying(300, 200, 1.0, seed=17)
    a[17, 33] = np.nan
    A = _t(a, dtype)
    fn = {"subspace": lambda **kw: rs.subspace(A, 10, 5, 3, **kw),
          "single_pass": lambda **kw: rs.single_pass(A, 10, 5, **kw),
          "row_sweep": lambda **kw: rs.block_krylov(A, 10, 5, 2, mode="row", **kw)}[call]
    with pytest.raises(rs.RsvdError) as e:
        fn(seed=SEED, check=True)
    assert e.value.code == 4 and e.value.flags & FLAG_NONFINITE
    # without check the call returns; the word is read afterwards
    _, _, _, ws = fn(seed=SEED, return_workspace=True)
    code, flags = rs.device_status(ws)
    assert code == 4 and flags & FLAG_NONFINITE


def test_small_svd_barrier_timeout_is_reported():
    # s = 100 > 80 columns: a single call takes the multi-workgroup small SVD
    m, n, k, p, v = 600, 400, 90, 10, 2
    a = _decaying(m, n, 1.0, seed=19)
    A = _t(a)
    with pytest.raises(rs.RsvdError) as e:
        rs.subspace(A, k, p, v, seed=SEED, sync_spins=1, check=True)
    assert e.value.code == 4 and e.value.flags & FLAG_SYNC_TIMEOUT
    # the default wait: no flag, and the oracle's result
    U, S, V, ws = rs.subspace(A, k, p, v, seed=SEED, return_workspace=True, check=True)
    code, flags = rs.device_status(ws)
    assert code == 0 and not flags & FLAG_SYNC_TIMEOUT
    ref = orsvd.alg2_gensubit(a, k, p, v, SEED)
    assert np.max(np.abs(S.cpu().numpy() - ref.S) / ref.S) <= 1e-10


def test_grad_on_rank_deficient_krylov_basis_raises():
    # rank 20 < v (k + p) = 36: the TSVD of R_K cuts, the adjoint would not model it
    a = _decaying(300, 200, 1.0, seed=23, rank=20)
    A = _t(a).requires_grad_(True)
    with pytest.raises(rs.RsvdError) as e:
        rag.row_sweep_svd(A, 8, 4, 3, seed=SEED)
    assert e.value.flags & FLAG_TRUNCATED
