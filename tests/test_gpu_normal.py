"""GPU: truncated eigendecompositions of J^T J (Sect. 4.2) against the FP64
oracle on the same seeded inputs: Alg. 4 (Nystrom), Alg. 5 (pinched) and
Alg. 2 by the J / J^T rule, for v = 2..5 views.  Tolerances, relative, on
sqrt(lam2) (the singular values of J the methods estimate): 1e-10 on the FP64
path, 1e-4 on the FP32 path; eigenvectors by |cos| against the oracle's.
Beside the oracle: exact recovery of an exactly rank-k J, and the
equivalences of Sect. 4.2.3 checked between the GPU's own methods.
"""

import sys

import numpy as np
import pytest

import synth
from oracle import normal as onormal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1804_07531_amd as rs  # noqa: E402

DEV = torch.device("cuda:0")
SEED = synth.METHOD_SEED
ORACLE = {"nystrom": onormal.nystrom, "pinched": onormal.pinched, "subspace": onormal.subspace_rule}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _check(V, lam2, ref, tol, vec_tol, nvec=None):
    V = V.double().cpu().numpy()
    lam2 = lam2.cpu().numpy()
    rel = np.abs(np.sqrt(lam2) - np.sqrt(ref.lam2)) / np.sqrt(ref.lam2)
    nv = V.shape[1] if nvec is None else nvec
    dv = np.max(np.abs(np.abs(np.sum(V[:, :nv] * ref.V[:, :nv], axis=0)) - 1.0))
    say(f"  sqrt(lam2) rel err {rel.max():.2e}, vectors {dv:.2e}")
    assert rel.max() <= tol
    assert dv <= vec_tol


@pytest.mark.parametrize("v", [2, 3, 4, 5])
@pytest.mark.parametrize("method", ["nystrom", "pinched", "subspace"])
def test_normal_fp64(method, v):
    m, n, k, p = 800, 500, 12, 6
    sigma = np.arange(1, 501, dtype=np.float64) ** -1.0
    j = synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 11)
    say(f"normal {method} v={v} f64 {m}x{n} k={k} p={p}")
    V, lam2 = rs.normal_tevd(_t(j), k, p, v, method=method, seed=SEED, check=True)
    _check(V, lam2, ORACLE[method](j, k, p, v, SEED), 1e-10, 1e-7)


@pytest.mark.parametrize("method", ["nystrom", "pinched", "subspace"])
def test_normal_wide_and_transposed_storage(method):
    # m < n, J given through the storage of J^T
    m, n, k, p = 300, 700, 10, 5
    sigma = np.arange(1, 301, dtype=np.float64) ** -1.5
    j = synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 12)
    for v in (2, 3):
        V, lam2 = rs.normal_tevd(_t(j.T), k, p, v, method=method, trans=True, seed=SEED)
        _check(V, lam2, ORACLE[method](j, k, p, v, SEED), 1e-10, 1e-7)


@pytest.mark.parametrize("method", ["nystrom", "pinched", "subspace"])
def test_normal_fp32(method):
    m, n, k, p = 3000, 1200, 30, 10
    sigma = np.arange(1, 1201, dtype=np.float64) ** -1.0
    j32 = synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 13).astype(np.float32)
    for v in (2, 3):
        V, lam2 = rs.normal_tevd(_t(j32, torch.float32), k, p, v, method=method, seed=SEED)
        _check(V, lam2, ORACLE[method](j32.astype(np.float64), k, p, v, SEED), 1e-4, 1e-2, nvec=10)


@pytest.mark.parametrize("method", ["nystrom", "pinched", "subspace"])
def test_normal_exact_recovery(method):
    m, n, k, p = 600, 400, 10, 5
    sigma = np.zeros(400)
    sigma[:k] = 10.0 ** -np.linspace(0, 2, k)
    j = synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 14)
    V, lam2 = rs.normal_tevd(_t(j), k, p, 3, method=method, seed=SEED)
    got = np.sqrt(lam2.cpu().numpy())
    assert np.max(np.abs(got - sigma[:k]) / sigma[:k]) <= 1e-11


def test_normal_equivalences():
    # Sect. 4.2.3: Nystrom with v views spans what Alg. 2 on J (even v) or J^T (odd v)
    # spans, pinched with v views what Alg. 2 on J^T (even v) or J (odd v) spans; the
    # eigenvalues agree up to the Nystrom shift (2.2e-16 ||Y_r||)
    m, n, k, p = 800, 500, 12, 6
    sigma = np.arange(1, 501, dtype=np.float64) ** -1.0
    J = _t(synth.spectral_matrix(m, n, sigma, synth.GEN_SEED + 15))
    for v in (3, 4):
        _, ln = rs.normal_tevd(J, k, p, v, method="nystrom", seed=SEED)
        _, ls = rs.normal_tevd(J, k, p, v, method="subspace", seed=SEED)
        assert np.max(np.abs(ln.cpu().numpy() - ls.cpu().numpy()) / ls.cpu().numpy()) <= 1e-10
    # pinched(v) against Alg. 2 with v views on J^T (even v) or J (odd v)
    Jt = J.t().contiguous()
    for v in (2, 3):
        _, lp = rs.normal_tevd(J, k, p, v, method="pinched", seed=SEED)
        _, S, _ = rs.subspace(Jt if v % 2 == 0 else J, k, p, v, seed=SEED)
        s2 = S.cpu().numpy() ** 2
        assert np.max(np.abs(lp.cpu().numpy() - s2) / s2) <= 1e-10


def test_normal_argument_errors():
    J = _t(np.ones((50, 40)))
    for args, code in [((5, 2, 1, "nystrom"), 1), ((5, 2, 2, 7), 1), ((30, 20, 2, "pinched"), 2)]:
        k, p, v, method = args
        with pytest.raises(rs.RsvdError) as e:
            rs.normal_tevd(J, k, p, v, method=method)
        assert e.value.code == code
