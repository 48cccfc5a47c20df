"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the randomized SVD itself: it only builds
data matrices with prescribed singular spectra, quantizes them to the storage
formats the library reads, and draws the shapes of a batch.  The Gaussian test
matrices the method draws are NOT here: the GPU library and the oracle each
generate those from their own implementation of the counter-based generator.

Matrices (Sect. 8.1 of the paper and the library's workloads):

* ``spectral_matrix``     A = U diag(sigma) V^T with Haar-distributed U, V
                          (QR of a seeded Gaussian, columns sign-fixed so that
                          diag(R) > 0, which makes the law exactly Haar).
* ``low_rank_noise``      diag(1,..,1 (R times), 0, ..) + sqrt(eta R / 2n^2)(G + G^T)
* ``poly_decay``          diag(1 (R times), 2^-rho, 3^-rho, ...)
* ``exp_decay``           diag(1 (R times), 10^-theta, 10^-2theta, ...)

Seeds: data generator seed = 20180524 + workload id; the method's test-matrix
seed = 1804075310 + trial.
"""

import math

import numpy as np

GEN_SEED = 20180524
METHOD_SEED = 1804075310


# --------------------------------------------------------------------------
# CPU (numpy) generators
# --------------------------------------------------------------------------

def haar(rows, cols, rng):
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def spectral_matrix(m, n, sigma, seed, noise=0.0):
    """m x n FP64 matrix U diag(sigma) V^T (+ optional iid Gaussian noise whose
    spectral norm is about noise * sigma_1)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.size
    rng = np.random.default_rng(seed)
    u = haar(m, r, rng)
    v = haar(n, r, rng)
    a = (u * sigma[None, :]) @ v.T
    if noise:
        tau = noise * sigma[0] / (math.sqrt(m) + math.sqrt(n))
        a = a + tau * rng.standard_normal((m, n))
    return a


def low_rank_noise(n, rank, eta, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    a = math.sqrt(eta * rank / (2.0 * n * n)) * (g + g.T)
    a[np.arange(rank), np.arange(rank)] += 1.0
    return a


def poly_decay_spectrum(n, rank, rho):
    return np.concatenate([np.ones(rank), np.arange(2, n - rank + 2, dtype=np.float64) ** (-rho)])


def exp_decay_spectrum(n, rank, theta):
    return np.concatenate([np.ones(rank), 10.0 ** (-theta * np.arange(1, n - rank + 1))])


def diag_matrix(sigma):
    return np.diag(np.asarray(sigma, dtype=np.float64))


def workload_c1():
    """2000 x 1000 FP64, sigma_j = j^-2, Haar U and V (full spectrum)."""
    sigma = np.arange(1, 1001, dtype=np.float64) ** -2.0
    return spectral_matrix(2000, 1000, sigma, GEN_SEED + 1), sigma


def batch_shapes(count=512, seed=GEN_SEED):
    """Shapes of the batched workload: m log-uniform in [500, 8000], n
    log-uniform in [200, 4000], k uniform in {8..64}."""
    rng = np.random.default_rng(seed)
    m = np.rint(np.exp(rng.uniform(math.log(500), math.log(8000), count))).astype(int)
    n = np.rint(np.exp(rng.uniform(math.log(200), math.log(4000), count))).astype(int)
    k = rng.integers(8, 65, count)
    return m, n, k


# --------------------------------------------------------------------------
# storage formats
# --------------------------------------------------------------------------

def to_bf16_bits(a):
    """Round FP32/FP64 values to BF16 (nearest, ties to even); returns uint16 bits."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def _e4m3_positive_values():
    vals = []
    for byte in range(0x7F):                     # 0x00 .. 0x7E: all finite non-negative codes
        exp, man = byte >> 3, byte & 7
        vals.append((2.0 ** -6) * man / 8.0 if exp == 0 else (2.0 ** (exp - 7)) * (1 + man / 8.0))
    return np.array(vals)


_E4M3_POS = _e4m3_positive_values()


def to_e4m3_bits(x):
    """Round to OCP FP8 E4M3 (nearest, ties to even), saturating at +-448."""
    x = np.asarray(x, dtype=np.float64)
    mag = np.minimum(np.abs(x), 448.0)
    hi = np.clip(np.searchsorted(_E4M3_POS, mag, side="left"), 0, 0x7E)
    lo = np.clip(hi - 1, 0, 0x7E)
    dlo = mag - _E4M3_POS[lo]
    dhi = _E4M3_POS[hi] - mag
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo).astype(np.uint8)
    code = np.where(mag == _E4M3_POS[hi], hi, code).astype(np.uint8)
    sign = np.where((x < 0) & (code != 0), 0x80, 0).astype(np.uint8)
    return code | sign


def to_fp8_rows(a):
    """Per-row scaled FP8: scale_i = max_j |a_ij| / 448 (FP32; 1 for an all-zero
    row) and bits = e4m3(a_ij / scale_i)."""
    a = np.asarray(a, dtype=np.float64)
    scale = (np.max(np.abs(a), axis=1) / 448.0).astype(np.float32)
    scale[scale == 0] = 1.0
    bits = to_e4m3_bits(a / scale.astype(np.float64)[:, None])
    return bits, scale


# --------------------------------------------------------------------------
# GPU (torch) generators for the full-size workloads
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def haar_torch(rows, cols, gen, device):
    torch = _torch()
    g = torch.randn(rows, cols, generator=gen, device=device, dtype=torch.float64)
    q, r = torch.linalg.qr(g)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def spectral_matrix_torch(m, n, sigma, seed, noise=0.0, dtype=None, device="cuda", chunk=8192):
    """Device-resident U diag(sigma) V^T (+ noise), built in FP64 and stored in
    ``dtype`` (default float32), one block of rows at a time."""
    torch = _torch()
    dtype = dtype or torch.float32
    sig = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    r = sig.numel()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    u = haar_torch(m, r, gen, device)
    v = haar_torch(n, r, gen, device)
    vt = (v * sig[None, :]).t().contiguous()
    del v
    out = torch.empty(m, n, dtype=dtype, device=device)
    tau = noise * float(sigma[0]) / (math.sqrt(m) + math.sqrt(n)) if noise else 0.0
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        blk = u[r0:r1] @ vt
        if tau:
            blk += tau * torch.randn(r1 - r0, n, generator=gen, device=device, dtype=torch.float64)
        out[r0:r1] = blk.to(dtype)
    del u, vt
    return out
