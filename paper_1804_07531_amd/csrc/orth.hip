// Orthonormalization of a panel: the paper's qr (Sect. 2) after every view
// (Alg. 1, 2, 9), computed as CholeskyQR2 with a shifted first round when
// the Gram matrix is too ill-conditioned (shifted CholeskyQR3 of Fukaya,
// Kannan, Nakatsukasa, Yamamoto & Yanagisawa, SIAM J. Sci. Comput. 2020).
//
// For a panel P = Y^T (s x len):
//   G = Y^T Y = P P^T                       (FP64, matrix cores)
//   R = chol(G [+ shift I])^T, R^-1         (FP64, one workgroup)
//   Q^T = R^-T P                            (FP64 arithmetic, result in the working type)
// repeated, with R_total = R_k ... R_1 when the caller needs the triangular
// factor (R_c or R_r of Alg. 2).
#include <algorithm>

#include "common.h"
#include "orth.h"

namespace {

template <typename T>
__device__ __forceinline__ void load4d(const T* p, int64_t k, int64_t kmax, bool ok, bool vec, double out[4]) {
    if (ok && vec && k + 3 < kmax) {
        if constexpr (sizeof(T) == 4) {
            const floatx4 f = *reinterpret_cast<const floatx4*>(p);
            out[0] = f[0]; out[1] = f[1]; out[2] = f[2]; out[3] = f[3];
        } else {
            const double2 a = *reinterpret_cast<const double2*>(p);
            const double2 b = *reinterpret_cast<const double2*>(p + 2);
            out[0] = a.x; out[1] = a.y; out[2] = b.x; out[3] = b.y;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) out[t] = (ok && k + t < kmax) ? (double)p[t] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Cross product of two panels: C (s1 x s2, FP64) = P1 P2^T, partial over a
// split of the long index.  Each wave computes one 16x16 tile.  With
// symmetric != 0 (P1 == P2) only tiles ta <= tb are computed and mirrored.
// grid.x: groups of 4 tile tasks; grid.y: splits.
// ---------------------------------------------------------------------------
template <typename T1, typename T2>
__global__ void __launch_bounds__(256)
cross_kernel(const T1* __restrict__ P1, int64_t ld1, int s1, const T2* __restrict__ P2, int64_t ld2, int s2,
             int64_t len, int symmetric, double* __restrict__ out, int64_t split_stride, int64_t chunk,
             const int* enable) {
    if (enable && *enable == 0) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    const int nt1 = (s1 + 15) / 16, nt2 = (s2 + 15) / 16;
    int64_t task = (int64_t)blockIdx.x * 4 + wave;
    int ta, tb;
    if (symmetric) {  // enumerate the upper triangle of tiles row by row
        int64_t t = task;
        ta = 0;
        while (ta < nt1 && t >= nt1 - ta) {
            t -= nt1 - ta;
            ++ta;
        }
        if (ta >= nt1) return;
        tb = ta + (int)t;
    } else {
        if (task >= (int64_t)nt1 * nt2) return;
        ta = (int)(task / nt2);
        tb = (int)(task % nt2);
    }
    const int64_t kb = (int64_t)blockIdx.y * chunk;
    const int64_t ke = std::min<int64_t>(len, kb + chunk);
    const int ra = 16 * ta + i, rb = 16 * tb + i;
    const bool oka = ra < s1, okb = rb < s2;
    const T1* pa = P1 + (int64_t)(oka ? ra : 0) * ld1;
    const T2* pb = P2 + (int64_t)(okb ? rb : 0) * ld2;
    const bool vec = (((uintptr_t)P1 | (uintptr_t)P2) & 15) == 0 && ld1 % 4 == 0 && ld2 % 4 == 0 && kb % 4 == 0;
    doublex4 acc = {0, 0, 0, 0};
    for (int64_t k = kb; k < ke; k += 16) {
        const int64_t kk = k + 4 * g;
        double a[4], b[4];
        load4d(pa + kk, kk, ke, oka, vec, a);
        load4d(pb + kk, kk, ke, okb, vec, b);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], acc, 0, 0, 0);
    }
    double* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * ta + mfma16<double>::row(g, r), col = 16 * tb + i;
        if (row < s1 && col < s2) {
            o[(int64_t)row * s2 + col] = acc[r];
            if (symmetric && ta != tb) o[(int64_t)col * s2 + row] = acc[r];
        }
    }
}

__global__ void __launch_bounds__(256)
sum_parts_f64_kernel(const double* __restrict__ parts, int nparts, int64_t stride, int64_t total,
                     double* __restrict__ out, const int* enable) {
    if (enable && *enable == 0) return;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = parts[e];
        for (int p = 1; p < nparts; ++p) acc += parts[p * stride + e];
        out[e] = acc;
    }
}

// ---------------------------------------------------------------------------
// Cholesky factorization G = L L^T (L lower), R = L^T, and R^-1, by ONE wave
// (64 lanes; lane l owns rows l, l+64, ...).  A single wave needs no
// workgroup barriers between the s column steps; the work matrix W (s x s,
// leading dimension ldw) lives in LDS when it fits, else in global scratch.
//
// First attempt without shift; if a pivot falls to <= 1e3 eps G_jj the
// factorization restarts on G + sigma I with
// sigma = 11 (len s + s (s+1)) eps trace(G) (trace(G) >= ||Y||_2^2), sets
// the SHIFTED status bit and *need_more = 1 (the caller then runs one more
// CholeskyQR round).  A pivot that is still <= 0 after the shift (possible
// only for an all-zero column) leaves a degenerate column (zero in R, unit
// in the inverse) and sets the PIVOT bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() { __syncthreads(); }  // one-wave block: a memory fence

// sum_{l < n} x[l] y[l] with four independent partial sums (keeps LDS loads in flight)
__device__ __forceinline__ double dot4(const double* __restrict__ x, const double* __restrict__ y, int n) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int l = 0;
    for (; l + 4 <= n; l += 4) {
        a0 += x[l] * y[l];
        a1 += x[l + 1] * y[l + 1];
        a2 += x[l + 2] * y[l + 2];
        a3 += x[l + 3] * y[l + 3];
    }
    for (; l < n; ++l) a0 += x[l] * y[l];
    return (a0 + a1) + (a2 + a3);
}

__global__ void __launch_bounds__(64)
chol_inv_kernel(const double* __restrict__ G, int s, double shift_factor, double* __restrict__ R,
                double* __restrict__ Rinv, double* __restrict__ gscratch, uint32_t* status, int* need_more,
                const int* enable) {
    if (enable && *enable == 0) return;
    extern __shared__ double lds[];
    const bool in_lds = gscratch == nullptr;
    const int ldw = s + 1;
    double* W = in_lds ? lds : gscratch;
    __shared__ double col_tmp[1024];
    __shared__ unsigned char unit_sh[1024];
    __shared__ double piv;
    const int lane = threadIdx.x;

    double tr = 0.0;
    for (int a = lane; a < s; a += 64) tr += G[(int64_t)a * s + a];
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off);
    const double shift = shift_factor * tr;

    // Crout order: column j of L from the finished columns 0..j-1,
    //   L[j][j] = sqrt(G[j][j] - sum_l L[j][l]^2),
    //   L[a][j] = (G[a][j] - sum_l L[a][l] L[j][l]) / L[j][j],  a > j (one row per lane).
    for (int attempt = 0; attempt < 2; ++attempt) {
        for (int a = lane; a < s; a += 64) {
            for (int b = 0; b <= a; ++b)
                W[a * ldw + b] = G[(int64_t)a * s + b] + ((attempt == 1 && a == b) ? shift : 0.0);
            unit_sh[a] = 0;
        }
        wave_sync();
        bool failed = false;
        for (int j = 0; j < s; ++j) {
            const double* wj = W + j * ldw;
            if (lane == (j & 63)) piv = wj[j] - dot4(wj, wj, j);
            wave_sync();
            const double d = piv;
            bool unit_col = false;
            if (attempt == 0) {
                if (!(d > 1e3 * 2.220446049250313e-16 * G[(int64_t)j * s + j]) || !(d > 0.0)) {
                    failed = true;  // uniform across the wave: every lane read the same d
                    break;
                }
            } else if (!(d > 0.0)) {
                unit_col = true;
            }
            const double rjj = unit_col ? 1.0 : sqrt(d);
            const double inv = 1.0 / rjj;
            for (int a = j + 1 + lane; a < s; a += 64) {
                double* wa = W + a * ldw;
                wa[j] = unit_col ? 0.0 : (wa[j] - dot4(wa, wj, j)) * inv;
            }
            if (lane == 0) {
                W[j * ldw + j] = rjj;
                if (unit_col) {
                    unit_sh[j] = 1;
                    rsvd_flag(status, RSVD_FLAG_PIVOT);
                }
            }
            wave_sync();
        }
        if (!failed) break;
        if (lane == 0) {
            rsvd_flag(status, RSVD_FLAG_SHIFTED);
            if (need_more) *need_more = 1;
        }
        wave_sync();
    }

    // R = L^T (upper; zeros below the diagonal).  A degenerate column of Y
    // (zero after the shift) gets a zero row in R and a unit diagonal in the
    // inverse, so that Q's column is zero and Y = Q R still holds.
    for (int e = lane; e < s * s; e += 64) {
        const int a = e / s, b = e % s;
        R[e] = (b >= a && !(a == b && unit_sh[a])) ? W[b * ldw + a] : 0.0;
    }
    // in-place inverse of the lower triangle, last column first:
    // Linv[j][j] = 1/L[j][j]; Linv[a][j] = -Linv[j][j] sum_{l=j+1..a} Linv[a][l] L[l][j]
    for (int j = s - 1; j >= 0; --j) {
        for (int a = j + 1 + lane; a < s; a += 64) col_tmp[a] = W[a * ldw + j];
        wave_sync();
        const double djj = 1.0 / W[j * ldw + j];
        for (int a = j + 1 + lane; a < s; a += 64) {
            const double* wa = W + a * ldw;
            W[a * ldw + j] = -dot4(wa + j + 1, col_tmp + j + 1, a - j) * djj;
        }
        if (lane == 0) W[j * ldw + j] = djj;
        wave_sync();
    }
    // R^-1 = Linv^T
    for (int e = lane; e < s * s; e += 64) {
        const int a = e / s, b = e % s;
        Rinv[e] = (b >= a) ? W[b * ldw + a] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Coefficient apply on panels (FP64 arithmetic):
//   OUT[a][x] = beta OUT[a][x] + alpha sum_b C[b][a] IN[b][x],  a < s_out, b < s_in.
// With C = R^-1 this is Q^T = R^-T Y^T.  One wave owns 16*NI columns and
// every output row; OUT may alias IN (s_in == s_out, beta == 0) because a
// wave reads all rows of its columns before writing any.  `triangular`
// skips the blocks of an upper-triangular C that are zero.
// ---------------------------------------------------------------------------
template <typename TI, typename TO, int NI>
__global__ void __launch_bounds__(256)
apply_coeff_kernel(const TI* __restrict__ IN, int64_t ldi, int s_in, int64_t len, const double* __restrict__ C,
                   int64_t ldc, int s_out, int triangular, double alpha, double beta, TO* OUT, int64_t ldo,
                   const int* enable) {
    if (enable && *enable == 0) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    const int64_t x0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * NI);
    if (x0 >= len) return;
    const int nt = (s_out + 15) / 16;
    doublex4 acc[16][NI];
#pragma unroll
    for (int a = 0; a < 16; ++a)
#pragma unroll
        for (int c = 0; c < NI; ++c) acc[a][c] = doublex4{0, 0, 0, 0};
    for (int k0 = 0; k0 < s_in; k0 += 16) {
        double bv[NI][4];
#pragma unroll
        for (int c = 0; c < NI; ++c) {
            const int64_t x = x0 + 16 * c + i;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int b = k0 + 4 * g + t;
                bv[c][t] = (b < s_in && x < len) ? (double)IN[(int64_t)b * ldi + x] : 0.0;
            }
        }
#pragma unroll
        for (int ta = 0; ta < 16; ++ta) {
            if (ta >= nt) break;
            if (triangular && 16 * ta + 15 < k0) continue;  // C[b][a] = 0 for b > a
            double av[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int b = k0 + 4 * g + t, a = 16 * ta + i;
                av[t] = (b < s_in && a < s_out) ? C[(int64_t)b * ldc + a] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int c = 0; c < NI; ++c)
                    acc[ta][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[c][t], acc[ta][c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int ta = 0; ta < 16; ++ta) {
        if (ta >= nt) break;
#pragma unroll
        for (int c = 0; c < NI; ++c) {
            const int64_t x = x0 + 16 * c + i;
            if (x >= len) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = 16 * ta + mfma16<double>::row(g, r);
                if (a < s_out) {
                    TO* d = OUT + (int64_t)a * ldo + x;
                    const double prev = beta != 0.0 ? beta * (double)*d : 0.0;
                    *d = (TO)(prev + alpha * acc[ta][c][r]);
                }
            }
        }
    }
}

// Upper-triangular products on s x s matrices (one workgroup):
// side 0: Racc <- R Racc;  side 1: Racc <- Racc R.
__global__ void __launch_bounds__(1024)
trmm_upper_kernel(const double* __restrict__ R, double* __restrict__ Racc, double* __restrict__ tmp, int s, int side,
                  const int* enable) {
    if (enable && *enable == 0) return;
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int a = e / s, b = e % s;
        double acc = 0.0;
        if (side == 0)
            for (int l = a; l <= b; ++l) acc += R[a * s + l] * Racc[l * s + b];
        else
            for (int l = a; l <= b; ++l) acc += Racc[a * s + l] * R[l * s + b];
        tmp[e] = (b >= a) ? acc : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) Racc[e] = tmp[e];
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int64_t cross_splits(int s1, int s2, int64_t len, int symmetric, int num_cu) {
    const int64_t nt1 = ceil_div(s1, 16), nt2 = ceil_div(s2, 16);
    const int64_t tasks = symmetric ? nt1 * (nt1 + 1) / 2 : nt1 * nt2;
    const int64_t groups = ceil_div(tasks, 4);
    int64_t splits = 1;
    while (groups * splits < 2 * num_cu && ceil_div(len, splits * 2) >= 512 && splits < 512) splits *= 2;
    return splits;
}

size_t cross_scratch_doubles(int s1, int s2, int64_t len, int symmetric, int num_cu) {
    const int64_t splits = cross_splits(s1, s2, len, symmetric, num_cu);
    return (size_t)splits * s1 * s2;
}

rsvd_status run_cross(int dtype1, const void* P1, int64_t ld1, int s1, int dtype2, const void* P2, int64_t ld2,
                      int s2, int64_t len, int symmetric, double* out, double* scratch, int num_cu,
                      const int* enable, hipStream_t st) {
    const int64_t splits = cross_splits(s1, s2, len, symmetric, num_cu);
    const int64_t chunk = round_up(ceil_div(len, splits), 16);
    const int64_t nsp = ceil_div(len, chunk);
    const int64_t nt1 = ceil_div(s1, 16), nt2 = ceil_div(s2, 16);
    const int64_t tasks = symmetric ? nt1 * (nt1 + 1) / 2 : nt1 * nt2;
    dim3 grid((unsigned)ceil_div(tasks, 4), (unsigned)nsp);
    double* dst = nsp > 1 ? scratch : out;
    const int64_t stride = (int64_t)s1 * s2;
#define RSVD_CROSS(T1, T2)                                                                                    \
    hipLaunchKernelGGL((cross_kernel<T1, T2>), grid, dim3(256), 0, st, (const T1*)P1, ld1, s1, (const T2*)P2, \
                       ld2, s2, len, symmetric, dst, stride, chunk, enable)
    if (dtype1 == RSVD_F32 && dtype2 == RSVD_F32) RSVD_CROSS(float, float);
    else if (dtype1 == RSVD_F64 && dtype2 == RSVD_F64) RSVD_CROSS(double, double);
    else if (dtype1 == RSVD_F32 && dtype2 == RSVD_F64) RSVD_CROSS(float, double);
    else if (dtype1 == RSVD_F64 && dtype2 == RSVD_F32) RSVD_CROSS(double, float);
    else return RSVD_EUNSUPPORTED;
#undef RSVD_CROSS
    RSVD_LAUNCH_CHECK();
    if (nsp > 1) {
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(stride, 256), 4096);
        hipLaunchKernelGGL(sum_parts_f64_kernel, dim3(blocks), dim3(256), 0, st, (const double*)scratch, (int)nsp,
                           stride, stride, out, enable);
        RSVD_LAUNCH_CHECK();
    }
    return RSVD_OK;
}

bool chol_fits_lds(int s) { return (size_t)s * (s + 1) * sizeof(double) <= 136 * 1024; }

rsvd_status run_chol_inv(const double* G, int s, int64_t len, double* R, double* Rinv, double* gscratch,
                         uint32_t* status, int* need_more, const int* enable, hipStream_t st) {
    const double eps = 2.220446049250313e-16;
    const double shift_factor = 11.0 * ((double)len * s + (double)s * (s + 1)) * eps;
    const bool lds = chol_fits_lds(s);
    const size_t shmem = lds ? (size_t)s * (s + 1) * sizeof(double) : 0;
    if (shmem > 0 && hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_inv_kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem) != hipSuccess)
        return RSVD_EHIP;
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(64), shmem, st, G, s, shift_factor, R, Rinv,
                       lds ? nullptr : gscratch, status, need_more, enable);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_trmm_upper(const double* R, double* Racc, double* tmp, int s, int side, const int* enable,
                           hipStream_t st) {
    hipLaunchKernelGGL(trmm_upper_kernel, dim3(1), dim3(1024), 0, st, R, Racc, tmp, s, side, enable);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_apply_coeff(int dtype_in, const void* IN, int64_t ldi, int s_in, int64_t len, const double* C,
                            int64_t ldc, int s_out, int triangular, double alpha, double beta, int dtype_out,
                            void* OUT, int64_t ldo, const int* enable, hipStream_t st) {
    if (s_out > 256) return RSVD_EUNSUPPORTED;
    constexpr int NI = 1;
    dim3 grid((unsigned)ceil_div(len, 4 * 16 * NI));
#define RSVD_APPLY(TI, TO)                                                                                       \
    hipLaunchKernelGGL((apply_coeff_kernel<TI, TO, NI>), grid, dim3(256), 0, st, (const TI*)IN, ldi, s_in, len, \
                       C, ldc, s_out, triangular, alpha, beta, (TO*)OUT, ldo, enable)
    if (dtype_in == RSVD_F32 && dtype_out == RSVD_F32) RSVD_APPLY(float, float);
    else if (dtype_in == RSVD_F64 && dtype_out == RSVD_F64) RSVD_APPLY(double, double);
    else if (dtype_in == RSVD_F64 && dtype_out == RSVD_F32) RSVD_APPLY(double, float);
    else if (dtype_in == RSVD_F32 && dtype_out == RSVD_F64) RSVD_APPLY(float, double);
    else return RSVD_EUNSUPPORTED;
#undef RSVD_APPLY
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_apply_rinv(int dtype_in, const void* YT, int64_t ldy, int s, int64_t len, const double* Rinv,
                           int dtype_out, void* QT, int64_t ldq, const int* enable, hipStream_t st) {
    return run_apply_coeff(dtype_in, YT, ldy, s, len, Rinv, s, s, 1, 1.0, 0.0, dtype_out, QT, ldq, enable, st);
}
