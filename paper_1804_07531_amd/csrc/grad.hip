// Kernels of the hand-written adjoint of the row-sweep block Krylov method:
// the dense gradient assembly G = alpha A + sum_seg scale_seg L_seg^T R_seg
// from thin panels, ||A||_F^2, and small FP64 coefficient builders.
#include <algorithm>

#include "common.h"
#include "grad.h"

namespace {

// ---------------------------------------------------------------------------
// G (m x n, row-major, ldg) = alpha A + sum over segments of
// scale * L^T R, with L a panel (rows x m) and R a panel (rows x n).  One
// workgroup per 64 x 64 tile of G; each wave owns a 32 x 32 quarter (2 x 2
// matrix-core tiles); 16 panel rows at a time are staged through LDS.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
outer_update_kernel(const T* __restrict__ A, int64_t lda, double alpha, int64_t m, int64_t n, OuterSegs<T> segs,
                    T* __restrict__ G, int64_t ldg) {
    __shared__ T Ls[16][64 + 1];
    __shared__ T Rs[16][64 + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, x = lane & 15;
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    typename mfma16<T>::acc acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = {0, 0, 0, 0};
    for (int sg = 0; sg < segs.count; ++sg) {
        const T* L = segs.L[sg];
        const T* R = segs.R[sg];
        const int64_t ldl = segs.ldl[sg], ldr = segs.ldr[sg];
        const int rows = segs.rows[sg];
        const T sc = (T)segs.scale[sg];
        for (int t0 = 0; t0 < rows; t0 += 16) {
            __syncthreads();
            for (int e = tid; e < 16 * 64; e += 256) {
                const int t = e >> 6, c = e & 63;
                const bool tr = t0 + t < rows;
                Ls[t][c] = (tr && i0 + c < m) ? sc * L[(int64_t)(t0 + t) * ldl + i0 + c] : (T)0;
                Rs[t][c] = (tr && j0 + c < n) ? R[(int64_t)(t0 + t) * ldr + j0 + c] : (T)0;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = 4 * q + g;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = mfma16<T>::step(Ls[t][wi + 16 * a + x], Rs[t][wj + 16 * b + x], acc[a][b]);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + wi + 16 * a + mfma16<T>::row(g, r);
                const int64_t j = j0 + wj + 16 * b + x;
                if (i < m && j < n) G[i * ldg + j] = (T)(alpha * (double)A[i * lda + j]) + acc[a][b][r];
            }
}

// ---------------------------------------------------------------------------
// The same update in FP32 for panels whose rows start on 16-byte boundaries
// (m, n and every leading dimension multiples of 4).  No LDS: each wave owns
// a 64 x 64 block of G and takes its operands straight from the panels, one
// float4 per lane and panel for every 4 panel rows.  Lane 16 g + x loads
// L[t + g][i0 + 4 x .. i0 + 4 x + 3]; element c of that float4 feeds the
// 16x16x4 product whose 16 output rows are i0 + 4 rho + c (rho = 0..15), so
// the 4 x 4 products of a step cover the wave's 64 rows and 64 columns
// (columns likewise from R).  A lane's four accumulators of one output row
// then hold four adjacent columns, which go out as one float4 beside one
// float4 load of A.  Four waves per workgroup make a 128 x 128 tile; the
// workgroups of one XCD (workgroup id modulo 8) take contiguous groups of
// 8 x 8 tiles, so the panel rows they stream stay in that XCD's L2.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
outer_update_f32x4_kernel(const float* __restrict__ A, int64_t lda, float alpha, int64_t m, int64_t n,
                          OuterSegs<float> segs, float* __restrict__ G, int64_t ldg, int tiles_m, int tiles_n) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, x = lane & 15;
    // workgroup id -> tile: XCD-contiguous, then 8 x 8 groups walked down the rows
    const int ntiles = tiles_m * tiles_n;
    const int per_xcd = (ntiles + 7) / 8;
    const int lin = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (lin >= ntiles) return;
    const int group_rows = 8;
    const int gsize = group_rows * tiles_n;
    const int grp = lin / gsize, in_grp = lin % gsize;
    const int rows_here = min(group_rows, tiles_m - grp * group_rows);
    const int tm = grp * group_rows + in_grp % rows_here, tn = in_grp / rows_here;
    const int64_t i0 = (int64_t)tm * 128 + (wave >> 1) * 64, j0 = (int64_t)tn * 128 + (wave & 1) * 64;
    const int64_t li = i0 + 4 * x, rj = j0 + 4 * x;   // this lane's 4 rows (columns) of the operands
    const bool lin_ok = li < m, rin_ok = rj < n;

    floatx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0, 0, 0, 0};
    const floatx4 zero = {0, 0, 0, 0};
    for (int sg = 0; sg < segs.count; ++sg) {
        const float* L = segs.L[sg] + li;
        const float* R = segs.R[sg] + rj;
        const int64_t ldl = segs.ldl[sg], ldr = segs.ldr[sg];
        const int rows = segs.rows[sg];
        const float sc = (float)segs.scale[sg];
        auto load = [&](int t, floatx4& lv, floatx4& rv) {
            const bool ok = t + g < rows;
            lv = (ok && lin_ok) ? *reinterpret_cast<const floatx4*>(L + (int64_t)(t + g) * ldl) : zero;
            rv = (ok && rin_ok) ? *reinterpret_cast<const floatx4*>(R + (int64_t)(t + g) * ldr) : zero;
        };
        auto step = [&](floatx4 lv, const floatx4& rv) {
            lv *= sc;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(lv[a], rv[b], acc[a][b], 0, 0, 0);
        };
        // steps of 4 panel rows, the loads of two steps in flight ahead of
        // the one being multiplied (loads past the last row give zeros and
        // touch no memory)
        const int nst = (rows + 3) / 4;
        floatx4 l0, r0, l1, r1, l2, r2;
        load(0, l0, r0);
        load(4, l1, r1);
        int j = 0;
        for (; j + 3 <= nst; j += 3) {
            load(4 * (j + 2), l2, r2);
            step(l0, r0);
            load(4 * (j + 3), l0, r0);
            step(l1, r1);
            load(4 * (j + 4), l1, r1);
            step(l2, r2);
        }
        if (j < nst) step(l0, r0);
        if (j + 1 < nst) step(l1, r1);
    }
    // G = alpha A + acc: accumulator r of lane (g, x) in product (a, b) is
    // row i0 + 4 (4 g + r) + a, column j0 + 4 x + b
    if (!rin_ok) return;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + 4 * (4 * g + r) + a;
            if (i >= m) continue;
            const floatx4 av = *reinterpret_cast<const floatx4*>(A + i * lda + rj);
            floatx4 o;
#pragma unroll
            for (int b = 0; b < 4; ++b) o[b] = alpha * av[b] + acc[a][b][r];
            *reinterpret_cast<floatx4*>(G + i * ldg + rj) = o;
        }
}

// Partial sums of squares of A (FP64 accumulation), one per block.
template <typename T>
__global__ void __launch_bounds__(256)
frob_partial_kernel(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n, double* __restrict__ part) {
    __shared__ double red[4];
    double acc = 0.0;
    const int64_t total = m * n;
    // element e = r n + c of a grid-stride loop; (r, c) advance by the stride
    // instead of a 64-bit division per element, four loads ahead of their sums
    const int64_t S = (int64_t)gridDim.x * blockDim.x;
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < total) {
        int64_t r = e / n, c = e % n;
        const int64_t dr = S / n, dc = S % n;
        auto advance = [&]() {
            r += dr;
            c += dc;
            if (c >= n) {
                c -= n;
                ++r;
            }
        };
        for (; e + 3 * S < total; e += 4 * S) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[u] = (double)A[r * lda + c];
                advance();
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += v[u] * v[u];
        }
        for (; e < total; e += S) {
            const double v = (double)A[r * lda + c];
            acc += v * v;
            advance();
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// E = sum(part) - sum_i lam_i^2, in a fixed order (one thread).
__global__ void loss_e_kernel(const double* __restrict__ part, int nparts, const double* __restrict__ lam, int nl,
                              double* __restrict__ E) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double fa = 0.0, fb = 0.0;
    int i = 0;
    for (; i + 16 <= nparts; i += 16) {   // sixteen loads ahead of their sums, same order
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = part[i + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) fa += v[u];
    }
    for (; i < nparts; ++i) fa += part[i];
    for (int i = 0; i < nl; ++i) fb += lam[i] * lam[i];
    *E = fa - fb;
}

// Ctot ((k + sk) x sk) = Cb Cc with Cb[b][l] = dS_b U~[l][b] (b < k),
// -2 dE [b - k == l] (b >= k), and Cc = C2^T, where C2 (W_K S_K^-1, or R_K^-1
// when the TSVD of R_K was skipped) is the coefficient matrix the forward
// applied to form B^T.
__global__ void grad_coeff_kernel(const double* __restrict__ Ut, const double* __restrict__ dS, double dE, int k,
                                  const double* __restrict__ C2, int sk, double* __restrict__ C) {
    const int rows = k + sk;
    // consecutive threads take consecutive rows b of one column a: the reads of
    // Ut (row l, column b) are then coalesced and those of C2 (row a) broadcast
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rows * sk; e += gridDim.x * blockDim.x) {
        const int a = e / rows, b = e % rows;
        double v = 0.0;
        if (b < k) {
            const double d = dS ? dS[b] : 0.0;
            int l = 0;
            for (; l + 8 <= sk; l += 8) {   // eight terms' loads ahead of their sums, same order
                double u[8], w[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    u[q] = Ut[(int64_t)(l + q) * sk + b];
                    w[q] = C2[(int64_t)a * sk + l + q];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) v += u[q] * w[q];
            }
            for (; l < sk; ++l) v += Ut[(int64_t)l * sk + b] * C2[(int64_t)a * sk + l];
            v *= d;
        } else {
            const int l = b - k;
            v = -2.0 * dE * C2[(int64_t)a * sk + l];
        }
        C[(int64_t)b * sk + a] = v;
    }
}
// S = the symmetric matrix built from the upper triangle of N (s x s).
__global__ void sym_upper_kernel(const double* __restrict__ N, int s, double* __restrict__ S) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < s * s; e += gridDim.x * blockDim.x) {
        const int a = e / s, b = e % s;
        S[e] = a <= b ? N[e] : N[(int64_t)b * s + a];
    }
}

__global__ void transpose_f64_kernel(const double* __restrict__ X, int s, double* __restrict__ Y) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < s * s; e += gridDim.x * blockDim.x) {
        const int a = e / s, b = e % s;
        Y[(int64_t)b * s + a] = X[e];
    }
}

// Y[b][a] = X[b][a] * d[a] for a < cols (X with leading dimension ldx).
__global__ void scale_cols_kernel(const double* __restrict__ X, int ldx, int rows, int cols, const double* __restrict__ d,
                                  double* __restrict__ Y) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols; e += gridDim.x * blockDim.x) {
        const int b = e / cols, a = e % cols;
        Y[e] = X[(int64_t)b * ldx + a] * (d ? d[a] : 0.0);
    }
}

// Sets bit `bit` of *status when S[l] < tau S[0] for some l (the Krylov
// basis would be cut, which the adjoint does not model).
__global__ void rank_check_kernel(const double* __restrict__ S, int n, double tau, uint32_t* status, uint32_t bit,
                                  const int* enable) {
    if (enable && *enable == 0) return;   // no SVD was taken: nothing can be cut
    for (int l = threadIdx.x; l < n; l += blockDim.x)
        if (!(S[l] >= tau * S[0])) rsvd_flag(status, bit);
}

template <typename T>
__global__ void __launch_bounds__(256)
fill_zero_kernel(T* __restrict__ p, int64_t count) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = (T)0;
}

}  // namespace

int64_t frob_parts() { return 2048; }

rsvd_status run_frob_sq(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, double* part,
                        const double* lam, int nl, double* E, hipStream_t st) {
    const int nb = (int)std::min<int64_t>(frob_parts(), std::max<int64_t>(1, ceil_div(m * n, 256)));
    if (dtype == RSVD_F64)
        hipLaunchKernelGGL(frob_partial_kernel<double>, dim3(nb), dim3(256), 0, st, (const double*)A, lda, m, n, part);
    else if (dtype == RSVD_F32)
        hipLaunchKernelGGL(frob_partial_kernel<float>, dim3(nb), dim3(256), 0, st, (const float*)A, lda, m, n, part);
    else
        return RSVD_EUNSUPPORTED;
    hipLaunchKernelGGL(loss_e_kernel, dim3(1), dim3(64), 0, st, (const double*)part, nb, lam, nl, E);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

static bool aligned4(const void* p, int64_t ld) { return ((uintptr_t)p & 15) == 0 && ld % 4 == 0; }

template <typename T>
static rsvd_status outer_t(const T* A, int64_t lda, double alpha, int64_t m, int64_t n, const OuterSegs<T>& segs, T* G,
                           int64_t ldg, hipStream_t st) {
    if constexpr (sizeof(T) == 4) {
        bool vec = m % 4 == 0 && n % 4 == 0 && aligned4(A, lda) && aligned4(G, ldg);
        for (int i = 0; i < segs.count; ++i) vec = vec && aligned4(segs.L[i], segs.ldl[i]) && aligned4(segs.R[i], segs.ldr[i]);
        if (vec) {
            const int tiles_m = (int)ceil_div(m, 128), tiles_n = (int)ceil_div(n, 128);
            const int per_xcd = (int)ceil_div((int64_t)tiles_m * tiles_n, 8);
            hipLaunchKernelGGL(outer_update_f32x4_kernel, dim3((unsigned)(8 * per_xcd)), dim3(256), 0, st, A, lda,
                               (float)alpha, m, n, segs, G, ldg, tiles_m, tiles_n);
            RSVD_LAUNCH_CHECK();
            return RSVD_OK;
        }
    }
    dim3 grid((unsigned)ceil_div(n, 64), (unsigned)ceil_div(m, 64));
    hipLaunchKernelGGL(outer_update_kernel<T>, grid, dim3(256), 0, st, A, lda, alpha, m, n, segs, G, ldg);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_outer_update_f32(const float* A, int64_t lda, double alpha, int64_t m, int64_t n,
                                 const OuterSegs<float>& segs, float* G, int64_t ldg, hipStream_t st) {
    return outer_t<float>(A, lda, alpha, m, n, segs, G, ldg, st);
}

rsvd_status run_outer_update_f64(const double* A, int64_t lda, double alpha, int64_t m, int64_t n,
                                 const OuterSegs<double>& segs, double* G, int64_t ldg, hipStream_t st) {
    return outer_t<double>(A, lda, alpha, m, n, segs, G, ldg, st);
}

rsvd_status run_grad_coeff(const double* Ut, const double* dS, double dE, int k, const double* C2, int sk, double* C,
                           hipStream_t st) {
    hipLaunchKernelGGL(grad_coeff_kernel, dim3((unsigned)ceil_div((int64_t)(k + sk) * sk, 256)), dim3(256), 0, st, Ut,
                       dS, dE, k, C2, sk, C);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_sym_upper(const double* N, int s, double* S, hipStream_t st) {
    hipLaunchKernelGGL(sym_upper_kernel, dim3((unsigned)ceil_div((int64_t)s * s, 256)), dim3(256), 0, st, N, s, S);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_transpose_f64(const double* X, int s, double* Y, hipStream_t st) {
    hipLaunchKernelGGL(transpose_f64_kernel, dim3((unsigned)ceil_div((int64_t)s * s, 256)), dim3(256), 0, st, X, s, Y);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_scale_cols(const double* X, int ldx, int rows, int cols, const double* d, double* Y, hipStream_t st) {
    hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)std::max<int64_t>(1, ceil_div((int64_t)rows * cols, 256))),
                       dim3(256), 0, st, X, ldx, rows, cols, d, Y);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_rank_check(const double* S, int n, double tau, uint32_t* status, uint32_t bit, hipStream_t st,
                           const int* enable) {
    hipLaunchKernelGGL(rank_check_kernel, dim3(1), dim3(256), 0, st, S, n, tau, status, bit, enable);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_fill_zero(int dtype, void* p, int64_t count, hipStream_t st) {
    const unsigned blocks = (unsigned)std::min<int64_t>(std::max<int64_t>(1, ceil_div(count, 256)), 8192);
    if (dtype == RSVD_F64) hipLaunchKernelGGL(fill_zero_kernel<double>, dim3(blocks), dim3(256), 0, st, (double*)p, count);
    else hipLaunchKernelGGL(fill_zero_kernel<float>, dim3(blocks), dim3(256), 0, st, (float*)p, count);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}
