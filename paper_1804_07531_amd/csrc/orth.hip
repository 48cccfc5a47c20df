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
#include "launch.h"
#include "orth.h"

namespace {

// Four consecutive values of a panel row, loaded with one or two 16-byte loads
// and read as FP64 when used.
template <typename T> struct raw4;
template <> struct raw4<float> {
    floatx4 v;
    __device__ __forceinline__ void load(const float* p) { v = *reinterpret_cast<const floatx4*>(p); }
    __device__ __forceinline__ double get(int t) const { return v[t]; }
};
template <> struct raw4<double> {
    double2 a, b;
    __device__ __forceinline__ void load(const double* p) {
        a = *reinterpret_cast<const double2*>(p);
        b = *reinterpret_cast<const double2*>(p + 2);
    }
    __device__ __forceinline__ double get(int t) const { return t == 0 ? a.x : t == 1 ? a.y : t == 2 ? b.x : b.y; }
};

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
struct cross_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const T1*  P1;
        int64_t ld1;
        int s1;
        const T2*  P2;
        int64_t ld2;
        int s2;
        int64_t len;
        int symmetric;
        double*  out;
        int64_t split_stride;
        int64_t chunk;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [P1, ld1, s1, P2, ld2, s2, len, symmetric, out, split_stride, chunk, enable] = args_;
        if (enable && *enable == 0) return;
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int g = lane >> 4, i = lane & 15;
        const int nt1 = (s1 + 15) / 16, nt2 = (s2 + 15) / 16;
        int64_t task = (int64_t)vg.bx * 4 + wave;
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
        const int64_t kb = (int64_t)vg.by * chunk;
        const int64_t ke = std::min<int64_t>(len, kb + chunk);
        const int ra = 16 * ta + i, rb = 16 * tb + i;
        const bool oka = ra < s1, okb = rb < s2;
        const T1* pa = P1 + (int64_t)(oka ? ra : 0) * ld1;
        const T2* pb = P2 + (int64_t)(okb ? rb : 0) * ld2;
        const bool vec = (((uintptr_t)P1 | (uintptr_t)P2) & 15) == 0 && ld1 % 4 == 0 && ld2 % 4 == 0 && kb % 4 == 0;
        doublex4 acc = {0, 0, 0, 0};
        int64_t k = kb;
        if (sizeof(T1) == 4 && sizeof(T2) == 4 && vec) {
            // FP32 panels, whole 16-wide steps: unguarded 16-byte loads kept D steps
            // ahead of the products, so that a wave waits on L2 once per D steps
            // instead of once per step (a row past s1 or s2 reads row 0 and is
            // zeroed after the load).  FP64 Grams are small here and were slower.
            constexpr int D = 4;
            const int64_t nfull = (ke - kb) / 16;
            raw4<T1> ra[D];
            raw4<T2> rb[D];
            auto fetch = [&](int d, int64_t step) {
                ra[d].load(pa + kb + 16 * step + 4 * g);
                rb[d].load(pb + kb + 16 * step + 4 * g);
            };
            auto products = [&](const raw4<T1>& va, const raw4<T2>& vb) {
    #pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(oka ? va.get(t) : 0.0, okb ? vb.get(t) : 0.0, acc, 0, 0,
                                                               0);
            };
    #pragma unroll
            for (int d = 0; d < D; ++d)
                if (d < nfull) fetch(d, d);
            int64_t t = 0;
            for (; t + D <= nfull; t += D) {
    #pragma unroll
                for (int d = 0; d < D; ++d) {
                    const raw4<T1> va = ra[d];
                    const raw4<T2> vb = rb[d];
                    if (t + d + D < nfull) fetch(d, t + d + D);
                    products(va, vb);
                }
            }
    #pragma unroll
            for (int d = 0; d < D; ++d)
                if (t + d < nfull) products(ra[d], rb[d]);
            k = kb + 16 * nfull;
        }
        for (; k < ke; k += 16) {
            const int64_t kk = k + 4 * g;
            double a[4], b[4];
            load4d(pa + kk, kk, ke, oka, vec, a);
            load4d(pb + kk, kk, ke, okb, vec, b);
    #pragma unroll
            for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], acc, 0, 0, 0);
        }
        double* o = out + (int64_t)vg.by * split_stride;
    #pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * ta + mfma16<double>::row(g, r), col = 16 * tb + i;
            if (row < s1 && col < s2) {
                o[(int64_t)row * s2 + col] = acc[r];
                if (symmetric && ta != tb) o[(int64_t)col * s2 + row] = acc[r];
            }
        }
    }
};

struct sum_parts_f64_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const double*  parts;
        int nparts;
        int64_t stride;
        int64_t total;
        double*  out;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [parts, nparts, stride, total, out, enable] = args_;
        if (enable && *enable == 0) return;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)vg.gx * blockDim.x) {
            // partials in order p = 0, 1, ...; sixteen loads go out before their sums
            double acc = parts[e];
            int p = 1;
            for (; p + 16 <= nparts; p += 16) {
                double v[16];
    #pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = parts[(int64_t)(p + u) * stride + e];
    #pragma unroll
                for (int u = 0; u < 16; ++u) acc += v[u];
            }
            for (; p < nparts; ++p) acc += parts[(int64_t)p * stride + e];
            out[e] = acc;
        }
    }
};

// ---------------------------------------------------------------------------
// Cholesky factorization G = L L^T (L lower), R = L^T and R^-1, blocked in
// 16 x 16 tiles for one workgroup of four waves.
//
// For each block column J: one wave factors the diagonal tile (right-looking,
// in a small LDS tile) and inverts it; the panel tiles below become
// L_IJ = A_IJ L_JJ^-T and the trailing tiles are updated
// A_IK -= L_IJ L_KJ^T, both as 16x16x16 FP64 matrix-core products spread
// over the waves.  L^-1 is then formed one block diagonal at a time,
// Linv_IJ = -Linv_II sum_{K=J..I-1} L_IK Linv_KJ, and stored transposed in
// the unused upper half of the work matrix W, where it already reads as
// R^-1 = Linv^T.  The strict lower part of each diagonal inverse is kept
// transposed in the strict upper part of its diagonal tile and its diagonal
// in a separate vector.
//
// Pivoting rule: a first attempt without shift; if a pivot falls to
// <= 1e3 eps G_jj the factorization restarts on G + sigma I with
// sigma = 11 (len s + s (s+1)) eps trace(G) (trace(G) >= ||Y||_2^2), sets
// the SHIFTED status bit and *need_more = 1 (the caller then runs one more
// CholeskyQR round).  A pivot still <= 0 after the shift (only an all-zero
// column) leaves a degenerate column: zero in R, unit in the inverse, so
// that Q's column is zero and Y = Q R still holds (PIVOT status bit).
//
// f64 matrix-core convention used below: a tile product over k = 0..15 runs
// four steps t; lane l = 16 g + x supplies A[x][4t+g] and B[4t+g][x], and
// accumulator register r of lane (g, x) holds C[g + 4r][x].  That result
// layout is also the B-operand layout, so a product's result can feed the
// next product without moving data.
// ---------------------------------------------------------------------------
constexpr int CT = 16;  // tile size

__device__ __forceinline__ doublex4 mma_tile_abt(const double* __restrict__ A, int lda, const double* __restrict__ B,
                                                 int ldb, int g, int x, doublex4 acc) {
    // acc += A B^T for 16x16 tiles (row-major, leading dimensions lda, ldb)
#pragma unroll
    for (int t = 0; t < 4; ++t)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[x * lda + 4 * t + g], B[x * ldb + 4 * t + g], acc, 0, 0, 0);
    return acc;
}

constexpr int kCholThreads = 1024;   // 16 waves: the trailing updates are 16 tile tasks wide

template <bool IN_LDS>
__device__ __forceinline__ void chol_blocked_body(double* __restrict__ W, const double* __restrict__ G, int s,
                                                  double shift_factor, double near_id_tol2, double* __restrict__ R,
                                                  double* __restrict__ Rinv, uint32_t* status, int* need_more) {
    const int sp = (s + CT - 1) / CT * CT;       // padded order (padding: unit diagonal)
    const int nbk = sp / CT;
    const int ldw = sp + 1;
    __shared__ double tile[CT * (CT + 1)];      // diagonal tile being factored
    __shared__ double dinv_diag[512];           // diagonals of the diagonal-tile inverses
    __shared__ unsigned char unit_sh[512];
    constexpr int NW = kCholThreads / 64;
    __shared__ double red[NW];
    __shared__ double gdiag[512];               // diagonal of G: read in the column loop, kept off global memory
    __shared__ int fail;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, x = lane & 15;
    constexpr int ldt = CT + 1;

    // A Gram G = I + E close to the identity (the second CholeskyQR round) has the
    // factor R = I + up(E) + O(|E|^2) and R^-1 = I - up(E) + O(|E|^2), where up(E)
    // is the strict upper part of E plus half its diagonal (R^T R = I + E to first
    // order).  With |E|_F^2 <= near_id_tol2 the second-order terms stay below
    // near_id_tol2 / 2, and the factors are written in that closed form.
    if (near_id_tol2 > 0.0) {
        double e2 = 0.0;
        for (int e = tid; e < s * s; e += kCholThreads) {
            const int a = e / s, b = e % s;
            if (b > a) continue;
            const double v = G[(int64_t)a * s + b] - (a == b ? 1.0 : 0.0);
            e2 += (a == b ? 1.0 : 2.0) * v * v;
        }
        for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off);
        if (lane == 0) red[wave] = e2;
        __syncthreads();
        double e2sum = 0.0;
        for (int w = 0; w < NW; ++w) e2sum += red[w];   // same order in every thread
        __syncthreads();                                 // red is reused below
        if (e2sum <= near_id_tol2) {                     // uniform over the workgroup
            for (int e = tid; e < s * s; e += kCholThreads) {
                const int a = e / s, b = e % s;
                double f = 0.0;
                if (b > a) f = G[(int64_t)b * s + a];
                else if (b == a) f = 0.5 * (G[(int64_t)a * s + a] - 1.0);
                const double id = a == b ? 1.0 : 0.0;
                R[e] = b >= a ? id + f : 0.0;
                Rinv[e] = b >= a ? id - f : 0.0;
            }
            return;
        }
    }

    double tr = 0.0;
    for (int a = tid; a < s; a += kCholThreads) {
        const double d = G[(int64_t)a * s + a];
        gdiag[a] = d;
        tr += d;
    }
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off);
    if (lane == 0) red[wave] = tr;
    __syncthreads();
    double trace = 0.0;
    for (int w = 0; w < NW; ++w) trace += red[w];   // same order in every thread
    // a non-finite entry of the panel (from a non-finite A) makes its column's Gram
    // diagonal non-finite; the pivot rule below would turn that column into a zero
    // column and hide it, so it is reported here
    if (tid == 0 && !isfinite(trace)) rsvd_flag(status, RSVD_FLAG_NONFINITE);
    const double shift = shift_factor * trace;

    for (int attempt = 0; attempt < 2; ++attempt) {
        for (int e = tid; e < sp * sp; e += kCholThreads) {
            const int a = e / sp, b = e % sp;
            if (b > a) continue;
            double v;
            if (a < s) v = G[(int64_t)a * s + b] + ((attempt == 1 && a == b) ? shift : 0.0);
            else v = (a == b) ? 1.0 : 0.0;
            W[a * ldw + b] = v;
        }
        for (int a = tid; a < sp; a += kCholThreads) unit_sh[a] = 0;
        if (tid == 0) fail = 0;
        __syncthreads();
        for (int J = 0; J < nbk; ++J) {
            const int j0 = J * CT;
            // ---- diagonal tile: factor and invert (wave 0, in LDS)
            if (wave == 0) {
                for (int e = lane; e < CT * CT; e += 64) {
                    const int r = e / CT, c = e % CT;
                    tile[r * ldt + c] = c <= r ? W[(j0 + r) * ldw + j0 + c] : 0.0;
                }
                bool failed = false;
                for (int j = 0; j < CT; ++j) {
                    const double d = tile[j * ldt + j];
                    bool unit_col = false;
                    const int gj = j0 + j;
                    if (gj < s) {
                        if (attempt == 0) {
                            if (!(d > 1e3 * 2.220446049250313e-16 * gdiag[gj]) || !(d > 0.0)) {
                                failed = true;   // uniform over the wave
                                break;
                            }
                        } else if (!(d > 0.0)) {
                            unit_col = true;
                        }
                    }
                    const double rjj = unit_col ? 1.0 : sqrt(d);
                    const double inv = 1.0 / rjj;
                    if (lane > j && lane < CT) tile[lane * ldt + j] = unit_col ? 0.0 : tile[lane * ldt + j] * inv;
                    if (lane == 0) {
                        tile[j * ldt + j] = rjj;
                        if (unit_col) {
                            unit_sh[gj] = 1;
                            rsvd_flag(status, RSVD_FLAG_PIVOT);
                        }
                    }
                    // trailing part of the tile: lanes (g, x): row x, columns j+1+g, j+5+g, ...
                    if (x > j) {
                        const double lxj = tile[x * ldt + j];
                        for (int c = j + 1 + g; c <= x; c += 4) tile[x * ldt + c] -= lxj * tile[c * ldt + j];
                    }
                }
                if (failed) {
                    if (lane == 0) fail = 1;
                } else {
                    // inverse of the lower-triangular tile: lane c (< 16) computes column c by
                    // forward substitution, Dinv[r][c] = -(sum_{l=c..r-1} L[r][l] Dinv[l][c]) / L[r][r]
                    double col[CT];
                    if (lane < CT) {
                        const int c = lane;
#pragma unroll
                        for (int r = 0; r < CT; ++r) {
                            double v = 0.0;
                            if (r == c) v = 1.0 / tile[r * ldt + r];
                            else if (r > c) {
                                double acc = 0.0;
#pragma unroll
                                for (int l = 0; l < CT; ++l)
                                    if (l >= c && l < r) acc += tile[r * ldt + l] * col[l];
                                v = -acc / tile[r * ldt + r];
                            }
                            col[r] = v;
                        }
                    }
                    // write back L's tile (lower incl. diagonal) and Dinv (strict lower part
                    // transposed into the strict upper part, diagonal into dinv_diag)
                    for (int e = lane; e < CT * CT; e += 64) {
                        const int r = e / CT, c = e % CT;
                        if (c <= r) W[(j0 + r) * ldw + j0 + c] = tile[r * ldt + c];
                    }
                    if (lane < CT) {
                        const int c = lane;
                        dinv_diag[j0 + c] = col[c];
#pragma unroll
                        for (int r = 0; r < CT; ++r)
                            if (r > c) W[(j0 + c) * ldw + j0 + r] = col[r];
                    }
                }
            }
            __syncthreads();
            if (fail) break;   // uniform after the barrier
            // ---- panel: L_IJ = A_IJ Dinv_J^T for I > J
            for (int I = J + 1 + wave; I < nbk; I += NW) {
                double* aij = W + (I * CT) * ldw + j0;
                // B = Dinv_J (lower): B[c][k] = Dinv[c][k]; only k <= c nonzero
                double bv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 4 * t + g;
                    bv[t] = (k < x) ? W[(j0 + k) * ldw + j0 + x] : (k == x ? dinv_diag[j0 + x] : 0.0);
                }
                doublex4 acc = {0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aij[x * ldw + 4 * t + g], bv[t], acc, 0, 0, 0);
                // all loads of the tile precede these stores within the wave (the tile is the wave's alone)
#pragma unroll
                for (int r = 0; r < 4; ++r) aij[(g + 4 * r) * ldw + x] = acc[r];
            }
            __syncthreads();
            // ---- trailing update: A_IK -= L_IJ L_KJ^T for J < K <= I
            const int nt = nbk - J - 1;
            const int tasks = nt * (nt + 1) / 2;
            for (int task = wave; task < tasks; task += NW) {
                int I = 0, rem = task;  // enumerate (I, K) row by row of the trailing block triangle
                while (rem > I) {
                    rem -= I + 1;
                    ++I;
                }
                const int K = rem;
                const int gi = (J + 1 + I) * CT, gk = (J + 1 + K) * CT;
                doublex4 acc = {0, 0, 0, 0};
                acc = mma_tile_abt(W + gi * ldw + j0, ldw, W + gk * ldw + j0, ldw, g, x, acc);
                double* aik = W + gi * ldw + gk;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (I != K || x <= g + 4 * r) aik[(g + 4 * r) * ldw + x] -= acc[r];
            }
            __syncthreads();
        }
        if (!fail) break;
        if (tid == 0) {
            rsvd_flag(status, RSVD_FLAG_SHIFTED);
            if (need_more) *need_more = 1;
        }
        __syncthreads();
    }

    // ---- R = L^T (upper); a degenerate column gets a zero row in R
    for (int e = tid; e < s * s; e += kCholThreads) {
        const int a = e / s, b = e % s;
        R[e] = (b >= a && !(a == b && unit_sh[a])) ? W[b * ldw + a] : 0.0;
    }
    __syncthreads();
    // ---- L^-1 one block diagonal at a time; Linv_IJ^T stored in W's tile (J, I)
    for (int d = 1; d < nbk; ++d) {
        for (int J = wave; J + d < nbk; J += NW) {
            const int I = J + d;
            // T = sum_{K=J..I-1} L_IK Linv_KJ  (B operand: Linv_KJ[k][x])
            doublex4 tacc = {0, 0, 0, 0};
            for (int K = J; K < I; ++K) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 4 * t + g;
                    double b;
                    if (K == J) b = (k > x) ? W[(J * CT + x) * ldw + J * CT + k] : (k == x ? dinv_diag[J * CT + x] : 0.0);
                    else b = W[(J * CT + x) * ldw + K * CT + k];      // Linv_KJ^T stored at tile (J, K)
                    tacc = __builtin_amdgcn_mfma_f64_16x16x4f64(W[(I * CT + x) * ldw + K * CT + 4 * t + g], b, tacc,
                                                                0, 0, 0);
                }
            }
            // Linv_IJ = -Dinv_I T: the result layout of T is the B-operand layout
            doublex4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = 4 * t + g;
                // A operand is Dinv_I[x][k]: strict lower part lives transposed at W[I*CT + k][I*CT + x]
                const double av = (k < x) ? W[(I * CT + k) * ldw + I * CT + x] : (k == x ? dinv_diag[I * CT + x] : 0.0);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, tacc[t], acc, 0, 0, 0);
            }
            // store Linv_IJ[row][col] transposed at W[J*CT + col][I*CT + row]
#pragma unroll
            for (int r = 0; r < 4; ++r) W[(J * CT + x) * ldw + I * CT + g + 4 * r] = -acc[r];
        }
        __syncthreads();
    }
    // ---- R^-1 = Linv^T: upper part; diagonal tiles from the tile inverses
    for (int e = tid; e < s * s; e += kCholThreads) {
        const int a = e / s, b = e % s;
        double v = 0.0;
        if (b > a) v = W[a * ldw + b];              // same tile: Dinv strict lower transposed; else Linv^T
        else if (b == a) v = dinv_diag[a];
        Rinv[e] = v;
    }
}

template <bool IN_LDS>
struct chol_inv_kernel_op {
    static constexpr int kThreads = kCholThreads;
    struct Args {
        const double*  G;
        int s;
        double shift_factor;
        double near_id_tol2;
        double*  R;
        double*  Rinv;
        double*  gscratch;
        uint32_t* status;
        int* need_more;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [G, s, shift_factor, near_id_tol2, R, Rinv, gscratch, status, need_more, enable] = args_;
        if (enable && *enable == 0) return;
        extern __shared__ double lds[];
        if constexpr (IN_LDS) chol_blocked_body<true>(lds, G, s, shift_factor, near_id_tol2, R, Rinv, status, need_more);
        else chol_blocked_body<false>(gscratch, G, s, shift_factor, near_id_tol2, R, Rinv, status, need_more);
    }
};

// ---------------------------------------------------------------------------
// Coefficient apply on panels (FP64 arithmetic):
//   OUT[a][x] = beta OUT[a][x] + alpha sum_b C[b][a] IN[b][x],  a < s_out, b < s_in.
// With C = R^-1 this is Q^T = R^-T Y^T.  One wave owns 16*NI columns and
// every output row (s_out <= 16 MT <= 256; MT of 8, 12, 14 or 16 tiles by
// s_out, fewer tiles leaving room for more waves); the four waves share the
// rows of C, staged through LDS 16 at a time.  OUT may alias IN (s_in ==
// s_out, beta == 0) because a wave reads all rows of its columns before
// writing any.  `triangular` skips the blocks of an upper-triangular C that
// are zero.
// ---------------------------------------------------------------------------
template <typename TI, typename TO, int NI, int MT, bool TOUT = false>
struct apply_coeff_kernel_op {
    // TOUT: OUT is row-major len x s_out (OUT[x * ldo + a]) instead of a panel
    // MT: output tiles of 16 rows a wave can hold (s_out <= 16 MT)
    static constexpr int kThreads = 256;
    struct Args {
        const TI*  IN;
        int64_t ldi;
        int s_in;
        int64_t len;
        const double*  C;
        int64_t ldc;
        int s_out;
        int triangular;
        int a_off;
        double alpha;
        double beta;
        TO* OUT;
        int64_t ldo;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [IN, ldi, s_in, len, C, ldc, s_out, triangular, a_off, alpha, beta, OUT, ldo, enable] = args_;
        if (enable && *enable == 0) return;   // uniform over the grid
        // 16 rows of C at a time, staged through LDS for the whole workgroup (the four
        // waves share them; a wave past the end of the panel still helps to stage)
        __shared__ double cs[16][16 * MT + 1];
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int g = lane >> 4, i = lane & 15;
        const int64_t x0 = ((int64_t)vg.bx * 4 + wave) * (16 * NI);
        if (((int64_t)vg.bx * 4) * (16 * NI) >= len) return;   // uniform: no wave of this workgroup has columns
        const bool active = x0 < len;
        const int nt = (s_out + 15) / 16;
        doublex4 acc[MT][NI];
    #pragma unroll
        for (int a = 0; a < MT; ++a)
    #pragma unroll
            for (int c = 0; c < NI; ++c) acc[a][c] = doublex4{0, 0, 0, 0};
        // the panel values of a block of 16 rows are loaded one block ahead, so
        // that their HBM latency runs under the previous block's products.  The
        // loads read clamped, in-bounds positions and are masked only when the
        // next block takes them: a load guarded where it is issued compiled to a
        // branch and a wait per element, four round trips to memory per block.
        TI braw[NI][4];
        auto load_panel = [&](int kb0) {
    #pragma unroll
            for (int c = 0; c < NI; ++c) {
                const int64_t x = x0 + 16 * c + i;
                const int64_t xc = x < len ? x : len - 1;
    #pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int b = kb0 + 4 * g + t;
                    braw[c][t] = IN[(int64_t)(b < s_in ? b : s_in - 1) * ldi + xc];
                }
            }
        };
        if (active && s_in > 0) load_panel(0);
        for (int k0 = 0; k0 < s_in; k0 += 16) {
            __syncthreads();   // the previous block of C is consumed
            for (int e = threadIdx.x; e < 16 * 16 * nt; e += 256) {
                const int r = e / (16 * nt), a = e % (16 * nt);
                cs[r][a] = (k0 + r < s_in && a < s_out) ? C[(int64_t)(k0 + r) * ldc + a] : 0.0;
            }
            __syncthreads();
            if (!active) continue;
            double bv[NI][4];
    #pragma unroll
            for (int c = 0; c < NI; ++c) {
                const bool xin = x0 + 16 * c + i < len;
    #pragma unroll
                for (int t = 0; t < 4; ++t) bv[c][t] = (xin && k0 + 4 * g + t < s_in) ? (double)braw[c][t] : 0.0;
            }
            if (k0 + 16 < s_in) load_panel(k0 + 16);
            // fully unrolled with predicates (no break or continue), so that acc stays in registers
    #pragma unroll
            for (int ta = 0; ta < MT; ++ta) {
                const bool zero_block = triangular && a_off + 16 * ta + 15 < k0;   // C[b][a] = 0 for b > a
                if (ta < nt && !zero_block) {
                    double av[4];
    #pragma unroll
                    for (int t = 0; t < 4; ++t) av[t] = cs[4 * g + t][16 * ta + i];
    #pragma unroll
                    for (int t = 0; t < 4; ++t)
    #pragma unroll
                        for (int c = 0; c < NI; ++c)
                            acc[ta][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[c][t], acc[ta][c], 0, 0, 0);
                }
            }
        }
        if (!active) return;
    #pragma unroll
        for (int ta = 0; ta < MT; ++ta) {
    #pragma unroll
            for (int c = 0; c < NI; ++c) {
                const int64_t x = x0 + 16 * c + i;
    #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = 16 * ta + mfma16<double>::row(g, r);
                    if (ta < nt && x < len && a < s_out) {
                        TO* d = TOUT ? OUT + x * ldo + a : OUT + (int64_t)a * ldo + x;
                        const double prev = beta != 0.0 ? beta * (double)*d : 0.0;
                        *d = (TO)(prev + alpha * acc[ta][c][r]);
                    }
                }
            }
        }
    }
};

// The same apply for FP32 panels in and out, on FP32 matrix cores: the
// coefficients are rounded to FP32 as they are staged through LDS, 16 rows
// of C at a time for the whole workgroup, and sums are FP32.  The rounding
// this adds is of the order of the FP32 storage of the panels themselves
// (|OUT| error ~ s_in u32 |C| |IN|); the Gram and the factors stay FP64.
// A wave owns 32 columns (two 16-column tiles) and every output row.
template <int MT>   // output tiles of 16 rows a wave holds (s_out <= 16 MT)
struct apply_coeff_f32_kernel_op {
    static constexpr int kThreads = 256;
    static constexpr int NI = 2;
    struct Args {
        const float* IN;
        int64_t ldi;
        int s_in;
        int64_t len;
        const double* C;
        int64_t ldc;
        int s_out;
        int triangular;
        int a_off;
        double alpha;
        double beta;
        float* OUT;
        int64_t ldo;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& a) {
        if (a.enable && *a.enable == 0) return;
        __shared__ float cs[16][16 * MT + 4];   // C[k0 + b][a] for b < 16, a < s_out
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, i = lane & 15;
        const int64_t x0 = ((int64_t)vg.bx * 4 + wave) * (16 * NI);
        const int nt = (a.s_out + 15) / 16;
        floatx4 acc[MT][NI];
#pragma unroll
        for (int ta = 0; ta < MT; ++ta)
#pragma unroll
            for (int c = 0; c < NI; ++c) acc[ta][c] = floatx4{0, 0, 0, 0};
        // panel values one block ahead, read at clamped positions and masked when
        // taken (as in the FP64-sum apply above)
        float braw[NI][4];
        auto load_panel = [&](int kb0) {
#pragma unroll
            for (int c = 0; c < NI; ++c) {
                const int64_t x = x0 + 16 * c + i;
                const int64_t xc = x < a.len ? x : a.len - 1;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int b = kb0 + 4 * g + t;
                    braw[c][t] = a.IN[(int64_t)(b < a.s_in ? b : a.s_in - 1) * a.ldi + xc];
                }
            }
        };
        if (x0 < a.len && a.s_in > 0) load_panel(0);
        for (int k0 = 0; k0 < a.s_in; k0 += 16) {
            __syncthreads();   // the previous chunk of C has been read
            for (int e = tid; e < 16 * 16 * MT; e += 256) {
                const int b = e / (16 * MT), col = e % (16 * MT);
                cs[b][col] = (k0 + b < a.s_in && col < a.s_out) ? (float)a.C[(int64_t)(k0 + b) * a.ldc + col] : 0.0f;
            }
            __syncthreads();
            if (x0 >= a.len) continue;   // uniform over the wave; the barriers above are the workgroup's
            float bv[NI][4];
#pragma unroll
            for (int c = 0; c < NI; ++c) {
                const bool xin = x0 + 16 * c + i < a.len;
#pragma unroll
                for (int t = 0; t < 4; ++t) bv[c][t] = (xin && k0 + 4 * g + t < a.s_in) ? braw[c][t] : 0.0f;
            }
            if (k0 + 16 < a.s_in) load_panel(k0 + 16);
            // fully unrolled with predicates (no break or continue), so that acc stays in registers
#pragma unroll
            for (int ta = 0; ta < MT; ++ta) {
                const bool zero_block = a.triangular && a.a_off + 16 * ta + 15 < k0;   // C[b][a] = 0 for b > a
                if (ta < nt && !zero_block) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float av = cs[4 * g + t][16 * ta + i];
#pragma unroll
                        for (int c = 0; c < NI; ++c)
                            acc[ta][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[c][t], acc[ta][c], 0, 0, 0);
                    }
                }
            }
        }
        if (x0 >= a.len) return;
        const float alpha = (float)a.alpha, beta = (float)a.beta;
#pragma unroll
        for (int ta = 0; ta < MT; ++ta) {
#pragma unroll
            for (int c = 0; c < NI; ++c) {
                const int64_t x = x0 + 16 * c + i;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * ta + mfma16<float>::row(g, r);
                    if (ta < nt && x < a.len && row < a.s_out) {
                        float* d = a.OUT + (int64_t)row * a.ldo + x;
                        const float prev = beta != 0.0f ? beta * *d : 0.0f;
                        *d = prev + alpha * acc[ta][c][r];
                    }
                }
            }
        }
    }
};

// Upper-triangular products on s x s matrices: side 0: Racc <- R Racc;
// side 1: Racc <- Racc R.  One wave per 16x16 output tile (FP64 matrix
// cores), written to tmp; a second kernel copies tmp back.
struct trmm_upper_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const double*  R;
        const double*  Racc;
        double*  tmp;
        int s;
        int side;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [R, Racc, tmp, s, side, enable] = args_;
        if (enable && *enable == 0) return;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, x = lane & 15;
        const int nt = (s + 15) / 16;
        const int tile = vg.bx * 4 + wave;
        if (tile >= nt * nt) return;
        const int ti = tile / nt, tj = tile % nt;
        const double* A = side == 0 ? R : Racc;
        const double* B = side == 0 ? Racc : R;
        doublex4 acc = {0, 0, 0, 0};
        if (tj >= ti) {
            // the next block's values load (at clamped positions) during this block's
            // products and are masked when used, so that no load waits on its own
            const int row = ti * 16 + x, col = tj * 16 + x;
            const int rowc = row < s ? row : s - 1, colc = col < s ? col : s - 1;
            double ra[4], rb[4];
            auto load = [&](int kb) {
    #pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = kb * 16 + 4 * t + g, kc = k < s ? k : s - 1;
                    ra[t] = A[(int64_t)rowc * s + kc];
                    rb[t] = B[(int64_t)kc * s + colc];
                }
            };
            load(ti);
            for (int kb = ti; kb <= tj; ++kb) {      // both factors upper triangular
                double av[4], bv[4];
    #pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = kb * 16 + 4 * t + g;
                    av[t] = (row < s && k < s) ? ra[t] : 0.0;
                    bv[t] = (k < s && col < s) ? rb[t] : 0.0;
                }
                if (kb < tj) load(kb + 1);
    #pragma unroll
                for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], acc, 0, 0, 0);
            }
        }
    #pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = ti * 16 + g + 4 * r, col = tj * 16 + x;
            if (row < s && col < s) tmp[(int64_t)row * s + col] = (col >= row) ? acc[r] : 0.0;
        }
    }
};

struct copy_f64_enabled_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const double*  src;
        double*  dst;
        int64_t count;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [src, dst, count, enable] = args_;
        if (enable && *enable == 0) return;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)vg.gx * blockDim.x)
            dst[e] = src[e];
    }
};

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
    while (ceil_div(len, splits) > 2048 && splits < 512) splits *= 2;   // bound the serial length per workgroup
    return splits;
}

size_t cross_scratch_doubles(int s1, int s2, int64_t len, int symmetric, int num_cu) {
    const int64_t splits = cross_splits(s1, s2, len, symmetric, num_cu);
    return (size_t)splits * s1 * s2;
}

rsvd_status run_cross(int dtype1, const void* P1, int64_t ld1, int s1, int dtype2, const void* P2, int64_t ld2,
                      int s2, int64_t len, int symmetric, double* out, double* scratch, int num_cu,
                      const int* enable, hipStream_t st) {
    launch_phase();
    const int64_t splits = cross_splits(s1, s2, len, symmetric, num_cu);
    const int64_t chunk = round_up(ceil_div(len, splits), 16);
    const int64_t nsp = ceil_div(len, chunk);
    const int64_t nt1 = ceil_div(s1, 16), nt2 = ceil_div(s2, 16);
    const int64_t tasks = symmetric ? nt1 * (nt1 + 1) / 2 : nt1 * nt2;
    dim3 grid((unsigned)ceil_div(tasks, 4), (unsigned)nsp);
    double* dst = nsp > 1 ? scratch : out;
    const int64_t stride = (int64_t)s1 * s2;
#define RSVD_CROSS(T1, T2)                                                                                    \
    launch_op<cross_kernel_op<T1, T2>>(grid, dim3(256), 0, st, {(const T1*)P1, ld1, s1, (const T2*)P2, \
                       ld2, s2, len, symmetric, dst, stride, chunk, enable})
    if (dtype1 == RSVD_F32 && dtype2 == RSVD_F32) RSVD_CROSS(float, float);
    else if (dtype1 == RSVD_F64 && dtype2 == RSVD_F64) RSVD_CROSS(double, double);
    else if (dtype1 == RSVD_F32 && dtype2 == RSVD_F64) RSVD_CROSS(float, double);
    else if (dtype1 == RSVD_F64 && dtype2 == RSVD_F32) RSVD_CROSS(double, float);
    else return RSVD_EUNSUPPORTED;
#undef RSVD_CROSS
    RSVD_LAUNCH_CHECK();
    if (nsp > 1) {
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(stride, 256), 4096);
        launch_op<sum_parts_f64_kernel_op>(dim3(blocks), dim3(256), 0, st, {(const double*)scratch, (int)nsp, stride, stride, out, enable});
        RSVD_LAUNCH_CHECK();
    }
    return RSVD_OK;
}

bool chol_fits_lds(int s) {
    const size_t sp = (size_t)(s + 15) / 16 * 16;
    return sp * (sp + 1) * sizeof(double) <= 133 * 1024;
}

rsvd_status run_chol_inv(const double* G, int s, int64_t len, double* R, double* Rinv, double* gscratch,
                         uint32_t* status, int* need_more, const int* enable, hipStream_t st, double near_id_tol2) {
    launch_phase();
    const double eps = 2.220446049250313e-16;
    const double shift_factor = 11.0 * ((double)len * s + (double)s * (s + 1)) * eps;
    if (s > 512) return RSVD_EUNSUPPORTED;
    const bool lds = chol_fits_lds(s);
    const size_t sp = (size_t)(s + 15) / 16 * 16;
    const size_t shmem = lds ? sp * (sp + 1) * sizeof(double) : 0;
    if (lds) {
        if (hipFuncSetAttribute(op_single_fn<chol_inv_kernel_op<true>>(),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem) != hipSuccess)
            return RSVD_EHIP;
        launch_op<chol_inv_kernel_op<true>>(dim3(1), dim3(kCholThreads), shmem, st, {G, s, shift_factor, near_id_tol2, R, Rinv, nullptr, status, need_more, enable});
    } else {
        launch_op<chol_inv_kernel_op<false>>(dim3(1), dim3(kCholThreads), 0, st, {G, s, shift_factor, near_id_tol2, R, Rinv, gscratch, status, need_more, enable});
    }
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_trmm_upper(const double* R, double* Racc, double* tmp, int s, int side, const int* enable,
                           hipStream_t st) {
    launch_phase();
    const int nt = (s + 15) / 16;
    launch_op<trmm_upper_kernel_op>(dim3((unsigned)ceil_div((int64_t)nt * nt, 4)), dim3(256), 0, st, {R, Racc, tmp, s, side, enable});
    launch_op<copy_f64_enabled_kernel_op>(dim3((unsigned)ceil_div((int64_t)s * s, 256)), dim3(256), 0, st, {(const double*)tmp, Racc, (int64_t)s * s, enable});
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_apply_coeff(int dtype_in, const void* IN, int64_t ldi, int s_in, int64_t len, const double* C,
                            int64_t ldc, int s_out, int triangular, double alpha, double beta, int dtype_out,
                            void* OUT, int64_t ldo, const int* enable, hipStream_t st, bool f32_sums) {
    launch_phase();
    constexpr int NI = 1;
    dim3 grid((unsigned)ceil_div(len, 4 * 16 * NI));
    const size_t osz = dtype_out == RSVD_F64 ? 8 : 4;
    // output rows in one slice up to 256 (the widest accumulator tile), else in
    // balanced slices of at most 224 rows (narrower tiles leave room for more waves)
    const int slices = s_out <= 256 ? 1 : (s_out + 223) / 224;
    const int slice = slices == 1 ? s_out : round_up((s_out + slices - 1) / slices, 16);
    for (int a0 = 0; a0 < s_out; a0 += slice) {
        const int so = std::min(slice, s_out - a0);
        const double* Cs = C + a0;
        void* Os = (char*)OUT + (size_t)a0 * ldo * osz;
#define RSVD_APPLY_MT(TI, TO, MT)                                                                                 \
    launch_op<apply_coeff_kernel_op<TI, TO, NI, MT>>(grid, dim3(256), 0, st, {(const TI*)IN, ldi, s_in, len, \
                       Cs, ldc, so, triangular, a0, alpha, beta, (TO*)Os, ldo, enable})
#define RSVD_APPLY(TI, TO)                                                                                       \
    do {                                                                                                         \
        if (so <= 128) RSVD_APPLY_MT(TI, TO, 8);                                                                 \
        else if (so <= 192) RSVD_APPLY_MT(TI, TO, 12);                                                           \
        else if (so <= 224) RSVD_APPLY_MT(TI, TO, 14);                                                           \
        else RSVD_APPLY_MT(TI, TO, 16);                                                                          \
    } while (0)
        if (dtype_in == RSVD_F32 && dtype_out == RSVD_F32 && f32_sums) {
            auto f32 = [&](auto op) {
                using Op = decltype(op);
                launch_op<Op>(dim3((unsigned)ceil_div(len, 4 * 16 * Op::NI)), dim3(256), 0, st,
                              {(const float*)IN, ldi, s_in, len, Cs, ldc, so, triangular, a0, alpha, beta,
                                       (float*)Os, ldo, enable});
            };
            if (so <= 128) f32(apply_coeff_f32_kernel_op<8>{});
            else if (so <= 192) f32(apply_coeff_f32_kernel_op<12>{});
            else if (so <= 224) f32(apply_coeff_f32_kernel_op<14>{});
            else f32(apply_coeff_f32_kernel_op<16>{});
        } else if (dtype_in == RSVD_F32 && dtype_out == RSVD_F32) RSVD_APPLY(float, float);
        else if (dtype_in == RSVD_F64 && dtype_out == RSVD_F64) RSVD_APPLY(double, double);
        else if (dtype_in == RSVD_F64 && dtype_out == RSVD_F32) RSVD_APPLY(double, float);
        else if (dtype_in == RSVD_F32 && dtype_out == RSVD_F64) RSVD_APPLY(float, double);
        else return RSVD_EUNSUPPORTED;
#undef RSVD_APPLY
#undef RSVD_APPLY_MT
        RSVD_LAUNCH_CHECK();
    }
    return RSVD_OK;
}

struct copy_panel_kernel_f32_op {
    static constexpr int kThreads = 256;
    struct Args {
        const float*  src;
        int64_t lds;
        float*  dst;
        int64_t ldd;
        int rows;
        int64_t cols;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [src, lds, dst, ldd, rows, cols, enable] = args_;
        if (enable && *enable == 0) return;
        const int64_t total = (int64_t)rows * cols;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)vg.gx * blockDim.x)
            dst[(e / cols) * ldd + e % cols] = src[(e / cols) * lds + e % cols];
    }
};

struct copy_panel_kernel_f64_op {
    static constexpr int kThreads = 256;
    struct Args {
        const double*  src;
        int64_t lds;
        double*  dst;
        int64_t ldd;
        int rows;
        int64_t cols;
        const int* enable;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [src, lds, dst, ldd, rows, cols, enable] = args_;
        if (enable && *enable == 0) return;
        const int64_t total = (int64_t)rows * cols;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)vg.gx * blockDim.x)
            dst[(e / cols) * ldd + e % cols] = src[(e / cols) * lds + e % cols];
    }
};

rsvd_status run_copy_panel(int dtype, const void* src, int64_t lds, void* dst, int64_t ldd, int rows, int64_t cols,
                           const int* enable, hipStream_t st) {
    launch_phase();
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div((int64_t)rows * cols, 256), 16384);
    if (dtype == RSVD_F64)
        launch_op<copy_panel_kernel_f64_op>(dim3(blocks), dim3(256), 0, st, {(const double*)src, lds, (double*)dst, ldd, rows, cols, enable});
    else if (dtype == RSVD_F32)
        launch_op<copy_panel_kernel_f32_op>(dim3(blocks), dim3(256), 0, st, {(const float*)src, lds, (float*)dst, ldd, rows, cols, enable});
    else
        return RSVD_EUNSUPPORTED;
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_lift_rows(int dtype_p, const void* P, int64_t ldp, int s, int64_t len, const double* F, int ldf,
                          int k, int dtype_o, void* out, int64_t ldo, hipStream_t st) {
    launch_phase();
    if (s > 512) return RSVD_EUNSUPPORTED;
    constexpr int NI = 1;
    dim3 grid((unsigned)ceil_div(len, 4 * 16 * NI));
    const size_t osz = dtype_o == RSVD_F64 ? 8 : 4;
    const int slices = k <= 256 ? 1 : (k + 223) / 224;
    const int slice = slices == 1 ? k : round_up((k + slices - 1) / slices, 16);
    for (int c0 = 0; c0 < k; c0 += slice) {
        const int kc = std::min(slice, k - c0);
        const double* Fs = F + c0;
        void* Os = (char*)out + (size_t)c0 * osz;   // columns c0.. of the row-major output
#define RSVD_LIFT_MT(TP, TO, MT)                                                                                 \
    launch_op<apply_coeff_kernel_op<TP, TO, NI, MT, true>>(grid, dim3(256), 0, st,                               \
        {(const TP*)P, ldp, s, len, Fs, ldf, kc, 0, 0, 1.0, 0.0, \
                                                          (TO*)Os, ldo, nullptr})
#define RSVD_LIFT(TP, TO)                                                                                        \
    do {                                                                                                         \
        if (kc <= 128) RSVD_LIFT_MT(TP, TO, 8);                                                                  \
        else if (kc <= 192) RSVD_LIFT_MT(TP, TO, 12);                                                            \
        else if (kc <= 224) RSVD_LIFT_MT(TP, TO, 14);                                                            \
        else RSVD_LIFT_MT(TP, TO, 16);                                                                           \
    } while (0)
        if (dtype_p == RSVD_F32 && dtype_o == RSVD_F32) RSVD_LIFT(float, float);
        else if (dtype_p == RSVD_F64 && dtype_o == RSVD_F64) RSVD_LIFT(double, double);
        else if (dtype_p == RSVD_F64 && dtype_o == RSVD_F32) RSVD_LIFT(double, float);
        else return RSVD_EUNSUPPORTED;
#undef RSVD_LIFT
#undef RSVD_LIFT_MT
        RSVD_LAUNCH_CHECK();
    }
    return RSVD_OK;
}

rsvd_status run_apply_rinv(int dtype_in, const void* YT, int64_t ldy, int s, int64_t len, const double* Rinv,
                           int dtype_out, void* QT, int64_t ldq, const int* enable, hipStream_t st,
                           bool f32_sums) {
    return run_apply_coeff(dtype_in, YT, ldy, s, len, Rinv, s, s, 1, 1.0, 0.0, dtype_out, QT, ldq, enable, st,
                           f32_sums);
}
