// The views of A (the paper's "products of A with a thin matrix", Sect. 1, 3).
//
// Every thin matrix is kept as a *panel*: its transpose, s x len, row-major
// (len = m for range-side matrices, n for co-range-side ones).  With that
// layout a lane's matrix-core operand is one contiguous 16-byte load along
// the contraction index, for A as well as for the thin operand.
//
//   range view    Y^T (s x m) = (A X)^T,   X given as X^T (s x n)
//   co-range view Z^T (s x n) = (A^T Y)^T, Y given as Y^T (s x m)
//
// Matrix-core layout (16x16x4, FP32 or FP64): lane l = 16 g + i supplies
// A_op[i][g] and B_op[g][j = i]; accumulator register r of lane l holds
// C[row(g, r)][i] (mfma16<T>::row).  Within one 16-wide step of the contraction index the k
// order is permuted: lane group g takes k = 4 g + t in sub-step t, so one
// 4-vector load per lane feeds four matrix-core steps.
//
// Neither view stages A through LDS: every wave owns a disjoint tile of A
// and streams it from HBM into registers; the thin operand is shared by the
// waves of a workgroup through the L1 cache.
#include <algorithm>

#include "common.h"
#include "views.h"

namespace {

template <typename T> struct vec4 { T x[4]; };

template <typename T>
__device__ __forceinline__ vec4<T> load4(const T* p) {
    vec4<T> v;
    if constexpr (sizeof(T) == 4) {
        const floatx4 f = *reinterpret_cast<const floatx4*>(p);
        v.x[0] = f[0]; v.x[1] = f[1]; v.x[2] = f[2]; v.x[3] = f[3];
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        v.x[0] = a.x; v.x[1] = a.y; v.x[2] = b.x; v.x[3] = b.y;
    }
    return v;
}

// Guarded scalar gather of p[0..3] (elements with k >= kmax read as 0).
template <typename T>
__device__ __forceinline__ vec4<T> load4_guard(const T* p, int64_t k, int64_t kmax, bool ok) {
    vec4<T> v;
#pragma unroll
    for (int t = 0; t < 4; ++t) v.x[t] = (ok && k + t < kmax) ? p[t] : T(0);
    return v;
}

// ---------------------------------------------------------------------------
// Range view: Y^T[j][r] = sum_c A[r][c] X^T[j][c]
// grid.x: row tiles of 64*MR... rows (4 waves x 16*MR rows); grid.y: K splits.
// Each wave: 16*MR rows x 16*NB thin columns, all in registers.
// ---------------------------------------------------------------------------
template <typename T, int NB, int MR, bool VEC>
__global__ void __launch_bounds__(256)
range_view_kernel(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                  const T* __restrict__ XT, int64_t ldx, int s,
                  T* __restrict__ out, int64_t ldo, int64_t split_stride, int64_t k_chunk, int accumulate) {
    typedef typename mfma16<T>::acc acc_t;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MR);
    if (row0 >= m) return;
    const int64_t kb = (int64_t)blockIdx.y * k_chunk;
    const int64_t ke = std::min<int64_t>(n, kb + k_chunk);

    acc_t acc[MR][NB];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const T* arow[MR];
    bool arow_ok[MR];
#pragma unroll
    for (int a = 0; a < MR; ++a) {
        const int64_t r = row0 + 16 * a + i;
        arow_ok[a] = r < m;
        arow[a] = A + (arow_ok[a] ? r : 0) * lda;
    }
    const T* xrow[NB];
    bool xrow_ok[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = 16 * b + i;
        xrow_ok[b] = j < s;
        xrow[b] = XT + (int64_t)(xrow_ok[b] ? j : 0) * ldx;
    }

    const int64_t kfull = kb + ((ke - kb) / 16) * 16;
    int64_t k = kb;
    if (VEC) {
        for (; k < kfull; k += 16) {
            const int64_t kk = k + 4 * g;
            vec4<T> av[MR], bv[NB];
#pragma unroll
            for (int a = 0; a < MR; ++a) av[a] = arow_ok[a] ? load4(arow[a] + kk) : vec4<T>{};
#pragma unroll
            for (int b = 0; b < NB; ++b) bv[b] = xrow_ok[b] ? load4(xrow[b] + kk) : vec4<T>{};
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int a = 0; a < MR; ++a)
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[a][b] = mfma16<T>::step(av[a].x[t], bv[b].x[t], acc[a][b]);
        }
    }
    for (; k < ke; k += 16) {  // tail (and the whole loop when A is not 16-byte aligned)
        const int64_t kk = k + 4 * g;
        vec4<T> av[MR], bv[NB];
#pragma unroll
        for (int a = 0; a < MR; ++a) av[a] = load4_guard(arow[a] + kk, kk, ke, arow_ok[a]);
#pragma unroll
        for (int b = 0; b < NB; ++b) bv[b] = load4_guard(xrow[b] + kk, kk, ke, xrow_ok[b]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int a = 0; a < MR; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[a][b] = mfma16<T>::step(av[a].x[t], bv[b].x[t], acc[a][b]);
    }

    T* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = 16 * b + i;
        if (j >= s) continue;
#pragma unroll
        for (int a = 0; a < MR; ++a) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + 16 * a + mfma16<T>::row(g, r);
                if (row < m) {
                    T* d = o + (int64_t)j * ldo + row;
                    *d = accumulate ? *d + acc[a][b][r] : acc[a][b][r];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Co-range view: Z^T[j][c] = sum_r A[r][c] Y^T[j][r]
// grid.x: column tiles (4 waves x 16*MR columns); grid.y: splits of the rows.
// ---------------------------------------------------------------------------
template <typename T, int NB, int MR, bool VEC>
__global__ void __launch_bounds__(256)
corange_view_kernel(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                    const T* __restrict__ YT, int64_t ldy, int s,
                    T* __restrict__ out, int64_t ldo, int64_t split_stride, int64_t r_chunk, int accumulate) {
    typedef typename mfma16<T>::acc acc_t;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    const int64_t col0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MR);
    if (col0 >= n) return;
    const int64_t rb = (int64_t)blockIdx.y * r_chunk;
    const int64_t re = std::min<int64_t>(m, rb + r_chunk);

    acc_t acc[MR][NB];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    bool col_ok[MR];
#pragma unroll
    for (int a = 0; a < MR; ++a) col_ok[a] = col0 + 16 * a + i < n;
    const T* yrow[NB];
    bool yrow_ok[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = 16 * b + i;
        yrow_ok[b] = j < s;
        yrow[b] = YT + (int64_t)(yrow_ok[b] ? j : 0) * ldy;
    }

    const int64_t rfull = rb + ((re - rb) / 16) * 16;
    int64_t r = rb;
    for (; r < rfull; r += 16) {
        const int64_t rr = r + 4 * g;
        vec4<T> av[MR], bv[NB];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const T* p = A + rr * lda + col0 + 16 * a + i;
#pragma unroll
            for (int t = 0; t < 4; ++t) av[a].x[t] = col_ok[a] ? p[t * lda] : T(0);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (VEC) bv[b] = yrow_ok[b] ? load4(yrow[b] + rr) : vec4<T>{};
            else bv[b] = load4_guard(yrow[b] + rr, rr, re, yrow_ok[b]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int a = 0; a < MR; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[a][b] = mfma16<T>::step(av[a].x[t], bv[b].x[t], acc[a][b]);
    }
    for (; r < re; r += 16) {
        const int64_t rr = r + 4 * g;
        vec4<T> av[MR], bv[NB];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const T* p = A + col0 + 16 * a + i;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                av[a].x[t] = (col_ok[a] && rr + t < re) ? p[(rr + t) * lda] : T(0);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) bv[b] = load4_guard(yrow[b] + rr, rr, re, yrow_ok[b]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int a = 0; a < MR; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[a][b] = mfma16<T>::step(av[a].x[t], bv[b].x[t], acc[a][b]);
    }

    T* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = 16 * b + i;
        if (j >= s) continue;
#pragma unroll
        for (int a = 0; a < MR; ++a) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t c = col0 + 16 * a + mfma16<T>::row(g, q);
                if (c < n) {
                    T* d = o + (int64_t)j * ldo + c;
                    *d = accumulate ? *d + acc[a][b][q] : acc[a][b][q];
                }
            }
        }
    }
}

// Sum of `parts` partial panels (rows x cols, leading dimension ld, parts
// spaced split_stride apart) into out, in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256)
reduce_parts_kernel(const T* __restrict__ parts, int nparts, int64_t split_stride, int64_t rows, int64_t cols,
                    int64_t ld, T* __restrict__ out, int64_t ldo, int accumulate) {
    const int64_t total = rows * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rr = e / cols, cc = e % cols;
        T acc = parts[rr * ld + cc];
        for (int p = 1; p < nparts; ++p) acc += parts[p * split_stride + rr * ld + cc];
        out[rr * ldo + cc] = accumulate ? out[rr * ldo + cc] + acc : acc;
    }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

template <typename T, int NB, int MR>
void launch_range_t(const ViewArgs& v, bool vec, dim3 grid, hipStream_t st, T* out, int64_t ldo,
                    int64_t split_stride, int64_t k_chunk, int acc) {
    if (vec)
        hipLaunchKernelGGL((range_view_kernel<T, NB, MR, true>), grid, dim3(256), 0, st, (const T*)v.A, v.lda, v.m,
                           v.n, (const T*)v.thin, v.ld_thin, v.s, out, ldo, split_stride, k_chunk, acc);
    else
        hipLaunchKernelGGL((range_view_kernel<T, NB, MR, false>), grid, dim3(256), 0, st, (const T*)v.A, v.lda, v.m,
                           v.n, (const T*)v.thin, v.ld_thin, v.s, out, ldo, split_stride, k_chunk, acc);
}

template <typename T, int NB, int MR>
void launch_corange_t(const ViewArgs& v, bool vec, dim3 grid, hipStream_t st, T* out, int64_t ldo,
                      int64_t split_stride, int64_t r_chunk, int acc) {
    if (vec)
        hipLaunchKernelGGL((corange_view_kernel<T, NB, MR, true>), grid, dim3(256), 0, st, (const T*)v.A, v.lda, v.m,
                           v.n, (const T*)v.thin, v.ld_thin, v.s, out, ldo, split_stride, r_chunk, acc);
    else
        hipLaunchKernelGGL((corange_view_kernel<T, NB, MR, false>), grid, dim3(256), 0, st, (const T*)v.A, v.lda,
                           v.m, v.n, (const T*)v.thin, v.ld_thin, v.s, out, ldo, split_stride, r_chunk, acc);
}

// Number of 16-column blocks needed for s, rounded to an instantiated width.
int pick_nb(int s) {
    const int nb = (int)ceil_div(s, 16);
    if (nb <= 1) return 1;
    if (nb <= 2) return 2;
    if (nb <= 4) return 4;
    if (nb <= 6) return 6;
    if (nb <= 8) return 8;
    if (nb <= 12) return 12;
    return 16;
}

#define RSVD_NB_SWITCH(NBV, CALL) \
    switch (NBV) {                \
        case 1: CALL(1); break;   \
        case 2: CALL(2); break;   \
        case 4: CALL(4); break;   \
        case 6: CALL(6); break;   \
        case 8: CALL(8); break;   \
        case 12: CALL(12); break; \
        default: CALL(16); break; \
    }

template <typename T>
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

int view_max_width() { return 256; }

// Plan of a range view: rows per workgroup and K splits.
ViewPlan plan_range(const ViewArgs& v, int num_cu) {
    ViewPlan p;
    p.nb = pick_nb(v.s);
    const int mr = (v.dtype == RSVD_F64) ? 1 : (p.nb <= 8 ? 2 : 1);
    p.mr = mr;
    const int64_t rows_per_wg = 4 * 16 * mr;
    p.tiles = ceil_div(v.m, rows_per_wg);
    // split K until the grid covers the chip about twice (never below 256 columns per split)
    int64_t splits = 1;
    while (p.tiles * splits < 2 * num_cu && ceil_div(v.n, splits * 2) >= 256 && splits < 64) splits *= 2;
    p.splits = splits;
    p.chunk = round_up(ceil_div(v.n, splits), 16);
    p.splits = ceil_div(v.n, p.chunk);
    return p;
}

ViewPlan plan_corange(const ViewArgs& v, int num_cu) {
    ViewPlan p;
    p.nb = pick_nb(v.s);
    const int mr = (v.dtype == RSVD_F64) ? 1 : (p.nb <= 8 ? 2 : 1);
    p.mr = mr;
    const int64_t cols_per_wg = 4 * 16 * mr;
    p.tiles = ceil_div(v.n, cols_per_wg);
    int64_t splits = 1;
    while (p.tiles * splits < 2 * num_cu && ceil_div(v.m, splits * 2) >= 256 && splits < 256) splits *= 2;
    p.chunk = round_up(ceil_div(v.m, splits), 16);
    p.splits = ceil_div(v.m, p.chunk);
    return p;
}

size_t view_partial_elems(const ViewPlan& p, int64_t s, int64_t len) {
    return p.splits > 1 ? (size_t)p.splits * (size_t)s * (size_t)len : 0;
}

template <typename T>
static rsvd_status run_range_t(const ViewArgs& v, const ViewPlan& p, T* out, int64_t ldo, T* partial, int accumulate,
                               hipStream_t st) {
    const bool vec = aligned16<T>(v.A) && aligned16<T>(v.thin) && (v.lda % 4 == 0) && (v.ld_thin % 4 == 0);
    dim3 grid((unsigned)p.tiles, (unsigned)p.splits);
    T* dst = p.splits > 1 ? partial : out;
    const int64_t ld_dst = p.splits > 1 ? v.m : ldo;
    const int64_t stride = (int64_t)v.s * v.m;
    const int dacc = p.splits > 1 ? 0 : accumulate;
#define RSVD_RANGE_CALL(NBV)                                                                      \
    do {                                                                                          \
        if (p.mr == 2) launch_range_t<T, NBV, 2>(v, vec, grid, st, dst, ld_dst, stride, p.chunk, dacc); \
        else launch_range_t<T, NBV, 1>(v, vec, grid, st, dst, ld_dst, stride, p.chunk, dacc);           \
    } while (0)
    RSVD_NB_SWITCH(p.nb, RSVD_RANGE_CALL);
#undef RSVD_RANGE_CALL
    RSVD_LAUNCH_CHECK();
    if (p.splits > 1) {
        const int64_t total = (int64_t)v.s * v.m;
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 8192);
        hipLaunchKernelGGL(reduce_parts_kernel<T>, dim3(blocks), dim3(256), 0, st, partial, (int)p.splits, stride,
                           (int64_t)v.s, v.m, v.m, out, ldo, accumulate);
        RSVD_LAUNCH_CHECK();
    }
    return RSVD_OK;
}

template <typename T>
static rsvd_status run_corange_t(const ViewArgs& v, const ViewPlan& p, T* out, int64_t ldo, T* partial,
                                 int accumulate, hipStream_t st) {
    const bool vec = aligned16<T>(v.thin) && (v.ld_thin % 4 == 0);
    dim3 grid((unsigned)p.tiles, (unsigned)p.splits);
    T* dst = p.splits > 1 ? partial : out;
    const int64_t ld_dst = p.splits > 1 ? v.n : ldo;
    const int64_t stride = (int64_t)v.s * v.n;
    const int dacc = p.splits > 1 ? 0 : accumulate;
#define RSVD_CORANGE_CALL(NBV)                                                                      \
    do {                                                                                            \
        if (p.mr == 2) launch_corange_t<T, NBV, 2>(v, vec, grid, st, dst, ld_dst, stride, p.chunk, dacc); \
        else launch_corange_t<T, NBV, 1>(v, vec, grid, st, dst, ld_dst, stride, p.chunk, dacc);           \
    } while (0)
    RSVD_NB_SWITCH(p.nb, RSVD_CORANGE_CALL);
#undef RSVD_CORANGE_CALL
    RSVD_LAUNCH_CHECK();
    if (p.splits > 1) {
        const int64_t total = (int64_t)v.s * v.n;
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 8192);
        hipLaunchKernelGGL(reduce_parts_kernel<T>, dim3(blocks), dim3(256), 0, st, partial, (int)p.splits, stride,
                           (int64_t)v.s, v.n, v.n, out, ldo, accumulate);
        RSVD_LAUNCH_CHECK();
    }
    return RSVD_OK;
}

rsvd_status run_range(const ViewArgs& v, const ViewPlan& p, void* out, int64_t ldo, void* partial, int accumulate,
                      hipStream_t st) {
    if (v.dtype == RSVD_F64) return run_range_t<double>(v, p, (double*)out, ldo, (double*)partial, accumulate, st);
    if (v.dtype == RSVD_F32) return run_range_t<float>(v, p, (float*)out, ldo, (float*)partial, accumulate, st);
    return RSVD_EUNSUPPORTED;
}

rsvd_status run_corange(const ViewArgs& v, const ViewPlan& p, void* out, int64_t ldo, void* partial, int accumulate,
                        hipStream_t st) {
    if (v.dtype == RSVD_F64) return run_corange_t<double>(v, p, (double*)out, ldo, (double*)partial, accumulate, st);
    if (v.dtype == RSVD_F32) return run_corange_t<float>(v, p, (float*)out, ldo, (float*)partial, accumulate, st);
    return RSVD_EUNSUPPORTED;
}
