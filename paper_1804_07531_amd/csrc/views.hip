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
#include <cstdint>
#include <cstdlib>

#include "common.h"
#include "launch.h"
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
struct range_view_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const T*  A;
        int64_t lda;
        int64_t m;
        int64_t n;
        const T*  XT;
        int64_t ldx;
        int s;
        T*  out;
        int64_t ldo;
        int64_t split_stride;
        int64_t k_chunk;
        int accumulate;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [A, lda, m, n, XT, ldx, s, out, ldo, split_stride, k_chunk, accumulate] = args_;
        typedef typename mfma16<T>::acc acc_t;
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int g = lane >> 4, i = lane & 15;
        const int64_t row0 = ((int64_t)vg.bx * 4 + wave) * (16 * MR);
        if (row0 >= m) return;
        const int64_t kb = (int64_t)vg.by * k_chunk;
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
        if (VEC && k < kfull) {
            // Loads are unconditional so the loop has no branches and the waits
            // can count: two register buffers alternate, the loads of one step
            // stay in flight while the matrix cores work on the other.  A row of
            // A past m (or a thin row past s) reads row 0 instead; it only feeds
            // output rows (columns) that are never stored, since C[i][j] depends
            // on row i of one operand and column j of the other alone.
            vec4<T> a0[MR], b0[NB], a1[MR], b1[NB];
            auto load_step = [&](int64_t kk, vec4<T>* av, vec4<T>* bv) {
    #pragma unroll
                for (int a = 0; a < MR; ++a) av[a] = load4(arow[a] + kk);
    #pragma unroll
                for (int b = 0; b < NB; ++b) bv[b] = load4(xrow[b] + kk);
            };
            auto mma_step = [&](const vec4<T>* av, const vec4<T>* bv) {
    #pragma unroll
                for (int t = 0; t < 4; ++t)
    #pragma unroll
                    for (int a = 0; a < MR; ++a)
    #pragma unroll
                        for (int b = 0; b < NB; ++b) acc[a][b] = mfma16<T>::step(av[a].x[t], bv[b].x[t], acc[a][b]);
            };
            // an odd leading step is peeled so the loop body below is a single
            // basic block (the waits then count across the back edge)
            if (((kfull - k) / 16) & 1) {
                load_step(k + 4 * g, a0, b0);
                mma_step(a0, b0);
                k += 16;
            }
            if (k < kfull) {
                const int64_t klast = kfull - 32;  // start of the last step pair
                load_step(k + 4 * g, a0, b0);
                for (; k < kfull; k += 32) {
                    // the scheduling barriers keep each step's loads ahead of the
                    // previous step's matrix-core work (the scheduler would
                    // otherwise sink them next to their use)
                    load_step(k + 16 + 4 * g, a1, b1);
                    __builtin_amdgcn_sched_barrier(0);
                    mma_step(a0, b0);
                    __builtin_amdgcn_sched_barrier(0);
                    load_step(std::min(k + 32, klast) + 4 * g, a0, b0);
                    __builtin_amdgcn_sched_barrier(0);
                    mma_step(a1, b1);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            k = kfull;
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
    
        T* o = out + (int64_t)vg.by * split_stride;
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
};

// ---------------------------------------------------------------------------
// Co-range view: Z^T[j][c] = sum_r A[r][c] Y^T[j][r]
// grid.x: column tiles (4 waves x 16*MR columns); grid.y: splits of the rows.
// ---------------------------------------------------------------------------
template <typename T, int NB, int MR, bool VEC>
struct corange_view_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const T*  A;
        int64_t lda;
        int64_t m;
        int64_t n;
        const T*  YT;
        int64_t ldy;
        int s;
        T*  out;
        int64_t ldo;
        int64_t split_stride;
        int64_t r_chunk;
        int accumulate;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [A, lda, m, n, YT, ldy, s, out, ldo, split_stride, r_chunk, accumulate] = args_;
        typedef typename mfma16<T>::acc acc_t;
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int g = lane >> 4, i = lane & 15;
        const int64_t col0 = ((int64_t)vg.bx * 4 + wave) * (16 * MR);
        if (col0 >= n) return;
        const int64_t rb = (int64_t)vg.by * r_chunk;
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
        int64_t acol[MR];
    #pragma unroll
        for (int a = 0; a < MR; ++a) acol[a] = col_ok[a] ? col0 + 16 * a + i : 0;
        if (r < rfull) {
            // branch-free loads and two alternating register buffers, as in the
            // range view (a column of A past n, or a thin row past s, only feeds
            // outputs that are never stored)
            vec4<T> a0[MR], b0[NB], a1[MR], b1[NB];
            auto load_step = [&](int64_t rr, vec4<T>* av, vec4<T>* bv) {
    #pragma unroll
                for (int a = 0; a < MR; ++a) {
                    const T* p = A + rr * lda + acol[a];
    #pragma unroll
                    for (int t = 0; t < 4; ++t) av[a].x[t] = p[t * lda];
                }
    #pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (VEC) bv[b] = load4(yrow[b] + rr);
                    else bv[b] = load4_guard(yrow[b] + rr, rr, re, true);
                }
            };
            auto mma_step = [&](const vec4<T>* av, const vec4<T>* bv) {
    #pragma unroll
                for (int t = 0; t < 4; ++t)
    #pragma unroll
                    for (int a = 0; a < MR; ++a)
    #pragma unroll
                        for (int b = 0; b < NB; ++b) acc[a][b] = mfma16<T>::step(av[a].x[t], bv[b].x[t], acc[a][b]);
            };
            if (((rfull - r) / 16) & 1) {
                load_step(r + 4 * g, a0, b0);
                mma_step(a0, b0);
                r += 16;
            }
            if (r < rfull) {
                const int64_t rlast = rfull - 32;
                load_step(r + 4 * g, a0, b0);
                for (; r < rfull; r += 32) {
                    load_step(r + 16 + 4 * g, a1, b1);
                    __builtin_amdgcn_sched_barrier(0);
                    mma_step(a0, b0);
                    __builtin_amdgcn_sched_barrier(0);
                    load_step(std::min(r + 32, rlast) + 4 * g, a0, b0);
                    __builtin_amdgcn_sched_barrier(0);
                    mma_step(a1, b1);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            r = rfull;
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
    
        T* o = out + (int64_t)vg.by * split_stride;
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
};

// ---------------------------------------------------------------------------
// FP32 views through a three-stage LDS ring (gfx950 direct-to-LDS loads).
//
// Each 16-wide step of the contraction index is one stage: the A tile and
// the thin tile of the step are copied from HBM straight into LDS with
// global_load_lds_dwordx4 (16 bytes per lane, no registers), two steps
// ahead of the step the matrix cores work on.  A wave waits only for its
// own copies of the current stage (an exact s_waitcnt vmcnt, every wave
// issues the same number of copies per step) and a plain s_barrier then
// makes every wave's copies visible; the same barrier tells every wave that
// the slot about to be refilled has been read.  The three stages are three
// separate LDS arrays and the loop is unrolled by three, so the compiler
// can see which stage each copy writes and does not drain the queue before
// the LDS reads.  After the last full step the ragged tail (fewer than 16)
// goes through guarded register loads.
// ---------------------------------------------------------------------------
template <int NLOADS>
__device__ __forceinline__ void wait_own_copies_then_barrier() {
    wait_vmcnt<NLOADS>();
    bare_barrier();
}

// Range view, FP32.  A wave owns 16*MR rows and all 16*NB thin columns; the
// thin tile of a stage (NB fragment blocks of 1 KB) is copied cooperatively,
// NB/4 blocks per wave.  Fragment block layout: lane l = 16 g + i holds the
// 4 values [row or column i][k0 + 4 g .. k0 + 4 g + 3].  One 16-wide step
// reads 64 bytes of each row of A, half of a 128-byte cache line.  With four
// row blocks per wave (one workgroup per CU, room in LDS) a stage holds two
// steps and both halves of each line are copied back to back: with one step
// per stage the second half came a stage later and the line was fetched
// from HBM again (8.3 GB read per launch at 65536 x 16384 for 4.3 GB of A).
template <int NB, int MR>
struct range_view_lds_kernel_op {
    static constexpr int kThreads = 256;
    static constexpr int kMinBlocks = 2;
    struct Args {
        const float*  A;
        int64_t lda;
        int64_t m;
        int64_t n;
        const float*  XT;
        int64_t ldx;
        int s;
        float*  out;
        int64_t ldo;
        int64_t split_stride;
        int64_t k_chunk;
        int accumulate;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [A, lda, m, n, XT, ldx, s, out, ldo, split_stride, k_chunk, accumulate] = args_;
        // every wave copies XB thin blocks per stage; when NB is not a multiple
        // of four, the copies past block NB - 1 fill spare slots that no product
        // reads (from clamped, in-bounds rows), so that all waves wait for the
        // same number of copies
        constexpr int XB = (NB + 3) / 4;
        constexpr int KS = MR == 4 ? 2 : 1;   // 16-wide contraction steps per stage
        constexpr int SB = 4 * MR + 4 * XB;   // 1 KB fragment blocks per step
        constexpr int BLK = KS * SB;          // ... per stage
        constexpr int NL = KS * (MR + XB);    // copies per wave per stage
        __shared__ floatx4 st0[BLK * 64];
        __shared__ floatx4 st1[BLK * 64];
        __shared__ floatx4 st2[BLK * 64];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
        const int64_t row0 = ((int64_t)vg.bx * 4 + wave) * (16 * MR);
        const int64_t kb = (int64_t)vg.by * k_chunk;
        const int64_t ke = std::min<int64_t>(n, kb + k_chunk);
        const int64_t nsteps = (ke - kb) / (16 * KS);   // full stages
    
        // copy sources; rows past the edge read the last row (they only feed outputs that are not stored)
        const float* asrc[MR];
    #pragma unroll
        for (int a = 0; a < MR; ++a) asrc[a] = A + std::min<int64_t>(row0 + 16 * a + i, m - 1) * lda + kb + 4 * g;
        const float* xsrc[XB];
    #pragma unroll
        for (int q = 0; q < XB; ++q) xsrc[q] = XT + (int64_t)std::min(16 * (wave + 4 * q) + i, s - 1) * ldx + kb + 4 * g;
    
        floatx4 acc[MR][NB];
    #pragma unroll
        for (int a = 0; a < MR; ++a)
    #pragma unroll
            for (int b = 0; b < NB; ++b) acc[a][b] = floatx4{0, 0, 0, 0};
    
        auto issue = [&](int64_t t, floatx4* stg) {
    #pragma unroll
            for (int a = 0; a < MR; ++a)
    #pragma unroll
                for (int u = 0; u < KS; ++u)
                    lds_copy16(asrc[a] + 16 * (KS * t + u), stg + (u * SB + wave * MR + a) * 64);
    #pragma unroll
            for (int q = 0; q < XB; ++q)
    #pragma unroll
                for (int u = 0; u < KS; ++u)
                    lds_copy16(xsrc[q] + 16 * (KS * t + u), stg + (u * SB + 4 * MR + wave + 4 * q) * 64);
        };
        auto fragments = [&](const floatx4* blk, floatx4 (&av)[MR], floatx4 (&bv)[NB]) {
    #pragma unroll
            for (int a = 0; a < MR; ++a) av[a] = blk[(wave * MR + a) * 64 + lane];
    #pragma unroll
            for (int b = 0; b < NB; ++b) bv[b] = blk[(4 * MR + b) * 64 + lane];
        };
        auto products = [&](const floatx4 (&av)[MR], const floatx4 (&bv)[NB]) {
    #pragma unroll
            for (int tt = 0; tt < 4; ++tt)
    #pragma unroll
                for (int a = 0; a < MR; ++a)
    #pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][tt], bv[b][tt], acc[a][b], 0, 0, 0);
        };
        auto step = [&](int64_t t, floatx4* cur, floatx4* nxt) {
            wait_own_copies_then_barrier<NL>();
            floatx4 av[MR], bv[NB];
            fragments(cur, av, bv);
            // refill the slot read by the previous stage (a repeat of the last
            // stage near the end keeps the per-stage copy count uniform)
            issue(std::min<int64_t>(t + 2, nsteps - 1), nxt);
            products(av, bv);
    #pragma unroll
            for (int u = 1; u < KS; ++u) {
                fragments(cur + u * SB * 64, av, bv);
                products(av, bv);
            }
        };
        if (nsteps > 0) {
            issue(0, st0);
            issue(std::min<int64_t>(1, nsteps - 1), st1);
            int64_t t = 0;
            for (; t + 3 <= nsteps; t += 3) {
                step(t, st0, st2);
                step(t + 1, st1, st0);
                step(t + 2, st2, st1);
            }
            if (t < nsteps) step(t, st0, st2);
            if (t + 1 < nsteps) step(t + 1, st1, st0);
            wait_all_vmem();  // drain the repeated copies before the workgroup exits
        }
        // ragged tail of the contraction (fewer than 16 * KS left)
        for (int64_t k = kb + 16 * KS * nsteps; k < ke; k += 16) {
            const int64_t kk = k + 4 * g;
            vec4<float> av[MR], bv[NB];
    #pragma unroll
            for (int a = 0; a < MR; ++a) {
                const int64_t r = row0 + 16 * a + i;
                av[a] = load4_guard(A + (r < m ? r : 0) * lda + kk, kk, ke, r < m);
            }
    #pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = 16 * b + i;
                bv[b] = load4_guard(XT + (int64_t)(j < s ? j : 0) * ldx + kk, kk, ke, j < s);
            }
    #pragma unroll
            for (int tt = 0; tt < 4; ++tt)
    #pragma unroll
                for (int a = 0; a < MR; ++a)
    #pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x[tt], bv[b].x[tt], acc[a][b], 0, 0, 0);
        }
        if (row0 >= m) return;
        float* o = out + (int64_t)vg.by * split_stride;
    #pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = 16 * b + i;
            if (j >= s) continue;
    #pragma unroll
            for (int a = 0; a < MR; ++a) {
    #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row0 + 16 * a + 4 * g + r;
                    if (row < m) {
                        float* d = o + (int64_t)j * ldo + row;
                        *d = accumulate ? *d + acc[a][b][r] : acc[a][b][r];
                    }
                }
            }
        }
    }
};

// Co-range view, FP32.  A wave owns 16*MR columns of A and all thin columns;
// a stage holds the 16 x 64*MR tile of A (row-major, copied 16 bytes per
// lane, MR copies per wave) and NB thin fragment blocks.
template <int NB, int MR>
struct corange_view_lds_kernel_op {
    static constexpr int kThreads = 256;
    static constexpr int kMinBlocks = 2;
    struct Args {
        const float*  A;
        int64_t lda;
        int64_t m;
        int64_t n;
        const float*  YT;
        int64_t ldy;
        int s;
        float*  out;
        int64_t ldo;
        int64_t split_stride;
        int64_t r_chunk;
        int accumulate;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [A, lda, m, n, YT, ldy, s, out, ldo, split_stride, r_chunk, accumulate] = args_;
        // XB thin blocks per wave and stage, spare slots as in the range view
        constexpr int XB = (NB + 3) / 4;
        constexpr int AW = 64 * MR;           // columns of the workgroup's A tile
        constexpr int ABLK = 4 * MR;          // A tile = 16 rows x AW columns = 4*MR KB
        constexpr int BLK = ABLK + 4 * XB;
        constexpr int NL = MR + XB;
        __shared__ floatx4 st0[BLK * 64];
        __shared__ floatx4 st1[BLK * 64];
        __shared__ floatx4 st2[BLK * 64];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
        const int64_t cw0 = (int64_t)vg.bx * AW;                 // first column of the workgroup
        const int64_t col0 = cw0 + (int64_t)wave * 16 * MR;          // first column of this wave
        const int64_t rb = (int64_t)vg.by * r_chunk;
        const int64_t re = std::min<int64_t>(m, rb + r_chunk);
        const int64_t nsteps = (re - rb) / 16;
    
        // A tile copies: copy q (q = wave*MR + a) covers rows q*(4/MR) .. of the
        // step, lane l takes row q*(4/MR) + l/(16*MR) and the 4 columns 4*(l%(16*MR)).
        const int64_t ncl = round_up(n, 4) - 4;                      // last 4-aligned column start inside a row
        const float* asrc[MR];
    #pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int q = wave * MR + a;
            const int row = q * (4 / MR) + lane / (16 * MR);
            const int64_t col = std::min<int64_t>(cw0 + 4 * (lane % (16 * MR)), ncl);
            asrc[a] = A + (rb + row) * lda + col;
        }
        const float* ysrc[XB];
    #pragma unroll
        for (int q = 0; q < XB; ++q) ysrc[q] = YT + (int64_t)std::min(16 * (wave + 4 * q) + i, s - 1) * ldy + rb + 4 * g;
    
        floatx4 acc[MR][NB];
    #pragma unroll
        for (int a = 0; a < MR; ++a)
    #pragma unroll
            for (int b = 0; b < NB; ++b) acc[a][b] = floatx4{0, 0, 0, 0};
    
        auto issue = [&](int64_t t, floatx4* stg) {
    #pragma unroll
            for (int a = 0; a < MR; ++a)
                lds_copy16(asrc[a] + 16 * t * lda, stg + (wave * MR + a) * 64);
    #pragma unroll
            for (int q = 0; q < XB; ++q)
                lds_copy16(ysrc[q] + 16 * t, stg + (ABLK + wave + 4 * q) * 64);
        };
        auto step = [&](int64_t t, floatx4* cur, floatx4* nxt) {
            wait_own_copies_then_barrier<NL>();
            const float* at = reinterpret_cast<const float*>(cur);   // 16 x AW row-major
            floatx4 av[MR], bv[NB];
    #pragma unroll
            for (int a = 0; a < MR; ++a) {
                const int c = wave * 16 * MR + 16 * a + i;
    #pragma unroll
                for (int tt = 0; tt < 4; ++tt) av[a][tt] = at[(4 * g + tt) * AW + c];
            }
    #pragma unroll
            for (int b = 0; b < NB; ++b) bv[b] = cur[(ABLK + b) * 64 + lane];
            issue(std::min<int64_t>(t + 2, nsteps - 1), nxt);
    #pragma unroll
            for (int tt = 0; tt < 4; ++tt)
    #pragma unroll
                for (int a = 0; a < MR; ++a)
    #pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][tt], bv[b][tt], acc[a][b], 0, 0, 0);
        };
        if (nsteps > 0) {
            issue(0, st0);
            issue(std::min<int64_t>(1, nsteps - 1), st1);
            int64_t t = 0;
            for (; t + 3 <= nsteps; t += 3) {
                step(t, st0, st2);
                step(t + 1, st1, st0);
                step(t + 2, st2, st1);
            }
            if (t < nsteps) step(t, st0, st2);
            if (t + 1 < nsteps) step(t + 1, st1, st0);
            wait_all_vmem();
        }
        for (int64_t r = rb + 16 * nsteps; r < re; r += 16) {
            const int64_t rr = r + 4 * g;
            vec4<float> av[MR], bv[NB];
    #pragma unroll
            for (int a = 0; a < MR; ++a) {
                const int64_t c = col0 + 16 * a + i;
    #pragma unroll
                for (int tt = 0; tt < 4; ++tt)
                    av[a].x[tt] = (c < n && rr + tt < re) ? A[(rr + tt) * lda + c] : 0.0f;
            }
    #pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = 16 * b + i;
                bv[b] = load4_guard(YT + (int64_t)(j < s ? j : 0) * ldy + rr, rr, re, j < s);
            }
    #pragma unroll
            for (int tt = 0; tt < 4; ++tt)
    #pragma unroll
                for (int a = 0; a < MR; ++a)
    #pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x[tt], bv[b].x[tt], acc[a][b], 0, 0, 0);
        }
        if (col0 >= n) return;
        float* o = out + (int64_t)vg.by * split_stride;
    #pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = 16 * b + i;
            if (j >= s) continue;
    #pragma unroll
            for (int a = 0; a < MR; ++a) {
    #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t c = col0 + 16 * a + 4 * g + q;
                    if (c < n) {
                        float* d = o + (int64_t)j * ldo + c;
                        *d = accumulate ? *d + acc[a][b][q] : acc[a][b][q];
                    }
                }
            }
        }
    }
};

// The LDS-ring kernels are built for every thin width pick_nb returns, with
// two 16-row (column) blocks per wave up to 8 thin blocks.
#define RSVD_LDS_SWITCH(NBV, MRV, LAUNCH)                 \
    do {                                                  \
        if ((MRV) == 2) {                                 \
            switch (NBV) {                                \
                case 1: LAUNCH(1, 2); break;              \
                case 2: LAUNCH(2, 2); break;              \
                case 4: LAUNCH(4, 2); break;              \
                case 6: LAUNCH(6, 2); break;              \
                default: LAUNCH(8, 2); break;             \
            }                                             \
        } else {                                          \
            switch (NBV) {                                \
                case 1: LAUNCH(1, 1); break;              \
                case 2: LAUNCH(2, 1); break;              \
                case 4: LAUNCH(4, 1); break;              \
                case 6: LAUNCH(6, 1); break;              \
                case 8: LAUNCH(8, 1); break;              \
                case 12: LAUNCH(12, 1); break;            \
                default: LAUNCH(16, 1); break;            \
            }                                             \
        }                                                 \
    } while (0)

template <int NB, int MR>
static void launch_range_lds(const ViewArgs& v, dim3 grid, hipStream_t st, float* out, int64_t ldo, int64_t stride,
                             int64_t chunk, int acc) {
    launch_op<range_view_lds_kernel_op<NB, MR>>(grid, dim3(256), 0, st, {(const float*)v.A, v.lda, v.m, v.n, (const float*)v.thin, v.ld_thin, v.s, out, ldo, stride, chunk, acc});
}

template <int NB, int MR>
static void launch_corange_lds(const ViewArgs& v, dim3 grid, hipStream_t st, float* out, int64_t ldo, int64_t stride,
                               int64_t chunk, int acc) {
    launch_op<corange_view_lds_kernel_op<NB, MR>>(grid, dim3(256), 0, st, {(const float*)v.A, v.lda, v.m, v.n, (const float*)v.thin, v.ld_thin, v.s, out, ldo, stride, chunk, acc});
}

// Sum of `parts` partial panels (rows x cols, leading dimension ld, parts
// spaced split_stride apart) into out, in a fixed order.
template <typename T>
struct reduce_parts_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const T*  parts;
        int nparts;
        int64_t split_stride;
        int64_t rows;
        int64_t cols;
        int64_t ld;
        T*  out;
        int64_t ldo;
        int accumulate;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [parts, nparts, split_stride, rows, cols, ld, out, ldo, accumulate] = args_;
        const int64_t total = rows * cols;
        const bool flat = ld == cols && ldo == cols;
        const bool small = total <= (int64_t)UINT32_MAX;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < total;
             e += (int64_t)vg.gx * blockDim.x) {
            int64_t src = e, dst = e;
            if (!flat) {
                int64_t rr, cc;
                if (small) {
                    rr = (uint32_t)e / (uint32_t)cols;
                    cc = (uint32_t)e - (uint32_t)rr * (uint32_t)cols;
                } else {
                    rr = e / cols;
                    cc = e % cols;
                }
                src = rr * ld + cc;
                dst = rr * ldo + cc;
            }
            // the partials in order p = 0, 1, ...; eight loads go out before their sums
            T acc = parts[src];
            int p = 1;
            for (; p + 8 <= nparts; p += 8) {
                T v[8];
    #pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = parts[(int64_t)(p + u) * split_stride + src];
    #pragma unroll
                for (int u = 0; u < 8; ++u) acc += v[u];
            }
            for (; p < nparts; ++p) acc += parts[(int64_t)p * split_stride + src];
            out[dst] = accumulate ? out[dst] + acc : acc;
        }
    }
};

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

template <typename T, int NB, int MR>
void launch_range_t(const ViewArgs& v, bool vec, dim3 grid, hipStream_t st, T* out, int64_t ldo,
                    int64_t split_stride, int64_t k_chunk, int acc) {
    if (vec)
        launch_op<range_view_kernel_op<T, NB, MR, true>>(grid, dim3(256), 0, st, {(const T*)v.A, v.lda, v.m, v.n, (const T*)v.thin, v.ld_thin, v.s, out, ldo, split_stride, k_chunk, acc});
    else
        launch_op<range_view_kernel_op<T, NB, MR, false>>(grid, dim3(256), 0, st, {(const T*)v.A, v.lda, v.m, v.n, (const T*)v.thin, v.ld_thin, v.s, out, ldo, split_stride, k_chunk, acc});
}

template <typename T, int NB, int MR>
void launch_corange_t(const ViewArgs& v, bool vec, dim3 grid, hipStream_t st, T* out, int64_t ldo,
                      int64_t split_stride, int64_t r_chunk, int acc) {
    if (vec)
        launch_op<corange_view_kernel_op<T, NB, MR, true>>(grid, dim3(256), 0, st, {(const T*)v.A, v.lda, v.m, v.n, (const T*)v.thin, v.ld_thin, v.s, out, ldo, split_stride, r_chunk, acc});
    else
        launch_op<corange_view_kernel_op<T, NB, MR, false>>(grid, dim3(256), 0, st, {(const T*)v.A, v.lda, v.m, v.n, (const T*)v.thin, v.ld_thin, v.s, out, ldo, split_stride, r_chunk, acc});
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

// Tiles and contraction splits of a view.  Two rows (columns) of 16 per
// wave for FP32 thin widths up to 128, one for short outputs (panels); the
// contraction is split until the grid covers the chip about twice, but
// never so far that the partial sums (splits x s x len) exceed about half
// the bytes of A the view reads (a concern only for the short panels of the
// one-view sweep and the row-sweep Krylov blocks: full views need no split).
// The FP32 co-range kernel also takes two 16-column blocks per wave with 12
// or 16 thin blocks (255 registers, no spills): at 4096 x 16384 with s = 241
// that runs at 114 TF/s against 100 with one block.  The FP32 range view of
// a long output (32768 rows or more) with 4, 6 or 8 thin blocks takes four
// row blocks per wave (64 rows; up to 252 registers), each thin fragment read
// from LDS then feeding four products: at 65536 x 16384 with s = 120,
// 118 TF/s against 105 with two, one workgroup per CU and no split.
static ViewPlan plan_view(int64_t out_len, int64_t contraction, int s, int dtype, int mr_hint, int num_cu,
                          bool corange = false) {
    ViewPlan p;
    p.nb = pick_nb(s);
    const int nb_mr2 = corange ? 16 : 8;          // widest thin tile with two 16-row (column) blocks per wave
    int mr = (dtype == RSVD_F64) ? 1 : (p.nb <= 8 ? 2 : 1);
    if (corange && p.nb > 8) mr = 2;
    if (out_len < 8192) mr = 1;
    if (mr_hint == 1 || mr_hint == 2) mr = mr_hint;
    if (dtype == RSVD_F64 || p.nb > nb_mr2) mr = 1;   // two blocks per wave only for FP32
    if (!corange && dtype == RSVD_F32 && mr_hint == 0 && out_len >= 32768 && p.nb >= 4 && p.nb <= 8) mr = 4;
    p.mr = mr;
    p.tiles = ceil_div(out_len, 4 * 16 * p.mr);
    const int64_t s_pad = 16 * (int64_t)p.nb;
    // four row blocks per wave leave room for one workgroup per CU
    const int64_t fill = mr == 4 ? num_cu : 2 * num_cu;
    int64_t splits = 1;
    while (p.tiles * splits < fill && ceil_div(contraction, splits * 2) >= 256 &&
           (splits * 2) * s_pad * 2 <= contraction && splits < 256)
        splits *= 2;
    p.chunk = round_up(ceil_div(contraction, splits), mr == 4 ? 32 : 16);   // whole LDS stages
    p.splits = ceil_div(contraction, p.chunk);
    return p;
}

ViewPlan plan_range(const ViewArgs& v, int num_cu) { return plan_view(v.m, v.n, v.s, v.dtype, v.mr_hint, num_cu); }

ViewPlan plan_corange(const ViewArgs& v, int num_cu) {
    return plan_view(v.n, v.m, v.s, v.dtype, v.mr_hint, num_cu, true);
}

size_t view_partial_elems(const ViewPlan& p, int64_t s, int64_t len) {
    return p.splits > 1 ? (size_t)p.splits * (size_t)s * (size_t)len : 0;
}

template <typename T>
static rsvd_status run_range_t(const ViewArgs& v, const ViewPlan& p, T* out, int64_t ldo, T* partial, int accumulate,
                               bool slots_only, hipStream_t st) {
    const bool vec = aligned16<T>(v.A) && aligned16<T>(v.thin) && (v.lda % 4 == 0) && (v.ld_thin % 4 == 0);
    dim3 grid((unsigned)p.tiles, (unsigned)p.splits);
    const bool to_slots = p.splits > 1 || slots_only;
    T* dst = to_slots ? partial : out;
    const int64_t ld_dst = to_slots ? v.m : ldo;
    const int64_t stride = (int64_t)v.s * v.m;
    const int dacc = p.splits > 1 && !slots_only ? 0 : accumulate;
    if constexpr (sizeof(T) == 4) {
        if (vec) {
            float* d = (float*)dst;
#define RSVD_RANGE_LDS(NBV, MRV) launch_range_lds<NBV, MRV>(v, grid, st, d, ld_dst, stride, p.chunk, dacc)
            if (p.mr == 4 && p.nb == 4) RSVD_RANGE_LDS(4, 4);
            else if (p.mr == 4 && p.nb == 6) RSVD_RANGE_LDS(6, 4);
            else if (p.mr == 4) RSVD_RANGE_LDS(8, 4);
            else RSVD_LDS_SWITCH(p.nb, p.mr, RSVD_RANGE_LDS);
#undef RSVD_RANGE_LDS
            goto launched;
        }
    }
    {
        // the register-path kernels take at most two row blocks per wave
        if (p.mr == 4) grid.x = (unsigned)ceil_div(v.m, 128);
        const int mr_reg = p.mr == 4 ? 2 : p.mr;
#define RSVD_RANGE_CALL(NBV)                                                                      \
    do {                                                                                          \
        if (mr_reg == 2) launch_range_t<T, NBV, 2>(v, vec, grid, st, dst, ld_dst, stride, p.chunk, dacc); \
        else launch_range_t<T, NBV, 1>(v, vec, grid, st, dst, ld_dst, stride, p.chunk, dacc);           \
    } while (0)
        RSVD_NB_SWITCH(p.nb, RSVD_RANGE_CALL);
#undef RSVD_RANGE_CALL
    }
launched:
    RSVD_LAUNCH_CHECK();
    if (p.splits > 1 && !slots_only) {
        const int64_t total = (int64_t)v.s * v.m;
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 8192);
        launch_op<reduce_parts_kernel_op<T>>(dim3(blocks), dim3(256), 0, st, {partial, (int)p.splits, stride, (int64_t)v.s, v.m, v.m, out, ldo, accumulate});
        RSVD_LAUNCH_CHECK();
    }
    return RSVD_OK;
}

template <typename T>
static rsvd_status run_corange_t(const ViewArgs& v, const ViewPlan& p, T* out, int64_t ldo, T* partial,
                                 int accumulate, bool slots_only, hipStream_t st) {
    const bool vec = aligned16<T>(v.thin) && (v.ld_thin % 4 == 0);
    dim3 grid((unsigned)p.tiles, (unsigned)p.splits);
    const bool to_slots = p.splits > 1 || slots_only;
    T* dst = to_slots ? partial : out;
    const int64_t ld_dst = to_slots ? v.n : ldo;
    const int64_t stride = (int64_t)v.s * v.n;
    const int dacc = p.splits > 1 && !slots_only ? 0 : accumulate;
    if constexpr (sizeof(T) == 4) {
        if (vec && aligned16<T>(v.A) && v.lda % 4 == 0 && v.n >= 4) {
            float* d = (float*)dst;
#define RSVD_CORANGE_LDS(NBV, MRV) launch_corange_lds<NBV, MRV>(v, grid, st, d, ld_dst, stride, p.chunk, dacc)
            if (p.mr == 2 && p.nb == 12) RSVD_CORANGE_LDS(12, 2);
            else if (p.mr == 2 && p.nb == 16) RSVD_CORANGE_LDS(16, 2);
            else RSVD_LDS_SWITCH(p.nb, p.mr, RSVD_CORANGE_LDS);
#undef RSVD_CORANGE_LDS
            goto launched;
        }
    }
    {
        // the register-path kernels take two column blocks per wave only up to 8 thin blocks
        if (p.mr == 2 && p.nb > 8) grid.x = (unsigned)ceil_div(v.n, 64);
        const int mr_reg = p.nb > 8 ? 1 : p.mr;
#define RSVD_CORANGE_CALL(NBV)                                                                      \
    do {                                                                                            \
        if (mr_reg == 2) launch_corange_t<T, NBV, 2>(v, vec, grid, st, dst, ld_dst, stride, p.chunk, dacc); \
        else launch_corange_t<T, NBV, 1>(v, vec, grid, st, dst, ld_dst, stride, p.chunk, dacc);           \
    } while (0)
        RSVD_NB_SWITCH(p.nb, RSVD_CORANGE_CALL);
#undef RSVD_CORANGE_CALL
    }
launched:
    RSVD_LAUNCH_CHECK();
    if (p.splits > 1 && !slots_only) {
        const int64_t total = (int64_t)v.s * v.n;
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 8192);
        launch_op<reduce_parts_kernel_op<T>>(dim3(blocks), dim3(256), 0, st, {partial, (int)p.splits, stride, (int64_t)v.s, v.n, v.n, out, ldo, accumulate});
        RSVD_LAUNCH_CHECK();
    }
    return RSVD_OK;
}

rsvd_status run_range(const ViewArgs& v, const ViewPlan& p, void* out, int64_t ldo, void* partial, int accumulate,
                      hipStream_t st, bool slots_only) {
    launch_phase();
    if (v.dtype == RSVD_F64)
        return run_range_t<double>(v, p, (double*)out, ldo, (double*)partial, accumulate, slots_only, st);
    if (v.dtype == RSVD_F32)
        return run_range_t<float>(v, p, (float*)out, ldo, (float*)partial, accumulate, slots_only, st);
    return RSVD_EUNSUPPORTED;
}

rsvd_status run_corange(const ViewArgs& v, const ViewPlan& p, void* out, int64_t ldo, void* partial, int accumulate,
                        hipStream_t st, bool slots_only) {
    launch_phase();
    if (v.dtype == RSVD_F64)
        return run_corange_t<double>(v, p, (double*)out, ldo, (double*)partial, accumulate, slots_only, st);
    if (v.dtype == RSVD_F32)
        return run_corange_t<float>(v, p, (float*)out, ldo, (float*)partial, accumulate, slots_only, st);
    return RSVD_EUNSUPPORTED;
}

ViewPlan cap_splits(const ViewPlan& p, int64_t contraction, int64_t max_splits) {
    ViewPlan q = p;
    if (q.splits <= max_splits) return q;
    q.chunk = round_up(ceil_div(contraction, max_splits), 16);
    q.splits = ceil_div(contraction, q.chunk);
    return q;
}

rsvd_status run_reduce_view_parts(int dtype, const void* parts, int nparts, int64_t s, int64_t len, void* out,
                                  int64_t ldo, int accumulate, hipStream_t st) {
    // a follow-up of the view that filled the slots: it shares that view's batch phase
    const int64_t total = s * len;
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 8192);
    if (dtype == RSVD_F64)
        launch_op<reduce_parts_kernel_op<double>>(dim3(blocks), dim3(256), 0, st, {(const double*)parts, nparts, total, s, len, len, (double*)out, ldo, accumulate});
    else if (dtype == RSVD_F32)
        launch_op<reduce_parts_kernel_op<float>>(dim3(blocks), dim3(256), 0, st, {(const float*)parts, nparts, total, s, len, len, (float*)out, ldo, accumulate});
    else
        return RSVD_EUNSUPPORTED;
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_reduce_parts_f32(const float* parts, int nparts, int64_t stride, int64_t rows, int64_t cols,
                                 float* out, int64_t ldo, int accumulate, hipStream_t st) {
    const int64_t total = rows * cols;
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 8192);
    launch_op<reduce_parts_kernel_op<float>>(dim3(blocks), dim3(256), 0, st, {parts, nparts, stride, rows, cols, cols, out, ldo, accumulate});
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}
