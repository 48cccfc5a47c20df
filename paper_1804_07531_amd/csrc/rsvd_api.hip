// Host drivers and the C ABI (include/rsvd.h).
//
// Each algorithm is written once against a Ctx; a "dry" Ctx runs the same
// code without launching anything and only sums the workspace it would
// carve, which is how rsvd_workspace_bytes() agrees with the calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "launch.h"
#include "grad.h"
#include "orth.h"
#include "philox.h"
#include "small.h"
#include "srft.h"
#include "views.h"

namespace {

constexpr int kPlanCUs = 256;        // default planning constant (MI355X compute units); affects only splits
constexpr uint32_t TAG_OMEGA = 1;    // range test matrix
constexpr uint32_t TAG_PSI = 2;      // co-range test matrix
constexpr uint32_t TAG_PHI = 3;      // core test matrix Phi_r^T (s_c x m)
constexpr uint32_t TAG_PHI2 = 4;     // core test matrix Phi_c^T (s_c x n)
constexpr uint32_t TAG_SRFT_SIGN_R = 6, TAG_SRFT_SAMPLE_R = 7;   // SRFT Phi_r (length m): signs, sample
constexpr uint32_t TAG_SRFT_SIGN_C = 8, TAG_SRFT_SAMPLE_C = 9;   // SRFT Phi_c (length n)
constexpr size_t kHeader = 256;      // status word + flags at the start of the workspace
constexpr int kLcWord = 5;           // header word: the l_c of the last one-view post-processing
constexpr int kMaxWidth = 512;       // widest panel the orthonormalization and small SVD handle

struct Arena {
    char* base;
    size_t off = kHeader;
    template <class T>
    T* take(size_t count) {
        off = (size_t)round_up((int64_t)off, 256);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct Ctx {
    bool dry;
    hipStream_t st;
    Arena ar;
    uint32_t* status = nullptr;
    int* flags = nullptr;  // per-orthonormalization "one more round" flags (kHeader holds 56 of them)
    int next_flag = 0;
    rsvd_view_trace* trace = nullptr;
    int trace_depth = 0;
    int f32_mode = RSVD_F32_MFMA;
    int plan_cus = kPlanCUs;   // compute units the split planning assumes (0: no contraction splits)
    int view_mr = 0;           // rows (columns) of 16 per wave in the FP32/FP64 views (0: automatic)
    unsigned sync_spins = 0;   // bounded-wait polls of the multi-workgroup small SVD (0: its default)
};

// Event pair around one view (no-op without a trace hook; views nested in a
// timed view are not timed separately).
struct ViewTimer {
    Ctx& ctx;
    int slot = -1;
    ViewTimer(Ctx& c, int kind) : ctx(c) {
        rsvd_view_trace* t = ctx.trace;
        ++ctx.trace_depth;
        if (ctx.dry || !t || !t->events || t->used >= t->capacity) return;
        // whole views and passes (depth 1), or with `inner` the products inside a pass
        const bool pass = kind == 2 || kind == 3;
        if (t->inner ? (ctx.trace_depth == 1 && pass) || ctx.trace_depth > 2 : ctx.trace_depth > 1) return;
        slot = t->used++;
        if (t->kind) t->kind[slot] = kind;
        (void)hipEventRecord(t->events[2 * slot], ctx.st);
    }
    ~ViewTimer() {
        --ctx.trace_depth;
        if (slot >= 0) (void)hipEventRecord(ctx.trace->events[2 * slot + 1], ctx.st);
    }
};

#define CALL(expr)                                   \
    do {                                             \
        if (!ctx.dry) {                              \
            rsvd_status e_ = (expr);                 \
            if (e_ != RSVD_OK) return e_;            \
        }                                            \
    } while (0)

#define TRY(expr)                                \
    do {                                         \
        rsvd_status e_ = (expr);                 \
        if (e_ != RSVD_OK) return e_;            \
    } while (0)

// Logical matrix A (m x n) over the stored buffer.
struct Mat {
    int dtype;
    const char* data;
    int64_t m, n, ld;
    int trans;
    size_t esize;
    const float* row_scale;  // FP8: one scale per stored row
};

size_t dtype_size(int d) { return d == RSVD_F64 ? 8 : d == RSVD_F32 ? 4 : d == RSVD_BF16 ? 2 : 1; }

Mat make_mat(const rsvd_mat* A) {
    Mat a;
    a.dtype = A->dtype;
    a.data = (const char*)A->data;
    a.m = A->m;
    a.n = A->n;
    a.ld = A->ld;
    a.trans = A->trans;
    a.esize = dtype_size(A->dtype);
    a.row_scale = A->row_scale;
    return a;
}

Mat rows_of(const Mat& a, int64_t r0, int64_t r1) {
    Mat b = a;
    b.m = r1 - r0;
    b.data = a.trans ? a.data + r0 * a.esize : a.data + r0 * a.ld * a.esize;
    if (a.row_scale && !a.trans) b.row_scale = a.row_scale + r0;
    return b;
}

Mat transposed(const Mat& a) {
    Mat b = a;
    b.m = a.n;
    b.n = a.m;
    b.trans = !a.trans;
    return b;
}

int work_dtype(int dtype) { return dtype == RSVD_F64 ? RSVD_F64 : RSVD_F32; }

struct set_int_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        int* p;
        int v;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [p, v] = args_;
     *p = v; 
    }
};
struct clear_header_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        uint32_t* h;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [h] = args_;
        if (threadIdx.x < kHeader / 4) h[threadIdx.x] = 0u;
    }
};

bool low_precision(int dtype) { return dtype == RSVD_BF16 || dtype == RSVD_FP8_E4M3; }

// A view through the BF16 / FP8 matrix-core kernels.  Returns false (and
// does nothing) when the launch does not apply: an FP32 A whose split form
// does not fit or is not aligned takes the FP32 path instead.
rsvd_status lp_view(Ctx& ctx, const Mat& a, const void* XT, int64_t ldx, int s, void* YT, int64_t ldy, int accumulate,
                    bool accurate, bool* done) {
    *done = false;
    const bool split_f32 = a.dtype == RSVD_F32 && ctx.f32_mode == RSVD_F32_BF16X6;
    if (!low_precision(a.dtype) && !split_f32) return RSVD_OK;
    LpArgs v;
    v.dtype = a.dtype;
    v.A = a.data;
    v.lda = a.ld;
    const bool cor = a.trans != 0;   // the stored matrix is A^T: A X = S^T X
    v.m = cor ? a.n : a.m;
    v.n = cor ? a.m : a.n;
    v.row_scale = cor ? nullptr : a.row_scale;
    v.thin_kind = (split_f32 || accurate) ? LP_THIN_BF16X3 : a.dtype == RSVD_FP8_E4M3 ? LP_THIN_FP8 : LP_THIN_BF16;
    v.s = s;
    // the planning (dry) pass sees the caller's pointer too, so both passes take the same branch
    if (s > view_max_width() || !lp_fits(v, cor) || !lp_aligned(a.dtype, a.data, a.ld)) {
        if (split_f32) return RSVD_OK;
        return s > view_max_width() || !lp_fits(v, cor) ? RSVD_EUNSUPPORTED : RSVD_EINVAL;
    }
    void* buf = ctx.ar.take<char>(lp_thin_bytes(v.thin_kind, s, a.n));
    const ViewPlan p = plan_lp(v, cor, ctx.plan_cus);
    float* part = ctx.ar.take<float>(p.splits > 1 ? (size_t)p.splits * s * a.m : 0);
    CALL(lp_prepare_thin((const float*)XT, ldx, s, a.n, cor ? a.row_scale : nullptr, v.thin_kind, buf, v, ctx.st));
    CALL(run_lp(v, p, cor, (float*)YT, ldy, part, accumulate, ctx.st));
    *done = true;
    return RSVD_OK;
}

// Contraction-split slots carried across the blocks of one sweep whose output
// sums the blocks' products (Z = sum_b A_b^T Y_b, W = sum_b Psi_b A_b): every
// block adds into the same slots, and carry_finish sums them into the output
// once, in a fixed order, after the last block.  The first block fixes the
// slot count (later blocks are never longer, so their plans are capped to
// it).  Without splits the blocks add into the output directly.  Views that
// take the BF16 / FP8 kernels or slices of the thin dimension do not carry:
// they reduce per block as usual.
struct SplitCarry {
    int blocks = 0;          // blocks that took the carried form
    int64_t splits = 0;      // slots (1: the blocks add into the output)
    void* part = nullptr;
    void* out = nullptr;
    int64_t ldo = 0, len = 0;
    int s = 0, dtype = 0, acc0 = 0;
};

// Y^T (s x m) [+]= (A X)^T for a panel X^T (s x n).  Widths above the
// kernel's limit are processed in slices of the thin dimension.  For a
// BF16 / FP8 A, accurate selects the FP32-accurate thin operand (three
// BF16 planes) over the quantized one.
// The sums of contraction splits are launched after the products of all
// slices, outside the trace hook's timing of the view, so that a traced view
// is the time of its product kernels alone.
rsvd_status range_view(Ctx& ctx, const Mat& a, const void* XT, int64_t ldx, int s, void* YT, int64_t ldy,
                       int accumulate, int kind = 0, bool accurate = false, SplitCarry* carry = nullptr) {
    struct SplitSum {
        int dtype, nparts;
        const void* part;
        int64_t s, len, ldo;
        void* out;
        int accumulate;
    };
    SplitSum sums[8];   // one per slice of the thin dimension (s <= 512, slices of at least 128)
    int nsums = 0;
    {
    ViewTimer timer(ctx, kind);
    const size_t ws = dtype_size(work_dtype(a.dtype));
    // slices of the thin dimension: 128 for FP64 (wider accumulators spill), else the kernels' 256
    const int slice = a.dtype == RSVD_F64 ? 128 : view_max_width();
    for (int j0 = 0; j0 < s; j0 += slice) {
        const int sj = std::min(slice, s - j0);
        const char* x = (const char*)XT + (size_t)j0 * ldx * ws;
        char* y = (char*)YT + (size_t)j0 * ldy * ws;
        bool done = false;
        TRY(lp_view(ctx, a, x, ldx, sj, y, ldy, accumulate, accurate, &done));
        if (done) continue;
        ViewArgs v;
        v.dtype = work_dtype(a.dtype);
        v.A = a.data;
        v.lda = a.ld;
        v.thin = x;
        v.ld_thin = ldx;
        v.s = sj;
        v.mr_hint = ctx.view_mr;
        // both kernels contract over a.n and write a.m outputs per thin column
        if (!a.trans) {
            v.m = a.m;
            v.n = a.n;
        } else {  // stored B = A^T (n x m): A X = B^T X
            v.m = a.n;
            v.n = a.m;
        }
        ViewPlan p = a.trans ? plan_corange(v, ctx.plan_cus) : plan_range(v, ctx.plan_cus);
        void* part;
        int acc = accumulate;
        const bool carried = carry && sj == s;
        if (carried) {
            if (carry->blocks == 0) {
                carry->splits = p.splits;
                carry->part = ctx.ar.take<char>(view_partial_elems(p, sj, a.m) * ws);
                carry->out = y;
                carry->ldo = ldy;
                carry->len = a.m;
                carry->s = sj;
                carry->dtype = v.dtype;
                carry->acc0 = accumulate;
                if (p.splits > 1) acc = 0;
            } else {
                p = cap_splits(p, a.n, carry->splits);
                acc = 1;
            }
            ++carry->blocks;
            part = carry->part;
        } else {
            part = ctx.ar.take<char>(view_partial_elems(p, sj, a.m) * ws);
        }
        // once the first block filled slots, every later block adds into them, even one short
        // enough for a single split; a view that does not carry fills its own slots and sums
        // them below
        const bool own_sum = !carried && p.splits > 1;
        const bool slots = (carried && carry->splits > 1) || own_sum;
        if (own_sum) {
            if (nsums >= 8) return RSVD_EUNSUPPORTED;
            sums[nsums++] = SplitSum{v.dtype, (int)p.splits, part, sj, a.m, ldy, y, accumulate};
            acc = 0;
        }
        if (!a.trans) CALL(run_range(v, p, y, ldy, part, acc, ctx.st, slots));
        else CALL(run_corange(v, p, y, ldy, part, acc, ctx.st, slots));
    }
    }
    for (int i = 0; i < nsums; ++i)
        CALL(run_reduce_view_parts(sums[i].dtype, sums[i].part, sums[i].nparts, sums[i].s, sums[i].len, sums[i].out,
                                   sums[i].ldo, sums[i].accumulate, ctx.st));
    return RSVD_OK;
}

// The output of a carried sweep: the sum of its split slots (nothing to do
// when the blocks added into the output directly or did not carry).
rsvd_status carry_finish(Ctx& ctx, const SplitCarry& c) {
    if (c.blocks == 0 || c.splits <= 1) return RSVD_OK;
    CALL(run_reduce_view_parts(c.dtype, c.part, (int)c.splits, c.s, c.len, c.out, c.ldo, c.acc0, ctx.st));
    return RSVD_OK;
}

// Z^T (s x n) [+]= (A^T Y)^T for a panel Y^T (s x m).
rsvd_status corange_view(Ctx& ctx, const Mat& a, const void* YT, int64_t ldy, int s, void* ZT, int64_t ldz,
                         int accumulate, bool accurate = false, SplitCarry* carry = nullptr) {
    return range_view(ctx, transposed(a), YT, ldy, s, ZT, ldz, accumulate, 1, accurate, carry);
}

// CholeskyQR2 (+ a third round after a shifted first round) of a panel
// P (s x len).  Q may alias P.  If Rout is given it receives the triangular
// factor R of P^T = Q^T-panel^T R; if Rinv_out is given, R^-1.
rsvd_status orth(Ctx& ctx, int dtype_in, const void* P, int64_t ldp, int s, int64_t len, int dtype_out, void* Q,
                 int64_t ldq, double* Rout, double* Rinv_out = nullptr) {
    if (s > kMaxWidth) return RSVD_EUNSUPPORTED;
    double* G = ctx.ar.take<double>((size_t)s * s);
    double* R = ctx.ar.take<double>((size_t)s * s);
    double* Rinv = ctx.ar.take<double>((size_t)s * s);
    double* tmp = ctx.ar.take<double>((size_t)s * s);
    double* scr = ctx.ar.take<double>(cross_scratch_doubles(s, s, len, 1, ctx.plan_cus));
    double* gscr = chol_fits_lds(s) ? nullptr : ctx.ar.take<double>((size_t)round_up(s, 16) * (round_up(s, 16) + 1));
    // above 256 columns Q = P R^-1 is applied in 256-row slices of the output, which must not
    // overwrite the panel they read: go through a second panel
    const bool wide = s > 256;
    void* T = wide ? ctx.ar.take<char>((size_t)s * len * dtype_size(dtype_out)) : nullptr;
    int* more = ctx.flags ? ctx.flags + (ctx.next_flag++ % 56) : nullptr;
    // a Gram within sqrt(u) of the identity (u: unit roundoff of the output panel) is
    // factored in closed form, exact to u/2: this is the usual second round
    const double near_id_tol2 = dtype_out == RSVD_F64 ? 0x1p-53 : 0x1p-24;
    if (!ctx.dry) {
        launch_phase();
        launch_op<set_int_kernel_op>(dim3(1), dim3(1), 0, ctx.st, {more, 0});
        RSVD_LAUNCH_CHECK();
    }
    for (int round = 0; round < 3; ++round) {
        const int* en = round == 2 ? more : nullptr;
        const void* src = round == 0 ? P : Q;
        const int dsrc = round == 0 ? dtype_in : dtype_out;
        const int64_t lsrc = round == 0 ? ldp : ldq;
        CALL(run_cross(dsrc, src, lsrc, s, dsrc, src, lsrc, s, len, 1, G, scr, ctx.plan_cus, en, ctx.st));
        CALL(run_chol_inv(G, s, len, R, Rinv, gscr, ctx.status, round == 0 ? more : nullptr, en, ctx.st,
                          near_id_tol2));
        // the first round's R^-1 carries the condition number of P and is applied with FP64 sums;
        // later rounds apply a near-identity R^-1 to an almost orthonormal Q, where FP32 sums
        // on FP32 matrix cores lose nothing that FP32 storage keeps
        const bool f32_sums = round > 0;
        if (wide) {
            CALL(run_apply_rinv(dsrc, src, lsrc, s, len, Rinv, dtype_out, T, len, en, ctx.st, f32_sums));
            CALL(run_copy_panel(dtype_out, T, len, Q, ldq, s, len, en, ctx.st));
        } else {
            CALL(run_apply_rinv(dsrc, src, lsrc, s, len, Rinv, dtype_out, Q, ldq, en, ctx.st, f32_sums));
        }
        if (Rout) {
            if (round == 0) CALL(run_copy_f64(R, Rout, (int64_t)s * s, ctx.st));
            else CALL(run_trmm_upper(R, Rout, tmp, s, 0, en, ctx.st));
        }
        if (Rinv_out) {
            if (round == 0) CALL(run_copy_f64(Rinv, Rinv_out, (int64_t)s * s, ctx.st));
            else CALL(run_trmm_upper(Rinv, Rinv_out, tmp, s, 1, en, ctx.st));
        }
    }
    return RSVD_OK;
}


// U = Q_c-panel^T Fu[:, :k], V = Q_r-panel^T Fv[:, :k], S = sigma[:k], then the joint sign fix.
rsvd_status finish(Ctx& ctx, int wdt_c, const void* QcT, int64_t ldc, int sc, int64_t m, int wdt_r, const void* QrT,
                   int64_t ldr, int sr, int64_t n, const double* Fu, int ldfu, const double* Fv, int ldfv,
                   const double* sigma, int k, int out_dtype, rsvd_out* out) {
    double* pval = ctx.ar.take<double>((size_t)sign_chunks(m) * k);
    int64_t* pidx = ctx.ar.take<int64_t>((size_t)sign_chunks(m) * k);
    double* sgn = ctx.ar.take<double>((size_t)k);
    CALL(run_lift(wdt_c, QcT, ldc, sc, m, Fu, ldfu, k, out_dtype, out->U, k, ctx.st));
    CALL(run_lift(wdt_r, QrT, ldr, sr, n, Fv, ldfv, k, out_dtype, out->V, k, ctx.st));
    CALL(run_copy_f64(sigma, out->S, k, ctx.st));
    CALL(run_signs(out_dtype, out->U, m, out->V, n, k, pval, pidx, sgn, ctx.st));
    return RSVD_OK;
}

// Small SVD M (s x s) = L diag(sig) Rv^T, with scratch when M does not fit LDS.
// A zero *enable skips it (device-side decision; L, Rv and sig are then left as they are).
rsvd_status small_svd(Ctx& ctx, const double* M, int s, double* L, double* Rv, double* sig,
                      const int* enable = nullptr) {
    const size_t jn = small_svd_scratch_doubles(s);
    double* jscr = jn ? ctx.ar.take<double>(jn) : nullptr;
    CALL(run_small_svd(M, s, L, Rv, sig, jscr, ctx.status, enable, ctx.st, ctx.sync_spins));
    return RSVD_OK;
}

// The same SVD, with the one-sided Jacobi run on the columns of M^T (the rows of
// M): M^T = Rv diag(sigma) L^T.  For the triangular factors that end Alg. 2 and
// Alg. 7 this converges in fewer sweeps (7 instead of 8, and 8 instead of 10,
// in an emulation with sigma_j = j^-1.5, s = 120).  The right vectors then come
// from the columns and the left ones from M w / sigma^2; the methods use the
// leading k of both.
rsvd_status small_svd_rows(Ctx& ctx, const double* M, int s, double* L, double* Rv, double* sig,
                           const int* enable = nullptr) {
    double* Mt = ctx.ar.take<double>((size_t)s * s);
    CALL(run_transpose_small_f64(M, Mt, s, ctx.st));
    return small_svd(ctx, Mt, s, Rv, L, sig, enable);
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------

rsvd_status check_common(const rsvd_mat* A, int k, int p, const rsvd_opts* o, const rsvd_out* out, bool need_out) {
    if (!A) return RSVD_EINVAL;
    if (A->dtype != RSVD_F64 && A->dtype != RSVD_F32 && A->dtype != RSVD_BF16 && A->dtype != RSVD_FP8_E4M3)
        return RSVD_EINVAL;
    if (A->m <= 0 || A->n <= 0) return RSVD_ESHAPE;
    if (A->trans != 0 && A->trans != 1) return RSVD_EINVAL;
    if (A->ld < (A->trans ? A->m : A->n)) return RSVD_ESHAPE;
    if (!A->data) return RSVD_EINVAL;
    if (A->dtype == RSVD_FP8_E4M3 && !A->row_scale) return RSVD_EINVAL;
    if (A->dtype != RSVD_FP8_E4M3 && A->row_scale) return RSVD_EINVAL;
    if (k < 1 || p < 0) return RSVD_EINVAL;
    if ((int64_t)k + p > std::min(A->m, A->n)) return RSVD_ESHAPE;
    if (o) {
        if (o->refine && A->dtype != RSVD_BF16 && A->dtype != RSVD_FP8_E4M3) return RSVD_EINVAL;
        if (o->block_rows < 0 || o->psi_rows < 0 || o->trunc_tau < 0 || o->core_rows < 0) return RSVD_EINVAL;
        if (o->f32_mode != RSVD_F32_MFMA && o->f32_mode != RSVD_F32_BF16X6) return RSVD_EINVAL;
        if (o->krylov_mode < 0 || o->krylov_mode > 2) return RSVD_EINVAL;
    }
    if (need_out && (!out || !out->U || !out->S || !out->V)) return RSVD_EINVAL;
    if (low_precision(A->dtype) && !lp_aligned(A->dtype, A->data, A->ld)) return RSVD_EINVAL;
    return RSVD_OK;
}

rsvd_opts opts_or_default(const rsvd_opts* o) {
    rsvd_opts d;
    rsvd_default_opts(&d);
    return o ? *o : d;
}

// ---------------------------------------------------------------------------
// Alg. 2: generalized subspace iteration
// ---------------------------------------------------------------------------
rsvd_status alg_subspace(Ctx& ctx, const Mat& a, int k, int p, int v, const rsvd_opts& o, rsvd_out* out) {
    const int s = k + p;
    if (s > kMaxWidth) return RSVD_EUNSUPPORTED;
    const int wdt = work_dtype(a.dtype);
    const size_t we = dtype_size(wdt);
    // panel rows padded to 16 bytes so that every row of a thin matrix is aligned
    const int64_t ldn = round_up(a.n, 4), ldm = round_up(a.m, 4);
    void* XT = ctx.ar.take<char>((size_t)s * ldn * we);  // Q_r panel (starts as Omega^T)
    void* YT = ctx.ar.take<char>((size_t)s * ldm * we);  // Q_c panel
    double* Rfin = ctx.ar.take<double>((size_t)s * s);
    double* L = ctx.ar.take<double>((size_t)s * s);
    double* Rv = ctx.ar.take<double>((size_t)s * s);
    double* sig = ctx.ar.take<double>((size_t)s);
    CALL(launch_gaussian(o.seed, TAG_OMEGA, 0, s, a.n, 0, wdt, XT, ldn, ctx.st));
    for (int j = 1; j <= v; ++j) {
        const bool last = j == v;
        const bool accurate = last && o.refine;   // BF16 / FP8 A: the refinement view
        if (j % 2 == 1) {   // [Q_c, R_c] = qr(A Q_r)
            TRY(range_view(ctx, a, XT, ldn, s, YT, ldm, 0, 0, accurate));
            TRY(orth(ctx, wdt, YT, ldm, s, a.m, wdt, YT, ldm, last ? Rfin : nullptr));
        } else {            // [Q_r, R_r] = qr(A^T Q_c)
            TRY(corange_view(ctx, a, YT, ldm, s, XT, ldn, 0, accurate));
            TRY(orth(ctx, wdt, XT, ldn, s, a.n, wdt, XT, ldn, last ? Rfin : nullptr));
        }
    }
    TRY(small_svd_rows(ctx, Rfin, s, L, Rv, sig));
    if (v % 2 == 0)  // R_r = V^ Lam U^^T: left factor -> V^, right factor -> U^
        return finish(ctx, wdt, YT, ldm, s, a.m, wdt, XT, ldn, s, a.n, Rv, s, L, s, sig, k, wdt, out);
    // R_c = U^ Lam V^^T
    return finish(ctx, wdt, YT, ldm, s, a.m, wdt, XT, ldn, s, a.n, L, s, Rv, s, sig, k, wdt, out);
}

// ---------------------------------------------------------------------------
// Alg. 7: one view
// ---------------------------------------------------------------------------
__global__ void small_gemm_kernel(const double* __restrict__ A, int64_t a_i, int64_t a_l, const double* __restrict__ B,
                                  int64_t b_l, int64_t b_j, int rows, int cols, int inner, double* __restrict__ C) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols; e += gridDim.x * blockDim.x) {
        const int i = e / cols, j = e % cols;
        double acc = 0.0;
        int l = 0;
        for (; l + 8 <= inner; l += 8) {   // eight terms' loads ahead of their sums, same order
            double u[8], w[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                u[q] = A[i * a_i + (l + q) * a_l];
                w[q] = B[(l + q) * b_l + j * b_j];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += u[q] * w[q];
        }
        for (; l < inner; ++l) acc += A[i * a_i + l * a_l] * B[l * b_l + j * b_j];
        C[e] = acc;
    }
}

// C (rows x cols, row-major) = A B for small FP64 operands with element
// strides: A[i][l] at A + i a_i + l a_l, B[l][j] at B + l b_l + j b_j.
rsvd_status gemm_small(Ctx& ctx, const double* A, int64_t a_i, int64_t a_l, const double* B, int64_t b_l,
                       int64_t b_j, int rows, int cols, int inner, double* C) {
    if (ctx.dry) return RSVD_OK;
    const int64_t total = (int64_t)rows * cols;
    hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 4096))),
                       dim3(256), 0, ctx.st, A, a_i, a_l, B, b_l, b_j, rows, cols, inner, C);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

// The side stream of the current device (default priority, created on first
// use, held until the process ends), or null if it cannot be created.
std::mutex g_side_mu;
std::map<int, hipStream_t> g_side;

hipStream_t side_stream() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(g_side_mu);
    auto it = g_side.find(dev);
    if (it != g_side.end()) return it->second;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    g_side[dev] = st;
    return st;
}

// One sweep over the row blocks of A: Y[b] = A_b X and Z = sum_b A_b^T T[b],
// each block's two products back to back.  The row sweep of Sect. 7.3 takes
// T[b] = Y[b] (thin_is_y); the one-view pass takes T[b] = Psi[:, b]^T, the
// block's columns of a panel T (s_t x m, leading dimension ldt).  The mode is
// an argument, never read off T: the planning pass sees every workspace
// pointer as null and must size the same views as the executing pass.
//
// The row sweep's co-range products carry their split slots across the
// blocks (one sum per sweep instead of one per 1024-row block).  The one-view
// pass sums each panel's splits at once: on its 4096 x 16384 panels with
// s_w = 241 the four splits hold 63 MB, and adding into carried slots (a read
// and a write of them per panel) cost 45 us per panel against 14 us for the
// panel's own sum.
//
// In the row sweep the range product of a block depends only on X, so the
// range products run on the side stream, ahead of the co-range products on
// the caller's stream, each of which waits for its block's Y[b]: the range
// product of block b + 1 then overlaps the co-range product of block b,
// which the short products of one 1024-row block alone leave the chip partly
// idle for (7% off the 32768 x 8192, v = 4 forward).  The one-view pass keeps
// one stream: its 4096-row panel products fill the chip, and overlapping them
// measured 2% slower.  The caller's stream waits for all of it.
rsvd_status block_sweep(Ctx& ctx, const Mat& a, int64_t rows, const void* X, int64_t ldx, int sx, char* Y,
                        int64_t ldy, bool thin_is_y, const char* T, int64_t ldt, int st, void* Z, int64_t ldz) {
    const size_t we = dtype_size(work_dtype(a.dtype));
    hipStream_t side = (ctx.dry || !thin_is_y) ? nullptr : side_stream();
    hipEvent_t ev_in = nullptr, ev_y = nullptr;
    if (side) {
        if (hipEventCreateWithFlags(&ev_in, hipEventDisableTiming) != hipSuccess) side = nullptr;
        else if (hipEventCreateWithFlags(&ev_y, hipEventDisableTiming) != hipSuccess) {
            (void)hipEventDestroy(ev_in);
            side = nullptr;
        }
    }
    auto done = [&](rsvd_status e) {
        if (side) {
            (void)hipEventDestroy(ev_in);
            (void)hipEventDestroy(ev_y);
        }
        return e;
    };
    auto join = [&](hipEvent_t ev, hipStream_t from, hipStream_t to) {
        return hipEventRecord(ev, from) == hipSuccess && hipStreamWaitEvent(to, ev, 0) == hipSuccess;
    };
    if (side && !join(ev_in, ctx.st, side)) return done(RSVD_EHIP);
    SplitCarry zc;
    for (int64_t r0 = 0; r0 < a.m; r0 += rows) {
        const int64_t r1 = std::min(a.m, r0 + rows);
        const Mat ab = rows_of(a, r0, r1);
        char* yb = Y + (size_t)r0 * we;
        const hipStream_t own = ctx.st;
        if (side) ctx.st = side;
        const rsvd_status e = range_view(ctx, ab, X, ldx, sx, yb, ldy, 0);
        ctx.st = own;
        if (e != RSVD_OK) return done(e);
        if (side && !join(ev_y, side, ctx.st)) return done(RSVD_EHIP);
        const rsvd_status f = thin_is_y
                                  ? corange_view(ctx, ab, yb, ldy, sx, Z, ldz, r0 > 0 ? 1 : 0, false, &zc)
                                  : corange_view(ctx, ab, T + (size_t)r0 * we, ldt, st, Z, ldz, r0 > 0 ? 1 : 0);
        if (f != RSVD_OK) return done(f);
    }
    return done(carry_finish(ctx, zc));
}

// Rows per panel of a one-view sweep: block_rows if given (for the
// one-view method this option is not the row-sweep block size but the panel
// height), else the largest multiple of 256 rows within 256 MiB, the size of
// the Infinity Cache. Taller panels mean fewer launches and fewer partial sums
// of W to reduce; the second product on a panel re-reads rows that the first
// one has just brought through the cache.
int64_t panel_rows(const Mat& a, int64_t requested) {
    if (requested > 0 && requested != 1024) return requested;
    const int64_t bytes_per_row = a.n * (int64_t)a.esize;
    const int64_t rows = ((int64_t)256 << 20) / std::max<int64_t>(1, bytes_per_row);
    return std::max<int64_t>(256, rows / 256 * 256);
}

// Sect. 6.7, the extended one-view sketch with the improved reconstruction
// (eq. bwzimproved), Gaussian core test matrices: Y_c = A Omega_r, Y_r^T =
// Psi A (s rows: l1 = l2), Z = Phi_r^T A Phi_c, all three from one sweep over
// row panels of A; then Q_c, Q_r, U_c T_c = qr(Phi_r^T Q_c), U_r T_r =
// qr(Phi_c^T Q_r), C = T_c^-1 U_c^T Z U_r T_r^-T and A ~ Q_c [[C]]_k Q_r^T.
rsvd_status alg_extended_one_view(Ctx& ctx, const Mat& a, int k, int p, const rsvd_opts& o, rsvd_out* out) {
    const int s = k + p;
    const int sc = o.core_rows;
    if (s > kMaxWidth || sc > 4 * kMaxWidth) return RSVD_EUNSUPPORTED;
    const int wdt = work_dtype(a.dtype);
    const size_t we = dtype_size(wdt);
    const int sx = s + sc;                                   // thin rows of the sweep
    void* XT = ctx.ar.take<char>((size_t)sx * a.n * we);     // [Omega_r^T; Phi_c^T] (s + s_c) x n
    void* PsiP = ctx.ar.take<char>((size_t)s * a.m * we);    // Psi = Omega_c^T (s x m)
    void* PhiP = ctx.ar.take<char>((size_t)sc * a.m * we);   // Phi_r^T (s_c x m)
    void* YT = ctx.ar.take<char>((size_t)sx * a.m * we);     // [Y_c^T; (A Phi_c)^T], then Q_c^T in the top rows
    void* W = ctx.ar.take<char>((size_t)s * a.n * we);       // Y_r^T = Psi A, then Q_r^T
    double* Z = ctx.ar.take<double>((size_t)sc * sc);
    double* PQc = ctx.ar.take<double>((size_t)s * sc);        // (Phi_r^T Q_c)^T as a panel (s x s_c), then U_c^T
    double* PQr = ctx.ar.take<double>((size_t)s * sc);        // (Phi_c^T Q_r)^T as a panel, then U_r^T
    double* Tcinv = ctx.ar.take<double>((size_t)s * s);
    double* Trinv = ctx.ar.take<double>((size_t)s * s);
    double* M1 = ctx.ar.take<double>((size_t)s * sc);         // U_c^T Z
    double* M2 = ctx.ar.take<double>((size_t)s * s);          // U_c^T Z U_r
    double* M3 = ctx.ar.take<double>((size_t)s * s);          // T_c^-1 U_c^T Z U_r
    double* C = ctx.ar.take<double>((size_t)s * s);
    double* L = ctx.ar.take<double>((size_t)s * s);
    double* Rv = ctx.ar.take<double>((size_t)s * s);
    double* sig = ctx.ar.take<double>((size_t)s);
    double* scr = ctx.ar.take<double>(std::max(cross_scratch_doubles(sc, sc, a.m, 0, ctx.plan_cus),
                                               std::max(cross_scratch_doubles(s, sc, a.m, 0, ctx.plan_cus),
                                                        cross_scratch_doubles(s, sc, a.n, 0, ctx.plan_cus))));
    char* Phi2 = (char*)XT + (size_t)s * a.n * we;            // Phi_c^T rows of the thin panel
    const char* TP = (const char*)YT + (size_t)s * a.m * we;  // (A Phi_c)^T rows

    CALL(launch_gaussian(o.seed, TAG_OMEGA, 0, s, a.n, 0, wdt, XT, a.n, ctx.st));
    CALL(launch_gaussian(o.seed, TAG_PSI, 0, s, a.m, 0, wdt, PsiP, a.m, ctx.st));
    if (o.core_kind == RSVD_CORE_SRFT) {
        // the paper's SRFTs: Phi_c^T and Phi_r^T as subsampled randomized DCT panels
        int* pos_c = ctx.ar.take<int>((size_t)sc);
        int* pos_r = ctx.ar.take<int>((size_t)sc);
        CALL(run_srft_panel(o.seed, TAG_SRFT_SIGN_C, TAG_SRFT_SAMPLE_C, a.n, sc, pos_c, wdt, Phi2, a.n, ctx.st));
        CALL(run_srft_panel(o.seed, TAG_SRFT_SIGN_R, TAG_SRFT_SAMPLE_R, a.m, sc, pos_r, wdt, PhiP, a.m, ctx.st));
    } else {
        CALL(launch_gaussian(o.seed, TAG_PHI2, 0, sc, a.n, 0, wdt, Phi2, a.n, ctx.st));
        CALL(launch_gaussian(o.seed, TAG_PHI, 0, sc, a.m, 0, wdt, PhiP, a.m, ctx.st));
    }
    // one sweep over row panels: [Y_c; A Phi_c][b] = A_b [Omega_r, Phi_c] and W += Psi[:, b] A_b
    {
        ViewTimer timer(ctx, 2);
        const int64_t rows = panel_rows(a, o.block_rows);
        TRY(block_sweep(ctx, a, rows, XT, a.n, sx, (char*)YT, a.m, false, (const char*)PsiP, a.m, s, W, a.n));
    }
    // Z = Phi_r^T (A Phi_c): s_c x s_c, FP64 sums over the long side
    CALL(run_cross(wdt, PhiP, a.m, sc, wdt, TP, a.m, sc, a.m, 0, Z, scr, ctx.plan_cus, nullptr, ctx.st));
    // Q_c R_c = Y_c, Q_r R_r = Y_r
    TRY(orth(ctx, wdt, YT, a.m, s, a.m, wdt, YT, a.m, nullptr));
    TRY(orth(ctx, wdt, W, a.n, s, a.n, wdt, W, a.n, nullptr));
    // U_c T_c = Phi_r^T Q_c and U_r T_r = Phi_c^T Q_r (panels s x s_c)
    CALL(run_cross(wdt, YT, a.m, s, wdt, PhiP, a.m, sc, a.m, 0, PQc, scr, ctx.plan_cus, nullptr, ctx.st));
    CALL(run_cross(wdt, W, a.n, s, wdt, Phi2, a.n, sc, a.n, 0, PQr, scr, ctx.plan_cus, nullptr, ctx.st));
    TRY(orth(ctx, RSVD_F64, PQc, sc, s, sc, RSVD_F64, PQc, sc, nullptr, Tcinv));
    TRY(orth(ctx, RSVD_F64, PQr, sc, s, sc, RSVD_F64, PQr, sc, nullptr, Trinv));
    // C = T_c^-1 (U_c^T Z U_r) T_r^-T; U_c^T and U_r^T are the panels PQc, PQr (s x s_c)
    if (!ctx.dry) {
        const dim3 b(256);
        hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)ceil_div((int64_t)s * sc, 256)), b, 0, ctx.st, PQc,
                           (int64_t)sc, (int64_t)1, Z, (int64_t)sc, (int64_t)1, s, sc, sc, M1);
        hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)ceil_div((int64_t)s * s, 256)), b, 0, ctx.st, M1,
                           (int64_t)sc, (int64_t)1, PQr, (int64_t)1, (int64_t)sc, s, s, sc, M2);
        hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)ceil_div((int64_t)s * s, 256)), b, 0, ctx.st, Tcinv,
                           (int64_t)s, (int64_t)1, M2, (int64_t)s, (int64_t)1, s, s, s, M3);
        hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)ceil_div((int64_t)s * s, 256)), b, 0, ctx.st, M3,
                           (int64_t)s, (int64_t)1, Trinv, (int64_t)1, (int64_t)s, s, s, s, C);
        RSVD_LAUNCH_CHECK();
    }
    // [[C]]_k: C = L S Rv^T, U = Q_c L_k, V = Q_r Rv_k
    TRY(small_svd(ctx, C, s, L, Rv, sig));
    return finish(ctx, wdt, YT, a.m, s, a.m, wdt, W, a.n, s, a.n, L, s, Rv, s, sig, k, wdt, out);
}

rsvd_status one_view_small(Ctx& ctx, int wdt, void* YT, int64_t ldy, int64_t m, const void* W, int64_t ldw, int64_t n,
                           const void* PsiP, int64_t ldpsi, int k, int p, int sw, const rsvd_opts& o, rsvd_out* out);

rsvd_status alg_single_pass(Ctx& ctx, const Mat& a, int k, int p, const rsvd_opts& o, rsvd_out* out) {
    if (o.core_rows > 0) return alg_extended_one_view(ctx, a, k, p, o, out);
    const int s = k + p;
    const int64_t sw64 = o.psi_rows ? o.psi_rows : 2 * (int64_t)s + 1;
    if (sw64 < s || sw64 > a.m) return RSVD_ESHAPE;
    const int sw = (int)sw64;
    if (s > kMaxWidth || sw > 4 * kMaxWidth) return RSVD_EUNSUPPORTED;
    const int wdt = work_dtype(a.dtype);
    const size_t we = dtype_size(wdt);
    void* XT = ctx.ar.take<char>((size_t)s * a.n * we);      // Omega^T
    void* PsiP = ctx.ar.take<char>((size_t)sw * a.m * we);   // Psi (s_w x m)
    void* YT = ctx.ar.take<char>((size_t)s * a.m * we);      // Y^T, then Q_c^T
    void* W = ctx.ar.take<char>((size_t)sw * a.n * we);      // W = Psi A (s_w x n)
    double* PQ = ctx.ar.take<double>((size_t)s * sw);         // (Psi Q_c)^T as a panel (s x s_w)
    double* Qh = ctx.ar.take<double>((size_t)s * sw);         // Q^ as a panel
    double* Rhinv = ctx.ar.take<double>((size_t)s * s);       // R^^-1
    double* M2T = ctx.ar.take<double>((size_t)sw * s);        // (R^^-1 Q^^T)^T = Q^ R^^-T (s_w x s)
    double* XP = ctx.ar.take<double>((size_t)s * a.n);        // X (s x n), then Q_r^T
    double* Rr = ctx.ar.take<double>((size_t)s * s);
    double* L = ctx.ar.take<double>((size_t)s * s);
    double* Rv = ctx.ar.take<double>((size_t)s * s);
    double* sig = ctx.ar.take<double>((size_t)s);
    double* scr = ctx.ar.take<double>(cross_scratch_doubles(s, sw, a.m, 0, ctx.plan_cus));

    // a) Omega_r and b) Omega_c^T = Psi
    CALL(launch_gaussian(o.seed, TAG_OMEGA, 0, s, a.n, 0, wdt, XT, a.n, ctx.st));
    CALL(launch_gaussian(o.seed, TAG_PSI, 0, sw, a.m, 0, wdt, PsiP, a.m, ctx.st));
    // a) Y_c = A Omega_r and b) Y_r^T = W = Psi A in one sweep over row
    // panels of A: Y[b] = A_b Omega, W += Psi[:, b] A_b, the two products on a
    // panel back to back.
    {
        ViewTimer timer(ctx, 2);
        const int64_t rows = panel_rows(a, o.block_rows);
        TRY(block_sweep(ctx, a, rows, XT, a.n, s, (char*)YT, a.m, false, (const char*)PsiP, a.m, sw, W, a.n));
    }
    if (o.one_view_method != RSVD_ONE_VIEW_TROPP || o.lc_rule != RSVD_LC_FULL)
        return one_view_small(ctx, wdt, YT, a.m, a.m, W, a.n, a.n, PsiP, a.m, k, p, sw, o, out);
    if (!ctx.dry && ctx.status)
        launch_op<set_int_kernel_op>(dim3(1), dim3(1), 0, ctx.st, {(int*)(ctx.status + kLcWord), p});
    // [Q_c, ~] = qr(Y_c)
    TRY(orth(ctx, wdt, YT, a.m, s, a.m, wdt, YT, a.m, nullptr));
    // (Psi Q_c)^T = Q_c^T Psi^T: panel s x s_w
    CALL(run_cross(wdt, YT, a.m, s, wdt, PsiP, a.m, sw, a.m, 0, PQ, scr, ctx.plan_cus, nullptr, ctx.st));
    // [Q^, R^] = qr(Psi Q_c)
    TRY(orth(ctx, RSVD_F64, PQ, sw, s, sw, RSVD_F64, Qh, sw, nullptr, Rhinv));
    // X = R^^-1 Q^^T W: first M2^T = Q^ R^^-T (s_w x s), then X = M2 W
    if (!ctx.dry) {
        hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)ceil_div((int64_t)sw * s, 256)), dim3(256), 0, ctx.st, Qh,
                           (int64_t)1, (int64_t)sw, Rhinv, (int64_t)1, (int64_t)s, sw, s, s, M2T);
        RSVD_LAUNCH_CHECK();
    }
    CALL(run_apply_coeff(wdt, W, a.n, sw, a.n, M2T, s, s, 0, 1.0, 0.0, RSVD_F64, XP, a.n, nullptr, ctx.st));
    // tsvd(X, k) through X^T = Q_r R_r:  R_r = L S Rv^T  =>  X = Rv S (Q_r L)^T
    TRY(orth(ctx, RSVD_F64, XP, a.n, s, a.n, RSVD_F64, XP, a.n, Rr));
    TRY(small_svd_rows(ctx, Rr, s, L, Rv, sig));
    return finish(ctx, wdt, YT, a.m, s, a.m, RSVD_F64, XP, a.n, s, a.n, Rv, s, L, s, sig, k, wdt, out);
}

// ---------------------------------------------------------------------------
// Sect. 6.5 and 6.6: one-view post-processing in the small space.
//
// From the sketches Y (Q_Y R_Y after CholeskyQR) and W = Psi A (W^T = Q_W R_W,
// Q_W an FP64 panel), every quantity a choice of l_c and of Alg. 7 / Alg. 8
// needs is an s_w-sized matrix:
//   Q_c = Q_Y L_Y[:, :j]       (j = k + l_c; R_Y = L_Y S_Y (.)^T),
//   Psi Q_c = (Psi Q_Y) L_Y[:, :j] = Q^ R^,
//   X = R^^-1 Q^^T W = M Q_W^T with M = R^^-1 Q^^T R_W^T (j x s_w),
//   Alg. 7: M^T = Q_m R_m, R_m = L_m S (R_v)^T, so M = R_v S (Q_m L_m)^T and
//           U = Q_Y (L_Y[:, :j] R_v[:, :k]), V = Q_W (Q_m L_m[:, :k]);
//   Alg. 8: Q_r = Q_W L_W[:, :j] (R_W = L_W S_W (.)^T), W Q_r = R_W^T L_W[:, :j],
//           X^ = M L_W[:, :j] = L_x S R_x^T,
//           U = Q_Y (L_Y[:, :j] L_x[:, :k]), V = Q_W (L_W[:, :j] R_x[:, :k]).
// The spectrum of X(l_c) is that of M.  Each candidate l_c leaves its
// coefficient matrices (s x k and s_w x k) and k singular values in a slot;
// the minimum-variance rule picks a slot on the device.
// ---------------------------------------------------------------------------

// eq. MinVar over candidates c = 0..l1 (spec: (l1 + 1) x k leading singular
// values, one row per c): for 0 <= c < l1 the population variance of the
// ratios lambda(c-1)/lambda(c) (c > 0), lambda(c)/lambda(c) and
// lambda(c+1)/lambda(c), each mean taken in a fixed order; the smallest
// variance wins, ties to the smallest c (a NaN variance never wins, so a
// NaN at c = 0 keeps c = 0).  Copies the chosen slot into the final
// coefficients and records the choice in the header word *lc_out.  One
// workgroup.
__global__ void __launch_bounds__(256)
minvar_select_kernel(const double* __restrict__ spec, int k, int l1, const double* __restrict__ CU,
                     const double* __restrict__ CV, const double* __restrict__ SG, int64_t cu_len, int64_t cv_len,
                     double* __restrict__ CUf, double* __restrict__ CVf, double* __restrict__ SGf,
                     uint32_t* __restrict__ lc_out) {
    __shared__ double var_sh[512];
    __shared__ int pick_sh;
    for (int c = threadIdx.x; c < l1; c += blockDim.x) {
        const double* lc0 = spec + (int64_t)c * k;
        const double* lp = spec + (int64_t)(c + 1) * k;
        const double* lm = c > 0 ? spec + (int64_t)(c - 1) * k : nullptr;
        const int cnt = (c > 0 ? 3 : 2) * k;
        double sum = 0.0;
        for (int i = 0; i < k; ++i) {
            if (lm) sum += lm[i] / lc0[i];
            sum += lc0[i] / lc0[i];
            sum += lp[i] / lc0[i];
        }
        const double mean = sum / cnt;
        double ss = 0.0;
        for (int i = 0; i < k; ++i) {
            double d;
            if (lm) {
                d = lm[i] / lc0[i] - mean;
                ss += d * d;
            }
            d = lc0[i] / lc0[i] - mean;
            ss += d * d;
            d = lp[i] / lc0[i] - mean;
            ss += d * d;
        }
        var_sh[c] = ss / cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int best = 0;
        if (l1 > 0) {
            double bv = var_sh[0];
            for (int c = 1; c < l1; ++c)
                if (var_sh[c] < bv) {
                    bv = var_sh[c];
                    best = c;
                }
        }
        pick_sh = best;
        *lc_out = (uint32_t)best;
    }
    __syncthreads();
    const int c = pick_sh;
    for (int64_t e = threadIdx.x; e < cu_len; e += blockDim.x) CUf[e] = CU[c * cu_len + e];
    for (int64_t e = threadIdx.x; e < cv_len; e += blockDim.x) CVf[e] = CV[c * cv_len + e];
    for (int e = threadIdx.x; e < k; e += blockDim.x) SGf[e] = SG[(int64_t)c * k + e];
}

__global__ void copy_prefix_kernel(const double* __restrict__ src, int64_t count, double* __restrict__ dst) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

rsvd_status copy_small(Ctx& ctx, const double* src, int64_t count, double* dst) {
    if (ctx.dry || count <= 0) return RSVD_OK;
    hipLaunchKernelGGL(copy_prefix_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(count, 256), 1024)), dim3(256), 0,
                       ctx.st, src, count, dst);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

// The fixed l_c of a rule other than the minimum-variance one (-1 for that one).
int fixed_lc(const rsvd_opts& o, int p) {
    if (o.lc_rule == RSVD_LC_FIXED) return o.lc;
    if (o.lc_rule == RSVD_LC_RATIO) return (int)std::floor(o.lc_alpha * (double)p);
    if (o.lc_rule == RSVD_LC_MINVAR) return -1;
    return p;
}

// YT: the range sketch panel (s x m, overwritten with Q_Y), W: the co-range
// sketch panel (s_w x n, read only), PsiP: Psi (s_w x m).
rsvd_status one_view_small(Ctx& ctx, int wdt, void* YT, int64_t ldy, int64_t m, const void* W, int64_t ldw, int64_t n,
                           const void* PsiP, int64_t ldpsi, int k, int p, int sw, const rsvd_opts& o, rsvd_out* out) {
    const int s = k + p;
    if (s > kMaxWidth || sw > kMaxWidth) return RSVD_EUNSUPPORTED;
    const bool woolfe = o.one_view_method == RSVD_ONE_VIEW_WOOLFE;
    const int lc_fix = fixed_lc(o, p);
    const bool minvar = lc_fix < 0;
    const int c0 = minvar ? 0 : lc_fix, c1 = minvar ? p : lc_fix;
    const int ncand = c1 - c0 + 1;
    double* RY = ctx.ar.take<double>((size_t)s * s);
    double* LY = ctx.ar.take<double>((size_t)s * s);
    double* RvY = ctx.ar.take<double>((size_t)s * s);
    double* sgY = ctx.ar.take<double>((size_t)s);
    double* PQ = ctx.ar.take<double>((size_t)s * sw);          // (Psi Q_Y)^T: panel s x s_w
    double* QW = ctx.ar.take<double>((size_t)sw * n);          // Q_W^T: FP64 panel s_w x n
    double* RW = ctx.ar.take<double>((size_t)sw * sw);
    double* LW = woolfe ? ctx.ar.take<double>((size_t)sw * sw) : nullptr;
    double* RvW = woolfe ? ctx.ar.take<double>((size_t)sw * sw) : nullptr;
    double* sgW = woolfe ? ctx.ar.take<double>((size_t)sw) : nullptr;
    double* T = ctx.ar.take<double>((size_t)s * sw);           // (Psi Q_c)^T, then Q^^T
    double* Rhi = ctx.ar.take<double>((size_t)s * s);          // R^^-1
    double* N = ctx.ar.take<double>((size_t)s * sw);           // Q^^T R_W^T
    double* Mp = ctx.ar.take<double>((size_t)s * sw);          // M (j x s_w)
    double* Qm = ctx.ar.take<double>((size_t)s * sw);          // Q_m^T
    double* Rm = ctx.ar.take<double>((size_t)s * s);
    double* L2 = ctx.ar.take<double>((size_t)s * s);
    double* R2 = ctx.ar.take<double>((size_t)s * s);
    double* sg2 = ctx.ar.take<double>((size_t)s);
    double* Xh = woolfe ? ctx.ar.take<double>((size_t)s * s) : nullptr;
    const int64_t cu_len = (int64_t)s * k, cv_len = (int64_t)sw * k;
    double* CU = ctx.ar.take<double>((size_t)ncand * cu_len);
    double* CV = ctx.ar.take<double>((size_t)ncand * cv_len);
    double* SG = ctx.ar.take<double>((size_t)ncand * k);
    double* SPEC = minvar ? ctx.ar.take<double>((size_t)ncand * k) : nullptr;
    double* CUf = minvar ? ctx.ar.take<double>((size_t)cu_len) : CU;
    double* CVf = minvar ? ctx.ar.take<double>((size_t)cv_len) : CV;
    double* SGf = minvar ? ctx.ar.take<double>((size_t)k) : SG;
    double* scr = ctx.ar.take<double>(std::max(cross_scratch_doubles(s, sw, m, 0, ctx.plan_cus),
                                               cross_scratch_doubles(s, sw, sw, 0, ctx.plan_cus)));

    // Y = Q_Y R_Y; (Psi Q_Y)^T; W^T = Q_W R_W; R_Y = L_Y S_Y Rv_Y^T
    TRY(orth(ctx, wdt, YT, ldy, s, m, wdt, YT, ldy, RY));
    CALL(run_cross(wdt, YT, ldy, s, wdt, PsiP, ldpsi, sw, m, 0, PQ, scr, ctx.plan_cus, nullptr, ctx.st));
    TRY(orth(ctx, wdt, W, ldw, sw, n, RSVD_F64, QW, n, RW));
    TRY(small_svd(ctx, RY, s, LY, RvY, sgY));
    if (woolfe) TRY(small_svd(ctx, RW, sw, LW, RvW, sgW));
    for (int c = c0; c <= c1; ++c) {
        const int j = k + c, slot = c - c0;
        // (Psi Q_c)^T = L_Y[:, :j]^T (Psi Q_Y)^T, then [Q^, R^] = qr(Psi Q_c)
        CALL(run_apply_coeff(RSVD_F64, PQ, sw, s, sw, LY, s, j, 0, 1.0, 0.0, RSVD_F64, T, sw, nullptr, ctx.st));
        TRY(orth(ctx, RSVD_F64, T, sw, j, sw, RSVD_F64, T, sw, nullptr, Rhi));
        // M = R^^-1 (Q^^T R_W^T)
        CALL(run_cross(RSVD_F64, T, sw, j, RSVD_F64, RW, sw, sw, sw, 0, N, scr, ctx.plan_cus, nullptr, ctx.st));
        TRY(gemm_small(ctx, Rhi, j, 1, N, sw, 1, j, sw, j, Mp));
        if (!woolfe || minvar) {
            // M^T = Q_m R_m, R_m = L_m S Rv_m^T: spectrum of X(l_c), and Alg. 7's factors
            TRY(orth(ctx, RSVD_F64, Mp, sw, j, sw, RSVD_F64, Qm, sw, Rm));
            TRY(small_svd(ctx, Rm, j, L2, R2, sg2));
            if (minvar) TRY(copy_small(ctx, sg2, k, SPEC + (size_t)slot * k));
            if (!woolfe) {
                TRY(gemm_small(ctx, LY, s, 1, R2, j, 1, s, k, j, CU + slot * cu_len));     // L_Y[:, :j] Rv_m[:, :k]
                TRY(gemm_small(ctx, Qm, 1, sw, L2, j, 1, sw, k, j, CV + slot * cv_len));   // Q_m L_m[:, :k]
                TRY(copy_small(ctx, sg2, k, SG + (size_t)slot * k));
            }
        }
        if (woolfe) {
            // X^ = M L_W[:, :j] = L_x S R_x^T
            TRY(gemm_small(ctx, Mp, sw, 1, LW, sw, 1, j, j, sw, Xh));
            TRY(small_svd(ctx, Xh, j, L2, R2, sg2));
            TRY(gemm_small(ctx, LY, s, 1, L2, j, 1, s, k, j, CU + slot * cu_len));         // L_Y[:, :j] L_x[:, :k]
            TRY(gemm_small(ctx, LW, sw, 1, R2, j, 1, sw, k, j, CV + slot * cv_len));       // L_W[:, :j] R_x[:, :k]
            TRY(copy_small(ctx, sg2, k, SG + (size_t)slot * k));
        }
    }
    if (!ctx.dry) {
        uint32_t* lc_word = ctx.status ? ctx.status + kLcWord : nullptr;
        if (minvar) {
            hipLaunchKernelGGL(minvar_select_kernel, dim3(1), dim3(256), 0, ctx.st, SPEC, k, p, CU, CV, SG, cu_len,
                               cv_len, CUf, CVf, SGf, lc_word);
        } else if (lc_word) {
            launch_op<set_int_kernel_op>(dim3(1), dim3(1), 0, ctx.st, {(int*)lc_word, lc_fix});
        }
        RSVD_LAUNCH_CHECK();
    }
    return finish(ctx, wdt, YT, ldy, s, m, RSVD_F64, QW, n, sw, n, CUf, k, CVf, k, SGf, k, wdt, out);
}

// ---------------------------------------------------------------------------
// Sect. 4.2: truncated eigendecompositions of the normal matrix J^T J.
// ---------------------------------------------------------------------------

// Alg. 3: `views` >= 1 alternating views of a started from Omega (a.n x s):
// view j multiplies by A (odd j) or A^T (even j) and orthonormalizes.  The
// co-range panel XT (s x a.n) starts as Omega^T, the range panel YT is
// s x a.m; the newest basis is the range basis in YT for odd `views` and the
// co-range basis in XT for even `views`.
rsvd_status alg3_views(Ctx& ctx, const Mat& a, int s, int views, uint64_t seed, void* XT, int64_t ldx, void* YT,
                       int64_t ldy) {
    const int wdt = work_dtype(a.dtype);
    CALL(launch_gaussian(seed, TAG_OMEGA, 0, s, a.n, 0, wdt, XT, ldx, ctx.st));
    for (int j = 1; j <= views; ++j) {
        if (j % 2 == 1) {
            TRY(range_view(ctx, a, XT, ldx, s, YT, ldy, 0));
            TRY(orth(ctx, wdt, YT, ldy, s, a.m, wdt, YT, ldy, nullptr));
        } else {
            TRY(corange_view(ctx, a, YT, ldy, s, XT, ldx, 0));
            TRY(orth(ctx, wdt, XT, ldx, s, a.n, wdt, XT, ldx, nullptr));
        }
    }
    return RSVD_OK;
}

// The co-range basis Q_r (n x s) of J after `views` views, from Alg. 3 on J
// (even `views`) or on J^T (odd `views`), left in the panel Pn (s x ldn);
// Pm (s x ldm) is scratch.  views = 0: Q_r = orth(Omega).
rsvd_status normal_basis(Ctx& ctx, const Mat& j, int s, int views, uint64_t seed, void* Pn, int64_t ldn, void* Pm,
                         int64_t ldm) {
    const int wdt = work_dtype(j.dtype);
    if (views == 0) {
        CALL(launch_gaussian(seed, TAG_OMEGA, 0, s, j.n, 0, wdt, Pn, ldn, ctx.st));
        return orth(ctx, wdt, Pn, ldn, s, j.n, wdt, Pn, ldn, nullptr);
    }
    if (views % 2 == 0) return alg3_views(ctx, j, s, views, seed, Pn, ldn, Pm, ldm);
    return alg3_views(ctx, transposed(j), s, views, seed, Pm, ldm, Pn, ldn);   // range basis of J^T
}

// nu = c sqrt(lambda_max), lambda_max the largest eigenvalue of a Gram
// (the square of the largest singular value of the panel).
__global__ void nystrom_nu_kernel(const double* __restrict__ lam_max, double c, double* __restrict__ nu) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *nu = c * sqrt(fmax(*lam_max, 0.0));
}

// out (FP64 panel) = Y + nu Q for panels Y, Q of the working type.
template <typename T>
__global__ void shift_panel_kernel(const T* __restrict__ Y, const T* __restrict__ Q, int64_t ld, int rows,
                                   int64_t len, const double* __restrict__ nu, double* __restrict__ out,
                                   int64_t ldo) {
    const double c = *nu;
    const int64_t total = (int64_t)rows * len;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / len, x = e % len;
        out[r * ldo + x] = (double)Y[r * ld + x] + c * (double)Q[r * ld + x];
    }
}

// Bs = (B + B^T) / 2 (s x s).
__global__ void symmetrize_kernel(const double* __restrict__ B, int s, double* __restrict__ Bs) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < s * s; e += gridDim.x * blockDim.x) {
        const int a = e / s, b = e % s;
        Bs[e] = 0.5 * (B[e] + B[b * s + a]);
    }
}

// lam2[i] = sig[i]^2 - nu (nu may be null), negative values set to 0.
__global__ void eig_from_sv_kernel(const double* __restrict__ sig, int k, const double* __restrict__ nu,
                                   double* __restrict__ lam2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const double v = sig[i] * sig[i] - (nu ? *nu : 0.0);
        lam2[i] = v > 0.0 ? v : 0.0;
    }
}

// Sign of each column of V (n x k): its entry of largest magnitude made positive.
rsvd_status sign_columns(Ctx& ctx, int wdt, void* V, int64_t n, int k) {
    double* pval = ctx.ar.take<double>((size_t)sign_chunks(n) * k);
    int64_t* pidx = ctx.ar.take<int64_t>((size_t)sign_chunks(n) * k);
    double* sgn = ctx.ar.take<double>((size_t)k);
    void* dummy = ctx.ar.take<char>((size_t)k * dtype_size(wdt));   // a one-row partner the sign is also applied to
    CALL(run_signs(wdt, V, n, dummy, 1, k, pval, pidx, sgn, ctx.st));
    return RSVD_OK;
}

enum { NORMAL_NYSTROM = 0, NORMAL_PINCHED = 1, NORMAL_SUBSPACE = 2 };

// Alg. 4, Alg. 5, or Alg. 2 by the J / J^T rule (Sect. 4.2.1), v >= 2 views of
// J (m x n): V (n x k, working type) and the k leading eigenvalues lam2 of
// J^T J.
rsvd_status alg_normal(Ctx& ctx, const Mat& j, int k, int p, int v, int method, const rsvd_opts& o, void* V,
                       double* lam2) {
    const int s = k + p;
    if (s > kMaxWidth) return RSVD_EUNSUPPORTED;
    const int wdt = work_dtype(j.dtype);
    const size_t we = dtype_size(wdt);
    const dim3 b256(256);
    if (method == NORMAL_SUBSPACE) {
        // even v: Alg. 2 on J, V = its right factor; odd v: Alg. 2 on J^T, V = its left factor
        const bool on_t = v % 2 == 1;
        void* Utmp = ctx.ar.take<char>((size_t)j.m * k * we);   // the factor on J's row side (m x k) either way
        double* sig = ctx.ar.take<double>((size_t)k);
        rsvd_out o2;
        o2.S = sig;
        o2.U = on_t ? V : Utmp;
        o2.V = on_t ? Utmp : V;
        TRY(alg_subspace(ctx, on_t ? transposed(j) : j, k, p, v, o, &o2));
        if (!ctx.dry) {
            hipLaunchKernelGGL(eig_from_sv_kernel, dim3(1), b256, 0, ctx.st, sig, k, (const double*)nullptr, lam2);
            RSVD_LAUNCH_CHECK();
        }
        return sign_columns(ctx, wdt, V, j.n, k);
    }
    const int64_t ldn = round_up(j.n, 4), ldm = round_up(j.m, 4);
    void* Pn = ctx.ar.take<char>((size_t)s * ldn * we);   // Q_r
    void* Pm = ctx.ar.take<char>((size_t)s * ldm * we);
    double* R = ctx.ar.take<double>((size_t)s * s);
    double* L = ctx.ar.take<double>((size_t)s * s);
    double* Rv = ctx.ar.take<double>((size_t)s * s);
    double* sig = ctx.ar.take<double>((size_t)s);
    if (method == NORMAL_PINCHED) {
        // Q_r from v - 1 views (Alg. 3 on J^T for even v, on J for odd v), B_c = J Q_r,
        // B_c^T B_c = R^T R = Rv S^2 Rv^T: V = Q_r Rv_k, lam2 = S^2
        TRY(normal_basis(ctx, j, s, v - 1, o.seed, Pn, ldn, Pm, ldm));
        TRY(range_view(ctx, j, Pn, ldn, s, Pm, ldm, 0));
        TRY(orth(ctx, wdt, Pm, ldm, s, j.m, wdt, Pm, ldm, R));
        TRY(small_svd(ctx, R, s, L, Rv, sig));
        CALL(run_lift(wdt, Pn, ldn, s, j.n, Rv, s, k, wdt, V, k, ctx.st));
        if (!ctx.dry) {
            hipLaunchKernelGGL(eig_from_sv_kernel, dim3(1), b256, 0, ctx.st, sig, k, (const double*)nullptr, lam2);
            RSVD_LAUNCH_CHECK();
        }
        return sign_columns(ctx, wdt, V, j.n, k);
    }
    // Alg. 4: Q_r from v - 2 views; Y_r = J^T (J Q_r); nu = 2.2e-16 ||Y_r||_2; Y~ = Y_r + nu Q_r;
    // B = Q_r^T Y~; C_L = chol((B + B^T)/2) = R^T; F^T = Y~ R^-1 = Q_F R_F, R_F = L S Rv^T;
    // V = Q_F L_k, lam2 = S^2 - nu
    void* Yr = ctx.ar.take<char>((size_t)s * ldn * we);
    double* Yt = ctx.ar.take<double>((size_t)s * j.n);
    double* G = ctx.ar.take<double>((size_t)s * s);
    double* B = ctx.ar.take<double>((size_t)s * s);
    double* Bs = ctx.ar.take<double>((size_t)s * s);
    double* Rinv = ctx.ar.take<double>((size_t)s * s);
    double* nu = ctx.ar.take<double>(1);
    double* gscr = chol_fits_lds(s) ? nullptr : ctx.ar.take<double>((size_t)round_up(s, 16) * (round_up(s, 16) + 1));
    double* scr = ctx.ar.take<double>(cross_scratch_doubles(s, s, j.n, 0, ctx.plan_cus));
    int* more = ctx.flags ? ctx.flags + (ctx.next_flag++ % 56) : nullptr;
    TRY(normal_basis(ctx, j, s, v - 2, o.seed, Pn, ldn, Pm, ldm));
    TRY(range_view(ctx, j, Pn, ldn, s, Pm, ldm, 0));
    TRY(corange_view(ctx, j, Pm, ldm, s, Yr, ldn, 0));
    CALL(run_cross(wdt, Yr, ldn, s, wdt, Yr, ldn, s, j.n, 1, G, scr, ctx.plan_cus, nullptr, ctx.st));
    TRY(small_svd(ctx, G, s, L, Rv, sig));                 // sig[0] = ||Y_r||_2^2
    if (!ctx.dry) {
        hipLaunchKernelGGL(nystrom_nu_kernel, dim3(1), dim3(64), 0, ctx.st, sig, 2.2e-16, nu);
        const int64_t total = (int64_t)s * j.n;
        const dim3 g((unsigned)std::min<int64_t>(ceil_div(total, 256), 8192));
        if (wdt == RSVD_F64)
            hipLaunchKernelGGL(shift_panel_kernel<double>, g, b256, 0, ctx.st, (const double*)Yr, (const double*)Pn,
                               ldn, s, j.n, (const double*)nu, Yt, j.n);
        else
            hipLaunchKernelGGL(shift_panel_kernel<float>, g, b256, 0, ctx.st, (const float*)Yr, (const float*)Pn,
                               ldn, s, j.n, (const double*)nu, Yt, j.n);
        RSVD_LAUNCH_CHECK();
    }
    CALL(run_cross(wdt, Pn, ldn, s, RSVD_F64, Yt, j.n, s, j.n, 0, B, scr, ctx.plan_cus, nullptr, ctx.st));
    if (!ctx.dry) {
        hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)ceil_div((int64_t)s * s, 256)), b256, 0, ctx.st, B, s,
                           Bs);
        launch_op<set_int_kernel_op>(dim3(1), dim3(1), 0, ctx.st, {more, 0});
        RSVD_LAUNCH_CHECK();
    }
    CALL(run_chol_inv(Bs, s, j.n, R, Rinv, gscr, ctx.status, more, nullptr, ctx.st));
    CALL(run_apply_rinv(RSVD_F64, Yt, j.n, s, j.n, Rinv, RSVD_F64, Yt, j.n, nullptr, ctx.st));   // F^T panel
    TRY(orth(ctx, RSVD_F64, Yt, j.n, s, j.n, RSVD_F64, Yt, j.n, R));
    TRY(small_svd(ctx, R, s, L, Rv, sig));
    CALL(run_lift(RSVD_F64, Yt, j.n, s, j.n, L, s, k, wdt, V, k, ctx.st));
    if (!ctx.dry) {
        hipLaunchKernelGGL(eig_from_sv_kernel, dim3(1), b256, 0, ctx.st, sig, k, (const double*)nu, lam2);
        RSVD_LAUNCH_CHECK();
    }
    return sign_columns(ctx, wdt, V, j.n, k);
}

// ---------------------------------------------------------------------------
// Alg. 9: generalized block Krylov (ALTERNATING)
// ---------------------------------------------------------------------------
rsvd_status alg_krylov_alternating(Ctx& ctx, const Mat& a, int k, int p, int v, const rsvd_opts& o, rsvd_out* out) {
    const int s = k + p;
    const int nblk = v % 2 == 0 ? v / 2 : (v - 1) / 2;
    const int sk = nblk * s;
    if (sk > kMaxWidth) return RSVD_EUNSUPPORTED;
    if ((int64_t)sk > std::min(a.m, a.n)) return RSVD_ESHAPE;
    const int wdt = work_dtype(a.dtype);
    const size_t we = dtype_size(wdt);
    void* XT = ctx.ar.take<char>((size_t)sk * a.n * we);   // K_r blocks (odd v) / current Q_r
    void* YT = ctx.ar.take<char>((size_t)sk * a.m * we);   // K_c blocks (even v) / current Q_c
    double* Rfin = ctx.ar.take<double>((size_t)sk * sk);
    double* L = ctx.ar.take<double>((size_t)sk * sk);
    double* Rv = ctx.ar.take<double>((size_t)sk * sk);
    double* sig = ctx.ar.take<double>((size_t)sk);
    // Q_r^0 = Omega: block 0 of the co-range panel
    CALL(launch_gaussian(o.seed, TAG_OMEGA, 0, s, a.n, 0, wdt, XT, a.n, ctx.st));
    int cblk = 0, rblk = 0;          // where the latest Q_c^j / Q_r^j live (block index)
    for (int j = 1; j <= v - 1; ++j) {
        const bool qr_it = j < v - 1;
        if (j % 2 == 1) {   // Q_c^j = [qr](A Q_r^{j-1})
            const int dst = v % 2 == 0 ? (j - 1) / 2 : 0;
            void* y = (char*)YT + (size_t)dst * s * a.m * we;
            const void* x = (const char*)XT + (size_t)rblk * s * a.n * we;
            TRY(range_view(ctx, a, x, a.n, s, y, a.m, 0));
            if (qr_it) TRY(orth(ctx, wdt, y, a.m, s, a.m, wdt, y, a.m, nullptr));
            cblk = dst;
        } else {            // Q_r^j = [qr](A^T Q_c^{j-1})
            const int dst = v % 2 == 1 ? (j - 2) / 2 : 0;
            void* x = (char*)XT + (size_t)dst * s * a.n * we;
            const void* y = (const char*)YT + (size_t)cblk * s * a.m * we;
            TRY(corange_view(ctx, a, y, a.m, s, x, a.n, 0));
            if (qr_it) TRY(orth(ctx, wdt, x, a.n, s, a.n, wdt, x, a.n, nullptr));
            rblk = dst;
        }
    }
    if (v % 2 == 0) {
        // [Q_c, ~] = qr(K_c); [Q_r, R_r] = qr(A^T Q_c); tsvd(R_r)
        TRY(orth(ctx, wdt, YT, a.m, sk, a.m, wdt, YT, a.m, nullptr));
        TRY(corange_view(ctx, a, YT, a.m, sk, XT, a.n, 0));
        TRY(orth(ctx, wdt, XT, a.n, sk, a.n, wdt, XT, a.n, Rfin));
        TRY(small_svd_rows(ctx, Rfin, sk, L, Rv, sig));
        return finish(ctx, wdt, YT, a.m, sk, a.m, wdt, XT, a.n, sk, a.n, Rv, sk, L, sk, sig, k, wdt, out);
    }
    // [Q_r, ~] = qr(K_r); [Q_c, R_c] = qr(A Q_r); tsvd(R_c)
    TRY(orth(ctx, wdt, XT, a.n, sk, a.n, wdt, XT, a.n, nullptr));
    TRY(range_view(ctx, a, XT, a.n, sk, YT, a.m, 0));
    TRY(orth(ctx, wdt, YT, a.m, sk, a.m, wdt, YT, a.m, Rfin));
    TRY(small_svd_rows(ctx, Rfin, sk, L, Rv, sig));
    return finish(ctx, wdt, YT, a.m, sk, a.m, wdt, XT, a.n, sk, a.n, L, sk, Rv, sk, sig, k, wdt, out);
}

// ---------------------------------------------------------------------------
// Sect. 7.3: row-wise accuracy-enhanced block Krylov (ROW_SWEEP)
// ---------------------------------------------------------------------------
// Coefficients of Q_c = Q_K C1 and B^T = Z C2 after the TSVD R = P S W^T of
// R_K.  With *need_svd == 0 (krylov_need_svd_kernel: no column can be cut) the
// SVD was skipped: C1 = I and C2 = R^-1, so Q_c = Q_K, with the same span as
// Q_K P; K is then well conditioned and the triangular inverse from the
// CholeskyQR is accurate.  Otherwise C1[a][c] = P[a][c] and C2[a][c] =
// W[a][c] / S_c for the kept columns (S_c >= tau S_0), else 0.  The SVD is
// then taken on the rows of R (Jacobi on R^T), so that W comes from the
// rotated columns and C2, which alone forms B, is accurate; P = R W / S carries
// rounding of order eps S_0 / S_c and enters only Q_c.  R^-1 P would lose the
// leading columns to cancellation when K is rank-deficient (the CholeskyQR
// inverse is then huge).
__global__ void krylov_coeff_kernel(const double* __restrict__ P, const double* __restrict__ Wr,
                                    const double* __restrict__ Rinv, const double* __restrict__ S, int n, double tau,
                                    const int* __restrict__ need_svd, double* __restrict__ C1,
                                    double* __restrict__ C2) {
    if (need_svd && *need_svd == 0) {
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
            C1[e] = (e / n == e % n) ? 1.0 : 0.0;
            C2[e] = Rinv[e];
        }
        return;
    }
    const double s0 = S[0];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
        const int c = e % n;
        const bool keep = s0 > 0.0 && S[c] >= tau * s0;
        C1[e] = keep ? P[e] : 0.0;
        C2[e] = keep ? Wr[e] / S[c] : 0.0;
    }
}

// *need_svd = 0 when the TSVD of R (n x n upper triangular, with its inverse
// Rinv) provably keeps every column: kappa_2(R) <= ||R||_F ||R^-1||_F < 1 / tau,
// so S_c >= tau S_0 for all c.  Else 1 (also for non-finite input).  One
// workgroup of 256 threads; fixed-order reduction.
__global__ void __launch_bounds__(256)
krylov_need_svd_kernel(const double* __restrict__ R, const double* __restrict__ Rinv, int n, double tau,
                       int* __restrict__ need_svd) {
    __shared__ double red[2][4];
    double nr = 0.0, ni = 0.0;
    int e = threadIdx.x;
    for (; e + 7 * (int)blockDim.x < n * n; e += 8 * blockDim.x) {   // eight loads ahead, same order
        double r[8], q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            r[u] = R[e + u * blockDim.x];
            q[u] = Rinv[e + u * blockDim.x];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            nr += r[u] * r[u];
            ni += q[u] * q[u];
        }
    }
    for (; e < n * n; e += blockDim.x) {
        nr += R[e] * R[e];
        ni += Rinv[e] * Rinv[e];
    }
    for (int off = 32; off > 0; off >>= 1) {
        nr += __shfl_xor(nr, off);
        ni += __shfl_xor(ni, off);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = nr;
        red[1][threadIdx.x >> 6] = ni;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double a = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        const double b = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        const bool safe = a > 0.0 && b > 0.0 && sqrt(a) * sqrt(b) * tau < 1.0;
        *need_svd = safe ? 0 : 1;
    }
}

// Flag slot and kernel launch of krylov_need_svd_kernel (nullptr: always take the SVD).
int* krylov_need_svd(Ctx& ctx, const double* R, const double* Rinv, int n, double tau) {
    if (ctx.dry || !ctx.flags) return nullptr;
    int* need = ctx.flags + (ctx.next_flag++ % 56);
    hipLaunchKernelGGL(krylov_need_svd_kernel, dim3(1), dim3(256), 0, ctx.st, R, Rinv, n, tau, need);
    if (hipPeekAtLastError() != hipSuccess) return nullptr;   // the SVD path then runs unconditionally
    return need;
}

rsvd_status alg_krylov_row_sweep(Ctx& ctx, const Mat& a, int k, int p, int v, const rsvd_opts& o, rsvd_out* out,
                                 bool swap_out) {
    const int s = k + p;
    const int sk = v * s;
    if (sk > kMaxWidth) return RSVD_EUNSUPPORTED;
    if ((int64_t)sk > std::min(a.m, a.n)) return RSVD_ESHAPE;
    const int wdt = work_dtype(a.dtype);
    const size_t we = dtype_size(wdt);
    const int64_t rows = o.block_rows > 0 ? o.block_rows : 1024;
    const double tau = o.trunc_tau > 0 ? o.trunc_tau : (wdt == RSVD_F64 ? 0x1p-40 : 0x1p-20);
    void* Xall = ctx.ar.take<char>((size_t)sk * a.n * we);   // [X_0; ...; X_{v-1}]  (co-range side)
    void* Kp = ctx.ar.take<char>((size_t)sk * a.m * we);     // [Y_1; ...; Y_v] = (A X)^T, then Q_c^T
    void* Zp = ctx.ar.take<char>((size_t)sk * a.n * we);     // [Z_1; ...; Z_v] = (A^T K)^T, then B, then Q_r^T
    double* Cx = ctx.ar.take<double>((size_t)sk * s);
    double* RK = ctx.ar.take<double>((size_t)sk * sk);
    double* RKinv = ctx.ar.take<double>((size_t)sk * sk);
    double* L = ctx.ar.take<double>((size_t)sk * sk);
    double* Rv = ctx.ar.take<double>((size_t)sk * sk);
    double* sig = ctx.ar.take<double>((size_t)sk);
    double* C1 = ctx.ar.take<double>((size_t)sk * sk);
    double* C2 = ctx.ar.take<double>((size_t)sk * sk);
    double* Rr = ctx.ar.take<double>((size_t)sk * sk);
    size_t scr_need = 0;  // the projection's cross product uses j*s rows for j = 1..v-1
    for (int j = 1; j < v; ++j) scr_need = std::max(scr_need, cross_scratch_doubles(j * s, s, a.n, 0, ctx.plan_cus));
    double* scr = ctx.ar.take<double>(scr_need);
    void* Kq = ctx.ar.take<char>((size_t)sk * a.m * we);     // Q_K^T
    void* Bt = ctx.ar.take<char>((size_t)sk * a.n * we);     // B = (A^T Q_c)^T panel

    // X_0 = orth(Omega)
    CALL(launch_gaussian(o.seed, TAG_OMEGA, 0, s, a.n, 0, wdt, Xall, a.n, ctx.st));
    TRY(orth(ctx, wdt, Xall, a.n, s, a.n, wdt, Xall, a.n, nullptr));
    for (int j = 1; j <= v; ++j) {
        const void* X = (const char*)Xall + (size_t)(j - 1) * s * a.n * we;
        char* Y = (char*)Kp + (size_t)(j - 1) * s * a.m * we;
        char* Z = (char*)Zp + (size_t)(j - 1) * s * a.n * we;
        // one sweep over row blocks: Y[b] = A_b X, Z += A_b^T Y[b]
        ViewTimer timer(ctx, 3);
        TRY(block_sweep(ctx, a, rows, X, a.n, s, Y, a.m, true, nullptr, 0, 0, Z, a.n));
        if (j < v) {
            // X_j = orth(Z_j projected twice off span[X_0..X_{j-1}])
            char* Xj = (char*)Xall + (size_t)j * s * a.n * we;
            const int sb = j * s;
            if (!ctx.dry && hipMemcpyAsync(Xj, Z, (size_t)s * a.n * we, hipMemcpyDeviceToDevice, ctx.st) != hipSuccess)
                return RSVD_EHIP;
            for (int rep = 0; rep < 2; ++rep) {
                CALL(run_cross(wdt, Xall, a.n, sb, wdt, Xj, a.n, s, a.n, 0, Cx, scr, ctx.plan_cus, nullptr, ctx.st));
                CALL(run_apply_coeff(wdt, Xall, a.n, sb, a.n, Cx, s, s, 0, -1.0, 1.0, wdt, Xj, a.n, nullptr, ctx.st));
            }
            TRY(orth(ctx, wdt, Xj, a.n, s, a.n, wdt, Xj, a.n, nullptr));
        }
    }
    // [Q_K, R_K] = qr(K); R_K = P S W^T; Q_c = Q_K P_r; B^T = A^T Q_c = Z W_r S_r^-1 (= Z R_K^-1 P_r)
    TRY(orth(ctx, wdt, Kp, a.m, sk, a.m, wdt, Kq, a.m, RK, RKinv));
    int* need = krylov_need_svd(ctx, RK, RKinv, sk, tau);
    TRY(small_svd_rows(ctx, RK, sk, L, Rv, sig, need));   // W from the columns of R_K^T: C2 = W / S
    if (!ctx.dry) {
        hipLaunchKernelGGL(krylov_coeff_kernel, dim3((unsigned)ceil_div((int64_t)sk * sk, 256)), dim3(256), 0, ctx.st,
                           L, Rv, RKinv, sig, sk, tau, need, C1, C2);
        RSVD_LAUNCH_CHECK();
    }
    CALL(run_apply_coeff(wdt, Kq, a.m, sk, a.m, C1, sk, sk, 0, 1.0, 0.0, wdt, Kp, a.m, nullptr, ctx.st));
    CALL(run_apply_coeff(wdt, Zp, a.n, sk, a.n, C2, sk, sk, 0, 1.0, 0.0, wdt, Bt, a.n, nullptr, ctx.st));
    // [Q_r, R_r] = qr(B^T); R_r = V^ Lam U^^T
    TRY(orth(ctx, wdt, Bt, a.n, sk, a.n, wdt, Bt, a.n, Rr));
    TRY(small_svd_rows(ctx, Rr, sk, L, Rv, sig));
    if (!swap_out) return finish(ctx, wdt, Kp, a.m, sk, a.m, wdt, Bt, a.n, sk, a.n, Rv, sk, L, sk, sig, k, wdt, out);
    // on A^T: U_A = V_{A^T}, V_A = U_{A^T}; the sign fix is applied to the new U
    return finish(ctx, wdt, Bt, a.n, sk, a.n, wdt, Kp, a.m, sk, a.m, L, sk, Rv, sk, sig, k, wdt, out);
}

// ---------------------------------------------------------------------------
// Row-sweep block Krylov with its loss terms and their adjoint.
//
// Forward (Sect. 7.3, as alg_krylov_row_sweep): X_0 = orth(Omega); sweep j
// forms Y_j = A X_{j-1} and Z_j = A^T Y_j; X_j = orth of Z_j projected
// twice off [X_0 .. X_{j-1}]; K = [Y_1 .. Y_v] = Q_K R_K, R_K = P S W^T,
// Q_c = Q_K P, B^T = A^T Q_c = Z W S^-1 = Q_r R_r, R_r = V^ Lam U^^T.
// Outputs: sigma = Lam[:k], E = ||A - Q_c Q_c^T A||_F^2 = ||A||_F^2 - sum Lam^2.
//
// Adjoint of L = sum_i dS_i sigma_i + dE E with Omega fixed (K at full
// numerical rank; a cut of the TSVD of R_K sets RSVD_FLAG_TRUNCATED):
//   direct term   Q_c U~_k diag(dS) V~_k^T + 2 dE (A - Q_c B),  V~ = Q_r V^, U~ = U^;
//   basis term    Gq = A V~_k diag(dS) U~_k^T - 2 dE A B^T, K_bar = (I - Q_c Q_c^T) Gq S^-1 W^T
//                 (F depends on range(K) only, and K = Q_c S W^T);
//   sweeps j = v..1: for j < v, X_bar_j -> W_bar = (X_bar - X sym(X^T X_bar)) R_j^-T
//                 (QR adjoint with no R gradient), Z_bar = (I - C C^T) W_bar,
//                 C_bar = -(W_bar Z^T C + Z W_bar^T C) onto X_bar_0..j-1, G += Y_j Z_bar^T,
//                 Y_bar_j += A Z_bar; then G += Y_bar_j X_{j-1}^T, X_bar_{j-1} += A^T Y_bar_j.
// All thin algebra runs on panels; the dense G = 2 dE A + sum L^T R is one
// matrix-core pass over the output.
// ---------------------------------------------------------------------------
constexpr uint32_t RSVD_FLAG_TRUNCATED = 8u;

// Small-factor record of the row-sweep gradient: the SVDs of R_K (P_K, W_K,
// S_K) and of R_r (V^, U^, lambda), 4 sk^2 + 2 sk doubles.
size_t grad_kept_doubles(int sk) { return 4 * (size_t)sk * sk + 2 * (size_t)sk; }

// small_svd, or its result copied from / to a kept record (keep_mode 2 / 1).
rsvd_status small_svd_kept(Ctx& ctx, const double* M, int s, double* L, double* Rv, double* sig, double* kept,
                           int keep_mode, bool rows = false, const int* enable = nullptr) {
    const size_t ss = (size_t)s * s;
    if (keep_mode == 2) {
        CALL(run_copy_f64(kept, L, (int64_t)ss, ctx.st));
        CALL(run_copy_f64(kept + ss, Rv, (int64_t)ss, ctx.st));
        CALL(run_copy_f64(kept + 2 * ss, sig, s, ctx.st));
        return RSVD_OK;
    }
    TRY(rows ? small_svd_rows(ctx, M, s, L, Rv, sig, enable) : small_svd(ctx, M, s, L, Rv, sig, enable));
    if (keep_mode == 1) {
        CALL(run_copy_f64(L, kept, (int64_t)ss, ctx.st));
        CALL(run_copy_f64(Rv, kept + ss, (int64_t)ss, ctx.st));
        CALL(run_copy_f64(sig, kept + 2 * ss, s, ctx.st));
    }
    return RSVD_OK;
}

rsvd_status alg_row_sweep_grad(Ctx& ctx, const Mat& a, int k, int p, int v, const rsvd_opts& o, rsvd_out* out,
                               double* E_out, const double* dS, double dE, void* G, int64_t ldg,
                               double* kept = nullptr, int keep_mode = 0) {
    const int s = k + p;
    const int sk = v * s;
    if (sk > kMaxWidth) return RSVD_EUNSUPPORTED;
    if ((int64_t)sk > std::min(a.m, a.n)) return RSVD_ESHAPE;
    const int wdt = work_dtype(a.dtype);
    const size_t we = dtype_size(wdt);
    const int64_t m = a.m, n = a.n;
    const int64_t rows = o.block_rows > 0 ? o.block_rows : 1024;
    const double tau = o.trunc_tau > 0 ? o.trunc_tau : (wdt == RSVD_F64 ? 0x1p-40 : 0x1p-20);
    auto panel = [&](int r, int64_t len) { return ctx.ar.take<char>((size_t)r * len * we); };
    char* Xall = panel(sk, n);     // X_0 .. X_{v-1}
    char* Kp = panel(sk, m);       // K = [Y_1 .. Y_v]
    char* Zp = panel(sk, n);       // [Z_1 .. Z_v]
    char* Kq = panel(sk, m);       // Q_K
    char* Qc = panel(sk, m);       // Q_c
    char* Bt = panel(sk, n);       // B = (A^T Q_c)^T panel
    char* Qr = panel(sk, n);       // Q_r
    double* Rinv = ctx.ar.take<double>((size_t)std::max(1, v - 1) * s * s);  // R_j^-1, j = 1..v-1
    double* Cx = ctx.ar.take<double>((size_t)sk * s);
    double* RK = ctx.ar.take<double>((size_t)sk * sk);
    double* RKinv = ctx.ar.take<double>((size_t)sk * sk);
    double* PK = ctx.ar.take<double>((size_t)sk * sk);
    double* WK = ctx.ar.take<double>((size_t)sk * sk);
    double* SK = ctx.ar.take<double>((size_t)sk);
    double* C1 = ctx.ar.take<double>((size_t)sk * sk);
    double* C2 = ctx.ar.take<double>((size_t)sk * sk);
    double* Rr = ctx.ar.take<double>((size_t)sk * sk);
    double* Vh = ctx.ar.take<double>((size_t)sk * sk);
    double* Uh = ctx.ar.take<double>((size_t)sk * sk);
    double* lam = ctx.ar.take<double>((size_t)sk);
    double* fpart = ctx.ar.take<double>((size_t)frob_parts());
    double* Eloc = ctx.ar.take<double>(1);
    size_t scr_need = cross_scratch_doubles(sk, sk, m, 0, ctx.plan_cus);
    for (int j = 1; j < v; ++j) {
        scr_need = std::max(scr_need, cross_scratch_doubles(j * s, s, n, 0, ctx.plan_cus));
        scr_need = std::max(scr_need, cross_scratch_doubles(s, j * s, n, 0, ctx.plan_cus));
    }
    scr_need = std::max(scr_need, cross_scratch_doubles(s, s, n, 0, ctx.plan_cus));
    double* scr = ctx.ar.take<double>(scr_need);

    // ---------------- forward
    CALL(launch_gaussian(o.seed, TAG_OMEGA, 0, s, n, 0, wdt, Xall, n, ctx.st));
    TRY(orth(ctx, wdt, Xall, n, s, n, wdt, Xall, n, nullptr));
    for (int j = 1; j <= v; ++j) {
        const char* X = Xall + (size_t)(j - 1) * s * n * we;
        char* Y = Kp + (size_t)(j - 1) * s * m * we;
        char* Z = Zp + (size_t)(j - 1) * s * n * we;
        ViewTimer timer(ctx, 3);
        TRY(block_sweep(ctx, a, rows, X, n, s, Y, m, true, nullptr, 0, 0, Z, n));
        if (j < v) {
            char* Xj = Xall + (size_t)j * s * n * we;
            const int sb = j * s;
            CALL(run_copy_panel(wdt, Z, n, Xj, n, s, n, nullptr, ctx.st));
            for (int rep = 0; rep < 2; ++rep) {
                CALL(run_cross(wdt, Xall, n, sb, wdt, Xj, n, s, n, 0, Cx, scr, ctx.plan_cus, nullptr, ctx.st));
                CALL(run_apply_coeff(wdt, Xall, n, sb, n, Cx, s, s, 0, -1.0, 1.0, wdt, Xj, n, nullptr, ctx.st));
            }
            TRY(orth(ctx, wdt, Xj, n, s, n, wdt, Xj, n, nullptr, Rinv + (size_t)(j - 1) * s * s));
        }
    }
    TRY(orth(ctx, wdt, Kp, m, sk, m, wdt, Kq, m, RK, RKinv));
    const size_t half = grad_kept_doubles(sk) / 2;   // the R_K record, then the R_r record
    int* need = krylov_need_svd(ctx, RK, RKinv, sk, tau);
    TRY(small_svd_kept(ctx, RK, sk, PK, WK, SK, kept, keep_mode, true, need));
    if (!ctx.dry) {
        hipLaunchKernelGGL(krylov_coeff_kernel, dim3((unsigned)ceil_div((int64_t)sk * sk, 256)), dim3(256), 0, ctx.st,
                           PK, WK, RKinv, SK, sk, tau, need, C1, C2);
        RSVD_LAUNCH_CHECK();
    }
    CALL(run_rank_check(SK, sk, tau, ctx.status, RSVD_FLAG_TRUNCATED, ctx.st, need));
    CALL(run_apply_coeff(wdt, Kq, m, sk, m, C1, sk, sk, 0, 1.0, 0.0, wdt, Qc, m, nullptr, ctx.st));
    CALL(run_apply_coeff(wdt, Zp, n, sk, n, C2, sk, sk, 0, 1.0, 0.0, wdt, Bt, n, nullptr, ctx.st));
    TRY(orth(ctx, wdt, Bt, n, sk, n, wdt, Qr, n, Rr));
    TRY(small_svd_kept(ctx, Rr, sk, Vh, Uh, lam, kept ? kept + half : nullptr, keep_mode, true));
    CALL(run_frob_sq(a.dtype, a.data, a.ld, m, n, fpart, lam, sk, E_out ? E_out : Eloc, ctx.st));
    if (out) TRY(finish(ctx, wdt, Qc, m, sk, m, wdt, Qr, n, sk, n, Uh, sk, Vh, sk, lam, k, wdt, out));
    if (!G) return RSVD_OK;

    // ---------------- adjoint
    const int q1 = k + sk;
    char* T1 = panel(q1, n);          // [V~_k ; B] panels
    char* AT1 = panel(q1, m);         // A [V~_k, B^T] as a panel
    char* Mp = panel(sk, m);          // Gq S^-1 W^T, then K_bar = [Y_bar_1 .. Y_bar_v]
    char* Xbar = panel(sk, n);
    char* Wb = panel(s, n);
    char* Tmp = panel(s, n);
    char* Zbar = panel(std::max(1, v - 1) * s, n);   // Z_bar_1 .. Z_bar_{v-1}
    char* Uk = panel(k, m);           // (Q_c U~_k diag(dS))^T
    double* Ct = ctx.ar.take<double>((size_t)q1 * sk);
    double* D = ctx.ar.take<double>((size_t)sk * sk);
    double* N = ctx.ar.take<double>((size_t)s * s);
    double* Ssym = ctx.ar.take<double>((size_t)s * s);
    double* RinvT = ctx.ar.take<double>((size_t)s * s);
    double* E1 = ctx.ar.take<double>((size_t)sk * s);
    double* F1 = ctx.ar.take<double>((size_t)s * sk);
    double* F2 = ctx.ar.take<double>((size_t)s * sk);
    double* Ud = ctx.ar.take<double>((size_t)sk * k);
    double* zeros = dS ? nullptr : ctx.ar.take<double>((size_t)k);
    if (!dS) {
        CALL(run_fill_zero(RSVD_F64, zeros, k, ctx.st));
        dS = zeros;
    }
    // A [V~_k, B^T]: V~_k panel = V^_k^T Q_r-panel, then B^T's panel
    CALL(run_apply_coeff(wdt, Qr, n, sk, n, Vh, sk, k, 0, 1.0, 0.0, wdt, T1, n, nullptr, ctx.st));
    CALL(run_copy_panel(wdt, Bt, n, T1 + (size_t)k * n * we, n, sk, n, nullptr, ctx.st));
    TRY(range_view(ctx, a, T1, n, q1, AT1, m, 0));
    // M = Gq S^-1 W^T, K_bar = M - Q_c (Q_c^T M)
    CALL(run_grad_coeff(Uh, dS, dE, k, C2, sk, Ct, ctx.st));
    CALL(run_apply_coeff(wdt, AT1, m, q1, m, Ct, sk, sk, 0, 1.0, 0.0, wdt, Mp, m, nullptr, ctx.st));
    CALL(run_cross(wdt, Qc, m, sk, wdt, Mp, m, sk, m, 0, D, scr, ctx.plan_cus, nullptr, ctx.st));
    CALL(run_apply_coeff(wdt, Qc, m, sk, m, D, sk, sk, 0, -1.0, 1.0, wdt, Mp, m, nullptr, ctx.st));
    CALL(run_fill_zero(wdt, Xbar, (int64_t)sk * n, ctx.st));
    for (int j = v; j >= 1; --j) {
        char* Ybar = Mp + (size_t)(j - 1) * s * m * we;
        if (j < v) {
            const int sb = j * s;
            const char* Xj = Xall + (size_t)j * s * n * we;
            char* Xbj = Xbar + (size_t)j * s * n * we;
            const char* Zj = Zp + (size_t)(j - 1) * s * n * we;
            char* Zbj = Zbar + (size_t)(j - 1) * s * n * we;
            // W_bar^T = R_j^-1 (X_bar - X sym(X^T X_bar))^T
            CALL(run_cross(wdt, Xj, n, s, wdt, Xbj, n, s, n, 0, N, scr, ctx.plan_cus, nullptr, ctx.st));
            CALL(run_sym_upper(N, s, Ssym, ctx.st));
            CALL(run_copy_panel(wdt, Xbj, n, Tmp, n, s, n, nullptr, ctx.st));
            CALL(run_apply_coeff(wdt, Xj, n, s, n, Ssym, s, s, 0, -1.0, 1.0, wdt, Tmp, n, nullptr, ctx.st));
            CALL(run_transpose_f64(Rinv + (size_t)(j - 1) * s * s, s, RinvT, ctx.st));
            CALL(run_apply_coeff(wdt, Tmp, n, s, n, RinvT, s, s, 0, 1.0, 0.0, wdt, Wb, n, nullptr, ctx.st));
            // Z_bar = (I - C C^T) W_bar with C = [X_0 .. X_{j-1}]
            CALL(run_cross(wdt, Xall, n, sb, wdt, Wb, n, s, n, 0, E1, scr, ctx.plan_cus, nullptr, ctx.st));
            CALL(run_copy_panel(wdt, Wb, n, Zbj, n, s, n, nullptr, ctx.st));
            CALL(run_apply_coeff(wdt, Xall, n, sb, n, E1, s, s, 0, -1.0, 1.0, wdt, Zbj, n, nullptr, ctx.st));
            // C_bar = -(W_bar (Z^T C) + Z (W_bar^T C)) onto X_bar_0 .. X_bar_{j-1}
            CALL(run_cross(wdt, Zj, n, s, wdt, Xall, n, sb, n, 0, F1, scr, ctx.plan_cus, nullptr, ctx.st));
            CALL(run_cross(wdt, Wb, n, s, wdt, Xall, n, sb, n, 0, F2, scr, ctx.plan_cus, nullptr, ctx.st));
            CALL(run_apply_coeff(wdt, Wb, n, s, n, F1, sb, sb, 0, -1.0, 1.0, wdt, Xbar, n, nullptr, ctx.st));
            CALL(run_apply_coeff(wdt, Zj, n, s, n, F2, sb, sb, 0, -1.0, 1.0, wdt, Xbar, n, nullptr, ctx.st));
            // Z_j = A^T Y_j: Y_bar_j += A Z_bar_j
            TRY(range_view(ctx, a, Zbj, n, s, Ybar, m, 1));
        }
        // Y_j = A X_{j-1}: X_bar_{j-1} += A^T Y_bar_j
        TRY(corange_view(ctx, a, Ybar, m, s, Xbar + (size_t)(j - 1) * s * n * we, n, 1));
    }
    // G = 2 dE A + U_k diag(dS) V~_k^T - 2 dE Q_c B + sum_j Y_bar_j X_{j-1}^T + sum_{j<v} Y_j Z_bar_j^T
    CALL(run_scale_cols(Uh, sk, sk, k, dS, Ud, ctx.st));
    CALL(run_apply_coeff(wdt, Qc, m, sk, m, Ud, k, k, 0, 1.0, 0.0, wdt, Uk, m, nullptr, ctx.st));
    if (!ctx.dry) {
        const char* Ls[4] = {Uk, Qc, Mp, Kp};
        const char* Rs[4] = {T1, Bt, Xall, Zbar};
        const int rws[4] = {k, sk, sk, (v - 1) * s};
        const double scl[4] = {1.0, -2.0 * dE, 1.0, 1.0};
        const int cnt = v > 1 ? 4 : 3;
        if (wdt == RSVD_F64) {
            OuterSegs<double> sg{};
            for (int i = 0; i < cnt; ++i) {
                sg.L[i] = (const double*)Ls[i];
                sg.R[i] = (const double*)Rs[i];
                sg.ldl[i] = m;
                sg.ldr[i] = n;
                sg.rows[i] = rws[i];
                sg.scale[i] = scl[i];
            }
            sg.count = cnt;
            TRY(run_outer_update_f64((const double*)a.data, a.ld, 2.0 * dE, m, n, sg, (double*)G, ldg, ctx.st));
        } else {
            OuterSegs<float> sg{};
            for (int i = 0; i < cnt; ++i) {
                sg.L[i] = (const float*)Ls[i];
                sg.R[i] = (const float*)Rs[i];
                sg.ldl[i] = m;
                sg.ldr[i] = n;
                sg.rows[i] = rws[i];
                sg.scale[i] = scl[i];
            }
            sg.count = cnt;
            TRY(run_outer_update_f32((const float*)a.data, a.ld, 2.0 * dE, m, n, sg, (float*)G, ldg, ctx.st));
        }
    }
    return RSVD_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing (rsvd_subspace_noalloc).
// One array per GPU, held from the library's load to the end of the process;
// every call on a GPU shares it.  Host code uses only the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocDevices] = {};

// The current device's address of `scratch`, looked up once per device.
rsvd_status noalloc_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return RSVD_EHIP;
    if (dev < 0 || dev >= kNoAllocDevices) return RSVD_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RSVD_EHIP;
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return RSVD_OK;
}

// ---------------------------------------------------------------------------
// call frame shared by the entry points
// ---------------------------------------------------------------------------
enum { ALG_SUB = 0, ALG_ONE = 1, ALG_KRY = 2 };

rsvd_status dispatch(Ctx& ctx, int algo, const Mat& a, int k, int p, int v, const rsvd_opts& o, rsvd_out* out) {
    if (algo == ALG_SUB) return alg_subspace(ctx, a, k, p, v, o, out);
    if (algo == ALG_ONE) return alg_single_pass(ctx, a, k, p, o, out);
    if (o.krylov_mode == RSVD_KRYLOV_ALTERNATING) return alg_krylov_alternating(ctx, a, k, p, v, o, out);
    if (o.krylov_mode == RSVD_KRYLOV_ROW_SWEEP) return alg_krylov_row_sweep(ctx, a, k, p, v, o, out, false);
    return alg_krylov_row_sweep(ctx, transposed(a), k, p, v, o, out, true);
}

rsvd_status check_algo(const rsvd_mat* A, int k, int p, int v, int algo, const rsvd_opts& o) {
    if (low_precision(A->dtype) && algo != ALG_SUB) return RSVD_EUNSUPPORTED;
    if (algo == ALG_SUB && v < 2) return RSVD_EINVAL;
    if (algo == ALG_ONE && v != 1) return RSVD_EINVAL;
    if (algo == ALG_KRY) {
        if (o.krylov_mode == RSVD_KRYLOV_ALTERNATING && v < 2) return RSVD_EINVAL;
        if (o.krylov_mode != RSVD_KRYLOV_ALTERNATING && v < 1) return RSVD_EINVAL;
        if (o.krylov_mode != RSVD_KRYLOV_ALTERNATING && (int64_t)v * (k + p) > std::min(A->m, A->n))
            return RSVD_ESHAPE;
    }
    if (o.one_view_method != RSVD_ONE_VIEW_TROPP && o.one_view_method != RSVD_ONE_VIEW_WOOLFE) return RSVD_EINVAL;
    if (o.lc_rule < RSVD_LC_FULL || o.lc_rule > RSVD_LC_MINVAR) return RSVD_EINVAL;
    if (o.lc_rule == RSVD_LC_FIXED && (o.lc < 0 || o.lc > p)) return RSVD_EINVAL;
    if (o.lc_rule == RSVD_LC_RATIO && !(o.lc_alpha >= 0.0 && o.lc_alpha <= 1.0)) return RSVD_EINVAL;
    if (o.core_kind != RSVD_CORE_GAUSSIAN && o.core_kind != RSVD_CORE_SRFT) return RSVD_EINVAL;
    const bool one_view_opts = o.one_view_method != RSVD_ONE_VIEW_TROPP || o.lc_rule != RSVD_LC_FULL;
    if (one_view_opts && (algo != ALG_ONE || o.core_rows > 0)) return RSVD_EINVAL;
    if (o.core_kind != RSVD_CORE_GAUSSIAN && (algo != ALG_ONE || o.core_rows == 0)) return RSVD_EINVAL;
    if (o.core_rows != 0 && algo != ALG_ONE) return RSVD_EINVAL;
    if (algo == ALG_ONE && o.core_rows > 0) {   // extended sketch: l1 = l2, s <= s_c <= min(m, n)
        if (o.psi_rows != 0 && o.psi_rows != k + p) return RSVD_EINVAL;
        if (o.core_rows < k + p || o.core_rows > std::min(A->m, A->n)) return RSVD_ESHAPE;
        if (o.core_rows > 4 * kMaxWidth) return RSVD_EUNSUPPORTED;
        if (o.core_kind == RSVD_CORE_SRFT && std::max(A->m, A->n) >= ((int64_t)1 << 31)) return RSVD_EUNSUPPORTED;
    } else if (algo == ALG_ONE) {
        const int64_t sw = o.psi_rows ? o.psi_rows : 2 * (int64_t)(k + p) + 1;
        if (sw < k + p || sw > A->m) return RSVD_ESHAPE;
        if (o.one_view_method == RSVD_ONE_VIEW_WOOLFE && sw > A->n) return RSVD_ESHAPE;
        if (one_view_opts && sw > kMaxWidth) return RSVD_EUNSUPPORTED;
    }
    return RSVD_OK;
}

size_t plan_bytes(const rsvd_mat* A, int k, int p, int v, int algo, const rsvd_opts& o, rsvd_status* err) {
    Ctx ctx{true, nullptr, Arena{nullptr}};
    ctx.f32_mode = o.f32_mode;
    rsvd_out dummy{nullptr, nullptr, nullptr};
    *err = dispatch(ctx, algo, make_mat(A), k, p, v, o, &dummy);
    return ctx.ar.off;
}

rsvd_status run_call(int algo, const rsvd_mat* A, int k, int p, int v, const rsvd_opts* op, rsvd_out* out, void* ws,
                     size_t ws_bytes, hipStream_t st) {
    rsvd_status e = check_common(A, k, p, op, out, true);
    if (e != RSVD_OK) return e;
    const rsvd_opts o = opts_or_default(op);
    e = check_algo(A, k, p, v, algo, o);
    if (e != RSVD_OK) return e;
    rsvd_status perr;
    const size_t need = plan_bytes(A, k, p, v, algo, o, &perr);
    if (perr != RSVD_OK) return perr;
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return RSVD_EWORKSPACE;
    Ctx ctx{false, st, Arena{(char*)ws}};
    ctx.status = (uint32_t*)ws;
    ctx.flags = (int*)((char*)ws + 32);
    ctx.trace = o.trace;
    ctx.f32_mode = o.f32_mode;
    ctx.sync_spins = o.sync_spins;
    if (ctx.trace) ctx.trace->used = 0;
    launch_op<clear_header_kernel_op>(dim3(1), dim3(64), 0, st, {(uint32_t*)ws});
    RSVD_LAUNCH_CHECK();
    return dispatch(ctx, algo, make_mat(A), k, p, v, o, out);
}

__global__ void philox_words_kernel(const uint32_t* __restrict__ ctr, int64_t count, uint32_t k0, uint32_t k1,
                                    uint32_t* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c[4] = {ctr[e], ctr[count + e], ctr[2 * count + e], ctr[3 * count + e]};
        philox4x32_10(c, k0, k1);
        for (int w = 0; w < 4; ++w) out[w * count + e] = c[w];
    }
}

// ---------------------------------------------------------------------------
// Sect. 6.1: one-view sketches of A = sum_i H_i, updated by linear updates.
// The workspace holds Omega^T (s x n), Psi (s_w x m), Y^T (s x m), W (s_w x n)
// and, for the post-processing, a copy of Y^T and the one-view arena.
// ---------------------------------------------------------------------------
struct StreamBufs {
    void* OmT;
    void* Psi;
    void* YT;
    void* W;
    void* Yc;
};

StreamBufs stream_bufs(Ctx& ctx, int64_t m, int64_t n, int s, int sw, size_t we) {
    StreamBufs b;
    b.OmT = ctx.ar.take<char>((size_t)s * n * we);
    b.Psi = ctx.ar.take<char>((size_t)sw * m * we);
    b.YT = ctx.ar.take<char>((size_t)s * m * we);
    b.W = ctx.ar.take<char>((size_t)sw * n * we);
    b.Yc = ctx.ar.take<char>((size_t)s * m * we);
    return b;
}

template <typename T>
__global__ void zero_fill_kernel(T* __restrict__ p, int64_t count) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = T(0);
}

// One sparse update sum_e v_e e_{r_e} e_{c_e}^T: Y[r, :] += v Omega[c, :] and
// W[:, c] += v Psi[:, r] for every entry, as FP atomic adds on the panels
// (repeated coordinates add up; the order of the adds is not fixed).  An
// entry outside A is skipped and sets RSVD_FLAG_BAD_ENTRY.  Thread t of the
// grid-stride loop takes (entry, thin index) pairs.
template <typename T>
__global__ void stream_entries_kernel(int64_t nnz, const int64_t* __restrict__ rows, const int64_t* __restrict__ cols,
                                      const T* __restrict__ vals, int64_t m, int64_t n, int s, int sw,
                                      const T* __restrict__ OmT, const T* __restrict__ Psi, T* __restrict__ YT,
                                      T* __restrict__ W, uint32_t* __restrict__ status) {
    const int width = s + sw;
    const int64_t total = nnz * width;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / width;
        const int j = (int)(t % width);
        const int64_t r = rows[e], c = cols[e];
        if (r < 0 || r >= m || c < 0 || c >= n) {
            if (j == 0) rsvd_flag(status, RSVD_FLAG_BAD_ENTRY);
            continue;
        }
        const T v = vals[e];
        if (j < s) unsafeAtomicAdd(YT + (int64_t)j * m + r, v * OmT[(int64_t)j * n + c]);
        else unsafeAtomicAdd(W + (int64_t)(j - s) * n + c, v * Psi[(int64_t)(j - s) * m + r]);
    }
}

// ---------------------------------------------------------------------------
// Batches: the per-matrix driver of Alg. 2 is recorded once per matrix
// (launch_op hands every launch to the recorder instead of a stream); the
// i-th launch of every matrix then runs as one batched launch per kernel,
// blockIdx.z selecting the matrix, in the order i = 0, 1, ...  A matrix's
// launches keep their order, and matrices are independent, so the batch
// computes exactly what the per-matrix calls compute.
// ---------------------------------------------------------------------------
struct RecordedLaunch {
    const void* batched_fn;
    const void* single_fn;
    std::vector<char> job;
    dim3 grid;
    unsigned threads;
    size_t shmem;
    int phase, sub;      // driver step and launch within the step
};

struct MatrixRecorder : LaunchRecorder {
    std::vector<RecordedLaunch> seq;
    int cur_phase = 0, cur_sub = 0;
    void phase() override {
        ++cur_phase;
        cur_sub = 0;
    }
    void add(const void* batched_fn, const void* single_fn, const void* job, size_t job_size, dim3 grid,
             unsigned threads, size_t shmem) override {
        RecordedLaunch r;
        r.batched_fn = batched_fn;
        r.single_fn = single_fn;
        r.job.assign((const char*)job, (const char*)job + job_size);
        r.grid = grid;
        r.threads = threads;
        r.shmem = shmem;
        r.phase = cur_phase;
        r.sub = cur_sub++;
        seq.push_back(std::move(r));
    }
};

struct RecorderScope {
    explicit RecorderScope(LaunchRecorder* r) { launch_recorder() = r; }
    ~RecorderScope() { launch_recorder() = nullptr; }
};

}  // namespace

struct rsvd_stream {
    int64_t m = 0, n = 0;
    int k = 0, p = 0, sw = 0, wdt = RSVD_F64;
    rsvd_opts o;
    size_t ws_bytes = 0;
    char* ws = nullptr;
};

struct rsvd_batch_plan {
    struct Group {
        const void* fn;
        unsigned gx, gy, gz, threads;
        size_t shmem;
        size_t table_off;   // offset of the job table inside the workspace
        size_t job_size;
    };
    int nb = 0, p = 0, v = 0;
    std::vector<rsvd_mat> mats;
    std::vector<int> ks;
    std::vector<rsvd_out> outs;
    rsvd_opts o;
    rsvd_batch_tuning tuning;
    std::vector<size_t> arena_off;   // start of each matrix's workspace
    size_t tables_off = 0, ws_bytes = 0;
    std::vector<Group> groups;
    std::vector<char> tables;        // host copy of every job table (uploaded by bind)
    void* ws = nullptr;
};

namespace {

// Records every matrix against workspace base `ws` and builds the groups.
rsvd_status batch_record(rsvd_batch_plan& P, char* ws) {
    P.groups.clear();
    P.tables.clear();
    std::vector<MatrixRecorder> recs(P.nb);
    for (int b = 0; b < P.nb; ++b) {
        RecorderScope scope(&recs[b]);
        Ctx ctx{false, nullptr, Arena{ws + P.arena_off[b]}};
        ctx.status = (uint32_t*)(ws + P.arena_off[b]);
        ctx.flags = (int*)(ws + P.arena_off[b] + 32);
        ctx.plan_cus = P.tuning.plan_cus;
        ctx.view_mr = P.tuning.view_mr;
        launch_phase();
        launch_op<clear_header_kernel_op>(dim3(1), dim3(64), 0, nullptr, {(uint32_t*)ctx.status});   // recorded
        rsvd_out out = P.outs[b];
        TRY(dispatch(ctx, ALG_SUB, make_mat(&P.mats[b]), P.ks[b], P.p, P.v, P.o, &out));
    }
    // group by (driver step, launch within the step), then by kernel; every
    // matrix's launches keep their order since (phase, sub) increases along it
    std::map<std::pair<int, int>, std::vector<const RecordedLaunch*>> bykey;
    for (auto& r : recs)
        for (const RecordedLaunch& L : r.seq) bykey[{L.phase, L.sub}].push_back(&L);
    size_t off = 0;
    for (auto& kv : bykey) {
        std::map<const void*, std::vector<const RecordedLaunch*>> byfn;
        std::vector<const void*> order;
        for (const RecordedLaunch* L : kv.second) {
            if (!byfn.count(L->batched_fn)) order.push_back(L->batched_fn);
            byfn[L->batched_fn].push_back(L);
        }
        for (const void* fn : order) {
            const auto& v = byfn[fn];
            rsvd_batch_plan::Group g;
            g.fn = fn;
            g.gx = g.gy = 1;
            g.gz = (unsigned)v.size();
            g.threads = 0;
            g.shmem = 0;
            g.job_size = v[0]->job.size();
            off = (size_t)round_up((int64_t)off, 256);
            g.table_off = off;
            P.tables.resize(off + g.job_size * v.size());
            for (size_t q = 0; q < v.size(); ++q) {
                g.gx = std::max(g.gx, v[q]->grid.x);
                g.gy = std::max(g.gy, v[q]->grid.y);
                g.threads = std::max(g.threads, v[q]->threads);
                g.shmem = std::max(g.shmem, v[q]->shmem);
                std::memcpy(P.tables.data() + off + q * g.job_size, v[q]->job.data(), g.job_size);
            }
            off += g.job_size * v.size();
            P.groups.push_back(g);
        }
    }
    return RSVD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void rsvd_default_opts(rsvd_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->krylov_mode = RSVD_KRYLOV_ALTERNATING;
    o->block_rows = 1024;
    o->f32_mode = RSVD_F32_MFMA;
}

const char* rsvd_status_string(rsvd_status s) {
    switch (s) {
        case RSVD_OK: return "ok";
        case RSVD_EINVAL: return "invalid argument";
        case RSVD_ESHAPE: return "invalid shape";
        case RSVD_EWORKSPACE: return "workspace too small or misaligned";
        case RSVD_EBREAKDOWN: return "numerical breakdown (non-finite result)";
        case RSVD_EHIP: return "HIP runtime error";
        case RSVD_EUNSUPPORTED: return "unsupported by this build";
    }
    return "unknown status";
}

size_t rsvd_workspace_bytes(const rsvd_mat* A, int k, int p, int v, int algo, const rsvd_opts* op) {
    if (check_common(A, k, p, op, nullptr, false) != RSVD_OK) return 0;
    if (algo < 0 || algo > 2) return 0;
    const rsvd_opts o = opts_or_default(op);
    if (check_algo(A, k, p, v, algo, o) != RSVD_OK) return 0;
    rsvd_status e;
    const size_t b = plan_bytes(A, k, p, v, algo, o, &e);
    return e == RSVD_OK ? b : 0;
}

rsvd_status rsvd_subspace(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o, rsvd_out* out, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
    return run_call(ALG_SUB, A, k, p, v, o, out, ws, ws_bytes, stream);
}

rsvd_status rsvd_single_pass(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o, rsvd_out* out, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
    return run_call(ALG_ONE, A, k, p, v, o, out, ws, ws_bytes, stream);
}

static rsvd_status check_normal(const rsvd_mat* J, int k, int p, int v, int method, const rsvd_opts* op) {
    rsvd_status e = check_common(J, k, p, op, nullptr, false);
    if (e != RSVD_OK) return e;
    if (J->dtype != RSVD_F64 && J->dtype != RSVD_F32) return RSVD_EUNSUPPORTED;
    if (method < NORMAL_NYSTROM || method > NORMAL_SUBSPACE || v < 2) return RSVD_EINVAL;
    const rsvd_opts o = opts_or_default(op);
    if (o.core_rows != 0 || o.one_view_method != RSVD_ONE_VIEW_TROPP || o.lc_rule != RSVD_LC_FULL ||
        o.core_kind != RSVD_CORE_GAUSSIAN || o.refine)
        return RSVD_EINVAL;
    return RSVD_OK;
}

static size_t normal_plan_bytes(const rsvd_mat* J, int k, int p, int v, int method, const rsvd_opts& o,
                                rsvd_status* err) {
    Ctx ctx{true, nullptr, Arena{nullptr}};
    ctx.f32_mode = o.f32_mode;
    *err = alg_normal(ctx, make_mat(J), k, p, v, method, o, nullptr, nullptr);
    return ctx.ar.off;
}

size_t rsvd_normal_workspace_bytes(const rsvd_mat* J, int k, int p, int v, int method, const rsvd_opts* op) {
    if (check_normal(J, k, p, v, method, op) != RSVD_OK) return 0;
    rsvd_status e;
    const size_t b = normal_plan_bytes(J, k, p, v, method, opts_or_default(op), &e);
    return e == RSVD_OK ? b : 0;
}

rsvd_status rsvd_normal_tevd(const rsvd_mat* J, int k, int p, int v, int method, const rsvd_opts* op, void* V,
                             double* lam2, void* ws, size_t ws_bytes, hipStream_t st) {
    rsvd_status e = check_normal(J, k, p, v, method, op);
    if (e != RSVD_OK) return e;
    if (!V || !lam2) return RSVD_EINVAL;
    const rsvd_opts o = opts_or_default(op);
    rsvd_status perr;
    const size_t need = normal_plan_bytes(J, k, p, v, method, o, &perr);
    if (perr != RSVD_OK) return perr;
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return RSVD_EWORKSPACE;
    Ctx ctx{false, st, Arena{(char*)ws}};
    ctx.status = (uint32_t*)ws;
    ctx.flags = (int*)((char*)ws + 32);
    ctx.trace = o.trace;
    ctx.f32_mode = o.f32_mode;
    ctx.sync_spins = o.sync_spins;
    if (ctx.trace) ctx.trace->used = 0;
    launch_op<clear_header_kernel_op>(dim3(1), dim3(64), 0, st, {(uint32_t*)ws});
    RSVD_LAUNCH_CHECK();
    return alg_normal(ctx, make_mat(J), k, p, v, method, o, V, lam2);
}

rsvd_status rsvd_extended_sizes(int k, int64_t budget, int64_t m, int64_t n, int* l1, int64_t* sc) {
    if (!l1 || !sc || k < 1 || budget < 1 || m < 1 || n < 1) return RSVD_EINVAL;
    // l1 = l2 = floor(0.8 floor(T/2 - k)); storage (2k + l1 + l2 + 1)(m + n) + s_c (s_c + 2) <= T (m + n)
    const double half = std::floor((double)budget / 2.0 - (double)k);
    const int64_t l = (int64_t)std::floor(0.8 * half);
    const int64_t room = (budget - 2 * (int64_t)k - 2 * l - 1) * (m + n);
    int64_t c = room >= 0 ? (int64_t)std::floor(std::sqrt(1.0 + (double)room)) - 1 : -1;
    while (c >= 0 && c * (c + 2) > room) --c;
    while (room >= 0 && (c + 1) * (c + 3) <= room) ++c;
    c = std::min<int64_t>(c, std::min(m, n));
    if (l < 0 || c < (int64_t)k + l) return RSVD_ESHAPE;
    *l1 = (int)l;
    *sc = c;
    return RSVD_OK;
}

size_t rsvd_noalloc_max_bytes(void) { return kNoAllocBytes; }

rsvd_status rsvd_subspace_noalloc(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o, rsvd_out* out,
                                  hipStream_t stream) {
    // the plan is checked before the scratch array is touched: an oversized or invalid request does nothing
    rsvd_status e = check_common(A, k, p, o, out, true);
    if (e != RSVD_OK) return e;
    const rsvd_opts op = opts_or_default(o);
    e = check_algo(A, k, p, v, ALG_SUB, op);
    if (e != RSVD_OK) return e;
    rsvd_status perr;
    const size_t need = plan_bytes(A, k, p, v, ALG_SUB, op, &perr);
    if (perr != RSVD_OK) return perr;
    if (need > kNoAllocBytes) return RSVD_EWORKSPACE;
    void* ws = nullptr;
    e = noalloc_scratch(&ws);
    if (e != RSVD_OK) return e;
    return run_call(ALG_SUB, A, k, p, v, o, out, ws, kNoAllocBytes, stream);
}

rsvd_status rsvd_block_krylov(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o, rsvd_out* out, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
    return run_call(ALG_KRY, A, k, p, v, o, out, ws, ws_bytes, stream);
}

static rsvd_status check_grad(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o) {
    rsvd_status e = check_common(A, k, p, o, nullptr, false);
    if (e != RSVD_OK) return e;
    if (A->dtype != RSVD_F64 && A->dtype != RSVD_F32) return RSVD_EUNSUPPORTED;
    if (A->trans) return RSVD_EUNSUPPORTED;
    if (o && o->krylov_mode != RSVD_KRYLOV_ROW_SWEEP) return RSVD_EUNSUPPORTED;
    if (v < 1) return RSVD_EINVAL;
    if ((int64_t)v * (k + p) > std::min(A->m, A->n)) return RSVD_ESHAPE;
    return RSVD_OK;
}

static size_t grad_plan_bytes(const rsvd_mat* A, int k, int p, int v, const rsvd_opts& o, int with_grad,
                              rsvd_status* err) {
    Ctx ctx{true, nullptr, Arena{nullptr}};
    ctx.f32_mode = o.f32_mode;
    rsvd_out dummy{nullptr, nullptr, nullptr};
    char fake;
    *err = alg_row_sweep_grad(ctx, make_mat(A), k, p, v, o, &dummy, nullptr, nullptr, 0.0,
                              with_grad ? (void*)&fake : nullptr, A->n);
    return ctx.ar.off;
}

size_t rsvd_grad_workspace_bytes(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* op, int with_grad) {
    if (check_grad(A, k, p, v, op) != RSVD_OK) return 0;
    const rsvd_opts o = opts_or_default(op);
    rsvd_status e;
    const size_t b = grad_plan_bytes(A, k, p, v, o, with_grad, &e);
    return e == RSVD_OK ? b : 0;
}

size_t rsvd_grad_kept_doubles(int k, int p, int v) {
    if (k < 1 || p < 0 || v < 1) return 0;
    return grad_kept_doubles(v * (k + p));
}

rsvd_status rsvd_block_krylov_grad(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* op, rsvd_out* out,
                                   double* E, const double* dS, double dE, void* G, int64_t ldg, void* ws,
                                   size_t ws_bytes, hipStream_t stream) {
    return rsvd_block_krylov_grad_kept(A, k, p, v, op, out, E, dS, dE, G, ldg, nullptr, 0, ws, ws_bytes, stream);
}

rsvd_status rsvd_block_krylov_grad_kept(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* op, rsvd_out* out,
                                        double* E, const double* dS, double dE, void* G, int64_t ldg, double* kept,
                                        int keep_mode, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (keep_mode < 0 || keep_mode > 2 || (keep_mode != 0 && !kept)) return RSVD_EINVAL;
    rsvd_status e = check_grad(A, k, p, v, op);
    if (e != RSVD_OK) return e;
    if (out && (!out->U || !out->S || !out->V)) return RSVD_EINVAL;
    if (G && ldg < A->n) return RSVD_ESHAPE;
    rsvd_opts o = opts_or_default(op);
    o.krylov_mode = RSVD_KRYLOV_ROW_SWEEP;
    rsvd_status perr;
    const size_t need = grad_plan_bytes(A, k, p, v, o, G != nullptr, &perr);
    if (perr != RSVD_OK) return perr;
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return RSVD_EWORKSPACE;
    Ctx ctx{false, stream, Arena{(char*)ws}};
    ctx.status = (uint32_t*)ws;
    ctx.flags = (int*)((char*)ws + 32);
    ctx.trace = o.trace;
    ctx.f32_mode = o.f32_mode;
    if (ctx.trace) ctx.trace->used = 0;
    launch_op<clear_header_kernel_op>(dim3(1), dim3(64), 0, stream, {(uint32_t*)ws});
    RSVD_LAUNCH_CHECK();
    return alg_row_sweep_grad(ctx, make_mat(A), k, p, v, o, out, E, dS, dE, G, ldg, kept, keep_mode);
}

void rsvd_default_batch_tuning(rsvd_batch_tuning* t) {
    if (!t) return;
    t->plan_cus = 256;
    t->view_mr = 0;
}

rsvd_status rsvd_batch_plan_create(int nb, const rsvd_mat* As, const int* ks, int p, int v, const rsvd_opts* op,
                                   const rsvd_out* outs, const rsvd_batch_tuning* tuning, rsvd_batch_plan** plan,
                                   size_t* ws_bytes) {
    if (!plan || !ws_bytes || nb < 1 || nb > 65535 || !As || !ks || !outs) return RSVD_EINVAL;
    *plan = nullptr;
    rsvd_opts o = opts_or_default(op);
    if (o.trace || o.f32_mode != RSVD_F32_MFMA) return RSVD_EUNSUPPORTED;
    rsvd_batch_plan* P = new rsvd_batch_plan();
    P->nb = nb;
    P->p = p;
    P->v = v;
    P->o = o;
    if (tuning) P->tuning = *tuning;
    else rsvd_default_batch_tuning(&P->tuning);
    if (P->tuning.plan_cus < 0 || P->tuning.view_mr < 0 || P->tuning.view_mr > 2) {
        delete P;
        return RSVD_EINVAL;
    }
    P->mats.assign(As, As + nb);
    P->ks.assign(ks, ks + nb);
    P->outs.assign(outs, outs + nb);
    size_t off = 0;
    for (int b = 0; b < nb; ++b) {
        rsvd_status e = check_common(&As[b], ks[b], p, &o, &outs[b], true);
        if (e == RSVD_OK && (As[b].dtype != RSVD_F64 && As[b].dtype != RSVD_F32)) e = RSVD_EUNSUPPORTED;
        if (e == RSVD_OK) e = check_algo(&As[b], ks[b], p, v, ALG_SUB, o);
        if (e != RSVD_OK) {
            delete P;
            return e;
        }
        Ctx ctx{true, nullptr, Arena{nullptr}};
        ctx.plan_cus = P->tuning.plan_cus;
        ctx.view_mr = P->tuning.view_mr;
        rsvd_out dummy{nullptr, nullptr, nullptr};
        e = dispatch(ctx, ALG_SUB, make_mat(&As[b]), ks[b], p, v, o, &dummy);
        if (e != RSVD_OK) {
            delete P;
            return e;
        }
        P->arena_off.push_back(off);
        off = (size_t)round_up((int64_t)(off + ctx.ar.off), 256);
    }
    P->tables_off = off;
    // the job tables' size does not depend on the base address: record once against a stand-in base
    rsvd_status e = batch_record(*P, (char*)(uintptr_t)4096);
    if (e != RSVD_OK) {
        delete P;
        return e;
    }
    P->ws_bytes = off + P->tables.size();
    *ws_bytes = P->ws_bytes;
    *plan = P;
    return RSVD_OK;
}

rsvd_status rsvd_batch_plan_bind(rsvd_batch_plan* P, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!P || !ws || ((uintptr_t)ws & 255) || ws_bytes < P->ws_bytes) return RSVD_EWORKSPACE;
    rsvd_status e = batch_record(*P, (char*)ws);
    if (e != RSVD_OK) return e;
    if (P->tables_off + P->tables.size() > ws_bytes) return RSVD_EWORKSPACE;
    for (const auto& g : P->groups) {
        if (g.shmem > 64 * 1024 &&
            hipFuncSetAttribute(g.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.shmem) != hipSuccess)
            return RSVD_EHIP;
    }
    if (hipMemcpyAsync((char*)ws + P->tables_off, P->tables.data(), P->tables.size(), hipMemcpyHostToDevice,
                       stream) != hipSuccess)
        return RSVD_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return RSVD_EHIP;
    P->ws = ws;
    return RSVD_OK;
}

rsvd_status rsvd_subspace_batched(const rsvd_batch_plan* P, hipStream_t stream) {
    if (!P || !P->ws) return RSVD_EINVAL;
    for (const auto& g : P->groups) {
        const void* table = (const char*)P->ws + P->tables_off + g.table_off;
        void* args[] = {(void*)&table};
        if (hipLaunchKernel(g.fn, dim3(g.gx, g.gy, g.gz), dim3(g.threads), args, g.shmem, stream) != hipSuccess)
            return RSVD_EHIP;
    }
    return RSVD_OK;
}

int rsvd_batch_plan_launches(const rsvd_batch_plan* P) { return P ? (int)P->groups.size() : 0; }

void rsvd_batch_plan_destroy(rsvd_batch_plan* P) { delete P; }

static rsvd_status stream_finish_body(Ctx& ctx, const rsvd_stream& S, rsvd_out* out) {
    const size_t we = dtype_size(S.wdt);
    const StreamBufs b = stream_bufs(ctx, S.m, S.n, S.k + S.p, S.sw, we);
    CALL(run_copy_panel(S.wdt, b.YT, S.m, b.Yc, S.m, S.k + S.p, S.m, nullptr, ctx.st));
    return one_view_small(ctx, S.wdt, b.Yc, S.m, S.m, b.W, S.n, S.n, b.Psi, S.m, S.k, S.p, S.sw, S.o, out);
}

rsvd_status rsvd_stream_create(int64_t m, int64_t n, int k, int p, int dtype, const rsvd_opts* op, rsvd_stream** st,
                               size_t* ws_bytes) {
    if (!st || !ws_bytes) return RSVD_EINVAL;
    *st = nullptr;
    *ws_bytes = 0;
    if (dtype != RSVD_F64 && dtype != RSVD_F32) return RSVD_EINVAL;
    if (m <= 0 || n <= 0) return RSVD_ESHAPE;
    if (k < 1 || p < 0) return RSVD_EINVAL;
    if ((int64_t)k + p > std::min(m, n)) return RSVD_ESHAPE;
    const rsvd_opts o = opts_or_default(op);
    if (o.core_rows != 0 || o.refine || o.trace) return RSVD_EINVAL;
    if (o.one_view_method != RSVD_ONE_VIEW_TROPP && o.one_view_method != RSVD_ONE_VIEW_WOOLFE) return RSVD_EINVAL;
    if (o.lc_rule < RSVD_LC_FULL || o.lc_rule > RSVD_LC_MINVAR) return RSVD_EINVAL;
    if (o.lc_rule == RSVD_LC_FIXED && (o.lc < 0 || o.lc > p)) return RSVD_EINVAL;
    if (o.lc_rule == RSVD_LC_RATIO && !(o.lc_alpha >= 0.0 && o.lc_alpha <= 1.0)) return RSVD_EINVAL;
    const int64_t s = k + p;
    const int64_t sw = o.psi_rows ? o.psi_rows : 2 * s + 1;
    if (sw < s || sw > m) return RSVD_ESHAPE;
    if (o.one_view_method == RSVD_ONE_VIEW_WOOLFE && sw > n) return RSVD_ESHAPE;
    if (s > kMaxWidth || sw > kMaxWidth) return RSVD_EUNSUPPORTED;
    rsvd_stream* S = new rsvd_stream;
    S->m = m;
    S->n = n;
    S->k = k;
    S->p = p;
    S->sw = (int)sw;
    S->wdt = dtype;
    S->o = o;
    Ctx ctx{true, nullptr, Arena{nullptr}};
    rsvd_out dummy{nullptr, nullptr, nullptr};
    const rsvd_status e = stream_finish_body(ctx, *S, &dummy);
    if (e != RSVD_OK) {
        delete S;
        return e;
    }
    S->ws_bytes = ctx.ar.off;
    *st = S;
    *ws_bytes = S->ws_bytes;
    return RSVD_OK;
}

rsvd_status rsvd_stream_bind(rsvd_stream* S, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!S) return RSVD_EINVAL;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < S->ws_bytes) return RSVD_EWORKSPACE;
    S->ws = (char*)ws;
    Ctx ctx{false, stream, Arena{S->ws}};
    const int s = S->k + S->p;
    const size_t we = dtype_size(S->wdt);
    const StreamBufs b = stream_bufs(ctx, S->m, S->n, s, S->sw, we);
    launch_op<clear_header_kernel_op>(dim3(1), dim3(64), 0, stream, {(uint32_t*)ws});
    RSVD_LAUNCH_CHECK();
    TRY(launch_gaussian(S->o.seed, TAG_OMEGA, 0, s, S->n, 0, S->wdt, b.OmT, S->n, stream));
    TRY(launch_gaussian(S->o.seed, TAG_PSI, 0, S->sw, S->m, 0, S->wdt, b.Psi, S->m, stream));
    const int64_t ny = (int64_t)s * S->m, nw = (int64_t)S->sw * S->n;
    const dim3 blk(256);
    if (S->wdt == RSVD_F64) {
        hipLaunchKernelGGL(zero_fill_kernel<double>, dim3((unsigned)std::min<int64_t>(ceil_div(ny, 256), 8192)), blk,
                           0, stream, (double*)b.YT, ny);
        hipLaunchKernelGGL(zero_fill_kernel<double>, dim3((unsigned)std::min<int64_t>(ceil_div(nw, 256), 8192)), blk,
                           0, stream, (double*)b.W, nw);
    } else {
        hipLaunchKernelGGL(zero_fill_kernel<float>, dim3((unsigned)std::min<int64_t>(ceil_div(ny, 256), 8192)), blk,
                           0, stream, (float*)b.YT, ny);
        hipLaunchKernelGGL(zero_fill_kernel<float>, dim3((unsigned)std::min<int64_t>(ceil_div(nw, 256), 8192)), blk,
                           0, stream, (float*)b.W, nw);
    }
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status rsvd_stream_add_dense(rsvd_stream* S, int64_t r0, int64_t c0, const rsvd_mat* H, hipStream_t stream) {
    if (!S || !H) return RSVD_EINVAL;
    if (!S->ws) return RSVD_EWORKSPACE;
    if (H->dtype != S->wdt || !H->data || H->row_scale) return RSVD_EINVAL;
    if (H->trans != 0 && H->trans != 1) return RSVD_EINVAL;
    if (H->m <= 0 || H->n <= 0 || H->ld < (H->trans ? H->m : H->n)) return RSVD_ESHAPE;
    if (r0 < 0 || c0 < 0 || r0 + H->m > S->m || c0 + H->n > S->n) return RSVD_ESHAPE;
    Ctx ctx{false, stream, Arena{nullptr}};
    ctx.plan_cus = 0;     // no contraction splits: the views accumulate straight into the sketches
    const int s = S->k + S->p;
    const size_t we = dtype_size(S->wdt);
    Ctx lay{true, nullptr, Arena{S->ws}};
    const StreamBufs b = stream_bufs(lay, S->m, S->n, s, S->sw, we);
    const Mat h = make_mat(H);
    // Y[r0 .. r0 + h.m) += H Omega[c0 .. c0 + h.n),  W[:, c0 .. c0 + h.n) += Psi[:, r0 .. r0 + h.m) H
    TRY(range_view(ctx, h, (const char*)b.OmT + (size_t)c0 * we, S->n, s, (char*)b.YT + (size_t)r0 * we, S->m, 1));
    TRY(corange_view(ctx, h, (const char*)b.Psi + (size_t)r0 * we, S->m, S->sw, (char*)b.W + (size_t)c0 * we, S->n,
                     1));
    return RSVD_OK;
}

rsvd_status rsvd_stream_add_entries(rsvd_stream* S, int64_t nnz, const int64_t* rows, const int64_t* cols,
                                    const void* vals, hipStream_t stream) {
    if (!S || nnz < 0) return RSVD_EINVAL;
    if (!S->ws) return RSVD_EWORKSPACE;
    if (nnz == 0) return RSVD_OK;
    if (!rows || !cols || !vals) return RSVD_EINVAL;
    const int s = S->k + S->p;
    const size_t we = dtype_size(S->wdt);
    Ctx lay{true, nullptr, Arena{S->ws}};
    const StreamBufs b = stream_bufs(lay, S->m, S->n, s, S->sw, we);
    const int64_t total = nnz * (s + S->sw);
    const dim3 grid((unsigned)std::min<int64_t>(ceil_div(total, 256), 16384));
    if (S->wdt == RSVD_F64)
        hipLaunchKernelGGL(stream_entries_kernel<double>, grid, dim3(256), 0, stream, nnz, rows, cols,
                           (const double*)vals, S->m, S->n, s, S->sw, (const double*)b.OmT, (const double*)b.Psi,
                           (double*)b.YT, (double*)b.W, (uint32_t*)S->ws);
    else
        hipLaunchKernelGGL(stream_entries_kernel<float>, grid, dim3(256), 0, stream, nnz, rows, cols,
                           (const float*)vals, S->m, S->n, s, S->sw, (const float*)b.OmT, (const float*)b.Psi,
                           (float*)b.YT, (float*)b.W, (uint32_t*)S->ws);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status rsvd_stream_finish(rsvd_stream* S, rsvd_out* out, hipStream_t stream) {
    if (!S || !out || !out->U || !out->S || !out->V) return RSVD_EINVAL;
    if (!S->ws) return RSVD_EWORKSPACE;
    Ctx ctx{false, stream, Arena{S->ws}};
    ctx.status = (uint32_t*)S->ws;
    ctx.flags = (int*)(S->ws + 32);
    ctx.sync_spins = S->o.sync_spins;
    return stream_finish_body(ctx, *S, out);
}

void rsvd_stream_destroy(rsvd_stream* S) { delete S; }

rsvd_status rsvd_device_status(const void* ws, hipStream_t stream, uint32_t* flags) {
    if (!ws) return RSVD_EINVAL;
    if (hipStreamSynchronize(stream) != hipSuccess) return RSVD_EHIP;
    uint32_t word = 0;
    if (hipMemcpy(&word, ws, sizeof(word), hipMemcpyDeviceToHost) != hipSuccess) return RSVD_EHIP;
    if (flags) *flags = word;
    if (word & (RSVD_FLAG_NONFINITE | RSVD_FLAG_SYNC_TIMEOUT)) return RSVD_EBREAKDOWN;
    return (word & RSVD_FLAG_BAD_ENTRY) ? RSVD_ESHAPE : RSVD_OK;
}

rsvd_status rsvd_one_view_lc(const void* ws, hipStream_t stream, int* lc) {
    if (!ws || !lc) return RSVD_EINVAL;
    if (hipStreamSynchronize(stream) != hipSuccess) return RSVD_EHIP;
    uint32_t word = 0;
    if (hipMemcpy(&word, (const uint32_t*)ws + kLcWord, sizeof(word), hipMemcpyDeviceToHost) != hipSuccess)
        return RSVD_EHIP;
    *lc = (int)word;
    return RSVD_OK;
}

rsvd_status rsvd_gaussian(uint64_t seed, uint32_t tag, uint32_t batch, int64_t rows, int64_t cols, int long_is_row,
                          int dtype, void* out, int64_t ld, hipStream_t stream) {
    if (rows < 0 || cols < 0 || !out || ld < cols) return RSVD_EINVAL;
    if (dtype != RSVD_F64 && dtype != RSVD_F32) return RSVD_EINVAL;
    if ((long_is_row ? rows : cols) > (int64_t)4 * 0xFFFFFFFFll) return RSVD_ESHAPE;
    return launch_gaussian(seed, tag, batch, rows, cols, long_is_row, dtype, out, ld, stream);
}

rsvd_status rsvd_philox_words(const uint32_t* ctr, int64_t count, uint32_t key0, uint32_t key1, uint32_t* out,
                              hipStream_t stream) {
    if (count < 0 || !ctr || !out) return RSVD_EINVAL;
    if (count == 0) return RSVD_OK;
    hipLaunchKernelGGL(philox_words_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(count, 256), 4096)), dim3(256), 0,
                       stream, ctr, count, key0, key1, out);
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

size_t rsvd_view_workspace_bytes(const rsvd_mat* A, int s, const rsvd_opts* o) {
    if (!A || s < 1 || A->m <= 0 || A->n <= 0) return 0;
    const rsvd_opts op = opts_or_default(o);
    const Mat a = make_mat(A);
    Ctx ctx{true, nullptr, Arena{nullptr}};
    ctx.f32_mode = op.f32_mode;
    if (range_view(ctx, a, nullptr, a.n, s, nullptr, a.m, 0, 0, op.refine != 0) != RSVD_OK) return 0;
    const size_t r = ctx.ar.off;
    Ctx ctx2{true, nullptr, Arena{nullptr}};
    ctx2.f32_mode = op.f32_mode;
    if (corange_view(ctx2, a, nullptr, a.m, s, nullptr, a.n, 0, op.refine != 0) != RSVD_OK) return 0;
    return std::max(r, ctx2.ar.off);
}

static rsvd_status check_view(const rsvd_mat* A, int s, const void* in, void* outp, const rsvd_opts* o, void* ws,
                              size_t ws_bytes) {
    if (!A || !A->data || !in || !outp || s < 1) return RSVD_EINVAL;
    if (A->dtype != RSVD_F64 && A->dtype != RSVD_F32 && !low_precision(A->dtype)) return RSVD_EINVAL;
    if ((A->dtype == RSVD_FP8_E4M3) != (A->row_scale != nullptr)) return RSVD_EINVAL;
    if (A->m <= 0 || A->n <= 0 || A->ld < (A->trans ? A->m : A->n)) return RSVD_ESHAPE;
    if (low_precision(A->dtype) && !lp_aligned(A->dtype, A->data, A->ld)) return RSVD_EINVAL;
    if (o && o->f32_mode != RSVD_F32_MFMA && o->f32_mode != RSVD_F32_BF16X6) return RSVD_EINVAL;
    const size_t need = rsvd_view_workspace_bytes(A, s, o);
    if (need == 0) return RSVD_EUNSUPPORTED;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need) return RSVD_EWORKSPACE;
    return RSVD_OK;
}

rsvd_status rsvd_view_range(const rsvd_mat* A, int s, const void* XT, void* YT, const rsvd_opts* o, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
    rsvd_status e = check_view(A, s, XT, YT, o, ws, ws_bytes);
    if (e != RSVD_OK) return e;
    const rsvd_opts op = opts_or_default(o);
    Ctx ctx{false, stream, Arena{(char*)ws}};
    ctx.f32_mode = op.f32_mode;
    const Mat a = make_mat(A);
    return range_view(ctx, a, XT, a.n, s, YT, a.m, 0, 0, op.refine != 0);
}

rsvd_status rsvd_view_corange(const rsvd_mat* A, int s, const void* YT, void* ZT, const rsvd_opts* o, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
    rsvd_status e = check_view(A, s, YT, ZT, o, ws, ws_bytes);
    if (e != RSVD_OK) return e;
    const rsvd_opts op = opts_or_default(o);
    Ctx ctx{false, stream, Arena{(char*)ws}};
    ctx.f32_mode = op.f32_mode;
    const Mat a = make_mat(A);
    return corange_view(ctx, a, YT, a.m, s, ZT, a.n, 0, op.refine != 0);
}

}  // extern "C"

LaunchRecorder*& launch_recorder() {
    static thread_local LaunchRecorder* r = nullptr;
    return r;
}
