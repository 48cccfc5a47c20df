// Host-side interface of the view kernels (views.hip).
#pragma once

#include <stdint.h>

#include "rsvd.h"

// One view: A (m x n, row-major, leading dimension lda) times a thin operand
// given as a panel (s x len row-major, leading dimension ld_thin).
struct ViewArgs {
    int dtype;          // RSVD_F64 or RSVD_F32: type of A and of the panels
    const void* A;
    int64_t lda, m, n;
    const void* thin;
    int64_t ld_thin;
    int s;
    int mr_hint = 0;    // 1 or 2 rows (columns) of 16 per wave; 0: chosen by the plan
};

struct ViewPlan {
    int nb = 1;         // 16-wide blocks of the thin dimension
    int mr = 1;         // 16-row (or column) blocks of A per wave
    int64_t tiles = 0;  // workgroups along the output's long side
    int64_t splits = 1; // splits of the contraction (partials + fixed-order sum)
    int64_t chunk = 0;  // contraction length per split
};

int view_max_width();
ViewPlan plan_range(const ViewArgs& v, int num_cu);
ViewPlan plan_corange(const ViewArgs& v, int num_cu);
size_t view_partial_elems(const ViewPlan& p, int64_t s, int64_t len);

// Y^T (s x m, leading dimension ldo) = (A X)^T (accumulate != 0: added to out).
// With slots_only, the products only fill the split slots in partial (s x m
// each, s * m elements apart; accumulate != 0: added to what the slots hold;
// a plan with one split fills the first slot), and run_reduce_view_parts
// later sums them.
rsvd_status run_range(const ViewArgs& v, const ViewPlan& p, void* out, int64_t ldo, void* partial, int accumulate,
                      hipStream_t st, bool slots_only = false);
// Z^T (s x n, leading dimension ldo) = (A^T Y)^T; slots_only as for run_range.
rsvd_status run_corange(const ViewArgs& v, const ViewPlan& p, void* out, int64_t ldo, void* partial, int accumulate,
                        hipStream_t st, bool slots_only = false);
// The plan with at most max_splits contraction splits.
ViewPlan cap_splits(const ViewPlan& p, int64_t contraction, int64_t max_splits);
// out (s x len, leading dimension ldo) [+]= the sum of nparts split slots
// (s x len each, packed), in a fixed order.  A follow-up of the view that
// filled the slots: it opens no batch phase of its own.
rsvd_status run_reduce_view_parts(int dtype, const void* parts, int nparts, int64_t s, int64_t len, void* out,
                                  int64_t ldo, int accumulate, hipStream_t st);

rsvd_status launch_gaussian(uint64_t seed, uint32_t tag, uint32_t batch, int64_t rows, int64_t cols,
                            int long_is_row, int dtype, void* out, int64_t ld, hipStream_t stream);

// Sum of nparts partial panels (rows x cols, parts `stride` elements apart)
// into out (leading dimension ldo), in a fixed order.
rsvd_status run_reduce_parts_f32(const float* parts, int nparts, int64_t stride, int64_t rows, int64_t cols,
                                 float* out, int64_t ldo, int accumulate, hipStream_t st);

// ---------------------------------------------------------------------------
// Views on BF16 / FP8 matrix cores (views_lp.hip).  The stored matrix S
// (m x n, row-major, leading dimension lda) is BF16, FP8 E4M3 with one
// scale per stored row, or FP32 split into three BF16 parts; the thin
// operand is prepared from an FP32 panel by lp_prepare_thin.
// ---------------------------------------------------------------------------
enum { LP_THIN_BF16 = 1, LP_THIN_BF16X3 = 3, LP_THIN_FP8 = 8 };

struct LpArgs {
    int dtype = RSVD_BF16;           // RSVD_BF16, RSVD_FP8_E4M3 or RSVD_F32 (split)
    const void* A = nullptr;
    int64_t lda = 0, m = 0, n = 0;
    const float* row_scale = nullptr; // FP8: one scale per stored row (range views apply it to the output)
    int thin_kind = LP_THIN_BF16;
    const void* planes = nullptr;     // prepared thin operand
    int64_t ldp = 0, pstride = 0;
    const float* thin_scale = nullptr; // FP8 thin: one scale per thin column
    int s = 0;
};

int64_t lp_plane_ld(int64_t len);
size_t lp_thin_bytes(int thin_kind, int s, int64_t len);
bool lp_aligned(int dtype, const void* A, int64_t lda);
bool lp_fits(const LpArgs& v, bool corange);
// Thin operand from an FP32 panel P (s x len, leading dimension ld); fills
// the thin fields of v.  len_scale (may be null) multiplies column r of P.
rsvd_status lp_prepare_thin(const float* P, int64_t ld, int s, int64_t len, const float* len_scale, int thin_kind,
                            void* buf, LpArgs& v, hipStream_t st);
ViewPlan plan_lp(const LpArgs& v, bool corange, int num_cu);
// corange = false: Y^T (s x m) = (S X)^T; true: Z^T (s x n) = (S^T Y)^T.
rsvd_status run_lp(const LpArgs& v, const ViewPlan& p, bool corange, float* out, int64_t ldo, float* partial,
                   int accumulate, hipStream_t st);
