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
rsvd_status run_range(const ViewArgs& v, const ViewPlan& p, void* out, int64_t ldo, void* partial, int accumulate,
                      hipStream_t st);
// Z^T (s x n, leading dimension ldo) = (A^T Y)^T.
rsvd_status run_corange(const ViewArgs& v, const ViewPlan& p, void* out, int64_t ldo, void* partial, int accumulate,
                        hipStream_t st);

rsvd_status launch_gaussian(uint64_t seed, uint32_t tag, uint32_t batch, int64_t rows, int64_t cols,
                            int long_is_row, int dtype, void* out, int64_t ld, hipStream_t stream);
