// Host-side interface of the SRFT test matrices (srft.hip).
#pragma once

#include <stdint.h>

#include "rsvd.h"

// Panel Phi^T (s_c x L, row-major, leading dimension ld, FP64 or FP32) of the
// subsampled randomized DCT of one side of length L (Sect. 6.7).  pos is
// device scratch for s_c ints (the sampled frequencies).  Requires
// 1 <= s_c <= L < 2^31.
rsvd_status run_srft_panel(uint64_t seed, uint32_t sign_tag, uint32_t sample_tag, int64_t L, int sc, int* pos,
                           int dtype, void* out, int64_t ld, hipStream_t st);
