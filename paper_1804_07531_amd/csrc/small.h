// Host-side interface of the small dense steps (small.hip).
#pragma once

#include <stdint.h>

#include "rsvd.h"

bool jacobi_fits_lds(int s);
// Doubles of global scratch run_small_svd needs for order s (0 when it runs in LDS).
size_t small_svd_scratch_doubles(int s);
// M (s x s FP64) = L diag(sigma) Rv^T, sorted by decreasing sigma; column c of
// L / Rv (row-major s x s) is the c-th singular vector.
// spin_limit: polls before the multi-workgroup form's bounded barrier wait gives up (0: default).
rsvd_status run_small_svd(const double* M, int s, double* L, double* Rv, double* sigma, double* gscratch,
                          uint32_t* status, const int* enable, hipStream_t st, unsigned spin_limit = 0);
// out (len x k, leading dimension ldo) = P^T F[:, :k] for a panel P (s x len).
rsvd_status run_lift(int dtype_p, const void* P, int64_t ldp, int s, int64_t len, const double* F, int ldf, int k,
                     int dtype_o, void* out, int64_t ldo, hipStream_t st);
int64_t sign_chunks(int64_t len);
// Joint sign fix of (U, V): the largest-magnitude entry of each column of U is made positive.
rsvd_status run_signs(int dtype, void* U, int64_t m, void* V, int64_t n, int k, double* pval, int64_t* pidx,
                      double* sgn, hipStream_t st);
rsvd_status run_copy_f64(const double* src, double* dst, int64_t count, hipStream_t st);
// Y = X^T (s x s, row-major FP64; Y must not alias X).
rsvd_status run_transpose_small_f64(const double* X, double* Y, int s, hipStream_t st);
