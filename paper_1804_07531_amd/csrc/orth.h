// Host-side interface of the orthonormalization kernels (orth.hip).
#pragma once

#include <stdint.h>

#include "rsvd.h"

int64_t cross_splits(int s1, int s2, int64_t len, int symmetric, int num_cu);
size_t cross_scratch_doubles(int s1, int s2, int64_t len, int symmetric, int num_cu);
// out (s1 x s2, FP64, row-major) = P1 P2^T for panels P1 (s1 x len), P2 (s2 x len).
rsvd_status run_cross(int dtype1, const void* P1, int64_t ld1, int s1, int dtype2, const void* P2, int64_t ld2,
                      int s2, int64_t len, int symmetric, double* out, double* scratch, int num_cu,
                      const int* enable, hipStream_t st);

bool chol_fits_lds(int s);
// G = L L^T, R = L^T, Rinv = R^-1 (all s x s FP64 row-major); shifted retry as described in orth.hip.
// With near_id_tol2 > 0, a G with ||G - I||_F^2 <= near_id_tol2 gets its factors in closed form,
// exact to second order in G - I.
rsvd_status run_chol_inv(const double* G, int s, int64_t len, double* R, double* Rinv, double* gscratch,
                         uint32_t* status, int* need_more, const int* enable, hipStream_t st,
                         double near_id_tol2 = 0.0);
// side 0: Racc <- R Racc; side 1: Racc <- Racc R (upper triangular s x s).
rsvd_status run_trmm_upper(const double* R, double* Racc, double* tmp, int s, int side, const int* enable,
                           hipStream_t st);
// OUT[a][x] = beta OUT[a][x] + alpha sum_b C[b][a] IN[b][x] on panels (FP64 arithmetic).  Above
// s_out = 256 the output is written in slices of at most 224 rows, so OUT must not alias IN.  f32_sums
// lets FP32 panels (in and out) take FP32 matrix cores with FP32 sums; callers set it only where
// the sums cannot cancel (C close to orthogonal).
// out (len x k, row-major, ldo) = P^T F[:, :k] for a panel P (s x len) and F (s x ldf, FP64):
// the lift U = Q_c U^_k, on matrix cores with FP64 sums (the apply with a row-major store).
rsvd_status run_lift_rows(int dtype_p, const void* P, int64_t ldp, int s, int64_t len, const double* F, int ldf,
                          int k, int dtype_o, void* out, int64_t ldo, hipStream_t st);
rsvd_status run_apply_coeff(int dtype_in, const void* IN, int64_t ldi, int s_in, int64_t len, const double* C,
                            int64_t ldc, int s_out, int triangular, double alpha, double beta, int dtype_out,
                            void* OUT, int64_t ldo, const int* enable, hipStream_t st, bool f32_sums = false);
// Q^T = R^-T Y^T (panels s x len); QT may alias YT.  f32_sums as above.
rsvd_status run_apply_rinv(int dtype_in, const void* YT, int64_t ldy, int s, int64_t len, const double* Rinv,
                           int dtype_out, void* QT, int64_t ldq, const int* enable, hipStream_t st,
                           bool f32_sums = false);
// Copy of a rows x cols panel (skipped when *enable == 0).
rsvd_status run_copy_panel(int dtype, const void* src, int64_t lds, void* dst, int64_t ldd, int rows, int64_t cols,
                           const int* enable, hipStream_t st);
