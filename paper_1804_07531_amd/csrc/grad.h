// Host-side interface of the adjoint kernels (grad.hip).
#pragma once

#include <stdint.h>

#include "rsvd.h"

// Up to four (L, R) panel pairs of a low-rank sum sum_seg scale L^T R.
template <typename T>
struct OuterSegs {
    const T* L[4];
    const T* R[4];
    int64_t ldl[4];
    int64_t ldr[4];
    int rows[4];
    double scale[4];
    int count;
};

int64_t frob_parts();
// E = ||A||_F^2 - sum_{i < nl} lam_i^2 (FP64; part holds frob_parts() doubles).
rsvd_status run_frob_sq(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, double* part,
                        const double* lam, int nl, double* E, hipStream_t st);
// G = alpha A + sum_seg scale_seg L_seg^T R_seg (panels rows x m and rows x n).
rsvd_status run_outer_update_f32(const float* A, int64_t lda, double alpha, int64_t m, int64_t n,
                                 const OuterSegs<float>& segs, float* G, int64_t ldg, hipStream_t st);
rsvd_status run_outer_update_f64(const double* A, int64_t lda, double alpha, int64_t m, int64_t n,
                                 const OuterSegs<double>& segs, double* G, int64_t ldg, hipStream_t st);
// Coefficients of the Q_c adjoint: C2 is the forward's B^T coefficient matrix.
rsvd_status run_grad_coeff(const double* Ut, const double* dS, double dE, int k, const double* C2, int sk, double* C,
                           hipStream_t st);
rsvd_status run_sym_upper(const double* N, int s, double* S, hipStream_t st);
rsvd_status run_transpose_f64(const double* X, int s, double* Y, hipStream_t st);
rsvd_status run_scale_cols(const double* X, int ldx, int rows, int cols, const double* d, double* Y, hipStream_t st);
rsvd_status run_rank_check(const double* S, int n, double tau, uint32_t* status, uint32_t bit, hipStream_t st,
                           const int* enable = nullptr);
rsvd_status run_fill_zero(int dtype, void* p, int64_t count, hipStream_t st);
