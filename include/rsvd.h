/*
 * rsvd.h -- pass-efficient randomized low-rank SVD on one MI355X (gfx950).
 *
 * C ABI of the library.  The method is Bjarkason, "Pass-Efficient Randomized
 * Algorithms for Low-Rank Matrix Approximation Using Any Number of Views"
 * (2018).  Every entry point returns an approximate rank-k SVD
 * A ~ U diag(S) V^T of an m x n matrix A from a budget of v views, where one
 * view is one full read of A (the paper's "number of times the matrix is
 * accessed", Sect. 1).
 *
 * Letters: target rank k (the paper's p), oversampling p (the paper's l),
 * sketch width s = k + p.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * - All array pointers are DEVICE pointers unless stated otherwise; structs
 *   passed by pointer live in host memory and are read before the call
 *   returns.
 * - All matrices are row-major.  A is m x n with leading dimension ld >= n
 *   (elements).  With trans = 1 the buffer holds A^T row-major (n x m, leading
 *   dimension ld >= m), i.e. A column-major; results are still those of A.
 * - Outputs: U is m x k, V is n x k (row-major, leading dimension k), in FP64
 *   when A is FP64 and in FP32 otherwise; S holds k FP64 values in
 *   descending order.  Each pair (u_i, v_i) is sign-fixed jointly so that the
 *   entry of largest magnitude of u_i is positive (ties: lowest row index).
 * - Gaussian test matrices are drawn from a counter-based generator
 *   (Philox4x32-10 + Box-Muller) keyed by opts->seed, so a call is a pure
 *   function of (A, k, p, v, opts): entry (long index i, short index j) of the
 *   range test matrix Omega (n x s) uses counter (i>>2, j, 0, 1) and output
 *   word i&3; the co-range test matrix Psi (s_w x m, entry (j, i)) uses tag 2.
 * - The caller owns A, the outputs and the workspace.  The library never
 *   allocates device memory on the call path, never frees caller memory and
 *   keeps no mutable global state (except the per-GPU scratch array of
 *   rsvd_subspace_noalloc, which is the library's).  Query the workspace size with
 *   rsvd_workspace_bytes() and pass a buffer of at least that many bytes,
 *   aligned to 256 bytes.
 * - Every call is asynchronous on the given HIP stream: kernels are enqueued
 *   and the call returns; no host synchronization happens inside a call.
 * - Argument checking is synchronous and complete before the first launch:
 *   a call that returns an error enqueues nothing.  Numerical trouble found on
 *   the device (a non-finite singular value) is recorded in the workspace's
 *   status word; read it with rsvd_device_status().
 * - Calls that share one workspace buffer must be ordered (same stream or
 *   explicit events); calls with distinct workspaces may overlap.
 */
#ifndef RSVD_H
#define RSVD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSVD_OK = 0,
    RSVD_EINVAL = 1,        /* bad scalar argument or option, or a null pointer */
    RSVD_ESHAPE = 2,        /* sizes violate k + p <= min(m, n) or a similar rule */
    RSVD_EWORKSPACE = 3,    /* workspace too small or misaligned */
    RSVD_EBREAKDOWN = 4,    /* device reported non-finite results or a barrier timeout */
    RSVD_EHIP = 5,          /* a HIP runtime call failed */
    RSVD_EUNSUPPORTED = 6   /* valid request this build does not implement */
} rsvd_status;

typedef enum {
    RSVD_F64 = 0,           /* IEEE binary64 */
    RSVD_F32 = 1,           /* IEEE binary32 */
    RSVD_BF16 = 2,          /* bfloat16 (upper half of binary32) */
    RSVD_FP8_E4M3 = 3       /* OCP FP8 E4M3 (bias 7, max 448) with one FP32 scale per stored row */
} rsvd_dtype;
/* BF16 and FP8 matrices: the stored values (times the row scales) are the
 * matrix whose SVD is computed.  They are accepted by rsvd_subspace and the
 * view entry points only (other algorithms return RSVD_EUNSUPPORTED), need a
 * 16-byte aligned data pointer and ld * element size a multiple of 16
 * (RSVD_EINVAL otherwise), and return U and V in FP32. */

typedef enum {
    RSVD_ALGO_SUBSPACE = 0,
    RSVD_ALGO_SINGLE_PASS = 1,
    RSVD_ALGO_BLOCK_KRYLOV = 2
} rsvd_algo;

typedef enum {
    RSVD_KRYLOV_ALTERNATING = 0,  /* Alg. 9 as printed: one product with A or A^T per view */
    RSVD_KRYLOV_ROW_SWEEP = 1,    /* Sect. 7.3: each view reads A once and forms A X and A^T (A X) */
    RSVD_KRYLOV_COL_SWEEP = 2     /* the same on A^T (column-wise access) */
} rsvd_krylov_mode;

typedef enum {
    RSVD_F32_MFMA = 0,      /* FP32 views on FP32 matrix cores (FP32 products, FP32 accumulation) */
    RSVD_F32_BF16X6 = 1     /* FP32 views on BF16 matrix cores: A = a1 + a2 + a3 and X = x1 + x2 + x3
                               split exactly into BF16 parts, the six products a_i x_j with
                               i + j <= 4 (each exact in FP32) accumulated in FP32; the dropped
                               terms are below 2^-26 |a x|.  Needs a 16-byte aligned A with
                               ld % 4 == 0 and s <= 192 (wider or unaligned views use RSVD_F32_MFMA) */
} rsvd_f32_mode;

/* One-view post-processing (Sect. 6.5): the variant that turns the two
 * sketches into a rank-k SVD. */
typedef enum {
    RSVD_ONE_VIEW_TROPP = 0,    /* Alg. 7: X = (Psi Q_c)^+ W, A ~ Q_c [[X]]_k */
    RSVD_ONE_VIEW_WOOLFE = 1    /* Alg. 8: Q_r from W^T as well; X^ solves (Psi Q_c) X^ = W Q_r
                                   (eq. lstsqWoolfe), A ~ Q_c [[X^]]_k Q_r^T */
} rsvd_one_view_method;

/* How many of the p oversampling columns of the range sketch the one-view
 * post-processing keeps (Sect. 6.6): Q_c holds the k + l_c leading left
 * singular vectors of Y = A Omega, 0 <= l_c <= l_1 = p. */
typedef enum {
    RSVD_LC_FULL = 0,       /* l_c = l_1: Q_c is an orthonormal basis of Y (Tropp's baseline) */
    RSVD_LC_FIXED = 1,      /* l_c = opts.lc */
    RSVD_LC_RATIO = 2,      /* l_c = floor(alpha l_1), alpha = opts.lc_alpha (eq. lcutfixedratio, Sect. 6.6.1) */
    RSVD_LC_MINVAR = 3      /* the minimum-variance l_c of eq. MinVar (Sect. 6.6.2): for every l_c = 0..l_1 the
                               k leading singular values lambda(l_c) of X(l_c) = (Psi Q_c)^+ W are formed; the
                               choice minimizes, over 0 <= c < l_1, the population variance of the ratios
                               lambda(c-1)/lambda(c), lambda(c)/lambda(c), lambda(c+1)/lambda(c) (the first
                               block omitted for c = 0), ties to the smallest c.  Chosen on the device; read it
                               back with rsvd_one_view_lc() */
} rsvd_lc_rule;

/* Test matrices of the core sketch Z = Phi_r^T A Phi_c (Sect. 6.7). */
typedef enum {
    RSVD_CORE_GAUSSIAN = 0, /* Gaussian Phi_r^T (s_c x m, tag 3) and Phi_c^T (s_c x n, tag 4) */
    RSVD_CORE_SRFT = 1      /* the paper's subsampled randomized trigonometric transforms Phi = D C^T P (L x s_c,
                               L = m or n): D a diagonal of random signs, C the orthonormal DCT-II
                               (C[f][j] = a_f cos(pi (2j + 1) f / (2L)), a_0 = sqrt(1/L), a_f = sqrt(2/L)),
                               P the s_c frequencies of the smallest generator words.  The sign of position j is
                               the top bit of word j & 3 of counter (j >> 2, 0, 0, tag) (tag 6 for Phi_r, 8 for
                               Phi_c); the sample holds the s_c positions with the smallest (word under tag 7 or
                               9, position) pairs, in increasing order */
} rsvd_core_kind;

typedef struct {
    rsvd_dtype dtype;
    int64_t m, n;           /* A is m x n */
    int64_t ld;             /* leading dimension in elements of the stored rows */
    int trans;              /* 0: data is A row-major; 1: data is A^T row-major */
    const void* data;       /* device pointer */
    const float* row_scale; /* FP8 only: one device FP32 scale per stored row r, the stored matrix being
                               row_scale[r] * e4m3(data[r, :]) (rows of A for trans = 0, of A^T for 1) */
} rsvd_mat;

/* Optional timing hook.  When rsvd_opts.trace is not NULL, a call records
 * events[2u] before and events[2u+1] after the kernels of its u-th view
 * (u = 0 .. capacity-1, on the call's stream) and sets kind[u] (0: range
 * view A X, 1: co-range view A^T Y, 2: the one-view pass forming both
 * sketches, 3: one row sweep forming A X and A^T A X) and used.  With
 * inner = 1 the passes of kinds 2 and 3 are not recorded as a whole; the
 * range and co-range products they take on each panel or block are, one pair
 * each (kinds 0 and 1).  The events are created by the caller
 * (hipEventCreate); the library only records them. */
typedef struct {
    hipEvent_t* events;     /* 2 * capacity events */
    int capacity;           /* event pairs available */
    int used;               /* out: pairs recorded */
    int* kind;              /* out: capacity entries (host memory) */
    int inner;              /* 0: whole views and passes; 1: the products inside the passes */
} rsvd_view_trace;

typedef struct {
    uint64_t seed;          /* key of the test-matrix generator */
    int refine;             /* BF16/FP8 only.  0: every view multiplies the stored A by the thin operand
                               rounded to BF16 (BF16 A) or to FP8 E4M3 with one power-of-two scale
                               per thin column, the smallest with max |x| / scale <= 448 (FP8 A,
                               on FP8 matrix cores; a contraction over stored rows first folds the
                               row scales into the thin operand).  1: the same, except the last view,
                               which multiplies the exact stored values by an FP32-accurate thin
                               operand (three BF16 parts), FP32 accumulation throughout */
    int krylov_mode;        /* rsvd_krylov_mode, block Krylov only */
    int64_t block_rows;     /* rows per block of a row sweep (0 = 1024); for the one-view method the
                               panel height of its sweep (0 or 1024 = about 96 MiB of A per panel) */
    int64_t psi_rows;       /* single pass: rows of Psi (0 = 2s + 1) */
    int core_rows;          /* single pass: 0, or s_c >= k+p rows of the Gaussian core sketch
                               Z = Phi_r^T A Phi_c (Sect. 6.7); psi_rows must then be 0 or k+p */
    double trunc_tau;       /* row sweep: relative cut of R_K's pseudo-inverse (0 = default) */
    int f32_mode;           /* rsvd_f32_mode for FP32 views */
    rsvd_view_trace* trace; /* optional timing hook (host struct), NULL for none */
    int one_view_method;    /* single pass without a core sketch: rsvd_one_view_method (default Tropp) */
    int lc_rule;            /* single pass without a core sketch: rsvd_lc_rule (default RSVD_LC_FULL) */
    int lc;                 /* RSVD_LC_FIXED: 0 <= lc <= p */
    double lc_alpha;        /* RSVD_LC_RATIO: 0 <= lc_alpha <= 1 */
    int core_kind;          /* rsvd_core_kind of the core sketch (core_rows > 0) */
    uint32_t sync_spins;    /* polls after which the bounded device-wide wait of the multi-workgroup small
                               SVD gives up and sets status bit 4 (0 = the default of 2^22); a small value
                               lets a test drive the timeout path with every kernel still exiting */
} rsvd_opts;

typedef struct {
    void* U;                /* m x k */
    double* S;              /* k */
    void* V;                /* n x k */
} rsvd_out;

/* Fills *o with the defaults (seed 0, no refinement, ALTERNATING, 1024-row
 * blocks, Psi with 2s+1 rows, default tau, FP32 on matrix cores). */
void rsvd_default_opts(rsvd_opts* o);

/* Workspace bytes a call with these arguments needs (0 when the arguments
 * are invalid).  algo is an rsvd_algo.  o may be NULL for the defaults. */
size_t rsvd_workspace_bytes(const rsvd_mat* A, int k, int p, int v, int algo, const rsvd_opts* o);

/*
 * Generalized randomized subspace iteration, Alg. 2 (Sect. 4), v >= 2 views.
 * Q_r starts as the Gaussian Omega (n x s); view j multiplies by A (odd j)
 * or A^T (even j) and orthonormalizes.  Even v returns the SVD of
 * Q_c Q_c^T A (small SVD of R_r), odd v that of A Q_r Q_r^T (small SVD of
 * R_c).  Requires 1 <= k, 0 <= p, k + p <= min(m, n).
 */
rsvd_status rsvd_subspace(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o,
                          rsvd_out* out, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * rsvd_subspace without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The call runs exactly the kernels of
 * rsvd_subspace on a scratch array the library holds on each GPU it runs on
 * (rsvd_noalloc_max_bytes() bytes, 32 MiB, from the library's load to the
 * end of the process); it allocates nothing and calls no allocating routine.
 * A request whose workspace (rsvd_workspace_bytes with RSVD_ALGO_SUBSPACE)
 * exceeds that size returns RSVD_EWORKSPACE and does nothing.  Every call on
 * one GPU shares that GPU's array, which keeps the last call's contents (the
 * status word included, so rsvd_device_status cannot be pointed at it):
 * calls that overlap on one GPU, on different streams or from different host
 * threads without ordering, race and give wrong results.  Otherwise as
 * rsvd_subspace; the first call on a device looks up the array's address
 * (RSVD_EHIP if that fails).
 */
rsvd_status rsvd_subspace_noalloc(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o, rsvd_out* out,
                                  hipStream_t stream);

/* Bytes of the per-GPU scratch array of rsvd_subspace_noalloc. */
size_t rsvd_noalloc_max_bytes(void);

/*
 * One-view method, Alg. 7 (Sect. 6.5) with l_c = l_1 (Tropp's baseline),
 * v must be 1.  One read of A forms both sketches Y = A Omega (m x s) and
 * W = Psi A (s_w x n, s_w = psi_rows or 2s+1 by the moderate-decay rule of
 * Sect. 6.3); then Q_c = orth(Y), [Q^, R^] = qr(Psi Q_c),
 * X = R^^-1 Q^^T W, [U^, S, V] = tsvd(X, k), U = Q_c U^.
 * Requires s <= s_w <= m.
 *
 * With o->one_view_method = RSVD_ONE_VIEW_WOOLFE (Alg. 8) or an lc_rule
 * other than RSVD_LC_FULL (Sect. 6.6), the same sweep is followed by the
 * post-processing in the small space: Y = Q_Y R_Y and W^T = Q_W R_W
 * (CholeskyQR, FP64 factors), R_Y = L_Y S_Y (.)^T, Q_c = Q_Y L_Y[:, :k+l_c]
 * (the k + l_c leading left singular vectors of Y), [Q^, R^] = qr(Psi Q_c)
 * and M = R^^-1 Q^^T R_W^T, so that X = M Q_W^T.  Alg. 7: [U~, S, V~] =
 * tsvd(M, k), U = Q_c U~, V = Q_W V~.  Alg. 8: Q_r = Q_W L_W[:, :k+l_c]
 * with R_W = L_W S_W (.)^T, X^ = M L_W[:, :k+l_c] (k+l_c square),
 * [U~, S, V~] = tsvd(X^, k), U = Q_c U~, V = Q_r V~.  The l_c chosen is
 * recorded in the workspace (rsvd_one_view_lc).  Requires s_w <= 512 and,
 * for Alg. 8, s_w <= n; not combined with a core sketch (RSVD_EINVAL).
 *
 * With o->core_rows = s_c > 0: the extended one-view sketch of Sect. 6.7 with
 * the improved reconstruction (eq. bwzimproved), Gaussian test matrices in
 * place of the paper's SRFTs.  The same read of A forms Y_c = A Omega_r,
 * Y_r^T = Psi A with k + p rows (l1 = l2) and Z = Phi_r^T A Phi_c (s_c x s_c);
 * then Q_c, Q_r, U_c T_c = qr(Phi_r^T Q_c), U_r T_r = qr(Phi_c^T Q_r),
 * C = T_c^-1 U_c^T Z U_r T_r^-T, [U^, S, V^] = tsvd(C, k), U = Q_c U^,
 * V = Q_r V^.  Requires k + p <= s_c <= min(m, n), psi_rows 0 or k + p
 * (else RSVD_ESHAPE / RSVD_EINVAL); FP32 or FP64 storage.  o->core_kind =
 * RSVD_CORE_SRFT takes the paper's SRFT core test matrices instead of
 * Gaussians (s_c <= 2048).
 */
rsvd_status rsvd_single_pass(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o,
                             rsvd_out* out, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Block Krylov methods (Sect. 7).
 * ALTERNATING: Alg. 9 with v >= 2 views (v - 1 + one final view).
 * ROW_SWEEP: the row-wise accuracy-enhanced variant (Sect. 7.3 with the
 *   single-sweep products of Sect. 6.8): each of v >= 1 views reads A once
 *   and yields Y = A X and Z = A^T Y; the basis of K = [Y_1..Y_v] and
 *   B^T = A^T Q_c are formed from these sketches without a further view.
 *   Requires v * s <= min(m, n).
 * COL_SWEEP: ROW_SWEEP applied to A^T.
 */
rsvd_status rsvd_block_krylov(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o,
                              rsvd_out* out, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Row-sweep block Krylov (the ROW_SWEEP method above, Sect. 7.3) with two loss
 * terms and their gradient with respect to A, Omega held fixed.
 * Forward: as rsvd_block_krylov (out may be NULL), plus
 *   E = ||A - Q_c Q_c^T A||_F^2 = ||A||_F^2 - ||Q_c^T A||_F^2   (device FP64 scalar, may be NULL),
 * where Q_c is the method's orthonormal basis of K = [A X_0 .. A X_{v-1}].
 * Gradient (when G is not NULL): G (m x n, row-major, leading dimension
 * ldg, A's dtype) = dL/dA for L = sum_i dS[i] sigma_i + dE * E, dS a device
 * FP64 array of k entries (NULL = zeros).  The adjoint is hand-written: it
 * recomputes the sketches (nothing is kept between calls), propagates
 * through the sweeps, the projections, the orthonormalizations and the
 * small SVDs, and assembles G = 2 dE A + (a sum of thin outer products).
 * It assumes K has full numerical rank; if the TSVD of R_K would cut a
 * column, bit 3 (value 8) of the status word is set (rsvd_device_status).
 * Requires A in FP64 or FP32 with trans = 0, o->krylov_mode ROW_SWEEP (or o
 * NULL), v >= 1 and v (k + p) <= min(m, n).
 */
rsvd_status rsvd_block_krylov_grad(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o, rsvd_out* out,
                                   double* E, const double* dS, double dE, void* G, int64_t ldg, void* ws,
                                   size_t ws_bytes, hipStream_t stream);

/* Workspace of rsvd_block_krylov_grad (with_grad = 0: forward and E only). */
size_t rsvd_grad_workspace_bytes(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o, int with_grad);

/*
 * rsvd_block_krylov_grad with the two small SVDs of the forward (of R_K and
 * of R_r, both s_K x s_K with s_K = v (k + p)) carried from a forward call to
 * the backward call on the same A, k, p, v and options, as an autograd
 * forward and backward do.  `kept` is a device FP64 record of
 * rsvd_grad_kept_doubles(k, p, v) entries, owned by the caller:
 *   keep_mode 0: not used (this is rsvd_block_krylov_grad);
 *   keep_mode 1: the call computes the small SVDs and writes them to kept;
 *   keep_mode 2: the call reads them from kept instead of computing them.
 * Everything else, the sketches included, is recomputed either way: on the
 * same inputs the views and reductions are deterministic, so mode 2 equals
 * mode 0 bit for bit when kept came from a mode-1 call on the same inputs;
 * reading a record from other inputs gives wrong results without an error.
 * The workspace of rsvd_grad_workspace_bytes suffices in every mode.
 * RSVD_EINVAL for another mode or a NULL kept with mode 1 or 2.
 */
rsvd_status rsvd_block_krylov_grad_kept(const rsvd_mat* A, int k, int p, int v, const rsvd_opts* o, rsvd_out* out,
                                        double* E, const double* dS, double dE, void* G, int64_t ldg, double* kept,
                                        int keep_mode, void* ws, size_t ws_bytes, hipStream_t stream);

/* Entries of the record of rsvd_block_krylov_grad_kept (0 for invalid sizes). */
size_t rsvd_grad_kept_doubles(int k, int p, int v);

/* ---------------------------------------------------------------------------
 * Batches of independent matrices (Alg. 2 on each).
 *
 * A plan records the launches rsvd_subspace would make for every matrix
 * and groups the i-th launch of all matrices into one batched launch per
 * kernel (the matrix is blockIdx.z), so a call costs a few dozen launches
 * however many matrices it holds.  rsvd_subspace_batched enqueues kernels
 * only (no allocation, copy or synchronization), so a caller may capture it
 * into one HIP graph and replay it; each replay recomputes all outputs.
 * Matrices are FP64 or FP32 (any shapes, leading dimensions and ranks);
 * opts as for rsvd_subspace (f32_mode must be RSVD_F32_MFMA, no trace).
 * ------------------------------------------------------------------------ */
typedef struct rsvd_batch_plan rsvd_batch_plan;   /* opaque, host memory */

/* Tile choices a batch is planned with (the autotuner's search space). */
typedef struct {
    int plan_cus;           /* compute units the contraction-split planning assumes; 0 = no splits */
    int view_mr;            /* 16-row blocks per wave in the views: 1, 2, or 0 = automatic */
} rsvd_batch_tuning;

void rsvd_default_batch_tuning(rsvd_batch_tuning* t);   /* plan_cus = 256, view_mr = 0 */

/* Validates every matrix (as rsvd_subspace would), plans the batch and
 * returns the workspace bytes it needs.  As, ks (ranks) and outs are host
 * arrays of nb entries (1 <= nb <= 65535) whose device pointers must stay
 * valid while the plan is used; tuning may be NULL. */
rsvd_status rsvd_batch_plan_create(int nb, const rsvd_mat* As, const int* ks, int p, int v, const rsvd_opts* o,
                                   const rsvd_out* outs, const rsvd_batch_tuning* tuning, rsvd_batch_plan** plan,
                                   size_t* ws_bytes);

/* Binds a device workspace (256-byte aligned, at least the planned bytes)
 * and uploads the job tables into it; synchronizes `stream`.  Not capturable. */
rsvd_status rsvd_batch_plan_bind(rsvd_batch_plan* plan, void* ws, size_t ws_bytes, hipStream_t stream);

/* Enqueues the whole batch on `stream` (kernel launches only). */
rsvd_status rsvd_subspace_batched(const rsvd_batch_plan* plan, hipStream_t stream);

/* Number of kernel launches one rsvd_subspace_batched call makes. */
int rsvd_batch_plan_launches(const rsvd_batch_plan* plan);

void rsvd_batch_plan_destroy(rsvd_batch_plan* plan);

/* ---------------------------------------------------------------------------
 * Truncated eigendecompositions of the normal matrix J^T J (Sect. 4.2), the
 * inverse-problem use of the views: J^T J ~ V diag(lam2) V^T from v >= 2
 * views of J (m x n, FP64 or FP32, any storage order).
 * ------------------------------------------------------------------------ */
typedef enum {
    RSVD_NORMAL_NYSTROM = 0,    /* Alg. 4 (prolonged sketch): Q_r from v - 2 views (Alg. 3 on J for even v, on
                                   J^T for odd v; orth(Omega) for v = 2), Y_r = J^T (J Q_r), nu = 2.2e-16 ||Y_r||_2,
                                   Y_r += nu Q_r, B = Q_r^T Y_r, C_L = chol((B + B^T)/2), F = C_L^-1 Y_r^T,
                                   [~, Lam, V] = tsvd(F, k), lam2 = max(Lam^2 - nu, 0).  nu and everything after
                                   the views are FP64 on either path */
    RSVD_NORMAL_PINCHED = 1,    /* Alg. 5 (pinched sketch): Q_r from v - 1 views (Alg. 3 on J^T for even v, on J
                                   for odd v), B_c = J Q_r, [lam2, V^] = tevd(B_c^T B_c, k) (taken as the SVD of
                                   B_c's triangular factor), V = Q_r V^ */
    RSVD_NORMAL_SUBSPACE = 2    /* Alg. 2 by the J / J^T rule of Sect. 4.2.1: on J for even v (V its right
                                   factor), on J^T for odd v (V its left factor); lam2 = sigma^2 */
} rsvd_normal_method;

/* V (n x k, row-major, the working type) and lam2 (k FP64 eigenvalues of
 * J^T J, descending); each column of V is sign-fixed so that its entry of
 * largest magnitude is positive (ties: lowest index).  Requires v >= 2,
 * 1 <= k, 0 <= p, k + p <= min(m, n); the Gaussian Omega is drawn as for
 * rsvd_subspace (on J^T, with J^T's column count).  opts: seed, trace,
 * f32_mode, sync_spins (other fields at their defaults, else RSVD_EINVAL). */
rsvd_status rsvd_normal_tevd(const rsvd_mat* J, int k, int p, int v, int method, const rsvd_opts* o, void* V,
                             double* lam2, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of rsvd_normal_tevd (0 when the arguments are invalid). */
size_t rsvd_normal_workspace_bytes(const rsvd_mat* J, int k, int p, int v, int method, const rsvd_opts* o);

/* ---------------------------------------------------------------------------
 * One-view sketches of a matrix given as a stream of linear updates
 * (Sect. 6.1, eq. streammat and eq. streammatmult): A = sum_i H_i is never
 * formed.  The sketches Y = A Omega (m x s) and W = Psi A (s_w x n) of the
 * one-view method are kept in a caller-owned workspace; every update adds
 * H_i Omega to Y and Psi H_i to W, and rsvd_stream_finish runs the one-view
 * post-processing on them exactly as rsvd_single_pass would on the summed
 * matrix (the same Omega, Psi, method and l_c rule).  FP64 or FP32 sketches;
 * the stream handle is host memory owned by the caller.
 * ------------------------------------------------------------------------ */
typedef struct rsvd_stream rsvd_stream;   /* opaque, host memory */

/* Validates the sizes (as rsvd_single_pass would, with s_w <= 512) and the
 * one-view options in o (seed, psi_rows, one_view_method, lc_rule, lc,
 * lc_alpha; no core sketch, refinement or trace: RSVD_EINVAL), creates the
 * handle and returns the workspace bytes it needs.  dtype is RSVD_F64 or
 * RSVD_F32: the type of the sketches and of every update. */
rsvd_status rsvd_stream_create(int64_t m, int64_t n, int k, int p, int dtype, const rsvd_opts* o, rsvd_stream** st,
                               size_t* ws_bytes);

/* Binds a workspace (256-byte aligned, at least the bytes create returned)
 * and starts from A = 0: enqueues the generation of Omega and Psi and the
 * zeroing of Y and W on `stream`.  Binding again restarts the stream. */
rsvd_status rsvd_stream_bind(rsvd_stream* st, void* ws, size_t ws_bytes, hipStream_t stream);

/* A dense update H (h.m x h.n, the dtype of the stream, trans allowed) placed
 * at rows r0.., columns c0.. of A (zero elsewhere):
 * Y[r0 .. r0 + h.m) += H Omega[c0 .. c0 + h.n) and W[:, c0 .. c0 + h.n) +=
 * Psi[:, r0 .. r0 + h.m) H, on the view kernels (H is read twice, the
 * second time mostly from cache).  RSVD_ESHAPE if the block leaves A. */
rsvd_status rsvd_stream_add_dense(rsvd_stream* st, int64_t r0, int64_t c0, const rsvd_mat* H, hipStream_t stream);

/* A sparse update of nnz entries (rows[e], cols[e], vals[e]) (device arrays;
 * vals of the stream's dtype; repeated coordinates add up): Y[r, :] +=
 * v Omega[c, :] and W[:, c] += v Psi[:, r], as floating-point atomic adds (the
 * order of the additions, hence the last bits, is not fixed).  Entries
 * outside A are skipped and set bit 5 of the status word (rsvd_device_status
 * then returns RSVD_ESHAPE). */
rsvd_status rsvd_stream_add_entries(rsvd_stream* st, int64_t nnz, const int64_t* rows, const int64_t* cols,
                                    const void* vals, hipStream_t stream);

/* The one-view post-processing (Alg. 7 or Alg. 8 with the l_c rule of the
 * create options) of the current sketches into out (U m x k, S k, V n x k).
 * The sketches are left as they are, so more updates and further finishes
 * may follow.  rsvd_device_status and rsvd_one_view_lc read the bound
 * workspace. */
rsvd_status rsvd_stream_finish(rsvd_stream* st, rsvd_out* out, hipStream_t stream);

void rsvd_stream_destroy(rsvd_stream* st);

/* Waits for `stream`, then reads the status word a previous call left in
 * `ws`: RSVD_EBREAKDOWN if a non-finite value was produced or the small
 * SVD's device-wide barrier timed out (bit 2 or bit 4), else RSVD_ESHAPE if a
 * streamed update entry lay outside A (bit 5), RSVD_OK otherwise.  If flags
 * is not NULL it receives the raw word
 * (bit 0: a shifted Cholesky was needed; bit 1: a Cholesky pivot stayed
 * non-positive after the shift; bit 2: non-finite values (singular values, or
 * a sketch whose Gram is not finite); bit 3:
 * rsvd_block_krylov_grad met a Krylov basis below full numerical rank; bit 4:
 * the workgroups of the multi-workgroup small SVD did not all meet at a
 * device-wide barrier within its bounded wait, so the result is invalid;
 * bit 5: a streamed update entry outside A was skipped). */
rsvd_status rsvd_device_status(const void* ws, hipStream_t stream, uint32_t* flags);

/* Sizes of the extended one-view sketch (Sect. 6.7) for a storage budget of
 * T = budget columns' worth of thin storage, the choice the paper found best
 * (eq. bwzafac8): l_1 = l_2 = floor(0.8 floor(T/2 - k)) and the largest core
 * size s_c with (2k + l_1 + l_2 + 1)(m + n) + s_c (s_c + 2) <= T (m + n),
 * capped at min(m, n).  Call rsvd_single_pass with p = *l1 and
 * core_rows = *sc.  RSVD_ESHAPE when the budget leaves l_1 < 0 or
 * s_c < k + l_1; host computation only. */
rsvd_status rsvd_extended_sizes(int k, int64_t budget, int64_t m, int64_t n, int* l1, int64_t* sc);

/* Waits for `stream`, then reads the l_c a previous rsvd_single_pass (or
 * rsvd_stream_finish) call with this workspace used in its one-view
 * post-processing (Sect. 6.6): the fixed or ratio value, or the one the
 * minimum-variance rule chose on the device; l_1 = p for the default path. */
rsvd_status rsvd_one_view_lc(const void* ws, hipStream_t stream, int* lc);

/* Static description of a status code. */
const char* rsvd_status_string(rsvd_status s);

/* ---------------------------------------------------------------------------
 * Building blocks of the views, exported for tests and measurement.  Same
 * conventions as above; they enqueue on `stream` and return immediately.
 * ------------------------------------------------------------------------ */

/* Gaussian test matrix (Sect. 2 randn) of `rows` x `cols` written row-major
 * to out (leading dimension ld): entry (r, c) has long index r and short
 * index c when long_is_row, else long c and short r.  dtype is RSVD_F64 or
 * RSVD_F32 (FP32 values are the round-to-nearest FP32 of the FP64 value). */
rsvd_status rsvd_gaussian(uint64_t seed, uint32_t tag, uint32_t batch, int64_t rows, int64_t cols,
                          int long_is_row, int dtype, void* out, int64_t ld, hipStream_t stream);

/* One range view Y = A X.  Thin matrices are passed as panels, i.e. their
 * transposes stored row-major: XT is X^T (s x n, leading dimension n) and
 * YT receives Y^T (s x m, leading dimension m).  The working dtype of the
 * panels is FP64 for an FP64 A and FP32 otherwise.  o (may be NULL) selects
 * the FP32 mode (f32_mode) and, for a BF16/FP8 A, the cheap (refine = 0) or
 * FP32-accurate (refine = 1) thin operand. */
rsvd_status rsvd_view_range(const rsvd_mat* A, int s, const void* X, void* Y, const rsvd_opts* o,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* One co-range view Z = A^T Y with YT = Y^T (s x m) and ZT = Z^T (s x n). */
rsvd_status rsvd_view_corange(const rsvd_mat* A, int s, const void* Y, void* Z, const rsvd_opts* o,
                              void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace for the two view entry points above. */
size_t rsvd_view_workspace_bytes(const rsvd_mat* A, int s, const rsvd_opts* o);

/* Raw Philox4x32-10 output for `count` counters: ctr holds the four counter
 * words word-major (ctr[w * count + i], device memory), out receives the
 * four output words the same way.  Exported so the generator can be checked
 * bit for bit against its published known answers. */
rsvd_status rsvd_philox_words(const uint32_t* ctr, int64_t count, uint32_t key0, uint32_t key1, uint32_t* out,
                              hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_H */
