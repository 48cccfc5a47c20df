// Small dense steps after the views: the SVD of the s x s core factor
// (tsvd of R_r or R_c in Alg. 2, of R_K / R_r in the Krylov methods) and the
// lifts U = Q_c U^_k, V = Q_r V^_k.
#include <algorithm>

#include "common.h"
#include "launch.h"
#include "small.h"

namespace {

// ---------------------------------------------------------------------------
// SVD of an s x s FP64 matrix M = L diag(sigma) Rv^T by one-sided Jacobi
// (Hestenes): the columns of W = M J are orthogonalized by plane rotations in
// round-robin order until every pair satisfies |w_p . w_q| <= tol ||w_p|| ||w_q||.
// Then sigma_c = ||w_c||, L[:, c] = w_c / sigma_c and, since M^T L = Rv diag(sigma),
// Rv[:, c] = M^T w_c / sigma_c^2.  Outputs are sorted by decreasing sigma.
// W is stored column by column (W[c * s + r]) in LDS (orders up to 128; wider
// matrices go to the block kernel below).
// A group of TPP threads rotates one column pair per step; each thread keeps
// its RPT rows of both columns in registers for the whole step.
// ---------------------------------------------------------------------------
template <int RPT>
__device__ __forceinline__ void jacobi_svd_body(double* __restrict__ W, const double* __restrict__ M, int s, int tpp,
                                                double* __restrict__ L, double* __restrict__ Rv,
                                                double* __restrict__ sigma, uint32_t* status) {
    __shared__ int rotated;
    __shared__ double sig_sh[1024];
    __shared__ int rank_sh[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < s * s; e += nt) {
        const int r = e / s, c = e % s;
        W[c * s + r] = M[e];
    }
    const int sp = s + (s & 1);          // even number of slots (slot s is a dummy when s is odd)
    const int npairs = sp / 2;
    const int groups = nt / tpp;
    const int grp = tid / tpp, gl = tid % tpp;
    const double tol = (double)s * 2.220446049250313e-16;
    __syncthreads();

    int sweeps = 0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int step = 0; step < sp - 1; ++step) {
            for (int pr = grp; pr < npairs; pr += groups) {
                const int qa = pr, qb = sp - 1 - pr;
                const int p = qa == 0 ? 0 : 1 + (qa - 1 + step) % (sp - 1);
                const int q = 1 + (qb - 1 + step) % (sp - 1);
                const bool live = p < s && q < s;
                double* wp = W + (int64_t)(live ? p : 0) * s;
                double* wq = W + (int64_t)(live ? q : 0) * s;
                double x[RPT], y[RPT];
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = gl + i * tpp;
                    const bool ok = live && r < s;
                    x[i] = ok ? wp[r] : 0.0;
                    y[i] = ok ? wq[r] : 0.0;
                }
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    al += x[i] * x[i];
                    be += y[i] * y[i];
                    ga += x[i] * y[i];
                }
                for (int off = tpp / 2; off > 0; off >>= 1) {
                    al += __shfl_xor(al, off, tpp);
                    be += __shfl_xor(be, off, tpp);
                    ga += __shfl_xor(ga, off, tpp);
                }
                if (live && al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t);
                    const double sn = c * t;
#pragma unroll
                    for (int i = 0; i < RPT; ++i) {
                        const int r = gl + i * tpp;
                        if (r < s) {
                            wp[r] = c * x[i] - sn * y[i];
                            wq[r] = sn * x[i] + c * y[i];
                        }
                    }
                    if (gl == 0) rotated = 1;
                }
            }
            __syncthreads();
        }
        const int any = rotated;
        sweeps = sweep + 1;
        __syncthreads();
        if (!any) break;
    }
    if (tid == 0 && status) status[4] = (uint32_t)sweeps;  // diagnostic: sweeps of the last small SVD

    // singular values and their order
    for (int c = tid; c < s; c += nt) {
        double acc = 0.0;
        for (int r = 0; r < s; ++r) acc += W[(int64_t)c * s + r] * W[(int64_t)c * s + r];
        sig_sh[c] = sqrt(acc);
    }
    __syncthreads();
    for (int c = tid; c < s; c += nt) {
        const double v = sig_sh[c];
        int rk = 0;
        for (int d = 0; d < s; ++d) {
            const double u = sig_sh[d];
            rk += (u > v) || (u == v && d < c);
        }
        rank_sh[c] = rk;
        sigma[rk] = v;
        if (!isfinite(v)) rsvd_flag(status, RSVD_FLAG_NONFINITE);
    }
    __syncthreads();
    for (int e = tid; e < s * s; e += nt) {
        const int r = e / s, c = e % s;
        const double sv = sig_sh[c];
        L[(int64_t)r * s + rank_sh[c]] = sv > 0.0 ? W[(int64_t)c * s + r] / sv : 0.0;
    }
    for (int e = tid; e < s * s; e += nt) {
        const int x = e / s, c = e % s;
        const double sv = sig_sh[c];
        double acc = 0.0;
        for (int r = 0; r < s; ++r) acc += M[(int64_t)r * s + x] * W[(int64_t)c * s + r];
        Rv[(int64_t)x * s + rank_sh[c]] = sv > 0.0 ? acc / (sv * sv) : 0.0;
    }
}

// One instantiation per placement of W (LDS or global scratch), so that
// every access compiles to LDS or global instructions.
template <int RPT, bool IN_LDS>
struct jacobi_svd_kernel_op {
    static constexpr int kThreads = 1024;
    struct Args {
        const double*  M;
        int s;
        int tpp;
        double*  L;
        double*  Rv;
        double*  sigma;
        double*  gscratch;
        uint32_t* status;
        const int* enable;
    };
    static Args make(const double*  M, int s, int tpp, double*  L, double*  Rv, double*  sigma, double*  gscratch, uint32_t* status, const int* enable) {
        Args a_;
        a_.M = M;
        a_.s = s;
        a_.tpp = tpp;
        a_.L = L;
        a_.Rv = Rv;
        a_.sigma = sigma;
        a_.gscratch = gscratch;
        a_.status = status;
        a_.enable = enable;
        return a_;
    }
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto M = args_.M;
        const auto s = args_.s;
        const auto tpp = args_.tpp;
        const auto L = args_.L;
        const auto Rv = args_.Rv;
        const auto sigma = args_.sigma;
        const auto gscratch = args_.gscratch;
        const auto status = args_.status;
        const auto enable = args_.enable;
        if (enable && *enable == 0) return;
        extern __shared__ double lds[];
        if constexpr (IN_LDS) jacobi_svd_body<RPT>(lds, M, s, tpp, L, Rv, sigma, status);
        else jacobi_svd_body<RPT>(gscratch, M, s, tpp, L, Rv, sigma, status);
    }
};

// ---------------------------------------------------------------------------
// SVD of an s x s FP64 matrix M = L diag(sigma) Rv^T by block one-sided
// Jacobi.  The columns of W = M (padded with zero columns to whole blocks)
// form blocks of JB columns; each step pairs the blocks round-robin, and one
// wave per block pair (2 JB columns C) forms the Gram G = C^T C on FP64
// matrix cores, runs one cyclic Jacobi sweep on G (JP - 1 rounds of JB
// disjoint plane rotations, accumulated into J) and applies C <- C J on
// matrix cores.  Steps repeat until a whole sweep finds every block pair
// orthogonal to |G_ac| <= s eps sqrt(G_aa G_cc).  Then sigma_c = ||w_c||,
// L[:, c] = w_c / sigma_c and Rv[:, c] = M^T w_c / sigma_c^2, sorted by
// decreasing sigma.  A sweep needs 2 s / JB - 1 workgroup barriers instead
// of the s - 1 of the column-pair method.  W lives in LDS when it fits,
// else in global scratch (s x round_up(s, 2 JB) doubles).
// ---------------------------------------------------------------------------
constexpr int JB = 8;
constexpr int JP = 2 * JB;
constexpr int JWAVES = 16;

__device__ __forceinline__ int rr_slot_index(int slot, int round, int n) {
    // index held by `slot` in round `round` of the round-robin on n indices
    return slot == 0 ? 0 : 1 + (slot - 1 + round) % (n - 1);
}

template <bool IN_LDS>
__device__ __forceinline__ void block_jacobi_body(double* __restrict__ W, const double* __restrict__ M, int s,
                                                  double* __restrict__ L, double* __restrict__ Rv,
                                                  double* __restrict__ sigma, uint32_t* status) {
    __shared__ double Gs[JWAVES][JP][JP + 1];
    __shared__ double Js[JWAVES][JP][JP + 1];
    __shared__ double coef_a[JWAVES][JP], coef_b[JWAVES][JP];
    __shared__ int partner[JWAVES][JP];
    __shared__ int rotated;
    __shared__ double sig_sh[512];
    __shared__ int rank_sh[512];
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int sp = (s + JP - 1) / JP * JP;
    const int nb = sp / JB;
    for (int e = tid; e < s * sp; e += nt) {
        const int c = e / s, r = e % s;
        W[e] = c < s ? M[(int64_t)r * s + c] : 0.0;
    }
    const double tol = (double)s * 2.220446049250313e-16;
    double (*G)[JP + 1] = Gs[wave];
    double (*J)[JP + 1] = Js[wave];
    __syncthreads();

    int sweeps = 0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int step = 0; step < nb - 1; ++step) {
            for (int pr = wave; pr < nb / 2; pr += nwaves) {
                const int P = rr_slot_index(pr, step, nb), Q = rr_slot_index(nb - 1 - pr, step, nb);
                auto col = [&](int a) { return a < JB ? P * JB + a : Q * JB + (a - JB); };
                // G = C^T C: lane (g, x) supplies C[r0 + g][x] as both operands; 16 loads are
                // issued before their matrix-core steps so that they overlap
                doublex4 acc = {0, 0, 0, 0};
                const double* cx = W + (int64_t)col(x) * s;
                for (int r0 = 0; r0 < s; r0 += 64) {
                    double v[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) v[u] = (r0 + 4 * u + g < s) ? cx[r0 + 4 * u + g] : 0.0;
#pragma unroll
                    for (int u = 0; u < 16; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u], v[u], acc, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) G[g + 4 * r][x] = acc[r];
                for (int e = lane; e < JP * JP; e += 64) J[e / JP][e % JP] = (e / JP == e % JP) ? 1.0 : 0.0;
                __builtin_amdgcn_wave_barrier();
                // largest scaled off-diagonal entry
                double off = 0.0;
                for (int e = lane; e < JP * JP; e += 64) {
                    const int a = e / JP, c = e % JP;
                    const double d = G[a][a] * G[c][c];
                    if (a != c && d > 0.0) off = fmax(off, fabs(G[a][c]) / sqrt(d));
                }
                for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o));
                if (!(off > tol)) continue;   // uniform over the wave
                if (lane == 0) rotated = 1;
                // one cyclic Jacobi sweep on G, rotations accumulated in J
                for (int rd = 0; rd < JP - 1; ++rd) {
                    if (lane < JB) {
                        const int p = rr_slot_index(lane, rd, JP), q = rr_slot_index(JP - 1 - lane, rd, JP);
                        const double al = G[p][p], be = G[q][q], ga = G[p][q];
                        double c = 1.0, sn = 0.0;
                        if (al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                            const double zeta = (be - al) / (2.0 * ga);
                            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                            c = 1.0 / sqrt(1.0 + t * t);
                            sn = c * t;
                        }
                        // new column p = c col_p - sn col_q, new column q = c col_q + sn col_p
                        coef_a[wave][p] = c;
                        coef_b[wave][p] = -sn;
                        partner[wave][p] = q;
                        coef_a[wave][q] = c;
                        coef_b[wave][q] = sn;
                        partner[wave][q] = p;
                    }
                    __builtin_amdgcn_wave_barrier();
                    double gn[JP * JP / 64], jn[JP * JP / 64];
#pragma unroll
                    for (int t = 0; t < JP * JP / 64; ++t) {
                        const int e = lane + 64 * t, i = e / JP, j = e % JP;
                        const int pi = partner[wave][i], pj = partner[wave][j];
                        const double ai = coef_a[wave][i], bi = coef_b[wave][i];
                        const double aj = coef_a[wave][j], bj = coef_b[wave][j];
                        gn[t] = ai * (aj * G[i][j] + bj * G[i][pj]) + bi * (aj * G[pi][j] + bj * G[pi][pj]);
                        jn[t] = aj * J[i][j] + bj * J[i][pj];
                    }
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int t = 0; t < JP * JP / 64; ++t) {
                        const int e = lane + 64 * t, i = e / JP, j = e % JP;
                        G[i][j] = gn[t];
                        J[i][j] = jn[t];
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                // C <- C J, two 16-row tiles at a time (a tile reads and writes only its own rows)
                double jv[JP / 4];
#pragma unroll
                for (int kq = 0; kq < JP / 4; ++kq) jv[kq] = J[4 * kq + g][x];
                for (int r0 = 0; r0 < s; r0 += 32) {
                    double av[2][JP / 4];
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int kq = 0; kq < JP / 4; ++kq) {
                            const int row = r0 + 16 * h + x;
                            av[h][kq] = row < s ? W[(int64_t)col(4 * kq + g) * s + row] : 0.0;
                        }
                    doublex4 o[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int kq = 0; kq < JP / 4; ++kq)
                            o[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][kq], jv[kq], o[h], 0, 0, 0);
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = r0 + 16 * h + g + 4 * r;
                            if (row < s) W[(int64_t)col(x) * s + row] = o[h][r];
                        }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
        }
        const int any = rotated;
        sweeps = sweep + 1;
        __syncthreads();
        if (!any) break;
    }
    if (tid == 0 && status) status[4] = (uint32_t)sweeps;  // diagnostic: sweeps of the last small SVD

    // column norms: one wave per column, lanes over rows
    for (int c = wave; c < sp; c += nwaves) {
        double acc = 0.0;
        for (int r = lane; r < s; r += 64) acc += W[(int64_t)c * s + r] * W[(int64_t)c * s + r];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) sig_sh[c] = sqrt(acc);
    }
    __syncthreads();
    for (int c = tid; c < sp; c += nt) {
        const double v = sig_sh[c];
        int rk = 0;
        for (int d = 0; d < sp; ++d) {
            const double u = sig_sh[d];
            rk += (u > v) || (u == v && d < c);
        }
        rank_sh[c] = rk;
        if (rk < s) {
            sigma[rk] = v;
            if (!isfinite(v)) rsvd_flag(status, RSVD_FLAG_NONFINITE);
        }
    }
    __syncthreads();
    for (int e = tid; e < s * sp; e += nt) {
        const int c = e / s, r = e % s;
        const int rk = rank_sh[c];
        if (rk >= s) continue;
        const double sv = sig_sh[c];
        L[(int64_t)r * s + rk] = sv > 0.0 ? W[e] / sv : 0.0;
    }
    // Rv[x][rank(c)] = (M^T W)[x][c] / sigma_c^2 on FP64 matrix cores, one 16 x 16 tile per wave:
    // lane (g, i) supplies M^T[x0 + i][k = r0 + g] = M[r0 + g][x0 + i] and W[c0 + i][r0 + g]
    const int ntx = (s + 15) / 16, ntc = sp / 16;
    for (int tile = wave; tile < ntx * ntc; tile += nwaves) {
        const int x0 = (tile / ntc) * 16, c0 = (tile % ntc) * 16;
        doublex4 acc = {0, 0, 0, 0};
        for (int r0 = 0; r0 < s; r0 += 64) {
            double mv[16], wv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int r = r0 + 4 * u + g;
                mv[u] = (r < s && x0 + x < s) ? M[(int64_t)r * s + x0 + x] : 0.0;
                wv[u] = r < s ? W[(int64_t)(c0 + x) * s + r] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(mv[u], wv[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int xx = x0 + g + 4 * r, c = c0 + x;
            if (xx >= s) continue;
            const int rk = rank_sh[c];
            if (rk >= s) continue;
            const double sv = sig_sh[c];
            Rv[(int64_t)xx * s + rk] = sv > 0.0 ? acc[r] / (sv * sv) : 0.0;
        }
    }
}

template <bool IN_LDS>
struct block_jacobi_kernel_op {
    static constexpr int kThreads = 1024;
    struct Args {
        const double* M;
        int s;
        double* L;
        double* Rv;
        double* sigma;
        double* gscratch;
        uint32_t* status;
        const int* enable;
    };
    static Args make(const double* M, int s, double* L, double* Rv, double* sigma, double* gscratch, uint32_t* status,
                     const int* enable) {
        return Args{M, s, L, Rv, sigma, gscratch, status, enable};
    }
    static __device__ __forceinline__ void run(const VGrid vg, const Args& a) {
        (void)vg;
        if (a.enable && *a.enable == 0) return;
        extern __shared__ double lds_w[];
        if constexpr (IN_LDS) block_jacobi_body<true>(lds_w, a.M, a.s, a.L, a.Rv, a.sigma, a.status);
        else block_jacobi_body<false>(a.gscratch, a.M, a.s, a.L, a.Rv, a.sigma, a.status);
    }
};

// out[x][c] = sum_a P[a][x] F[a][c] for c < k  (P: s x len panel, F: s x ldf FP64);
// F is staged through LDS 256 rows at a time.
template <typename TP, typename TO>
struct lift_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const TP*  P;
        int64_t ldp;
        int s;
        int64_t len;
        const double*  F;
        int ldf;
        int k;
        TO*  out;
        int64_t ldo;
    };
    static Args make(const TP*  P, int64_t ldp, int s, int64_t len, const double*  F, int ldf, int k, TO*  out, int64_t ldo) {
        Args a_;
        a_.P = P;
        a_.ldp = ldp;
        a_.s = s;
        a_.len = len;
        a_.F = F;
        a_.ldf = ldf;
        a_.k = k;
        a_.out = out;
        a_.ldo = ldo;
        return a_;
    }
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto P = args_.P;
        const auto ldp = args_.ldp;
        const auto s = args_.s;
        const auto len = args_.len;
        const auto F = args_.F;
        const auto ldf = args_.ldf;
        const auto k = args_.k;
        const auto out = args_.out;
        const auto ldo = args_.ldo;
        constexpr int KC = 32;
        __shared__ double fs[256 * KC];
        const int c0 = vg.by * KC;
        const int kc = std::min(KC, k - c0);
        const int64_t x = (int64_t)vg.bx * blockDim.x + threadIdx.x;
        double acc[KC];
    #pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = 0.0;
        for (int a0 = 0; a0 < s; a0 += 256) {
            const int sa = std::min(256, s - a0);
            __syncthreads();
            for (int e = threadIdx.x; e < sa * KC; e += blockDim.x) {
                const int a = e / KC, c = e % KC;
                fs[e] = (c < kc) ? F[(int64_t)(a0 + a) * ldf + c0 + c] : 0.0;
            }
            __syncthreads();
            if (x < len) {
                for (int a = 0; a < sa; ++a) {
                    const double pv = (double)P[(int64_t)(a0 + a) * ldp + x];
    #pragma unroll
                    for (int c = 0; c < KC; ++c) acc[c] += pv * fs[a * KC + c];
                }
            }
        }
        if (x >= len) return;
        TO* o = out + x * ldo + c0;
    #pragma unroll
        for (int c = 0; c < KC; ++c)
            if (c < kc) o[c] = (TO)acc[c];
    }
};

// Per row chunk and column: the entry of largest magnitude (first on ties).
template <typename T>
struct sign_partial_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const T*  U;
        int64_t len;
        int k;
        int64_t ldu;
        int64_t rows_per_chunk;
        double*  pval;
        int64_t*  pidx;
    };
    static Args make(const T*  U, int64_t len, int k, int64_t ldu, int64_t rows_per_chunk, double*  pval, int64_t*  pidx) {
        Args a_;
        a_.U = U;
        a_.len = len;
        a_.k = k;
        a_.ldu = ldu;
        a_.rows_per_chunk = rows_per_chunk;
        a_.pval = pval;
        a_.pidx = pidx;
        return a_;
    }
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto U = args_.U;
        const auto len = args_.len;
        const auto k = args_.k;
        const auto ldu = args_.ldu;
        const auto rows_per_chunk = args_.rows_per_chunk;
        const auto pval = args_.pval;
        const auto pidx = args_.pidx;
        const int64_t r0 = (int64_t)vg.bx * rows_per_chunk;
        const int64_t r1 = std::min<int64_t>(len, r0 + rows_per_chunk);
        for (int c = threadIdx.x; c < k; c += blockDim.x) {
            double best = -1.0, bval = 0.0;
            int64_t bidx = -1;
            for (int64_t r = r0; r < r1; ++r) {
                const double v = (double)U[r * ldu + c];
                if (fabs(v) > best) {
                    best = fabs(v);
                    bval = v;
                    bidx = r;
                }
            }
            pval[(int64_t)vg.bx * k + c] = bval;
            pidx[(int64_t)vg.bx * k + c] = bidx;
        }
    }
};

// One wave per column: the first chunk (in row order) holding the largest
// magnitude decides the sign.
struct sign_final_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const double*  pval;
        const int64_t*  pidx;
        int nchunks;
        int k;
        double*  sgn;
    };
    static Args make(const double*  pval, const int64_t*  pidx, int nchunks, int k, double*  sgn) {
        Args a_;
        a_.pval = pval;
        a_.pidx = pidx;
        a_.nchunks = nchunks;
        a_.k = k;
        a_.sgn = sgn;
        return a_;
    }
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto pval = args_.pval;
        const auto pidx = args_.pidx;
        const auto nchunks = args_.nchunks;
        const auto k = args_.k;
        const auto sgn = args_.sgn;
        const int lane = threadIdx.x & 63;
        const int c = vg.bx * 4 + (threadIdx.x >> 6);
        if (c >= k) return;
        double best = -1.0, bval = 0.0;
        int bchunk = 1 << 30;
        for (int p = lane; p < nchunks; p += 64) {
            const double v = pval[(int64_t)p * k + c];
            if (pidx[(int64_t)p * k + c] >= 0 && fabs(v) > best) {
                best = fabs(v);
                bval = v;
                bchunk = p;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off), ov = __shfl_xor(bval, off);
            const int oc = __shfl_xor(bchunk, off);
            if (ob > best || (ob == best && oc < bchunk)) {
                best = ob;
                bval = ov;
                bchunk = oc;
            }
        }
        if (lane == 0) sgn[c] = bval < 0.0 ? -1.0 : 1.0;
    }
};

template <typename T>
struct apply_sign_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        T*  X;
        int64_t len;
        int k;
        int64_t ldx;
        const double*  sgn;
    };
    static Args make(T*  X, int64_t len, int k, int64_t ldx, const double*  sgn) {
        Args a_;
        a_.X = X;
        a_.len = len;
        a_.k = k;
        a_.ldx = ldx;
        a_.sgn = sgn;
        return a_;
    }
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto X = args_.X;
        const auto len = args_.len;
        const auto k = args_.k;
        const auto ldx = args_.ldx;
        const auto sgn = args_.sgn;
        const int64_t total = len * k;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)vg.gx * blockDim.x) {
            const int64_t r = e / k;
            const int c = (int)(e % k);
            if (sgn[c] < 0.0) X[r * ldx + c] = -X[r * ldx + c];
        }
    }
};

struct copy_f64_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const double*  src;
        double*  dst;
        int64_t count;
    };
    static Args make(const double*  src, double*  dst, int64_t count) {
        Args a_;
        a_.src = src;
        a_.dst = dst;
        a_.count = count;
        return a_;
    }
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto src = args_.src;
        const auto dst = args_.dst;
        const auto count = args_.count;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)vg.gx * blockDim.x)
            dst[e] = src[e];
    }
};

}  // namespace

static size_t block_jacobi_w_doubles(int s) { return (size_t)s * ((s + JP - 1) / JP * JP); }

// Up to 128 columns the column-pair kernel runs with W in LDS (its s - 1
// barriers per sweep are cheap there); wider matrices use the block kernel
// with W in global scratch (2 s / JB - 1 barriers per sweep).
bool jacobi_fits_lds(int s) { return (size_t)s * s * sizeof(double) <= 128 * 1024; }

size_t small_svd_scratch_doubles(int s) { return jacobi_fits_lds(s) ? 0 : block_jacobi_w_doubles(s); }

rsvd_status run_small_svd(const double* M, int s, double* L, double* Rv, double* sigma, double* gscratch,
                          uint32_t* status, const int* enable, hipStream_t st) {
    launch_phase();
    if (s > 512 || s < 1) return RSVD_EUNSUPPORTED;
    if (jacobi_fits_lds(s)) {
        constexpr int RPT = 16;                          // rows of a column pair held per thread
        const int npairs = (s + (s & 1)) / 2;
        int tpp = 1;
        while (tpp < 16 && tpp * RPT < s) tpp <<= 1;     // threads per pair
        const int threads = (int)std::min<int64_t>(1024, round_up((int64_t)npairs * tpp, 64));
        const size_t shmem = (size_t)s * s * sizeof(double);
        if (hipFuncSetAttribute(op_single_fn<jacobi_svd_kernel_op<RPT, true>>(),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem) != hipSuccess)
            return RSVD_EHIP;
        launch_op<jacobi_svd_kernel_op<RPT, true>>(dim3(1), dim3(threads), shmem, st,
                                                   jacobi_svd_kernel_op<RPT, true>::make(M, s, tpp, L, Rv, sigma,
                                                                                         nullptr, status, enable));
    } else {
        if (!gscratch) return RSVD_EINVAL;
        launch_op<block_jacobi_kernel_op<false>>(dim3(1), dim3(64 * JWAVES), 0, st,
                                                 block_jacobi_kernel_op<false>::make(M, s, L, Rv, sigma, gscratch,
                                                                                     status, enable));
    }
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_lift(int dtype_p, const void* P, int64_t ldp, int s, int64_t len, const double* F, int ldf, int k,
                     int dtype_o, void* out, int64_t ldo, hipStream_t st) {
    launch_phase();
    if (s > 512) return RSVD_EUNSUPPORTED;
    dim3 grid((unsigned)ceil_div(len, 256), (unsigned)ceil_div(k, 32));
#define RSVD_LIFT(TP, TO)                                                                                          \
    launch_op<lift_kernel_op<TP, TO>>(grid, dim3(256), 0, st, lift_kernel_op<TP, TO>::make((const TP*)P, ldp, s, len, F, ldf, k, (TO*)out, \
                       ldo))
    if (dtype_p == RSVD_F32 && dtype_o == RSVD_F32) RSVD_LIFT(float, float);
    else if (dtype_p == RSVD_F64 && dtype_o == RSVD_F64) RSVD_LIFT(double, double);
    else if (dtype_p == RSVD_F64 && dtype_o == RSVD_F32) RSVD_LIFT(double, float);
    else return RSVD_EUNSUPPORTED;
#undef RSVD_LIFT
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

int64_t sign_chunks(int64_t len) { return std::max<int64_t>(1, std::min<int64_t>(256, ceil_div(len, 256))); }

rsvd_status run_signs(int dtype, void* U, int64_t m, void* V, int64_t n, int k, double* pval, int64_t* pidx,
                      double* sgn, hipStream_t st) {
    launch_phase();
    const int64_t nch = sign_chunks(m);
    const int64_t rows = ceil_div(m, nch);
    const unsigned gu = (unsigned)std::min<int64_t>(ceil_div(m * k, 256), 8192);
    const unsigned gv = (unsigned)std::min<int64_t>(ceil_div(n * k, 256), 8192);
    if (dtype == RSVD_F64) {
        launch_op<sign_partial_kernel_op<double>>(dim3((unsigned)nch), dim3(256), 0, st, sign_partial_kernel_op<double>::make((const double*)U, m, k, (int64_t)k, rows, pval, pidx));
        launch_op<sign_final_kernel_op>(dim3((unsigned)ceil_div(k, 4)), dim3(256), 0, st, sign_final_kernel_op::make(pval, pidx, (int)nch, k, sgn));
        launch_op<apply_sign_kernel_op<double>>(dim3(gu), dim3(256), 0, st, apply_sign_kernel_op<double>::make((double*)U, m, k, (int64_t)k, sgn));
        launch_op<apply_sign_kernel_op<double>>(dim3(gv), dim3(256), 0, st, apply_sign_kernel_op<double>::make((double*)V, n, k, (int64_t)k, sgn));
    } else {
        launch_op<sign_partial_kernel_op<float>>(dim3((unsigned)nch), dim3(256), 0, st, sign_partial_kernel_op<float>::make((const float*)U, m, k, (int64_t)k, rows, pval, pidx));
        launch_op<sign_final_kernel_op>(dim3((unsigned)ceil_div(k, 4)), dim3(256), 0, st, sign_final_kernel_op::make(pval, pidx, (int)nch, k, sgn));
        launch_op<apply_sign_kernel_op<float>>(dim3(gu), dim3(256), 0, st, apply_sign_kernel_op<float>::make((float*)U, m, k, (int64_t)k, sgn));
        launch_op<apply_sign_kernel_op<float>>(dim3(gv), dim3(256), 0, st, apply_sign_kernel_op<float>::make((float*)V, n, k, (int64_t)k, sgn));
    }
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_copy_f64(const double* src, double* dst, int64_t count, hipStream_t st) {
    launch_phase();
    launch_op<copy_f64_kernel_op>(dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(count, 256), 1024))), dim3(256), 0, st, copy_f64_kernel_op::make(src, dst, count));
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}
