// Small dense steps after the views: the SVD of the s x s core factor
// (tsvd of R_r or R_c in Alg. 2, of R_K / R_r in the Krylov methods) and the
// lifts U = Q_c U^_k, V = Q_r V^_k.
#include <algorithm>
#include <utility>

#include "common.h"
#include "launch.h"
#include "small.h"
#include "orth.h"

namespace {

// Lanes of one wave exchanging data through LDS: the wave runs in lockstep and
// its LDS operations complete in order, so no instruction is needed, but the
// compiler must not move a load above another lane's store (it may, across a
// bare wave barrier, when the store sits in a branch this lane does not take).
// The wavefront-scope fences make the exchange a release/acquire pair.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Plane rotation that makes columns x, y (al = x.x, be = y.y, ga = x.y)
// orthogonal: the smaller root t of t^2 + 2 zeta t - 1 = 0, zeta =
// (be - al) / (2 ga), written as t = sz |2 ga| / (|d| + sqrt(d^2 + 4 ga^2))
// with d = be - al and sz the sign of zeta (+1 for zeta = 0), which takes one
// square root and one division; c = 1 / sqrt(1 + t^2), sn = c t.  Returns
// false (c = 1, sn = 0) when |ga| <= tol sqrt(al be).
__device__ __forceinline__ bool jacobi_rotation(double al, double be, double ga, double tol, double& c, double& sn) {
    c = 1.0;
    sn = 0.0;
    if (!(al > 0.0 && be > 0.0 && ga * ga > tol * tol * al * be)) return false;
    const double d = be - al;
    const double two_ga = 2.0 * ga;
    const double sz = (d == 0.0 || ((d > 0.0) == (ga > 0.0))) ? 1.0 : -1.0;
    const double t = sz * fabs(two_ga) / (fabs(d) + sqrt(d * d + two_ga * two_ga));
    c = rsqrt(1.0 + t * t);
    sn = c * t;
    return true;
}

// Same rotation with the square root and the divisions taken from the
// hardware reciprocal square root and reciprocal estimates.  Only the angle
// carries their error (a slightly inexact angle slows convergence but leaves
// W = M J exact up to rounding); c is refined by two Newton steps for
// 1 / sqrt(1 + t^2), so that c^2 + sn^2 = 1 to rounding and every rotation is
// orthogonal.  Inputs far from 1 in scale take the exact formula.
__device__ __forceinline__ bool jacobi_rotation_fast(double al, double be, double ga, double tol, double& c,
                                                     double& sn) {
    c = 1.0;
    sn = 0.0;
    if (!(al > 0.0 && be > 0.0 && ga * ga > tol * tol * al * be)) return false;
    const double d = be - al;
    const double two_ga = 2.0 * ga;
    const double r2 = d * d + two_ga * two_ga;
    if (!(r2 > 0x1p-900 && r2 < 0x1p900)) return jacobi_rotation(al, be, ga, tol, c, sn);
    const double sz = (d == 0.0 || ((d > 0.0) == (ga > 0.0))) ? 1.0 : -1.0;
    const double r = r2 * __builtin_amdgcn_rsq(r2);
    const double t = sz * fabs(two_ga) * __builtin_amdgcn_rcp(fabs(d) + r);
    const double u = 1.0 + t * t;
    double y = __builtin_amdgcn_rsq(u);
    y = y * (1.5 - 0.5 * u * y * y);
    y = y * (1.5 - 0.5 * u * y * y);
    c = y;
    sn = y * t;
    return true;
}

// ---------------------------------------------------------------------------
// SVD of an s x s FP64 matrix M = L diag(sigma) Rv^T by block one-sided
// Jacobi.  The columns of W = M (padded with zero columns to whole blocks)
// form blocks of JB columns; each step pairs the blocks round-robin.  For
// every block pair (2 JB columns C) one wave forms the Gram G = C^T C on FP64
// matrix cores; then one cyclic Jacobi sweep on G (JP - 1 rounds of JB
// disjoint plane rotations, accumulated into J) runs with sixteen lanes per
// pair, four pairs per wave; finally C <- C J on matrix cores.  Steps repeat
// until a whole sweep finds every block pair orthogonal to
// |G_ac| <= s eps sqrt(G_aa G_cc).  Then sigma_c = ||w_c||, L[:, c] =
// w_c / sigma_c and Rv[:, c] = M^T w_c / sigma_c^2, sorted by decreasing
// sigma.  W lives in LDS when it fits, else in global scratch
// (s x round_up(s, 2 JB) doubles).
//
// Inner sweep: lane j of a pair's sixteen keeps column j of G and row j of J
// in registers.  A round publishes the columns through LDS, and each lane
// reads its partner's column and the rotation inputs, applies its column's
// rotation (G <- G R), then reads all sixteen coefficients and applies the
// row rotations (G <- R^T G) and J <- J R in registers.  The rounds are
// unrolled, so the row partners are constants.
// ---------------------------------------------------------------------------
constexpr int JB = 8;
constexpr int JP = 2 * JB;
constexpr int JR = JP - 1;            // rounds of one inner sweep
constexpr int JSTR = JP + 2;          // LDS stride of a 16 x 16 pair matrix (16-byte aligned rows)
constexpr int JSLOTS_LDS = 8;         // block pairs of the LDS form (s <= 128)
constexpr int JSLOTS_GLOBAL = 32;     // block pairs of the global form (s <= 512)
constexpr int JTHREADS = 512;

__device__ __forceinline__ int rr_slot_index(int slot, int round, int n) {
    // index held by `slot` in round `round` of the round-robin on n indices
    return slot == 0 ? 0 : 1 + (slot - 1 + round) % (n - 1);
}
// the same on JP indices, and its inverse (the slot of index idx)
__host__ __device__ constexpr int rr_index(int slot, int rd) { return slot == 0 ? 0 : 1 + (slot - 1 + rd) % (JP - 1); }
__host__ __device__ constexpr int rr_slot(int idx, int rd) {
    return idx == 0 ? 0 : 1 + (idx - 1 + (JP - 1) - rd) % (JP - 1);
}

// Round RD of the inner sweep for lane j of a pair: publish column j of G,
// read the partner column and the rotation inputs, rotate the column pair
// (G <- G R), publish this column's coefficients, then apply the row
// rotations (G <- R^T G) and J <- J R.  Row pairs are constants of the round.
template <int RD>
__device__ __forceinline__ void pair_round(double* __restrict__ X, double2* __restrict__ T, int j, double tol,
                                           double (&gc)[JP], double (&jr)[JP]) {
    // the lane's partner arithmetic of this round stays in this round (hoisted
    // over all fifteen rounds it would not fit in registers)
    asm volatile("" : "+v"(j));
    if (RD > 0) {
#pragma unroll
        for (int r = 0; r < JP; r += 2) *(double2*)&X[j * JSTR + r] = make_double2(gc[r], gc[r + 1]);
    }
    wave_lds_sync();
    const int sl = rr_slot(j, RD);
    const bool lead = sl < JB;
    const int pj = rr_index(JP - 1 - sl, RD);
    const int p = lead ? j : pj, q = lead ? pj : j;
    const double al = X[p * JSTR + p], be = X[q * JSTR + q], ga = X[q * JSTR + p];
    double pc[JP];
#pragma unroll
    for (int r = 0; r < JP; r += 2) {
        const double2 v = *(const double2*)&X[pj * JSTR + r];
        pc[r] = v.x;
        pc[r + 1] = v.y;
    }
    double c, sn;
    jacobi_rotation_fast(al, be, ga, tol, c, sn);
    // new column p = c col_p - sn col_q, new column q = c col_q + sn col_p; the coefficients are
    // published first so that reading all sixteen back overlaps the column update
    const double a = c, b = lead ? -sn : sn;
    T[j] = make_double2(a, b);
    wave_lds_sync();
    double2 co[JP];
#pragma unroll
    for (int r = 0; r < JP; ++r) co[r] = T[r];
#pragma unroll
    for (int r = 0; r < JP; ++r) gc[r] = a * gc[r] + b * pc[r];
#pragma unroll
    for (int l = 0; l < JB; ++l) {
        const int rp = rr_index(l, RD), rq = rr_index(JP - 1 - l, RD);
        const double2 cp = co[rp], cq = co[rq];
        const double gp = gc[rp], gq = gc[rq];
        gc[rp] = cp.x * gp + cp.y * gq;
        gc[rq] = cq.x * gq + cq.y * gp;
        const double jp = jr[rp], jq = jr[rq];
        jr[rp] = cp.x * jp + cp.y * jq;
        jr[rq] = cq.x * jq + cq.y * jp;
    }
    // finish J's update in this round: deferred, it would keep every round's
    // coefficients live
#pragma unroll
    for (int r = 0; r < JP; ++r) asm volatile("" : "+v"(jr[r]));
    wave_lds_sync();
}

template <int... RD>
__device__ __forceinline__ void pair_rounds(double* __restrict__ X, double2* __restrict__ T, int j, double tol,
                                            double (&gc)[JP], double (&jr)[JP], std::integer_sequence<int, RD...>) {
    (pair_round<RD>(X, T, j, tol, gc, jr), ...);
}

// One cyclic sweep on the pair matrix X (column c at X[c * JSTR], G on entry,
// overwritten); row j of the accumulated rotation J goes to Jrow.
__device__ __forceinline__ void pair_inner_sweep(double* __restrict__ X, double2* __restrict__ T, int j, double tol,
                                                 double* __restrict__ Jrow) {
    double gc[JP], jr[JP];
#pragma unroll
    for (int r = 0; r < JP; r += 2) {
        const double2 v = *(const double2*)&X[j * JSTR + r];
        gc[r] = v.x;
        gc[r + 1] = v.y;
    }
#pragma unroll
    for (int r = 0; r < JP; ++r) jr[r] = r == j ? 1.0 : 0.0;
    pair_rounds(X, T, j, tol, gc, jr, std::make_integer_sequence<int, JR>{});
#pragma unroll
    for (int r = 0; r < JP; r += 2) *(double2*)&Jrow[r] = make_double2(jr[r], jr[r + 1]);
}

// The same sweep with one 2 x 2 block per lane of a whole wave: lane 8 a + b
// holds rows {p_a, q_a} x columns {p_b, q_b} of G and the same entries of J,
// where (p_l, q_l) is pair l of the round.  Pair a's rotation comes from the
// diagonal block of lane 9 a; every lane then updates its block in
// registers (G <- R_a^T G R_b, J <- J R_b, R = [[c, s], [-s, c]]) and writes
// it back, so a round costs one broadcast of eight rotations and one LDS
// round trip of four G and four J entries.  G: column c at X[c * JSTR]
// (overwritten); J: row r at Jm[r * JSTR], the identity on entry.
template <int RD>
__device__ __forceinline__ void pair64_round(double* __restrict__ X, double* __restrict__ Jm, double2* __restrict__ T,
                                             int a, int b, double tol) {
    asm volatile("" : "+v"(a), "+v"(b));   // keep this round's index arithmetic in this round
    const int pa = rr_index(a, RD), qa = rr_index(JP - 1 - a, RD);
    const int pb = rr_index(b, RD), qb = rr_index(JP - 1 - b, RD);
    double g00 = X[pb * JSTR + pa], g01 = X[qb * JSTR + pa], g10 = X[pb * JSTR + qa], g11 = X[qb * JSTR + qa];
    const double j00 = Jm[pa * JSTR + pb], j01 = Jm[pa * JSTR + qb], j10 = Jm[qa * JSTR + pb], j11 = Jm[qa * JSTR + qb];
    if (a == b) {
        double c, sn;
        jacobi_rotation_fast(g00, g11, g01, tol, c, sn);
        T[a] = make_double2(c, sn);
    }
    wave_lds_sync();
    const double2 ra = T[a], rb = T[b];
    const double t00 = g00 * rb.x - g01 * rb.y, t01 = g00 * rb.y + g01 * rb.x;
    const double t10 = g10 * rb.x - g11 * rb.y, t11 = g10 * rb.y + g11 * rb.x;
    g00 = ra.x * t00 - ra.y * t10;
    g01 = ra.x * t01 - ra.y * t11;
    g10 = ra.y * t00 + ra.x * t10;
    g11 = ra.y * t01 + ra.x * t11;
    // each entry belongs to one lane in a round, so the block is written back in place
    X[pb * JSTR + pa] = g00;
    X[qb * JSTR + pa] = g01;
    X[pb * JSTR + qa] = g10;
    X[qb * JSTR + qa] = g11;
    Jm[pa * JSTR + pb] = j00 * rb.x - j01 * rb.y;
    Jm[pa * JSTR + qb] = j00 * rb.y + j01 * rb.x;
    Jm[qa * JSTR + pb] = j10 * rb.x - j11 * rb.y;
    Jm[qa * JSTR + qb] = j10 * rb.y + j11 * rb.x;
    wave_lds_sync();
}

template <int... RD>
__device__ __forceinline__ void pair64_rounds(double* __restrict__ X, double* __restrict__ Jm, double2* __restrict__ T,
                                              int a, int b, double tol, std::integer_sequence<int, RD...>) {
    (pair64_round<RD>(X, Jm, T, a, b, tol), ...);
}

// One cyclic sweep of a pair matrix on a whole wave; J (row-major, stride
// JSTR) is written to Jm.  T holds eight double2 of scratch.
__device__ __forceinline__ void pair_sweep64(double* __restrict__ X, double* __restrict__ Jm, double2* __restrict__ T,
                                             int lane, double tol) {
    for (int e = lane; e < JP * JP; e += 64) Jm[(e >> 4) * JSTR + (e & 15)] = (e >> 4) == (e & 15) ? 1.0 : 0.0;
    wave_lds_sync();
    pair64_rounds(X, Jm, T, lane >> 3, lane & 7, tol, std::make_integer_sequence<int, JR>{});
}

template <bool IN_LDS, int NS>
__device__ __forceinline__ void block_jacobi_body(double* __restrict__ W, const double* __restrict__ M, int s,
                                                  double* __restrict__ L, double* __restrict__ Rv,
                                                  double* __restrict__ sigma, uint32_t* status) {
    __shared__ __align__(16) double Gs[NS][JP * JSTR];
    __shared__ __align__(16) double Js[NS][JP * JSTR];
    __shared__ __align__(16) double2 Ts[NS][JP];
    __shared__ int flag[NS];
    __shared__ int rotated;
    static_assert(NS * JP * JSTR >= 512, "the final phase reuses the pair slots for 512 norms and ranks");
    double* const sig_sh = &Gs[0][0];   // after the sweeps: column norms
    int* const rank_sh = (int*)&Js[0][0];
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int sp = (s + JP - 1) / JP * JP;
    const int nb = sp / JB;
    const int npairs = nb / 2;
    for (int e = tid; e < s * sp; e += nt) {
        const int c = e / s, r = e % s;
        W[e] = c < s ? M[(int64_t)r * s + c] : 0.0;
    }
    const double tol = (double)s * 2.220446049250313e-16;
    if (tid == 0) rotated = 0;
    __syncthreads();

    int sweeps = 0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        for (int step = 0; step < nb - 1; ++step) {
            // G = C^T C per pair: lane (g, x) supplies C[r0 + g][x] as both operands; 16 loads are
            // issued before their matrix-core steps so that they overlap
            for (int pr = wave; pr < npairs; pr += nwaves) {
                const int P = rr_slot_index(pr, step, nb), Q = rr_slot_index(nb - 1 - pr, step, nb);
                const int cx_col = x < JB ? P * JB + x : Q * JB + (x - JB);
                doublex4 acc = {0, 0, 0, 0};
                const double* cx = W + (int64_t)cx_col * s;
                for (int r0 = 0; r0 < s; r0 += 64) {
                    double v[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) v[u] = (r0 + 4 * u + g < s) ? cx[r0 + 4 * u + g] : 0.0;
#pragma unroll
                    for (int u = 0; u < 16; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u], v[u], acc, 0, 0, 0);
                }
                double* X = Gs[pr];
#pragma unroll
                for (int r = 0; r < 4; ++r) X[x * JSTR + g + 4 * r] = acc[r];
                wave_lds_sync();
                // any scaled off-diagonal entry above tol (compared in squares)
                bool off = false;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = g + 4 * r;
                    const double d = X[a * JSTR + a] * X[x * JSTR + x];
                    off |= a != x && d > 0.0 && acc[r] * acc[r] > tol * tol * d;
                }
                const bool any = __builtin_amdgcn_ballot_w64(off) != 0;
                if (lane == 0) {
                    flag[pr] = any ? 1 : 0;
                    if (any) rotated = 1;
                }
            }
            __syncthreads();
            // one cyclic sweep per pair, sixteen lanes each
            static_assert(NS % 4 == 0, "a wave sweeps four pair slots");
            if constexpr (NS <= 8) {
                // one pair per wave (npairs <= NS <= the workgroup's waves)
                if (wave < npairs) pair_sweep64(Gs[wave], Js[wave], Ts[wave], lane, tol);
            } else if (4 * wave < npairs) {
                // slot < NS since 4 wave < npairs <= NS; a slot at or past npairs holds no pair and
                // its lanes work on that unused slot's stale contents, whose J is never applied
                const int slot = 4 * wave + g;
                pair_inner_sweep(Gs[slot], Ts[slot], x, tol, &Js[slot][x * JSTR]);
            }
            __syncthreads();
            // C <- C J, two 16-row tiles at a time (a tile reads and writes only its own rows)
            for (int pr = wave; pr < npairs; pr += nwaves) {
                if (!flag[pr]) continue;   // uniform over the wave
                const int P = rr_slot_index(pr, step, nb), Q = rr_slot_index(nb - 1 - pr, step, nb);
                auto col = [&](int a) { return a < JB ? P * JB + a : Q * JB + (a - JB); };
                const double* J = Js[pr];
                double jv[JP / 4];
#pragma unroll
                for (int kq = 0; kq < JP / 4; ++kq) jv[kq] = J[(4 * kq + g) * JSTR + x];
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
                    wave_lds_sync();
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = r0 + 16 * h + g + 4 * r;
                            if (row < s) W[(int64_t)col(x) * s + row] = o[h][r];
                        }
                    wave_lds_sync();
                }
            }
            __syncthreads();
        }
        const int any = rotated;
        sweeps = sweep + 1;
        __syncthreads();
        if (tid == 0) rotated = 0;
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

template <bool IN_LDS, int NS>
struct block_jacobi_kernel_op {
    static constexpr int kThreads = JTHREADS;
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
    static __device__ __forceinline__ void run(const VGrid vg, const Args& a) {
        (void)vg;
        if (a.enable && *a.enable == 0) return;
        extern __shared__ double lds_w[];
        if constexpr (IN_LDS) block_jacobi_body<true, NS>(lds_w, a.M, a.s, a.L, a.Rv, a.sigma, a.status);
        else block_jacobi_body<false, NS>(a.gscratch, a.M, a.s, a.L, a.Rv, a.sigma, a.status);
    }
};

// ---------------------------------------------------------------------------
// Wide form of the block one-sided Jacobi SVD (s above the LDS form's limit):
// one workgroup per block pair, W in global scratch.  Each step a workgroup
// stages its pair's 2 JB columns into LDS with coalesced loads, forms the
// Gram there (four waves over row chunks, partials summed in LDS), sweeps it
// once as above, applies C <- C J in LDS and writes the columns back; then
// all workgroups meet at a grid barrier before the next pairing.  A sweep
// ends the iteration when no workgroup found its pair above tolerance.  The
// final phase (norms, order, L, Rv) is shared out over the workgroups.
//
// The barrier counts arrivals in global memory; its wait is bounded, and a
// wait that runs out sets a flag that makes every later wait return at once
// and marks the status word, so a grid that is not co-resident ends with an
// error rather than a hang.  The host launches this form only outside batch
// recording (a grouped launch could hold more workgroups than fit at once).
// ---------------------------------------------------------------------------
constexpr int JW_THREADS = 256;
constexpr unsigned kBarrierSpins = 1u << 22;
constexpr int kSyncWords = 64;      // barrier count, timeout flag, per-sweep rotation counts
constexpr int kMaxSweeps = kSyncWords - 2;

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned* err, unsigned target, unsigned spin_limit) {
    // every thread waits for its own stores to reach L2, the workgroup barrier then holds
    // them all; thread 0's agent-scope release publishes them (one L2 write-back per
    // workgroup), and its agent-scope acquire after the wait makes the other workgroups'
    // stores visible before the closing workgroup barrier releases the waves
    wait_all_vmem();
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
            if (++spins > spin_limit) {
                __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

struct block_jacobi_wide_op {
    static constexpr int kThreads = JW_THREADS;
    struct Args {
        const double* M;
        int s;
        double* L;
        double* Rv;
        double* sigma;
        double* W;
        unsigned* sync;   // kSyncWords zeroed words
        uint32_t* status;
        const int* enable;
        unsigned spin_limit;   // polls of one bounded barrier wait
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& a) {
        if (a.enable && *a.enable == 0) return;   // uniform over the grid
        extern __shared__ __align__(16) double jw_lds[];
        const double* __restrict__ M = a.M;
        double* __restrict__ W = a.W;
        const int s = a.s;
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int g = lane >> 4, x = lane & 15;
        const int sp = (s + JP - 1) / JP * JP;
        const int nb = sp / JB;
        const int nwg = (int)vg.gx, pr = (int)vg.bx;
        const int cstr = (s + 31) / 32 * 32 + 4;   // LDS column stride: 16 columns x 4 rows hit distinct banks
        double* Cs = jw_lds;                             // 2 JB staged columns
        double* Gp = Cs + JP * cstr;                     // four partial Grams
        double* Gs = Gp + 4 * JP * JSTR;                 // four sweep slots (slot 0 is the pair's)
        double* Js = Gs + 4 * JP * JSTR;
        double2* Ts = (double2*)(Js + 4 * JP * JSTR);
        __shared__ int need_sh, more_sh;
        unsigned* bar = a.sync;
        unsigned* err = a.sync + 1;
        unsigned* rot = a.sync + 2;
        unsigned nbar = 0;
        const double tol = (double)s * 2.220446049250313e-16;

        // W = M (column c at W + c s), zero columns up to sp
        for (int64_t e = (int64_t)pr * JW_THREADS + tid; e < (int64_t)s * sp; e += (int64_t)nwg * JW_THREADS) {
            const int c = (int)(e / s), r = (int)(e % s);
            W[e] = c < s ? M[(int64_t)r * s + c] : 0.0;
        }
        grid_barrier(bar, err, ++nbar * nwg, a.spin_limit);

        int sweeps = 0;
        for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
            for (int step = 0; step < nb - 1; ++step) {
                const int P = rr_slot_index(pr, step, nb), Q = rr_slot_index(nb - 1 - pr, step, nb);
                auto col = [&](int c) { return c < JB ? P * JB + c : Q * JB + (c - JB); };
                // stage the pair's columns: eight loads in flight per thread before their LDS stores
                for (int e0 = tid; e0 < JP * s; e0 += 8 * JW_THREADS) {
                    double v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * JW_THREADS;
                        v[u] = e < JP * s ? W[(int64_t)col(e / s) * s + e % s] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * JW_THREADS;
                        if (e < JP * s) Cs[(e / s) * cstr + e % s] = v[u];
                    }
                }
                __syncthreads();
                // partial Grams over 16-row chunks, chunk ch on wave ch % 4
                {
                    doublex4 acc = {0, 0, 0, 0};
                    for (int r0 = 16 * wave; r0 < s; r0 += 64) {
                        double v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) v[u] = (r0 + 4 * u + g < s) ? Cs[x * cstr + r0 + 4 * u + g] : 0.0;
#pragma unroll
                        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u], v[u], acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) Gp[wave * JP * JSTR + x * JSTR + g + 4 * r] = acc[r];
                }
                __syncthreads();
                {
                    const int c = tid >> 4, r = tid & 15;   // element (row r, column c)
                    const int o = c * JSTR + r;
                    Gs[o] = (Gp[o] + Gp[JP * JSTR + o]) + (Gp[2 * JP * JSTR + o] + Gp[3 * JP * JSTR + o]);
                }
                __syncthreads();
                {
                    const int c = tid >> 4, r = tid & 15;
                    const double d = Gs[r * JSTR + r] * Gs[c * JSTR + c], v = Gs[c * JSTR + r];
                    const bool off = r != c && d > 0.0 && v * v > tol * tol * d;
                    const int need = __syncthreads_or(off ? 1 : 0);
                    if (tid == 0) need_sh = need;
                }
                __syncthreads();
                if (need_sh) {
                    if (wave == 0) pair_sweep64(Gs, Js, Ts, lane, tol);
                    __syncthreads();
                    // C <- C J in place, 32-row tiles (a tile reads and writes only its own rows)
                    double jv[JP / 4];
#pragma unroll
                    for (int kq = 0; kq < JP / 4; ++kq) jv[kq] = Js[(4 * kq + g) * JSTR + x];
                    for (int r0 = 32 * wave; r0 < s; r0 += 128) {
                        double av[2][JP / 4];
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int kq = 0; kq < JP / 4; ++kq) {
                                const int row = r0 + 16 * h + x;
                                av[h][kq] = row < s ? Cs[(4 * kq + g) * cstr + row] : 0.0;
                            }
                        doublex4 o[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int kq = 0; kq < JP / 4; ++kq)
                                o[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][kq], jv[kq], o[h], 0, 0, 0);
                        wave_lds_sync();
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int row = r0 + 16 * h + g + 4 * r;
                                if (row < s) Cs[x * cstr + row] = o[h][r];
                            }
                        wave_lds_sync();
                    }
                    __syncthreads();
                    for (int e0 = tid; e0 < JP * s; e0 += 8 * JW_THREADS) {
                        double v[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int e = e0 + u * JW_THREADS;
                            v[u] = e < JP * s ? Cs[(e / s) * cstr + e % s] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int e = e0 + u * JW_THREADS;
                            if (e < JP * s) W[(int64_t)col(e / s) * s + e % s] = v[u];
                        }
                    }
                    if (tid == 0) __hip_atomic_fetch_add(&rot[sweep], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                grid_barrier(bar, err, ++nbar * nwg, a.spin_limit);
            }
            sweeps = sweep + 1;
            // every workgroup reads the same count: all increments of this sweep precede the barrier
            if (tid == 0)
                more_sh = __hip_atomic_load(&rot[sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u &&
                          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
            __syncthreads();
            if (!more_sh) break;
        }
        if (pr == 0 && tid == 0 && a.status) {
            a.status[4] = (uint32_t)sweeps;
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
                rsvd_flag(a.status, RSVD_FLAG_SYNC_TIMEOUT);
        }

        // every workgroup: column norms and their order (same arithmetic everywhere)
        double* sig_sh = Cs;                 // sp doubles
        int* rank_sh = (int*)(Cs + 512);     // sp ints
        __syncthreads();
        for (int c = wave; c < sp; c += 4) {
            double acc = 0.0;
            for (int r = lane; r < s; r += 64) acc += W[(int64_t)c * s + r] * W[(int64_t)c * s + r];
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            if (lane == 0) sig_sh[c] = sqrt(acc);
        }
        __syncthreads();
        for (int c = tid; c < sp; c += JW_THREADS) {
            const double v = sig_sh[c];
            int rk = 0;
            for (int d = 0; d < sp; ++d) {
                const double u = sig_sh[d];
                rk += (u > v) || (u == v && d < c);
            }
            rank_sh[c] = rk;
            if (pr == 0 && rk < s) {
                a.sigma[rk] = v;
                if (!isfinite(v)) rsvd_flag(a.status, RSVD_FLAG_NONFINITE);
            }
        }
        __syncthreads();
        // L: columns shared out over the workgroups
        for (int c = pr; c < sp; c += nwg) {
            const int rk = rank_sh[c];
            if (rk >= s) continue;
            const double sv = sig_sh[c];
            for (int r = tid; r < s; r += JW_THREADS) a.L[(int64_t)r * s + rk] = sv > 0.0 ? W[(int64_t)c * s + r] / sv : 0.0;
        }
        // Rv[x][rank(c)] = (M^T W)[x][c] / sigma_c^2, 16 x 16 tiles shared out over all waves of the grid
        const int ntx = (s + 15) / 16, ntc = sp / 16;
        for (int tile = pr * 4 + wave; tile < ntx * ntc; tile += nwg * 4) {
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
                a.Rv[(int64_t)xx * s + rk] = sv > 0.0 ? acc[r] / (sv * sv) : 0.0;
            }
        }
    }
};

struct zero_words_op {
    static constexpr int kThreads = 64;
    struct Args {
        unsigned* p;
        int n;
    };
    static __device__ __forceinline__ void run(const VGrid, const Args& a) {
        for (int i = threadIdx.x; i < a.n; i += 64) a.p[i] = 0u;
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
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [U, len, k, ldu, rows_per_chunk, pval, pidx] = args_;
        const int64_t r0 = (int64_t)vg.bx * rows_per_chunk;
        const int64_t r1 = std::min<int64_t>(len, r0 + rows_per_chunk);
        for (int c = threadIdx.x; c < k; c += blockDim.x) {
            double best = -1.0, bval = 0.0;
            int64_t bidx = -1;
            auto visit = [&](double v, int64_t r) {
                if (fabs(v) > best) {
                    best = fabs(v);
                    bval = v;
                    bidx = r;
                }
            };
            // rows in order; eight loads go out before their comparisons
            int64_t r = r0;
            for (; r + 8 <= r1; r += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = (double)U[(r + u) * ldu + c];
#pragma unroll
                for (int u = 0; u < 8; ++u) visit(v[u], r + u);
            }
            for (; r < r1; ++r) visit((double)U[r * ldu + c], r);
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
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [pval, pidx, nchunks, k, sgn] = args_;
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
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [X, len, k, ldx, sgn] = args_;
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
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [src, dst, count] = args_;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)vg.gx * blockDim.x)
            dst[e] = src[e];
    }
};

// Y = X^T for s x s row-major FP64 matrices.
struct transpose_f64_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        const double*  X;
        double*  Y;
        int64_t s;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [X, Y, s] = args_;
        for (int64_t e = vg.bx * (int64_t)blockDim.x + threadIdx.x; e < s * s; e += (int64_t)vg.gx * blockDim.x)
            Y[(e % s) * s + e / s] = X[e];
    }
};

}  // namespace

static size_t block_jacobi_w_doubles(int s) { return (size_t)s * ((s + JP - 1) / JP * JP); }

// W (s x round_up(s, 16) doubles) sits in LDS when it fits beside the eight
// pair slots of the LDS form (s up to 121); wider matrices keep W in global
// scratch.
static constexpr size_t kJacobiSlotsLds =
    2 * sizeof(double) * JSLOTS_LDS * JP * JSTR + sizeof(double2) * JSLOTS_LDS * JP + sizeof(int) * (JSLOTS_LDS + 1);
static constexpr size_t kLdsBytes = 160 * 1024;
bool jacobi_fits_lds(int s) {
    return s <= JSLOTS_LDS * JP && block_jacobi_w_doubles(s) * sizeof(double) + kJacobiSlotsLds + 256 <= kLdsBytes;
}

// Global scratch: W, then the wide form's synchronization words (also for
// LDS-sized cores, which take the wide form outside batches).
size_t small_svd_scratch_doubles(int s) { return s <= 80 ? 0 : block_jacobi_w_doubles(s) + kSyncWords / 2; }

static size_t wide_lds_bytes(int s) {
    const int cstr = (s + 31) / 32 * 32 + 4;
    return sizeof(double) * ((size_t)JP * cstr + 3 * 4 * JP * JSTR) + sizeof(double2) * 4 * JP;
}

rsvd_status run_small_svd(const double* M, int s, double* L, double* Rv, double* sigma, double* gscratch,
                          uint32_t* status, const int* enable, hipStream_t st, unsigned spin_limit) {
    launch_phase();
    if (s > 512 || s < 1) return RSVD_EUNSUPPORTED;
    // one workgroup with W in LDS for batches and narrow cores; the
    // multi-workgroup form otherwise (its grid barrier costs more than it
    // saves below about 80 columns)
    if (jacobi_fits_lds(s) && (launch_recorder() || s <= 80)) {
        using Op = block_jacobi_kernel_op<true, JSLOTS_LDS>;
        const size_t shmem = block_jacobi_w_doubles(s) * sizeof(double);
        if (hipFuncSetAttribute(op_single_fn<Op>(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem) !=
            hipSuccess)
            return RSVD_EHIP;
        launch_op<Op>(dim3(1), dim3(Op::kThreads), shmem, st, {M, s, L, Rv, sigma, nullptr, status, enable});
    } else if (launch_recorder()) {
        // grouped batch launches do not guarantee that a matrix's workgroups are resident together
        if (!gscratch) return RSVD_EINVAL;
        using Op = block_jacobi_kernel_op<false, JSLOTS_GLOBAL>;
        launch_op<Op>(dim3(1), dim3(Op::kThreads), 0, st, {M, s, L, Rv, sigma, gscratch, status, enable});
    } else {
        if (!gscratch) return RSVD_EINVAL;
        unsigned* sync = (unsigned*)(gscratch + block_jacobi_w_doubles(s));
        launch_op<zero_words_op>(dim3(1), dim3(64), 0, st, {sync, kSyncWords});
        using Op = block_jacobi_wide_op;
        const size_t shmem = wide_lds_bytes(s);
        if (hipFuncSetAttribute(op_single_fn<Op>(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem) !=
            hipSuccess)
            return RSVD_EHIP;
        const int npairs = (s + JP - 1) / JP;
        launch_op<Op>(dim3(npairs), dim3(Op::kThreads), shmem, st,
                      {M, s, L, Rv, sigma, gscratch, sync, status, enable,
                               spin_limit ? spin_limit : kBarrierSpins});
    }
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_lift(int dtype_p, const void* P, int64_t ldp, int s, int64_t len, const double* F, int ldf, int k,
                     int dtype_o, void* out, int64_t ldo, hipStream_t st) {
    // on matrix cores: the coefficient apply with a row-major store
    return run_lift_rows(dtype_p, P, ldp, s, len, F, ldf, k, dtype_o, out, ldo, st);
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
        launch_op<sign_partial_kernel_op<double>>(dim3((unsigned)nch), dim3(256), 0, st, {(const double*)U, m, k, (int64_t)k, rows, pval, pidx});
        launch_op<sign_final_kernel_op>(dim3((unsigned)ceil_div(k, 4)), dim3(256), 0, st, {pval, pidx, (int)nch, k, sgn});
        launch_op<apply_sign_kernel_op<double>>(dim3(gu), dim3(256), 0, st, {(double*)U, m, k, (int64_t)k, sgn});
        launch_op<apply_sign_kernel_op<double>>(dim3(gv), dim3(256), 0, st, {(double*)V, n, k, (int64_t)k, sgn});
    } else {
        launch_op<sign_partial_kernel_op<float>>(dim3((unsigned)nch), dim3(256), 0, st, {(const float*)U, m, k, (int64_t)k, rows, pval, pidx});
        launch_op<sign_final_kernel_op>(dim3((unsigned)ceil_div(k, 4)), dim3(256), 0, st, {pval, pidx, (int)nch, k, sgn});
        launch_op<apply_sign_kernel_op<float>>(dim3(gu), dim3(256), 0, st, {(float*)U, m, k, (int64_t)k, sgn});
        launch_op<apply_sign_kernel_op<float>>(dim3(gv), dim3(256), 0, st, {(float*)V, n, k, (int64_t)k, sgn});
    }
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_transpose_small_f64(const double* X, double* Y, int s, hipStream_t st) {
    launch_phase();
    const int64_t count = (int64_t)s * s;
    launch_op<transpose_f64_kernel_op>(dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(count, 256), 1024))), dim3(256), 0, st, {X, Y, s});
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

rsvd_status run_copy_f64(const double* src, double* dst, int64_t count, hipStream_t st) {
    launch_phase();
    launch_op<copy_f64_kernel_op>(dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(count, 256), 1024))), dim3(256), 0, st, {src, dst, count});
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}
