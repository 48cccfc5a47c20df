// Test matrices of the SRFT core sketch (Sect. 6.7): for one side of length L,
// Phi = D C^T P (L x s_c) with D a diagonal of random signs, C the orthonormal
// DCT-II (C[f][j] = a_f cos(pi (2j + 1) f / (2L)), a_0 = sqrt(1/L),
// a_f = sqrt(2/L)) and P the s_c sampled frequencies.  Column c of Phi is the
// sign-flipped row P[c] of C; the kernels write Phi^T as a panel, the layout
// of every thin operand of the views.
//
// Random bits come from the counter-based generator of the Gaussian test
// matrices: position j uses output word j & 3 of Philox4x32-10 at counter
// (j >> 2, 0, 0, tag).  The sign of j is the top bit of its word under the
// sign tag; the sample holds the s_c positions with the smallest
// (word under the sample tag, position) pairs, in increasing order.
#include <algorithm>

#include "common.h"
#include "philox.h"
#include "srft.h"

namespace {

__device__ __forceinline__ uint32_t srft_word(uint64_t seed, uint32_t tag, int64_t j) {
    uint32_t c[4] = {(uint32_t)(j >> 2), 0u, 0u, tag};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return c[j & 3];
}

// The 64-bit sort key of position j: generator word above, position below
// (positions are unique, so keys are).
__device__ __forceinline__ uint64_t srft_key(uint64_t seed, uint32_t tag, int64_t j) {
    return ((uint64_t)srft_word(seed, tag, j) << 32) | (uint64_t)j;
}

constexpr int kSelectThreads = 1024;

// One workgroup: the s_c-th smallest key by an 8-bit radix select (eight
// passes from the top digit, each a histogram of the keys that share the
// digits chosen so far), then the keys not above it, i.e. exactly the s_c
// smallest, compacted in increasing position order (thread t scans a
// contiguous range of positions and writes at the exclusive prefix count).
__global__ void __launch_bounds__(kSelectThreads)
srft_sample_kernel(uint64_t seed, uint32_t tag, int64_t L, int sc, int* __restrict__ pos) {
    __shared__ unsigned hist[256];
    __shared__ uint64_t prefix_sh;
    __shared__ int64_t rank_sh;
    __shared__ int64_t cnt_sh[kSelectThreads];
    const int tid = threadIdx.x;
    uint64_t prefix = 0;
    int64_t rank = sc;   // 1-based rank of the wanted key within the keys matching `prefix`
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        for (int b = tid; b < 256; b += kSelectThreads) hist[b] = 0u;
        __syncthreads();
        for (int64_t j = tid; j < L; j += kSelectThreads) {
            const uint64_t key = srft_key(seed, tag, j);
            if (pass == 0 || (key >> (shift + 8)) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int64_t below = 0;
            int b = 0;
            while (b < 255 && below + (int64_t)hist[b] < rank) below += hist[b++];
            rank_sh = rank - below;
            prefix_sh = (prefix << 8) | (uint64_t)b;
        }
        __syncthreads();
        prefix = prefix_sh;
        rank = rank_sh;
        __syncthreads();
    }
    const uint64_t thr = prefix;
    const int64_t chunk = (L + kSelectThreads - 1) / kSelectThreads;
    const int64_t j0 = (int64_t)tid * chunk, j1 = j0 + chunk < L ? j0 + chunk : L;
    int64_t c = 0;
    for (int64_t j = j0; j < j1; ++j) c += srft_key(seed, tag, j) <= thr ? 1 : 0;
    cnt_sh[tid] = c;
    __syncthreads();
    if (tid == 0) {
        int64_t acc = 0;
        for (int t = 0; t < kSelectThreads; ++t) {
            const int64_t v = cnt_sh[t];
            cnt_sh[t] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int64_t o = cnt_sh[tid];
    for (int64_t j = j0; j < j1; ++j)
        if (srft_key(seed, tag, j) <= thr && o < sc) pos[o++] = (int)j;
}

// out[c][j] = d_j a_f cos(pi t / (2L)) with f = pos[c] and t = (2j + 1) f
// reduced modulo 4L (the cosine's period in the integer (2j + 1) f), so the
// angle carries one rounding however large (2j + 1) f is.
template <typename T>
__global__ void srft_fill_kernel(uint64_t seed, uint32_t sign_tag, int64_t L, int sc, const int* __restrict__ pos,
                                 T* __restrict__ out, int64_t ld) {
    const int64_t total = (int64_t)sc * L;
    const double a0 = sqrt(1.0 / (double)L), af = sqrt(2.0 / (double)L);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / L);
        const int64_t j = e % L;
        const uint64_t f = (uint64_t)pos[c];
        const uint64_t t = ((2u * (uint64_t)j + 1u) * f) % (4u * (uint64_t)L);
        const double v = cospi((double)t / (2.0 * (double)L));
        const double sign = (srft_word(seed, sign_tag, j) >> 31) ? -1.0 : 1.0;
        out[(int64_t)c * ld + j] = (T)(sign * (f == 0 ? a0 : af) * v);
    }
}

}  // namespace

rsvd_status run_srft_panel(uint64_t seed, uint32_t sign_tag, uint32_t sample_tag, int64_t L, int sc, int* pos,
                           int dtype, void* out, int64_t ld, hipStream_t st) {
    if (sc < 1 || L < sc || L >= ((int64_t)1 << 31) || ld < L || !pos || !out) return RSVD_EINVAL;
    hipLaunchKernelGGL(srft_sample_kernel, dim3(1), dim3(kSelectThreads), 0, st, seed, sample_tag, L, sc, pos);
    const int64_t total = (int64_t)sc * L;
    const dim3 grid((unsigned)std::min<int64_t>(ceil_div(total, 256), 16384));
    if (dtype == RSVD_F64)
        hipLaunchKernelGGL(srft_fill_kernel<double>, grid, dim3(256), 0, st, seed, sign_tag, L, sc, (const int*)pos,
                           (double*)out, ld);
    else if (dtype == RSVD_F32)
        hipLaunchKernelGGL(srft_fill_kernel<float>, grid, dim3(256), 0, st, seed, sign_tag, L, sc, (const int*)pos,
                           (float*)out, ld);
    else
        return RSVD_EINVAL;
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}
