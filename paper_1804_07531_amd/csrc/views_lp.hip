// Views on BF16 matrix cores: A stored in BF16, in FP8 E4M3 (one FP32
// scale per stored row), or in FP32 split exactly into three BF16 parts;
// the thin operand is prepared from an FP32 panel as one BF16 plane (a
// quantized cheap view), three BF16 planes hi + mid + lo (an FP32-accurate
// view), or one FP8 plane with one scale per thin column (the cheap view of
// an FP8 matrix, on FP8 matrix cores).  Accumulation is FP32 throughout.
//
// Exactness of the splits: for an FP32 value x, hi = bf16(x), mid =
// bf16(x - hi), lo = bf16(x - hi - mid) are each computed without rounding
// error in FP32 and hi + mid + lo = x exactly (8 + 8 + 8 significant bits).
// A BF16 x BF16 product is exact in FP32.  So a BF16 or FP8 A times the
// three thin planes is A X up to FP32 accumulation only; an FP32 A split as
// a1 + a2 + a3 times x1 + x2 + x3 keeps the six products with i + j <= 4 and
// drops terms below 2^-26 |a x|, under the FP32 unit roundoff.
#include <algorithm>

#include "common.h"
#include "views.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

namespace {

// ---------------------------------------------------------------------------
// element conversions
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    __bf16 h = (__bf16)x;  // round to nearest even (v_cvt_pk_bf16_f32)
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// x = hi + mid + lo exactly (see the header comment).
__device__ __forceinline__ void split3(float x, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
    hi = bf16_bits(x);
    const float r1 = x - bf16_to_f32(hi);
    mid = bf16_bits(r1);
    const float r2 = r1 - bf16_to_f32(mid);
    lo = bf16_bits(r2);
}

// OCP E4M3 (bias 7, no infinities, max 448): value of a byte.
__device__ __forceinline__ float e4m3_to_f32(uint32_t b) {
    const uint32_t e = (b >> 3) & 15u, mnt = b & 7u;
    const float mag = e ? __uint_as_float(((e + 120u) << 23) | (mnt << 20)) : (float)mnt * 0x1p-9f;
    return (b & 0x80u) ? -mag : mag;
}

// Round to nearest even into OCP E4M3, saturating at +-448.
__device__ __forceinline__ uint32_t f32_to_e4m3(float x) {
    const uint32_t sign = x < 0.0f ? 0x80u : 0u;
    float a = fminf(fabsf(x), 448.0f);
    uint32_t code;
    if (a < 0x1p-6f) {
        code = (uint32_t)rintf(a * 512.0f);  // subnormal steps of 2^-9 (8 -> the smallest normal)
    } else {
        uint32_t u = __float_as_uint(a);
        u = (u + 0x7FFFFu + ((u >> 20) & 1u)) & ~0xFFFFFu;   // keep 3 mantissa bits, ties to even
        const uint32_t e = (u >> 23) - 120u, mnt = (u >> 20) & 7u;
        code = (e > 15u || (e == 15u && mnt == 7u)) ? 0x7Eu : ((e << 3) | mnt);
    }
    return sign | code;
}

// ---------------------------------------------------------------------------
// thin operand preparation
// ---------------------------------------------------------------------------
// NT BF16 planes (s x ldp, zero past len) from an FP32 panel (s x len):
// NT = 1: bf16(x); NT = 3: hi, mid, lo.  len_scale (optional) multiplies
// element (c, r) by len_scale[r] first (row scales of a stored FP8 matrix
// folded into the thin operand of a contraction over its rows).
template <int NT>
__global__ void __launch_bounds__(256)
thin_split_kernel(const float* __restrict__ P, int64_t ld, int s, int64_t len, const float* __restrict__ len_scale,
                  uint16_t* __restrict__ planes, int64_t ldp) {
    const int64_t total = (int64_t)s * ldp;
    const int64_t pstride = total;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / ldp, r = e % ldp;
        float x = 0.0f;
        if (r < len) {
            x = P[c * ld + r];
            if (len_scale) x *= len_scale[r];
        }
        if (NT == 1) {
            planes[e] = bf16_bits(x);
        } else {
            uint16_t h, mi, lo;
            split3(x, h, mi, lo);
            planes[e] = h;
            planes[pstride + e] = mi;
            planes[2 * pstride + e] = lo;
        }
    }
}

// Per-row maxima |x| of a (optionally len-scaled) panel -> scale: the
// smallest power of two d with max / d <= 448 (max = f 2^E, f in [0.5, 1),
// 448 = 0.875 2^9 gives d = 2^(E - 9 + [f > 0.875])), so that x / d is exact.
__global__ void __launch_bounds__(256)
thin_amax_kernel(const float* __restrict__ P, int64_t ld, int64_t len, const float* __restrict__ len_scale,
                 float* __restrict__ scale) {
    __shared__ float red[4];
    const int c = blockIdx.x;
    float mx = 0.0f;
    int64_t r = threadIdx.x;
    for (; r + 7 * (int64_t)blockDim.x < len; r += 8 * (int64_t)blockDim.x) {   // eight loads ahead
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = P[(int64_t)c * ld + r + u * blockDim.x];
        if (len_scale) {
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] *= len_scale[r + u * blockDim.x];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) mx = fmaxf(mx, fabsf(x[u]));
    }
    for (; r < len; r += blockDim.x) {
        float x = P[(int64_t)c * ld + r];
        if (len_scale) x *= len_scale[r];
        mx = fmaxf(mx, fabsf(x));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        int e = 0;
        const float f = frexpf(mx, &e);
        scale[c] = mx > 0.0f ? ldexpf(1.0f, e - 9 + (f > 0.875f ? 1 : 0)) : 1.0f;
    }
}

__global__ void __launch_bounds__(256)
thin_fp8_kernel(const float* __restrict__ P, int64_t ld, int s, int64_t len, const float* __restrict__ len_scale,
                const float* __restrict__ scale, uint8_t* __restrict__ plane, int64_t ldp) {
    const int64_t total = (int64_t)s * ldp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / ldp, r = e % ldp;
        uint32_t code = 0;
        if (r < len) {
            float x = P[c * ld + r];
            if (len_scale) x *= len_scale[r];
            code = f32_to_e4m3(x * (1.0f / scale[c]));   // scale is a power of two: exact
        }
        plane[e] = (uint8_t)code;
    }
}

// ---------------------------------------------------------------------------
// A-side traits.  AK 0: BF16 A; 1: FP32 A split into three BF16 parts;
// 2: FP8 E4M3 A converted exactly to BF16.
// ---------------------------------------------------------------------------
template <int AK>
struct LpA {
    static constexpr int KS = 32;                   // contraction per stage (one 32-deep matrix-core step)
    static constexpr int BYTES = AK == 0 ? 2 : AK == 1 ? 4 : 1;
    static constexpr int NA = AK == 1 ? 3 : 1;      // BF16 parts of an A value
};

__device__ __forceinline__ bf16x8 as_bf(uintx4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ uintx4 pack_bf(const uint16_t (&h)[8]) {
    uintx4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = (uint32_t)h[2 * q] | ((uint32_t)h[2 * q + 1] << 16);
    return r;
}

// BF16 parts of 8 A values given as FP32.
template <int AK>
__device__ __forceinline__ void a_parts_f32(const float (&x)[8], bf16x8 (&out)[LpA<AK>::NA]) {
    if constexpr (AK == 1) {
        uint16_t h[8], mi[8], lo[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) split3(x[t], h[t], mi[t], lo[t]);
        out[0] = as_bf(pack_bf(h));
        out[1] = as_bf(pack_bf(mi));
        out[2] = as_bf(pack_bf(lo));
    } else {
        uint16_t h[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h[t] = bf16_bits(x[t]);
        out[0] = as_bf(pack_bf(h));
    }
}

// 8 FP8 bytes (two words) -> BF16 (exact).
__device__ __forceinline__ bf16x8 fp8x8_to_bf(uint32_t w0, uint32_t w1) {
    uint16_t h[8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        h[t] = bf16_bits(e4m3_to_f32((w0 >> (8 * t)) & 0xFFu));
        h[4 + t] = bf16_bits(e4m3_to_f32((w1 >> (8 * t)) & 0xFFu));
    }
    return as_bf(pack_bf(h));
}

// acc += A-parts x thin-planes with the product set of (AK, NT).
template <int AK, int NT>
__device__ __forceinline__ floatx4 lp_mma(const bf16x8 (&a)[LpA<AK>::NA], const bf16x8 (&x)[NT], floatx4 acc) {
    if constexpr (AK == 1) {
        static_assert(NT == 3, "a split FP32 A pairs with three thin planes");
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], x[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], x[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], x[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], x[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], x[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], x[0], acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int p = NT - 1; p >= 0; --p) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], x[p], acc, 0, 0, 0);
    }
    return acc;
}

// Guarded load of one A element as FP32 (tail paths).
template <int AK>
__device__ __forceinline__ float a_elem(const void* A, int64_t off) {
    if constexpr (AK == 0) return bf16_to_f32(((const uint16_t*)A)[off]);
    else if constexpr (AK == 1) return ((const float*)A)[off];
    else return e4m3_to_f32(((const uint8_t*)A)[off]);
}

// ---------------------------------------------------------------------------
// Range view of the stored matrix S (m x n): Y^T (s x m) = (S X)^T, with X
// given as NT BF16 planes of X^T (s x ldp).  A wave owns 16*MR rows and all
// 16*NB thin columns.  Three-stage LDS ring fed by direct-to-LDS copies
// (one exact vmcnt wait + one barrier per stage, as the FP32 kernels).
// Lane l = 16 g + i of a fragment holds row (or thin column) i and the
// contraction indices k0 + 8 g + (0..7); both operands use the same
// assignment, so the matrix core pairs equal k.  A stage of S is one 1 KB
// copy per 16 x 32 BF16 fragment, two per FP32 fragment, and for FP8 one
// copy per wave holding its 32 rows x 32 bytes (so FP8 needs MR = 2).
// ---------------------------------------------------------------------------
template <int AK, int NT, int NB, int MR>
__global__ void __launch_bounds__(256)
range_lp_kernel(const void* __restrict__ Av, int64_t lda, int64_t m, int64_t n, const float* __restrict__ row_scale,
                const uint16_t* __restrict__ planes, int64_t ldp, int64_t pstride, int s,
                float* __restrict__ out, int64_t ldo, int64_t split_stride, int64_t k_chunk, int accumulate) {
    using T = LpA<AK>;
    constexpr int KS = T::KS, NA = T::NA;
    static_assert(AK != 2 || MR == 2, "an FP8 copy covers 32 rows");
    constexpr int CPW = AK == 1 ? 2 * MR : AK == 0 ? MR : 1;   // A copies per wave per stage
    constexpr int ABLK = 4 * CPW;
    constexpr int TB = NT * NB;                // 1 KB blocks of the thin operand per stage
    static_assert(TB % 4 == 0, "thin blocks split evenly over the four waves");
    constexpr int BLK = ABLK + TB;
    constexpr int NL = CPW + TB / 4;           // copies per wave per stage
    __shared__ uintx4 st0[BLK * 64];
    __shared__ uintx4 st1[BLK * 64];
    __shared__ uintx4 st2[BLK * 64];
    const char* A = (const char*)Av;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MR);
    const int64_t kb = (int64_t)blockIdx.y * k_chunk;
    const int64_t ke = std::min<int64_t>(n, kb + k_chunk);
    const int64_t nsteps = (ke - kb) / KS;

    const char* asrc[CPW];
    if constexpr (AK == 2) {
        const int64_t r = std::min<int64_t>(row0 + (lane & 31), m - 1);
        asrc[0] = A + r * lda + kb + 16 * (lane >> 5);
    } else {
#pragma unroll
        for (int a = 0; a < MR; ++a)
#pragma unroll
            for (int c = 0; c < CPW / MR; ++c) {
                const int64_t r = std::min<int64_t>(row0 + 16 * a + i, m - 1);
                asrc[a * (CPW / MR) + c] = A + (r * lda + kb + 8 * g + 4 * c) * T::BYTES;
            }
    }
    const uint16_t* xsrc[TB / 4];
#pragma unroll
    for (int u = 0; u < TB / 4; ++u) {
        const int q = wave + 4 * u;
        const int p = q / NB, b = q % NB;
        xsrc[u] = planes + p * pstride + (int64_t)std::min(16 * b + i, s - 1) * ldp + kb + 8 * g;
    }

    floatx4 acc[MR][NB];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = floatx4{0, 0, 0, 0};

    auto issue = [&](int64_t t, uintx4* stg) {
#pragma unroll
        for (int a = 0; a < CPW; ++a) lds_copy16(asrc[a] + t * KS * T::BYTES, stg + (wave * CPW + a) * 64);
#pragma unroll
        for (int u = 0; u < TB / 4; ++u) lds_copy16(xsrc[u] + t * KS, stg + (ABLK + wave + 4 * u) * 64);
    };
    auto step = [&](int64_t t, uintx4* cur, uintx4* nxt) {
        wait_vmcnt<NL>();
        bare_barrier();
        issue(std::min<int64_t>(t + 2, nsteps - 1), nxt);
        bf16x8 af[MR][NA];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            if constexpr (AK == 0) {
                af[a][0] = as_bf(cur[(wave * MR + a) * 64 + lane]);
            } else if constexpr (AK == 1) {
                const uintx4 v0 = cur[((wave * MR + a) * 2 + 0) * 64 + lane];
                const uintx4 v1 = cur[((wave * MR + a) * 2 + 1) * 64 + lane];
                float x[8];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    x[q] = __uint_as_float(v0[q]);
                    x[4 + q] = __uint_as_float(v1[q]);
                }
                a_parts_f32<AK>(x, af[a]);
            } else {
                // row 16 a + i sits in copy lane 16 a + i + 32 (g >> 1), bytes 8 (g & 1) .. + 7
                const uint32_t* w = (const uint32_t*)(cur + wave * 64 + 16 * a + i + 32 * (g >> 1)) + 2 * (g & 1);
                af[a][0] = fp8x8_to_bf(w[0], w[1]);
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            bf16x8 xf[NT];
#pragma unroll
            for (int p = 0; p < NT; ++p) xf[p] = as_bf(cur[(ABLK + p * NB + b) * 64 + lane]);
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = lp_mma<AK, NT>(af[a], xf, acc[a][b]);
        }
    };
    if (nsteps > 0) {
        issue(0, st0);
        issue(std::min<int64_t>(1, nsteps - 1), st1);
        int64_t t = 0;
        for (; t + 3 <= nsteps; t += 3) {
            step(t, st0, st2);
            step(t + 1, st1, st0);
            step(t + 2, st2, st1);
        }
        if (t < nsteps) step(t, st0, st2);
        if (t + 1 < nsteps) step(t + 1, st1, st0);
        wait_all_vmem();
    }
    // ragged tail of the contraction: guarded element loads, k = kk + 8 g + (0..7)
    for (int64_t kk = kb + KS * nsteps; kk < ke; kk += 32) {
        bf16x8 af[MR][NA];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int64_t r = row0 + 16 * a + i;
            float x[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int64_t k = kk + 8 * g + t;
                x[t] = (r < m && k < ke) ? a_elem<AK>(A, r * lda + k) : 0.0f;
            }
            if constexpr (AK == 1) {
                a_parts_f32<1>(x, af[a]);
            } else {
                bf16x8 tmp[1];
                a_parts_f32<0>(x, tmp);   // BF16 and FP8 values are exact in BF16
                af[a][0] = tmp[0];
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = std::min(16 * b + i, s - 1);
            bf16x8 xf[NT];
#pragma unroll
            for (int p = 0; p < NT; ++p) {
                // planes are zero past len and at least round_up(len, 128) long
                const uint16_t* src = planes + p * pstride + (int64_t)j * ldp + kk + 8 * g;
                uint16_t h8[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) h8[t] = src[t];
                xf[p] = as_bf(pack_bf(h8));
            }
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = lp_mma<AK, NT>(af[a], xf, acc[a][b]);
        }
    }
    if (row0 >= m) return;
    float* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int a = 0; a < MR; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + 16 * a + 4 * g + r;
            if (row >= m) continue;
            const float sc = row_scale ? row_scale[row] : 1.0f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = 16 * b + i;
                if (j >= s) continue;
                float* d = o + (int64_t)j * ldo + row;
                const float v = acc[a][b][r] * sc;
                *d = accumulate ? *d + v : v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Range view with 64 rows per wave (BF16 A, or FP8 A converted to BF16).
// Each thin fragment read from LDS feeds four row blocks instead of one or
// two: with 32 or 16 rows per wave the thin tile's LDS reads, not HBM or
// the matrix cores, bound the view.  The 64 x 16 NB accumulators take most
// of the register file (AGPRs included), so a workgroup (256 rows) has the
// CU to itself and the ring is as deep as the LDS allows: NS = 2 to 4
// stages, copies running NS - 1 stages ahead.
// Thin blocks are copied four per stage round; when NT NB is not a
// multiple of four, the spare copies repeat the last block into unused
// slots.
// ---------------------------------------------------------------------------
template <int AK, int NT, int NB, int NS>
__global__ void __launch_bounds__(256, 1)
range_lp4_kernel(const void* __restrict__ Av, int64_t lda, int64_t m, int64_t n, const float* __restrict__ row_scale,
                 const uint16_t* __restrict__ planes, int64_t ldp, int64_t pstride, int s,
                 float* __restrict__ out, int64_t ldo, int64_t split_stride, int64_t k_chunk, int accumulate) {
    static_assert(AK == 0 || AK == 2, "BF16 A or FP8 A");
    static_assert(NS >= 2 && NS <= 4, "two to four stages");
    constexpr int MR = 4;
    constexpr int KS = 32;
    constexpr int CPW = AK == 0 ? MR : MR / 2;   // A copies per wave per stage (FP8: one per 32 rows)
    constexpr int ABLK = 4 * CPW;
    constexpr int TB = NT * NB;
    constexpr int TBP = (TB + 3) / 4 * 4;
    constexpr int BLK = ABLK + TBP;
    constexpr int NL = CPW + TBP / 4;           // copies per wave per stage
    constexpr int BYTES = AK == 0 ? 2 : 1;
    __shared__ uintx4 st0[BLK * 64];
    __shared__ uintx4 st1[BLK * 64];
    __shared__ uintx4 st2[NS >= 3 ? BLK * 64 : 1];
    __shared__ uintx4 st3[NS == 4 ? BLK * 64 : 1];
    const char* A = (const char*)Av;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MR);
    const int64_t kb = (int64_t)blockIdx.y * k_chunk;
    const int64_t ke = std::min<int64_t>(n, kb + k_chunk);
    const int64_t nsteps = (ke - kb) / KS;

    const char* asrc[CPW];
    if constexpr (AK == 2) {
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int64_t r = std::min<int64_t>(row0 + 32 * c + (lane & 31), m - 1);
            asrc[c] = A + r * lda + kb + 16 * (lane >> 5);
        }
    } else {
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int64_t r = std::min<int64_t>(row0 + 16 * a + i, m - 1);
            asrc[a] = A + (r * lda + kb + 8 * g) * BYTES;
        }
    }
    const uint16_t* xsrc[TBP / 4];
#pragma unroll
    for (int u = 0; u < TBP / 4; ++u) {
        const int q = std::min(wave + 4 * u, TB - 1);   // spare copies repeat the last block
        const int p = q / NB, b = q % NB;
        xsrc[u] = planes + p * pstride + (int64_t)std::min(16 * b + i, s - 1) * ldp + kb + 8 * g;
    }

    floatx4 acc[MR][NB];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = floatx4{0, 0, 0, 0};

    auto issue = [&](int64_t t, uintx4* stg) {
#pragma unroll
        for (int c = 0; c < CPW; ++c) lds_copy16(asrc[c] + t * KS * BYTES, stg + (wave * CPW + c) * 64);
#pragma unroll
        for (int u = 0; u < TBP / 4; ++u) lds_copy16(xsrc[u] + t * KS, stg + (ABLK + wave + 4 * u) * 64);
    };
    auto step = [&](int64_t t, uintx4* cur, uintx4* nxt) {
        wait_vmcnt<(NS - 2) * NL>();
        bare_barrier();
        issue(std::min<int64_t>(t + NS - 1, nsteps - 1), nxt);
        bf16x8 af[MR][1];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            if constexpr (AK == 0) {
                af[a][0] = as_bf(cur[(wave * MR + a) * 64 + lane]);
            } else {
                // row 16 a + i: copy (a >> 1), lane 16 (a & 1) + i + 32 (g >> 1), bytes 8 (g & 1) .. + 7
                const uint32_t* w =
                    (const uint32_t*)(cur + (wave * CPW + (a >> 1)) * 64 + 16 * (a & 1) + i + 32 * (g >> 1)) + 2 * (g & 1);
                af[a][0] = fp8x8_to_bf(w[0], w[1]);
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            bf16x8 xf[NT];
#pragma unroll
            for (int p = 0; p < NT; ++p) xf[p] = as_bf(cur[(ABLK + p * NB + b) * 64 + lane]);
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = lp_mma<0, NT>(af[a], xf, acc[a][b]);
        }
    };
    if (nsteps > 0) {
        issue(0, st0);
        if constexpr (NS == 4) {
            issue(std::min<int64_t>(1, nsteps - 1), st1);
            issue(std::min<int64_t>(2, nsteps - 1), st2);
            int64_t t = 0;
            for (; t + 4 <= nsteps; t += 4) {
                step(t, st0, st3);
                step(t + 1, st1, st0);
                step(t + 2, st2, st1);
                step(t + 3, st3, st2);
            }
            if (t < nsteps) step(t, st0, st3);
            if (t + 1 < nsteps) step(t + 1, st1, st0);
            if (t + 2 < nsteps) step(t + 2, st2, st1);
        } else if constexpr (NS == 3) {
            issue(std::min<int64_t>(1, nsteps - 1), st1);
            int64_t t = 0;
            for (; t + 3 <= nsteps; t += 3) {
                step(t, st0, st2);
                step(t + 1, st1, st0);
                step(t + 2, st2, st1);
            }
            if (t < nsteps) step(t, st0, st2);
            if (t + 1 < nsteps) step(t + 1, st1, st0);
        } else {
            int64_t t = 0;
            for (; t + 2 <= nsteps; t += 2) {
                step(t, st0, st1);
                step(t + 1, st1, st0);
            }
            if (t < nsteps) step(t, st0, st1);
        }
        wait_all_vmem();
    }
    // ragged tail of the contraction: guarded element loads, k = kk + 8 g + (0..7)
    for (int64_t kk = kb + KS * nsteps; kk < ke; kk += 32) {
        bf16x8 af[MR][1];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int64_t r = row0 + 16 * a + i;
            float x[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int64_t k = kk + 8 * g + t;
                x[t] = (r < m && k < ke) ? a_elem<AK>(A, r * lda + k) : 0.0f;
            }
            bf16x8 tmp[1];
            a_parts_f32<0>(x, tmp);   // BF16 and FP8 values are exact in BF16
            af[a][0] = tmp[0];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = std::min(16 * b + i, s - 1);
            bf16x8 xf[NT];
#pragma unroll
            for (int p = 0; p < NT; ++p) {
                // planes are zero past len and at least round_up(len, 128) long
                const uint16_t* src = planes + p * pstride + (int64_t)j * ldp + kk + 8 * g;
                uint16_t h8[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) h8[t] = src[t];
                xf[p] = as_bf(pack_bf(h8));
            }
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = lp_mma<0, NT>(af[a], xf, acc[a][b]);
        }
    }
    if (row0 >= m) return;
    float* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int a = 0; a < MR; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + 16 * a + 4 * g + r;
            if (row >= m) continue;
            const float sc = row_scale ? row_scale[row] : 1.0f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = 16 * b + i;
                if (j >= s) continue;
                float* d = o + (int64_t)j * ldo + row;
                const float v = acc[a][b][r] * sc;
                *d = accumulate ? *d + v : v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Co-range view of the stored matrix S (m x n): Z^T (s x n) = (S^T Y)^T,
// with Y given as NT BF16 planes of Y^T (s x ldp).  A wave owns 16*MR
// columns of S; a stage holds KS rows x 64*MR columns of S, row-major in
// 16-byte chunks, with the chunk index of row r XOR-ed with
// ((r >> 3) & 3) * CW so that the four lane groups, which read rows 8
// apart, fall on different LDS banks.
// ---------------------------------------------------------------------------
// Workgroups per CU the co-range ring leaves room for: two when two rings
// (three stages of the A tile and the thin tile each) fit the LDS.  With two,
// the compiler also keeps a wave within 256 VGPRs and accumulates in them;
// with the accumulators in AGPRs it moves them between registers at every
// pass of the unrolled loop (the BF16 co-range at s = 220: 3.16 ms with one,
// 2.84 ms with the accumulators in VGPRs).
template <int AK, int NT, int NB, int MR>
constexpr int corange_lp_min_blocks() {
    constexpr int bytes = AK == 0 ? 2 : AK == 1 ? 4 : 1;
    constexpr int stage_kb = 32 * (64 * MR * bytes / 16) / 64 + NT * NB;
    return 2 * 3 * stage_kb <= 156 ? 2 : 1;
}

template <int AK, int NT, int NB, int MR>
__global__ void __launch_bounds__(256, (corange_lp_min_blocks<AK, NT, NB, MR>()))
corange_lp_kernel(const void* __restrict__ Av, int64_t lda, int64_t m, int64_t n,
                  const uint16_t* __restrict__ planes, int64_t ldp, int64_t pstride, int s,
                  float* __restrict__ out, int64_t ldo, int64_t split_stride, int64_t r_chunk, int accumulate) {
    using T = LpA<AK>;
    constexpr int KS = T::KS, NA = T::NA, BYTES = T::BYTES;
    constexpr int AW = 64 * MR;                       // columns of the workgroup
    constexpr int CH = AW * BYTES / 16;               // 16-byte chunks per tile row
    constexpr int ABLK = KS * CH / 64;                // 1 KB blocks of A per stage
    static_assert(ABLK % 4 == 0, "A copies split evenly over the four waves");
    constexpr int TB = NT * NB;
    static_assert(TB % 4 == 0, "thin blocks split evenly over the four waves");
    constexpr int BLK = ABLK + TB;
    constexpr int NL = ABLK / 4 + TB / 4;
    constexpr int RS = 3;                             // lane groups read rows 8 apart
    constexpr int CW = BYTES;                         // chunks spanned by 16 consecutive columns
    static_assert(CH >= 4 * CW, "swizzle stays inside a tile row");
    __shared__ uintx4 st0[BLK * 64];
    __shared__ uintx4 st1[BLK * 64];
    __shared__ uintx4 st2[BLK * 64];
    const char* A = (const char*)Av;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
    const int64_t cw0 = (int64_t)blockIdx.x * AW;
    const int64_t col0 = cw0 + (int64_t)wave * 16 * MR;
    const int64_t rb = (int64_t)blockIdx.y * r_chunk;
    const int64_t re = std::min<int64_t>(m, rb + r_chunk);
    const int64_t nsteps = (re - rb) / KS;
    const int64_t last_cb = (((n - 1) * BYTES) / 16) * 16;   // last 16-byte chunk holding a column of S

    const char* asrc[ABLK / 4];
#pragma unroll
    for (int u = 0; u < ABLK / 4; ++u) {
        const int L = 64 * (wave + 4 * u) + lane;
        const int row = L / CH, slot = L % CH;
        const int chunk = slot ^ (((row >> RS) & 3) * CW);
        const int64_t cb = std::min<int64_t>(cw0 * BYTES + 16 * chunk, last_cb);
        asrc[u] = A + (rb + row) * lda * BYTES + cb;
    }
    const uint16_t* ysrc[TB / 4];
#pragma unroll
    for (int u = 0; u < TB / 4; ++u) {
        const int q = wave + 4 * u;
        const int p = q / NB, b = q % NB;
        ysrc[u] = planes + p * pstride + (int64_t)std::min(16 * b + i, s - 1) * ldp + rb + 8 * g;
    }

    floatx4 acc[MR][NB];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = floatx4{0, 0, 0, 0};

    auto issue = [&](int64_t t, uintx4* stg) {
#pragma unroll
        for (int u = 0; u < ABLK / 4; ++u) lds_copy16(asrc[u] + t * KS * lda * BYTES, stg + (wave + 4 * u) * 64);
#pragma unroll
        for (int u = 0; u < TB / 4; ++u) lds_copy16(ysrc[u] + t * KS, stg + (ABLK + wave + 4 * u) * 64);
    };
    auto step = [&](int64_t t, uintx4* cur, uintx4* nxt) {
        wait_vmcnt<NL>();
        bare_barrier();
        issue(std::min<int64_t>(t + 2, nsteps - 1), nxt);
        const char* at = (const char*)cur;
        bf16x8 af[MR][NA];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int cl = wave * 16 * MR + 16 * a + i;     // column inside the tile
            const int cbyte = cl * BYTES;
            float x[8];
            uint16_t hb[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int row = 8 * g + t;
                const int slot = (cbyte >> 4) ^ (((row >> RS) & 3) * CW);
                const char* pe = at + (row * CH + slot) * 16 + (cbyte & 15);
                if constexpr (AK == 0) hb[t] = *(const uint16_t*)pe;
                else if constexpr (AK == 1) x[t] = *(const float*)pe;
                else hb[t] = bf16_bits(e4m3_to_f32(*(const uint8_t*)pe));
            }
            if constexpr (AK == 1) a_parts_f32<1>(x, af[a]);
            else af[a][0] = as_bf(pack_bf(hb));
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            bf16x8 yf[NT];
#pragma unroll
            for (int p = 0; p < NT; ++p) yf[p] = as_bf(cur[(ABLK + p * NB + b) * 64 + lane]);
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = lp_mma<AK, NT>(af[a], yf, acc[a][b]);
        }
    };
    if (nsteps > 0) {
        issue(0, st0);
        issue(std::min<int64_t>(1, nsteps - 1), st1);
        int64_t t = 0;
        for (; t + 3 <= nsteps; t += 3) {
            step(t, st0, st2);
            step(t + 1, st1, st0);
            step(t + 2, st2, st1);
        }
        if (t < nsteps) step(t, st0, st2);
        if (t + 1 < nsteps) step(t + 1, st1, st0);
        wait_all_vmem();
    }
    // ragged tail of the rows: guarded element loads, row = rr + 8 g + (0..7)
    for (int64_t rr = rb + KS * nsteps; rr < re; rr += 32) {
        bf16x8 af[MR][NA];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int64_t c = col0 + 16 * a + i;
            float x[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int64_t r = rr + 8 * g + t;
                x[t] = (c < n && r < re) ? a_elem<AK>(A, r * lda + c) : 0.0f;
            }
            if constexpr (AK == 1) {
                a_parts_f32<1>(x, af[a]);
            } else {
                bf16x8 tmp[1];
                a_parts_f32<0>(x, tmp);
                af[a][0] = tmp[0];
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = std::min(16 * b + i, s - 1);
            bf16x8 yf[NT];
#pragma unroll
            for (int p = 0; p < NT; ++p) {
                const uint16_t* src = planes + p * pstride + (int64_t)j * ldp + rr + 8 * g;
                uint16_t h8[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) h8[t] = src[t];
                yf[p] = as_bf(pack_bf(h8));
            }
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = lp_mma<AK, NT>(af[a], yf, acc[a][b]);
        }
    }
    if (col0 >= n) return;
    float* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = 16 * b + i;
        if (j >= s) continue;
#pragma unroll
        for (int a = 0; a < MR; ++a) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t c = col0 + 16 * a + 4 * g + q;
                if (c < n) {
                    float* d = o + (int64_t)j * ldo + c;
                    *d = accumulate ? *d + acc[a][b][q] : acc[a][b][q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP8 x FP8 views on the 16x16x128 FP8 matrix cores (unit block scales).
// Lane l = 16 g + i of a fragment holds 32 bytes: row (or thin column) i,
// contraction indices k0 + 32 g + (0..31), as two 16-byte copies.
// ---------------------------------------------------------------------------
__device__ __forceinline__ floatx4 mma_fp8(const uintx4& a0, const uintx4& a1, const uintx4& b0, const uintx4& b1,
                                           floatx4 acc) {
    intx8 a, b;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a[q] = (int)a0[q];
        a[4 + q] = (int)a1[q];
        b[q] = (int)b0[q];
        b[4 + q] = (int)b1[q];
    }
    // formats 0/0 = E4M3 x E4M3; scales 127 = 2^0 (E8M0)
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
}

template <int NB, int MR>
__global__ void __launch_bounds__(256)
range_fp8_kernel(const uint8_t* __restrict__ A, int64_t lda, int64_t m, int64_t n, const float* __restrict__ row_scale,
                 const uint8_t* __restrict__ plane, int64_t ldp, const float* __restrict__ thin_scale, int s,
                 float* __restrict__ out, int64_t ldo, int64_t split_stride, int64_t k_chunk, int accumulate) {
    constexpr int KS = 128;
    constexpr int ABLK = 4 * MR * 2;
    constexpr int TB = NB * 2;
    static_assert(TB % 4 == 0, "thin blocks split evenly over the four waves");
    constexpr int BLK = ABLK + TB;
    constexpr int NL = MR * 2 + TB / 4;
    __shared__ uintx4 st0[BLK * 64];
    __shared__ uintx4 st1[BLK * 64];
    __shared__ uintx4 st2[BLK * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MR);
    const int64_t kb = (int64_t)blockIdx.y * k_chunk;
    const int64_t ke = std::min<int64_t>(n, kb + k_chunk);
    const int64_t nsteps = (ke - kb) / KS;

    const uint8_t* asrc[MR * 2];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
            asrc[a * 2 + c] = A + std::min<int64_t>(row0 + 16 * a + i, m - 1) * lda + kb + 32 * g + 16 * c;
    const uint8_t* xsrc[TB / 4];
#pragma unroll
    for (int u = 0; u < TB / 4; ++u) {
        const int q = wave + 4 * u, b = q >> 1, c = q & 1;
        xsrc[u] = plane + (int64_t)std::min(16 * b + i, s - 1) * ldp + kb + 32 * g + 16 * c;
    }
    floatx4 acc[MR][NB];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = floatx4{0, 0, 0, 0};

    auto issue = [&](int64_t t, uintx4* stg) {
#pragma unroll
        for (int a = 0; a < MR * 2; ++a) lds_copy16(asrc[a] + t * KS, stg + (wave * MR * 2 + a) * 64);
#pragma unroll
        for (int u = 0; u < TB / 4; ++u) lds_copy16(xsrc[u] + t * KS, stg + (ABLK + wave + 4 * u) * 64);
    };
    auto step = [&](int64_t t, uintx4* cur, uintx4* nxt) {
        wait_vmcnt<NL>();
        bare_barrier();
        issue(std::min<int64_t>(t + 2, nsteps - 1), nxt);
        uintx4 av[MR][2];
#pragma unroll
        for (int a = 0; a < MR; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) av[a][c] = cur[((wave * MR + a) * 2 + c) * 64 + lane];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uintx4 x0 = cur[(ABLK + 2 * b) * 64 + lane], x1 = cur[(ABLK + 2 * b + 1) * 64 + lane];
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = mma_fp8(av[a][0], av[a][1], x0, x1, acc[a][b]);
        }
    };
    if (nsteps > 0) {
        issue(0, st0);
        issue(std::min<int64_t>(1, nsteps - 1), st1);
        int64_t t = 0;
        for (; t + 3 <= nsteps; t += 3) {
            step(t, st0, st2);
            step(t + 1, st1, st0);
            step(t + 2, st2, st1);
        }
        if (t < nsteps) step(t, st0, st2);
        if (t + 1 < nsteps) step(t + 1, st1, st0);
        wait_all_vmem();
    }
    // ragged tail: guarded byte loads, k = kk + 32 g + (0..31)
    for (int64_t kk = kb + KS * nsteps; kk < ke; kk += KS) {
        uintx4 av[MR][2];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int64_t r = row0 + 16 * a + i;
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int64_t k = kk + 32 * g + 16 * c + 4 * q + t;
                        const uint32_t byte = (r < m && k < ke) ? A[r * lda + k] : 0u;
                        w |= byte << (8 * t);
                    }
                    av[a][c][q] = w;
                }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = std::min(16 * b + i, s - 1);
            uintx4 xv[2];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // the plane is zero past len and at least round_up(len, 128) long
                    const uint8_t* src = plane + (int64_t)j * ldp + kk + 32 * g + 16 * c + 4 * q;
                    xv[c][q] = (uint32_t)src[0] | ((uint32_t)src[1] << 8) | ((uint32_t)src[2] << 16) |
                               ((uint32_t)src[3] << 24);
                }
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = mma_fp8(av[a][0], av[a][1], xv[0], xv[1], acc[a][b]);
        }
    }
    if (row0 >= m) return;
    float* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int a = 0; a < MR; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + 16 * a + 4 * g + r;
            if (row >= m) continue;
            const float sc = row_scale[row];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = 16 * b + i;
                if (j >= s) continue;
                float* d = o + (int64_t)j * ldo + row;
                const float v = acc[a][b][r] * sc * thin_scale[j];
                *d = accumulate ? *d + v : v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP8 range view for tall matrices, with A streamed from HBM straight into
// registers.  The FP8 view above stages both operands in a three-stage LDS
// ring; at one workgroup per CU that is two stages (32 KB of A) in flight,
// too little for the HBM latency, and the waves wait on memory about half
// their time.  Here each wave owns 16 MR rows and loads its own A fragments
// with 16-byte vector loads into a ring of NS register slots, so NS - 1
// stages of A (NS - 1 times 16 KB per wave pair of row blocks) are in flight
// per wave; only the thin tile, which all four waves share, goes through an
// NS-stage LDS ring.  The contraction index of a 128-deep stage is permuted
// the same way on both operands: half c of lane group g holds bytes
// 16 g + 64 c .. + 15, so one load instruction covers 64 contiguous bytes of
// each of 16 rows.  The accumulators (16 MR x 16 NB per wave) take most of
// the register file: one workgroup per CU.
// ---------------------------------------------------------------------------
template <int NB, int MR, int NS>
__global__ void __launch_bounds__(256, 1)
range_fp8_rs_kernel(const uint8_t* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                    const float* __restrict__ row_scale, const uint8_t* __restrict__ plane, int64_t ldp,
                    const float* __restrict__ thin_scale, int s, float* __restrict__ out, int64_t ldo,
                    int64_t split_stride, int64_t k_chunk, int accumulate) {
    static_assert(NB % 2 == 0, "thin copies split evenly over the four waves");
    static_assert(NS >= 2 && NS <= 4, "two to four stages");
    constexpr int KS = 128;
    constexpr int TB = NB * 2;          // 1 KB thin copies per stage (two per 16-column block)
    constexpr int NL = TB / 4 + MR * 2; // vector-memory operations per wave per stage
    __shared__ uintx4 tst[NS][TB * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MR);
    const int64_t kb = (int64_t)blockIdx.y * k_chunk;
    const int64_t ke = std::min<int64_t>(n, kb + k_chunk);
    const int64_t nsteps = (ke - kb) / KS;

    const uint8_t* asrc[MR];
#pragma unroll
    for (int a = 0; a < MR; ++a) asrc[a] = A + std::min<int64_t>(row0 + 16 * a + i, m - 1) * lda + kb + 16 * g;
    const uint8_t* xsrc[TB / 4];
#pragma unroll
    for (int u = 0; u < TB / 4; ++u) {
        const int q = wave + 4 * u, b = q >> 1, c = q & 1;
        xsrc[u] = plane + (int64_t)std::min(16 * b + i, s - 1) * ldp + kb + 16 * g + 64 * c;
    }
    floatx4 acc[MR][NB];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = floatx4{0, 0, 0, 0};
    uintx4 av[NS][MR][2];

    // stage t into ring slot `slot`: this wave's thin copies, then its A fragments
    auto issue = [&](int64_t t, int slot) {
        const int64_t off = t * KS;
#pragma unroll
        for (int u = 0; u < TB / 4; ++u) lds_copy16(xsrc[u] + off, &tst[slot][(wave + 4 * u) * 64]);
#pragma unroll
        for (int a = 0; a < MR; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) av[slot][a][c] = *(const uintx4*)(asrc[a] + off + 64 * c);
    };
    auto step = [&](int64_t t, int slot) {
        wait_vmcnt<(NS - 2) * NL>();   // stage t (issued NS - 1 stages ago) has landed for this wave
        bare_barrier();                // ... and for the other waves; slot (t - 1) % NS is free
        const int nslot = slot == 0 ? NS - 1 : slot - 1;
        issue(std::min<int64_t>(t + NS - 1, nsteps - 1), nslot);
        // thin fragments read from LDS two blocks ahead of their matrix-core steps, so
        // the LDS latency hides behind the steps of the blocks before (one wave per SIMD
        // has no other wave to hide it)
        uintx4 xb[3][2];
        auto load_x = [&](int b) {
            xb[b % 3][0] = tst[slot][(2 * b) * 64 + lane];
            xb[b % 3][1] = tst[slot][(2 * b + 1) * 64 + lane];
        };
        load_x(0);
        if (NB > 1) load_x(1);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b + 2 < NB) load_x(b + 2);
            // keeps the reads ahead: without it the scheduler sinks them to their use
            // and folds the three buffers into one
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int a = 0; a < MR; ++a)
                acc[a][b] = mma_fp8(av[slot][a][0], av[slot][a][1], xb[b % 3][0], xb[b % 3][1], acc[a][b]);
        }
    };
    if (nsteps > 0) {
#pragma unroll
        for (int u = 0; u < NS - 1; ++u) issue(std::min<int64_t>(u, nsteps - 1), u);
        int64_t t = 0;
        for (; t + NS <= nsteps; t += NS) {
#pragma unroll
            for (int u = 0; u < NS; ++u) step(t + u, u);
        }
#pragma unroll
        for (int u = 0; u < NS; ++u)
            if (t + u < nsteps) step(t + u, u);
        wait_all_vmem();
    }
    // ragged tail: guarded byte loads, k = kk + 32 g + 16 c + (0..15) on both operands
    for (int64_t kk = kb + KS * nsteps; kk < ke; kk += KS) {
        uintx4 tv[MR][2];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int64_t r = row0 + 16 * a + i;
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2) {
                        const int64_t k = kk + 32 * g + 16 * c + 4 * q + t2;
                        const uint32_t byte = (r < m && k < ke) ? A[r * lda + k] : 0u;
                        w |= byte << (8 * t2);
                    }
                    tv[a][c][q] = w;
                }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = std::min(16 * b + i, s - 1);
            uintx4 xv[2];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // the plane is zero past len and at least round_up(len, 128) long
                    const uint8_t* src = plane + (int64_t)j * ldp + kk + 32 * g + 16 * c + 4 * q;
                    xv[c][q] = (uint32_t)src[0] | ((uint32_t)src[1] << 8) | ((uint32_t)src[2] << 16) |
                               ((uint32_t)src[3] << 24);
                }
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = mma_fp8(tv[a][0], tv[a][1], xv[0], xv[1], acc[a][b]);
        }
    }
    if (row0 >= m) return;
    float* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int a = 0; a < MR; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + 16 * a + 4 * g + r;
            if (row >= m) continue;
            const float sc = row_scale[row];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = 16 * b + i;
                if (j >= s) continue;
                float* d = o + (int64_t)j * ldo + row;
                const float v = acc[a][b][r] * sc * thin_scale[j];
                *d = accumulate ? *d + v : v;
            }
        }
    }
}

// FP8 co-range view: stage = 128 rows x 64*MR columns of S (bytes), chunks
// swizzled by (row >> 5) & 3 since the lane groups read rows 32 apart.
template <int NB, int MR>
__global__ void __launch_bounds__(256)
corange_fp8_kernel(const uint8_t* __restrict__ A, int64_t lda, int64_t m, int64_t n, const uint8_t* __restrict__ plane,
                   int64_t ldp, const float* __restrict__ thin_scale, int s, float* __restrict__ out, int64_t ldo,
                   int64_t split_stride, int64_t r_chunk, int accumulate) {
    constexpr int KS = 128;
    constexpr int AW = 64 * MR;
    constexpr int CH = AW / 16;
    constexpr int ABLK = KS * CH / 64;
    constexpr int TB = NB * 2;
    static_assert(ABLK % 4 == 0 && TB % 4 == 0, "copies split evenly over the four waves");
    constexpr int BLK = ABLK + TB;
    constexpr int NL = ABLK / 4 + TB / 4;
    __shared__ uintx4 st0[BLK * 64];
    __shared__ uintx4 st1[BLK * 64];
    __shared__ uintx4 st2[BLK * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
    const int64_t cw0 = (int64_t)blockIdx.x * AW;
    const int64_t col0 = cw0 + (int64_t)wave * 16 * MR;
    const int64_t rb = (int64_t)blockIdx.y * r_chunk;
    const int64_t re = std::min<int64_t>(m, rb + r_chunk);
    const int64_t nsteps = (re - rb) / KS;
    const int64_t last_cb = ((n - 1) / 16) * 16;

    const uint8_t* asrc[ABLK / 4];
#pragma unroll
    for (int u = 0; u < ABLK / 4; ++u) {
        const int L = 64 * (wave + 4 * u) + lane;
        const int row = L / CH, slot = L % CH;
        const int chunk = slot ^ ((row >> 5) & 3);
        asrc[u] = A + (rb + row) * lda + std::min<int64_t>(cw0 + 16 * chunk, last_cb);
    }
    const uint8_t* ysrc[TB / 4];
#pragma unroll
    for (int u = 0; u < TB / 4; ++u) {
        const int q = wave + 4 * u, b = q >> 1, c = q & 1;
        ysrc[u] = plane + (int64_t)std::min(16 * b + i, s - 1) * ldp + rb + 32 * g + 16 * c;
    }
    floatx4 acc[MR][NB];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = floatx4{0, 0, 0, 0};

    auto issue = [&](int64_t t, uintx4* stg) {
#pragma unroll
        for (int u = 0; u < ABLK / 4; ++u) lds_copy16(asrc[u] + t * KS * lda, stg + (wave + 4 * u) * 64);
#pragma unroll
        for (int u = 0; u < TB / 4; ++u) lds_copy16(ysrc[u] + t * KS, stg + (ABLK + wave + 4 * u) * 64);
    };
    auto step = [&](int64_t t, uintx4* cur, uintx4* nxt) {
        wait_vmcnt<NL>();
        bare_barrier();
        issue(std::min<int64_t>(t + 2, nsteps - 1), nxt);
        const uint8_t* at = (const uint8_t*)cur;
        uintx4 av[MR][2];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int cl = wave * 16 * MR + 16 * a + i;
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int row = 32 * g + 16 * c + 4 * q + t;
                        const int slot = (cl >> 4) ^ ((row >> 5) & 3);
                        w |= (uint32_t)at[(row * CH + slot) * 16 + (cl & 15)] << (8 * t);
                    }
                    av[a][c][q] = w;
                }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uintx4 y0 = cur[(ABLK + 2 * b) * 64 + lane], y1 = cur[(ABLK + 2 * b + 1) * 64 + lane];
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = mma_fp8(av[a][0], av[a][1], y0, y1, acc[a][b]);
        }
    };
    if (nsteps > 0) {
        issue(0, st0);
        issue(std::min<int64_t>(1, nsteps - 1), st1);
        int64_t t = 0;
        for (; t + 3 <= nsteps; t += 3) {
            step(t, st0, st2);
            step(t + 1, st1, st0);
            step(t + 2, st2, st1);
        }
        if (t < nsteps) step(t, st0, st2);
        if (t + 1 < nsteps) step(t + 1, st1, st0);
        wait_all_vmem();
    }
    for (int64_t rr = rb + KS * nsteps; rr < re; rr += KS) {
        uintx4 av[MR][2];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
            const int64_t c = col0 + 16 * a + i;
#pragma unroll
            for (int cc = 0; cc < 2; ++cc)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int64_t r = rr + 32 * g + 16 * cc + 4 * q + t;
                        const uint32_t byte = (c < n && r < re) ? A[r * lda + c] : 0u;
                        w |= byte << (8 * t);
                    }
                    av[a][cc][q] = w;
                }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = std::min(16 * b + i, s - 1);
            uintx4 yv[2];
#pragma unroll
            for (int cc = 0; cc < 2; ++cc)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint8_t* src = plane + (int64_t)j * ldp + rr + 32 * g + 16 * cc + 4 * q;
                    yv[cc][q] = (uint32_t)src[0] | ((uint32_t)src[1] << 8) | ((uint32_t)src[2] << 16) |
                                ((uint32_t)src[3] << 24);
                }
#pragma unroll
            for (int a = 0; a < MR; ++a) acc[a][b] = mma_fp8(av[a][0], av[a][1], yv[0], yv[1], acc[a][b]);
        }
    }
    if (col0 >= n) return;
    float* o = out + (int64_t)blockIdx.y * split_stride;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = 16 * b + i;
        if (j >= s) continue;
        const float ts = thin_scale[j];
#pragma unroll
        for (int a = 0; a < MR; ++a) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t c = col0 + 16 * a + 4 * g + q;
                if (c < n) {
                    float* d = o + (int64_t)j * ldo + c;
                    const float v = acc[a][b][q] * ts;
                    *d = accumulate ? *d + v : v;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int lp_a_kind(int dtype) { return dtype == RSVD_BF16 ? 0 : dtype == RSVD_F32 ? 1 : 2; }
int lp_bytes(int dtype) { return dtype == RSVD_BF16 ? 2 : dtype == RSVD_F32 ? 4 : 1; }

// LDS kilobytes of one stage of a launch.
int lp_stage_kb(int ak, int nt, int nb, int mr, bool corange, bool fp8) {
    if (fp8) return 8 * mr + 2 * nb;
    const int bytes = ak == 0 ? 2 : ak == 1 ? 4 : 1;
    const int a_kb = corange ? 32 * (64 * mr * bytes / 16) / 64 : (ak == 1 ? 8 * mr : ak == 0 ? 4 * mr : 4);
    return a_kb + nt * nb;
}

// Whether the three-stage ring of a BF16-path launch fits the 160 KB LDS.
template <int AK, int NT, int NB, int MR, bool CORANGE>
constexpr bool lp_ring_fits() {
    constexpr int bytes = AK == 0 ? 2 : AK == 1 ? 4 : 1;
    constexpr int a_kb = CORANGE ? 32 * (64 * MR * bytes / 16) / 64 : (AK == 1 ? 8 * MR : AK == 0 ? 4 * MR : 4);
    return 3 * (a_kb + NT * NB) <= 156;
}

int lp_nb(int s) {
    const int nb = (int)ceil_div(s, 16);
    return nb <= 4 ? 4 : nb <= 8 ? 8 : nb <= 12 ? 12 : 16;
}

#define LP_NB_SWITCH(NBV, CALL)   \
    switch (NBV) {                \
        case 4: CALL(4); break;   \
        case 8: CALL(8); break;   \
        case 12: CALL(12); break; \
        default: CALL(16); break; \
    }

template <int AK, int NT, int NB, int MR>
void launch_range_lp_mr(const LpArgs& v, dim3 grid, hipStream_t st, float* d, int64_t ldd, int64_t stride,
                        int64_t chunk, int acc) {
    hipLaunchKernelGGL((range_lp_kernel<AK, NT, NB, MR>), grid, dim3(256), 0, st, v.A, v.lda, v.m, v.n, v.row_scale,
                       (const uint16_t*)v.planes, v.ldp, v.pstride, v.s, d, ldd, stride, chunk, acc);
}

template <int AK, int NT, int NB>
void launch_range_lp(int mr, const LpArgs& v, dim3 grid, hipStream_t st, float* d, int64_t ldd, int64_t stride,
                     int64_t chunk, int acc) {
    if constexpr (AK == 2) {
        if constexpr (lp_ring_fits<AK, NT, NB, 2, false>())
            launch_range_lp_mr<AK, NT, NB, 2>(v, grid, st, d, ldd, stride, chunk, acc);
    } else {
        if constexpr (lp_ring_fits<AK, NT, NB, 2, false>()) {
            if (mr == 2) {
                launch_range_lp_mr<AK, NT, NB, 2>(v, grid, st, d, ldd, stride, chunk, acc);
                return;
            }
        }
        if constexpr (lp_ring_fits<AK, NT, NB, 1, false>())
            launch_range_lp_mr<AK, NT, NB, 1>(v, grid, st, d, ldd, stride, chunk, acc);
    }
}

// Stages of the 64-rows-per-wave range ring that fit the LDS (0: none).
constexpr int lp4_stage_kb(int ak, int nt, int nb) { return 4 * (ak == 0 ? 4 : 2) + (nt * nb + 3) / 4 * 4; }
constexpr int lp4_stages(int ak, int nt, int nb) {
    return 4 * lp4_stage_kb(ak, nt, nb) <= 156   ? 4
           : 3 * lp4_stage_kb(ak, nt, nb) <= 156 ? 3
           : 2 * lp4_stage_kb(ak, nt, nb) <= 156 ? 2
                                                 : 0;
}

template <int AK, int NT, int NB>
void launch_range_lp4(const LpArgs& v, dim3 grid, hipStream_t st, float* d, int64_t ldd, int64_t stride,
                      int64_t chunk, int acc) {
    constexpr int NS = lp4_stages(AK, NT, NB);
    static_assert(NS > 0, "the ring fits the LDS");
    hipLaunchKernelGGL((range_lp4_kernel<AK, NT, NB, NS>), grid, dim3(256), 0, st, v.A, v.lda, v.m, v.n,
                       v.row_scale, (const uint16_t*)v.planes, v.ldp, v.pstride, v.s, d, ldd, stride, chunk, acc);
}

template <int AK, int NT, int NB, int MR>
void launch_corange_lp_mr(const LpArgs& v, dim3 grid, hipStream_t st, float* d, int64_t ldd, int64_t stride,
                          int64_t chunk, int acc) {
    hipLaunchKernelGGL((corange_lp_kernel<AK, NT, NB, MR>), grid, dim3(256), 0, st, v.A, v.lda, v.m, v.n,
                       (const uint16_t*)v.planes, v.ldp, v.pstride, v.s, d, ldd, stride, chunk, acc);
}

template <int AK, int NT, int NB>
void launch_corange_lp(int mr, const LpArgs& v, dim3 grid, hipStream_t st, float* d, int64_t ldd, int64_t stride,
                       int64_t chunk, int acc) {
    if constexpr (AK == 2) {
        if constexpr (lp_ring_fits<AK, NT, NB, 2, true>())
            launch_corange_lp_mr<AK, NT, NB, 2>(v, grid, st, d, ldd, stride, chunk, acc);
    } else {
        if constexpr (lp_ring_fits<AK, NT, NB, 2, true>()) {
            if (mr == 2) {
                launch_corange_lp_mr<AK, NT, NB, 2>(v, grid, st, d, ldd, stride, chunk, acc);
                return;
            }
        }
        if constexpr (lp_ring_fits<AK, NT, NB, 1, true>())
            launch_corange_lp_mr<AK, NT, NB, 1>(v, grid, st, d, ldd, stride, chunk, acc);
    }
}

// Stages of the register-streamed FP8 range ring (thin tile 2 NB KB per stage).
constexpr int kFp8RsStages = 3;

template <int NB>
void launch_range_fp8(int mr, const LpArgs& v, dim3 grid, hipStream_t st, float* d, int64_t ldd, int64_t stride,
                      int64_t chunk, int acc) {
    if constexpr (NB <= 14) {
        if (mr == 4) {
            hipLaunchKernelGGL((range_fp8_rs_kernel<NB, 4, kFp8RsStages>), grid, dim3(256), 0, st,
                               (const uint8_t*)v.A, v.lda, v.m, v.n, v.row_scale, (const uint8_t*)v.planes, v.ldp,
                               v.thin_scale, v.s, d, ldd, stride, chunk, acc);
            return;
        }
    }
    if (mr == 2)
        hipLaunchKernelGGL((range_fp8_kernel<NB, 2>), grid, dim3(256), 0, st, (const uint8_t*)v.A, v.lda, v.m, v.n,
                           v.row_scale, (const uint8_t*)v.planes, v.ldp, v.thin_scale, v.s, d, ldd, stride, chunk, acc);
    else
        hipLaunchKernelGGL((range_fp8_kernel<NB, 1>), grid, dim3(256), 0, st, (const uint8_t*)v.A, v.lda, v.m, v.n,
                           v.row_scale, (const uint8_t*)v.planes, v.ldp, v.thin_scale, v.s, d, ldd, stride, chunk, acc);
}

template <int NB>
void launch_corange_fp8(int mr, const LpArgs& v, dim3 grid, hipStream_t st, float* d, int64_t ldd, int64_t stride,
                        int64_t chunk, int acc) {
    if (mr == 2)
        hipLaunchKernelGGL((corange_fp8_kernel<NB, 2>), grid, dim3(256), 0, st, (const uint8_t*)v.A, v.lda, v.m, v.n,
                           (const uint8_t*)v.planes, v.ldp, v.thin_scale, v.s, d, ldd, stride, chunk, acc);
    else
        hipLaunchKernelGGL((corange_fp8_kernel<NB, 1>), grid, dim3(256), 0, st, (const uint8_t*)v.A, v.lda, v.m, v.n,
                           (const uint8_t*)v.planes, v.ldp, v.thin_scale, v.s, d, ldd, stride, chunk, acc);
}

}  // namespace

int64_t lp_plane_ld(int64_t len) { return round_up(len, 128); }

size_t lp_thin_bytes(int thin_kind, int s, int64_t len) {
    const int64_t ldp = lp_plane_ld(len);
    if (thin_kind == LP_THIN_FP8) return (size_t)s * ldp + 256 + (size_t)s * 4;
    return (size_t)thin_kind * s * ldp * 2;
}

bool lp_aligned(int dtype, const void* A, int64_t lda) {
    const int64_t bytes = lp_bytes(dtype);
    return ((uintptr_t)A & 15) == 0 && (lda * bytes) % 16 == 0;
}

rsvd_status lp_prepare_thin(const float* P, int64_t ld, int s, int64_t len, const float* len_scale, int thin_kind,
                            void* buf, LpArgs& v, hipStream_t st) {
    const int64_t ldp = lp_plane_ld(len);
    const int64_t total = (int64_t)s * ldp;
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 16384);
    v.ldp = ldp;
    v.pstride = total;
    v.s = s;
    v.planes = buf;
    v.thin_scale = nullptr;
    if (thin_kind == LP_THIN_FP8) {
        uint8_t* plane = (uint8_t*)buf;
        float* scale = (float*)((char*)buf + round_up(total, 256));
        hipLaunchKernelGGL(thin_amax_kernel, dim3(s), dim3(256), 0, st, P, ld, len, len_scale, scale);
        hipLaunchKernelGGL(thin_fp8_kernel, dim3(blocks), dim3(256), 0, st, P, ld, s, len, len_scale,
                           (const float*)scale, plane, ldp);
        v.thin_scale = scale;
    } else if (thin_kind == LP_THIN_BF16) {
        hipLaunchKernelGGL(thin_split_kernel<1>, dim3(blocks), dim3(256), 0, st, P, ld, s, len, len_scale,
                           (uint16_t*)buf, ldp);
    } else {
        hipLaunchKernelGGL(thin_split_kernel<3>, dim3(blocks), dim3(256), 0, st, P, ld, s, len, len_scale,
                           (uint16_t*)buf, ldp);
    }
    v.thin_kind = thin_kind;
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}

// Whether a range view takes the 64-rows-per-wave kernel: a BF16 A (or an
// FP8 A through BF16) with BF16 thin planes, and enough rows to give every
// CU a 256-row workgroup without splitting the contraction.
static bool lp4_applies(const LpArgs& v, bool corange, int num_cu) {
    const int ak = lp_a_kind(v.dtype);
    return !corange && v.thin_kind != LP_THIN_FP8 && ak != 1 && v.m >= (int64_t)256 * num_cu;
}

// Whether an FP8 range view takes the register-streamed kernel: enough rows to
// give every CU a 256-row workgroup without splitting the contraction.
static bool fp8_rs_applies(const LpArgs& v, bool corange, int num_cu) {
    // up to 14 thin blocks: 16 would not leave the A ring its registers
    return !corange && v.thin_kind == LP_THIN_FP8 && v.m >= (int64_t)256 * num_cu && v.s <= 224;
}

// Thin blocks of the 64-rows-per-wave kernel: ceil(s / 16), with 14 between 12 and 16.
static int lp4_nb(int s) {
    const int nb = (int)ceil_div(s, 16);
    return nb <= 4 ? 4 : nb <= 8 ? 8 : nb <= 12 ? 12 : nb <= 14 ? 14 : 16;
}

// Tiles and splits: as the FP32 plan, with chunks in whole stages and the
// rows (columns) per wave reduced until the ring fits the LDS; tall range
// views take 64 rows per wave (mr = 4).
ViewPlan plan_lp(const LpArgs& v, bool corange, int num_cu) {
    ViewPlan p;
    const bool fp8 = v.thin_kind == LP_THIN_FP8;
    const int ak = lp_a_kind(v.dtype);
    const int nt = fp8 ? 1 : v.thin_kind;
    p.nb = lp_nb(v.s);
    const int64_t out_len = corange ? v.n : v.m;
    const int64_t contraction = corange ? v.m : v.n;
    int mr = (out_len < 8192) ? 1 : 2;
    while (mr > 1 && 3 * lp_stage_kb(ak, nt, p.nb, mr, corange, fp8) > 156) --mr;
    if (!fp8 && ak == 2) mr = 2;   // FP8 A through the BF16 path: 32 rows (columns) per wave
    if (lp4_applies(v, corange, num_cu) || fp8_rs_applies(v, corange, num_cu)) {
        p.nb = lp4_nb(v.s);
        mr = 4;
    }
    p.mr = mr;
    p.tiles = ceil_div(out_len, 64 * mr);
    const int ks = fp8 ? 128 : 32;
    const int64_t s_pad = 16 * (int64_t)p.nb;
    int64_t splits = 1;
    while (p.tiles * splits < 2 * num_cu && ceil_div(contraction, splits * 2) >= 4 * ks &&
           (splits * 2) * s_pad * 8 <= contraction && splits < 256)
        splits *= 2;
    p.chunk = round_up(ceil_div(contraction, splits), ks);
    p.splits = ceil_div(contraction, p.chunk);
    return p;
}

bool lp_fits(const LpArgs& v, bool corange) {
    const bool fp8 = v.thin_kind == LP_THIN_FP8;
    const int ak = lp_a_kind(v.dtype);
    const int nt = fp8 ? 1 : v.thin_kind;
    return 3 * lp_stage_kb(ak, nt, lp_nb(v.s), (!fp8 && ak == 2) ? 2 : 1, corange, fp8) <= 156;
}

rsvd_status run_lp(const LpArgs& v, const ViewPlan& p, bool corange, float* out, int64_t ldo, float* partial,
                   int accumulate, hipStream_t st) {
    if (v.s > 256 || !lp_fits(v, corange)) return RSVD_EUNSUPPORTED;
    if (!lp_aligned(v.dtype, v.A, v.lda)) return RSVD_EINVAL;
    const int64_t out_len = corange ? v.n : v.m;
    dim3 grid((unsigned)p.tiles, (unsigned)p.splits);
    float* dst = p.splits > 1 ? partial : out;
    const int64_t ldd = p.splits > 1 ? out_len : ldo;
    const int64_t stride = (int64_t)v.s * out_len;
    const int dacc = p.splits > 1 ? 0 : accumulate;
    const int ak = lp_a_kind(v.dtype);
    if (v.thin_kind == LP_THIN_FP8) {
        if (v.dtype != RSVD_FP8_E4M3) return RSVD_EINVAL;
        if (p.mr == 4) {
            if (corange) return RSVD_EINVAL;
            switch (p.nb) {
                case 4: launch_range_fp8<4>(4, v, grid, st, dst, ldd, stride, p.chunk, dacc); break;
                case 8: launch_range_fp8<8>(4, v, grid, st, dst, ldd, stride, p.chunk, dacc); break;
                case 12: launch_range_fp8<12>(4, v, grid, st, dst, ldd, stride, p.chunk, dacc); break;
                case 14: launch_range_fp8<14>(4, v, grid, st, dst, ldd, stride, p.chunk, dacc); break;
                default: return RSVD_EINVAL;   // the plan takes this kernel up to 14 thin blocks only
            }
        } else {
#define LP_FP8(NBV)                                                                        \
    if (corange) launch_corange_fp8<NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc); \
    else launch_range_fp8<NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc)
            LP_NB_SWITCH(p.nb, LP_FP8);
#undef LP_FP8
        }
    } else if (p.mr == 4) {
        if (corange || ak == 1) return RSVD_EINVAL;
#define LP_R4(NBV)                                                                                      \
    if (v.thin_kind == LP_THIN_BF16) {                                                                  \
        if (ak == 0) launch_range_lp4<0, 1, NBV>(v, grid, st, dst, ldd, stride, p.chunk, dacc);         \
        else launch_range_lp4<2, 1, NBV>(v, grid, st, dst, ldd, stride, p.chunk, dacc);                 \
    } else {                                                                                            \
        if (ak == 0) launch_range_lp4<0, 3, NBV>(v, grid, st, dst, ldd, stride, p.chunk, dacc);         \
        else launch_range_lp4<2, 3, NBV>(v, grid, st, dst, ldd, stride, p.chunk, dacc);                 \
    }
        switch (p.nb) {
            case 4: LP_R4(4); break;
            case 8: LP_R4(8); break;
            case 12: LP_R4(12); break;
            case 14: LP_R4(14); break;
            default: LP_R4(16); break;
        }
#undef LP_R4
    } else if (v.thin_kind == LP_THIN_BF16) {
        if (ak == 1) return RSVD_EINVAL;
#define LP_B1(NBV)                                                                                          \
    if (ak == 0) {                                                                                          \
        if (corange) launch_corange_lp<0, 1, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);       \
        else launch_range_lp<0, 1, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);                 \
    } else {                                                                                                \
        if (corange) launch_corange_lp<2, 1, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);       \
        else launch_range_lp<2, 1, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);                 \
    }
        LP_NB_SWITCH(p.nb, LP_B1);
#undef LP_B1
    } else {
#define LP_B3(NBV)                                                                                          \
    if (ak == 0) {                                                                                          \
        if (corange) launch_corange_lp<0, 3, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);       \
        else launch_range_lp<0, 3, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);                 \
    } else if (ak == 1) {                                                                                   \
        if (corange) launch_corange_lp<1, 3, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);       \
        else launch_range_lp<1, 3, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);                 \
    } else {                                                                                                \
        if (corange) launch_corange_lp<2, 3, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);       \
        else launch_range_lp<2, 3, NBV>(p.mr, v, grid, st, dst, ldd, stride, p.chunk, dacc);                 \
    }
        LP_NB_SWITCH(p.nb, LP_B3);
#undef LP_B3
    }
    RSVD_LAUNCH_CHECK();
    if (p.splits > 1) return run_reduce_parts_f32(partial, (int)p.splits, stride, v.s, out_len, out, ldo, accumulate, st);
    return RSVD_OK;
}
