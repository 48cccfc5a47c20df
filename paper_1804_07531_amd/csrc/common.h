// Shared device/host helpers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsvd.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

#define RSVD_WAVE 64

// Status word bits written by kernels into the workspace header.
#define RSVD_FLAG_SHIFTED 1u
#define RSVD_FLAG_PIVOT 2u
#define RSVD_FLAG_NONFINITE 4u
#define RSVD_FLAG_SYNC_TIMEOUT 16u   // the wide small SVD's workgroups did not meet at a grid barrier in time
#define RSVD_FLAG_BAD_ENTRY 32u      // a streamed update entry lay outside A and was skipped

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Record a status flag (vector atomic OR on a global word).
__device__ inline void rsvd_flag(uint32_t* status, uint32_t bit) {
    if (status) atomicOr(status, bit);
}

// ---------------------------------------------------------------------------
// Element loads of the stored A, converted to the working type.
// ---------------------------------------------------------------------------
template <typename T> struct elem;
template <> struct elem<double> { static __device__ __forceinline__ double ld(const double* p) { return *p; } };
template <> struct elem<float> { static __device__ __forceinline__ float ld(const float* p) { return *p; } };

// ---------------------------------------------------------------------------
// 16x16x4 matrix-core step in the working precision.  Operand layout (both
// FP32 and FP64 variants): lane l = 16 g + i supplies A[i][kk = g] and
// B[kk = g][j = i].  Accumulator register r of lane l holds C[row(g, r)][i]
// with row = 4 g + r for FP32 and row = g + 4 r for FP64 (the two
// instructions interleave their result rows differently; checked on gfx950).
// ---------------------------------------------------------------------------
template <typename T> struct mfma16;
template <> struct mfma16<float> {
    typedef floatx4 acc;
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};
template <> struct mfma16<double> {
    typedef doublex4 acc;
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};

// Device-only instructions used by the streaming kernels.  Their bodies exist
// only in the device compilation pass: the host pass, which must still emit
// the launch stubs of the kernel templates that call them, cannot lower
// these builtins.
__device__ __forceinline__ void lds_copy16(const void* gsrc, void* lds_dst) {
#if defined(__HIP_DEVICE_COMPILE__)
    // global_load_lds_dwordx4: lane l writes 16 bytes at lds_dst + 16 l
    __builtin_amdgcn_global_load_lds(gsrc, lds_dst, 16, 0, 0);
#endif
}

template <int NLOADS>
__device__ __forceinline__ void wait_vmcnt() {
#if defined(__HIP_DEVICE_COMPILE__)
    // s_waitcnt vmcnt(NLOADS) with expcnt and lgkmcnt left alone
    __builtin_amdgcn_s_waitcnt((NLOADS & 15) | (7 << 4) | (15 << 8) | (((NLOADS >> 4) & 3) << 14));
#endif
}

__device__ __forceinline__ void wait_all_vmem() {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_s_waitcnt(0);
#endif
}

__device__ __forceinline__ void bare_barrier() {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_s_barrier();
#endif
}

// Host-side launch checking.
#define RSVD_LAUNCH_CHECK()                               \
    do {                                                  \
        hipError_t e_ = hipGetLastError();                \
        if (e_ != hipSuccess) return RSVD_EHIP;           \
    } while (0)
