// Gaussian test matrices from a counter-based generator.
//
// The paper's randn (Sect. 2) asks for independent standard Gaussian entries.
// Here every entry is a pure function of (seed, tag, batch, long index i,
// short index j): Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) on the
// counter (i >> 2, j, batch, tag) with key (seed mod 2^32, seed >> 32) gives
// four 32-bit words; word w becomes the uniform (w + 1/2) 2^-32, and the
// Box-Muller transform (Box & Muller 1958) of words (0,1) and (2,3) gives
// four normals, of which entry i takes number i & 3.  The value is evaluated
// in FP64 and rounded once to the working precision.
#include "common.h"
#include "launch.h"
#include "philox.h"

namespace {

// Each thread evaluates one Philox block: 4 consecutive long indices of one
// short index, and writes them to the row-major output.
template <typename T>
struct gaussian_fill_kernel_op {
    static constexpr int kThreads = 256;
    struct Args {
        uint64_t seed;
        uint32_t tag;
        uint32_t batch;
        int64_t n_long;
        int64_t n_short;
        int long_is_row;
        T*  out;
        int64_t ld;
    };
    static __device__ __forceinline__ void run(const VGrid vg, const Args& args_) {
        const auto [seed, tag, batch, n_long, n_short, long_is_row, out, ld] = args_;
        const int64_t nq = ceil_div(n_long, 4);
        const int64_t total = nq * n_short;
        for (int64_t idx = vg.bx * (int64_t)blockDim.x + threadIdx.x; idx < total;
             idx += (int64_t)vg.gx * blockDim.x) {
            int64_t q, j;
            if (long_is_row) {      // neighbouring threads write neighbouring columns
                q = idx / n_short;
                j = idx % n_short;
            } else {                // neighbouring threads write neighbouring 4-wide groups of one row
                j = idx / nq;
                q = idx % nq;
            }
            double z[4];
            philox_normal4(seed, tag, batch, (uint32_t)q, (uint32_t)j, z);
    #pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t i = 4 * q + t;
                if (i < n_long) {
                    if (long_is_row) out[i * ld + j] = (T)z[t];
                    else out[j * ld + i] = (T)z[t];
                }
            }
        }
    }
};

}  // namespace

rsvd_status launch_gaussian(uint64_t seed, uint32_t tag, uint32_t batch, int64_t rows, int64_t cols,
                            int long_is_row, int dtype, void* out, int64_t ld, hipStream_t stream) {
    launch_phase();
    const int64_t n_long = long_is_row ? rows : cols;
    const int64_t n_short = long_is_row ? cols : rows;
    if (n_long <= 0 || n_short <= 0) return RSVD_OK;
    const int64_t total = ceil_div(n_long, 4) * n_short;
    const int64_t blocks = std::min<int64_t>(ceil_div(total, 256), 65536);
    if (dtype == RSVD_F64)
        launch_op<gaussian_fill_kernel_op<double>>(dim3((unsigned)blocks), dim3(256), 0, stream, {seed, tag, batch, n_long, n_short, long_is_row, (double*)out, ld});
    else if (dtype == RSVD_F32)
        launch_op<gaussian_fill_kernel_op<float>>(dim3((unsigned)blocks), dim3(256), 0, stream, {seed, tag, batch, n_long, n_short, long_is_row, (float*)out, ld});
    else
        return RSVD_EINVAL;
    RSVD_LAUNCH_CHECK();
    return RSVD_OK;
}
