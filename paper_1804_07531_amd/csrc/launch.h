// Launching kernels one matrix at a time or as a batch.
//
// A kernel on the batched path is written as an Op: a struct with the
// workgroup size kThreads, its arguments Args (an aggregate: call sites pass
// a braced list in field order, and run() copies them into locals with one
// structured binding) and a device function run(vg, args) in which the
// workgroup coordinates come from vg instead of blockIdx / gridDim.
// launch_op launches op_single<Op> on a stream; while a LaunchRecorder is
// installed (planning a batch) it records the launch instead, and the batch
// later replays every recorded step of every matrix as one op_batched<Op>
// launch in which blockIdx.z selects the matrix's job.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

struct VGrid {
    unsigned bx, by, gx, gy;
};

// Workgroups per compute unit the compiler should leave room for: an Op may
// set kMinBlocks (as the second argument of __launch_bounds__); 0 leaves the
// compiler's default.
template <class Op, class = void>
struct op_min_blocks {
    static constexpr int value = 0;
};
template <class Op>
struct op_min_blocks<Op, decltype((void)Op::kMinBlocks)> {
    static constexpr int value = Op::kMinBlocks;
};

template <class Op>
__global__ void __launch_bounds__(Op::kThreads) op_single(typename Op::Args a) {
    Op::run(VGrid{blockIdx.x, blockIdx.y, gridDim.x, gridDim.y}, a);
}

template <class Op>
__global__ void __launch_bounds__(Op::kThreads, (op_min_blocks<Op>::value > 0 ? op_min_blocks<Op>::value : 1))
op_single_mb(typename Op::Args a) {
    Op::run(VGrid{blockIdx.x, blockIdx.y, gridDim.x, gridDim.y}, a);
}

template <class Op>
struct OpJob {
    typename Op::Args a;
    unsigned gx, gy;
};

template <class Op>
__global__ void __launch_bounds__(Op::kThreads, (op_min_blocks<Op>::value > 0 ? op_min_blocks<Op>::value : 1))
op_batched(const OpJob<Op>* __restrict__ jobs) {
    const OpJob<Op>* j = jobs + blockIdx.z;
    const unsigned gx = j->gx, gy = j->gy;
    if (blockIdx.x >= gx || blockIdx.y >= gy) return;
    const typename Op::Args a = j->a;
    Op::run(VGrid{blockIdx.x, blockIdx.y, gx, gy}, a);
}

// Receives the launches of one matrix's call while a batch is planned.
struct LaunchRecorder {
    virtual ~LaunchRecorder() {}
    virtual void add(const void* batched_fn, const void* single_fn, const void* job, size_t job_size, dim3 grid,
                     unsigned threads, size_t shmem) = 0;
    // a new step of the driver begins (its launches, including optional
    // follow-ups such as partial-sum reductions, share the step)
    virtual void phase() {}
};

// The single-launch kernel of an Op (for hipFuncSetAttribute).
template <class Op>
inline const void* op_single_fn() {
    if constexpr (op_min_blocks<Op>::value > 0) return reinterpret_cast<const void*>(&op_single_mb<Op>);
    else return reinterpret_cast<const void*>(&op_single<Op>);
}

// The recorder of the current thread (null outside batch planning).
LaunchRecorder*& launch_recorder();

// Marks the start of a driver step (no-op outside batch planning).
inline void launch_phase() {
    if (LaunchRecorder* r = launch_recorder()) r->phase();
}

// A failed launch is left in HIP's last error (not read here), for the
// caller's next launch check to report.
template <class Op>
inline void launch_op(dim3 grid, dim3 block, size_t shmem, hipStream_t st, const typename Op::Args& a) {
    if (LaunchRecorder* r = launch_recorder()) {
        OpJob<Op> j;
        j.a = a;
        j.gx = grid.x;
        j.gy = grid.y;
        r->add(reinterpret_cast<const void*>(&op_batched<Op>), op_single_fn<Op>(), &j, sizeof(j), grid, block.x,
               shmem);
        return;
    }
    if constexpr (op_min_blocks<Op>::value > 0) hipLaunchKernelGGL(op_single_mb<Op>, grid, block, shmem, st, a);
    else hipLaunchKernelGGL(op_single<Op>, grid, block, shmem, st, a);
}


