// pm_batch.hip -- batched row and column passes: one launch covers every
// mask of a batch, each work-group taking one task (mask, first line) and
// running the pass body for that mask's size.  Compiled once per pass mode
// (PM_BATCH_WHICH = 0 .. 5), in parallel.
#include "pm_kernels.hpp"

#ifndef PM_BATCH_WHICH
#error "compile with -DPM_BATCH_WHICH=<0..5>"
#endif

namespace pm {

// Lines per work-group for a transform of length L at kBatchThreads threads.
template <int L>
struct BatchShape {
    static constexpr int G = kBatchThreads / LineShape<L>::T;
};

constexpr int batch_lds_floats2() {
    int m = 0;
    const int f[5] = {LdsPlan<64, BatchShape<64>::G>::FLOATS2, LdsPlan<128, BatchShape<128>::G>::FLOATS2,
                      LdsPlan<256, BatchShape<256>::G>::FLOATS2, LdsPlan<512, BatchShape<512>::G>::FLOATS2,
                      LdsPlan<1024, BatchShape<1024>::G>::FLOATS2};
    for (int i = 0; i < 5; ++i) m = f[i] > m ? f[i] : m;
    return m;
}
constexpr int kBatchLds = batch_lds_floats2();

template <int MODE>
__global__ void __launch_bounds__(kBatchThreads) k_col_batch(BatchParams p) {
    __shared__ float2 lds[kBatchLds];
    __shared__ double red[kBatchThreads / 64];
    const BatchTask task = p.tasks[blockIdx.x];
    const BatchMask mk = p.masks[task.mask];
    ColParams a{};
    a.X = mk.X;
    a.mhat = mk.mhat;
    a.tw = p.tw;
    a.W = mk.W;
    a.invN = 1.0 / ((double)mk.H * (double)mk.W);
    double* slot = p.part + blockIdx.x;
    switch (mk.H) {
        case 64: a.tw_step = kBatchMaxLen / 64; col_body<64, BatchShape<64>::G, MODE>(a, task.first, slot, lds, red); break;
        case 128: a.tw_step = kBatchMaxLen / 128; col_body<128, BatchShape<128>::G, MODE>(a, task.first, slot, lds, red); break;
        case 256: a.tw_step = kBatchMaxLen / 256; col_body<256, BatchShape<256>::G, MODE>(a, task.first, slot, lds, red); break;
        case 512: a.tw_step = kBatchMaxLen / 512; col_body<512, BatchShape<512>::G, MODE>(a, task.first, slot, lds, red); break;
        case 1024: a.tw_step = 1; col_body<1024, BatchShape<1024>::G, MODE>(a, task.first, slot, lds, red); break;
        default: break;
    }
}

template <int MODE>
__global__ void __launch_bounds__(kBatchThreads) k_row_batch(BatchParams p) {
    __shared__ float2 lds[kBatchLds];
    __shared__ double red[kBatchThreads / 64];
    const BatchTask task = p.tasks[blockIdx.x];
    const BatchMask mk = p.masks[task.mask];
    RowParams a{};
    a.X = mk.X;
    a.tw = p.tw;
    a.H = mk.H;
    const float* pin = nullptr;
    float* pout = nullptr;
    if constexpr ((MODE & RIN_PHASE) != 0) pin = p.io->phases_in[task.mask];
    if constexpr ((MODE & ROUT_PHASE) != 0) pout = p.io->phases_out[task.mask];
    double* slot = p.part + blockIdx.x;
    switch (mk.W) {
        case 64: a.tw_step = kBatchMaxLen / 64; row_body<64, BatchShape<64>::G, MODE>(a, task.first, pin, pout, slot, lds, red); break;
        case 128: a.tw_step = kBatchMaxLen / 128; row_body<128, BatchShape<128>::G, MODE>(a, task.first, pin, pout, slot, lds, red); break;
        case 256: a.tw_step = kBatchMaxLen / 256; row_body<256, BatchShape<256>::G, MODE>(a, task.first, pin, pout, slot, lds, red); break;
        case 512: a.tw_step = kBatchMaxLen / 512; row_body<512, BatchShape<512>::G, MODE>(a, task.first, pin, pout, slot, lds, red); break;
        case 1024: a.tw_step = 1; row_body<1024, BatchShape<1024>::G, MODE>(a, task.first, pin, pout, slot, lds, red); break;
        default: break;
    }
}

template <int MODE>
hipError_t launch_batch_col(const BatchParams& p, int grid, hipStream_t s) {
    k_col_batch<MODE><<<grid, kBatchThreads, 0, s>>>(p);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_batch_row(const BatchParams& p, int grid, hipStream_t s) {
    k_row_batch<MODE><<<grid, kBatchThreads, 0, s>>>(p);
    return hipGetLastError();
}

#if PM_BATCH_WHICH == 0
template hipError_t launch_batch_col<COL_ITER_NE>(const BatchParams&, int, hipStream_t);
#elif PM_BATCH_WHICH == 1
template hipError_t launch_batch_col<COL_ERR>(const BatchParams&, int, hipStream_t);
#elif PM_BATCH_WHICH == 2
template hipError_t launch_batch_row<ROW_INIT>(const BatchParams&, int, hipStream_t);
#elif PM_BATCH_WHICH == 3
template hipError_t launch_batch_row<ROW_ITER_NE>(const BatchParams&, int, hipStream_t);
#elif PM_BATCH_WHICH == 4
template hipError_t launch_batch_row<ROW_LAST_NE>(const BatchParams&, int, hipStream_t);
#elif PM_BATCH_WHICH == 5
template hipError_t launch_batch_row<ROW_LAST_FWD_NE>(const BatchParams&, int, hipStream_t);
#endif

}  // namespace pm
