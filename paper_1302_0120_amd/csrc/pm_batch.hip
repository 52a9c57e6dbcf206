// pm_batch.hip -- batched row and column passes: one launch covers every
// mask of a batch, each work-group taking one task (mask, first line) and
// running the pass body for that mask's size under the FFT schedule SCHED.
// Compiled once per (pass mode, schedule): PM_BATCH_WHICH = 0 .. 5 and
// PM_BATCH_SCHED = 0 .. kBatchSchedules - 1, in parallel.
#include <hip/hip_ext.h>

#include "pm_kernels.hpp"

#ifndef PM_BATCH_WHICH
#error "compile with -DPM_BATCH_WHICH=<0..5>"
#endif
#ifndef PM_BATCH_SCHED
#error "compile with -DPM_BATCH_SCHED=<schedule>"
#endif

namespace pm {

template <int SCHED, int L>
struct BatchShape {
    static constexpr int P = batch_points(SCHED, L);
    static constexpr int G = batch_lines(SCHED, L);
    static constexpr int FLOATS2 = LdsPlan<L, G, 1>::FLOATS2;  // one exchange buffer (LdsPlan)
    // Last FFT stage across lanes where the tile has the lane layout for it
    // (a strip of kC columns, or 4 rows): 16-16-4 at 1024.
    static constexpr bool SW_COL = lane_swap_plan(L, P) && G == kC;
    static constexpr bool SW_ROW = lane_swap_plan(L, P) && G == 4;
};

template <int SCHED>
constexpr int batch_lds_floats2() {
    const int f[5] = {BatchShape<SCHED, 64>::FLOATS2, BatchShape<SCHED, 128>::FLOATS2,
                      BatchShape<SCHED, 256>::FLOATS2, BatchShape<SCHED, 512>::FLOATS2,
                      BatchShape<SCHED, 1024>::FLOATS2};
    int m = 0;
    for (int i = 0; i < 5; ++i) m = f[i] > m ? f[i] : m;
    return m;
}

// One case per transform length: the staged twiddle table of (L, P) and the
// pass body with one LDS exchange buffer (LdsPlan, NBMAX = 1).
#define PM_COL_CASE(L)                                                                    \
    case L:                                                                               \
        a.tw = p.tw + batch_twiddle_offset(SCHED, L);                                     \
        col_body<L, BatchShape<SCHED, L>::P, BatchShape<SCHED, L>::G, MODE,               \
                 BatchShape<SCHED, L>::SW_COL, 1>(                                        \
            a, task.first, slot, lds, red);                                               \
        break;
#define PM_ROW_CASE(L)                                                                    \
    case L:                                                                               \
        a.tw = p.tw + batch_twiddle_offset(SCHED, L);                                     \
        row_body<L, BatchShape<SCHED, L>::P, BatchShape<SCHED, L>::G, MODE,               \
                 BatchShape<SCHED, L>::SW_ROW, 1>(                                        \
            a, task.first, pin, pout, slot, lds, red);                                    \
        break;

template <int MODE, int SCHED>
__global__ void __launch_bounds__(kBatchThreads) k_col_batch(BatchParams p) {
    __shared__ float2 lds[batch_lds_floats2<SCHED>()];
    __shared__ double red[kBatchThreads / 64];
    const BatchTask task = p.tasks[blockIdx.x];
    const BatchMask mk = p.masks[task.mask];
    ColParams a{};
    a.X = mk.X;
    a.mhat = mk.mhat;
    a.W = mk.W;
    a.invN = 1.0 / ((double)mk.H * (double)mk.W);
    double* slot = p.part + blockIdx.x * red_slots(kBatchThreads);
    switch (mk.H) {
        PM_COL_CASE(64)
        PM_COL_CASE(128)
        PM_COL_CASE(256)
        PM_COL_CASE(512)
        PM_COL_CASE(1024)
        default: break;
    }
}

template <int MODE, int SCHED>
__global__ void __launch_bounds__(kBatchThreads) k_row_batch(BatchParams p) {
    __shared__ float2 lds[batch_lds_floats2<SCHED>()];
    __shared__ double red[kBatchThreads / 64];
    const BatchTask task = p.tasks[blockIdx.x];
    const BatchMask mk = p.masks[task.mask];
    RowParams a{};
    a.X = mk.X;
    a.H = mk.H;
    const float* pin = nullptr;
    float* pout = nullptr;
    if constexpr ((MODE & RIN_PHASE) != 0) pin = p.io->phases_in[task.mask];
    if constexpr ((MODE & ROUT_PHASE) != 0) pout = p.io->phases_out[task.mask];
    double* slot = p.part + blockIdx.x * red_slots(kBatchThreads);
    switch (mk.W) {
        PM_ROW_CASE(64)
        PM_ROW_CASE(128)
        PM_ROW_CASE(256)
        PM_ROW_CASE(512)
        PM_ROW_CASE(1024)
        default: break;
    }
}

template <typename K>
hipError_t launch_k(K kern, const BatchParams& p, int grid, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (ev0 != nullptr || ev1 != nullptr) {
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBatchThreads), 0, s, ev0, ev1, 0, p);
    } else {
        kern<<<grid, kBatchThreads, 0, s>>>(p);
    }
    return hipGetLastError();
}

template <int MODE, int SCHED>
hipError_t launch_batch_col(const BatchParams& p, int grid, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    return launch_k(k_col_batch<MODE, SCHED>, p, grid, s, ev0, ev1);
}

template <int MODE, int SCHED>
hipError_t launch_batch_row(const BatchParams& p, int grid, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    return launch_k(k_row_batch<MODE, SCHED>, p, grid, s, ev0, ev1);
}

#define PM_INST_COL(MODE) \
    template hipError_t launch_batch_col<MODE, PM_BATCH_SCHED>(const BatchParams&, int, hipStream_t, hipEvent_t, hipEvent_t);
#define PM_INST_ROW(MODE) \
    template hipError_t launch_batch_row<MODE, PM_BATCH_SCHED>(const BatchParams&, int, hipStream_t, hipEvent_t, hipEvent_t);

#if PM_BATCH_WHICH == 0
PM_INST_COL(COL_ITER_NE)
#elif PM_BATCH_WHICH == 1
PM_INST_COL(COL_ERR)
#elif PM_BATCH_WHICH == 2
PM_INST_ROW(ROW_INIT)
#elif PM_BATCH_WHICH == 3
PM_INST_ROW(ROW_ITER_NE)
#elif PM_BATCH_WHICH == 4
PM_INST_ROW(ROW_LAST_NE)
#elif PM_BATCH_WHICH == 5
PM_INST_ROW(ROW_LAST_FWD_NE)
#endif

}  // namespace pm
