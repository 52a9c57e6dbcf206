// pm_pass.hip -- instantiates the row and column passes for one transform
// length, given at compile time as PM_L (the build compiles this file once
// per supported length, in parallel).
#include <hip/hip_ext.h>

#include "pm_kernels.hpp"

#ifndef PM_L
#error "compile with -DPM_L=<transform length>"
#endif

#define PM_CAT2(a, b) a##b
#define PM_CAT(a, b) PM_CAT2(a, b)

namespace pm {

namespace {

template <typename Params>
hipError_t launch(void (*kern)(Params), int grid, int block, hipStream_t s, hipEvent_t ev0,
                  hipEvent_t ev1, const Params& p) {
    if (ev0 != nullptr || ev1 != nullptr) {
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, ev0, ev1, 0, p);
    } else {
        kern<<<grid, block, 0, s>>>(p);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t PM_CAT(launch_row_, PM_L)(int mode, const RowParams& p, int grid, hipStream_t s,
                                     hipEvent_t ev0, hipEvent_t ev1) {
    const int block = kGR * LineShape<PM_L>::T;
    switch (mode) {
        case ROW_INIT: return launch(k_row<PM_L, ROW_INIT>, grid, block, s, ev0, ev1, p);
        case ROW_ITER: return launch(k_row<PM_L, ROW_ITER>, grid, block, s, ev0, ev1, p);
        case ROW_LAST: return launch(k_row<PM_L, ROW_LAST>, grid, block, s, ev0, ev1, p);
        case ROW_LAST_FWD: return launch(k_row<PM_L, ROW_LAST_FWD>, grid, block, s, ev0, ev1, p);
        case ROW_GAP: return launch(k_row<PM_L, ROW_GAP>, grid, block, s, ev0, ev1, p);
        case ROW_FFT_FWD: return launch(k_row<PM_L, ROW_FFT_FWD>, grid, block, s, ev0, ev1, p);
        case ROW_FFT_INV: return launch(k_row<PM_L, ROW_FFT_INV>, grid, block, s, ev0, ev1, p);
        case ROW_ITER_NE: return launch(k_row<PM_L, ROW_ITER_NE>, grid, block, s, ev0, ev1, p);
        case ROW_LAST_NE: return launch(k_row<PM_L, ROW_LAST_NE>, grid, block, s, ev0, ev1, p);
        default: return hipErrorInvalidValue;
    }
}

hipError_t PM_CAT(launch_col_, PM_L)(int mode, const ColParams& p, int grid, hipStream_t s,
                                     hipEvent_t ev0, hipEvent_t ev1) {
    const int block = kC * LineShape<PM_L>::T;
    switch (mode) {
        case COL_ITER: return launch(k_col<PM_L, COL_ITER>, grid, block, s, ev0, ev1, p);
        case COL_ERR: return launch(k_col<PM_L, COL_ERR>, grid, block, s, ev0, ev1, p);
        case COL_FFT_FWD: return launch(k_col<PM_L, COL_FFT_FWD>, grid, block, s, ev0, ev1, p);
        case COL_FFT_INV: return launch(k_col<PM_L, COL_FFT_INV>, grid, block, s, ev0, ev1, p);
        case COL_ITER_NE: return launch(k_col<PM_L, COL_ITER_NE>, grid, block, s, ev0, ev1, p);
        case COL_INIT_BIT: return launch(k_col<PM_L, COL_INIT_BIT>, grid, block, s, ev0, ev1, p);
        case COL_POW: return launch(k_col<PM_L, COL_POW>, grid, block, s, ev0, ev1, p);
        default: return hipErrorInvalidValue;
    }
}

hipError_t PM_CAT(launch_adj_row_, PM_L)(int mode, const AdjParams& p, int batch, hipStream_t s) {
    const dim3 grid(p.H / kGR, batch), block(kGR * LineShape<PM_L>::T);
    switch (mode) {
        case ROW_INIT: k_row_adj<PM_L, ROW_INIT><<<grid, block, 0, s>>>(p); break;
        case ROW_GRAD: k_row_adj<PM_L, ROW_GRAD><<<grid, block, 0, s>>>(p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t PM_CAT(launch_adj_col_, PM_L)(const AdjParams& p, int batch, hipStream_t s) {
    const dim3 grid(p.W / kC, batch), block(kC * LineShape<PM_L>::T);
    k_col_adj<PM_L><<<grid, block, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace pm
