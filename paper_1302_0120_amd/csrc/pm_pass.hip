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

// When a pass has no more work-groups than the GPU has CUs (p.spread), the
// launch reserves extra dynamic LDS so that no CU can hold two of them: the
// dispatcher then gives every work-group a CU of its own instead of doubling
// up some CUs while others idle (measured: about 0.6 us per 1024^2 pass).
constexpr size_t kSpreadLds = 80 * 1024 + 256;  // more than half of the 160 KB per CU

template <typename Params>
hipError_t launch(void (*kern)(Params), int grid, int block, hipStream_t s, hipEvent_t ev0,
                  hipEvent_t ev1, const Params& p) {
    size_t dyn = 0;
    if (p.spread) {
        hipFuncAttributes attr{};
        hipError_t e = hipFuncGetAttributes(&attr, (const void*)kern);
        if (e != hipSuccess) return e;
        if (attr.sharedSizeBytes < kSpreadLds) {
            dyn = kSpreadLds - attr.sharedSizeBytes;
            e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
            if (e != hipSuccess) return e;
        }
    }
    // grid.y: the masks of a uniform batch (R_MANY / C_MANY modes), else 1
    const dim3 g(grid, p.nb > 1 ? p.nb : 1);
    if (ev0 != nullptr || ev1 != nullptr) {
        hipExtLaunchKernelGGL(kern, g, dim3(block), dyn, s, ev0, ev1, 0, p);
    } else {
        kern<<<g, block, dyn, s>>>(p);
    }
    return hipGetLastError();
}

}  // namespace

// Row modes of the solves, each also built with R_ILLUM (illumination p).
#define PM_ROW_SOLVE_MODES(X) \
    X(ROW_INIT) X(ROW_ITER) X(ROW_LAST) X(ROW_LAST_FWD) X(ROW_GAP) X(ROW_ITER_NE) X(ROW_LAST_NE) \
    X(ROW_INIT_Z) X(ROW_RAAR) X(ROW_RAAR_LAST) X(ROW_RAAR_LAST_FWD) \
    X(ROW_LAST_FIELD) X(ROW_LAST_FIELD_FWD) X(ROW_LAST_FIELD_NE)
// Row modes of uniform batches, each also built with R_ILLUM.
#define PM_ROW_MANY_MODES(X) \
    X(ROW_INIT_MANY) X(ROW_ITER_MANY) X(ROW_ITER_NE_MANY) X(ROW_LAST_MANY) X(ROW_LAST_FWD_MANY) X(ROW_LAST_NE_MANY)
#define PM_ROW_CASE(M)                                                                         \
    case M: return launch(k_row<PM_L, M, G>, grid, block, s, ev0, ev1, p);                     \
    case M | R_ILLUM: return launch(k_row<PM_L, M | R_ILLUM, G>, grid, block, s, ev0, ev1, p);

namespace {

template <int G>
hipError_t launch_rows(int mode, const RowParams& p, int grid, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const int block = G * LineShape<PM_L>::T;
    switch (mode) {
        PM_ROW_SOLVE_MODES(PM_ROW_CASE)
        case ROW_FFT_FWD: return launch(k_row<PM_L, ROW_FFT_FWD, G>, grid, block, s, ev0, ev1, p);
        case ROW_FFT_INV: return launch(k_row<PM_L, ROW_FFT_INV, G>, grid, block, s, ev0, ev1, p);
        case ROW_INIT_FIELD: return launch(k_row<PM_L, ROW_INIT_FIELD, G>, grid, block, s, ev0, ev1, p);
        case ROW_COPY_FIELD: return launch(k_row<PM_L, ROW_COPY_FIELD, G>, grid, block, s, ev0, ev1, p);
        case ROW_COPY: return launch(k_row<PM_L, ROW_COPY, G>, grid, block, s, ev0, ev1, p);
        PM_ROW_MANY_MODES(PM_ROW_CASE)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
#undef PM_ROW_CASE
#undef PM_ROW_SOLVE_MODES
#undef PM_ROW_MANY_MODES

// The row tile is p.H / grid rows: row_lines(PM_L), or row_lines_alt(PM_L)
// where the length has one.
hipError_t PM_CAT(launch_row_, PM_L)(int mode, const RowParams& p, int grid, hipStream_t s,
                                     hipEvent_t ev0, hipEvent_t ev1) {
    if (grid <= 0) return hipErrorInvalidValue;
    const int g = p.H / grid;
    if (g * grid != p.H) return hipErrorInvalidValue;
    if (g == row_lines(PM_L)) return launch_rows<row_lines(PM_L)>(mode, p, grid, s, ev0, ev1);
    if constexpr (row_lines_alt(PM_L) != 0) {
        if (g == row_lines_alt(PM_L)) return launch_rows<row_lines_alt(PM_L)>(mode, p, grid, s, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

// The column tile is p.W / grid columns, which must be col_lines(PM_L).
hipError_t PM_CAT(launch_col_, PM_L)(int mode, const ColParams& p, int grid, hipStream_t s,
                                     hipEvent_t ev0, hipEvent_t ev1) {
    if (grid <= 0 || p.W != grid * col_lines(PM_L)) return hipErrorInvalidValue;
    const int block = col_lines(PM_L) * LineShape<PM_L>::T;
    switch (mode) {
        case COL_ITER: return launch(k_col<PM_L, COL_ITER>, grid, block, s, ev0, ev1, p);
        case COL_ERR: return launch(k_col<PM_L, COL_ERR>, grid, block, s, ev0, ev1, p);
        case COL_FFT_FWD: return launch(k_col<PM_L, COL_FFT_FWD>, grid, block, s, ev0, ev1, p);
        case COL_FFT_INV: return launch(k_col<PM_L, COL_FFT_INV>, grid, block, s, ev0, ev1, p);
        case COL_ITER_NE: return launch(k_col<PM_L, COL_ITER_NE>, grid, block, s, ev0, ev1, p);
        case COL_INIT_BIT: return launch(k_col<PM_L, COL_INIT_BIT>, grid, block, s, ev0, ev1, p);
        case COL_POW: return launch(k_col<PM_L, COL_POW>, grid, block, s, ev0, ev1, p);
        case COL_COPY: return launch(k_col<PM_L, COL_COPY>, grid, block, s, ev0, ev1, p);
        case COL_ITER_MANY: return launch(k_col<PM_L, COL_ITER_MANY>, grid, block, s, ev0, ev1, p);
        case COL_ITER_NE_MANY: return launch(k_col<PM_L, COL_ITER_NE_MANY>, grid, block, s, ev0, ev1, p);
        case COL_ERR_MANY: return launch(k_col<PM_L, COL_ERR_MANY>, grid, block, s, ev0, ev1, p);
        default: return hipErrorInvalidValue;
    }
}

hipError_t PM_CAT(launch_adj_row_, PM_L)(int mode, const AdjParams& p, int batch, hipStream_t s) {
    const dim3 grid(p.H / row_lines(PM_L), batch), block(row_lines(PM_L) * LineShape<PM_L>::T);
    switch (mode) {
        case ROW_INIT: k_row_adj<PM_L, ROW_INIT><<<grid, block, 0, s>>>(p); break;
        case ROW_GRAD: k_row_adj<PM_L, ROW_GRAD><<<grid, block, 0, s>>>(p); break;
        case ROW_ADAM: k_row_adj<PM_L, ROW_ADAM><<<grid, block, 0, s>>>(p); break;
        case ROW_ADAM_LAST: k_row_adj<PM_L, ROW_ADAM_LAST><<<grid, block, 0, s>>>(p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t PM_CAT(launch_adj_col_, PM_L)(int mode, const AdjParams& p, int batch, hipStream_t s) {
    const dim3 grid(p.W / kC, batch), block(kC * LineShape<PM_L>::T);
    switch (mode) {
        case COL_LOSS: k_col_adj<PM_L, COL_LOSS><<<grid, block, 0, s>>>(p); break;
        case COL_LOSS_T: k_col_adj<PM_L, COL_LOSS_T><<<grid, block, 0, s>>>(p); break;
        case COL_LOSS_ONLY_T: k_col_adj<PM_L, COL_LOSS_ONLY_T><<<grid, block, 0, s>>>(p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pm

#ifdef PM_TIMELINE
// Timeline records of this transform length's passes (pm_trace.h): copies
// the ring buffer (2 * kTlLaunches * kTlWg * kTlFields 64-bit words) and the
// launch counts (2 * kTlWg 32-bit words) to host memory; 0 or -1.
extern "C" int PM_CAT(phasemask_timeline_read_, PM_L)(void* records, void* counts) {
    if (hipMemcpyFromSymbol(records, HIP_SYMBOL(pm::tl_buf), sizeof(pm::tl_buf)) != hipSuccess) return -1;
    if (hipMemcpyFromSymbol(counts, HIP_SYMBOL(pm::tl_cnt), sizeof(pm::tl_cnt)) != hipSuccess) return -1;
    return 0;
}
// Restarts the launch counts of this length's passes; 0 or -1.
extern "C" int PM_CAT(phasemask_timeline_reset_, PM_L)() {
    static const unsigned zeros[2][pm::kTlWg] = {};
    return hipMemcpyToSymbol(HIP_SYMBOL(pm::tl_cnt), zeros, sizeof(zeros)) == hipSuccess ? 0 : -1;
}
#endif
