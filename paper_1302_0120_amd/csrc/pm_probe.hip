// pm_probe.hip -- measures the arithmetic rate of one 16-point DFT stage on
// the vector ALUs (the butterflies every pass runs) and as FP32 matrix
// products on the matrix cores, for the choice of unit (DFT-as-matmul costs
// 16 complex multiply-adds per point where the radix-16 butterfly costs
// about 10 real operations; the matrix cores run FP32 at twice the rate of
// the non-packed vector ALUs).  Both kernels work on data already in
// registers and repeat the stage `reps` times, so only the arithmetic is
// timed; the matrix version's operands are loaded straight into the
// layouts the instruction wants, which a real pass would first have to
// produce by a cross-lane exchange, so the measurement favours it.
#include <hip/hip_ext.h>

#include "pm_fft.hpp"

namespace pm {

namespace {

constexpr int kProbeThreads = 256;  // 4 waves
using f4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;

// Vector ALUs: every thread transforms its 16 points with the radix-16
// butterfly of the passes, forward then inverse (scaled by 1/16, so values
// stay bounded), reps / 2 times.  Points t of thread i: in[16 i + t].
__global__ void __launch_bounds__(kProbeThreads) k_dft16_valu(const float2* in, float2* out, int reps) {
    const size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
    float2 x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = in[i * 16 + t];
    for (int r = 0; r < reps; r += 2) {
        dft<16, false>(x);
        dft<16, true>(x);
#pragma unroll
        for (int t = 0; t < 16; ++t) x[t] = make_float2(x[t].x * 0.0625f, x[t].y * 0.0625f);
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) out[i * 16 + t] = x[t];
}

// Matrix cores: a wave holds 4 blocks of 16 butterflies; block b computes
// Y = F X, F[k][t] = exp(-2 pi i k t / 16), X[t][j] = in[1024 w + 256 b +
// 16 t + j], as real products Yr = Fr Xr - Fi Xi, Yi = Fr Xi + Fi Xr, each
// split over the K dimension t into four 16x16x4 products (lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 (l / 16) + r][l % 16]
// in register r).  The products accumulate over the reps, so none can be
// dropped; out[1024 w + 256 b + 16 k + j] = Y[k][j] summed over the reps.
__global__ void __launch_bounds__(kProbeThreads) k_dft16_mfma(const float2* in, float2* out, int reps) {
    const int lane = threadIdx.x & 63;
    const size_t w = ((size_t)blockIdx.x * kProbeThreads + threadIdx.x) / 64;
    const int row = lane % 16, kq = lane / 16;
    float fr[4], fi[4], nfi[4];
    const TurnTable<16> tt{};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = (row * (4 * q + kq)) % 16;
        fr[q] = tt.c[e];
        fi[q] = -tt.s[e];
        nfi[q] = tt.s[e];
    }
    float xr[4][4], xi[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float2 v = in[w * 1024 + b * 256 + (4 * q + kq) * 16 + row];
            xr[b][q] = v.x;
            xi[b][q] = v.y;
        }
    f4 yr[4], yi[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        yr[b] = f4{0.f, 0.f, 0.f, 0.f};
        yi[b] = f4{0.f, 0.f, 0.f, 0.f};
    }
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                yr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[q], xr[b][q], yr[b], 0, 0, 0);
                yr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(nfi[q], xi[b][q], yr[b], 0, 0, 0);
                yi[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[q], xi[b][q], yi[b], 0, 0, 0);
                yi[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fi[q], xr[b][q], yi[b], 0, 0, 0);
            }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            out[w * 1024 + b * 256 + (4 * kq + r) * 16 + row] = make_float2(yr[b][r], yi[b][r]);
}

}  // namespace

hipError_t launch_probe_dft16(int matrix, const float2* in, float2* out, int waves, int reps, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1) {
    const int grid = waves / 4;
    if (matrix)
        hipExtLaunchKernelGGL(k_dft16_mfma, dim3(grid), dim3(kProbeThreads), 0, s, ev0, ev1, 0, in, out, reps);
    else
        hipExtLaunchKernelGGL(k_dft16_valu, dim3(grid), dim3(kProbeThreads), 0, s, ev0, ev1, 0, in, out, reps);
    return hipGetLastError();
}

}  // namespace pm
