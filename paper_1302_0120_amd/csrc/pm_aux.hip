// pm_aux.hip -- small kernels around the iteration: per-call pointer block,
// target normalisation and tiling, FP64 history finalisation.
#include <float.h>

#include "pm_kernels.hpp"

namespace pm {

// Rewrites the per-call pointer block (4 pointers), one lane per pointer.
__global__ void k_set_io(PmIo* io, PmIo val) {
    const unsigned long long vals[4] = {
        (unsigned long long)val.target, (unsigned long long)val.phase_in,
        (unsigned long long)val.phase_out, (unsigned long long)val.hist};
    const int i = threadIdx.x;
    if (i < 4) reinterpret_cast<unsigned long long*>(io)[i] = vals[i];
}

constexpr int kAuxThreads = 256;

// Partial sums of m^2 in FP64, one per work-group (grid-stride over float4).
__global__ void __launch_bounds__(kAuxThreads) k_norm_partial(const PmIo* io, int n, double* part) {
    __shared__ double red[kAuxThreads / 64];
    const float4* m4 = reinterpret_cast<const float4*>(io->target);
    const int n4 = n / 4;
    double acc = 0.0;
    for (int i = blockIdx.x * kAuxThreads + threadIdx.x; i < n4; i += gridDim.x * kAuxThreads) {
        const float4 q = m4[i];
        acc = fma((double)q.x, (double)q.x, acc);
        acc = fma((double)q.y, (double)q.y, acc);
        acc = fma((double)q.z, (double)q.z, acc);
        acc = fma((double)q.w, (double)q.w, acc);
    }
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// mhat = m / ||m|| in the strip-tiled layout.  Every work-group sums the
// partials itself in the same fixed order, so all see the same norm.
// One thread per 4 consecutive pixels of a row (= one strip chunk, kC = 4).
__global__ void __launch_bounds__(kAuxThreads)
k_target_tile(const PmIo* io, int H, int W, const double* part, int npart, float* mhat) {
    static_assert(kC == 4, "one float4 per strip chunk");
    __shared__ double red[kAuxThreads / 64];
    __shared__ double inv_norm;
    double acc = 0.0;
    for (int i = threadIdx.x; i < npart; i += kAuxThreads) acc += part[i];
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) inv_norm = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
    __syncthreads();
    const double inv = inv_norm;
    const int w4 = W / 4;
    const int i = blockIdx.x * kAuxThreads + threadIdx.x;
    if (i < H * w4) {
        const int y = i / w4;
        const int q = i - y * w4;
        const float4 m = reinterpret_cast<const float4*>(io->target)[i];
        float4 o;
        o.x = (float)((double)m.x * inv);
        o.y = (float)((double)m.y * inv);
        o.z = (float)((double)m.z * inv);
        o.w = (float)((double)m.w * inv);
        reinterpret_cast<float4*>(mhat)[(size_t)q * H + y] = o;
    }
}

// History entry e = first_entry + blockIdx.x: even entries are Fourier
// errors, E_F = sqrt(sum of partials); odd entries are gaps,
// G = sqrt(sum / N).  Partials of entry e sit at part[e * stride + wg].
__global__ void __launch_bounds__(kAuxThreads)
k_finalize(const double* part, int stride, int nwg_col, int nwg_row, double invN,
           const PmIo* io, int first_entry) {
    __shared__ double red[kAuxThreads / 64];
    const int e = first_entry + blockIdx.x;
    const int nwg = (e & 1) ? nwg_row : nwg_col;
    const double* p = part + (size_t)e * stride;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nwg; i += kAuxThreads) acc += p[i];
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) {
        double* hist = io->hist;
        if (hist != nullptr) hist[blockIdx.x] = (e & 1) ? sqrt(tot * invN) : sqrt(tot);
    }
}

// out = atan2(sin phi, cos phi): the phase of u^0 for a zero-iteration solve.
__global__ void __launch_bounds__(kAuxThreads) k_wrap_phase(const PmIo* io, int n) {
    const int i = blockIdx.x * kAuxThreads + threadIdx.x;
    if (i < n) {
        float sn, cs;
        sincosf(io->phase_in[i], &sn, &cs);
        io->phase_out[i] = atan2f(sn, cs);
    }
}

hipError_t launch_set_io(PmIo* io, const PmIo& val, hipStream_t s) {
    k_set_io<<<1, 64, 0, s>>>(io, val);
    return hipGetLastError();
}

hipError_t launch_norm_partial(const PmIo* io, int n, double* part, int grid, hipStream_t s) {
    k_norm_partial<<<grid, kAuxThreads, 0, s>>>(io, n, part);
    return hipGetLastError();
}

hipError_t launch_target_tile(const PmIo* io, int H, int W, const double* part, int npart,
                              float* mhat, hipStream_t s) {
    const int grid = (H * (W / 4) + kAuxThreads - 1) / kAuxThreads;
    k_target_tile<<<grid, kAuxThreads, 0, s>>>(io, H, W, part, npart, mhat);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* part, int stride, int nwg_col, int nwg_row, double invN,
                           const PmIo* io, int first_entry, int count, hipStream_t s) {
    k_finalize<<<count, kAuxThreads, 0, s>>>(part, stride, nwg_col, nwg_row, invN, io, first_entry);
    return hipGetLastError();
}

hipError_t launch_wrap_phase(const PmIo* io, int n, hipStream_t s) {
    k_wrap_phase<<<(n + kAuxThreads - 1) / kAuxThreads, kAuxThreads, 0, s>>>(io, n);
    return hipGetLastError();
}

}  // namespace pm
