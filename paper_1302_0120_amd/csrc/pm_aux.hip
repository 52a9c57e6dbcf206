// pm_aux.hip -- small kernels around the iteration: per-call pointer block,
// target normalisation and tiling, FP64 history finalisation.
#include <float.h>

#include "pm_kernels.hpp"

namespace pm {

// Rewrites a device-resident pointer block (PmIo, BatchIo: pointers only),
// one lane per 8-byte word, every word of the struct.
template <class Block>
__device__ __forceinline__ void set_words(Block* dst, const Block& val) {
    constexpr int kWords = (int)(sizeof(Block) / sizeof(unsigned long long));
    static_assert(sizeof(Block) == kWords * sizeof(unsigned long long), "pointer blocks hold pointers only");
    static_assert(kWords <= 64, "one lane per word");
    unsigned long long w[kWords];
    __builtin_memcpy(w, &val, sizeof(val));
    const int i = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kWords; ++k)
        if (i == k) reinterpret_cast<unsigned long long*>(dst)[k] = w[k];
}

__global__ void k_set_io(PmIo* io, PmIo val) { set_words(io, val); }

constexpr int kAuxThreads = 256;

// Partial sums of x^2 in FP64, one per work-group (grid-stride over float4).
__device__ __forceinline__ void sq_partial(const float* x, int n, double* part, double* red) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const int n4 = n / 4;
    double acc = 0.0;
#pragma unroll 4
    for (int i = blockIdx.x * kAuxThreads + threadIdx.x; i < n4; i += gridDim.x * kAuxThreads) {
        const float4 q = x4[i];
        acc = fma((double)q.x, (double)q.x, acc);
        acc = fma((double)q.y, (double)q.y, acc);
        acc = fma((double)q.z, (double)q.z, acc);
        acc = fma((double)q.w, (double)q.w, acc);
    }
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Mask blockIdx.y of a uniform batch (0 for one mask).
__global__ void __launch_bounds__(kAuxThreads) k_norm_partial(const PmIo* io, int n, double* part) {
    __shared__ double red[red_slots(kAuxThreads)];
    sq_partial(io->target + (size_t)blockIdx.y * n, n, part + (size_t)blockIdx.y * gridDim.x, red);
}

__global__ void __launch_bounds__(kAuxThreads) k_sq_partial(const float* x, int n, double* part) {
    __shared__ double red[red_slots(kAuxThreads)];
    sq_partial(x, n, part, red);
}

// Natural [H][W] floats to the strip-tiled layout, one float4 per thread;
// block 0 also sums the `npart` partials in a fixed order into *sum.
__global__ void __launch_bounds__(kAuxThreads)
k_tile_plain(const float* src, int H, int W, float* dst, const double* part, int npart, double* sum) {
    static_assert(kC == 4, "one float4 per strip chunk");
    const int w4 = W / 4;
    const int i = blockIdx.x * kAuxThreads + threadIdx.x;
    if (i < H * w4) {
        const int y = i / w4;
        const int q = i - y * w4;
        reinterpret_cast<float4*>(dst)[(size_t)q * H + y] = reinterpret_cast<const float4*>(src)[i];
    }
    if (blockIdx.x == 0) {
        __shared__ double red[red_slots(kAuxThreads)];
        double acc = 0.0;
        for (int k = threadIdx.x; k < npart; k += kAuxThreads) acc += part[k];
        const double tot = block_sum<kAuxThreads>(acc, red);
        if (threadIdx.x == 0) *sum = tot;
    }
}

// mhat = m / ||m|| in the strip-tiled layout.  Every work-group sums the
// partials itself in the same fixed order, so all see the same norm.
// One thread per 4 consecutive pixels of a row (= one strip chunk, kC = 4).
// Mask blockIdx.y of a uniform batch (0 for one mask).
__global__ void __launch_bounds__(kAuxThreads)
k_target_tile(const PmIo* io, int H, int W, const double* part, int npart, float* mhat, const double* pn2) {
    static_assert(kC == 4, "one float4 per strip chunk");
    __shared__ double red[red_slots(kAuxThreads)];
    __shared__ double inv_norm;
    const size_t mb = (size_t)blockIdx.y * H * W;
    part += (size_t)blockIdx.y * npart;
    mhat += mb;
    // this thread's four pixels, loaded while the partials are summed
    const int w4 = W / 4;
    const int i = blockIdx.x * kAuxThreads + threadIdx.x;
    const bool in = i < H * w4;
    const float4 m = in ? reinterpret_cast<const float4*>(io->target + mb)[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    double acc = 0.0;
    for (int k = threadIdx.x; k < npart; k += kAuxThreads) acc += part[k];
    const double tot = block_sum<kAuxThreads>(acc, red);
    // p = 1: m / ||m||.  Illumination p: m ||p|| / (||m|| sqrt(N)), the
    // energy-matched target on the scale of unnormalised transforms.
    if (threadIdx.x == 0) {
        if (pn2 == nullptr) {
            inv_norm = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
        } else {
            inv_norm = tot > 0.0 ? sqrt(pn2[0] / ((double)H * (double)W)) / sqrt(tot) : 0.0;
        }
    }
    __syncthreads();
    const double inv = inv_norm;
    if (in) {
        const int y = i / w4;
        const int q = i - y * w4;
        float4 o;
        o.x = (float)((double)m.x * inv);
        o.y = (float)((double)m.y * inv);
        o.z = (float)((double)m.z * inv);
        o.w = (float)((double)m.w * inv);
        reinterpret_cast<float4*>(mhat)[(size_t)q * H + y] = o;
    }
}

// History entry e = first_entry + blockIdx.x * entry_step: even entries are Fourier
// errors, E_F = sqrt(sum of partials); odd entries are gaps,
// G = sqrt(sum / N).  The n_col (n_row) partials of entry e sit at
// part[e * stride + i].
// With an illumination p (pn2 = ||p||^2 on the device) the errors are
// relative to ||p||: E_F = sqrt(sum N / ||p||^2), G = sqrt(sum / ||p||^2).
// Mask blockIdx.y of a uniform batch (0 for one mask): partials from
// part + blockIdx.y part_bstride, entries to io->hist + blockIdx.y gridDim.x.
__global__ void __launch_bounds__(kAuxThreads)
k_finalize(const double* part, int stride, int n_col, int n_row, double invN,
           const PmIo* io, int first_entry, int entry_step, const double* pn2, size_t part_bstride) {
    __shared__ double red[red_slots(kAuxThreads)];
    const int e = first_entry + blockIdx.x * entry_step;
    const int nwg = (e & 1) ? n_row : n_col;
    const double* p = part + (size_t)blockIdx.y * part_bstride + (size_t)e * stride;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nwg; i += kAuxThreads) acc += p[i];
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) {
        double* hist = io->hist;
        const double ef2 = pn2 == nullptr ? 1.0 : 1.0 / (invN * pn2[0]);
        const double g2 = pn2 == nullptr ? invN : 1.0 / pn2[0];
        if (hist != nullptr)
            hist[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = (e & 1) ? sqrt(tot * g2) : sqrt(tot * ef2);
    }
}

// Input checks (PM_FLAG_VALIDATE): flags[0] gets bit 1 for a negative
// entry (when `nonneg`), bit 2 for a non-finite one; flags[1] is set when
// any entry is non-zero.  Plain vector atomics; flags are cleared by the
// host before the launch.
__global__ void __launch_bounds__(kAuxThreads) k_validate(const float* x, int n, int nonneg, int* flags) {
    int bad = 0, nz = 0;
    for (int i = blockIdx.x * kAuxThreads + threadIdx.x; i < n; i += gridDim.x * kAuxThreads) {
        const float v = x[i];
        if (!isfinite(v)) bad |= 2;
        else if (nonneg && v < 0.0f) bad |= 1;
        if (v != 0.0f) nz = 1;
    }
    if (bad) atomicOr(&flags[0], bad);
    if (nz) atomicOr(&flags[1], 1);
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

// ----- batched preparation ---------------------------------------------------

__global__ void k_set_batch_io(BatchIo* io, BatchIo val) { set_words(io, val); }

// Sum of m^2 over one task's kPrepPixels pixels (4 float4 per thread).
__global__ void __launch_bounds__(kAuxThreads)
k_batch_norm(const BatchIo* io, const BatchTask* tasks, double* part_m) {
    static_assert(kPrepPixels == kAuxThreads * 16, "4 float4 per thread");
    __shared__ double red[red_slots(kAuxThreads)];
    const BatchTask task = tasks[blockIdx.x];
    const float4* m4 = reinterpret_cast<const float4*>(io->targets[task.mask] + task.first);
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float4 q = m4[t * kAuxThreads + threadIdx.x];
        acc = fma((double)q.x, (double)q.x, acc);
        acc = fma((double)q.y, (double)q.y, acc);
        acc = fma((double)q.z, (double)q.z, acc);
        acc = fma((double)q.w, (double)q.w, acc);
    }
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) part_m[blockIdx.x] = tot;
}

// mhat = m / ||m|| (strip-tiled) for one task's pixels; the norm is summed
// from the mask's partials in a fixed order by every work-group.
__global__ void __launch_bounds__(kAuxThreads)
k_batch_tile(const BatchIo* io, const BatchMask* masks, const BatchTask* tasks, const int* mask_prep0,
             const double* part_m) {
    __shared__ double red[red_slots(kAuxThreads)];
    __shared__ double inv_norm;
    const BatchTask task = tasks[blockIdx.x];
    const BatchMask mk = masks[task.mask];
    const int p0 = mask_prep0[task.mask];
    const int np = mk.H * mk.W / kPrepPixels;
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += kAuxThreads) acc += part_m[p0 + i];
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) inv_norm = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
    __syncthreads();
    const double inv = inv_norm;
    const float4* m4 = reinterpret_cast<const float4*>(io->targets[task.mask]);
    float4* out4 = reinterpret_cast<float4*>(mk.mhat);
    const int w4 = mk.W / 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int i = task.first / 4 + t * kAuxThreads + threadIdx.x;
        const int y = i / w4;
        const int q = i - y * w4;
        const float4 m = m4[i];
        float4 o;
        o.x = (float)((double)m.x * inv);
        o.y = (float)((double)m.y * inv);
        o.z = (float)((double)m.z * inv);
        o.w = (float)((double)m.w * inv);
        out4[(size_t)q * mk.H + y] = o;
    }
}

// phases_out = atan2(sin phi, cos phi) for a zero-iteration batched solve.
__global__ void __launch_bounds__(kAuxThreads)
k_batch_wrap(const BatchIo* io, const BatchTask* tasks) {
    const BatchTask task = tasks[blockIdx.x];
    const float* in = io->phases_in[task.mask] + task.first;
    float* out = io->phases_out[task.mask] + task.first;
    for (int i = threadIdx.x; i < kPrepPixels; i += kAuxThreads) {
        float sn, cs;
        sincosf(in[i], &sn, &cs);
        out[i] = atan2f(sn, cs);
    }
}

// final_err[mask] = sqrt(sum of the mask's column-pass partials).
__global__ void __launch_bounds__(kAuxThreads)
k_batch_finalize(const BatchIo* io, const BatchMask* masks, const double* part) {
    __shared__ double red[red_slots(kAuxThreads)];
    const BatchMask mk = masks[blockIdx.x];
    double acc = 0.0;
    constexpr int NS = red_slots(kBatchThreads);  // partials per column work-group
    for (int i = threadIdx.x; i < mk.col_wgs * NS; i += kAuxThreads) acc += part[mk.col_wg0 * NS + i];
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0 && io->final_err != nullptr) io->final_err[blockIdx.x] = sqrt(tot);
}

hipError_t launch_set_batch_io(BatchIo* io, const BatchIo& val, hipStream_t s) {
    k_set_batch_io<<<1, 64, 0, s>>>(io, val);
    return hipGetLastError();
}

hipError_t launch_batch_norm(const BatchIo* io, const BatchTask* tasks, int ntasks, double* part_m,
                             hipStream_t s) {
    k_batch_norm<<<ntasks, kAuxThreads, 0, s>>>(io, tasks, part_m);
    return hipGetLastError();
}

hipError_t launch_batch_tile(const BatchIo* io, const BatchMask* masks, const BatchTask* tasks, int ntasks,
                             const int* mask_prep0, const double* part_m, hipStream_t s) {
    k_batch_tile<<<ntasks, kAuxThreads, 0, s>>>(io, masks, tasks, mask_prep0, part_m);
    return hipGetLastError();
}

hipError_t launch_batch_wrap(const BatchIo* io, const BatchMask* masks, const BatchTask* tasks, int ntasks,
                             hipStream_t s) {
    (void)masks;
    k_batch_wrap<<<ntasks, kAuxThreads, 0, s>>>(io, tasks);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchIo* io, const BatchMask* masks, int count, const double* part,
                                 hipStream_t s) {
    k_batch_finalize<<<count, kAuxThreads, 0, s>>>(io, masks, part);
    return hipGetLastError();
}

// out[b] = sum of one row of partials, fixed order (one work-group per row).
__global__ void __launch_bounds__(kAuxThreads) k_sum_rows(const double* part, int nwg, double* out) {
    __shared__ double red[red_slots(kAuxThreads)];
    const double* p = part + (size_t)blockIdx.x * nwg;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nwg; i += kAuxThreads) acc += p[i];
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

hipError_t launch_sum_rows(const double* part, int nwg, double* out, int count, hipStream_t s) {
    k_sum_rows<<<count, kAuxThreads, 0, s>>>(part, nwg, out);
    return hipGetLastError();
}

// k_sum_rows into io->hist (read through the per-call pointer block).
__global__ void __launch_bounds__(kAuxThreads) k_sum_rows_io(const double* part, int nwg, const PmIo* io) {
    __shared__ double red[red_slots(kAuxThreads)];
    const double* p = part + (size_t)blockIdx.x * nwg;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nwg; i += kAuxThreads) acc += p[i];
    const double tot = block_sum<kAuxThreads>(acc, red);
    if (threadIdx.x == 0) io->hist[blockIdx.x] = tot;
}

hipError_t launch_sum_rows_io(const double* part, int nwg, const PmIo* io, int count, hipStream_t s) {
    k_sum_rows_io<<<count, kAuxThreads, 0, s>>>(part, nwg, io);
    return hipGetLastError();
}

// ----- Adam solves on the intensity loss ----------------------------------------

// Set-up over batch x H x W pixels, one thread per 4 adjacent pixels of a
// row (W is a multiple of 4): the working phase (natural layout) from
// io->phase_in, the intensity io->target into the strip-tiled layout (a
// strip row of kC = 4 pixels is one float4), and zero moments.
__global__ void __launch_bounds__(kAuxThreads)
k_adam_prep(const PmIo* io, int H, int W, int batch, float* phase, float* inten, float* m, float* v) {
    const size_t q = (size_t)blockIdx.x * kAuxThreads + threadIdx.x;  // float4 index
    const size_t per = (size_t)H * (W / 4);
    if (q >= per * (size_t)batch) return;
    const size_t b = q / per;
    const size_t r = q % per;
    const int y = (int)(r / (W / 4));
    const int s4 = (int)(r % (W / 4));  // strip index (4 columns)
    const size_t n = (size_t)H * W;
    const float4 ph = reinterpret_cast<const float4*>(io->phase_in + b * n)[(size_t)y * (W / 4) + s4];
    const float4 it = reinterpret_cast<const float4*>(io->target + b * n)[(size_t)y * (W / 4) + s4];
    reinterpret_cast<float4*>(phase + b * n)[(size_t)y * (W / 4) + s4] = ph;
    reinterpret_cast<float4*>(inten + b * n)[(size_t)s4 * H + y] = it;
    const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    reinterpret_cast<float4*>(m + b * n)[(size_t)y * (W / 4) + s4] = z;
    reinterpret_cast<float4*>(v + b * n)[(size_t)y * (W / 4) + s4] = z;
}

hipError_t launch_adam_prep(const PmIo* io, int H, int W, int batch, float* phase, float* inten, float* m,
                            float* v, hipStream_t s) {
    const size_t quads = (size_t)batch * H * (W / 4);
    const unsigned grid = (unsigned)((quads + kAuxThreads - 1) / kAuxThreads);
    k_adam_prep<<<grid, kAuxThreads, 0, s>>>(io, H, W, batch, phase, inten, m, v);
    return hipGetLastError();
}

// io->phase_out = phase, n floats (n a multiple of 4).
__global__ void __launch_bounds__(kAuxThreads) k_adam_out(const PmIo* io, const float* phase, size_t n4) {
    const size_t q = (size_t)blockIdx.x * kAuxThreads + threadIdx.x;
    if (q < n4) reinterpret_cast<float4*>(io->phase_out)[q] = reinterpret_cast<const float4*>(phase)[q];
}

hipError_t launch_adam_out(const PmIo* io, const float* phase, size_t n, hipStream_t s) {
    const size_t n4 = n / 4;
    k_adam_out<<<(unsigned)((n4 + kAuxThreads - 1) / kAuxThreads), kAuxThreads, 0, s>>>(io, phase, n4);
    return hipGetLastError();
}

// ----- physical error (Eq. 8) and target maxima -------------------------------

__global__ void __launch_bounds__(kAuxThreads) k_max_partial(const float* x, int n, float* part) {
    __shared__ float redf[red_slots(kAuxThreads)];
    const float4* x4 = reinterpret_cast<const float4*>(x);
    float mx = 0.0f;
    for (int i = blockIdx.x * kAuxThreads + threadIdx.x; i < n / 4; i += gridDim.x * kAuxThreads) {
        const float4 q = x4[i];
        mx = fmaxf(fmaxf(mx, fmaxf(q.x, q.y)), fmaxf(q.z, q.w));
    }
    mx = block_max<kAuxThreads>(mx, redf);
    if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

// E_lit = sum over lit pixels of (t_d rel / t_l - t_d) [rel > t_l], rel = |It - Ir| / It;
// E_dark = sum over dark pixels of (Ir - t_d) [Ir > t_d]; It = m^2 / max m^2,
// Ir = |U|^2 / max |U|^2, lit where It > t_d (Eq. 8a / 8b, reading in the
// design notes).  One thread per 4 consecutive strip-tiled pixels.
__global__ void __launch_bounds__(kAuxThreads)
k_physical_error(const float* pw, const double* pw_max_part, int n_pw_max, const float* target,
                 const float* tmax_part, int ntmax, int H, int W, double t_lit, double t_dark,
                 double* scratch) {
    static_assert(kC == 4, "one float4 per strip chunk");
    __shared__ double red[red_slots(kAuxThreads)];
    __shared__ float redf[red_slots(kAuxThreads)];
    __shared__ double pmax_s;
    double pm = 0.0;
    for (int i = threadIdx.x; i < n_pw_max; i += kAuxThreads) pm = fmax(pm, pw_max_part[i]);
    float tm = 0.0f;
    for (int i = threadIdx.x; i < ntmax; i += kAuxThreads) tm = fmaxf(tm, tmax_part[i]);
    tm = block_max<kAuxThreads>(tm, redf);
    pm = (double)block_max<kAuxThreads>((float)pm, redf);  // the partial maxima are floats
    if (threadIdx.x == 0) pmax_s = pm;
    __syncthreads();
    const double pmax = pmax_s;
    const double mx2 = (double)tm * (double)tm;
    const int i4 = blockIdx.x * kAuxThreads + threadIdx.x;  // float4 index, strip-tiled
    double e_lit = 0.0, e_dark = 0.0;
    if (i4 < H * W / 4) {
        const int s = i4 / H;   // strip
        const int y = i4 - s * H;
        const float4 q = reinterpret_cast<const float4*>(pw)[i4];
        const float4 m = reinterpret_cast<const float4*>(target + (size_t)y * W)[s];
        const float qs[4] = {q.x, q.y, q.z, q.w};
        const float ms[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double it = ((double)ms[k] * (double)ms[k]) / mx2;
            const double ir = (double)qs[k] / pmax;
            if (it > t_dark) {
                const double rel = fabs(it - ir) / it;
                if (rel - t_lit > 0.0) e_lit += t_dark * rel / t_lit - t_dark;
            } else if (ir - t_dark > 0.0) {
                e_dark += ir - t_dark;
            }
        }
    }
    const double a = block_sum<kAuxThreads>(e_lit, red);
    __syncthreads();
    const double b = block_sum<kAuxThreads>(e_dark, red);
    if (threadIdx.x == 0) {
        scratch[2 * blockIdx.x] = a;
        scratch[2 * blockIdx.x + 1] = b;
    }
}

__global__ void __launch_bounds__(kAuxThreads) k_pair_sum(const double* scratch, int n, double* out) {
    __shared__ double red[red_slots(kAuxThreads)];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += kAuxThreads) {
        a += scratch[2 * i];
        b += scratch[2 * i + 1];
    }
    const double ta = block_sum<kAuxThreads>(a, red);
    __syncthreads();
    const double tb = block_sum<kAuxThreads>(b, red);
    if (threadIdx.x == 0) {
        out[0] = ta;
        out[1] = tb;
    }
}

hipError_t launch_max_partial(const float* x, int n, float* part, int grid, hipStream_t s) {
    k_max_partial<<<grid, kAuxThreads, 0, s>>>(x, n, part);
    return hipGetLastError();
}

hipError_t launch_physical_error(const float* pw, const double* pw_max_part, int n_pw_max, const float* target,
                                 const float* tmax_part, int ntmax, int H, int W, double t_lit, double t_dark,
                                 double* scratch, double* out, hipStream_t s) {
    const int grid = (H * W / 4 + kAuxThreads - 1) / kAuxThreads;
    k_physical_error<<<grid, kAuxThreads, 0, s>>>(pw, pw_max_part, n_pw_max, target, tmax_part, ntmax, H, W,
                                                  t_lit, t_dark, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pair_sum<<<1, kAuxThreads, 0, s>>>(scratch, grid, out);
    return hipGetLastError();
}

// ----- one-mask helpers -------------------------------------------------------

hipError_t launch_set_io(PmIo* io, const PmIo& val, hipStream_t s) {
    k_set_io<<<1, 64, 0, s>>>(io, val);
    return hipGetLastError();
}

hipError_t launch_norm_partial(const PmIo* io, int n, double* part, int grid, hipStream_t s, int batch) {
    if (batch < 1) return hipErrorInvalidValue;
    k_norm_partial<<<dim3(grid, batch), kAuxThreads, 0, s>>>(io, n, part);
    return hipGetLastError();
}

hipError_t launch_target_tile(const PmIo* io, int H, int W, const double* part, int npart,
                              float* mhat, hipStream_t s, const double* pn2, int batch) {
    if (batch < 1) return hipErrorInvalidValue;
    const int grid = (H * (W / 4) + kAuxThreads - 1) / kAuxThreads;
    k_target_tile<<<dim3(grid, batch), kAuxThreads, 0, s>>>(io, H, W, part, npart, mhat, pn2);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* part, int stride, int n_col, int n_row, double invN,
                           const PmIo* io, int first_entry, int count, hipStream_t s, int entry_step,
                           const double* pn2, int batch, size_t part_bstride) {
    if (batch < 1) return hipErrorInvalidValue;
    k_finalize<<<dim3(count, batch), kAuxThreads, 0, s>>>(part, stride, n_col, n_row, invN, io, first_entry,
                                                          entry_step, pn2, part_bstride);
    return hipGetLastError();
}

hipError_t launch_illum_prep(const float* p, int H, int W, double* part, int grid, float* illum,
                             double* pn2, hipStream_t s) {
    k_sq_partial<<<grid, kAuxThreads, 0, s>>>(p, H * W, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int tgrid = (H * (W / 4) + kAuxThreads - 1) / kAuxThreads;
    k_tile_plain<<<tgrid, kAuxThreads, 0, s>>>(p, H, W, illum, part, grid, pn2);
    return hipGetLastError();
}

hipError_t launch_validate(const float* x, int n, bool nonneg, int* flags, hipStream_t s) {
    k_validate<<<256, kAuxThreads, 0, s>>>(x, n, nonneg ? 1 : 0, flags);
    return hipGetLastError();
}

hipError_t launch_wrap_phase(const PmIo* io, int n, hipStream_t s) {
    k_wrap_phase<<<(n + kAuxThreads - 1) / kAuxThreads, kAuxThreads, 0, s>>>(io, n);
    return hipGetLastError();
}

}  // namespace pm
