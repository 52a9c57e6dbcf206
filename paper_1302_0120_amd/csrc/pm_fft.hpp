// pm_fft.hpp -- device-side Stockham FFT for gfx950, used by the fused
// projection kernels.  The transform is the F of Eq. 2 / Eq. 4b (unnormalised
// here: the method only uses the phase of F u, and P_S divides every modulus
// out, so no 1/N scaling pass is ever needed).
//
// Scheme (Stockham autosort, radix-2^k, natural order in and out):
//   * A line of L points is handled by T = L / P threads; thread j holds the
//     P points  x[j + T t], t = 0 .. P-1, in registers.
//   * Stage s (sub-transform length NS so far, radix R) runs butterflies
//     b = j + T m, m = 0 .. P/R - 1.  Butterfly b reads x[b + q L/R]
//     (= register slot m + q P/R of its thread), multiplies input q by
//     exp(-+2 pi i q (b mod NS) / (NS R)), does an R-point DFT, and writes
//     output q to position (b - b mod NS) R + b mod NS + q NS.
//   * Between stages the outputs go through LDS and each thread gathers its
//     next inputs x[j + T t]; the last stage's outputs land exactly in the
//     thread's own slots, so a line needs (#stages - 1) LDS exchanges and the
//     first read / last write can go straight to or from global memory.
//   * Radix sequence: P, P, ..., then the remaining factor (each divides P).
//   * Twiddles come from a table tw[i] = exp(-2 pi i i / L) computed on the
//     host in double precision and rounded once to float; each thread loads
//     the ones it needs into registers at kernel start.
#pragma once
#include <hip/hip_runtime.h>

namespace pm {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * (-i) for the forward transform, a * (+i) for the inverse.
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// cos and sin of 2 pi e / 16, e = 0 .. 15.
__device__ constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
__device__ constexpr float kSin16[16] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

// a * exp(-+2 pi i E / 16) with E known at compile time.
template <int E, bool INV>
__device__ __forceinline__ float2 tw16(float2 a) {
    constexpr int e = E & 15;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 4) {
        return rot90<INV>(a);
    } else if constexpr (e == 8) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (e == 12) {
        return rot90<!INV>(a);
    } else {
        const float c = kCos16[e];
        const float s = INV ? kSin16[e] : -kSin16[e];
        return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

// In-register DFTs of R = 2, 4, 8, 16 points, natural order in and out.
// Each first forms sums and differences of input pairs, so equal inputs give
// exact zeros off the zero frequency (the constant-field tie-break case).
template <bool INV>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
    const float2 s02 = cadd(x0, x2), d02 = csub(x0, x2);
    const float2 s13 = cadd(x1, x3), d13 = rot90<INV>(csub(x1, x3));
    x0 = cadd(s02, s13);
    x2 = csub(s02, s13);
    x1 = cadd(d02, d13);
    x3 = csub(d02, d13);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&x)[R]) {
    if constexpr (R == 2) {
        const float2 t = csub(x[0], x[1]);
        x[0] = cadd(x[0], x[1]);
        x[1] = t;
    } else if constexpr (R == 4) {
        dft4<INV>(x[0], x[1], x[2], x[3]);
    } else if constexpr (R == 8) {
        // Even / odd halves, then one radix-2 layer with exp(-+i pi k / 4).
        dft4<INV>(x[0], x[2], x[4], x[6]);
        dft4<INV>(x[1], x[3], x[5], x[7]);
        const float2 o1 = tw16<2, INV>(x[3]);
        const float2 o2 = tw16<4, INV>(x[5]);
        const float2 o3 = tw16<6, INV>(x[7]);
        const float2 y0 = cadd(x[0], x[1]), y4 = csub(x[0], x[1]);
        const float2 y1 = cadd(x[2], o1), y5 = csub(x[2], o1);
        const float2 y2 = cadd(x[4], o2), y6 = csub(x[4], o2);
        const float2 y3 = cadd(x[6], o3), y7 = csub(x[6], o3);
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
        x[4] = y4; x[5] = y5; x[6] = y6; x[7] = y7;
    } else if constexpr (R == 16) {
        // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle
        // exp(-+2 pi i n2 k1 / 16), DFT4 over n2; output k1 + 4 k2 sits in
        // slot 4 k1 + k2 and is renamed into natural order at the end.
        dft4<INV>(x[0], x[4], x[8], x[12]);
        dft4<INV>(x[1], x[5], x[9], x[13]);
        dft4<INV>(x[2], x[6], x[10], x[14]);
        dft4<INV>(x[3], x[7], x[11], x[15]);
        x[5] = tw16<1, INV>(x[5]);
        x[6] = tw16<2, INV>(x[6]);
        x[7] = tw16<3, INV>(x[7]);
        x[9] = tw16<2, INV>(x[9]);
        x[10] = tw16<4, INV>(x[10]);
        x[11] = tw16<6, INV>(x[11]);
        x[13] = tw16<3, INV>(x[13]);
        x[14] = tw16<6, INV>(x[14]);
        x[15] = tw16<9, INV>(x[15]);
        dft4<INV>(x[0], x[1], x[2], x[3]);
        dft4<INV>(x[4], x[5], x[6], x[7]);
        dft4<INV>(x[8], x[9], x[10], x[11]);
        dft4<INV>(x[12], x[13], x[14], x[15]);
        float2 y[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) y[k1 + 4 * k2] = x[4 * k1 + k2];
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = y[k];
    } else {
        static_assert(R == 2 || R == 4 || R == 8 || R == 16, "unsupported radix");
    }
}

// Padded LDS index: one spare element after every 16, against bank conflicts
// of the strided Stockham writes.  Lines of one work-group are a further 8
// elements apart (16 banks), so the 4 lines that share a wave fall on
// different banks.
__device__ __forceinline__ constexpr int lds_pad(int i) { return i + (i >> 4); }
#ifndef PM_LDS_LINE_EXTRA
#define PM_LDS_LINE_EXTRA 8
#endif
__host__ __device__ constexpr int lds_line_len(int L) { return L + L / 16 + PM_LDS_LINE_EXTRA; }

// Radix of the stage that starts at sub-transform length NS.
__host__ __device__ constexpr int stage_radix(int L, int P, int NS) {
    return (L / NS) >= P ? P : (L / NS);
}

// Twiddles a thread multiplies in the stages that start at NS and later:
// (P/R)(R-1) per stage with NS > 1.
__host__ __device__ constexpr int twiddles_from(int L, int P, int NS) {
    return NS >= L ? 0
                   : (NS > 1 ? (P / stage_radix(L, P, NS)) * (stage_radix(L, P, NS) - 1) : 0) +
                         twiddles_from(L, P, NS * stage_radix(L, P, NS));
}

// The thread's twiddle factors for a whole line transform, loaded once from
// the table before any barrier (so their latency overlaps the data loads);
// the inverse transform uses their conjugates.
template <int L, int P>
struct LineTwiddles {
    static constexpr int COUNT = twiddles_from(L, P, 1) > 0 ? twiddles_from(L, P, 1) : 1;
    float2 w[COUNT];
};

template <int L, int P, int NS, int OFF>
__device__ __forceinline__ void load_twiddles_from(LineTwiddles<L, P>& tw, int j, const float2* __restrict__ table,
                                                   int step) {
    if constexpr (NS < L) {
        constexpr int T = L / P;
        constexpr int R = stage_radix(L, P, NS);
        constexpr int M = P / R;
        if constexpr (NS > 1) {
            constexpr int STRIDE = L / (NS * R);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int k = (j + T * m) & (NS - 1);
#pragma unroll
                for (int q = 1; q < R; ++q) tw.w[OFF + m * (R - 1) + (q - 1)] = table[q * k * STRIDE * step];
            }
            load_twiddles_from<L, P, NS * R, OFF + M * (R - 1)>(tw, j, table, step);
        } else {
            load_twiddles_from<L, P, NS * R, OFF>(tw, j, table, step);
        }
    }
}

// `table` holds exp(-2 pi i k / (L step)); entry k step is exp(-2 pi i k / L),
// so one table of the largest length serves every shorter power of two.
template <int L, int P>
__device__ __forceinline__ void load_twiddles(LineTwiddles<L, P>& tw, int j, const float2* __restrict__ table,
                                              int step) {
    load_twiddles_from<L, P, 1, 0>(tw, j, table, step);
}

// LDS exchange buffers per line: two (alternating, one barrier per
// exchange) when that leaves room for two work-groups per CU, else one (two
// barriers per exchange).  `stride` is the distance between the buffers.
template <int L, int G>
struct LdsPlan {
    static constexpr int LP = lds_line_len(L);
    static constexpr int NBUF = (2 * G * LP * 8 <= 80 * 1024) ? 2 : 1;
    static constexpr int FLOATS2 = NBUF * G * LP;  // float2 elements per work-group
    static constexpr int STRIDE = G * LP;
};

// Number of LDS exchanges in one line transform (= stages - 1).
__host__ __device__ constexpr int exchanges_from(int L, int P, int NS) {
    return NS * stage_radix(L, P, NS) >= L ? 0 : 1 + exchanges_from(L, P, NS * stage_radix(L, P, NS));
}

// One Stockham stage on the thread's P register points (see header); OFF is
// this stage's first entry in the thread's twiddle registers, PAR the LDS
// buffer this stage's exchange uses when NBUF == 2.
template <int L, int P, int NS, int OFF, bool INV, int NBUF, int PAR>
__device__ __forceinline__ void fft_stage(float2 (&v)[P], int j, float2* line, int stride,
                                          const LineTwiddles<L, P>& tw) {
    constexpr int T = L / P;
    constexpr int R = stage_radix(L, P, NS);
    constexpr int M = P / R;
    constexpr bool LAST = (NS * R == L);
    float2* buf = (NBUF == 2 && PAR == 1) ? line + stride : line;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float2 x[R];
#pragma unroll
        for (int q = 0; q < R; ++q) x[q] = v[m + q * M];
        const int b = j + T * m;
        const int k = b & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                float2 w = tw.w[OFF + m * (R - 1) + (q - 1)];
                if constexpr (INV) w.y = -w.y;
                x[q] = cmul(x[q], w);
            }
        }
        dft<R, INV>(x);
        if constexpr (LAST) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[m + q * M] = x[q];
        } else {
            const int base = (b - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[lds_pad(base + q * NS)] = x[q];
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < P; ++t) v[t] = buf[lds_pad(j + T * t)];
        // With one buffer the next stage's writes must wait for every read;
        // with two they go to the other buffer, whose last reads finished
        // before the barrier above.
        if constexpr (NBUF == 1) __syncthreads();
        fft_stage<L, P, NS * R, (NS > 1 ? OFF + M * (R - 1) : OFF), INV, NBUF, PAR ^ 1>(v, j, line,
                                                                                     stride, tw);
    }
}

// Full length-L transform of one line; every thread of the work-group must
// call it (it contains work-group barriers).  Consecutive transforms in one
// kernel must pass PAR = the parity after the previous one
// (fft_parity_after) so that the buffers keep alternating.
template <int L, int P, bool INV, int NBUF, int PAR>
__device__ __forceinline__ void fft_line(float2 (&v)[P], int j, float2* line, int stride,
                                         const LineTwiddles<L, P>& tw) {
    fft_stage<L, P, 1, 0, INV, NBUF, PAR>(v, j, line, stride, tw);
}

template <int L, int P, int PAR>
__host__ __device__ constexpr int fft_parity_after() {
    return (PAR + exchanges_from(L, P, 1)) & 1;
}

// Points per thread for a line of L points.
__host__ __device__ constexpr int points_per_thread(int L) {
    return L >= 256 ? 16 : (L >= 32 ? 8 : 4);
}

}  // namespace pm
