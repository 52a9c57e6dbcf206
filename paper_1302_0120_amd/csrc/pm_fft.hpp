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
//     first read / last write can go straight to or from global memory.  A
//     last radix-2 stage after a radix-P stage can instead swap operands
//     between the two halves of a wave (fft_last_radix2_lanes).
//   * Radix sequence: P, P, ..., then the remaining factor (each divides P)
//     for powers of two; fixed mixed-radix sequences (radices 4, 6, 10, 12,
//     20, 30) for the non-power-of-two lengths 600, 800, 1080 and 1920,
//     whose butterfly index b and sub-length NS are then not powers of two
//     (b mod NS is a true modulo).
//   * Twiddles come from a staged table (one block per stage, see
//     twiddle_block) computed on the host in double precision and rounded
//     once to float; each thread loads the ones it needs into registers at
//     kernel start (or, for the long mixed-radix plans, reads them from the
//     table stage by stage).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "pm_common.h"

namespace pm {

// Pointer to element i of a device array, from a base pointer and a 32-bit
// element offset.  The byte offset is formed in 32 bits and zero-extended,
// which lets the compiler use the scalar-base form of the global memory
// instructions (base in scalar registers, one 32-bit offset per lane)
// instead of 64-bit address arithmetic on every lane.  Offsets stay below
// 2^29 elements: the largest array indexed this way holds 4096^2 elements.
template <class T>
__device__ __forceinline__ T* elem_ptr(T* base, unsigned i) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + (size_t)(i * (unsigned)sizeof(T)));
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Products are written with explicit fused multiply-adds and the library
// is compiled without automatic contraction, so every instantiation of a
// formula (any line count, either pass, one-mask or batched) rounds the
// same way and gives bitwise the same result.
//
// a * (c + i s): (a.x c - a.y s, a.x s + a.y c), one rounding per product
// term pair.
__device__ __forceinline__ float2 cmul_cs(float2 a, float c, float s) {
    return make_float2(fmaf(a.x, c, -(a.y * s)), fmaf(a.x, s, a.y * c));
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) { return cmul_cs(a, b.x, b.y); }
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
        return cmul_cs(a, c, s);
    }
}

// In-register DFTs of R = 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 30 points,
// natural order in and out.
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

// Radix-3 DFT from its definition with w = exp(-+2 pi i / 3):
// X0 = x0 + (x1 + x2); X1,2 = x0 - (x1 + x2)/2 -+ i (sqrt(3)/2)(x1 - x2).
template <bool INV>
__device__ __forceinline__ void dft3(float2& x0, float2& x1, float2& x2) {
    constexpr float S3 = 0.86602540378443865f;  // sin(2 pi / 3)
    const float2 s = cadd(x1, x2);
    const float2 d = csub(x1, x2);
    const float2 t = make_float2(fmaf(-0.5f, s.x, x0.x), fmaf(-0.5f, s.y, x0.y));
    const float2 r = rot90<INV>(make_float2(S3 * d.x, S3 * d.y));  // -+i (sqrt3/2) d
    x0 = cadd(x0, s);
    x1 = cadd(t, r);
    x2 = csub(t, r);
}

// Radix-5 DFT from its definition with w = exp(-+2 pi i / 5), pairing
// n with 5 - n (s = pair sums, d = pair differences):
//   X_{1,4} = x0 + c1 s1 + c2 s2 -+ i (S1 d1 + S2 d2),
//   X_{2,3} = x0 + c2 s1 + c1 s2 -+ i (S2 d1 - S1 d2),
// c_k = cos(2 pi k / 5), S_k = sin(2 pi k / 5).  The cosine parts are formed
// as x0 - (s1 + s2)/4 +- (sqrt5/4)(s1 - s2) (c1 + c2 = -1/2, c1 - c2 =
// sqrt5/2), so equal inputs give exact zeros off the zero frequency.
template <bool INV>
__device__ __forceinline__ void dft5(float2& x0, float2& x1, float2& x2, float2& x3, float2& x4) {
    constexpr float Q5 = 0.55901699437494742f;   // sqrt(5) / 4
    constexpr float S1 = 0.95105651629515357f;   // sin(2 pi / 5)
    constexpr float S2 = 0.58778525229247313f;   // sin(4 pi / 5)
    const float2 s1 = cadd(x1, x4), d1 = csub(x1, x4);
    const float2 s2 = cadd(x2, x3), d2 = csub(x2, x3);
    const float2 t1 = cadd(s1, s2), t2 = csub(s1, s2);
    const float2 a = make_float2(fmaf(-0.25f, t1.x, x0.x), fmaf(-0.25f, t1.y, x0.y));
    const float2 m2 = make_float2(Q5 * t2.x, Q5 * t2.y);
    const float2 a1 = cadd(a, m2), a2 = csub(a, m2);
    const float2 b1 = rot90<INV>(make_float2(fmaf(S1, d1.x, S2 * d2.x), fmaf(S1, d1.y, S2 * d2.y)));
    const float2 b2 = rot90<INV>(make_float2(fmaf(S2, d1.x, -(S1 * d2.x)), fmaf(S2, d1.y, -(S1 * d2.y))));
    x0 = cadd(x0, t1);
    x1 = cadd(a1, b1);
    x4 = csub(a1, b1);
    x2 = cadd(a2, b2);
    x3 = csub(a2, b2);
}

// cos and sin of 2 pi e / d for the internal twiddles of composite radices,
// evaluated at compile time in double: the angle reduced to [-pi, pi], then
// the Taylor series (30 terms; the largest term at pi is below 6, so the
// cancellation error stays near 1e-15), rounded once to float.  Values
// within 1e-12 of 0 are snapped to 0 (the quarter turns).
__host__ __device__ constexpr double ct_angle(int e, int d) {
    int r = ((e % d) + d) % d;
    if (2 * r > d) r -= d;
    return 6.283185307179586476925286766559 * (double)r / (double)d;
}
__host__ __device__ constexpr double ct_sin(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return (sum < 1e-12 && sum > -1e-12) ? 0.0 : sum;
}
__host__ __device__ constexpr double ct_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return (sum < 1e-12 && sum > -1e-12) ? 0.0 : sum;
}

template <int D>
struct TurnTable {
    float c[D], s[D];
    constexpr TurnTable() : c(), s() {
        for (int e = 0; e < D; ++e) {
            c[e] = (float)ct_cos(ct_angle(e, D));
            s[e] = (float)ct_sin(ct_angle(e, D));
        }
    }
};

// R = R1 R2 by one Cooley-Tukey step: n = R2 n1 + n2, k = k1 + R1 k2.
// DFT_R1 over n1 for each n2, twiddle exp(-+2 pi i n2 k1 / R), DFT_R2 over
// n2 for each k1.  All indices are compile-time constants once the loops
// are unrolled, so the twiddles are immediate constants.
template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&x)[R]);

template <int R1, int R2, bool INV>
__device__ __forceinline__ void dft_ct(float2 (&x)[R1 * R2]) {
    constexpr int R = R1 * R2;
    constexpr TurnTable<R> tt{};
    float2 y[R];  // y[n2 R1 + k1]
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        float2 col[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) col[n1] = x[R2 * n1 + n2];
        dft<R1, INV>(col);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            const int e = (n2 * k1) % R;
            if (e == 0) {
                y[n2 * R1 + k1] = col[k1];
            } else {
                const float c = tt.c[e];
                const float sn = INV ? tt.s[e] : -tt.s[e];
                y[n2 * R1 + k1] = cmul_cs(col[k1], c, sn);
            }
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        float2 row[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) row[n2] = y[n2 * R1 + k1];
        dft<R2, INV>(row);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) x[k1 + R1 * k2] = row[k2];
    }
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&x)[R]) {
    if constexpr (R == 3) {
        dft3<INV>(x[0], x[1], x[2]);
    } else if constexpr (R == 5) {
        dft5<INV>(x[0], x[1], x[2], x[3], x[4]);
    } else if constexpr (R == 6) {
        dft_ct<3, 2, INV>(x);
    } else if constexpr (R == 10) {
        dft_ct<5, 2, INV>(x);
    } else if constexpr (R == 12) {
        dft_ct<3, 4, INV>(x);
    } else if constexpr (R == 20) {
        dft_ct<4, 5, INV>(x);
    } else if constexpr (R == 30) {
        dft_ct<10, 3, INV>(x);
    } else if constexpr (R == 2) {
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
        static_assert(R == 2 || R == 3 || R == 4 || R == 5 || R == 6 || R == 8 || R == 10 || R == 12 ||
                          R == 16 || R == 20 || R == 30,
                      "unsupported radix");
    }
}

// LDS index of element i of a line of L points.  The padding scheme is a
// tuning knob per length (every scheme is a bijection onto a line of
// lds_line_len elements, so results do not depend on it):
//   0: one spare element after every 16;  1: after every 32;  2: none;
//   3: after every 16 and another after every 256.
// PM_LDS_PAD applies up to 1024 points, PM_LDS_PAD_LONG to 2048 and 4096.
// Lines of one work-group are PM_LDS_LINE_EXTRA elements further apart, so
// the lines that share a wave fall on different banks.  Measured on MI355X
// (1024^2 and 800 x 600 solves, 11 layouts): no padding with lines 4
// elements apart (any extra of 4 mod 8) is fastest, 5.5% faster than one
// spare per 16 with lines 8 apart at 1024^2 and 8% faster at 800 x 600.
// For 2048 and 4096 points (16 points per thread, so the first exchange
// writes each wave's outputs 16 elements apart), one spare per 32 is
// fastest: 2048^2 -3.8%, 4096^2 -9.6% per solve against no padding (one
// spare per 16: -3.3% and -7.8%); at 1024^2 it costs 1-3%.
#ifndef PM_LDS_PAD
#define PM_LDS_PAD 2
#endif
#ifndef PM_LDS_PAD_LONG
#define PM_LDS_PAD_LONG 1
#endif
#ifndef PM_LDS_LINE_EXTRA
#define PM_LDS_LINE_EXTRA 4
#endif
__host__ __device__ constexpr int lds_pad_scheme(int L) {
    return (L == 2048 || L == 4096) ? PM_LDS_PAD_LONG : PM_LDS_PAD;
}
// A layout code LAY = scheme * 64 + extra names a padding scheme (as above)
// and the extra elements between consecutive lines (< 64).  Each pass
// type takes its layout as a template argument; lds_layout(L) is the
// default, row_lds_layout(L) the one-mask row pass's (PM_ROW_LDS_LAYOUT
// overrides it at every power-of-two length up to 1024).
__host__ __device__ constexpr int lds_layout(int L) { return lds_pad_scheme(L) * 64 + PM_LDS_LINE_EXTRA; }
#ifndef PM_ROW_LDS_LAYOUT
#define PM_ROW_LDS_LAYOUT -1
#endif
// The row swizzle also at 512 points (two-row tiles, same exchange patterns:
// 512 row pass conflict-free; 512^2 x 50 solve 0.4150 -> 0.4128 ms).
#ifndef PM_ROW_SWZ_512
#define PM_ROW_SWZ_512 1
#endif
__host__ __device__ constexpr int row_lds_layout(int L) {
    return (PM_ROW_LDS_LAYOUT >= 0 && L <= 1024 && (L & (L - 1)) == 0) ? PM_ROW_LDS_LAYOUT
         : (L == 1024 || (L == 512 && PM_ROW_SWZ_512)) ? 4 * 64 + 8
                                                       : lds_layout(L);
}
// The intensity-loss row passes keep the unswizzled layout at 512: there the
// swizzle made the 16 x 512^2 Adam solve 5% slower (0.0475 -> 0.0499 ms per
// step).
__host__ __device__ constexpr int adj_row_lds_layout(int L) { return L == 512 ? lds_layout(L) : row_lds_layout(L); }
// Schemes 4 and 5 are swizzles without spare slots: element i of a line
// sits at i ^ mask(i), mask(i) = (bit 4 of i) << 2 ^ key (scheme 4) or
// (bits 3-4 of i) << 1 ^ key (scheme 5), where `key` (0, 2, 4 or 6) is a
// per-line constant the pass chooses.  The mask only flips bits 1-2 and is
// steered by bits 3-4, which it never flips, so each map is a bijection of
// [0, L) that keeps 16-byte pairs together, and adding a multiple of 32 to
// i adds it to the slot (one base address serves a thread's strided reads).
__host__ __device__ constexpr int lds_pad_lay(int lay, int i) {
    return lay / 64 == 0 ? i + (i >> 4)
         : lay / 64 == 1 ? i + (i >> 5)
         : lay / 64 == 2 ? i
         : lay / 64 == 3 ? i + (i >> 4) + (i >> 8)
                         : i;
}
__host__ __device__ constexpr int lds_swizzle_mask(int lay, int i, int key) {
    return lay / 64 == 4 ? ((((i >> 4) & 1) << 2) ^ key) : lay / 64 == 5 ? ((((i >> 3) & 3) << 1) ^ key) : 0;
}
__host__ __device__ constexpr bool lds_swizzled(int lay) { return lay / 64 == 4 || lay / 64 == 5; }
__host__ __device__ constexpr int lds_index(int lay, int i, int key) {
    return lds_swizzled(lay) ? (i ^ lds_swizzle_mask(lay, i, key)) : lds_pad_lay(lay, i);
}
#ifndef PM_COL_LDS_LAYOUT
#define PM_COL_LDS_LAYOUT -1
#endif
// Columns per one-mask column work-group at 1024 points (col_lines): 4 (a
// whole strip) or 2 (half strips).
#ifndef PM_COL_LINES_1024
#define PM_COL_LINES_1024 4
#endif
#ifndef PM_COL_LINES_512
#define PM_COL_LINES_512 4
#endif

// Layout of the one-mask column pass (PM_COL_LDS_LAYOUT overrides it at
// 1024).  Half strips at 1024 hold two lines whose lanes alternate, as the
// two-row tiles of the row pass do, and take the row pass's swizzle.
__host__ __device__ constexpr int col_lds_layout(int L) {
    return (PM_COL_LDS_LAYOUT >= 0 && L == 1024) ? PM_COL_LDS_LAYOUT
         : ((L == 1024 && PM_COL_LINES_1024 == 2) || (L == 512 && PM_COL_LINES_512 == 2)) ? 4 * 64 + 8
                                                                                          : lds_layout(L);
}
__host__ __device__ constexpr int lds_line_len_lay(int L, int lay) { return lds_pad_lay(lay, L) + lay % 64; }
__host__ __device__ constexpr int lds_pad(int L, int i) { return lds_pad_lay(lds_layout(L), i); }
__host__ __device__ constexpr int lds_line_len(int L) { return lds_line_len_lay(L, lds_layout(L)); }

// LDS-resident transforms.  For lengths whose register plan would need too
// many points per thread (1920 needs P = 60 and spills), every stage reads
// its butterfly inputs from LDS and writes its outputs back to LDS, so the
// stage radices need not divide the points per thread: T threads per line
// share the L / R butterflies of a stage in rounds.  Costs one more LDS
// write and read per transform (the line enters and leaves LDS in natural
// order) and, with ragged rounds, some idle lanes.  PM_LDS_MODE_<L> selects
// the scheme for the other mixed-radix lengths; measured on MI355X, LDS mode
// is faster for 600 (column pass 9.2 -> 6.9 us at 800 x 600) and 1080 (22
// -> 14 us at 1080 x 1920), slower for 800 (7.1 -> 8.0 us).
#ifndef PM_LDS_MODE_600
#define PM_LDS_MODE_600 1
#endif
#ifndef PM_LDS_MODE_800
#define PM_LDS_MODE_800 0
#endif
#ifndef PM_LDS_MODE_1080
#define PM_LDS_MODE_1080 1
#endif
__host__ __device__ constexpr bool lds_mode(int L) {
    return L == 1920 || (L == 600 && PM_LDS_MODE_600) || (L == 800 && PM_LDS_MODE_800) ||
           (L == 1080 && PM_LDS_MODE_1080);
}
// Threads per line in LDS mode.
#ifndef PM_LDS_T_1920
#define PM_LDS_T_1920 128
#endif
#ifndef PM_LDS_T_600
#define PM_LDS_T_600 60
#endif
#ifndef PM_LDS_T_800
#define PM_LDS_T_800 80
#endif
#ifndef PM_LDS_R_800
#define PM_LDS_R_800 0
#endif
__host__ __device__ constexpr int lds_threads(int L) {
    return L == 1920 ? PM_LDS_T_1920 : (L == 600 ? PM_LDS_T_600 : (L == 800 ? PM_LDS_T_800 : 120));
}
// Radix sequences in LDS mode (largest radix first, where no inter-stage
// twiddles are needed): 1920 = 16*12*10, 600 = 10*6*10, 800 = 20*10*4
// (PM_LDS_R_800 = 1: 10*10*8), 1080 = 30*6*6.
__host__ __device__ constexpr int lds_stage_radix(int L, int NS) {
    return L == 1920 ? (NS == 1 ? 16 : (NS == 16 ? 12 : 10))
         : L == 600 ? (NS == 1 ? 10 : (NS == 10 ? 6 : 10))
         : (L == 800 && PM_LDS_R_800 == 1) ? (NS == 1 ? 10 : (NS == 10 ? 10 : 8))
         : L == 800 ? (NS == 1 ? 20 : (NS == 20 ? 10 : 4))
                    : (NS == 1 ? 30 : 6);
}
__host__ __device__ constexpr int lds_num_stages(int L, int NS = 1) {
    return NS >= L ? 0 : 1 + lds_num_stages(L, NS * lds_stage_radix(L, NS));
}
// LDS mode preloads its inter-stage twiddles into registers only for 600
// points (measured: 800 x 600 solve 3% faster); for 1080 the extra
// registers halve the work-groups per CU (pass 14 -> 20 us), for 1920 it
// is neutral, so those read the table stage by stage.
__host__ __device__ constexpr bool lds_preload(int L) { return L == 600; }

// Inter-stage twiddles a thread multiplies in LDS mode from sub-length NS on
// (R - 1 per butterfly round of every stage with NS > 1).
__host__ __device__ constexpr int lds_twiddles_from(int L, int NS) {
    return NS >= L ? 0
                   : (NS > 1 ? ((L / lds_stage_radix(L, NS) + lds_threads(L) - 1) / lds_threads(L)) *
                                   (lds_stage_radix(L, NS) - 1)
                             : 0) +
                         lds_twiddles_from(L, NS * lds_stage_radix(L, NS));
}

// Radix of the stage that starts at sub-transform length NS.  Powers of two
// take P, P, ..., remainder.  The non-power-of-two lengths of common SLM
// panels (800 x 600, 1920 x 1080) take fixed mixed-radix sequences whose
// radices divide P: 800 = 10*10*2*2*2 (P = 10; 20*10*4 with P = 20),
// 600 = 6*10*10 (P = 30), 1080 = 30*6*6 (P = 30), 1920 = 12*10*4*4 (P = 60).
// The largest radix goes first, where no inter-stage twiddles are needed.
__host__ __device__ constexpr int stage_radix(int L, int P, int NS) {
    if (L == 800 && P == 10) return NS <= 10 ? 10 : 2;
    if (L == 800) return NS == 1 ? 20 : (NS == 20 ? 10 : 4);
    if (L == 600) return NS == 1 ? 6 : 10;
    if (L == 1080) return NS == 1 ? 30 : 6;
    if (L == 1920) return NS == 1 ? 12 : (NS == 12 ? 10 : 4);
    return (L / NS) >= P ? P : (L / NS);
}

// Twiddles a thread multiplies in the stages that start at NS and later:
// (P/R)(R-1) per stage with NS > 1.
__host__ __device__ constexpr int twiddles_from(int L, int P, int NS) {
    return NS >= L ? 0
                   : (NS > 1 ? (P / stage_radix(L, P, NS)) * (stage_radix(L, P, NS) - 1) : 0) +
                         twiddles_from(L, P, NS * stage_radix(L, P, NS));
}

// Radix of the stage at sub-length NS in the scheme the length uses.
__host__ __device__ constexpr int line_stage_radix(int L, int P, int NS) {
    return lds_mode(L) ? lds_stage_radix(L, NS) : stage_radix(L, P, NS);
}

// Staged twiddle table of a line plan (L, P): one block per stage with
// NS > 1, in stage order; the block of the stage at NS with radix R holds
// (R - 1) NS entries, entry (q - 1) NS + k = exp(-2 pi i q k / (NS R)) for
// q = 1 .. R - 1 and k = 0 .. NS - 1.  A wave's threads read consecutive k
// for a fixed q, so each table read of a wave touches a few contiguous
// cache lines instead of one line per lane.  twiddle_block gives the first
// entry of the stage at NS (stages before it summed from `cur` on).
__host__ __device__ constexpr int twiddle_block(int L, int P, int NS, int cur = 1) {
    return cur >= NS ? 0
                     : (cur > 1 ? (line_stage_radix(L, P, cur) - 1) * cur : 0) +
                           twiddle_block(L, P, NS, cur * line_stage_radix(L, P, cur));
}
__host__ __device__ constexpr int twiddle_entries(int L, int P) { return twiddle_block(L, P, L); }

// The batched plans keep the staged tables of every schedule and power-of-two
// length in one buffer, schedule by schedule, lengths ascending; this is the
// first entry of (schedule sched, length L), and with sched = kBatchSchedules
// the total.
__host__ __device__ constexpr int batch_twiddle_offset(int sched, int L) {
    int off = 0;
    for (int s = 0; s < kBatchSchedules; ++s) {
        for (int l = kBatchMinLen; l <= kBatchMaxLen; l *= 2) {
            if (s == sched && l == L) return off;
            off += twiddle_entries(l, batch_points(s, l));
        }
    }
    return off;
}

// The thread's twiddle factors for a whole line transform, loaded once from
// the table before any barrier (so their latency overlaps the data loads);
// the inverse transform uses their conjugates.  Plans that need more than
// kMaxTwiddleRegs of them (the 1920-point plan, 144 factors) would not fit
// the register file next to their data, so their stages read the factors
// from the table (an L1-resident few KB) instead.  (Up to 56 preloaded:
// the 600-point plan needs 54 and measured 13% faster preloaded.)
#ifndef PM_MAX_TWIDDLE_REGS
#define PM_MAX_TWIDDLE_REGS 56
#endif
constexpr int kMaxTwiddleRegs = PM_MAX_TWIDDLE_REGS;

template <int L, int P>
struct LineTwiddles {
    static constexpr int NEED = lds_mode(L) ? lds_twiddles_from(L, 1) : twiddles_from(L, P, 1);
    static constexpr bool PRELOAD = lds_mode(L) ? lds_preload(L) : NEED <= kMaxTwiddleRegs;
    static constexpr int COUNT = (PRELOAD && NEED > 0) ? NEED : 1;
    float2 w[COUNT];
    const float2* table;   // the staged table of (L, P)
};

template <int L, int P, int NS, int OFF>
__device__ __forceinline__ void load_twiddles_from(LineTwiddles<L, P>& tw, int j, const float2* __restrict__ table) {
    if constexpr (NS < L) {
        constexpr int T = L / P;
        constexpr int R = stage_radix(L, P, NS);
        constexpr int M = P / R;
        if constexpr (NS > 1) {
            constexpr int BLOCK = twiddle_block(L, P, NS);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const unsigned k = (unsigned)((j + T * m) % NS);
#pragma unroll
                for (int q = 1; q < R; ++q)
                    tw.w[OFF + m * (R - 1) + (q - 1)] = *elem_ptr(table, BLOCK + (q - 1) * NS + k);
            }
            load_twiddles_from<L, P, NS * R, OFF + M * (R - 1)>(tw, j, table);
        } else {
            load_twiddles_from<L, P, NS * R, OFF>(tw, j, table);
        }
    }
}

// LDS mode: the twiddles of every round of every stage (rounds past the
// last butterfly load a harmless entry and are never used).
template <int L, int P, int NS, int OFF>
__device__ __forceinline__ void lds_load_twiddles_from(LineTwiddles<L, P>& tw, int j,
                                                       const float2* __restrict__ table) {
    if constexpr (NS < L) {
        constexpr int T = lds_threads(L);
        constexpr int R = lds_stage_radix(L, NS);
        constexpr int NB = L / R;
        constexpr int ROUNDS = (NB + T - 1) / T;
        if constexpr (NS > 1) {
            constexpr int BLOCK = twiddle_block(L, P, NS);
#pragma unroll
            for (int m = 0; m < ROUNDS; ++m) {
                const int b = j + T * m;
                const unsigned k = (unsigned)(b < NB ? b % NS : 0);
#pragma unroll
                for (int q = 1; q < R; ++q)
                    tw.w[OFF + m * (R - 1) + (q - 1)] = *elem_ptr(table, BLOCK + (q - 1) * NS + k);
            }
            lds_load_twiddles_from<L, P, NS * R, OFF + ROUNDS * (R - 1)>(tw, j, table);
        } else {
            lds_load_twiddles_from<L, P, NS * R, OFF>(tw, j, table);
        }
    }
}

// `table` is the staged twiddle table of (L, P) (twiddle_block).
template <int L, int P>
__device__ __forceinline__ void load_twiddles(LineTwiddles<L, P>& tw, int j, const float2* __restrict__ table) {
    tw.table = table;
    if constexpr (LineTwiddles<L, P>::PRELOAD) {
        if constexpr (lds_mode(L)) {
            lds_load_twiddles_from<L, P, 1, 0>(tw, j, table);
        } else {
            load_twiddles_from<L, P, 1, 0>(tw, j, table);
        }
    }
}

// LDS exchange buffers per line: two (alternating, one barrier per
// exchange) when that leaves room for two work-groups per CU, else one (two
// barriers per exchange).  NBMAX = 1 asks for one buffer wherever the scheme
// allows it (LDS mode always ping-pongs): the batched passes, whose many
// independent work-groups gain more from twice the work-groups per CU than
// they lose to the second barrier (64-mask workload: 2970 -> 3570 masks/s;
// the one-mask 1024^2 solve, one work-group per CU, is 1% slower that way).
// `stride` is the distance between the buffers.
template <int L, int G, int NBMAX = 2, int LAY = lds_layout(L)>
struct LdsPlan {
    static constexpr int LP = lds_line_len_lay(L, LAY);
    static constexpr int NBUF = (lds_mode(L) || (NBMAX == 2 && 2 * G * LP * 8 <= 80 * 1024)) ? 2 : 1;
    static constexpr int FLOATS2 = NBUF * G * LP;  // float2 elements per work-group
    static constexpr int STRIDE = G * LP;
};

// Number of LDS exchanges in one line transform (= stages - 1).
__host__ __device__ constexpr int exchanges_from(int L, int P, int NS) {
    return NS * stage_radix(L, P, NS) >= L ? 0 : 1 + exchanges_from(L, P, NS * stage_radix(L, P, NS));
}

// Sub-length at which the last stage of the register scheme starts.
__host__ __device__ constexpr int last_stage_ns(int L, int P, int NS = 1) {
    return NS * stage_radix(L, P, NS) >= L ? NS : last_stage_ns(L, P, NS * stage_radix(L, P, NS));
}

// Plans whose last stage has radix Q = 2 or 4 right after a stage of radix P
// (one butterfly per thread), e.g. 8-8-8-2 at 1024, 16-16-2 at 512, 8-8-2 at
// 128, 16-16-4 at 1024: there the last stage can take its operands across
// lanes instead of through LDS (fft_last_radix2_lanes, _radix4_lanes),
// provided lanes i + 64 k / Q, k < Q, of every wave hold threads j + k T / Q
// of one line.  T % 16 == 0 keeps the lane layouts of the passes whole.
// lane_group is that Q, 0 for other plans.
__host__ __device__ constexpr int lane_group(int L, int P) {
    return (!lds_mode(L) && last_stage_ns(L, P) > P && stage_radix(L, P, last_stage_ns(L, P) / P) == P &&
            (L / P) % 16 == 0 &&
            (stage_radix(L, P, last_stage_ns(L, P)) == 2 || stage_radix(L, P, last_stage_ns(L, P)) == 4))
               ? stage_radix(L, P, last_stage_ns(L, P))
               : 0;
}
__host__ __device__ constexpr bool lane_swap_plan(int L, int P) { return lane_group(L, P) != 0; }

// Exchanges one float between the halves of a wave: afterwards lanes 0..31
// hold in `hi` the `lo` of lane i + 32, and lanes 32..63 hold in `lo` the
// `hi` of lane i - 32; the other two values stay.
__device__ __forceinline__ void swap_halves(float& lo, float& hi) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    lo = __uint_as_float(r[0]);
    hi = __uint_as_float(r[1]);
}

// The same between the quarters of each half: afterwards lanes of quarters
// 0 and 2 hold in `hi` the `lo` of lane i + 16, and lanes of quarters 1 and 3
// hold in `lo` the `hi` of lane i - 16.
__device__ __forceinline__ void swap_quarters(float& lo, float& hi) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    lo = __uint_as_float(r[0]);
    hi = __uint_as_float(r[1]);
}

// The last stage (radix 2, sub-length L/2) of a lane_swap_plan, with lanes i
// and i + 32 holding threads j and j + T/2 of the line.  After the stage
// before it, v[q] of thread j is element (L/2)(j / (T/2)) + j % (T/2) +
// (T/2) q.  Butterfly m of thread j pairs elements p = j + T m and p + L/2:
// for the lower thread p is its own v[2m] and p + L/2 the partner's v[2m];
// for the upper thread p is the partner's v[2m + 1] and p + L/2 its own.
// Swapping v[2m + 1] of the lower lanes with v[2m] of the upper lanes hands
// every thread both operands.  Twiddles, arithmetic and the result slots
// (v[m], v[m + P/2]) are those of the LDS exchange path, so both give
// identical results.
template <int L, int P, int OFF, bool INV>
__device__ __forceinline__ void fft_last_radix2_lanes(float2 (&v)[P], int j, const LineTwiddles<L, P>& tw) {
    constexpr int T = L / P;
    constexpr int NS = L / 2;
    constexpr int H2 = P / 2;
    float2 y[P];
#pragma unroll
    for (int m = 0; m < H2; ++m) {
        float2 a = v[2 * m];
        float2 b = v[2 * m + 1];
        swap_halves(a.x, b.x);
        swap_halves(a.y, b.y);
        const int k = j + T * m;  // < L/2, so this is also (j + T m) mod NS
        float2 w;
        if constexpr (LineTwiddles<L, P>::PRELOAD) {
            w = tw.w[OFF + m];
        } else {
            w = *elem_ptr(tw.table, (unsigned)(twiddle_block(L, P, NS) + k));
        }
        if constexpr (INV) w.y = -w.y;
        float2 x[2] = {a, cmul(b, w)};
        dft<2, INV>(x);
        y[m] = x[0];
        y[m + H2] = x[1];
    }
#pragma unroll
    for (int t = 0; t < P; ++t) v[t] = y[t];
}

// The last stage (radix 4, sub-length L/4) of a plan with lane_group 4,
// lanes i, i + 16, i + 32, i + 48 holding threads j, j + T/4, j + T/2,
// j + 3T/4 of the line (quarter s of the wave holds the threads with
// j / (T/4) = s).  After the stage before it, v[q] of the thread in quarter r
// is element (L/4) r + j % (T/4) + (T/4) q.  Butterfly m of the thread in
// quarter s takes elements b + (L/4) r, r < 4, with b = j + T m, i.e. v[s +
// 4m] of the thread in quarter r: for each m the 4 x 4 block v[4m .. 4m + 3]
// of the four threads is transposed (one half swap and one quarter swap per
// pair of registers), after which v[4m + r] holds input r.  Twiddles,
// arithmetic and result slots (v[m + q P/4]) are those of the LDS path.
template <int L, int P, int OFF, bool INV>
__device__ __forceinline__ void fft_last_radix4_lanes(float2 (&v)[P], int j, const LineTwiddles<L, P>& tw) {
    constexpr int T = L / P;
    constexpr int NS = L / 4;
    constexpr int M = P / 4;
    float2 y[P];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float2 x[4] = {v[4 * m], v[4 * m + 1], v[4 * m + 2], v[4 * m + 3]};
        swap_halves(x[0].x, x[2].x);
        swap_halves(x[0].y, x[2].y);
        swap_halves(x[1].x, x[3].x);
        swap_halves(x[1].y, x[3].y);
        swap_quarters(x[0].x, x[1].x);
        swap_quarters(x[0].y, x[1].y);
        swap_quarters(x[2].x, x[3].x);
        swap_quarters(x[2].y, x[3].y);
        const int k = j + T * m;  // < L/4, so this is also (j + T m) mod NS
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            float2 w;
            if constexpr (LineTwiddles<L, P>::PRELOAD) {
                w = tw.w[OFF + m * 3 + (r - 1)];
            } else {
                w = *elem_ptr(tw.table, (unsigned)(twiddle_block(L, P, NS) + (r - 1) * NS + k));
            }
            if constexpr (INV) w.y = -w.y;
            x[r] = cmul(x[r], w);
        }
        dft<4, INV>(x);
#pragma unroll
        for (int q = 0; q < 4; ++q) y[m + q * M] = x[q];
    }
#pragma unroll
    for (int t = 0; t < P; ++t) v[t] = y[t];
}

// One Stockham stage on the thread's P register points (see header); OFF is
// this stage's first entry in the thread's twiddle registers, PAR the LDS
// buffer this stage's exchange uses when NBUF == 2.  SW: the lanes hold
// their threads as fft_last_radix2_lanes needs, so a lane_swap_plan runs its
// last stage across lanes.
template <int L, int P, int NS, int OFF, bool INV, int NBUF, int PAR, bool SW, int LAY = lds_layout(L)>
__device__ __forceinline__ void fft_stage(float2 (&v)[P], int j, float2* line, int stride,
                                          const LineTwiddles<L, P>& tw, int key = 0) {
    constexpr int T = L / P;
    constexpr int R = stage_radix(L, P, NS);
    constexpr int M = P / R;
    constexpr bool LAST = (NS * R == L);
    constexpr int QN = lane_group(L, P);
    constexpr bool LANES_NEXT = SW && QN != 0 && !LAST && NS * R * QN == L;
    float2* buf = (NBUF == 2 && PAR == 1) ? line + stride : line;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float2 x[R];
#pragma unroll
        for (int q = 0; q < R; ++q) x[q] = v[m + q * M];
        const int b = j + T * m;
        const int k = b % NS;
        if constexpr (NS > 1) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                float2 w;
                if constexpr (LineTwiddles<L, P>::PRELOAD) {
                    w = tw.w[OFF + m * (R - 1) + (q - 1)];
                } else {
                    w = *elem_ptr(tw.table, (unsigned)(twiddle_block(L, P, NS) + (q - 1) * NS + k));
                }
                if constexpr (INV) w.y = -w.y;
                x[q] = cmul(x[q], w);
            }
        }
        dft<R, INV>(x);
        if constexpr (LAST || LANES_NEXT) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[m + q * M] = x[q];
        } else if constexpr (lds_swizzled(LAY) && NS == 1 && R % 2 == 0 && R >= 8) {
            // R contiguous outputs from base = R b: bits 3-4 of base + q equal
            // those of base (q < R, R a multiple of 8), so one mask permutes the
            // 16-byte pairs of the group.
            const int base = b * R;
            const int msk = lds_swizzle_mask(LAY, base, key);
#pragma unroll
            for (int q = 0; q < R; q += 2)
                *reinterpret_cast<float4*>(buf + base + (q ^ msk)) = make_float4(x[q].x, x[q].y, x[q + 1].x, x[q + 1].y);
        } else if constexpr (lds_swizzled(LAY) && NS % 8 == 0) {
            // q NS leaves bits 1-2 alone, so slot(base + q NS) = (base ^ mask) + q NS
            const int base = (b - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[(base ^ lds_swizzle_mask(LAY, base + q * NS, key)) + q * NS] = x[q];
        } else {
            const int base = (b - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[lds_index(LAY, base + q * NS, key)] = x[q];
        }
    }
    if constexpr (LANES_NEXT) {
        static_assert(M == 1, "one butterfly per thread before the cross-lane stage");
        if constexpr (QN == 2) {
            fft_last_radix2_lanes<L, P, (NS > 1 ? OFF + M * (R - 1) : OFF), INV>(v, j, tw);
        } else {
            fft_last_radix4_lanes<L, P, (NS > 1 ? OFF + M * (R - 1) : OFF), INV>(v, j, tw);
        }
    } else if constexpr (!LAST) {
        __syncthreads();
        if constexpr (lds_swizzled(LAY) && T % 32 == 0) {
            // T t is a multiple of 32: one swizzled base, constant offsets
            const int rb = lds_index(LAY, j, key);
#pragma unroll
            for (int t = 0; t < P; ++t) v[t] = buf[rb + T * t];
        } else {
#pragma unroll
            for (int t = 0; t < P; ++t) v[t] = buf[lds_index(LAY, j + T * t, key)];
        }
        // With one buffer the next stage's writes must wait for every read;
        // with two they go to the other buffer, whose last reads finished
        // before the barrier above.
        if constexpr (NBUF == 1) __syncthreads();
        fft_stage<L, P, NS * R, (NS > 1 ? OFF + M * (R - 1) : OFF), INV, NBUF, PAR ^ 1, SW, LAY>(v, j, line,
                                                                                              stride, tw, key);
    }
}

// LDS-mode stages from sub-length NS on: read src, write dst, barrier, swap.
// Thread j takes butterflies b = j + T m of each stage (the last round may
// leave some threads idle); butterfly b reads src[b + q L/R], multiplies by
// exp(-+2 pi i q (b mod NS) / (NS R)), does the R-point DFT and writes
// dst[(b - b mod NS) R + b mod NS + q NS], as in the register scheme.
template <int L, int P, int NS, int OFF, bool INV>
__device__ __forceinline__ void lds_stages(float2* src, float2* dst, int j, const LineTwiddles<L, P>& tw) {
    if constexpr (NS < L) {
        constexpr int T = lds_threads(L);
        constexpr int R = lds_stage_radix(L, NS);
        constexpr int NB = L / R;
        constexpr int ROUNDS = (NB + T - 1) / T;
#pragma unroll
        for (int m = 0; m < ROUNDS; ++m) {
            const int b = j + T * m;
            if (NB % T == 0 || b < NB) {
                float2 x[R];
#pragma unroll
                for (int q = 0; q < R; ++q) x[q] = src[b + q * NB];
                const int k = b % NS;
                if constexpr (NS > 1) {
#pragma unroll
                    for (int q = 1; q < R; ++q) {
                        float2 w;
                        if constexpr (LineTwiddles<L, P>::PRELOAD) {
                            w = tw.w[OFF + m * (R - 1) + (q - 1)];
                        } else {
                            w = *elem_ptr(tw.table, (unsigned)(twiddle_block(L, P, NS) + (q - 1) * NS + k));
                        }
                        if constexpr (INV) w.y = -w.y;
                        x[q] = cmul(x[q], w);
                    }
                }
                dft<R, INV>(x);
                const int base = (b - k) * R + k;
#pragma unroll
                for (int q = 0; q < R; ++q) dst[base + q * NS] = x[q];
            }
        }
        __syncthreads();
        lds_stages<L, P, NS * R, (NS > 1 ? OFF + ROUNDS * (R - 1) : OFF), INV>(dst, src, j, tw);
    }
}

// Whole LDS-mode transform of one line held as v[t] = x[j + T t]: into LDS,
// the stages, back into registers.  Ends with a barrier, so the next
// transform may reuse both buffers.
template <int L, int P, bool INV>
__device__ __forceinline__ void fft_line_lds(float2 (&v)[P], int j, float2* a, float2* b,
                                             const LineTwiddles<L, P>& tw) {
    constexpr int T = lds_threads(L);
    static_assert(T * P == L, "LDS-mode lines hold L / T points per thread");
#pragma unroll
    for (int t = 0; t < P; ++t) a[j + T * t] = v[t];
    __syncthreads();
    lds_stages<L, P, 1, 0, INV>(a, b, j, tw);
    float2* res = (lds_num_stages(L) % 2 == 0) ? a : b;
#pragma unroll
    for (int t = 0; t < P; ++t) v[t] = res[j + T * t];
    __syncthreads();
}

// Full length-L transform of one line; every thread of the work-group must
// call it (it contains work-group barriers).  Consecutive transforms in one
// kernel must pass PAR = the parity after the previous one
// (fft_parity_after, with the same SW) so that the buffers keep alternating.
// SW: see fft_stage.
template <int L, int P, bool INV, int NBUF, int PAR, bool SW = false, int LAY = lds_layout(L)>
__device__ __forceinline__ void fft_line(float2 (&v)[P], int j, float2* line, int stride,
                                         const LineTwiddles<L, P>& tw, int key = 0) {
    if constexpr (lds_mode(L)) {
        static_assert(NBUF == 2, "LDS mode ping-pongs between two buffers");
        fft_line_lds<L, P, INV>(v, j, line, line + stride, tw);
    } else {
        fft_stage<L, P, 1, 0, INV, NBUF, PAR, SW, LAY>(v, j, line, stride, tw, key);
    }
}

template <int L, int P, int PAR, bool SW = false>
__host__ __device__ constexpr int fft_parity_after() {
    return lds_mode(L) ? PAR
                       : (PAR + exchanges_from(L, P, 1) - ((SW && lane_swap_plan(L, P)) ? 1 : 0)) & 1;
}

// Points per thread for a line of L points.  The one-mask passes run one
// work-group of 4 lines per CU or fewer, so more threads per line (smaller
// P) hide more latency, at the cost of more stages: measured on MI355X
// (solve time per iteration), P = 4 (radix 4-4-4 ... with the last stage
// across lanes) is fastest for 64 .. 256 points (64^2: 6.0 -> 5.2 us
// against P = 8; 256^2: 8.5 -> 6.4 us against P = 16), P = 8 for 512
// (8-8-8: 10.1 -> 8.5 us against 16-16-2) and 1024 (8-8-8-2: P = 16 is 8%
// slower, P = 4 12%), P = 16 from 2048 on (P = 8 is within 0.5% at 2048
// and does not fit a 4-line work-group at 4096).
__host__ __device__ constexpr int points_per_thread(int L) {
    return lds_mode(L) ? L / lds_threads(L)
         : L == 800 ? 10
         : L == 600 ? 30
         : L == 1080 ? 30
         : L == 1920 ? 60
         : (L == 512 || L == 1024) ? 8
         : (L >= 64 && L <= 256) ? 4
         : (L >= 2048 ? 16 : (L >= 32 ? 8 : 4));
}

// Rows per work-group of the one-mask row pass for rows of W points.  Rows
// of 128 .. 4096 points (powers of two) take 2-row work-groups, twice as
// many as 4-row ones, paired on XCDs (pass_tile) so that the two
// work-groups reading the two halves of the same 128-byte lines share one
// L2: measured per iteration, 256^2 -1%, 512^2 -4%, 1024^2 -1.4%, 2048^2
// -4.6%, 4096^2 -2.8%, 128^2 even, against 4-row work-groups (without the
// pairing, 2-row work-groups were 9-17% slower: each XCD then fetched whole
// lines for half their bytes).  The mixed-radix lengths keep 4 rows.
#ifndef PM_ROWS_800
#define PM_ROWS_800 4
#endif
#ifndef PM_ROWS_1920
#define PM_ROWS_1920 4
#endif
__host__ __device__ constexpr int row_lines(int W) {
    return W == 800 ? PM_ROWS_800
         : W == 1920 ? PM_ROWS_1920
         : ((W & (W - 1)) == 0 && W >= 128 && W <= 4096) ? 2
                                                           : kGR;
}

// Columns per work-group of the one-mask column pass for columns of H
// points: a whole strip (kC columns), or half a strip with the two halves
// paired on one XCD (pass_tile) as for the rows.  A half strip reads 16
// bytes of each 32-byte strip row, against 64 of each 128-byte line for a
// half row tile; measured per iteration against whole strips: 4096^2 -3%
// (two work-groups per CU instead of one), 128^2 -1.7%, 256^2 -1%, but 512^2
// +4.5%, 1024^2 +6%, 2048^2 +4%, so only 128, 256 and 4096 take half strips.
__host__ __device__ constexpr int col_lines(int H) {
    return (H == 128 || H == 256 || H == 4096 || (H == 1024 && PM_COL_LINES_1024 == 2) ||
            (H == 512 && PM_COL_LINES_512 == 2))
               ? 2
               : kC;
}

// A second, taller row tile for 1920-point rows (0: none).  A 1920-point
// row work-group holds 123 KB of LDS at 4 rows, so one fits on a CU and
// 1080 rows make 270 work-groups: two rounds on 256 CUs, the second nearly
// empty.  Five rows (154 KB, 216 work-groups) run in one round; the plan
// takes them when that is the case (rows_for_plan).
__host__ __device__ constexpr int row_lines_alt(int W) { return W == 1920 ? 5 : 0; }

// Rows per work-group of the one-mask row pass of an H x W plan on a GPU with
// `cus` compute units: the taller tile where it turns two rounds of
// work-groups into one, else row_lines(W).
__host__ __device__ constexpr int rows_for_plan(int H, int W, int cus) {
    return (row_lines_alt(W) != 0 && H % row_lines_alt(W) == 0 && H / row_lines(W) > cus &&
            H / row_lines_alt(W) <= cus)
               ? row_lines_alt(W)
               : row_lines(W);
}

}  // namespace pm
