// pm_kernels.hpp -- the fused row and column passes of one Gerchberg-Saxton
// iteration (Eq. 6), templated on the transform length and on the number of
// lines a work-group owns.
//
// One iteration = two passes over the iterate:
//   column pass:  forward column FFT -> M-hat of Eq. 5 (keep the phase of
//                 each Fourier coefficient, take the target modulus) ->
//                 inverse column FFT, plus the FP64 Fourier-error partials;
//   row pass:     inverse row FFT (completes P_M, Eq. 4b) -> P_S of Eq. 4a
//                 (unit modulus) -> forward row FFT of the next iteration,
//                 plus the FP64 gap partials.
// The very first row pass forms exp(i phi0) instead (u^0 in S, Eq. 1); the
// last one writes the phase of u^n.
//
// The bodies (col_body, row_body) serve both the one-mask kernels below and
// the batched kernels, which pick the body per work-group from the size of
// the mask it works on.
#pragma once
#include <float.h>

#include "pm_common.h"
#include "pm_fft.hpp"
#include "pm_trace.h"

namespace pm {

// Deterministic work-group sum of one double per thread: a fixed xor
// butterfly inside each reduction group, then group results added in group
// order by thread 0.  The result is valid in thread 0 only.  All threads
// must call; `red` holds red_slots(NT) doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    constexpr int WS = red_width(NT);
    constexpr int NW = red_slots(NT);
#pragma unroll
    for (int off = WS / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WS);
    if constexpr (NW == 1) {
        return v;
    } else {
        if (threadIdx.x % WS == 0) red[threadIdx.x / WS] = v;
        __syncthreads();
        double s = 0.0;
        if (threadIdx.x == 0) {
#pragma unroll
            for (int w = 0; w < NW; ++w) s += red[w];
        }
        return s;
    }
}

#ifndef PM_DPP_SUM
#define PM_DPP_SUM 1
#endif
// A double moved between lanes by the DPP pattern CTRL (within rows of 16
// lanes, every source lane valid).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// One FP64 partial per reduction group (see red_width), in a fixed order,
// written by the group's first lane to slot[group].  No barrier; all threads
// must call.  Groups of 16, 32 or 64 lanes (aligned rows of 16 lanes, all
// active, since the work-group size is a multiple of the group size): four
// DPP steps inside each row (pairs, quads, eights, sixteens: every lane then
// holds its row's sum), then rows added from lane reads -- (row 0 + row 1)
// + (row 2 + row 3) for 64, row 0 + row 1 and row 2 + row 3 for 32.  These
// stay in the vector unit, where a cross-lane shuffle goes through the LDS
// crossbar once per step (still used for smaller groups).
template <int NT>
__device__ __forceinline__ void group_sum_store(double v, double* slot) {
    constexpr int WS = red_width(NT);
    if constexpr (WS >= 16 && PM_DPP_SUM) {
        v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]: lane ^ 1
        v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]: lane ^ 2
        v += dpp_f64<0x141>(v);  // row_half_mirror: lane i <-> 7 - i in each 8
        v += dpp_f64<0x140>(v);  // row_mirror: lane i <-> 15 - i in each 16
        if constexpr (WS == 64) {
            const double s = (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
            if (threadIdx.x % 64 == 0) slot[threadIdx.x / 64] = s;
        } else if constexpr (WS == 32) {
            const double s0 = readlane_f64(v, 0) + readlane_f64(v, 16);
            const double s1 = readlane_f64(v, 32) + readlane_f64(v, 48);
            if (threadIdx.x % 32 == 0) slot[threadIdx.x / 32] = (threadIdx.x % 64 == 0) ? s0 : s1;
        } else {
            if (threadIdx.x % 16 == 0) slot[threadIdx.x / 16] = v;
        }
    } else {
#pragma unroll
        for (int off = WS / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WS);
        if (threadIdx.x % WS == 0) slot[threadIdx.x / WS] = v;
    }
}

// The same for a maximum (stored as a double).
template <int NT>
__device__ __forceinline__ void group_max_store(float v, double* slot) {
    constexpr int WS = red_width(NT);
#pragma unroll
    for (int off = WS / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, WS));
    if (threadIdx.x % WS == 0) slot[threadIdx.x / WS] = (double)v;
}

// Store of one iterate element that the next pass reads on other XCDs: a
// relaxed device-scope store writes through this XCD's L2, so the data is in
// the shared Infinity Cache when the kernel ends instead of waiting for the
// end-of-kernel L2 write-back (about 1.5 us per pass at 1024 x 1024).
__device__ __forceinline__ void store_shared(float2* p, float2 v) {
    const unsigned long long bits =
        ((unsigned long long)__float_as_uint(v.y) << 32) | (unsigned long long)__float_as_uint(v.x);
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), bits, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Work-group maximum of one float per thread, returned to every thread.
// Max is exact, so the order does not matter.  All threads must call;
// `redf` holds red_slots(NT) floats.
template <int NT>
__device__ __forceinline__ float block_max(float v, float* redf) {
    constexpr int WS = red_width(NT);
    constexpr int NW = red_slots(NT);
#pragma unroll
    for (int off = WS / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, WS));
    if constexpr (NW > 1) {
        if (threadIdx.x % WS == 0) redf[threadIdx.x / WS] = v;
        __syncthreads();
        v = redf[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) v = fmaxf(v, redf[w]);
        __syncthreads();
    }
    return v;
}

// Whether row tiles of G rows can take the cross-lane last stage of (W, P):
// a lane group must hold whole rows of whole strips (lane_group times G
// divides 16).
__host__ __device__ constexpr bool row_lanes_ok(int W, int P, int G) {
    return lane_swap_plan(W, P) && 16 % (lane_group(W, P) * G) == 0;
}

// The same for column tiles of G columns: whole strips, or half a strip with
// a lane group of 32 / Q rows per column (T a multiple of 32).
__host__ __device__ constexpr bool col_lanes_ok(int H, int P, int G) {
    return lane_swap_plan(H, P) && (G % kC == 0 || (G == 2 && (H / P) % 32 == 0));
}

// Tile (of G rows, or of G columns) that pass work-group `wg` of `nwg` works
// on.  Work-groups are dealt to the 8 XCDs of the GPU in turn (wg mod 8), so
// with 2-line tiles the two halves 2g and 2g + 1 of a 4-row group (a strip)
// are given to work-groups wg and wg + 8 (same XCD): the lines one half
// loads are then in that XCD's L2 for the other.  Work-groups past the last
// multiple of 16 keep their own index, so the map is a bijection of
// [0, nwg) for any nwg; other tile sizes use the identity.
// With 3-row tiles, four consecutive tiles (12 rows: three whole 128-byte
// rows of every strip) go to work-groups wg, wg + 8, wg + 16, wg + 24.
#ifndef PM_TILE3_XCD
#define PM_TILE3_XCD 1
#endif
template <int G>
__host__ __device__ __forceinline__ int pass_tile(int wg, int nwg) {
    if constexpr (G == 2) {
        if (wg < (nwg & ~15)) return 2 * ((wg / 16) * 8 + (wg & 7)) + ((wg / 8) & 1);
    }
    if constexpr (G == 3 && PM_TILE3_XCD) {
        if (wg < (nwg & ~31)) return 4 * ((wg / 32) * 8 + (wg & 7)) + ((wg / 8) & 3);
    }
    return wg;
}

template <int L, int PP = points_per_thread(L)>
struct LineShape {
    static constexpr int P = PP;                    // points per thread (radix schedule)
    static constexpr int T = L / P;                 // threads per line
};

// Column pass over G columns: G / kC adjacent strips starting at strip
// `first` (G a multiple of kC), or (G = 2) half `first` mod 2 of strip
// `first` / 2.  Thread tid = (sl, j, c), c fastest: strip strip0 + sl,
// column c of that strip, rows j + T t.  For a fixed t a wave's loads are
// 64 / kC consecutive rows of one strip (one contiguous run), or with half
// strips 32 rows of its two columns.
// `lds` holds LdsPlan<H, G, NBMAX>::FLOATS2 elements, `red` red_slots(G T) doubles;
// the FP64 partials go to part_slot[0 .. red_slots(G T)); a.tw is the staged
// twiddle table of (H, P).  SW (one strip, G = kC): with Q = lane_group(H, P),
// lanes i + 64 k / Q (k < Q) of a wave hold rows j + k T / Q of one column,
// 16 / Q rows per lane group and column, so the plan runs its last FFT stage
// across lanes.
template <int H, int P, int G, int MODE, bool SW = false, int NBMAX = 2, int LAY = lds_layout(H)>
__device__ __forceinline__ void col_body(const ColParams& a, int first, double* part_slot,
                                         float2* lds, double* red) {
    constexpr int T = LineShape<H, P>::T;
    constexpr int NT = G * T;
    using LD = LdsPlan<H, G, NBMAX, LAY>;
    constexpr int LP = LD::LP;
    static_assert(G % kC == 0 || G == 2, "whole strips, or half a strip, per work-group");
    PM_TL_DECL
    PM_TL_STAMP(0);

    const int tid = threadIdx.x;
    constexpr bool HALF = G < kC;
    const int strip0 = HALF ? first >> 1 : first;
    const int c0 = HALF ? (first & 1) * 2 : 0;  // first column of the tile in its strip
    int c, j, sl;
    if constexpr (SW) {
        constexpr int Q = lane_group(H, P);
        const int lane = tid & 63;
        if constexpr (HALF) {
            static_assert(Q != 0 && T % 32 == 0, "half strips: whole lane groups");
            c = c0 + (lane & 1);
            j = (tid >> 6) * (32 / Q) + ((lane >> 1) % (32 / Q)) + (lane / (64 / Q)) * (T / Q);
            sl = 0;
        } else {
            static_assert(Q != 0 && G == kC && kC == 4 && T % 16 == 0, "one strip, whole lane groups");
            c = lane & 3;
            j = (tid >> 6) * (16 / Q) + ((lane >> 2) % (16 / Q)) + (lane / (64 / Q)) * (T / Q);
            sl = 0;
        }
    } else if constexpr (HALF) {
        c = c0 + (tid & 1);
        j = (tid >> 1) % T;
        sl = 0;
    } else {
        c = tid & (kC - 1);
        j = (tid / kC) % T;
        sl = tid / (kC * T);
    }
    // Element (row j + T t, column c) of strip strip0 + sl: a uniform base
    // per t plus a per-thread 32-bit offset, in the strip-tiled layout and in
    // the natural row-major layout.
    const unsigned toff = (unsigned)((sl * H + j) * kC + c);
    const unsigned noff = (unsigned)(j * a.W + sl * kC + c);
    auto tiled = [&](auto* base, int t) {
        return elem_ptr(base + ((size_t)strip0 * H * kC + (size_t)T * t * kC), toff);
    };
    auto natural = [&](auto* base, int t) {
        return elem_ptr(base + ((size_t)T * t * a.W + (size_t)strip0 * kC), noff);
    };
    LineTwiddles<H, P> tw;
    load_twiddles(tw, j, a.tw);
    float mt[P];
    if constexpr ((MODE & (C_PROJ | C_ERR)) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) mt[t] = *tiled(a.mhat, t);
    }
    float2 v[P];
    if constexpr ((MODE & C_BIT) != 0) {
        // 1-bit pattern: lit where m^2 / max(m^2) > t_dark, both in IEEE double
        // (a correctly rounded division, as in any double evaluation of it).
        float mx = 0.0f;
        for (int i = tid; i < a.ntmax; i += NT) mx = fmaxf(mx, a.tmax_part[i]);
        mx = block_max<NT>(mx, reinterpret_cast<float*>(red));
        const double mx2 = (double)mx * (double)mx;
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const double m = (double)*natural(a.tnat, t);
            v[t] = make_float2((m * m) / mx2 > a.t_dark ? 1.0f : 0.0f, 0.0f);
        }
    } else if constexpr ((MODE & CIN_NAT) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) v[t] = *natural(a.nat_in, t);
    } else {
#pragma unroll
        for (int t = 0; t < P; ++t) v[t] = *tiled(a.X, t);
    }
    PM_TL_WAIT();
    PM_TL_STAMP(1);
    float2* line = lds + (sl * kC + c - c0) * LP;
    // Layout scheme 5 (whole strips, lines 4 mod 16 elements apart) needs no
    // per-column key: the swizzle alone puts the four columns' accesses of a
    // wave on disjoint banks in each exchange.  Scheme 4 (half strips, lines
    // 8 mod 16 apart) flips bit 1 of the second column's indices, as for the
    // second row of a two-row tile.
    const int key = (LAY / 64 == 4 && c != c0) ? 2 : 0;
    static_assert(LAY / 64 != 5 || (G == kC && LP % 16 == 4), "swizzled columns: whole strips, lines 4 mod 16 apart");
    static_assert(LAY / 64 != 4 || (G == 2 && LP % 16 == 8), "swizzled half strips: lines 8 mod 16 apart");

    constexpr int PAR1 = (MODE & C_FWD) != 0 ? fft_parity_after<H, P, 0, SW>() : 0;
    if constexpr ((MODE & C_FWD) != 0)
        fft_line<H, P, false, LD::NBUF, 0, SW, LAY>(v, j, line, LD::STRIDE, tw, key);

    // Per-thread partial of this pass's FP64 sum (Fourier error or loss);
    // reduced at the very end, after the stores, into one partial per
    // reduction group (part_slot[0 .. red_slots(NT))).
    double acc = 0.0;
    float mx = 0.0f;  // C_POW: per-thread maximum

    if constexpr ((MODE & (C_PROJ | C_ERR)) != 0) {
        // U = unnormalised DFT of u, so |U|/N is the unitary modulus over
        // sqrt(N); mhat = m / ||m||.  E_F^2 = sum (|U|/N - mhat)^2.
        constexpr bool ERR = (MODE & C_NOERR) == 0;
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const float m = mt[t];
            const float2 U = v[t];
            const float a2 = fmaf(U.x, U.x, U.y * U.y);
            // |U|^2 >= FLT_MIN excludes denormals, so the raw hardware
            // reciprocal square root applies; below it the tie-break of
            // Eq. 5 takes phase 0 and |U| counts as 0.
            const bool nz = a2 >= FLT_MIN;
            const float r = nz ? __builtin_amdgcn_rsqf(a2) : 0.0f;
            if constexpr (ERR) {
                const double d = fma((double)(a2 * r), a.invN, -(double)m);
                acc = fma(d, d, acc);
            }
            if constexpr ((MODE & C_PROJ) != 0) {
                const float q = m * r;
                v[t] = nz ? make_float2(U.x * q, U.y * q) : make_float2(m, 0.0f);
            }
        }
    }

    if constexpr ((MODE & C_POW) != 0) {
        // |U_unitary|^2 = |U|^2 / N (for N a power of two, an exact scaling).
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const float q = fmaf(v[t].x, v[t].x, v[t].y * v[t].y) * (float)a.invN;
            *tiled(a.pw, t) = q;
            mx = fmaxf(mx, q);
        }
    }

    if constexpr ((MODE & C_LOSS) != 0) {
        // Intensity loss L = sum_k (|U_k|^2 - I_k)^2 with unitary U: the
        // unnormalised U here gives |U_unitary|^2 = |U|^2 / N (exact scaling).
        // The residual-weighted field r U feeds the adjoint transform; its
        // 1/sqrt(N) factors are folded into the gradient scale.
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const float I = (MODE & C_ITILED) != 0 ? *tiled(a.inten, t) : *natural(a.inten, t);
            const float2 U = v[t];
            const float r = fmaf(fmaf(U.x, U.x, U.y * U.y), (float)a.invN, -I);
            acc = fma((double)r, (double)r, acc);
            v[t] = make_float2(U.x * r, U.y * r);
        }
    }

    if constexpr ((MODE & C_INV) != 0)
        fft_line<H, P, true, LD::NBUF, PAR1, SW, LAY>(v, j, line, LD::STRIDE, tw, key);

    PM_TL_STAMP(2);
    if constexpr ((MODE & COUT_TILED) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) store_shared(tiled(a.X, t), v[t]);
    }
    if constexpr ((MODE & COUT_NAT) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) *natural(a.nat_out, t) = v[t];
    }
    PM_TL_WAIT();
    PM_TL_STAMP(3);

    constexpr bool SUM = ((MODE & (C_PROJ | C_ERR)) != 0 && (MODE & C_NOERR) == 0) || (MODE & C_LOSS) != 0;
    if constexpr (SUM) group_sum_store<NT>(acc, part_slot);
    if constexpr ((MODE & C_POW) != 0) group_max_store<NT>(mx, part_slot);
    PM_TL_COMMIT(0);
}

// Row pass over G adjacent rows starting at `row0`.  Thread tid = (jhi, rho,
// c), c fastest: row row0 + rho, thread index within the row j = jhi kC + c.
// For a fixed t the element (row, j + T t) lies in strip jhi + (T / kC) t at
// column c, so a wave's loads are runs of G kC contiguous elements; a.tw is
// the staged twiddle table of (W, P).  SW (row_lanes_ok): with Q =
// lane_group(W, P), lanes i + 64 k / Q (k < Q) of a wave hold threads
// j + k T / Q of one row (jhi + k T / (4 Q)), 16 / (Q G) strips per lane
// group, so the plan runs its last FFT stage across lanes.
template <int W, int P, int G, int MODE, bool SW = false, int NBMAX = 2, int LAY = lds_layout(W)>
__device__ __forceinline__ void row_body(const RowParams& a, int row0, const float* phase_in,
                                         float* phase_out, double* part_slot, float2* lds,
                                         double* red) {
    constexpr int T = LineShape<W, P>::T;
    constexpr int NT = G * T;
    static_assert(T % kC == 0, "row threads must cover whole strips");
    using LD = LdsPlan<W, G, NBMAX, LAY>;
    constexpr int LP = LD::LP;
    PM_TL_DECL
    PM_TL_STAMP(0);

    const int tid = threadIdx.x;
    int c, rho, jhi;
    if constexpr (SW) {
        constexpr int Q = lane_group(W, P);
        constexpr int JG = 16 / (Q * G);  // strips per lane group
        static_assert(Q != 0 && kC == 4 && T % 16 == 0 && JG >= 1 && JG * Q * G == 16,
                      "whole rows and strips per lane group");
        const int lane = tid & 63;
        c = lane & 3;
        rho = (lane >> 2) % G;
        jhi = (tid >> 6) * JG + ((lane / (4 * G)) % JG) + (lane / (64 / Q)) * (T / (4 * Q));
    } else {
        c = tid & (kC - 1);
        rho = (tid / kC) % G;
        jhi = tid / (kC * G);
    }
    const int j = jhi * kC + c;
    const int H = a.H;
    // Element (row row0 + rho, column j + T t): a uniform base per t plus a
    // per-thread 32-bit offset.  Strip-tiled: strip jhi + (T / kC) t, row,
    // column c; natural: row-major.
    const unsigned toff = (unsigned)((jhi * H + rho) * kC + c);
    const unsigned noff = (unsigned)(rho * W + j);
    auto tiled = [&](auto* base, int t) {
        return elem_ptr(base + ((size_t)row0 * kC + (size_t)T * t * H), toff);
    };
    auto natural = [&](auto* base, int t) { return elem_ptr(base + ((size_t)row0 * W + (size_t)T * t), noff); };
    LineTwiddles<W, P> tw;
    load_twiddles(tw, j, a.tw);
    float2 v[P];
    // Illumination amplitude p of Eq. 1 (S = fields of modulus p): the
    // projections below take modulus p instead of 1.
    constexpr bool ILLUM = (MODE & R_ILLUM) != 0;
    static_assert(!ILLUM || (MODE & ROUT_PHASE) == 0 || (MODE & (R_PS | R_RAAR)) != 0,
                  "with an illumination the phase is written by P_S or the RAAR update");
    float pil[ILLUM ? P : 1];
    if constexpr (ILLUM) {
#pragma unroll
        for (int t = 0; t < P; ++t) pil[t] = *tiled(a.illum, t);
    }

    if constexpr ((MODE & RIN_PHASE) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) {
            float sn, cs;
            sincosf(*natural(phase_in, t), &sn, &cs);
            if constexpr (ILLUM) {
                v[t] = make_float2(pil[t] * cs, pil[t] * sn);
            } else {
                v[t] = make_float2(cs, sn);
            }
        }
    } else if constexpr ((MODE & RIN_NAT) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) v[t] = *natural(a.nat_in, t);
    } else {
#pragma unroll
        for (int t = 0; t < P; ++t) v[t] = *tiled(a.X, t);
    }
    float2 zx[(MODE & R_RAAR) != 0 ? P : 1];
    if constexpr ((MODE & R_RAAR) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) zx[t] = *tiled(a.Z, t);
    }
    if constexpr ((MODE & R_STOREZ) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) *tiled(a.Z, t) = v[t];
    }
    PM_TL_WAIT();
    PM_TL_STAMP(1);
    float2* line = lds + rho * LP;
    // Swizzle key of this row's LDS line (layout scheme 4, two-row tiles:
    // the second row lies 8 mod 16 elements further and flips bit 1 of every
    // index, so in each exchange the two rows' accesses of a wave fall on
    // disjoint banks).
    const int key = (LAY / 64 == 4 && rho != 0) ? 2 : 0;
    static_assert(LAY / 64 != 4 || (G == 2 && LP % 16 == 8), "swizzled rows: two-row tiles, lines 8 mod 16 apart");

    constexpr int PAR1 = (MODE & R_INV) != 0 ? fft_parity_after<W, P, 0, SW>() : 0;
    if constexpr ((MODE & R_INV) != 0)
        fft_line<W, P, true, LD::NBUF, 0, SW, LAY>(v, j, line, LD::STRIDE, tw, key);

    // Per-thread gap partial; reduced at the very end (see col_body).
    double acc = 0.0;

    if constexpr ((MODE & R_PS) != 0) {
        // w = P_M u^nu with unit scale (the target was divided by ||m||, so
        // the unnormalised inverse leaves |w| on the scale of p = 1).
        constexpr bool ERR = (MODE & R_NOERR) == 0;
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const float2 w = v[t];
            const float a2 = fmaf(w.x, w.x, w.y * w.y);
            // Tie-break of Eq. 4a below FLT_MIN (phase 0), as in the column pass.
            const bool nz = a2 >= FLT_MIN;
            const float r = nz ? __builtin_amdgcn_rsqf(a2) : 0.0f;
            const float2 e = nz ? make_float2(w.x * r, w.y * r) : make_float2(1.0f, 0.0f);
            if constexpr (ERR) {
                double p = 1.0;
                if constexpr (ILLUM) p = (double)pil[t];
                const double d = (double)(a2 * r) - p;
                acc = fma(d, d, acc);
            }
            if constexpr (ILLUM) {
                // the phase of the mask is that of e (also where p = 0)
                if constexpr ((MODE & ROUT_PHASE) != 0) *natural(phase_out, t) = atan2f(e.y, e.x);
                v[t] = make_float2(pil[t] * e.x, pil[t] * e.y);
            } else {
                v[t] = e;
            }
        }
    }

    if constexpr ((MODE & R_RAAR) != 0) {
        // RAAR: x+ = beta P_S(2w - x) + beta x + (1 - 2 beta) w with w = P_M x
        // (the unnormalised inverse of the target-scaled M-hat leaves w on the
        // scale of x).  Tie-break of P_S below FLT_MIN as in Eq. 4a.
        const float b = a.beta;
        const float c = 1.0f - 2.0f * b;
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const float2 w = v[t];
            const float2 x = zx[t];
            const float2 y = make_float2(fmaf(2.0f, w.x, -x.x), fmaf(2.0f, w.y, -x.y));
            const float a2 = fmaf(y.x, y.x, y.y * y.y);
            const bool nz = a2 >= FLT_MIN;
            const float r = nz ? __builtin_amdgcn_rsqf(a2) : 0.0f;
            float2 ps = nz ? make_float2(y.x * r, y.y * r) : make_float2(1.0f, 0.0f);
            if constexpr (ILLUM) ps = make_float2(pil[t] * ps.x, pil[t] * ps.y);
            const float2 xn = make_float2(fmaf(c, w.x, fmaf(b, x.x, b * ps.x)), fmaf(c, w.y, fmaf(b, x.y, b * ps.y)));
            if constexpr ((MODE & ROUT_PHASE) != 0) {
                // last pass: the mask is the shadow P_S x^n
                const float q2 = fmaf(xn.x, xn.x, xn.y * xn.y);
                const bool qz = q2 >= FLT_MIN;
                const float qr = qz ? __builtin_amdgcn_rsqf(q2) : 0.0f;
                const float2 e = qz ? make_float2(xn.x * qr, xn.y * qr) : make_float2(1.0f, 0.0f);
                if constexpr (ILLUM) {
                    *natural(phase_out, t) = atan2f(e.y, e.x);
                    v[t] = make_float2(pil[t] * e.x, pil[t] * e.y);
                } else {
                    v[t] = e;
                }
            } else {
                *tiled(a.Z, t) = xn;
                v[t] = xn;
            }
        }
    }

    if constexpr ((MODE & ROUT_PHASE) != 0 && !ILLUM) {
#pragma unroll
        for (int t = 0; t < P; ++t) *natural(phase_out, t) = atan2f(v[t].y, v[t].x);
    }
    if constexpr ((MODE & ROUT_NAT) != 0) {
#pragma unroll
        for (int t = 0; t < P; ++t) *natural(a.nat_out, t) = v[t];
    }
    if constexpr ((MODE & ROUT_GRAD) != 0) {
        // v = unnormalised inverse of r U, i.e. N F^H(r U) up to the scale the
        // column pass left out; dL/dphi = 4 Im(e^{-i phi} F^H(r U)).
#pragma unroll
        for (int t = 0; t < P; ++t) {
            float sn, cs;
            sincosf(*natural(phase_in, t), &sn, &cs);
            *natural(phase_out, t) = a.gscale * fmaf(cs, v[t].y, -(sn * v[t].x));
        }
    }
    if constexpr ((MODE & R_ADAM) != 0) {
        // v = unnormalised inverse of r U, as for ROUT_GRAD: the gradient of
        // the intensity loss is g = 4 Im(e^{-i phi} F^H(r U)) (scale folded
        // into gscale).  Adam (Kingma and Ba, Algorithm 1) on each pixel:
        //   m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
        //   phi <- phi - (lr / (1 - beta1^k)) m / (sqrt(v) / sqrt(1 - beta2^k) + eps),
        // then (R_FWD) exp(i phi) of the new phase feeds the forward row
        // transform of the next step.
        const float omb1 = 1.0f - a.beta1;
        const float omb2 = 1.0f - a.beta2;
#pragma unroll
        for (int t = 0; t < P; ++t) {
            float sn, cs;
            const float ph = *natural(phase_in, t);
            sincosf(ph, &sn, &cs);
            const float g = a.gscale * fmaf(cs, v[t].y, -(sn * v[t].x));
            float* mp = natural(a.am, t);
            float* vp = natural(a.av, t);
            const float m1 = fmaf(a.beta1, *mp, omb1 * g);
            const float v1 = fmaf(a.beta2, *vp, omb2 * (g * g));
            const float denom = sqrtf(v1) / a.adam_bc2s + a.eps;
            const float ph1 = ph - (a.adam_step * m1) / denom;
            *mp = m1;
            *vp = v1;
            *natural(phase_out, t) = ph1;
            if constexpr ((MODE & R_FWD) != 0) {
                sincosf(ph1, &sn, &cs);
                v[t] = make_float2(cs, sn);
            }
        }
    }
    if constexpr ((MODE & R_FWD) != 0) {
        fft_line<W, P, false, LD::NBUF, PAR1, SW, LAY>(v, j, line, LD::STRIDE, tw, key);
        PM_TL_STAMP(2);
#pragma unroll
        for (int t = 0; t < P; ++t) store_shared(tiled(a.X, t), v[t]);
        PM_TL_WAIT();
        PM_TL_STAMP(3);
    }
    if constexpr ((MODE & ROUT_TILED) != 0) {
        static_assert((MODE & (R_INV | R_FWD | R_PS | RIN_TILED)) == RIN_TILED, "copy of the iterate only");
#pragma unroll
        for (int t = 0; t < P; ++t) store_shared(tiled(a.X, t), v[t]);
    }
    if constexpr ((MODE & R_PS) != 0 && (MODE & R_NOERR) == 0) group_sum_store<NT>(acc, part_slot);
    PM_TL_COMMIT(1);
}

// One-mask kernels: kC columns (one strip) or G rows per work-group
// (row_lines(W), or row_lines_alt(W) where the plan takes it).
template <int H, int MODE, int G = col_lines(H)>
__global__ void __launch_bounds__(G * LineShape<H>::T)
k_col(ColParams a) {
    constexpr int NT = G * LineShape<H>::T;
    __shared__ __align__(16) float2 lds[LdsPlan<H, G, 2, col_lds_layout(H)>::FLOATS2];
    __shared__ double red[red_slots(NT)];
    if constexpr ((MODE & C_MANY) != 0) {
        // mask blockIdx.y of a uniform batch: its iterate, target, partials
        const size_t mb = (size_t)blockIdx.y * H * a.W;
        a.X += mb;
        a.mhat += mb;
        a.part += blockIdx.y * a.part_bstride;
    }
    col_body<H, LineShape<H>::P, G, MODE, col_lanes_ok(H, LineShape<H>::P, G), 2, col_lds_layout(H)>(
        a, pass_tile<G>(blockIdx.x, gridDim.x), a.part + blockIdx.x * red_slots(NT), lds, red);
}

// Field modes read / write the caller's complex fields through the pointer
// block (so a captured graph serves any buffers) and otherwise run as the
// natural-layout modes.
__host__ __device__ constexpr int field_as_nat(int mode) {
    return (mode & ~(RIN_FIELD | ROUT_FIELD)) | ((mode & RIN_FIELD) != 0 ? RIN_NAT : 0) |
           ((mode & ROUT_FIELD) != 0 ? ROUT_NAT : 0);
}

template <int W, int MODE, int G = row_lines(W)>
__global__ void __launch_bounds__(G * LineShape<W>::T)
k_row(RowParams a) {
    constexpr int NT = G * LineShape<W>::T;
    __shared__ __align__(16) float2 lds[LdsPlan<W, G, 2, row_lds_layout(W)>::FLOATS2];
    __shared__ double red[red_slots(NT)];
    const float* pin = nullptr;
    float* pout = nullptr;
    if constexpr ((MODE & RIN_PHASE) != 0) pin = a.io->phase_in;
    if constexpr ((MODE & ROUT_PHASE) != 0) pout = a.io->phase_out;
    if constexpr ((MODE & RIN_FIELD) != 0) a.nat_in = a.io->field_in;
    if constexpr ((MODE & ROUT_FIELD) != 0) a.nat_out = a.io->field_out;
    if constexpr ((MODE & R_MANY) != 0) {
        // mask blockIdx.y of a uniform batch: its iterate, phases, partials
        // (the illumination p, when set, is the plan's and shared by the masks)
        static_assert((MODE & (R_RAAR | R_STOREZ | RIN_NAT | ROUT_NAT | RIN_FIELD | ROUT_FIELD)) == 0,
                      "uniform batches: the phase-in, phase-out solve modes");
        const size_t mb = (size_t)blockIdx.y * a.H * W;
        a.X += mb;
        if (pin != nullptr) pin += mb;
        if (pout != nullptr) pout += mb;
        a.part += blockIdx.y * a.part_bstride;
    }
    row_body<W, LineShape<W>::P, G, field_as_nat(MODE), row_lanes_ok(W, LineShape<W>::P, G), 2, row_lds_layout(W)>(
        a, pass_tile<G>(blockIdx.x, gridDim.x) * G, pin, pout, a.part + blockIdx.x * red_slots(NT), lds, red);
}

// Intensity-loss kernels over a batch of same-size phases, sample = blockIdx.y.
// Forward: ROW_INIT (exp(i phi), row FFT) then the column kernel (COL_LOSS).
// Backward: ROW_GRAD.  Adam steps: the column kernel (COL_LOSS_T) then
// ROW_ADAM, whose phase input and output are both p.phase / p.grad (the
// caller passes the same buffer: the update is in place).
template <int W, int MODE>
__global__ void __launch_bounds__(row_lines(W) * LineShape<W>::T)
k_row_adj(AdjParams p) {
    constexpr int NT = row_lines(W) * LineShape<W>::T;
    __shared__ __align__(16) float2 lds[LdsPlan<W, row_lines(W), 2, adj_row_lds_layout(W)>::FLOATS2];
    __shared__ double red[red_slots(NT)];
    const size_t n = (size_t)p.H * W;
    const size_t b = blockIdx.y;
    RowParams a{};
    a.X = p.saved + b * n;
    a.tw = p.twW;
    a.H = p.H;
    float* out = nullptr;
    if constexpr ((MODE & ROUT_GRAD) != 0) {
        a.gscale = (float)(4.0 * p.grad_loss[b] / (double)n);
        out = p.grad + b * n;
    }
    if constexpr ((MODE & R_ADAM) != 0) {
        // the gradient of the sample's own loss (unit upstream gradient),
        // the phase updated in place
        a.gscale = (float)(4.0 / (double)n);
        out = p.grad + b * n;
        a.am = p.am + b * n;
        a.av = p.av + b * n;
        a.adam_step = p.adam_step;
        a.adam_bc2s = p.adam_bc2s;
        a.beta1 = p.beta1;
        a.beta2 = p.beta2;
        a.eps = p.eps;
    }
    row_body<W, LineShape<W>::P, row_lines(W), MODE, row_lanes_ok(W, LineShape<W>::P, row_lines(W)), 2,
             adj_row_lds_layout(W)>(a, pass_tile<row_lines(W)>(blockIdx.x, gridDim.x) * row_lines(W), p.phase + b * n,
                                out, nullptr, lds, red);
}

// Strip of loss column work-group x of `nx`: work-groups are dealt to the 8
// XCDs in turn, so with nx a multiple of 8 this gives XCD k the contiguous
// strips [k nx / 8, (k + 1) nx / 8).  The natural-layout intensity is read
// 16 bytes per row per strip; adjacent strips on one XCD then share each
// 128-byte line through that XCD's L2 instead of every XCD fetching whole
// lines for a quarter of their bytes.
__host__ __device__ __forceinline__ int xcd_strip(int x, int nx) {
    return (nx % 8 == 0) ? (x % 8) * (nx / 8) + x / 8 : x;
}

template <int H, int MODE>
__global__ void __launch_bounds__(kC * LineShape<H>::T)
k_col_adj(AdjParams p) {
    constexpr int NT = kC * LineShape<H>::T;
    __shared__ float2 lds[LdsPlan<H, kC>::FLOATS2];
    __shared__ double red[red_slots(NT)];
    const size_t n = (size_t)H * p.W;
    const size_t b = blockIdx.y;
    ColParams a{};
    a.X = p.saved + b * n;
    a.tw = p.twH;
    a.W = p.W;
    a.invN = 1.0 / (double)n;
    a.inten = p.inten + b * n;
    const int strip = xcd_strip(blockIdx.x, gridDim.x);
    col_body<H, LineShape<H>::P, kC, MODE, col_lanes_ok(H, LineShape<H>::P, kC)>(
        a, strip, p.part + (size_t)(p.part_row0 + b) * p.nwg + strip * red_slots(NT), lds, red);
}

}  // namespace pm
