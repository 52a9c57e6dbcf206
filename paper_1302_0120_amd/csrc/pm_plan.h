// pm_plan.h -- host-side plan tables (no device calls): the staged twiddle
// tables the FFT passes read, built in double precision and rounded once.
// Shared by the library's plan set-up and the host consistency check.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

#include "pm_common.h"
#include "pm_fft.hpp"

namespace pm {

// Staged twiddle table of the line plan (L, P) (layout: twiddle_block in
// pm_fft.hpp): entry (q - 1) NS + k of the stage at NS with radix R is
// exp(-2 pi i q k / (NS R)) = exp(-2 pi i e / L) with e = q k L / (NS R) < L,
// evaluated in double and rounded once to float.  At least one entry, so a
// plan without inter-stage twiddles still has a table to point at.
inline std::vector<float2> staged_twiddles(int L, int P) {
    std::vector<float2> t(std::max(1, twiddle_entries(L, P)), make_float2(1.0f, 0.0f));
    const double two_pi = 6.283185307179586476925286766559;
    for (int ns = 1; ns < L; ns *= line_stage_radix(L, P, ns)) {
        const int R = line_stage_radix(L, P, ns);
        if (ns == 1) continue;
        const int base = twiddle_block(L, P, ns);
        for (int q = 1; q < R; ++q) {
            for (int k = 0; k < ns; ++k) {
                const int e = q * k * (L / (ns * R));
                const double a = two_pi * (double)e / (double)L;
                t[(size_t)(base + (q - 1) * ns + k)] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
            }
        }
    }
    return t;
}

// The batched plans' tables: every schedule and power-of-two length in one
// buffer, at batch_twiddle_offset(schedule, length).
inline std::vector<float2> batch_twiddles() {
    std::vector<float2> tw((size_t)batch_twiddle_offset(kBatchSchedules, 0));
    for (int sc = 0; sc < kBatchSchedules; ++sc) {
        for (int l = kBatchMinLen; l <= kBatchMaxLen; l *= 2) {
            const std::vector<float2> t = staged_twiddles(l, batch_points(sc, l));
            const int n = twiddle_entries(l, batch_points(sc, l));
            std::copy(t.begin(), t.begin() + n, tw.begin() + batch_twiddle_offset(sc, l));
        }
    }
    return tw;
}

}  // namespace pm
