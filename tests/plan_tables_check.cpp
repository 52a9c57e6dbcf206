// Host-side consistency check of the transform plans (compiled and run by
// tests/test_plan_tables_cpu.py; no GPU needed).  Every line plan the
// library can build -- one-mask lengths with points_per_thread, batched
// lengths with batch_points of every schedule -- is walked stage by stage:
//   * the stage radices multiply to the line length;
//   * the staged twiddle table blocks tile [0, twiddle_entries) exactly, and
//     every entry's exponent q k L / (NS R) lies in [0, L);
//   * the batched table offsets add up schedule by schedule;
// the cross-lane and row-tile choices are checked on known plans, the
// row-pass work-group to tile map on a range of grid sizes, the padded LDS
// index of every length, and the one-mask kernels' static LDS.  The twiddle
// tables the library builds (pm_plan.h) are compared with the definition
// exp(-2 pi i q k / (NS R)) entry by entry; tests/test_plan_tables_cpu.py
// also runs this check built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code.
// Prints "ok" and exits 0, or prints the first violation and exits 1.
#include <cstdio>
#include <vector>

#include <cmath>

#include "pm_common.h"
#include "pm_fft.hpp"
#include "pm_kernels.hpp"
#include "pm_plan.h"

namespace {

int failures = 0;

void check(bool ok, const char* what, int a = 0, int b = 0, int c = 0) {
    if (!ok && failures++ == 0) std::printf("violation: %s (%d, %d, %d)\n", what, a, b, c);
}

void walk(int L, int P) {
    long prod = 1;
    int next_block = 0;
    for (int ns = 1; ns < L; ns *= pm::line_stage_radix(L, P, ns)) {
        const int R = pm::line_stage_radix(L, P, ns);
        check(R >= 2 && L % (ns * R) == 0, "stage radix divides the remaining length", L, P, ns);
        if (R < 2) return;
        prod *= R;
        if (!pm::lds_mode(L)) check(P % R == 0, "register-scheme radix divides P", L, P, R);
        if (ns > 1) {
            check(pm::twiddle_block(L, P, ns) == next_block, "twiddle blocks are contiguous", L, P, ns);
            next_block += (R - 1) * ns;
            for (int q = 1; q < R; ++q)
                for (int k = 0; k < ns; ++k) {
                    const long e = (long)q * k * (L / (ns * R));
                    check(e >= 0 && e < L, "twiddle exponent in range", L, q, k);
                }
        }
    }
    check(prod == L, "radices multiply to L", L, P, (int)prod);
    check(pm::twiddle_entries(L, P) == next_block, "twiddle_entries is the last block end", L, P, next_block);
    check(pm::twiddle_entries(L, P) < L, "staged table shorter than L", L, P);
}

// LDS layout of a line: the padded index maps [0, L) one to one into the
// line's lds_line_len slots.
void lds_line(int L) {
    const int LP = pm::lds_line_len(L);
    std::vector<int> hit(LP, 0);
    for (int i = 0; i < L; ++i) {
        const int a = pm::lds_pad(L, i);
        check(a >= 0 && a < LP, "padded LDS index inside the line", L, i, a);
        if (a >= 0 && a < LP) check(++hit[a] == 1, "padded LDS index one to one", L, i, a);
    }
}

// The one-mask passes' layouts (row_lds_layout, col_lds_layout; schemes 4
// and 5 swizzle each line with a per-line key): one to one into the line,
// 16-byte pairs kept together, for every key a pass can use (0, 2, 4, 6).
void pass_lds_line(int L, int lay) {
    const int LP = pm::lds_line_len_lay(L, lay);
    const int keys[] = {0, 2, 4, 6};
    for (int key : keys) {
        if (key != 0 && lay / 64 < 4) continue;
        std::vector<int> hit(LP, 0);
        for (int i = 0; i < L; ++i) {
            const int a = pm::lds_index(lay, i, key);
            check(a >= 0 && a < LP, "pass LDS index inside the line", L, i, a);
            if (a >= 0 && a < LP) check(++hit[a] == 1, "pass LDS index one to one", L, i, a);
            if ((i & 1) == 0) check(pm::lds_index(lay, i + 1, key) == a + 1, "16-byte pairs kept together", L, i);
        }
    }
}

// The library's staged table of (L, P) against its definition, entry by
// entry (float rounding of the double value), and every entry on the unit
// circle.
void twiddle_values(int L, int P) {
    const std::vector<float2> t = pm::staged_twiddles(L, P);
    check((int)t.size() == std::max(1, pm::twiddle_entries(L, P)), "table size", L, P);
    const double two_pi = 6.283185307179586476925286766559;
    for (int ns = 1; ns < L; ns *= pm::line_stage_radix(L, P, ns)) {
        const int R = pm::line_stage_radix(L, P, ns);
        if (ns == 1) continue;
        for (int q = 1; q < R; ++q)
            for (int k = 0; k < ns; ++k) {
                const float2 w = t[pm::twiddle_block(L, P, ns) + (q - 1) * ns + k];
                const double a = two_pi * q * k / ((double)ns * R);
                check(std::fabs(w.x - std::cos(a)) <= 1e-7 && std::fabs(w.y + std::sin(a)) <= 1e-7,
                      "twiddle entry is exp(-2 pi i q k / (NS R))", L, q, k);
            }
    }
}

// Static LDS of the one-mask pass kernels (exchange buffers and FP64
// reduction slots) within the 160 KiB of a CU.
template <int L>
void lds_budget() {
    constexpr int T = pm::LineShape<L>::T;
    constexpr int budget = 160 * 1024;
    constexpr int gc = pm::col_lines(L), gr = pm::row_lines(L);
    check(pm::LdsPlan<L, gc, 2, pm::col_lds_layout(L)>::FLOATS2 * 8 + pm::red_slots(gc * T) * 8 <= budget,
          "column pass LDS", L, gc);
    check(pm::LdsPlan<L, gr, 2, pm::row_lds_layout(L)>::FLOATS2 * 8 + pm::red_slots(gr * T) * 8 <= budget,
          "row pass LDS", L, gr);
    if constexpr (pm::row_lines_alt(L) != 0) {
        constexpr int ga = pm::row_lines_alt(L);
        check(pm::LdsPlan<L, ga>::FLOATS2 * 8 + pm::red_slots(ga * T) * 8 <= budget, "taller row tile LDS", L, ga);
    }
}

}  // namespace

int main() {
    const int lengths[] = {16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 600, 800, 1080, 1920};
    for (int L : lengths) {
        twiddle_values(L, pm::points_per_thread(L));
        walk(L, pm::points_per_thread(L));
        check(L % pm::points_per_thread(L) == 0, "P divides L", L);
    }
    int off = 0;
    for (int s = 0; s < pm::kBatchSchedules; ++s) {
        for (int L = pm::kBatchMinLen; L <= pm::kBatchMaxLen; L *= 2) {
            walk(L, pm::batch_points(s, L));
            check(pm::batch_twiddle_offset(s, L) == off, "batched table offsets add up", s, L, off);
            off += pm::twiddle_entries(L, pm::batch_points(s, L));
        }
    }
    check(pm::batch_twiddle_offset(pm::kBatchSchedules, 0) == off, "batched table total", off);
    {
        const std::vector<float2> bt = pm::batch_twiddles();
        check((int)bt.size() == off, "batched table size", (int)bt.size(), off);
        for (int s = 0; s < pm::kBatchSchedules; ++s)
            for (int L = pm::kBatchMinLen; L <= pm::kBatchMaxLen; L *= 2) {
                const std::vector<float2> t = pm::staged_twiddles(L, pm::batch_points(s, L));
                for (int i = 0; i < pm::twiddle_entries(L, pm::batch_points(s, L)); ++i) {
                    const float2 a = bt[pm::batch_twiddle_offset(s, L) + i];
                    check(a.x == t[i].x && a.y == t[i].y, "batched table holds each plan's table", s, L, i);
                }
            }
    }
    // cross-lane last stages: radix 2 after radix P, radix 4 after radix P
    check(pm::lane_group(1024, 8) == 2, "8-8-8-2 takes its radix-2 stage across lanes");
    check(pm::lane_group(512, 8) == 0, "8-8-8 has no last stage across lanes");
    check(pm::lane_group(512, 16) == 2, "16-16-2 takes its radix-2 stage across lanes");
    check(pm::lane_group(1024, 16) == 4, "16-16-4 takes its radix-4 stage across lanes");
    check(pm::lane_group(256, 4) == 4 && pm::lane_group(64, 4) == 4, "4-4-4(-4) across lanes");
    check(pm::lane_group(128, 4) == 2, "4-4-4-2 across lanes");
    check(pm::lane_group(4096, 16) == 0 && pm::lane_group(2048, 16) == 0, "16-16-16 and 16-16-8 stay in LDS");
    check(pm::lane_group(800, 10) == 0 && pm::lane_group(1920, pm::points_per_thread(1920)) == 0,
          "mixed-radix plans stay in LDS");
    // row tiles: five 1920-point rows per work-group only where that makes one round
    check(pm::rows_for_plan(1080, 1920, 256) == 5, "1080 rows of 1920 take 5-row tiles on 256 CUs");
    check(pm::rows_for_plan(1920, 1920, 256) == 4, "1920 rows of 1920 keep 4-row tiles");
    check(pm::rows_for_plan(600, 1920, 256) == 4, "600 rows of 1920 fit one round with 4-row tiles");
    check(pm::rows_for_plan(1080, 1920, 304) == 4, "270 tiles fit 304 CUs");
    check(pm::rows_for_plan(1080, 1024, 256) == pm::row_lines(1024), "only 1920-point rows have a taller tile");
    // 2-row tiles: the work-group -> tile map is a bijection, and the two
    // halves of every whole group of 16 work-groups sit on one XCD (wg mod 8)
    for (int nwg : {1, 8, 16, 30, 128, 150, 256, 300, 512, 540, 1024, 2048}) {
        std::vector<int> seen(nwg, 0), where(nwg, -1);
        for (int wg = 0; wg < nwg; ++wg) {
            const int t = pm::pass_tile<2>(wg, nwg);
            check(t >= 0 && t < nwg, "row tile in range", nwg, wg, t);
            if (t < 0 || t >= nwg) continue;
            ++seen[t];
            where[t] = wg;
        }
        for (int t = 0; t < nwg; ++t) check(seen[t] == 1, "row tiles are a bijection", nwg, t);
        for (int g = 0; 2 * g + 1 < (nwg & ~15); ++g)
            check(where[2 * g] % 8 == where[2 * g + 1] % 8, "row tile halves share an XCD", nwg, g);
        check(pm::pass_tile<4>(7, nwg) == 7, "4-row tiles keep their index", nwg);
        // 3-row tiles: a bijection, and the four tiles of every 12 rows of a
        // whole group of 32 work-groups sit on one XCD
        std::vector<int> seen3(nwg, 0), where3(nwg, -1);
        for (int wg = 0; wg < nwg; ++wg) {
            const int t = pm::pass_tile<3>(wg, nwg);
            check(t >= 0 && t < nwg, "3-row tile in range", nwg, wg, t);
            if (t < 0 || t >= nwg) continue;
            ++seen3[t];
            where3[t] = wg;
        }
        for (int t = 0; t < nwg; ++t) check(seen3[t] == 1, "3-row tiles are a bijection", nwg, t);
        for (int g = 0; 4 * g + 3 < (nwg & ~31); ++g)
            for (int r = 1; r < 4; ++r)
                check(where3[4 * g] % 8 == where3[4 * g + r] % 8, "3-row tile groups share an XCD", nwg, g);
    }
    check(pm::col_lines(1024) == pm::kC && pm::col_lines(4096) == 2 && pm::col_lines(600) == pm::kC,
          "column tile widths");
    for (int H : {128, 256, 4096})
        check(pm::col_lines(H) != 2 || pm::col_lanes_ok(H, pm::points_per_thread(H), 2) ==
                                           pm::lane_swap_plan(H, pm::points_per_thread(H)),
              "half-strip column tiles keep the cross-lane stage", H);
    check(pm::row_lines(1024) == 2 && pm::row_lines(4096) == 2 && pm::row_lines(64) == 4 &&
              pm::row_lines(1920) == 4 && pm::row_lines(600) == 4 && pm::row_lines(1080) == 4,
          "row tile heights");
    // the loss column pass's strip map: a bijection, contiguous strips per XCD
    for (int nx : {4, 16, 128, 150, 256, 1024}) {
        std::vector<int> hit(nx, 0);
        for (int x = 0; x < nx; ++x) {
            const int s = pm::xcd_strip(x, nx);
            check(s >= 0 && s < nx, "strip map in range", nx, x, s);
            if (s >= 0 && s < nx) check(++hit[s] == 1, "strip map one to one", nx, x, s);
            if (nx % 8 == 0) check(s / (nx / 8) == x % 8, "XCD x % 8 takes a contiguous run of strips", nx, x);
        }
    }
    for (int L : lengths) {
        lds_line(L);
        pass_lds_line(L, pm::row_lds_layout(L));
        pass_lds_line(L, pm::col_lds_layout(L));
        if (L == 1024) pass_lds_line(L, 5 * 64 + 4);  // the column swizzle the build knob selects
    }
    lds_budget<16>(); lds_budget<32>(); lds_budget<64>(); lds_budget<128>(); lds_budget<256>();
    lds_budget<512>(); lds_budget<1024>(); lds_budget<2048>(); lds_budget<4096>();
    lds_budget<600>(); lds_budget<800>(); lds_budget<1080>(); lds_budget<1920>();
    if (failures == 0) std::printf("ok\n");
    return failures == 0 ? 0 : 1;
}
