// Per-work-group timelines of the one-mask row and column passes, for
// profiling builds only (PM_TIMELINE defined; `python -m
// paper_1302_0120_amd.build --timeline` writes libphasemask_timeline.so).
//
// The first thread of every work-group records the device wall clock
// (wall_clock64, a constant-rate counter common to all XCDs) at five points
// of the pass body: entry, its loads arrived, before its stores, its stores
// acknowledged, and the end; with the HW_ID and XCC_ID hardware registers
// and the launch's sequence number.  Waiting for the loads and for the store
// acknowledgements is forced (s_waitcnt vmcnt(0)), which slows a solve by
// about a fifth, so the phases are upper bounds.  Each translation unit (one
// per transform length) keeps the last kTlLaunches launches of each pass
// type, for work-groups 0 .. kTlWg - 1 of the first batch entry.
// In ordinary builds every macro below is empty.
#pragma once

#ifdef PM_TIMELINE
namespace pm {
constexpr int kTlLaunches = 32;
constexpr int kTlWg = 1024;
constexpr int kTlFields = 8;
// tl_buf[pass][launch % kTlLaunches][work-group] = {t_entry, t_loaded,
// t_compute_done, t_stored, t_end, HW_ID, XCC_ID, launch}; pass 0 = column,
// 1 = row.  tl_cnt[pass][work-group] counts the work-group's launches (one
// writer per element: work-group blockIdx.x of consecutive launches).
static __device__ unsigned long long tl_buf[2][kTlLaunches][kTlWg][kTlFields];
static __device__ unsigned tl_cnt[2][kTlWg];
}  // namespace pm
#define PM_TL_DECL unsigned long long tl_t[5] = {0, 0, 0, 0, 0};
#define PM_TL_STAMP(i)                              \
    do {                                            \
        if (threadIdx.x == 0) tl_t[i] = wall_clock64(); \
    } while (0)
#define PM_TL_WAIT() asm volatile("s_waitcnt vmcnt(0)" ::: "memory")
#define PM_TL_COMMIT(pass)                                                                  \
    do {                                                                                    \
        if (threadIdx.x == 0 && blockIdx.x < (unsigned)::pm::kTlWg && blockIdx.y == 0) {     \
            tl_t[4] = wall_clock64();                                                       \
            const unsigned seq = ::pm::tl_cnt[pass][blockIdx.x];                            \
            ::pm::tl_cnt[pass][blockIdx.x] = seq + 1;                                       \
            unsigned long long* r = ::pm::tl_buf[pass][seq % ::pm::kTlLaunches][blockIdx.x]; \
            for (int q = 0; q < 5; ++q) r[q] = tl_t[q];                                     \
            r[5] = (unsigned)__builtin_amdgcn_s_getreg(0xF804); /* HW_ID, 32 bits */        \
            r[6] = (unsigned)__builtin_amdgcn_s_getreg(0xF814); /* XCC_ID, 32 bits */       \
            r[7] = seq;                                                                     \
        }                                                                                   \
    } while (0)
#else
#define PM_TL_DECL
#define PM_TL_STAMP(i) \
    do {               \
    } while (0)
#define PM_TL_WAIT() \
    do {             \
    } while (0)
#define PM_TL_COMMIT(pass) \
    do {                   \
    } while (0)
#endif
