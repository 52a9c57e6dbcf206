// phasemask.cpp -- host side of the C ABI declared in include/phasemask.h:
// plan creation (workspace, FP64-derived twiddle tables), argument checks,
// the launch sequence of one solve, and its capture into a HIP graph.
#include "phasemask.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <list>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "pm_common.h"
#include "pm_fft.hpp"
#include "pm_plan.h"

namespace {

thread_local std::string g_last_error;

pm_status fail(pm_status s, const std::string& why) {
    g_last_error = why;
    return s;
}

pm_status fail_hip(hipError_t e, const char* what) {
    // The runtime also keeps a failed call's error as its last error, which
    // the next launch check (hipGetLastError) would report as its own: the
    // failure is handled here, so clear it.
    (void)hipGetLastError();
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PM_ENOMEM : PM_EDEVICE;
}

bool pow2_in_range(int n) { return n >= 16 && n <= 4096 && (n & (n - 1)) == 0; }

int log2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Slot of a supported one-mask transform length in the launcher tables:
// log2(L) - 4 for the powers of two 16 .. 4096, then 600, 800, 1080 and
// 1920 (the mixed-radix plans); -1 when unsupported.
int len_slot(int n) {
    if (pow2_in_range(n)) return log2i(n) - 4;
    if (n == 600) return 9;
    if (n == 800) return 10;
    if (n == 1080) return 11;
    if (n == 1920) return 12;
    return -1;
}

using AdjRowLauncher = hipError_t (*)(int, const pm::AdjParams&, int, hipStream_t);
using AdjColLauncher = hipError_t (*)(int, const pm::AdjParams&, int, hipStream_t);
const AdjRowLauncher kAdjRow[13] = {pm::launch_adj_row_16,   pm::launch_adj_row_32,   pm::launch_adj_row_64,
                                    pm::launch_adj_row_128,  pm::launch_adj_row_256,  pm::launch_adj_row_512,
                                    pm::launch_adj_row_1024, pm::launch_adj_row_2048, pm::launch_adj_row_4096,
                                    pm::launch_adj_row_600,  pm::launch_adj_row_800,
    pm::launch_adj_row_1080, pm::launch_adj_row_1920};
const AdjColLauncher kAdjCol[13] = {pm::launch_adj_col_16,   pm::launch_adj_col_32,   pm::launch_adj_col_64,
                                    pm::launch_adj_col_128,  pm::launch_adj_col_256,  pm::launch_adj_col_512,
                                    pm::launch_adj_col_1024, pm::launch_adj_col_2048, pm::launch_adj_col_4096,
                                    pm::launch_adj_col_600,  pm::launch_adj_col_800,
    pm::launch_adj_col_1080, pm::launch_adj_col_1920};

using RowLauncher = hipError_t (*)(int, const pm::RowParams&, int, hipStream_t, hipEvent_t, hipEvent_t);
using ColLauncher = hipError_t (*)(int, const pm::ColParams&, int, hipStream_t, hipEvent_t, hipEvent_t);

// Indexed by len_slot(L).
const RowLauncher kRowLaunch[13] = {pm::launch_row_16,   pm::launch_row_32,   pm::launch_row_64,
                                    pm::launch_row_128,  pm::launch_row_256,  pm::launch_row_512,
                                    pm::launch_row_1024, pm::launch_row_2048, pm::launch_row_4096,
                                    pm::launch_row_600,  pm::launch_row_800,
    pm::launch_row_1080, pm::launch_row_1920};
const ColLauncher kColLaunch[13] = {pm::launch_col_16,   pm::launch_col_32,   pm::launch_col_64,
                                    pm::launch_col_128,  pm::launch_col_256,  pm::launch_col_512,
                                    pm::launch_col_1024, pm::launch_col_2048, pm::launch_col_4096,
                                    pm::launch_col_600,  pm::launch_col_800,
    pm::launch_col_1080, pm::launch_col_1920};

// What a captured solve graph was recorded for (its kernel arguments bake
// in the iteration count, the algorithm and its scalars).
struct SolveKey {
    int n_iter = 0;
    bool hist = false;
    int algo = 0;        // kAlgoGS, kAlgoRAAR, kAlgoGSField, kAlgoAdam
    float beta = 0.0f;   // RAAR relaxation
    int batch = 0;       // Adam: samples
    double lr = 0.0, beta1 = 0.0, beta2 = 0.0, eps = 0.0;  // Adam
    int chain = -1;      // Adam: the steps of chain `chain` of `chains` only (-1: the whole solve)
    int chains = 1;
    bool operator==(const SolveKey& o) const {
        return n_iter == o.n_iter && hist == o.hist && algo == o.algo && beta == o.beta && batch == o.batch &&
               lr == o.lr && beta1 == o.beta1 && beta2 == o.beta2 && eps == o.eps && chain == o.chain &&
               chains == o.chains;
    }
};

struct GraphEntry {
    SolveKey key;
    hipGraphExec_t exec;
};

// Work-groups of the target-norm partial pass: each thread then loads one or
// two float4 of an 800 x 600 or 1024^2 target (with 64 work-groups, 8 or 16
// in a row; the pass took 7.8 us at 800 x 600).
constexpr int kNormGrid = 512;
// Default cache budget of one group of masks in a batched solve (the
// working sets of the masks whose iterations run together);
// PHASEMASK_GROUP_MB overrides it, 0 = all masks in one group.  With
// kBatchChains groups in flight at once, 4 x 48 MiB stays inside the 256 MB
// last-level cache of an MI355X.  Measured on the 64-mask workload (385 MB
// of iterates and targets): 18.0 ms per batch, against 22.6 ms for one
// group and 19.6 ms for 224 MiB groups on one chain.
constexpr size_t kBatchGroupBytes = (size_t)48 << 20;
// Default number of concurrent chains the groups are spread over
// (PHASEMASK_CHAINS overrides, 1..8).
constexpr int kBatchChains = 4;
// Concurrent chains of launches in an Adam solve of several samples (one
// group of samples per chain; PHASEMASK_ADAM_CHAINS).  One by default: two
// chains took the 16 x 512^2 solve from 9.3 to 8.4 ms in a process holding
// only the Adam plan, but from 9.7 to 10.9 ms after other plans had run,
// where the two chains' streams shared one of the runtime's four hardware
// queues (with GPU_MAX_HW_QUEUES=8 they gained there too).
constexpr int kAdamChains = 1;
constexpr size_t kMaxCachedGraphs = 8;

// Iterations per schedule the batched tuner times (groups on chains, as a
// solve runs them).
constexpr int kTuneIterations = 6;
// Relative margin by which a later FFT schedule must beat the best earlier one
// to be chosen (the two schedules of the 64-mask workload time within about
// 1% of each other, and without a margin the choice flipped between runs).
constexpr double kTuneMargin = 0.02;

}  // namespace

// A run of masks of a batched plan whose iterations are enqueued together
// (column tasks [c0, c1), row tasks [r0, r1) of the active layout), sized so
// that their iterates and targets stay resident in the last-level cache
// while all iterations run.
struct pm_batch_group {
    int c0, c1, r0, r1;
    size_t bytes;  // working set of the group's masks
    int chain;     // chain of launches the group runs on
};

struct pm_plan {
    int H = 0, W = 0, N = 0;
    unsigned flags = 0;
    int device = 0;
    hipStream_t stream = nullptr;      // caller's stream
    hipStream_t cap_stream = nullptr;  // private stream used only for graph capture
    int rows = 0;                      // rows per row-pass work-group (rows_for_plan)
    int nwg_row = 0, nwg_col = 0, stride = 0;
    int slots_row = 0, slots_col = 0;  // FP64 partials per row / column pass (one per reduction group)
    int slots_adj = 0;                 // per sample of the loss column pass (whole-strip work-groups)
    int num_cu = 0;                    // compute units of the device
    float2* X = nullptr;
    float* mhat = nullptr;
    float2* twW = nullptr;
    float2* twH = nullptr;
    double* part_m = nullptr;
    float* part_mx = nullptr;          // per-work-group maxima of a target
    float* pw = nullptr;               // |U|^2 / N scratch of the physical error, on first use
    float2* Z = nullptr;               // RAAR's SLM-plane point, on first use
    float* illum = nullptr;            // illumination amplitude p, strip-tiled, on first use
    double* pn2 = nullptr;             // ||p||^2 on the device
    bool illum_on = false;             // solves use p (else p = 1)
    int* vflags = nullptr;             // PM_FLAG_VALIDATE: two check words on the device
    double* part = nullptr;
    size_t part_entries = 0;           // capacity of `part` in history entries
    pm::PmIo* io = nullptr;
    size_t ws_bytes = 0;
    // A caller-owned workspace (phasemask_set_workspace) holding X, mhat and
    // the partials; the plan then owns none of the three.
    bool ws_borrowed = false;
    hipEvent_t order_ev = nullptr;     // orders the handle's work across a stream switch
    // Adam solves (phasemask_solve_adam), allocated for adam_cap samples on
    // first use: the transform buffer, working phase, moments (natural
    // layout) and the strip-tiled intensity.
    int adam_cap = 0;
    int adam_chains = 0;               // concurrent chains of an Adam solve (0: not chosen yet)
    float2* a_saved = nullptr;
    float* a_phase = nullptr;
    float* a_m = nullptr;
    float* a_v = nullptr;
    float* a_inten = nullptr;
    // Uniform batches (phasemask_solve_many), allocated on first use for
    // many_cap masks of many_entries history entries each: the iterates,
    // rescaled targets, target-norm partials and FP64 error partials of
    // every mask (mask b's partials many_entries * stride doubles further).
    int many_cap = 0;
    size_t many_entries = 0;
    float2* m_X = nullptr;
    float* m_mhat = nullptr;
    double* m_partm = nullptr;
    double* m_part = nullptr;
    // Device address of the allocation-free solve's scratch array on the
    // plan's device (looked up at create), or null with the lookup's error.
    unsigned char* scratch = nullptr;
    hipError_t scratch_err = hipSuccess;
    std::list<GraphEntry> graphs;      // most recently used first
    bool dead = false;

    // Batched plans (phasemask_create_batched) only.
    bool batched = false;
    int count = 0;
    int n_col_tasks = 0, n_row_tasks = 0, n_prep_tasks = 0;
    void* batch_ws = nullptr;          // iterates and rescaled targets of every mask
    pm::BatchMask* masks = nullptr;
    pm::BatchTask* col_tasks = nullptr;
    pm::BatchTask* row_tasks = nullptr;
    pm::BatchTask* prep_tasks = nullptr;
    int* mask_prep0 = nullptr;
    pm::BatchIo* bio = nullptr;
    float2* tw_batch = nullptr;
    int sched = 0;                     // FFT schedule of the batched passes
    size_t batch_ws_bytes = 0;
    size_t group_bytes = 0;            // cache budget of one group (0 = one group)
    std::vector<pm_batch_group> groups;
    // Groups are spread over `chains` independent chains of launches (the
    // caller's stream plus side streams joined by events), which a graph
    // runs concurrently.
    int chains = 1;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> fork_ev, join_ev;
};

namespace {

void drop_graphs(pm_plan* h) {
    for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

void free_plan(pm_plan* h) {
    drop_graphs(h);
    for (hipStream_t x : h->side) (void)hipStreamDestroy(x);
    for (hipEvent_t x : h->fork_ev) (void)hipEventDestroy(x);
    for (hipEvent_t x : h->join_ev) (void)hipEventDestroy(x);
    (void)hipFree(h->batch_ws);
    (void)hipFree(h->masks);
    (void)hipFree(h->col_tasks);
    (void)hipFree(h->row_tasks);
    (void)hipFree(h->prep_tasks);
    (void)hipFree(h->mask_prep0);
    (void)hipFree(h->bio);
    (void)hipFree(h->tw_batch);
    if (!h->ws_borrowed) {
        (void)hipFree(h->X);
        (void)hipFree(h->mhat);
        (void)hipFree(h->part);
    }
    if (h->order_ev) (void)hipEventDestroy(h->order_ev);
    (void)hipFree(h->twW);
    (void)hipFree(h->twH);
    (void)hipFree(h->part_m);
    (void)hipFree(h->part_mx);
    (void)hipFree(h->pw);
    (void)hipFree(h->Z);
    (void)hipFree(h->illum);
    (void)hipFree(h->a_saved);
    (void)hipFree(h->a_phase);
    (void)hipFree(h->a_m);
    (void)hipFree(h->a_v);
    (void)hipFree(h->a_inten);
    (void)hipFree(h->m_X);
    (void)hipFree(h->m_mhat);
    (void)hipFree(h->m_partm);
    (void)hipFree(h->m_part);
    (void)hipFree(h->pn2);
    (void)hipFree(h->vflags);
    (void)hipFree(h->io);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
}

// Plans returned by phasemask_create / _create_batched and not yet destroyed.
// Every entry point checks its handle here before touching it, so a destroyed
// handle (or any other pointer) is refused with PM_ESTATE instead of being
// dereferenced -- unless a later plan happens to occupy the same address.
std::mutex g_live_mu;
std::set<const pm_plan*> g_live;

void plan_register(const pm_plan* h) {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(h);
}
bool plan_unregister(const pm_plan* h) {
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.erase(h) == 1;
}
bool plan_live(const pm_plan* h) {
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.count(h) == 1;
}

// A live plan of either kind.
pm_status check_any(pm_plan* h) {
    if (h == nullptr) return fail(PM_EINVAL, "null handle");
    if (!plan_live(h)) return fail(PM_ESTATE, "not a live plan (destroyed, or never created)");
    if (h->dead) return fail(PM_ESTATE, "handle is in an unusable state");
    return PM_OK;
}

pm_status check_handle(pm_plan* h, bool batched = false) {
    pm_status st = check_any(h);
    if (st != PM_OK) return st;
    if (h->batched != batched)
        return fail(PM_ESTATE, batched ? "handle is not a batched plan" : "handle is a batched plan");
    return PM_OK;
}

// Layout of a caller-owned workspace (phasemask_set_workspace): the iterate,
// the rescaled target and the partial sums, each 256-byte aligned.
struct WsLayout {
    size_t mhat_off, part_off;
};
size_t align256(size_t b) { return (b + 255) / 256 * 256; }
WsLayout ws_layout(const pm_plan* h) {
    const size_t x = align256((size_t)h->N * sizeof(float2));
    return WsLayout{x, x + align256((size_t)h->N * sizeof(float))};
}

// History entries of partials the calls other than the solves need: two
// (phasemask_error, phasemask_time_passes), or the physical error's
// per-block pairs.
size_t min_partial_entries(const pm_plan* h) {
    const size_t nblk = ((size_t)h->N / 4 + 255) / 256;
    return std::max<size_t>(2, 1 + (2 * nblk + h->stride - 1) / h->stride);
}

// Makes sure `part` holds `entries` history entries of partials.
pm_status ensure_partials(pm_plan* h, size_t entries) {
    if (entries <= h->part_entries) return PM_OK;
    if (h->ws_borrowed) {
        std::ostringstream os;
        os << "the workspace set by phasemask_set_workspace holds partial sums for " << h->part_entries
           << " error-history entries; this call needs " << entries << " (see phasemask_workspace_size)";
        return fail(PM_EINVAL, os.str());
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    drop_graphs(h);  // captured graphs hold the old pointer
    size_t want = h->part_entries ? h->part_entries : 64;
    while (want < entries) want *= 2;
    double* p = nullptr;
    e = hipMalloc(&p, want * (size_t)h->stride * sizeof(double));
    if (e != hipSuccess) return fail_hip(e, "hipMalloc(partials)");
    (void)hipFree(h->part);
    h->ws_bytes += (want - h->part_entries) * (size_t)h->stride * sizeof(double);
    h->part = p;
    h->part_entries = want;
    return PM_OK;
}

pm::RowParams row_params(pm_plan* h, double* part) {
    pm::RowParams r{};
    r.X = h->X;
    r.tw = h->twW;
    r.io = h->io;
    r.part = part;
    r.H = h->H;
    r.illum = h->illum_on ? h->illum : nullptr;
    r.spread = h->nwg_row <= h->num_cu;
    return r;
}

// A solve-path row mode, with the illumination variant when one is set.
int rmode(const pm_plan* h, int mode) { return h->illum_on ? (mode | pm::R_ILLUM) : mode; }

// ||p||^2 on the device for the error scales, or null for p = 1.
const double* pnorm2(const pm_plan* h) { return h->illum_on ? h->pn2 : nullptr; }

pm::ColParams col_params(pm_plan* h, double* part) {
    pm::ColParams c{};
    c.X = h->X;
    c.mhat = h->mhat;
    c.tw = h->twH;
    c.part = part;
    c.W = h->W;
    c.invN = 1.0 / (double)h->N;
    c.spread = h->nwg_col <= h->num_cu;
    return c;
}

#define PM_TRY(expr, what)                          \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

// PM_FLAG_VALIDATE: checks `n` floats at x on the device (sign only when
// `nonneg`; all zero is an error only when `need_nonzero`) and waits for the
// result.  `what` names the argument in the error message.
pm_status validate_input(pm_plan* h, const float* x, bool nonneg, bool need_nonzero, const char* what,
                         int floats_per_pixel = 1) {
    if ((h->flags & PM_FLAG_VALIDATE) == 0 || x == nullptr) return PM_OK;
    PM_TRY(hipMemsetAsync(h->vflags, 0, 2 * sizeof(int), h->stream), "hipMemsetAsync(check)");
    PM_TRY(pm::launch_validate(x, h->N * floats_per_pixel, nonneg, h->vflags, h->stream), "input check");
    int f[2] = {0, 0};
    PM_TRY(hipMemcpyAsync(f, h->vflags, sizeof(f), hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync(check)");
    PM_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize(check)");
    if (f[0] & 2) return fail(PM_EINVAL, std::string(what) + " has a non-finite entry");
    if (f[0] & 1) return fail(PM_EINVAL, std::string(what) + " has a negative entry");
    if (need_nonzero && f[1] == 0) return fail(PM_EINVAL, std::string(what) + " is all zero");
    return PM_OK;
}


// Target normalisation + tiling (the rescaled m used by every column pass).
pm_status enqueue_target(pm_plan* h, hipStream_t s) {
    PM_TRY(pm::launch_norm_partial(h->io, h->N, h->part_m, kNormGrid, s), "target norm");
    PM_TRY(pm::launch_target_tile(h->io, h->H, h->W, h->part_m, kNormGrid, h->mhat, s, pnorm2(h)), "target tile");
    return PM_OK;
}

// Solve algorithms (one captured graph per algorithm, n_iter and history).
enum : int {
    kAlgoGS = 0,       // alternating projections, phases in and out
    kAlgoRAAR = 1,     // RAAR, phases in and out
    kAlgoGSField = 2,  // alternating projections, complex fields in and out
    kAlgoAdam = 3,     // Adam on the intensity loss, phases in and out
    kAlgoMany = 4,     // alternating projections on a uniform batch of masks
};

// The whole solve after the pointer block is set: target preparation,
// u^0, n_iter iterations, final error and history finalisation.
pm_status enqueue_solve(pm_plan* h, hipStream_t s, int n_iter, bool hist, int algo = kAlgoGS, float beta = 0.0f) {
    const int lw = len_slot(h->W), lh = len_slot(h->H);
    const RowLauncher row = kRowLaunch[lw];
    const ColLauncher col = kColLaunch[lh];
    // Partials of history entry e; without a history the passes write none
    // and the plan holds a single entry.
    auto pe = [&](int e) { return hist ? h->part + (size_t)e * h->stride : h->part; };
    const bool field = algo == kAlgoGSField;
    // u^0: exp(i phi0) (times p), or the caller's field as given.
    const int init_mode = field ? pm::ROW_INIT_FIELD : rmode(h, pm::ROW_INIT);

    if (n_iter == 0) {
        if (field) {
            PM_TRY(row(pm::ROW_COPY_FIELD, row_params(h, nullptr), h->nwg_row, s, nullptr, nullptr), "field copy");
        } else {
            PM_TRY(pm::launch_wrap_phase(h->io, h->N, s), "wrap phase");
        }
        if (!hist) return PM_OK;
        pm_status st = enqueue_target(h, s);
        if (st != PM_OK) return st;
        PM_TRY(row(init_mode, row_params(h, nullptr), h->nwg_row, s, nullptr, nullptr), "row init");
        PM_TRY(col(pm::COL_ERR, col_params(h, pe(0)), h->nwg_col, s, nullptr, nullptr), "column error");
        PM_TRY(pm::launch_finalize(h->part, h->stride, h->slots_col, h->slots_row, 1.0 / h->N, h->io, 0, 1, s, 1, pnorm2(h)),
               "finalize");
        return PM_OK;
    }
    pm_status st = enqueue_target(h, s);
    if (st != PM_OK) return st;
    if (algo == kAlgoRAAR) {
        // RAAR: x^0 = exp(i phi0) kept in Z; history = E_F(x^nu) at entries
        // 2 nu and E_F(P_S x^n) at entry 2 n, finalised with step 2.
        pm::RowParams rp = row_params(h, nullptr);
        rp.Z = h->Z;
        rp.beta = beta;
        PM_TRY(row(rmode(h, pm::ROW_INIT_Z), rp, h->nwg_row, s, nullptr, nullptr), "row init");
        for (int nu = 0; nu < n_iter; ++nu) {
            PM_TRY(col(hist ? pm::COL_ITER : pm::COL_ITER_NE, col_params(h, pe(2 * nu)), h->nwg_col, s, nullptr,
                       nullptr),
                   "column pass");
            const bool last = nu == n_iter - 1;
            const int mode = !last ? pm::ROW_RAAR : (hist ? pm::ROW_RAAR_LAST_FWD : pm::ROW_RAAR_LAST);
            PM_TRY(row(rmode(h, mode), rp, h->nwg_row, s, nullptr, nullptr), "RAAR row pass");
        }
        if (hist) {
            PM_TRY(col(pm::COL_ERR, col_params(h, pe(2 * n_iter)), h->nwg_col, s, nullptr, nullptr), "column error");
            PM_TRY(pm::launch_finalize(h->part, h->stride, h->slots_col, h->slots_row, 1.0 / h->N, h->io, 0, n_iter + 1,
                                       s, 2, pnorm2(h)),
                   "finalize");
        }
        return PM_OK;
    }
    PM_TRY(row(init_mode, row_params(h, nullptr), h->nwg_row, s, nullptr, nullptr), "row init");
    // Without a history the passes skip their error partial sums.
    const int col_mode = hist ? pm::COL_ITER : pm::COL_ITER_NE;
    const int row_mode = hist ? pm::ROW_ITER : pm::ROW_ITER_NE;
    const int last_mode = field ? (hist ? pm::ROW_LAST_FIELD_FWD : pm::ROW_LAST_FIELD_NE)
                                : (hist ? pm::ROW_LAST_FWD : pm::ROW_LAST_NE);
    for (int nu = 0; nu < n_iter; ++nu) {
        PM_TRY(col(col_mode, col_params(h, pe(2 * nu)), h->nwg_col, s, nullptr, nullptr), "column pass");
        const bool last = nu == n_iter - 1;
        const int mode = !last ? row_mode : last_mode;
        PM_TRY(row(rmode(h, mode), row_params(h, pe(2 * nu + 1)), h->nwg_row, s, nullptr, nullptr), "row pass");
    }
    if (hist) {
        PM_TRY(col(pm::COL_ERR, col_params(h, pe(2 * n_iter)), h->nwg_col, s, nullptr, nullptr), "column error");
        PM_TRY(pm::launch_finalize(h->part, h->stride, h->slots_col, h->slots_row, 1.0 / h->N, h->io, 0,
                                   2 * n_iter + 1, s, 1, pnorm2(h)),
               "finalize");
    }
    return PM_OK;
}

// A uniform batch of `batch` masks (phasemask_solve_many): the one-mask
// solve's sequence with every launch covering all masks (grid.y = mask),
// each mask with its own iterate, rescaled target, partials and history.
pm_status enqueue_many(pm_plan* h, hipStream_t s, int n_iter, bool hist, int batch) {
    const RowLauncher row = kRowLaunch[len_slot(h->W)];
    const ColLauncher col = kColLaunch[len_slot(h->H)];
    const size_t bstride = h->many_entries * (size_t)h->stride;
    auto pe = [&](int e) { return hist ? h->m_part + (size_t)e * h->stride : h->m_part; };
    pm::RowParams rp = row_params(h, nullptr);
    rp.X = h->m_X;
    rp.nb = batch;
    rp.part_bstride = bstride;
    rp.spread = (long)h->nwg_row * batch <= h->num_cu;
    pm::ColParams cp = col_params(h, nullptr);
    cp.X = h->m_X;
    cp.mhat = h->m_mhat;
    cp.nb = batch;
    cp.part_bstride = bstride;
    cp.spread = (long)h->nwg_col * batch <= h->num_cu;
    auto rpe = [&](double* part) {
        pm::RowParams r = rp;
        r.part = part;
        return r;
    };
    auto cpe = [&](double* part) {
        pm::ColParams c = cp;
        c.part = part;
        return c;
    };
    if (n_iter == 0) {
        PM_TRY(pm::launch_wrap_phase(h->io, h->N * batch, s), "wrap phase");
        if (!hist) return PM_OK;
    }
    PM_TRY(pm::launch_norm_partial(h->io, h->N, h->m_partm, kNormGrid, s, batch), "target norm");
    PM_TRY(pm::launch_target_tile(h->io, h->H, h->W, h->m_partm, kNormGrid, h->m_mhat, s, pnorm2(h), batch),
           "target tile");
    PM_TRY(row(rmode(h, pm::ROW_INIT_MANY), rpe(nullptr), h->nwg_row, s, nullptr, nullptr), "row init");
    const int col_mode = hist ? pm::COL_ITER_MANY : pm::COL_ITER_NE_MANY;
    const int row_mode = hist ? pm::ROW_ITER_MANY : pm::ROW_ITER_NE_MANY;
    const int last_mode = hist ? pm::ROW_LAST_FWD_MANY : pm::ROW_LAST_NE_MANY;
    for (int nu = 0; nu < n_iter; ++nu) {
        PM_TRY(col(col_mode, cpe(pe(2 * nu)), h->nwg_col, s, nullptr, nullptr), "column pass");
        const int mode = nu < n_iter - 1 ? row_mode : last_mode;
        PM_TRY(row(rmode(h, mode), rpe(pe(2 * nu + 1)), h->nwg_row, s, nullptr, nullptr), "row pass");
    }
    if (hist) {
        PM_TRY(col(pm::COL_ERR_MANY, cpe(pe(2 * n_iter)), h->nwg_col, s, nullptr, nullptr), "column error");
        PM_TRY(pm::launch_finalize(h->m_part, h->stride, h->slots_col, h->slots_row, 1.0 / h->N, h->io, 0,
                                   2 * n_iter + 1, s, 1, pnorm2(h), batch, bstride),
               "finalize");
    }
    return PM_OK;
}

pm_status enqueue_batch(pm_plan* h, hipStream_t s, int n_iter, bool err);
pm_status enqueue_adam(pm_plan* h, hipStream_t s, const SolveKey& k);
pm_status enqueue_adam_chain(pm_plan* h, hipStream_t s, const SolveKey& k);

// The whole sequence of one solve, as the key describes it.
pm_status enqueue_key(pm_plan* h, hipStream_t s, const SolveKey& k) {
    if (h->batched) return enqueue_batch(h, s, k.n_iter, k.hist);
    if (k.algo == kAlgoAdam) return k.chain >= 0 ? enqueue_adam_chain(h, s, k) : enqueue_adam(h, s, k);
    if (k.algo == kAlgoMany) return enqueue_many(h, s, k.n_iter, k.hist, k.batch);
    return enqueue_solve(h, s, k.n_iter, k.hist, k.algo, k.beta);
}

// Replays (capturing on first use) the graph of one solve shape, on the
// handle's stream or on `stream`.
pm_status launch_graph(pm_plan* h, const SolveKey& key, hipStream_t stream = nullptr) {
    hipStream_t ls = stream != nullptr ? stream : h->stream;
    for (auto it = h->graphs.begin(); it != h->graphs.end(); ++it) {
        if (it->key == key) {
            h->graphs.splice(h->graphs.begin(), h->graphs, it);
            PM_TRY(hipGraphLaunch(it->exec, ls), "hipGraphLaunch");
            return PM_OK;
        }
    }
    hipGraph_t graph = nullptr;
    PM_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    pm_status st = enqueue_key(h, h->cap_stream, key);
    hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
    if (st != PM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ec != hipSuccess) return fail_hip(ec, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail_hip(ei, "hipGraphInstantiate");
    if (h->graphs.size() >= kMaxCachedGraphs) {
        (void)hipGraphExecDestroy(h->graphs.back().exec);
        h->graphs.pop_back();
    }
    h->graphs.push_front(GraphEntry{key, exec});
    PM_TRY(hipGraphLaunch(exec, ls), "hipGraphLaunch");
    return PM_OK;
}

pm_status launch_graph(pm_plan* h, int n_iter, bool hist, int algo = kAlgoGS, float beta = 0.0f) {
    SolveKey k;
    k.n_iter = n_iter;
    k.hist = hist;
    k.algo = algo;
    k.beta = beta;
    return launch_graph(h, k);
}

// ----- batched solves ----------------------------------------------------------

bool batch_len_ok(int n) {
    return n >= pm::kBatchMinLen && n <= pm::kBatchMaxLen && (n & (n - 1)) == 0;
}

pm::BatchParams batch_params(pm_plan* h, const pm::BatchTask* tasks) {
    pm::BatchParams p{};
    p.masks = h->masks;
    p.tasks = tasks;
    p.tw = h->tw_batch;
    p.io = h->bio;
    p.part = h->part;
    return p;
}

template <int SCHED>
hipError_t batch_col_s(int mode, const pm::BatchParams& p, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (mode) {
        case pm::COL_ITER_NE: return pm::launch_batch_col<pm::COL_ITER_NE, SCHED>(p, grid, s, e0, e1);
        case pm::COL_ERR: return pm::launch_batch_col<pm::COL_ERR, SCHED>(p, grid, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <int SCHED>
hipError_t batch_row_s(int mode, const pm::BatchParams& p, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (mode) {
        case pm::ROW_INIT: return pm::launch_batch_row<pm::ROW_INIT, SCHED>(p, grid, s, e0, e1);
        case pm::ROW_ITER_NE: return pm::launch_batch_row<pm::ROW_ITER_NE, SCHED>(p, grid, s, e0, e1);
        case pm::ROW_LAST_NE: return pm::launch_batch_row<pm::ROW_LAST_NE, SCHED>(p, grid, s, e0, e1);
        case pm::ROW_LAST_FWD_NE: return pm::launch_batch_row<pm::ROW_LAST_FWD_NE, SCHED>(p, grid, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

// Column (row) pass over tasks [t0, t1) of the active layout (t1 < 0: all).
// The error partial of a task is written at part[task - t0].
hipError_t batch_col(pm_plan* h, int mode, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                     int t0 = 0, int t1 = -1) {
    if (t1 < 0) t1 = h->n_col_tasks;
    const pm::BatchParams p = batch_params(h, h->col_tasks + t0);
    static_assert(pm::kBatchSchedules == 2, "one dispatch case per schedule");
    return h->sched == 0 ? batch_col_s<0>(mode, p, t1 - t0, s, e0, e1) : batch_col_s<1>(mode, p, t1 - t0, s, e0, e1);
}

hipError_t batch_row(pm_plan* h, int mode, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                     int t0 = 0, int t1 = -1) {
    if (t1 < 0) t1 = h->n_row_tasks;
    const pm::BatchParams p = batch_params(h, h->row_tasks + t0);
    return h->sched == 0 ? batch_row_s<0>(mode, p, t1 - t0, s, e0, e1) : batch_row_s<1>(mode, p, t1 - t0, s, e0, e1);
}

// n_iter iterations of every mask: all iterations of one group of masks
// before the next group of the same chain, so that the group's working set
// stays cache-resident across its iterations; groups alternate between the
// chains, which run concurrently (fork and join through events on s).  The
// last row pass of a group runs in `last_mode`.
pm_status enqueue_groups(pm_plan* h, hipStream_t s, int n_iter, int last_mode) {
    const int chains = std::min<int>(h->chains, (int)h->groups.size());
    for (int c = 1; c < chains; ++c) {
        PM_TRY(hipEventRecord(h->fork_ev[c - 1], s), "hipEventRecord(fork)");
        PM_TRY(hipStreamWaitEvent(h->side[c - 1], h->fork_ev[c - 1], 0), "hipStreamWaitEvent(fork)");
    }
    for (const pm_batch_group& g : h->groups) {
        const int c = g.chain < chains ? g.chain : 0;
        hipStream_t cs = c == 0 ? s : h->side[c - 1];
        for (int nu = 0; nu < n_iter; ++nu) {
            PM_TRY(batch_col(h, pm::COL_ITER_NE, cs, nullptr, nullptr, g.c0, g.c1), "batch column pass");
            const int mode = nu < n_iter - 1 ? pm::ROW_ITER_NE : last_mode;
            PM_TRY(batch_row(h, mode, cs, nullptr, nullptr, g.r0, g.r1), "batch row pass");
        }
    }
    for (int c = 1; c < chains; ++c) {
        PM_TRY(hipEventRecord(h->join_ev[c - 1], h->side[c - 1]), "hipEventRecord(join)");
        PM_TRY(hipStreamWaitEvent(s, h->join_ev[c - 1], 0), "hipStreamWaitEvent(join)");
    }
    return PM_OK;
}

// Whole batched solve after the pointer block is set.
pm_status enqueue_batch(pm_plan* h, hipStream_t s, int n_iter, bool err) {
    if (n_iter == 0) {
        PM_TRY(pm::launch_batch_wrap(h->bio, h->masks, h->prep_tasks, h->n_prep_tasks, s), "batch wrap");
        if (!err) return PM_OK;
    }
    PM_TRY(pm::launch_batch_norm(h->bio, h->prep_tasks, h->n_prep_tasks, h->part_m, s), "batch norm");
    PM_TRY(pm::launch_batch_tile(h->bio, h->masks, h->prep_tasks, h->n_prep_tasks, h->mask_prep0, h->part_m, s),
           "batch tile");
    PM_TRY(batch_row(h, pm::ROW_INIT, s), "batch row init");
    pm_status st = enqueue_groups(h, s, n_iter, err ? pm::ROW_LAST_FWD_NE : pm::ROW_LAST_NE);
    if (st != PM_OK) return st;
    if (err) {
        PM_TRY(batch_col(h, pm::COL_ERR, s), "batch column error");
        PM_TRY(pm::launch_batch_finalize(h->bio, h->masks, h->count, h->part, s), "batch finalize");
    }
    return PM_OK;
}

// ----- batched schedule tuner --------------------------------------------------

struct BatchLayout {
    std::vector<pm::BatchMask> masks;
    std::vector<pm::BatchTask> col, row;
    std::vector<int> seq;              // masks in task order
    std::vector<int> row0, rows;       // each mask's row tasks
};

// Task lists of one schedule; masks in `order` (largest first).
BatchLayout batch_layout(int sched, int count, const int* heights, const int* widths,
                         const std::vector<int>& order, const std::vector<float2*>& xs,
                         const std::vector<float*>& ms) {
    BatchLayout l;
    l.masks.resize(count);
    for (int i : order) {
        const int H = heights[i], W = widths[i];
        pm::BatchMask& mk = l.masks[i];
        mk.H = H;
        mk.W = W;
        mk.X = xs[i];
        mk.mhat = ms[i];
        const int gc = pm::batch_lines(sched, H) / pm::kC;  // strips per column work-group
        mk.col_wg0 = (int)l.col.size();
        for (int s0 = 0; s0 < W / pm::kC; s0 += gc) l.col.push_back(pm::BatchTask{i, s0});
        mk.col_wgs = (int)l.col.size() - mk.col_wg0;
        const int gr = pm::batch_lines(sched, W);
        l.seq.push_back(i);
        l.row0.resize(count);
        l.rows.resize(count);
        l.row0[i] = (int)l.row.size();
        for (int r0 = 0; r0 < H; r0 += gr) l.row.push_back(pm::BatchTask{i, r0});
        l.rows[i] = (int)l.row.size() - l.row0[i];
    }
    return l;
}

// Consecutive masks (in task order) whose working sets (iterate 8 B/px and
// target 4 B/px) add up to at most `budget` bytes form one group; a mask
// larger than the budget forms a group of its own.  budget 0: one group.
std::vector<pm_batch_group> batch_groups(const BatchLayout& l, size_t budget) {
    std::vector<pm_batch_group> g;
    size_t bytes = 0;
    for (int i : l.seq) {
        const pm::BatchMask& mk = l.masks[i];
        const size_t b = (size_t)mk.H * mk.W * (sizeof(float2) + sizeof(float));
        if (g.empty() || (budget > 0 && bytes + b > budget)) {
            g.push_back(pm_batch_group{mk.col_wg0, mk.col_wg0, l.row0[i], l.row0[i], 0, 0});
            bytes = 0;
        }
        g.back().c1 = mk.col_wg0 + mk.col_wgs;
        g.back().r1 = l.row0[i] + l.rows[i];
        g.back().bytes += b;
        bytes += b;
    }
    return g;
}

// Spreads the groups over `chains` chains, each group (largest first, in the
// order they were formed) to the chain with the fewest bytes so far, so the
// concurrent chains finish at about the same time.
void assign_chains(std::vector<pm_batch_group>& g, int chains) {
    std::vector<size_t> load((size_t)std::max(chains, 1), 0);
    for (pm_batch_group& x : g) {
        const size_t c = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        x.chain = (int)c;
        load[c] += x.bytes;
    }
}

hipError_t upload_layout(pm_plan* h, const BatchLayout& l) {
    hipError_t e = hipMemcpy(h->masks, l.masks.data(), l.masks.size() * sizeof(pm::BatchMask), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(h->col_tasks, l.col.data(), l.col.size() * sizeof(pm::BatchTask), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(h->row_tasks, l.row.data(), l.row.size() * sizeof(pm::BatchTask), hipMemcpyHostToDevice);
    h->n_col_tasks = (int)l.col.size();
    h->n_row_tasks = (int)l.row.size();
    h->groups = batch_groups(l, h->group_bytes);
    assign_chains(h->groups, h->chains);
    return e;
}

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;
bool g_tune_file_read = false;

std::string tune_key(int device, int count, const int* heights, const int* widths) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
    std::vector<std::pair<int, int>> sz;
    for (int i = 0; i < count; ++i) sz.emplace_back(heights[i], widths[i]);
    std::sort(sz.begin(), sz.end());
    std::ostringstream os;
    os << arch.substr(0, arch.find(':')) << '|';
    for (auto& p : sz) os << p.first << 'x' << p.second << ',';
    return os.str();
}

// Average device time of one batched iteration run the way a solve runs it:
// `iters` iterations of every group on the plan's concurrent chains,
// captured in a graph (on the capture stream) and replayed twice on the
// plan's stream; the second replay is timed.
pm_status time_batch(pm_plan* h, int iters, double* ms_out) {
    hipGraph_t graph = nullptr;
    PM_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture(tune)");
    pm_status st = enqueue_groups(h, h->cap_stream, iters, pm::ROW_ITER_NE);
    hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
    if (st != PM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ec != hipSuccess) return fail_hip(ec, "hipStreamEndCapture(tune)");
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail_hip(e, "hipGraphInstantiate(tune)");
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipGraphLaunch(exec, h->stream);  // untimed
    if (e == hipSuccess) e = hipEventRecord(a, h->stream);
    if (e == hipSuccess) e = hipGraphLaunch(exec, h->stream);
    if (e == hipSuccess) e = hipEventRecord(b, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipGraphExecDestroy(exec);
    if (e != hipSuccess) return fail_hip(e, "tune timing");
    *ms_out = (double)ms / iters;
    return PM_OK;
}

// Picks the FFT schedule of a batched plan: PHASEMASK_SCHEDULE forces one;
// otherwise a cached choice for the same sizes on the same architecture
// (in-process, and the file named by PHASEMASK_TUNE_CACHE if set); otherwise
// every schedule is timed on the plan's zeroed buffers and the fastest kept.
pm_status tune_batch(pm_plan* h, const std::vector<BatchLayout>& layouts, const std::string& key) {
    const char* force = std::getenv("PHASEMASK_SCHEDULE");
    if (force != nullptr && force[0] != '\0') {
        const int f = std::atoi(force);
        if (f < 0 || f >= pm::kBatchSchedules) return fail(PM_EINVAL, "PHASEMASK_SCHEDULE out of range");
        h->sched = f;
        return PM_OK;
    }
    if (h->flags & PM_FLAG_NO_TUNE) {
        h->sched = 0;
        return PM_OK;
    }
    const char* path = std::getenv("PHASEMASK_TUNE_CACHE");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!g_tune_file_read && path != nullptr && path[0] != '\0') {
            g_tune_file_read = true;
            std::ifstream in(path);
            std::string k;
            int v;
            while (in >> k >> v)
                if (v >= 0 && v < pm::kBatchSchedules) g_tune_cache[k] = v;
        }
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            h->sched = it->second;
            return PM_OK;
        }
    }
    PM_TRY(hipMemsetAsync(h->batch_ws, 0, h->batch_ws_bytes, h->stream), "hipMemsetAsync(tune)");
    double best = 1e30;
    int best_s = 0;
    for (int sc = 0; sc < pm::kBatchSchedules; ++sc) {
        h->sched = sc;
        PM_TRY(upload_layout(h, layouts[sc]), "upload layout");
        double ms = 0.0;
        const pm_status tst = time_batch(h, kTuneIterations, &ms);
        if (tst != PM_OK) return tst;
        if (std::getenv("PHASEMASK_LOG") != nullptr)
            std::fprintf(stderr, "phasemask tune %s schedule %d: %.1f us/iteration\n", key.c_str(), sc, ms * 1e3);
        // a later schedule must win by kTuneMargin: near-ties keep the
        // earlier one, so repeated plan creations choose alike
        if (ms < best * (1.0 - kTuneMargin)) {
            best = ms;
            best_s = sc;
        }
    }
    h->sched = best_s;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best_s;
    if (path != nullptr && path[0] != '\0') {
        std::ofstream outf(path, std::ios::app);
        outf << key << ' ' << best_s << '\n';
    }
    return PM_OK;
}

bool misaligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) != 0; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

extern "C" {

const char* phasemask_status_string(pm_status s) {
    switch (s) {
        case PM_OK: return "PM_OK";
        case PM_EINVAL: return "PM_EINVAL: invalid argument";
        case PM_EUNSUPPORTED: return "PM_EUNSUPPORTED: unsupported size";
        case PM_ENOMEM: return "PM_ENOMEM: out of memory";
        case PM_EDEVICE: return "PM_EDEVICE: device error";
        case PM_ESTATE: return "PM_ESTATE: bad handle state";
    }
    return "unknown pm_status";
}

const char* phasemask_last_error(void) { return g_last_error.c_str(); }

namespace {
hipError_t scratch_address(int device, unsigned char** out);  // allocation-free solve (below)
}  // namespace

pm_status phasemask_create(pm_handle* out, int height, int width, unsigned flags, void* stream) {
    if (out == nullptr) return fail(PM_EINVAL, "out is NULL");
    *out = nullptr;
    if (len_slot(height) < 0 || len_slot(width) < 0)
        return fail(PM_EUNSUPPORTED,
                    "height and width must each be a power of two in [16, 4096], 600, 800, 1080 or 1920");
    if ((flags & ~(PM_FLAG_NO_GRAPH | PM_FLAG_VALIDATE)) != 0) return fail(PM_EINVAL, "unknown flag bits");
    pm_plan* h = new (std::nothrow) pm_plan;
    if (h == nullptr) return fail(PM_ENOMEM, "host allocation failed");
    h->H = height;
    h->W = width;
    h->N = height * width;
    h->flags = flags;
    h->stream = (hipStream_t)stream;
    auto bail = [&](hipError_t e, const char* what) {
        pm_status s = fail_hip(e, what);
        free_plan(h);
        return s;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device)) != hipSuccess)
        return bail(e, "hipDeviceGetAttribute");
    h->rows = pm::rows_for_plan(height, width, h->num_cu);
    h->nwg_row = height / h->rows;
    h->nwg_col = width / pm::col_lines(height);
    // Threads per work-group: lines x (length / points per thread).
    h->slots_row = h->nwg_row * pm::red_slots(h->rows * (width / pm::points_per_thread(width)));
    h->slots_col = h->nwg_col * pm::red_slots(pm::col_lines(height) * (height / pm::points_per_thread(height)));
    h->slots_adj = (width / pm::kC) * pm::red_slots(pm::kC * (height / pm::points_per_thread(height)));
    h->stride = h->slots_row > h->slots_col ? h->slots_row : h->slots_col;
    if (h->stride < h->slots_adj) h->stride = h->slots_adj;
    if (h->stride < kNormGrid) h->stride = kNormGrid;
    const size_t n = (size_t)h->N;
    if ((e = hipMalloc(&h->X, n * sizeof(float2))) != hipSuccess) return bail(e, "hipMalloc(iterate)");
    if ((e = hipMalloc(&h->mhat, n * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc(target)");
    const std::vector<float2> tw_w = pm::staged_twiddles(width, pm::points_per_thread(width));
    const std::vector<float2> tw_h = pm::staged_twiddles(height, pm::points_per_thread(height));
    if ((e = hipMalloc(&h->twW, tw_w.size() * sizeof(float2))) != hipSuccess) return bail(e, "hipMalloc(twiddles)");
    if ((e = hipMalloc(&h->twH, tw_h.size() * sizeof(float2))) != hipSuccess) return bail(e, "hipMalloc(twiddles)");
    if ((e = hipMalloc(&h->part_m, kNormGrid * sizeof(double))) != hipSuccess) return bail(e, "hipMalloc(norm)");
    if ((e = hipMalloc(&h->part_mx, kNormGrid * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc(max)");
    if ((e = hipMalloc(&h->io, sizeof(pm::PmIo))) != hipSuccess) return bail(e, "hipMalloc(io)");
    h->ws_bytes = n * (sizeof(float2) + sizeof(float)) + (tw_w.size() + tw_h.size()) * sizeof(float2) +
                  kNormGrid * sizeof(double) + sizeof(pm::PmIo);
    if ((e = hipMemcpy(h->twW, tw_w.data(), tw_w.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "hipMemcpy(twiddles)");
    if ((e = hipMemcpy(h->twH, tw_h.data(), tw_h.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "hipMemcpy(twiddles)");
    if ((e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(e, "hipStreamCreate");
    // Set-up of the allocation-free solve on this device (the plan's device
    // is current here); a failed lookup only disables that entry point.
    h->scratch_err = scratch_address(h->device, &h->scratch);
    if ((flags & PM_FLAG_VALIDATE) != 0 && (e = hipMalloc(&h->vflags, 2 * sizeof(int))) != hipSuccess)
        return bail(e, "hipMalloc(check)");
    if (std::getenv("PHASEMASK_LOG") != nullptr) {
        auto line = [](int L) {
            std::ostringstream os;
            os << L << " points: " << (pm::lds_mode(L) ? "LDS" : "register") << " scheme, "
               << pm::points_per_thread(L) << " points x " << L / pm::points_per_thread(L) << " threads";
            return os.str();
        };
        std::fprintf(stderr, "phasemask plan %dx%d: rows %s, %d work-groups of %d rows; columns %s, %d work-groups; "
                     "workspace %zu bytes\n", height, width, line(width).c_str(), h->nwg_row,
                     h->rows, line(height).c_str(), h->nwg_col, h->ws_bytes);
    }
    plan_register(h);
    *out = h;
    return PM_OK;
}

pm_status phasemask_destroy(pm_handle h) {
    if (h == nullptr) return fail(PM_EINVAL, "null handle");
    if (!plan_unregister(h)) return fail(PM_ESTATE, "not a live plan (destroyed, or never created)");
    (void)hipStreamSynchronize(h->stream);
    free_plan(h);
    return PM_OK;
}

pm_status phasemask_set_stream(pm_handle h, void* stream) {
    pm_status st = check_any(h);
    if (st != PM_OK) return st;
    const hipStream_t ns = (hipStream_t)stream;
    if (ns == h->stream) return PM_OK;
    // The handle's buffers (pointer block, iterate, target, partials) serve
    // every call, so work enqueued on the new stream waits for everything the
    // handle enqueued on the old one.
    if (h->order_ev == nullptr) {
        hipError_t e = hipEventCreateWithFlags(&h->order_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            h->order_ev = nullptr;
            return fail_hip(e, "hipEventCreate(stream order)");
        }
    }
    PM_TRY(hipEventRecord(h->order_ev, h->stream), "hipEventRecord(stream order)");
    PM_TRY(hipStreamWaitEvent(ns, h->order_ev, 0), "hipStreamWaitEvent(stream order)");
    h->stream = ns;
    return PM_OK;
}

pm_status phasemask_set_illumination(pm_handle h, const float* illumination) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (illumination != nullptr && misaligned(illumination, 16))
        return fail(PM_EINVAL, "illumination must be 16-byte aligned");
    const bool on = illumination != nullptr;
    if ((st = validate_input(h, illumination, true, true, "illumination")) != PM_OK) return st;
    if (on != h->illum_on) {
        // Captured graphs hold the kernels of the other case.
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
        drop_graphs(h);
    }
    if (!on) {
        h->illum_on = false;
        return PM_OK;
    }
    if (h->illum == nullptr) {
        hipError_t e = hipMalloc(&h->illum, (size_t)h->N * sizeof(float));
        if (e != hipSuccess) return fail_hip(e, "hipMalloc(illumination)");
        e = hipMalloc(&h->pn2, sizeof(double));
        if (e != hipSuccess) {
            (void)hipFree(h->illum);
            h->illum = nullptr;
            return fail_hip(e, "hipMalloc(illumination norm)");
        }
        h->ws_bytes += (size_t)h->N * sizeof(float) + sizeof(double);
    }
    PM_TRY(pm::launch_illum_prep(illumination, h->H, h->W, h->part_m, kNormGrid, h->illum, h->pn2, h->stream),
           "illumination set-up");
    h->illum_on = true;
    return PM_OK;
}

size_t phasemask_workspace_bytes(pm_handle h) { return (h != nullptr && plan_live(h)) ? h->ws_bytes : 0; }

size_t phasemask_workspace_size(pm_handle h, int n_iter) {
    if (h == nullptr || !plan_live(h) || h->dead || h->batched || n_iter < 0) return 0;
    return ws_layout(h).part_off + std::max(min_partial_entries(h), 2 * (size_t)n_iter + 1) * (size_t)h->stride *
                                       sizeof(double);
}

pm_status phasemask_set_workspace(pm_handle h, void* dev_ptr, size_t bytes) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    const WsLayout l = ws_layout(h);
    const size_t min_bytes = phasemask_workspace_size(h, 0);
    if (dev_ptr != nullptr) {
        if (misaligned(dev_ptr, 256)) return fail(PM_EINVAL, "workspace must be 256-byte aligned");
        if (bytes < min_bytes) {
            std::ostringstream os;
            os << "workspace of " << bytes << " bytes is below the minimum of " << min_bytes
               << " (phasemask_workspace_size(h, 0))";
            return fail(PM_EINVAL, os.str());
        }
    }
    // Captured graphs and queued work refer to the current buffers.
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    drop_graphs(h);
    const size_t own = (size_t)h->N * (sizeof(float2) + sizeof(float)) + h->part_entries * (size_t)h->stride * sizeof(double);
    if (dev_ptr == nullptr) {
        if (!h->ws_borrowed) return PM_OK;
        float2* x = nullptr;
        float* m = nullptr;
        e = hipMalloc(&x, (size_t)h->N * sizeof(float2));
        if (e == hipSuccess) e = hipMalloc(&m, (size_t)h->N * sizeof(float));
        if (e != hipSuccess) {
            (void)hipFree(x);
            return fail_hip(e, "hipMalloc(workspace)");
        }
        h->X = x;
        h->mhat = m;
        h->part = nullptr;
        h->part_entries = 0;
        h->ws_borrowed = false;
        h->ws_bytes += (size_t)h->N * (sizeof(float2) + sizeof(float));
        return PM_OK;
    }
    if (!h->ws_borrowed) {
        (void)hipFree(h->X);
        (void)hipFree(h->mhat);
        (void)hipFree(h->part);
        h->ws_bytes -= own;
    }
    char* base = (char*)dev_ptr;
    h->X = (float2*)base;
    h->mhat = (float*)(base + l.mhat_off);
    h->part = (double*)(base + l.part_off);
    h->part_entries = (bytes - l.part_off) / ((size_t)h->stride * sizeof(double));
    h->ws_borrowed = true;
    return PM_OK;
}

namespace {

// Argument checks shared by phasemask_solve and phasemask_solve_noalloc.
pm_status check_solve_args(pm_plan* h, const float* target_amplitude, const float* init_phase, int n_iter,
                           const float* out_phase, const double* err_history) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!target_amplitude || !init_phase || !out_phase) return fail(PM_EINVAL, "null array argument");
    if (n_iter < 0) return fail(PM_EINVAL, "n_iter must be >= 0");
    if (misaligned(target_amplitude, 16)) return fail(PM_EINVAL, "target must be 16-byte aligned");
    if (misaligned(init_phase, 4) || misaligned(out_phase, 4) || misaligned(err_history, 8))
        return fail(PM_EINVAL, "misaligned array argument");
    const size_t nb = (size_t)h->N * sizeof(float);
    if (overlaps(out_phase, nb, target_amplitude, nb)) return fail(PM_EINVAL, "out_phase overlaps the target");
    if (err_history && overlaps(err_history, (2 * (size_t)n_iter + 1) * sizeof(double), target_amplitude, nb))
        return fail(PM_EINVAL, "err_history overlaps the target");
    return PM_OK;
}

}  // namespace

pm_status phasemask_solve(pm_handle h, const float* target_amplitude, const float* init_phase, int n_iter,
                          float* out_phase, double* err_history) {
    pm_status st = check_solve_args(h, target_amplitude, init_phase, n_iter, out_phase, err_history);
    if (st != PM_OK) return st;
    const bool hist = err_history != nullptr;
    if ((st = validate_input(h, target_amplitude, true, true, "target")) != PM_OK) return st;
    if ((st = validate_input(h, init_phase, false, false, "init_phase")) != PM_OK) return st;
    st = ensure_partials(h, hist ? 2 * (size_t)n_iter + 1 : 1);
    if (st != PM_OK) return st;
    pm::PmIo io{target_amplitude, init_phase, out_phase, err_history};
    PM_TRY(pm::launch_set_io(h->io, io, h->stream), "set io");
    if (h->flags & PM_FLAG_NO_GRAPH) return enqueue_solve(h, h->stream, n_iter, hist);
    return launch_graph(h, n_iter, hist);
}

namespace {

// Makes the uniform-batch buffers hold `batch` masks of `entries` history
// entries each (growing them synchronises the stream and drops the graphs).
pm_status ensure_many(pm_plan* h, int batch, size_t entries) {
    entries = std::max<size_t>(entries, 2);
    if (batch <= h->many_cap && entries <= h->many_entries) return PM_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    drop_graphs(h);
    const int cap = std::max(batch, h->many_cap);
    const size_t ent = std::max(entries, h->many_entries);
    const size_t n = (size_t)h->N * cap;
    float2* x = nullptr;
    float* m = nullptr;
    double* pm_ = nullptr;
    double* pt = nullptr;
    if ((e = hipMalloc(&x, n * sizeof(float2))) != hipSuccess || (e = hipMalloc(&m, n * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&pm_, (size_t)kNormGrid * cap * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&pt, ent * (size_t)h->stride * cap * sizeof(double))) != hipSuccess) {
        (void)hipFree(x);
        (void)hipFree(m);
        (void)hipFree(pm_);
        (void)hipFree(pt);
        return fail_hip(e, "hipMalloc(uniform batch)");
    }
    const size_t old_bytes = h->many_cap == 0 ? 0
        : (size_t)h->N * h->many_cap * (sizeof(float2) + sizeof(float)) + (size_t)kNormGrid * h->many_cap * sizeof(double) +
              h->many_entries * (size_t)h->stride * h->many_cap * sizeof(double);
    (void)hipFree(h->m_X);
    (void)hipFree(h->m_mhat);
    (void)hipFree(h->m_partm);
    (void)hipFree(h->m_part);
    h->m_X = x;
    h->m_mhat = m;
    h->m_partm = pm_;
    h->m_part = pt;
    h->many_cap = cap;
    h->many_entries = ent;
    h->ws_bytes = h->ws_bytes - old_bytes + n * (sizeof(float2) + sizeof(float)) + (size_t)kNormGrid * cap * sizeof(double) +
                  ent * (size_t)h->stride * cap * sizeof(double);
    return PM_OK;
}

}  // namespace

pm_status phasemask_solve_many(pm_handle h, int batch, const float* target_amplitude, const float* init_phase,
                               int n_iter, float* out_phase, double* err_history) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (batch < 1 || batch > 65535) return fail(PM_EINVAL, "batch must be in [1, 65535]");
    if ((long long)h->N * batch > 0x7fffffffLL)
        return fail(PM_EINVAL, "batch * height * width must be below 2^31 pixels");
    if (!target_amplitude || !init_phase || !out_phase) return fail(PM_EINVAL, "null array argument");
    if (n_iter < 0 || n_iter > (1 << 20)) return fail(PM_EINVAL, "n_iter must be in [0, 2^20]");
    if (misaligned(target_amplitude, 16)) return fail(PM_EINVAL, "target must be 16-byte aligned");
    if (misaligned(init_phase, 4) || misaligned(out_phase, 4) || misaligned(err_history, 8))
        return fail(PM_EINVAL, "misaligned array argument");
    const size_t nb = (size_t)h->N * batch * sizeof(float);
    const size_t hb = (2 * (size_t)n_iter + 1) * batch * sizeof(double);
    if (overlaps(out_phase, nb, target_amplitude, nb)) return fail(PM_EINVAL, "out_phase overlaps the target");
    if (err_history && (overlaps(err_history, hb, target_amplitude, nb) || overlaps(err_history, hb, out_phase, nb) ||
                        overlaps(err_history, hb, init_phase, nb)))
        return fail(PM_EINVAL, "err_history overlaps an array argument");
    const bool hist = err_history != nullptr;
    if ((st = validate_input(h, target_amplitude, true, false, "target", batch)) != PM_OK) return st;
    if ((st = validate_input(h, init_phase, false, false, "init_phase", batch)) != PM_OK) return st;
    if ((st = ensure_many(h, batch, hist ? 2 * (size_t)n_iter + 1 : 1)) != PM_OK) return st;
    pm::PmIo io{target_amplitude, init_phase, out_phase, err_history};
    PM_TRY(pm::launch_set_io(h->io, io, h->stream), "set io");
    if (h->flags & PM_FLAG_NO_GRAPH) return enqueue_many(h, h->stream, n_iter, hist, batch);
    SolveKey k;
    k.n_iter = n_iter;
    k.hist = hist;
    k.algo = kAlgoMany;
    k.batch = batch;
    return launch_graph(h, k);
}

// ----- allocation-free solve ----------------------------------------------------

// Scratch of phasemask_solve_noalloc: the iterate, the rescaled target, the
// target-norm partials, the pointer block and the FP64 error partials of one
// solve.  A file-scope device array: every GPU the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, never a device address; the kernels get the per-device address
// that hipGetSymbolAddress returns (scratch_address).
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
struct ScratchSlot {
    std::once_flag once;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[kMaxScratchDevices];

// Address of `scratch` on `device`, which must be the current device; looked
// up once per device and kept.
hipError_t scratch_address(int device, unsigned char** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    ScratchSlot& slot = g_scratch[device];
    std::call_once(slot.once, [&slot] { slot.err = hipGetSymbolAddress(&slot.ptr, HIP_SYMBOL(scratch)); });
    if (slot.err == hipSuccess) *out = static_cast<unsigned char*>(slot.ptr);
    return slot.err;
}

// Where one solve's buffers sit in the scratch array (each part 256-byte
// aligned); `end` is the bytes the solve needs.
struct NoAllocLayout {
    size_t x, mhat, part_m, io, part, end;
};
NoAllocLayout noalloc_layout(const pm_plan* h, size_t entries) {
    NoAllocLayout l{};
    size_t o = 0;
    l.x = o;
    o += align256((size_t)h->N * sizeof(float2));
    l.mhat = o;
    o += align256((size_t)h->N * sizeof(float));
    l.part_m = o;
    o += align256(kNormGrid * sizeof(double));
    l.io = o;
    o += align256(sizeof(pm::PmIo));
    l.part = o;
    o += entries * (size_t)h->stride * sizeof(double);
    l.end = o;
    return l;
}

// Points the plan's solve buffers at other memory for the lifetime of the
// object (the kernels take the pointers as launch arguments, so restoring
// them after the launches are enqueued is safe).
class BufferSwap {
  public:
    BufferSwap(pm_plan* h, float2* x, float* mhat, double* part_m, pm::PmIo* io, double* part)
        : h_(h), x_(h->X), mhat_(h->mhat), part_m_(h->part_m), io_(h->io), part_(h->part) {
        h->X = x;
        h->mhat = mhat;
        h->part_m = part_m;
        h->io = io;
        h->part = part;
    }
    ~BufferSwap() {
        h_->X = x_;
        h_->mhat = mhat_;
        h_->part_m = part_m_;
        h_->io = io_;
        h_->part = part_;
    }
    BufferSwap(const BufferSwap&) = delete;
    BufferSwap& operator=(const BufferSwap&) = delete;

  private:
    pm_plan* h_;
    float2* x_;
    float* mhat_;
    double* part_m_;
    pm::PmIo* io_;
    double* part_;
};

}  // namespace

pm_status phasemask_solve_noalloc(pm_handle h, const float* target_amplitude, const float* init_phase, int n_iter,
                                  float* out_phase, double* err_history) {
    pm_status st = check_solve_args(h, target_amplitude, init_phase, n_iter, out_phase, err_history);
    if (st != PM_OK) return st;
    if (h->scratch == nullptr)
        return fail(PM_EDEVICE, std::string("no address for the scratch array on this device: ") +
                                    hipGetErrorString(h->scratch_err));
    const bool hist = err_history != nullptr;
    const NoAllocLayout l = noalloc_layout(h, hist ? 2 * (size_t)n_iter + 1 : 1);
    if (l.end > kNoAllocScratchBytes) {
        std::ostringstream os;
        os << "a " << h->H << "x" << h->W << " solve of " << n_iter << " iterations"
           << (hist ? " with a history" : "") << " needs " << l.end
           << " bytes of scratch; the allocation-free solve has " << kNoAllocScratchBytes;
        return fail(PM_EINVAL, os.str());
    }
    unsigned char* base = h->scratch;
    BufferSwap swap(h, reinterpret_cast<float2*>(base + l.x), reinterpret_cast<float*>(base + l.mhat),
                    reinterpret_cast<double*>(base + l.part_m), reinterpret_cast<pm::PmIo*>(base + l.io),
                    reinterpret_cast<double*>(base + l.part));
    pm::PmIo io{target_amplitude, init_phase, out_phase, err_history};
    PM_TRY(pm::launch_set_io(h->io, io, h->stream), "set io");
    return enqueue_solve(h, h->stream, n_iter, hist);
}

pm_status phasemask_solve_field(pm_handle h, const float* target_amplitude, const void* init_field, int n_iter,
                                void* out_field, double* err_history) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!target_amplitude || !init_field || !out_field) return fail(PM_EINVAL, "null array argument");
    if (n_iter < 0) return fail(PM_EINVAL, "n_iter must be >= 0");
    if (misaligned(target_amplitude, 16)) return fail(PM_EINVAL, "target must be 16-byte aligned");
    if (misaligned(init_field, 8) || misaligned(out_field, 8) || misaligned(err_history, 8))
        return fail(PM_EINVAL, "misaligned array argument");
    const size_t nb = (size_t)h->N * sizeof(float);
    const size_t nf = (size_t)h->N * sizeof(float2);
    if (overlaps(out_field, nf, target_amplitude, nb)) return fail(PM_EINVAL, "out_field overlaps the target");
    const bool hist = err_history != nullptr;
    if (hist && overlaps(err_history, (2 * (size_t)n_iter + 1) * sizeof(double), target_amplitude, nb))
        return fail(PM_EINVAL, "err_history overlaps the target");
    if (hist && (overlaps(err_history, (2 * (size_t)n_iter + 1) * sizeof(double), out_field, nf) ||
                 overlaps(err_history, (2 * (size_t)n_iter + 1) * sizeof(double), init_field, nf)))
        return fail(PM_EINVAL, "err_history overlaps a field");
    if ((st = validate_input(h, target_amplitude, true, true, "target")) != PM_OK) return st;
    if ((st = validate_input(h, (const float*)init_field, false, false, "init_field", 2)) != PM_OK) return st;
    st = ensure_partials(h, hist ? 2 * (size_t)n_iter + 1 : 1);
    if (st != PM_OK) return st;
    pm::PmIo io{target_amplitude, nullptr, nullptr, err_history, (const float2*)init_field, (float2*)out_field};
    PM_TRY(pm::launch_set_io(h->io, io, h->stream), "set io");
    if (h->flags & PM_FLAG_NO_GRAPH) return enqueue_solve(h, h->stream, n_iter, hist, kAlgoGSField);
    return launch_graph(h, n_iter, hist, kAlgoGSField);
}

pm_status phasemask_solve_raar(pm_handle h, const float* target_amplitude, const float* init_phase, int n_iter,
                               double beta, float* out_phase, double* err_history) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!target_amplitude || !init_phase || !out_phase) return fail(PM_EINVAL, "null array argument");
    if (n_iter < 0) return fail(PM_EINVAL, "n_iter must be >= 0");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(PM_EINVAL, "beta must be in (0, 1]");
    if (misaligned(target_amplitude, 16)) return fail(PM_EINVAL, "target must be 16-byte aligned");
    if (misaligned(init_phase, 4) || misaligned(out_phase, 4) || misaligned(err_history, 8))
        return fail(PM_EINVAL, "misaligned array argument");
    const size_t nb = (size_t)h->N * sizeof(float);
    if (overlaps(out_phase, nb, target_amplitude, nb)) return fail(PM_EINVAL, "out_phase overlaps the target");
    const bool hist = err_history != nullptr;
    if (hist && overlaps(err_history, ((size_t)n_iter + 1) * sizeof(double), target_amplitude, nb))
        return fail(PM_EINVAL, "err_history overlaps the target");
    if ((st = validate_input(h, target_amplitude, true, true, "target")) != PM_OK) return st;
    if ((st = validate_input(h, init_phase, false, false, "init_phase")) != PM_OK) return st;
    st = ensure_partials(h, hist ? 2 * (size_t)n_iter + 1 : 1);
    if (st != PM_OK) return st;
    if (h->Z == nullptr) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
        drop_graphs(h);
        e = hipMalloc(&h->Z, (size_t)h->N * sizeof(float2));
        if (e != hipSuccess) return fail_hip(e, "hipMalloc(RAAR state)");
        h->ws_bytes += (size_t)h->N * sizeof(float2);
    }
    pm::PmIo io{target_amplitude, init_phase, out_phase, err_history};
    PM_TRY(pm::launch_set_io(h->io, io, h->stream), "set io");
    if (h->flags & PM_FLAG_NO_GRAPH) return enqueue_solve(h, h->stream, n_iter, hist, kAlgoRAAR, (float)beta);
    return launch_graph(h, n_iter, hist, kAlgoRAAR, (float)beta);
}

pm_status phasemask_error(pm_handle h, const float* target_amplitude, const float* phase, double* errors) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!target_amplitude || !phase || !errors) return fail(PM_EINVAL, "null array argument");
    if (misaligned(target_amplitude, 16)) return fail(PM_EINVAL, "target must be 16-byte aligned");
    if (misaligned(phase, 4) || misaligned(errors, 8)) return fail(PM_EINVAL, "misaligned array argument");
    if ((st = validate_input(h, target_amplitude, true, true, "target")) != PM_OK) return st;
    if ((st = validate_input(h, phase, false, false, "phase")) != PM_OK) return st;
    st = ensure_partials(h, 2);
    if (st != PM_OK) return st;
    pm::PmIo io{target_amplitude, phase, nullptr, errors};
    hipStream_t s = h->stream;
    PM_TRY(pm::launch_set_io(h->io, io, s), "set io");
    st = enqueue_target(h, s);
    if (st != PM_OK) return st;
    const RowLauncher row = kRowLaunch[len_slot(h->W)];
    const ColLauncher col = kColLaunch[len_slot(h->H)];
    PM_TRY(row(rmode(h, pm::ROW_INIT), row_params(h, nullptr), h->nwg_row, s, nullptr, nullptr), "row init");
    PM_TRY(col(pm::COL_ITER, col_params(h, h->part), h->nwg_col, s, nullptr, nullptr), "column pass");
    PM_TRY(row(rmode(h, pm::ROW_GAP), row_params(h, h->part + h->stride), h->nwg_row, s, nullptr, nullptr),
           "row gap");
    PM_TRY(pm::launch_finalize(h->part, h->stride, h->slots_col, h->slots_row, 1.0 / h->N, h->io, 0, 2, s, 1,
                               pnorm2(h)),
           "finalize");
    return PM_OK;
}

pm_status phasemask_fft2(pm_handle h, const void* in, void* out, int inverse) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!in || !out) return fail(PM_EINVAL, "null array argument");
    if (misaligned(in, 8) || misaligned(out, 8)) return fail(PM_EINVAL, "complex arrays must be 8-byte aligned");
    hipStream_t s = h->stream;
    const RowLauncher row = kRowLaunch[len_slot(h->W)];
    const ColLauncher col = kColLaunch[len_slot(h->H)];
    pm::RowParams rp = row_params(h, nullptr);
    pm::ColParams cp = col_params(h, nullptr);
    if (!inverse) {
        rp.nat_in = (const float2*)in;
        cp.nat_out = (float2*)out;
        PM_TRY(row(pm::ROW_FFT_FWD, rp, h->nwg_row, s, nullptr, nullptr), "row fft");
        PM_TRY(col(pm::COL_FFT_FWD, cp, h->nwg_col, s, nullptr, nullptr), "column fft");
    } else {
        cp.nat_in = (const float2*)in;
        rp.nat_out = (float2*)out;
        PM_TRY(col(pm::COL_FFT_INV, cp, h->nwg_col, s, nullptr, nullptr), "column ifft");
        PM_TRY(row(pm::ROW_FFT_INV, rp, h->nwg_row, s, nullptr, nullptr), "row ifft");
    }
    return PM_OK;
}

pm_status phasemask_create_batched(pm_handle* out, int count, const int* heights, const int* widths,
                                   unsigned flags, void* stream) {
    if (out == nullptr) return fail(PM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || heights == nullptr || widths == nullptr) return fail(PM_EINVAL, "need count >= 1 and sizes");
    if ((flags & ~(PM_FLAG_NO_GRAPH | PM_FLAG_NO_TUNE)) != 0) return fail(PM_EINVAL, "unknown flag bits");
    for (int i = 0; i < count; ++i)
        if (!batch_len_ok(heights[i]) || !batch_len_ok(widths[i]))
            return fail(PM_EUNSUPPORTED, "batched sizes must be powers of two in [64, 1024]");
    pm_plan* h = new (std::nothrow) pm_plan;
    if (h == nullptr) return fail(PM_ENOMEM, "host allocation failed");
    h->batched = true;
    h->count = count;
    h->flags = flags;
    h->stream = (hipStream_t)stream;
    h->group_bytes = kBatchGroupBytes;
    if (const char* g = std::getenv("PHASEMASK_GROUP_MB"); g != nullptr && g[0] != '\0') {
        const long mb = std::atol(g);
        if (mb < 0 || mb > (1L << 20)) {
            delete h;
            return fail(PM_EINVAL, "PHASEMASK_GROUP_MB out of range");
        }
        h->group_bytes = (size_t)mb << 20;
    }
    h->chains = kBatchChains;
    if (const char* c = std::getenv("PHASEMASK_CHAINS"); c != nullptr && c[0] != '\0') {
        const long n = std::atol(c);
        if (n < 1 || n > 8) {
            delete h;
            return fail(PM_EINVAL, "PHASEMASK_CHAINS out of range");
        }
        h->chains = (int)n;
    }
    auto bail = [&](hipError_t e, const char* what) {
        pm_status st = fail_hip(e, what);
        free_plan(h);
        return st;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(e, "hipGetDevice");

    // Work order: larger masks first, so their work-groups start first.
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (long)heights[a] * widths[a] > (long)heights[b] * widths[b];
    });
    size_t off = 0;
    std::vector<size_t> xoff(count), moff(count);
    for (int i = 0; i < count; ++i) {
        const size_t n = (size_t)heights[i] * widths[i];
        xoff[i] = off;
        off += ((n * sizeof(float2) + 255) / 256) * 256;
        moff[i] = off;
        off += ((n * sizeof(float) + 255) / 256) * 256;
    }
    if ((e = hipMalloc(&h->batch_ws, off)) != hipSuccess) return bail(e, "hipMalloc(batch workspace)");
    h->batch_ws_bytes = off;
    std::vector<float2*> xs(count);
    std::vector<float*> ms(count);
    for (int i = 0; i < count; ++i) {
        xs[i] = (float2*)((char*)h->batch_ws + xoff[i]);
        ms[i] = (float*)((char*)h->batch_ws + moff[i]);
    }
    std::vector<BatchLayout> layouts;
    size_t max_col = 0, max_row = 0;
    for (int sc = 0; sc < pm::kBatchSchedules; ++sc) {
        layouts.push_back(batch_layout(sc, count, heights, widths, order, xs, ms));
        max_col = std::max(max_col, layouts.back().col.size());
        max_row = std::max(max_row, layouts.back().row.size());
    }
    std::vector<pm::BatchTask> prep;
    std::vector<int> prep0(count);
    for (int i : order) {
        prep0[i] = (int)prep.size();
        for (int p0 = 0; p0 < heights[i] * widths[i]; p0 += pm::kPrepPixels) prep.push_back(pm::BatchTask{i, p0});
    }
    h->n_prep_tasks = (int)prep.size();
    const size_t npart = std::max(max_col, max_row) * pm::red_slots(pm::kBatchThreads);
    if ((e = hipMalloc(&h->masks, count * sizeof(pm::BatchMask))) != hipSuccess) return bail(e, "hipMalloc(masks)");
    if ((e = hipMalloc(&h->col_tasks, max_col * sizeof(pm::BatchTask))) != hipSuccess) return bail(e, "hipMalloc(tasks)");
    if ((e = hipMalloc(&h->row_tasks, max_row * sizeof(pm::BatchTask))) != hipSuccess) return bail(e, "hipMalloc(tasks)");
    if ((e = hipMalloc(&h->prep_tasks, prep.size() * sizeof(pm::BatchTask))) != hipSuccess) return bail(e, "hipMalloc(tasks)");
    if ((e = hipMalloc(&h->mask_prep0, count * sizeof(int))) != hipSuccess) return bail(e, "hipMalloc(prep index)");
    if ((e = hipMalloc(&h->part, npart * sizeof(double))) != hipSuccess) return bail(e, "hipMalloc(partials)");
    if ((e = hipMalloc(&h->part_m, prep.size() * sizeof(double))) != hipSuccess) return bail(e, "hipMalloc(norm)");
    if ((e = hipMalloc(&h->bio, sizeof(pm::BatchIo))) != hipSuccess) return bail(e, "hipMalloc(io)");
    const std::vector<float2> tw = pm::batch_twiddles();
    if ((e = hipMalloc(&h->tw_batch, tw.size() * sizeof(float2))) != hipSuccess) return bail(e, "hipMalloc(twiddles)");
    h->part_entries = 1;
    h->stride = (int)npart;
    if ((e = hipMemcpy(h->prep_tasks, prep.data(), prep.size() * sizeof(pm::BatchTask), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(h->mask_prep0, prep0.data(), count * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(h->tw_batch, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "hipMemcpy(plan)");
    if ((e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(e, "hipStreamCreate");
    for (int c = 1; c < h->chains; ++c) {
        hipStream_t x = nullptr;
        hipEvent_t f = nullptr, j = nullptr;
        if ((e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking)) != hipSuccess) return bail(e, "hipStreamCreate");
        h->side.push_back(x);
        if ((e = hipEventCreateWithFlags(&f, hipEventDisableTiming)) != hipSuccess) return bail(e, "hipEventCreate");
        h->fork_ev.push_back(f);
        if ((e = hipEventCreateWithFlags(&j, hipEventDisableTiming)) != hipSuccess) return bail(e, "hipEventCreate");
        h->join_ev.push_back(j);
    }
    const std::string key = tune_key(h->device, count, heights, widths);
    pm_status ts = tune_batch(h, layouts, key);
    if (ts != PM_OK) {
        free_plan(h);
        return ts;
    }
    if ((e = upload_layout(h, layouts[h->sched])) != hipSuccess) return bail(e, "hipMemcpy(layout)");
    h->ws_bytes = off + npart * sizeof(double) + prep.size() * (sizeof(double) + sizeof(pm::BatchTask)) +
                  (max_col + max_row) * sizeof(pm::BatchTask) + count * (sizeof(pm::BatchMask) + sizeof(int)) +
                  sizeof(pm::BatchIo) + tw.size() * sizeof(float2);
    plan_register(h);
    *out = h;
    return PM_OK;
}

pm_status phasemask_solve_batched(pm_handle h, const float* const* targets, const float* const* init_phases,
                                  int n_iter, float* const* out_phases, double* final_err) {
    pm_status st = check_handle(h, true);
    if (st != PM_OK) return st;
    if (!targets || !init_phases || !out_phases) return fail(PM_EINVAL, "null pointer-array argument");
    if (n_iter < 0) return fail(PM_EINVAL, "n_iter must be >= 0");
    if (misaligned(targets, 8) || misaligned(init_phases, 8) || misaligned(out_phases, 8) ||
        misaligned(final_err, 8))
        return fail(PM_EINVAL, "misaligned argument");
    pm::BatchIo io{targets, init_phases, out_phases, final_err};
    PM_TRY(pm::launch_set_batch_io(h->bio, io, h->stream), "set batch io");
    const bool err = final_err != nullptr;
    if (h->flags & PM_FLAG_NO_GRAPH) return enqueue_batch(h, h->stream, n_iter, err);
    return launch_graph(h, n_iter, err);
}

pm_status phasemask_intensity_loss_fwd(pm_handle h, int batch, const float* phase,
                                       const float* target_intensity, double* loss, void* saved) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!phase || !target_intensity || !loss || !saved) return fail(PM_EINVAL, "null array argument");
    if (batch < 1 || batch > 65535) return fail(PM_EINVAL, "batch must be in [1, 65535]");
    if (misaligned(phase, 4) || misaligned(target_intensity, 4) || misaligned(loss, 8) || misaligned(saved, 8))
        return fail(PM_EINVAL, "misaligned array argument");
    st = ensure_partials(h, (size_t)batch);
    if (st != PM_OK) return st;
    pm::AdjParams p{};
    p.saved = (float2*)saved;
    p.phase = phase;
    p.inten = target_intensity;
    p.part = h->part;
    p.twW = h->twW;
    p.twH = h->twH;
    p.H = h->H;
    p.W = h->W;
    p.nwg = h->slots_adj;
    hipStream_t s = h->stream;
    PM_TRY(kAdjRow[len_slot(h->W)](pm::ROW_INIT, p, batch, s), "loss row pass");
    PM_TRY(kAdjCol[len_slot(h->H)](pm::COL_LOSS, p, batch, s), "loss column pass");
    PM_TRY(pm::launch_sum_rows(h->part, h->slots_adj, loss, batch, s), "loss sum");
    return PM_OK;
}

pm_status phasemask_intensity_loss_bwd(pm_handle h, int batch, const float* phase, const void* saved,
                                       const double* grad_loss, float* grad_phase) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!phase || !saved || !grad_loss || !grad_phase) return fail(PM_EINVAL, "null array argument");
    if (batch < 1 || batch > 65535) return fail(PM_EINVAL, "batch must be in [1, 65535]");
    if (misaligned(phase, 4) || misaligned(saved, 8) || misaligned(grad_loss, 8) || misaligned(grad_phase, 4))
        return fail(PM_EINVAL, "misaligned array argument");
    pm::AdjParams p{};
    p.saved = (float2*)saved;
    p.phase = phase;
    p.grad = grad_phase;
    p.grad_loss = grad_loss;
    p.twW = h->twW;
    p.twH = h->twH;
    p.H = h->H;
    p.W = h->W;
    p.nwg = h->slots_adj;
    PM_TRY(kAdjRow[len_slot(h->W)](pm::ROW_GRAD, p, batch, h->stream), "gradient row pass");
    return PM_OK;
}

// ----- Adam solves on the intensity loss -------------------------------------

// The whole Adam solve after the pointer block is set: set-up, the row
// transform of exp(i phi^0), then per step the loss column pass (loss of
// phi^{k-1}, residual-weighted field back through the inverse column
// transform) and the Adam row pass (inverse row transform, gradient, update
// to phi^k, forward row transform of exp(i phi^k)); with a history, the loss
// of phi^n and the fixed-order sums; finally the phase to the caller.
namespace {

pm::AdjParams adam_params(pm_plan* h, const SolveKey& k) {
    pm::AdjParams p{};
    p.saved = h->a_saved;
    p.phase = h->a_phase;
    p.grad = h->a_phase;  // the update is in place
    p.inten = h->a_inten;
    p.part = h->part;
    p.twW = h->twW;
    p.twH = h->twH;
    p.H = h->H;
    p.W = h->W;
    p.nwg = h->slots_adj;
    p.am = h->a_m;
    p.av = h->a_v;
    p.beta1 = (float)k.beta1;
    p.beta2 = (float)k.beta2;
    p.eps = (float)k.eps;
    return p;
}

// The samples are independent: contiguous groups of them run their steps
// on concurrent chains, so that one chain's kernel boundaries overlap
// another's passes.  Each sample keeps its own buffers and partial rows, so
// the results do not depend on the grouping.  This is chain k.chain of
// k.chains: the row transform of exp(i phi^0), the steps and (with a
// history) the loss of phi^n of its samples, all on stream s.
pm_status enqueue_adam_chain(pm_plan* h, hipStream_t s, const SolveKey& k) {
    const int batch = k.batch, n = k.n_iter, c = k.chain;
    const int b0 = (int)((long)batch * c / k.chains);
    const int gb = (int)((long)batch * (c + 1) / k.chains) - b0;
    if (gb == 0) return PM_OK;
    pm::AdjParams q = adam_params(h, k);
    const size_t off = (size_t)b0 * h->N;
    q.saved += off;
    q.phase += off;
    q.grad += off;
    q.inten += off;
    q.am += off;
    q.av += off;
    const AdjRowLauncher row = kAdjRow[len_slot(h->W)];
    const AdjColLauncher col = kAdjCol[len_slot(h->H)];
    if (n > 0 || k.hist) PM_TRY(row(pm::ROW_INIT, q, gb, s), "Adam row init");
    for (int step = 1; step <= n; ++step) {
        q.part_row0 = (k.hist ? (step - 1) * batch : 0) + b0;
        PM_TRY(col(pm::COL_LOSS_T, q, gb, s), "Adam loss column pass");
        // bias corrections of step k (evaluated in double, rounded once)
        q.adam_step = (float)(k.lr / (1.0 - std::pow(k.beta1, (double)step)));
        q.adam_bc2s = (float)std::sqrt(1.0 - std::pow(k.beta2, (double)step));
        const int mode = (step < n || k.hist) ? pm::ROW_ADAM : pm::ROW_ADAM_LAST;
        PM_TRY(row(mode, q, gb, s), "Adam row pass");
    }
    if (k.hist) {
        q.part_row0 = n * batch + b0;
        PM_TRY(col(pm::COL_LOSS_ONLY_T, q, gb, s), "Adam final loss");
    }
    return PM_OK;
}

// The whole Adam solve after the pointer block is set: set-up of all
// samples on s, the chains (chain 0 on s, the others on side streams forked
// from s and joined back; each a captured graph of its own unless
// PM_FLAG_NO_GRAPH, so that every graph stays a single chain of kernels),
// then the fixed-order loss sums and the phases to the caller.  With one
// chain and graphs, all of it is one captured graph.
pm_status enqueue_adam(pm_plan* h, hipStream_t s, const SolveKey& k, bool graphs) {
    const int batch = k.batch, n = k.n_iter;
    // one chain: the whole solve is one graph
    if (graphs && std::min(h->adam_chains, batch) == 1) return launch_graph(h, k, s);
    PM_TRY(pm::launch_adam_prep(h->io, h->H, h->W, batch, h->a_phase, h->a_inten, h->a_m, h->a_v, s),
           "Adam set-up");
    const int chains = std::min(h->adam_chains, batch);
    for (int c = 1; c < chains; ++c) {
        PM_TRY(hipEventRecord(h->fork_ev[c - 1], s), "hipEventRecord(fork)");
        PM_TRY(hipStreamWaitEvent(h->side[c - 1], h->fork_ev[c - 1], 0), "hipStreamWaitEvent(fork)");
    }
    for (int c = 0; c < chains; ++c) {
        SolveKey kc = k;
        kc.chain = c;
        kc.chains = chains;
        hipStream_t cs = c == 0 ? s : h->side[c - 1];
        pm_status st = graphs ? launch_graph(h, kc, cs) : enqueue_adam_chain(h, cs, kc);
        if (st != PM_OK) return st;
    }
    for (int c = 1; c < chains; ++c) {
        PM_TRY(hipEventRecord(h->join_ev[c - 1], h->side[c - 1]), "hipEventRecord(join)");
        PM_TRY(hipStreamWaitEvent(s, h->join_ev[c - 1], 0), "hipStreamWaitEvent(join)");
    }
    if (k.hist)
        PM_TRY(pm::launch_sum_rows_io(h->part, h->slots_adj, h->io, (n + 1) * batch, s), "Adam loss sums");
    PM_TRY(pm::launch_adam_out(h->io, h->a_phase, (size_t)batch * h->N, s), "Adam output");
    return PM_OK;
}

pm_status enqueue_adam(pm_plan* h, hipStream_t s, const SolveKey& k) { return enqueue_adam(h, s, k, false); }

}  // namespace

pm_status phasemask_solve_adam(pm_handle h, int batch, const float* target_intensity, const float* init_phase,
                               int n_steps, double lr, double beta1, double beta2, double eps, float* out_phase,
                               double* loss_history) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!target_intensity || !init_phase || !out_phase) return fail(PM_EINVAL, "null array argument");
    if (batch < 1 || batch > 65535) return fail(PM_EINVAL, "batch must be in [1, 65535]");
    if (n_steps < 0) return fail(PM_EINVAL, "n_steps must be >= 0");
    if (!(lr > 0.0 && std::isfinite(lr))) return fail(PM_EINVAL, "lr must be positive and finite");
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0))
        return fail(PM_EINVAL, "beta1 and beta2 must be in [0, 1)");
    if (!(eps > 0.0 && std::isfinite(eps))) return fail(PM_EINVAL, "eps must be positive and finite");
    if (misaligned(target_intensity, 16) || misaligned(init_phase, 16) || misaligned(out_phase, 16) ||
        misaligned(loss_history, 8))
        return fail(PM_EINVAL, "target_intensity, init_phase and out_phase must be 16-byte aligned");
    const size_t nb = (size_t)batch * h->N * sizeof(float);
    if (overlaps(out_phase, nb, target_intensity, nb)) return fail(PM_EINVAL, "out_phase overlaps the target");
    const size_t hb = ((size_t)n_steps + 1) * batch * sizeof(double);
    if (loss_history && (overlaps(loss_history, hb, target_intensity, nb) || overlaps(loss_history, hb, out_phase, nb) ||
                         overlaps(loss_history, hb, init_phase, nb)))
        return fail(PM_EINVAL, "loss_history overlaps an array");
    // concurrent chains (PHASEMASK_ADAM_CHAINS=<1..8>, default kAdamChains),
    // chosen at the handle's first Adam solve
    int chains = h->adam_chains;
    if (chains == 0) {
        chains = kAdamChains;
        if (const char* c = std::getenv("PHASEMASK_ADAM_CHAINS"); c != nullptr && c[0] != '\0') {
            const long v = std::atol(c);
            if (v < 1 || v > 8) return fail(PM_EINVAL, "PHASEMASK_ADAM_CHAINS out of range");
            chains = (int)v;
        }
    }
    if (h->adam_cap < batch) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
        drop_graphs(h);  // captured graphs hold the old buffers
        const size_t n = (size_t)batch * h->N;
        float2* sv = nullptr;
        float *ph = nullptr, *m = nullptr, *v = nullptr, *it = nullptr;
        e = hipMalloc(&sv, n * sizeof(float2));
        if (e == hipSuccess) e = hipMalloc(&ph, n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&m, n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&v, n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&it, n * sizeof(float));
        if (e != hipSuccess) {
            (void)hipFree(sv);
            (void)hipFree(ph);
            (void)hipFree(m);
            (void)hipFree(v);
            (void)hipFree(it);
            return fail_hip(e, "hipMalloc(Adam state)");
        }
        const size_t old = (size_t)h->adam_cap * h->N * (sizeof(float2) + 4 * sizeof(float));
        (void)hipFree(h->a_saved);
        (void)hipFree(h->a_phase);
        (void)hipFree(h->a_m);
        (void)hipFree(h->a_v);
        (void)hipFree(h->a_inten);
        h->a_saved = sv;
        h->a_phase = ph;
        h->a_m = m;
        h->a_v = v;
        h->a_inten = it;
        h->ws_bytes += n * (sizeof(float2) + 4 * sizeof(float)) - old;
        h->adam_cap = batch;
    }
    if (h->adam_chains == 0) {
        // a side stream with its fork and join events per chain after the first
        for (int c = (int)h->side.size() + 1; c < chains; ++c) {
            hipStream_t x = nullptr;
            hipEvent_t f = nullptr, j = nullptr;
            hipError_t e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&f, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
            if (e != hipSuccess) {
                if (x) (void)hipStreamDestroy(x);
                if (f) (void)hipEventDestroy(f);
                if (j) (void)hipEventDestroy(j);
                return fail_hip(e, "side stream of an Adam chain");
            }
            h->side.push_back(x);
            h->fork_ev.push_back(f);
            h->join_ev.push_back(j);
        }
        h->adam_chains = chains;
    }
    const bool hist = loss_history != nullptr;
    const size_t rows = hist ? ((size_t)n_steps + 1) * batch : (size_t)batch;
    st = ensure_partials(h, (rows * h->slots_adj + h->stride - 1) / h->stride);
    if (st != PM_OK) return st;
    pm::PmIo io{target_intensity, init_phase, out_phase, loss_history};
    PM_TRY(pm::launch_set_io(h->io, io, h->stream), "set io");
    SolveKey k;
    k.n_iter = n_steps;
    k.hist = hist;
    k.algo = kAlgoAdam;
    k.batch = batch;
    k.lr = lr;
    k.beta1 = beta1;
    k.beta2 = beta2;
    k.eps = eps;
    return enqueue_adam(h, h->stream, k, (h->flags & PM_FLAG_NO_GRAPH) == 0);
}

pm_status phasemask_initial_phase(pm_handle h, const float* target_amplitude, double t_dark, float* out_phase) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!target_amplitude || !out_phase) return fail(PM_EINVAL, "null array argument");
    if (misaligned(target_amplitude, 16) || misaligned(out_phase, 4)) return fail(PM_EINVAL, "misaligned array argument");
    if (!(t_dark >= 0.0 && t_dark < 1.0)) return fail(PM_EINVAL, "t_dark must be in [0, 1)");
    if (overlaps(out_phase, (size_t)h->N * sizeof(float), target_amplitude, (size_t)h->N * sizeof(float)))
        return fail(PM_EINVAL, "out_phase overlaps the target");
    if ((st = validate_input(h, target_amplitude, true, true, "target")) != PM_OK) return st;
    hipStream_t s = h->stream;
    pm::PmIo io{target_amplitude, nullptr, out_phase, nullptr};
    PM_TRY(pm::launch_set_io(h->io, io, s), "set io");
    PM_TRY(pm::launch_max_partial(target_amplitude, h->N, h->part_mx, kNormGrid, s), "target max");
    pm::ColParams cp = col_params(h, nullptr);
    cp.tnat = target_amplitude;
    cp.tmax_part = h->part_mx;
    cp.ntmax = kNormGrid;
    cp.t_dark = t_dark;
    const RowLauncher row = kRowLaunch[len_slot(h->W)];
    const ColLauncher col = kColLaunch[len_slot(h->H)];
    PM_TRY(col(pm::COL_INIT_BIT, cp, h->nwg_col, s, nullptr, nullptr), "1-bit inverse column pass");
    PM_TRY(row(pm::ROW_LAST_NE, row_params(h, nullptr), h->nwg_row, s, nullptr, nullptr), "inverse row pass");
    return PM_OK;
}

pm_status phasemask_physical_error(pm_handle h, const float* target_amplitude, const float* phase, double t_lit,
                                   double t_dark, double* errors) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!target_amplitude || !phase || !errors) return fail(PM_EINVAL, "null array argument");
    if (misaligned(target_amplitude, 16) || misaligned(phase, 4) || misaligned(errors, 8))
        return fail(PM_EINVAL, "misaligned array argument");
    if (!(t_lit > 0.0) || !(t_dark >= 0.0 && t_dark < 1.0)) return fail(PM_EINVAL, "need t_lit > 0, 0 <= t_dark < 1");
    if ((st = validate_input(h, target_amplitude, true, true, "target")) != PM_OK) return st;
    if ((st = validate_input(h, phase, false, false, "phase")) != PM_OK) return st;
    st = ensure_partials(h, min_partial_entries(h));
    if (st != PM_OK) return st;
    if (h->pw == nullptr) {
        hipError_t e = hipMalloc(&h->pw, (size_t)h->N * sizeof(float));
        if (e != hipSuccess) return fail_hip(e, "hipMalloc(power)");
        h->ws_bytes += (size_t)h->N * sizeof(float);
    }
    hipStream_t s = h->stream;
    pm::PmIo io{target_amplitude, phase, nullptr, nullptr};
    PM_TRY(pm::launch_set_io(h->io, io, s), "set io");
    PM_TRY(pm::launch_max_partial(target_amplitude, h->N, h->part_mx, kNormGrid, s), "target max");
    const RowLauncher row = kRowLaunch[len_slot(h->W)];
    const ColLauncher col = kColLaunch[len_slot(h->H)];
    PM_TRY(row(rmode(h, pm::ROW_INIT), row_params(h, nullptr), h->nwg_row, s, nullptr, nullptr), "row init");
    pm::ColParams cp = col_params(h, h->part);
    cp.pw = h->pw;
    PM_TRY(col(pm::COL_POW, cp, h->nwg_col, s, nullptr, nullptr), "power column pass");
    PM_TRY(pm::launch_physical_error(h->pw, h->part, h->slots_col, target_amplitude, h->part_mx, kNormGrid, h->H,
                                     h->W, t_lit, t_dark, h->part + h->stride, errors, s),
           "physical error");
    return PM_OK;
}

pm_status phasemask_probe_dft16(int matrix_units, const void* in, void* out, int waves, int reps, float* ms) {
    if (!in || !out || !ms) return fail(PM_EINVAL, "null argument");
    if (waves < 4 || waves > (1 << 20) || waves % 4 != 0) return fail(PM_EINVAL, "waves must be a multiple of 4 in [4, 2^20]");
    if (reps < 2 || reps > (1 << 20) || reps % 2 != 0) return fail(PM_EINVAL, "reps must be even, in [2, 2^20]");
    if (misaligned(in, 8) || misaligned(out, 8)) return fail(PM_EINVAL, "misaligned array argument");
    if (overlaps(in, (size_t)waves * 1024 * sizeof(float2), out, (size_t)waves * 1024 * sizeof(float2)))
        return fail(PM_EINVAL, "out overlaps in");
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess)
        e = pm::launch_probe_dft16(matrix_units != 0, (const float2*)in, (float2*)out, waves, reps, nullptr, a, b);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail_hip(e, "DFT-16 probe");
    return PM_OK;
}

#ifdef PM_TIMELINE
// Rate of the device wall clock the timeline records count (kHz), or -1.
extern "C" int phasemask_timeline_clock_khz() {
    int khz = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return -1;
    return khz;
}
#endif

int phasemask_batch_schedule(pm_handle h) { return (h != nullptr && plan_live(h) && h->batched) ? h->sched : -1; }

pm_status phasemask_batch_config(pm_handle h, int* schedule, int* chains, size_t* group_bytes) {
    pm_status st = check_any(h);
    if (st != PM_OK) return st;
    if (!h->batched) return fail(PM_ESTATE, "handle is not a batched plan");
    if (schedule) *schedule = h->sched;
    if (chains) *chains = h->chains;
    if (group_bytes) *group_bytes = h->group_bytes;
    return PM_OK;
}

pm_status phasemask_probe_exchange(pm_handle h, void* buffer, int reps, float* ms) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!buffer || !ms) return fail(PM_EINVAL, "null argument");
    if (reps < 1 || reps > 10000) return fail(PM_EINVAL, "reps must be in [1, 10000]");
    if (misaligned(buffer, 16)) return fail(PM_EINVAL, "buffer must be 16-byte aligned");
    const RowLauncher row = kRowLaunch[len_slot(h->W)];
    const ColLauncher col = kColLaunch[len_slot(h->H)];
    pm::ColParams cp = col_params(h, h->part);
    pm::RowParams rp = row_params(h, nullptr);
    cp.X = (float2*)buffer;
    rp.X = (float2*)buffer;
    // The pairs go into one graph (captured per call: the buffer is a kernel
    // argument), launched once untimed and once between the events.
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail_hip(e, "hipStreamBeginCapture(exchange)");
    hipError_t el = hipSuccess;
    for (int r = 0; r < reps && el == hipSuccess; ++r) {
        el = col(pm::COL_COPY, cp, h->nwg_col, h->cap_stream, nullptr, nullptr);
        if (el == hipSuccess) el = row(pm::ROW_COPY, rp, h->nwg_row, h->cap_stream, nullptr, nullptr);
    }
    e = hipStreamEndCapture(h->cap_stream, &graph);
    if (el != hipSuccess) {
        cleanup();
        return fail_hip(el, "exchange pass");
    }
    if (e != hipSuccess) {
        cleanup();
        return fail_hip(e, "hipStreamEndCapture(exchange)");
    }
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) == hipSuccess &&
        (e = hipEventCreate(&e0)) == hipSuccess && (e = hipEventCreate(&e1)) == hipSuccess &&
        (e = hipGraphLaunch(exec, h->stream)) == hipSuccess && (e = hipEventRecord(e0, h->stream)) == hipSuccess &&
        (e = hipGraphLaunch(exec, h->stream)) == hipSuccess && (e = hipEventRecord(e1, h->stream)) == hipSuccess &&
        (e = hipEventSynchronize(e1)) == hipSuccess)
        e = hipEventElapsedTime(ms, e0, e1);
    cleanup();
    if (e != hipSuccess) return fail_hip(e, "exchange probe");
    return PM_OK;
}

pm_status phasemask_time_passes(pm_handle h, const float* target_amplitude, const float* phase, int reps,
                                float* col_ms, float* row_ms) {
    pm_status st = check_handle(h);
    if (st != PM_OK) return st;
    if (!target_amplitude || !phase || !col_ms || !row_ms) return fail(PM_EINVAL, "null argument");
    if (reps < 1 || reps > 100000) return fail(PM_EINVAL, "reps must be in [1, 100000]");
    if (misaligned(target_amplitude, 16)) return fail(PM_EINVAL, "target must be 16-byte aligned");
    if (misaligned(phase, 4)) return fail(PM_EINVAL, "misaligned array argument");
    st = ensure_partials(h, 2);
    if (st != PM_OK) return st;
    hipStream_t s = h->stream;
    pm::PmIo io{target_amplitude, phase, nullptr, nullptr};
    PM_TRY(pm::launch_set_io(h->io, io, s), "set io");
    st = enqueue_target(h, s);
    if (st != PM_OK) return st;
    const RowLauncher row = kRowLaunch[len_slot(h->W)];
    const ColLauncher col = kColLaunch[len_slot(h->H)];
    PM_TRY(row(rmode(h, pm::ROW_INIT), row_params(h, nullptr), h->nwg_row, s, nullptr, nullptr), "row init");
    std::vector<hipEvent_t> ev(4 * (size_t)reps, nullptr);
    auto cleanup = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (auto& e : ev) {
        hipError_t ee = hipEventCreate(&e);
        if (ee != hipSuccess) {
            cleanup();
            return fail_hip(ee, "hipEventCreate");
        }
    }
    hipError_t err = hipSuccess;
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        err = col(pm::COL_ITER, col_params(h, h->part), h->nwg_col, s, ev[4 * r], ev[4 * r + 1]);
        if (err == hipSuccess)
            err = row(rmode(h, pm::ROW_ITER), row_params(h, h->part + h->stride), h->nwg_row, s, ev[4 * r + 2],
                      ev[4 * r + 3]);
    }
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    double tc = 0.0, tr = 0.0;
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        float a = 0.f, b = 0.f;
        err = hipEventElapsedTime(&a, ev[4 * r], ev[4 * r + 1]);
        if (err == hipSuccess) err = hipEventElapsedTime(&b, ev[4 * r + 2], ev[4 * r + 3]);
        tc += a;
        tr += b;
    }
    cleanup();
    if (err != hipSuccess) return fail_hip(err, "timed passes");
    *col_ms = (float)(tc / reps);
    *row_ms = (float)(tr / reps);
    return PM_OK;
}

}  // extern "C"
