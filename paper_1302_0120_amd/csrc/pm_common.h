// pm_common.h -- types shared by the host plan code and the kernel
// translation units (no kernels here).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pm {

// Iterate layout in device memory ("strip-tiled"): the [H][W] complex field is
// split into W/kC strips of kC adjacent columns; strip s is stored as a
// contiguous [H][kC] block, so element (y, x) sits at
//     ((x / kC) * H + y) * kC + (x % kC).
// A column pass reads one strip as one contiguous block; a row pass that
// owns G adjacent rows reads G*kC contiguous elements per strip (128 bytes
// for 4 rows; with 2-row work-groups the two halves of each 128-byte line
// are read by two work-groups placed on one XCD, pass_tile).  The
// rescaled target uses the same layout.
// Reduction groups of a work-group of NT threads: the largest power of two
// that divides NT, at most one wave.  A group is a run of whole lanes, so
// in-group shuffles never read an inactive lane (a work-group of 80 threads
// is one full wave and a quarter wave: five groups of 16).  The passes write
// one FP64 partial per group (red_slots(NT) per work-group), so no
// work-group barrier is needed for their sums.
__host__ __device__ constexpr int red_width(int NT) { return (NT & -NT) < 64 ? (NT & -NT) : 64; }
__host__ __device__ constexpr int red_slots(int NT) { return NT / red_width(NT); }

constexpr int kC = 4;    // columns per strip = columns per column work-group
#ifndef PM_KGR
#define PM_KGR 4
#endif
constexpr int kGR = PM_KGR;  // rows per row work-group (a tuning knob)

// Per-call pointers.  Kernels replayed from a captured graph read them from
// this device-resident block, which a one-thread kernel rewrites before each
// replay, so one graph serves any caller buffers.
struct PmIo {
    const float* target;   // [H][W] target amplitude m
    const float* phase_in; // [H][W] initial phase
    float* phase_out;      // [H][W] output phase
    double* hist;          // error history (or the two errors of a mask), may be null
    const float2* field_in;  // [H][W] complex initial field u^0 (field solves)
    float2* field_out;       // [H][W] complex output field u^n (field solves)
};

// Row-pass modes (bit sets).
enum : int {
    RIN_PHASE = 1,    // read a phase image, form exp(i phi)
    RIN_TILED = 2,    // read the tiled iterate
    RIN_NAT = 4,      // read a natural-layout complex image
    R_INV = 8,        // inverse row transform
    R_PS = 16,        // P_S (Eq. 4a) + gap partial sum
    R_FWD = 32,       // forward row transform, write the tiled iterate
    ROUT_PHASE = 64,  // write atan2 of the projected field
    ROUT_NAT = 128,   // write a natural-layout complex image
    R_NOERR = 256,    // P_S without the gap partial sum
    ROUT_GRAD = 512,  // intensity-loss gradient 4 gscale Im(e^{-i phi} g)
    R_RAAR = 1024,    // RAAR update of the SLM-plane point x (kept in Z) from w = P_M x
    R_STOREZ = 2048,  // store the initial field to Z (RAAR start)
    R_ILLUM = 4096,   // illumination amplitude p of Eq. 1 on S (else p = 1)
    RIN_FIELD = 8192,   // read the natural-layout complex field io->field_in (as RIN_NAT)
    ROUT_FIELD = 16384, // write the natural-layout complex field to io->field_out (as ROUT_NAT)
    R_ADAM = 32768,     // intensity-loss gradient, Adam update of the phase (and with R_FWD the
                        // row FFT of exp(i phase) of the updated phase)
    ROUT_TILED = 65536, // write the tiled iterate as read, no transform (exchange probe)
    R_MANY = 131072,    // one of a uniform batch of masks (blockIdx.y): iterate, phases and
                        // partials offset by the mask's index (phasemask_solve_many)
};
constexpr int ROW_INIT = RIN_PHASE | R_FWD;
constexpr int ROW_ITER = RIN_TILED | R_INV | R_PS | R_FWD;
constexpr int ROW_LAST = RIN_TILED | R_INV | R_PS | ROUT_PHASE;
constexpr int ROW_LAST_FWD = RIN_TILED | R_INV | R_PS | ROUT_PHASE | R_FWD;
constexpr int ROW_GAP = RIN_TILED | R_INV | R_PS;
constexpr int ROW_FFT_FWD = RIN_NAT | R_FWD;
constexpr int ROW_FFT_INV = RIN_TILED | R_INV | ROUT_NAT;
constexpr int ROW_ITER_NE = ROW_ITER | R_NOERR;
constexpr int ROW_LAST_NE = ROW_LAST | R_NOERR;
constexpr int ROW_LAST_FWD_NE = ROW_LAST_FWD | R_NOERR;
constexpr int ROW_GRAD = RIN_TILED | R_INV | ROUT_GRAD;
constexpr int ROW_INIT_Z = RIN_PHASE | R_STOREZ | R_FWD;
constexpr int ROW_RAAR = RIN_TILED | R_INV | R_RAAR | R_FWD;
// Last RAAR pass: phase of the shadow P_S x^n, and (with _FWD) its row FFT
// for the final Fourier error.
constexpr int ROW_RAAR_LAST = RIN_TILED | R_INV | R_RAAR | ROUT_PHASE;
constexpr int ROW_RAAR_LAST_FWD = RIN_TILED | R_INV | R_RAAR | ROUT_PHASE | R_FWD;
// Field solves: u^0 given as a complex field, u^n returned as one (the row
// pass's field after P_S, before the next forward transform).
constexpr int ROW_INIT_FIELD = RIN_FIELD | R_FWD;
constexpr int ROW_LAST_FIELD = RIN_TILED | R_INV | R_PS | ROUT_FIELD;
constexpr int ROW_LAST_FIELD_FWD = RIN_TILED | R_INV | R_PS | ROUT_FIELD | R_FWD;
constexpr int ROW_LAST_FIELD_NE = ROW_LAST_FIELD | R_NOERR;
constexpr int ROW_COPY_FIELD = RIN_FIELD | ROUT_FIELD;  // u^n = u^0 (no iterations)
// Adam steps on the intensity loss: the row pass of step k (gradient of
// phi^{k-1}, update to phi^k, and the forward row transform for step k + 1).
constexpr int ROW_ADAM = RIN_TILED | R_INV | R_ADAM | R_FWD;
constexpr int ROW_ADAM_LAST = RIN_TILED | R_INV | R_ADAM;
// Exchange probe: the passes' loads and stores of the iterate with nothing
// between them (each element written back where it was read).
constexpr int ROW_COPY = RIN_TILED | ROUT_TILED;
// Uniform batches of masks (phasemask_solve_many): the phase-in, phase-out
// solve modes, one mask per blockIdx.y.
constexpr int ROW_INIT_MANY = ROW_INIT | R_MANY;
constexpr int ROW_ITER_MANY = ROW_ITER | R_MANY;
constexpr int ROW_ITER_NE_MANY = ROW_ITER_NE | R_MANY;
constexpr int ROW_LAST_MANY = ROW_LAST | R_MANY;
constexpr int ROW_LAST_FWD_MANY = ROW_LAST_FWD | R_MANY;
constexpr int ROW_LAST_NE_MANY = ROW_LAST_NE | R_MANY;

// Column-pass modes (bit sets).
enum : int {
    CIN_TILED = 1,
    CIN_NAT = 2,
    C_FWD = 4,        // forward column transform
    C_PROJ = 8,       // M-hat (Eq. 5) + Fourier-error partial sum
    C_ERR = 16,       // Fourier-error partial sum only
    C_INV = 32,       // inverse column transform
    COUT_TILED = 64,
    COUT_NAT = 128,
    C_NOERR = 256,    // M-hat without the Fourier-error partial sum
    C_LOSS = 512,     // intensity residual r = |U|^2/N - I, loss partials, U <- r U
    C_BIT = 1024,     // load the 1-bit target pattern (lit where m^2 / max m^2 > t_dark)
    C_POW = 2048,     // store |U|^2 / N (float, strip-tiled) and the work-group maximum
    C_ITILED = 4096,  // C_LOSS: the target intensity is strip-tiled (else natural layout)
    C_MANY = 8192,    // one of a uniform batch of masks (blockIdx.y), as R_MANY
};
constexpr int COL_ITER = CIN_TILED | C_FWD | C_PROJ | C_INV | COUT_TILED;
constexpr int COL_ERR = CIN_TILED | C_FWD | C_ERR;
constexpr int COL_FFT_FWD = CIN_TILED | C_FWD | COUT_NAT;
constexpr int COL_FFT_INV = CIN_NAT | C_INV | COUT_TILED;
constexpr int COL_ITER_NE = COL_ITER | C_NOERR;
constexpr int COL_LOSS = CIN_TILED | C_FWD | C_LOSS | C_INV | COUT_TILED;
constexpr int COL_INIT_BIT = C_BIT | C_INV | COUT_TILED;
constexpr int COL_POW = CIN_TILED | C_FWD | C_POW;
// Adam steps: the loss column pass on a strip-tiled intensity, and the loss
// of the final phase alone.
constexpr int COL_LOSS_T = COL_LOSS | C_ITILED;
constexpr int COL_LOSS_ONLY_T = CIN_TILED | C_FWD | C_LOSS | C_ITILED;
constexpr int COL_COPY = CIN_TILED | COUT_TILED;
constexpr int COL_ITER_MANY = COL_ITER | C_MANY;
constexpr int COL_ITER_NE_MANY = COL_ITER_NE | C_MANY;
constexpr int COL_ERR_MANY = COL_ERR | C_MANY;

struct RowParams {
    float2* X;             // tiled iterate
    const float2* tw;      // staged twiddle table of the row plan (W, P)
    const PmIo* io;
    const float2* nat_in;  // natural-layout input (RIN_NAT)
    float2* nat_out;       // natural-layout output (ROUT_NAT)
    double* part;          // one gap partial per work-group (R_PS), null without
    int H;
    float gscale;          // ROUT_GRAD: gradient scale 4 g_out / N
    float2* Z;             // R_RAAR / R_STOREZ: SLM-plane point x, strip-tiled
    float beta;            // R_RAAR: relaxation parameter
    const float* illum;    // R_ILLUM: illumination amplitude p, strip-tiled (float per pixel)
    int spread;            // launch at most one work-group per CU (grid fits the CUs)
    // R_ADAM: first and second moments (natural layout) and the step's
    // scalars: lr / (1 - beta1^k), sqrt(1 - beta2^k), beta1, beta2, eps
    float* am;
    float* av;
    float adam_step, adam_bc2s, beta1, beta2, eps;
    // R_MANY: masks in the launch (grid.y) and doubles between two masks'
    // partials
    int nb;
    size_t part_bstride;
};

struct ColParams {
    float2* X;             // tiled iterate
    const float* mhat;     // tiled target divided by its 2-norm
    const float2* tw;      // staged twiddle table of the column plan (H, P)
    const float2* nat_in;
    float2* nat_out;
    double* part;          // one Fourier-error partial per work-group
    int W;
    double invN;           // 1 / (H W)
    const float* inten;    // C_LOSS: target intensity, natural layout [H][W]
    const float* tnat;     // C_BIT: target amplitude, natural layout [H][W]
    const float* tmax_part;// C_BIT: per-work-group maxima of the target
    int ntmax;
    double t_dark;         // C_BIT: lit threshold on the normalised intensity
    float* pw;             // C_POW: |U|^2 / N, strip-tiled
    int spread;            // launch at most one work-group per CU (grid fits the CUs)
    int nb;                // C_MANY: masks in the launch (grid.y)
    size_t part_bstride;   // C_MANY: doubles between two masks' partials
};

// Intensity-loss passes over a batch of same-size phases (blockIdx.y = sample).
struct AdjParams {
    float2* saved;              // [batch][N] tiled work buffer, kept from forward to backward
    const float* phase;         // [batch][H][W]
    const float* inten;         // [batch][H][W] target intensity (strip-tiled with C_ITILED)
    float* grad;                // [batch][H][W] gradient (backward); updated phase (R_ADAM)
    const double* grad_loss;    // [batch] upstream gradient of each sample's loss (backward)
    double* part;               // loss partials: row part_row0 + b of nwg slots per sample
    const float2* twW;
    const float2* twH;
    int H, W, nwg;
    int part_row0;
    // R_ADAM: moments [batch][H][W] and the step's scalars (as RowParams)
    float* am;
    float* av;
    float adam_step, adam_bc2s, beta1, beta2, eps;
};

// Launchers, one pair per supported transform length (powers of two 16 ..
// 4096, and the mixed-radix lengths 600, 800, 1080 and 1920), defined
// in the per-length kernel translation units.  `grid` is the number of
// work-groups; the block size is fixed by the length.  With non-null
// events the launch records the kernel's own start and end on them
// (hipExtLaunchKernelGGL), for timing a single pass.
#define PM_DECLARE_LAUNCHERS(L)                                                        \
    hipError_t launch_row_##L(int mode, const RowParams& p, int grid, hipStream_t s,    \
                              hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);      \
    hipError_t launch_col_##L(int mode, const ColParams& p, int grid, hipStream_t s,    \
                              hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
#define PM_DECLARE_ADJ_LAUNCHERS(L)                                                              \
    hipError_t launch_adj_row_##L(int mode, const AdjParams& p, int batch, hipStream_t s);  \
    hipError_t launch_adj_col_##L(int mode, const AdjParams& p, int batch, hipStream_t s);
PM_DECLARE_ADJ_LAUNCHERS(16)
PM_DECLARE_ADJ_LAUNCHERS(32)
PM_DECLARE_ADJ_LAUNCHERS(64)
PM_DECLARE_ADJ_LAUNCHERS(128)
PM_DECLARE_ADJ_LAUNCHERS(256)
PM_DECLARE_ADJ_LAUNCHERS(512)
PM_DECLARE_ADJ_LAUNCHERS(1024)
PM_DECLARE_ADJ_LAUNCHERS(2048)
PM_DECLARE_ADJ_LAUNCHERS(4096)
PM_DECLARE_ADJ_LAUNCHERS(600)
PM_DECLARE_ADJ_LAUNCHERS(800)
PM_DECLARE_ADJ_LAUNCHERS(1080)
PM_DECLARE_ADJ_LAUNCHERS(1920)
#undef PM_DECLARE_ADJ_LAUNCHERS

PM_DECLARE_LAUNCHERS(16)
PM_DECLARE_LAUNCHERS(32)
PM_DECLARE_LAUNCHERS(64)
PM_DECLARE_LAUNCHERS(128)
PM_DECLARE_LAUNCHERS(256)
PM_DECLARE_LAUNCHERS(512)
PM_DECLARE_LAUNCHERS(1024)
PM_DECLARE_LAUNCHERS(2048)
PM_DECLARE_LAUNCHERS(4096)
PM_DECLARE_LAUNCHERS(600)
PM_DECLARE_LAUNCHERS(800)
PM_DECLARE_LAUNCHERS(1080)
PM_DECLARE_LAUNCHERS(1920)
#undef PM_DECLARE_LAUNCHERS

// ---------------------------------------------------------------------------
// Batched solves: masks of several sizes (powers of two in
// [kBatchMinLen, kBatchMaxLen] per side) advance together, one column-pass
// kernel and one row-pass kernel per iteration for the whole batch.  Every
// work-group has kBatchThreads threads and takes one task (a mask and its
// first strip or row); it owns kBatchThreads / T lines of that mask.
constexpr int kBatchThreads = 256;
constexpr int kBatchMinLen = 64;
constexpr int kBatchMaxLen = 1024;
constexpr int kPrepPixels = 4096;  // pixels per task of the batched target preparation

// FFT schedules of the batched passes.  A schedule fixes, per transform
// length L, the points per thread P (hence the radix sequence P, P, ...,
// remainder: 16-16-2 or 8-8-8 at L = 512) and, at kBatchThreads threads, the
// lines per work-group G = kBatchThreads P / L (the tile).  The plan's tuner
// times every schedule on the plan's own buffers and keeps the fastest.
constexpr int kBatchSchedules = 2;
__host__ __device__ constexpr int batch_points(int sched, int L) {
    return sched == 0 ? (L >= 256 ? 16 : 8)
                      : (L >= 1024 ? 16 : (L >= 256 ? 8 : (L == 128 ? 16 : 4)));
}
__host__ __device__ constexpr int batch_lines(int sched, int L) {
    return kBatchThreads * batch_points(sched, L) / L;
}

struct BatchMask {
    int H, W;
    int col_wg0, col_wgs;  // this mask's column-pass work-groups (first, count)
    float2* X;             // tiled iterate
    float* mhat;           // tiled rescaled target
};

struct BatchTask {
    int mask;
    int first;             // first strip (column pass), first row (row pass), first pixel (prep)
};

struct BatchIo {
    const float* const* targets;     // device array of count device pointers
    const float* const* phases_in;
    float* const* phases_out;
    double* final_err;               // count doubles, may be null
};

struct BatchParams {
    const BatchMask* masks;
    const BatchTask* tasks;          // one per work-group of this launch
    const float2* tw;                // staged twiddle tables, batch_twiddle_offset
    const BatchIo* io;
    double* part;                    // one partial per work-group (error passes)
};

// Batched passes; MODE is one of the column / row modes, SCHED the FFT
// schedule.  Explicit instantiations live in pm_batch.hip.  With non-null
// events the launch records its own start and end on them.
template <int MODE, int SCHED>
hipError_t launch_batch_col(const BatchParams& p, int grid, hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);
template <int MODE, int SCHED>
hipError_t launch_batch_row(const BatchParams& p, int grid, hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);

// Batched preparation kernels (pm_aux.hip).  Prep tasks cover kPrepPixels
// pixels of one mask each; mask_prep0[i] is mask i's first prep task.
hipError_t launch_set_batch_io(BatchIo* io, const BatchIo& val, hipStream_t s);
hipError_t launch_batch_norm(const BatchIo* io, const BatchTask* tasks, int ntasks, double* part_m,
                             hipStream_t s);
hipError_t launch_batch_tile(const BatchIo* io, const BatchMask* masks, const BatchTask* tasks,
                             int ntasks, const int* mask_prep0, const double* part_m, hipStream_t s);
hipError_t launch_batch_wrap(const BatchIo* io, const BatchMask* masks, const BatchTask* tasks,
                             int ntasks, hipStream_t s);
hipError_t launch_batch_finalize(const BatchIo* io, const BatchMask* masks, int count,
                                 const double* part, hipStream_t s);

// Small kernels (pm_aux.hip).
hipError_t launch_set_io(PmIo* io, const PmIo& val, hipStream_t s);
// With batch > 1 (a uniform batch of masks, one per grid.y): mask b's target
// is io->target + b n, its partials part + b grid.
hipError_t launch_norm_partial(const PmIo* io, int n, double* part, int grid, hipStream_t s, int batch = 1);
// mhat = m / ||m||, or with an illumination (pn2 = device pointer to ||p||^2)
// m ||p|| / (||m|| sqrt(N)), strip-tiled.  Batches as launch_norm_partial
// (mask b's partials at part + b npart, its mhat at mhat + b H W).
hipError_t launch_target_tile(const PmIo* io, int H, int W, const double* part, int npart,
                              float* mhat, hipStream_t s, const double* pn2 = nullptr, int batch = 1);
// History entries first_entry + k * entry_step, k < count, into hist[k].
// pn2: ||p||^2 on the device with an illumination, else null (p = 1).
// With batch > 1, mask b's partials start at part + b part_bstride and its
// entries go to io->hist + b count.
hipError_t launch_finalize(const double* part, int stride, int n_col, int n_row, double invN,
                           const PmIo* io, int first_entry, int count, hipStream_t s, int entry_step = 1,
                           const double* pn2 = nullptr, int batch = 1, size_t part_bstride = 0);
// Illumination set-up: p (natural layout [H][W]) copied to the strip-tiled
// `illum`, and ||p||^2 (FP64, fixed summation order) to *pn2; `part` holds
// `grid` doubles of scratch.
hipError_t launch_illum_prep(const float* p, int H, int W, double* part, int grid, float* illum,
                             double* pn2, hipStream_t s);
hipError_t launch_wrap_phase(const PmIo* io, int n, hipStream_t s);
// Input check of PM_FLAG_VALIDATE over n floats (see k_validate).
hipError_t launch_validate(const float* x, int n, bool nonneg, int* flags, hipStream_t s);
// Per-work-group maxima of a float array (n a multiple of 4).
hipError_t launch_max_partial(const float* x, int n, float* part, int grid, hipStream_t s);
// Physical error of Eq. 8 (E_lit, E_dark) from the strip-tiled power
// |U|^2 / N, the natural-layout target and the partial maxima of both;
// `scratch` holds 2 doubles per work-group of grid n / 1024.
hipError_t launch_physical_error(const float* pw, const double* pw_max_part, int n_pw_max, const float* target,
                                 const float* tmax_part, int ntmax, int H, int W, double t_lit, double t_dark,
                                 double* scratch, double* out, hipStream_t s);
// Arithmetic-rate probe of one 16-point DFT stage (pm_probe.hip): matrix = 0
// on the vector ALUs, 1 as FP32 matrix products; `waves` (a multiple of 4)
// waves of 1024 complex points each, in and out; the launch records its own
// start and end on ev0 / ev1.
hipError_t launch_probe_dft16(int matrix, const float2* in, float2* out, int waves, int reps, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1);

// out[b] = sum of part[b * nwg .. b * nwg + nwg) in a fixed order, b < count.
hipError_t launch_sum_rows(const double* part, int nwg, double* out, int count, hipStream_t s);
// The same into io->hist (the per-call pointer block).
hipError_t launch_sum_rows_io(const double* part, int nwg, const PmIo* io, int count, hipStream_t s);
// Adam solve set-up over `batch` samples of H x W: phase = io->phase_in,
// inten (strip-tiled) = io->target, moments m = v = 0.
hipError_t launch_adam_prep(const PmIo* io, int H, int W, int batch, float* phase, float* inten, float* m,
                            float* v, hipStream_t s);
// io->phase_out = phase over batch x H x W floats.
hipError_t launch_adam_out(const PmIo* io, const float* phase, size_t n, hipStream_t s);

}  // namespace pm
