/*
 * phasemask.h -- C ABI of the MI355X (gfx950) phase-mask library.
 *
 * The library computes phase-only spatial-light-modulator (SLM) masks by the
 * method of alternating projections (Gerchberg-Saxton), Kramer, Hagemann and
 * Luke, "Real-Time Phase Masks for Interactive Stimulation of Optogenetic
 * Neurons" (arXiv:1302.0120):
 *
 *   find u in S cap M                                  (Eq. 3)
 *   S = { u : |u_jk| = p_jk },  here p = 1              (Eq. 1)
 *   M = { u : |(F u)_jk| = m_jk }                       (Eq. 2)
 *   u^{nu+1} = P_S P_M u^nu                              (Eq. 6)
 *
 * with P_S of Eq. 4a and P_M of Eq. 4b / Eq. 5.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Images are row-major [height][width] (height = n_y rows, width = n_x),
 *    contiguous, with no padding between rows.
 *  * The Fourier plane is in natural DFT order: zero frequency at [0][0];
 *    forward kernel exp(-2 pi i (k_y y / height + k_x x / width)).
 *  * Complex arrays are interleaved pairs of float (re, im), 8 bytes per
 *    element.
 *  * Sizes: height and width must each be a power of two in [16, 4096], or
 *    600, 800, 1080 or 1920 (the mixed-radix transforms of 800 x 600 and
 *    1920 x 1080 SLM panels, in either orientation, also paired with any
 *    supported length); anything else returns PM_EUNSUPPORTED.  The batched entry points take powers of two
 *    only (see phasemask_create_batched).
 *  * All array arguments are DEVICE pointers owned by the caller, on the
 *    device that was current when the handle was created, unless a comment
 *    says otherwise.  The library never frees them.  Alignment: the target
 *    amplitude 16 bytes, complex arrays and doubles 8 bytes, other floats
 *    4 bytes; a misaligned pointer returns PM_EINVAL.
 *  * Every call is asynchronous on the handle's stream (see
 *    phasemask_set_stream) unless a comment says otherwise: results are valid
 *    once that stream's work up to the call has completed.  Calls on one
 *    handle must not run concurrently from several host threads.
 *  * Every call returns a pm_status.  Nothing throws across the ABI.  After
 *    PM_EINVAL or PM_EUNSUPPORTED the handle is unchanged and still usable;
 *    phasemask_last_error() gives a human-readable reason.
 *  * Error norms are relative to ||p|| = sqrt(N), N = height * width, with
 *    the target rescaled to the energy of the SLM field,
 *    m~ = m sqrt(N) / ||m||, which leaves the iterates unchanged:
 *      E_F = || |F u| - m~ || / sqrt(N)      = d(u, M) / ||p||      (Eq. 7 as
 *            printed, since u lies in S)
 *      G   = || |P_M u| - 1 || / sqrt(N)     = d(P_M u, S) / ||p||  (Eq. 7,
 *            the sentence after it: points of M and their projections on S)
 *    Zero tie-break of Eq. 4a / Eq. 5: a pixel or Fourier coefficient whose
 *    squared modulus is below FLT_MIN takes the phase theta = 0.
 */
#ifndef PHASEMASK_H
#define PHASEMASK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pm_plan* pm_handle;

typedef enum {
    PM_OK = 0,
    PM_EINVAL = -1,        /* bad argument (null pointer, negative count, ...) */
    PM_EUNSUPPORTED = -2,  /* size outside {2^k: 16..4096} + {600, 800, 1080, 1920} */
    PM_ENOMEM = -3,        /* device or host allocation failed                */
    PM_EDEVICE = -4,       /* a HIP call or kernel launch failed              */
    PM_ESTATE = -5         /* handle destroyed or in an unusable state        */
} pm_status;

/* Flags for phasemask_create. */
#define PM_FLAG_NO_GRAPH 0x1u   /* launch kernels one by one instead of
                                   replaying a captured HIP graph           */
#define PM_FLAG_NO_TUNE 0x2u    /* batched plans: use FFT schedule 0 instead
                                   of timing the schedules at creation      */
#define PM_FLAG_VALIDATE 0x4u   /* one-mask plans: before each call check the
                                   inputs on the device (target >= 0, finite,
                                   not all zero; phases finite; illumination
                                   >= 0, finite, not all zero) and return
                                   PM_EINVAL if a check fails.  Synchronises
                                   the handle's stream on every call.       */

/*
 * Create a plan for masks of height x width pixels (Sec. II: n_y = height,
 * n_x = width).  Allocates the plan's device workspace (the iterate, the
 * rescaled target, twiddle tables and reduction partials: about 12 bytes per
 * pixel, plus FP64 partial sums of N / 128 to N / 16 bytes (N = height x
 * width), at least 4 KiB, per error-history entry, grown on demand) on the
 * current device.
 * `stream` is a hipStream_t (NULL = the null stream) used by every later
 * call until phasemask_set_stream changes it.
 * With the environment variable PHASEMASK_LOG set, the plan's transform
 * schemes and work-group counts are printed to stderr.
 * Errors: PM_EINVAL if out is NULL; PM_EUNSUPPORTED for sizes outside the
 * supported set; PM_ENOMEM, PM_EDEVICE.  On error *out is set to NULL.
 */
pm_status phasemask_create(pm_handle* out, int height, int width,
                           unsigned flags, void* stream);

/* Release the plan and its workspace.  Synchronises the handle's stream
 * first.  Destroying NULL returns PM_EINVAL.  The library keeps a registry
 * of live plans: every call given a handle that is not one (destroyed, or
 * never returned by a create call) returns PM_ESTATE without touching it --
 * unless a later plan happens to occupy the same address -- and the size
 * queries return 0 (phasemask_batch_schedule -1). */
pm_status phasemask_destroy(pm_handle h);

/*
 * Use `stream` (a hipStream_t, NULL = null stream) for subsequent calls.
 * Every call of a handle shares its device buffers (pointer block, iterate,
 * rescaled target, partial sums), so the handle's calls are ordered: when
 * the stream changes, an event recorded on the previous stream makes the new
 * stream wait for everything the handle enqueued before the switch (work of
 * the caller on either stream is not otherwise ordered).  Switching to the
 * current stream does nothing.
 * Errors: PM_EINVAL (NULL handle), PM_EDEVICE.
 */
pm_status phasemask_set_stream(pm_handle h, void* stream);

/*
 * Illumination amplitude p of Eq. 1: the set S becomes the fields whose
 * pixel moduli equal p (not 1), so u^0 = p exp(i init_phase), P_S of Eq. 4a
 * gives each pixel modulus p (a zero pixel takes p exp(i 0)), and the errors
 * are relative to ||p|| with the target energy-matched to ||p||:
 *     E_F = || |F u| - m ||p|| / ||m|| || / ||p||,
 *     G   = || |P_M u| - p || / ||p||.
 * Applies to phasemask_solve, phasemask_solve_many (one p for every mask
 * of the batch), phasemask_solve_field (whose P_S then gives
 * modulus p; its init_field is taken as given), phasemask_solve_raar,
 * phasemask_error, phasemask_physical_error (whose field is
 * u = p exp(i phase)) and phasemask_time_passes until changed; the output phase is that of the
 * projected field before the factor p (also defined where p = 0).  Not
 * applied by phasemask_initial_phase, phasemask_fft2 or the intensity-loss
 * entry points.
 *
 *   illumination  float[height*width] DEVICE array, natural layout, p >= 0
 *                 and not all zero (not checked), 16-byte aligned; or NULL
 *                 to return to p = 1.  Copied on the handle's stream (with
 *                 ||p||^2 summed in FP64), so the caller may reuse it once
 *                 that stream has passed this call.
 * The first call allocates 4 bytes per pixel.  Switching between p and
 * p = 1 synchronises the stream and drops the handle's captured graphs.
 * Errors: PM_EINVAL (misaligned), PM_ESTATE (batched handle), PM_ENOMEM,
 * PM_EDEVICE.
 */
pm_status phasemask_set_illumination(pm_handle h, const float* illumination);

/*
 * Run n_iter iterations of Eq. 6 starting from u^0 = exp(i init_phase) and
 * write the phase of u^{n_iter}.
 *
 *   target_amplitude  float[height*width], m >= 0, finite, not all zero,
 *                     natural DFT order (Eq. 2).  Only its direction matters
 *                     for the iterates (any positive scale gives the same u).
 *                     (An all-zero target, not checked, makes M = {0}: the
 *                     result is the tie-break phase 0 and every error is 1.)
 *   init_phase        float[height*width], radians, any real value.
 *   n_iter            >= 0.
 *   out_phase         float[height*width]; receives the FP32 atan2(Im u, Re u),
 *                     in [-pi, pi] up to FP32 rounding (the float nearest pi
 *                     is slightly above pi).  May alias init_phase; must not
 *                     overlap target_amplitude.
 *   err_history       NULL, or double[2*n_iter + 1] receiving
 *                     [E_F^0, G^0, E_F^1, G^1, ..., E_F^{n-1}, G^{n-1}, E_F^n]
 *                     (E_F^nu measured on u^nu before projecting, G^nu on
 *                     P_M u^nu; the final entry costs one extra transform).
 *                     Reductions are in FP64 and deterministic: repeating a
 *                     call gives bitwise identical results.
 * The plan keeps 2 n_iter + 1 entries of FP64 partial sums for a history
 * (grown on first use, which synchronises the stream and drops the captured
 * graphs); a solve without a history writes none and grows nothing.
 * Errors: PM_EINVAL for a NULL array, n_iter < 0, or overlapping output and
 * target; PM_ENOMEM if the partial-sum buffer for n_iter cannot be grown;
 * PM_EDEVICE if a launch fails.
 */
pm_status phasemask_solve(pm_handle h, const float* target_amplitude,
                          const float* init_phase, int n_iter,
                          float* out_phase, double* err_history);

/*
 * The alternating projections of Sec. II (Eqs. 4a, 5, 6) on a uniform batch
 * of `batch` masks of the plan's size, e.g. a stream of stimulation patterns
 * for the same SLM panel (Sec. I: frame rates of 0.1-1 kHz): every pass of
 * the solve is one launch over all masks, so the GPU holds several tiles per
 * CU where one mask holds one.  Mask b's arrays follow mask b - 1's:
 *   target_amplitude  float[batch][height][width] (16-byte aligned), m >= 0;
 *   init_phase        float[batch][height][width];
 *   out_phase         float[batch][height][width], may alias init_phase;
 *   err_history       double[batch][2 n_iter + 1] or NULL, mask b's history
 *                     as phasemask_solve writes it.
 * Each mask's phases and history are bitwise those of phasemask_solve on
 * that mask alone (same kernels and summation order), also with the
 * illumination of phasemask_set_illumination, which every mask of the batch
 * shares.  The plan keeps the batch's iterates, rescaled targets and
 * partial sums (12 bytes per pixel and mask, plus, with a history, 2 n_iter + 1
 * entries of partials), allocated on first use for the
 * largest batch and history seen, which synchronises the
 * stream and drops the captured graphs; without PM_FLAG_NO_GRAPH the solve
 * is one captured graph per (n_iter, batch, history).
 * Errors: PM_EINVAL for a NULL array, batch outside [1, 65535] or with
 * batch * height * width >= 2^31, n_iter outside [0, 2^20], misalignment or
 * overlapping arrays (out_phase with the
 * target, err_history with any array); PM_ESTATE (batched handle);
 * PM_ENOMEM; PM_EDEVICE.
 */
pm_status phasemask_solve_many(pm_handle h, int batch, const float* target_amplitude,
                               const float* init_phase, int n_iter,
                               float* out_phase, double* err_history);

/*
 * For callers that cannot allocate device memory when they solve (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * phasemask_solve without any allocation.  Same arguments, results (bitwise)
 * and errors as phasemask_solve, except:
 *   - the iterate, the rescaled target, the pointer block and the FP64
 *     partial sums live in a scratch array the library holds on every GPU
 *     it runs on (32 MiB each, until the process ends; its device address is
 *     looked up once per device, at phasemask_create), not in the plan;
 *   - it enqueues the solve's kernels on the handle's stream one by one (no
 *     graph, no synchronisation, no allocation, no memset), so a caller may
 *     capture it;
 *   - PM_FLAG_VALIDATE is not honoured (its check would synchronise);
 *   - the solve must fit in the array: 12 bytes per pixel plus, with a
 *     history, 2 n_iter + 1 entries of FP64 partial sums (16 KiB per entry
 *     at 1024 x 1024, so 1024 x 1024 fits with histories of up to 639
 *     iterations; 2048 x 2048 does not fit); else PM_EINVAL stating the
 *     bytes needed.
 * Nothing in the array needs to start at zero (each call writes every byte
 * it reads before reading it), but every call on one GPU shares that GPU's
 * array: calls whose work can overlap on one GPU (other streams, plans or
 * host threads) race on it and give undefined results, so order them.
 */
pm_status phasemask_solve_noalloc(pm_handle h, const float* target_amplitude,
                                  const float* init_phase, int n_iter,
                                  float* out_phase, double* err_history);

/*
 * The iteration of phasemask_solve on complex fields: the state of the
 * method is the SLM field u (Eq. 6), so a solve that hands it back exactly
 * can be resumed exactly.  u^0 = init_field as given (a point of S, Eq. 1,
 * normally: unit modulus, or modulus p with an illumination; a field off S
 * is used as it is, so E_F^0 is then || |F u^0| - m~ || / ||p||), and
 * out_field receives u^{n_iter}: with n_iter >= 1 the FP32 result of the last
 * P_S (Eq. 4a), bitwise the value the next iteration would transform, so
 *   solve_field(a + b, u0)  ==  solve_field(b, solve_field(a, u0))
 * bitwise in the field and in the history entries they share.
 *   init_field   complex float[height*width] (interleaved re, im), natural
 *                layout, 8-byte aligned; finite.
 *   n_iter       >= 0 (0: out_field = init_field, history [E_F^0]).
 *   out_field    complex float[height*width]; may alias init_field; must not
 *                overlap the target or the history.
 *   target_amplitude, err_history   as for phasemask_solve.
 * Errors: as phasemask_solve.
 */
pm_status phasemask_solve_field(pm_handle h, const float* target_amplitude, const void* init_field,
                                int n_iter, void* out_field, double* err_history);

/*
 * Relaxed averaged alternating reflections (RAAR), the algorithm the paper
 * names for projection problems where alternating projections stagnate
 * (Sec. IV.B).  With R_S = 2 P_S - I and R_M = 2 P_M - I:
 *   x^{nu+1} = beta/2 (R_S R_M + I) x^nu + (1 - beta) P_M x^nu
 *            = beta P_S(2 P_M x^nu - x^nu) + beta x^nu + (1 - 2 beta) P_M x^nu,
 * from x^0 = exp(i init_phase); the mask is the shadow P_S x^n and out_phase
 * receives its phase.  Arguments as for phasemask_solve, plus
 *   beta          relaxation in (0, 1] (beta = 1: Douglas-Rachford).
 *   err_history   NULL or double[n_iter + 1]:
 *                 [E_F(x^0), ..., E_F(x^{n-1}), E_F(P_S x^n)].
 * The plan keeps an 8-byte-per-pixel state buffer after the first call.
 * Errors: as phasemask_solve, and PM_EINVAL for beta outside (0, 1].
 */
pm_status phasemask_solve_raar(pm_handle h, const float* target_amplitude,
                               const float* init_phase, int n_iter, double beta,
                               float* out_phase, double* err_history);

/*
 * Errors of a given phase-only mask u = exp(i phase) against a target:
 * errors[0] = E_F, errors[1] = G (definitions above; equal to entries 0 and
 * 1 of the history of a solve started at `phase`).
 *   target_amplitude, phase   as for phasemask_solve.
 *   errors                    double[2], device.
 * Errors: PM_EINVAL for NULL arrays; PM_EDEVICE.
 */
pm_status phasemask_error(pm_handle h, const float* target_amplitude,
                          const float* phase, double* errors);

/*
 * The paper's initial mask (Sec. IV, first paragraph), read as: binarise the
 * target (lit where m^2 / max m^2 > t_dark, an IEEE double comparison),
 * back-propagate the 1-bit pattern with the inverse transform and keep the
 * phase (the projection onto S, Eq. 4a, with its zero tie-break).  The paper
 * uses t_dark = 3e-4, its dark tolerance of Eq. 8b.
 *   target_amplitude  as for phasemask_solve.
 *   out_phase         float[height*width] receives the phase (FP32 atan2);
 *                     must not overlap the target.
 * Errors: PM_EINVAL for NULL, misaligned or overlapping arrays, or t_dark
 * outside [0, 1); PM_EDEVICE.
 */
pm_status phasemask_initial_phase(pm_handle h, const float* target_amplitude,
                                  double t_dark, float* out_phase);

/*
 * Physical error of the mask exp(i phase) against a target (Eq. 8a, 8b):
 *   errors[0] = E_lit  = sum over lit pixels  (t_dark rel / t_lit - t_dark) [rel > t_lit]
 *   errors[1] = E_dark = sum over dark pixels (I_r - t_dark) [I_r > t_dark]
 * with I_t = m^2 / max m^2, I_r = |F u|^2 / max |F u|^2, rel = |I_t - I_r| / I_t
 * and a pixel lit where I_t > t_dark (the paper calls both quantities
 * intensities and leaves their scale and the lit/dark split unstated; this is
 * the reading above).  The paper's tolerances are t_lit = 0.1, t_dark = 3e-4
 * (Sec. II, the paragraph defining the physical error).  FP64 sums; the
 * plan keeps a 4-byte-per-pixel scratch buffer after the first call.
 *   errors            DEVICE double[2].
 * Errors: PM_EINVAL for NULL or misaligned arrays, t_lit <= 0 or t_dark
 * outside [0, 1); PM_ENOMEM; PM_EDEVICE.
 */
pm_status phasemask_physical_error(pm_handle h, const float* target_amplitude,
                                   const float* phase, double t_lit, double t_dark,
                                   double* errors);

/*
 * Unnormalised complex 2-D DFT through the library's own FFT passes (the
 * transform inside P_M, Eq. 4b):
 *   inverse = 0:  out[k] = sum_x in[x] exp(-2 pi i (k_y y/height + k_x x/width))
 *   inverse = 1:  out[x] = sum_k in[k] exp(+2 pi i (...))   (no 1/N factor)
 * in, out: complex float[height*width] (interleaved re, im).  They may be
 * the same buffer.
 * Errors: PM_EINVAL for NULL arrays; PM_EDEVICE.
 */
pm_status phasemask_fft2(pm_handle h, const void* in, void* out, int inverse);

/*
 * Batched plans: `count` independent masks of uneven sizes solved together,
 * e.g. the masks of one frame of an interactive stimulation loop (the paper
 * asks for frame rates of 0.1 to 1 kHz, Sec. I).  Every iteration of Eq. 6
 * runs as one column-pass launch and one row-pass launch over the masks of
 * a group; the whole solve is one captured graph.  Groups: consecutive
 * masks (largest first) whose working sets (12 bytes per pixel) add up to
 * at most 48 MiB; a group runs all its iterations before the next group of
 * its chain, and the groups are spread over 4 chains of launches that run
 * concurrently (balanced by bytes), so that the chains' working sets stay
 * in the last-level cache together.  The environment variables
 * PHASEMASK_GROUP_MB=<m> (0 = one group) and PHASEMASK_CHAINS=<1..8> set
 * these at creation.  Results do not depend on the grouping or chains.
 *   heights, widths   HOST arrays of `count` sizes, each a power of two in
 *                     [64, 1024] (else PM_EUNSUPPORTED).
 * FFT schedules: the batched passes have several compiled schedules (points
 * per thread, i.e. radix sequence, and lines per work-group).  At creation
 * the plan picks one: the environment variable PHASEMASK_SCHEDULE=<k>
 * forces schedule k; else a choice cached for the same multiset of sizes on
 * the same GPU architecture (in this process, or in the file named by
 * PHASEMASK_TUNE_CACHE, one "key schedule" line per entry, appended to);
 * else each schedule runs a few iterations on the plan's own buffers, grouped
 * and spread over the chains as a solve runs them (one captured graph,
 * replayed on `stream`, synchronised), and the fastest is kept.  PM_FLAG_NO_TUNE selects
 * schedule 0 without timing.  PHASEMASK_LOG=1 prints the timings to stderr.
 * Errors: PM_EINVAL for NULL arguments, count < 1 or an out-of-range
 * PHASEMASK_SCHEDULE, PHASEMASK_GROUP_MB or PHASEMASK_CHAINS; PM_ENOMEM;
 * PM_EDEVICE.
 * A batched handle works with phasemask_solve_batched, phasemask_set_stream,
 * phasemask_workspace_bytes and phasemask_destroy; other entry points
 * return PM_ESTATE for it.
 */
pm_status phasemask_create_batched(pm_handle* out, int count, const int* heights,
                                   const int* widths, unsigned flags, void* stream);

/*
 * n_iter iterations of Eq. 6 for every mask of a batched plan.
 *   targets, init_phases, out_phases   DEVICE arrays of `count` device
 *                     pointers (8-byte aligned), entry i pointing at mask i's
 *                     float[height_i * width_i] image, laid out and
 *                     constrained as for phasemask_solve (targets 16-byte
 *                     aligned; out_phases[i] may alias init_phases[i]).
 *   final_err         NULL, or DEVICE double[count] receiving E_F^n of each
 *                     returned mask (the last history entry of a one-mask
 *                     solve).
 * Results equal `count` separate phasemask_solve calls on the same inputs
 * up to FP32 rounding; where a mask's sides run the one-mask radix plans
 * (schedule 1 at 64 and 512 points) its phases are bitwise equal and its
 * error equal up to the order of the FP64 sums.
 * Errors: PM_EINVAL for NULL pointer arrays, n_iter < 0 or misaligned
 * arguments; PM_ESTATE for a one-mask handle; PM_EDEVICE.
 */
pm_status phasemask_solve_batched(pm_handle h, const float* const* targets,
                                  const float* const* init_phases, int n_iter,
                                  float* const* out_phases, double* final_err);

/* FFT schedule a batched plan runs (0 .. schedules-1), or -1 for a NULL or
 * one-mask handle. */
int phasemask_batch_schedule(pm_handle h);

/* Configuration a batched plan runs with: FFT schedule (picked at creation
 * by the plan's tuner, which times every schedule on the plan's own
 * buffers and keeps the lowest-numbered one unless a later schedule is more
 * than 2% faster, cached per architecture and set of sizes, in-process and in the
 * file named by PHASEMASK_TUNE_CACHE; PHASEMASK_SCHEDULE forces one,
 * PM_FLAG_NO_TUNE takes 0), number of concurrent chains of launches
 * (PHASEMASK_CHAINS, default 4) and the cache budget of one group of masks
 * in bytes (PHASEMASK_GROUP_MB, default 48 MiB; 0 = one group).  Any output
 * pointer may be NULL.
 * Errors: PM_EINVAL for a NULL handle, PM_ESTATE for a one-mask handle. */
pm_status phasemask_batch_config(pm_handle h, int* schedule, int* chains, size_t* group_bytes);

/*
 * Intensity loss and its gradient (differentiable phase optimisation beside
 * the projections; not in the paper, which notes that other reconstruction
 * algorithms plug into the same machinery, Sec. V).  For each of `batch`
 * phases of the plan's size:
 *   L_b(phi) = sum_k ( |(F exp(i phi_b))_k|^2 - I_{b,k} )^2,  F unitary
 *   dL_b/dphi_j = 4 Im( exp(-i phi_j) (F^H (r . U))_j ),  r = |U|^2 - I_b.
 * A phase-only field has sum_k |U_k|^2 = N, so targets scaled to
 * sum_k I_k = N are the natural choice (the library does not rescale).
 *
 * Forward:  phase, target_intensity   float[batch][height][width];
 *           loss                      DEVICE double[batch];
 *           saved                     DEVICE complex float[batch][height*width]
 *                                     (8-byte aligned) that the backward
 *                                     call reads; its layout is internal.
 * Backward: grad_loss                 DEVICE double[batch], the upstream
 *                                     gradient of each loss;
 *           grad_phase                float[batch][height][width] receives
 *                                     grad_loss_b * dL_b/dphi.
 *           phase and saved must be the forward call's, unchanged.
 * Errors: PM_EINVAL for NULL or misaligned arrays or batch outside
 * [1, 65535]; PM_ENOMEM; PM_EDEVICE.
 */
pm_status phasemask_intensity_loss_fwd(pm_handle h, int batch, const float* phase,
                                       const float* target_intensity, double* loss,
                                       void* saved);
pm_status phasemask_intensity_loss_bwd(pm_handle h, int batch, const float* phase,
                                       const void* saved, const double* grad_loss,
                                       float* grad_phase);

/*
 * Gradient-based phase optimisation beside GS (not in the paper; its Sec. V
 * notes that other reconstruction methods plug into the same framework):
 * n_steps of Adam (Kingma and Ba 2015, Algorithm 1) on the intensity loss
 * of phasemask_intensity_loss_fwd, for `batch` phases of height x width at
 * once.  From m = v = 0, step k = 1 .. n_steps on each sample:
 *   g   = d loss / d phi at phi^{k-1}  (the intensity-loss adjoint),
 *   m   = beta1 m + (1 - beta1) g,   v = beta2 v + (1 - beta2) g^2,
 *   phi^k = phi^{k-1} - (lr / (1 - beta1^k)) m / (sqrt(v) / sqrt(1 - beta2^k) + eps),
 * elementwise in FP32 (bias corrections in double, rounded once).  Each step
 * is two fused passes: the loss column pass (forward column transform,
 * residual, loss partials, inverse column transform) and a row pass that
 * runs the inverse row transform, the gradient, the update and the forward
 * row transform of exp(i phi^k).
 *   target_intensity  float[batch][height][width], I >= 0, natural DFT order,
 *                     on the scale of |F e^{i phi}|^2 with unitary F (sums
 *                     to N when matched in energy).
 *   init_phase        float[batch][height][width], radians.
 *   n_steps           >= 0.
 *   lr, beta1, beta2, eps   lr > 0 and finite; beta1, beta2 in [0, 1);
 *                     eps > 0 and finite.
 *   out_phase         float[batch][height][width] receiving phi^{n_steps};
 *                     may alias init_phase; must not overlap the target.
 *   loss_history      NULL, or double[(n_steps + 1) * batch]: entry
 *                     k * batch + b = loss of sample b at phi^k (FP64,
 *                     deterministic).
 * The three float arrays must be 16-byte aligned (history 8).  The plan
 * keeps the Adam state (24 bytes per pixel and sample, allocated on first
 * use for the largest batch seen, which synchronises the stream and drops
 * the captured graphs).  The illumination of phasemask_set_illumination does
 * not apply (the loss is that of exp(i phi)).  Without PM_FLAG_NO_GRAPH the
 * solve is one captured graph per (n_steps, batch, history, lr, beta1,
 * beta2, eps), like phasemask_solve.  PHASEMASK_ADAM_CHAINS=<1..8> (read at
 * the handle's first Adam solve; default 1) runs the samples in contiguous
 * groups on that many concurrent chains of launches: the handle's stream
 * and side streams forked from it and joined back, each chain its own
 * captured graph.  The results do not depend on it; the speed does: two
 * chains gained 10% in a process holding only the Adam plan and lost 12%
 * in one that had created and run other plans first, where the chains'
 * streams shared one of the runtime's hardware queues (GPU_MAX_HW_QUEUES,
 * default 4; with 8 the two chains gained 11% there too).
 * Errors: PM_EINVAL for a NULL array, batch outside [1, 65535], n_steps < 0,
 * a hyper-parameter out of range, misalignment or overlapping arrays, or an
 * out-of-range PHASEMASK_ADAM_CHAINS; PM_ENOMEM; PM_EDEVICE.
 */
pm_status phasemask_solve_adam(pm_handle h, int batch, const float* target_intensity,
                               const float* init_phase, int n_steps, double lr,
                               double beta1, double beta2, double eps,
                               float* out_phase, double* loss_history);

/*
 * Measurement (roofline accounting of the two passes that run n_iter times,
 * Eq. 6): average device duration in milliseconds of one column pass
 * (forward column FFT, Eq. 5 projection, inverse column FFT) and of one row
 * pass (inverse row FFT, Eq. 4a projection, forward row FFT).  Prepares the
 * iterate of a solve started at `phase` against `target_amplitude`, then runs
 * `reps` iterations, each pass launched with its own start/end events
 * (recorded by the kernel launch itself, so host launch gaps are excluded).
 * The iterate left behind is discarded.  Synchronises the stream; col_ms and
 * row_ms are HOST pointers.
 * Errors: PM_EINVAL for NULL arguments or reps outside [1, 100000];
 * PM_EDEVICE.
 */
pm_status phasemask_time_passes(pm_handle h, const float* target_amplitude,
                                const float* phase, int reps,
                                float* col_ms, float* row_ms);

/*
 * Arithmetic-rate probe for the choice of unit for the FFT butterflies (no
 * handle; the null stream; synchronises).  Runs one 16-point DFT stage over
 * waves x 1024 complex points, reps times, with the data in registers:
 *   matrix_units = 0: on the vector ALUs with the radix-16 butterfly of the
 *     passes, as forward-then-inverse pairs scaled by 1/16 (reps / 2 pairs);
 *     out = in transformed so (about in).
 *   matrix_units = 1: as FP32 matrix products (v_mfma_f32_16x16x4_f32), each
 *     wave 4 blocks of 16 butterflies, Y = F X with F[k][t] = exp(-2 pi i k t
 *     / 16), X[t][j] = in[1024 w + 256 b + 16 t + j], accumulated over the
 *     reps: out[1024 w + 256 b + 16 k + j] = reps * Y[k][j].
 *   in, out   complex float[waves * 1024], device, not overlapping.
 *   waves     a multiple of 4 in [4, 2^20]; reps even, in [2, 2^20].
 *   ms        receives the kernel's own duration.
 * Both versions do 16 x reps DFT points per thread-lane of work, so
 * waves * 1024 * reps / ms compares the units' rates for this stage.
 * Errors: PM_EINVAL for bad arguments; PM_EDEVICE.
 */
pm_status phasemask_probe_dft16(int matrix_units, const void* in, void* out, int waves, int reps, float* ms);

/*
 * Data-movement probe of a one-mask plan: the iterate exchange of Sec. II's
 * iteration without its arithmetic.  Runs reps pairs of the plan's own
 * column and row pass kernels (same thread maps, tiles, work-groups per CU
 * and launch order as a solve) in a copy mode that stores every element of
 * the iterate where it was loaded, with the same write-through stores, so
 * each pass reads what the other pass wrote from other XCDs, as in a solve.
 *   buffer  device complex float[height * width] (16-byte aligned), any
 *           contents; copied in place 2 * reps times, so it is unchanged on
 *           return (bitwise).  The plan's own buffers are not touched.
 *   reps    pairs, in [1, 10000].
 *   ms      receives the duration of the reps pairs (one captured graph,
 *           launched once untimed and once between events on the handle's
 *           stream; the call synchronises).
 * ms / reps is the time one iteration's two passes take for moving their
 * data alone: the floor for the iteration that this data movement sets.
 * Errors: PM_EINVAL (NULL handle or argument, reps out of range,
 * misalignment), PM_ESTATE (batched handle), PM_EDEVICE.
 */
pm_status phasemask_probe_exchange(pm_handle h, void* buffer, int reps, float* ms);

/* Plan facts.  Bytes of device memory the plan currently owns (a workspace
 * set by phasemask_set_workspace is the caller's and not counted). */
size_t phasemask_workspace_bytes(pm_handle h);

/*
 * Caller-owned workspace, e.g. from the PyTorch caching allocator.  The
 * workspace of a one-mask plan holds the iterate (complex, 8 bytes per
 * pixel), the rescaled target (4 bytes per pixel) and the FP64 partial sums
 * of the error norms (a fixed number of doubles per error-history entry),
 * each part 256-byte aligned.
 *
 * phasemask_workspace_size: bytes a workspace needs for solves of up to
 * n_iter iterations with a history (2 n_iter + 1 entries; every other entry
 * point needs at most the size for n_iter = 0, except an intensity-loss call
 * of `batch` phases, which needs batch entries: the size for n_iter =
 * batch / 2).  0 for a NULL or batched handle or n_iter < 0.
 *
 * phasemask_set_workspace: the plan releases its own iterate, target and
 * partial-sum buffers and works in [dev_ptr, dev_ptr + bytes) from then on;
 * dev_ptr = NULL returns to plan-owned buffers (allocated here, partials
 * grown on demand).  Synchronises the handle's stream first and drops the
 * captured graphs (they hold the old buffers).  The caller keeps the memory
 * allocated, on the plan's device, until the plan is destroyed or another
 * workspace is set, and must not touch it while the plan's work runs.  Its
 * contents need no initialisation.  A later call that needs more partial
 * sums than the workspace holds returns PM_EINVAL instead of growing them.
 * Buffers created on first use (RAAR state, illumination, power image of the
 * physical error) stay plan-owned.
 * Errors: PM_EINVAL for a workspace not 256-byte aligned or smaller than
 * phasemask_workspace_size(h, 0); PM_ESTATE for a batched handle;
 * PM_ENOMEM (returning to plan-owned buffers); PM_EDEVICE.
 */
size_t phasemask_workspace_size(pm_handle h, int n_iter);
pm_status phasemask_set_workspace(pm_handle h, void* dev_ptr, size_t bytes);

/* Static text for a status code. */
const char* phasemask_status_string(pm_status s);

/* Reason for the last non-PM_OK status returned on the calling host thread
 * (static or thread-local text, valid until the next call). */
const char* phasemask_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PHASEMASK_H */
