"""Benchmark: Gerchberg-Saxton phase masks on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one complete solve of the 1024 x 1024 spot workload (100 spots,
sigma 2 px, amplitudes in [0.5, 1], uniform random initial phase, seed 3):
target normalisation, u^0, 100 iterations of Eq. 6 (two fused passes each),
the FP64 error history and the output phase, replayed from the captured
graph with inputs resident in device memory.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GS iters/s & ms per 1024² mask (fp32, 100 it); batched masks/s vs plain GS"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Algorithmic bytes per pixel of one launch (see the design notes):
COL_BYTES_PER_PX = 8 + 8 + 4   # read iterate, write iterate, read rescaled target
ROW_BYTES_PER_PX = 8 + 8       # read iterate, write iterate
# One Adam step on the intensity loss: loss row pass (phase 4, saved 8),
# loss column pass (saved 8 + 8, intensity 4), gradient row pass (saved 8,
# phase 4, gradient 4), fused Adam (phase, gradient, two moments read, phase
# and moments written: 28).
ADAM_STEP_BYTES_PER_PX = 12 + 20 + 16 + 28
# The library's Adam solve, per step: loss column pass (transform 8 + 8,
# tiled intensity 4) and the Adam row pass (transform 8 in and out, phase
# and both moments in and out: 8 + 8 + 24).
ADAM_FUSED_BYTES_PER_PX = 20 + 40

# Measured HBM/MALL traffic per launch (rocprofv3 FETCH_SIZE x 1.9992 +
# WRITE_SIZE x 1.0, factors from a plain 64 MiB copy; summary under profiles/),
# valid only for the kernel sources it was taken on (hash below).
KERNEL_SOURCES = ("pm_common.h", "pm_fft.hpp", "pm_kernels.hpp", "pm_pass.hip")
TRAFFIC_SOURCE_HASH = "0d28a96a29195a3f"
TRAFFIC_BYTES = {"row pass": 16947061, "column pass": 21131672}


def kernel_source_hash() -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_1302_0120_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def environment(torch):
    """Where the numbers were measured."""
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    prop = torch.cuda.get_device_properties(0)
    return {"gpu": prop.name, "arch": getattr(prop, "gcnArchName", "unknown"),
            "compute_units": prop.multi_processor_count, "hip": torch.version.hip,
            "torch": torch.__version__, "host_cpu": cpu, "host_threads": os.cpu_count()}


def _median_of_reps(fn, reps=3):
    """1 warm-up call, then `reps` timed calls; the median duration in s."""
    import statistics
    fn()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
    return statistics.median(times)


def cpu_baseline(m, phi0, n_iter_sample, reps=3):
    """The FP64 oracle, as it stands, on a bounded sample of the workload
    (its first n_iter_sample iterations): 1 warm-up (2 iterations: FFT
    set-up) + `reps` timed runs, median."""
    from oracle import gs
    import statistics
    gs.gs_solve(m, phi0, 2)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        gs.gs_solve(m, phi0, n_iter_sample)
        times.append(time.perf_counter() - t0)
    dt = statistics.median(times)
    return n_iter_sample / dt, dt


def cpu_fp32_gs(m, phi0, n_iter, workers):
    """A multithreaded FP32 CPU run of the same iteration, the analogue of the
    paper's multithreaded CPU comparison (Sec. IV.A: FFTW on 12 threads):
    complex64 2-D FFTs by scipy.fft on `workers` threads, the projections of
    Eq. 4a and Eq. 5 in NumPy, no error history.  A timing baseline only:
    nothing here is used as a reference for results."""
    import numpy as np
    import scipy.fft as sfft
    mm = m.astype(np.float32)
    ones = np.ones_like(mm)

    def project(z, modulus):
        # modulus * z / |z|; modulus (phase 0) where z = 0
        a = np.abs(z)
        nz = a > 0
        np.divide(modulus, a, out=a, where=nz)
        out = z * a
        if not nz.all():
            out[~nz] = modulus[~nz]
        return out

    def run():
        u = np.exp(1j * phi0.astype(np.float32)).astype(np.complex64)
        for _ in range(n_iter):
            U = sfft.fft2(u, workers=workers, overwrite_x=True)
            w = sfft.ifft2(project(U, mm), workers=workers, overwrite_x=True)
            u = project(w, ones)
        return u
    return _median_of_reps(run)


def host_cpu_model():
    """CPU model as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return "unknown"


def copy_bandwidth(torch, nbytes, reps=200):
    """Device-to-device copy of `nbytes` (the iterate of the workload) back to
    back on torch's current stream, the bandwidth a pass moving the same
    working set could reach: read + write bytes over the mean copy time
    (events on the stream the copies run on)."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(20):
        b.copy_(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / reps
    return 2 * nbytes / (us * 1e-6) / 1e9, us


def bench_batched(torch, binding, synth, steps, plain_too=True, progress=False):
    """64 masks of sizes drawn from {256, 512, 1024}^2 (1-200 spots each), 100
    iterations: one batched graph launch versus the same masks solved one by
    one with the one-mask path (each with its own plan and graph; skipped
    with plain_too=False).  Both report the final Fourier error of every
    mask."""
    n_iter = 100
    say = (lambda m: print(m, flush=True)) if progress else (lambda m: None)
    probs = synth.batched_problems()
    shapes = [m.shape for m, _ in probs]
    dev = torch.device("cuda", 0)
    targets = [torch.from_numpy(m).to(dev) for m, _ in probs]
    phases = [torch.from_numpy(p).to(dev) for _, p in probs]
    outs = [torch.empty_like(p) for p in phases]
    err = torch.empty(len(probs), dtype=torch.float64, device=dev)
    say("batched: plan (tuner)")
    bp = binding.BatchedPhaseMask(shapes, device=dev)
    say("batched: first solve")
    bp.solve(targets, phases, n_iter, outs=outs, final_err=err)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        bp.solve(targets, phases, n_iter, outs=outs, final_err=err)
        say(f"batched: timed solve {k + 1} of {steps} enqueued")
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    sum_px = sum(h * w for h, w in shapes)
    gbs = (COL_BYTES_PER_PX + ROW_BYTES_PER_PX) * sum_px * n_iter / t_batch / 1e9
    res = {
        "workload": "64 masks, sizes uniform over {256,512,1024}^2 (seed 4), 1-200 spots, 100 it",
        "sum_pixels": sum_px,
        "masks_per_s": len(probs) / t_batch,
        "ms_per_batch": t_batch * 1e3,
        "algorithmic_gbs": gbs,
        "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
        "max_final_error": float(err.max().item()),
        "schedule": bp.schedule,
    }
    if not plain_too:
        return res

    plans = {}
    hists = [torch.empty(2 * n_iter + 1, dtype=torch.float64, device=dev) for _ in probs]
    def plain():
        for i, shp in enumerate(shapes):
            if shp not in plans:
                plans[shp] = binding.PhaseMask(*shp, device=dev)
            plans[shp].solve(targets[i], phases[i], n_iter, out=outs[i], history=hists[i])
    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / steps
    res.update({
        "plain_masks_per_s": len(probs) / t_plain,
        "plain_ms": t_plain * 1e3,
        "speedup_vs_plain": t_plain / t_batch,
    })
    return res


def bench_batched_uniform(torch, binding, synth, steps, count=16, size=1024):
    """`count` masks of the headline's size (the 1024 x 1024 spot workload's
    sizes, 1-200 spots each, 100 iterations) through the batched path: how
    far the same pass design gets once every CU holds several tiles, which
    the single mask cannot give it."""
    n_iter = 100
    probs = synth.batched_problems(count=count, sizes=(size,))
    dev = torch.device("cuda", 0)
    targets = [torch.from_numpy(m).to(dev) for m, _ in probs]
    phases = [torch.from_numpy(p).to(dev) for _, p in probs]
    outs = [torch.empty_like(p) for p in phases]
    err = torch.empty(count, dtype=torch.float64, device=dev)
    bp = binding.BatchedPhaseMask([(size, size)] * count, device=dev)
    bp.solve(targets, phases, n_iter, outs=outs, final_err=err)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bp.solve(targets, phases, n_iter, outs=outs, final_err=err)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    gbs = (COL_BYTES_PER_PX + ROW_BYTES_PER_PX) * count * size * size * n_iter / t / 1e9
    return {"workload": f"{count} masks of {size}x{size}, 1-200 spots, 100 it", "masks_per_s": count / t,
            "ms_per_batch": t * 1e3, "gs_iterations_per_s": count * n_iter / t,
            "algorithmic_gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "max_final_error": float(err.max().item()), "schedule": bp.schedule}


def bench_mfma_probe(torch, binding, waves=4096, reps=200):
    """One 16-point DFT stage (the radix of the largest FFT plans) over
    waves x 1024 points, reps times, with the data in registers: on the
    vector ALUs (the passes' butterflies) and as FP32 matrix products
    (16 complex multiply-adds per point, operands preloaded in the matrix
    layout).  Points per second of stage work for each."""
    x = torch.randn(waves * 1024, dtype=torch.complex64, device="cuda")
    binding.probe_dft16(False, x, 2)
    binding.probe_dft16(True, x, 2)
    _, ms_v = binding.probe_dft16(False, x, reps)
    _, ms_m = binding.probe_dft16(True, x, reps)
    pts = waves * 1024 * reps
    rv, rm = pts / (ms_v * 1e-3), pts / (ms_m * 1e-3)
    return {"stage": "16-point DFT", "points": pts,
            "vector_alu_points_per_s": rv, "matrix_core_points_per_s": rm,
            "matrix_over_vector": rm / rv,
            "matrix_tflops": 128 * rm / 1e12, "matrix_peak_tflops_fp32": 157.3}


def bench_many(torch, binding, synth, h, w, n_iter, count, steps):
    """`count` masks of h x w (1-200 spots each) solved together as a
    uniform batch (phasemask_solve_many, FP64 histories): ms per batch and
    per mask, masks/s and algorithmic GB/s (36 B/px per iteration)."""
    import numpy as np
    dev = torch.device("cuda", 0)
    ms_, ps_ = [], []
    for b in range(count):
        rng = np.random.default_rng(7000 + b)
        ms_.append(synth.spot_amplitude(h, w, int(rng.integers(1, 201)), 2.0, 0.5, 1.0, rng))
        ps_.append(synth.uniform_phase(h, w, rng))
    md = torch.from_numpy(np.stack(ms_)).to(dev)
    pd = torch.from_numpy(np.stack(ps_)).to(dev)
    plan = binding.PhaseMask(h, w, device=dev)
    out = torch.empty_like(pd)
    hist = torch.empty((count, 2 * n_iter + 1), dtype=torch.float64, device=dev)
    for _ in range(3):
        plan.solve_many(md, pd, n_iter, out=out, history=hist)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve_many(md, pd, n_iter, out=out, history=hist)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    gbs = (COL_BYTES_PER_PX + ROW_BYTES_PER_PX) * count * h * w * n_iter / t / 1e9
    plan.close()
    return {"masks": count, "n_iter": n_iter, "ms_per_batch": t * 1e3, "ms_per_mask": t * 1e3 / count,
            "masks_per_s": count / t, "gs_iterations_per_s": count * n_iter / t, "algorithmic_gbs": gbs,
            "frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "max_final_error": float(hist[:, -1].max().item())}


def bench_paper_slm(torch, binding, synth, steps=20):
    """The paper's own timing case as context: an 800 x 600 SLM (600 rows of
    800 pixels), 25 iterations, spot target; ms per solve with the target
    resident, and with the target uploaded from pinned host memory first
    (the paper's figure includes its upload).  Also 5 iterations, the
    paper's usable-mask count."""
    spec = synth.SPOTS_800x600
    h, w, n_iter = spec.height, spec.width, spec.n_iter
    m, phi0 = synth.spot_problem(spec)
    dev = torch.device("cuda", 0)
    host_m = torch.from_numpy(m).pin_memory()
    md = host_m.to(dev)
    pd = torch.from_numpy(phi0).to(dev)
    plan = binding.PhaseMask(h, w, device=dev)
    out = torch.empty((h, w), dtype=torch.float32, device=dev)
    res = {"workload": "gs_spots_800x600_25it", "height": h, "width": w, "n_iter": n_iter,
           "paper_ms_incl_upload": 45.0, "paper_gpu": "Tesla C2070 (FP32)"}

    def timed(k, upload):
        hist = torch.empty(2 * k + 1, dtype=torch.float64, device=dev)
        for _ in range(30):  # warm-up runs exactly what is timed (the first pinned uploads are slow)
            if upload:
                md.copy_(host_m, non_blocking=True)
            plan.solve(md, pd, k, out=out, history=hist)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            if upload:
                md.copy_(host_m, non_blocking=True)
            plan.solve(md, pd, k, out=out, history=hist)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, float(hist[-1].item())

    res["ms_per_mask"], res["final_fourier_error"] = timed(n_iter, False)
    res["ms_per_mask_incl_upload"], _ = timed(n_iter, True)
    res["ms_per_mask_5it_incl_upload"], _ = timed(5, True)
    res["speedup_vs_paper"] = res["paper_ms_incl_upload"] / res["ms_per_mask_incl_upload"]
    # a uniform batch of the panel's masks (phasemask_solve_many): every
    # pass one launch over all masks
    res["many"] = bench_many(torch, binding, synth, h, w, n_iter, 16, steps)
    # the iterate exchange alone (the passes in copy mode), per iteration
    xbuf = torch.zeros((h, w), dtype=torch.complex64, device=dev)
    plan.probe_exchange(xbuf, 10)
    res["exchange_us_per_iteration"] = plan.probe_exchange(xbuf, 200) * 1e3 / 200
    plan.close()
    return res


def bench_other_configs(torch, binding, synth, steps=20):
    """The other one-mask spot workloads: 64 x 64 (5 spots, 100 iterations),
    512 x 512 (20 spots, 50 iterations) and the larger 2048 x 2048 (100
    spots, 50 iterations) and 4096 x 4096 (100 spots, 20 iterations), each
    one graph-replayed solve with the FP64 history, inputs resident; ms per
    mask and the final Fourier error."""
    dev = torch.device("cuda", 0)
    res = {}
    for name, spec in (("spots64x100", synth.SPOTS_64), ("spots512x50", synth.SPOTS_512),
                       ("spots2048x50", synth.SPOTS_2048), ("spots4096x20", synth.SPOTS_4096)):
        m, phi0 = synth.spot_problem(spec)
        md = torch.from_numpy(m).to(dev)
        pd = torch.from_numpy(phi0).to(dev)
        plan = binding.PhaseMask(spec.height, spec.width, device=dev)
        out = torch.empty_like(pd)
        hist = torch.empty(2 * spec.n_iter + 1, dtype=torch.float64, device=dev)
        for _ in range(3):
            plan.solve(md, pd, spec.n_iter, out=out, history=hist)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.solve(md, pd, spec.n_iter, out=out, history=hist)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[name] = {"height": spec.height, "width": spec.width, "n_iter": spec.n_iter, "ms_per_mask": ms,
                     "us_per_iteration": ms * 1e3 / spec.n_iter, "final_fourier_error": float(hist[-1].item())}
        plan.close()
    return res


def bench_next_rows(torch, binding, synth, m, phi0, plan_steps=10, reps=100):
    """The other device entry points on the same 1024 x 1024 workload: RAAR
    (100 iterations), the paper's initial mask, the physical error of Eq. 8,
    and a GS solve under a Gaussian illumination p (with the pass timings of
    its row pass, which also reads p).  Algorithmic bytes per pixel: RAAR
    iteration 20 (column) + 32 (row: iterate and the point x in and out);
    illuminated GS iteration 20 + 20 (row also reads p)."""
    h, w = m.shape
    npx = h * w
    n_iter = 100
    dev = torch.device("cuda", 0)
    md = torch.from_numpy(m).to(dev)
    pd = torch.from_numpy(phi0).to(dev)
    plan = binding.PhaseMask(h, w, device=dev)
    out = torch.empty((h, w), dtype=torch.float32, device=dev)

    def per_call(fn, k=plan_steps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    res = {"workload": "gs_spots_1024x1024", "n_iter": n_iter}
    ms = per_call(lambda: plan.solve_raar(md, pd, n_iter, 0.9, out=out))
    res["raar"] = {"beta": 0.9, "ms_per_mask": ms,
                   "algorithmic_gbs": (20 + 32) * npx * n_iter / (ms * 1e-3) / 1e9}
    res["initial_phase_ms"] = per_call(lambda: plan.initial_phase(md, out=out))
    res["physical_error_ms"] = per_call(lambda: plan.physical_error(md, pd))
    p = torch.from_numpy(synth.gaussian_illumination(h, w, waist=0.4)).to(dev)
    plan.set_illumination(p)
    ms = per_call(lambda: plan.solve(md, pd, n_iter, out=out))
    col_ms, row_ms = plan.time_passes(md, pd, reps=reps)
    res["illumination"] = {"profile": "gaussian waist 0.4", "ms_per_mask": ms,
                           "passes_us": {"column": col_ms * 1e3, "row": row_ms * 1e3},
                           "row_gbs": 20 * npx / (row_ms * 1e-3) / 1e9,
                           "algorithmic_gbs": 40 * npx * n_iter / (ms * 1e-3) / 1e9}
    plan.close()
    return res


def bench_adjoint(torch, binding, synth, lr, steps=200):
    """16 x 512^2 phases, 50-spot intensity targets I = m^2 scaled to sum N:
    200 Adam steps on the intensity loss versus 200 GS iterations on the
    amplitude m = sqrt(I), compared by the Fourier-plane error E_F of the
    resulting masks."""
    import numpy as np
    batch, n = 16, 512
    it_np, ph_np = synth.intensity_problems(batch=batch, size=n, n_spots=50)
    it_np = (it_np.astype(np.float64) * (n * n / it_np.astype(np.float64).sum(axis=(1, 2), keepdims=True)))
    it_np = it_np.astype(np.float32)
    m_np = np.sqrt(it_np.astype(np.float64)).astype(np.float32)
    dev = torch.device("cuda", 0)
    it_d = torch.from_numpy(it_np).to(dev)
    m_list = [torch.from_numpy(m_np[b]).to(dev) for b in range(batch)]
    ph0 = torch.from_numpy(ph_np).to(dev)
    bp = binding.BatchedPhaseMask([(n, n)] * batch, device=dev)

    def ef_of(phases):
        _, e = bp.solve(m_list, [phases[b] for b in range(batch)], 0)
        return e

    # Adam on the intensity loss, three ways: the library's Adam solve (two
    # fused passes per step, the whole run one graph replay), and PyTorch's
    # fused Adam on the library's loss and adjoint kernels, recorded into a
    # graph per step and run eagerly.
    plan_a = binding.PhaseMask(n, n, device=dev)
    out_a = torch.empty_like(ph0)
    plan_a.solve_adam(it_d, ph0, steps, lr, out=out_a)  # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, loss_hist = plan_a.solve_adam(it_d, ph0, steps, lr, out=out_a)
    torch.cuda.synchronize()
    t_adam = time.perf_counter() - t0

    def torch_adam_run(capture):
        p = ph0.clone().requires_grad_(True)
        st = binding.AdamIntensityStep(p, it_d, lr=lr, capture=capture)  # warms up, then resets
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st.step()
        torch.cuda.synchronize()
        return p, time.perf_counter() - t0
    p_eager, t_torch_eager = torch_adam_run(False)
    p_graph, t_torch_graph = torch_adam_run(True)
    assert torch.equal(p_graph, p_eager), "captured and eager Adam runs differ"
    ef_adam = ef_of(out_a).mean().item()
    ef_torch = ef_of(p_graph.detach()).mean().item()
    # GS on the amplitudes, same initial phases, batched
    outs = [torch.empty((n, n), dtype=torch.float32, device=dev) for _ in range(batch)]
    phs = [ph0[b] for b in range(batch)]
    bp.solve(m_list, phs, steps, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, e_gs = bp.solve(m_list, phs, steps, outs=outs)
    torch.cuda.synchronize()
    t_gs = time.perf_counter() - t0
    ef_gs = e_gs.mean().item()
    # GS iterations (mean history over the batch) needed to reach Adam's error
    hist = torch.zeros(2 * steps + 1, dtype=torch.float64, device=dev)
    plan = binding.PhaseMask(n, n, device=dev)
    for b in range(batch):
        _, h = plan.solve(m_list[b], phs[b], steps)
        hist += h
    ef_hist = (hist[0::2] / batch).cpu().numpy()
    reach = np.nonzero(ef_hist <= ef_adam)[0]
    nu_equal = int(reach[0]) if reach.size else None
    return {
        "workload": "16 x 512^2 phases, 50-spot intensity targets (seeds 500+b), sum I = N",
        "adam": {"steps": steps, "lr": lr, "ms_per_step": t_adam * 1e3 / steps,
                 "total_ms": t_adam * 1e3, "final_fourier_error_mean": ef_adam,
                 "final_loss_mean": float(loss_hist[-1].mean().item()),
                 "launch": "phasemask_solve_adam: one graph, 2 fused passes per step",
                 "algorithmic_gbs": ADAM_FUSED_BYTES_PER_PX * batch * n * n / (t_adam / steps) / 1e9,
                 "torch_adam": {"graph_ms_per_step": t_torch_graph * 1e3 / steps,
                                "eager_ms_per_step": t_torch_eager * 1e3 / steps,
                                "final_fourier_error_mean": ef_torch,
                                "algorithmic_gbs": ADAM_STEP_BYTES_PER_PX * batch * n * n
                                / (t_torch_graph / steps) / 1e9}},
        "gs": {"iterations": steps, "total_ms": t_gs * 1e3, "final_fourier_error_mean": ef_gs},
        "gs_iterations_to_adam_error": nu_equal,
        "gs_ms_to_adam_error": (t_gs * 1e3 * nu_equal / steps) if nu_equal is not None else None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=32,
                    help="iterations of the FP64 oracle timed for the CPU baseline (per rep)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-versus-plain measurement")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched workload (no one-by-one comparison), printing its steps "
                         "and one JSON object: for counter runs under rocprofv3")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the Adam-versus-GS measurement")
    ap.add_argument("--no-paper-slm", action="store_true",
                    help="skip the 800x600 / 25-iteration context measurement")
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip RAAR / initial mask / physical error / illumination timings")
    ap.add_argument("--adam-lr", type=float, default=0.1,
                    help="chosen from {0.01, 0.03, 0.1} by the final Fourier error of the workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 64 MiB device copy 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); masks are independent, "
              "so more GPUs would each run their own share", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        nbytes = 64 << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}))
        return

    from paper_1302_0120_amd import binding, synth

    if args.only_batched:
        print(json.dumps({"batched": bench_batched(torch, binding, synth, args.batched_steps,
                                                   plain_too=False, progress=True)}), flush=True)
        return

    spec = synth.SPOTS_1024
    h, w, n_iter = spec.height, spec.width, spec.n_iter
    npx = h * w
    m, phi0 = synth.spot_problem(spec)
    dev = torch.device("cuda", 0)
    md = torch.from_numpy(m).to(dev)
    pd = torch.from_numpy(phi0).to(dev)
    plan = binding.PhaseMask(h, w, device=dev)
    out = torch.empty((h, w), dtype=torch.float32, device=dev)
    hist = torch.empty(2 * n_iter + 1, dtype=torch.float64, device=dev)

    for _ in range(args.warmup):
        plan.solve(md, pd, n_iter, out=out, history=hist)
    torch.cuda.synchronize()
    # The solves run on torch's current stream (the plan follows it), so
    # these events bracket the timed region on the kernels' own stream.
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        plan.solve(md, pd, n_iter, out=out, history=hist)
    ev1.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    region_ms = ev0.elapsed_time(ev1) / args.steps
    final_ef = float(hist[-1].item())

    # Per-iteration device time inside the timed solves: the difference
    # between the n_iter-iteration solve and a short one of the same plan
    # (same graph shape, so the per-solve work -- target preparation, u^0,
    # final error, finalisation -- cancels).
    n_short = 20
    hist_s = torch.empty(2 * n_short + 1, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        plan.solve(md, pd, n_short, out=out, history=hist_s)
    ev0.record()
    for _ in range(args.steps):
        plan.solve(md, pd, n_short, out=out, history=hist_s)
    ev1.record()
    torch.cuda.synchronize()
    short_ms = ev0.elapsed_time(ev1) / args.steps
    iter_us = (region_ms - short_ms) * 1e3 / (n_iter - n_short)

    # Dominant kernel: the launches' own start/end events over an eager
    # iteration sequence on the same stream give each pass's share of an
    # iteration; its average duration in the timed solves is that share of
    # the per-iteration time above.
    col_ms, row_ms = plan.time_passes(md, pd, reps=args.kernel_reps)
    col_us = iter_us * col_ms / (col_ms + row_ms)
    row_us = iter_us * row_ms / (col_ms + row_ms)
    if col_ms >= row_ms:
        kname, kms, kbytes = "column pass", col_us * 1e-3, COL_BYTES_PER_PX * npx
    else:
        kname, kms, kbytes = "row pass", row_us * 1e-3, ROW_BYTES_PER_PX * npx
    achieved = kbytes / (kms * 1e-3) / 1e9
    traffic = TRAFFIC_BYTES[kname] if kernel_source_hash() == TRAFFIC_SOURCE_HASH else None
    solve_gbs = (COL_BYTES_PER_PX + ROW_BYTES_PER_PX) * npx * n_iter / (ms_per_step * 1e-3) / 1e9
    copy_gbs, copy_us = copy_bandwidth(torch, npx * 8)
    # The iterate exchange alone: the plan's own column and row passes in
    # copy mode (same maps, tiles and launch order, each pass reading what
    # the other wrote on other XCDs), per iteration.
    xbuf = torch.zeros((h, w), dtype=torch.complex64, device=dev)
    plan.probe_exchange(xbuf, 10)
    exchange_us = plan.probe_exchange(xbuf, args.kernel_reps) * 1e3 / args.kernel_reps

    line = {
        "metric": METRIC,
        "value": n_iter * args.steps / dt,
        "unit": "GS it/s (1024x1024 mask)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_mask": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gs_spots_1024x1024_100it", "height": h, "width": w,
                   "n_iter": n_iter, "n_spots": spec.n_spots, "sigma_px": spec.sigma,
                   "amplitude": [spec.amp_low, spec.amp_high], "seed": spec.seed,
                   "history": "fp64 E_F/G per iteration", "launch": "hip graph"},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel_us": kms * 1e3, "bytes_per_launch": kbytes,
                     # measured copy of the same working set (the 8 MiB iterate
                     # read and written), and the kernel's fraction of it
                     "copy_gbs": copy_gbs, "copy_us": copy_us, "frac_of_copy": achieved / copy_gbs,
                     # one iteration's two passes moving their data alone (no
                     # arithmetic), and the iteration's speed relative to it
                     "exchange_us_per_iteration": exchange_us,
                     "frac_of_exchange": exchange_us / iter_us},
        # per-launch durations in the timed solves (per-iteration device
        # time split by the eager launch-event ratio), and the eager ones
        "passes_us": {"column": col_us, "row": row_us},
        "passes_eager_us": {"column": col_ms * 1e3, "row": row_ms * 1e3},
        "iteration_us": iter_us,
        "solve_algorithmic_gbs": solve_gbs,
        "final_fourier_error": final_ef,
        "env": environment(torch),
    }
    if not args.no_batched:
        line["batched"] = bench_batched(torch, binding, synth, args.batched_steps)
        line["batched_uniform_1024"] = bench_batched_uniform(torch, binding, synth, args.batched_steps)
        line["batched_uniform_1024"]["one_mask_kernels"] = bench_many(torch, binding, synth, 1024, 1024, 100, 16,
                                                                      args.batched_steps)
    if not args.no_adjoint:
        line["adjoint"] = bench_adjoint(torch, binding, synth, args.adam_lr)
    if not args.no_paper_slm:
        line["paper_slm"] = bench_paper_slm(torch, binding, synth)
    if not args.no_next_rows:
        line["mfma_probe"] = bench_mfma_probe(torch, binding)
        line["next_rows"] = bench_next_rows(torch, binding, synth, m, phi0)
        line["other_configs"] = bench_other_configs(torch, binding, synth)
    if not args.no_cpu_baseline:
        rate, cdt = cpu_baseline(m, phi0, args.cpu_iters)
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        t32 = cpu_fp32_gs(m, phi0, n_iter, threads)
        line["cpu_baseline"] = {
            "value": rate, "unit": "GS it/s (1024x1024 mask)", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy oracle, first {args.cpu_iters} of the {n_iter} iterations of "
                      f"the same 1024x1024 spot workload, single thread; median of 3 runs after "
                      f"a warm-up, {cdt:.2f} s per run",
            "cpu_model": host_cpu_model(),
            "gpu_over_cpu": line["value"] / rate,
            # the analogue of the paper's multithreaded CPU comparison
            "fp32_multithreaded": {
                "value": n_iter / t32, "unit": "GS it/s (1024x1024 mask)", "cores": threads,
                "ms_per_mask": t32 * 1e3,
                "sample": f"scipy.fft complex64 on {threads} threads, all {n_iter} iterations, "
                          f"no history; median of 3 runs after a warm-up",
                "gpu_over_cpu": line["value"] / (n_iter / t32)}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
