"""GPU test of phasemask_solve_noalloc, the allocation-free variant of
phasemask_solve: through the C ABI, against phasemask_solve on the same
inputs, on two calls in a row (the second smaller, in the scratch array the
first one left behind), with no change in the device's free memory."""
import ctypes

import numpy as np
import pytest

from paper_1302_0120_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pmb():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1302_0120_amd import binding
    return binding


def _problem(h, w, spots, seed):
    rng = np.random.default_rng(seed)
    m = synth.spot_amplitude(h, w, spots, 2.0, 0.5, 1.0, rng)
    phi0 = synth.uniform_phase(h, w, rng)
    return torch.from_numpy(m).cuda(), torch.from_numpy(phi0).cuda()


def _noalloc(pmb, plan, md, pd, n_iter, out, hist):
    """One call through the C ABI; returns the status."""
    return pmb.lib.phasemask_solve_noalloc(plan._h, ctypes.c_void_p(md.data_ptr()),
                                           ctypes.c_void_p(pd.data_ptr()), int(n_iter),
                                           ctypes.c_void_p(out.data_ptr()),
                                           None if hist is None else ctypes.c_void_p(hist.data_ptr()))


def test_noalloc_matches_solve_on_two_calls(pmb):
    cases = [((1024, 1024), 100, 3), ((256, 256), 7, 4)]  # second call smaller
    runs = []
    for (h, w), n, seed in cases:
        print(f"noalloc: {h}x{w}, {n} iterations", flush=True)
        md, pd = _problem(h, w, 40, seed)
        plan = pmb.PhaseMask(h, w)
        ref, href = plan.solve(md, pd, n)
        torch.cuda.synchronize()
        out = torch.full_like(pd, float("nan"))
        hist = torch.full((2 * n + 1,), float("nan"), dtype=torch.float64, device="cuda")
        runs.append((plan, md, pd, n, out, hist, ref.clone(), href.clone()))
    # eager launches on this stream once before the memory reading (the
    # runtime may set up per-stream launch state on its first eager launch)
    warm = pmb.PhaseMask(256, 256, flags=pmb.PM_FLAG_NO_GRAPH)
    warm.solve(runs[1][1], runs[1][2], 1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for plan, md, pd, n, out, hist, _, _ in runs:
        plan._stream()
        assert _noalloc(pmb, plan, md, pd, n, out, hist) == 0, pmb.lib.phasemask_last_error()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"noalloc: device free memory before {free0}, after {free1}", flush=True)
    assert free1 == free0
    for plan, md, pd, n, out, hist, ref, href in runs:
        print(f"noalloc {plan.shape}: output equal {torch.equal(out, ref)}, history equal "
              f"{torch.equal(hist, href)}", flush=True)
        assert torch.equal(out, ref) and torch.equal(hist, href)
    # without a history, and once more after the smaller call
    plan, md, pd, n, out, _, ref, _ = runs[0]
    out.fill_(float("nan"))
    assert _noalloc(pmb, plan, md, pd, n, out, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_rejects_what_does_not_fit(pmb):
    md, pd = _problem(1024, 1024, 10, 5)
    plan = pmb.PhaseMask(1024, 1024)
    out = torch.empty_like(pd)
    big = 5000
    hist = torch.empty(2 * big + 1, dtype=torch.float64, device="cuda")
    assert _noalloc(pmb, plan, md, pd, big, out, hist) == -1
    assert b"scratch" in pmb.lib.phasemask_last_error()
    md2, pd2 = _problem(2048, 2048, 10, 6)
    plan2 = pmb.PhaseMask(2048, 2048)
    out2 = torch.empty_like(pd2)
    assert _noalloc(pmb, plan2, md2, pd2, 1, out2, None) == -1
    assert b"scratch" in pmb.lib.phasemask_last_error()
    # the plan still works afterwards, through both entry points
    ref, _ = plan.solve(md, pd, 3)
    assert _noalloc(pmb, plan, md, pd, 3, out, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
