"""GPU parity of the general illumination amplitude p of Eq. 1 (S = fields of
modulus p) against the FP64 oracle's gs_solve / raar_solve with p.

Fields are compared as p exp(i phi) (the oracle's u), so pixels with p = 0
carry no weight; tolerances are the phase-only ones (one iteration 1e-5
relative L2 and per history entry, final error after a full run 1e-3)."""
import math

import numpy as np
import pytest

from oracle import gs
from paper_1302_0120_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pmb():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1302_0120_amd import binding
    return binding


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _problem(h, w, seed, aperture=None):
    rng = np.random.default_rng(seed)
    m = synth.spot_amplitude(h, w, 15, 2.0, 0.5, 1.0, rng)
    phi0 = synth.uniform_phase(h, w, rng)
    p = synth.gaussian_illumination(h, w, waist=0.4, aperture=aperture)
    return m, phi0, p


def test_uniform_illumination_is_the_phase_only_solve(pmb):
    """p = 1 given explicitly gives bitwise the phases of the phase-only
    solve; None switches back."""
    h, w = 128, 256
    m, phi0, _ = _problem(h, w, 11)
    md, pd = _dev(m), _dev(phi0)
    plan = pmb.PhaseMask(h, w)
    ph0, h0 = plan.solve(md, pd, 7)
    ph0, h0 = ph0.clone(), h0.clone()
    plan.set_illumination(torch.ones(h, w, device="cuda"))
    ph1, h1 = plan.solve(md, pd, 7)
    assert torch.equal(ph0, ph1)
    assert torch.max(torch.abs(h0 - h1) / h0).item() <= 1e-14
    plan.set_illumination(None)
    ph2, h2 = plan.solve(md, pd, 7)
    assert torch.equal(ph0, ph2) and torch.equal(h0, h2)


@pytest.mark.parametrize("shape,aperture", [((64, 64), None), ((256, 128), None), ((512, 512), 0.45),
                                            ((600, 800), None), ((1024, 1024), 0.4), ((1080, 1920), 0.45)])
def test_one_iteration_with_illumination(pmb, shape, aperture):
    h, w = shape
    print(f"illumination one iteration {shape} aperture={aperture}", flush=True)
    m, phi0, p = _problem(h, w, 20 + h + w, aperture)
    plan = pmb.PhaseMask(h, w)
    plan.set_illumination(_dev(p))
    ph, hist = plan.solve(_dev(m), _dev(phi0), 1)
    ref = gs.gs_solve(m, phi0, 1, p=p)
    u = p.astype(np.float64) * np.exp(1j * ph.cpu().numpy().astype(np.float64))
    assert _rel_l2(u, ref["u"]) <= 1e-5
    hg = hist.cpu().numpy()
    assert np.max(np.abs(hg - ref["history"]) / ref["history"]) <= 1e-5, (hg, ref["history"])


def test_full_run_with_illumination(pmb):
    h = w = 512
    m, phi0, p = _problem(h, w, 5)
    plan = pmb.PhaseMask(h, w)
    plan.set_illumination(_dev(p))
    md = _dev(m)
    ph, hist = plan.solve(md, _dev(phi0), 50)
    hg = hist.cpu().numpy()
    hr = gs.gs_solve(m, phi0, 50, p=p)["history"]
    assert abs(hg[-1] - hr[-1]) / hr[-1] <= 1e-3, (hg[-1], hr[-1])
    assert np.max(np.abs(hg[:3] - hr[:3]) / hr[:3]) <= 1e-5
    assert np.all(np.diff(hg) <= 1e-6 * hg[:-1])
    # the reported final error is that of the returned mask under the same p
    e = plan.error(md, ph).cpu().numpy()
    assert abs(e[0] - hg[-1]) / hg[-1] <= 1e-5


def test_siemens_star_with_illumination(pmb):
    """The paper's second target (a Siemens star) under a Gaussian beam:
    final error after 20 iterations within 1e-3 of the oracle."""
    h = w = 256
    m = synth.siemens_star(h, w, n_spokes=24)
    phi0 = synth.uniform_phase(h, w, np.random.default_rng(3))
    p = synth.gaussian_illumination(h, w, waist=0.5)
    plan = pmb.PhaseMask(h, w)
    plan.set_illumination(_dev(p))
    _, hist = plan.solve(_dev(m), _dev(phi0), 20)
    hg = hist.cpu().numpy()
    hr = gs.gs_solve(m, phi0, 20, p=p)["history"]
    assert abs(hg[-1] - hr[-1]) / hr[-1] <= 1e-3, (hg[-1], hr[-1])
    assert np.max(np.abs(hg[:3] - hr[:3]) / hr[:3]) <= 1e-5


def test_error_and_physical_error_with_illumination(pmb):
    h, w = 256, 256
    m, phi0, p = _problem(h, w, 9, aperture=0.45)
    plan = pmb.PhaseMask(h, w)
    plan.set_illumination(_dev(p))
    md, pd = _dev(m), _dev(phi0)
    e = plan.error(md, pd).cpu().numpy()
    ref = gs.gs_solve(m, phi0, 1, p=p)["history"][:2]  # E_F^0, G^0 of u^0 = p exp(i phi0)
    assert np.max(np.abs(e - ref) / ref) <= 1e-5, (e, ref)
    pe = plan.physical_error(md, pd).cpu().numpy()
    pref = gs.physical_error(m, p.astype(np.float64) * np.exp(1j * phi0.astype(np.float64)))
    for k in range(2):
        assert abs(pe[k] - pref[k]) <= 1e-4 * max(pref[k], 1e-6), (k, pe[k], pref[k])


def test_raar_with_illumination(pmb):
    h, w = 128, 128
    m, phi0, p = _problem(h, w, 13)
    plan = pmb.PhaseMask(h, w)
    plan.set_illumination(_dev(p))
    ph, hist = plan.solve_raar(_dev(m), _dev(phi0), 1, 0.7)
    ref = gs.raar_solve(m, phi0, 1, 0.7, p=p)
    u = p.astype(np.float64) * np.exp(1j * ph.cpu().numpy().astype(np.float64))
    assert _rel_l2(u, ref["u"]) <= 1e-5
    assert np.max(np.abs(hist.cpu().numpy() - ref["history"]) / ref["history"]) <= 1e-5


def test_zero_illumination_pixels_keep_a_defined_phase(pmb):
    """Where p = 0 the output phase is that of the projected field before
    the factor p: finite and in [-pi, pi] (FP32 pi rounds up)."""
    h = w = 128
    m, phi0, p = _problem(h, w, 17, aperture=0.3)
    assert np.count_nonzero(p == 0) > 0
    plan = pmb.PhaseMask(h, w)
    plan.set_illumination(_dev(p))
    ph, _ = plan.solve(_dev(m), _dev(phi0), 5)
    o = ph.cpu().numpy()
    assert np.all(np.isfinite(o)) and np.all(np.abs(o) <= np.float32(math.pi))


def test_illumination_argument_errors_and_reuse(pmb):
    """A misaligned illumination pointer is rejected before any work; the
    plan stays usable, and a batched handle refuses illumination."""
    h = w = 64
    m, phi0, p = _problem(h, w, 23)
    plan = pmb.PhaseMask(h, w)
    buf = torch.zeros(h * w + 1, device="cuda")
    st = pmb.lib.phasemask_set_illumination(plan._h, buf.data_ptr() + 4)
    assert st == -1
    ph0, _ = plan.solve(_dev(m), _dev(phi0), 3)
    plan.set_illumination(_dev(p))
    plan.set_illumination(_dev(p))          # a second copy replaces the first
    ph1, h1 = plan.solve(_dev(m), _dev(phi0), 3)
    ref = gs.gs_solve(m, phi0, 3, p=p)["history"]
    assert np.max(np.abs(h1.cpu().numpy()[:3] - ref[:3]) / ref[:3]) <= 1e-5
    plan.set_illumination(None)
    ph2, _ = plan.solve(_dev(m), _dev(phi0), 3)
    assert torch.equal(ph0, ph2)
    bp = pmb.BatchedPhaseMask([(64, 64)])
    assert pmb.lib.phasemask_set_illumination(bp._h, None) == -5
