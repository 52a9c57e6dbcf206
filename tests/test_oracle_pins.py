"""Pins for the FP64 oracle: each test checks the oracle against something
other than itself -- a brute-force transform, a closed form, a theorem about
projections, an invariance of the method, or finite differences -- so that a
dropped term, a wrong sign or index, or a transposed operand fails one of
them.  CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import gs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# The transform F (Eq. 2, Eq. 4b): brute force and closed forms
# --------------------------------------------------------------------------

def _brute_dft2(u, sign):
    """Textbook O(N^2) 2-D DFT from its defining double sum, unitary scale."""
    h, w = u.shape
    out = np.zeros((h, w), dtype=np.complex128)
    ys = np.arange(h)[:, None]
    xs = np.arange(w)[None, :]
    for ky in range(h):
        for kx in range(w):
            ph = sign * 2.0 * math.pi * (ky * ys / h + kx * xs / w)
            out[ky, kx] = np.sum(u * (np.cos(ph) + 1j * np.sin(ph)))
    return out / math.sqrt(h * w)


@pytest.mark.parametrize("shape", [(16, 16), (8, 16), (16, 8)])
def test_dft_matches_brute_force(shape):
    rng = np.random.default_rng(7)
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    tol = 1e-12 * np.linalg.norm(u)
    assert np.max(np.abs(gs.F(u) - _brute_dft2(u, -1.0))) <= tol
    assert np.max(np.abs(gs.F_inv(u) - _brute_dft2(u, +1.0))) <= tol


@pytest.mark.parametrize("shape", [(8, 16), (16, 8), (32, 32)])
def test_dft_closed_forms(shape):
    h, w = shape
    n = h * w
    # delta at the origin -> constant 1/sqrt(N)
    d = np.zeros(shape, complex)
    d[0, 0] = 1.0
    assert np.allclose(gs.F(d), np.full(shape, 1 / math.sqrt(n)), atol=1e-15, rtol=0)
    # constant -> sqrt(N) delta
    c = np.ones(shape, complex)
    e = np.zeros(shape, complex)
    e[0, 0] = math.sqrt(n)
    assert np.max(np.abs(gs.F(c) - e)) <= 1e-13
    # plane wave exp(+2 pi i (a y/h + b x/w)) -> sqrt(N) delta at (a, b):
    # pins the forward sign and which axis is rows
    a, b = 3, 5
    ys = np.arange(h)[:, None]
    xs = np.arange(w)[None, :]
    pw = np.exp(2j * math.pi * (a * ys / h + b * xs / w))
    e = np.zeros(shape, complex)
    e[a, b] = math.sqrt(n)
    assert np.max(np.abs(gs.F(pw) - e)) <= 1e-12


def test_parseval_and_inverse():
    rng = np.random.default_rng(8)
    u = rng.standard_normal((32, 64)) + 1j * rng.standard_normal((32, 64))
    U = gs.F(u)
    assert abs(np.linalg.norm(U) - np.linalg.norm(u)) <= 1e-13 * np.linalg.norm(u)
    assert np.max(np.abs(gs.F_inv(U) - u)) <= 1e-13 * np.linalg.norm(u)


# --------------------------------------------------------------------------
# Projections P_S (Eq. 4a) and P_M (Eq. 4b, Eq. 5)
# --------------------------------------------------------------------------

def test_PS_modulus_phase_idempotent():
    rng = np.random.default_rng(9)
    u = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    v = gs.P_S(u)
    assert np.max(np.abs(np.abs(v) - 1.0)) <= 1e-15
    assert np.max(np.abs(np.angle(v) - np.angle(u))) <= 1e-15
    assert np.max(np.abs(gs.P_S(v) - v)) <= 1e-15
    p = rng.uniform(0.5, 2.0, (8, 8))
    vp = gs.P_S(u, p)
    assert np.max(np.abs(np.abs(vp) - p)) <= 1e-15


def test_PS_is_nearest_point_brute_force():
    """No random point of S on a 4x4 grid is closer to u than P_S u."""
    rng = np.random.default_rng(10)
    u = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    d0 = np.linalg.norm(u - gs.P_S(u))
    thetas = rng.uniform(0, 2 * math.pi, (10000, 4, 4))
    d = np.linalg.norm((u[None] - np.exp(1j * thetas)).reshape(10000, -1), axis=1)
    assert d0 < d.min()


def test_PS_with_illumination_is_nearest_point_brute_force():
    """With an illumination p (Eq. 1), S = {|z| = p}: no random point of S
    is closer to u than P_S(u, p); a pixel with p = 0 maps to 0."""
    rng = np.random.default_rng(12)
    u = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    p = rng.uniform(0.2, 2.0, (4, 4))
    p[2, 1] = 0.0
    v = gs.P_S(u, p)
    assert v[2, 1] == 0.0
    d0 = np.linalg.norm(u - v)
    thetas = rng.uniform(0, 2 * math.pi, (10000, 4, 4))
    d = np.linalg.norm((u[None] - p[None] * np.exp(1j * thetas)).reshape(10000, -1), axis=1)
    assert d0 < d.min()


def test_PS_zero_tie_break():
    u = np.zeros((4, 4), complex)
    u[1, 2] = 3 - 4j
    v = gs.P_S(u)
    assert v[0, 0] == 1.0 and v[3, 3] == 1.0
    assert abs(v[1, 2] - (0.6 - 0.8j)) <= 1e-15


def test_PM_lands_in_M_and_is_idempotent():
    rng = np.random.default_rng(11)
    m = rng.uniform(0, 1, (16, 32))
    mt = gs.matched_target(m)
    u = rng.standard_normal((16, 32)) + 1j * rng.standard_normal((16, 32))
    v = gs.P_M(u, mt)
    assert np.max(np.abs(np.abs(gs.F(v)) - mt)) <= 1e-12
    assert np.max(np.abs(gs.P_M(v, mt) - v)) <= 1e-12
    # energy matching: ||m~|| = sqrt(N) = ||p||
    assert abs(np.linalg.norm(mt) - math.sqrt(m.size)) <= 1e-12


def test_PM_is_nearest_point_brute_force():
    """No random point of M (F^{-1} of m~ with random phases) beats P_M u."""
    rng = np.random.default_rng(12)
    m = rng.uniform(0, 1, (4, 4))
    mt = gs.matched_target(m)
    u = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    d0 = np.linalg.norm(u - gs.P_M(u, mt))
    thetas = rng.uniform(0, 2 * math.pi, (10000, 4, 4))
    cands = gs.F_inv(mt[None] * np.exp(1j * thetas))
    d = np.linalg.norm((u[None] - cands).reshape(10000, -1), axis=1)
    assert d0 < d.min()


def test_constant_phase_tie_break():
    """A constant field has exact zeros off DC, so Eq. 5 takes theta = 0 there:
    V_k = m~_k for k != 0, and V_0 = m~_0 exp(i c)."""
    c = 0.7
    rng = np.random.default_rng(13)
    m = rng.uniform(0.1, 1, (16, 16))
    mt = gs.matched_target(m)
    U = gs.F(np.full((16, 16), np.exp(1j * c)))
    V = gs.M_hat(U, mt)
    expect = mt.astype(complex)
    expect[0, 0] = mt[0, 0] * np.exp(1j * c)
    assert np.max(np.abs(V - expect)) <= 1e-15


# --------------------------------------------------------------------------
# The iteration (Eq. 6), its error norms (Eq. 7) and invariances
# --------------------------------------------------------------------------

def _spots(h, w, seed, k=5):
    from paper_1302_0120_amd import synth
    rng = np.random.default_rng(seed)
    m = synth.spot_amplitude(h, w, k, 1.5, 1.0, 1.0, rng)
    phi = synth.uniform_phase(h, w, rng)
    return m, phi


def test_history_equals_distances():
    """E_F^nu = ||u^nu - P_M u^nu|| / sqrt N and G^nu = ||P_M u^nu - u^{nu+1}|| / sqrt N,
    measured in the SLM plane (the oracle measures them in the Fourier plane)."""
    m, phi = _spots(32, 64, 1)
    n = m.size
    mt = gs.matched_target(m)
    res = gs.gs_solve(m, phi, 6)
    h = res["history"]
    u = np.exp(1j * phi.astype(np.float64))
    for nu in range(6):
        v = gs.P_M(u, mt)
        u_next = gs.P_S(v)
        assert abs(h[2 * nu] - np.linalg.norm(u - v) / math.sqrt(n)) <= 1e-12
        assert abs(h[2 * nu + 1] - np.linalg.norm(v - u_next) / math.sqrt(n)) <= 1e-12
        u = u_next
    assert np.max(np.abs(u - res["u"])) <= 1e-12
    assert abs(h[12] - np.linalg.norm(u - gs.P_M(u, mt)) / math.sqrt(n)) <= 1e-12


def test_monotone_chain():
    """For alternating projections d(u,M) >= d(P_M u, S) >= d(P_S P_M u, M) >= ...:
    each step's distance is at most the previous one (nearest-point property)."""
    m, phi = _spots(64, 64, 1)
    h = gs.gs_solve(m, phi, 100)["history"]
    assert np.all(np.diff(h) <= 1e-12)
    assert h[-1] < h[0]


def test_unnormalised_transforms_and_target_scale_give_same_iterates():
    """The device path runs unnormalised FFTs with a rescaled target and never
    divides by N; the iterates must not change."""
    m, phi = _spots(32, 32, 2)
    res = gs.gs_solve(m, phi, 10)
    u = np.exp(1j * phi.astype(np.float64))
    m_raw = 7.3 * m.astype(np.float64)
    for _ in range(10):
        U = np.fft.fft2(u)            # unnormalised forward
        V = m_raw * U / np.abs(U)
        w = np.fft.ifft2(V) * u.size  # unnormalised inverse
        u = w / np.abs(w)
    assert np.max(np.abs(u - res["u"])) <= 1e-12


def test_equivariances():
    m, phi = _spots(32, 32, 3)
    phi = phi.astype(np.float64)
    base = gs.gs_solve(m, phi, 8)
    # global phase: u^nu -> u^nu exp(i a), same errors
    a = 0.9
    r = gs.gs_solve(m, phi + a, 8)
    assert np.max(np.abs(r["u"] - base["u"] * np.exp(1j * a))) <= 1e-12
    assert np.max(np.abs(r["history"] - base["history"])) <= 1e-12
    # circular shift of the SLM field: |F u| unchanged, iterates shifted
    r = gs.gs_solve(m, np.roll(phi, (5, -3), axis=(0, 1)), 8)
    assert np.max(np.abs(r["u"] - np.roll(base["u"], (5, -3), axis=(0, 1)))) <= 1e-12
    # twin: conj(u(-x)) has the conjugate spectrum, same modulus
    twin = -np.roll(phi[::-1, ::-1], (1, 1), axis=(0, 1))
    r = gs.gs_solve(m, twin, 8)
    base_twin = np.conj(np.roll(base["u"][::-1, ::-1], (1, 1), axis=(0, 1)))
    assert np.max(np.abs(r["u"] - base_twin)) <= 1e-12


def _consistent(h, w, seed_true=31, seed_init=32):
    rng = np.random.default_rng(seed_true)
    phit = rng.uniform(0, 2 * math.pi, (h, w))
    m = np.abs(np.fft.fft2(np.exp(1j * phit)))  # |F| of a known mask, any scale
    return m, phit, np.random.default_rng(seed_init)


def test_consistent_target_fixed_point():
    """Started at a solution of S cap M the iteration stays there: E_F ~ 0."""
    m, phit, _ = _consistent(64, 64)
    h = gs.gs_solve(m, phit, 20)["history"]
    assert h.max() <= 1e-13


def test_consistent_target_local_convergence():
    """Started near a solution the error falls monotonically towards 0."""
    m, phit, rng = _consistent(64, 64)
    phi0 = phit + rng.uniform(-0.3, 0.3, phit.shape)
    h = gs.gs_solve(m, phi0, 100)["history"]
    assert np.all(np.diff(h) <= 1e-12)
    assert h[0] > 0.05 and h[-1] <= 5e-3


def test_mask_errors_match_history():
    m, phi = _spots(32, 32, 4)
    res = gs.gs_solve(m, phi, 3)
    ef, g = gs.mask_errors(m, phi)
    assert abs(ef - res["history"][0]) <= 1e-14
    assert abs(g - res["history"][1]) <= 1e-14
    assert gs.gs_solve(m, phi, 0)["history"].shape == (1,)


def test_output_phase_in_range_and_unit_modulus():
    m, phi = _spots(32, 32, 5)
    res = gs.gs_solve(m, phi, 5)
    assert np.all(res["phi"] <= math.pi) and np.all(res["phi"] > -math.pi)
    assert np.max(np.abs(np.abs(res["u"]) - 1.0)) <= 1e-15


# --------------------------------------------------------------------------
# Physical error, Eq. 8
# --------------------------------------------------------------------------

def _golden_tolerances():
    vals = {}
    with open(os.path.join(GOLDEN, "physical_error_tolerances.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_physical_error_closed_form():
    """Target = one lit pixel at b; mask = plane wave lighting pixel a != b.
    The lit pixel is fully off: E_lit = t_d / t_l - t_d.  The dark pixel a
    carries normalised intensity 1: E_dark = 1 - t_d."""
    tol = _golden_tolerances()
    t_l, t_d = tol["t_lit"], tol["t_dark"]
    h, w = 8, 16
    a, b = (2, 3), (5, 1)
    ys = np.arange(h)[:, None]
    xs = np.arange(w)[None, :]
    u = np.exp(2j * math.pi * (a[0] * ys / h + a[1] * xs / w))
    m = np.zeros((h, w))
    m[b] = 1.0
    e_lit, e_dark = gs.physical_error(m, u, t_l, t_d)
    assert abs(e_lit - (t_d / t_l - t_d)) <= 1e-15
    assert abs(e_dark - (1.0 - t_d)) <= 1e-12
    # consistent target: no violation at all
    m2 = np.zeros((h, w))
    m2[a] = 1.0
    assert gs.physical_error(m2, u, t_l, t_d) == (0.0, 0.0)


def test_physical_error_intensity_reading():
    """Eq. 8 compares intensities (squared moduli), each normalised to its
    peak; the lit set is where the target intensity exceeds t_d.  A
    non-degenerate closed form tells intensities from amplitudes apart:

    * target amplitudes 1 at k1, 1/2 at k2, 1/100 at k4, 0 elsewhere, so the
      normalised target intensities are 1, 1/4 and 1e-4 (k4 is dark, since
      1e-4 < t_d, although its amplitude ratio 1e-2 exceeds t_d);
    * mask u = a e1 + b e2 + c e3 of plane waves at k1, k2, k3 (k3 dark),
      whose unitary transform is sqrt(N) (a, b, c) at (k1, k2, k3), so the
      normalised reconstructed intensities are 1, (b/a)^2, (c/a)^2, 0.

    Lit k1 matches exactly; lit k2 deviates by rel = |1/4 - (b/a)^2| / (1/4)
    and costs t_d rel / t_l - t_d; dark k3 costs (c/a)^2 - t_d; dark k4 has
    no reconstructed light.  An amplitude reading (|F u| and m) gives other
    numbers for every one of these terms."""
    tol = _golden_tolerances()
    t_l, t_d = tol["t_lit"], tol["t_dark"]
    h, w = 8, 16
    k1, k2, k3, k4 = (1, 2), (3, 7), (6, 11), (4, 0)
    a, b, c = 2.0, 1.6, 0.2          # b/a = 0.8, c/a = 0.1
    ys = np.arange(h)[:, None]
    xs = np.arange(w)[None, :]

    def wave(k):
        return np.exp(2j * math.pi * (k[0] * ys / h + k[1] * xs / w))

    u = a * wave(k1) + b * wave(k2) + c * wave(k3)
    m = np.zeros((h, w))
    m[k1], m[k2], m[k4] = 1.0, 0.5, 0.01
    e_lit, e_dark = gs.physical_error(m, u, t_l, t_d)
    rel = abs(0.25 - 0.64) / 0.25
    assert abs(e_lit - (t_d * rel / t_l - t_d)) <= 1e-14
    assert abs(e_dark - (0.01 - t_d)) <= 1e-14
    # the amplitude reading would give these instead (far outside the bounds)
    rel_amp = abs(0.5 - 0.8) / 0.5
    assert abs(e_lit - (t_d * rel_amp / t_l - t_d)) > 1e-4
    assert abs(e_dark - (0.1 - t_d)) > 1e-2


# --------------------------------------------------------------------------
# Intensity-loss gradient (the differentiable form beside the projections)
# --------------------------------------------------------------------------

def test_intensity_gradient_vs_finite_differences():
    rng = np.random.default_rng(5)
    n = 64
    phi = rng.uniform(0, 2 * math.pi, (n, n))
    it = rng.uniform(0, 2, (n, n))
    it *= (n * n) / it.sum()
    g = gs.intensity_loss_grad(phi, it)
    hstep = 1e-6
    for _ in range(8):
        j = tuple(rng.integers(0, n, 2))
        pp = phi.copy()
        pm = phi.copy()
        pp[j] += hstep
        pm[j] -= hstep
        fd = (gs.intensity_loss(pp, it) - gs.intensity_loss(pm, it)) / (2 * hstep)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])) + 1e-6 * np.abs(g).max()


def test_intensity_gradient_invariants():
    rng = np.random.default_rng(6)
    phi = rng.uniform(0, 2 * math.pi, (32, 32))
    it = rng.uniform(0, 2, (32, 32))
    g = gs.intensity_loss_grad(phi, it)
    # global-phase invariance of L: the gradient sums to zero
    assert abs(g.sum()) <= 1e-9 * np.abs(g).sum()
    # at an exact solution (I = |F e^{i phi}|^2) the gradient vanishes
    it_exact = np.abs(gs.F(np.exp(1j * phi))) ** 2
    assert np.abs(gs.intensity_loss_grad(phi, it_exact)).max() <= 1e-12
    assert gs.intensity_loss(phi, it_exact) <= 1e-24


def test_stored_history_regression():
    """The oracle still reproduces the stored history of the 64x64 spot case
    (written by tests/golden/make_golden.py from the oracle itself): guards
    against unintended drift of the checker."""
    from paper_1302_0120_amd import synth
    stored = np.loadtxt(os.path.join(GOLDEN, "gs_spots64_history.txt"))
    m, phi0 = synth.spot_problem(synth.SPOTS_64)
    h = gs.gs_solve(m, phi0, 100)["history"]
    assert stored.shape == h.shape
    assert np.max(np.abs(h - stored)) <= 1e-13


# --------------------------------------------------------------------------
# General illumination p (Eq. 1), RAAR, the paper's initial mask
# --------------------------------------------------------------------------

def test_general_illumination_distances_and_chain():
    """With p != 1 the history still equals SLM-plane distances relative to
    ||p||, the iterates keep modulus p, and the chain is monotone."""
    m, phi = _spots(32, 32, 6)
    rng = np.random.default_rng(61)
    pp = rng.uniform(0.3, 1.5, m.shape)
    res = gs.gs_solve(m, phi, 8, p=pp)
    h = res["history"]
    mt = gs.matched_target(m, pp)
    pn = np.linalg.norm(pp)
    assert abs(np.linalg.norm(mt) - pn) <= 1e-12 * pn
    u = pp * np.exp(1j * phi.astype(np.float64))
    for nu in range(8):
        v = gs.P_M(u, mt)
        un = gs.P_S(v, pp)
        assert abs(h[2 * nu] - np.linalg.norm(u - v) / pn) <= 1e-12
        assert abs(h[2 * nu + 1] - np.linalg.norm(v - un) / pn) <= 1e-12
        u = un
    assert np.max(np.abs(np.abs(res["u"]) - pp)) <= 1e-13
    assert np.all(np.diff(h) <= 1e-12)
    # p = 1 given explicitly reproduces the phase-only solve
    r1 = gs.gs_solve(m, phi, 8, p=np.ones_like(pp))
    r0 = gs.gs_solve(m, phi, 8)
    assert np.max(np.abs(r1["history"] - r0["history"])) <= 1e-15


def test_raar_reductions():
    """beta = 1/2: x+ = P_S(2 P_M x - x)/2 + x/2 (the average of x and the
    reflection step), checked step by step; at a solution of S cap M every
    beta leaves x fixed; RAAR does not blow up and its shadow improves on a
    consistent target from a nearby start."""
    m, phi = _spots(16, 16, 7)
    mt = gs.matched_target(m)
    x = np.exp(1j * phi.astype(np.float64))
    res = gs.raar_solve(m, phi, 3, 0.5)
    for _ in range(3):
        pm = gs.P_M(x, mt)
        x = 0.5 * gs.P_S(2 * pm - x) + 0.5 * x
    assert np.max(np.abs(x - res["x"])) <= 1e-12
    assert res["history"].shape == (4,)
    rng = np.random.default_rng(41)
    phit = rng.uniform(0, 2 * np.pi, (32, 32))
    mc = np.abs(gs.F(np.exp(1j * phit)))
    for beta in (0.5, 0.9, 1.0):
        r = gs.raar_solve(mc, phit, 5, beta)
        assert r["history"].max() <= 1e-13
    r = gs.raar_solve(mc, phit + rng.uniform(-0.3, 0.3, phit.shape), 60, 0.9)
    assert r["history"][-1] < 0.5 * r["history"][0]


def test_paper_initial_phase():
    """A single lit pixel at frequency (a, b) back-propagates to the plane
    wave exp(+2 pi i (a y/h + b x/w)): the initial mask is that wave's phase.
    A target lit everywhere back-propagates to sqrt(N) delta_0: phase 0."""
    h, w = 16, 32
    a, b = 3, 5
    m = np.zeros((h, w))
    m[a, b] = 2.0
    phi = gs.paper_initial_phase(m)
    ys = np.arange(h)[:, None]
    xs = np.arange(w)[None, :]
    want = np.exp(2j * np.pi * (a * ys / h + b * xs / w))
    assert np.max(np.abs(np.exp(1j * phi) - want)) <= 1e-12
    assert np.max(np.abs(gs.paper_initial_phase(np.ones((h, w))))) == 0.0


def test_paper_initial_phase_thresholds_intensity():
    """The 1-bit target is lit where the normalised INTENSITY m^2 / max m^2
    exceeds t_d.  A second pixel whose amplitude ratio r lies between t_d
    and sqrt(t_d) is dark under that reading (r^2 < t_d) although r > t_d:
    the initial mask stays the single plane wave of the first pixel.  With
    r above sqrt(t_d) the pixel is lit, and the back-propagated pattern is
    the sum of two plane waves, whose phase differs."""
    t_d = 3e-4
    h, w = 16, 32
    a, b = (3, 5), (7, 2)
    ys = np.arange(h)[:, None]
    xs = np.arange(w)[None, :]
    want = np.exp(2j * np.pi * (a[0] * ys / h + a[1] * xs / w))
    m = np.zeros((h, w))
    m[a] = 1.0
    m[b] = 0.005                      # t_d < 0.005 < sqrt(t_d) = 0.0173
    phi = gs.paper_initial_phase(m, t_d)
    assert np.max(np.abs(np.exp(1j * phi) - want)) <= 1e-12
    m[b] = 0.02                       # 0.02^2 = 4e-4 > t_d: lit
    two = want + np.exp(2j * np.pi * (b[0] * ys / h + b[1] * xs / w))
    phi2 = gs.paper_initial_phase(m, t_d)
    nz = np.abs(two) > 1e-3
    assert np.max(np.abs(np.exp(1j * phi2[nz]) - two[nz] / np.abs(two[nz]))) <= 1e-9
    assert np.max(np.abs(np.exp(1j * phi2) - want)) > 0.5


def test_one_iteration_sensitivity_rule():
    """The tolerance rule of the one-iteration parity tests: on the small
    spot cases the oracle's own change under an FP32-level perturbation of
    phi^0 is far below the stated 1e-5 (so the literal bound applies), and
    a perturbation of zero changes nothing."""
    import parity_util
    from paper_1302_0120_amd import synth
    for h, w in [(16, 16), (64, 64), (32, 128)]:
        rng = np.random.default_rng(100 + h + w)
        m = synth.spot_amplitude(h, w, 8, 2.0, 0.5, 1.0, rng)
        phi0 = synth.uniform_phase(h, w, rng)
        tol, s = parity_util.one_iteration_tolerance(m, phi0)
        assert s < 1e-6 and tol == 1e-5
    old = parity_util.EPS32
    try:
        parity_util.EPS32 = 0.0
        assert parity_util.oracle_sensitivity(m, phi0) == 0.0
    finally:
        parity_util.EPS32 = old


def test_start_from_a_field():
    """Eq. 6 from a given field u^0.  P_M keeps only the phase of F u
    (Eq. 5), so it is unchanged when u is scaled by c > 0: from u^0 =
    2 exp(i phi) the iterates u^1, u^2, ... are those from exp(i phi) and
    G^0 is unchanged, while E_F^0 measures |F u^0| = 2 |F exp(i phi)|."""
    m, phi = _spots(16, 32, 8)
    n = m.size
    a = gs.gs_solve(m, phi, 4)
    b = gs.gs_solve(m, None, 4, u0=2.0 * np.exp(1j * phi.astype(np.float64)))
    assert np.max(np.abs(a["u"] - b["u"])) <= 1e-12
    assert np.max(np.abs(a["history"][1:] - b["history"][1:])) <= 1e-12
    mt = gs.matched_target(m)
    U = gs.F(np.exp(1j * phi.astype(np.float64)))
    assert abs(b["history"][0] - np.linalg.norm(2.0 * np.abs(U) - mt) / math.sqrt(n)) <= 1e-12
    with pytest.raises(ValueError):
        gs.gs_solve(m, phi, 1, u0=np.exp(1j * phi))


def _adam_problem(n=16, seed=77):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:n, 0:n]
    m = np.zeros((n, n))
    for cy, cx in rng.uniform(n / 4, 3 * n / 4, (3, 2)):
        m += np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2 * 1.5 ** 2))
    it = m * m
    it *= n * n / it.sum()
    phi0 = rng.uniform(0.0, 2.0 * np.pi, (n, n))
    return it, phi0


def test_adam_first_step_closed_form():
    """Adam's bias corrections make the first step lr g / (|g| + eps) in
    every coordinate (Kingma and Ba, Sec. 2: m_hat = g, v_hat = g^2 at t = 1)."""
    it, phi0 = _adam_problem()
    lr, eps = 0.05, 1e-8
    g = gs.intensity_loss_grad(phi0, it)
    out = gs.adam_intensity(phi0, it, 1, lr, eps=eps)
    assert np.max(np.abs(out["phi"] - (phi0 - lr * g / (np.abs(g) + eps)))) <= 1e-15
    # with eps far below |g| every coordinate moves by lr against its gradient
    big = np.abs(g) > 1e3 * eps
    assert big.mean() > 0.9
    assert np.allclose(np.abs(out["phi"] - phi0)[big], lr, rtol=1e-6, atol=0)


def test_adam_matches_torch_adam_in_fp64():
    """An independent implementation (torch.optim.Adam, float64 on the CPU)
    fed the oracle's gradients gives the oracle's trajectory."""
    torch = pytest.importorskip("torch")
    it, phi0 = _adam_problem(seed=78)
    lr, b1, b2, eps, steps = 0.03, 0.9, 0.99, 1e-6, 6
    p = torch.tensor(phi0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(b1, b2), eps=eps)
    for _ in range(steps):
        opt.zero_grad()
        p.grad = torch.tensor(gs.intensity_loss_grad(p.detach().numpy(), it), dtype=torch.float64)
        opt.step()
    out = gs.adam_intensity(phi0, it, steps, lr, b1, b2, eps)
    assert np.max(np.abs(out["phi"] - p.detach().numpy())) <= 1e-12
    assert out["losses"].shape == (steps + 1,)
    assert out["losses"][0] == gs.intensity_loss(phi0, it)


def test_adam_reduces_the_loss():
    it, phi0 = _adam_problem(seed=79)
    out = gs.adam_intensity(phi0, it, 40, 0.02)
    assert out["losses"][-1] < 0.8 * out["losses"][0]
