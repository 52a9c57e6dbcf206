"""Seeded input recipe: determinism, dtypes, draw order, spot placement."""
import numpy as np

from paper_1302_0120_amd import synth


def test_spot_problem_deterministic_fp32():
    m1, p1 = synth.spot_problem(synth.SPOTS_64)
    m2, p2 = synth.spot_problem(synth.SPOTS_64)
    assert m1.dtype == np.float32 and p1.dtype == np.float32
    assert m1.shape == (64, 64) and p1.shape == (64, 64)
    assert np.array_equal(m1, m2) and np.array_equal(p1, p2)
    assert p1.min() >= 0.0 and p1.max() <= np.float32(2 * np.pi)
    assert m1.min() >= 0.0


def test_spots_sit_in_inner_half_of_display_frame():
    rng = np.random.default_rng(0)
    m = synth.spot_amplitude(64, 64, 1, 1.0, 1.0, 1.0, rng)
    disp = np.fft.fftshift(m)            # back to display order
    y, x = np.unravel_index(np.argmax(disp), disp.shape)
    assert 16 <= y <= 48 and 16 <= x <= 48
    assert abs(disp.max() - 1.0) < 0.5


def test_draw_order_centres_amplitudes_phase():
    rng = np.random.default_rng(5)
    c = rng.uniform([8, 8], [24, 24], size=(3, 2))
    a = rng.uniform(0.5, 1.0, size=3)
    ph = rng.uniform(0, 2 * np.pi, size=(32, 32)).astype(np.float32)
    rng2 = np.random.default_rng(5)
    synth.spot_amplitude(32, 32, 3, 2.0, 0.5, 1.0, rng2)
    assert np.array_equal(synth.uniform_phase(32, 32, rng2), ph)
    assert c.shape == (3, 2) and a.shape == (3,)


def test_batched_problem_sizes():
    probs = synth.batched_problems(count=8, sizes=(16, 32), max_spots=4)
    assert len(probs) == 8
    for m, p in probs:
        assert m.shape == p.shape and m.shape[0] in (16, 32)
        assert m.dtype == np.float32
    again = synth.batched_problems(count=8, sizes=(16, 32), max_spots=4)
    assert all(np.array_equal(a[0], b[0]) for a, b in zip(probs, again))


def test_siemens_star_structure():
    h, w = 128, 256
    m = synth.siemens_star(h, w, n_spokes=12)
    assert m.dtype == np.float32 and m.shape == (h, w)
    assert set(np.unique(m)) <= {0.0, 1.0}
    d = np.fft.fftshift(m)  # display coordinates
    # the centre disc and the frame beyond r_outer are dark
    assert d[h // 2, w // 2] == 0.0 and d[0, 0] == 0.0
    # about half of the annulus is lit (12 bright sectors out of 24)
    yy = np.arange(h)[:, None] - h // 2
    xx = np.arange(w)[None, :] - w // 2
    r = np.hypot(yy, xx)
    ann = (r >= 0.03 * h) & (r <= 0.35 * h)
    assert abs(d[ann].mean() - 0.5) < 0.05
    # bright on the +x axis just past r_inner (angle 0: sin 0 = 0 >= 0)
    assert d[h // 2, w // 2 + 20] == 1.0


def test_gaussian_illumination_profile():
    h, w = 64, 96
    p = synth.gaussian_illumination(h, w, waist=0.4)
    assert p.dtype == np.float32 and p.shape == (h, w)
    assert np.all(p > 0) and p.max() <= 1.0
    # symmetric about the panel centre (between pixels)
    assert np.array_equal(p, p[::-1, :]) and np.array_equal(p, p[:, ::-1])
    pa = synth.gaussian_illumination(h, w, waist=0.4, aperture=0.3)
    assert np.count_nonzero(pa == 0) > 0 and np.all(pa[pa > 0] == p[pa > 0])
