"""Seeded synthetic inputs: spot-pattern targets and random initial phases,
plus a Siemens-star target and a Gaussian illumination profile.

The paper benchmarks on optical stimulation patterns (OSPs) made of bright
spots on a dark background (Sec. IV, first paragraph) and notes random phases
as the alternative initial mask (Sec. IV).  This module draws exactly those
inputs from a seed.  It holds none of the method's arithmetic (no transform,
no projection); both the device path and the CPU checker consume the arrays
it returns, so the two always start from identical fp32 values.

Conventions
-----------
* Arrays are row-major ``[height][width]`` (``height`` = n_y rows, ``width``
  = n_x pixels per row).
* Spots are placed in *display* coordinates (zero frequency at the image
  centre) and the image is then moved to natural DFT order (zero frequency at
  ``[0][0]``) by one ``ifftshift``.
* Draw order from one ``numpy.random.default_rng(seed)``: spot centres
  (k x 2), spot amplitudes (k), then the initial phase (height x width).
* A spot is ``a * exp(-r^2 / (2 sigma^2))``; overlapping spots add; there is
  no background offset.  Each spot is evaluated on a window of radius
  ``40 sigma``: beyond it every term is below ``exp(-800)``, which is exactly
  zero in float64, so the window changes no value.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "spot_amplitude",
    "uniform_phase",
    "SpotSpec",
    "SPOTS_64",
    "SPOTS_512",
    "SPOTS_1024",
    "SPOTS_800x600",
    "SPOTS_2048",
    "SPOTS_4096",
    "spot_problem",
    "batched_problems",
    "intensity_problems",
    "siemens_star",
    "gaussian_illumination",
]


def _spot_image(height: int, width: int, centres: np.ndarray, amps: np.ndarray,
                sigma: float) -> np.ndarray:
    """Sum of Gaussian spots on a display-centred float64 grid."""
    img = np.zeros((height, width), dtype=np.float64)
    rad = int(math.ceil(40.0 * sigma))
    inv = 1.0 / (2.0 * sigma * sigma)
    for (cy, cx), a in zip(centres, amps):
        y0 = max(0, int(math.floor(cy)) - rad)
        y1 = min(height, int(math.floor(cy)) + rad + 2)
        x0 = max(0, int(math.floor(cx)) - rad)
        x1 = min(width, int(math.floor(cx)) + rad + 2)
        yy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
        xx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
        img[y0:y1, x0:x1] += a * np.exp(-(yy * yy + xx * xx) * inv)
    return img


def spot_amplitude(height: int, width: int, n_spots: int, sigma: float,
                   amp_low: float, amp_high: float,
                   rng: np.random.Generator) -> np.ndarray:
    """Target amplitude m (fp32, natural DFT order) made of ``n_spots`` spots.

    Centres are uniform over the inner half of the display frame,
    ``[n/4, 3n/4)`` per axis; amplitudes are uniform in
    ``[amp_low, amp_high]`` (a constant when the two are equal).
    """
    if n_spots < 1:
        raise ValueError("need at least one spot")
    lo = np.array([height / 4.0, width / 4.0])
    hi = np.array([3.0 * height / 4.0, 3.0 * width / 4.0])
    centres = rng.uniform(lo, hi, size=(n_spots, 2))
    amps = rng.uniform(amp_low, amp_high, size=n_spots)
    img = _spot_image(height, width, centres, amps, sigma)
    return np.ascontiguousarray(np.fft.ifftshift(img).astype(np.float32))


def uniform_phase(height: int, width: int, rng: np.random.Generator) -> np.ndarray:
    """Initial phase, uniform on [0, 2 pi), fp32."""
    return rng.uniform(0.0, 2.0 * math.pi, size=(height, width)).astype(np.float32)


@dataclass(frozen=True)
class SpotSpec:
    """One spot-pattern workload: size, spots and iteration count."""
    height: int
    width: int
    n_spots: int
    sigma: float
    amp_low: float
    amp_high: float
    n_iter: int
    seed: int


# 64 x 64, 5 unit spots of sigma 1.5 px, 100 iterations (CPU-sized case).
SPOTS_64 = SpotSpec(64, 64, 5, 1.5, 1.0, 1.0, 100, 1)
# 512 x 512, 20 unit spots of sigma 2 px, 50 iterations.
SPOTS_512 = SpotSpec(512, 512, 20, 2.0, 1.0, 1.0, 50, 2)
# 1024 x 1024, 100 spots of sigma 2 px with amplitudes in [0.5, 1], 100 iterations.
SPOTS_1024 = SpotSpec(1024, 1024, 100, 2.0, 0.5, 1.0, 100, 3)
# The SLM panel of the paper's timing (800 x 600 pixels: 600 rows of 800),
# 25 iterations; 20 spots of sigma 2 px with amplitudes in [0.5, 1].
SPOTS_800x600 = SpotSpec(600, 800, 20, 2.0, 0.5, 1.0, 25, 6)
# Larger masks: 2048 x 2048 (50 iterations) and 4096 x 4096 (20 iterations),
# 100 spots of sigma 2 px with amplitudes in [0.5, 1].
SPOTS_2048 = SpotSpec(2048, 2048, 100, 2.0, 0.5, 1.0, 50, 7)
SPOTS_4096 = SpotSpec(4096, 4096, 100, 2.0, 0.5, 1.0, 20, 8)


def spot_problem(spec: SpotSpec, seed: int | None = None):
    """(target amplitude, initial phase) for a spot workload, both fp32."""
    rng = np.random.default_rng(spec.seed if seed is None else seed)
    m = spot_amplitude(spec.height, spec.width, spec.n_spots, spec.sigma,
                       spec.amp_low, spec.amp_high, rng)
    phi0 = uniform_phase(spec.height, spec.width, rng)
    return m, phi0


def batched_problems(count: int = 64, sizes=(256, 512, 1024), size_seed: int = 4,
                     base_seed: int = 1000, max_spots: int = 200, sigma: float = 2.0):
    """Uneven batch: square masks with sizes drawn uniformly from ``sizes``.

    Mask i uses its own generator seeded ``base_seed + i``: first the spot
    count (uniform on 1..max_spots), then centres, amplitudes in [0.5, 1] and
    the initial phase.  Returns a list of (target, phase) fp32 pairs.
    """
    size_rng = np.random.default_rng(size_seed)
    picks = size_rng.integers(0, len(sizes), size=count)
    out = []
    for i, p in enumerate(picks):
        n = int(sizes[int(p)])
        rng = np.random.default_rng(base_seed + i)
        k = int(rng.integers(1, max_spots + 1))
        m = spot_amplitude(n, n, k, sigma, 0.5, 1.0, rng)
        phi0 = uniform_phase(n, n, rng)
        out.append((m, phi0))
    return out


def intensity_problems(batch: int = 16, size: int = 512, n_spots: int = 50,
                       sigma: float = 2.0, base_seed: int = 500):
    """Targets for intensity-loss phase optimisation: I = m^2 of a spot
    pattern, plus a uniform initial phase, per batch entry (fp32)."""
    ts, ps = [], []
    for b in range(batch):
        rng = np.random.default_rng(base_seed + b)
        m = spot_amplitude(size, size, n_spots, sigma, 0.5, 1.0, rng)
        ts.append((m.astype(np.float64) ** 2).astype(np.float32))
        ps.append(uniform_phase(size, size, rng))
    return np.stack(ts), np.stack(ps)


def siemens_star(height: int, width: int, n_spokes: int = 36, r_outer: float = 0.35,
                 r_inner: float = 0.03) -> np.ndarray:
    """Binary Siemens-star target amplitude (fp32, natural DFT order), the
    resolution pattern of the paper's second experiment (Sec. IV, Fig. 4).

    In display coordinates (centre at ``(height // 2, width // 2)``) a pixel
    is bright (1) when its polar angle t satisfies ``sin(n_spokes t) >= 0``
    and its radius lies in ``[r_inner, r_outer] * min(height, width)``, else
    dark (0).  Deterministic: no random draws.
    """
    if n_spokes < 1:
        raise ValueError("need at least one spoke")
    n = float(min(height, width))
    yy = np.arange(height, dtype=np.float64)[:, None] - height // 2
    xx = np.arange(width, dtype=np.float64)[None, :] - width // 2
    r = np.hypot(yy, xx)
    t = np.arctan2(yy, xx)
    lit = (np.sin(n_spokes * t) >= 0.0) & (r >= r_inner * n) & (r <= r_outer * n)
    return np.ascontiguousarray(np.fft.ifftshift(lit.astype(np.float32)))


def gaussian_illumination(height: int, width: int, waist: float = 0.5,
                          aperture: float | None = None) -> np.ndarray:
    """Illumination amplitude p on the SLM (Eq. 1) of a Gaussian laser beam
    centred on the panel: ``p = exp(-r^2 / (waist * min(height, width))^2)``
    with r measured from ``(height / 2, width / 2)`` in pixels.  With
    ``aperture`` set, p = 0 beyond radius ``aperture * min(height, width)``
    (a circular stop).  fp32, SLM pixel order (no shift).
    """
    n = float(min(height, width))
    yy = np.arange(height, dtype=np.float64)[:, None] + 0.5 - height / 2.0
    xx = np.arange(width, dtype=np.float64)[None, :] + 0.5 - width / 2.0
    r2 = yy * yy + xx * xx
    p = np.exp(-r2 / (waist * n) ** 2)
    if aperture is not None:
        p[r2 > (aperture * n) ** 2] = 0.0
    return np.ascontiguousarray(p.astype(np.float32))
