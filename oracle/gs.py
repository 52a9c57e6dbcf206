"""Plain FP64 CPU oracle for the method of alternating projections
(Gerchberg-Saxton) that computes a phase-only SLM mask.

TEST INFRASTRUCTURE ONLY.  This module is the checker, not the product: only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the device library and imports nothing
from it.  Everything here is slow on purpose: float64/complex128 NumPy, no
blocking, no fusion, steps in the paper's order and notation.

Notation (Sec. II of the paper)
-------------------------------
* ``u`` in C^N is the field on the SLM, N = n_x * n_y, stored row-major as a
  ``[n_y][n_x]`` array (rows = y, columns = x).
* ``p`` >= 0 is the illumination amplitude on the SLM (Eq. 1); p = 1 (a
  phase-only SLM) unless given.
* ``m`` >= 0 is the target amplitude of the optical stimulation pattern
  (Eq. 2), in natural DFT order (zero frequency at ``[0][0]``).
* ``F`` is the 2-D discrete Fourier transform, taken unitary here (forward
  kernel exp(-2 pi i (k_y y / n_y + k_x x / n_x)) / sqrt(N)) so that the
  projections of Eq. 4 are nearest-point maps in the Euclidean norm
  (Sec. II: a projection maps a point to its nearest points).

Readings where the paper is silent (each also listed in the design notes):
* Scale of m.  The iterates do not depend on any positive scale of m (P_M
  keeps only the phase of Fu, P_S divides every modulus out), so the oracle
  works with the energy-matched target  m~ = m * ||p|| / ||m||  (Parseval:
  ||F u|| = ||u|| = ||p|| for u in S).  Error norms are reported relative to
  ||p||.
* Zero tie-break of Eq. 4a and Eq. 5.  The set-valued branch (u = 0) takes
  theta = 0, and "zero" means |z|^2 below the smallest normal float64.
* Gap, Eq. 7.  For u in S the printed formula ||P_S u - P_M u|| equals
  ||u - P_M u|| = d(u, M), reported here as the Fourier-plane error E_F.
  The sentence after Eq. 7 (accumulation points in M and their projections
  onto S) is d(P_M u, S), reported as the gap G.  Both are relative to ||p||.
* Iteration count.  ``n_iter`` applications of P_S P_M (Eq. 6) starting from
  u^0 = p exp(i phi0); the returned mask is u^n.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "DBL_MIN",
    "F",
    "F_inv",
    "matched_target",
    "P_S",
    "M_hat",
    "P_M",
    "fourier_error",
    "gap",
    "mask_errors",
    "gs_solve",
    "physical_error",
    "intensity_loss",
    "intensity_loss_grad",
    "raar_solve",
    "paper_initial_phase",
]

DBL_MIN = np.finfo(np.float64).tiny


def F(u: np.ndarray) -> np.ndarray:
    """Unitary 2-D DFT over the last two axes (rows = y, columns = x).

    Models Fraunhofer propagation from the SLM to the specimen (Sec. II,
    the sentence before Eq. 2)."""
    return np.fft.fft2(np.asarray(u, dtype=np.complex128), axes=(-2, -1), norm="ortho")


def F_inv(v: np.ndarray) -> np.ndarray:
    """Inverse of the unitary 2-D DFT (also its adjoint)."""
    return np.fft.ifft2(np.asarray(v, dtype=np.complex128), axes=(-2, -1), norm="ortho")


def matched_target(m: np.ndarray, p: np.ndarray | None = None) -> np.ndarray:
    """Energy-matched target m~ = m ||p|| / ||m|| (float64)."""
    m = np.asarray(m, dtype=np.float64)
    n = m.shape[-2] * m.shape[-1]
    p_norm = np.sqrt(n) if p is None else np.linalg.norm(np.asarray(p, dtype=np.float64))
    return m * (p_norm / np.linalg.norm(m))


def _phase_of(z: np.ndarray) -> np.ndarray:
    """z / |z| where |z|^2 >= DBL_MIN, else exp(i 0) = 1 (tie-break theta = 0)."""
    a2 = z.real * z.real + z.imag * z.imag
    nz = a2 >= DBL_MIN
    out = np.ones_like(z)
    out[nz] = z[nz] / np.sqrt(a2[nz])
    return out


def P_S(u: np.ndarray, p: np.ndarray | None = None) -> np.ndarray:
    """Projection onto S, Eq. 4a: every pixel keeps its phase and takes
    modulus p (p = 1 if omitted); a zero pixel takes p exp(i 0)."""
    ph = _phase_of(np.asarray(u, dtype=np.complex128))
    return ph if p is None else np.asarray(p, dtype=np.float64) * ph


def M_hat(Fu: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Fourier-plane amplitude adaption, Eq. 5: every coefficient keeps its
    phase and takes modulus m; a zero coefficient takes m exp(i 0)."""
    return np.asarray(m, dtype=np.float64) * _phase_of(np.asarray(Fu, dtype=np.complex128))


def P_M(u: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Projection onto M, Eq. 4b: F^{-1} of M_hat(F u)."""
    return F_inv(M_hat(F(u), m))


def fourier_error(u: np.ndarray, m: np.ndarray) -> float:
    """E_F = || |F u| - m~ || / ||p||  (p = 1, so ||p|| = sqrt N).

    For u in S this is d(u, M) / ||p|| (Parseval), the literal Eq. 7."""
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[-2] * u.shape[-1]
    mt = matched_target(m)
    return float(np.linalg.norm(np.abs(F(u)) - mt) / np.sqrt(n))


def gap(v: np.ndarray) -> float:
    """G = d(v, S) / ||p|| = || |v| - 1 || / sqrt N for a point v of M
    (the prose reading of Eq. 7, p = 1)."""
    v = np.asarray(v, dtype=np.complex128)
    n = v.shape[-2] * v.shape[-1]
    return float(np.linalg.norm(np.abs(v) - 1.0) / np.sqrt(n))


def mask_errors(m: np.ndarray, phi: np.ndarray) -> tuple[float, float]:
    """(E_F, G) of the phase-only mask u = exp(i phi) against target m."""
    u = np.exp(1j * np.asarray(phi, dtype=np.float64))
    mt = matched_target(m)
    return fourier_error(u, m), gap(P_M(u, mt))


def gs_solve(m: np.ndarray, phi0: np.ndarray | None, n_iter: int, p: np.ndarray | None = None,
             u0: np.ndarray | None = None) -> dict:
    """Method of alternating projections, Eq. 6 (p = 1 unless given).

    u^0 = p exp(i phi0) (a point of S, Eq. 1), or the complex field ``u0``
    as given when ``phi0`` is None (Eq. 6 starts from any point; the state
    of the method is the field); for nu = 0 .. n_iter-1:
        U      = F u^nu                          (Eq. 2 / Eq. 4b)
        E_F^nu = || |U| - m~ || / ||p||           (error before projecting)
        V      = M_hat(U)                         (Eq. 5)
        w      = F^{-1} V  = P_M u^nu             (Eq. 4b)
        G^nu   = || |w| - p || / ||p||            (Eq. 7, prose reading)
        u^{nu+1} = P_S w                          (Eq. 4a)
    and finally E_F^n of the returned mask.

    Returns a dict with the field ``u`` (= u^n), the phase ``phi`` =
    angle(u^n) in (-pi, pi], and ``history`` = [E_F^0, G^0, ..., E_F^{n-1},
    G^{n-1}, E_F^n] (length 2 n_iter + 1).
    """
    if n_iter < 0:
        raise ValueError("n_iter must be >= 0")
    m = np.asarray(m, dtype=np.float64)
    if (phi0 is None) == (u0 is None):
        raise ValueError("give exactly one of phi0 and u0")
    start = np.asarray(phi0 if u0 is None else u0)
    if m.shape != start.shape or m.ndim != 2:
        raise ValueError("target and initial point must be 2-D arrays of one shape")
    pp = np.ones_like(m) if p is None else np.asarray(p, dtype=np.float64)
    p_norm = np.linalg.norm(pp)
    mt = matched_target(m, pp)
    if u0 is None:
        u = pp * np.exp(1j * np.asarray(phi0, dtype=np.float64))
    else:
        u = np.asarray(u0, dtype=np.complex128)
    hist = []
    for _ in range(n_iter):
        U = F(u)
        hist.append(float(np.linalg.norm(np.abs(U) - mt) / p_norm))
        w = F_inv(M_hat(U, mt))
        hist.append(float(np.linalg.norm(np.abs(w) - pp) / p_norm))
        u = P_S(w, pp)
    hist.append(float(np.linalg.norm(np.abs(F(u)) - mt) / p_norm))
    return {"u": u, "phi": np.angle(u), "history": np.array(hist)}


def raar_solve(m: np.ndarray, phi0: np.ndarray, n_iter: int, beta: float,
               p: np.ndarray | None = None) -> dict:
    """Relaxed averaged alternating reflections, the alternative the paper
    names for problems where alternating projections stagnate (Sec. IV.B).

    With the reflectors R_S = 2 P_S - I and R_M = 2 P_M - I:
        x^{nu+1} = beta/2 (R_S R_M + I) x^nu + (1 - beta) P_M x^nu
                 = beta P_S(2 P_M x^nu - x^nu) + beta x^nu + (1 - 2 beta) P_M x^nu,
    started from x^0 = p exp(i phi0).  The mask is the shadow P_S x^n.
    History: [E_F(x^0), E_F(x^1), ..., E_F(x^{n-1}), E_F(P_S x^n)] with
    E_F(x) = || |F x| - m~ || / ||p|| (length n_iter + 1).  beta = 1 gives
    the Douglas-Rachford average of reflections.
    """
    if n_iter < 0:
        raise ValueError("n_iter must be >= 0")
    m = np.asarray(m, dtype=np.float64)
    pp = np.ones_like(m) if p is None else np.asarray(p, dtype=np.float64)
    p_norm = np.linalg.norm(pp)
    mt = matched_target(m, pp)
    x = pp * np.exp(1j * np.asarray(phi0, dtype=np.float64))
    hist = []
    for _ in range(n_iter):
        U = F(x)
        hist.append(float(np.linalg.norm(np.abs(U) - mt) / p_norm))
        pm = F_inv(M_hat(U, mt))
        x = beta * P_S(2.0 * pm - x, pp) + beta * x + (1.0 - 2.0 * beta) * pm
    u = P_S(x, pp)
    hist.append(float(np.linalg.norm(np.abs(F(u)) - mt) / p_norm))
    return {"x": x, "u": u, "phi": np.angle(u), "history": np.array(hist)}


def paper_initial_phase(m: np.ndarray, t_d: float = 3e-4) -> np.ndarray:
    """The paper's initial mask (Sec. IV, first paragraph), read as: binarise
    the target pattern (lit where the normalised target intensity m~^2 /
    max m~^2 exceeds t_d, the dark tolerance of Eq. 8b), take the inverse
    transform of that 1-bit pattern back to the SLM plane, and keep its phase
    (the projection onto S of the back-propagated pattern).  Phase 0 where
    the back-propagated field is exactly zero (tie-break of Eq. 4a)."""
    it = np.asarray(m, dtype=np.float64) ** 2
    b = (it / it.max() > t_d).astype(np.float64)
    return np.angle(P_S(F_inv(b)))


def physical_error(m: np.ndarray, u: np.ndarray, t_l: float = 0.1,
                   t_d: float = 3e-4) -> tuple[float, float]:
    """Physical error of Eq. 8a/8b: (E_lit, E_dark).

    Reading (the paper calls both u and m intensities here, leaves their
    scale and the lit/dark split unstated): target intensity I_t = m~^2 and
    reconstructed intensity I_r = |F u|^2, each divided by its own maximum;
    a pixel is lit when I_t > t_d, dark otherwise; the sums are as printed.
    Tolerances t_l = 0.1 (relative, lit) and t_d = 3e-4 (absolute, dark)
    are the paper's (Sec. II, last paragraph).
    """
    it = matched_target(m) ** 2
    ir = np.abs(F(u)) ** 2
    it = it / it.max()
    ir = ir / ir.max()
    lit = it > t_d
    rel = np.abs(it[lit] - ir[lit]) / it[lit]
    e_lit = float(np.sum((t_d * rel / t_l - t_d) * (rel - t_l > 0)))
    d = ir[~lit]
    e_dark = float(np.sum((d - t_d) * (d - t_d > 0)))
    return e_lit, e_dark


def intensity_loss(phi: np.ndarray, target_intensity: np.ndarray) -> float:
    """L(phi) = sum_k ( |(F exp(i phi))_k|^2 - I_k )^2 with unitary F.

    Not in the paper: the gradient-based alternative that sits beside the
    projection method.  The caller chooses the scale of I (sum I = N matches
    the energy of a phase-only field)."""
    U = F(np.exp(1j * np.asarray(phi, dtype=np.float64)))
    r = np.abs(U) ** 2 - np.asarray(target_intensity, dtype=np.float64)
    return float(np.sum(r * r))


def intensity_loss_grad(phi: np.ndarray, target_intensity: np.ndarray) -> np.ndarray:
    """dL/dphi_j = 4 Im( exp(-i phi_j) (F^H (r . U))_j ),  r = |U|^2 - I.

    Chain rule: d|U_k|^2/dphi_j = 2 Re( conj(U_k) F_kj i u_j ), summed with
    the weight 2 r_k over k; F^H = F^{-1} for the unitary transform."""
    u = np.exp(1j * np.asarray(phi, dtype=np.float64))
    U = F(u)
    r = np.abs(U) ** 2 - np.asarray(target_intensity, dtype=np.float64)
    g = F_inv(r * U)
    return 4.0 * np.imag(np.conj(u) * g)


def adam_intensity(phi0: np.ndarray, target_intensity: np.ndarray, n_steps: int, lr: float,
                   beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> dict:
    """n_steps of Adam on intensity_loss from phi0, in FP64.

    Not in the paper: gradient-based phase optimisation beside the
    projection method.  Adam as published by Kingma and Ba (2015,
    Algorithm 1): from m = v = 0, at step t = 1, 2, ...
        g = grad L(theta),  m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
        m_hat = m / (1 - beta1^t),  v_hat = v / (1 - beta2^t),
        theta = theta - lr m_hat / (sqrt(v_hat) + eps).
    Returns the final phase and the losses [L(phi^0), ..., L(phi^n)]."""
    phi = np.asarray(phi0, dtype=np.float64).copy()
    it = np.asarray(target_intensity, dtype=np.float64)
    m = np.zeros_like(phi)
    v = np.zeros_like(phi)
    losses = [intensity_loss(phi, it)]
    for t in range(1, n_steps + 1):
        g = intensity_loss_grad(phi, it)
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        m_hat = m / (1.0 - beta1 ** t)
        v_hat = v / (1.0 - beta2 ** t)
        phi = phi - lr * m_hat / (np.sqrt(v_hat) + eps)
        losses.append(intensity_loss(phi, it))
    return {"phi": phi, "losses": np.array(losses)}
