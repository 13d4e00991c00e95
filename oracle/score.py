"""Continuous correlation score, its gradient and gradient-ascent refinement.

TEST INFRASTRUCTURE ONLY (see package docstring).

Not in the paper: the continuous analogue of its normalised polar correlation,
used for sub-grid orientation refinement.  Ingredients, all from the paper:
  * observed weights w_m = q_m^gamma I_m^(omega/2)                 (Eq. image_polar)
  * predicted weights v_g = |g|^gamma (|F_g|^2 D(s_g))^(omega/2), with the
    kinematical spot intensity |F_g|^2 D(s_g), D = exp(-s^2 / 2 sigma_e^2) the
    Gaussian shape factor (Eq. shape_gaussian, Eq. excitation error) and
    sigma_e the excitation tolerance (0.02 1/A, the paper's example value);
  * a Gaussian kernel of width sigma_c = delta / 2 on the in-plane distance
    between a peak and a projected reflection;
  * normalisation of the template, as the plan's A(phi1, theta2) does:

  S(theta) = sum_m sum_g w_m v_g K_mg / sqrt(sum_g v_g^2),
  K_mg = exp(-[(qx_m - x_g)^2 + (qy_m - y_g)^2] / (2 sigma_c^2)),
  (x_g, y_g, z_g) = Exp(theta)^T m0^T g,  m = m0 Exp(theta)  (sample -> crystal).

Reading: with the normalisation, observed and predicted weights are parallel
at the true orientation of a noise-free pattern, so S peaks there; tilts are
seen through the excitation errors (an unnormalised score would instead reward
tilting extra reflections onto the Ewald sphere).
Gradient in theta: d(Exp(theta)^T u)/dtheta = [r]x J_r(theta), r = Exp(theta)^T u
(SO(3) right Jacobian).

Refinement reading: every step re-centres (theta = 0) and moves by l along
grad/|grad|; l starts at 0.25 deg, doubles on success up to 0.5 deg, halves on
failure; stop when l < 1e-4 deg or after max_iter trials; among several
candidates the one with the largest S wins (ties -> the earlier one).
"""
import math
import numpy as np

from .plan import excitation_error

SIGMA_EXC = 0.02


def hat(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def expm_so3(th):
    """Rodrigues: Exp(theta) = I + sin t/t [th]x + (1 - cos t)/t^2 [th]x^2."""
    th = np.asarray(th, dtype=np.float64)
    t = float(np.linalg.norm(th))
    K = hat(th)
    if t < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + math.sin(t) / t * K + (1.0 - math.cos(t)) / (t * t) * K @ K


def right_jacobian(th):
    th = np.asarray(th, dtype=np.float64)
    t = float(np.linalg.norm(th))
    K = hat(th)
    if t < 1e-8:
        return np.eye(3) - 0.5 * K + K @ K / 6.0
    return np.eye(3) - (1.0 - math.cos(t)) / (t * t) * K + (t - math.sin(t)) / (t ** 3) * K @ K


def _terms(refl, qx, qy, I, m0, theta, prm, sigma_e):
    qx = np.asarray(qx, np.float64)
    qy = np.asarray(qy, np.float64)
    I = np.asarray(I, np.float64)
    q = np.sqrt(qx * qx + qy * qy)
    w = q ** prm.gamma * I ** (0.5 * prm.omega)
    R = np.asarray(m0, np.float64) @ expm_so3(theta)
    r = refl["g"] @ R                           # rows r_g = R^T g
    s = excitation_error(r, prm.k0)
    F2 = np.abs(refl["F"]) ** 2
    v = refl["q"] ** prm.gamma * (F2 * np.exp(-s * s / (2.0 * sigma_e * sigma_e))) ** (0.5 * prm.omega)
    dx = qx[:, None] - r[None, :, 0]
    dy = qy[:, None] - r[None, :, 1]
    sig2 = (0.5 * prm.delta) ** 2
    K = np.exp(-(dx * dx + dy * dy) / (2.0 * sig2))
    return q, w, v, r, s, dx, dy, sig2, K


def score(refl, qx, qy, I, m0, theta, prm, sigma_e=SIGMA_EXC):
    """S(theta) for one pattern (0 when no reflection carries weight)."""
    _, w, v, _, _, _, _, _, K = _terms(refl, qx, qy, I, m0, theta, prm, sigma_e)
    nv = math.sqrt(float(np.sum(v * v)))
    return 0.0 if nv == 0.0 else float(w @ K @ v) / nv


def score_grad(refl, qx, qy, I, m0, theta, prm, sigma_e=SIGMA_EXC):
    """(S, dS/dtheta [3], dS/dqx [M], dS/dqy [M]) for one pattern."""
    q, w, v, r, s, dx, dy, sig2, K = _terms(refl, qx, qy, I, m0, theta, prm, sigma_e)
    nv = math.sqrt(float(np.sum(v * v)))
    M = len(w)
    if nv == 0.0:
        return 0.0, np.zeros(3), np.zeros(M), np.zeros(M)
    a = w @ K                                   # [G]: sum_m w_m K_mg
    Nn = float(a @ v)
    S = Nn / nv
    k0 = prm.k0
    x, y, z = r[:, 0], r[:, 1], r[:, 2]
    D = np.sqrt(x * x + y * y + (k0 + z) ** 2)
    dsdr = np.stack([-x / D - s * x / D ** 2, -y / D - s * y / D ** 2,
                     -(k0 + z) / D - s * (k0 + z) / D ** 2], axis=1)
    dvdr = (v * 0.5 * prm.omega * (-s / (sigma_e * sigma_e)))[:, None] * dsdr
    WK = w[:, None] * K * v[None, :]
    dNdr = a[:, None] * dvdr
    dNdr[:, 0] += np.sum(WK * dx, axis=0) / sig2
    dNdr[:, 1] += np.sum(WK * dy, axis=0) / sig2
    dSdr = dNdr / nv - (Nn / nv ** 3) * v[:, None] * dvdr
    Jr = right_jacobian(theta)
    gth = np.zeros(3)
    for gi in range(len(r)):
        gth += dSdr[gi] @ hat(r[gi]) @ Jr
    with np.errstate(divide="ignore", invalid="ignore"):
        inv_q2 = np.where(q > 0, 1.0 / (q * q), 0.0)
    Kv = K @ v                                  # [M]
    dwx = prm.gamma * w * np.asarray(qx, np.float64) * inv_q2
    dwy = prm.gamma * w * np.asarray(qy, np.float64) * inv_q2
    dqx = (dwx * Kv - np.sum(WK * dx, axis=1) / sig2) / nv
    dqy = (dwy * Kv - np.sum(WK * dy, axis=1) / sig2) / nv
    return S, gth, dqx, dqy


def refine_one(refl, qx, qy, I, m_init, prm, max_iter=64, step0_deg=0.25, step_max_deg=0.5,
               step_min_deg=1e-4, sigma_e=SIGMA_EXC):
    """Gradient ascent from one starting orientation; returns (m, S, trials)."""
    m = np.asarray(m_init, np.float64).copy()
    S = score(refl, qx, qy, I, m, np.zeros(3), prm, sigma_e)
    l = math.radians(step0_deg)
    lmax, lmin = math.radians(step_max_deg), math.radians(step_min_deg)
    _, gth, _, _ = score_grad(refl, qx, qy, I, m, np.zeros(3), prm, sigma_e)
    it = 0
    while it < max_iter and l >= lmin:
        gn = float(np.linalg.norm(gth))
        if gn == 0.0:
            break
        th = l * gth / gn
        St = score(refl, qx, qy, I, m, th, prm, sigma_e)
        it += 1
        if St > S:
            m = m @ expm_so3(th)
            S = St
            l = min(2.0 * l, lmax)
            _, gth, _, _ = score_grad(refl, qx, qy, I, m, np.zeros(3), prm, sigma_e)
        else:
            l *= 0.5
    return m, S, it


def refine(refl, qx, qy, I, candidates, prm, max_iter=64, sigma_e=SIGMA_EXC):
    """Refine every candidate orientation; keep the largest S (ties -> earlier)."""
    best = None
    for mc in candidates:
        m, S, _ = refine_one(refl, qx, qy, I, mc, prm, max_iter=max_iter, sigma_e=sigma_e)
        if best is None or S > best[1]:
            best = (m, S)
    return best
