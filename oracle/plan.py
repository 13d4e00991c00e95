"""Orientation plan P(zone, phi3, q_s) in FP64.

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Methods > Calculation of Kinematical Diffraction Patterns (Eq.
excitation error) and Methods > Generation of an Orientation Plan (the P0
expression, the normalisation A and P = A P0, default gamma = omega = 1).

Readings taken where the paper is silent or ambiguous:
  * beam along +z with |k| = 1/lambda, alpha = 0 (foil normal to the beam);
  * phi_a = 2 pi a / N_phi, a = 0..N_phi-1, no half-bin offset;
  * radial axis: "shells" = the unique |g| (the paper's q_s), or "uniform" =
    bin centres (s + 1/2) k_max / N_r.  In uniform mode each g reaches the bins
    near |g| through rho = |g| - q_s inside the square root, and its amplitude
    factor is |g|^gamma (equal to q_s^gamma in shells mode);
  * kernel: the paper's cone max(1 - d/delta, 0); optional Gaussian
    exp(-d^2 / 2 sigma^2) cut at d < 3 sigma (same family for plan and image);
  * a zone whose P0 is identically zero gets A = 0 (never selected).
"""
import math
import numpy as np

from . import crystal as _crystal
from . import zones as _zones

CONE = 0
GAUSS = 1
UNIFORM = 0
SHELLS = 1


def excitation_error(gp, k0):
    """Eq. excitation error with alpha = 0 and k = (0, 0, k0):
    s_g = -g.(2k + g) / (2 |k + g|)."""
    gp = np.asarray(gp, dtype=np.float64)
    num = -(2.0 * k0 * gp[..., 2] + np.sum(gp * gp, axis=-1))
    den = 2.0 * np.sqrt(gp[..., 0] ** 2 + gp[..., 1] ** 2 + (k0 + gp[..., 2]) ** 2)
    return num / den


def wrap_angle(x):
    """mod(x + pi, 2 pi) - pi with a floor-mod, as in the plan expression."""
    return np.mod(np.asarray(x, dtype=np.float64) + math.pi, 2.0 * math.pi) - math.pi


def kernel(d, delta, kind=CONE, sigma=None):
    """Correlation kernel of distance d: cone max(1 - d/delta, 0) (paper) or the
    optional cut Gaussian."""
    d = np.asarray(d, dtype=np.float64)
    if kind == CONE:
        return np.maximum(1.0 - d / delta, 0.0)
    if sigma is None:
        sigma = 0.5 * delta
    return np.where(d < 3.0 * sigma, np.exp(-d * d / (2.0 * sigma * sigma)), 0.0)


def kernel_radius(delta, kind=CONE, sigma=None):
    if kind == CONE:
        return delta
    return 3.0 * (0.5 * delta if sigma is None else sigma)


def radial_axis(mode, k_max, n_radial=None, q_refl=None, tol=1e-9):
    """q_s: uniform bin centres, or the unique reflection radii (shells)."""
    if mode == UNIFORM:
        return (np.arange(n_radial, dtype=np.float64) + 0.5) * (k_max / n_radial)
    qs = []
    for q in np.sort(np.asarray(q_refl, dtype=np.float64)):
        if not qs or q - qs[-1] > tol:
            qs.append(q)
    return np.array(qs)


class Params:
    """Plan parameters (defaults: delta = 0.08 1/A, gamma = omega = 1, 300 kV)."""

    def __init__(self, k_max, n_radial=32, n_angular=90, delta=0.08, gamma=1.0, omega=1.0,
                 accel_kV=300.0, zone_step_deg=5.0, radial=UNIFORM, kind=CONE, sigma=None):
        self.k_max = float(k_max)
        self.n_radial = int(n_radial)
        self.n_angular = int(n_angular)
        self.delta = float(delta)
        self.gamma = float(gamma)
        self.omega = float(omega)
        self.accel_kV = float(accel_kV)
        self.zone_step_deg = float(zone_step_deg)
        self.radial = int(radial)
        self.kind = int(kind)
        self.sigma = None if sigma is None else float(sigma)

    @property
    def k0(self):
        return 1.0 / _crystal.electron_wavelength(self.accel_kV)


class Phase:
    """One crystal phase: lattice rows, fractional basis, zone triangles or an
    explicit zone list."""

    def __init__(self, lattice, frac_xyz, triangles=None, zones=None, species=None, f_q=None, f_tab=None):
        self.lattice = np.asarray(lattice, dtype=np.float64)
        self.frac = np.asarray(frac_xyz, dtype=np.float64).reshape(-1, 3)
        self.triangles = triangles
        self.zones = None if zones is None else np.asarray(zones, dtype=np.float64)
        self.species = species
        self.f_q = f_q
        self.f_tab = f_tab


def zone_plan(refl, w, q_s, prm):
    """Unnormalised P0[a, s] for one zone axis w (Generation of an Orientation Plan).

    P0 = sum_g |g|^gamma |F_g|^omega K(sqrt(s_g^2 + rho^2 + (wrap(phi_a - gamma_g) q_s)^2)),
    with g' = M12^T g, s_g from g' (Eq. excitation error) and gamma_g = atan2(g'_y, g'_x).
    """
    M = _zones.zone_rotation(w)
    gp = refl["g"] @ M                       # rows of g' = M12^T g
    sg = excitation_error(gp, prm.k0)
    gam = np.arctan2(gp[:, 1], gp[:, 0])
    amp = refl["q"] ** prm.gamma * np.abs(refl["F"]) ** prm.omega
    R = kernel_radius(prm.delta, prm.kind, prm.sigma)
    phi = 2.0 * math.pi * np.arange(prm.n_angular) / prm.n_angular
    P0 = np.zeros((prm.n_angular, len(q_s)))
    for i in np.nonzero(np.abs(sg) < R)[0]:
        if prm.radial == SHELLS:
            cols = np.nonzero(np.abs(q_s - refl["q"][i]) <= 1e-9)[0]
            rho = np.zeros(len(cols))
        else:
            cols = np.nonzero(np.abs(q_s - refl["q"][i]) < R)[0]
            rho = refl["q"][i] - q_s[cols]
        if len(cols) == 0:
            continue
        dphi = wrap_angle(phi[:, None] - gam[i])
        d = np.sqrt(sg[i] ** 2 + rho[None, :] ** 2 + (dphi * q_s[None, cols]) ** 2)
        P0[:, cols] += amp[i] * kernel(d, prm.delta, prm.kind, prm.sigma)
    return P0


def build(phases, prm):
    """Full normalised plan over all phases (zones concatenated phase by phase).

    Returns dict: P float[Z, N_phi, N_r] (A P0), A float[Z], q_s, zones [Z,3],
    zone_phase int[Z], M12 [Z,3,3], refl (list per phase)."""
    reflist, zl, zp = [], [], []
    for ip, ph in enumerate(phases):
        refl = _crystal.reflections(ph.lattice, ph.frac, prm.k_max, ph.species, ph.f_q, ph.f_tab)
        reflist.append(refl)
        z = ph.zones if ph.zones is not None else _zones.zone_grid(ph.triangles, prm.zone_step_deg)
        zl.append(np.array([v / np.linalg.norm(v) for v in z]))
        zp.append(np.full(len(z), ip, dtype=np.int64))
    zones_all = np.concatenate(zl)
    zone_phase = np.concatenate(zp)
    if prm.radial == SHELLS:
        q_s = radial_axis(SHELLS, prm.k_max, q_refl=np.concatenate([r["q"] for r in reflist]))
    else:
        q_s = radial_axis(UNIFORM, prm.k_max, prm.n_radial)
    Z = len(zones_all)
    P = np.zeros((Z, prm.n_angular, len(q_s)))
    A = np.zeros(Z)
    for iz in range(Z):
        P0 = zone_plan(reflist[zone_phase[iz]], zones_all[iz], q_s, prm)
        nrm = math.sqrt(float(np.sum(P0 * P0)))
        A[iz] = 0.0 if nrm == 0.0 else 1.0 / nrm
        P[iz] = A[iz] * P0
    M12 = np.array([_zones.zone_rotation(w) for w in zones_all])
    return {"P": P, "A": A, "q_s": q_s, "zones": zones_all, "zone_phase": zone_phase,
            "M12": M12, "refl": reflist, "params": prm}
