"""Sparse polar diffraction image X(phi3, q_s) in FP64.

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Methods > Correlation Pattern Matching, Eq. image_polar:
X(phi_a, q_s) = sum over peaks with |q_m - q_s| < delta of
q_m^gamma I_m^(omega/2) max{1 - sqrt((q_m - q_s)^2 + wrap(phi_a - gamma_m)^2 q_s^2)/delta, 0},
with q_m = sqrt(qx^2 + qy^2) and gamma_m = arctan2(qy, qx).
For the cone kernel the |q_m - q_s| < delta restriction is implied by the
kernel's support; the optional Gaussian kernel uses its own 3-sigma cut.
"""
import math
import numpy as np

from .plan import kernel, wrap_angle


def peak_polar(qx, qy, I, gamma, omega):
    """Polar coordinates and weights w_m = q_m^gamma I_m^(omega/2) of a peak list."""
    qx = np.asarray(qx, dtype=np.float64)
    qy = np.asarray(qy, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    q = np.sqrt(qx * qx + qy * qy)
    g = np.arctan2(qy, qx)
    w = q ** gamma * I ** (0.5 * omega)
    return q, g, w


def polar_image(qx, qy, I, q_s, n_angular, prm):
    """X[a, s] for one pattern (Eq. image_polar), evaluated cell by cell."""
    q, g, w = peak_polar(qx, qy, I, prm.gamma, prm.omega)
    phi = 2.0 * math.pi * np.arange(n_angular) / n_angular
    X = np.zeros((n_angular, len(q_s)))
    for m in range(len(q)):
        dq = q[m] - np.asarray(q_s)[None, :]
        dphi = wrap_angle(phi[:, None] - g[m])
        d = np.sqrt(dq * dq + (dphi * np.asarray(q_s)[None, :]) ** 2)
        X += w[m] * kernel(d, prm.delta, prm.kind, prm.sigma)
    return X
