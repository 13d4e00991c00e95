"""Forward kinematical diffraction pattern for a given orientation (FP64).

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Methods > Calculation of Kinematical Diffraction Patterns.  For each
reciprocal lattice point, rotate into the sample frame, compute its excitation
error (Eq. excitation error), attenuate |F|^2 by the Gaussian shape factor
D = exp(-s^2 / 2 sigma^2) (Eq. shape_gaussian) and project onto the image plane.
Used only by the oracle's own pins (self-recovery, symmetry).
"""
import numpy as np

from .plan import excitation_error


def pattern(refl, m, k0, sigma=0.02, rel_cut=0.01, k_max=None):
    """Peaks (qx, qy, I) for orientation m (d = m d0, sample -> crystal).

    A reflection g (crystal frame) sits at g_s = m^T g in the sample frame.
    Kept when |F|^2 D(s_g) > rel_cut * max|F|^2 (and |g| < k_max if given)."""
    gs = refl["g"] @ np.asarray(m, dtype=np.float64)     # rows m^T g
    sg = excitation_error(gs, k0)
    I0 = np.abs(refl["F"]) ** 2
    I = I0 * np.exp(-sg * sg / (2.0 * sigma * sigma))
    keep = I > rel_cut * I0.max()
    if k_max is not None:
        keep &= refl["q"] < k_max
    return gs[keep, 0], gs[keep, 1], I[keep]
