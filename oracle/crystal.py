"""Crystal: reciprocal lattice, reflection list and structure factors (FP64).

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Methods > Structure Factor Calculations (reciprocal basis without 2*pi,
lattice points g_hkl = h a* + k b* + l c* inside |g| < q_max, structure factor
F_hkl = sum_n f_n(|g|) exp(-2 pi i (h,k,l).p_n)).
"""
import math
import numpy as np


def reciprocal_basis(lattice):
    """Rows a*, b*, c* for a lattice given as rows a, b, c (Cartesian, Angstrom).

    Structure Factor Calculations: a* = (b x c)/V with V = a.(b x c), cyclic;
    no 2*pi factor, so reciprocal coordinates are spatial frequencies.
    """
    L = np.asarray(lattice, dtype=np.float64)
    a, b, c = L[0], L[1], L[2]
    V = float(np.dot(a, np.cross(b, c)))
    if V == 0.0:
        raise ValueError("degenerate lattice")
    return np.array([np.cross(b, c) / V, np.cross(c, a) / V, np.cross(a, b) / V])


def electron_wavelength(accel_kV):
    """Relativistic electron wavelength in Angstrom for an accelerating voltage.

    Kinematical Diffraction: |k| = 1/lambda with lambda relativistically corrected.
    CODATA constants; lambda = h / sqrt(2 m0 e V (1 + e V / (2 m0 c^2))).
    """
    h = 6.62607015e-34
    m0 = 9.1093837015e-31
    e = 1.602176634e-19
    c = 299792458.0
    V = accel_kV * 1e3
    return h / math.sqrt(2.0 * m0 * e * V * (1.0 + e * V / (2.0 * m0 * c * c))) * 1e10


def scattering_factor(species, q, f_q=None, f_tab=None):
    """Atomic scattering factor f_n(|g|).

    The paper uses the Lobato & Van Dyck parameterisation, whose coefficient
    table is not available here.  Reading: f == 1 unless a caller gives a table
    of knots f_q (1/Angstrom) and values f_tab[species, knot]; then linear
    interpolation, clamped at the ends.
    """
    if f_q is None or f_tab is None or len(f_q) == 0:
        return np.ones_like(np.asarray(q, dtype=np.float64))
    return np.interp(q, np.asarray(f_q, np.float64), np.asarray(f_tab, np.float64)[species])


def reflections(lattice, frac_xyz, k_max, species=None, f_q=None, f_tab=None, rel_cut=1e-12):
    """All reciprocal lattice points 0 < |g| < k_max with their structure factors.

    Structure Factor Calculations.  The (h,k,l) range: since g.a = h exactly,
    |h| <= |g||a| < k_max |a|, so |h| <= ceil(k_max |a|) (likewise k, l) is an
    exact bound (the paper's "shortest vector" range, read as this bound).
    Reflections with |F|^2 <= rel_cut * max|F|^2 are dropped: they are the
    forbidden reflections, carrying only round-off.

    Returns dict: hkl int[G,3], g float[G,3] (crystal Cartesian), q float[G] (|g|),
    F complex[G].
    """
    L = np.asarray(lattice, dtype=np.float64)
    B = reciprocal_basis(L)
    frac = np.asarray(frac_xyz, dtype=np.float64).reshape(-1, 3)
    if species is None:
        species = np.zeros(len(frac), dtype=np.int64)
    hmax = [int(math.ceil(k_max * np.linalg.norm(L[i]))) for i in range(3)]
    rh = np.arange(-hmax[0], hmax[0] + 1)
    rk = np.arange(-hmax[1], hmax[1] + 1)
    rl = np.arange(-hmax[2], hmax[2] + 1)
    H, K, Lh = np.meshgrid(rh, rk, rl, indexing="ij")
    hkl = np.stack([H.ravel(), K.ravel(), Lh.ravel()], axis=1)
    g = hkl.astype(np.float64) @ B
    q = np.sqrt(np.sum(g * g, axis=1))
    keep = (q > 0.0) & (q < k_max)
    hkl, g, q = hkl[keep], g[keep], q[keep]
    F = np.zeros(len(q), dtype=np.complex128)
    for n in range(len(frac)):
        fn = scattering_factor(int(species[n]), q, f_q, f_tab)
        F += fn * np.exp(-2j * np.pi * (hkl.astype(np.float64) @ frac[n]))
    I = np.abs(F) ** 2
    if len(I):
        keep = I > rel_cut * I.max()
        hkl, g, q, F = hkl[keep], g[keep], q[keep], F[keep]
    return {"hkl": hkl, "g": g, "q": q, "F": F}
