"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms,
textbook extinction rules, the paper's worked-example statements (Methods >
Generation of an Orientation Plan, Correlation Pattern Matching), the paper's
own FFT route, invariants, brute force and finite differences.
"""
import math

import numpy as np
import pytest

from oracle import correlate, crystal, directsum, image, kinematics, metrics, plan, score, zones
import synth

A_FCC = 4.08
FCC_BASIS = [[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]
BCC_BASIS = [[0, 0, 0], [0.5, 0.5, 0.5]]
HCP_LAT = np.array([[2.95, 0, 0], [-2.95 / 2, 2.95 * math.sqrt(3) / 2, 0], [0, 0, 4.68]])
HCP_BASIS = [[1 / 3, 2 / 3, 0.25], [2 / 3, 1 / 3, 0.75]]


def fcc_phase():
    return plan.Phase(np.eye(3) * A_FCC, FCC_BASIS, triangles=[zones.cubic_triangle()])


# ---------------------------------------------------------------- crystal ----

@pytest.mark.parametrize("lat", [np.eye(3) * A_FCC, HCP_LAT,
                                 np.array([[3.1, 0.2, 0.1], [0.4, 4.2, -0.3], [0.2, 0.5, 5.3]])])
def test_reciprocal_basis_duality(lat):
    B = crystal.reciprocal_basis(lat)
    assert np.allclose(lat @ B.T, np.eye(3), atol=1e-14)


def test_fcc_shells_and_extinction():
    r = crystal.reflections(np.eye(3) * A_FCC, FCC_BASIS, 1.2)
    h = r["hkl"]
    parity = np.mod(h, 2)
    allowed = np.all(parity == parity[:, :1], axis=1)       # all even or all odd
    assert allowed.all()                                      # forbidden ones dropped
    assert np.allclose(np.abs(r["F"]) ** 2, 16.0, atol=1e-9)  # 4 f, f = 1
    shells = np.unique(np.round(r["q"], 9))
    assert np.allclose(shells[:3], [math.sqrt(3) / A_FCC, 2 / A_FCC, math.sqrt(8) / A_FCC], atol=1e-12)


def test_bcc_extinction():
    r = crystal.reflections(np.eye(3) * 2.87, BCC_BASIS, 2.0)
    assert np.all(np.sum(r["hkl"], axis=1) % 2 == 0)
    assert np.allclose(np.abs(r["F"]) ** 2, 4.0, atol=1e-9)


def test_hcp_structure_factor_classes():
    r = crystal.reflections(HCP_LAT, HCP_BASIS, 2.0)
    h, k, l = r["hkl"].T
    m3 = np.mod(h + 2 * k, 3)
    expect = np.where(m3 == 0, np.where(l % 2 == 0, 4.0, 0.0), np.where(l % 2 == 0, 1.0, 3.0))
    assert np.allclose(np.abs(r["F"]) ** 2, expect, atol=1e-9)
    assert not np.any(expect == 0)


def test_structure_factor_with_scattering_factor_table():
    """Two species on a simple cubic cell (a = 3 A: species 0 at the origin,
    species 1 at the body centre), with a caller's f table of knots 0, 1, 2 1/A:
    F_hkl = f0(|g|) + (-1)^(h+k+l) f1(|g|), each f the straight line between its
    neighbouring knots, written out by hand here."""
    lat = np.eye(3) * 3.0
    r = crystal.reflections(lat, [[0, 0, 0], [0.5, 0.5, 0.5]], 1.5, species=[0, 1],
                            f_q=[0.0, 1.0, 2.0], f_tab=[[2.0, 1.0, 0.5], [1.0, 0.8, 0.2]])

    def f0(q):
        return 2.0 - q if q <= 1.0 else 1.0 - 0.5 * (q - 1.0)

    def f1(q):
        return 1.0 - 0.2 * q if q <= 1.0 else 0.8 - 0.6 * (q - 1.0)

    n_expected = sum(1 for h in range(-5, 6) for k in range(-5, 6) for l in range(-5, 6)
                     if 0 < math.sqrt(h * h + k * k + l * l) / 3.0 < 1.5)
    assert len(r["q"]) == n_expected
    for (h, k, l), q, F in zip(r["hkl"], r["q"], r["F"]):
        assert abs(q - math.sqrt(h * h + k * k + l * l) / 3.0) < 1e-14
        expect = f0(q) + (-1) ** int(h + k + l) * f1(q)
        assert abs(F - expect) < 1e-12, (h, k, l, F, expect)
    # (1,0,0): 2 - 1/3 - (1 - 0.2/3); (2,2,2): |g| = 1.1547, both on the second segment
    i100 = [i for i, t in enumerate(r["hkl"]) if tuple(t) == (1, 0, 0)][0]
    assert abs(r["F"][i100] - (5.0 / 3.0 - (1.0 - 0.2 / 3.0))) < 1e-12


def test_reflection_set_equals_wider_brute_force():
    lat = np.eye(3) * A_FCC
    r = crystal.reflections(lat, [[0, 0, 0]], 1.5)   # primitive cubic: no extinctions
    B = crystal.reciprocal_basis(lat)
    rng = range(-14, 15)
    brute = {(h, k, l) for h in rng for k in rng for l in rng
             if 0 < np.linalg.norm(np.array([h, k, l]) @ B) < 1.5}
    assert set(map(tuple, r["hkl"].tolist())) == brute


def test_wavelength_300kV():
    # relativistic electron wavelength at 300 kV is 0.019687 A (standard value)
    assert abs(crystal.electron_wavelength(300.0) - 0.0196875) < 2e-7


# ------------------------------------------------------------------ zones ----

@pytest.mark.parametrize("step,count", [(5.0, 55), (2.0, 300), (1.0, 1081)])
def test_cubic_zone_counts(step, count):
    Zs = zones.zone_grid([zones.cubic_triangle()], step)
    assert len(Zs) == count
    v0, v1, v2 = zones.cubic_triangle()
    for v in (v0, v1, v2):
        assert np.min(np.linalg.norm(Zs - v, axis=1)) < 1e-12
    # inside the spherical triangle: same side of every great-circle edge
    n01, n12, n20 = np.cross(v0, v1), np.cross(v1, v2), np.cross(v2, v0)
    sgn = np.sign(np.dot(v2, n01))
    assert np.all(sgn * Zs @ n01 >= -1e-12) and np.all(sgn * Zs @ n12 >= -1e-12) and np.all(sgn * Zs @ n20 >= -1e-12)
    assert np.allclose(np.linalg.norm(Zs, axis=1), 1.0, atol=1e-14)


def test_hex_wedge_count():
    assert len(zones.zone_grid(zones.hex_wedge_triangles(), 1.0)) == 2 * 4186 - 91


def test_zone_rotation_maps_beam_to_zone():
    rng = np.random.default_rng(3)
    ws = list(zones.zone_grid([zones.cubic_triangle()], 2.0)) + list(rng.normal(size=(50, 3)))
    ws += [np.array([0, 0, -1.0]), np.array([1.0, 0, 0])]
    for w in ws:
        w = w / np.linalg.norm(w)
        M = zones.zone_rotation(w)
        assert np.allclose(M @ [0, 0, 1.0], w, atol=1e-14)
        assert np.allclose(M.T @ M, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(M) - 1.0) < 1e-14


# ------------------------------------------------------------- kinematics ----

def test_excitation_error_zero_on_ewald_sphere():
    k0 = 1.0 / crystal.electron_wavelength(300.0)
    rng = np.random.default_rng(4)
    for _ in range(20):
        u = np.array([*rng.normal(scale=0.05, size=2), 1.0])
        u /= np.linalg.norm(u)
        g = k0 * u - np.array([0, 0, k0])          # k' = k + g with |k'| = k0
        assert abs(plan.excitation_error(g, k0)) < 1e-12


def test_excitation_error_along_beam_closed_form():
    k0 = 50.0
    for gz in (-0.3, -0.01, 0.02, 0.5):
        s = plan.excitation_error(np.array([0.0, 0.0, gz]), k0)
        assert abs(s - (-gz * (2 * k0 + gz) / (2 * (k0 + gz)))) < 1e-14
        assert abs(s + gz) < 0.01 * abs(gz)


# ------------------------------------------------------------------- plan ----

def test_plan_normalised_per_zone():
    prm = plan.Params(k_max=1.2, n_radial=32, n_angular=90, zone_step_deg=5.0)
    pl = plan.build([fcc_phase()], prm)
    ss = np.sum(pl["P"] ** 2, axis=(1, 2))
    assert np.allclose(ss[pl["A"] > 0], 1.0, atol=1e-12)
    assert np.all(pl["P"] >= 0)


def test_plan_001_first_shell_is_200_with_four_spots():
    """Worked example: at [001] the first row of the plan is the four {200} spots."""
    prm = plan.Params(k_max=1.5, n_angular=360, radial=plan.SHELLS, zone_step_deg=2.0)
    ph = plan.Phase(np.eye(3) * A_FCC, FCC_BASIS, zones=[[0, 0, 1.0]])
    pl = plan.build([ph], prm)
    P = pl["P"][0]
    first = np.nonzero(P.sum(axis=0) > 0)[0][0]
    assert abs(pl["q_s"][first] - 2.0 / A_FCC) < 1e-12
    row = P[:, first]
    peaks = [a for a in range(360) if row[a] > 0 and row[a] >= row[a - 1] and row[a] > row[(a + 1) % 360]]
    assert peaks == [0, 90, 180, 270]


# ------------------------------------------------------------------ image ----

def test_image_single_peak_closed_form():
    prm = plan.Params(k_max=2.0, n_radial=64, n_angular=360, gamma=1.0, omega=1.0)
    q_s = plan.radial_axis(plan.UNIFORM, 2.0, 64)
    s0, a0 = 20, 37
    q, g, I = q_s[s0], 2 * math.pi * a0 / 360, 9.0
    X = image.polar_image([q * math.cos(g)], [q * math.sin(g)], [I], q_s, 360, prm)
    w = q * 3.0
    assert abs(X[a0, s0] - w) < 1e-12 * w
    for j in range(-8, 9):
        expect = w * max(1 - abs(j * 2 * math.pi / 360 * q) / prm.delta, 0)
        assert abs(X[(a0 + j) % 360, s0] - expect) < 1e-12
    far = np.abs(q_s - q) >= prm.delta
    assert np.all(X[:, far] == 0)


def test_image_single_peak_gaussian_closed_form():
    """Gaussian kernel option: a peak at the centre of cell (a0, s0) gives w there,
    w exp(-d^2 / 2 sigma^2) at the cells whose distance d (radial offset, arc
    length of the angular offset at q_s, or both) is below 3 sigma, and 0 beyond."""
    sigma = 0.03
    prm = plan.Params(k_max=2.0, n_radial=64, n_angular=360, kind=plan.GAUSS, sigma=sigma)
    q_s = plan.radial_axis(plan.UNIFORM, 2.0, 64)
    s0, a0 = 40, 101
    q, g, I = q_s[s0], 2 * math.pi * a0 / 360, 4.0
    X = image.polar_image([q * math.cos(g)], [q * math.sin(g)], [I], q_s, 360, prm)
    w = q * 2.0
    assert abs(X[a0, s0] - w) < 1e-12 * w
    dphi = 2 * math.pi / 360
    dq = 2.0 / 64
    for i in range(-4, 5):
        for j in range(-12, 13):
            d = math.sqrt((i * dq) ** 2 + (j * dphi * q_s[s0 + i]) ** 2)
            expect = w * math.exp(-d * d / (2 * sigma * sigma)) if d < 3 * sigma else 0.0
            assert abs(X[(a0 + j) % 360, s0 + i] - expect) < 1e-12 * w, (i, j)
    far = np.abs(q_s - q) >= 3 * sigma
    assert np.all(X[:, far] == 0)
    assert X[(a0 + 180) % 360, s0] == 0


# ------------------------------------------------------------ correlation ----

def _rand_sparse(rng, shape, frac):
    x = rng.random(shape)
    x[rng.random(shape) > frac] = 0
    return x


@pytest.mark.parametrize("Z,N,R", [(3, 8, 3), (5, 16, 4), (4, 90, 32)])
def test_direct_sum_equals_paper_fft_route(Z, N, R):
    rng = np.random.default_rng(Z * N)
    P = _rand_sparse(rng, (Z, N, R), 0.3)
    X = _rand_sparse(rng, (N, R), 0.2)
    C, Cm = correlate.correlate_direct(P, X)
    F, Fm = correlate.correlate_fft(P, X)
    sc = max(1.0, np.abs(F).max())
    assert np.abs(C - F).max() < 1e-12 * sc and np.abs(Cm - Fm).max() < 1e-12 * sc


def _small_plan():
    prm = plan.Params(k_max=1.2, n_radial=32, n_angular=90, zone_step_deg=5.0)
    return plan.build([fcc_phase()], prm)


def test_rotation_rolls_correlogram_and_mirror_swaps_branches():
    pl = _small_plan()
    prm = pl["params"]
    d = synth.make("small")
    o = d["offsets"]
    qx, qy, I = (np.asarray(d[k][o[3]:o[4]], np.float64) for k in ("qx", "qy", "I"))
    X = image.polar_image(qx, qy, I, pl["q_s"], 90, prm)
    C, Cm = correlate.correlate_direct(pl["P"], X)
    j = 7
    ang = j * 2 * math.pi / 90
    rx, ry = qx * math.cos(ang) - qy * math.sin(ang), qx * math.sin(ang) + qy * math.cos(ang)
    Cr, Cmr = correlate.correlate_direct(pl["P"], image.polar_image(rx, ry, I, pl["q_s"], 90, prm))
    sc = np.abs(C).max()
    assert np.abs(Cr - np.roll(C, j, axis=1)).max() < 1e-10 * sc
    assert np.abs(Cmr - np.roll(Cm, -j, axis=1)).max() < 1e-10 * sc
    Cf, Cmf = correlate.correlate_direct(pl["P"], image.polar_image(qx, -qy, I, pl["q_s"], 90, prm))
    assert np.abs(Cf - Cm).max() < 1e-12 * sc and np.abs(Cmf - C).max() < 1e-12 * sc


@pytest.mark.parametrize("w,period", [([0, 0, 1], 90), ([0, 1, 1], 180), ([1, 1, 1], 60)])
def test_zone_symmetry_of_correlation(w, period):
    """Worked example: [001], [011], [111] give 4-, 2- and 6-fold phi3 correlation."""
    prm = plan.Params(k_max=1.5, n_radial=96, n_angular=360)
    ph = plan.Phase(np.eye(3) * A_FCC, FCC_BASIS, zones=[w])
    pl = plan.build([ph], prm)
    refl = pl["refl"][0]
    qx, qy, I = kinematics.pattern(refl, pl["M12"][0], prm.k0, k_max=1.5)
    X = image.polar_image(qx, qy, I, pl["q_s"], 360, prm)
    C, Cm = correlate.correlate_direct(pl["P"], X)
    sc = C.max()
    assert np.abs(np.roll(C[0], period) - C[0]).max() < 1e-12 * sc
    assert np.abs(np.roll(Cm[0], period) - Cm[0]).max() < 1e-12 * sc
    assert C[0, 0] >= sc * (1 - 1e-12)           # the true in-plane bin is a maximum


def test_self_recovery_noise_free_grid_patterns():
    """A noise-free kinematical pattern at a grid orientation returns its zone and bin
    (up to exact ties) at k_max = 2.0, N_phi = 360."""
    prm = plan.Params(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=5.0)
    pl = plan.build([fcc_phase()], prm)
    refl = pl["refl"][0]
    for z in range(len(pl["zones"])):
        n = (37 * z + 11) % 360
        m = correlate.orientation(pl["M12"][z], n, 0.0, 0, 360)
        qx, qy, I = kinematics.pattern(refl, m, prm.k0, k_max=2.0)
        X = image.polar_image(qx, qy, I, pl["q_s"], 360, prm)
        C, Cm = correlate.correlate_direct(pl["P"], X)
        assert (z, n, 0) in correlate.tie_set(C, Cm, rel=1e-9)


def test_generator_patterns_recovered_by_oracle():
    """Noise-free generator patterns (its own geometry, tabulated reflections) are
    indexed by the oracle to within the grid resolution: generator and oracle agree
    on geometry, sign and frame conventions."""
    prm = plan.Params(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=2.0)
    pl = plan.build([fcc_phase()], prm)
    t = synth.load_table("fcc_a4.08")
    R = synth.haar_rotations(np.random.default_rng(9), 12)
    G = metrics.cubic_rotations()
    errs = []
    for m in R:
        qx, qy, I = synth.recorded_peaks(t, m, 2.0)
        keep = I > 0.01 * t["F2"].max()
        X = image.polar_image(qx[keep], qy[keep], I[keep], pl["q_s"], 360, prm)
        res, _, _ = correlate.match(pl, X)
        errs.append(metrics.misorientation_deg(res[0]["orient"], m, G))
    assert np.median(errs) < 1.5 and max(errs) < 3.0


def test_parabolic_offset_exact_vertex():
    for x0 in (-0.45, -0.1, 0.0, 0.3, 0.49):
        f = lambda x: 3.0 - 2.0 * (x - x0) ** 2
        assert abs(correlate.parabolic_offset(f(-1), f(0), f(1)) - x0) < 1e-12
    assert correlate.parabolic_offset(1.0, 1.0, 1.0) == 0.0
    assert correlate.parabolic_offset(0.0, 1.0, 5.0) == 0.0      # not concave
    assert correlate.parabolic_offset(0.0, 1.0, 1.0) == 0.5      # clamped


@pytest.mark.parametrize("N", [32, 33])
def test_spectral_bound_is_an_upper_bound_and_tight_for_a_spike(N):
    rng = np.random.default_rng(2)
    R = 20
    P = _rand_sparse(rng, (6, N, R), 0.3)
    X = _rand_sparse(rng, (N, R), 0.3)
    C, Cm = correlate.correlate_direct(P, X)
    best = np.maximum(C.max(1), Cm.max(1))
    # the all-exact form equals (1/N) sum over the FULL spectrum of the larger modulus
    Ph, Xh = np.fft.fft(P, axis=1), np.fft.fft(X, axis=0)
    full = np.maximum(np.abs(np.sum(np.conj(Ph) * Xh[None], axis=2)),
                      np.abs(np.sum(np.conj(Ph) * np.conj(Xh)[None], axis=2))).sum(1) / N
    U = correlate.spectral_bound(P, X)
    assert np.allclose(U, full, rtol=1e-12)
    assert np.all(U >= best - 1e-12)
    Nk = N // 2 + 1
    assert np.array_equal(correlate.spectral_bound(P, X, exact_freqs=Nk + 3), U)
    # split forms: every split and block size is still an upper bound; finer
    # blocks (and more exact frequencies) never loosen it
    for kc in (0, 1, 4, 9, Nk - 1):
        for blk in (3, 8):
            Ub = correlate.spectral_bound(P, X, exact_freqs=kc, block=blk)
            assert np.all(Ub >= best - 1e-12), (kc, blk)
            assert np.all(Ub >= U - 1e-12), (kc, blk)
        nested = [correlate.spectral_bound(P, X, exact_freqs=kc, block=blk) for blk in (1, 2, 4, R)]
        for lo, hi in zip(nested, nested[1:]):     # each partition refines the next
            assert np.all(hi >= lo - 1e-12), kc
        if kc > 0:
            assert np.all(correlate.spectral_bound(P, X, exact_freqs=kc - 1, block=4) >= nested[2] - 1e-12)
    # tight for a single spike in plan and image at the same radius, in both forms
    P1 = np.zeros((1, N, 5))
    P1[0, 3, 2] = 2.0
    X1 = np.zeros((N, 5))
    X1[9, 2] = 1.5
    C1, Cm1 = correlate.correlate_direct(P1, X1)
    for kc, blk in ((None, 8), (0, 5), (0, 1), (5, 2)):
        assert abs(correlate.spectral_bound(P1, X1, exact_freqs=kc, block=blk)[0] - max(C1.max(), Cm1.max())) < 1e-12


@pytest.mark.parametrize("kind", [plan.CONE, plan.GAUSS])
def test_c_direct_sum_matches_numpy_oracle(kind):
    if kind == plan.CONE:
        pl = _small_plan()
    else:
        prm = plan.Params(k_max=1.2, n_radial=32, n_angular=90, zone_step_deg=5.0, kind=plan.GAUSS)
        pl = plan.build([fcc_phase()], prm)
    d = synth.make("small")
    zs = directsum.zone_scores(pl, d["offsets"][:9], d["qx"], d["qy"], d["I"], nthreads=2)
    for p in range(8):
        o = d["offsets"]
        X = image.polar_image(d["qx"][o[p]:o[p + 1]], d["qy"][o[p]:o[p + 1]], d["I"][o[p]:o[p + 1]],
                              pl["q_s"], 90, pl["params"])
        C, Cm = correlate.correlate_direct(pl["P"], X)
        sc, n, mi = correlate.zone_best(C, Cm)
        assert np.abs(zs["score"][p] - sc).max() < 1e-12 * sc.max()
        # the chosen (n, branch) is NumPy's, or one tied with it up to FP64 summation order
        both = np.stack([C, Cm], axis=2)
        zi = np.arange(len(sc))
        got = both[zi, zs["n"][p], zs["mirror"][p]]
        assert np.all(got >= sc - 1e-12 * sc.max())
        same = (zs["n"][p] == n) & (zs["mirror"][p] == mi)
        assert same.mean() > 0.9 if kind == plan.GAUSS else same.all()
        # the neighbours reported for the parabola are the correlogram's own
        br = np.where(zs["mirror"][p][:, None] == 1, Cm, C)
        N = C.shape[1]
        assert np.abs(zs["cm1"][p] - br[zi, (zs["n"][p] - 1) % N]).max() < 1e-12 * sc.max()
        assert np.abs(zs["cp1"][p] - br[zi, (zs["n"][p] + 1) % N]).max() < 1e-12 * sc.max()


# ------------------------------------------------------------------ score ----

def _score_case():
    prm = plan.Params(k_max=2.0)
    refl = crystal.reflections(np.eye(3) * A_FCC, FCC_BASIS, 2.0)
    m_true = synth.haar_rotations(np.random.default_rng(12), 1)[0]
    qx, qy, I = kinematics.pattern(refl, m_true, prm.k0, k_max=2.0)
    return prm, refl, m_true, qx, qy, I


def test_score_gradient_matches_finite_differences():
    prm, refl, m_true, qx, qy, I = _score_case()
    rng = np.random.default_rng(1)
    m0 = m_true @ score.expm_so3(np.radians(0.6) * rng.normal(size=3) / math.sqrt(3))
    th = np.radians(0.8) * rng.normal(size=3) / math.sqrt(3)
    S, gth, gx, gy = score.score_grad(refl, qx, qy, I, m0, th, prm)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (score.score(refl, qx, qy, I, m0, th + e, prm) - score.score(refl, qx, qy, I, m0, th - e, prm)) / (2 * h)
        assert abs(fd - gth[j]) < 1e-6 * max(1.0, np.abs(gth).max())
    for i in range(0, len(qx), max(1, len(qx) // 5)):
        h2 = 1e-7
        qp, qm = qx.copy(), qx.copy()
        qp[i] += h2
        qm[i] -= h2
        fd = (score.score(refl, qp, qy, I, m0, th, prm) - score.score(refl, qm, qy, I, m0, th, prm)) / (2 * h2)
        assert abs(fd - gx[i]) < 1e-5 * max(1.0, abs(gx[i]))


def test_refinement_recovers_off_grid_truth():
    prm, refl, m_true, qx, qy, I = _score_case()
    G = metrics.cubic_rotations()
    rng = np.random.default_rng(7)
    ax = rng.normal(size=3)
    m_init = m_true @ score.expm_so3(np.radians(0.5) * ax / np.linalg.norm(ax))
    m, S, _ = score.refine_one(refl, qx, qy, I, m_init, prm, max_iter=64)
    assert metrics.misorientation_deg(m, m_init, G) > 0.45
    assert metrics.misorientation_deg(m, m_true, G) < 0.05
    assert S > score.score(refl, qx, qy, I, m_init, np.zeros(3), prm)


# ---------------------------------------------------------------- metrics ----

def test_misorientation_symmetry_and_known_angle():
    G = metrics.cubic_rotations()
    assert len(G) == 24 and len(metrics.hexagonal_rotations()) == 12
    m = synth.haar_rotations(np.random.default_rng(5), 1)[0]
    for S in G:
        assert metrics.misorientation_deg(m, S @ m, G) < 1e-6
    assert abs(metrics.misorientation_deg(m, m @ zones.Rz(math.radians(5.0)), G) - 5.0) < 1e-9
    for S in metrics.hexagonal_rotations():
        assert np.allclose(S.T @ S, np.eye(3)) and abs(np.linalg.det(S) - 1) < 1e-12


# ------------------------------------------------ overlapping patterns ----

def test_multi_edit_rule_closed_form():
    """The peak edit of Matching of Overlapping Diffraction Patterns, at known
    distances from one simulated peak: removed inside the deletion radius,
    scaled by (d - r_del) / (r_k - r_del) up to the kernel reach, kept beyond."""
    from oracle import multi
    r_del, r_k = 0.03, 0.08
    d = np.array([0.0, 0.01, 0.03, 0.055, 0.08, 0.2])
    I = np.array([2.0, 2.0, 2.0, 2.0, 2.0, 2.0])
    out = multi.edit_intensities(d, np.zeros_like(d), I, [0.0], [0.0], r_del, r_k)
    np.testing.assert_allclose(out, [0.0, 0.0, 0.0, 1.0, 2.0, 2.0], rtol=0, atol=1e-15)
    # the nearest of several simulated peaks decides
    out = multi.edit_intensities([0.5], [0.0], [1.0], [0.0, 0.445], [0.0, 0.0], r_del, r_k)
    np.testing.assert_allclose(out, [(0.055 - r_del) / (r_k - r_del)], rtol=1e-12)


def test_multi_recovers_two_grid_grains_and_stops():
    """Two noise-free grains at grid orientations summed into one pattern (the
    second at 0.6 of the intensity; 8 and 11 peaks): the iterative procedure
    returns both grains, each at its grid orientation, the higher original
    correlogram value first, with the original pattern's correlogram values; a
    third round, every peak deleted, finds nothing, and a single grain alone is
    found once."""
    from oracle import multi
    prm = plan.Params(k_max=1.2, n_radial=32, n_angular=90, zone_step_deg=5.0)
    pl = plan.build([fcc_phase()], prm)
    t = synth.load_table("fcc_a4.08")
    G = metrics.cubic_rotations()
    (za, na), (zb, nb) = (7, 13), (41, 58)
    ma = correlate.orientation(pl["M12"][za], na, 0.0, 0, 90)
    mb = correlate.orientation(pl["M12"][zb], nb, 0.0, 0, 90)
    parts = []
    for m, s in ((ma, 1.0), (mb, 0.6)):
        qx, qy, I = synth.recorded_peaks(t, m, 1.2)
        keep = I > 0.01 * t["F2"].max()
        parts.append((qx[keep], qy[keep], s * I[keep]))
    qx = np.concatenate([parts[0][0], parts[1][0]])
    qy = np.concatenate([parts[0][1], parts[1][1]])
    I = np.concatenate([parts[0][2], parts[1][2]])
    res = multi.match_multi(pl, qx, qy, I, n_orient=3, r_del=0.04)
    assert res[0] is not None and res[1] is not None and res[2] is None
    found = [r["orient"] for r in res[:2]]
    for m in (ma, mb):
        assert sorted(metrics.misorientation_deg(f, m, G) for f in found)[0] < 0.5
        assert sorted(metrics.misorientation_deg(f, m, G) for f in found)[1] > 10.0
    res = res[:2]
    X0 = image.polar_image(qx, qy, I, pl["q_s"], 90, prm)
    C0, Cm0 = correlate.correlate_direct(pl["P"], X0)
    for r in res:
        assert r["score"] == (Cm0 if r["mirror"] else C0)[r["zone"], r["n"]]
    assert res[0]["score"] > res[1]["score"] > 0.0
    alone = multi.match_multi(pl, *parts[0], n_orient=3, r_del=0.04)
    assert alone[0] is not None and metrics.misorientation_deg(alone[0]["orient"], ma, G) < 0.5
    assert alone[1] is None and alone[2] is None


def test_multi_c_variant_equals_plain_procedure():
    """The scan-sized variant (plain-C direct sum for each round's maximum) takes
    the same decisions and reports the same original-pattern values as the numpy
    procedure, on seeded overlapping patterns."""
    from oracle import multi
    prm = plan.Params(k_max=1.2, n_radial=32, n_angular=90, zone_step_deg=5.0)
    pl = plan.build([fcc_phase()], prm)
    d = synth.make("overlap", n=6, k_max=1.2)
    o = d["offsets"]
    for p in range(6):
        args = (d["qx"][o[p]:o[p + 1]].astype(np.float64), d["qy"][o[p]:o[p + 1]].astype(np.float64),
                d["I"][o[p]:o[p + 1]].astype(np.float64))
        a = multi.match_multi(pl, *args, 3, 0.04)
        b = multi.match_multi_c(pl, *args, 3, 0.04)
        for ra, rb in zip(a, b):
            assert (ra is None) == (rb is None)
            if ra is None:
                continue
            assert (ra["zone"], ra["n"], ra["mirror"]) == (rb["zone"], rb["n"], rb["mirror"])
            assert abs(ra["score"] - rb["score"]) <= 1e-9 * abs(ra["score"])


# ------------------------------------------------------- fiber texture ----

@pytest.mark.parametrize("axis", [[0, 0, 1], [1, 1, 1], [1, 2, 0.3]])
def test_fiber_grid_geometry(axis):
    """Fiber-texture zone sets: the axis comes first; every direction is a unit
    vector within theta_max of the axis, on rings of polar angle i*step; a full
    ring of polar angle theta has ceil(360 sin(theta) / step) points whose
    neighbours are at most `step` of arc apart; a wedge keeps its two ends."""
    step, tmax = 2.0, 10.0
    w = zones.fiber_grid(axis, tmax, step)
    f = np.asarray(axis, float) / np.linalg.norm(axis)
    np.testing.assert_allclose(w[0], f, atol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-14)
    th = np.degrees(np.arccos(np.clip(w @ f, -1, 1)))
    assert th.max() <= tmax + 1e-9
    rings = np.round(th / step).astype(int)
    np.testing.assert_allclose(th, rings * step, atol=1e-9)
    for i in range(1, int(tmax / step) + 1):
        ring = w[rings == i]
        assert len(ring) == math.ceil(360.0 * math.sin(math.radians(i * step)) / step - 1e-9)
        # neighbours around the ring: arc length along the ring circle <= step
        c = ring - np.outer(ring @ f, f)
        ang = np.sort(np.degrees(np.arctan2(c @ np.cross(f, c[0] / np.linalg.norm(c[0])), c @ (c[0] / np.linalg.norm(c[0])))) % 360.0)
        gaps = np.diff(np.concatenate([ang, [ang[0] + 360.0]]))
        assert gaps.max() * math.sin(math.radians(i * step)) <= step + 1e-9
    wedge = zones.fiber_grid(axis, tmax, step, 0.0, 90.0)
    assert len(wedge) == 1 + sum(math.ceil(90.0 * math.sin(math.radians(i * step)) / step - 1e-9) + 1
                                 for i in range(1, 6))
