"""Seeded synthetic diffraction scans shaped like the paper's workloads.

This module is the one input source shared by the oracle-side tests and the
HIP path.  It holds none of the matching method's arithmetic: the reflections
of each test crystal (positions g and intensities |F|^2, and the beam
wavenumber) are data, read from tables/*.json that an oracle script wrote; here
there is only geometry (rotating those vectors into the sample frame, their
distance to the Ewald sphere, projection) and random draws from
numpy.random.Generator(PCG64(seed)).

Measurement model (a stand-in for the paper's missing datasets): a reflection
at sample-frame position g_s is recorded at (g_s,x, g_s,y) with intensity
|F|^2 exp(-e^2 / (2 sigma^2)), e = k0 - |k0 z + g_s| (its distance to the Ewald
sphere), sigma = 0.02 1/A; positions get N(0, 0.005^2) jitter per axis (half
the 0.01 1/A reciprocal pixel of the paper's simulations), intensities a
(1 + 0.05 N(0,1)) factor, and some configurations add spurious peaks.

Configurations (name -> recipe):
  small   128 Haar-random FCC orientations, peaks with I > 1% of max |F|^2, |g| < 1.2,
          0-2 spurious peaks                                        (seed 1001)
  scan    256x256 FCC scan, 50 Voronoi grains, |g| < 2.0, >= 10 peaks per grain
          (redrawn otherwise), at most the 60 strongest, noise + spurious (seed 1002)
  hcp     the same geometry with the HCP crystal                     (seed 1003)
  multi   512x512 scan, 200 grains, phase per grain uniform in {FCC, BCC, HCP},
          n ~ round(exp(U(ln 3, ln 150))) strongest reflections, noise (seed 1004)
  refine  65,536 Haar-random FCC orientations, noise as 'scan'       (seed 1005)
  overlap patterns that each sum the peaks of two Haar-random FCC grains (the
          second's intensities scaled by U(0.4, 0.9)), per grain the reflections
          above 1% of max |F|^2 (at most its 40 strongest), noise as 'scan' (seed 1006)
  frames  raw size x size detector frames (float32 counts) of Haar-random FCC grains: each
          recorded peak (at most the 40 strongest above 1% of max |F|^2, jitter as 'scan')
          drawn as a probe disk (radius 3.5 px, 1 px linear edge) of amplitude 1000 I/max|F|^2
          centred at its sub-pixel position, an unscattered beam of amplitude 3000 on the
          optical axis (size/2, size/2), background 2 + N(0, 3^2) + shot noise N(0, signal);
          |q| = k_max falls (size/2 - 4) px from the axis; plus the vacuum probe image
          (the same disk on the axis, noise-free); optionally the frames of a scan of Voronoi
          grains instead of independent orientations                 (seed 1007)
"""
import json
import math
import os

import numpy as np

_TABLES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tables")
PHASE_NAMES = ("fcc_a4.08", "bcc_a2.87", "hcp_a2.95_c4.68")


def load_table(name):
    with open(os.path.join(_TABLES, name + ".json")) as f:
        d = json.load(f)
    return {"g": np.asarray(d["g"], np.float64), "F2": np.asarray(d["F2"], np.float64),
            "k0": float(d["k0"]), "lattice": np.asarray(d["lattice"], np.float64),
            "frac_xyz": np.asarray(d["frac_xyz"], np.float64), "name": name}


def haar_rotations(rng, n):
    """n uniformly random rotation matrices (normalised 4-D Gaussian quaternions)."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def recorded_peaks(table, m, k_max, sigma=0.02):
    """Noise-free recorded peaks for orientation m (d = m d0): (qx, qy, I), all
    reflections with |g| < k_max, strongest first."""
    g = table["g"]
    keep = np.sqrt(np.sum(g * g, axis=1)) < k_max
    gs = g[keep] @ np.asarray(m, np.float64)          # rows m^T g
    k0 = table["k0"]
    e = k0 - np.sqrt(gs[:, 0] ** 2 + gs[:, 1] ** 2 + (k0 + gs[:, 2]) ** 2)
    I = table["F2"][keep] * np.exp(-e * e / (2.0 * sigma * sigma))
    o = np.argsort(-I, kind="stable")
    return gs[o, 0], gs[o, 1], I[o]


def _noisy(rng, qx, qy, I, jitter=0.005, inoise=0.05):
    n = len(qx)
    return (qx + rng.normal(0.0, jitter, n), qy + rng.normal(0.0, jitter, n),
            I * (1.0 + inoise * rng.normal(size=n)))


def _spurious(rng, I_real, k_max):
    cnt = int(rng.integers(0, 3))
    r = k_max * np.sqrt(rng.random(cnt))
    t = 2.0 * math.pi * rng.random(cnt)
    med = float(np.median(I_real)) if len(I_real) else 1.0
    return r * np.cos(t), r * np.sin(t), rng.uniform(0.1, 1.0, cnt) * med


def _pack(lists, truth, phase, meta):
    counts = np.array([len(l[0]) for l in lists], dtype=np.int64)
    offsets = np.zeros(len(lists) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    cat = lambda i: (np.concatenate([l[i] for l in lists]).astype(np.float32) if len(lists)
                     else np.zeros(0, np.float32))
    out = {"offsets": offsets, "qx": cat(0), "qy": cat(1), "I": cat(2),
           "truth": np.asarray(truth, np.float64), "phase": np.asarray(phase, np.int32)}
    out.update(meta)
    return out


def voronoi_labels(rng, ny, nx, n_grains):
    """Nearest seed (ties -> lower id) of every pixel centre; seeds uniform in the scan."""
    seeds = rng.random((n_grains, 2)) * np.array([ny, nx])
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    best = np.zeros((ny, nx), dtype=np.int64)
    bd = np.full((ny, nx), np.inf)
    for i in range(n_grains):
        d = (yy - seeds[i, 0]) ** 2 + (xx - seeds[i, 1]) ** 2
        upd = d < bd
        best[upd] = i
        bd[upd] = d[upd]
    return best.ravel()


def small(seed=1001, n=128, k_max=1.2):
    rng = np.random.default_rng(seed)
    t = load_table("fcc_a4.08")
    R = haar_rotations(rng, n)
    lists = []
    for i in range(n):
        qx, qy, I = recorded_peaks(t, R[i], k_max)
        keep = I > 0.01 * t["F2"].max()
        qx, qy, I = _noisy(rng, qx[keep], qy[keep], I[keep])
        sx, sy, sI = _spurious(rng, I, k_max)
        lists.append((np.concatenate([qx, sx]), np.concatenate([qy, sy]), np.concatenate([I, sI])))
    return _pack(lists, R, np.zeros(n), {"name": "small", "k_max": k_max, "phases": ["fcc_a4.08"]})


def _grain_patterns(rng, tables, grain_phase, k_max, min_peaks, max_peaks, rel_cut, ragged=None):
    """Noise-free peak lists per grain (orientation redrawn until >= min_peaks)."""
    G = len(grain_phase)
    R = np.zeros((G, 3, 3))
    base = []
    for i in range(G):
        t = tables[grain_phase[i]]
        while True:
            m = haar_rotations(rng, 1)[0]
            qx, qy, I = recorded_peaks(t, m, k_max)
            if ragged is None:
                keep = I > rel_cut * t["F2"].max()
                qx, qy, I = qx[keep], qy[keep], I[keep]
                if len(qx) >= min_peaks:
                    qx, qy, I = qx[:max_peaks], qy[:max_peaks], I[:max_peaks]
                    break
            else:
                nk = ragged[i]
                qx, qy, I = qx[:nk], qy[:nk], I[:nk]
                break
        R[i] = m
        base.append((qx, qy, I))
    return R, base


def scan(seed=1002, ny=256, nx=256, n_grains=50, k_max=2.0, phase_name="fcc_a4.08", spurious=True):
    rng = np.random.default_rng(seed)
    t = load_table(phase_name)
    lab = voronoi_labels(rng, ny, nx, n_grains)
    R, base = _grain_patterns(rng, [t], np.zeros(n_grains, dtype=np.int64), k_max, 10, 60, 0.01)
    lists = []
    for p in range(ny * nx):
        qx, qy, I = _noisy(rng, *base[lab[p]])
        if spurious:
            sx, sy, sI = _spurious(rng, I, k_max)
            qx, qy, I = np.concatenate([qx, sx]), np.concatenate([qy, sy]), np.concatenate([I, sI])
        lists.append((qx, qy, I))
    return _pack(lists, R[lab], np.zeros(ny * nx), {"name": "scan", "k_max": k_max, "phases": [phase_name],
                                                     "grain": lab, "shape": (ny, nx)})


def hard(seed=1008, ny=256, nx=256, n_grains=50, k_max=2.0, drop=0.2, inoise=0.3, spurious=(5, 10)):
    """The scan's geometry with degraded peak lists (the regime of the paper's
    dynamical and experimental patterns, where intensities depart from the
    kinematical ones and peaks are missed or spurious): each real peak is
    dropped with probability `drop`, intensities are multiplied by
    (1 + inoise N(0, 1)) (clipped at 0), and 5-10 spurious peaks (positions
    area-uniform in |q| < k_max, intensities U(0.1, 1) of the median) are
    added."""
    rng = np.random.default_rng(seed)
    t = load_table("fcc_a4.08")
    lab = voronoi_labels(rng, ny, nx, n_grains)
    R, base = _grain_patterns(rng, [t], np.zeros(n_grains, dtype=np.int64), k_max, 10, 60, 0.01)
    lists = []
    for p in range(ny * nx):
        bx, by, bI = base[lab[p]]
        keep = rng.random(len(bx)) >= drop
        qx, qy, I = _noisy(rng, bx[keep], by[keep], bI[keep], inoise=inoise)
        I = np.maximum(I, 0.0)
        cnt = int(rng.integers(spurious[0], spurious[1] + 1))
        r = k_max * np.sqrt(rng.random(cnt))
        a = 2.0 * math.pi * rng.random(cnt)
        med = float(np.median(bI)) if len(bI) else 1.0
        lists.append((np.concatenate([qx, r * np.cos(a)]), np.concatenate([qy, r * np.sin(a)]),
                      np.concatenate([I, rng.uniform(0.1, 1.0, cnt) * med])))
    return _pack(lists, R[lab], np.zeros(ny * nx), {"name": "hard", "k_max": k_max, "phases": ["fcc_a4.08"],
                                                     "grain": lab, "shape": (ny, nx)})


def hcp(seed=1003, ny=256, nx=256, n_grains=50, k_max=2.0):
    d = scan(seed, ny, nx, n_grains, k_max, "hcp_a2.95_c4.68")
    d["name"] = "hcp"
    return d


def multi(seed=1004, ny=512, nx=512, n_grains=200, k_max=2.0):
    rng = np.random.default_rng(seed)
    tables = [load_table(n) for n in PHASE_NAMES]
    lab = voronoi_labels(rng, ny, nx, n_grains)
    gphase = rng.integers(0, 3, n_grains)
    npix = ny * nx
    nk = np.rint(np.exp(rng.uniform(math.log(3), math.log(150), npix))).astype(np.int64)
    R, base = _grain_patterns(rng, tables, gphase, k_max, 0, 10 ** 9, 0.0, ragged=np.full(n_grains, 10 ** 9))
    lists = []
    for p in range(npix):
        bx, by, bI = base[lab[p]]
        k = min(int(nk[p]), len(bx))
        lists.append(_noisy(rng, bx[:k], by[:k], bI[:k]))
    return _pack(lists, R[lab], gphase[lab], {"name": "multi", "k_max": k_max, "phases": list(PHASE_NAMES),
                                              "grain": lab, "shape": (ny, nx)})


def refine(seed=1005, n=65536, k_max=2.0, phase_name="fcc_a4.08"):
    rng = np.random.default_rng(seed)
    t = load_table(phase_name)
    R = haar_rotations(rng, n)
    lists = []
    for i in range(n):
        qx, qy, I = recorded_peaks(t, R[i], k_max)
        keep = I > 0.01 * t["F2"].max()
        qx, qy, I = qx[keep][:60], qy[keep][:60], I[keep][:60]
        lists.append(_noisy(rng, qx, qy, I))
    return _pack(lists, R, np.zeros(n), {"name": "refine", "k_max": k_max, "phases": [phase_name]})


def overlap(seed=1006, n=4096, k_max=2.0, second=(0.4, 0.9), per_grain=40):
    rng = np.random.default_rng(seed)
    t = load_table("fcc_a4.08")
    R = haar_rotations(rng, 2 * n).reshape(n, 2, 3, 3)
    lists = []
    for i in range(n):
        parts = []
        for j in range(2):
            qx, qy, I = recorded_peaks(t, R[i, j], k_max)
            keep = I > 0.01 * t["F2"].max()
            qx, qy, I = qx[keep][:per_grain], qy[keep][:per_grain], I[keep][:per_grain]
            if j == 1:
                I = I * rng.uniform(*second)
            parts.append((qx, qy, I))
        qx = np.concatenate([parts[0][0], parts[1][0]])
        qy = np.concatenate([parts[0][1], parts[1][1]])
        I = np.concatenate([parts[0][2], parts[1][2]])
        lists.append(_noisy(rng, qx, qy, I))
    return _pack(lists, R, np.zeros(n), {"name": "overlap", "k_max": k_max, "phases": ["fcc_a4.08"]})


def probe_disk(size, cy, cx, radius=3.5):
    """A probe disk of the given radius with a 1 px linear edge, centred at (cy, cx)."""
    y, x = np.meshgrid(np.arange(size), np.arange(size), indexing="ij")
    rho = np.sqrt((y - cy) ** 2 + (x - cx) ** 2)
    return np.clip(radius + 0.5 - rho, 0.0, 1.0)


def frames(seed=1007, n=256, size=128, k_max=2.0, per_grain=40, radius=3.5, grain_map=None):
    """grain_map=(ny, nx, n_grains): the frames of an ny x nx scan whose pixels take
    the orientation of the nearest of n_grains Voronoi seeds (n = ny * nx), as in
    'scan'; else n Haar-random orientations."""
    rng = np.random.default_rng(seed)
    t = load_table("fcc_a4.08")
    if grain_map is not None:
        ny, nx, ng = grain_map
        lab = voronoi_labels(rng, ny, nx, ng)
        R = haar_rotations(rng, ng)[lab]
        n = ny * nx
    else:
        R = haar_rotations(rng, n)
    c = size // 2
    pix = k_max / (size / 2 - 4)
    w = int(math.ceil(radius + 1.5))
    oy, ox = np.meshgrid(np.arange(-w, w + 1), np.arange(-w, w + 1), indexing="ij")
    out = np.empty((n, size, size), np.float32)
    peaks_y, peaks_x, amps = [], [], []
    Fmax = t["F2"].max()
    for i in range(n):
        qx, qy, I = recorded_peaks(t, R[i], k_max)
        keep = I > 0.01 * Fmax
        qx, qy, I = _noisy(rng, qx[keep][:per_grain], qy[keep][:per_grain], I[keep][:per_grain])
        py = np.concatenate([[float(c)], c + qy / pix])
        px = np.concatenate([[float(c)], c + qx / pix])
        a = np.concatenate([[3000.0], 1000.0 * np.maximum(I, 0.0) / Fmax])
        sig = np.zeros((size, size))
        iy = np.rint(py).astype(np.int64)
        ix = np.rint(px).astype(np.int64)
        yy = iy[:, None, None] + oy[None]
        xx = ix[:, None, None] + ox[None]
        rho = np.sqrt((yy - py[:, None, None]) ** 2 + (xx - px[:, None, None]) ** 2)
        val = a[:, None, None] * np.clip(radius + 0.5 - rho, 0.0, 1.0)
        ok = (yy >= 0) & (yy < size) & (xx >= 0) & (xx < size) & (val > 0)
        np.add.at(sig, (yy[ok], xx[ok]), val[ok])
        f = 2.0 + sig + rng.normal(0.0, 3.0, sig.shape) + rng.normal(size=sig.shape) * np.sqrt(sig)
        out[i] = f
        peaks_y.append(py[1:])
        peaks_x.append(px[1:])
        amps.append(a[1:])
    return {"name": "frames", "frames": out, "probe": probe_disk(size, c, c, radius).astype(np.float32),
            "center": (float(c), float(c)), "pixel_size": pix, "k_max": k_max, "truth": R,
            "peaks_y": peaks_y, "peaks_x": peaks_x, "amplitude": amps, "phases": ["fcc_a4.08"]}


def subset(d, idx):
    """Patterns idx of a generated scan, re-packed (for bounded oracle samples)."""
    idx = np.asarray(idx, dtype=np.int64)
    off = d["offsets"]
    lists = [(d["qx"][off[i]:off[i + 1]], d["qy"][off[i]:off[i + 1]], d["I"][off[i]:off[i + 1]]) for i in idx]
    return _pack(lists, d["truth"][idx], d["phase"][idx], {"name": d["name"] + "_subset", "k_max": d["k_max"],
                                                            "phases": d["phases"]})


CONFIGS = {"small": small, "scan": scan, "hcp": hcp, "multi": multi, "refine": refine, "overlap": overlap,
           "frames": frames, "hard": hard}


def make(name, **kw):
    return CONFIGS[name](**kw)
