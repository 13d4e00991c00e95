"""Pins of the disk-detection oracle (oracle/disks.py) to brute force, the
correlation theorem, closed forms and hand-built correlation maps."""
import numpy as np
import pytest

import synth
from oracle import disks


def test_correlation_equals_brute_force_sum():
    rng = np.random.default_rng(5)
    f = rng.normal(size=(8, 8))
    t = rng.normal(size=(8, 8))
    C = disks.correlate(f, t)
    B = np.zeros((8, 8))
    for y in range(8):
        for x in range(8):
            s = 0.0
            for u in range(8):
                for v in range(8):
                    s += f[(y + u) % 8, (x + v) % 8] * t[u, v]
            B[y, x] = s
    assert np.max(np.abs(C - B)) < 1e-12


def test_correlation_theorem():
    """The DFT of a circular cross-correlation is F(f) times the conjugate of F(t)."""
    rng = np.random.default_rng(6)
    f = rng.normal(size=(32, 24))
    t = np.zeros((32, 24))
    t[rng.integers(0, 32, 40), rng.integers(0, 24, 40)] = rng.normal(size=40)
    C = disks.correlate(f, t)
    ref = np.fft.ifft2(np.fft.fft2(f) * np.conj(np.fft.fft2(t))).real
    assert np.max(np.abs(C - ref)) < 1e-11


def test_single_disk_closed_form():
    """One disk of amplitude h on a zero frame: by Cauchy-Schwarz the unique
    maximum is at its centre with value h * sum(t^2); the two neighbours on each
    axis are equal, so the sub-pixel offset is zero."""
    probe = synth.probe_disk(64, 32, 32, 3.5)
    t = disks.probe_template(probe, 32, 32)
    h, y0, x0 = 7.0, 21, 40
    frame = h * synth.probe_disk(64, y0, x0, 3.5)
    qx, qy, I, ys, xs = disks.detect(frame, t, edge=4, min_rel=0.5, min_spacing=3, max_peaks=8,
                                     cy=32.0, cx=32.0, pixel_size=0.1)
    assert list(ys) == [y0] and list(xs) == [x0]
    assert abs(I[0] - h * np.sum(t * t)) < 1e-10 * I[0]
    assert abs(qx[0] - (x0 - 32) * 0.1) < 1e-12 and abs(qy[0] - (y0 - 32) * 0.1) < 1e-12


def test_subpixel_vertex_of_a_quadratic():
    """With a unit template at the origin the correlation is the frame itself; on
    a quadratic bump the three-point parabola gives the vertex exactly, per axis."""
    t = np.zeros((64, 64))
    t[0, 0] = 1.0
    y, x = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    y0, x0 = 30.7, 20.3
    frame = np.maximum(0.0, 100.0 - 2.0 * (x - x0) ** 2 - 3.0 * (y - y0) ** 2)
    qx, qy, I, ys, xs = disks.detect(frame, t, edge=2, min_rel=0.5, min_spacing=3, max_peaks=4,
                                     cy=32.0, cx=32.0, pixel_size=1.0)
    assert list(ys) == [31] and list(xs) == [20]
    assert abs(qx[0] - (x0 - 32.0)) < 1e-9
    assert abs(qy[0] - (y0 - 32.0)) < 1e-9
    assert abs(I[0] - frame[31, 20]) < 1e-12


def _spikes(H, W, spikes):
    f = np.zeros((H, W))
    for (yy, xx), v in spikes.items():
        f[yy, xx] = v
    return f


@pytest.mark.parametrize("max_peaks,min_abs,expect", [
    (8, 0.0, [(20, 20), (60, 100), (40, 40), (10, 60)]),
    (2, 0.0, [(20, 20), (60, 100)]),
    (8, 60.0, [(20, 20), (60, 100)]),
])
def test_selection_rules_on_a_hand_built_map(max_peaks, min_abs, expect):
    """Unit template, so C is the map below; expected lists written by hand:
    (2,2) lies in the 4-pixel edge band; (64,64) is within 3 px of the axis;
    (20,23) is 3 px from the stronger (20,20) (spacing 5); (60,100) ties with
    (20,20) and comes after it in raster order; (10,60) at 0.6 passes
    0.005 * 100; (50,10) at 0.4 does not; the plateau (80,80)-(80,81) has no
    strict maximum."""
    H = W = 128
    t = np.zeros((H, W))
    t[0, 0] = 1.0
    f = _spikes(H, W, {(20, 20): 100.0, (20, 23): 90.0, (40, 40): 50.0, (2, 2): 200.0, (64, 64): 300.0,
                       (50, 10): 0.4, (10, 60): 0.6, (60, 100): 100.0, (80, 80): 70.0, (80, 81): 70.0})
    qx, qy, I, ys, xs = disks.detect(f, t, edge=4, min_rel=0.005, min_abs=min_abs, min_spacing=5,
                                     max_peaks=max_peaks, cy=64.0, cx=64.0, r_excl=3.0, pixel_size=1.0)
    assert list(zip(ys.tolist(), xs.tolist())) == expect
    assert np.all(np.diff(I) <= 0)


def test_detection_finds_the_rendered_disks():
    """Synthetic frames: every rendered disk well inside the frame, away from the
    axis and from other disks, and bright enough, is found within 0.25 px."""
    d = synth.frames(n=6, size=128)
    cy, cx = d["center"]
    t = disks.probe_template(d["probe"], int(cy), int(cx))
    pix = d["pixel_size"]
    found = missed = 0
    for i in range(6):
        qx, qy, I, ys, xs = disks.detect(d["frames"][i], t, edge=5, min_rel=0.005, min_spacing=5,
                                         max_peaks=64, cy=cy, cx=cx, r_excl=4.0, pixel_size=pix)
        px, py = qx / pix + cx, qy / pix + cy
        ty, tx, a = d["peaks_y"][i], d["peaks_x"][i], d["amplitude"][i]
        for j in range(len(ty)):
            others = np.hypot(ty - ty[j], tx - tx[j])
            others[j] = np.inf
            if (a[j] < 30 or min(ty[j], tx[j]) < 8 or max(ty[j], tx[j]) > 120 or others.min() < 9
                    or np.hypot(ty[j] - cy, tx[j] - cx) < 9):
                continue
            dist = np.hypot(py - ty[j], px - tx[j])
            if dist.min() < 0.25:
                found += 1
            else:
                missed += 1
    assert found >= 50 and missed == 0, (found, missed)


def test_decision_margin_sees_a_near_tie():
    H = W = 64
    t = np.zeros((H, W))
    t[0, 0] = 1.0
    f = _spikes(H, W, {(20, 20): 100.0, (30, 30): 50.0})
    kw = dict(edge=4, min_rel=0.005, min_abs=0.0, min_spacing=5, max_peaks=8, cy=32.0, cx=32.0, r_excl=0.0)
    assert disks.decision_margin(f, **kw) > 0.1
    f[20, 21] = 100.0 - 1e-9          # a neighbour within 1e-9 of the maximum
    assert disks.decision_margin(f, **kw) < 1e-9
