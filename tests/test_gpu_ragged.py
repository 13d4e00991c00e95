"""Patterns longer than the polar kernel's peak cache, against the FP64 oracle.

The polar pass prepares at most 128 peaks at once with 32 radial columns per
pass (256 with 16 columns); a longer pattern takes the path that re-prepares
its peaks batch by batch for every radial tile.  These tests build patterns of
127 to 400 peaks (peak lists of several scan patterns laid over one another,
as in a pattern that crosses a grain boundary) at the scan's plan (k_max = 2,
128 radial x 360 angular bins, 1081 zones) and compare, with both pass widths:

  * X and FFT{X} cell by cell with the oracle (Eq. image_polar, then numpy's
    rfft of the oracle's X) within 1e-6 of the pattern's largest value: every
    cell is a sum of a few FP32 kernel values (each within a few ulp), and the
    FFT adds ~log2(360) roundings relative to the spectrum's scale;
  * the decisions, tie-aware, against the plain-C FP64 direct sum (FP32 and
    BF16 contractions);
  * data errors (NaN position or intensity, negative intensity) placed in any
    wave's share of the peaks and beyond either cache size: the pattern is
    flagged (zone -1, score 0) and its image is zero.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import directsum
from tests import helpers

pytestmark = pytest.mark.gpu

COUNTS = [127, 128, 129, 140, 200, 255, 256, 257, 300, 384, 400, 150]
# (peaks in the pattern, index of the bad peak, field, value)
BAD = [(100, 70, "qx", np.nan), (120, 99, "I", -1.0), (200, 130, "I", -0.5), (300, 200, "qy", np.nan),
       (350, 300, "I", -2.0), (400, 390, "I", np.nan), (260, 257, "qx", np.inf)]


@pytest.fixture(scope="module")
def acom():
    from paper_2111_00171_amd import acom as a
    a.lib()
    return a


def _long_patterns(d, counts, seed):
    """Each pattern: the peaks of randomly drawn scan patterns, one after the
    other, cut at the wanted count."""
    rng = np.random.default_rng(seed)
    o = d["offsets"]
    n = len(o) - 1
    lists = []
    for c in counts:
        parts, tot = [], 0
        while tot < c:
            p = int(rng.integers(n))
            take = min(c - tot, int(o[p + 1] - o[p]))
            sl = slice(o[p], o[p] + take)
            parts.append((d["qx"][sl], d["qy"][sl], d["I"][sl]))
            tot += take
        lists.append(tuple(np.concatenate([q[i] for q in parts]).astype(np.float32) for i in range(3)))
    return lists


def _pack(lists):
    off = np.concatenate([[0], np.cumsum([len(l[0]) for l in lists])]).astype(np.int64)
    return {"offsets": off, "qx": np.concatenate([l[0] for l in lists]),
            "qy": np.concatenate([l[1] for l in lists]), "I": np.concatenate([l[2] for l in lists])}


@pytest.fixture(scope="module")
def long_set(acom):
    d = synth.make("scan")
    lists = _long_patterns(d, COUNTS, 41)
    bad = _long_patterns(d, [b[0] for b in BAD], 42)
    for (n, i, field, v), l in zip(BAD, bad):
        k = {"qx": 0, "qy": 1, "I": 2}[field]
        l[k][i] = v
    dd = _pack(lists + bad)
    opl = helpers.oracle_plan(["fcc"], **helpers.SCAN)
    gpl = helpers.gpu_plan(["fcc"], precisions=("fp32", "bf16"), **helpers.SCAN)
    return dd, opl, gpl


@pytest.mark.parametrize("cols", [32, 16])
def test_long_patterns_image_and_spectrum(acom, long_set, cols):
    dd, opl, gpl = long_set
    pk = acom.Peaks.from_host(dd)
    try:
        acom.set_tuning(polar_cols=cols)
        X = gpl.polar_image(pk).cpu().numpy()
        Xr, Xi = gpl.polar_spectrum(pk)
        Xr, Xi = Xr.cpu().numpy(), Xi.cpu().numpy()
    finally:
        acom.set_tuning(polar_cols=32)
    worst_x = worst_f = 0.0
    for p in range(len(COUNTS)):
        Xo = helpers.oracle_image(opl, dd, p)
        sc = np.abs(Xo).max()
        ex = np.abs(X[p] - Xo).max() / sc
        F = np.fft.rfft(Xo, axis=0)
        scf = np.abs(F).max()
        ef = max(np.abs(Xr[p] - F.real).max(), np.abs(Xi[p] - F.imag).max()) / scf
        worst_x, worst_f = max(worst_x, ex), max(worst_f, ef)
        assert ex <= 1e-6, (p, COUNTS[p], ex)
        assert ef <= 1e-6, (p, COUNTS[p], ef)
    print(f"cols {cols}: max |X - oracle| / max X = {worst_x:.2e}, spectrum {worst_f:.2e}")
    for j in range(len(BAD)):
        p = len(COUNTS) + j
        assert np.all(X[p] == 0) and np.all(Xr[p] == 0) and np.all(Xi[p] == 0), BAD[j]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_long_patterns_decisions(acom, long_set, precision):
    dd, opl, gpl = long_set
    pk = acom.Peaks.from_host(dd)
    out = {}
    try:
        for cols in (32, 16):
            acom.set_tuning(polar_cols=cols)
            r = gpl.match(pk, top_k=2, precision=precision)
            torch.cuda.synchronize()
            out[cols] = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    finally:
        acom.set_tuning(polar_cols=32)
    for k in ("zone", "bin", "mirror", "score"):
        assert np.array_equal(out[32][k], out[16][k]), k
    res = out[32]
    nl = len(COUNTS)
    sub = {"offsets": dd["offsets"][:nl + 1], "qx": dd["qx"], "qy": dd["qy"], "I": dd["I"]}
    zs = directsum.zone_scores(opl, sub["offsets"], sub["qx"], sub["qy"], sub["I"])
    for p in range(nl):
        sc = zs["score"][p]
        mx = sc.max()
        z = int(res["zone"][p, 0])
        assert z >= 0 and sc[z] >= mx - 1e-5 * mx, (p, COUNTS[p], z, sc[z], mx)
        assert abs(res["score"][p, 0] - sc[z]) <= 1e-5 * mx
        z2 = int(res["zone"][p, 1])
        others = np.delete(sc, z)
        assert z2 >= 0 and sc[z2] >= others.max() - 1e-5 * mx
    for j in range(len(BAD)):
        p = nl + j
        assert np.all(res["zone"][p] == -1) and np.all(res["score"][p] == 0), BAD[j]
        assert res["n_evaluated"][p] == 0
