"""Multi-phase plans (concatenated phases, argmax over all of them), the
hexagonal two-triangle zone set, and capture of acom_match in a HIP graph."""
import numpy as np
import pytest
import torch

import synth
from oracle import correlate
from tests import helpers

pytestmark = pytest.mark.gpu

MULTI = dict(k_max=2.0, n_radial=64, n_angular=180, zone_step_deg=5.0)


@pytest.fixture(scope="module")
def acom():
    from paper_2111_00171_amd import acom as a
    a.lib()
    return a


def test_hcp_two_triangle_plan_matches_oracle(acom):
    cfg = dict(k_max=1.6, n_radial=32, n_angular=120, zone_step_deg=10.0)
    opl = helpers.oracle_plan(["hcp"], **cfg)
    gpl = helpers.gpu_plan(["hcp"], keep_f64=True, precisions=("fp32",), **cfg)
    assert gpl.n_zones == len(opl["zones"]) == 2 * 55 - 10
    assert np.allclose(gpl.info()["zones"], opl["zones"], atol=1e-14)
    P = gpl.angular_f64()
    assert np.abs(P - opl["P"]).max() < 1e-12 * np.abs(opl["P"]).max()


@pytest.fixture(scope="module")
def multi(acom):
    d = synth.multi(ny=16, nx=16, n_grains=12)
    opl = helpers.oracle_plan(["fcc", "bcc", "hcp"], **MULTI)
    gpl = helpers.gpu_plan(["fcc", "bcc", "hcp"], **MULTI)
    return d, opl, gpl


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_multiphase_match(acom, multi, precision):
    d, opl, gpl = multi
    assert gpl.n_phases == 3 and gpl.n_zones == len(opl["zones"])
    info = gpl.info()
    assert np.array_equal(info["zone_phase"], opl["zone_phase"])
    res = gpl.match(acom.Peaks.from_host(d), top_k=2, precision=precision)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in res.items() if v is not None}
    pats = list(range(0, 256, 7))
    for p in pats:
        Xo = helpers.oracle_image(opl, d, p)
        Co, Cmo = correlate.correlate_direct(opl["P"], Xo)
        sc, _, _ = correlate.zone_best(Co, Cmo)
        mx = sc.max()
        z = int(res["zone"][p, 0])
        assert sc[z] >= mx - 1e-5 * mx
        assert res["phase"][p, 0] == opl["zone_phase"][z]
    # phase identification against the generator's truth (patterns with >= 8 peaks)
    cnt = np.diff(d["offsets"])
    ok = [res["phase"][p, 0] == d["phase"][p] for p in range(256) if cnt[p] >= 8]
    assert np.mean(ok) > 0.9


def test_match_in_hip_graph(acom, multi):
    """acom_match allocates nothing and never synchronises: captured once, the
    graph replays on new peak data and reproduces eager results bit for bit."""
    d, opl, gpl = multi
    pk = acom.Peaks.from_host(d)
    n = pk.n_patterns
    ws = torch.empty(gpl.match_workspace_bytes("bf16", 128), dtype=torch.uint8, device="cuda")
    out = gpl.empty_matches(n, 2, True, "cuda")
    gpl.match(pk, 2, "bf16", 128, ws, out=out)       # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpl.match(pk, 2, "bf16", 128, ws, out=out)
    rng = np.random.default_rng(3)
    for rep in range(3):
        ang = rng.uniform(-0.3, 0.3)
        qx = d["qx"] * np.cos(ang) - d["qy"] * np.sin(ang)
        qy = d["qx"] * np.sin(ang) + d["qy"] * np.cos(ang)
        I = d["I"] * rng.uniform(0.8, 1.2, len(d["I"]))
        pk.qx.copy_(torch.tensor(qx, dtype=torch.float32))
        pk.qy.copy_(torch.tensor(qy, dtype=torch.float32))
        pk.intensity.copy_(torch.tensor(I, dtype=torch.float32))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = {k: v.clone() for k, v in out.items() if v is not None}
        fresh = acom.Peaks(d["offsets"], qx, qy, I)
        ref = gpl.match(fresh, 2, "bf16", 128)
        torch.cuda.synchronize()
        for k in ("zone", "bin", "mirror", "score", "phi3", "orient", "n_evaluated"):
            assert torch.equal(got[k], ref[k]), (rep, k)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_autotune_keeps_results(acom, multi, precision):
    """The autotuner picks a contraction shape by timing; matching with it gives
    the same decisions and exact scores as the library's default shape."""
    d, opl, gpl = multi
    pk = acom.Peaks.from_host(d)
    ref = gpl.match(pk, top_k=2, precision=precision, chunk=128)
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ref.items() if v is not None}
    shape = gpl.autotune(pk, precision, chunk=128)
    assert shape["tile"] in ("64x64", "large") and shape["order"] in (0, 1) and shape["ms"] > 0.0
    assert shape["radii_per_step"] in ((16, 32) if precision == "fp32" else (32, 64, 128))
    res = gpl.match(pk, top_k=2, precision=precision, chunk=128)
    torch.cuda.synchronize()
    for k in ("zone", "bin", "mirror", "score"):
        assert np.array_equal(res[k].cpu().numpy(), ref[k]), k


def test_concurrent_matches_on_two_streams(acom, multi):
    """The plan is read-only after acom_build_plan and launch settings belong to
    the calling host thread, so matches on two streams at once (interleaved
    from one thread, then from two threads, one of which changes its own
    launch settings meanwhile) give the sequential results bit for bit."""
    import threading
    d, opl, gpl = multi
    rng = np.random.default_rng(9)
    sets = []
    for k in range(2):
        ang = rng.uniform(-0.5, 0.5)
        qx = d["qx"] * np.cos(ang) - d["qy"] * np.sin(ang)
        qy = d["qx"] * np.sin(ang) + d["qy"] * np.cos(ang)
        sets.append(acom.Peaks(d["offsets"], qx, qy, d["I"]))
    ref = []
    for pk in sets:
        r = gpl.match(pk, 2, "bf16", 128)
        torch.cuda.synchronize()
        ref.append({k: v.clone() for k, v in r.items() if v is not None})
    keys = ("zone", "bin", "mirror", "score", "phi3", "orient", "n_evaluated")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ws = [torch.empty(gpl.match_workspace_bytes("bf16", 128), dtype=torch.uint8, device="cuda") for _ in range(2)]
    outs = [gpl.empty_matches(sets[0].n_patterns, 2, True, "cuda") for _ in range(2)]
    torch.cuda.synchronize()
    # one thread, two streams, launches interleaved
    for rep in range(3):
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                gpl.match(sets[k], 2, "bf16", 128, ws[k], out=outs[k])
        torch.cuda.synchronize()
        for k in range(2):
            for key in keys:
                assert torch.equal(outs[k][key], ref[k][key]), (rep, k, key)
    # two threads, each on its own stream
    errors = []

    def worker(k):
        try:
            if k == 1:
                acom.set_tuning(polar_cols=16, bound_tile=0)  # this thread's settings only
            for rep in range(4):
                with torch.cuda.stream(streams[k]):
                    gpl.match(sets[k], 2, "bf16", 128, ws[k], out=outs[k])
                streams[k].synchronize()
                for key in keys:
                    if not torch.equal(outs[k][key], ref[k][key]):
                        errors.append((k, rep, key))
        except Exception as e:  # reported below
            errors.append((k, repr(e)))

    th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors


def test_plan_above_16384_zones(acom):
    """A hexagonal 6/m wedge at 0.7 degree (16,900 zones): the exact pass keeps
    the pattern's bound row in the workspace instead of LDS.  Decisions match
    the plain-C FP64 direct sum, and equal those of the LDS path (forced by
    raising the limit) bit for bit; on the FCC plan the in-place path forced by
    a zero limit equals the default LDS path."""
    from oracle import directsum
    cfg = dict(k_max=1.6, n_radial=32, n_angular=90, zone_step_deg=0.7)
    opl = helpers.oracle_plan(["hcp"], **cfg)
    gpl = helpers.gpu_plan(["hcp"], precisions=("fp32", "bf16"), **cfg)
    assert gpl.n_zones == 16900 > 16384
    d = synth.subset(synth.make("hcp"), np.arange(0, 65536, 1024))
    pk = acom.Peaks.from_host(d)
    out = {}
    try:
        for lim in (16384, 32768):
            acom.set_tuning(exact_u_lds_max=lim)
            r = gpl.match(pk, top_k=4, precision="bf16")
            torch.cuda.synchronize()
            out[lim] = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    finally:
        acom.set_tuning(exact_u_lds_max=16384)
    for k in ("zone", "bin", "mirror", "score", "phi3", "n_evaluated"):
        assert np.array_equal(out[16384][k], out[32768][k]), k
    res = out[16384]
    zs = directsum.zone_scores(opl, d["offsets"], d["qx"], d["qy"], d["I"])
    for p in range(len(d["offsets"]) - 1):
        sc = zs["score"][p]
        mx = sc.max()
        z = int(res["zone"][p, 0])
        assert z >= 0 and sc[z] >= mx - 1e-5 * mx, (p, z)
        assert abs(res["score"][p, 0] - sc[z]) <= 1e-5 * mx
    # the in-place path on a plan whose rows would fit LDS
    d2, _, gpl2 = None, None, helpers.gpu_plan(["fcc"], precisions=("fp32",), **MULTI)
    pk2 = acom.Peaks.from_host(synth.multi(ny=8, nx=8, n_grains=6))
    try:
        a = gpl2.match(pk2, top_k=3, precision="fp32")
        acom.set_tuning(exact_u_lds_max=0)
        b = gpl2.match(pk2, top_k=3, precision="fp32")
        torch.cuda.synchronize()
    finally:
        acom.set_tuning(exact_u_lds_max=16384)
    for k in ("zone", "bin", "mirror", "score", "phi3", "n_evaluated"):
        assert torch.equal(a[k], b[k]), k


# launch orders: the exact pass's default grid (XCD runs of 1024 patterns), one
# range per XCD, runs of 3 and 100 (partial last groups), plain order, and the
# persistent workgroups on XCD-local queues; the polar pass XCD-grouped
LAUNCH_ORDERS = [dict(), dict(exact_xcd_block=0), dict(exact_xcd_block=3), dict(exact_xcd_block=100),
                 dict(exact_xcd=0), dict(exact_persist=1), dict(polar_xcd=1)]
DEFAULT_ORDER = dict(exact_persist=0, exact_xcd=1, exact_xcd_block=1024, polar_xcd=0)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_launch_orders_and_persistent_exact_pass_agree(acom, multi, precision):
    """Every launch order of the exact and polar passes gives the default
    launch's results bit for bit: on the three-phase plan, and on 20,000 scan patterns in
    chunks of 8,192 (a ragged last chunk; the persistent queues are reset per
    chunk by the polar pass)."""
    d, opl, gpl = multi
    cases = [(gpl, acom.Peaks.from_host(d), 0)]
    scan_plan = helpers.gpu_plan(["fcc"], precisions=("fp32", "bf16"), **helpers.SCAN)
    cases.append((scan_plan, acom.Peaks.from_host(synth.subset(synth.make("scan"), np.arange(20000) * 3)), 8192))
    for pl, pk, chunk in cases:
        out = []
        try:
            for tune in LAUNCH_ORDERS:
                acom.set_tuning(**tune)
                r = pl.match(pk, top_k=3, precision=precision, chunk=chunk)
                torch.cuda.synchronize()
                out.append({k: v.cpu().numpy() for k, v in r.items() if v is not None})
                acom.set_tuning(**DEFAULT_ORDER)
        finally:
            acom.set_tuning(**DEFAULT_ORDER)
        for tune, o in zip(LAUNCH_ORDERS[1:], out[1:]):
            for k in ("zone", "phase", "bin", "mirror", "score", "phi3", "orient", "n_evaluated"):
                assert np.array_equal(out[0][k], o[k]), (chunk, tune, k)
        assert (out[0]["zone"][:, 0] >= 0).mean() > 0.95
