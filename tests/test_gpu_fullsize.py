"""Full-size runs in the launch configuration the benchmark times (one chunk of
65,536 patterns per launch), each checked on sampled patterns against the FP64
oracle computed one pattern at a time:

  - the 256x256 HCP scan against the 8281-zone 6/m wedge plan, top-8 with
    BF16 and FP16 contractions and FP32 rescoring;
  - the 512x512 three-phase scan (262,144 patterns with 3-150 peaks) against
    the concatenated 10,443-zone plan, BF16 (oracle sample over the whole
    range of peak counts, three of them above 128 peaks);
  - 65,536 off-grid FCC patterns: top-4 grid candidates (FP32 and BF16
    contractions, FP32 rescoring) refined on the continuous score, against the
    oracle's refinement of the same candidates.

Tolerances: a reported zone's oracle score is within 1e-5 of the oracle's
maximum (ties between symmetry-equivalent zones are equal to FP32 rounding),
and the reported FP32 score equals the oracle's value there within 1e-5 of the
maximum; the refined winner is a candidate whose oracle-refined score is the
oracle's best within 1e-4 (twins can tie), and its orientation agrees with the
oracle's refinement of that candidate within 0.01 degree (the two ascents take
the same steps up to FP32 rounding of the gradient).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import crystal, directsum, metrics, score
from oracle import plan as oplan
from tests import helpers

pytestmark = pytest.mark.gpu

CHUNK = 65536


@pytest.fixture(scope="module")
def acom():
    from paper_2111_00171_amd import acom as a
    a.lib()
    return a


def _oracle_scores(opl, d, idx):
    sub = synth.subset(d, idx)
    return directsum.zone_scores(opl, sub["offsets"], sub["qx"], sub["qy"], sub["I"])


def _check_sampled(zs, res, idx, top):
    for i, p in enumerate(idx):
        sc = zs["score"][i]
        mx = sc.max()
        z = int(res["zone"][p, 0])
        assert z >= 0 and sc[z] >= mx - 1e-5 * mx, (p, z, sc[z], mx)
        assert abs(res["score"][p, 0] - sc[z]) <= 1e-5 * mx, (p, res["score"][p, 0], sc[z])
        if top > 1:  # the rest of the list: valid zones in non-increasing order of exact score
            s = res["score"][p]
            assert np.all(np.diff(s[s > 0]) <= 1e-6 * mx)


def test_hcp_full_size_sampled(acom):
    d = synth.make("hcp")
    opl = helpers.oracle_plan(["hcp"], **helpers.SCAN)
    gpl = helpers.gpu_plan(["hcp"], precisions=("fp32", "bf16", "fp16"), **helpers.SCAN)
    assert gpl.n_zones == 8281
    pk = acom.Peaks.from_host(d)
    idx = np.sort(np.random.default_rng(81).choice(len(d["offsets"]) - 1, 8, replace=False))
    zs = _oracle_scores(opl, d, idx)
    for prec in ("bf16", "fp16"):
        res = gpl.match(pk, top_k=8, precision=prec, chunk=CHUNK)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in res.items() if v is not None}
        assert np.all(res["zone"][:, 0] >= 0)
        _check_sampled(zs, res, idx, 8)


def test_multiphase_full_size_sampled(acom):
    d = synth.make("multi")
    assert len(d["offsets"]) - 1 == 262144
    opl = helpers.oracle_plan(["fcc", "bcc", "hcp"], **helpers.SCAN)
    gpl = helpers.gpu_plan(["fcc", "bcc", "hcp"], precisions=("fp32", "bf16"), **helpers.SCAN)
    assert gpl.n_zones == 10443
    res = gpl.match(acom.Peaks.from_host(d), top_k=1, precision="bf16", chunk=CHUNK)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in res.items() if v is not None}
    # sampled over the whole 3-150 range of peak counts, with three patterns
    # above 128 peaks (the polar pass's multi-batch path)
    cnt = np.diff(d["offsets"])
    rng = np.random.default_rng(82)
    idx = np.sort(np.concatenate([rng.choice(len(cnt), 6, replace=False),
                                  rng.choice(np.nonzero(cnt > 128)[0], 3, replace=False)]))
    assert (cnt[idx] > 128).sum() >= 3
    _check_sampled(_oracle_scores(opl, d, idx), res, idx, 1)
    for p in idx:
        assert res["phase"][p, 0] == opl["zone_phase"][res["zone"][p, 0]]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_refine_full_size_sampled(acom, precision):
    d = synth.make("refine")
    n = len(d["offsets"]) - 1
    gpl = helpers.gpu_plan(["fcc"], precisions=("fp32", "bf16"), **helpers.SCAN)
    pk = acom.Peaks.from_host(d)
    res = gpl.match(pk, top_k=4, precision=precision, chunk=CHUNK)
    init = res["orient"].reshape(n, 4, 9)
    m, S, cand = gpl.refine(pk, init, max_iter=64)
    torch.cuda.synchronize()
    m = m.cpu().numpy()
    S = S.cpu().numpy()
    cand = cand.cpu().numpy()
    init = init.cpu().numpy().reshape(n, 4, 3, 3)
    refl = crystal.reflections(np.eye(3) * helpers.A_FCC, helpers.FCC_FRAC, 2.0)
    prm = oplan.Params(k_max=2.0)
    G = metrics.cubic_rotations()
    o = d["offsets"]
    idx = np.random.default_rng(83).choice(n, 24 if precision == "fp32" else 12, replace=False)
    mis = []
    for p in idx:
        args = [d[k][o[p]:o[p + 1]].astype(np.float64) for k in ("qx", "qy", "I")]
        # the oracle refines every candidate; the GPU's winner must be one whose
        # refined score is the oracle's best up to FP32 resolution (candidates
        # of equal score, such as twins, are ties), and its orientation the
        # oracle's refinement of that same candidate
        ref = [score.refine_one(refl, *args, init[p, j], prm, max_iter=64)[:2] for j in range(4)]
        So = max(r[1] for r in ref)
        c = int(cand[p])
        assert ref[c][1] >= So - 1e-4 * abs(So), (p, c, [r[1] for r in ref])
        assert abs(S[p] - ref[c][1]) <= 1e-4 * abs(So) + 1e-6, (p, S[p], ref[c][1])
        # an end point as good as the oracle's (FP64 score within 1e-4 of its
        # end score), within where the two ascents stop
        Sg = score.score(refl, *args, m[p].astype(np.float64), np.zeros(3), prm)
        assert Sg >= ref[c][1] - 1e-4 * abs(So) - 1e-6, (p, Sg, ref[c][1])
        mis.append(metrics.misorientation_deg(m[p], ref[c][0], G))
    assert np.median(mis) <= 0.01 and max(mis) <= 0.05, mis
