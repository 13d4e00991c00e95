"""Matching of overlapping diffraction patterns (acom_match_multi) against the
FP64 oracle (oracle/multi.py), through the C ABI.

Each round depends on the previous rounds' orientations, which FP32 and FP64
may pick differently among exact ties (symmetry-equivalent zones give the same
forward pattern, but not bit for bit).  So the check replays the oracle on the
GPU's own decisions: for every pattern and round, the oracle edits the peaks
with the GPU's previous orientations (FP32 matrices taken to FP64), and then
  - the GPU's (zone, bin, branch) must lie in the oracle's tie set of the
    edited pattern's correlogram (1e-5 of its maximum: FP32 resolution);
  - the GPU's score must equal the ORIGINAL pattern's correlogram at that
    (zone, bin, branch) within 1e-5 of the original maximum;
  - a round the GPU reports empty must be one where the oracle finds nothing
    (every peak deleted) or only a non-positive original value.
The edit itself is continuous in the distance (0 at the deletion radius, 1 at
the kernel reach), so FP32 positions change it only by rounding.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import correlate, image, kinematics, multi
from tests import helpers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def acom():
    from paper_2111_00171_amd import acom as a
    a.lib()
    return a


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_match_multi_replayed_by_oracle(acom, precision):
    d = synth.make("overlap", n=48, k_max=1.2)
    opl = helpers.oracle_plan(["fcc"], **helpers.SMALL)
    gpl = helpers.gpu_plan(["fcc"], **helpers.SMALL)
    pk = acom.Peaks.from_host(d)
    r_del, n_orient = 0.04, 3
    res = gpl.match_multi(pk, n_orient=n_orient, deletion_radius=r_del, precision=precision, chunk=32)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in res.items() if v is not None}
    prm = opl["params"]
    N = prm.n_angular
    o = d["offsets"]
    rounds_found = 0
    for p in range(len(o) - 1):
        qx = d["qx"][o[p]:o[p + 1]].astype(np.float64)
        qy = d["qy"][o[p]:o[p + 1]].astype(np.float64)
        I = d["I"][o[p]:o[p + 1]].astype(np.float64)
        X0 = image.polar_image(qx, qy, I, opl["q_s"], N, prm)
        C0, Cm0 = correlate.correlate_direct(opl["P"], X0)
        mx0 = max(C0.max(), Cm0.max())
        ended = False
        for r in range(n_orient):
            z = int(res["zone"][p, r])
            if ended:
                assert z == -1, (p, r)
                continue
            X = image.polar_image(qx, qy, I, opl["q_s"], N, prm)
            if not np.any(X != 0):
                assert z == -1, (p, r)
                ended = True
                continue
            C, Cm = correlate.correlate_direct(opl["P"], X)
            both = np.stack([C, Cm], axis=2)
            mx = both.max()
            if z < 0:
                # the GPU found nothing: the oracle's best has no positive original value
                zo, no, mo = np.unravel_index(np.argmax(both), both.shape)
                assert (Cm0 if mo else C0)[zo, no] <= 1e-5 * mx0, (p, r)
                ended = True
                continue
            n, m = int(res["bin"][p, r]), int(res["mirror"][p, r])
            assert both[z, n, m] >= mx - 1e-5 * mx, (p, r, z, n, m)
            assert abs(res["score"][p, r] - (Cm0 if m else C0)[z, n]) <= 1e-5 * mx0, (p, r)
            rounds_found += 1
            sx, sy, _ = kinematics.pattern(opl["refl"][0], res["orient"][p, r].astype(np.float64), prm.k0,
                                           rel_cut=0.01)
            I = multi.edit_intensities(qx, qy, I, sx, sy, r_del, prm.delta)
    assert rounds_found >= 2 * (len(o) - 1)


def test_match_multi_round_zero_is_match(acom):
    """Round 0 of acom_match_multi is acom_match's top-1 (the same kernels on the
    same peaks), bit for bit; invalid arguments are rejected."""
    d = synth.make("overlap", n=40, k_max=1.2)
    gpl = helpers.gpu_plan(["fcc"], **helpers.SMALL)
    pk = acom.Peaks.from_host(d)
    one = gpl.match(pk, top_k=1, precision="fp32")
    mm = gpl.match_multi(pk, n_orient=2, deletion_radius=0.04, precision="fp32")
    torch.cuda.synchronize()
    for k in ("zone", "bin", "mirror", "score", "phi3"):
        assert torch.equal(mm[k][:, 0], one[k][:, 0]), k
    with pytest.raises(acom.AcomError):
        gpl.match_multi(pk, n_orient=0)
    with pytest.raises(acom.AcomError):
        gpl.match_multi(pk, deletion_radius=0.08)  # not below the kernel reach (delta)
    with pytest.raises(acom.AcomError):
        gpl.match_multi(pk, rel_cut=0.0)
