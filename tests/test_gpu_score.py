"""Continuous score, hand-written backward and refinement on the GPU against the
FP64 oracle (oracle/score.py, itself pinned to finite differences at 1e-6).

Tolerances, from the arithmetic:
  * S is a normalised sum of a few thousand FP32 products of exponentials:
    1e-4 relative (FP32 emulation of the kernel's arithmetic: ~1e-6);
  * dS/dtheta against the oracle's analytic gradient, and against central
    differences of the oracle's FP64 score (h = 1e-6 rad, truncation and
    rounding both below 1e-8 of the gradient): every component within 1e-4 of
    the gradient's norm, at orientations 0.3-0.6 degree off the optimum.  An
    FP32 emulation of the kernel's operations gives 1.4e-5 at worst (1.5e-6
    median) on this set: the rounding of g, m^T g and the excitation error
    propagate through d v / d s ~ s / sigma_e^2;
  * dS/dq (per peak) within 1e-4 of the largest peak-gradient component;
  * finite differences of the GPU's own FP32 score (Richardson, h = 2e-3 rad)
    carry the FP32 rounding noise of S divided by h (~1e-4 of the gradient):
    checked at 1e-3 as a second, independent check.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import crystal, metrics, score
from oracle import plan as oplan
from tests import helpers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2111_00171_amd import acom
    refl = crystal.reflections(np.eye(3) * helpers.A_FCC, helpers.FCC_FRAC, 2.0)
    prm = oplan.Params(k_max=2.0)
    gpl = acom.Plan([acom.fcc(zones=[[0, 0, 1.0]])],
                    acom.PlanParams(k_max=2.0, n_radial=32, n_angular=90, precisions=["fp32"]))
    d = synth.refine(n=96)
    rng = np.random.default_rng(31)
    base = np.stack([m @ score.expm_so3(np.radians(0.5) * v / np.linalg.norm(v))
                     for m, v in zip(d["truth"], rng.normal(size=(96, 3)))])
    theta = np.radians(0.3) * rng.normal(size=(96, 3))
    return acom, refl, prm, gpl, d, base, theta


def _peaks(d, p):
    o = d["offsets"]
    return (np.asarray(d["qx"][o[p]:o[p + 1]], np.float64), np.asarray(d["qy"][o[p]:o[p + 1]], np.float64),
            np.asarray(d["I"][o[p]:o[p + 1]], np.float64))


def test_score_and_gradients_match_oracle(setup):
    acom, refl, prm, gpl, d, base, theta = setup
    pk = acom.Peaks.from_host(d)
    b = torch.tensor(base.reshape(-1, 9), dtype=torch.float32, device="cuda")
    th = torch.tensor(theta, dtype=torch.float32, device="cuda")
    S = gpl.score(pk, b, th).cpu().numpy()
    dth, dqx, dqy = gpl.score_grad(pk, b, th, peak_grads=True)
    dth, dqx, dqy = dth.cpu().numpy(), dqx.cpu().numpy(), dqy.cpu().numpy()
    o = d["offsets"]
    worst = (0.0, 0.0)
    for p in range(0, 96, 4):
        qx, qy, I = _peaks(d, p)
        So, go, gxo, gyo = score.score_grad(refl, qx, qy, I, base[p], theta[p], prm)
        assert abs(S[p] - So) <= 1e-4 * abs(So)
        e_th = np.abs(dth[p] - go).max() / np.linalg.norm(go)
        gq = np.concatenate([gxo, gyo])
        e_q = max(np.abs(dqx[o[p]:o[p + 1]] - gxo).max(), np.abs(dqy[o[p]:o[p + 1]] - gyo).max()) / np.abs(gq).max()
        worst = (max(worst[0], e_th), max(worst[1], e_q))
        assert e_th <= 1e-4, (p, e_th)
        assert e_q <= 1e-4, (p, e_q)
    print(f"gradient vs oracle: theta {worst[0]:.2e}, peaks {worst[1]:.2e} (relative)")


def test_gradient_against_finite_differences(setup):
    """Richardson-extrapolated central differences (O(h^4) truncation) of the
    FP32 score; h = 2e-3 rad keeps the rounding term eps * S / h near 1e-4 of the
    gradient norm, while the plain central difference at that step would carry a
    truncation error of ~1e-3 (tilts move s_g by |g| h against sigma_e = 0.02)."""
    acom, refl, prm, gpl, d, base, theta = setup
    pk = acom.Peaks.from_host(d)
    b = torch.tensor(base.reshape(-1, 9), dtype=torch.float32, device="cuda")
    th = torch.tensor(theta, dtype=torch.float32, device="cuda")
    g, _, _ = gpl.score_grad(pk, b, th)
    g = g.cpu().numpy()

    def central(h):
        out = np.zeros_like(g)
        for j in range(3):
            e = torch.zeros_like(th)
            e[:, j] = h
            out[:, j] = ((gpl.score(pk, b, th + e).double() - gpl.score(pk, b, th - e).double()) / (2 * h)).cpu().numpy()
        return out

    h = 2e-3
    fd = (4.0 * central(h / 2) - central(h)) / 3.0
    nrm = np.linalg.norm(g, axis=1)
    rel = np.abs(fd - g).max(axis=1) / nrm
    print("fd check: max relative error", rel.max(), "median", np.median(rel))
    assert np.all(rel <= 1e-3)


def test_gradient_against_oracle_finite_differences(setup):
    """The GPU's dS/dtheta against central differences of the oracle's FP64
    score (h = 1e-6 rad): within 1e-4 of the gradient's norm."""
    acom, refl, prm, gpl, d, base, theta = setup
    pk = acom.Peaks.from_host(d)
    b = torch.tensor(base.reshape(-1, 9), dtype=torch.float32, device="cuda")
    th = torch.tensor(theta, dtype=torch.float32, device="cuda")
    g, _, _ = gpl.score_grad(pk, b, th)
    g = g.cpu().numpy()
    bf = b.cpu().numpy().astype(np.float64).reshape(-1, 3, 3)
    tf = th.cpu().numpy().astype(np.float64)
    h = 1e-6
    worst = 0.0
    for p in range(1, 96, 6):
        qx, qy, I = _peaks(d, p)
        fd = np.zeros(3)
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            fd[j] = (score.score(refl, qx, qy, I, bf[p], tf[p] + e, prm)
                     - score.score(refl, qx, qy, I, bf[p], tf[p] - e, prm)) / (2 * h)
        rel = np.abs(g[p] - fd).max() / np.linalg.norm(fd)
        worst = max(worst, rel)
        assert rel <= 1e-4, (p, rel)
    print(f"gradient vs FP64 finite differences: {worst:.2e} (relative)")


def test_autograd_function(setup):
    """ContinuousScore differentiates S with respect to theta and the peak
    positions; its backward equals acom_score_grad with the upstream weights."""
    acom, refl, prm, gpl, d, base, theta = setup
    pk = acom.Peaks.from_host(d)
    b = torch.tensor(base.reshape(-1, 9), dtype=torch.float32, device="cuda")
    th = torch.tensor(theta, dtype=torch.float32, device="cuda", requires_grad=True)
    qx = pk.qx.clone().requires_grad_(True)
    qy = pk.qy.clone().requires_grad_(True)
    S = acom.ContinuousScore.apply(th, qx, qy, gpl, pk, b)
    w = torch.linspace(0.5, 1.5, S.numel(), device="cuda")
    (S * w).sum().backward()
    g, gx, gy = gpl.score_grad(pk, b, th.detach(), dS=w.contiguous(), peak_grads=True)
    assert torch.allclose(th.grad, g, rtol=1e-6, atol=1e-6)
    assert torch.equal(qx.grad, gx) and torch.equal(qy.grad, gy)
    # moved peaks: the Function scores the positions it is given
    qx2 = (pk.qx + 0.01).requires_grad_(True)
    S2 = acom.ContinuousScore.apply(th.detach(), qx2, pk.qy, gpl, pk, b)
    moved = acom.Peaks(pk.offsets, pk.qx + 0.01, pk.qy, pk.intensity)
    assert torch.equal(S2, gpl.score(moved, b, th.detach()))
    S2.sum().backward()
    _, gx2, _ = gpl.score_grad(moved, b, th.detach(), peak_grads=True)
    assert torch.equal(qx2.grad, gx2)
    # the peak gradient agrees with the oracle's (pattern 0, every peak)
    o = d["offsets"]
    qx0, qy0, I0 = _peaks(d, 0)
    _, _, gxo, gyo = score.score_grad(refl, qx0, qy0, I0, base[0], theta[0], prm)
    gq = np.abs(np.concatenate([gxo, gyo])).max()
    assert np.abs(qx.grad[o[0]:o[1]].cpu().numpy() / 0.5 - gxo).max() <= 1e-4 * gq
    assert np.abs(qy.grad[o[0]:o[1]].cpu().numpy() / 0.5 - gyo).max() <= 1e-4 * gq


def test_refinement_matches_oracle_and_truth(setup):
    acom, refl, prm, gpl, d, base, theta = setup
    pk = acom.Peaks.from_host(d)
    rng = np.random.default_rng(5)
    far = synth.haar_rotations(rng, 96)
    cands = np.stack([base, far], axis=1)            # the right basin first, a wrong one second
    init = torch.tensor(cands.reshape(96, 2, 9), dtype=torch.float32, device="cuda")
    work = torch.zeros(96, 2, dtype=torch.int32, device="cuda")
    m, S, c = gpl.refine(pk, init, max_iter=64, work=work)
    m, S, c = m.cpu().numpy(), S.cpu().numpy(), c.cpu().numpy()
    # the work counts: every pattern evaluated its candidates with the gradient
    # at least once, and took trial steps (pairs = peaks x kept reflections)
    w = work.cpu().numpy()
    npk = np.diff(d["offsets"])
    assert np.all(w[:, 1] >= 2 * npk) and np.all(w[:, 0] > 0)
    G = metrics.cubic_rotations()
    mis_truth, mis_oracle = [], []
    for p in range(96):
        mis_truth.append(metrics.misorientation_deg(m[p], d["truth"][p], G))
    for p in range(0, 96, 8):
        qx, qy, I = _peaks(d, p)
        mo, So = score.refine(refl, qx, qy, I, list(cands[p]), prm, max_iter=64)
        mis_oracle.append(metrics.misorientation_deg(m[p], mo, G))
        assert abs(S[p] - So) <= 1e-3 * abs(So)
    assert np.all(c == 0)
    assert np.median(mis_oracle) <= 0.01 and max(mis_oracle) <= 0.05
    assert np.percentile(mis_truth, 90) <= 0.1


@pytest.mark.parametrize("phase_name,ph", [("bcc_a2.87", 1), ("hcp_a2.95_c4.68", 2)])
def test_refinement_on_other_phases(phase_name, ph):
    """Refinement with per-candidate phases on a three-phase plan (FCC, BCC,
    HCP): off-grid BCC or HCP patterns, candidates (the right phase near the
    truth, the FCC phase at the same matrix, the right phase far away), each
    refined on its own phase's reflections; the GPU's winner and score equal
    the oracle's refinement of the same candidates."""
    from paper_2111_00171_amd import acom
    lat = {"bcc_a2.87": (np.eye(3) * 2.87, helpers.BCC_FRAC), "hcp_a2.95_c4.68": (np.array(helpers.HCP_LAT), helpers.HCP_FRAC)}
    refls = [crystal.reflections(np.eye(3) * helpers.A_FCC, helpers.FCC_FRAC, 2.0),
             crystal.reflections(np.eye(3) * 2.87, helpers.BCC_FRAC, 2.0),
             crystal.reflections(np.array(helpers.HCP_LAT), helpers.HCP_FRAC, 2.0)]
    prm = oplan.Params(k_max=2.0)
    gpl = acom.Plan([acom.fcc(zones=[[0, 0, 1.0]]), acom.bcc(zones=[[0, 0, 1.0]]), acom.hcp(zones=[[0, 0, 1.0]])],
                    acom.PlanParams(k_max=2.0, n_radial=32, n_angular=90, precisions=["fp32"]))
    n = 48
    d = synth.refine(seed=1105 + ph, n=n, phase_name=phase_name)
    rng = np.random.default_rng(ph)
    near = np.stack([m @ score.expm_so3(np.radians(0.4) * v / np.linalg.norm(v))
                     for m, v in zip(d["truth"], rng.normal(size=(n, 3)))])
    far = synth.haar_rotations(rng, n)
    cands = np.stack([near, near, far], axis=1)
    cph = np.tile(np.array([ph, 0, ph], np.int32), (n, 1))
    pk = acom.Peaks.from_host(d)
    init = torch.tensor(cands.reshape(n, 3, 9), dtype=torch.float32, device="cuda")
    m, S, c = gpl.refine(pk, init, cand_phase=torch.tensor(cph, device="cuda"), max_iter=64)
    m, S, c = m.cpu().numpy(), S.cpu().numpy(), c.cpu().numpy()
    G = metrics.cubic_rotations() if ph == 1 else metrics.hexagonal_rotations()
    c32 = init.cpu().numpy().astype(np.float64).reshape(n, 3, 3, 3)
    mis_oracle = []
    for p in range(0, n, 4):
        qx, qy, I = _peaks(d, p)
        # the GPU's winner: a candidate of the oracle's best refined score up to
        # FP32 resolution, ending where the oracle's refinement of that candidate
        # ends, up to where either ascent stops (the FP64 score at the GPU's end
        # point is the oracle's end score up to 1e-4)
        allr = [score.refine_one(refls[cph[p, j]], qx, qy, I, c32[p, j], prm, max_iter=64) for j in range(3)]
        jb = int(np.argmax([r[1] for r in allr]))
        best = (allr[jb][0], allr[jb][1], jb)
        cj = int(c[p])
        assert allr[cj][1] >= best[1] - 1e-4 * abs(best[1]), (p, cj, best[2])
        assert abs(S[p] - allr[cj][1]) <= 1e-4 * abs(best[1]), (p, S[p], allr[cj][1])
        Sg = score.score(refls[cph[p, cj]], qx, qy, I, m[p].astype(np.float64), np.zeros(3), prm)
        assert Sg >= allr[cj][1] - 1e-4 * abs(best[1]), (p, Sg, allr[cj][1])
        mis_oracle.append(metrics.misorientation_deg(m[p], allr[cj][0], G))
    assert np.median(mis_oracle) <= 0.01 and max(mis_oracle) <= 0.05, mis_oracle
    assert np.mean(c == 0) > 0.8
    mis = [metrics.misorientation_deg(m[p], d["truth"][p], G) for p in range(n)]
    assert np.median(mis) < 0.1


def test_reflection_cap_is_an_error():
    """With omega = 0 every reflection takes part; FCC up to k_max = 3 has
    more than the 1024 the kernels hold, so the score is NaN and refinement
    reports the pattern as an error (candidate -2), never a truncated sum."""
    from paper_2111_00171_amd import acom
    assert len(crystal.reflections(np.eye(3) * helpers.A_FCC, helpers.FCC_FRAC, 3.0)["q"]) > 1024
    gpl = acom.Plan([acom.fcc(zones=[[0, 0, 1.0]])],
                    acom.PlanParams(k_max=3.0, n_radial=32, n_angular=90, omega=0.0, precisions=["fp32"]))
    d = synth.subset(synth.refine(n=8), np.arange(8))
    pk = acom.Peaks.from_host(d)
    b = torch.tensor(d["truth"].reshape(-1, 9), dtype=torch.float32, device="cuda")
    th = torch.zeros(8, 3, dtype=torch.float32, device="cuda")
    S = gpl.score(pk, b, th)
    dth, dqx, _ = gpl.score_grad(pk, b, th, peak_grads=True)
    assert torch.isnan(S).all() and torch.isnan(dth).all() and torch.isnan(dqx).all()
    m, Sr, c = gpl.refine(pk, b.reshape(8, 1, 9), max_iter=8)
    assert torch.isnan(Sr).all() and (c == -2).all()
