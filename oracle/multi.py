"""Matching of overlapping diffraction patterns (FP64).

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Methods > Matching of Overlapping Diffraction Patterns.  The procedure,
in the paper's order:
  1. find the best-fit orientation of the pattern with the correlation match;
  2. compute the forward diffraction pattern of that orientation
     (Methods > Calculation of Kinematical Diffraction Patterns, here
     kinematics.pattern: reflections above rel_cut of the largest |F|^2 after
     the Gaussian shape factor of the excitation error);
  3. remove every experimental peak within the deletion radius of a simulated
     peak; scale the intensity of a peak outside that radius but within the
     correlation kernel's reach by the linear factor
     (distance - deletion radius) / (kernel reach - deletion radius);
  4. repeat the match on the edited peaks until the requested number of
     orientations is found or none is found any more.
The score reported for each orientation is the value of the ORIGINAL pattern's
correlogram at that orientation's (zone, bin, branch), as the paper reports.

Readings (the paper leaves them open): the distance of a peak is to the
NEAREST simulated peak; "the correlation kernel size" is the kernel's reach
(delta for the cone kernel); the orientation simulated is the reported one,
with its parabolic sub-bin offset; a round whose match is empty or whose score
is not above zero (or is below a caller's threshold) ends the search.
"""
import numpy as np

from . import correlate, image, kinematics
from .plan import CONE, kernel_radius


def edit_intensities(qx, qy, I, sim_x, sim_y, r_del, r_k):
    """Step 3 for one pattern: the edited intensities (FP64)."""
    I = np.asarray(I, dtype=np.float64)
    if len(sim_x) == 0:
        return I.copy()
    dx = np.asarray(qx, dtype=np.float64)[:, None] - np.asarray(sim_x, dtype=np.float64)[None, :]
    dy = np.asarray(qy, dtype=np.float64)[:, None] - np.asarray(sim_y, dtype=np.float64)[None, :]
    d = np.sqrt(np.min(dx * dx + dy * dy, axis=1))
    f = np.where(d < r_del, 0.0, np.where(d < r_k, (d - r_del) / (r_k - r_del), 1.0))
    return I * f


def match_multi(plan, qx, qy, I, n_orient, r_del, rel_cut=0.01, min_score=0.0, sigma_exc=0.02):
    """Up to n_orient orientations of one pattern (list of dicts, None where a
    round found nothing; every round after the first None is None)."""
    prm = plan["params"]
    N = plan["P"].shape[1]
    r_k = kernel_radius(prm.delta, prm.kind, prm.sigma)
    X0 = image.polar_image(qx, qy, I, plan["q_s"], N, prm)
    C0, Cm0 = correlate.correlate_direct(plan["P"], X0)
    I_cur = np.asarray(I, dtype=np.float64).copy()
    out = []
    done = False
    for r in range(n_orient):
        if done:
            out.append(None)
            continue
        if r == 0:
            X, C, Cm = X0, C0, Cm0
        else:
            X = image.polar_image(qx, qy, I_cur, plan["q_s"], N, prm)
            C, Cm = correlate.correlate_direct(plan["P"], X)
        best = correlate.match(plan, X, top_k=1, C=C, Cm=Cm)[0][0]
        if best["zone"] < 0:
            done = True
            out.append(None)
            continue
        z, n, mi = best["zone"], best["n"], best["mirror"]
        score = float((Cm0 if mi else C0)[z, n])
        if not (score > 0.0 and score >= min_score):
            done = True
            out.append(None)
            continue
        out.append(dict(zone=z, phase=best["phase"], n=n, mirror=mi, score=score, orient=best["orient"],
                        edited_score=best["score"]))
        refl = plan["refl"][best["phase"]]
        sx, sy, _ = kinematics.pattern(refl, best["orient"], prm.k0, sigma=sigma_exc, rel_cut=rel_cut)
        I_cur = edit_intensities(qx, qy, I_cur, sx, sy, r_del, r_k)
    return out


def match_multi_c(plan, qx, qy, I, n_orient, r_del, rel_cut=0.01, min_score=0.0, sigma_exc=0.02, nthreads=0):
    """The same procedure with each round's full correlogram maximum taken by the
    plain-C direct sum (directsum.zone_scores: per zone, the best (n, branch);
    the best zone, ties to the smaller index) and the original pattern's value at
    the chosen (zone, bin, branch) by the numpy direct sum over that zone alone.
    For scan-sized plans, where the numpy correlogram of every zone is slow."""
    from . import directsum
    prm = plan["params"]
    N = plan["P"].shape[1]
    r_k = kernel_radius(prm.delta, prm.kind, prm.sigma)
    qx = np.asarray(qx, dtype=np.float64)
    qy = np.asarray(qy, dtype=np.float64)
    X0 = image.polar_image(qx, qy, I, plan["q_s"], N, prm)
    I_cur = np.asarray(I, dtype=np.float64).copy()
    off = np.array([0, len(qx)], dtype=np.int64)
    out = []
    done = False
    for r in range(n_orient):
        if done or not np.any(I_cur > 0.0):
            done = True
            out.append(None)
            continue
        zs = directsum.zone_scores(plan, off, qx, qy, I_cur, nthreads)
        sc = zs["score"][0]
        z = int(np.argmax(sc))
        if not (sc[z] > 0.0):
            done = True
            out.append(None)
            continue
        n, mi = int(zs["n"][0, z]), int(zs["mirror"][0, z])
        offp = correlate.parabolic_offset(zs["cm1"][0, z], sc[z], zs["cp1"][0, z])
        m = correlate.orientation(plan["M12"][z], n, offp, mi, N)
        Cz, Cmz = correlate.correlate_direct(plan["P"][z:z + 1], X0)
        score = float((Cmz if mi else Cz)[0, n])
        if not (score > 0.0 and score >= min_score):
            done = True
            out.append(None)
            continue
        out.append(dict(zone=z, phase=int(plan["zone_phase"][z]), n=n, mirror=mi, score=score, orient=m))
        refl = plan["refl"][int(plan["zone_phase"][z])]
        sx, sy, _ = kinematics.pattern(refl, m, prm.k0, sigma=sigma_exc, rel_cut=rel_cut)
        I_cur = edit_intensities(qx, qy, I_cur, sx, sy, r_del, r_k)
    return out
