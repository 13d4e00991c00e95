"""Orientation error metrics (FP64).

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Results (mean zone-axis misorientation for kinematical and dynamical
tests).  Misorientation of two orientations is the smallest rotation angle
between them over the proper rotations of the crystal's point group; the zone
axis error is the smallest angle between the zone axes over the Laue group
(proper rotations and their negatives).
"""
import itertools
import math
import numpy as np


def cubic_rotations():
    """The 24 proper rotations of 432: signed permutation matrices with det +1."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([-1.0, 1.0], repeat=3):
            M = np.zeros((3, 3))
            for i in range(3):
                M[i, perm[i]] = signs[i]
            if np.linalg.det(M) > 0:
                out.append(M)
    return out


def hexagonal_rotations():
    """The 12 proper rotations of 622 (6-fold axis z, 2-fold axes in the basal plane
    every 30 degrees starting at x)."""
    out = []
    for k in range(6):
        a = k * math.pi / 3.0
        c, s = math.cos(a), math.sin(a)
        out.append(np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]]))
    for k in range(6):
        a = k * math.pi / 6.0
        c2, s2 = math.cos(2 * a), math.sin(2 * a)
        out.append(np.array([[c2, s2, 0.0], [s2, -c2, 0.0], [0.0, 0.0, -1.0]]))
    return out


def rotation_angle(R):
    """Angle of rotation R from both its cosine (trace) and its sine (the
    antisymmetric part): well conditioned at every angle, so FP32 matrices a
    few units of rounding from orthogonal read as a few 1e-7 rad, where the
    arccos of the trace alone would read their rounding as ~3e-4 rad."""
    R = np.asarray(R, np.float64)
    s = 0.5 * math.sqrt((R[2, 1] - R[1, 2]) ** 2 + (R[0, 2] - R[2, 0]) ** 2 + (R[1, 0] - R[0, 1]) ** 2)
    c = 0.5 * (float(np.trace(R)) - 1.0)
    return math.atan2(s, c)


def misorientation_deg(m1, m2, group):
    """min over S in group of angle(m1^T S m2), degrees."""
    m1 = np.asarray(m1, np.float64)
    m2 = np.asarray(m2, np.float64)
    return math.degrees(min(rotation_angle(m1.T @ S @ m2) for S in group))


def zone_axis_error_deg(m1, m2, group):
    """Angle between zone axes w = m z over the Laue group (S and -S)."""
    w1 = np.asarray(m1, np.float64)[:, 2]
    w2 = np.asarray(m2, np.float64)[:, 2]
    best = math.pi
    for S in group:
        for sg in (1.0, -1.0):
            c = float(np.dot(w1, sg * (S @ w2)))
            best = min(best, math.acos(max(-1.0, min(1.0, c))))
    return math.degrees(best)
