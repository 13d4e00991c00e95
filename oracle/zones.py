"""Zone-axis grid and zone rotations (FP64).

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Methods > Generation of an Orientation Plan.  Three boundary vectors
delimit the symmetry-reduced set of zone axes; a 2-D grid spanning them is
built with spherical linear interpolation (Shoemake); the rotation taking the
beam axis z onto a zone axis is the inverse of the first two factors of the
Z-X-Z Euler product of Eq. rotation_matrices.
"""
import math
import numpy as np


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def _angle(u, v):
    return math.acos(max(-1.0, min(1.0, float(np.dot(u, v)))))


def slerp(p0, p1, t):
    """Spherical linear interpolation between unit vectors (Shoemake 1985)."""
    om = _angle(p0, p1)
    if om < 1e-12:
        return np.array(p0, dtype=np.float64)
    s = math.sin(om)
    return (math.sin((1.0 - t) * om) * p0 + math.sin(t * om) * p1) / s


def triangle_grid(v0, v1, v2, step_deg):
    """SLERP grid over the spherical triangle (v0, v1, v2).

    Reading (the paper gives the method, not the indexing): N = ceil(angle(v0,v1)
    / step - 1e-6) rows; row i holds a_i = slerp(v0,v1,i/N), b_i = slerp(v0,v2,i/N)
    and the i+1 points slerp(a_i, b_i, j/i), j = 0..i (row 0 is v0 alone).
    That gives (N+1)(N+2)/2 zone axes, corners included.
    """
    v0, v1, v2 = _unit(v0), _unit(v1), _unit(v2)
    N = max(1, int(math.ceil(math.degrees(_angle(v0, v1)) / step_deg - 1e-6)))
    pts = []
    for i in range(N + 1):
        a = slerp(v0, v1, i / N)
        b = slerp(v0, v2, i / N)
        if i == 0:
            pts.append(v0.copy())
            continue
        for j in range(i + 1):
            pts.append(slerp(a, b, j / i))
    return np.array(pts)


def zone_grid(triangles, step_deg, dedup_tol=1e-9):
    """Concatenate the grids of one or more triangles, dropping any point within
    dedup_tol of an earlier one (shared edges of adjacent triangles)."""
    out = np.zeros((0, 3))
    for tri in triangles:
        for p in triangle_grid(tri[0], tri[1], tri[2], step_deg):
            if len(out) == 0 or np.min(np.linalg.norm(out - p, axis=1)) > dedup_tol:
                out = np.vstack([out, p])
    return out


def Rz(phi):
    """Rotation about z as printed in Eq. rotation_matrices: [[C,-S,0],[S,C,0],[0,0,1]]."""
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def Rx_paper(theta):
    """Middle factor of Eq. rotation_matrices as printed: [[1,0,0],[0,C,S],[0,-S,C]]."""
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, s], [0.0, -s, c]])


def Ry_pi():
    """Rotation by pi about y: diag(-1, 1, -1) (used for the mirror branch)."""
    return np.diag([-1.0, 1.0, -1.0])


def zone_euler(w):
    """(phi1, theta2) with Rz(phi1) Rx_paper(theta2) z = w.

    From the printed matrices, Rz(phi1) Rx(theta2) z = (-S1 S2, C1 S2, C2), so
    theta2 = arccos(w_z), phi1 = atan2(-w_x, w_y); phi1 = 0 on the z axis.
    """
    w = _unit(w)
    th = math.acos(max(-1.0, min(1.0, w[2])))
    if math.hypot(w[0], w[1]) < 1e-12:
        ph = 0.0
    else:
        ph = math.atan2(-w[0], w[1])
    return ph, th


def zone_rotation(w):
    """M12 = Rz(phi1) Rx(theta2): the first two factors of Eq. rotation_matrices.

    Its inverse (transpose) rotates crystal vectors into the frame where the zone
    axis is the beam direction z (Generation of an Orientation Plan)."""
    ph, th = zone_euler(w)
    return Rz(ph) @ Rx_paper(th)


def cubic_triangle():
    """[001], [011], [111]: the fcc boundary vectors named in the paper."""
    return [np.array([0.0, 0.0, 1.0]), _unit([0.0, 1.0, 1.0]), _unit([1.0, 1.0, 1.0])]


def hex_wedge_triangles():
    """Two triangles z -> x(0 deg) -> 30 deg and z -> 60 deg -> 30 deg in the basal
    plane: a 6/m-style wedge (reading for the ~8,000-zone hexagonal plan)."""
    z = np.array([0.0, 0.0, 1.0])
    e0 = np.array([1.0, 0.0, 0.0])
    e30 = np.array([math.cos(math.radians(30)), math.sin(math.radians(30)), 0.0])
    e60 = np.array([math.cos(math.radians(60)), math.sin(math.radians(60)), 0.0])
    return [[z, e0, e30], [z, e60, e30]]


def fiber_grid(axis, theta_max_deg, step_deg, phi0_deg=0.0, phi1_deg=360.0):
    """Zone axes of a fiber-texture plan (Orientation plans of other types:
    fiber texture): directions within theta_max of the fiber axis f.

    Reading (the paper gives the idea, not the grid): rings of polar angle
    theta_i = i * step about f, i = 0 .. floor(theta_max / step); ring 0 is f;
    ring i has points spaced at most `step` of arc along it: over a full circle
    n_i = ceil(360 sin(theta_i) / step) points at phi0 + j 360 / n_i, over a
    wedge [phi0, phi1] n_i = ceil((phi1 - phi0) sin(theta_i) / step) equal
    intervals with both ends.  Azimuth 0 is unit(f x e), e the coordinate axis
    least aligned with f (ties to the lower index); 90 degrees is f x u.
    """
    f = np.asarray(axis, dtype=np.float64)
    f = f / np.linalg.norm(f)
    e = np.zeros(3)
    e[int(np.argmin(np.abs(f)))] = 1.0
    u = np.cross(f, e)
    u /= np.linalg.norm(u)
    v = np.cross(f, u)
    full = phi1_deg - phi0_deg >= 360.0 - 1e-9
    out = [f]
    for i in range(1, int(math.floor(theta_max_deg / step_deg + 1e-9)) + 1):
        th = math.radians(i * step_deg)
        if full:
            m = max(1, math.ceil(360.0 * math.sin(th) / step_deg - 1e-9))
            phis = [phi0_deg + j * 360.0 / m for j in range(m)]
        else:
            m = max(1, math.ceil((phi1_deg - phi0_deg) * math.sin(th) / step_deg - 1e-9))
            phis = [phi0_deg + j * (phi1_deg - phi0_deg) / m for j in range(m + 1)]
        for ph in phis:
            p = math.radians(ph)
            out.append(math.cos(th) * f + math.sin(th) * (math.cos(p) * u + math.sin(p) * v))
    return np.array(out)
