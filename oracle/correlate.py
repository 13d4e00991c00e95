"""Correlogram, mirror branch and the per-pattern decision (FP64).

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Methods > Correlation Pattern Matching.  The paper computes
C = sum_s IFFT{ FFT{P}^* FFT{X} } along phi3 and the mirror C_mirror with
FFT{X}^* (the mirror of the pattern), then takes, per zone, the maximum of C
and C_mirror and the highest value overall.  With the inverse FFT normalised by
1/N this is exactly the circular cross-correlation

    C[z, n]      = sum_s sum_a P[z, a, s] X[(a + n) mod N, s]
    C_mirror[z,n]= sum_s sum_a P[z, a, s] X[(-a - n) mod N, s]

so the oracle computes that plain definition as a direct sum (skipping cells
where X = 0, an identical sum).  `correlate_fft` is the paper's own FFT route,
kept as an independent second computation for the pins.

Readings (the paper is silent):
  * ties: the lexicographically smallest (zone, n, mirror) wins;
  * sub-bin refinement: a 3-point parabola through the cyclic neighbours of the
    winning bin in its own branch, offset clamped to [-1/2, 1/2], 0 if the
    parabola is not concave;
  * orientation of bin n (+ offset) in zone z: phi3 = -(n + offset) 2 pi / N,
    m = M12(w_z) Rz(phi3), times Ry(pi) on the right for the mirror branch;
  * several phases: the argmax over the concatenation of their plans.
"""
import math
import numpy as np

from .zones import Rz, Ry_pi


def correlate_direct(P, X, zchunk=32):
    """Direct sum over the nonzero cells of X.  P [Z, N, Nr], X [N, Nr] ->
    (C [Z, N], Cm [Z, N])."""
    P = np.asarray(P, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    Z, N, _ = P.shape
    b, s = np.nonzero(X)
    x = X[b, s]
    n = np.arange(N)
    idx = (b[None, :] - n[:, None]) % N           # [N, J]
    idxm = (-b[None, :] - n[:, None]) % N
    C = np.zeros((Z, N))
    Cm = np.zeros((Z, N))
    if len(x) == 0:
        return C, Cm
    for z0 in range(0, Z, zchunk):
        Pz = P[z0:z0 + zchunk]
        C[z0:z0 + zchunk] = Pz[:, idx, s[None, :]] @ x
        Cm[z0:z0 + zchunk] = Pz[:, idxm, s[None, :]] @ x
    return C, Cm


def correlate_fft(P, X):
    """The paper's FFT route: sum_s IFFT{FFT{P}^* FFT{X}} and the same with FFT{X}^*."""
    Ph = np.fft.fft(np.asarray(P, dtype=np.float64), axis=1)
    Xh = np.fft.fft(np.asarray(X, dtype=np.float64), axis=0)
    C = np.fft.ifft(np.conj(Ph) * Xh[None], axis=1).real.sum(axis=2)
    Cm = np.fft.ifft(np.conj(Ph) * np.conj(Xh)[None], axis=1).real.sum(axis=2)
    return C, Cm


def spectral_bound(P, X, exact_freqs=None, block=8):
    """U[z] >= max_n max(C, C_mirror)[z, n], an upper bound used to skip zones
    that cannot win.  Not a quantity of the paper.

    Over the half spectrum k = 0 .. N/2 (w_k = 1 at k = 0 and N/2, else 2, so
    the full spectrum is counted; |G_{N-k}| = |G_k| for real P and X):

      U[z] = (1/N) sum_k w_k T_k[z],
      T_k = max(|G_k|, |G'_k|)                        for k <  exact_freqs,
      T_k = sum_b ||Phat_{k,b}|| ||Xhat_{k,b}||       for k >= exact_freqs,

    with G_k = sum_s conj(Phat_ks) Xhat_ks, G'_k the same with conj(Xhat)
    (mirror), and b the blocks of `block` consecutive radii (the last one
    shorter when the radial count is not a multiple).  The first form is the
    triangle inequality on the inverse DFT of either branch with the larger
    modulus per frequency; the second bounds both moduli by Cauchy-Schwarz on
    each radial block.  exact_freqs = None (or >= N/2 + 1): every frequency
    takes the first form."""
    Ph = np.fft.rfft(np.asarray(P, dtype=np.float64), axis=1)    # [Z, Nk, R]
    Xh = np.fft.rfft(np.asarray(X, dtype=np.float64), axis=0)    # [Nk, R]
    N = np.asarray(P).shape[1]
    Nk = Ph.shape[1]
    w = np.full(Nk, 2.0)
    w[0] = 1.0
    if N % 2 == 0:
        w[-1] = 1.0
    kc = Nk if exact_freqs is None else min(int(exact_freqs), Nk)
    G = np.sum(np.conj(Ph[:, :kc]) * Xh[None, :kc], axis=2)
    Gm = np.sum(np.conj(Ph[:, :kc]) * np.conj(Xh)[None, :kc], axis=2)
    U = (w[:kc] * np.maximum(np.abs(G), np.abs(Gm))).sum(axis=1)
    if kc < Nk:
        R = Xh.shape[1]
        for b0 in range(0, R, block):
            xb = np.sqrt(np.sum(np.abs(Xh[kc:, b0:b0 + block]) ** 2, axis=1))          # [Nk - kc]
            pb = np.sqrt(np.sum(np.abs(Ph[:, kc:, b0:b0 + block]) ** 2, axis=2))     # [Z, Nk - kc]
            U += pb @ (w[kc:] * xb)
    return U / N


def zone_best(C, Cm):
    """Per zone: best value over (n, branch) and its (n, mirror), ties -> smallest
    n, then the non-mirror branch.  Returns (score[Z], n[Z], mirror[Z])."""
    both = np.stack([C, Cm], axis=2)              # [Z, N, 2]; flat index = 2 n + mirror
    Z, N, _ = both.shape
    flat = both.reshape(Z, 2 * N)
    arg = np.argmax(flat, axis=1)                 # numpy returns the first maximum
    return flat[np.arange(Z), arg], arg // 2, arg % 2


def rank_zones(score):
    """Zones in decreasing score, ties -> smaller zone index."""
    Z = len(score)
    return np.lexsort((np.arange(Z), -np.asarray(score)))


def parabolic_offset(cm1, c0, cp1):
    """Vertex of the parabola through (-1, cm1), (0, c0), (1, cp1), clamped to
    [-1/2, 1/2]; 0 when the curvature is not negative."""
    den = cm1 - 2.0 * c0 + cp1
    if not den < 0.0:
        return 0.0
    return float(min(0.5, max(-0.5, 0.5 * (cm1 - cp1) / den)))


def orientation(M12, n, offset, mirror, N):
    """Orientation matrix m (sample -> crystal) of bin n + offset in a zone."""
    phi3 = -(n + offset) * 2.0 * math.pi / N
    m = M12 @ Rz(phi3)
    if mirror:
        m = m @ Ry_pi()
    return m


def match(plan, X, top_k=1, C=None, Cm=None):
    """Full decision for one pattern: top_k distinct zones with (zone, phase, n,
    mirror, score, offset, phi3, orientation).  Zero image -> zone -1."""
    P = plan["P"]
    N = P.shape[1]
    if C is None:
        C, Cm = correlate_direct(P, X)
    out = []
    if not np.any(np.asarray(X) != 0):
        return [dict(zone=-1, phase=-1, n=0, mirror=0, score=0.0, offset=0.0, phi3=0.0,
                     orient=np.zeros((3, 3)))], C, Cm
    score, nb, mb = zone_best(C, Cm)
    order = rank_zones(score)
    for z in order[:top_k]:
        n, mi = int(nb[z]), int(mb[z])
        br = Cm if mi else C
        off = parabolic_offset(br[z, (n - 1) % N], br[z, n], br[z, (n + 1) % N])
        out.append(dict(zone=int(z), phase=int(plan["zone_phase"][z]), n=n, mirror=mi,
                        score=float(score[z]), offset=off,
                        phi3=-(n + off) * 2.0 * math.pi / N,
                        orient=orientation(plan["M12"][z], n, off, mi, N)))
    return out, C, Cm


def tie_set(C, Cm, rel=1e-9, abs_tol=0.0):
    """All (zone, n, mirror) whose value is within rel*|max| + abs_tol of the maximum."""
    both = np.stack([C, Cm], axis=2)
    mx = both.max()
    z, n, m = np.nonzero(both >= mx - rel * abs(mx) - abs_tol)
    return set(zip(z.tolist(), n.tolist(), m.tolist()))
