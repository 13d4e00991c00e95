"""Bragg disk detection on raw diffraction frames by correlation template matching (FP64).

TEST INFRASTRUCTURE ONLY (see package docstring).

Paper: Methods > Correlation Pattern Matching (the peak list of each pattern
comes from template matching with the vacuum probe) and Methods > Software
Implementation (each frame is correlated with the image of the probe over
vacuum; disk positions are the correlation maxima and the correlation value at
a maximum is the peak's intensity).  The paper cites the detector and does not
spell it out, so every step below is a stated reading:

  template   the probe image circularly shifted so that its centre pixel
             (cy0, cx0) sits at the origin: t[u, v] = probe[(u+cy0) % H, (v+cx0) % W];
  correlate  circular cross-correlation C[y, x] = sum_{u,v} f[(y+u) % H, (x+v) % W] t[u, v]
             (a disk centred on (y0, x0) correlates most at (y0, x0));
  candidates pixels of the interior (at least `edge` pixels from every border,
             and not closer than `r_excl` to the optical axis (cy, cx)) whose
             C is strictly greater than all 8 neighbours;
  threshold  keep candidates with C > max(min_abs, min_rel * largest candidate C);
  spacing    greedy in order of decreasing C (equal C: lower raster index y*W+x
             first): a candidate is kept when no kept peak lies closer than
             `min_spacing` pixels; at most `max_peaks` are kept;
  sub-pixel  per axis, the vertex of the parabola through C at the peak and its
             two neighbours, dx = (C[x-1] - C[x+1]) / (2 (C[x-1] - 2 C[x] + C[x+1]));
  output     qx = (x + dx - cx) * pixel_size, qy = (y + dy - cy) * pixel_size,
             I = C[y, x], in the keep order.
"""
import numpy as np


def probe_template(probe, cy0, cx0):
    """The probe image with its centre pixel moved to the origin (circular shift)."""
    return np.roll(np.asarray(probe, np.float64), (-int(cy0), -int(cx0)), axis=(0, 1))


def correlate(frame, template):
    """Circular cross-correlation by its definition: a sum over the template's
    nonzero taps of the frame shifted by that tap (zero taps add nothing)."""
    f = np.asarray(frame, np.float64)
    t = np.asarray(template, np.float64)
    C = np.zeros_like(f)
    for u, v in zip(*np.nonzero(t)):
        C += t[u, v] * np.roll(f, (-u, -v), axis=(0, 1))     # f[(y+u) % H, (x+v) % W]
    return C


def interior_mask(H, W, edge, cy, cx, r_excl):
    y, x = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    m = (y >= edge) & (y < H - edge) & (x >= edge) & (x < W - edge)
    if r_excl > 0:
        m &= (y - cy) ** 2 + (x - cx) ** 2 >= r_excl * r_excl
    return m


def neighbour_max(C):
    """Largest of the 8 neighbours of every pixel (circular; only interior
    pixels, at least one pixel from the border, are ever used)."""
    nb = np.full_like(C, -np.inf)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                nb = np.maximum(nb, np.roll(C, (-dy, -dx), axis=(0, 1)))
    return nb


def select(C, edge, min_rel, min_abs, min_spacing, max_peaks, cy, cx, r_excl):
    """Candidates, threshold and greedy spacing on a correlation map.
    Returns the kept (y, x) in keep order and the threshold used."""
    H, W = C.shape
    if edge < 1:
        raise ValueError("edge must be at least 1")
    cand = interior_mask(H, W, edge, cy, cx, r_excl) & (C > neighbour_max(C))
    ys, xs = np.nonzero(cand)
    if len(ys) == 0:
        return [], max(min_abs, 0.0)
    vals = C[ys, xs]
    thr = max(min_abs, min_rel * float(vals.max()))
    order = sorted(range(len(ys)), key=lambda i: (-vals[i], ys[i] * W + xs[i]))
    kept = []
    s2 = min_spacing * min_spacing
    for i in order:
        if not (vals[i] > thr):
            break
        if all((ys[i] - y) ** 2 + (xs[i] - x) ** 2 >= s2 for y, x in kept):
            kept.append((int(ys[i]), int(xs[i])))
            if len(kept) == max_peaks:
                break
    return kept, thr


def parabolic_vertex(cm, c0, cp):
    """Vertex offset of the parabola through (-1, cm), (0, c0), (1, cp)."""
    return (cm - cp) / (2.0 * (cm - 2.0 * c0 + cp))


def detect(frame, template, *, edge=4, min_rel=0.005, min_abs=0.0, min_spacing=5, max_peaks=64,
           cy=64.0, cx=64.0, r_excl=0.0, pixel_size=1.0, C=None):
    """Peaks (qx, qy, I, y, x) of one frame, strongest first."""
    if C is None:
        C = correlate(frame, template)
    kept, _ = select(C, edge, min_rel, min_abs, min_spacing, max_peaks, cy, cx, r_excl)
    n = len(kept)
    qx, qy, I = np.zeros(n), np.zeros(n), np.zeros(n)
    ys, xs = np.zeros(n, np.int64), np.zeros(n, np.int64)
    for i, (y, x) in enumerate(kept):
        dx = parabolic_vertex(C[y, x - 1], C[y, x], C[y, x + 1])
        dy = parabolic_vertex(C[y - 1, x], C[y, x], C[y + 1, x])
        qx[i] = (x + dx - cx) * pixel_size
        qy[i] = (y + dy - cy) * pixel_size
        I[i] = C[y, x]
        ys[i], xs[i] = y, x
    return qx, qy, I, ys, xs


def decision_margin(C, edge, min_rel, min_abs, min_spacing, max_peaks, cy, cx, r_excl):
    """Smallest gap, relative to max |C|, between two values whose order decides
    the detected set: a near-threshold pixel's C against its largest neighbour
    and against the threshold, two candidates closer than min_spacing, and the
    last kept candidate against the next.  A second implementation in another
    precision can only disagree with this one on frames with a small margin."""
    H, W = C.shape
    scale = float(np.abs(C).max()) or 1.0
    inner = interior_mask(H, W, edge, cy, cx, r_excl)
    nb = neighbour_max(C)
    kept, thr = select(C, edge, min_rel, min_abs, min_spacing, max_peaks, cy, cx, r_excl)
    gaps = [np.inf]
    near = inner & (C > thr - 1e-3 * scale)
    if near.any():
        gaps.append(float(np.abs(C - nb)[near].min()))
    cand = inner & (C > nb)
    ys, xs = np.nonzero(cand)
    vals = C[ys, xs]
    if len(vals):
        gaps.append(float(np.abs(vals - thr).min()))
        strong = vals > thr - 1e-3 * scale
        ys, xs, vals = ys[strong], xs[strong], vals[strong]
        s2 = min_spacing * min_spacing
        for i in range(len(vals)):
            close = ((ys - ys[i]) ** 2 + (xs - xs[i]) ** 2 < s2)
            close[i] = False
            if close.any():
                gaps.append(float(np.abs(vals[close] - vals[i]).min()))
        if len(kept) == max_peaks:
            last = C[kept[-1]]
            ks = set(kept)
            rest = [v for y, x, v in zip(ys, xs, vals) if (int(y), int(x)) not in ks and v > thr]
            if rest:
                gaps.append(float(np.abs(np.asarray(rest) - last).min()))
    return min(gaps) / scale
