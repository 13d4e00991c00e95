"""Python binding of libacom (the C ABI declared in include/acom.h).

Argument marshalling only: every step of the matching path runs in the HIP
kernels of libacom.so.  PyTorch supplies device memory and the current stream.
If the library has not been built, `lib()` raises: there is no fallback.
"""
import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libacom.so")

FP32, BF16, FP16 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16}
CONE, GAUSS = 0, 1
UNIFORM, SHELLS = 0, 1

c_int32, c_int64, c_double, c_void_p, c_size_t = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
P = ctypes.POINTER


class _Phase(ctypes.Structure):
    _fields_ = [("lattice", c_double * 9), ("n_atoms", c_int32), ("frac_xyz", P(c_double)),
                ("species", P(c_int32)), ("n_f", c_int32), ("f_q", P(c_double)), ("f_tab", P(c_double)),
                ("n_triangles", c_int32), ("triangles", c_double * 18), ("n_zones_explicit", c_int32),
                ("zones_explicit", P(c_double))]


class _Params(ctypes.Structure):
    _fields_ = [("k_max", c_double), ("delta", c_double), ("gamma", c_double), ("omega", c_double),
                ("accel_kV", c_double), ("zone_step_deg", c_double), ("gauss_sigma", c_double),
                ("sigma_exc", c_double), ("n_radial", c_int32), ("n_angular", c_int32), ("radial", c_int32),
                ("kernel", c_int32), ("precisions", c_int32), ("keep_f64", c_int32),
                ("bound_exact_freqs", c_int32), ("bound_block_radii", c_int32),
                ("bound_exact_freqs_16bit", c_int32)]


class _Peaks(ctypes.Structure):
    _fields_ = [("n_patterns", c_int64), ("total_peaks", c_int64), ("offsets", c_void_p), ("qx", c_void_p),
                ("qy", c_void_p), ("intensity", c_void_p)]


class _Matches(ctypes.Structure):
    _fields_ = [("zone", c_void_p), ("phase", c_void_p), ("bin", c_void_p), ("mirror", c_void_p),
                ("score", c_void_p), ("phi3", c_void_p), ("orient", c_void_p), ("n_evaluated", c_void_p)]


class _DiskParams(ctypes.Structure):
    _fields_ = [("size", c_int32), ("edge", c_int32), ("min_rel", ctypes.c_float), ("min_abs", ctypes.c_float),
                ("min_spacing", c_int32), ("max_peaks", c_int32), ("center_y", ctypes.c_float),
                ("center_x", ctypes.c_float), ("exclusion_radius", ctypes.c_float), ("pixel_size", ctypes.c_float)]


_lib = None


def lib():
    """The loaded libacom.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libacom.so not found at {LIB_PATH}: run `python -m paper_2111_00171_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        sig = {
            "acom_build_plan": [P(_Phase), c_int32, P(_Params), c_void_p, P(c_void_p)],
            "acom_plan_info": [c_void_p, P(c_int32), P(c_int32), P(c_int32), P(c_int32), P(c_double), P(c_double),
                               P(c_int32), P(c_double)],
            "acom_plan_copy_f64": [c_void_p, P(c_double)],
            "acom_plan_bound_split": [c_void_p, c_int32, P(c_int32), P(c_int32)],
            "acom_plan_destroy": [c_void_p],
            "acom_match_workspace_size": [c_void_p, c_int32, c_int32, P(c_size_t)],
            "acom_match": [c_void_p, P(_Peaks), c_int32, c_int32, c_int32, c_void_p, c_size_t, P(_Matches), c_void_p],
            "acom_match_noalloc": [c_void_p, P(_Peaks), c_int32, c_int32, P(_Matches), c_void_p],
            "acom_match_noalloc_chunk": [c_void_p, c_int32, P(c_int32)],
            "acom_match_multi_workspace_size": [c_void_p, c_int32, c_int32, c_int64, P(c_size_t)],
            "acom_fiber_zones": [P(c_double), c_double, c_double, c_double, c_double, c_void_p, c_int32, P(c_int32)],
            "acom_simulate_count": [c_void_p, c_int64, c_void_p, c_void_p, ctypes.c_float, c_void_p, c_void_p,
                                    c_void_p],
            "acom_simulate_fill": [c_void_p, c_int64, c_void_p, c_void_p, ctypes.c_float, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p],
            "acom_match_multi": [c_void_p, P(_Peaks), c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float, c_int32,
                                 c_int32, c_void_p, c_size_t, P(_Matches), c_void_p],
            "acom_autotune": [c_void_p, P(_Peaks), c_int32, c_int32, c_void_p, c_size_t, c_void_p, P(c_int32),
                              P(ctypes.c_float)],
            "acom_debug_workspace_size": [c_void_p, c_int64, P(c_size_t)],
            "acom_polar_image": [c_void_p, P(_Peaks), c_void_p, c_void_p, c_size_t, c_void_p],
            "acom_polar_spectrum": [c_void_p, P(_Peaks), c_void_p, c_void_p, c_void_p, c_size_t, c_void_p],
            "acom_correlate": [c_void_p, P(_Peaks), c_void_p, c_void_p, c_size_t, c_void_p],
            "acom_bound": [c_void_p, P(_Peaks), c_int32, c_void_p, c_void_p, c_size_t, c_void_p],
            "acom_score": [c_void_p, P(_Peaks), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
            "acom_score_grad": [c_void_p, P(_Peaks), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p],
            "acom_refine": [c_void_p, P(_Peaks), c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                            c_void_p, c_void_p],
            "acom_disk_template": [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p],
            "acom_detect_disks": [c_void_p, c_int64, c_void_p, P(_DiskParams), c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_void_p],
            "acom_gather_peaks": [c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_int64, c_void_p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = st
        L.acom_set_tuning.argtypes = [c_int32, c_int32]
        L.acom_set_tuning.restype = st
        L.acom_profile_begin.argtypes = [c_int32]
        L.acom_profile_read.argtypes = [c_int32, P(c_double), P(c_int32)]
        L.acom_profile_end.argtypes = []
        for f in (L.acom_profile_begin, L.acom_profile_read, L.acom_profile_end):
            f.restype = st
        L.acom_status_string.argtypes = [ctypes.c_int]
        L.acom_status_string.restype = ctypes.c_char_p
        L.acom_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


class AcomError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(status, what):
    if status != 0:
        L = lib()
        raise AcomError(status, f"{what}: {L.acom_status_string(status).decode()}: {L.acom_last_error().decode()}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _ptr(t, dtype, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return c_void_p(t.data_ptr())


def _need(t, shape, name):
    """Device arrays handed to the library by pointer must hold what the call
    reads: check the element count against the expected shape."""
    if t is None:
        return
    import math as _m
    if t.numel() != _m.prod(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} ({_m.prod(shape)} elements), got {tuple(t.shape)}")


# ------------------------------------------------------------------ inputs --

def cubic_triangle():
    """[001], [011], [111]: the boundary vectors of the cubic fundamental zone."""
    return [[0.0, 0.0, 1.0], [0.0, 1.0, 1.0], [1.0, 1.0, 1.0]]


def hex_wedge_triangles():
    """z -> 0 deg -> 30 deg and z -> 60 deg -> 30 deg in the basal plane (two triangles)."""
    c30, s30 = math.cos(math.radians(30)), math.sin(math.radians(30))
    c60, s60 = math.cos(math.radians(60)), math.sin(math.radians(60))
    return [[[0, 0, 1.0], [1.0, 0, 0], [c30, s30, 0]], [[0, 0, 1.0], [c60, s60, 0], [c30, s30, 0]]]


@dataclass
class Phase:
    lattice: Sequence[Sequence[float]]
    frac_xyz: Sequence[Sequence[float]]
    triangles: Optional[List] = None          # one or two [v0, v1, v2]
    zones: Optional[Sequence[Sequence[float]]] = None
    species: Optional[Sequence[int]] = None
    f_q: Optional[Sequence[float]] = None
    f_tab: Optional[Sequence[Sequence[float]]] = None


def fiber_zones(axis, theta_max_deg, step_deg, phi_range_deg=(0.0, 360.0)):
    """Zone axes of a fiber-texture plan (acom_fiber_zones): within theta_max of
    `axis`, optionally in an azimuthal wedge; (n, 3) numpy array for the
    `zones` argument of fcc / bcc / hcp."""
    import numpy as np
    ax = (c_double * 3)(*[float(v) for v in axis])
    cnt = c_int32()
    _check(lib().acom_fiber_zones(ax, float(theta_max_deg), float(phi_range_deg[0]), float(phi_range_deg[1]),
                                  float(step_deg), None, 0, ctypes.byref(cnt)), "acom_fiber_zones")
    buf = (c_double * (3 * cnt.value))()
    _check(lib().acom_fiber_zones(ax, float(theta_max_deg), float(phi_range_deg[0]), float(phi_range_deg[1]),
                                  float(step_deg), ctypes.cast(buf, c_void_p), cnt.value, ctypes.byref(cnt)),
           "acom_fiber_zones")
    return np.array(buf[:]).reshape(-1, 3)


def fcc(a=4.08, triangles=None, zones=None):
    return Phase(lattice=[[a, 0, 0], [0, a, 0], [0, 0, a]],
                 frac_xyz=[[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]],
                 triangles=[cubic_triangle()] if (triangles is None and zones is None) else triangles, zones=zones)


def bcc(a=2.87, triangles=None, zones=None):
    return Phase(lattice=[[a, 0, 0], [0, a, 0], [0, 0, a]], frac_xyz=[[0, 0, 0], [0.5, 0.5, 0.5]],
                 triangles=[cubic_triangle()] if (triangles is None and zones is None) else triangles, zones=zones)


def hcp(a=2.95, c=4.68, triangles=None, zones=None):
    return Phase(lattice=[[a, 0, 0], [-a / 2, a * math.sqrt(3) / 2, 0], [0, 0, c]],
                 frac_xyz=[[1 / 3, 2 / 3, 0.25], [2 / 3, 1 / 3, 0.75]],
                 triangles=hex_wedge_triangles() if (triangles is None and zones is None) else triangles,
                 zones=zones)


@dataclass
class PlanParams:
    k_max: float
    n_radial: int = 32
    n_angular: int = 90
    delta: float = 0.08
    gamma: float = 1.0
    omega: float = 1.0
    accel_kV: float = 300.0
    zone_step_deg: float = 5.0
    radial: int = UNIFORM
    kernel: int = CONE
    gauss_sigma: float = 0.0
    sigma_exc: float = 0.02
    precisions: Sequence[str] = field(default_factory=lambda: ["fp32"])
    keep_f64: bool = False
    bound_exact_freqs: int = 0      # 0: the library's default split (FP32 operands)
    bound_block_radii: int = 0
    bound_exact_freqs_16bit: int = 0


class Peaks:
    """CSR peak lists on the device (offsets int64, qx / qy / intensity float32)."""

    def __init__(self, offsets, qx, qy, intensity, device="cuda"):
        self.offsets = torch.as_tensor(offsets, dtype=torch.int64).to(device).contiguous()
        self.qx = torch.as_tensor(qx, dtype=torch.float32).to(device).contiguous()
        self.qy = torch.as_tensor(qy, dtype=torch.float32).to(device).contiguous()
        self.intensity = torch.as_tensor(intensity, dtype=torch.float32).to(device).contiguous()
        self.n_patterns = int(self.offsets.numel()) - 1
        self.total_peaks = int(self.qx.numel())
        if self.qy.numel() != self.total_peaks or self.intensity.numel() != self.total_peaks:
            raise ValueError("qx, qy and intensity must have the same length")
        if self.n_patterns < 0:
            raise ValueError("offsets needs n_patterns + 1 entries")

    @classmethod
    def from_host(cls, d, device="cuda"):
        return cls(d["offsets"], d["qx"], d["qy"], d["I"], device)

    def c(self):
        return _Peaks(self.n_patterns, self.total_peaks, _ptr(self.offsets, torch.int64, "offsets").value,
                      _ptr(self.qx, torch.float32, "qx").value, _ptr(self.qy, torch.float32, "qy").value,
                      _ptr(self.intensity, torch.float32, "intensity").value)


class DiskDetector:
    """Bragg disk detection on raw N x N frames (N = 64 or 128) by correlation
    with the vacuum probe image (acom_disk_template / acom_detect_disks /
    acom_gather_peaks).  probe: (N, N) float32 device tensor; probe_center:
    its centre pixel (row, column); center: the optical axis of the frames in
    pixels; pixel_size: 1/A per pixel."""

    def __init__(self, probe, probe_center, center, pixel_size, edge=4, min_rel=0.005, min_abs=0.0,
                 min_spacing=5, max_peaks=64, exclusion_radius=0.0, stream=None):
        N = int(probe.shape[-1])
        if probe.shape != (N, N):
            raise ValueError("probe must be square")
        self.size = N
        self.max_peaks = int(max_peaks)
        self.params = _DiskParams(N, int(edge), float(min_rel), float(min_abs), int(min_spacing), int(max_peaks),
                                  float(center[0]), float(center[1]), float(exclusion_radius), float(pixel_size))
        self.spectrum = torch.empty((N, N // 2 + 1, 2), dtype=torch.float32, device=probe.device)
        _check(lib().acom_disk_template(_ptr(probe, torch.float32, "probe"), N, int(probe_center[0]),
                                        int(probe_center[1]), c_void_p(self.spectrum.data_ptr()), _stream(stream)),
               "acom_disk_template")

    def detect(self, frames, with_pixels=False, stream=None):
        """Per-frame slots: dict(counts, offsets, qx, qy, I (n, max_peaks), pixel, flags)."""
        if frames.dim() != 3 or tuple(frames.shape[1:]) != (self.size, self.size):
            raise ValueError(f"frames must be (n, {self.size}, {self.size}), got {tuple(frames.shape)}")
        n = int(frames.shape[0])
        dev = frames.device
        out = {"counts": torch.empty(n, dtype=torch.int32, device=dev),
               "offsets": torch.empty(n + 1, dtype=torch.int64, device=dev),
               "flags": torch.empty(n, dtype=torch.int32, device=dev)}
        for k in ("qx", "qy", "I"):
            out[k] = torch.zeros((n, self.max_peaks), dtype=torch.float32, device=dev)
        out["pixel"] = (torch.full((n, self.max_peaks), -1, dtype=torch.int32, device=dev) if with_pixels
                        else None)
        _check(lib().acom_detect_disks(_ptr(frames, torch.float32, "frames"), n,
                                       c_void_p(self.spectrum.data_ptr()), ctypes.byref(self.params),
                                       c_void_p(out["counts"].data_ptr()), c_void_p(out["offsets"].data_ptr()),
                                       c_void_p(out["qx"].data_ptr()), c_void_p(out["qy"].data_ptr()),
                                       c_void_p(out["I"].data_ptr()), _ptr(out["pixel"], torch.int32, "pixel"),
                                       c_void_p(out["flags"].data_ptr()), _stream(stream)), "acom_detect_disks")
        return out

    def gather(self, det, out=None, stream=None, sync=True):
        """CSR Peaks from the slots of detect().  sync=True reads the total (a
        host synchronisation) and returns arrays of exactly that length;
        sync=False returns arrays of the slot capacity n * max_peaks (the
        offsets bound every row, which is all acom_match needs), so the whole
        frames -> peaks -> match sequence runs without a host round trip."""
        n = int(det["counts"].numel())
        dev = det["counts"].device
        total = int(det["offsets"][-1].item()) if sync else n * self.max_peaks
        if out is None:
            out = tuple(torch.empty(total, dtype=torch.float32, device=dev) for _ in range(3))
        qx, qy, I = out
        _check(lib().acom_gather_peaks(n, self.max_peaks, c_void_p(det["counts"].data_ptr()),
                                       c_void_p(det["offsets"].data_ptr()), c_void_p(det["qx"].data_ptr()),
                                       c_void_p(det["qy"].data_ptr()), c_void_p(det["I"].data_ptr()),
                                       c_void_p(qx.data_ptr()), c_void_p(qy.data_ptr()), c_void_p(I.data_ptr()),
                                       min(qx.numel(), qy.numel(), I.numel()), _stream(stream)), "acom_gather_peaks")
        return Peaks(det["offsets"], qx[:total], qy[:total], I[:total], device=dev)

    def peaks(self, frames, stream=None, sync=True):
        return self.gather(self.detect(frames, stream=stream), stream=stream, sync=sync)


class Plan:
    """An orientation plan built on the device by acom_build_plan."""

    def __init__(self, phases: Sequence[Phase], params: PlanParams, stream=None):
        L = lib()
        self._keep = []
        arr = (_Phase * len(phases))()
        for i, ph in enumerate(phases):
            arr[i] = self._phase(ph)
        prm = _Params()
        prm.k_max = params.k_max
        prm.delta = params.delta
        prm.gamma = params.gamma
        prm.omega = params.omega
        prm.accel_kV = params.accel_kV
        prm.zone_step_deg = params.zone_step_deg
        prm.gauss_sigma = params.gauss_sigma
        prm.sigma_exc = params.sigma_exc
        prm.n_radial = params.n_radial
        prm.n_angular = params.n_angular
        prm.radial = params.radial
        prm.kernel = params.kernel
        prm.precisions = sum(1 << PRECISIONS[p] for p in params.precisions)
        prm.keep_f64 = 1 if params.keep_f64 else 0
        prm.bound_exact_freqs = params.bound_exact_freqs
        prm.bound_block_radii = params.bound_block_radii
        prm.bound_exact_freqs_16bit = params.bound_exact_freqs_16bit
        h = c_void_p()
        _check(L.acom_build_plan(arr, len(phases), ctypes.byref(prm), _stream(stream), ctypes.byref(h)),
               "acom_build_plan")
        self._h = h
        self.params = params
        self._keep = None
        Z, R, N, nph = c_int32(), c_int32(), c_int32(), c_int32()
        _check(L.acom_plan_info(h, ctypes.byref(Z), ctypes.byref(R), ctypes.byref(N), ctypes.byref(nph),
                                None, None, None, None), "acom_plan_info")
        self.n_zones, self.n_radial, self.n_angular, self.n_phases = Z.value, R.value, N.value, nph.value

    def _phase(self, ph):
        c = _Phase()
        lat = [float(v) for row in ph.lattice for v in row]
        for i in range(9):
            c.lattice[i] = lat[i]
        frac = (c_double * (3 * len(ph.frac_xyz)))(*[float(v) for row in ph.frac_xyz for v in row])
        self._keep.append(frac)
        c.n_atoms = len(ph.frac_xyz)
        c.frac_xyz = ctypes.cast(frac, P(c_double))
        if ph.species is not None:
            sp = (c_int32 * len(ph.species))(*[int(v) for v in ph.species])
            self._keep.append(sp)
            c.species = ctypes.cast(sp, P(c_int32))
        if ph.f_q is not None:
            fq = (c_double * len(ph.f_q))(*[float(v) for v in ph.f_q])
            ft = (c_double * (len(ph.f_tab) * len(ph.f_q)))(*[float(v) for row in ph.f_tab for v in row])
            self._keep += [fq, ft]
            c.n_f = len(ph.f_q)
            c.f_q = ctypes.cast(fq, P(c_double))
            c.f_tab = ctypes.cast(ft, P(c_double))
        if ph.zones is not None:
            z = (c_double * (3 * len(ph.zones)))(*[float(v) for row in ph.zones for v in row])
            self._keep.append(z)
            c.n_zones_explicit = len(ph.zones)
            c.zones_explicit = ctypes.cast(z, P(c_double))
        else:
            tris = ph.triangles
            c.n_triangles = len(tris)
            for t, tri in enumerate(tris):
                for i in range(3):
                    for j in range(3):
                        c.triangles[9 * t + 3 * i + j] = float(tri[i][j])
        return c

    def info(self):
        import numpy as np
        Z, R = self.n_zones, self.n_radial
        qs = (c_double * R)()
        zs = (c_double * (3 * Z))()
        zp = (c_int32 * Z)()
        A = (c_double * Z)()
        _check(lib().acom_plan_info(self._h, None, None, None, None, qs, zs, zp, A), "acom_plan_info")
        return {"q_s": np.array(qs[:]), "zones": np.array(zs[:]).reshape(Z, 3), "zone_phase": np.array(zp[:]),
                "norm_A": np.array(A[:])}

    def bound_split(self, precision="fp32"):
        """(Kc, radii per block) of the contraction pass's split bound."""
        kc, bb = c_int32(), c_int32()
        _check(lib().acom_plan_bound_split(self._h, PRECISIONS[precision], ctypes.byref(kc), ctypes.byref(bb)),
               "acom_plan_bound_split")
        return kc.value, bb.value

    def angular_f64(self):
        import numpy as np
        out = np.zeros((self.n_zones, self.n_angular, self.n_radial))
        _check(lib().acom_plan_copy_f64(self._h, out.ctypes.data_as(P(c_double))), "acom_plan_copy_f64")
        return out

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().acom_plan_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- match
    def match_workspace_bytes(self, precision="fp32", chunk=0):
        n = c_size_t()
        _check(lib().acom_match_workspace_size(self._h, PRECISIONS[precision], int(chunk), ctypes.byref(n)),
               "acom_match_workspace_size")
        return n.value

    def match(self, peaks: Peaks, top_k=1, precision="fp32", chunk=0, workspace=None, orient=True, stream=None,
              out=None):
        """Top-k matches of every pattern (dict of device tensors)."""
        n = peaks.n_patterns
        dev = peaks.offsets.device
        if workspace is None:
            workspace = torch.empty(self.match_workspace_bytes(precision, chunk), dtype=torch.uint8, device=dev)
        if out is None:
            out = self.empty_matches(n, top_k, orient, dev)
        m = _Matches(*(None if out.get(k) is None else out[k].data_ptr()
                       for k in ("zone", "phase", "bin", "mirror", "score", "phi3", "orient", "n_evaluated")))
        pk = peaks.c()
        _check(lib().acom_match(self._h, ctypes.byref(pk), int(top_k), PRECISIONS[precision], int(chunk),
                                c_void_p(workspace.data_ptr()), workspace.numel(), ctypes.byref(m), _stream(stream)),
               "acom_match")
        return out

    def match_noalloc(self, peaks: Peaks, top_k=1, precision="fp32", orient=True, stream=None, out=None):
        """acom_match_noalloc: the same results as match() with the library's
        static scratch instead of a workspace (calls on one GPU must not overlap)."""
        n = peaks.n_patterns
        if out is None:
            out = self.empty_matches(n, top_k, orient, peaks.offsets.device)
        m = _Matches(*(None if out.get(k) is None else out[k].data_ptr()
                       for k in ("zone", "phase", "bin", "mirror", "score", "phi3", "orient", "n_evaluated")))
        pk = peaks.c()
        _check(lib().acom_match_noalloc(self._h, ctypes.byref(pk), int(top_k), PRECISIONS[precision],
                                        ctypes.byref(m), _stream(stream)), "acom_match_noalloc")
        return out

    def match_multi_workspace_bytes(self, total_peaks, precision="fp32", chunk=0):
        n = c_size_t()
        _check(lib().acom_match_multi_workspace_size(self._h, PRECISIONS[precision], int(chunk), int(total_peaks),
                                                     ctypes.byref(n)), "acom_match_multi_workspace_size")
        return n.value

    def match_multi(self, peaks: Peaks, n_orient=3, deletion_radius=0.04, rel_cut=0.01, min_score=0.0,
                    precision="fp32", chunk=0, workspace=None, stream=None, out=None):
        """Up to n_orient orientations per pattern from overlapping patterns
        (acom_match_multi): dict of device tensors of shape (n, n_orient)
        (orient (n, n_orient, 3, 3)); zone -1 where a round found nothing."""
        n = peaks.n_patterns
        dev = peaks.offsets.device
        if workspace is None:
            workspace = torch.empty(self.match_multi_workspace_bytes(peaks.total_peaks, precision, chunk),
                                    dtype=torch.uint8, device=dev)
        if out is None:
            out = self.empty_matches(n, n_orient, True, dev)
            out["n_evaluated"] = None
        m = _Matches(*(None if out.get(k) is None else out[k].data_ptr()
                       for k in ("zone", "phase", "bin", "mirror", "score", "phi3", "orient", "n_evaluated")))
        pk = peaks.c()
        _check(lib().acom_match_multi(self._h, ctypes.byref(pk), int(n_orient), float(deletion_radius),
                                      float(rel_cut), float(min_score), PRECISIONS[precision], int(chunk),
                                      c_void_p(workspace.data_ptr()), workspace.numel(), ctypes.byref(m),
                                      _stream(stream)), "acom_match_multi")
        return out

    def simulate(self, orient, phase=None, rel_cut=0.01, stream=None, events=None):
        """Forward kinematical patterns of orientations orient (n, 3, 3) on the
        plan's device (acom_simulate_count / _fill): (offsets, qx, qy, intensity)
        device tensors, peaks in the plan's reflection order.  events: optional
        dict of (start, end) torch.cuda.Event pairs under "count" and "fill",
        recorded around the two calls on the launch stream."""
        orient = orient.reshape(-1, 9)
        n = orient.shape[0]
        dev = orient.device
        counts = torch.empty(n, dtype=torch.int32, device=dev)
        offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
        _need(phase, (n,), "phase")
        ph = _ptr(phase, torch.int32, "phase")
        st = torch.cuda.current_stream() if stream is None else stream

        def rec(key, i):
            if events is not None and key in events:
                events[key][i].record(st)

        rec("count", 0)
        _check(lib().acom_simulate_count(self._h, n, _ptr(orient, torch.float32, "orient"), ph, float(rel_cut),
                                         c_void_p(counts.data_ptr()), c_void_p(offsets.data_ptr()), _stream(st)),
               "acom_simulate_count")
        rec("count", 1)
        total = int(offsets[-1].item())  # synchronises
        f32 = dict(dtype=torch.float32, device=dev)
        qx, qy, I = torch.empty(total, **f32), torch.empty(total, **f32), torch.empty(total, **f32)
        rec("fill", 0)
        _check(lib().acom_simulate_fill(self._h, n, _ptr(orient, torch.float32, "orient"), ph, float(rel_cut),
                                        c_void_p(offsets.data_ptr()), c_void_p(qx.data_ptr()), c_void_p(qy.data_ptr()),
                                        c_void_p(I.data_ptr()), _stream(st)), "acom_simulate_fill")
        rec("fill", 1)
        return offsets, qx, qy, I

    def autotune(self, peaks: Peaks, precision="fp32", chunk=0, workspace=None, stream=None):
        """Time every contraction launch shape on the first chunk of `peaks` and
        keep the fastest for `precision` in the calling thread's launch settings
        (acom_autotune; the plan itself is not modified)."""
        dev = peaks.offsets.device
        if workspace is None:
            workspace = torch.empty(self.match_workspace_bytes(precision, chunk), dtype=torch.uint8, device=dev)
        shape = (c_int32 * 3)()
        ms = ctypes.c_float()
        pk = peaks.c()
        _check(lib().acom_autotune(self._h, ctypes.byref(pk), PRECISIONS[precision], int(chunk),
                                   c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream), shape,
                                   ctypes.byref(ms)), "acom_autotune")
        tile = {0: "64x64", 1: "large"}.get(shape[0], str(shape[0]))
        return {"tile": tile, "radii_per_step": shape[1], "order": shape[2], "ms": ms.value}

    @staticmethod
    def empty_matches(n, top_k, orient=True, device="cuda"):
        i32 = dict(dtype=torch.int32, device=device)
        f32 = dict(dtype=torch.float32, device=device)
        return {"zone": torch.empty(n, top_k, **i32), "phase": torch.empty(n, top_k, **i32),
                "bin": torch.empty(n, top_k, **i32), "mirror": torch.empty(n, top_k, **i32),
                "score": torch.empty(n, top_k, **f32), "phi3": torch.empty(n, top_k, **f32),
                "orient": torch.empty(n, top_k, 3, 3, **f32) if orient else None,
                "n_evaluated": torch.empty(n, **i32)}

    # ------------------------------------------------------------- debug
    def _debug_ws(self, n, dev):
        b = c_size_t()
        _check(lib().acom_debug_workspace_size(self._h, n, ctypes.byref(b)), "acom_debug_workspace_size")
        return torch.empty(b.value, dtype=torch.uint8, device=dev)

    def polar_image(self, peaks: Peaks, stream=None):
        n = peaks.n_patterns
        dev = peaks.offsets.device
        X = torch.zeros(n, self.n_angular, self.n_radial, dtype=torch.float32, device=dev)
        ws = self._debug_ws(n, dev)
        pk = peaks.c()
        _check(lib().acom_polar_image(self._h, ctypes.byref(pk), c_void_p(X.data_ptr()), c_void_p(ws.data_ptr()),
                                      ws.numel(), _stream(stream)), "acom_polar_image")
        return X

    def polar_spectrum(self, peaks: Peaks, stream=None):
        n = peaks.n_patterns
        dev = peaks.offsets.device
        nk = self.n_angular // 2 + 1
        Xr = torch.zeros(n, nk, self.n_radial, dtype=torch.float32, device=dev)
        Xi = torch.zeros_like(Xr)
        ws = self._debug_ws(n, dev)
        pk = peaks.c()
        _check(lib().acom_polar_spectrum(self._h, ctypes.byref(pk), c_void_p(Xr.data_ptr()), c_void_p(Xi.data_ptr()),
                                         c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "acom_polar_spectrum")
        return Xr, Xi

    def correlate(self, peaks: Peaks, stream=None):
        n = peaks.n_patterns
        dev = peaks.offsets.device
        C = torch.zeros(n, self.n_zones, 2, self.n_angular, dtype=torch.float32, device=dev)
        ws = self._debug_ws(n, dev)
        pk = peaks.c()
        _check(lib().acom_correlate(self._h, ctypes.byref(pk), c_void_p(C.data_ptr()), c_void_p(ws.data_ptr()),
                                    ws.numel(), _stream(stream)), "acom_correlate")
        return C

    def bound(self, peaks: Peaks, precision="fp32", stream=None):
        n = peaks.n_patterns
        dev = peaks.offsets.device
        U = torch.zeros(n, self.n_zones, dtype=torch.float32, device=dev)
        ws = self._debug_ws(n, dev)
        pk = peaks.c()
        _check(lib().acom_bound(self._h, ctypes.byref(pk), PRECISIONS[precision], c_void_p(U.data_ptr()),
                                c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "acom_bound")
        return U

    # ------------------------------------------------------ score / refine
    def score(self, peaks: Peaks, base, theta, phase=None, stream=None):
        n = peaks.n_patterns
        _need(base, (n, 9), "base")
        _need(theta, (n, 3), "theta")
        _need(phase, (n,), "phase")
        S = torch.empty(n, dtype=torch.float32, device=peaks.offsets.device)
        pk = peaks.c()
        _check(lib().acom_score(self._h, ctypes.byref(pk), _ptr(base, torch.float32, "base"),
                                _ptr(theta, torch.float32, "theta"), _ptr(phase, torch.int32, "phase"),
                                _ptr(S, torch.float32, "S"), _stream(stream)), "acom_score")
        return S

    def score_grad(self, peaks: Peaks, base, theta, dS=None, phase=None, peak_grads=False, stream=None):
        n = peaks.n_patterns
        _need(base, (n, 9), "base")
        _need(theta, (n, 3), "theta")
        _need(dS, (n,), "dS")
        _need(phase, (n,), "phase")
        dev = peaks.offsets.device
        dth = torch.empty(n, 3, dtype=torch.float32, device=dev)
        dqx = torch.empty(peaks.total_peaks, dtype=torch.float32, device=dev) if peak_grads else None
        dqy = torch.empty_like(dqx) if peak_grads else None
        pk = peaks.c()
        _check(lib().acom_score_grad(self._h, ctypes.byref(pk), _ptr(base, torch.float32, "base"),
                                     _ptr(theta, torch.float32, "theta"), _ptr(phase, torch.int32, "phase"),
                                     _ptr(dS, torch.float32, "dS"), _ptr(dth, torch.float32, "dtheta"),
                                     _ptr(dqx, torch.float32, "dqx"), _ptr(dqy, torch.float32, "dqy"),
                                     _stream(stream)), "acom_score_grad")
        return dth, dqx, dqy

    def refine(self, peaks: Peaks, init_orient, cand_phase=None, max_iter=64, stream=None, work=None):
        n = peaks.n_patterns
        dev = peaks.offsets.device
        n_cand = int(init_orient.shape[1])
        _need(init_orient, (n, n_cand, 9), "init_orient")
        _need(cand_phase, (n, n_cand), "cand_phase")
        _need(work, (n, 2), "work")
        out = torch.empty(n, 3, 3, dtype=torch.float32, device=dev)
        S = torch.empty(n, dtype=torch.float32, device=dev)
        cand = torch.empty(n, dtype=torch.int32, device=dev)
        pk = peaks.c()
        _check(lib().acom_refine(self._h, ctypes.byref(pk), n_cand, _ptr(init_orient, torch.float32, "init_orient"),
                                 _ptr(cand_phase, torch.int32, "cand_phase"), int(max_iter),
                                 _ptr(out, torch.float32, "out"), _ptr(S, torch.float32, "S"),
                                 _ptr(cand, torch.int32, "cand"), _ptr(work, torch.int32, "work"), _stream(stream)),
               "acom_refine")
        return out, S, cand


KERNEL_KINDS = {"polar": 0, "bound": 1, "exact": 2}
TUNING_KEYS = {"bound_order": 0, "bound_kch16": 1, "exact_xcd": 2, "polar_xcd": 3, "bound_tile": 4, "skip_zero_radii": 5,
               "bound_kch32": 6, "polar_cols": 7, "exact_u_lds_max": 8, "exact_persist": 9,
               "exact_xcd_block": 10}


def set_tuning(**kw):
    """Launch-shape knobs of the calling thread (results do not depend on them):
    bound_order (0/1), bound_kch16 (32/64/128), exact_xcd (0/1), polar_xcd (0/1),
    bound_tile (0/1/2), skip_zero_radii (0/1), bound_kch32 (16/32), polar_cols
    (16/32), exact_u_lds_max (zones whose bound row the exact pass keeps in LDS), exact_persist (0/1),
    exact_xcd_block (patterns per XCD run of the exact pass's order; 0 = one range per XCD)."""
    for k, v in kw.items():
        _check(lib().acom_set_tuning(TUNING_KEYS[k], int(v)), "acom_set_tuning")


def profile_begin(capacity=4096):
    """Start recording HIP events around every kernel acom_match launches."""
    _check(lib().acom_profile_begin(int(capacity)), "acom_profile_begin")


def profile_read():
    """{kernel: (total_ms, launches)} of the records so far (synchronises them)."""
    out = {}
    for name, k in KERNEL_KINDS.items():
        t, n = c_double(), c_int32()
        _check(lib().acom_profile_read(k, ctypes.byref(t), ctypes.byref(n)), "acom_profile_read")
        out[name] = (t.value, n.value)
    return out


def profile_end():
    _check(lib().acom_profile_end(), "acom_profile_end")


class ContinuousScore(torch.autograd.Function):
    """S = acom_score at base Exp(theta) for the peaks at positions (qx, qy);
    backward through acom_score_grad, which gives dS/dtheta and, when qx or qy
    requires a gradient, dS/dqx and dS/dqy per peak.

    S = ContinuousScore.apply(theta, qx, qy, plan, peaks, base[, phase]):
    theta (n, 3), qx and qy (total_peaks,) float32 device tensors (the peak
    positions; peaks supplies the CSR offsets and the intensities, its own qx /
    qy are not read), base (n, 9)."""

    @staticmethod
    def forward(ctx, theta, qx, qy, plan, peaks, base, phase=None):
        theta_c = theta.detach().contiguous()
        pk = Peaks.__new__(Peaks)
        pk.offsets, pk.intensity = peaks.offsets, peaks.intensity
        pk.qx, pk.qy = qx.detach().contiguous(), qy.detach().contiguous()
        pk.n_patterns, pk.total_peaks = peaks.n_patterns, peaks.total_peaks
        if pk.qx.numel() != pk.total_peaks or pk.qy.numel() != pk.total_peaks:
            raise ValueError("qx and qy must have one entry per peak")
        ctx.plan, ctx.peaks, ctx.base, ctx.phase = plan, pk, base, phase
        ctx.save_for_backward(theta_c)
        return plan.score(pk, base, theta_c, phase)

    @staticmethod
    def backward(ctx, gS):
        (theta_c,) = ctx.saved_tensors
        need_q = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        dth, dqx, dqy = ctx.plan.score_grad(ctx.peaks, ctx.base, theta_c, gS.contiguous().float(), ctx.phase,
                                            peak_grads=need_q)
        return (dth if ctx.needs_input_grad[0] else None, dqx if ctx.needs_input_grad[1] else None,
                dqy if ctx.needs_input_grad[2] else None, None, None, None, None)
