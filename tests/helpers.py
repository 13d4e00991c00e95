"""Shared test helpers: the same crystal / plan parameters handed to the HIP
library (through the binding) and to the oracle."""
import math

import numpy as np

from oracle import plan as oplan
from oracle import zones as ozones

A_FCC = 4.08
FCC_FRAC = [[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]
BCC_FRAC = [[0, 0, 0], [0.5, 0.5, 0.5]]
HCP_LAT = [[2.95, 0, 0], [-2.95 / 2, 2.95 * math.sqrt(3) / 2, 0], [0, 0, 4.68]]
HCP_FRAC = [[1 / 3, 2 / 3, 0.25], [2 / 3, 1 / 3, 0.75]]

SMALL = dict(k_max=1.2, n_radial=32, n_angular=90, zone_step_deg=5.0)
SCAN = dict(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=1.0)


def oracle_plan(phases, k_max, n_radial, n_angular, zone_step_deg, radial=0, kernel=0, delta=0.08,
                gamma=1.0, omega=1.0):
    prm = oplan.Params(k_max=k_max, n_radial=n_radial, n_angular=n_angular, zone_step_deg=zone_step_deg,
                       radial=radial, kind=kernel, delta=delta, gamma=gamma, omega=omega)
    ph = []
    for kind in phases:
        if kind == "fcc":
            ph.append(oplan.Phase(np.eye(3) * A_FCC, FCC_FRAC, triangles=[ozones.cubic_triangle()]))
        elif kind == "bcc":
            ph.append(oplan.Phase(np.eye(3) * 2.87, BCC_FRAC, triangles=[ozones.cubic_triangle()]))
        elif kind == "hcp":
            ph.append(oplan.Phase(np.array(HCP_LAT), HCP_FRAC, triangles=ozones.hex_wedge_triangles()))
        else:
            raise ValueError(kind)
    return oplan.build(ph, prm)


def gpu_plan(phases, k_max, n_radial, n_angular, zone_step_deg, radial=0, kernel=0, delta=0.08, gamma=1.0,
             omega=1.0, precisions=("fp32", "bf16", "fp16"), keep_f64=False):
    from paper_2111_00171_amd import acom
    ph = [{"fcc": acom.fcc, "bcc": acom.bcc, "hcp": acom.hcp}[k]() for k in phases]
    prm = acom.PlanParams(k_max=k_max, n_radial=n_radial, n_angular=n_angular, zone_step_deg=zone_step_deg,
                          radial=radial, kernel=kernel, delta=delta, gamma=gamma, omega=omega,
                          precisions=list(precisions), keep_f64=keep_f64)
    return acom.Plan(ph, prm)


def oracle_image(pl, d, p):
    from oracle import image
    o = d["offsets"]
    return image.polar_image(d["qx"][o[p]:o[p + 1]], d["qy"][o[p]:o[p + 1]], d["I"][o[p]:o[p + 1]], pl["q_s"],
                             pl["P"].shape[1], pl["params"])
