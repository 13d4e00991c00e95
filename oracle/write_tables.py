"""Write the reflection tables read by the synthetic-scan generator.

TEST INFRASTRUCTURE (part of the oracle).  Run:  python -m oracle.write_tables
It calls only the oracle and writes synth/tables/<phase>.json with, for every
reflection 0 < |g| < 2.0 1/A of the phase: g (crystal Cartesian, 1/A), |F|^2
(f == 1) and the beam wavenumber k0 = 1/lambda at 300 kV.  The generator then
needs no structure-factor or wavelength arithmetic of its own.
"""
import json
import math
import os

import numpy as np

from . import crystal

PHASES = {
    "fcc_a4.08": (np.eye(3) * 4.08, [[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]),
    "bcc_a2.87": (np.eye(3) * 2.87, [[0, 0, 0], [0.5, 0.5, 0.5]]),
    "hcp_a2.95_c4.68": (np.array([[2.95, 0.0, 0.0],
                                  [-2.95 / 2, 2.95 * math.sqrt(3) / 2, 0.0],
                                  [0.0, 0.0, 4.68]]),
                        [[1 / 3, 2 / 3, 0.25], [2 / 3, 1 / 3, 0.75]]),
}
K_MAX = 2.0
ACCEL_KV = 300.0


def main():
    out_dir = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "synth", "tables")
    os.makedirs(out_dir, exist_ok=True)
    k0 = 1.0 / crystal.electron_wavelength(ACCEL_KV)
    for name, (lat, frac) in PHASES.items():
        r = crystal.reflections(lat, frac, K_MAX)
        doc = {"phase": name, "k_max": K_MAX, "accel_kV": ACCEL_KV, "k0": k0,
               "lattice": np.asarray(lat).tolist(), "frac_xyz": np.asarray(frac, float).tolist(),
               "g": np.round(r["g"], 15).tolist(), "F2": np.round(np.abs(r["F"]) ** 2, 12).tolist()}
        with open(os.path.join(out_dir, name + ".json"), "w") as f:
            json.dump(doc, f)
        print(name, len(r["q"]))


if __name__ == "__main__":
    main()
