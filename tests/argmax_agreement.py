"""Argmax agreement of the GPU matcher with the FP64 oracle on a seeded subset of
the 65,536-pattern scan (256 x 256 FCC, 1081 zones, 128 x 360 bins), or with
--workload hcp of the 256 x 256 HCP scan against the 8281-zone 6/m wedge (top-8,
one 65,536-pattern chunk per launch as the benchmark runs it).

Test infrastructure: the `compare` step calls the oracle (plain-C FP64 direct
sum over every zone, shift and branch).  The `gpu` step runs the library only.

    python -m tests.argmax_agreement gpu DECISIONS.npz [--workload scan|hcp]
    python -m tests.argmax_agreement compare DECISIONS.npz REPORT.json [--patterns 4096] [--seed 4242]
        [--workload scan|hcp]

Agreement per contraction precision, over the sampled patterns:
  - strict: the GPU's (zone, bin, mirror) is the oracle's lexicographically
    smallest argmax;
  - tie_aware_1e-5: the GPU's choice scores within 1e-5 relative of the oracle
    maximum (the resolution of an FP32 sum of this size);
  - tie_aware_1e-9: the same within 1e-9 (exact ties of symmetric zones).
Near-ties of the oracle (second-best zone within 1e-5 relative) are counted.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

PRECISIONS = ("fp32", "bf16", "fp16")


WORKLOADS = {"scan": ("fcc", 1, "scan: 256x256 FCC, 1081 zones, 128 radial x 360 angular bins, top-1"),
             "hcp": ("hcp", 8, "hcp: 256x256 HCP, 8281 zones (6/m wedge at 1 degree), 128 x 360 bins, top-8, "
                               "65,536 patterns per launch")}


def run_gpu(out_path, workload):
    import torch
    import synth
    from paper_2111_00171_amd import acom
    from tests import helpers
    phase, top_k, _ = WORKLOADS[workload]
    d = synth.make(workload)
    gpl = helpers.gpu_plan([phase], **helpers.SCAN)
    pk = acom.Peaks.from_host(d)
    res = {}
    for prec in PRECISIONS:
        r = gpl.match(pk, top_k=top_k, precision=prec, chunk=65536 if workload == "hcp" else 0)
        torch.cuda.synchronize()
        for k in ("zone", "bin", "mirror", "score"):
            res[f"{prec}_{k}"] = r[k][:, 0].cpu().numpy()
        print(prec, "done", flush=True)
    np.savez(out_path, **res)


def run_compare(dec_path, report_path, n_sample, seed, workload):
    import synth
    from oracle import correlate, directsum
    from tests import helpers
    phase, _, descr = WORKLOADS[workload]
    dec = np.load(dec_path)
    d = synth.make(workload)
    opl = helpers.oracle_plan([phase], **helpers.SCAN)
    n = len(d["offsets"]) - 1
    # in the random order, so that a report cut short is still a uniform sample
    idx = np.random.default_rng(seed).choice(n, n_sample, replace=False)
    t0 = time.perf_counter()
    zsc = []
    for b0 in range(0, n_sample, 64):
        sub = synth.subset(d, idx[b0:b0 + 64])
        zsc.append(directsum.zone_scores(opl, sub["offsets"], sub["qx"], sub["qy"], sub["I"]))
        done = b0 + len(sub["offsets"]) - 1
        print(f"oracle {done}/{n_sample} patterns, {time.perf_counter() - t0:.0f} s", flush=True)
        # the report so far (rewritten after every batch, so a long run can be cut short)
        _report(dec, d, opl, idx[:done], zsc, descr, seed, n_sample, time.perf_counter() - t0, report_path)


def _report(dec, d, opl, idx, zsc, descr, seed, n_planned, seconds, report_path):
    import synth
    from oracle import correlate
    from tests import helpers
    m = len(idx)
    score = np.concatenate([z["score"] for z in zsc])
    zn = np.concatenate([z["n"] for z in zsc])
    zm = np.concatenate([z["mirror"] for z in zsc])
    best = score.max(axis=1)
    ozone = np.argmax(score, axis=1)
    srt = np.sort(score, axis=1)
    near = int(np.sum(srt[:, -2] >= best - 1e-5 * np.abs(best)))
    report = {"workload": descr, "patterns": int(m), "patterns_planned": int(n_planned), "seed": int(seed),
              "oracle": "plain-C FP64 direct sum (oracle/directsum.c)",
              "oracle_near_ties_1e-5": near, "oracle_seconds": round(seconds, 1)}
    for prec in PRECISIONS:
        gz = dec[f"{prec}_zone"][idx]
        gn = dec[f"{prec}_bin"][idx]
        gm = dec[f"{prec}_mirror"][idx]
        strict = tie5 = tie9 = 0
        for i in range(m):
            z = int(gz[i])
            if z < 0:
                continue
            if z == ozone[i] and gn[i] == zn[i, z] and gm[i] == zm[i, z]:
                strict += 1
            if gn[i] == zn[i, z] and gm[i] == zm[i, z]:
                v = score[i, z]
            else:  # the GPU took another (bin, branch) of this zone: evaluate it in FP64
                sub = synth.subset(d, idx[i:i + 1])
                X = helpers.oracle_image(opl, sub, 0)
                C, Cm = correlate.correlate_direct(opl["P"][z:z + 1], X)
                v = (Cm if gm[i] else C)[0, int(gn[i])]
            tie5 += v >= best[i] - 1e-5 * abs(best[i])
            tie9 += v >= best[i] - 1e-9 * abs(best[i])
        report[prec] = {"strict": strict / m, "tie_aware_1e-5": tie5 / m, "tie_aware_1e-9": tie9 / m}
    print({p: report[p] for p in PRECISIONS}, flush=True)
    with open(report_path, "w") as f:
        json.dump(report, f, indent=1)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("step", choices=["gpu", "compare"])
    ap.add_argument("decisions")
    ap.add_argument("report", nargs="?")
    ap.add_argument("--patterns", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=4242)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="scan")
    a = ap.parse_args()
    if a.step == "gpu":
        run_gpu(a.decisions, a.workload)
    else:
        run_compare(a.decisions, a.report, a.patterns, a.seed, a.workload)


if __name__ == "__main__":
    main()
