#!/usr/bin/env python3
"""Diffraction patterns indexed per second on one MI355X.

Default workload ("scan"): a seeded synthetic 256 x 256 FCC (a = 4.08 A) scan
of 65,536 patterns with 10-60 Bragg peaks each (50 Voronoi grains, position
jitter, intensity noise, 0-2 spurious peaks), matched against the 1-degree
orientation plan of the cubic fundamental zone (1081 zone axes), 128 radial
bins to k_max = 2.0 1/A and 360 angular bins, top-1 match per pattern.

One step = one acom_match over the whole scan (peaks already resident in HBM):
polar image + FFT, MFMA bound contraction, exact FP32 pass, orientation.
`value` is the FP32-contraction rate; the BF16 (and optionally FP16)
contraction with FP32 rescoring is timed on the same inputs and reported
beside it.  The dominant kernel's roofline uses its average duration from HIP
events recorded on its launch stream during the timed steps.

The default run also times, as extra keys of the same line ("workloads"),
short runs of the HCP top-8 scan (BF16 / FP16 / FP32), the three-phase
262,144-pattern scan by HIP-graph replay (BF16) and the top-4 + refinement
workload, each with its own dominant-kernel time and a seeded oracle sample
of at least 64 patterns (--no-extra skips them).  Their oracle plans and
direct sums run in a worker process while the GPU is timed.

Other workloads (--workload), each printing one JSON line of the same form:
  hcp     256 x 256 HCP (a = 2.95, c = 4.68) scan against the 6/m wedge at 1
          degree (8281 zones); BF16 / FP16 / FP32 contraction, top-8 FP32
          rescoring.
  multi   512 x 512 three-phase scan (FCC + BCC + HCP plans concatenated,
          10,443 zones), ragged peak counts 3-150; BF16; the whole acom_match
          captured once in a HIP graph and timed by graph replays.
  refine  65,536 FCC patterns at random (off-grid) orientations: top-4 grid
          candidates (FP32 contraction) refined by gradient ascent on the
          continuous score (acom_refine, FP32).
  overlap 65,536 patterns of two overlapping FCC grains: up to two
          orientations each (acom_match_multi, BF16).
  simulate forward kinematical patterns of 65,536 orientations (CSR).
  detect  Bragg disk detection on 65,536 raw 128 x 128 frames (acom_detect_disks
          and acom_gather_peaks); frames/s, HBM roofline of the detection kernel.
  pipeline raw frames -> disk detection -> match (BF16, FP32 rescoring) with no
          host round trip; frames/s and orientation accuracy against the truth.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "diffraction patterns indexed/sec at 1 GPU, BF16 vs FP32 at ≥99.9% oracle argmax match"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}   # dense MFMA
HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bound_kernel_scan_traffic.json")
# Exact frequencies of the 16-bit split bound for the three-phase workload: its
# 10,443-zone plan and 3-150-peak patterns prune better with a tighter bound
# (measured: 72 -> 697k, 48 -> 543k, 96 -> 633k patterns/s); the library's
# default, 48, is the best on the FCC scan (4.19M against 4.08M at 64) and the
# HCP scan (1.00M against 0.94M at 64).
MULTI_KC16 = 72
DATA = "synthetic (seeded generator; the paper's datasets are not available)"

PLAN_CFG = {  # phases and plan parameters of each workload
    "scan": (["fcc"], dict(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=1.0)),
    "hcp": (["hcp"], dict(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=1.0)),
    "multi": (["fcc", "bcc", "hcp"], dict(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=1.0)),
    "refine": (["fcc"], dict(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=1.0)),
    "overlap": (["fcc"], dict(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=1.0)),
    "simulate": (["fcc"], dict(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=1.0)),
    "hard": (["fcc"], dict(k_max=2.0, n_radial=128, n_angular=360, zone_step_deg=1.0)),
}
DESCR = {
    "scan": "scan: 256x256 FCC scan, 65,536 patterns x 10-60 peaks, 1-degree plan (1081 zones), "
            "128 radial x 360 angular bins, top-1, FP32 contraction",
    "hcp": "hcp: 256x256 HCP scan, 65,536 patterns, 6/m wedge at 1 degree (8281 zones), 128 x 360 bins, "
           "top-8 FP32 rescoring",
    "multi": "multi: 512x512 three-phase scan (FCC 4.08 + BCC 2.87 + HCP), 262,144 patterns x 3-150 peaks, "
             "10,443 zones, 128 x 360 bins, top-1, BF16 contraction, one HIP-graph replay per step",
    "hard": "hard: the 256x256 FCC scan with degraded peak lists (20% of real peaks dropped, intensities x (1 + 0.3 "
            "N(0,1)), 5-10 spurious peaks each), 1081 zones, 128 x 360 bins, top-1",
    "refine": "refine: 65,536 FCC patterns at random orientations, top-4 grid candidates (FP32 contraction) "
              "refined by gradient ascent on the continuous score (<= 64 trials each)",
    "overlap": "overlap: 65,536 FCC patterns, each two overlapping grains (second at 0.4-0.9 intensity), "
               "up to 2 orientations per pattern by iterative match + forward pattern + peak deletion "
               "(deletion radius 0.04 1/A), BF16 contraction, 1-degree plan, 128 x 360 bins",
    "simulate": "simulate: forward kinematical patterns of 65,536 random FCC orientations (reflections with "
                "|g| < 2.0 1/A, kept above 1% of max |F|^2 after the excitation-error shape factor), CSR output",
    "pipeline": "pipeline: 65,536 raw 128x128 float32 frames (a 64x64 scan of 4 FCC Voronoi grains, tiled 16 times; "
                "the grain density of the 256x256 scan) -> Bragg disk "
                "detection (at most 64 peaks) -> CSR peaks without a host round trip -> match against the 1-degree "
                "plan (1081 zones, 128 x 360 bins), BF16 contraction, top-1 rescored in FP32",
    "detect": "detect: Bragg disk detection on 65,536 raw 128x128 float32 frames of FCC grains (4,096 distinct "
              "frames tiled 16 times; probe disk radius 3.5 px), correlation with the probe image, at most 64 "
              "peaks per frame (spacing 5 px, threshold 0.5% of the strongest, 4 px edge, 4 px beam exclusion), "
              "CSR output",
}
DISK_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "disk_detect_kernel_traffic.json")


def log(msg):
    """Progress of the run on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the contraction kernel's source: the bound section of match.hip
    (from its section marker to the next) and the shared header, so that the
    stored counters stay valid across changes to the other passes."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2111_00171_amd", "csrc", "match.hip"), "rb") as fh:
        src = fh.read()
    a = src.index(b"// " + b"-" * 60 + b" 2. bound ----")
    b = src.index(b"// " + b"-" * 60 + b" 3. exact ----")
    h.update(src[a:b])
    with open(os.path.join(ROOT, "paper_2111_00171_amd", "csrc", "acom_internal.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def disk_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2111_00171_amd", "csrc", "disks.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_disk_traffic(frames_per_launch):
    """HBM bytes per launch of the disk detection kernel from rocprofv3
    FETCH_SIZE/WRITE_SIZE counters (profiles/), or None if they were taken on a
    different kernel source or launch size."""
    if not os.path.exists(DISK_TRAFFIC_FILE):
        return None
    with open(DISK_TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("source_hash") != disk_source_hash() or t.get("frames_per_launch") != frames_per_launch:
        return None
    return t["bytes_per_launch"]


def measured_traffic(precision, launches_patterns):
    """HBM bytes per launch of the bound kernel on the scan workload from
    rocprofv3 FETCH_SIZE/WRITE_SIZE counters (profiles/), or None if they were
    taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash():
        return None
    e = t.get(precision)
    if not e or e.get("patterns_per_launch") != launches_patterns:
        return None
    return e["bytes_per_launch"]


def refine_roofline(work, ms):
    """ALU roofline of refine_kernel from its own work counts (acom_refine's
    out_work: (peak, reflection) pairs evaluated for S alone and with the
    gradient): 8 FLOP per pair for S (two differences, the squared distance,
    its scaling, the exponential, the weight and the sum) and 12 with the
    gradient (two more multiply-adds), against the FP32 vector peak without
    packed instructions (78.6 TFLOP/s)."""
    w = work.double().sum(0).cpu().numpy()
    flop = 8.0 * w[0] + 12.0 * w[1]
    tf = flop / (ms * 1e-3) / 1e12
    return {"kernel": "refine_kernel (one wavefront per pattern)", "bound": "alu", "achieved": round(tf, 3),
            "peak": 78.6, "unit": "TFLOP/s", "frac": round(tf / 78.6, 4), "flop_per_launch": flop,
            "pairs_score": float(w[0]), "pairs_score_and_gradient": float(w[1]), "refine_ms": round(ms, 3)}


def bound_flop_per_pattern(gpl, prec):
    """Algorithmic FLOP per pattern of the contraction pass's split bound with
    operands of `prec`: for every zone, the four real products of the Kc exact
    frequencies (8 Kc N_r) and one multiply-add per block-norm entry of the
    rest (2 (N_phi/2 + 1 - Kc) ceil(N_r / block))."""
    kc, bb = gpl.bound_split(prec)
    nk, R = gpl.n_angular // 2 + 1, gpl.n_radial
    return float(gpl.n_zones) * (8.0 * kc * R + 2.0 * (nk - kc) * (-(-R // bb)))


def full_contraction_flop_per_pattern(gpl):
    """8 Z (N_phi/2 + 1) N_r: every frequency's complex contraction, which the
    split bound replaces above Kc."""
    return 8.0 * gpl.n_zones * (gpl.n_angular // 2 + 1) * gpl.n_radial


def _oracle_plan(workload):
    from tests import helpers
    phases, cfg = PLAN_CFG[workload]
    return helpers.oracle_plan(phases, **cfg)


def cpu_baseline_match(workload, d, res_by_prec, sample_target_s=15.0, max_patterns=512):
    """The oracle (plain-C FP64 direct sum, OpenMP) on a bounded seeded sample;
    also the argmax agreement of each precision on that sample."""
    import numpy as np
    import synth
    from oracle import directsum

    t0 = time.perf_counter()
    opl = _oracle_plan(workload)
    log(f"{workload}: oracle plan built ({time.perf_counter() - t0:.1f} s)")
    rng = np.random.default_rng(2024)
    n = len(d["offsets"]) - 1
    idx_all = rng.permutation(n)
    # the oracle runs one pattern per thread: a first batch of `cores` patterns
    # calibrates, then one call takes the rest of about sample_target_s of work
    # (dynamic scheduling over more patterns than threads keeps them busy)
    cores = directsum.num_threads()
    batches, el = [], 0.0
    for b in range(2):
        lo = 0 if b == 0 else cores
        hi = cores if b == 0 else min(max_patterns, cores + int(cores * (sample_target_s - el) / el) // cores * cores)
        if hi <= lo:
            break
        idx = np.sort(idx_all[lo:hi])
        sub = synth.subset(d, idx)
        t0 = time.perf_counter()
        batches.append((idx, directsum.zone_scores(opl, sub["offsets"], sub["qx"], sub["qy"], sub["I"])))
        el += time.perf_counter() - t0
        log(f"{workload}: oracle on {hi - lo} patterns ({el:.1f} s in total)")
    idx = np.concatenate([i for i, _ in batches])
    zs = {k: np.concatenate([z[k] for _, z in batches]) for k in ("score", "n", "mirror")}
    m = len(idx)
    # the same oracle on one thread, on the first sampled pattern, when that
    # takes at most ~20 s (estimated from the all-thread rate)
    one_core = None
    if cores / (m / el) <= 20.0:
        sub1 = synth.subset(d, np.sort(idx_all[:1]))
        t0 = time.perf_counter()
        directsum.zone_scores(opl, sub1["offsets"], sub1["qx"], sub1["qy"], sub1["I"], 1)
        one_core = 1 / (time.perf_counter() - t0)
        log(f"{workload}: oracle on one thread, {one_core:.3f} patterns/s")
    agree = {}
    for prec, res in res_by_prec.items():
        zone = res["zone"][idx, 0]
        bins = res["bin"][idx, 0]
        mir = res["mirror"][idx, 0]
        ok_tie = ok_strict = 0
        for i in range(m):
            sc = zs["score"][i]
            mx = sc.max()
            z = int(zone[i])
            best = int(np.argmax(sc))
            strict = (z == best and int(bins[i]) == int(zs["n"][i][best]) and int(mir[i]) == int(zs["mirror"][i][best]))
            ok_strict += strict
            ok_tie += (z >= 0 and sc[z] >= mx - 1e-5 * mx)
        agree[prec] = {"tie_aware": ok_tie / m, "strict": ok_strict / m, "patterns": m}
    Z = opl["P"].shape[0]
    return ({"value": m / el, "unit": "patterns/s", "cores": cores, "kind": "oracle",
             "sample": f"{m} seeded patterns of the same workload; plain-C FP64 direct-sum correlation "
                       f"over all {Z} zones x 360 bins x 2 branches (OpenMP, {cores} threads); "
                       f"plan build excluded as on the GPU",
             "value_one_core": one_core, "cpu_model": cpu_model()}, agree)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_refine(d, init, res, sample_target_s=15.0, max_patterns=256):
    """The oracle refinement (FP64 score and gradient, the same ascent) on a
    bounded seeded sample from the GPU's top-4 grid candidates; also the
    misorientation between the GPU and oracle refinements on that sample."""
    import numpy as np
    from oracle import crystal, metrics, score
    from oracle import plan as oplan
    from tests import helpers

    refl = crystal.reflections(np.eye(3) * helpers.A_FCC, helpers.FCC_FRAC, 2.0)
    prm = oplan.Params(k_max=2.0)
    o = d["offsets"]
    G = metrics.cubic_rotations()
    rng = np.random.default_rng(2025)
    order = rng.permutation(len(o) - 1)
    done, mis, t_used = 0, [], 0.0
    while done < max_patterns and t_used < sample_target_s:
        p = int(order[done])
        t0 = time.perf_counter()
        mo, _ = score.refine(refl, d["qx"][o[p]:o[p + 1]].astype(np.float64), d["qy"][o[p]:o[p + 1]].astype(np.float64),
                             d["I"][o[p]:o[p + 1]].astype(np.float64), list(init[p]), prm, max_iter=64)
        t_used += time.perf_counter() - t0
        mis.append(metrics.misorientation_deg(res[p], mo, G))
        done += 1
        if done % 8 == 0:
            log(f"refine: oracle refined {done} patterns ({t_used:.1f} s)")
    return ({"value": done / t_used, "unit": "patterns/s", "cores": 1, "kind": "oracle",
             "sample": f"{done} seeded patterns; FP64 continuous-score refinement of the same 4 candidates "
                       f"(numpy, single thread); candidate search excluded"},
            {"gpu_vs_oracle_misorientation_deg": {"median": float(np.median(mis)), "max": float(np.max(mis)),
                                                  "patterns": done}})


def time_match(gpl, pk, prec, top_k, chunk, steps, warmup, n, flop_per_pattern, autotune=True):
    import torch
    from paper_2111_00171_amd import acom
    ws = torch.empty(gpl.match_workspace_bytes(prec, chunk), dtype=torch.uint8, device="cuda")
    out = gpl.empty_matches(n, top_k, True, "cuda")
    shape = gpl.autotune(pk, prec, chunk, ws) if autotune else None
    for _ in range(warmup):
        gpl.match(pk, top_k, prec, chunk, ws, out=out)
    torch.cuda.synchronize()
    acom.profile_begin(8192)
    t0 = time.perf_counter()
    for _ in range(steps):
        gpl.match(pk, top_k, prec, chunk, ws, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = acom.profile_read()
    acom.profile_end()
    kern = {k: {"avg_ms": (t / c if c else None), "launches": c} for k, (t, c) in prof.items()}
    b = prof["bound"]
    per_launch = min(chunk, n)
    flop_per_pattern = bound_flop_per_pattern(gpl, prec)  # the split depends on the operand precision
    achieved = flop_per_pattern * per_launch / (b[0] / b[1] * 1e-3) / 1e12
    nev = out["n_evaluated"].float()
    run = {"value": n * steps / el, "ms_per_step": el * 1e3 / steps, "kernels": kern, "contraction_shape": shape,
           "flop_per_pattern": flop_per_pattern,
           "bound_tflops": achieved, "bound_frac": achieved / PEAK_TFLOPS[prec],
           "zones_evaluated_mean": float(nev.mean()), "zones_evaluated_max": int(nev.max())}
    host = {k: out[k].cpu().numpy() for k in ("zone", "phase", "bin", "mirror", "score")}
    host["orient"] = out["orient"].cpu().numpy()
    del ws
    return run, host


def by_precision(runs):
    return {p: {"patterns_per_s": round(v["value"], 1), "ms_per_step": round(v["ms_per_step"], 3),
                "bound_tflops": round(v["bound_tflops"], 3), "bound_frac_of_peak": round(v["bound_frac"], 4),
                "kernel_avg_ms": {k: (None if kk["avg_ms"] is None else round(kk["avg_ms"], 4))
                                  for k, kk in v["kernels"].items()},
                "zones_evaluated_mean": round(v["zones_evaluated_mean"], 3),
                "zones_evaluated_max": v["zones_evaluated_max"],
                "contraction_shape": v["contraction_shape"]} for p, v in runs.items()}


def roofline(runs, prec, per_launch, flop_per_pattern, traffic):
    r = runs[prec]
    kern = r["kernels"]
    dominant = max(kern, key=lambda k: (kern[k]["avg_ms"] or 0) * kern[k]["launches"])
    return {"kernel": "bound_kernel (MFMA contraction, %s operands)" % prec, "bound": "mfma",
            "achieved": round(r["bound_tflops"], 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": round(r["bound_frac"], 4), "traffic": traffic,
            "algorithmic_flop_per_launch": r["flop_per_pattern"] * per_launch, "dominant_kernel_of_step": dominant}


def line(workload, value, ms, steps, warmup, dtype, cfg, roof, cpu, extra):
    out = {"metric": METRIC, "value": round(value, 1), "unit": "patterns/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": DATA, "config": {"workload": DESCR[workload], **cfg},
           "roofline": roof, "cpu_baseline": cpu}
    out.update(extra)
    return out


def run_match_workload(args, workload, defer_oracle=False):
    import numpy as np
    import torch
    import synth
    from paper_2111_00171_amd import acom

    precs = [p for p in args.precisions.split(",") if p]
    top_k = 8 if workload == "hcp" else 1
    t0 = time.perf_counter()
    d = synth.make(workload)
    t_gen = time.perf_counter() - t0
    log(f"{workload}: inputs generated ({len(d['offsets']) - 1} patterns, {t_gen:.1f} s)")
    phases, cfg = PLAN_CFG[workload]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gpl = acom.Plan([{"fcc": acom.fcc, "bcc": acom.bcc, "hcp": acom.hcp}[k]() for k in phases],
                    acom.PlanParams(precisions=precs, bound_exact_freqs=args.bound_exact_freqs,
                                    bound_block_radii=args.bound_block_radii,
                                    bound_exact_freqs_16bit=args.bound_exact_freqs_16bit, **cfg))
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    n = len(d["offsets"]) - 1
    pk = acom.Peaks.from_host(d)
    Z, R, N = gpl.n_zones, gpl.n_radial, gpl.n_angular
    flop_per_pattern = bound_flop_per_pattern(gpl, precs[0])
    runs, host = {}, {}
    log(f"{workload}: plan built ({Z} zones, {t_plan:.1f} s)")
    for prec in precs:
        runs[prec], host[prec] = time_match(gpl, pk, prec, top_k, args.chunk, args.steps, args.warmup, n,
                                            flop_per_pattern)
        log(f"{workload}: {prec} timed, {runs[prec]['value']:.0f} patterns/s")
    cpu = agree = None
    if not args.no_cpu_baseline and not defer_oracle:
        cpu, agree = cpu_baseline_match(workload, d, host)
        log(f"{workload}: oracle sample timed")
    main_prec = precs[0]
    per_launch = min(args.chunk, n)
    traffic = measured_traffic(main_prec, per_launch) if workload == "scan" else None
    extra = {"argmax_match_vs_oracle": agree, "by_precision": by_precision(runs),
             "plan_build_s": round(t_plan, 3), "input_generation_s": round(t_gen, 3)}
    if workload != "scan":
        # the generator's ground truth: misorientation of the top match within the 1-degree grid
        from oracle import metrics
        G = metrics.hexagonal_rotations() if workload == "hcp" else metrics.cubic_rotations()
        idx = np.random.default_rng(7).choice(n, 256, replace=False)
        mis = [metrics.misorientation_deg(host[main_prec]["orient"][p, 0], d["truth"][p], G) for p in idx]
        extra["misorientation_vs_truth_deg"] = {"median": float(np.median(mis)), "p90": float(np.percentile(mis, 90)),
                                                "patterns": 256, "precision": main_prec}
    kc, bb = gpl.bound_split(main_prec)
    ccfg = {"patterns": n, "peaks": int(d["offsets"][-1]), "zones": Z, "n_radial": R, "n_angular": N,
            "chunk": args.chunk, "top_k": top_k, "bound_exact_freqs": kc, "bound_block_radii": bb,
            "bound_exact_freqs_by_precision": {p: gpl.bound_split(p)[0] for p in precs}}
    extra["bound_flop_per_pattern"] = flop_per_pattern
    extra["full_contraction_flop_per_pattern"] = full_contraction_flop_per_pattern(gpl)
    r = runs[main_prec]
    out = line(workload, r["value"], r["ms_per_step"], args.steps, args.warmup,
               {"fp32": "f32", "bf16": "bf16", "fp16": "f16"}[main_prec], ccfg,
               roofline(runs, main_prec, per_launch, flop_per_pattern, traffic), cpu, extra)
    if defer_oracle:
        out["_deferred"] = (d, host)
    return out


def run_multi(args):
    """Batching: one acom_match over the whole ragged 3-phase scan captured in a
    HIP graph; a step is one graph replay."""
    import numpy as np
    import torch
    import synth
    from paper_2111_00171_amd import acom

    prec = "bf16"
    t0 = time.perf_counter()
    d = synth.make("multi")
    t_gen = time.perf_counter() - t0
    log(f"multi: inputs generated ({len(d['offsets']) - 1} patterns, {t_gen:.1f} s)")
    phases, cfg = PLAN_CFG["multi"]
    t0 = time.perf_counter()
    gpl = acom.Plan([{"fcc": acom.fcc, "bcc": acom.bcc, "hcp": acom.hcp}[k]() for k in phases],
                    acom.PlanParams(precisions=[prec], bound_exact_freqs=args.bound_exact_freqs,
                                    bound_block_radii=args.bound_block_radii,
                                    bound_exact_freqs_16bit=args.bound_exact_freqs_16bit or MULTI_KC16, **cfg))
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    n = len(d["offsets"]) - 1
    pk = acom.Peaks.from_host(d)
    Z, R, N = gpl.n_zones, gpl.n_radial, gpl.n_angular
    flop_per_pattern = bound_flop_per_pattern(gpl, prec)
    # kernel averages and the contraction roofline from an eager profiled run
    log(f"multi: plan built ({Z} zones, {t_plan:.1f} s)")
    run, host = time_match(gpl, pk, prec, 1, args.chunk, 2, 1, n, flop_per_pattern)
    log(f"multi: eager profiled run, {run['value']:.0f} patterns/s")
    # the graph: captured once, replayed
    ws = torch.empty(gpl.match_workspace_bytes(prec, args.chunk), dtype=torch.uint8, device="cuda")
    out = gpl.empty_matches(n, 1, True, "cuda")
    gpl.match(pk, 1, prec, args.chunk, ws, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpl.match(pk, 1, prec, args.chunk, ws, out=out)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    same = bool(np.array_equal(out["zone"].cpu().numpy(), host["zone"]))
    log(f"multi: graph replays timed, {n * args.steps / el:.0f} patterns/s")
    cpu = agree = None
    if not args.no_cpu_baseline:
        cpu, agree = cpu_baseline_match("multi", d, {prec: host})
    cnt = np.diff(d["offsets"])
    sel = np.flatnonzero(cnt >= 8)
    phase_ok = float(np.mean((host["zone"][sel, 0] >= 0) & (host["phase"][sel, 0] == d["phase"][sel])))
    per_launch = min(args.chunk, n)
    extra = {"argmax_match_vs_oracle": agree, "by_precision": by_precision({prec: run}),
             "graph_replay_matches_eager": same, "phase_identified_fraction_ge8_peaks": phase_ok,
             "plan_build_s": round(t_plan, 3), "input_generation_s": round(t_gen, 3)}
    ccfg = {"patterns": n, "peaks": int(d["offsets"][-1]), "zones": Z, "n_radial": R, "n_angular": N,
            "chunk": args.chunk, "top_k": 1, "graph": True, "bound_exact_freqs_16bit": gpl.bound_split("bf16")[0]}
    return line("multi", n * args.steps / el, el * 1e3 / args.steps, args.steps, args.warmup, "bf16", ccfg,
                roofline({prec: run}, prec, per_launch, flop_per_pattern, None), cpu, extra)


def run_refine(args):
    """Differentiation: top-4 grid candidates (FP32 contraction) refined on the
    continuous score; a step is acom_match + acom_refine over all patterns."""
    import numpy as np
    import torch
    import synth
    from paper_2111_00171_amd import acom
    from oracle import metrics

    t0 = time.perf_counter()
    d = synth.make("refine")
    t_gen = time.perf_counter() - t0
    log(f"refine: inputs generated ({len(d['offsets']) - 1} patterns, {t_gen:.1f} s)")
    phases, cfg = PLAN_CFG["refine"]
    gpl = acom.Plan([acom.fcc()], acom.PlanParams(precisions=["fp32", "bf16"], **cfg))
    n = len(d["offsets"]) - 1
    pk = acom.Peaks.from_host(d)
    ws = torch.empty(gpl.match_workspace_bytes("bf16", args.chunk), dtype=torch.uint8, device="cuda")
    out = gpl.empty_matches(n, 4, True, "cuda")

    shape = gpl.autotune(pk, "fp32", args.chunk, ws)
    work = torch.zeros(n, 2, dtype=torch.int32, device="cuda")

    def step():
        gpl.match(pk, 4, "fp32", args.chunk, ws, out=out)
        return gpl.refine(pk, out["orient"].reshape(n, 4, 9), max_iter=64)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_match = t_ref = 0.0
    acom.profile_begin(8192)
    for _ in range(args.steps):
        t0 = time.perf_counter()
        gpl.match(pk, 4, "fp32", args.chunk, ws, out=out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m, S, c = gpl.refine(pk, out["orient"].reshape(n, 4, 9), max_iter=64, work=work)
        torch.cuda.synchronize()
        t_ref += time.perf_counter() - t1
        t_match += t1 - t0
    el = t_match + t_ref
    prof = acom.profile_read()
    acom.profile_end()
    Z, R, N = gpl.n_zones, gpl.n_radial, gpl.n_angular
    flop_per_pattern = bound_flop_per_pattern(gpl, "fp32")
    b_ms = prof["bound"][0] / prof["bound"][1]
    per_launch = min(args.chunk, n)
    tflops = flop_per_pattern * per_launch / (b_ms * 1e-3) / 1e12
    log(f"refine: timed, {n * args.steps / el:.0f} patterns/s")
    m = m.cpu().numpy()
    init = out["orient"].reshape(n, 4, 3, 3).cpu().numpy()
    G = metrics.cubic_rotations()
    idx = np.random.default_rng(9).choice(n, 512, replace=False)
    mis_grid = [metrics.misorientation_deg(init[p, 0], d["truth"][p], G) for p in idx]
    mis_ref = [metrics.misorientation_deg(m[p], d["truth"][p], G) for p in idx]
    # the far tail: is the refined orientation a higher maximum of the score than
    # the truth (the score itself prefers it), or did the search stop short?
    truth = torch.tensor(np.ascontiguousarray(d["truth"].reshape(n, 9)), dtype=torch.float32, device="cuda")
    S_truth = gpl.score(pk, truth, torch.zeros(n, 3, dtype=torch.float32, device="cuda")).cpu().numpy()
    S_ref = S.cpu().numpy()
    far = [p for p, mr in zip(idx, mis_ref) if mr > 5.0]
    # the same refinement from BF16-contraction candidates (FP32 rescoring)
    out16 = gpl.empty_matches(n, 4, True, "cuda")
    gpl.match(pk, 4, "bf16", args.chunk, ws, out=out16)
    m16, _, _ = gpl.refine(pk, out16["orient"].reshape(n, 4, 9), max_iter=64)
    m16 = m16.cpu().numpy()
    mis16 = [metrics.misorientation_deg(m16[p], d["truth"][p], G) for p in idx]
    mis16_32 = [metrics.misorientation_deg(m16[p], m[p], G) for p in idx]
    tail = {"patterns_over_5deg": len(far),
            "refined_score_at_least_truth_score": int(sum(S_ref[p] >= S_truth[p] * (1.0 - 1e-5) for p in far))}
    cpu = ext = None
    if not args.no_cpu_baseline:
        cpu, ext = cpu_baseline_refine(d, init, m)
    extra = {"refinement_vs_truth_deg": {"grid_top1_median": float(np.median(mis_grid)),
                                         "refined_median": float(np.median(mis_ref)),
                                         "refined_p90": float(np.percentile(mis_ref, 90)),
                                         "refined_p99": float(np.percentile(mis_ref, 99)), "patterns": 512,
                                         "tail_over_5deg": tail,
                                         "bf16_candidates": {
                                             "refined_median": float(np.median(mis16)),
                                             "refined_p90": float(np.percentile(mis16, 90)),
                                             "vs_fp32_candidates_within_0.1deg": float(np.mean(np.array(mis16_32) < 0.1)),
                                             "vs_fp32_candidates_median": float(np.median(mis16_32))}},
             "refine_roofline": refine_roofline(work, t_ref * 1e3 / args.steps),
             "contraction_shape": shape, "ms_per_step_match": round(t_match * 1e3 / args.steps, 3),
             "ms_per_step_refine": round(t_ref * 1e3 / args.steps, 3),
             "oracle_comparison": ext, "input_generation_s": round(t_gen, 3)}
    ccfg = {"patterns": n, "peaks": int(d["offsets"][-1]), "zones": gpl.n_zones, "n_radial": gpl.n_radial,
            "n_angular": gpl.n_angular, "candidates": 4, "max_trials": 64}
    # the roofline of the step's dominant kernel: the refinement's (ALU, its
    # counted score and gradient work) or the FP32 contraction of the search
    contraction = {"kernel": "bound_kernel (MFMA contraction, fp32 operands) of the top-4 search", "bound": "mfma",
                   "achieved": round(tflops, 3), "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                   "frac": round(tflops / PEAK_TFLOPS["fp32"], 4), "traffic": None,
                   "algorithmic_flop_per_launch": flop_per_pattern * per_launch,
                   "kernel_avg_ms": {k: (round(t / c, 4) if c else None) for k, (t, c) in prof.items()}}
    rr = dict(extra["refine_roofline"], traffic=None)
    bound_ms = contraction["kernel_avg_ms"].get("bound") or 0.0
    if rr["refine_ms"] >= bound_ms:
        roof = dict(rr, other_kernel=contraction)
    else:
        roof = dict(contraction, other_kernel=rr)
    return line("refine", n * args.steps / el, el * 1e3 / args.steps, args.steps, args.warmup, "f32", ccfg, roof,
                cpu, extra)


def cpu_baseline_overlap(d, res, r_del, n_orient, budget_s=25.0):
    """The oracle (oracle/multi.match_multi_c: the plain-C direct sum for each
    round's maximum) on seeded patterns of the workload until ~budget_s of CPU
    time; also how often its decisions equal the GPU's."""
    import numpy as np
    from oracle import directsum, metrics, multi
    from tests import helpers
    G = metrics.cubic_rotations()
    phases, cfg = PLAN_CFG["overlap"]
    opl = helpers.oracle_plan(phases, **cfg)
    log("overlap: oracle plan built")
    cores = directsum.num_threads()
    o = d["offsets"]
    idx = np.random.default_rng(11).permutation(len(o) - 1)
    t0 = time.perf_counter()
    done = same = close = 0
    for p in idx:
        p = int(p)
        out = multi.match_multi_c(opl, d["qx"][o[p]:o[p + 1]], d["qy"][o[p]:o[p + 1]],
                                  d["I"][o[p]:o[p + 1]].astype(np.float64), n_orient, r_del, nthreads=cores)
        done += 1
        same += all((r is None and res["zone"][p, k] < 0) or
                    (r is not None and (r["zone"], r["n"], r["mirror"]) ==
                     (int(res["zone"][p, k]), int(res["bin"][p, k]), int(res["mirror"][p, k])))
                    for k, r in enumerate(out))
        # the same orientations up to the crystal's symmetry (a strict mismatch may be an exact tie)
        close += all((r is None and res["zone"][p, k] < 0) or
                     (r is not None and res["zone"][p, k] >= 0 and
                      metrics.misorientation_deg(r["orient"], res["orient"][p, k], G) < 0.5)
                     for k, r in enumerate(out))
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    log(f"overlap: oracle on {done} patterns ({el:.1f} s)")
    return ({"value": done / el, "unit": "patterns/s", "cores": cores, "kind": "oracle",
             "sample": f"{done} seeded patterns of the same workload; the oracle's iterative procedure with the "
                       f"plain-C FP64 direct sum over all zones for each of the {n_orient} rounds (OpenMP, "
                       f"{cores} threads); plan build excluded as on the GPU"},
            {"patterns": done, "all_rounds_identical_to_gpu": same,
             "all_rounds_within_0.5deg_of_gpu": close})


def run_overlap(args):
    """Matching of overlapping patterns: a step is one acom_match_multi call over
    all patterns (up to 3 rounds of polar + contraction + exact, the original
    pattern's rescoring and the peak edit)."""
    import numpy as np
    import torch
    import synth
    from paper_2111_00171_amd import acom
    from oracle import metrics

    prec, n_orient, r_del = "bf16", args.rounds, 0.04
    t0 = time.perf_counter()
    d = synth.make("overlap", n=65536, k_max=2.0)
    t_gen = time.perf_counter() - t0
    log(f"overlap: inputs generated ({len(d['offsets']) - 1} patterns, {t_gen:.1f} s)")
    phases, cfg = PLAN_CFG["overlap"]
    gpl = acom.Plan([acom.fcc()], acom.PlanParams(precisions=[prec], **cfg))
    n = len(d["offsets"]) - 1
    pk = acom.Peaks.from_host(d)
    Z, R, N = gpl.n_zones, gpl.n_radial, gpl.n_angular
    flop_per_pattern = bound_flop_per_pattern(gpl, prec)
    ws = torch.empty(gpl.match_multi_workspace_bytes(pk.total_peaks, prec, args.chunk), dtype=torch.uint8,
                     device="cuda")
    shape = gpl.autotune(pk, prec, args.chunk, ws)
    out = gpl.empty_matches(n, n_orient, True, "cuda")
    out["n_evaluated"] = None

    def step():
        gpl.match_multi(pk, n_orient, r_del, 0.01, 0.0, prec, args.chunk, ws, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    acom.profile_begin(8192)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = acom.profile_read()
    acom.profile_end()
    log(f"overlap: timed, {n * args.steps / el:.0f} patterns/s")
    kern = {k: {"avg_ms": (t / c if c else None), "launches": c} for k, (t, c) in prof.items()}
    b = prof["bound"]
    achieved = flop_per_pattern * min(args.chunk, n) / (b[0] / b[1] * 1e-3) / 1e12
    res = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    found = (res["zone"] >= 0).sum(axis=1)
    # the generator's two grains: each within 2 degrees of some found orientation
    G = metrics.cubic_rotations()
    idx = np.random.default_rng(7).choice(n, 1024, replace=False)
    both = one = 0
    for p in idx:
        orients = [res["orient"][p, k] for k in range(n_orient) if res["zone"][p, k] >= 0]
        hit = [any(metrics.misorientation_deg(m, d["truth"][p, j], G) < 2.0 for m in orients) for j in range(2)]
        both += all(hit)
        one += any(hit)
    cpu = check = None
    if not args.no_cpu_baseline:
        cpu, check = cpu_baseline_overlap(d, res, r_del, n_orient)
    roof = {"kernel": "bound_kernel (MFMA contraction, bf16 operands)", "bound": "mfma",
            "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS[prec], 4), "traffic": None,
            "algorithmic_flop_per_launch": flop_per_pattern * min(args.chunk, n),
            "dominant_kernel_of_step": "bound"}
    extra = {"kernel_avg_ms": {k: (None if v["avg_ms"] is None else round(v["avg_ms"], 4)) for k, v in kern.items()},
             "kernel_launches_per_step": {k: v["launches"] / args.steps for k, v in kern.items()},
             "orientations_found_per_pattern": {str(k): int((found == k).sum()) for k in range(n_orient + 1)},
             "grains_recovered_within_2deg": {"both": both / 1024, "at_least_one": one / 1024, "patterns": 1024},
             "oracle_check": check, "contraction_shape": shape, "input_generation_s": round(t_gen, 3)}
    ccfg = {"patterns": n, "peaks": int(d["offsets"][-1]), "zones": Z, "n_radial": R, "n_angular": N,
            "chunk": args.chunk, "rounds": n_orient, "deletion_radius": r_del}
    return line("overlap", n * args.steps / el, el * 1e3 / args.steps, args.steps, args.warmup, "bf16", ccfg, roof,
                cpu, extra)


def run_simulate(args):
    """Forward kinematical patterns: a step is acom_simulate_count, the read of
    the total, and acom_simulate_fill for all orientations."""
    import numpy as np
    import torch
    import synth
    from paper_2111_00171_amd import acom

    n = 65536
    R = synth.haar_rotations(np.random.default_rng(31), n)
    phases, cfg = PLAN_CFG["simulate"]
    gpl = acom.Plan([acom.fcc()], acom.PlanParams(precisions=["fp32"], **cfg))
    orient = torch.tensor(R.reshape(n, 9), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        gpl.simulate(orient)
    torch.cuda.synchronize()
    ev = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for k in ("count", "fill")} for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        off, qx, qy, I = gpl.simulate(orient, events=ev[i])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t_count = sum(e["count"][0].elapsed_time(e["count"][1]) for e in ev) / args.steps
    t_fill = sum(e["fill"][0].elapsed_time(e["fill"][1]) for e in ev) / args.steps
    total = int(off[-1].item())
    log(f"simulate: timed, {n * args.steps / el:.0f} patterns/s, {total / n:.1f} peaks per pattern, "
        f"count call {t_count:.4f} ms, fill call {t_fill:.4f} ms")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import kinematics
        from tests import helpers
        opl = helpers.oracle_plan(phases, **cfg)
        refl = opl["refl"][0]
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 10.0 and k < n:
            kinematics.pattern(refl, R[k], opl["params"].k0, sigma=0.02, rel_cut=0.01)
            k += 1
        cel = time.perf_counter() - t0
        cpu = {"value": k / cel, "unit": "patterns/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} of the same orientations; oracle/kinematics.pattern (numpy FP64, one thread)"}
    # per reflection: rotation 15, excitation error 14 (incl. sqrt and divide), shape factor 4 (incl. exp),
    # cut 1 = 34 operations, for the 536 reflections of the FCC plan (|g| < 2 1/A), in the fill pass
    n_refl = int(np.sum(np.linalg.norm(synth.load_table("fcc_a4.08")["g"], axis=1) < cfg["k_max"]))
    flop = 34.0 * n_refl * n
    tf = flop / (t_fill * 1e-3) / 1e12
    roof = {"kernel": "simulate_kernel<true> (fill: rotate, excitation error, shape factor, ordered compaction)",
            "bound": "alu", "achieved": round(tf, 3), "peak": 157.3, "unit": "TFLOP/s",
            "frac": round(tf / 157.3, 4), "traffic": None, "algorithmic_flop_per_launch": flop,
            "fill_call_ms": round(t_fill, 4), "count_call_ms": round(t_count, 4),
            "note": "one wavefront per pattern; exp, sqrt and divide issue as several instructions each"}
    ccfg = {"patterns": n, "peaks_per_pattern": round(total / n, 2), "k_max": cfg["k_max"]}
    return line("simulate", n * args.steps / el, el * 1e3 / args.steps, args.steps, args.warmup, "f32", ccfg, roof,
                cpu, {"metric": "forward kinematical patterns simulated/sec at 1 GPU"})


def run_detect(args):
    """Bragg disk detection: a step is acom_detect_disks (detection kernel and
    the counts scan) on all frames, the read of the total, and
    acom_gather_peaks into CSR arrays."""
    import numpy as np
    import torch
    import synth
    from paper_2111_00171_amd import acom

    n, U, N = 65536, 4096, 128
    t0 = time.perf_counter()
    d = synth.frames(seed=1007, n=U, size=N)
    log(f"detect: {U} distinct frames generated ({time.perf_counter() - t0:.1f} s)")
    fr = torch.tensor(d["frames"], device="cuda").repeat(n // U, 1, 1).contiguous()
    c = int(d["center"][0])
    prm = dict(edge=4, min_rel=0.005, min_abs=0.0, min_spacing=5, max_peaks=64, exclusion_radius=4.0)
    det = acom.DiskDetector(torch.tensor(d["probe"], device="cuda"), (c, c), d["center"], d["pixel_size"], **prm)
    cap = tuple(torch.empty(n * prm["max_peaks"], dtype=torch.float32, device="cuda") for _ in range(3))
    for _ in range(args.warmup):
        det.gather(det.detect(fr), out=cap)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        res = det.detect(fr)
        ev[i][1].record()
        pk = det.gather(res, out=cap)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t_det = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    total = int(pk.total_peaks)
    log(f"detect: timed, {n * args.steps / el:.0f} frames/s, detection call {t_det:.3f} ms, "
        f"{total / n:.1f} peaks per frame")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import disks
        t = disks.probe_template(d["probe"], c, c)
        kw = dict(edge=4, min_rel=0.005, min_abs=0.0, min_spacing=5, max_peaks=64, cy=d["center"][0],
                  cx=d["center"][1], r_excl=4.0, pixel_size=d["pixel_size"])
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 15.0 and k < U:
            disks.detect(d["frames"][k], t, **kw)
            k += 1
        cel = time.perf_counter() - t0
        cpu = {"value": k / cel, "unit": "frames/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {k} distinct frames; oracle/disks.detect (numpy FP64 direct correlation over "
                         f"the probe's nonzero taps, one thread)"}
    per_frame = N * N * 4 + 16                      # frame read; count, offset, flag
    alg = n * per_frame + total * 12                # + the kept peaks' slots
    gbs = alg / (t_det * 1e-3) / 1e9
    traffic = measured_disk_traffic(n)
    # the kernel is bound by VALU issue (its counters: 68 % of SIMD cycles issue
    # VALU work), so the roof is the vector rate: the correlation's algorithmic
    # FLOP, two real 2-D FFTs (2.5 N^2 log2 N^2 each) and the spectrum product
    # (6 N (N/2 + 1)), against the FP32 vector peak without packed instructions
    # (256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s; the 157.3
    # TFLOP/s figure counts packed FP32, which this build does not emit)
    import math
    fft_flop = 2 * 2.5 * N * N * math.log2(N * N) + 6 * N * (N // 2 + 1)
    tf = fft_flop * n / (t_det * 1e-3) / 1e12
    roof = {"kernel": "disk_detect_kernel<128> (+ the one-block counts scan in the same call)", "bound": "alu",
            "achieved": round(tf, 2), "peak": 78.6, "unit": "TFLOP/s", "frac": round(tf / 78.6, 4),
            "peak_with_packed_fp32": 157.3, "algorithmic_flop_per_frame": fft_flop,
            "traffic": traffic, "algorithmic_bytes_per_launch": alg,
            "hbm_GBps": round(gbs, 1), "hbm_frac": round(gbs / 8000.0, 4),
            "detect_call_ms": round(t_det, 4)}
    ccfg = {"frames": n, "frame": [N, N], "distinct_frames": U, "peaks_per_frame": round(total / n, 2),
            "max_peaks": prm["max_peaks"]}
    out = line("detect", n * args.steps / el, el * 1e3 / args.steps, args.steps, args.warmup, "f32", ccfg, roof,
               cpu, {"metric": "raw diffraction frames reduced to Bragg peak lists/sec at 1 GPU"})
    out["unit"] = "frames/s"
    return out


def run_pipeline(args):
    """Raw frames to orientations: a step is acom_detect_disks, acom_gather_peaks
    into capacity-sized CSR arrays (no host read of the total) and acom_match
    (BF16 contraction, FP32 top-1 rescoring) over all frames."""
    import numpy as np
    import torch
    import synth
    from oracle import metrics
    from paper_2111_00171_amd import acom

    n, U, N = 65536, 4096, 128
    prec = "bf16"
    t0 = time.perf_counter()
    d = synth.frames(seed=1007, size=N, grain_map=(64, 64, 4))  # a 64 x 64 scan of 4 grains
    log(f"pipeline: {U} distinct frames generated ({time.perf_counter() - t0:.1f} s)")
    fr = torch.tensor(d["frames"], device="cuda").repeat(n // U, 1, 1).contiguous()
    c = int(d["center"][0])
    det = acom.DiskDetector(torch.tensor(d["probe"], device="cuda"), (c, c), d["center"], d["pixel_size"], edge=4,
                            min_rel=0.005, min_abs=0.0, min_spacing=5, max_peaks=64, exclusion_radius=4.0)
    phases, cfg = PLAN_CFG["scan"]
    gpl = acom.Plan([acom.fcc()], acom.PlanParams(precisions=[prec], **cfg))
    Z, R, Nphi = gpl.n_zones, gpl.n_radial, gpl.n_angular
    flop_per_pattern = bound_flop_per_pattern(gpl, prec)
    cap = tuple(torch.empty(n * det.max_peaks, dtype=torch.float32, device="cuda") for _ in range(3))
    ws = torch.empty(gpl.match_workspace_bytes(prec, args.chunk), dtype=torch.uint8, device="cuda")
    out = gpl.empty_matches(n, 1, True, "cuda")
    pk = det.gather(det.detect(fr), out=cap, sync=False)
    shape = gpl.autotune(pk, prec, args.chunk, ws)

    def step():
        p = det.gather(det.detect(fr), out=cap, sync=False)
        gpl.match(p, 1, prec, args.chunk, ws, out=out)
        return p

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    acom.profile_begin(8192)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pk = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = acom.profile_read()
    acom.profile_end()
    b_ms = prof["bound"][0] / prof["bound"][1]
    tf = flop_per_pattern * min(args.chunk, n) / (b_ms * 1e-3) / 1e12
    log(f"pipeline: timed, {n * args.steps / el:.0f} frames/s")
    peaks_total = int(pk.offsets[-1].item())
    om = out["orient"][:U, 0].reshape(U, 3, 3).cpu().numpy()
    G = metrics.cubic_rotations()
    idx = np.random.default_rng(11).choice(U, 512, replace=False)
    mis = np.array([metrics.misorientation_deg(om[i], d["truth"][i], G) for i in idx])
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import directsum, disks
        t = disks.probe_template(d["probe"], c, c)
        opl = _oracle_plan("scan")
        kw = dict(edge=4, min_rel=0.005, min_abs=0.0, min_spacing=5, max_peaks=64, cy=d["center"][0],
                  cx=d["center"][1], r_excl=4.0, pixel_size=d["pixel_size"])
        cores = directsum.num_threads()
        m = cores
        t0 = time.perf_counter()
        lists = [disks.detect(d["frames"][i], t, **kw)[:3] for i in range(m)]
        offs = np.zeros(m + 1, np.int64)
        np.cumsum([len(l[0]) for l in lists], out=offs[1:])
        qx, qy, I = (np.concatenate([l[j] for l in lists]).astype(np.float32) for j in range(3))
        directsum.zone_scores(opl, offs, qx, qy, I)
        cel = time.perf_counter() - t0
        cpu = {"value": m / cel, "unit": "frames/s", "cores": cores, "kind": "oracle",
               "sample": f"the first {m} distinct frames: oracle/disks.detect (numpy FP64, one thread) then the "
                         f"plain-C FP64 direct-sum correlation over all {Z} zones (OpenMP, {cores} threads)"}
    roof = {"kernel": "bound_kernel (MFMA contraction, bf16 operands)", "bound": "mfma", "achieved": round(tf, 3),
            "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s", "frac": round(tf / PEAK_TFLOPS[prec], 4), "traffic": None,
            "algorithmic_flop_per_launch": flop_per_pattern * min(args.chunk, n),
            "kernel_avg_ms": {k: (round(t_ / c_, 4) if c_ else None) for k, (t_, c_) in prof.items()}}
    ccfg = {"frames": n, "frame": [N, N], "distinct_frames": U, "peaks_per_frame": round(peaks_total / n, 2),
            "zones": Z, "n_radial": R, "n_angular": Nphi, "chunk": args.chunk, "top_k": 1, "precision": prec}
    extra = {"metric": "raw diffraction frames indexed/sec at 1 GPU (disk detection + BF16 match, FP32 rescoring)",
             "orientation_vs_truth": {"frames": 512, "within_2deg": float(np.mean(mis < 2.0)),
                                      "median_deg": float(np.median(mis))},
             "contraction_shape": shape}
    o = line("pipeline", n * args.steps / el, el * 1e3 / args.steps, args.steps, args.warmup, "bf16", ccfg, roof,
             cpu, extra)
    o["unit"] = "frames/s"
    return o


def oracle_extra_samples(n_threads, n_sample=64):
    """Worker process (no GPU): the oracle plans of FCC, BCC and HCP and the
    plain-C FP64 direct sum of seeded samples of the HCP scan (8281 zones) and
    of the three-phase scan (the three plans concatenated, 10,443 zones)."""
    import numpy as np
    import synth
    from oracle import directsum
    from tests import helpers
    os.environ["OMP_NUM_THREADS"] = str(n_threads)
    cfg = PLAN_CFG["hcp"][1]
    t0 = time.perf_counter()
    plans = {k: helpers.oracle_plan([k], **cfg) for k in ("fcc", "bcc", "hcp")}
    t_plan = time.perf_counter() - t0
    out = {"plan_s": t_plan, "threads": n_threads}
    for name, seed in (("hcp", 3003), ("multi", 3004), ("hard", 3008)):
        d = synth.make(name)
        n = len(d["offsets"]) - 1
        idx = np.sort(np.random.default_rng(seed).choice(n, n_sample, replace=False))
        sub = synth.subset(d, idx)
        if name == "hcp":
            pl = plans["hcp"]
        elif name == "hard":
            pl = plans["fcc"]
        else:
            pl = dict(plans["fcc"])
            pl["P"] = np.concatenate([plans[k]["P"] for k in ("fcc", "bcc", "hcp")])
            pl["M12"] = np.concatenate([plans[k]["M12"] for k in ("fcc", "bcc", "hcp")])
            pl["zone_phase"] = np.concatenate([np.full(len(plans[k]["P"]), i) for i, k in enumerate(("fcc", "bcc", "hcp"))])
        t0 = time.perf_counter()
        zs = directsum.zone_scores(pl, sub["offsets"], sub["qx"], sub["qy"], sub["I"], n_threads)
        el = time.perf_counter() - t0
        # the oracle's top-1 orientation: best zone, its bin and branch, parabolic offset
        from oracle import correlate
        orient = []
        for i in range(n_sample):
            z = int(np.argmax(zs["score"][i]))
            off = correlate.parabolic_offset(zs["cm1"][i, z], zs["score"][i, z], zs["cp1"][i, z])
            orient.append(correlate.orientation(pl["M12"][z], int(zs["n"][i, z]), off, int(zs["mirror"][i, z]),
                                                pl["P"].shape[1]))
        out[name] = {"idx": idx, "score": zs["score"], "n": zs["n"], "mirror": zs["mirror"],
                     "orient": np.array(orient), "seconds": el, "zone_phase": pl["zone_phase"],
                     "peaks": np.diff(sub["offsets"])}
        if name == "multi":
            del pl
    return out


def _single_threaded():
    """Pool initializer: one BLAS / OpenMP thread per worker process."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"


def _refine_one_oracle(args):
    """Pool task: the oracle's refinement of one pattern's candidates."""
    import numpy as np
    from oracle import crystal, score
    from oracle import plan as oplan
    from tests import helpers
    qx, qy, I, cands = args
    refl = crystal.reflections(np.eye(3) * helpers.A_FCC, helpers.FCC_FRAC, 2.0)
    m, S = score.refine(refl, qx, qy, I, list(cands), oplan.Params(k_max=2.0), max_iter=64)
    return m, S


def _agreement(sample, res, prec):
    """Top-1 argmax agreement of the GPU's decisions with the oracle sample
    (tie-aware: within 1e-5 of the oracle's maximum; strict: the same zone, bin
    and branch), and the misorientation between the two top-1 orientations."""
    import numpy as np
    from oracle import metrics
    idx = sample["idx"]
    m = len(idx)
    ok_tie = ok_strict = 0
    mis = []
    zp = sample["zone_phase"]
    for i, p in enumerate(idx):
        sc = sample["score"][i]
        mx = sc.max()
        z = int(res["zone"][p, 0])
        best = int(np.argmax(sc))
        ok_tie += (z >= 0 and sc[z] >= mx - 1e-5 * mx)
        ok_strict += (z == best and int(res["bin"][p, 0]) == int(sample["n"][i][best])
                      and int(res["mirror"][p, 0]) == int(sample["mirror"][i][best]))
        G = metrics.hexagonal_rotations() if zp[best] == 2 or sample.get("hex") else metrics.cubic_rotations()
        if z >= 0 and zp[z] == zp[best]:
            mis.append(metrics.misorientation_deg(res["orient"][p, 0], sample["orient"][i], G))
    return {"tie_aware": ok_tie / m, "strict": ok_strict / m, "patterns": m,
            "patterns_over_128_peaks": int((sample["peaks"] > 128).sum()),
            "misorientation_vs_oracle_deg": {"median": float(np.median(mis)), "max": float(np.max(mis))},
            "precision": prec}


def extra_workloads(args, fut):
    """Short runs of the HCP, three-phase and refinement workloads for the
    default line, each summarised with its rate, kernel times and oracle check."""
    import numpy as np
    import torch
    import synth
    from paper_2111_00171_amd import acom
    from oracle import metrics
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    out = {}
    t_all = time.perf_counter()
    # --- HCP top-8, three contraction precisions
    d = synth.make("hcp")
    n = len(d["offsets"]) - 1
    phases, cfg = PLAN_CFG["hcp"]
    gpl = acom.Plan([acom.hcp()], acom.PlanParams(precisions=["fp32", "bf16", "fp16"], **cfg))
    pk = acom.Peaks.from_host(d)
    fpp = bound_flop_per_pattern(gpl, "bf16")
    runs, host = {}, {}
    t0 = time.perf_counter()
    for prec in ("bf16", "fp16", "fp32"):
        runs[prec], host[prec] = time_match(gpl, pk, prec, 8, args.chunk, 3, 1, n, fpp)
        log(f"hcp (extra): {prec} {runs[prec]['value']:.0f} patterns/s")
    t_hcp = time.perf_counter() - t0
    out["hcp"] = {"workload": DESCR["hcp"], "patterns": n, "zones": gpl.n_zones, "top_k": 8, "steps": 3,
                  "by_precision": by_precision(runs), "timed_s": round(t_hcp, 2),
                  "roofline_bf16": roofline(runs, "bf16", min(args.chunk, n), fpp, None)}
    del gpl, pk
    torch.cuda.empty_cache()
    # --- the scan with degraded peak lists, BF16 and FP32
    dh = synth.make("hard")
    nh = len(dh["offsets"]) - 1
    gpl = acom.Plan([acom.fcc()], acom.PlanParams(precisions=["fp32", "bf16"], **PLAN_CFG["hard"][1]))
    pk = acom.Peaks.from_host(dh)
    fpph = bound_flop_per_pattern(gpl, "bf16")
    runs_h, host_h = {}, {}
    t0 = time.perf_counter()
    for prec in ("bf16", "fp32"):
        runs_h[prec], host_h[prec] = time_match(gpl, pk, prec, 1, args.chunk, 3, 1, nh, fpph)
        log(f"hard (extra): {prec} {runs_h[prec]['value']:.0f} patterns/s")
    out["hard"] = {"workload": DESCR["hard"], "patterns": nh, "peaks_mean": float(np.diff(dh["offsets"]).mean()),
                   "steps": 3, "by_precision": by_precision(runs_h), "timed_s": round(time.perf_counter() - t0, 2)}
    Gc = metrics.cubic_rotations()
    idx_h = np.random.default_rng(7).choice(nh, 256, replace=False)
    mis_h = [metrics.misorientation_deg(host_h["bf16"]["orient"][p, 0], dh["truth"][p], Gc) for p in idx_h]
    out["hard"]["misorientation_vs_truth_deg"] = {"median": float(np.median(mis_h)),
                                                  "within_2deg": float(np.mean(np.array(mis_h) < 2.0)),
                                                  "patterns": 256, "precision": "bf16"}
    del gpl, pk
    torch.cuda.empty_cache()
    # --- three-phase scan, BF16, one HIP graph per step
    d3 = synth.make("multi")
    n3 = len(d3["offsets"]) - 1
    phases, cfg = PLAN_CFG["multi"]
    gpl = acom.Plan([acom.fcc(), acom.bcc(), acom.hcp()],
                    acom.PlanParams(precisions=["bf16"], bound_exact_freqs_16bit=MULTI_KC16, **cfg))
    pk = acom.Peaks.from_host(d3)
    fpp3 = bound_flop_per_pattern(gpl, "bf16")
    t0 = time.perf_counter()
    run3, host3 = time_match(gpl, pk, "bf16", 1, args.chunk, 1, 1, n3, fpp3)
    ws = torch.empty(gpl.match_workspace_bytes("bf16", args.chunk), dtype=torch.uint8, device="cuda")
    o3 = gpl.empty_matches(n3, 1, True, "cuda")
    gpl.match(pk, 1, "bf16", args.chunk, ws, out=o3)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpl.match(pk, 1, "bf16", args.chunk, ws, out=o3)
    g.replay()
    torch.cuda.synchronize()
    steps3 = 3
    t1 = time.perf_counter()
    for _ in range(steps3):
        g.replay()
    torch.cuda.synchronize()
    el3 = time.perf_counter() - t1
    same = bool(np.array_equal(o3["zone"].cpu().numpy(), host3["zone"]))
    t_multi = time.perf_counter() - t0
    log(f"multi (extra): graph replays {n3 * steps3 / el3:.0f} patterns/s")
    out["multi"] = {"workload": DESCR["multi"], "patterns": n3, "zones": gpl.n_zones, "steps": steps3,
                    "bound_exact_freqs_16bit": gpl.bound_split("bf16")[0],
                    "patterns_per_s": round(n3 * steps3 / el3, 1), "ms_per_step": round(el3 * 1e3 / steps3, 3),
                    "graph_replay_matches_eager": same, "eager": by_precision({"bf16": run3})["bf16"],
                    "timed_s": round(t_multi, 2),
                    "roofline_bf16": roofline({"bf16": run3}, "bf16", min(args.chunk, n3), fpp3, None)}
    del g, gpl, pk, ws, o3
    torch.cuda.empty_cache()
    # --- top-4 grid candidates (FP32) + refinement
    dr = synth.make("refine")
    nr = len(dr["offsets"]) - 1
    gpl = acom.Plan([acom.fcc()], acom.PlanParams(precisions=["fp32"], **PLAN_CFG["refine"][1]))
    pk = acom.Peaks.from_host(dr)
    ws = torch.empty(gpl.match_workspace_bytes("fp32", args.chunk), dtype=torch.uint8, device="cuda")
    orr = gpl.empty_matches(nr, 4, True, "cuda")
    gpl.match(pk, 4, "fp32", args.chunk, ws, out=orr)
    gpl.refine(pk, orr["orient"].reshape(nr, 4, 9), max_iter=64)
    torch.cuda.synchronize()
    stepsr, t_m, t_r = 3, 0.0, 0.0
    work = torch.zeros(nr, 2, dtype=torch.int32, device="cuda")
    t0 = time.perf_counter()
    for _ in range(stepsr):
        a = time.perf_counter()
        gpl.match(pk, 4, "fp32", args.chunk, ws, out=orr)
        torch.cuda.synchronize()
        b = time.perf_counter()
        m, S, c = gpl.refine(pk, orr["orient"].reshape(nr, 4, 9), max_iter=64, work=work)
        torch.cuda.synchronize()
        t_r += time.perf_counter() - b
        t_m += b - a
    t_ref = time.perf_counter() - t0
    m = m.cpu().numpy()
    init = orr["orient"].reshape(nr, 4, 3, 3).cpu().numpy()
    G = metrics.cubic_rotations()
    idx_t = np.random.default_rng(9).choice(nr, 512, replace=False)
    mis_t = [metrics.misorientation_deg(m[p], dr["truth"][p], G) for p in idx_t]
    log(f"refine (extra): {nr * stepsr / (t_m + t_r):.0f} patterns/s")
    del gpl, pk, ws, orr
    torch.cuda.empty_cache()
    # --- oracle checks: HCP and three-phase samples from the worker, refinement in a pool
    t0 = time.perf_counter()
    samples = fut.result()
    log(f"extra: oracle samples ready (waited {time.perf_counter() - t0:.1f} s)")
    samples["hcp"]["hex"] = True
    for prec in ("bf16", "fp16", "fp32"):
        out["hcp"]["by_precision"][prec]["argmax_match_vs_oracle"] = _agreement(samples["hcp"], host[prec], prec)
    out["multi"]["argmax_match_vs_oracle"] = _agreement(samples["multi"], host3, "bf16")
    for prec in ("bf16", "fp32"):
        out["hard"]["by_precision"][prec]["argmax_match_vs_oracle"] = _agreement(samples["hard"], host_h[prec], prec)
    zp = samples["multi"]["zone_phase"]
    out["multi"]["argmax_match_vs_oracle"]["phase_equal"] = float(np.mean(
        [zp[int(host3["zone"][p, 0])] == zp[int(np.argmax(samples["multi"]["score"][i]))]
         for i, p in enumerate(samples["multi"]["idx"])]))
    out["oracle_worker"] = {"plan_build_s": round(samples["plan_s"], 1), "threads": samples["threads"],
                            "hcp_sample_s": round(samples["hcp"]["seconds"], 1),
                            "multi_sample_s": round(samples["multi"]["seconds"], 1),
                            "hard_sample_s": round(samples["hard"]["seconds"], 1)}
    o = dr["offsets"]
    idx_r = np.sort(np.random.default_rng(3005).choice(nr, 64, replace=False))
    jobs = [(dr["qx"][o[p]:o[p + 1]].astype(np.float64), dr["qy"][o[p]:o[p + 1]].astype(np.float64),
             dr["I"][o[p]:o[p + 1]].astype(np.float64), init[p]) for p in idx_r]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=max(1, min(16, (os.cpu_count() or 2))), mp_context=mp.get_context("spawn"),
                             initializer=_single_threaded) as ex:
        ores = list(ex.map(_refine_one_oracle, jobs))
    t_or = time.perf_counter() - t0
    mis_o = [metrics.misorientation_deg(m[p], mo, G) for p, (mo, _) in zip(idx_r, ores)]
    dS = [abs(float(S[p]) - So) / abs(So) for p, (_, So) in zip(idx_r, ores)]
    out["refine"] = {"workload": DESCR["refine"], "patterns": nr, "steps": stepsr,
                     "patterns_per_s": round(nr * stepsr / (t_m + t_r), 1),
                     "ms_per_step_match": round(t_m * 1e3 / stepsr, 3), "ms_per_step_refine": round(t_r * 1e3 / stepsr, 3),
                     "refine_roofline": refine_roofline(work, t_r * 1e3 / stepsr),
                     "timed_s": round(t_ref, 2),
                     "refined_vs_truth_deg": {"median": float(np.median(mis_t)), "p90": float(np.percentile(mis_t, 90)),
                                              "patterns": 512},
                     "refined_vs_oracle_refinement_deg": {"median": float(np.median(mis_o)), "max": float(np.max(mis_o)),
                                                          "patterns": len(idx_r), "oracle_pool_s": round(t_or, 1)},
                     "score_vs_oracle_refinement_rel": {"median": float(np.median(dS)), "max": float(np.max(dS))}}
    out["extra_wall_s"] = round(time.perf_counter() - t_all, 1)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="scan", choices=["scan", "hcp", "hard", "multi", "refine", "overlap",
                                                             "simulate", "detect", "pipeline"])
    ap.add_argument("--precisions", default=None,
                    help="comma list; the first is `value` (scan: fp32,bf16,fp16; hcp: bf16,fp16,fp32)")
    ap.add_argument("--chunk", type=int, default=65536,
                    help="patterns per internal launch (65,536: one launch per step on the scan; ~19 GB of workspace)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--bound-exact-freqs", type=int, default=0,
                    help="plan parameter bound_exact_freqs (0: the library's default)")
    ap.add_argument("--bound-block-radii", type=int, default=0,
                    help="plan parameter bound_block_radii (0: the library's default)")
    ap.add_argument("--bound-exact-freqs-16bit", type=int, default=0,
                    help="plan parameter bound_exact_freqs_16bit (0: the library's default)")
    ap.add_argument("--no-extra", action="store_true",
                    help="default run: skip the HCP, three-phase and refinement extra keys")
    ap.add_argument("--rounds", type=int, default=2,
                    help="overlap workload: orientations sought per pattern (the generator draws two grains)")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="first copy this many GiB device-to-device (a plain copy kernel of known size, "
                         "for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); patterns are independent, so a "
              f"multi-GPU run shards the scan into contiguous pattern ranges with no exchange", file=sys.stderr)
        sys.exit(2)
    if args.precisions is None:
        args.precisions = "bf16,fp16,fp32" if args.workload == "hcp" else "fp32,bf16,fp16"

    fut = pool = None
    extra = args.workload == "scan" and not args.no_extra and not args.no_cpu_baseline
    if extra:  # the oracle worker starts before this process touches the GPU
        from concurrent.futures import ProcessPoolExecutor
        import multiprocessing as mp
        pool = ProcessPoolExecutor(max_workers=1, mp_context=mp.get_context("spawn"))
        fut = pool.submit(oracle_extra_samples, max(1, min(16, os.cpu_count() or 2) - 2))
    t_start = time.perf_counter()
    import torch
    if args.calibrate_copy_gib > 0:
        nb = int(args.calibrate_copy_gib * (1 << 30))
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload in ("scan", "hcp", "hard"):
        out = run_match_workload(args, args.workload, defer_oracle=extra)
    elif args.workload == "multi":
        out = run_multi(args)
    elif args.workload == "overlap":
        out = run_overlap(args)
    elif args.workload == "simulate":
        out = run_simulate(args)
    elif args.workload == "detect":
        out = run_detect(args)
    elif args.workload == "pipeline":
        out = run_pipeline(args)
    else:
        out = run_refine(args)
    if extra:
        out["workloads"] = extra_workloads(args, fut)
        pool.shutdown()
        # the scan's oracle baseline, timed once the worker has finished (no
        # other CPU load on the host)
        d, host = out.pop("_deferred")
        out["cpu_baseline"], out["argmax_match_vs_oracle"] = cpu_baseline_match("scan", d, host)
        log("scan: oracle sample timed")
    out["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
