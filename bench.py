"""Benchmark: mixed-precision matrix-free CP-ALS sweeps of the PPL tensor on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C3]

A step is one ALS sweep of the BF16-operand path (FP32 accumulation; FP64
Grams, block-sweep inverses, solves, normalisation, fit and eta): the four matrix-free
MTTKRP chains and the four factor updates, on synthetic MP2-shaped inputs
already resident in HBM.  The one-time ||R||^2 pass, the FP64 refinement sweep,
the energy contraction and the plain-FP64 comparison are timed separately and
reported beside the headline number.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "ALS sweeps/s + MTTKRP TFLOP/s (o=32,v=256,R=1024); time-to-fit vs plain FP64"
PEAK = {"bf16": 2516.6, "fp64": 78.6}  # dense MFMA TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0
CLASSES = ["kr_t2", "y", "z", "m", "g", "h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
GEMM_SRC = os.path.join(ROOT, "paper_2503_10380_amd", "csrc", "gemm.hip")


def class_flops(cfg):
    """Algorithmic flops of one launch of each MTTKRP kernel class (multiply-add = 2)."""
    o, v, x, r = cfg.o, cfg.v, cfg.nx, cfg.rank
    return {
        "kr_t2": 2.0 * o * o * v * v * r,   # tau = KR(gamma, rho)^T t
        "y": 2.0 * r * x * v * v,           # Y = F^T B
        "z": 2.0 * r * x * v * v,           # per-r Y tau
        "m": 2.0 * r * x * v * v,           # M = B . Z (split-K)
        "g": 2.0 * r * x * v * v,           # per-r G = Y_a^T Y_b
        "h": 2.0 * o * o * v * v * r,       # H = t . G (split-K)
    }


def class_bytes(cfg, esz=2, in_esz=None):
    """Algorithmic HBM bytes per launch: operands read once, result written once.
    esz: bytes per factor / intermediate element; in_esz: per t and B element
    (default esz; 1 for e4m3, whose per-row scales are negligible)."""
    o, v, x, r = cfg.o, cfg.v, cfg.nx, cfg.rank
    ei = esz if in_esz is None else in_esz
    return {
        "kr_t2": esz * (r * o * o + r * v * v) + ei * o * o * v * v,
        "y": esz * (r * v + r * x * v) + ei * x * v * v,
        "z": esz * (r * x * v + r * v * v + r * x * v),
        "m": esz * r * x * v + ei * x * v * v + 8 * r * v,
        "g": esz * (2 * r * x * v + r * v * v),
        "h": esz * r * v * v + ei * o * o * v * v + 8 * r * o * o,
    }


def sweep_flops(cfg):
    o, v, x, r = cfg.o, cfg.v, cfg.nx, cfg.rank
    return 4.0 * o * o * v * v * r + 14.0 * x * v * v * r


def gemm_src_hash():
    with open(GEMM_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel):
    """HBM bytes per launch of a kernel class from committed counter runs, if
    they were taken on the current GEMM source; None otherwise."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    if rec.get("gemm_src_sha256_16") != gemm_src_hash():
        return None
    k = rec.get("classes", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


# BF16 products of one ALS sweep in issue order (main stream).  While a
# side-stream inverse is pending the library cuts tau into four launches and
# Z and G into two (Y and the split-K products stay whole), so a class call is
# LAUNCHES[cls] consecutive BF16 GEMM dispatches (kernels named gemm_bf16*).
SWEEP_GEMMS = ["kr_t2", "z", "m", "y", "z", "m", "y", "g", "h"]
LAUNCHES = {"kr_t2": 4, "y": 1, "z": 2, "g": 2, "m": 1, "h": 1}


def digest_counters(fetch_csv, write_csv, steps, calib_mib, out_path):
    """HBM traffic per MTTKRP kernel class from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
    `bench.py --steps S --warmup W --no-cpu --no-compare --copy-calibration MIB`.
    The last S sweeps' BF16 GEMM dispatches are the timed sweeps, labelled by
    the fixed issue order (LAUNCHES[cls] dispatches per class call); a split-K
    reduction is charged to the GEMM before it.
    Each counter is scaled by (known bytes / counted bytes) of the plain device
    copies of MIB MiB issued first."""
    import csv

    def per_dispatch(path):
        rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
        return [(r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0) for r in rows]

    out = {"gemm_src_sha256_16": gemm_src_hash(), "classes": {}, "calibration": {}}
    per = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        d = per_dispatch(path)
        copies = [b for k, b in d if "copyBuffer" in k or "copy" in k.lower()][:3]
        known = calib_mib * (1 << 20)
        big = [b for b in copies if b > 0.25 * known]
        if not big:
            raise SystemExit(f"no copy-calibration dispatch found in {path}")
        factor = known / (sum(big) / len(big))
        out["calibration"][name] = {"known_bytes": known, "counted_bytes": sum(big) / len(big),
                                    "factor": factor}
        per_sweep = sum(LAUNCHES[c] for c in SWEEP_GEMMS)
        idx = [i for i, (k, _) in enumerate(d) if k.startswith("gemm_bf16")]
        idx = idx[-per_sweep * steps:]
        pos = 0
        for _ in range(steps):
            for cls in SWEEP_GEMMS:
                b = 0.0
                for i in idx[pos:pos + LAUNCHES[cls]]:
                    b += d[i][1]
                    if i + 1 < len(d) and d[i + 1][0].startswith("splitk_reduce_kernel"):
                        b += d[i + 1][1]
                pos += LAUNCHES[cls]
                per.setdefault(cls, {}).setdefault(name, []).append(b * factor)
    for cls, v in per.items():
        f = sum(v["fetch"]) / len(v["fetch"])
        w = sum(v["write"]) / len(v["write"])
        out["classes"][cls] = {"fetch_bytes_per_call": f, "write_bytes_per_call": w,
                               "bytes_per_call": f + w, "calls": len(v["fetch"]),
                               "launches_per_call": LAUNCHES[cls],
                               "bytes_per_launch": (f + w) / LAUNCHES[cls]}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def digest_mfma(csv_path, steps, out_path, n_cu=256, simd_per_cu=4, n_xcd=8):
    """Matrix-core utilisation per MTTKRP kernel class from one rocprofv3 --pmc
    run of SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE (per dispatch) of
    `bench.py --steps S --warmup W --no-cpu --no-compare`: for the last S
    sweeps' BF16 GEMM dispatches (labelled by the fixed issue order as in
    digest_counters).  A 16x16x32 BF16 MFMA counts 16 busy cycles on its SIMD,
    the rate at which 4 SIMDs x 256 CUs at 2.4 GHz give the 2.5 PFLOP/s dense
    peak, and GRBM_GUI_ACTIVE adds the active cycles of the n_xcd dies, so
        util = sum MFMA_BUSY / (simd_per_cu * n_cu * sum GUI_ACTIVE / n_xcd).
    The dispatch timestamps give a second reading of the same fraction at the
    nominal 2.4 GHz clock, and GUI_ACTIVE / n_xcd over the dispatch time gives
    the clock it implies."""
    import csv
    rows = sorted(csv.DictReader(open(csv_path)), key=lambda r: int(r["Dispatch_Id"]))
    per = {}
    for r in rows:
        d = per.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        if r.get("Start_Timestamp") and r.get("End_Timestamp"):
            d["ns"] = float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    disp = [per[k] for k in sorted(per)]
    idx = [i for i, d in enumerate(disp) if d["name"].startswith("gemm_bf16")]
    per_sweep = sum(LAUNCHES[c] for c in SWEEP_GEMMS)
    idx = idx[-per_sweep * steps:]
    acc = {}
    pos = 0
    for _ in range(steps):
        for cls in SWEEP_GEMMS:
            for i in idx[pos:pos + LAUNCHES[cls]]:
                a = acc.setdefault(cls, [0.0, 0.0, 0, 0.0])
                a[0] += disp[i].get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
                a[1] += disp[i].get("GRBM_GUI_ACTIVE", 0.0)
                a[2] += 1
                a[3] += disp[i].get("ns", 0.0)
            pos += LAUNCHES[cls]
    lanes = simd_per_cu * n_cu
    classes = {}
    for c, (busy, gui, n, ns) in acc.items():
        e = {"mfma_busy_cycles": busy, "gui_active_cycles": gui, "launches": n,
             "mfma_util": busy / (lanes * gui / n_xcd) if gui else None}
        if ns:
            e["dispatch_ns"] = ns
            e["mfma_util_at_2p4ghz"] = busy / (lanes * 2.4 * ns)
            e["implied_clock_ghz"] = gui / n_xcd / ns
        classes[c] = e
    out = {"n_cu": n_cu, "simd_per_cu": simd_per_cu, "n_xcd": n_xcd, "classes": classes}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def roofline_for(cls, flops, nbytes, launch_ms):
    """Roofline of one kernel class: bound by whichever of dense-BF16 MFMA time
    and HBM time is larger for its algorithmic flops and bytes."""
    t_mfma = flops / (PEAK["bf16"] * 1e12)
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    sec = launch_ms * 1e-3
    if t_hbm >= t_mfma:
        ach = nbytes / sec / 1e9
        return {"bound": "hbm", "kernel": cls, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": traffic_for(cls),
                "algorithmic_bytes_per_launch": nbytes, "algorithmic_flops_per_launch": flops,
                "avg_launch_ms": launch_ms, "tflops": flops / sec / 1e12}
    ach = flops / sec / 1e12
    return {"bound": "mfma", "kernel": cls, "achieved": ach, "peak": PEAK["bf16"],
            "unit": "TFLOP/s", "frac": ach / PEAK["bf16"], "traffic": traffic_for(cls),
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes,
            "avg_launch_ms": launch_ms, "hbm_gbs": nbytes / sec / 1e9}


def class_rooflines(rep, flops, nbytes):
    """Per-launch roofline of every MTTKRP class from an ALS report with timing."""
    out = {}
    for k in CLASSES:
        n = rep["n_class"][k]
        if not n or rep["ms_class"][k] <= 0:
            continue
        nl = LAUNCHES[k]
        r = roofline_for(k, flops[k] / nl, nbytes[k] / nl, rep["ms_class"][k] / (n * nl))
        r["launches_per_call"] = nl
        r["share_of_mttkrp_time"] = rep["ms_class"][k] / sum(rep["ms_class"][c] for c in CLASSES)
        out[k] = r
    return out


def dominant_class(rep, rooflines, tie=0.05):
    """The class taking the most time; classes within `tie` (relative) of it
    count as tied, and of those the one furthest from its roofline is taken,
    so that a near-tie never hides the weaker kernel."""
    top = max(rooflines, key=lambda k: rep["ms_class"][k])
    tied = [k for k in rooflines if rep["ms_class"][k] >= (1 - tie) * rep["ms_class"][top]]
    return min(tied, key=lambda k: rooflines[k]["frac"])


def cpu_baseline_whole(cfg, inp, fs, sweeps=2):
    """The FP64 oracle on the whole workload: R formed explicitly, then
    `sweeps` textbook ALS sweeps from the seeded start, timed (about 25 s of CPU
    work at o = 32, v = 256, X = 768, R = 1024 on 16 cores)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    t0 = time.perf_counter()
    r = oracle.form_r(inp.t, inp.b_vv)
    t_form = time.perf_counter() - t0
    print(f"cpu baseline: R formed in {t_form:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    oracle.cp_als(r, fs, sweeps, norm_r2=float(np.sum(r * r)))
    t_als = time.perf_counter() - t0
    return {
        "value": sweeps / t_als, "unit": "sweeps/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"{cfg.name} whole: R formed explicitly ({t_form:.1f} s), then {sweeps} textbook "
                   f"FP64 ALS sweeps from the seeded start, timed"),
        "r_formation_s": t_form, "sweeps": sweeps, "als_s": t_als,
    }


def cpu_baseline(cfg, inp, fs, occ=8):
    """The FP64 oracle on a bounded sample: R for the i, j < occ pairs, then one
    textbook ALS sweep on that sub-tensor.  MTTKRP work is linear in the number
    of (i, j) pairs, so it is scaled by (o/occ)^2; the R x R solves are not."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    t0 = time.perf_counter()
    rs = oracle.form_r_pairs(inp.t, inp.b_vv, occ)
    t_form = time.perf_counter() - t0
    sub = [np.array(fs[0][:occ]), np.array(fs[1][:occ]), np.array(fs[2]), np.array(fs[3])]
    t_m = [0.0]

    def timed_mttkrp(factors, mode):
        a = time.perf_counter()
        out = oracle.mttkrp(rs, factors, mode)
        t_m[0] += time.perf_counter() - a
        return out

    t0 = time.perf_counter()
    oracle.cp_als(rs, sub, 1, mttkrp_fn=timed_mttkrp)
    t_sweep = time.perf_counter() - t0
    scale = (cfg.o / occ) ** 2
    sweep_s = scale * t_m[0] + (t_sweep - t_m[0])
    return {
        "value": 1.0 / sweep_s, "unit": "sweeps/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"{cfg.name}: R formed for the {occ}x{occ} occupied pairs i,j<{occ} "
                   f"({occ * occ} of {cfg.o * cfg.o}); one textbook FP64 ALS sweep on that "
                   f"sub-tensor; MTTKRP time x{scale:.0f}, solves as measured"),
        "sweep_s_extrapolated": sweep_s,
        "r_formation_s_extrapolated": t_form * scale,
        "sample_wall_s": t_form + t_sweep,
    }


def cpu_oracle_runs(args):
    """The FP64 oracle on the host cores, per workload: C1 (R formed, 50
    sweeps) and C2 (R formed, 30 sweeps) whole; C3 with R formed whole and two
    sweeps timed; C4 with R formed for the first amplitude step and two sweeps
    timed; C5 extrapolated from the 6 x 6 occupied pairs (1/64 of the pairs:
    R for those pairs and one sweep on that sub-tensor, MTTKRP time x64)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    out = {"cores": int(threads), "cpu_count": os.cpu_count(), "kind": "oracle", "runs": {}}
    for name in ("C1", "C2"):
        cfg = synth.CONFIGS[name]
        inp = synth.make_inputs(cfg)
        fs = synth.init_factors(cfg)
        t0 = time.perf_counter()
        r = oracle.form_r(inp.t, inp.b_vv)
        t_form = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, _, hist = oracle.cp_als(r, fs, cfg.sweeps, norm_r2=float(np.sum(r * r)))
        t_als = time.perf_counter() - t0
        out["runs"][name] = {"r_formation_s": t_form, "sweeps": cfg.sweeps, "als_s": t_als,
                             "sweeps_per_s": cfg.sweeps / t_als, "fit": hist["fit"][-1]}
        print(f"cpu oracle {name}: {json.dumps(out['runs'][name])}", file=sys.stderr, flush=True)
    for name in ("C3", "C4"):
        cfg = synth.CONFIGS[name]
        inp = synth.make_inputs(cfg)
        fs = synth.init_factors(cfg)
        t = inp.t if name == "C3" else inp.t + synth.perturbation(cfg, 0, inp.t)
        print(f"cpu oracle {name}: forming R", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        r = oracle.form_r(t, inp.b_vv)
        t_form = time.perf_counter() - t0
        print(f"cpu oracle {name}: R formed in {t_form:.1f} s", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        _, _, hist = oracle.cp_als(r, fs, 2, norm_r2=float(np.sum(r * r)))
        t_als = time.perf_counter() - t0
        out["runs"][name] = {"r_formation_s": t_form, "sweeps": 2, "als_s": t_als,
                             "sweeps_per_s": 2 / t_als, "fit": hist["fit"][-1]}
        print(f"cpu oracle {name}: {json.dumps(out['runs'][name])}", file=sys.stderr, flush=True)
        del r
    cfg = synth.CONFIGS["C5"]
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    print("cpu oracle C5: 6 x 6 pair sample", file=sys.stderr, flush=True)
    out["runs"]["C5"] = dict(cpu_baseline(cfg, inp, fs, occ=6), extrapolated=True)
    print(f"cpu oracle C5: {json.dumps(out['runs']['C5'])}", file=sys.stderr, flush=True)
    return out


def time_to_fit(cp, torch, cfg, inp, fs, dev_t, dev_b, args):
    """Mixed path vs plain FP64 from a common warm start (the regime of a
    CCSD-like amplitude iteration).  The previous amplitude step is converged
    first (BF16 sweeps to |dfit| < 1e-3, then FP64 sweeps to |dfit| < 1e-6);
    the amplitudes then take one step t -> t + eps_0 (the sequence recipe) and
    both paths restart from those factors: plain FP64 ALS until |dfit| < tol,
    and BF16 sweeps until |dfit| < max(tol, floor) (for tol < 1e-4 the change is
    averaged over 8 sweeps, the BF16 fit having ~2e-6 evaluation noise) followed
    by FP64 refinement sweeps until |dfit| < tol.  Wall time excludes the one-time ||R||^2 pass, which both
    need.  Fit and energy of the mixed path are compared with the FP64 path's."""
    ctx = cp.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "bf16")
    ctx.load_t2(dev_t)
    ctx.load_df(dev_b)
    ctx.set_factors(*fs)
    prep = ctx.als(args.prep_sweeps, stop_rule=1, tol=1e-3, refine=args.prep_sweeps,
                   refine_tol=1e-6)
    state = ctx.get_factors()
    t1 = inp.t + synth.perturbation(cfg, 0, inp.t)
    dev_t1 = torch.tensor(t1, device="cuda")
    ctx.load_t2(dev_t1)
    ctx.norm_r2()
    c64 = cp.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    c64.load_t2(dev_t1)
    c64.load_df(dev_b)
    _, e_exact = c64.norm_r2()
    res = {"protocol": "common warm start after one amplitude step; stop when |dfit| < tol",
           "prep": {"sweeps": prep["sweeps"], "fit": prep["fit"]}, "energy_exact": e_exact}
    for tol in (1e-3, 1e-6):
        ctx.set_factors(*state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # BF16 sweeps until the fit change (averaged over 8 sweeps when tol is near
        # the BF16 noise level) reaches max(tol, floor), then FP64 refinement
        win = 1 if tol >= 1e-4 else 8
        rm = ctx.als(args.max_sweeps, stop_rule=1, tol=max(tol, args.bf16_floor),
                     refine=args.max_sweeps, refine_tol=tol, energy=True, stop_window=win)
        t_mixed = time.perf_counter() - t0
        c64.set_factors(*state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r64 = c64.als(args.max_sweeps, stop_rule=1, tol=tol, energy=True)
        t_64 = time.perf_counter() - t0
        res[f"tol_{tol:g}"] = {
            "fp64": {"sweeps": r64["sweeps"], "wall_s": t_64, "fit": r64["fit"],
                     "energy": r64["energy_cp"]},
            "mixed": {"bf16_sweeps": rm["sweeps"] - rm["refine_sweeps"],
                      "fp64_sweeps": rm["refine_sweeps"], "wall_s": t_mixed, "fit": rm["fit"],
                      "energy": rm["energy_cp"]},
            "speedup": t_64 / t_mixed,
            "fit_rel_diff": abs(rm["fit"] - r64["fit"]) / abs(r64["fit"]),
            "energy_abs_diff": abs(rm["energy_cp"] - r64["energy_cp"]),
            "energy_rel_diff": abs(rm["energy_cp"] - r64["energy_cp"]) / abs(r64["energy_cp"]),
        }
    res["fp64_ms_per_sweep"] = float(np.nanmean(r64["ms_hist"]))
    # the energy criterion (reading P14): both paths run until E_CP changes by
    # less than etol per FP64 sweep (capped at --max-sweeps); the mixed path's
    # BF16 phase stops on the windowed fit floor as above
    etol = args.energy_tol
    ctx.set_factors(*state)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rm = ctx.als(args.max_sweeps, stop_rule=1, tol=args.bf16_floor, stop_window=8,
                 refine=args.max_sweeps, refine_etol=etol, energy=True)
    t_mixed = time.perf_counter() - t0
    c64.set_factors(*state)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r64 = c64.als(args.max_sweeps, stop_rule=3, tol=etol, energy=True)
    t_64 = time.perf_counter() - t0
    eh64 = r64["energy_hist"]
    ehm = rm["energy_hist"][rm["sweeps"] - rm["refine_sweeps"]:]
    res[f"energy_tol_{etol:g}"] = {
        "fp64": {"sweeps": r64["sweeps"], "wall_s": t_64, "fit": r64["fit"],
                 "energy": r64["energy_cp"], "last_energy_change": float(abs(eh64[-1] - eh64[-2])),
                 "capped": r64["sweeps"] >= args.max_sweeps},
        "mixed": {"bf16_sweeps": rm["sweeps"] - rm["refine_sweeps"],
                  "fp64_sweeps": rm["refine_sweeps"], "wall_s": t_mixed, "fit": rm["fit"],
                  "energy": rm["energy_cp"],
                  "last_energy_change": float(abs(ehm[-1] - ehm[-2])) if len(ehm) > 1 else None,
                  "capped": rm["refine_sweeps"] >= args.max_sweeps},
        "speedup": t_64 / t_mixed,
        "fit_rel_diff": abs(rm["fit"] - r64["fit"]) / abs(r64["fit"]),
        "energy_abs_diff": abs(rm["energy_cp"] - r64["energy_cp"]),
        "energy_rel_diff": abs(rm["energy_cp"] - r64["energy_cp"]) / abs(r64["energy_cp"]),
    }
    c64.close()
    ctx.close()
    return res


def workload_leg(cp, torch, cfg, prec, args):
    """Sweep rate and MTTKRP throughput of one more workload and operand
    precision (the same protocol as the headline: --warmup sweeps, then
    --steps timed sweeps from the seeded random factors, then the same number
    with per-class events)."""
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    ctx = cp.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, prec)
    ctx.load_t2(torch.tensor(inp.t, device="cuda"))
    ctx.load_df(torch.tensor(inp.b_vv, device="cuda"))
    del inp
    ctx.norm_r2()
    ctx.set_factors(*fs)
    if args.warmup:
        ctx.als(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.als(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep = ctx.als(args.steps, timing=True)
    ctx.close()
    flops = class_flops(cfg)
    esz = 8 if prec == "fp64" else 2
    nbytes = class_bytes(cfg, esz=esz, in_esz={"fp64": 8, "bf16": 2, "fp8": 1}[prec])
    mt_ms = sum(rep["ms_class"][k] for k in CLASSES)
    tf = sweep_flops(cfg) * args.steps / (mt_ms * 1e-3) / 1e12
    peak = PEAK["fp64"] if prec == "fp64" else PEAK["bf16"]
    per = {}
    for k in CLASSES:
        n = rep["n_class"][k]
        if n and rep["ms_class"][k] > 0:
            sec = rep["ms_class"][k] * 1e-3 / n
            per[k] = {"ms_per_call": sec * 1e3, "tflops": flops[k] / sec / 1e12,
                      "frac_of_dtype_peak": flops[k] / sec / 1e12 / peak,
                      "gbs": nbytes[k] / sec / 1e9, "frac_of_hbm": nbytes[k] / sec / 1e9 / HBM_PEAK_GBS}
    return {"workload": cfg.name, "o": cfg.o, "v": cfg.v, "nx": cfg.nx, "rank": cfg.rank,
            "operands": prec, "sweeps_per_s": args.steps / wall, "ms_per_sweep": wall * 1e3 / args.steps,
            "mttkrp_tflops": tf, "mttkrp_frac_of_dtype_peak": tf / peak,
            "dtype_peak_tflops": peak, "per_class": per, "fit": rep["fit"]}


def _common_warm_start(cp, torch, cfg, inp, fs, dev_b, args):
    """Factors converged on the previous amplitude step (BF16 sweeps to
    |dfit| < 1e-3, then FP64 to 1e-6) and t after one amplitude step."""
    ctx = cp.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "bf16")
    ctx.load_t2(torch.tensor(inp.t, device="cuda"))
    ctx.load_df(dev_b)
    ctx.set_factors(*fs)
    prep = ctx.als(args.prep_sweeps, stop_rule=1, tol=1e-3, refine=args.prep_sweeps,
                   refine_tol=1e-6)
    state = ctx.get_factors()
    ctx.close()
    del ctx
    t1 = inp.t + synth.perturbation(cfg, 0, inp.t)
    return state, t1, prep


def precision_ablation(cp, torch, args):
    """FP64, BF16 and FP8 (e4m3 t and B with power-of-two scales) on one
    workload: sweep rate and per-class kernel times; the MTTKRP error of each
    mode against the FP64 path at the same factors; and, from a common warm
    start after one amplitude step, low-precision sweeps until the fit change
    (averaged over 8 sweeps) is below the precision's floor, then FP64
    refinement until |dfit| < tol, against plain FP64 ALS to the same tol."""
    cfg = synth.CONFIGS[args.config]
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    dev_b = torch.tensor(inp.b_vv, device="cuda")
    state, t1, prep = _common_warm_start(cp, torch, cfg, inp, fs, dev_b, args)
    dev_t = torch.tensor(t1, device="cuda")
    del inp
    tol = args.ablation_tol
    floors = {"bf16": args.bf16_floor, "fp8": args.fp8_floor}
    flops = class_flops(cfg)
    res = {"workload": cfg.name, "o": cfg.o, "v": cfg.v, "nx": cfg.nx, "rank": cfg.rank,
           "protocol": ("rate: --steps sweeps from the warm start after --warmup; mttkrp error: "
                        "all four modes at the warm-start factors vs the FP64 path; fit/energy: "
                        f"low-precision sweeps until |dfit| (8-sweep mean) < floor, then FP64 "
                        f"refinement until |dfit| < {tol:g}, vs FP64 ALS until |dfit| < {tol:g}"),
           "prep_sweeps": prep["sweeps"], "floors": floors, "precisions": {}}
    m64 = None
    ref = None
    for prec in ("fp64", "bf16", "fp8"):
        print(f"ablation: {prec}", file=sys.stderr, flush=True)
        ctx = cp.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, prec)
        ctx.load_t2(dev_t)
        ctx.load_df(dev_b)
        _, e_exact = ctx.norm_r2()
        ctx.set_factors(*state)
        ms = [ctx.mttkrp(m) for m in range(4)]
        if prec == "fp64":
            m64 = ms
        errs = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(ms, m64)]
        if args.warmup:
            ctx.als(args.warmup)
        ctx.set_factors(*state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.als(args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.set_factors(*state)
        rep = ctx.als(args.steps, timing=True)
        nbytes = class_bytes(cfg, esz=8 if prec == "fp64" else 2,
                             in_esz={"fp64": 8, "bf16": 2, "fp8": 1}[prec])
        per_class = {}
        for k in CLASSES:
            n = rep["n_class"][k]
            kms = rep["ms_class"][k]
            if n and kms > 0:
                per_class[k] = {"ms_per_call": kms / n, "tflops": flops[k] * n / (kms * 1e-3) / 1e12,
                                "gbs": nbytes[k] * n / (kms * 1e-3) / 1e9}
        mt_ms = sum(rep["ms_class"][k] for k in CLASSES)
        ctx.set_factors(*state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if prec == "fp64":
            r = ctx.als(args.max_sweeps, stop_rule=1, tol=tol, energy=True)
        else:
            r = ctx.als(args.max_sweeps, stop_rule=1, tol=max(tol, floors[prec]), stop_window=8,
                        refine=args.max_sweeps, refine_tol=tol, energy=True)
        t_fit = time.perf_counter() - t0
        entry = {
            "sweeps_per_s": args.steps / wall, "ms_per_sweep": wall * 1e3 / args.steps,
            "mttkrp_tflops": sweep_flops(cfg) * args.steps / (mt_ms * 1e-3) / 1e12,
            "per_class": per_class,
            "mttkrp_rel_err_vs_fp64": errs,
            "to_tol": {"low_sweeps": r["sweeps"] - r["refine_sweeps"],
                       "fp64_sweeps": r["refine_sweeps"] if prec != "fp64" else r["sweeps"],
                       "wall_s": t_fit, "fit": r["fit"], "energy": r["energy_cp"],
                       "energy_exact": e_exact, "fit_hist": [float(f) for f in r["fit_hist"]]},
        }
        if prec == "fp64":
            ref = entry["to_tol"]
        else:
            entry["to_tol"]["fit_rel_diff"] = abs(r["fit"] - ref["fit"]) / abs(ref["fit"])
            entry["to_tol"]["energy_abs_diff"] = abs(r["energy_cp"] - ref["energy"])
            entry["to_tol"]["energy_rel_diff"] = abs(r["energy_cp"] - ref["energy"]) / abs(ref["energy"])
            entry["to_tol"]["speedup_vs_fp64"] = ref["wall_s"] / t_fit
        res["precisions"][prec] = entry
        print(json.dumps({prec: entry}), file=sys.stderr, flush=True)
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    return res


def warmstart_experiment(cp, torch, args):
    """Learned vs plain vs first-order warm start over a CCSD-like amplitude
    sequence (C4 by default): t^(k+1) = t^(k) + 0.3^e eps_k, 20 steps, with
    e = k (the sequence as specified) or e = k mod 10 (--ws-period 10: later
    steps see the perturbation scales of the early ones).  Every step's
    reference fit fit*_k is that of plain-warm-started FP64 ALS run to
    |dfit| < 1e-9 (at most --ws-cap sweeps); its factors start the next step.
    Steps 1-10 train the per-column network on rows from those converged
    factors; on steps 11-20 each strategy starts from the same previous
    factors and runs FP64 sweeps.  Reported per strategy: the candidate the
    judge kept; the initial relative loss gap (||R - CP||^2 at the start minus
    that at fit*_k, over the latter); sweeps until |fit - fit*_k| / fit*_k <=
    1e-4 (the start itself counting as sweep 0; None if not reached within 60)
    and their wall time including the warm start."""
    cfg = synth.CONFIGS[args.config]
    inp = synth.make_inputs(cfg)
    dev_b = torch.tensor(inp.b_vv, device="cuda")
    ctx = cp.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    ctx.load_t2(torch.tensor(inp.t, device="cuda"))
    ctx.load_df(dev_b)
    ctx.set_factors(*synth.init_factors(cfg))
    t0 = time.perf_counter()
    r0 = ctx.als(args.ws_cap, stop_rule=1, tol=1e-9)
    net = cp.MLP(ctx.ws_in_dim, ctx.ws_out_dim, hidden=256, n_hidden=2,
                 capacity=10 * cfg.rank, seed=7)
    period = args.ws_period or None
    ts = [inp.t] + list(synth.amplitude_sequence(cfg, inp.t, 20, period=period))
    strategies = (("plain", cp.WS_PLAIN), ("first_order", cp.WS_FIRST_ORDER),
                  ("learned", cp.WS_LEARNED))

    def load_step(k):
        ctx.load_t2(torch.tensor(ts[k], device="cuda"))

    def converge_plain(k):
        load_step(k - 1)
        ctx.set_factors(*state)
        ctx.warm_start(ts[k] - ts[k - 1], cp.WS_PLAIN)
        return ctx.als(args.ws_cap, stop_rule=1, tol=1e-9)

    state = ctx.get_factors()
    train_sweeps = []
    for k in range(1, 11):
        r = converge_plain(k)
        train_sweeps.append(r["sweeps"])
        ctx.training_rows(net)
        state = ctx.get_factors()
        print(f"warmstart: training step {k}: {r['sweeps']} sweeps", file=sys.stderr, flush=True)
    t_train = time.perf_counter()
    net.standardize()
    hist = net.train(args.ws_epochs, lr=1e-3, batch=512, seed=1)
    t_train = time.perf_counter() - t_train
    rows = []
    for k in range(11, 21):
        prev = state
        ref = converge_plain(k)
        fit_star = ref["fit"]
        n2 = ctx.norm_r2()[0]
        f_s, inner_s, cp2_s = ctx.fit()
        res2_star = n2 - 2 * inner_s + cp2_s
        state = ctx.get_factors()
        row = {"fit_star": fit_star, "ref_sweeps": ref["sweeps"]}
        for name, strat in strategies:
            load_step(k - 1)
            ctx.set_factors(*prev)
            torch.cuda.synchronize()
            a = time.perf_counter()
            chosen = ctx.warm_start(ts[k] - ts[k - 1], strat, net if strat == cp.WS_LEARNED else None)
            torch.cuda.synchronize()
            ws_s = time.perf_counter() - a
            f0, inner0, cp20 = ctx.fit()
            rep = ctx.als(60)
            h = np.concatenate([[f0], rep["fit_hist"]])
            ok = np.abs(h - fit_star) / abs(fit_star) <= 1e-4
            n = int(np.argmax(ok)) if np.any(ok) else None
            wall = None if n is None else ws_s + float(np.sum(rep["ms_hist"][:n])) * 1e-3
            row[name] = {"chosen": int(chosen), "fit0": float(f0),
                         "loss_gap0": float((n2 - 2 * inner0 + cp20 - res2_star) / res2_star),
                         "sweeps_to_1e-4": n, "wall_s_to_1e-4": wall, "warm_start_s": ws_s}
        rows.append(row)
        print(f"warmstart: evaluation step {k}: " + ", ".join(
            f"{name} chosen {row[name]['chosen']} gap {row[name]['loss_gap0']:.3e}"
            for name, _ in strategies), file=sys.stderr, flush=True)
    summary = {}
    for name, _ in strategies:
        ns = [r[name]["sweeps_to_1e-4"] for r in rows]
        summary[name] = {
            "chosen_non_plain": int(sum(r[name]["chosen"] != cp.WS_PLAIN for r in rows)),
            "reached": int(sum(n is not None for n in ns)),
            "mean_sweeps_to_1e-4": float(np.mean([61 if n is None else n for n in ns])),
            "mean_wall_s_to_1e-4": float(np.mean([r[name]["wall_s_to_1e-4"] or np.nan
                                                  for r in rows])),
            "median_loss_gap0": float(np.median([r[name]["loss_gap0"] for r in rows])),
        }
    ctx.close()
    return {"metric": "warm start over an amplitude sequence: sweeps to |fit - fit*|/fit* <= 1e-4 "
                      "and initial loss gap, steps 11-20",
            "config": {"workload": cfg.name, "o": cfg.o, "v": cfg.v, "nx": cfg.nx,
                       "rank": cfg.rank, "als": "fp64", "decay_period": period},
            "step0": {"sweeps": r0["sweeps"], "fit": r0["fit"]},
            "train": {"steps": 10, "sweeps_per_step": train_sweeps, "rows": net.num_rows,
                      "epochs": args.ws_epochs, "loss_first": float(hist[0]),
                      "loss_last": float(hist[-1]), "loss_ratio": float(hist[0] / hist[-1]),
                      "train_s": t_train, "standardized": True},
            "summary": summary, "steps": rows,
            "wall_s": time.perf_counter() - t0}


def ccd_experiment(cp, torch, args):
    """The CCD-like Jacobi iteration on the pair-symmetrised CP ladder (C2 by
    default): t^(k) = (w + s R~(t^(k-1))) / D from the MP2 amplitudes, ALS to
    |dfit| < --ccd-tol per CC step (at most --ccd-cap sweeps, FP64), for each of
    the paper's three initial guesses.  Reported per CC step: ALS sweeps, fit,
    the guess used, E = <w, t> and its change, and ||dt|| (E and ||dt|| are
    diagnostics computed with torch on the amplitudes the library returns)."""
    cfg = synth.CONFIGS[args.config]
    inp = synth.make_inputs(cfg)
    w = synth.exchange_integrals(inp)
    s = synth.ccd_scale(inp)
    dev = [torch.tensor(x, device="cuda") for x in (w, inp.e_occ, inp.e_vir)]
    out = {"metric": "CCD-like Jacobi loop with the CP ladder: ALS sweeps per CC step by initial guess",
           "config": {"workload": cfg.name, "o": cfg.o, "v": cfg.v, "nx": cfg.nx, "rank": cfg.rank,
                      "als": "fp64", "tol": args.ccd_tol, "cap": args.ccd_cap,
                      "cc_steps": args.ccd_steps, "scale": s},
           "guesses": {}}
    for guess in cp.GUESSES:
        ctx = cp.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
        ctx.load_t2(torch.tensor(inp.t, device="cuda"))
        ctx.load_df(torch.tensor(inp.b_vv, device="cuda"))
        t_cur = torch.tensor(inp.t, device="cuda")
        e_prev = float(torch.sum(dev[0] * t_cur))
        rows = []

        def on_step(k, dt, rec):
            nonlocal t_cur
            t_cur = t_cur + dt
            rec["energy"] = float(torch.sum(dev[0] * t_cur))
            rec["dt_norm"] = float(torch.linalg.vector_norm(dt))

        t0 = time.perf_counter()
        hist = cp.ccd_loop(ctx, *dev, s, args.ccd_steps, guess=guess, seed=11, tol=args.ccd_tol,
                           max_sweeps=args.ccd_cap, on_step=on_step)
        wall = time.perf_counter() - t0
        for h in hist:
            h["d_energy"] = h["energy"] - e_prev
            e_prev = h["energy"]
            rows.append(h)
        ctx.close()
        later = [h["sweeps"] for h in rows[1:]]
        out["guesses"][guess] = {
            "steps": rows, "wall_s": wall,
            "sweeps_first_step": rows[0]["sweeps"],
            "mean_sweeps_later_steps": float(np.mean(later)) if later else None,
            "fit_first": rows[0]["fit"], "fit_last": rows[-1]["fit"],
            "last_abs_d_energy": abs(rows[-1]["d_energy"]),
        }
        print(json.dumps({guess: out["guesses"][guess]["mean_sweeps_later_steps"]}), file=sys.stderr,
              flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default=None,
                    help="workload (default C3; C4 for --experiment warmstart, C5 for precision)")
    ap.add_argument("--prep-sweeps", type=int, default=60,
                    help="cap on the BF16 and on the FP64 sweeps that converge the previous step")
    ap.add_argument("--bf16-floor", type=float, default=1e-6,
                    help="smallest (window-averaged) fit change the BF16 phase waits for")
    ap.add_argument("--energy-tol", type=float, default=1e-9,
                    help="time-to-fit energy leg: stop when |E_n - E_{n-1}| < this (Ha)")
    ap.add_argument("--max-sweeps", type=int, default=200,
                    help="cap on the sweeps of each time-to-fit run (and on the refinement)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--legs", default="C2:fp64,C5:bf16,C5:fp8",
                    help="extra workload:precision legs reported beside the headline "
                         "('' for none)")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--fp8-floor", type=float, default=1e-4,
                    help="precision ablation: fit-change floor of the FP8 sweeps")
    ap.add_argument("--ablation-tol", type=float, default=1e-5,
                    help="precision ablation: |dfit| tolerance of the FP64 phase")
    ap.add_argument("--ccd-steps", type=int, default=10)
    ap.add_argument("--ccd-tol", type=float, default=1e-3,
                    help="ccd: ALS stop |dfit| < tol per CC step (the paper's 1e-3)")
    ap.add_argument("--ccd-cap", type=int, default=100)
    ap.add_argument("--experiment", choices=["warmstart", "precision", "ccd", "cpu"],
                    help="warmstart: the learned warm-start experiment (C4 unless --config); "
                         "precision: the FP64 / BF16 / FP8 ablation (C5 unless --config)")
    ap.add_argument("--ws-epochs", type=int, default=300)
    ap.add_argument("--ws-cap", type=int, default=500,
                    help="warmstart: sweep cap of the |dfit| < 1e-9 reference runs")
    ap.add_argument("--ws-period", type=int, default=0,
                    help="warmstart: 0 = decay 0.3^k as specified, 10 = 0.3^(k mod 10)")
    ap.add_argument("--digest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this "
                         "script into profiles/traffic_counters.json and exit")
    ap.add_argument("--digest-mfma", metavar="CSV",
                    help="summarise a rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE "
                         "run of this script into profiles/mfma_busy_c3.json and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run three plain device copies of MIB MiB each, so that "
                         "HBM byte counters can be scaled against a kernel of known traffic")
    args = ap.parse_args()
    if args.experiment == "warmstart":
        import torch
        import paper_2503_10380_amd as cp
        args.config = args.config or "C4"
        print(json.dumps(warmstart_experiment(cp, torch, args)))
        return
    if args.experiment == "cpu":
        print(json.dumps(cpu_oracle_runs(args)))
        return
    if args.experiment == "ccd":
        import torch
        import paper_2503_10380_amd as cp
        args.config = args.config or "C2"
        print(json.dumps(ccd_experiment(cp, torch, args)))
        return
    if args.experiment == "precision":
        import torch
        import paper_2503_10380_amd as cp
        args.config = args.config or "C5"
        print(json.dumps(precision_ablation(cp, torch, args)))
        return
    if args.digest_mfma:
        digest_mfma(args.digest_mfma, args.steps, os.path.join(ROOT, "profiles", "mfma_busy_c3.json"))
        return
    if args.digest_counters:
        digest_counters(args.digest_counters[0], args.digest_counters[1], args.steps,
                        args.copy_calibration, TRAFFIC_FILE)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the sharded design over rank columns is described, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2503_10380_amd as cp

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy calibration: 3 copies of {args.copy_calibration} MiB", file=sys.stderr)
        del src, dst

    cfg = synth.CONFIGS[args.config or "C3"]
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    dev_t = torch.tensor(inp.t, device="cuda")
    dev_b = torch.tensor(inp.b_vv, device="cuda")

    ctx = cp.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "bf16")
    ctx.load_t2(dev_t)
    ctx.load_df(dev_b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norm_r2, e_exact = ctx.norm_r2()
    s0_ms = (time.perf_counter() - t0) * 1e3

    ctx.set_factors(*fs)
    if args.warmup:
        ctx.als(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep_plain = ctx.als(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    # per-kernel-class HIP-event timings come from a second pass of the same
    # length (the events add a little time between kernels)
    rep = ctx.als(args.steps, timing=True)

    flops = class_flops(cfg)
    nbytes = class_bytes(cfg)
    per_class = {}
    for k in CLASSES:
        n = rep["n_class"][k]
        ms = rep["ms_class"][k]
        per_class[k] = {"calls": n, "launches_per_call": LAUNCHES[k], "ms_total": ms,
                        "ms_per_call": ms / n if n else None,
                        "tflops": (flops[k] * n / (ms * 1e-3) / 1e12) if ms > 0 else None}
    per_class["solve"] = {"launches": rep["n_class"]["solve"], "ms_total": rep["ms_class"]["solve"]}
    per_class["fit"] = {"launches": rep["n_class"]["fit"], "ms_total": rep["ms_class"]["fit"]}
    per_class["inv"] = {"launches": rep["n_class"]["inv"], "ms_total": rep["ms_class"]["inv"],
                        "note": "W^-1 on the side stream for alpha/beta/gamma (overlapped)"}
    mttkrp_ms = sum(rep["ms_class"][k] for k in CLASSES)
    mttkrp_tflops = sweep_flops(cfg) * args.steps / (mttkrp_ms * 1e-3) / 1e12
    rooflines = class_rooflines(rep, flops, nbytes)
    dom = dominant_class(rep, rooflines)
    roofline = dict(rooflines[dom])
    for k in CLASSES:
        if per_class[k]["ms_per_call"]:
            r = rooflines[k]
            per_class[k].update({"bound": r["bound"], "frac": r["frac"],
                                 "gbs": nbytes[k] / (per_class[k]["ms_per_call"] * 1e-3) / 1e9})

    out = {
        "metric": METRIC, "value": args.steps / wall, "unit": "sweeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic MP2-shaped inputs (seeded DF tensor, orbital energies, MP2 amplitudes)",
        "config": {"workload": f"{cfg.name}: mixed-precision CP-ALS sweep of the DF-PPL tensor",
                   "o": cfg.o, "v": cfg.v, "nx": cfg.nx, "rank": cfg.rank,
                   "operands": "bf16", "accumulate": "fp32", "solve": "fp64"},
        "roofline": roofline,
        "roofline_per_class": {k: {f: r[f] for f in ("bound", "achieved", "unit", "frac",
                                                     "avg_launch_ms", "share_of_mttkrp_time")}
                               for k, r in rooflines.items()},
        "roofline_lowest": min(rooflines, key=lambda k: rooflines[k]["frac"]),
        "mttkrp_tflops": mttkrp_tflops,
        "mttkrp_frac_of_bf16_peak": mttkrp_tflops / PEAK["bf16"],
        "per_class": per_class,
        "fit_after_timed_sweeps": rep_plain["fit"],
        "ms_per_step_with_class_events": float(np.sum(rep["ms_hist"]) / rep["sweeps"]),
        "s0_norm_r2_ms": s0_ms,
        "norm_r2": norm_r2, "energy_exact": e_exact,
    }

    if not args.no_compare:
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        out["time_to_fit"] = time_to_fit(cp, torch, cfg, inp, fs, dev_t, dev_b, args)
    if args.legs:
        if "ctx" in locals():
            ctx.close()
            del ctx
        del dev_t, dev_b
        torch.cuda.empty_cache()
        out["legs"] = {}
        for leg in args.legs.split(","):
            name, prec = leg.split(":")
            print(f"leg {leg}", file=sys.stderr, flush=True)
            out["legs"][leg] = workload_leg(cp, torch, synth.CONFIGS[name], prec, args)
            torch.cuda.empty_cache()
    if not args.no_cpu:
        # whole up to C3's size (R 0.5 GB, ~25 s), else the pair sample
        whole = cfg.o ** 2 * cfg.v ** 2 * 8 <= (1 << 30)
        out["cpu_baseline"] = cpu_baseline_whole(cfg, inp, fs) if whole else cpu_baseline(cfg, inp, fs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
