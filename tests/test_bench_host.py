"""Host logic of bench.py (no GPU): the per-class flop accounting against the
credited MTTKRP flops of a sweep, the roofline bound choice, and the digest of
the HBM counter runs (calibration, launch grouping, split-K reductions)."""
import csv
import json

import pytest

import bench
import synth


def test_class_flops_add_up_to_the_sweep():
    """Every class call of one sweep (issue order) adds up to 4 o^2 v^2 R + 14 X v^2 R."""
    for name in ("C1", "C2", "C3", "C5"):
        cfg = synth.CONFIGS[name]
        f = bench.class_flops(cfg)
        total = sum(f[c] for c in bench.SWEEP_GEMMS)
        assert total == pytest.approx(bench.sweep_flops(cfg), rel=1e-12)
        assert set(bench.SWEEP_GEMMS) == set(bench.CLASSES) == set(bench.LAUNCHES)


def test_roofline_takes_the_binding_resource():
    # 1 GB at 8 TB/s (125 us) outweighs 1e11 flop at 2.5 PFLOP/s (40 us): HBM-bound
    r = bench.roofline_for("z", 1e11, 1e9, 0.25)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1e9 / 0.25e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
    # 1e12 flop against 100 MB: MFMA-bound
    r = bench.roofline_for("h", 1e12, 1e8, 1.0)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["frac"] == pytest.approx(1e12 / 1e-3 / 1e12 / bench.PEAK["bf16"])


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Value": v})


def test_digest_groups_launches_and_calibrates(tmp_path):
    """Three calibration copies (FETCH counts half of the copied bytes), a
    warm-up sweep that must be ignored, then two timed sweeps whose GEMM
    launches come LAUNCHES[cls] per call, M and H each followed by their
    split-K reduction."""
    calib_mib = 4
    per_launch = {c: 100.0 + 10 * i for i, c in enumerate(bench.CLASSES)}  # KiB
    reduce_kib = 7.0

    def rows(counter):
        out = [("__amd_rocclr_copyBuffer", calib_mib * 1024 * (0.5 if counter == "fetch" else 1.0))] * 3
        for sweep in range(3):  # sweep 0 is the warm-up
            for cls in bench.SWEEP_GEMMS:
                for _ in range(bench.LAUNCHES[cls]):
                    val = per_launch[cls] if sweep else 9999.0
                    out.append(("gemm_bf16_kernel<128, 128>", val))
                if cls in ("m", "h"):
                    out.append(("splitk_reduce_kernel", reduce_kib))
                out.append(("convert_kernel", 1.0))
        return out

    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fetch, rows("fetch"))
    _write(write, rows("write"))
    out = tmp_path / "t.json"
    bench.digest_counters(str(fetch), str(write), 2, calib_mib, str(out))
    d = json.load(open(out))
    assert d["calibration"]["fetch"]["factor"] == pytest.approx(2.0)
    assert d["calibration"]["write"]["factor"] == pytest.approx(1.0)
    for cls in bench.CLASSES:
        n = bench.LAUNCHES[cls]
        kib = n * per_launch[cls] + (reduce_kib if cls in ("m", "h") else 0.0)
        c = d["classes"][cls]
        assert c["fetch_bytes_per_call"] == pytest.approx(2.0 * kib * 1024)
        assert c["write_bytes_per_call"] == pytest.approx(kib * 1024)
        assert c["bytes_per_launch"] == pytest.approx(3.0 * kib * 1024 / n)
        assert c["calls"] == 2 * bench.SWEEP_GEMMS.count(cls)


def test_dominant_class_breaks_near_ties_toward_the_weaker_kernel():
    """The headline roofline goes to the class taking the most time, except
    that classes within 5 % of it are tied and the one furthest from its own
    roofline is reported; every class keeps its own roofline entry."""
    cfg = synth.CONFIGS["C3"]
    flops, nbytes = bench.class_flops(cfg), bench.class_bytes(cfg)
    ms = {"kr_t2": 4.5, "y": 11.0, "z": 11.2, "m": 6.8, "g": 5.5, "h": 3.6}
    rep = {"ms_class": dict(ms), "n_class": {"kr_t2": 20, "y": 40, "z": 40, "m": 40, "g": 20,
                                             "h": 20}}
    rl = bench.class_rooflines(rep, flops, nbytes)
    assert set(rl) == set(bench.CLASSES)
    # y moves fewer bytes than z in about the same time: further from its roofline
    assert rl["y"]["frac"] < rl["z"]["frac"]
    assert bench.dominant_class(rep, rl) == "y"
    # without a near-tie the largest time share wins
    rep["ms_class"]["z"] = 20.0
    rl = bench.class_rooflines(rep, flops, nbytes)
    assert bench.dominant_class(rep, rl) == "z"
    # per launch: a class call of y is LAUNCHES["y"] launches
    assert rl["y"]["avg_launch_ms"] == pytest.approx(11.0 / (40 * bench.LAUNCHES["y"]))


def test_digest_mfma_groups_launches(tmp_path):
    """Two counters per dispatch (one CSV row each): a warm-up sweep is ignored,
    and each class's utilisation is its summed MFMA-busy cycles over SIMDs x
    its summed active cycles per die."""
    busy = {c: 1000.0 * (i + 1) for i, c in enumerate(bench.CLASSES)}
    path = tmp_path / "m.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        did = 0
        for sweep in range(3):
            for cls in bench.SWEEP_GEMMS:
                for _ in range(bench.LAUNCHES[cls]):
                    b = busy[cls] if sweep else 1e9
                    w.writerow({"Dispatch_Id": did, "Kernel_Name": "gemm_bf16_kernel<...>",
                                "Counter_Name": "SQ_VALU_MFMA_BUSY_CYCLES", "Counter_Value": b})
                    w.writerow({"Dispatch_Id": did, "Kernel_Name": "gemm_bf16_kernel<...>",
                                "Counter_Name": "GRBM_GUI_ACTIVE", "Counter_Value": 10.0})
                    did += 1
                w.writerow({"Dispatch_Id": did, "Kernel_Name": "fit_rows_kernel",
                            "Counter_Name": "GRBM_GUI_ACTIVE", "Counter_Value": 5.0})
                did += 1
    out = tmp_path / "o.json"
    bench.digest_mfma(str(path), 2, str(out), n_cu=4, simd_per_cu=4, n_xcd=8)
    d = json.load(open(out))["classes"]
    for cls in bench.CLASSES:
        assert d[cls]["mfma_util"] == pytest.approx(busy[cls] / (16 * 10.0 / 8))
        assert d[cls]["launches"] == 2 * bench.SWEEP_GEMMS.count(cls) * bench.LAUNCHES[cls]


def test_cpu_baseline_whole_small():
    """The whole-workload CPU baseline forms R and times the requested sweeps
    (run here on the small C1 workload)."""
    cfg = synth.CONFIGS["C1"]
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    out = bench.cpu_baseline_whole(cfg, inp, fs, sweeps=2)
    assert out["kind"] == "oracle" and out["unit"] == "sweeps/s" and out["sweeps"] == 2
    assert out["value"] > 0 and out["r_formation_s"] >= 0 and out["cores"] >= 1
    assert "C1 whole" in out["sample"]
