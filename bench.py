"""Benchmark: SymFT per-shot sampling throughput on one MI355X.

Default workload (N=1): rotated surface-code Z-memory, distance 11, 11 rounds,
p = 1e-3 (241 qubits, 1441 records, 1320 detectors, 1 observable), 2^24 shots
per step on the pure-frame path.  One step = one symft_sample call that
writes all 2762 bit-packed rows for 2^24 shots, inputs (the compiled program)
already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
                    [--workload c2|c1|c3|c3fp64|c4|c4fp64|c5|c5fp64|c5k16|post|distill]

Prints one JSON line.  `roofline` prices the dominant kernel against HBM
bandwidth (record bytes written per launch / average launch time, measured
with HIP events on the launch stream); `cpu_baseline` times the CPU oracle
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shots/s on 1 MI355X (batched FP32 vs plain FP64) + % HBM roofline"
HBM_PEAK_GBS = 8000.0
# Measured HBM bytes per launch of the pure-frame kernel on a workload (FETCH_SIZE x 2.000 +
# WRITE_SIZE x 1.000, the scales read off a 1 GiB device copy), kept only while the kernel is
# the one the counters were taken on.
FRAME_TRAFFIC_BYTES = {"surface_d11_r11_p1e-3": (1563095 * 2 + 8400322) * 1024}
# The same for the active kernel with HBM-resident vectors (FP32, 2^16 shots).
ACTIVE_TRAFFIC_BYTES = {"near_clifford_n48_k16": (688241884 * 2 + 1133273003) * 1024}
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def _time_launches(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return t0.elapsed_time(t1) / steps, sum(per) / len(per), wall


LDS_BYTES = 160 * 1024


def _p0_error(prog, seed, n_shots):
    """Largest |Pr(m=0)| difference between the FP32 and FP64 kernels over the active
    measurements of n_shots shots, and how many exceed 1e-5 (the FP64 kernel matches the
    oracle within 1e-12 in the parity tests; a larger difference can only follow a draw that
    fell between the two precisions' thresholds, after which both branches are valid)."""
    import numpy as np
    a = prog.probe(0, n_shots, seed, precision="fp32")
    b = prog.probe(0, n_shots, seed, precision="fp64")
    ok = ~np.isnan(b)
    d = np.abs(a[ok] - b[ok])
    return {"max_abs": float(d.max(initial=0.0)), "over_1e-5": int((d > 1e-5).sum()),
            "measurements": int(d.size), "probed_shots": n_shots}


def _amp_error(prog, seed, n_shots):
    """Largest |amplitude| difference between the FP32 and FP64 kernels over the final active vectors of
    n_shots shots whose records agree in both precisions (a shot whose draw fell between the two
    precisions' thresholds took another branch and is left out; the count is reported)."""
    import numpy as np
    import paper_2607_28600_amd as S
    a32 = prog.probe_amplitudes(0, n_shots, seed, precision="fp32")
    a64 = prog.probe_amplitudes(0, n_shots, seed, precision="fp64")
    r32 = S.bits_to_numpy(prog.sample(n_shots, seed, precision="fp32"))
    r64 = S.bits_to_numpy(prog.sample(n_shots, seed, precision="fp64"))
    same = [s for s in range(n_shots)
            if np.array_equal((r32[:, s // 64] >> np.uint64(s % 64)) & np.uint64(1),
                              (r64[:, s // 64] >> np.uint64(s % 64)) & np.uint64(1))]
    d = np.abs(a32[same] - a64[same]) if same else np.zeros(1)
    return {"max_abs": float(d.max(initial=0.0)), "shots_compared": len(same), "probed_shots": n_shots,
            "amplitudes_per_shot": int(a64.shape[1])}


def _cpu_baseline(circ, seed, words, threads):
    from oracle import OracleCircuit
    oc = OracleCircuit(circ)
    t = time.perf_counter()
    oc.sample_words(seed, words, threads=threads)
    dt = time.perf_counter() - t
    return len(words) * 64 / dt, dt


def run(args):
    import torch
    import paper_2607_28600_amd as S
    from workloads import configs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    cores = os.cpu_count() or 1
    extra = {}
    wl = args.workload
    if wl in ("c1", "c2", "c3", "c3fp64", "c5", "c5fp64", "c5k16"):
        w = {"c1": configs.c1, "c2": configs.c2, "c3": configs.c3, "c3fp64": configs.c3,
             "c5": lambda: configs.c5(14), "c5fp64": lambda: configs.c5(14), "c5k16": lambda: configs.c5(16)}[wl]()
        prec = "fp32" if wl in ("c3", "c5", "c5k16") else "fp64"
        prog = S.Program(w.circuit)
        info = prog.info()
        tps = prog.autotune(prec) if info["k_max"] else 0  # launch configuration, outside the timed region
        words = (w.shots + 63) // 64
        out = torch.empty((prog.n_rows, words), dtype=torch.int64, device="cuda")

        def step():
            prog.sample_into(out, w.shots, w.seed, precision=prec, stream=stream.cuda_stream)

        ms_step, ms_kernel, wall = _time_launches(step, args.steps, args.warmup, stream)
        value = w.shots / (ms_step / 1e3)
        rec_bytes = prog.n_rows * words * 8
        if info["k_max"] == 0:
            achieved = rec_bytes / (ms_kernel / 1e3) / 1e9
            traffic = FRAME_TRAFFIC_BYTES.get(w.name) if w.shots == 1 << 24 else None
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": round(traffic / 1e9, 3) if traffic else None, "traffic_unit": "GB/launch",
                    "kernel": "frame_kernel", "bytes_per_launch": rec_bytes}
            dtype = "u64"
        elif (1 << info["k_max"]) * (8 if prec == "fp32" else 16) > LDS_BYTES or (13 <= info["k_max"] <= 14 and tps != 1024):
            # vectors streamed from HBM scratch (always at peak widths 13 and 14 unless one shot runs per
            # 1024-thread workgroup): one read and one write of the live vector per instruction
            nbytes = info["dense_bytes_per_shot"] * (1 if prec == "fp32" else 2) * w.shots
            achieved = nbytes / (ms_kernel / 1e3) / 1e9
            traffic = ACTIVE_TRAFFIC_BYTES.get(w.name) if prec == "fp32" and w.shots == 1 << 16 else None
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": round(traffic / 1e9, 1) if traffic else None, "traffic_unit": "GB/launch",
                    "kernel": "active_kernel", "bytes_per_launch": nbytes}
            dtype = "f32" if prec == "fp32" else "f64"
        else:
            flops = info["dense_flops_per_shot"] * w.shots
            achieved = flops / (ms_kernel / 1e3) / 1e12
            peak = FP32_PEAK_TFLOPS if prec == "fp32" else FP64_PEAK_TFLOPS
            roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4), "traffic": None, "kernel": "active_kernel",
                    "flops_per_launch": flops}
            dtype = "f32" if prec == "fp32" else "f64"
        if info["k_max"] and prec == "fp32":
            extra["p0_fp32_vs_fp64"] = _p0_error(prog, w.seed, 64)
            extra["amplitude_fp32_vs_fp64"] = _amp_error(prog, w.seed, 64)
        config = {"workload": w.name, "shots": w.shots, "rows": prog.n_rows, "k_max": info["k_max"],
                  "precision": prec if info["k_max"] else "n/a (integer path)"}
        if tps:
            config["threads_per_shot"] = tps
        n_cpu_words = {"c1": 256, "c2": 24, "c3": 64, "c3fp64": 64, "c5": 8, "c5fp64": 8, "c5k16": 2}[wl]
        sample_words = [int(i * words / n_cpu_words) for i in range(n_cpu_words)]
        circ, seed = w.circuit, w.seed
    elif wl in ("c4", "c4fp64"):
        ws = configs.c4()
        progs = [S.Program(x.circuit) for x in ws]
        outs = [torch.empty((p.n_rows, (x.shots + 63) // 64), dtype=torch.int64, device="cuda")
                for p, x in zip(progs, ws)]
        shots = [x.shots for x in ws]
        seeds = [x.seed for x in ws]
        prec = "fp64" if wl == "c4fp64" else "fp32"

        def step():
            S.sample_batch(progs, shots, seeds, outs, precision=prec, graph=True, stream=stream.cuda_stream)

        ms_step, ms_kernel, wall = _time_launches(step, args.steps, args.warmup, stream)
        total = sum(shots)
        value = total / (ms_step / 1e3)

        def plain_fp64():
            for p, x, o in zip(progs, ws, outs):
                p.sample_into(o, x.shots, x.seed, precision="fp64", stream=stream.cuda_stream)

        ms64, _, _ = _time_launches(plain_fp64, max(2, args.steps // 4), 1, stream)
        extra["fp64_per_circuit_launches"] = {"shots_per_s": round(total / (ms64 / 1e3), 1), "ms_per_step": round(ms64, 4)}
        extra[f"batched_{prec}_over_fp64_plain"] = round(ms64 / ms_step, 3)
        flops = sum(p.info()["dense_flops_per_shot"] * s for p, s in zip(progs, shots))
        achieved = flops / (ms_kernel / 1e3) / 1e12
        peak = FP32_PEAK_TFLOPS if prec == "fp32" else FP64_PEAK_TFLOPS
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None, "kernel": "active_kernel"}
        dtype = "f32" if prec == "fp32" else "f64"
        config = {"workload": "batch_128_near_clifford", "shots": total, "programs": len(ws), "precision": prec}
        if prec == "fp32":
            errs = [_p0_error(p, x.seed, 16) for p, x in list(zip(progs, ws))[::16]]
            extra["p0_fp32_vs_fp64"] = {"max_abs": max(e["max_abs"] for e in errs),
                                        "over_1e-5": sum(e["over_1e-5"] for e in errs),
                                        "measurements": sum(e["measurements"] for e in errs),
                                        "probed_shots": sum(e["probed_shots"] for e in errs),
                                        "programs": len(errs)}
        circ, seed = ws[0].circuit, ws[0].seed
        sample_words = list(range(16))
    elif wl in ("post", "distill"):
        # detector postselection with the aggregate-count output: a step is one call that returns the
        # discarded / logical-error flags and their counts for every shot; rejected shots stop their
        # dense work at the rejecting detector
        w = configs.postselect() if wl == "post" else configs.distill()
        prec = "fp32"
        prog = S.Program(w.circuit)
        info = prog.info()
        tps = prog.autotune(prec)
        words = (w.shots + 63) // 64
        post = list(range(prog.n_det))
        tps_counts = prog.autotune_counts(post, precision=prec)  # launch configuration, outside the timing
        flags = torch.empty((2, words), dtype=torch.int64, device="cuda")
        counts = torch.zeros(2, dtype=torch.int64, device="cuda")

        def step():
            prog.sample_counts_into(flags, counts, w.shots, w.seed, post=post, precision=prec,
                                    stream=stream.cuda_stream)

        ms_step, ms_kernel, wall = _time_launches(step, args.steps, args.warmup, stream)
        value = w.shots / (ms_step / 1e3)
        counts.zero_()
        step()
        n_disc, n_log = (int(x) for x in counts.cpu())
        out = torch.empty((prog.n_rows, words), dtype=torch.int64, device="cuda")

        def records():
            prog.sample_into(out, w.shots, w.seed, precision=prec, stream=stream.cuda_stream)

        ms_rec, ms_rec_kernel, _ = _time_launches(records, max(2, args.steps // 2), 1, stream)
        del out
        extra["discarded_fraction"] = round(n_disc / w.shots, 5)
        extra["logical_errors_per_kept_shot"] = round(n_log / max(1, w.shots - n_disc), 6)
        extra["full_records"] = {"shots_per_s": round(w.shots / (ms_rec / 1e3), 1), "ms_per_step": round(ms_rec, 4)}
        extra["counts_over_full_records"] = round(ms_rec / ms_step, 3)
        # the full dense work of every shot, priced on the records launch, which does all of it
        flops = info["dense_flops_per_shot"] * w.shots
        achieved = flops / (ms_rec_kernel / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": None,
                "kernel": "active_kernel (full-records launch)", "flops_per_launch": flops}
        dtype = "f32"
        config = {"workload": w.name, "shots": w.shots, "rows": prog.n_rows, "k_max": info["k_max"],
                  "precision": prec, "threads_per_shot": tps_counts, "threads_per_shot_full_records": tps,
                  "postselected_detectors": len(post),
                  "output": "per-shot discarded / logical-error flags + counts"}
        circ, seed = w.circuit, w.seed
        n_cpu_words = 16 if wl == "post" else 8192  # the width-5 distillation oracle runs ~1e5 shots/s
        sample_words = [int(i * words / n_cpu_words) for i in range(n_cpu_words)]
    else:
        raise SystemExit(f"unknown workload {wl}")

    if args.cpu_baseline:
        cpu_value, cpu_dt = _cpu_baseline(circ, seed, sample_words, threads=cores)
        cpu = {"value": round(cpu_value, 2), "unit": "shots/s", "cores": cores, "kind": "oracle",
               "sample": f"{len(sample_words)} 64-shot words spread over the workload's shot range "
                         f"({len(sample_words) * 64} shots, {cpu_dt:.1f} s)"}
    else:
        cpu = None
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
        "roofline": roof, "cpu_baseline": cpu,
    }
    line["kernel_ms_avg"] = round(ms_kernel, 4)
    if extra:
        line["extra"] = extra
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the sampler runs on one GPU only; shots shard by 64-shot word ranges, "
                                   "so N GPUs would each run this same kernel on 1/N of the words"}))
        raise SystemExit(2)
    run(args)


if __name__ == "__main__":
    main()
