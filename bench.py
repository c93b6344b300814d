"""Benchmark: SymFT per-shot sampling throughput on one MI355X.

Default workload (N=1): rotated surface-code Z-memory, distance 11, 11 rounds,
p = 1e-3 (241 qubits, 1441 records, 1320 detectors, 1 observable), 2^24 shots
per step on the pure-frame path.  One step = one symft_sample call that
writes all 2762 bit-packed rows for 2^24 shots, inputs (the compiled program)
already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-extras]
                    [--workload c2|c1|c3|c3fp64|c4|c4fp64|c5|c5fp64|c5k16|c5k16fp64|post|distill]

Prints one JSON line.  `roofline` prices the dominant kernel against its
bound (record bytes written per launch / average launch time for the frame
kernel, measured with HIP events on the launch stream).  The default line's
`extra` also carries the batched-FP32 vs per-circuit-FP64 comparison on the
128-program batch (both sides autotuned) and the step-synchronous frame
kernel's time.  The oracle leg (`cpu_baseline`, on unless --no-cpu-baseline)
times the CPU oracle on a bounded sample of the same workload and reports
the kernels' branch-probability and amplitude errors against the FP64 oracle
per configuration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shots/s on 1 MI355X (batched FP32 vs plain FP64) + % HBM roofline"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
LDS_BYTES = 160 * 1024
CSRC = os.path.join(ROOT, "paper_2607_28600_amd", "csrc")

# HBM bytes per launch measured with rocprofv3 (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 KiB, the scales
# read off a 1 GiB device copy; profiles/ holds the runs), keyed by (workload, kernel source), with the
# first 16 hex digits of the SHA-256 of the sources they were taken on (see _HEADERS).  A changed source
# reports traffic null until it is profiled again.
PROFILED_TRAFFIC = {
    ("surface_d11_r11_p1e-3", "sample_frame.hip"): ("9868ee569723208d", 13214566208),
}
# the kernel sources a traffic figure depends on: the kernel file, the shared headers and the host code that
# lays out the device program
_HEADERS = ["device_program.hpp", "launch_args.hpp", "philox.hpp", "frame_device.hpp", "frame_schedule.cpp", "capi.cpp"]


def _source_sha(name):
    h = hashlib.sha256()
    for f in [name] + _HEADERS:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _flops_per_shot(info):
    """Algorithmic flops per shot of the representation the program samples with: its product components
    (merges included) when selected, else the dense vector."""
    return info["product_flops_per_shot"] if info["product_selected"] else info["dense_flops_per_shot"]


def _representation(info):
    return "product components" if info["product_selected"] else "dense vector"


def _traffic(workload, source):
    rec = PROFILED_TRAFFIC.get((workload, source))
    if rec is None or _source_sha(source)[:16] != rec[0]:
        return None
    return rec[1]


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
    t0.record(stream)
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return t0.elapsed_time(t1) / steps, sum(per) / len(per)


def _c4_comparison(S, stream, steps, prec="fp32"):
    """The 128-program batch in one persistent graph-replayed launch (threads per shot from the batch
    autotuner) against 128 per-circuit plain FP64 launches, each program autotuned for FP64 first.
    Both launch configurations are chosen outside the timed region."""
    import torch
    from workloads import configs
    ws = configs.c4()
    progs = [S.Program(x.circuit) for x in ws]
    outs = [torch.empty((p.n_rows, (x.shots + 63) // 64), dtype=torch.int64, device="cuda")
            for p, x in zip(progs, ws)]
    shots = [x.shots for x in ws]
    seeds = [x.seed for x in ws]
    total = sum(shots)

    def batched():
        S.sample_batch(progs, shots, seeds, outs, precision=prec, graph=True, stream=stream.cuda_stream)

    ms_b, ms_b_kernel = _time_launches(batched, steps, 2, stream)
    for p in progs:
        p.autotune("fp64")

    def plain_fp64():
        for p, x, o in zip(progs, ws, outs):
            p.sample_into(o, x.shots, x.seed, precision="fp64", stream=stream.cuda_stream)

    ms_64, _ = _time_launches(plain_fp64, max(2, steps // 2), 1, stream)
    flops = sum(_flops_per_shot(p.info()) * s for p, s in zip(progs, shots))
    # the same batch with every member on the dense vector (symft_compile_opts.components = 1)
    dense = [S.Program(x.circuit, components="off") for x in ws]

    def batched_dense():
        S.sample_batch(dense, shots, seeds, outs, precision=prec, graph=True, stream=stream.cuda_stream)

    ms_bd, _ = _time_launches(batched_dense, max(2, steps // 2), 1, stream)
    n_prod = sum(p.info()["product_selected"] for p in progs)
    return {
        "shots": total, "programs": len(ws),
        f"batched_{prec}": {"ms_per_step": round(ms_b, 3), "shots_per_s": round(total / (ms_b / 1e3), 1),
                            "tflops": round(flops / (ms_b_kernel / 1e3) / 1e12, 3)},
        "per_circuit_fp64_autotuned": {"ms_per_step": round(ms_64, 3), "shots_per_s": round(total / (ms_64 / 1e3), 1)},
        f"batched_{prec}_over_per_circuit_fp64": round(ms_64 / ms_b, 3),
        "members_on_product_components": n_prod,
        f"batched_{prec}_dense_vector": {"ms_per_step": round(ms_bd, 3), "shots_per_s": round(total / (ms_bd / 1e3), 1)},
    }, (progs, ws, flops, ms_b_kernel)


# ------------------------------------------------------------------ oracle leg
def _cpu_baseline(circ, seed, words, threads):
    from oracle import OracleCircuit
    oc = OracleCircuit(circ)
    t = time.perf_counter()
    oc.sample_words(seed, words, threads=threads)
    dt = time.perf_counter() - t
    return len(words) * 64 / dt, dt


def _errors_vs_oracle(prog, w, n_p0, n_amp):
    """Branch-probability and final-amplitude errors of the kernels (FP32 and FP64) against the FP64
    oracle on the first shots of a workload.  Pr(m = 0) is compared on every active measurement up to a
    shot's first draw within 1e-5 of the oracle's threshold (past it the branches may differ); final
    amplitudes on shots whose records equal the oracle's, up to the Pauli-frame map the two
    representations differ by (index shift, sign character, global phase)."""
    import numpy as np
    import paper_2607_28600_amd as S
    from oracle import OracleCircuit
    from tests.parity_util import frame_match, p0_error
    oc = OracleCircuit(w.circuit)
    res = {}
    s0 = 64 * 3 + 5
    shots = list(range(s0, s0 + n_p0))
    want = oc.sample(w.seed, 64)
    for prec in ("fp32", "fp64"):
        p0 = prog.probe(s0, n_p0, w.seed, precision=prec)
        worst, cnt = p0_error(p0, oc, w.seed, shots, 1e-5)
        amp = prog.probe_amplitudes(0, n_amp, w.seed, precision=prec)
        rec = S.bits_to_numpy(prog.sample(64, w.seed, precision=prec))
        amp_err, checked, unmatched = 0.0, 0, 0
        for s in range(n_amp):
            bit = np.uint64(s)
            if not np.array_equal((rec[:, 0] >> bit) & np.uint64(1), (want[:, 0] >> bit) & np.uint64(1)):
                continue
            fs = oc.final_state(w.seed, s)
            m = frame_match(amp[s], fs["alpha"], 1e-4 if prec == "fp32" else 1e-9)
            if m is None:
                unmatched += 1
                continue
            amp_err = max(amp_err, m[2])
            checked += 1
        res[prec] = {"p0_max_abs_err": worst, "p0_compared": cnt, "amp_max_abs_err": amp_err,
                     "amp_shots": checked, "amp_shots_unmatched": unmatched,
                     "amplitudes_per_shot": int(amp.shape[1])}
    return res


def _oracle_errors_all(S):
    """Errors against the FP64 oracle for the near-Clifford configurations: C3, four C4 programs (widths
    4, 8, 12, 12), C5 at widths 14 and 16."""
    from workloads import configs
    out = {}
    cases = [("c3", configs.c3(), 24, 16)]
    c4 = configs.c4()
    cases += [(f"c4_{i}", c4[i], 8, 8) for i in (3, 7, 11, 59)]
    cases += [("c5_k14", configs.c5(14), 8, 4), ("c5_k16", configs.c5(16), 4, 2)]
    for name, w, n_p0, n_amp in cases:
        prog = S.Program(w.circuit)
        out[name] = _errors_vs_oracle(prog, w, n_p0, n_amp)
        out[name]["k_max"] = prog.k_max
    return out


# ------------------------------------------------------------------ workloads
def run(args):
    import torch
    import paper_2607_28600_amd as S
    from workloads import configs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    cores = os.cpu_count() or 1
    extra = {}
    errors_for = None  # workload whose errors the oracle leg reports
    wl = args.workload
    single = {"c1": (configs.c1, "fp64"), "c2": (configs.c2, "fp64"), "c3": (configs.c3, "fp32"),
              "c3fp64": (configs.c3, "fp64"), "c5": (lambda: configs.c5(14), "fp32"),
              "c5fp64": (lambda: configs.c5(14), "fp64"), "c5k16": (lambda: configs.c5(16), "fp32"),
              "c5k16fp64": (lambda: configs.c5(16), "fp64")}
    if wl in single:
        make, prec = single[wl]
        w = make()
        prog = S.Program(w.circuit)
        info = prog.info()
        tps = prog.autotune(prec) if info["k_max"] else 0  # launch configuration, outside the timed region
        words = (w.shots + 63) // 64
        out = torch.empty((prog.n_rows, words), dtype=torch.int64, device="cuda")

        def step():
            prog.sample_into(out, w.shots, w.seed, precision=prec, stream=stream.cuda_stream)

        ms_step, ms_kernel = _time_launches(step, args.steps, args.warmup, stream)
        value = w.shots / (ms_step / 1e3)
        rec_bytes = prog.n_rows * words * 8
        dtype = "u64" if info["k_max"] == 0 else ("f32" if prec == "fp32" else "f64")
        if info["k_max"] == 0:
            # the automatic choice for this call: small calls of small schedules take the wave-owned kernel
            fk = 1 if words <= int(info["frame_small_words"]) else int(info["frame_kernel"])
            kname, src = ("frame_wave_kernel", "sample_frame_wave.hip") if fk == 1 else ("frame_kernel", "sample_frame.hip")
            achieved = rec_bytes / (ms_kernel / 1e3) / 1e9
            traffic = _traffic(w.name, src) if w.shots == 1 << 24 else None
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": round(traffic / 1e9, 3) if traffic else None, "traffic_unit": "GB/launch",
                    "kernel": kname, "bytes_per_launch": rec_bytes}
            if args.extras and fk in (1, 2):
                # the other pure-frame kernel on the same launch, for comparison
                other = 2 if fk == 1 else 1

                def other_kernel():
                    prog.sample_into(out, w.shots, w.seed, stream=stream.cuda_stream, frame_kernel=other)
                key = "step_synchronous_frame_kernel" if other == 2 else "wave_owned_frame_kernel"
                try:
                    _, ms_ok = _time_launches(other_kernel, max(2, args.steps // 4), 1, stream)
                    extra[key] = {"ms_per_launch": round(ms_ok, 4),
                                  "frac": round(rec_bytes / (ms_ok / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
                except S.SymftError as e:  # the schedule does not fit that kernel
                    extra[key] = {"unavailable": str(e)}
        elif (not info["product_selected"] and (1 << info["k_max"]) * (8 if prec == "fp32" else 16) > LDS_BYTES
              and info["k_max"] >= 15):
            # vectors streamed from HBM scratch far beyond the caches: one read and one write of the live
            # vector per dense instruction
            nbytes = info["dense_bytes_per_shot"] * (1 if prec == "fp32" else 2) * w.shots
            achieved = nbytes / (ms_kernel / 1e3) / 1e9
            traffic = _traffic(w.name, "sample_active.hip") if prec == "fp32" and w.shots == 1 << 16 else None
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": round(traffic / 1e9, 1) if traffic else None, "traffic_unit": "GB/launch",
                    "kernel": "active_kernel", "bytes_per_launch": nbytes}
        else:
            # vectors in LDS, or at widths 13 and 14 in scratch that the L2 and the Infinity Cache hold:
            # priced against the vector ALU, with the flops of the representation that runs
            flops = _flops_per_shot(info) * w.shots
            achieved = flops / (ms_kernel / 1e3) / 1e12
            peak = FP32_PEAK_TFLOPS if prec == "fp32" else FP64_PEAK_TFLOPS
            roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4), "traffic": None,
                    "kernel": "lane_kernel" if tps == 1 else "active_kernel", "flops_per_launch": flops}
        config = {"workload": w.name, "shots": w.shots, "rows": prog.n_rows, "k_max": info["k_max"],
                  "precision": prec if info["k_max"] else "n/a (integer path)"}
        if tps:
            config["threads_per_shot"] = tps
        if info["k_max"]:
            config["representation"] = _representation(info)
        if info["k_max"] and info["product_selected"] and args.extras:
            # the same launch on the dense vector
            dprog = S.Program(w.circuit, components="off")
            dprog.autotune(prec)

            def dense_step():
                dprog.sample_into(out, w.shots, w.seed, precision=prec, stream=stream.cuda_stream)
            _, ms_d = _time_launches(dense_step, max(2, args.steps // 4), 1, stream)
            extra["dense_vector"] = {"ms_per_launch": round(ms_d, 4), "dense_over_product": round(ms_d / ms_kernel, 3),
                                     "dense_flops_per_shot": info["dense_flops_per_shot"],
                                     "product_flops_per_shot": info["product_flops_per_shot"]}
        if info["k_max"]:
            errors_for = (prog, w)
        n_cpu_words = {"c1": 256, "c2": 24, "c3": 64, "c3fp64": 64, "c5": 8, "c5fp64": 8, "c5k16": 2,
                       "c5k16fp64": 2}[wl]
        sample_words = [int(i * words / n_cpu_words) for i in range(n_cpu_words)]
        circ, seed = w.circuit, w.seed
        if wl == "c1" and args.extras:
            # the launch-latency-bound case: the same call eager, through the allocation-free entry point,
            # and captured once in a HIP graph and replayed (that entry point allocates nothing, so it can be
            # captured); every replay's records equal the eager call's
            eager = out.clone()
            prog.sample_noalloc_into(out, w.shots, w.seed, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            assert torch.equal(out, eager)

            def noalloc():
                prog.sample_noalloc_into(out, w.shots, w.seed, stream=stream.cuda_stream)
            ms_na, _ = _time_launches(noalloc, args.steps, args.warmup, stream)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, capture_error_mode="thread_local"):
                prog.sample_noalloc_into(out, w.shots, w.seed)
            out.fill_(-1)
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), "graph replay differs from the eager call"
            ms_g, _ = _time_launches(graph.replay, args.steps, args.warmup, stream)
            extra["c1_launch_latency"] = {"eager_us_per_call": round(ms_step * 1e3, 2),
                                          "noalloc_us_per_call": round(ms_na * 1e3, 2),
                                          "graph_replay_us_per_call": round(ms_g * 1e3, 2),
                                          "kernel_us": round(ms_kernel * 1e3, 2)}
        if wl == "c2" and args.extras:
            extra["c4_batch"], _ = _c4_comparison(S, stream, 6)
    elif wl in ("c4", "c4fp64"):
        prec = "fp64" if wl == "c4fp64" else "fp32"
        cmp, (progs, ws, flops, ms_kernel) = _c4_comparison(S, stream, args.steps, prec)
        ms_step = cmp[f"batched_{prec}"]["ms_per_step"]
        value = cmp["shots"] / (ms_step / 1e3)
        extra["c4_batch"] = cmp
        achieved = flops / (ms_kernel / 1e3) / 1e12
        peak = FP32_PEAK_TFLOPS if prec == "fp32" else FP64_PEAK_TFLOPS
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": "lane_batch_kernel + batch_kernel (one graph)"}
        dtype = "f32" if prec == "fp32" else "f64"
        config = {"workload": "batch_128_near_clifford", "shots": cmp["shots"], "programs": len(ws), "precision": prec,
                  "representation": "automatic per member"}
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

        ms_step, ms_kernel = _time_launches(step, args.steps, args.warmup, stream)
        value = w.shots / (ms_step / 1e3)
        counts.zero_()
        step()
        n_disc, n_log = (int(x) for x in counts.cpu())
        out = torch.empty((prog.n_rows, words), dtype=torch.int64, device="cuda")

        def records():
            prog.sample_into(out, w.shots, w.seed, precision=prec, stream=stream.cuda_stream)

        ms_rec, ms_rec_kernel = _time_launches(records, max(2, args.steps // 2), 1, stream)
        del out
        extra["discarded_fraction"] = round(n_disc / w.shots, 5)
        extra["logical_errors_per_kept_shot"] = round(n_log / max(1, w.shots - n_disc), 6)
        extra["full_records"] = {"shots_per_s": round(w.shots / (ms_rec / 1e3), 1), "ms_per_step": round(ms_rec, 4)}
        extra["counts_over_full_records"] = round(ms_rec / ms_step, 3)
        # the full work of every shot, priced on the records launch, which does all of it
        flops = _flops_per_shot(info) * w.shots
        achieved = flops / (ms_rec_kernel / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": None,
                "kernel": ("lane_kernel" if tps == 1 else "active_kernel") + " (full-records launch)",
                "flops_per_launch": flops}
        dtype = "f32"
        config = {"workload": w.name, "shots": w.shots, "rows": prog.n_rows, "k_max": info["k_max"],
                  "precision": prec, "threads_per_shot": tps_counts, "threads_per_shot_full_records": tps,
                  "postselected_detectors": len(post),
                  "output": "per-shot discarded / logical-error flags + counts"}
        circ, seed = w.circuit, w.seed
        n_cpu_words = 16 if wl == "post" else 8192  # the width-5 distillation oracle runs ~1e5 shots/s
        sample_words = [int(i * words / n_cpu_words) for i in range(n_cpu_words)]
        errors_for = (prog, w)
    else:
        raise SystemExit(f"unknown workload {wl}")

    if args.cpu_baseline:
        cpu_value, cpu_dt = _cpu_baseline(circ, seed, sample_words, threads=cores)
        cpu = {"value": round(cpu_value, 2), "unit": "shots/s", "cores": cores, "kind": "oracle",
               "sample": f"{len(sample_words)} 64-shot words spread over the workload's shot range "
                         f"({len(sample_words) * 64} shots, {cpu_dt:.1f} s)"}
        if args.extras:
            if wl == "c2":
                extra["errors_vs_fp64_oracle"] = _oracle_errors_all(S)
            elif errors_for is not None:
                extra["errors_vs_fp64_oracle"] = _errors_vs_oracle(errors_for[0], errors_for[1], 12, 8)
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
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="time only the workload itself (no comparisons, no error report)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the sampler runs on one GPU only; shots shard by 64-shot word ranges, "
                                   "so N GPUs would each run this same kernel on 1/N of the words"}))
        raise SystemExit(2)
    run(args)


if __name__ == "__main__":
    main()
