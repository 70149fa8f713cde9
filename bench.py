#!/usr/bin/env python3
"""Noisy-trajectory throughput on one MI355X.

Workload: 24-qubit 4x6 grid, 20 cycles of random sqrt(X)/sqrt(Y)/sqrt(W)
layers and four alternating CZ patterns; a depolarizing channel (p = 1e-3)
after every gate on each touched qubit, amplitude damping (gamma = 1e-3) on
every qubit after every moment, readout flips 2e-2; complex64 state, FP64
norms, one shot per trajectory, delayed inner-product branch selection.
A step is one batch of trajectories (default 1000) through the whole path:
per-trajectory draws and classification, fused gate sweeps, in-place inner
products where needed, and sampling with readout error.  The step's
trajectories are split over --streams states (default 2), each on its own
stream and host thread, run at once (qs_run_trajectories_concurrent): one
state's sweep ramps are filled by the other's gate work.

Prints one JSON line with the throughput, the fused-gate sweep's achieved
rate against its binding roofline (the sweep time is the span during which
at least one sweep ran, from HIP-event brackets on the states' streams inside
the timed region), the same step on one state, the conventional (naive)
method's throughput on a few trajectories, and the CPU oracle's rate on a
bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP32_PEAK_TFLOPS = 157.3
KERNEL_SOURCE = os.path.join(ROOT, "paper_2111_02396_amd", "csrc", "qs_kernels.hip")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "apply_tile_grid24_counters.md")


def kernel_source_digest() -> str:
    """SHA-256 prefix of the kernel source with comments and whitespace
    removed (a comment edit leaves the kernels, and their counters, as they were)."""
    import hashlib
    import re

    src = open(KERNEL_SOURCE, encoding="utf-8").read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per sweep launch from the committed counter summary, only if
    it was taken on the kernel source that is built now (else None)."""
    try:
        digest = kernel_source_digest()
        text = open(COUNTER_SUMMARY).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("kernel_source_sha256_prefix:", "traffic_bytes_per_launch:")))
    if fields.get("kernel_source_sha256_prefix", "").strip() != digest:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def trace_marker(qs, st) -> None:
    """Two norm passes back to back (norm_partials, reduce_records,
    norm_partials, reduce_records): a pattern the trajectory driver never
    launches, so a kernel trace of this command can be cut at these points
    (the timed region's sweeps lie between the first two markers)."""
    qs.qs_norm(st.h)
    qs.qs_norm(st.h)


def bench_copy(args) -> int:
    """Device-to-device copy of a 2^24-amplitude complex64 state (128 MiB read,
    128 MiB written per copy): the kernel of known traffic whose FETCH_SIZE /
    WRITE_SIZE readings scale the counters taken on the sweep kernels."""
    import torch

    a = torch.randn(1 << 24, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    nbytes = 2 * a.numel() * 8
    print(json.dumps({"metric": "device copy bandwidth (counter calibration)", "value": nbytes / dt / 1e9,
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "c64", "data": "synthetic",
                      "config": {"workload": "copy of a 2^24-amplitude complex64 state",
                                 "bytes_per_copy": nbytes}}), flush=True)
    return 0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(workload, cycles: int) -> dict:
    """The oracle (single thread, complex128) on the first `cycles` cycles of
    trajectory 0; scaled to whole trajectories by the cycle count."""
    import oracle
    import workloads as W

    c = workload.circuit
    total_moments = 1 + max(o.moment for o in c.ops)
    keep = 2 * cycles
    sub = W.Circuit(c.n, [o for o in c.ops if o.moment < keep])
    oracle.lib()
    t0 = time.perf_counter()
    oracle.run_trajectory(sub, 0, mode=0, seed=workload.seed)
    dt = time.perf_counter() - t0
    per_traj = dt * total_moments / keep
    return {
        "value": 1.0 / per_traj,
        "unit": "trajectories/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"trajectory 0, first {keep} of {total_moments} moments "
                   f"({len(sub.ops)} of {len(c.ops)} ops) in {dt:.1f} s, scaled by moments"),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--traj", type=int, default=1000, help="trajectories per step")
    ap.add_argument("--p-dep", type=float, default=1e-3)
    ap.add_argument("--rows", type=int, default=4, help="grid rows (the headline workload is 4 x 6)")
    ap.add_argument("--cols", type=int, default=6, help="grid columns")
    ap.add_argument("--max-fuse", type=int, default=0)
    ap.add_argument("--tile-bits", type=int, default=0,
                    help="LDS tile sweep width (0 = library default, 1 = one pass per fused gate)")
    ap.add_argument("--streams", type=int, default=2,
                    help="states (each on its own stream, driven by its own host thread) that a "
                         "step's trajectories are split over and run on at once")
    ap.add_argument("--inplace-traj", type=int, default=3,
                    help="trajectories timed with the conventional rule and in-place inner products")
    ap.add_argument("--naive-traj", type=int, default=3,
                    help="trajectories timed with the conventional method (0 = skip)")
    ap.add_argument("--cpu-cycles", type=int, default=1,
                    help="cycles of trajectory 0 timed on the oracle (0 = skip)")
    ap.add_argument("--workload", default="grid24",
                    choices=["grid24", "chain12", "grid28", "batched", "serving", "phase_damping",
                             "copy"],
                    help="grid24 (default): the headline line; batched / serving / phase_damping: "
                         "the other forms; copy: a plain device copy of a 24-qubit state, the "
                         "reference for calibrating HBM byte counters")
    ap.add_argument("--requests", type=int, default=60, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=0.0, help="serving: arrivals/s (0 = ~70%% load)")
    ap.add_argument("--max-qubits", type=int, default=26, help="serving: largest request")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only (--gpus 1): the library has no multi-GPU path; "
              "trajectories would shard by index range, one range per GPU",
              file=sys.stderr)
        return 2

    import torch

    import paper_2111_02396_amd as qs
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    qs.load()
    torch.cuda.set_device(0)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "chain12":
        return bench_chain12(args)
    if args.workload == "grid28":
        return bench_grid28(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "phase_damping":
        return bench_phase_damping(args)
    if args.workload == "copy":
        return bench_copy(args)
    w = W.grid24_workload(p_dep=args.p_dep, rows=args.rows, cols=args.cols)
    c = w.circuit
    n = c.n
    mc = qs.MarshalledCircuit(c)
    n_streams = max(1, args.streams)
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    bufs = [torch.zeros(1 << n, dtype=torch.complex64, device="cuda") for _ in range(n_streams)]
    states = [qs.State(n, b.data_ptr(), b.numel() * 8, sx.cuda_stream) for b, sx in zip(bufs, streams)]
    st, stream = states[0], streams[0]
    handles = [x.h for x in states]

    def step(offset: int, timed: bool, mode=qs.QS_KRAUS_DELAYED, n_traj=None, all_states=True):
        # a step: the trajectories split over every state, run at once
        hs = handles if (all_states and n_streams > 1) else st.h
        return qs.qs_run_trajectories(
            hs, c, n_traj or args.traj, seed=w.seed, traj_offset=offset, mode=mode,
            max_fuse=args.max_fuse, tile_bits=args.tile_bits, n_samples=w.n_samples,
            p0to1=w.e0, p1to0=w.e1,
            record_choices=False, time_kernels=timed, marshalled=mc)

    log(f"workload {w.name}: n={n}, ops={len(c.ops)}, channels={mc.n_channels}")
    for i in range(args.warmup):
        t0 = time.perf_counter()
        r = step(10_000_000 + i * args.traj, False)
        log(f"warmup {i}: {args.traj / (time.perf_counter() - t0):.1f} traj/s untimed-kernels, "
            f"gate sweeps/traj {r['gate_sweeps'] / args.traj:.1f}")

    trace_marker(qs, st)  # the timed region begins
    torch.cuda.synchronize()
    for sx in streams:
        sx.synchronize()
    t0 = time.perf_counter()
    gate_ms = 0.0
    gate_launches = 0
    zero_start = 0
    sweeps = 0
    gate_sweeps = 0
    slow = 0
    k_hist = [0] * 6
    for s in range(args.steps):
        r = step(s * args.traj, True)
        gate_ms += r["gate_kernel_ms"]
        gate_launches += r["gate_kernel_launches"]
        zero_start += r["zero_start_sweeps"]
        sweeps += r["sweeps"]
        gate_sweeps += r["gate_sweeps"]
        slow += int(r["n_slow"].sum())
        k_hist = [a + b for a, b in zip(k_hist, r["gate_k_launches"])]
        log(f"step {s}: {r['host_seconds']:.3f} s")
    for sx in streams:
        sx.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    trace_marker(qs, st)  # the timed region has ended
    total_traj = args.steps * args.traj
    value = total_traj / elapsed

    avg_gate_s = (gate_ms / 1e3) / max(gate_launches, 1)
    # algorithmic bytes: one read + one write of the complex64 state per sweep,
    # except a trajectory's first sweep, which starts from |0...0> written on
    # chip and only writes
    state_bytes = 8 * (1 << n)
    alg_bytes = 2 * state_bytes * gate_launches - state_bytes * zero_start
    bytes_per_launch = alg_bytes / max(gate_launches, 1)
    achieved = alg_bytes / (gate_ms / 1e3) / 1e9 if gate_ms > 0 else 0.0
    traffic = measured_traffic() if (args.rows, args.cols) == (4, 6) else None  # profiled at 4 x 6
    # complex mat-vec flops of the fused blocks applied (8 * 2^k per amplitude, Section 3.1)
    flops = sum(k_hist[k] * (8 << k) for k in range(1, 6)) * float(1 << n)
    flops_tf = flops / (gate_ms / 1e3) / 1e12 if gate_ms > 0 else 0.0

    # The sweep's binding roofline: the longer of its algorithmic bytes at the
    # HBM peak and its algorithmic flops at the FP32 MFMA peak.
    hbm_side = {"achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS,
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "roofline_us_per_launch": bytes_per_launch / (HBM_PEAK_GBPS * 1e3)}
    flops_per_launch = flops / max(gate_launches, 1)
    mfma_us = flops_per_launch / (FP32_PEAK_TFLOPS * 1e6)
    common = {
        "traffic": (traffic / 1e9) if traffic else None,
        "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "kernel": "fused-gate sweep (apply_tile / apply_direct): one read + one write of the state, "
                  "the sweep's fused blocks applied in LDS",
        "avg_launch_us": avg_gate_s * 1e6,
        "avg_launch_basis": ("time during which at least one sweep ran (union of the streams' "
                             "HIP-event brackets) / launches" if n_streams > 1 else
                             "HIP-event brackets of back-to-back sweeps / launches"),
        "launches": gate_launches,
        "zero_start_launches": zero_start,
    }
    if mfma_us > hbm_side["roofline_us_per_launch"]:
        roofline = {"bound": "mfma", "achieved": flops_tf, "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": flops_tf / FP32_PEAK_TFLOPS,
                    "algorithmic_flops_per_launch": flops_per_launch,
                    "roofline_us_per_launch": mfma_us,
                    "basis": "8*2^k flops per amplitude per fused k-qubit block (complex mat-vec)",
                    **common}
    else:
        roofline = {"bound": "hbm", **{k: v for k, v in hbm_side.items()}, **common}

    naive = None
    if args.naive_traj > 0:
        t1 = time.perf_counter()
        rn = step(20_000_000, False, mode=qs.QS_KRAUS_NAIVE, n_traj=args.naive_traj, all_states=False)
        dtn = time.perf_counter() - t1
        naive = {"value": args.naive_traj / dtn, "unit": "trajectories/s",
                 "trajectories": args.naive_traj,
                 "sweeps_per_traj": rn["sweeps"] / args.naive_traj}
        log(f"naive: {naive['value']:.3f} traj/s")

    inplace = None
    if args.inplace_traj > 0:
        t1 = time.perf_counter()
        ri = step(30_000_000, False, mode=qs.QS_KRAUS_CONVENTIONAL_INPLACE, n_traj=args.inplace_traj,
                  all_states=False)
        dti = time.perf_counter() - t1
        inplace = {"value": args.inplace_traj / dti, "unit": "trajectories/s",
                   "trajectories": args.inplace_traj,
                   "sweeps_per_traj": ri["sweeps"] / args.inplace_traj}
        log(f"conventional, in-place inner products: {inplace['value']:.3f} traj/s")

    single = None
    if n_streams > 1:
        # the same step on one state, for comparison (kernels untimed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step(60_000_000, False, all_states=False)
        stream.synchronize()
        dts = time.perf_counter() - t1
        single = {"value": args.traj / dts, "unit": "trajectories/s", "steps": 1}
        log(f"one state: {single['value']:.1f} traj/s")

    cpu = None
    if args.cpu_cycles > 0:
        log("timing the CPU oracle sample ...")
        cpu = cpu_baseline(w, args.cpu_cycles)

    for x in states:
        x.close()
    out = {
        "metric": "trajectories/s at 24q depth-20 noisy (HBM GB/s %peak); served p50/p99 latency",
        "value": value,
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "qubits": n,
            "trajectories_per_step": args.traj,
            "samples_per_trajectory": w.n_samples,
            "mode": "delayed",
            "max_fuse": args.max_fuse or 4,
            "tile_bits": args.tile_bits or 13,
            "parallelism": f"none (1 GPU); {n_streams} trajectory streams",
        },
        "roofline": roofline,
        "hbm": hbm_side,
        "cpu_baseline": cpu,
        "one_stream": single,
        "naive": naive,
        "speedup_vs_naive": (value / naive["value"]) if naive else None,
        "conventional_inplace": inplace,
        "speedup_vs_conventional_inplace": (value / inplace["value"]) if inplace else None,
        "gate_sweeps_per_traj": gate_sweeps / total_traj,
        "sweeps_per_traj": sweeps / total_traj,
        "slow_paths_per_traj": slow / total_traj,
        "gate_width_histogram": k_hist[1:],
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_chain12(args) -> int:
    """The 12-qubit chain (depth 20, depolarizing 1e-3 after every gate): 100
    trajectories x 1000 samples.  The 32 KiB state lives in LDS, so the run is
    latency bound: one persistent launch (qs_run_batched) for the whole step,
    and the same trajectories one qs_run_trajectories call each beside it."""
    import torch

    import paper_2111_02396_amd as qs
    import workloads as W

    w = W.chain12_workload()
    prepared = qs.PreparedBatch([w], record_choices=False)
    for _ in range(args.warmup):
        qs.qs_run_batched(prepared)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        _, stats = qs.qs_run_batched(prepared, time_kernels=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps * w.n_traj / dt
    mc = qs.MarshalledCircuit(w.circuit)
    with qs.State(w.circuit.n) as st:
        qs.qs_run_trajectories(st.h, w.circuit, 4, seed=w.seed, n_samples=w.n_samples,
                               max_fuse=w.max_fuse, record_choices=False, marshalled=mc)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        qs.qs_run_trajectories(st.h, w.circuit, w.n_traj, seed=w.seed, n_samples=w.n_samples,
                               max_fuse=w.max_fuse, record_choices=False, marshalled=mc)
        dt1 = time.perf_counter() - t1
    out = {
        "metric": "trajectories/s, 12-qubit chain depth 20, 1000 samples each",
        "value": value, "unit": "trajectories/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": w.name, "trajectories_per_step": w.n_traj,
                   "samples_per_trajectory": w.n_samples, "max_fuse": w.max_fuse},
        "us_per_trajectory": 1e6 * dt / (args.steps * w.n_traj),
        "samples_per_s": value * w.n_samples,
        "kernel_ms": stats["kernel_ms"],
        "one_call_per_range": {"value": w.n_traj / dt1, "unit": "trajectories/s",
                               "form": "qs_run_trajectories over the 100 trajectories"},
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_grid28(args) -> int:
    """The 28-qubit noiseless 4 x 7 grid (depth 20, blocks of <= 4 qubits): one
    2 GiB state evolved from |0...0>, then 10^5 samples; sweep time and rate
    against the rooflines."""
    import torch

    import paper_2111_02396_amd as qs
    import workloads as W

    w = W.grid28_workload()
    c = w.circuit
    n = c.n
    mc = qs.MarshalledCircuit(c)
    with qs.State(n) as st:
        def run(timed):
            return qs.qs_run_trajectories(st.h, c, 1, seed=w.seed, n_samples=w.n_samples,
                                          max_fuse=w.max_fuse, record_choices=False,
                                          time_kernels=timed, marshalled=mc)
        for _ in range(args.warmup):
            run(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = 0.0
        launches = 0
        k_hist = [0] * 6
        zero = 0
        for _ in range(args.steps):
            r = run(True)
            ms += r["gate_kernel_ms"]
            launches += r["gate_kernel_launches"]
            zero += r["zero_start_sweeps"]
            k_hist = [a + b for a, b in zip(k_hist, r["gate_k_launches"])]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    state_bytes = 8 * (1 << n)
    alg_bytes = 2 * state_bytes * launches - state_bytes * zero
    flops = sum(k_hist[k] * (8 << k) for k in range(1, 6)) * float(1 << n)
    sweep_s = ms / 1e3
    out = {
        "metric": "28-qubit noiseless grid: evolved states/s (with 1e5 samples each)",
        "value": args.steps / dt, "unit": "states/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": w.name, "qubits": n, "samples": w.n_samples,
                   "max_fuse": w.max_fuse},
        "sweeps_per_state": launches / args.steps,
        "avg_sweep_us": 1e6 * sweep_s / max(launches, 1),
        "sweep_hbm": {"achieved_GBps": alg_bytes / sweep_s / 1e9 if sweep_s > 0 else None,
                      "peak_GBps": HBM_PEAK_GBPS},
        "sweep_mfma": {"achieved_TFLOPs": flops / sweep_s / 1e12 if sweep_s > 0 else None,
                       "peak_TFLOPs": FP32_PEAK_TFLOPS},
        "non_sweep_ms_per_state": 1e3 * (dt - sweep_s) / args.steps,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_batched(args) -> int:
    """4096 trajectories = 256 circuits x 16, n ~ U{12..18}, depth ~ U{10..40},
    depolarizing 1e-3, in one persistent launch; the same work one trajectory
    per qs_run_trajectories call on a sample is the comparison."""
    import torch

    import paper_2111_02396_amd as qs
    import workloads as W

    items = W.batched_workload()
    n_traj = sum(w.n_traj for w in items)
    prepared = qs.PreparedBatch(items, record_choices=False)
    for _ in range(args.warmup):
        qs.qs_run_batched(prepared)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        _, stats = qs.qs_run_batched(prepared, time_kernels=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps * n_traj / dt
    # one trajectory per call, on every 16th circuit's trajectories
    sample = items[::16]
    t1 = time.perf_counter()
    done = 0
    for w in sample:
        with qs.State(w.circuit.n) as st:
            for t in range(w.n_traj):
                qs.qs_run_trajectories(st.h, w.circuit, 1, seed=w.seed, traj_offset=t,
                                       circuit_id=w.circuit_id, n_samples=w.n_samples,
                                       max_fuse=3, record_choices=False)
                done += 1
    dt1 = time.perf_counter() - t1
    per_call = done / dt1
    out = {
        "metric": "batched trajectories/s (persistent launch)",
        "value": value, "unit": "trajectories/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "batched 256 circuits x 16 trajectories, n 12-18, depth 10-40, "
                               "depolarizing 1e-3", "trajectories_per_step": n_traj},
        "kernel_ms": stats["kernel_ms"], "plan_seconds": stats["plan_seconds"],
        "resident_jobs": stats["resident_jobs"],
        "one_trajectory_per_call": {"value": per_call, "unit": "trajectories/s",
                                    "sample": f"{done} trajectories of {len(sample)} circuits"},
        "speedup_vs_one_per_call": value / per_call,
    }
    print(json.dumps(out), flush=True)
    return 0


def phase_damped_circuit(rows: int, cols: int, lam: float, cycles: int = 20):
    """Random grid circuit with a phase-damping channel after every gate on
    each qubit it touches (the paper's noise benchmark shape)."""
    import workloads as W

    c = W.grid_circuit(rows, cols, cycles, seed=0)
    ops = []
    pd = W.phase_damp(lam)
    for op in c.ops:
        ops.append(op)
        for q in op.qubits:
            ops.append(W.Op(W.CHANNEL, (q,), pd, op.moment, "phase_damp"))
    return W.Circuit(c.n, ops, f"grid{rows}x{cols}-pd{lam:g}")


def bench_phase_damping(args) -> int:
    """Trajectories/s against phase-damping strength, delayed inner products
    vs the conventional method, at 20 and 27 qubits."""
    import paper_2111_02396_amd as qs

    rows = []
    for (r, c_, n_traj, n_naive) in ((4, 5, 40, 4), (3, 9, 6, 1)):
        n = r * c_
        with qs.State(n) as st:
            for lam in (1e-4, 1e-3, 1e-2, 1e-1):
                circ = phase_damped_circuit(r, c_, lam)
                mc = qs.MarshalledCircuit(circ)
                qs.qs_run_trajectories(st.h, circ, 1, seed=0, traj_offset=99, n_samples=1,
                                       marshalled=mc, record_choices=False)
                t0 = time.perf_counter()
                rd = qs.qs_run_trajectories(st.h, circ, n_traj, seed=0, n_samples=1,
                                            marshalled=mc, record_choices=False)
                dd = time.perf_counter() - t0
                t1 = time.perf_counter()
                qs.qs_run_trajectories(st.h, circ, n_naive, seed=0, n_samples=1,
                                       mode=qs.QS_KRAUS_NAIVE, marshalled=mc, record_choices=False)
                dn = time.perf_counter() - t1
                row = {"qubits": n, "lambda": lam, "channels": mc.n_channels,
                       "delayed_traj_per_s": n_traj / dd, "naive_traj_per_s": n_naive / dn,
                       "slow_paths_per_traj": float(rd["n_slow"].mean()),
                       "speedup": (n_traj / dd) / (n_naive / dn)}
                log(json.dumps(row))
                rows.append(row)
    out = {"metric": "trajectories/s vs phase-damping strength (delayed vs conventional)",
           "value": rows[1]["delayed_traj_per_s"], "unit": "trajectories/s", "n_gpus": 1,
           "steps": 1, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
           "config": {"workload": "grid 4x5 and 3x9, 20 cycles, phase damping after every gate"},
           "sweep": rows}
    print(json.dumps(out), flush=True)
    return 0


def bench_serving(args) -> int:
    """Poisson arrivals of random grid circuits (n uniform up to --max-qubits,
    depth 10-40, depolarizing log-uniform in [1e-4, 1e-2], 1-1000
    trajectories, one shot each), admission by 16 * 2^n bytes."""
    import paper_2111_02396_amd as qs  # noqa: F401
    from paper_2111_02396_amd import serving
    import workloads as W

    def requests(rate):
        return W.serving_requests(args.requests, rate, seed=1, n_hi=args.max_qubits)

    rate = args.rate
    if rate <= 0:
        # offered load ~70%: modelled service time from a 6 TB/s sweep rate
        reqs = requests(1.0)
        work = sum(r.workload.n_traj * 30 * 16.0 * (1 << r.workload.circuit.n) / 6e12
                   + 2e-4 for r in reqs)
        rate = 0.7 * len(reqs) / work
    reqs = requests(rate)
    srv = serving.Server()
    stats = srv.run(reqs)
    d = stats.as_dict()
    lanes = {}
    for r in reqs:
        lanes[srv.results[r.rid].lane] = lanes.get(srv.results[r.rid].lane, 0) + 1
    out = {
        "metric": "served trajectories/s; p50/p99 request latency",
        "value": d["trajectories_per_s"], "unit": "trajectories/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": 1e3 * d["wall_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"serving {args.requests} requests, Poisson {rate:.2f}/s, "
                               f"n 10-{args.max_qubits}"},
        "p50_s": d["p50_s"], "p99_s": d["p99_s"], "requests": d["requests"], "lanes": lanes,
        "errors": sum(1 for r in reqs if srv.results[r.rid].error),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
