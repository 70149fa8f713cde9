#!/usr/bin/env python3
"""Noisy-trajectory throughput on one MI355X.

Workload (the headline): 24-qubit 4x6 grid, 20 cycles of random
sqrt(X)/sqrt(Y)/sqrt(W) layers and four alternating CZ patterns; a
depolarizing channel (p = 1e-3) after every gate on each touched qubit,
amplitude damping (gamma = 1e-3) on every qubit after every moment, readout
flips 2e-2; complex64 state, FP64 norms, one shot per trajectory, delayed
inner-product branch selection, fusion and tile widths autotuned.  A step is
one batch of trajectories (default 1000) through the whole path: per-
trajectory draws and classification, fused gate sweeps, in-place inner
products where needed, and sampling with readout error.  The step's
trajectories are split over --streams states (default 2), each on its own
stream and host thread, run at once (qs_run_trajectories_concurrent).

Prints one JSON line: the throughput; the fused-gate sweep's achieved HBM
rate against the 8 TB/s peak (algorithmic bytes over the span during which
at least one sweep ran, from HIP-event brackets on the states' streams inside
the timed region) with the sweep's compute floor (issued MFMA and VALU work)
beside it; the same step on one state; the conventional method on one state;
the CPU oracle on all host cores; and bounded sub-records for the other
workloads (depolarizing strengths, 26 and 28 qubits, the 28-qubit noiseless
grid, the 12-qubit chain, the batched launch, served requests).
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
FP32_MFMA_PEAK_TFLOPS = 157.3
# FP32 vector rate without packed instructions (the build disables them):
# half of the 157.3 TFLOP/s packed figure
FP32_VALU_PEAK_TFLOPS = 78.65
KERNEL_SOURCE = os.path.join(ROOT, "paper_2111_02396_amd", "csrc", "qs_kernels.hip")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "apply_tile_grid24_counters.md")

# Flops per amplitude of a fused k-qubit block: the algorithmic count of a
# complex 2^k x 2^k mat-vec (Section 3.1), and what the kernels issue: k = 3
# on MFMA in the real form, k = 4 and 5 on MFMA with three real products
# instead of four, k = 1 and 2 on VALU.
ALG_FLOPS = {k: 8 << k for k in range(1, 6)}
MFMA_FLOPS = {3: 64, 4: 96, 5: 192}
VALU_FLOPS = {1: 16, 2: 32}


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


def measured_traffic(tile_bits, path=COUNTER_SUMMARY):
    """HBM bytes per sweep launch from a committed counter summary, only if
    it was taken on the kernel source that is built now and on the tile
    width the run used (else None)."""
    try:
        digest = kernel_source_digest()
        text = open(path).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("kernel_source_sha256_prefix:", "traffic_bytes_per_launch:",
                                      "tile_bits:")))
    if fields.get("kernel_source_sha256_prefix", "").strip() != digest:
        return None
    if fields.get("tile_bits", "").strip() != str(tile_bits):
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


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def sweep_roofline(n, ms, launches, zero_start, k_hist):
    """The fused-gate sweep against its rooflines.  Units: one sweep launch.
    HBM: algorithmic bytes (one read and one write of the complex64 state;
    a trajectory's first sweep starts from |0...0> on chip and only writes).
    Compute: the MFMA and VALU work the kernels issue for the launch's blocks
    (they share the SIMDs' issue cycles, so their times add)."""
    amps = float(1 << n)
    state_bytes = 8 * amps
    launches = max(launches, 1)
    sec = ms / 1e3
    alg_bytes = 2 * state_bytes * launches - state_bytes * zero_start
    bytes_per_launch = alg_bytes / launches
    alg_flops = sum(k_hist[k] * ALG_FLOPS[k] for k in range(1, 6)) * amps
    mfma_flops = sum(k_hist[k] * MFMA_FLOPS.get(k, 0) for k in range(1, 6)) * amps
    valu_flops = sum(k_hist[k] * VALU_FLOPS.get(k, 0) for k in range(1, 6)) * amps
    hbm_us = bytes_per_launch / (HBM_PEAK_GBPS * 1e3)
    mfma_us = mfma_flops / launches / (FP32_MFMA_PEAK_TFLOPS * 1e6)
    valu_us = valu_flops / launches / (FP32_VALU_PEAK_TFLOPS * 1e6)
    gbps = alg_bytes / sec / 1e9 if sec > 0 else 0.0
    return {
        "avg_launch_us": 1e6 * sec / launches,
        "launches": launches,
        "zero_start_launches": zero_start,
        "hbm": {"achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                "algorithmic_bytes_per_launch": bytes_per_launch, "floor_us_per_launch": hbm_us},
        "compute": {
            "mfma_issued_tflops": mfma_flops / sec / 1e12 if sec > 0 else 0.0,
            "mfma_issued_frac": (mfma_flops / sec / 1e12) / FP32_MFMA_PEAK_TFLOPS if sec > 0 else 0.0,
            "algorithmic_tflops": alg_flops / sec / 1e12 if sec > 0 else 0.0,
            "algorithmic_frac_of_fp32_mfma_peak":
                (alg_flops / sec / 1e12) / FP32_MFMA_PEAK_TFLOPS if sec > 0 else 0.0,
            "mfma_floor_us_per_launch": mfma_us,
            "valu_floor_us_per_launch": valu_us,
            "floor_us_per_launch": mfma_us + valu_us,
            "basis": ("issued flops per amplitude: k=3 64 (real form), k=4 96 and k=5 192 "
                      "(three real products) on FP32 MFMA at 157.3 TFLOP/s; k=1 16 and k=2 32 "
                      "on FP32 VALU at 78.65 TFLOP/s (no packed FP32)"),
        },
        "bound": "hbm" if hbm_us >= mfma_us + valu_us else "mfma",
    }


def run_grid(qs, W, args, torch, rows=4, cols=6, p_dep=1e-3, n_traj=1000, steps=1, warmup=1,
             streams=2, max_fuse=0, tile_bits=0, workload=None, mark=False, graph=False):
    """Trajectory steps of a noisy grid on `streams` concurrent states;
    returns the rate, the sweep roofline and the plan the driver used."""
    w = workload or W.grid24_workload(p_dep=p_dep, rows=rows, cols=cols)
    c = w.circuit
    n = c.n
    mc = qs.MarshalledCircuit(c)
    sx = [torch.cuda.Stream() for _ in range(max(1, streams))]
    bufs = [torch.zeros(1 << n, dtype=torch.complex64, device="cuda") for _ in sx]
    states = [qs.State(n, b.data_ptr(), b.numel() * 8, s.cuda_stream) for b, s in zip(bufs, sx)]
    handles = [x.h for x in states] if len(states) > 1 else states[0].h
    try:
        def step(offset, timed):
            return qs.qs_run_trajectories(
                handles, c, n_traj, seed=w.seed, traj_offset=offset, max_fuse=max_fuse,
                tile_bits=tile_bits, n_samples=w.n_samples, p0to1=w.e0, p1to0=w.e1,
                record_choices=False, time_kernels=timed, graph=graph, marshalled=mc)

        tune_ms = 0.0
        for i in range(warmup):
            r = step(10_000_000 + i * n_traj, False)
            tune_ms += r["tune_ms"]
        if mark:
            trace_marker(qs, states[0])  # the timed region begins
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = 0.0
        launches = zero = gate_sweeps = sweeps = slow = replays = 0
        k_hist = [0] * 6
        used = None
        for s in range(steps):
            r = step(s * n_traj, True)
            ms += r["gate_kernel_ms"]
            launches += r["gate_kernel_launches"]
            zero += r["zero_start_sweeps"]
            gate_sweeps += r["gate_sweeps"]
            sweeps += r["sweeps"]
            slow += int(r["n_slow"].sum())
            k_hist = [a + b for a, b in zip(k_hist, r["gate_k_launches"])]
            used = (r["max_fuse_used"], r["tile_bits_used"])
            tune_ms += r["tune_ms"]
            replays += r["graph_replays"]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        if mark:
            trace_marker(qs, states[0])  # the timed region has ended
    finally:
        for x in states:
            x.close()
    total = steps * n_traj
    return {
        "workload": w.name, "qubits": n, "value": total / elapsed, "unit": "trajectories/s",
        "elapsed_s": elapsed, "trajectories": total, "streams": len(sx),
        "max_fuse": used[0], "tile_bits": used[1], "tune_ms": tune_ms,
        "gate_sweeps_per_traj": gate_sweeps / total, "sweeps_per_traj": sweeps / total,
        "slow_paths_per_traj": slow / total, "gate_width_histogram": k_hist[1:],
        "graph_replays_per_traj": replays / total,
        "sweep": sweep_roofline(n, ms, launches, zero, k_hist),
    }


def one_state_rate(qs, W, torch, w, n_traj, mode, max_fuse=0, tile_bits=0, warm=1, graph=False):
    """Trajectories/s of one state on one stream (kernels untimed)."""
    c = w.circuit
    mc = qs.MarshalledCircuit(c)
    s = torch.cuda.Stream()
    buf = torch.zeros(1 << c.n, dtype=torch.complex64, device="cuda")
    with qs.State(c.n, buf.data_ptr(), buf.numel() * 8, s.cuda_stream) as st:
        kw = dict(seed=w.seed, mode=mode, max_fuse=max_fuse, tile_bits=tile_bits,
                  n_samples=w.n_samples, p0to1=w.e0, p1to0=w.e1, record_choices=False,
                  graph=graph, marshalled=mc)
        if warm:
            qs.qs_run_trajectories(st.h, c, warm, traj_offset=50_000_000, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = qs.qs_run_trajectories(st.h, c, n_traj, traj_offset=60_000_000, **kw)
        s.synchronize()
        dt = time.perf_counter() - t0
    return {"value": n_traj / dt, "unit": "trajectories/s", "trajectories": n_traj,
            "sweeps_per_traj": r["sweeps"] / n_traj, "max_fuse": r["max_fuse_used"],
            "tile_bits": r["tile_bits_used"], "graph_replays": r["graph_replays"]}


def states_rate(qs, torch, w, n_traj, n_states, mode, max_fuse=0, tile_bits=0):
    """Trajectories/s of n_states states on their own streams, the range split
    over them (qs_run_trajectories_concurrent); one untimed warm-up call."""
    c = w.circuit
    mc = qs.MarshalledCircuit(c)
    streams = [torch.cuda.Stream() for _ in range(n_states)]
    states = [qs.State(c.n, hip_stream=st.cuda_stream) for st in streams]
    try:
        hs = [st.h for st in states]
        kw = dict(seed=w.seed, mode=mode, max_fuse=max_fuse, tile_bits=tile_bits,
                  n_samples=w.n_samples, p0to1=w.e0, p1to0=w.e1, record_choices=False, marshalled=mc)
        qs.qs_run_trajectories(hs, c, 2 * n_states, traj_offset=50_000_000, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = qs.qs_run_trajectories(hs, c, n_traj, traj_offset=60_000_000, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        for st in states:
            st.close()
    return {"value": n_traj / dt, "unit": "trajectories/s", "trajectories": n_traj, "states": n_states,
            "sweeps_per_traj": r["sweeps"] / n_traj, "max_fuse": r["max_fuse_used"],
            "tile_bits": r["tile_bits_used"]}


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count()
    return model, os.cpu_count(), affinity


def _oracle_prefix(args):
    """One trajectory's first `keep` moments on the oracle."""
    import oracle
    import workloads as W

    keep, t = args
    w = W.grid24_workload()
    c = w.circuit
    sub = W.Circuit(c.n, [o for o in c.ops if o.moment < keep])
    oracle.lib()
    t0 = time.perf_counter()
    oracle.run_trajectory(sub, t, mode=0, seed=w.seed)
    return time.perf_counter() - t0, len(sub.ops)


def cpu_baseline(cycles: int, workers: int) -> dict:
    """The oracle (single thread, complex128, unchanged) on the first
    `cycles` cycles of the headline workload, one trajectory per host thread
    on `workers` threads at once (trajectories are independent; the oracle's
    C call releases the interpreter lock, so the threads run in parallel):
    the all-core rate, scaled to whole trajectories by the moment count; and
    the same prefix alone on one core."""
    from concurrent.futures import ThreadPoolExecutor

    import workloads as W

    c = W.grid24_workload().circuit
    total_moments = 1 + max(o.moment for o in c.ops)
    keep = 2 * cycles
    dt1, n_ops = _oracle_prefix((keep, 0))
    single = keep / (total_moments * dt1)  # whole trajectories per second
    out = {"single_core": {"value": single, "unit": "trajectories/s", "cores": 1,
                           "sample": f"trajectory 0, first {keep} of {total_moments} moments "
                                     f"({n_ops} ops) in {dt1:.1f} s"}}
    model, ncpu, aff = cpu_info()
    if workers > 1:
        t0 = time.perf_counter()
        with ThreadPoolExecutor(workers) as pool:
            res = list(pool.map(_oracle_prefix, [(keep, t) for t in range(workers)]))
        wall = time.perf_counter() - t0
        rate = workers * keep / (total_moments * wall)
        sample = (f"{workers} trajectories at once, one per thread, each its first {keep} of "
                  f"{total_moments} moments, in {wall:.1f} s (slowest thread "
                  f"{max(dt for dt, _ in res):.1f} s), scaled by moments")
        out.update({"value": rate, "unit": "trajectories/s", "cores": workers, "kind": "oracle",
                    "sample": sample})
    else:
        out.update({"value": single, "unit": "trajectories/s", "cores": 1, "kind": "oracle",
                    "sample": out["single_core"]["sample"]})
    out.update({"cpu_model": model, "nproc": ncpu, "affinity_cpus": aff})
    return out


# ------------------------------------------------------------------ other workloads

def sub_chain12(qs, W, torch, steps=20):
    """The 12-qubit chain (depth 20, depolarizing 1e-3 after every gate): 100
    trajectories x 1000 samples in one persistent launch, and as one
    qs_run_trajectories call over the range."""
    w = W.chain12_workload()
    prepared = qs.PreparedBatch([w], record_choices=False)
    qs.qs_run_batched(prepared)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, stats = qs.qs_run_batched(prepared, time_kernels=True, copy=False)
    dt = time.perf_counter() - t0
    mc = qs.MarshalledCircuit(w.circuit)
    with qs.State(w.circuit.n) as st:
        qs.qs_run_trajectories(st.h, w.circuit, 4, seed=w.seed, n_samples=w.n_samples,
                               max_fuse=w.max_fuse, record_choices=False, marshalled=mc)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        qs.qs_run_trajectories(st.h, w.circuit, w.n_traj, seed=w.seed, n_samples=w.n_samples,
                               max_fuse=w.max_fuse, record_choices=False, marshalled=mc)
        dt1 = time.perf_counter() - t1
    return {"workload": w.name, "value": steps * w.n_traj / dt, "unit": "trajectories/s",
            "form": "one persistent launch per 100 trajectories",
            "us_per_trajectory": 1e6 * dt / (steps * w.n_traj),
            "samples_per_s": steps * w.n_traj * w.n_samples / dt,
            "kernel_ms": stats["kernel_ms"], "host_plan_ms": 1e3 * stats["plan_seconds"],
            "max_fuse": stats["max_fuse_used"],
            "one_call_per_range": {"value": w.n_traj / dt1, "unit": "trajectories/s"}}


def sub_grid28(qs, W, torch, steps=3, max_fuse=4):
    """The 28-qubit noiseless 4 x 7 grid (depth 20): one 2 GiB state from
    |0...0> and 10^5 samples per step."""
    w = W.grid28_workload()
    c = w.circuit
    n = c.n
    mc = qs.MarshalledCircuit(c)
    with qs.State(n) as st:
        def run(timed):
            return qs.qs_run_trajectories(st.h, c, 1, seed=w.seed, n_samples=w.n_samples,
                                          max_fuse=max_fuse, record_choices=False,
                                          time_kernels=timed, marshalled=mc)
        first = run(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = 0.0
        launches = zero = 0
        k_hist = [0] * 6
        for _ in range(steps):
            r = run(True)
            ms += r["gate_kernel_ms"]
            launches += r["gate_kernel_launches"]
            zero += r["zero_start_sweeps"]
            k_hist = [a + b for a, b in zip(k_hist, r["gate_k_launches"])]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    return {"workload": w.name, "value": steps / dt, "unit": "states/s (with 1e5 samples each)",
            "ms_per_state": 1e3 * dt / steps, "max_fuse": r["max_fuse_used"],
            "tile_bits": r["tile_bits_used"], "tune_ms": first["tune_ms"],
            "sweeps_per_state": launches / steps,
            "non_sweep_ms_per_state": (1e3 * dt - ms) / steps,
            "sweep": sweep_roofline(n, ms, launches, zero, k_hist)}


def sub_batched(qs, W, torch, steps=2):
    """4096 trajectories = 256 circuits x 16, n ~ U{12..18}, depth ~ U{10..40},
    depolarizing 1e-3, one persistent launch (fusion width autotuned); the same
    work one trajectory per qs_run_trajectories call on every 16th circuit."""
    items = W.batched_workload()
    n_traj = sum(w.n_traj for w in items)
    prepared = qs.PreparedBatch(items, record_choices=False)
    _, first = qs.qs_run_batched(prepared)  # tunes the fusion width once
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, stats = qs.qs_run_batched(prepared, time_kernels=True, copy=False)
    dt = time.perf_counter() - t0
    value = steps * n_traj / dt
    fixed = {}
    for f in (3,):
        qs.qs_run_batched(prepared, max_fuse=f)
        t1 = time.perf_counter()
        _, st3 = qs.qs_run_batched(prepared, max_fuse=f, time_kernels=True, copy=False)
        fixed[f"max_fuse_{f}"] = {"value": n_traj / (time.perf_counter() - t1),
                                  "kernel_ms": st3["kernel_ms"]}
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
    per_call = done / (time.perf_counter() - t1)
    return {"workload": "256 circuits x 16 trajectories, n 12-18, depth 10-40, depolarizing 1e-3",
            "value": value, "unit": "trajectories/s", "kernel_ms": stats["kernel_ms"],
            "host_plan_ms": 1e3 * stats["plan_seconds"], "max_fuse": stats["max_fuse_used"],
            "tune_ms": first["tune_ms"], "fixed_width": fixed,
            "one_trajectory_per_call": {"value": per_call, "unit": "trajectories/s",
                                        "sample": f"{done} trajectories of {len(sample)} circuits"},
            "speedup_vs_one_per_call": value / per_call}


def cap_large_requests(reqs):
    """Bounded variant for the top of the request range: a request of n >= 28
    qubits keeps at most 2^(33 - n) of its trajectories (32 q: 2, 30 q: 8,
    28 q: 32), so a run with 30-32-qubit requests takes minutes, not hours."""
    for r in reqs:
        n = r.workload.circuit.n
        if n >= 28:
            r.workload.n_traj = max(1, min(r.workload.n_traj, 1 << (33 - n)))
    return reqs


def sub_served(qs, W, requests=40, max_qubits=24, cap_large=False):
    """Poisson arrivals of random grid circuits (n uniform in 10..max_qubits,
    depth 10-40, depolarizing log-uniform in [1e-4, 1e-2], 1-1000
    trajectories, one shot each), admission by 16 * 2^n bytes, ~70% load."""
    from paper_2111_02396_amd import serving

    def make(rate):
        reqs = W.serving_requests(requests, rate, seed=1, n_hi=max_qubits)
        return cap_large_requests(reqs) if cap_large else reqs

    reqs = make(1.0)
    work = sum(r.workload.n_traj * 30 * 16.0 * (1 << r.workload.circuit.n) / 6e12 + 2e-4
               for r in reqs)
    rate = 0.7 * len(reqs) / work
    reqs = make(rate)
    srv = serving.Server()
    d = srv.run(reqs).as_dict()
    lanes = {}
    for r in reqs:
        lanes[srv.results[r.rid].lane] = lanes.get(srv.results[r.rid].lane, 0) + 1
    sizes = [r.workload.circuit.n for r in reqs]
    return {"workload": f"{requests} Poisson requests at {rate:.2f}/s, n 10-{max_qubits}"
                        + (" (n >= 28: at most 2^(33-n) trajectories)" if cap_large else ""),
            "largest_request_qubits": max(sizes), "requests_28_or_more_qubits": sum(n >= 28 for n in sizes),
            "value": d["trajectories_per_s"], "unit": "trajectories/s", "p50_s": d["p50_s"],
            "p99_s": d["p99_s"], "requests": d["requests"], "wall_s": d["wall_s"], "lanes": lanes,
            "errors": sum(1 for r in reqs if srv.results[r.rid].error)}


# ------------------------------------------------------------------ headline

def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--traj", type=int, default=1000, help="trajectories per step")
    ap.add_argument("--p-dep", type=float, default=1e-3)
    ap.add_argument("--rows", type=int, default=4, help="grid rows (the headline workload is 4 x 6)")
    ap.add_argument("--cols", type=int, default=6, help="grid columns")
    ap.add_argument("--max-fuse", type=int, default=0, help="0 = autotuned")
    ap.add_argument("--tile-bits", type=int, default=0,
                    help="LDS tile sweep width (0 = autotuned with the fusion width when "
                         "--max-fuse is 0, else 13; 1 = one pass per fused gate)")
    ap.add_argument("--streams", type=int, default=2,
                    help="states (each on its own stream and host thread) a step's "
                         "trajectories are split over and run on at once")
    ap.add_argument("--naive-traj", type=int, default=4,
                    help="trajectories timed with the conventional method (0 = skip)")
    ap.add_argument("--inplace-traj", type=int, default=3,
                    help="trajectories timed with the conventional rule and in-place inner products")
    ap.add_argument("--cpu-cycles", type=int, default=1,
                    help="cycles of each oracle trajectory timed for the CPU baseline (0 = skip)")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="oracle trajectories run at once (one host thread each) for the all-core CPU baseline")
    ap.add_argument("--extras", type=int, default=1,
                    help="1: add the bounded sub-records for the other workloads")
    ap.add_argument("--workload", default="grid24",
                    choices=["grid24", "chain12", "grid28", "batched", "serving", "phase_damping",
                             "copy"],
                    help="grid24 (default): the headline line; the others print their own line; "
                         "copy: a plain device copy, the reference for calibrating byte counters")
    ap.add_argument("--requests", type=int, default=60, help="serving: number of requests")
    ap.add_argument("--max-qubits", type=int, default=26, help="serving: largest request")
    ap.add_argument("--cap-large", type=int, default=0,
                    help="serving: 1 = requests of 28 or more qubits keep at most 2^(33-n) "
                         "trajectories (a bounded run at the top of the range)")
    ap.add_argument("--copy-qubits", type=int, default=24, help="copy: state size")
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
    if args.workload != "grid24":
        return other_workload(args, qs, W, torch)

    log(f"headline: {args.rows}x{args.cols} grid, {args.traj} trajectories per step, "
        f"{args.streams} streams")
    head = run_grid(qs, W, args, torch, rows=args.rows, cols=args.cols, p_dep=args.p_dep,
                    n_traj=args.traj, steps=args.steps, warmup=args.warmup, streams=args.streams,
                    max_fuse=args.max_fuse, tile_bits=args.tile_bits, mark=True)
    log(f"headline: {head['value']:.1f} traj/s, f={head['max_fuse']} tiles={head['tile_bits']}, "
        f"sweep {head['sweep']['avg_launch_us']:.2f} us")
    n = head["qubits"]
    sw = head["sweep"]
    traffic = measured_traffic(head["tile_bits"]) if (args.rows, args.cols) == (4, 6) else None
    roofline = {
        "bound": "hbm",
        "achieved": sw["hbm"]["achieved"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
        "frac": sw["hbm"]["frac"],
        "traffic": (traffic / 1e9) if traffic else None,
        "traffic_unit": ("GB per launch of apply_tile<13>: rocprofv3 FETCH_SIZE x 2.000 + "
                         "WRITE_SIZE x 1.000 (factors from a plain 2 GiB copy), "
                         "profiles/apply_tile_grid24_counters.md, which also gives the raw "
                         "TCC_EA0 request-counter bytes (null unless that summary matches the "
                         "built kernel source and the run's tile width)"),
        "counter_summaries": ["profiles/apply_tile_grid24_counters.md",
                              "profiles/apply_tile_grid24_pmc.md",
                              "profiles/apply_tile_grid28_counters.md"],
        "kernel": "fused-gate sweep apply_tile: one read and one write of the state, the sweep's "
                  "fused blocks applied in LDS",
        "avg_launch_us": sw["avg_launch_us"],
        "avg_launch_basis": ("time during which at least one sweep ran (union of the streams' "
                             "HIP-event brackets) / launches" if args.streams > 1 else
                             "HIP-event brackets of back-to-back sweeps / launches"),
        "launches": sw["launches"], "zero_start_launches": sw["zero_start_launches"],
        "algorithmic_bytes_per_launch": sw["hbm"]["algorithmic_bytes_per_launch"],
        "floor_us_per_launch": sw["hbm"]["floor_us_per_launch"],
        "compute": sw["compute"],
        "binding_floor": sw["bound"],
    }
    copy_ref = copy_reference(qs, torch)
    roofline["copy_reference"] = copy_ref
    roofline["frac_of_copy"] = sw["hbm"]["achieved"] / copy_ref["24q" if n <= 24 else "28q"]["GB_per_s"]
    roofline["copy_basis"] = ("achieved / the GB/s of qs_copy_state on a state of the same size "
                              "class (24q: cache-resident 128 MiB buffers; 28q: HBM-resident 2 GiB)")
    log(f"copy reference: {json.dumps(copy_ref)}")

    w = W.grid24_workload(p_dep=args.p_dep, rows=args.rows, cols=args.cols)
    single = one_state_rate(qs, W, torch, w, min(args.traj, 500), qs.QS_KRAUS_DELAYED,
                            args.max_fuse, args.tile_bits)
    log(f"one state: {single['value']:.1f} traj/s")
    naive = inplace = None
    if args.naive_traj > 0:
        naive = one_state_rate(qs, W, torch, w, args.naive_traj, qs.QS_KRAUS_NAIVE, 4, 0)
        log(f"naive: {naive['value']:.3f} traj/s")
    if args.inplace_traj > 0:
        inplace = one_state_rate(qs, W, torch, w, args.inplace_traj,
                                 qs.QS_KRAUS_CONVENTIONAL_INPLACE, 4, 0)
        log(f"conventional in place: {inplace['value']:.3f} traj/s")

    extras = {}
    if args.extras and (args.rows, args.cols) == (4, 6):
        log("autotune: fixed widths 4/13, 5/13 and 4/14 for comparison")
        for f, tb in ((4, 13), (5, 13), (4, 14)):
            r = run_grid(qs, W, args, torch, n_traj=500, steps=1, warmup=1, streams=args.streams,
                         max_fuse=f, tile_bits=tb)
            extras[f"fixed_widths_{f}_{tb}"] = {
                k: v for k, v in r.items()
                if k in ("value", "unit", "max_fuse", "tile_bits", "gate_sweeps_per_traj")}
            extras[f"fixed_widths_{f}_{tb}"]["avg_launch_us"] = r["sweep"]["avg_launch_us"]
        extras["depolarizing_strength"] = []
        for p in (1e-4, 1e-2):
            log(f"p = {p:g}")
            r = run_grid(qs, W, args, torch, p_dep=p, n_traj=500, steps=1, warmup=1,
                         streams=args.streams)
            extras["depolarizing_strength"].append(
                {"p": p, "value": r["value"], "unit": r["unit"],
                 "slow_paths_per_traj": r["slow_paths_per_traj"],
                 "gate_sweeps_per_traj": r["gate_sweeps_per_traj"], "max_fuse": r["max_fuse"],
                 "tile_bits": r["tile_bits"]})
        extras["larger_states"] = []
        for nq, nt in ((26, 100), (28, 24)):
            log(f"noisy grid at {nq} qubits")
            r = run_grid(qs, W, args, torch, n_traj=nt, steps=1, warmup=1, streams=args.streams,
                         workload=W.noisy_grid_workload(nq, n_traj=nt))
            if nq >= 28:
                r["sweep"]["hbm"]["frac_of_copy"] = r["sweep"]["hbm"]["achieved"] / copy_ref["28q"]["GB_per_s"]
            extras["larger_states"].append(
                {"qubits": nq, "workload": r["workload"], "value": r["value"], "unit": r["unit"],
                 "max_fuse": r["max_fuse"], "tile_bits": r["tile_bits"], "sweep": r["sweep"]})
        log("20-qubit grid (graph replay on and off) and 20-qubit phase damping")
        small = {}
        for streams in (2, 4):
            for graph in (True, False):
                r = run_grid(qs, W, args, torch, rows=4, cols=5, n_traj=1000, steps=1, warmup=1,
                             streams=streams, graph=graph)
                small[f"{streams}_streams_graph_{'on' if graph else 'off'}"] = {
                    k: r[k] for k in ("value", "unit", "max_fuse", "tile_bits",
                                      "graph_replays_per_traj", "slow_paths_per_traj")}
        pd = phase_damped_circuit(4, 5, 1e-3)
        wl = W.TrajectoryWorkload(pd.name, pd, n_traj=200, n_samples=1)
        for graph in (True, False):
            small[f"phase_damping_1e-3_one_state_graph_{'on' if graph else 'off'}"] = one_state_rate(
                qs, W, torch, wl, 200, qs.QS_KRAUS_DELAYED, 0, 0, graph=graph)
        extras["grid20"] = small
        log("grid28 (noiseless, f <= 4)")
        extras["grid28"] = sub_grid28(qs, W, torch)
        g28 = extras["grid28"]["sweep"]["hbm"]
        g28["frac_of_copy"] = g28["achieved"] / copy_ref["28q"]["GB_per_s"]
        extras["grid28_autotuned"] = {k: v for k, v in sub_grid28(qs, W, torch, max_fuse=0).items()
                                      if k in ("value", "unit", "ms_per_state", "max_fuse",
                                               "tile_bits", "tune_ms", "sweeps_per_state")}
        log("chain12")
        extras["chain12"] = sub_chain12(qs, W, torch)
        log("batched")
        extras["batched"] = sub_batched(qs, W, torch)
        log("served")
        extras["served"] = sub_served(qs, W)

    cpu = None
    if args.cpu_cycles > 0:
        log("timing the CPU oracle ...")
        cpu = cpu_baseline(args.cpu_cycles, args.cpu_workers)

    total_traj = args.steps * args.traj
    out = {
        "metric": "trajectories/s at 24q depth-20 noisy (HBM GB/s %peak); served p50/p99 latency",
        "value": head["value"],
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * head["elapsed_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": head["workload"],
            "qubits": n,
            "trajectories_per_step": args.traj,
            "samples_per_trajectory": w.n_samples,
            "mode": "delayed",
            "max_fuse": head["max_fuse"],
            "tile_bits": head["tile_bits"],
            "widths": "autotuned" if args.max_fuse == 0 else "fixed",
            "parallelism": f"none (1 GPU); {head['streams']} trajectory streams",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "one_stream": single,
        "naive": naive,
        "speedup_vs_naive": (single["value"] / naive["value"]) if naive else None,
        "speedup_vs_naive_basis": "one state on one stream for both methods",
        "speedup_vs_naive_two_streams": (head["value"] / naive["value"]) if naive else None,
        "conventional_inplace": inplace,
        "speedup_vs_conventional_inplace": (single["value"] / inplace["value"]) if inplace else None,
        "tune_ms": head["tune_ms"],
        "gate_sweeps_per_traj": head["gate_sweeps_per_traj"],
        "sweeps_per_traj": head["sweeps_per_traj"],
        "slow_paths_per_traj": head["slow_paths_per_traj"],
        "gate_width_histogram": head["gate_width_histogram"],
        "trajectories": total_traj,
        **extras,
    }
    print(json.dumps(out), flush=True)
    return 0


def copy_reference(qs, torch, qubit_sizes=(24, 28)):
    """Achievable bandwidth of a plain state copy (qs_copy_state: one read and
    one write of the state, like a sweep, with 16-byte accesses): at 24
    qubits the two 128 MiB states sit in the Infinity Cache, at 28 qubits (2
    GiB each) they do not.  torch's own device copy is timed beside it.
    Events on the default stream, outside the timed region."""
    out = {}
    for q in qubit_sizes:
        reps = 20 if q <= 24 else 5
        nbytes = 2 * (8 << q)

        def timed(fn):
            for _ in range(3):
                fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            return nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

        with qs.State(q) as a, qs.State(q) as b:
            gbps = timed(lambda: qs.qs_copy_state(b.h, a.h))
        x = torch.zeros(1 << q, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        tgbps = timed(lambda: y.copy_(x))
        del x, y
        torch.cuda.empty_cache()
        out[f"{q}q"] = {"bytes_per_copy": nbytes, "GB_per_s": gbps, "torch_copy_GB_per_s": tgbps}
    return out


# ------------------------------------------------------------------ standalone lines

def bench_copy(args, torch) -> int:
    """Device-to-device copy of a complex64 state: the kernel of known
    traffic whose FETCH_SIZE / WRITE_SIZE readings scale the counters taken
    on the sweep kernels."""
    a = torch.randn(1 << args.copy_qubits, dtype=torch.complex64, device="cuda")
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
                      "config": {"workload": f"copy of a 2^{args.copy_qubits}-amplitude complex64 state",
                                 "bytes_per_copy": nbytes}}), flush=True)
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


def other_workload(args, qs, W, torch) -> int:
    common = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic"}
    if args.workload == "copy":
        return bench_copy(args, torch)
    if args.workload == "chain12":
        r = sub_chain12(qs, W, torch, steps=args.steps)
        out = {"metric": "trajectories/s, 12-qubit chain depth 20, 1000 samples each", **common,
               "value": r["value"], "unit": r["unit"], "ms_per_step": 1e5 / r["value"],
               "config": {"workload": r["workload"]}, **{k: v for k, v in r.items() if k != "value"}}
    elif args.workload == "grid28":
        r = sub_grid28(qs, W, torch, steps=args.steps)
        out = {"metric": "28-qubit noiseless grid: evolved states/s (with 1e5 samples each)", **common,
               "value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_state"],
               "config": {"workload": r["workload"]}, **{k: v for k, v in r.items() if k != "value"}}
    elif args.workload == "batched":
        r = sub_batched(qs, W, torch, steps=args.steps)
        out = {"metric": "batched trajectories/s (persistent launch)", **common,
               "value": r["value"], "unit": r["unit"], "ms_per_step": 4096e3 / r["value"],
               "config": {"workload": r["workload"]}, **{k: v for k, v in r.items() if k != "value"}}
    elif args.workload == "serving":
        r = sub_served(qs, W, requests=args.requests, max_qubits=args.max_qubits,
                       cap_large=bool(args.cap_large))
        out = {"metric": "served trajectories/s; p50/p99 request latency", **common,
               "value": r["value"], "unit": r["unit"], "ms_per_step": 1e3 * r["wall_s"],
               "config": {"workload": r["workload"]}, **{k: v for k, v in r.items() if k != "value"}}
    else:  # phase damping
        rows = []
        for (r_, c_, n_traj, n_naive) in ((4, 5, 200, 4), (3, 9, 6, 1)):
            for lam in (1e-4, 1e-3, 1e-2, 1e-1):
                circ = phase_damped_circuit(r_, c_, lam)
                wl = W.TrajectoryWorkload(circ.name, circ, n_traj=n_traj, n_samples=1)
                d = one_state_rate(qs, W, torch, wl, n_traj, qs.QS_KRAUS_DELAYED, 0, 0)
                nv = one_state_rate(qs, W, torch, wl, n_naive, qs.QS_KRAUS_NAIVE, 4, 0, warm=0)
                d4 = states_rate(qs, torch, wl, 2 * n_traj, 4, qs.QS_KRAUS_DELAYED)
                row = {"qubits": r_ * c_, "lambda": lam, "delayed_traj_per_s": d["value"],
                       "naive_traj_per_s": nv["value"], "speedup": d["value"] / nv["value"],
                       "delayed_4_states_traj_per_s": d4["value"],
                       "max_fuse": d["max_fuse"], "tile_bits": d["tile_bits"]}
                log(json.dumps(row))
                rows.append(row)
        out = {"metric": "trajectories/s vs phase-damping strength (delayed vs conventional)",
               **common, "value": rows[1]["delayed_traj_per_s"], "unit": "trajectories/s",
               "ms_per_step": None,
               "config": {"workload": "grid 4x5 and 3x9, 20 cycles, phase damping after every gate"},
               "sweep": rows}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
