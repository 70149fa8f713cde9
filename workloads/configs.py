"""The five benchmark workloads, as seeded synthetic inputs.

The paper measures on generator-defined random circuits ("random circuits
with depth 20", Section 3.6; phase damping on random circuits, Fig.
perf_noise), not on a dataset; these recipes stand in for them.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .circuits import Circuit, chain_circuit, generic_grid_circuit, grid_circuit, readout_arrays


@dataclass
class TrajectoryWorkload:
    name: str
    circuit: Circuit
    n_traj: int
    seed: int = 0          # Philox key
    circuit_id: int = 0    # Philox counter word 2
    n_samples: int = 1
    e0: Optional[np.ndarray] = None   # readout P(1|0) per qubit
    e1: Optional[np.ndarray] = None   # readout P(0|1) per qubit
    max_fuse: int = 4


def chain12_workload() -> TrajectoryWorkload:
    """12-qubit chain, depth 20, depolarizing 1e-3 after every gate;
    100 trajectories x 1000 samples, Philox seed 0."""
    c = chain_circuit(12, 20, p_dep=1e-3, seed=0)
    return TrajectoryWorkload("chain12-depth20-dep1e-3", c, n_traj=100, seed=0,
                              n_samples=1000, max_fuse=3)


def grid28_workload() -> TrajectoryWorkload:
    """28-qubit 4x7 grid, depth 20, noiseless; one state, 1e5 samples."""
    c = grid_circuit(4, 7, 20, seed=0)
    return TrajectoryWorkload("grid4x7-depth20-noiseless", c, n_traj=1, seed=0,
                              n_samples=100000, max_fuse=4)


def grid24_workload(p_dep: float = 1e-3, gamma: float = 1e-3, readout: float = 2e-2,
                    n_traj: int = 1000, rows: int = 4, cols: int = 6) -> TrajectoryWorkload:
    """24-qubit 4x6 grid, depth 20: depolarizing after every gate, amplitude
    damping on every qubit after every moment, readout flips; 1 shot per
    trajectory."""
    c = grid_circuit(rows, cols, 20, p_dep=p_dep, gamma=gamma, seed=0)
    e0, e1 = readout_arrays(rows * cols, readout, readout)
    return TrajectoryWorkload(f"grid{rows}x{cols}-depth20-dep{p_dep:g}-ad{gamma:g}-ro{readout:g}",
                              c, n_traj=n_traj, seed=0, n_samples=1, e0=e0, e1=e1,
                              max_fuse=4)


def noisy_grid_workload(n: int, p_dep: float = 1e-3, gamma: float = 1e-3, readout: float = 2e-2,
                        n_traj: int = 100) -> TrajectoryWorkload:
    """The grid24 noise model on an n-qubit generic grid (R = floor(sqrt(n))
    rows, last row partial), depth 20: for sizes whose state no longer fits
    the device's last-level cache (26 and 28 qubits)."""
    c = generic_grid_circuit(n, 20, p_dep=p_dep, gamma=gamma, seed=0)
    e0, e1 = readout_arrays(n, readout, readout)
    return TrajectoryWorkload(f"ggrid{n}-depth20-dep{p_dep:g}-ad{gamma:g}-ro{readout:g}", c,
                              n_traj=n_traj, seed=0, n_samples=1, e0=e0, e1=e1, max_fuse=4)


def batched_workload(n_circuits: int = 256, traj_per_circuit: int = 16, seed: int = 0,
                     n_lo: int = 12, n_hi: int = 18, d_lo: int = 10, d_hi: int = 40,
                     p_dep: float = 1e-3) -> List[TrajectoryWorkload]:
    """Many small circuits of uneven sizes (qubit counts and depths uniform)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_circuits):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        c = generic_grid_circuit(n, d, p_dep=p_dep, seed=seed * 100003 + i)
        out.append(TrajectoryWorkload(f"batch{i}-n{n}-d{d}", c, n_traj=traj_per_circuit,
                                      seed=seed, circuit_id=i, n_samples=1, max_fuse=3))
    return out


@dataclass
class Request:
    rid: int
    arrival_s: float
    workload: TrajectoryWorkload


def serving_requests(n_requests: int, rate_hz: float, seed: int = 0, n_lo: int = 10,
                     n_hi: int = 32, d_lo: int = 10, d_hi: int = 40,
                     p_lo: float = 1e-4, p_hi: float = 1e-2, t_lo: int = 1,
                     t_hi: int = 1000) -> List[Request]:
    """Poisson arrivals; n, depth uniform; p and trajectory count log-uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        p = float(math.exp(rng.uniform(math.log(p_lo), math.log(p_hi))))
        nt = int(round(math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))))
        nt = max(t_lo, min(t_hi, nt))
        c = generic_grid_circuit(n, d, p_dep=p, seed=seed * 7919 + rid)
        w = TrajectoryWorkload(f"req{rid}-n{n}-d{d}", c, n_traj=nt, seed=seed, circuit_id=rid,
                               n_samples=1, max_fuse=4)
        out.append(Request(rid, t, w))
    return out
