"""GPU parity of the batched persistent launch (many small circuits in one
kernel) against the oracle and against the one-trajectory-per-call driver."""

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can be slow)

import workloads as W
from workloads.configs import TrajectoryWorkload
from gpu_helpers import SAMPLE_TIE, compare_choices

pytestmark = pytest.mark.gpu


def _items(specs):
    out = []
    for i, (n, depth, p, ntraj, nsamp) in enumerate(specs):
        c = W.generic_grid_circuit(n, depth, p_dep=p, seed=100 + i)
        e0, e1 = W.readout_arrays(n, 0.01, 0.02)
        out.append(TrajectoryWorkload(f"b{i}", c, n_traj=ntraj, seed=7, circuit_id=i,
                                      n_samples=nsamp, e0=e0, e1=e1, max_fuse=3))
    return out


def test_batched_matches_oracle(qs, orc):
    items = _items([(10, 6, 0.05, 3, 20), (12, 8, 0.03, 3, 20), (13, 5, 0.05, 2, 20),
                    (14, 5, 0.03, 2, 20), (15, 4, 0.05, 2, 20)])
    res, stats = qs.qs_run_batched(items)
    assert stats["jobs"] == sum(w.n_traj for w in items)
    assert stats["resident_jobs"] == 3 + 3 + 2
    for w, r in zip(items, res):
        m = orc.Marshalled(w.circuit)
        for t in range(w.n_traj):
            ref = orc.run_trajectory(w.circuit, t, seed=w.seed, circ=w.circuit_id,
                                     n_samples=w.n_samples, e0=w.e0, e1=w.e1, marshalled=m)
            _, tie = compare_choices(r["choices"][t], ref)
            assert tie == 0
            mism = np.nonzero(r["samples"][t] != ref["samples"])[0]
            assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE), (w.name, t, mism)


def test_batched_matches_oracle_and_driver_all_sizes(qs, orc):
    """Every size of the batched range, 12..18 qubits: n <= 13 keeps the state
    in LDS, 14..18 stream tiles of a per-workgroup slot.  Choices and samples
    against the oracle (samples may differ only at a prefix tie), and the
    batched launch against the one-call driver on the same trajectories."""
    items = _items([(n, 8, 0.01, 4, 8) for n in range(12, 19)])
    res, _ = qs.qs_run_batched(items)
    for w, r in zip(items, res):
        with qs.State(w.circuit.n) as st:
            d = qs.qs_run_trajectories(st.h, w.circuit, w.n_traj, seed=w.seed,
                                       circuit_id=w.circuit_id, n_samples=w.n_samples,
                                       p0to1=w.e0, p1to0=w.e1, max_fuse=3)
        assert np.array_equal(r["choices"], d["choices"])
        m = orc.Marshalled(w.circuit)
        for t in range(w.n_traj):
            ref = orc.run_trajectory(w.circuit, t, seed=w.seed, circ=w.circuit_id,
                                     n_samples=w.n_samples, e0=w.e0, e1=w.e1, marshalled=m)
            _, tie = compare_choices(r["choices"][t], ref)
            assert tie == 0
            for got in (r["samples"][t], d["samples"][t]):
                mism = np.nonzero(got != ref["samples"])[0]
                assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE), (w.name, t, mism)


def test_batched_offsets_and_determinism(qs):
    items = _items([(12, 6, 0.05, 6, 5), (16, 4, 0.05, 3, 5)])
    a, _ = qs.qs_run_batched(items)
    b, _ = qs.qs_run_batched(items)
    for x, y in zip(a, b):
        assert np.array_equal(x["samples"], y["samples"])
        assert np.array_equal(x["choices"], y["choices"])
    tail = _items([(12, 6, 0.05, 6, 5), (16, 4, 0.05, 3, 5)])
    for w in tail:
        w.traj_offset = 2
        w.n_traj -= 2
    c, _ = qs.qs_run_batched(tail)
    for x, z in zip(a, c):
        assert np.array_equal(x["choices"][2:], z["choices"])
        assert np.array_equal(x["samples"][2:], z["samples"])


def test_batched_rejects_non_mixtures(qs):
    c = W.generic_grid_circuit(10, 4, p_dep=0.01, gamma=0.01, seed=1)
    w = TrajectoryWorkload("ad", c, n_traj=1, n_samples=1)
    with pytest.raises(qs.QsError) as e:
        qs.qs_run_batched([w])
    assert e.value.code == qs.QS_ERR_NOT_SUPPORTED


def test_batched_heavy_noise_patched_blocks_match_oracle(qs, orc):
    """Every job draws its channels on the device and recomputes, in FP64,
    the fused blocks whose picks differ from the defaults.  Heavy noise (p =
    0.3) patches most blocks of most jobs; two circuits of different sizes
    (one resident, one tiled) give the channel table two ranges.  A large
    batch and a small one agree on their common trajectories (the launch
    shape does not change a job's result), and both agree with the oracle."""
    specs = [(12, 8, 0.3, 0, 6), (16, 5, 0.3, 0, 6)]
    items = _items(specs)
    nch = [qs.MarshalledCircuit(w.circuit).n_channels for w in items]
    for w, k in zip(items, nch):
        w.n_traj = 24000 // k + 3
    big, _ = qs.qs_run_batched(items)
    non_default = sum(int(np.count_nonzero(r["choices"])) for r in big)
    assert non_default > 8192, non_default
    small_items = _items(specs)
    for w in small_items:
        w.n_traj = 3
    small, _ = qs.qs_run_batched(small_items)
    for r_big, r_small in zip(big, small):
        assert np.array_equal(r_big["choices"][:3], r_small["choices"])
        assert np.array_equal(r_big["samples"][:3], r_small["samples"])
    for w, r in zip(items, big):
        m = orc.Marshalled(w.circuit)
        for t in (0, 1, w.n_traj - 1):
            ref = orc.run_trajectory(w.circuit, t, seed=w.seed, circ=w.circuit_id,
                                     n_samples=w.n_samples, e0=w.e0, e1=w.e1, marshalled=m)
            _, tie = compare_choices(r["choices"][t], ref)
            assert tie == 0
            mism = np.nonzero(r["samples"][t] != ref["samples"])[0]
            assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE), (w.name, t, mism)


@pytest.mark.parametrize("f", [2, 4, 5])
def test_batched_patched_wide_blocks_match_oracle(qs, orc, f):
    """Patched blocks of every width the planner forms at fusion width f
    (k = 5 blocks are recomputed 16 columns at a time), on a resident and a
    tiled circuit, against the oracle; the picks equal the one-call driver's."""
    items = _items([(11, 6, 0.2, 3, 16), (15, 4, 0.2, 2, 16)])
    res, stats = qs.qs_run_batched(items, max_fuse=f)
    assert stats["max_fuse_used"] == f
    for w, r in zip(items, res):
        assert np.count_nonzero(r["choices"]) > 0
        m = orc.Marshalled(w.circuit)
        for t in range(w.n_traj):
            ref = orc.run_trajectory(w.circuit, t, seed=w.seed, circ=w.circuit_id,
                                     n_samples=w.n_samples, e0=w.e0, e1=w.e1, marshalled=m)
            _, tie = compare_choices(r["choices"][t], ref)
            assert tie == 0
            mism = np.nonzero(r["samples"][t] != ref["samples"])[0]
            assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE), (w.name, f, t, mism)


def test_batched_without_recorded_choices(qs):
    """Choices not asked for are not written; the samples do not depend on it."""
    items = _items([(12, 6, 0.05, 4, 8), (16, 4, 0.05, 2, 8)])
    a, _ = qs.qs_run_batched(items)
    b, _ = qs.qs_run_batched(items, record_choices=False)
    for x, y in zip(a, b):
        assert "choices" not in y
        assert np.array_equal(x["samples"], y["samples"])


def _wide_noisy(n, seed, p):
    """Random gates on 1..5 unsorted targets, each followed by 1-qubit
    depolarizing on its targets and, for 2-qubit gates, 2-qubit
    depolarizing (16 Kraus operators) on the pair."""
    from workloads.circuits import CHANNEL, Op, depolarize2
    c = W.random_noisy_circuit(n, 24, seed, p_dep=p, gamma=0.0, max_k=5)
    ops = []
    for o in c.ops:
        ops.append(o)
        if o.kind != CHANNEL and o.k == 2:
            ops.append(Op(CHANNEL, o.qubits, depolarize2(p), o.moment, "depolarize2"))
    c.ops = ops
    return c


@pytest.mark.parametrize("f", [4, 5])
def test_batched_patched_blocks_with_wide_gates_match_oracle(qs, orc, f):
    """Blocks that hold a channel next to a 3- to 5-qubit gate with unsorted
    targets (the generic re-fusion path for operations on 4 or 5 qubits)
    and 2-qubit channels with 16 Kraus operators, on a resident and a tiled
    circuit, against the oracle."""
    items = []
    for i, n in enumerate((11, 14)):
        c = _wide_noisy(n, 40 + i, 0.25)
        assert max(o.k for o in c.ops) >= 4
        e0, e1 = W.readout_arrays(n, 0.01, 0.02)
        items.append(TrajectoryWorkload(f"w{i}", c, n_traj=3, seed=11, circuit_id=i,
                                        n_samples=16, e0=e0, e1=e1, max_fuse=f))
    res, _ = qs.qs_run_batched(items, max_fuse=f)
    for w, r in zip(items, res):
        assert np.count_nonzero(r["choices"]) > 0
        m = orc.Marshalled(w.circuit)
        for t in range(w.n_traj):
            ref = orc.run_trajectory(w.circuit, t, seed=w.seed, circ=w.circuit_id,
                                     n_samples=w.n_samples, e0=w.e0, e1=w.e1, marshalled=m)
            _, tie = compare_choices(r["choices"][t], ref)
            assert tie == 0
            mism = np.nonzero(r["samples"][t] != ref["samples"])[0]
            assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE), (w.name, f, t, mism)


def test_batched_samples_into_pinned_and_pageable_buffers(qs, monkeypatch):
    """An item with 16384 or more samples lands straight in a pinned caller
    buffer; pageable buffers go through the library's staging.  Both give
    the same samples, and views of a prepared batch's buffers hold the
    latest call's results."""
    items = _items([(12, 8, 0.02, 40, 1000), (11, 6, 0.02, 3, 20)])
    pinned = qs.PreparedBatch(items)
    a, _ = qs.qs_run_batched(pinned)
    v, _ = qs.qs_run_batched(pinned, copy=False)
    monkeypatch.setattr(qs, "_sample_buffer",
                        lambda n: (lambda x: (x, x))(np.zeros(max(n, 1), dtype=np.uint64)))
    pageable = qs.PreparedBatch(items)
    b, _ = qs.qs_run_batched(pageable)
    for x, y, z in zip(a, b, v):
        assert np.array_equal(x["samples"], y["samples"])
        assert np.array_equal(x["samples"], z["samples"])
        assert np.array_equal(x["choices"], y["choices"])
