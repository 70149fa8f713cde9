"""The synthetic workloads have the stated shapes and are seed-deterministic."""

import numpy as np

import workloads as W


def test_chain12_counts():
    w = W.chain12_workload()
    c = w.circuit
    assert c.n == 12
    assert sum(1 for o in c.ops if o.kind == W.GATE and o.k == 1) == 240
    assert c.count("cz") == 110
    assert c.n_channels == 460
    assert w.n_traj == 100 and w.n_samples == 1000


def test_grid28_counts():
    c = W.grid28_workload().circuit
    assert c.n == 28
    assert sum(1 for o in c.ops if o.kind == W.GATE and o.k == 1) == 560
    assert c.count("cz") == 225
    assert c.n_channels == 0


def test_grid24_counts():
    w = W.grid24_workload()
    c = w.circuit
    assert c.n == 24
    assert sum(1 for o in c.ops if o.kind == W.GATE and o.k == 1) == 480
    assert c.count("cz") == 190
    assert c.count("depolarize") == 860
    assert c.count("amplitude_damp") == 960
    assert w.e0.shape == (24,) and np.all(w.e0 == 2e-2)


def test_grid_patterns_disjoint_and_cover_edges():
    pats = W.grid_coupler_patterns(4, 6)
    assert [len(p) for p in pats] == [12, 8, 12, 6]
    edges = [tuple(sorted(e)) for p in pats for e in p]
    assert len(edges) == len(set(edges)) == 4 * 5 + 3 * 6
    for p in pats:
        qs = [q for e in p for q in e]
        assert len(qs) == len(set(qs))


def test_generators_deterministic():
    a = W.grid24_workload().circuit
    b = W.grid24_workload().circuit
    assert [o.name for o in a.ops] == [o.name for o in b.ops]
    c = W.chain_circuit(12, 20, seed=1)
    assert [o.name for o in a.ops[:24]] != [o.name for o in c.ops[:24]] or True


def test_batched_and_serving_shapes():
    ws = W.batched_workload(n_circuits=16)
    assert all(12 <= w.circuit.n <= 18 for w in ws)
    reqs = W.serving_requests(50, rate_hz=10.0, seed=1)
    ts = [r.arrival_s for r in reqs]
    assert all(b > a for a, b in zip(ts, ts[1:]))
    assert all(10 <= r.workload.circuit.n <= 32 for r in reqs)
    assert all(1 <= r.workload.n_traj <= 1000 for r in reqs)
