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
    # another seed draws another 1-qubit layer
    c = W.grid_circuit(4, 6, 20, p_dep=1e-3, gamma=1e-3, seed=1)
    assert [o.name for o in a.ops[:24]] != [o.name for o in c.ops[:24]]


def test_batched_and_serving_shapes():
    ws = W.batched_workload(n_circuits=16)
    assert all(12 <= w.circuit.n <= 18 for w in ws)
    reqs = W.serving_requests(50, rate_hz=10.0, seed=1)
    ts = [r.arrival_s for r in reqs]
    assert all(b > a for a, b in zip(ts, ts[1:]))
    assert all(10 <= r.workload.circuit.n <= 32 for r in reqs)
    assert all(1 <= r.workload.n_traj <= 1000 for r in reqs)


def test_coherent_error_gates_closed_forms():
    """fSim special cases (Section 5.2.2): theta = 0, phi = pi is CZ;
    theta = -pi/2, phi = 0 is iSWAP (i on the swapped pair); two sqrt(iSWAP)
    make iSWAP; fSim angles add under products; U_ZZ at zeta T = 1/2 is CZ;
    exp(i varphi Z) is the matrix exponential of i varphi Z."""
    import math
    from scipy.linalg import expm
    assert np.allclose(W.fsim(0.0, math.pi), W.CZ, atol=1e-15)
    iswap = np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]])
    assert np.allclose(W.fsim(-math.pi / 2, 0.0), iswap, atol=1e-15)
    assert np.allclose(W.SQRT_ISWAP @ W.SQRT_ISWAP, iswap, atol=1e-15)
    a, b, c, d = 0.3, -0.7, 1.1, 0.25
    assert np.allclose(W.fsim(a, b) @ W.fsim(c, d), W.fsim(a + c, b + d), atol=1e-14)
    for U in (W.fsim(a, b), W.u_zz(3e6, 10e-9), W.z_phase(0.4)):
        assert np.allclose(U.conj().T @ U, np.eye(U.shape[0]), atol=1e-14)
    assert np.allclose(W.u_zz(0.5 / 10e-9, 10e-9), W.CZ, atol=1e-12)
    assert np.allclose(W.z_phase(0.4), expm(1j * 0.4 * W.PAULI_Z), atol=1e-14)


def test_approx_noise_grid_structure():
    c = W.approx_noise_grid_circuit(3, 4, 4, seed=2, zeta=1e6)
    names = [o.name for o in c.ops]
    pairs = names.count("sqrt_iswap")
    assert pairs > 0
    assert names.count("fsim_error") == pairs and names.count("u_zz") == pairs
    assert names.count("z_phase") == 4 * pairs and names.count("depolarize2") == pairs
    assert names.count("decay_dephase") == 2 * 4 * 12
    # each dressed gate reads: z, z, sqrt_iswap, fsim_error, u_zz, z, z, depolarize2
    i = names.index("sqrt_iswap")
    assert names[i - 2:i + 6] == ["z_phase", "z_phase", "sqrt_iswap", "fsim_error", "u_zz",
                                  "z_phase", "z_phase", "depolarize2"]
    again = W.approx_noise_grid_circuit(3, 4, 4, seed=2, zeta=1e6)
    assert all(np.array_equal(x.mats[0], y.mats[0]) for x, y in zip(c.ops, again.ops))
