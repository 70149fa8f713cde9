"""Host-side checks of libqs that need no GPU: every symbol the header
declares is exported, argument validation, the fusion planner (Section 3.2),
Kraus bounds (Section 3.5) and the library's own Philox."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import dense

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_2111_02396_amd as qs

    if not os.path.exists(qs.LIB_PATH):
        from paper_2111_02396_amd import _build

        _build.build()
    qs.load()
    return qs


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "qs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qs_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported(lib):
    names = _declared_functions()
    assert len(names) >= 18
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (qs_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = lib.load()
    for n in names:
        assert hasattr(L, n)


def test_validation_before_device_work(lib):
    with pytest.raises(lib.QsError) as e:
        lib.qs_create_state(0)
    assert e.value.code == lib.QS_ERR_INVALID_ARGUMENT
    with pytest.raises(lib.QsError) as e:
        lib.qs_create_state(35)
    assert e.value.code == lib.QS_ERR_INVALID_ARGUMENT
    with pytest.raises(lib.QsError):
        lib.qs_destroy_state(None)
    assert "null" in lib.qs_last_error_message()
    with pytest.raises(lib.QsError) as e:
        lib.qs_copy_state(None, None)
    assert e.value.code == lib.QS_ERR_INVALID_ARGUMENT


def test_philox_matches_oracle(lib, orc):
    rng = np.random.default_rng(3)
    for _ in range(300):
        c = [int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        k = [int(x) for x in rng.integers(0, 2**32, size=2, dtype=np.uint64)]
        assert lib.qs_philox4x32_10(c, k) == orc.philox4x32_10(c, k)


@pytest.mark.parametrize("name,kraus,expect,mix", [
    ("depolarize", W.depolarize(1e-3), [1 - 1e-3] + [1e-3 / 3] * 3, True),
    ("amplitude_damp", W.amplitude_damp(1e-3), [1 - 1e-3, 0.0], False),
    ("phase_damp", W.phase_damp(0.2), [0.8, 0.0], False),
    ("bit_flip", W.bit_flip(0.1), [0.9, 0.1], True),
])
def test_kraus_bounds_closed_forms(lib, name, kraus, expect, mix):
    pbar, m = lib.qs_kraus_bounds(kraus)
    assert m == mix
    assert np.allclose(pbar, expect, rtol=0, atol=1e-15)


def test_kraus_bounds_general(lib, orc):
    rng = np.random.default_rng(4)
    for k in (1, 2):
        for _ in range(5):
            ks = [W.random_matrix(k, rng) for _ in range(3)]
            pb, _ = lib.qs_kraus_bounds(ks)
            ref = [max(np.linalg.svd(K, compute_uv=False).min() ** 2, 0.0) for K in ks]
            assert np.allclose(pb, ref, rtol=1e-12, atol=1e-14)
    pb, mix = lib.qs_kraus_bounds(W.decay_dephase(0.2, 1.0, 0.5))
    assert not mix
    ref, _ = orc.kraus_bounds(W.decay_dephase(0.2, 1.0, 0.5))
    assert np.allclose(pb, ref, atol=1e-15)


def _check_plan(lib, c, f):
    blocks, op_block = lib.qs_fusion_plan(c, f)
    U_ref = dense.circuit_unitary(c)
    U = np.eye(1 << c.n, dtype=np.complex128)
    for targets, m in blocks:
        assert len(targets) <= max(f, max(o.k for o in c.ops))
        assert list(targets) == sorted(targets)
        U = dense.full_operator(c.n, list(targets), m) @ U
    assert np.max(np.abs(U - U_ref)) < 1e-12
    assert np.all(op_block >= 0) and np.all(op_block < len(blocks))
    return blocks


@pytest.mark.parametrize("f", [1, 2, 3, 4, 5])
def test_fusion_equals_unfused(lib, f):
    c = W.random_gate_circuit(7, 80, seed=f, max_k=3)
    blocks = _check_plan(lib, c, f)
    if f >= 3:
        assert len(blocks) < len(c.ops)


def test_fusion_on_grid_layers(lib):
    c = W.grid_circuit(2, 4, 6, seed=3)
    for f in (2, 3, 4):
        blocks = _check_plan(lib, c, f)
        assert len(blocks) <= len(c.ops)
    # wider fusion never needs more blocks on this circuit
    n2 = len(lib.qs_fusion_plan(c, 2)[0])
    n4 = len(lib.qs_fusion_plan(c, 4)[0])
    assert n4 < n2


def test_fusion_wide_gates_alone(lib):
    rng = np.random.default_rng(8)
    ops = [W.Op(W.GATE, (0, 1, 2, 3, 4), [W.random_unitary(5, rng)]),
           W.Op(W.GATE, (2,), [W.SQRT_X]),
           W.Op(W.GATE, (5, 6), [W.CZ]),
           W.Op(W.GATE, (1, 3, 5), [W.random_unitary(3, rng)])]
    c = W.Circuit(7, ops)
    _check_plan(lib, c, 2)


def test_fusion_rejects_channels(lib):
    c = W.random_noisy_circuit(3, 2, seed=1)
    with pytest.raises(lib.QsError):
        lib.qs_fusion_plan(c, 3)


def test_grid24_plan_size(lib):
    """The default-pick plan of the benchmark circuit: report how many
    sweeps fusion leaves per trajectory at each width."""
    c = W.grid24_workload().circuit.gates_only()
    sizes = {f: len(lib.qs_fusion_plan(c, f)[0]) for f in (2, 3, 4, 5)}
    assert sizes[4] < sizes[2] < len(c.ops)


@pytest.mark.parametrize("tile_bits", [1, 10, 12, 13])
@pytest.mark.parametrize("f", [2, 4])
def test_sweep_grouping_keeps_order(lib, tile_bits, f):
    """Regrouping fused blocks into tile sweeps reorders them; the product in
    the new order must still equal the circuit."""
    c = W.grid_circuit(2, 5, 8, seed=2)  # 10 qubits: tiles are narrower than the state
    blocks, _ = lib.qs_fusion_plan(c, f)
    ns, order, sweep_of, bits = lib.qs_sweep_plan(c, f, tile_bits)
    assert sorted(order.tolist()) == list(range(len(blocks)))
    assert np.all(np.diff(sweep_of) >= 0)
    rng = np.random.default_rng(tile_bits + 10 * f)
    psi0 = rng.standard_normal(1 << c.n) + 1j * rng.standard_normal(1 << c.n)
    psi = psi0.copy()
    for b in order:
        targets, m = blocks[b]
        psi = dense.apply_tensor(psi, list(targets), m)
    ref = psi0.copy()
    for op in c.ops:
        ref = dense.apply_tensor(ref, list(op.qubits), op.mats[0])
    assert np.max(np.abs(psi - ref)) < 1e-12
    if tile_bits >= 10:
        for i, b in enumerate(order):
            mask = int(bits[sweep_of[i]])
            assert all((mask >> q) & 1 for q in blocks[b][0])
            assert mask & 0xF == 0xF
            assert bin(mask).count("1") <= tile_bits


def test_sweep_grouping_cuts_passes(lib):
    c = W.grid24_workload().circuit.gates_only()
    ns_off, *_ = lib.qs_sweep_plan(c, 4, 1)
    ns_13, *_ = lib.qs_sweep_plan(c, 4, 13)
    assert ns_13 * 2.5 < ns_off


def test_fusion_merges_subset_blocks(lib):
    """No block of the default grid plan is a qubit subset of the nearest
    block sharing a qubit with it (such blocks are folded in), and the plan
    still multiplies out to the circuit."""
    c = W.grid_circuit(2, 4, 6, seed=3)
    blocks = _check_plan(lib, c, 4)
    assert all(len(t) > 1 for t, _ in blocks)
    for i, (ti, _) in enumerate(blocks):
        later = [tj for tj, _ in blocks[i + 1:] if set(tj) & set(ti)]
        if later:
            assert not set(ti) <= set(later[0])


def test_batched_planning_without_trajectories(lib):
    """The batched call's host planning runs before any device work, so a
    batch with no trajectories completes on the host: an empty circuit (no
    ops, empty matrix pool) is a valid circuit, a repeated call reuses the
    cached circuit model, and a circuit with ops but no op records is
    rejected."""
    empty = W.Circuit(5, [])
    grid = W.grid_circuit(3, 4, 3, p_dep=0.01, seed=4)
    items = [W.TrajectoryWorkload("empty", empty, n_traj=0, n_samples=4),
             W.TrajectoryWorkload("grid", grid, n_traj=0, n_samples=4)]
    for _ in range(2):
        _, stats = lib.qs_run_batched(items, max_fuse=3)
        assert stats["jobs"] == 0
    pb = lib.PreparedBatch(items[1:])
    circ = ctypes.cast(pb.items[0].circuit, ctypes.POINTER(lib.QsCircuit)).contents
    circ.ops = None
    with pytest.raises(lib.QsError) as e:
        lib.qs_run_batched(pb, max_fuse=3)
    assert e.value.code == lib.QS_ERR_INVALID_ARGUMENT


def test_batched_planning_from_concurrent_threads(lib):
    """Several host threads plan batches at once (no trajectories, so no
    device work): the circuit-model cache, the batched plan cache and the
    planner's worker pool are shared, and every call must still succeed
    with the same counts."""
    from concurrent.futures import ThreadPoolExecutor

    circuits = [W.generic_grid_circuit(n, 6, p_dep=0.01, seed=s) for s, n in enumerate(range(10, 16))]

    def plan(seed):
        rng = np.random.default_rng(seed)
        picks = rng.permutation(len(circuits))[:4]
        items = [W.TrajectoryWorkload(f"c{i}", circuits[i], n_traj=0, n_samples=2, circuit_id=int(i))
                 for i in picks]
        out = []
        for _ in range(5):
            _, stats = lib.qs_run_batched(items, max_fuse=3)
            out.append(stats["jobs"])
        return out

    with ThreadPoolExecutor(max_workers=6) as ex:
        results = list(ex.map(plan, range(12)))
    assert all(r == [0] * 5 for r in results)
