"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bars: amplitudes within 1e-5 relative L2 (normalised states); FP64 norms to
rounding; Kraus choices and bitstrings bit-exact away from threshold ties.
"""

import math

import torch  # noqa: F401  (imported at collection: the first import can be slow)

import numpy as np
import pytest

import workloads as W
from gpu_helpers import (AMP_TOL, SAMPLE_TIE, compare_choices, random_state, rel_l2)

pytestmark = pytest.mark.gpu

TARGET_PATTERNS = {
    1: [[0], [1], [5], [6], [-1]],
    2: [[0, 1], [1, 0], [0, -1], [3, 7], [-2, -1], [6, 9]],
    3: [[0, 1, 2], [2, 0, 5], [6, 7, 8], [0, 6, -1], [4, 5, 6]],
    4: [[0, 1, 2, 3], [3, 1, 0, 2], [6, 7, 8, 9], [0, 3, 7, -1], [5, 6, -2, -1]],
    5: [[0, 1, 2, 3, 4], [4, 2, 0, 1, 3], [6, 7, 8, 9, 10], [0, 2, 6, 9, -1], [1, 5, 7, -2, -1]],
}


def _resolve(targets, n):
    return [t if t >= 0 else n + t for t in targets]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n", [11, 16, 21])
def test_apply_fused_gate_parity(qs, orc, k, n):
    rng = np.random.default_rng(1000 * k + n)
    psi0 = random_state(n, rng)
    with qs.State(n) as st:
        for pat in TARGET_PATTERNS[k]:
            t = _resolve(pat, n)
            U = W.random_matrix(k, rng)
            qs.qs_load_state_from_host(st.h, psi0)
            qs.qs_apply_fused_gate(st.h, t, U)
            got = qs.qs_copy_state_to_host(st.h)
            ref = psi0.astype(np.complex128)
            orc.apply_matrix(ref, t, U)
            err = rel_l2(got, ref)
            assert err < AMP_TOL, (k, n, t, err)


def test_norm_parity_and_determinism(qs, orc):
    rng = np.random.default_rng(5)
    for n in (3, 12, 20, 23):
        psi = (random_state(n, rng) * np.float32(1.7)).astype(np.complex64)
        with qs.State(n) as st:
            qs.qs_load_state_from_host(st.h, psi)
            a = qs.qs_norm(st.h)
            b = qs.qs_norm(st.h)
            assert a == b
            ref = orc.norm_sq(psi.astype(np.complex128))
            assert abs(a - ref) <= 1e-12 * ref


def test_circuit_parity(qs, orc):
    for n, ng, kmax, seed in [(10, 200, 3, 1), (14, 150, 5, 2), (17, 120, 4, 3)]:
        c = W.random_gate_circuit(n, ng, seed=seed, max_k=kmax)
        with qs.State(n) as st:
            for op in c.ops:
                qs.qs_apply_fused_gate(st.h, list(op.qubits), op.mats[0])
            got = qs.qs_copy_state_to_host(st.h)
        ref = orc.simulate(c)
        assert rel_l2(got, ref) < AMP_TOL


def test_invalid_arguments_leave_state(qs):
    rng = np.random.default_rng(2)
    psi = random_state(6, rng)
    with qs.State(6) as st:
        qs.qs_load_state_from_host(st.h, psi)
        for t in ([6], [1, 1], [-1], [0, 1, 2, 3, 4, 5]):
            with pytest.raises(qs.QsError) as e:
                qs.qs_apply_fused_gate(st.h, t, np.eye(1 << len(t)))
            assert e.value.code == qs.QS_ERR_INVALID_ARGUMENT
        bad = np.eye(2, dtype=np.complex128)
        bad[0, 0] = np.nan
        with pytest.raises(qs.QsError):
            qs.qs_apply_fused_gate(st.h, [0], bad)
        with pytest.raises(qs.QsError) as e:
            qs.qs_apply_channel(st.h, [0, 1, 2], [np.eye(8)], 0, 0, 0)
        assert e.value.code == qs.QS_ERR_NOT_SUPPORTED
        got = qs.qs_copy_state_to_host(st.h)
        assert np.array_equal(got, psi)


def test_zero_norm_reported(qs):
    with qs.State(4) as st:
        P1 = np.diag([0.0, 1.0]).astype(np.complex128)
        qs.qs_apply_fused_gate(st.h, [2], P1)  # annihilates |0000>
        assert qs.qs_norm(st.h) == 0.0
        with pytest.raises(qs.QsError) as e:
            qs.qs_sample_measurements(st.h, 0, 0, 4)
        assert e.value.code == qs.QS_ERR_ZERO_NORM


@pytest.mark.parametrize("n", [1, 5, 10, 13, 18])
def test_sampling_parity(qs, orc, n):
    rng = np.random.default_rng(40 + n)
    psi = random_state(n, rng)
    e0 = rng.uniform(0, 0.1, size=n)
    e1 = rng.uniform(0, 0.1, size=n)
    ns = 3000
    with qs.State(n) as st:
        qs.qs_load_state_from_host(st.h, psi)
        got = qs.qs_sample_measurements(st.h, 17, 3, ns, e0, e1)
        got_plain = qs.qs_sample_measurements(st.h, 17, 3, ns)
    ref, margins = orc.sample(psi.astype(np.complex128), 17, 3, 0, ns, e0, e1)
    ref_plain, _ = orc.sample(psi.astype(np.complex128), 17, 3, 0, ns)
    mism = np.nonzero(got != ref)[0]
    assert np.all(margins[mism] < SAMPLE_TIE), (mism[:5], margins[mism[:5]])
    assert len(mism) <= max(2, ns // 500)
    mism = np.nonzero(got_plain != ref_plain)[0]
    assert np.all(margins[mism] < SAMPLE_TIE)


def test_sampling_ghz_rule(qs, orc):
    n = 20
    psi = np.zeros(1 << n, dtype=np.complex64)
    psi[0] = psi[-1] = 1 / math.sqrt(2)
    with qs.State(n) as st:
        qs.qs_load_state_from_host(st.h, psi)
        got = qs.qs_sample_measurements(st.h, 11, 2, 400)
    for s, x in enumerate(got):
        u = orc.draw(11, s, 2, 0, 1)
        assert int(x) == (0 if u < 0.5 else (1 << n) - 1)


def _imperative_run(qs, c, seed, traj, mode, n_samples=0, e0=None, e1=None):
    choices, paths = [], []
    with qs.State(c.n) as st:
        ch = 0
        for op in c.ops:
            if op.kind == W.GATE:
                qs.qs_apply_fused_gate(st.h, list(op.qubits), op.mats[0])
            else:
                pick, path = qs.qs_apply_channel(st.h, list(op.qubits), op.mats, seed, traj, ch,
                                                 mode)
                choices.append(pick)
                paths.append(path)
                ch += 1
        state = qs.qs_copy_state_to_host(st.h)
        samples = qs.qs_sample_measurements(st.h, seed, traj, n_samples, e0, e1) if n_samples else None
    return np.array(choices), np.array(paths), state, samples


@pytest.mark.parametrize("mode", [0, 1], ids=["delayed", "naive"])
def test_channel_parity_imperative(qs, orc, mode):
    c = W.random_noisy_circuit(9, 25, seed=4, p_dep=0.05, gamma=0.08, lam=0.05)
    m = orc.Marshalled(c)
    ties = 0
    for traj in range(6):
        ch, paths, state, samples = _imperative_run(qs, c, 7, traj, mode, n_samples=50)
        ref = orc.run_trajectory(c, traj, mode=mode, seed=7, n_samples=50, return_state=True,
                                 marshalled=m)
        _, tie = compare_choices(ch, ref)
        ties += tie
        if tie:
            continue
        if mode == 0:
            assert np.array_equal(paths, ref["paths"])
        assert rel_l2(state, ref["state"]) < AMP_TOL
        mism = np.nonzero(samples != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
    assert ties <= 1


def _driver(qs, c, n_traj, mode, seed=0, traj_offset=0, n_samples=0, e0=None, e1=None,
            return_state=False, max_fuse=0, circuit_id=0, tile_bits=0):
    with qs.State(c.n) as st:
        return qs.qs_run_trajectories(st.h, c, n_traj, seed=seed, traj_offset=traj_offset,
                                      mode=mode, n_samples=n_samples, p0to1=e0, p1to0=e1,
                                      return_state=return_state, max_fuse=max_fuse,
                                      circuit_id=circuit_id, tile_bits=tile_bits)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["delayed", "naive", "conventional_inplace"])
@pytest.mark.parametrize("max_fuse", [2, 4, 5])
def test_driver_parity_noisy_grid(qs, orc, mode, max_fuse):
    """A 4x3 grid with the benchmark's noise kinds (depolarizing, amplitude
    damping, readout) at strengths that make inner products frequent.  The
    in-place conventional mode follows the conventional rule, so it is held to
    the oracle's conventional choices, with every channel on the inner-product
    path."""
    c = W.grid_circuit(4, 3, 8, p_dep=0.02, gamma=0.03, seed=5)
    e0, e1 = W.readout_arrays(12, 0.02, 0.05)
    m = orc.Marshalled(c)
    oracle_mode = 0 if mode == 0 else 1
    ties = 0
    for t in range(5):
        got = _driver(qs, c, 1, mode, seed=3, traj_offset=t, n_samples=40, e0=e0, e1=e1,
                      return_state=True, max_fuse=max_fuse)
        ref = orc.run_trajectory(c, t, mode=oracle_mode, seed=3, n_samples=40, e0=e0, e1=e1,
                                 return_state=True, marshalled=m)
        _, tie = compare_choices(got["choices"][0], ref)
        ties += tie
        if tie:
            continue
        if mode == 0:
            assert np.array_equal(got["paths"][0], ref["paths"])
            assert got["n_slow"][0] == int(np.sum(ref["paths"]))
        if mode == 2:
            assert np.all(got["paths"][0] == 1)
            assert got["n_slow"][0] == len(got["paths"][0])
        assert rel_l2(got["state"], ref["state"]) < AMP_TOL
        mism = np.nonzero(got["samples"][0] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
    assert ties <= 1


def test_driver_chain12_workload(qs, orc):
    """The 12-qubit chain workload: 100 trajectories x 1000 samples."""
    w = W.chain12_workload()
    c = w.circuit
    got = _driver(qs, c, w.n_traj, 0, seed=w.seed, n_samples=w.n_samples, max_fuse=w.max_fuse)
    m = orc.Marshalled(c)
    sample_mism = 0
    for t in range(w.n_traj):
        ref = orc.run_trajectory(c, t, mode=0, seed=w.seed, n_samples=w.n_samples, marshalled=m)
        _, tie = compare_choices(got["choices"][t], ref)
        assert tie == 0
        assert np.all(got["paths"][t] == 0)  # depolarizing only: never needs inner products
        mism = np.nonzero(got["samples"][t] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
        sample_mism += len(mism)
    assert sample_mism <= 10


def test_driver_delayed_equals_naive_for_depolarizing(qs):
    c = W.chain_circuit(10, 6, p_dep=0.05, seed=2)
    a = _driver(qs, c, 8, 0, seed=1, n_samples=20)
    b = _driver(qs, c, 8, 1, seed=1, n_samples=20)
    assert np.array_equal(a["choices"], b["choices"])
    mism = np.sum(a["samples"] != b["samples"])
    assert mism <= 2


def test_driver_resume_equals_uninterrupted(qs):
    c = W.grid_circuit(3, 3, 6, p_dep=0.05, gamma=0.05, seed=1)
    full = _driver(qs, c, 12, 0, seed=9, n_samples=5)
    a = _driver(qs, c, 5, 0, seed=9, n_samples=5)
    b = _driver(qs, c, 7, 0, seed=9, traj_offset=5, n_samples=5)
    assert np.array_equal(full["choices"], np.concatenate([a["choices"], b["choices"]]))
    assert np.array_equal(full["samples"], np.concatenate([a["samples"], b["samples"]]))


def test_driver_deterministic(qs):
    c = W.grid_circuit(3, 4, 6, p_dep=0.01, gamma=0.05, seed=4)
    a = _driver(qs, c, 6, 0, seed=2, n_samples=30, return_state=True)
    b = _driver(qs, c, 6, 0, seed=2, n_samples=30, return_state=True)
    assert np.array_equal(a["choices"], b["choices"])
    assert np.array_equal(a["samples"], b["samples"])
    assert np.array_equal(a["state"], b["state"])


def test_torch_buffer_and_stream(qs, orc):
    import torch

    n = 14
    c = W.random_gate_circuit(n, 40, seed=12, max_k=3)
    buf = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
    stream = torch.cuda.Stream()
    with qs.State(n, buf.data_ptr(), buf.numel() * 8, stream.cuda_stream) as st:
        for op in c.ops:
            qs.qs_apply_fused_gate(st.h, list(op.qubits), op.mats[0])
        qs.qs_flush(st.h)
        stream.synchronize()
        got = buf.cpu().numpy()
    assert rel_l2(got, orc.simulate(c)) < AMP_TOL


@pytest.mark.parametrize("tile_bits", [1, 10, 12, 13, 14])
@pytest.mark.parametrize("max_fuse", [2, 4])
def test_driver_tile_sweeps_16q(qs, orc, tile_bits, max_fuse):
    """16 qubits: tiles narrower than the state, fused blocks regrouped into
    LDS sweeps, slow paths splitting the sweeps."""
    c = W.grid_circuit(4, 4, 6, p_dep=0.01, gamma=0.02, seed=8)
    e0, e1 = W.readout_arrays(16, 0.01, 0.03)
    m = orc.Marshalled(c)
    ties = 0
    for t in range(2):
        got = _driver(qs, c, 1, 0, seed=4, traj_offset=t, n_samples=30, e0=e0, e1=e1,
                      return_state=True, max_fuse=max_fuse, tile_bits=tile_bits)
        ref = orc.run_trajectory(c, t, mode=0, seed=4, n_samples=30, e0=e0, e1=e1,
                                 return_state=True, marshalled=m)
        _, tie = compare_choices(got["choices"][0], ref)
        ties += tie
        if tie:
            continue
        assert np.array_equal(got["paths"][0], ref["paths"])
        assert rel_l2(got["state"], ref["state"]) < AMP_TOL
        mism = np.nonzero(got["samples"][0] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
    assert ties <= 1


@pytest.mark.parametrize("tile_bits", [0, 14])
def test_driver_noiseless_grid_matches_oracle_20q(qs, orc, tile_bits):
    c = W.grid_circuit(4, 5, 10, seed=3)
    got = _driver(qs, c, 1, 0, n_samples=200, return_state=True, tile_bits=tile_bits)
    ref = orc.run_trajectory(c, 0, n_samples=200, return_state=True)
    assert rel_l2(got["state"], ref["state"]) < AMP_TOL
    mism = np.nonzero(got["samples"][0] != ref["samples"])[0]
    assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)


def test_grid24_full_size_classification(qs, orc):
    """The benchmark workload at full size in the benchmark's launch
    configuration: every channel resolved from the bounds must pick the same
    Kraus operator as the oracle's rule on the same draw, and the channels
    that need inner products must be the same ones."""
    w = W.grid24_workload()
    c = w.circuit
    n_traj = 24
    got = _driver(qs, c, n_traj, 0, seed=w.seed, n_samples=1, e0=w.e0, e1=w.e1)
    m = orc.Marshalled(c)
    chans = [o for o in c.ops if o.kind == W.CHANNEL]
    bounds = {}
    dummy = orc.zero_state(1)
    slow_total = 0
    for t in range(n_traj):
        for j, op in enumerate(chans):
            key = id(op.mats)
            if key not in bounds:
                bounds[key] = orc.kraus_bounds(op.mats)
            pbar, mix = bounds[key]
            r = orc.draw(w.seed, j, t, 0, 0)
            res = orc.select_branch(dummy, [0], op.mats, 0, r, pbar=pbar, mixture=mix)
            if res["path"] == 0:
                assert got["paths"][t][j] == 0 or res["margin_fast"] < 1e-12
                if got["paths"][t][j] == 0:
                    assert got["choices"][t][j] == res["choice"] or res["margin_fast"] < 1e-12
            else:
                slow_total += 1
                assert got["paths"][t][j] == 1 or res["margin_fast"] < 1e-12
    assert slow_total == int(got["n_slow"].sum())
    assert np.all(got["samples"] < (1 << 24))


@pytest.mark.parametrize("mode", [0, 1], ids=["delayed", "naive"])
def test_driver_decay_dephasing_and_two_qubit_noise(qs, orc, mode):
    """Slow-path-heavy channels: the three-operator decay/dephasing channel on
    every qubit after every moment and two-qubit depolarizing after each CZ."""
    ops = []
    rng = np.random.default_rng(6)
    n = 11
    dd = W.decay_dephase(0.05, 1.0, 0.6)
    for layer in range(5):
        for q in range(n):
            ops.append(W.Op(W.GATE, (q,), [W.random_unitary(1, rng)], 2 * layer))
            ops.append(W.Op(W.CHANNEL, (q,), dd, 2 * layer))
        for q in range(layer % 2, n - 1, 2):
            ops.append(W.Op(W.GATE, (q, q + 1), [W.CZ], 2 * layer + 1))
            ops.append(W.Op(W.CHANNEL, (q + 1, q), W.depolarize2(0.05), 2 * layer + 1))
    c = W.Circuit(n, ops)
    m = orc.Marshalled(c)
    ties = 0
    for t in range(3):
        got = _driver(qs, c, 1, mode, seed=12, traj_offset=t, n_samples=25, return_state=True)
        ref = orc.run_trajectory(c, t, mode=mode, seed=12, n_samples=25, return_state=True,
                                 marshalled=m)
        _, tie = compare_choices(got["choices"][0], ref)
        ties += tie
        if tie:
            continue
        assert rel_l2(got["state"], ref["state"]) < AMP_TOL
        mism = np.nonzero(got["samples"][0] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
    assert ties <= 1


def test_phase_damping_slow_paths_scale_with_noise(qs):
    """Section 3.5: with phase damping the channels needing inner products
    grow linearly with the noise strength (sum over channels of 1 - s)."""
    counts = {}
    for lam in (1e-3, 1e-2, 1e-1):
        c = W.grid_circuit(3, 4, 6, seed=2)
        ops = []
        for op in c.ops:
            ops.append(op)
            if op.kind == W.GATE:
                for q in op.qubits:
                    ops.append(W.Op(W.CHANNEL, (q,), W.phase_damp(lam), op.moment))
        nc = W.Circuit(c.n, ops)
        r = _driver(qs, nc, 40, 0, seed=1)
        n_ch = sum(1 for o in ops if o.kind == W.CHANNEL)
        counts[lam] = (float(r["n_slow"].mean()), n_ch * lam)
    for lam, (got, expect) in counts.items():
        assert abs(got - expect) < 5 * np.sqrt(expect / 40) + 0.5, (lam, got, expect)


@pytest.mark.parametrize("shape,cycles,n_traj", [((3, 4), 6, 4), ((4, 5), 4, 1)])
@pytest.mark.parametrize("mode", [0, 1], ids=["delayed", "naive"])
def test_driver_approx_noise_model(qs, orc, mode, shape, cycles, n_traj):
    """Section 5.2's approximate noise model: sqrt(iSWAP) dressed with fSim
    and Z-phase coherent errors and U_ZZ (unitaries the planner fuses with
    the gates), 2-qubit depolarizing on every pair and decay/dephasing on
    every qubit after every moment."""
    c = W.approx_noise_grid_circuit(*shape, cycles, seed=4, zeta=2e6, p_dep2=0.02,
                                    step_time=0.5)
    m = orc.Marshalled(c)
    e0, e1 = W.readout_arrays(c.n, 0.02, 0.05)
    ties = 0
    for t in range(n_traj):
        got = _driver(qs, c, 1, mode, seed=21, traj_offset=t, n_samples=30, e0=e0, e1=e1,
                      return_state=True, max_fuse=4)
        ref = orc.run_trajectory(c, t, mode=mode, seed=21, n_samples=30, e0=e0, e1=e1,
                                 return_state=True, marshalled=m)
        _, tie = compare_choices(got["choices"][0], ref)
        ties += tie
        if tie:
            continue
        if mode == 0:
            assert np.array_equal(got["paths"][0], ref["paths"])
        assert rel_l2(got["state"], ref["state"]) < AMP_TOL
        mism = np.nonzero(got["samples"][0] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
    assert ties <= 1


@pytest.mark.parametrize("n_states,n_traj", [(2, 9), (3, 2), (4, 13)])
def test_driver_concurrent_states_match_one_state(qs, n_states, n_traj):
    """qs_run_trajectories_concurrent splits the range over states running at
    once; every output equals the single-state run of the same range."""
    import torch
    c = W.grid_circuit(4, 3, 8, p_dep=0.02, gamma=0.03, seed=5)
    e0, e1 = W.readout_arrays(12, 0.02, 0.05)
    kw = dict(seed=4, traj_offset=3, n_samples=7, p0to1=e0, p1to0=e1, return_state=True,
              z_expect=True)
    with qs.State(c.n) as one:
        ref = qs.qs_run_trajectories(one.h, c, n_traj, **kw)
    streams = [torch.cuda.Stream() for _ in range(n_states)]
    states = [qs.State(c.n, hip_stream=st.cuda_stream) for st in streams]
    try:
        got = qs.qs_run_trajectories([st.h for st in states], c, n_traj, **kw)
    finally:
        for st in states:
            st.close()
    for key in ("samples", "choices", "paths", "n_slow", "z_expect"):
        assert np.array_equal(got[key], ref[key]), key
    assert np.array_equal(got["state"], ref["state"])
    assert got["gate_sweeps"] == ref["gate_sweeps"]


def test_driver_concurrent_rejects_repeated_state(qs):
    c = W.grid_circuit(3, 4, 2, p_dep=0.01, seed=1)
    with qs.State(c.n) as st:
        with pytest.raises(qs.QsError):
            qs.qs_run_trajectories([st.h, st.h], c, 4, seed=1)


def test_driver_concurrent_kernel_timing(qs):
    """With kernel timing, a concurrent call reports the span during which
    its sweeps ran: positive, within the call's wall time, and no more than
    the single-state call's sweep time on the same range by a wide margin."""
    import torch
    c = W.grid_circuit(4, 4, 10, p_dep=0.01, gamma=0.01, seed=2)
    streams = [torch.cuda.Stream() for _ in range(2)]
    states = [qs.State(c.n, hip_stream=st.cuda_stream) for st in streams]
    try:
        r = qs.qs_run_trajectories([s_.h for s_ in states], c, 12, seed=3, time_kernels=True)
        one = qs.qs_run_trajectories(states[0].h, c, 12, seed=3, time_kernels=True)
    finally:
        for s_ in states:
            s_.close()
    assert r["gate_kernel_launches"] == one["gate_kernel_launches"] > 0
    assert 0.0 < r["gate_kernel_ms"] <= 1e3 * r["host_seconds"]
    assert r["gate_kernel_ms"] < 2.0 * one["gate_kernel_ms"]


def test_grid24_full_size_delayed_equals_conventional(qs):
    """The benchmark workload at full size: the delayed path (tile sweeps,
    device-side selection) and the conventional one (one scratch-state pass per
    Kraus trial) are separate code; away from threshold ties they pick the same
    Kraus operators, draw the same bitstring and end in the same state."""
    w = W.grid24_workload()
    c = w.circuit
    compared = 0
    for t in (0, 1, 2):
        kw = dict(seed=w.seed, traj_offset=t, n_samples=1, e0=w.e0, e1=w.e1, return_state=True,
                  max_fuse=w.max_fuse)
        a = _driver(qs, c, 1, 0, **kw)
        b = _driver(qs, c, 1, 1, **kw)
        if not np.array_equal(a["choices"][0], b["choices"][0]):
            continue  # a threshold tie between the two roundings
        compared += 1
        assert rel_l2(a["state"], b["state"]) < 2 * AMP_TOL
        assert np.array_equal(a["samples"], b["samples"])
    assert compared >= 2


def test_driver_two_qubit_channel_and_fused_reduced_density_matrix(qs, orc):
    """Inner products over both kinds of reduced density matrix: one-qubit
    amplitude damping (its matrix is formed by the last tile sweep before the
    channel when the tile holds the qubit) and a two-qubit channel that is not
    a mixture of unitaries (amplitude damping on both qubits at once, four
    Kraus operators; its 4x4 matrix comes from a read pass).  14 qubits, so
    tiles are narrower than the state; against the oracle."""
    rng = np.random.default_rng(21)
    n = 14
    ad = W.amplitude_damp(0.2)
    ad2 = [np.kron(b, a) for b in ad for a in ad]  # matrix bit 0 <-> first qubit
    ops = []
    for layer in range(10):
        for q in range(0, n - 1, 2):
            a, b = (q, q + 1) if layer % 2 == 0 else ((q + 1) % n, (q + 2) % n)
            ops.append(W.Op(W.GATE, (a, b), [W.random_unitary(2, rng)], layer, "u2"))
        for q in rng.choice(n, size=3, replace=False):
            ops.append(W.Op(W.CHANNEL, (int(q),), ad, layer, "amplitude_damp"))
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        ops.append(W.Op(W.CHANNEL, (a, b), ad2, layer, "amplitude_damp2"))
    c = W.Circuit(n, ops, "ad2")
    m = orc.Marshalled(c)
    slow = 0
    for t in range(3):
        got = _driver(qs, c, 1, 0, seed=5, traj_offset=t, n_samples=20, return_state=True,
                      max_fuse=4)
        ref = orc.run_trajectory(c, t, mode=0, seed=5, n_samples=20, return_state=True,
                                 marshalled=m)
        _, tie = compare_choices(got["choices"][0], ref)
        assert tie == 0
        assert np.array_equal(got["paths"][0], ref["paths"])
        slow += int(got["n_slow"][0])
        assert rel_l2(got["state"], ref["state"]) < AMP_TOL
        mism = np.nonzero(got["samples"][0] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
    assert slow >= 6


def test_autotuner_times_trajectories_when_inner_products_are_frequent(qs, orc):
    """Amplitude damping at gamma = 0.2 on a 16-qubit grid predicts about 19
    inner-product channels per trajectory, so the autotuner times whole
    trajectories (host planning included) instead of one default pass.  The
    tuned call equals a call with the chosen widths fixed, and matches the
    oracle."""
    c = W.grid_circuit(4, 4, 6, p_dep=0.02, gamma=0.2, seed=9)
    e0, e1 = W.readout_arrays(16, 0.01, 0.02)
    kw = dict(seed=4, mode=0, n_samples=20, p0to1=e0, p1to0=e1, traj_offset=7)
    with qs.State(16) as st:
        tuned = qs.qs_run_trajectories(st.h, c, 6, max_fuse=0, tile_bits=0, **kw)
        assert tuned["tune_ms"] > 0.0
        assert tuned["n_slow"].mean() > 5
        f, tb = tuned["max_fuse_used"], tuned["tile_bits_used"]
        fixed = qs.qs_run_trajectories(st.h, c, 6, max_fuse=f, tile_bits=tb, **kw)
    assert np.array_equal(tuned["choices"], fixed["choices"])
    assert np.array_equal(tuned["samples"], fixed["samples"])
    m = orc.Marshalled(c)
    ties = 0
    for t in range(3):
        ref = orc.run_trajectory(c, 7 + t, seed=4, n_samples=20, e0=e0, e1=e1, marshalled=m)
        _, tie = compare_choices(tuned["choices"][t], ref)
        ties += tie
        if tie:
            continue
        mism = np.nonzero(tuned["samples"][t] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
    assert ties <= 1
