"""Edge cases of the trajectory driver through the C ABI: empty circuits and
ranges, one-qubit states, channel-only circuits, the smallest tiled states,
and sizes that leave a ragged number of tiles per workgroup."""

import math

import torch  # noqa: F401  (imported at collection: the first import can be slow)

import numpy as np
import pytest

import workloads as W
from gpu_helpers import AMP_TOL, SAMPLE_TIE, compare_choices, rel_l2

pytestmark = pytest.mark.gpu


def _run(qs, c, n_traj, **kw):
    with qs.State(c.n) as st:
        return qs.qs_run_trajectories(st.h, c, n_traj, **kw)


def test_empty_circuit_samples_zero(qs):
    """No operations: every trajectory stays |0...0>; every sample reads 0."""
    c = W.Circuit(5, [])
    r = _run(qs, c, 4, n_samples=16, return_state=True, z_expect=True)
    assert np.all(r["samples"] == 0)
    assert r["state"][0] == 1 and np.all(r["state"][1:] == 0)
    assert np.array_equal(r["z_expect"], np.ones((4, 5)))


def test_zero_trajectories(qs):
    c = W.grid_circuit(3, 4, 2, p_dep=0.05, seed=1)
    r = _run(qs, c, 0, n_samples=3, z_expect=True)
    assert r["samples"].shape == (0, 3) and r["sweeps"] == 0


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["delayed", "naive", "conventional_inplace"])
def test_one_qubit_state(qs, orc, mode):
    """n = 1 (no tile sweeps): amplitude damping after a rotation."""
    th = 1.1
    ry = np.array([[math.cos(th / 2), -math.sin(th / 2)], [math.sin(th / 2), math.cos(th / 2)]])
    ops = [W.Op(W.GATE, (0,), [ry], 0), W.Op(W.CHANNEL, (0,), W.amplitude_damp(0.4), 0)]
    c = W.Circuit(1, ops)
    m = orc.Marshalled(c)
    oracle_mode = 0 if mode == 0 else 1
    for t in range(6):
        got = _run(qs, c, 1, seed=5, traj_offset=t, mode=mode, n_samples=8, return_state=True)
        ref = orc.run_trajectory(c, t, mode=oracle_mode, seed=5, n_samples=8, return_state=True,
                                 marshalled=m)
        _, tie = compare_choices(got["choices"][0], ref)
        if tie:
            continue
        assert rel_l2(got["state"], ref["state"]) < AMP_TOL
        mism = np.nonzero(got["samples"][0] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)


def test_channel_only_circuit(qs, orc):
    """Channels with no gates between them (every block is a channel pick)."""
    ops = []
    for q in range(10):
        ops.append(W.Op(W.CHANNEL, (q,), W.bit_flip(0.3), 0))
        ops.append(W.Op(W.CHANNEL, (q,), W.amplitude_damp(0.2), 0))
    c = W.Circuit(10, ops)
    m = orc.Marshalled(c)
    for t in range(4):
        got = _run(qs, c, 1, seed=2, traj_offset=t, n_samples=20, return_state=True)
        ref = orc.run_trajectory(c, t, mode=0, seed=2, n_samples=20, return_state=True,
                                 marshalled=m)
        _, tie = compare_choices(got["choices"][0], ref)
        if tie:
            continue
        assert rel_l2(got["state"], ref["state"]) < AMP_TOL
        mism = np.nonzero(got["samples"][0] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)


@pytest.mark.parametrize("n", [10, 14, 17, 19])
def test_tile_edges(qs, orc, n):
    """The smallest tiled state (one tile), a state with fewer tiles than
    workgroups, and sizes whose tiles do not split evenly over the grid."""
    c = W.generic_grid_circuit(n, 4, p_dep=0.02, gamma=0.02, seed=n)
    m = orc.Marshalled(c)
    ties = 0
    for t in range(2):
        got = _run(qs, c, 1, seed=9, traj_offset=t, n_samples=10, return_state=True)
        ref = orc.run_trajectory(c, t, mode=0, seed=9, n_samples=10, return_state=True,
                                 marshalled=m)
        _, tie = compare_choices(got["choices"][0], ref)
        ties += tie
        if tie:
            continue
        assert rel_l2(got["state"], ref["state"]) < AMP_TOL
    assert ties <= 1


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["delayed", "naive", "conventional_inplace"])
def test_state_after_run_is_last_trajectory(qs, mode):
    """After qs_run_trajectories the state holds the last trajectory's final
    vector (the one QS_TRAJ_RETURN_STATE copies out), whichever buffer the
    conventional method ended in."""
    c = W.grid_circuit(3, 4, 6, p_dep=0.05, gamma=0.1, seed=3)
    with qs.State(c.n) as st:
        r = qs.qs_run_trajectories(st.h, c, 5, seed=4, mode=mode, return_state=True)
        after = qs.qs_copy_state_to_host(st.h)
        assert np.array_equal(after, r["state"])
        # and with no trajectories the state is left as it was
        r0 = qs.qs_run_trajectories(st.h, c, 0, seed=4, mode=mode)
        assert np.array_equal(qs.qs_copy_state_to_host(st.h), after)


@pytest.mark.parametrize("n", [1, 9, 20])
def test_copy_state_between_streams(qs, n):
    """qs_copy_state copies every amplitude bit for bit, from a state on one
    stream to a state on another, after the source's pending gate, and drops
    the destination's pending work; mismatched sizes are refused."""
    rng = np.random.default_rng(n)
    amps = (rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)).astype(np.complex64)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with qs.State(n, hip_stream=s1.cuda_stream) as a, qs.State(n, hip_stream=s2.cuda_stream) as b:
        qs.qs_load_state_from_host(a.h, amps)
        h = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2)
        qs.qs_apply_fused_gate(a.h, [0], h)
        qs.qs_apply_fused_gate(b.h, [0], h)
        qs.qs_copy_state(b.h, a.h)
        got = qs.qs_copy_state_to_host(b.h)
        want = qs.qs_copy_state_to_host(a.h)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
        qs.qs_copy_state(a.h, a.h)
        assert np.array_equal(qs.qs_copy_state_to_host(a.h).view(np.uint64), want.view(np.uint64))
    with qs.State(n) as a, qs.State(n + 1) as b:
        with pytest.raises(qs.QsError) as e:
            qs.qs_copy_state(b.h, a.h)
        assert e.value.code == qs.QS_ERR_INVALID_ARGUMENT
