"""HIP-graph replay of the default plan (QS_TRAJ_GRAPH; small states,
delayed mode): the replayed trajectories match the oracle and are bit-identical to the same
trajectories launched directly, over many replays with direct trajectories
(those that need inner products) and synchronisations in between."""

import torch

import numpy as np
import pytest

import workloads as W
from gpu_helpers import AMP_TOL, SAMPLE_TIE, compare_choices, rel_l2

pytestmark = pytest.mark.gpu


def _run(qs, c, n_traj, graph, **kw):
    stream = torch.cuda.Stream()
    with qs.State(c.n, hip_stream=stream.cuda_stream) as st:
        return qs.qs_run_trajectories(st.h, c, n_traj, graph=graph, **kw)


@pytest.mark.parametrize("shape,max_fuse,tile_bits", [((4, 4), 4, 13), ((3, 4), 4, 0),
                                                      ((4, 5), 4, 12)])
def test_graph_replays_equal_direct_launches(qs, shape, max_fuse, tile_bits):
    # depolarizing (picked from the bounds: graph replays) and amplitude
    # damping (sometimes needs inner products: those trajectories run directly)
    c = W.grid_circuit(*shape, 8, p_dep=0.02, gamma=0.001, seed=7)
    e0, e1 = W.readout_arrays(c.n, 0.01, 0.03)
    kw = dict(seed=3, n_samples=16, p0to1=e0, p1to0=e1, return_state=True, z_expect=True,
              max_fuse=max_fuse, tile_bits=tile_bits)
    g = _run(qs, c, 24, True, **kw)
    d = _run(qs, c, 24, False, **kw)
    # a trajectory with no inner-product channel replays unless its norm bound
    # would need renormalising on the way
    direct_ok = 24 - int(np.count_nonzero(g["n_slow"]))
    assert 0.8 * direct_ok <= g["graph_replays"] <= direct_ok, (g["graph_replays"], direct_ok)
    assert g["graph_replays"] >= 8 and direct_ok < 24
    assert d["graph_replays"] == 0
    for key in ("samples", "choices", "paths", "n_slow", "z_expect"):
        assert np.array_equal(g[key], d[key]), key
    assert np.array_equal(g["state"], d["state"])
    assert g["gate_sweeps"] == d["gate_sweeps"]


def test_graph_replays_against_oracle(qs, orc):
    c = W.grid_circuit(4, 4, 6, p_dep=0.01, seed=11)
    m = orc.Marshalled(c)
    stream = torch.cuda.Stream()
    with qs.State(c.n, hip_stream=stream.cuda_stream) as st:
        got = qs.qs_run_trajectories(st.h, c, 6, seed=5, n_samples=40, max_fuse=4, z_expect=True,
                                     graph=True)
        # every trajectory ran as a replay; the state holds the last one
        assert got["graph_replays"] == 6
        last = qs.qs_copy_state_to_host(st.h)
    for t in range(6):
        ref = orc.run_trajectory(c, t, seed=5, n_samples=40, return_state=(t == 5), marshalled=m)
        _, tie = compare_choices(got["choices"][t], ref)
        assert tie == 0
        mism = np.nonzero(got["samples"][t] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE)
        if t == 5:
            assert rel_l2(last, ref["state"]) < AMP_TOL
            assert np.allclose(got["z_expect"][t], orc.z_expectations(ref["state"]), atol=1e-5)


def test_graph_call_repeated_with_eager_work_between(qs):
    """Several calls on one state, each capturing its own graph, with direct
    gate applications, norms and copies in between."""
    c = W.grid_circuit(3, 4, 6, p_dep=0.02, seed=2)
    stream = torch.cuda.Stream()
    with qs.State(c.n, hip_stream=stream.cuda_stream) as st:
        first = qs.qs_run_trajectories(st.h, c, 8, seed=1, n_samples=8, graph=True)
        for _ in range(3):
            qs.qs_apply_fused_gate(st.h, [0, 5], W.random_unitary(2, np.random.default_rng(0)))
            qs.qs_norm(st.h)
            again = qs.qs_run_trajectories(st.h, c, 8, seed=1, n_samples=8, graph=True)
            assert again["graph_replays"] == 8
            assert np.array_equal(again["samples"], first["samples"])
            assert np.array_equal(again["choices"], first["choices"])


def test_graph_with_concurrent_states(qs):
    """Four states on their own streams and host threads, each capturing and
    replaying its own graph while the others copy matrices and samples: the
    outputs equal the one-state run of the same range."""
    c = W.grid_circuit(4, 4, 8, p_dep=0.01, gamma=0.0005, seed=17)
    kw = dict(seed=8, n_samples=4, max_fuse=4, tile_bits=12, z_expect=True)
    ref = _run(qs, c, 48, False, **kw)
    streams = [torch.cuda.Stream() for _ in range(4)]
    for _ in range(2):
        states = [qs.State(c.n, hip_stream=s.cuda_stream) for s in streams]
        try:
            got = qs.qs_run_trajectories([st.h for st in states], c, 48, graph=True, **kw)
        finally:
            for st in states:
                st.close()
        assert got["graph_replays"] > 24
        for key in ("samples", "choices", "paths", "n_slow", "z_expect"):
            assert np.array_equal(got[key], ref[key]), key
