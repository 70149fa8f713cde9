"""The serving loop: every request completes under a tight memory budget,
and each request's results are the same alone and in the mix."""

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can be slow)

import workloads as W

pytestmark = pytest.mark.gpu


def _requests():
    return W.serving_requests(14, rate_hz=200.0, seed=3, n_lo=10, n_hi=21, d_lo=4, d_hi=10,
                              t_lo=1, t_hi=12)


def test_serving_alone_equals_mix(qs):
    from paper_2111_02396_amd import serving

    reqs = _requests()
    # budget for about two of the largest requests at once: forces queueing
    budget = 2 * serving.footprint_bytes(21) + serving.footprint_bytes(18)
    srv = serving.Server(budget_bytes=budget, slot_workers=3)
    stats = srv.run(reqs)
    assert all(srv.results[r.rid].error is None for r in reqs)
    assert stats.trajectories == sum(r.workload.n_traj for r in reqs)
    lanes = {srv.results[r.rid].lane for r in reqs}
    assert lanes == {"batch", "slot"}
    assert srv.used == 0
    for r in reqs:
        mix = srv.results[r.rid]
        alone = serving.run_alone(r)
        assert alone.lane == mix.lane
        assert np.array_equal(alone.samples, mix.samples), r.rid
        assert np.array_equal(alone.choices, mix.choices), r.rid
        assert mix.done_s >= mix.arrival_s


def test_serving_rejects_oversized(qs):
    from paper_2111_02396_amd import serving

    reqs = W.serving_requests(3, rate_hz=100.0, seed=5, n_lo=12, n_hi=12, t_hi=2)
    srv = serving.Server(budget_bytes=serving.footprint_bytes(11), slot_workers=1)
    srv.run(reqs)
    assert all(srv.results[r.rid].error for r in reqs)
    assert srv.used == 0


def test_serving_top_of_the_range_32_qubits(qs):
    """The serving range reaches 32 qubits (Section 4.1: a state takes 8 2^n
    bytes, up to twice that with non-unitary noise).  With room for the
    32-qubit request, one 30-qubit request and the small ones, the second
    30-qubit request is admitted only after a large one has released its
    16 2^n bytes; nothing admitted ever exceeds the budget; the large
    requests' results are the same alone and in the mix (the 32-qubit one
    runs the 64-bit index kernels)."""
    from paper_2111_02396_amd import serving
    from workloads.configs import Request, TrajectoryWorkload

    def req(rid, n, depth, p, n_traj, arrival):
        c = W.generic_grid_circuit(n, depth, p_dep=p, seed=40 + rid)
        return Request(rid, arrival, TrajectoryWorkload(f"r{rid}-n{n}", c, n_traj=n_traj, seed=9,
                                                        circuit_id=rid, n_samples=2, max_fuse=4))

    reqs = [req(0, 32, 4, 1e-3, 1, 0.0), req(1, 30, 6, 1e-3, 2, 0.0), req(2, 30, 4, 1e-3, 1, 0.001),
            req(3, 12, 8, 1e-2, 8, 0.0), req(4, 16, 6, 1e-2, 4, 0.002), req(5, 20, 6, 1e-3, 3, 0.003)]
    fp = serving.footprint_bytes
    budget = fp(32) + fp(30) + fp(20) + fp(16) + fp(12)
    srv = serving.Server(budget_bytes=budget, slot_workers=4)
    stats = srv.run(reqs)
    assert all(srv.results[r.rid].error is None for r in reqs)
    assert stats.trajectories == sum(r.workload.n_traj for r in reqs)
    assert srv.used == 0 and 0 < srv.peak_used <= budget
    assert {srv.results[r.rid].lane for r in reqs} == {"batch", "slot"}
    first_large_done = min(srv.results[0].done_s, srv.results[1].done_s)
    assert srv.results[2].admitted_s >= first_large_done - 1e-3
    for r in reqs[:3]:
        mix = srv.results[r.rid]
        alone = serving.run_alone(r)
        assert np.array_equal(alone.samples, mix.samples), r.rid
        assert np.array_equal(alone.choices, mix.choices), r.rid
