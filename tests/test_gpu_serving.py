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
