"""Pins for whole trajectories and sampling: averages over trajectories must
reproduce exact density-matrix evolution (Section 3.5: a trajectory picks one
Kraus operator per channel with probability p_i), and the sampler must follow
|psi|^2 and the readout confusion model (Section 5.1.2)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import dense


def _traj_average(orc, c, T, mode, seed):
    m = orc.Marshalled(c)
    dim = 1 << c.n
    acc = np.zeros((dim, dim), dtype=np.complex128)
    acc2 = np.zeros((dim, dim), dtype=np.float64)
    for t in range(T):
        psi = orc.run_trajectory(c, t, mode=mode, seed=seed, return_state=True,
                                 marshalled=m)["state"]
        outer = np.outer(psi, psi.conj())
        acc += outer
        acc2 += np.abs(outer) ** 2
    mean = acc / T
    var = np.maximum(acc2 / T - np.abs(mean) ** 2, 1e-30)
    return mean, np.sqrt(var / T)


@pytest.mark.parametrize("mode", [0, 1], ids=["delayed", "naive"])
def test_trajectory_average_matches_density_matrix(orc, mode):
    c = W.random_noisy_circuit(3, 8, seed=12, p_dep=0.15, gamma=0.25, lam=0.2, p_flip=0.1)
    rho = dense.density_evolve(c)
    assert abs(np.trace(rho) - 1) < 1e-12
    mean, se = _traj_average(orc, c, 3000, mode, seed=77)
    z = np.abs(mean - rho) / np.maximum(se, 1e-4)
    assert np.max(z) < 5.0, float(np.max(z))


def test_decay_dephase_trajectories(orc):
    ops = [W.Op(W.GATE, (0,), [W.SQRT_Y], 0), W.Op(W.GATE, (1,), [W.SQRT_X], 0)]
    for i in range(4):
        ops.append(W.Op(W.CHANNEL, (0,), W.decay_dephase(0.2, 1.0, 0.8), i + 1))
        ops.append(W.Op(W.CHANNEL, (1,), W.decay_dephase(0.1, 0.5, 2.0), i + 1))
        ops.append(W.Op(W.GATE, (0, 1), [W.CZ], i + 1))
    c = W.Circuit(2, ops)
    rho = dense.density_evolve(c)
    mean, se = _traj_average(orc, c, 4000, 0, seed=5)
    z = np.abs(mean - rho) / np.maximum(se, 1e-4)
    assert np.max(z) < 5.0


def test_two_qubit_depolarizing_trajectories(orc):
    ops = [W.Op(W.GATE, (0,), [W.SQRT_W], 0), W.Op(W.GATE, (0, 2), [W.CZ], 0),
           W.Op(W.CHANNEL, (2, 0), W.depolarize2(0.3), 1),
           W.Op(W.GATE, (1,), [W.SQRT_X], 1), W.Op(W.CHANNEL, (1, 2), W.depolarize2(0.2), 2)]
    c = W.Circuit(3, ops)
    rho = dense.density_evolve(c)
    mean, se = _traj_average(orc, c, 3000, 0, seed=9)
    assert np.max(np.abs(mean - rho) / np.maximum(se, 1e-4)) < 5.0


def test_sampled_distribution_with_readout(orc):
    """One shot per trajectory with readout flips: chi^2 against diag(rho)
    pushed through the per-qubit confusion matrices."""
    c = W.random_noisy_circuit(3, 6, seed=31, p_dep=0.1, gamma=0.2)
    e0, e1 = np.array([0.05, 0.1, 0.0]), np.array([0.2, 0.0, 0.15])
    rho = dense.density_evolve(c)
    q = dense.readout_distribution(np.real(np.diag(rho)), 3, e0, e1)
    m = orc.Marshalled(c)
    T = 8000
    xs = np.array([orc.run_trajectory(c, t, seed=4, n_samples=1, e0=e0, e1=e1,
                                      marshalled=m)["samples"][0] for t in range(T)],
                  dtype=np.int64)
    counts = np.bincount(xs, minlength=8)
    exp = q * T
    mask = exp > 5
    chi2 = float(np.sum((counts[mask] - exp[mask]) ** 2 / exp[mask]))
    assert chi2 < 35.0, chi2  # <= 7 dof


def test_sampler_follows_amplitudes(orc):
    rng = np.random.default_rng(3)
    n = 5
    psi = (rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)).astype(np.complex128)
    psi *= 3.0  # the sampler normalises by N itself
    p = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    xs, margins = orc.sample(psi, seed=1, traj=0, circ=0, n_samples=40000)
    counts = np.bincount(xs.astype(np.int64), minlength=1 << n)
    chi2 = float(np.sum((counts - p * 40000) ** 2 / (p * 40000)))
    assert chi2 < 80.0  # 31 dof
    assert np.all(margins >= 0)


def test_sampler_inverse_cdf_rule(orc):
    """GHZ: u < 1/2 must give 0...0 and u >= 1/2 must give 1...1."""
    n = 6
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = psi[-1] = 1 / math.sqrt(2)
    xs, _ = orc.sample(psi, seed=11, traj=2, circ=1, n_samples=500)
    for s, x in enumerate(xs):
        u = orc.draw(11, s, 2, 1, 1)
        assert int(x) == (0 if u < 0.5 else (1 << n) - 1)


def test_sampler_basis_state_and_readout(orc):
    n = 4
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0b0101] = 1.0
    xs, _ = orc.sample(psi, seed=0, traj=0, circ=0, n_samples=100)
    assert np.all(xs == 0b0101)
    e0, e1 = np.full(n, 0.25), np.full(n, 0.4)
    T = 20000
    xs, _ = orc.sample(psi, seed=0, traj=0, circ=0, n_samples=T, e0=e0, e1=e1)
    xs = xs.astype(np.int64)
    for q in range(n):
        true_b = (0b0101 >> q) & 1
        flip = np.mean(((xs >> q) & 1) != true_b)
        e = e1[q] if true_b else e0[q]
        assert abs(flip - e) < 5 * math.sqrt(e * (1 - e) / T)


def test_trajectories_are_seed_deterministic(orc):
    c = W.random_noisy_circuit(4, 10, seed=2, p_dep=0.1, gamma=0.1)
    a = orc.run_trajectory(c, 5, seed=9, n_samples=3, return_state=True)
    b = orc.run_trajectory(c, 5, seed=9, n_samples=3, return_state=True)
    assert np.array_equal(a["choices"], b["choices"])
    assert np.array_equal(a["samples"], b["samples"])
    assert np.array_equal(a["state"], b["state"])
    d = orc.run_trajectory(c, 6, seed=9, n_samples=3)
    e = orc.run_trajectory(c, 5, seed=10, n_samples=3)
    assert not (np.array_equal(a["choices"], d["choices"]) and
                np.array_equal(a["choices"], e["choices"]) and
                np.array_equal(a["samples"], d["samples"]))
