"""Pins for the oracle's channels, Kraus bounds and branch selection
(Section 3.5, Algorithm 2, and the conventional method it replaces)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import dense

CHANNELS = {
    "depolarize": W.depolarize(0.07),
    "amplitude_damp": W.amplitude_damp(0.2),
    "phase_damp": W.phase_damp(0.3),
    "bit_flip": W.bit_flip(0.1),
    "decay_dephase": W.decay_dephase(0.05, 1.0, 0.7),
}


@pytest.mark.parametrize("name", sorted(CHANNELS))
def test_completeness(name):
    ks = CHANNELS[name]
    S = sum(K.conj().T @ K for K in ks)
    assert np.max(np.abs(S - np.eye(2))) < 1e-15


def test_completeness_two_qubit_depolarizing():
    ks = W.depolarize2(0.05)
    assert len(ks) == 16
    S = sum(K.conj().T @ K for K in ks)
    assert np.max(np.abs(S - np.eye(4))) < 1e-14


def test_printed_third_decay_operator_is_incomplete():
    # the third operator as printed in Section 5.2.1 carries a 1 in its
    # upper-left entry; with it the sum of K^dag K is diag(2, 1)
    t, t1, tphi = 0.05, 1.0, 0.7
    ks = W.decay_dephase(t, t1, tphi)
    printed = ks[2].copy()
    printed[0, 0] = 1.0
    S = ks[0].conj().T @ ks[0] + ks[1].conj().T @ ks[1] + printed.conj().T @ printed
    assert abs(S[0, 0] - 2.0) < 1e-15 and abs(S[1, 1] - 1.0) < 1e-15


def test_decay_dephase_matches_channel_form():
    # the Kraus form reproduces the density-matrix form of Section 5.2.1
    t, t1, tphi = 0.05, 1.0, 0.7
    inv_t2 = 1 / (2 * t1) + 1 / tphi
    rho = np.array([[0.3, 0.2 - 0.1j], [0.2 + 0.1j, 0.7]])
    out = sum(K @ rho @ K.conj().T for K in W.decay_dephase(t, t1, tphi))
    e1, e2 = math.exp(-t / t1), math.exp(-t * inv_t2)
    ref = np.array([[1 - rho[1, 1] * e1, rho[0, 1] * e2], [rho[1, 0] * e2, rho[1, 1] * e1]])
    assert np.max(np.abs(out - ref)) < 1e-15


def test_bounds_closed_forms(orc):
    p, g, lam = 1e-3, 2e-3, 0.3
    pb, mix = orc.kraus_bounds(W.depolarize(p))
    assert mix and np.allclose(pb, [1 - p, p / 3, p / 3, p / 3], rtol=0, atol=4e-16)
    assert abs(pb.sum() - 1.0) < 1e-15
    pb, mix = orc.kraus_bounds(W.amplitude_damp(g))
    assert not mix and np.allclose(pb, [1 - g, 0.0], rtol=0, atol=4e-16)
    pb, mix = orc.kraus_bounds(W.phase_damp(lam))
    assert not mix and np.allclose(pb, [1 - lam, 0.0], rtol=0, atol=4e-16)
    pb, mix = orc.kraus_bounds(W.bit_flip(0.1))
    assert mix and np.allclose(pb, [0.9, 0.1], rtol=0, atol=4e-16)
    pb, mix = orc.kraus_bounds(W.depolarize2(0.05))
    assert mix and abs(pb.sum() - 1.0) < 1e-14


def _exact_probs(psi, n, targets, kraus):
    N = np.vdot(psi, psi).real
    return np.array([np.linalg.norm(dense.full_operator(n, targets, K) @ psi) ** 2 / N
                     for K in kraus])


PARTITION_CASES = [
    ("amplitude_damp", W.amplitude_damp(0.35), [1]),
    ("phase_damp", W.phase_damp(0.4), [2]),
    ("decay_dephase", W.decay_dephase(0.3, 1.0, 0.5), [0]),
    ("depolarize", W.depolarize(0.2), [1]),
    ("depolarize2", W.depolarize2(0.3), [2, 0]),
    ("random_kraus_pair", None, [0, 1]),
]


def _random_kraus_pair(rng):
    # a 2-qubit channel with two full-rank non-unitary Kraus operators
    A = W.random_matrix(2, rng)
    B = W.random_matrix(2, rng)
    S = A.conj().T @ A + B.conj().T @ B
    w, V = np.linalg.eigh(S)
    Sinv_half = V @ np.diag(w ** -0.5) @ V.conj().T
    return [A @ Sinv_half, B @ Sinv_half]


@pytest.mark.parametrize("mode", [0, 1], ids=["delayed", "naive"])
@pytest.mark.parametrize("case", PARTITION_CASES, ids=[c[0] for c in PARTITION_CASES])
def test_partition_of_unit_interval(orc, case, mode):
    """Sweep r over the midpoints of a 10^6 grid: the fraction of r that picks
    K_i must be p_i = <psi|K_i^dag K_i|psi>/<psi|psi> in both schemes."""
    name, kraus, targets = case
    rng = np.random.default_rng(17)
    if kraus is None:
        kraus = _random_kraus_pair(rng)
    n = 3
    psi = (rng.standard_normal(8) + 1j * rng.standard_normal(8)) * 1.7  # not normalised
    psi = psi.astype(np.complex128)
    m = 10 ** 6
    rs = (np.arange(m) + 0.5) / m
    picks = orc.select_many(psi, targets, kraus, mode, rs)
    frac = np.bincount(picks.astype(np.int64), minlength=len(kraus)) / m
    p = _exact_probs(psi, n, targets, kraus)
    assert abs(p.sum() - 1.0) < 1e-12
    assert np.max(np.abs(frac - p)) <= 1.5e-6, (frac, p)


def test_delayed_fast_path_skips_inner_products(orc):
    # r below the first bound: picked from the bounds alone
    psi = orc.zero_state(2)
    res = orc.select_branch(psi, [0], W.amplitude_damp(0.1), 0, 0.5)
    assert res["choice"] == 0 and res["path"] == 0
    res = orc.select_branch(psi, [0], W.amplitude_damp(0.1), 0, 0.95)
    assert res["path"] == 1
    # on |0>, K1 of amplitude damping has zero weight: the residual goes to K0
    assert res["choice"] == 0


def test_delayed_equals_naive_for_mixtures(orc):
    """If every K_i is proportional to a unitary the two schemes partition
    [0,1) identically, so the same draws give the same branches."""
    c = W.random_noisy_circuit(5, 30, seed=8, p_dep=0.2, gamma=0.0, p_flip=0.15)
    for t in range(20):
        a = orc.run_trajectory(c, t, mode=0, seed=3)
        b = orc.run_trajectory(c, t, mode=1, seed=3)
        assert np.array_equal(a["choices"], b["choices"])
        assert np.all(a["paths"] == 0)


def test_amplitude_damping_survival(orc):
    """|1> survives m amplitude-damping channels with probability (1-g)^m."""
    g, m, T = 0.05, 8, 4000
    ops = [W.Op(W.GATE, (0,), [W.PAULI_X], 0, "x")]
    ops += [W.Op(W.CHANNEL, (0,), W.amplitude_damp(g), i + 1, "ad") for i in range(m)]
    c = W.Circuit(1, ops)
    survive = 0
    for t in range(T):
        r = orc.run_trajectory(c, t, seed=21, return_state=True)
        survive += abs(r["state"][1]) > 0.5
    p = (1 - g) ** m
    sd = math.sqrt(p * (1 - p) / T)
    assert abs(survive / T - p) < 5 * sd


def test_depolarizing_flip_probability(orc):
    """Depolarizing p on |0>: X and Y flip the bit, so P(1) = 2p/3."""
    p, T = 0.3, 6000
    c = W.Circuit(1, [W.Op(W.CHANNEL, (0,), W.depolarize(p), 0, "dep")])
    res = [orc.run_trajectory(c, t, seed=5, n_samples=1)["samples"][0] for t in range(T)]
    f = np.mean(res)
    q = 2 * p / 3
    assert abs(f - q) < 5 * math.sqrt(q * (1 - q) / T)


def test_zero_norm_raises(orc):
    # K1 of amplitude damping annihilates |0>
    psi = orc.zero_state(1)
    with pytest.raises(ZeroDivisionError):
        orc.apply_kraus_normalised(psi, [0], W.amplitude_damp(0.3)[1])
