"""GPU parity of observable estimation (<Z_q> of every qubit in one read
pass, <O> on one or two qubits from the reduced density matrix, and the
trajectory driver's per-trajectory <Z_q>) against the CPU oracle.

Bars: on the same complex64 amplitudes both sides sum in FP64, so the
estimates agree to 1e-12 (absolute, times the observable's largest entry).
For driver trajectories the states themselves differ by at most AMP_TOL in
relative L2; for unit vectors |<a|Z|a> - <b|Z|b>| <= 2 |a - b|, so the bar
there is 2 AMP_TOL plus rounding.
"""

import math

import torch  # noqa: F401  (imported at collection: the first import can be slow)

import numpy as np
import pytest

import workloads as W
from gpu_helpers import AMP_TOL, compare_choices, random_state, rel_l2

pytestmark = pytest.mark.gpu

Z_DRIVER_TOL = 2 * AMP_TOL + 1e-6


def _ry(theta):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


@pytest.mark.parametrize("n", [1, 3, 7, 8, 9, 12, 18, 19, 20, 23])
def test_expectation_z_parity(qs, orc, n):
    """Sizes on both sides of every chunking regime: fewer than 256
    amplitudes, one chunk per workgroup, and up to 2048 workgroups with
    iteration bits."""
    rng = np.random.default_rng(70 + n)
    psi = (random_state(n, rng) * np.float32(0.6)).astype(np.complex64)
    with qs.State(n) as st:
        qs.qs_load_state_from_host(st.h, psi)
        got = qs.qs_expectation_z(st.h)
        again = qs.qs_expectation_z(st.h)
    assert np.array_equal(got, again)  # fixed reduction order
    ref = orc.z_expectations(psi.astype(np.complex128))
    assert np.max(np.abs(got - ref)) < 1e-12, (n, np.max(np.abs(got - ref)))


@pytest.mark.parametrize("n", [4, 10, 21])
def test_expectation_z_basis_states(qs, n):
    rng = np.random.default_rng(n)
    for x in [0, (1 << n) - 1] + [int(v) for v in rng.integers(0, 1 << n, size=4)]:
        psi = np.zeros(1 << n, dtype=np.complex64)
        psi[x] = -1j
        with qs.State(n) as st:
            qs.qs_load_state_from_host(st.h, psi)
            z = qs.qs_expectation_z(st.h)
        want = np.array([1.0 - 2.0 * ((x >> q) & 1) for q in range(n)])
        assert np.array_equal(z, want), x


def test_expectation_z_product_state_28q(qs):
    """A 28-qubit product state prepared on the device by one rotation per
    qubit: <Z_q> = cos theta_q at any size (bound: complex64 rounding)."""
    n = 28
    th = np.linspace(0.1, 3.0, n)
    with qs.State(n) as st:
        for q in range(n):
            qs.qs_apply_fused_gate(st.h, [q], _ry(th[q]))
        z = qs.qs_expectation_z(st.h)
    assert np.max(np.abs(z - np.cos(th))) < 1e-5


def _hermitian(k, rng):
    A = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    return A + A.conj().T


@pytest.mark.parametrize("n", [2, 11, 17, 22])
def test_expectation_parity(qs, orc, n):
    rng = np.random.default_rng(90 + n)
    psi = (random_state(n, rng) * np.float32(2.5)).astype(np.complex64)
    pats = [[0], [n - 1], [1, 0], [0, n - 1], [n - 1, n // 2 if n // 2 != n - 1 else 0]]
    with qs.State(n) as st:
        qs.qs_load_state_from_host(st.h, psi)
        for t in pats:
            if len(set(t)) != len(t) or max(t) >= n:
                continue
            O = _hermitian(len(t), rng)
            got = qs.qs_expectation(st.h, t, O)
            ref = orc.observable_expectation(psi.astype(np.complex128), t, O)
            assert abs(got - ref) < 1e-12 * np.max(np.abs(O)), (n, t, got, ref)


def test_expectation_rejects_bad_observables(qs):
    with qs.State(6) as st:
        with pytest.raises(qs.QsError):
            qs.qs_expectation(st.h, [0], np.array([[0, 1], [0, 0]], dtype=np.complex128))
        with pytest.raises(qs.QsError):
            qs.qs_expectation(st.h, [2, 2], np.eye(4))
        with pytest.raises(qs.QsError):
            qs.qs_expectation(st.h, [6], np.eye(2))
        with pytest.raises(qs.QsError):
            qs.qs_expectation(st.h, [0, 1, 2], np.eye(8))
        # the state is untouched and still answers
        assert np.array_equal(qs.qs_expectation_z(st.h), np.ones(6))


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["delayed", "naive", "conventional_inplace"])
def test_driver_z_expectations(qs, orc, mode):
    """Per-trajectory <Z_q> recorded by the driver on the noisy 4x3 grid,
    against the oracle's definition on the oracle's own trajectory state."""
    c = W.grid_circuit(4, 3, 8, p_dep=0.02, gamma=0.03, seed=5)
    m = orc.Marshalled(c)
    oracle_mode = 0 if mode == 0 else 1
    n_traj = 6
    with qs.State(c.n) as st:
        got = qs.qs_run_trajectories(st.h, c, n_traj, seed=8, mode=mode, z_expect=True,
                                     n_samples=3)
    assert got["z_expect"].shape == (n_traj, c.n)
    ties = 0
    for t in range(n_traj):
        ref = orc.run_trajectory(c, t, mode=oracle_mode, seed=8, n_samples=3,
                                 return_state=True, marshalled=m)
        _, tie = compare_choices(got["choices"][t], ref)
        ties += tie
        if tie:
            continue
        zr = orc.z_expectations(ref["state"])
        assert np.max(np.abs(got["z_expect"][t] - zr)) < Z_DRIVER_TOL, (t, got["z_expect"][t], zr)
    assert ties <= 1


def test_driver_z_expectations_grid24_last_state(qs, orc):
    """Full-size workload in the benchmark's configuration: the last
    trajectory's recorded <Z_q> equals the definition on the state the
    driver returns, and every value lies in [-1, 1]."""
    w = W.grid24_workload()
    with qs.State(w.circuit.n) as st:
        got = qs.qs_run_trajectories(st.h, w.circuit, 4, seed=w.seed, z_expect=True,
                                     n_samples=w.n_samples, p0to1=w.e0, p1to0=w.e1,
                                     return_state=True, max_fuse=w.max_fuse)
    z = got["z_expect"]
    assert np.all(np.abs(z) <= 1.0 + 1e-12)
    ref = orc.z_expectations(got["state"].astype(np.complex128))
    assert np.max(np.abs(z[-1] - ref)) < 1e-12
