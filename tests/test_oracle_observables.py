"""Pins for the oracle's observable estimates (per-trajectory <Z_q> and
<O> on one or two qubits, Section 3.5's estimator on the normalised state).

Each check rests on a closed form: product states of single-qubit
rotations (<Z> = cos theta, <X> = sin theta), basis states (+-1), GHZ and
Bell states (vanishing single-qubit <Z>, fixed two-qubit correlators), the
scale invariance of a normalised estimate, and an unnormalised state's
explicit probability sums on a tiny case written by hand.
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import dense

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.diag([1.0, -1.0]).astype(np.complex128)


def ry(theta):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def product_state(thetas):
    psi = np.array([1.0 + 0j])
    for th in thetas:  # qubit q is index bit q: later qubits are the outer factor
        psi = np.kron(ry(th) @ np.array([1.0, 0.0]), psi)
    return psi.astype(np.complex128)


def test_z_of_rotated_product_state(orc):
    rng = np.random.default_rng(3)
    th = rng.uniform(0, math.pi, size=7)
    z = orc.z_expectations(product_state(th))
    assert np.max(np.abs(z - np.cos(th))) < 1e-13


def test_x_and_y_of_rotated_product_state(orc):
    th = [0.3, 1.1, 2.0, 2.9]
    psi = product_state(th)
    for q, t in enumerate(th):
        assert abs(orc.observable_expectation(psi, [q], X) - math.sin(t)) < 1e-13
        assert abs(orc.observable_expectation(psi, [q], Y)) < 1e-13
        assert abs(orc.observable_expectation(psi, [q], Z) - math.cos(t)) < 1e-13


@pytest.mark.parametrize("n", [1, 3, 6])
def test_z_of_basis_states(orc, n):
    for x in range(1 << n):
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[x] = 1j  # a phase changes nothing
        want = np.array([1.0 - 2.0 * ((x >> q) & 1) for q in range(n)])
        assert np.array_equal(orc.z_expectations(psi), want)


def test_ghz_and_bell_correlators(orc):
    n = 5
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = psi[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(orc.z_expectations(psi))) < 1e-15
    for a, b in [(0, 1), (1, 4), (3, 2)]:
        assert abs(orc.observable_expectation(psi, [a, b], np.kron(Z, Z)) - 1.0) < 1e-14
    bell = np.zeros(4, dtype=np.complex128)
    bell[0] = bell[3] = 1 / math.sqrt(2)
    assert abs(orc.observable_expectation(bell, [0, 1], np.kron(X, X)) - 1.0) < 1e-14
    assert abs(orc.observable_expectation(bell, [0, 1], np.kron(Y, Y)) + 1.0) < 1e-14
    # singlet: every correlator is -1
    singlet = np.array([0, 1, -1, 0], dtype=np.complex128) / math.sqrt(2)
    for P in (X, Y, Z):
        assert abs(orc.observable_expectation(singlet, [0, 1], np.kron(P, P)) + 1.0) < 1e-14


def test_two_qubit_target_order(orc):
    # O = Z on matrix bit 0 only (I (x) Z in kron order): targets [a, b] reads qubit a
    O = np.kron(np.eye(2), Z)
    psi = product_state([0.4, 1.3, 2.2])
    assert abs(orc.observable_expectation(psi, [2, 0], O) - math.cos(2.2)) < 1e-13
    assert abs(orc.observable_expectation(psi, [0, 2], O) - math.cos(0.4)) < 1e-13


def test_unnormalised_state_by_hand(orc):
    # psi = (1, 2i, 0, 3) on two qubits: N = 14; qubit 0 is 1 on x = 1, 3
    # (weight 4 + 9), qubit 1 on x = 2, 3 (weight 0 + 9)
    psi = np.array([1, 2j, 0, 3], dtype=np.complex128)
    z = orc.z_expectations(psi)
    assert abs(z[0] - (14 - 2 * 13) / 14) < 1e-15
    assert abs(z[1] - (14 - 2 * 9) / 14) < 1e-15
    assert abs(orc.observable_expectation(psi, [1], Z) - z[1]) < 1e-15


def test_scale_invariance_and_dense_hermitian(orc):
    rng = np.random.default_rng(11)
    n = 5
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    z1 = orc.z_expectations(psi)
    z2 = orc.z_expectations(psi * (0.01 - 3j))
    assert np.max(np.abs(z1 - z2)) < 1e-13
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    O = A + A.conj().T
    t = [3, 1]
    full = dense.full_operator(n, t, O)
    want = (psi.conj() @ full @ psi).real / (psi.conj() @ psi).real
    assert abs(orc.observable_expectation(psi, t, O) - want) < 1e-12
