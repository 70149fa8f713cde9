"""Pins for the oracle's gate application (Algorithm 1), norm and expectation.

Each check uses something other than the oracle itself: two textbook dense
constructions (Kronecker product + permutation, tensor contraction), closed
forms (product states, GHZ), mirror circuits and norm preservation.
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import dense

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2)
# CNOT with control on matrix bit 0 (targets[0]) and target on matrix bit 1.
CNOT_C0 = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=np.complex128)


def _rand_state(n, rng):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)


def test_dense_constructions_agree():
    rng = np.random.default_rng(1)
    for n, k in [(3, 1), (4, 2), (5, 3), (6, 2)]:
        t = list(rng.choice(n, size=k, replace=False))
        U = W.random_matrix(k, rng)
        psi = _rand_state(n, rng)
        a = dense.full_operator(n, t, U) @ psi
        b = dense.apply_tensor(psi, t, U)
        assert np.allclose(a, b, atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_apply_matches_dense(orc, k):
    rng = np.random.default_rng(100 + k)
    for trial in range(6):
        n = int(rng.integers(k, 9))
        t = [int(x) for x in rng.choice(n, size=k, replace=False)]
        U = W.random_matrix(k, rng)  # need not be unitary
        psi = _rand_state(n, rng)
        ref = dense.full_operator(n, t, U) @ psi
        got = psi.copy()
        orc.apply_matrix(got, t, U)
        assert np.max(np.abs(got - ref)) < 1e-12, (n, t)


def test_target_order_matters(orc):
    # matrix bit j belongs to targets[j]: swapping the targets of a
    # non-symmetric gate changes the result exactly as the dense form says
    rng = np.random.default_rng(5)
    psi = _rand_state(4, rng)
    a, b = psi.copy(), psi.copy()
    orc.apply_matrix(a, [0, 2], CNOT_C0)
    orc.apply_matrix(b, [2, 0], CNOT_C0)
    assert not np.allclose(a, b)
    assert np.allclose(a, dense.apply_tensor(psi, [0, 2], CNOT_C0), atol=1e-14)
    assert np.allclose(b, dense.apply_tensor(psi, [2, 0], CNOT_C0), atol=1e-14)


def test_product_state_closed_form(orc):
    rng = np.random.default_rng(2)
    n = 7
    us = [W.random_unitary(1, rng) for _ in range(n)]
    psi = orc.zero_state(n)
    for q in range(n):
        orc.apply_matrix(psi, [q], us[q])
    for x in range(1 << n):
        amp = 1.0 + 0j
        for q in range(n):
            amp *= us[q][(x >> q) & 1, 0]
        assert abs(psi[x] - amp) < 1e-14


def test_ghz(orc):
    n = 9
    psi = orc.zero_state(n)
    orc.apply_matrix(psi, [0], H)
    for q in range(n - 1):
        orc.apply_matrix(psi, [q, q + 1], CNOT_C0)
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


def test_mirror_circuit_returns_to_zero(orc):
    c = W.random_gate_circuit(8, 60, seed=3, max_k=4)
    psi = orc.zero_state(8)
    for op in c.ops:
        orc.apply_matrix(psi, op.qubits, op.mats[0])
    for op in reversed(c.ops):
        orc.apply_matrix(psi, op.qubits, op.mats[0].conj().T)
    ref = orc.zero_state(8)
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_norm_preserved_and_sequential(orc):
    c = W.random_gate_circuit(10, 40, seed=4, max_k=5)
    psi = orc.simulate(c)
    assert abs(orc.norm_sq(psi) - 1.0) < 1e-12
    rng = np.random.default_rng(9)
    v = rng.standard_normal(1 << 6) + 1j * rng.standard_normal(1 << 6)
    assert abs(orc.norm_sq(v) - float(np.sum(np.abs(v) ** 2))) < 1e-12


def test_expectation_matches_dense(orc):
    rng = np.random.default_rng(6)
    for k in [1, 2, 3]:
        n = 6
        t = [int(x) for x in rng.choice(n, size=k, replace=False)]
        M = W.random_matrix(k, rng)
        psi = _rand_state(n, rng)
        ref = np.vdot(psi, dense.full_operator(n, t, M) @ psi)
        assert abs(orc.expectation(psi, t, M) - ref) < 1e-13


def test_gate_set_definitions():
    X, Y = W.PAULI_X, W.PAULI_Y
    Wg = (X + Y) / math.sqrt(2)
    for root, g in [(W.SQRT_X, X), (W.SQRT_Y, Y), (W.SQRT_W, Wg)]:
        assert np.allclose(root @ root, g, atol=1e-15)
        assert np.allclose(root.conj().T @ root, np.eye(2), atol=1e-15)
        # principal root: eigenvalues 1 and i
        ev = np.sort_complex(np.linalg.eigvals(root))
        assert np.allclose(sorted(ev, key=lambda z: z.imag), [1, 1j], atol=1e-12)
    assert np.allclose(W.CZ @ W.CZ, np.eye(4))


def test_circuit_unitary_vs_oracle(orc):
    c = W.chain_circuit(6, cycles=4, p_dep=None, seed=11)
    U = dense.circuit_unitary(c)
    psi = orc.simulate(c)
    assert np.max(np.abs(psi - U[:, 0])) < 1e-13
