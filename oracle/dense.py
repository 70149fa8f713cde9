"""Dense linear-algebra checks for the oracle (numpy, small n only).

TEST INFRASTRUCTURE ONLY.  Two textbook constructions of a k-qubit operator
on n qubits, both independent of Algorithm 1's index-group loop:

* ``full_operator``: P^T (I (x) U) P, with P the basis permutation that
  moves the target qubits to the lowest bit positions (np.kron);
* ``apply_tensor``: the state as an n-axis tensor contracted with U as a
  2k-axis tensor (np.tensordot).

``density_evolve`` propagates rho <- U rho U^dag and rho <- sum_i K_i rho K_i^dag
exactly, for comparing trajectory averages with the channel's action.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np


def _perm_matrix(n: int, targets: Sequence[int]) -> np.ndarray:
    """P with (P psi)[y] = psi[x], where bit j of y is bit targets[j] of x for
    j < k and the remaining qubits fill bits k.. in ascending order."""
    k = len(targets)
    rest = [q for q in range(n) if q not in targets]
    order = list(targets) + rest  # bit position in y  -> qubit in x
    dim = 1 << n
    P = np.zeros((dim, dim), dtype=np.complex128)
    for x in range(dim):
        y = 0
        for pos, q in enumerate(order):
            if (x >> q) & 1:
                y |= 1 << pos
        P[y, x] = 1.0
    return P


def full_operator(n: int, targets: Sequence[int], U: np.ndarray) -> np.ndarray:
    k = len(targets)
    P = _perm_matrix(n, targets)
    big = np.kron(np.eye(1 << (n - k), dtype=np.complex128), np.asarray(U, np.complex128))
    return P.T @ big @ P


def apply_tensor(psi: np.ndarray, targets: Sequence[int], U: np.ndarray) -> np.ndarray:
    """Returns U applied to psi via tensor contraction (psi unchanged)."""
    n = int(psi.size).bit_length() - 1
    k = len(targets)
    # C-order reshape: axis a holds qubit n-1-a
    T = np.asarray(psi, np.complex128).reshape([2] * n)
    # U as tensor: axes (out bit k-1 .. out bit 0, in bit k-1 .. in bit 0)
    Ut = np.asarray(U, np.complex128).reshape([2] * (2 * k))
    in_axes_u = list(range(k, 2 * k))           # in bit k-1-i at axis k+i
    state_axes = [n - 1 - targets[k - 1 - i] for i in range(k)]
    R = np.tensordot(Ut, T, axes=(in_axes_u, state_axes))
    # R axes: (out bit k-1..0, remaining state axes in order)
    rem = [a for a in range(n) if a not in state_axes]
    cur = [state_axes[i] for i in range(k)] + rem
    # move back: result axis cur[j] currently at position j
    inv = np.argsort(cur)
    R = np.transpose(R, inv)
    return R.reshape(-1)


def circuit_unitary(circuit) -> np.ndarray:
    dim = 1 << circuit.n
    M = np.eye(dim, dtype=np.complex128)
    for op in circuit.ops:
        if op.kind != 0:
            raise ValueError("gates only")
        M = full_operator(circuit.n, op.qubits, op.mats[0]) @ M
    return M


def density_evolve(circuit, rho: np.ndarray = None) -> np.ndarray:
    """Exact density-matrix evolution of a noisy circuit from |0...0><0...0|."""
    n = circuit.n
    dim = 1 << n
    if rho is None:
        rho = np.zeros((dim, dim), dtype=np.complex128)
        rho[0, 0] = 1.0
    for op in circuit.ops:
        if op.kind == 0:
            U = full_operator(n, op.qubits, op.mats[0])
            rho = U @ rho @ U.conj().T
        else:
            acc = np.zeros_like(rho)
            for K in op.mats:
                F = full_operator(n, op.qubits, K)
                acc += F @ rho @ F.conj().T
            rho = acc
    return rho


def readout_distribution(probs: np.ndarray, n: int, e0, e1) -> np.ndarray:
    """Push a distribution over true bitstrings through independent per-qubit
    confusion matrices [[1-e0, e1], [e0, 1-e1]] (column = true bit)."""
    P = np.asarray(probs, dtype=np.float64).reshape([2] * n)
    for q in range(n):
        A = np.array([[1 - e0[q], e1[q]], [e0[q], 1 - e1[q]]])
        ax = n - 1 - q
        P = np.moveaxis(np.tensordot(A, P, axes=([1], [ax])), 0, ax)
    return P.reshape(-1)
