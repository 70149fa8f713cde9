"""Closed-form states for checking the GPU path at sizes no oracle run
reaches (no simulation arithmetic of the method: each function states the
exact result of a special circuit).

* pair products: U on every qubit, a 2-qubit unitary on each pair
  (q, q + n/2), V on every qubit -- the state is the tensor product of the
  pairs' 4-vectors, so any amplitude is a product of n/2 numbers and the
  inverse CDF in index order can be followed bit by bit;
* GHZ: H then a CNOT chain, (|0...0> + |1...1>)/sqrt(2);
* mirror circuits: a circuit followed by its inverse is the identity.
"""

import math

import numpy as np

import workloads as W


def _kron_pair(a_hi, a_lo):
    """4x4 operator on a pair index a + 2 b (a: first qubit) from 1-qubit
    operators on the second (hi) and first (lo) qubit."""
    return np.kron(a_hi, a_lo)


def pair_product(n, seed):
    """U on every qubit, a random 2-qubit unitary on each pair (q, q + n/2),
    V on every qubit: a product of n/2 pair states.  Returns the circuit and
    each pair's 4-vector w_q (index x_q + 2 x_{q+n/2})."""
    rng = np.random.default_rng(seed)
    h = n // 2
    U = [W.random_unitary(1, rng) for _ in range(n)]
    P = [W.random_unitary(2, rng) for _ in range(h)]
    V = [W.random_unitary(1, rng) for _ in range(n)]
    ops = [W.Op(W.GATE, (q,), [U[q]], 0) for q in range(n)]
    ops += [W.Op(W.GATE, (q, q + h), [P[q]], 1) for q in range(h)]
    ops += [W.Op(W.GATE, (q,), [V[q]], 2) for q in range(n)]
    e = np.zeros(4, dtype=np.complex128)
    e[0] = 1.0
    w = [_kron_pair(V[q + h], V[q]) @ P[q] @ _kron_pair(U[q + h], U[q]) @ e for q in range(h)]
    return W.Circuit(n, ops, f"pairs{n}"), w


def pair_amplitudes(w, n, xs):
    h = n // 2
    amp = np.ones(len(xs), dtype=np.complex128)
    for q in range(h):
        idx = ((xs >> q) & 1) + 2 * ((xs >> (q + h)) & 1)
        amp *= w[q][idx]
    return amp


def pair_inverse_cdf(w, n, u):
    """Smallest x with u < C(x), C the inclusive prefix of |psi_x|^2 in index
    order, for the pair-product state: decided bit by bit from the top (the
    indices sharing the bits already decided form one contiguous range).
    Returns x and the distance from u to the nearest boundary met."""
    h = n // 2
    p = [np.abs(v) ** 2 / np.sum(np.abs(v) ** 2) for v in w]
    x, cum, mass, margin = 0, 0.0, 1.0, math.inf
    for j in range(n - 1, -1, -1):
        if j >= h:
            q = j - h
            p0 = p[q][0] + p[q][1]  # second qubit of pair q reads 0
        else:
            q = j
            b = (x >> (q + h)) & 1
            p0 = p[q][2 * b] / (p[q][2 * b] + p[q][2 * b + 1])  # first qubit, given the second
        boundary = cum + mass * p0
        margin = min(margin, abs(u - boundary))
        if u < boundary:
            mass = mass * p0
        else:
            cum = boundary
            mass = mass * (1.0 - p0)
            x |= 1 << j
    return x, margin


def pair_prefix(w, n, x):
    """Exclusive and inclusive prefix of |psi|^2 in index order at index x
    for the pair-product state: (sum over y < x, sum over y <= x), decided
    bit by bit from the top like pair_inverse_cdf."""
    h = n // 2
    p = [np.abs(v) ** 2 / np.sum(np.abs(v) ** 2) for v in w]
    cum, mass = 0.0, 1.0
    for j in range(n - 1, -1, -1):
        if j >= h:
            q = j - h
            p0 = p[q][0] + p[q][1]
        else:
            q = j
            b = (x >> (q + h)) & 1
            p0 = p[q][2 * b] / (p[q][2 * b] + p[q][2 * b + 1])
        if (x >> j) & 1:
            cum += mass * p0
            mass *= 1.0 - p0
        else:
            mass *= p0
    return cum, cum + mass


def ghz_circuit(n):
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
    # matrix bit 0 <-> control, bit 1 <-> target: |c=1,t=0> (index 1) <-> |1,1> (index 3)
    CNOT = np.eye(4, dtype=np.complex128)[[0, 3, 2, 1]]
    ops = [W.Op(W.GATE, (0,), [H], 0)]
    ops += [W.Op(W.GATE, (q, q + 1), [CNOT], 1 + q) for q in range(n - 1)]
    return W.Circuit(n, ops, f"ghz{n}")


def mirror_circuit(c):
    inv = [W.Op(o.kind, o.qubits, [np.conj(o.mats[0]).T], 10_000 - o.moment) for o in reversed(c.ops)]
    return W.Circuit(c.n, list(c.ops) + inv, c.name + "-mirror")
