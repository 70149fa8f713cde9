"""Circuit and noise-channel construction (inputs only).

Conventions used by every consumer of these objects:

* qubit q is bit q of an amplitude index (little-endian);
* an operation's matrix acts on ``qubits`` with matrix row/column bit j
  belonging to ``qubits[j]``;
* a circuit is a time-ordered list of operations grouped in moments
  (Cirq's Circuit -> Moment -> Operation model, Section 2 of the paper);
* a channel is a list of Kraus operators K_0..K_{m-1} (Section 2: channels
  are given through their Kraus operators; Section 3.5 samples one per
  channel and trajectory).

The 1-qubit gate set {sqrt(X), sqrt(Y), sqrt(W)} and the CZ layers are the
usual random-circuit construction; the paper only says "random circuits with
depth 20" (Section 3.6), so the layout below is this project's reading.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

GATE = 0
CHANNEL = 1

_S2 = math.sqrt(2.0)

PAULI_I = np.array([[1, 0], [0, 1]], dtype=np.complex128)
PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)

# Principal square roots of the involutions X, Y and W = (X + Y)/sqrt(2):
# for G with G^2 = I, ((1+i) I + (1-i) G) / 2 squares to G.
SQRT_X = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
SQRT_Y = 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128)
SQRT_W = 0.5 * np.array([[1 + 1j, -1j * _S2], [_S2, 1 + 1j]], dtype=np.complex128)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)

ONE_QUBIT_SET = (("sqrt_x", SQRT_X), ("sqrt_y", SQRT_Y), ("sqrt_w", SQRT_W))


@dataclass
class Op:
    """One gate or one channel in a circuit.

    ``mats`` is ``[U]`` for a gate and ``[K_0, ..., K_{m-1}]`` for a channel,
    each a complex128 array of shape (2^k, 2^k) with k = len(qubits).
    """

    kind: int
    qubits: Tuple[int, ...]
    mats: List[np.ndarray]
    moment: int = 0
    name: str = ""

    @property
    def k(self) -> int:
        return len(self.qubits)


@dataclass
class Circuit:
    n: int
    ops: List[Op] = field(default_factory=list)
    name: str = ""

    @property
    def n_channels(self) -> int:
        return sum(1 for o in self.ops if o.kind == CHANNEL)

    @property
    def n_gates(self) -> int:
        return sum(1 for o in self.ops if o.kind == GATE)

    def count(self, name: str) -> int:
        return sum(1 for o in self.ops if o.name == name)

    def gates_only(self) -> "Circuit":
        return Circuit(self.n, [o for o in self.ops if o.kind == GATE], self.name + "-noiseless")


# --------------------------------------------------------------------------
# Channels (Kraus lists).  Sources: Section 2 names depolarize, phase_damp,
# bit_flip; Section 5.2.1 gives the decay/dephasing channel; Section 5.2.3
# gives the depolarizing channel as (1-r) rho + r/(D^2-1) sum_{mu!=0} P rho P.
# --------------------------------------------------------------------------


def depolarize(p: float) -> List[np.ndarray]:
    """1-qubit depolarizing channel in the Section 5.2.3 form (D = 2)."""
    a = math.sqrt(1.0 - p)
    b = math.sqrt(p / 3.0)
    return [a * PAULI_I, b * PAULI_X, b * PAULI_Y, b * PAULI_Z]


def depolarize2(p: float) -> List[np.ndarray]:
    """2-qubit depolarizing channel in the Section 5.2.3 form (D = 4).

    Paulis are ordered P_a (x) P_b with matrix bit 0 on qubits[0]; the
    identity comes first.
    """
    paulis = [PAULI_I, PAULI_X, PAULI_Y, PAULI_Z]
    out = []
    for hi in range(4):
        for lo in range(4):
            m = np.kron(paulis[hi], paulis[lo])  # bit 0 (low) <- qubits[0]
            if hi == 0 and lo == 0:
                out.append(math.sqrt(1.0 - p) * m)
            else:
                out.append(math.sqrt(p / 15.0) * m)
    return out


def amplitude_damp(gamma: float) -> List[np.ndarray]:
    """Amplitude damping: the decay part of Section 5.2.1 (T_phi -> infinity)."""
    k0 = np.array([[1, 0], [0, math.sqrt(1.0 - gamma)]], dtype=np.complex128)
    k1 = np.array([[0, math.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    return [k0, k1]


def phase_damp(lam: float) -> List[np.ndarray]:
    """Phase damping (Cirq's phase_damp, named in Section 2)."""
    k0 = np.array([[1, 0], [0, math.sqrt(1.0 - lam)]], dtype=np.complex128)
    k1 = np.array([[0, 0], [0, math.sqrt(lam)]], dtype=np.complex128)
    return [k0, k1]


def bit_flip(p: float) -> List[np.ndarray]:
    return [math.sqrt(1.0 - p) * PAULI_I, math.sqrt(p) * PAULI_X]


def decay_dephase(t: float, t1: float, tphi: float) -> List[np.ndarray]:
    """Decay + dephasing channel of Section 5.2.1 with three Kraus operators.

    1/T2 = 1/(2 T1) + 1/T_phi.  The printed third operator has a 1 in its
    upper-left entry, which breaks completeness (sum K^dag K = diag(2, 1));
    this uses a zero there, which restores completeness and reproduces the
    channel's density-matrix form given in the same section.
    """
    inv_t2 = 1.0 / (2.0 * t1) + 1.0 / tphi
    e1 = math.exp(-t / t1)
    e2 = math.exp(-t * inv_t2)
    k0 = np.array([[1, 0], [0, e2]], dtype=np.complex128)
    k1 = np.array([[0, math.sqrt(1.0 - e1)], [0, 0]], dtype=np.complex128)
    k2 = np.array([[0, 0], [0, math.sqrt(max(e1 - e2 * e2, 0.0))]], dtype=np.complex128)
    return [k0, k1, k2]


# --------------------------------------------------------------------------
# Coherent (unitary) errors.
# --------------------------------------------------------------------------


def fsim(theta: float, phi: float) -> np.ndarray:
    """fSim(theta, phi) of Section 5.2.2: a rotation by theta between |01>
    and |10> (off-diagonal -i sin theta) and the phase e^{-i phi} on |11>.
    Symmetric under exchanging the two qubits, so the target order does not
    matter."""
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


SQRT_ISWAP = fsim(-math.pi / 4, 0.0)  # fSim at theta = -pi/4: the square root of iSWAP


def z_phase(varphi: float) -> np.ndarray:
    """Single-qubit Z phase error exp(i varphi Z) (Section 5.2.2)."""
    return np.diag([np.exp(1j * varphi), np.exp(-1j * varphi)]).astype(np.complex128)


def u_zz(zeta: float, gate_time: float) -> np.ndarray:
    """Control error of Section 4: exp(-i 2 pi zeta T |11><11|), a phase on
    |11> only."""
    return np.diag([1, 1, 1, np.exp(-2j * math.pi * zeta * gate_time)]).astype(np.complex128)


def approx_noise_grid_circuit(rows: int, cols: int, cycles: int, seed: int = 0,
                              dtheta: float = 0.01, dphi: float = 0.05,
                              zphase_sigma: float = 0.01, zeta: float = 0.0,
                              gate_time: float = 10e-9, p_dep1: float = 1e-3,
                              p_dep2: float = 5e-3, step_time: float = 0.025,
                              t1: float = 15.0, tphi: float = 30.0) -> Circuit:
    """Section 5.2's approximate noise model on a rows x cols grid.

    Per cycle: a random 1-qubit layer, each gate followed by 1-qubit
    depolarizing; then one coupler pattern of sqrt(iSWAP) gates, each
    dressed with its coherent errors -- exp(i varphi Z) on both qubits before
    and after, fSim(dtheta, dphi) right after the gate, and (zeta > 0) the
    U_ZZ control error -- then 2-qubit depolarizing on the pair.  Every
    moment ends with the decay/dephasing channel on every qubit (times in
    microseconds: step_time per moment, T1, T_phi).

    The Z phase angles are drawn once per gate instance from a normal
    distribution of width zphase_sigma (a calibrated, static error: the
    same in every trajectory), from the circuit's seed.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rows * cols
    pats = [p for p in grid_coupler_patterns(rows, cols) if p]
    dep1 = depolarize(p_dep1)
    dep2 = depolarize2(p_dep2)
    dd = decay_dephase(step_time, t1, tphi)
    err = fsim(dtheta, dphi)
    zz = u_zz(zeta, gate_time) if zeta else None
    ops: List[Op] = []
    moment = 0
    for cyc in range(cycles):
        layer = _one_qubit_layer(n, rng)
        for q in range(n):
            nm, u = layer[q]
            ops.append(Op(GATE, (q,), [u], moment, nm))
            ops.append(Op(CHANNEL, (q,), dep1, moment, "depolarize"))
        for q in range(n):
            ops.append(Op(CHANNEL, (q,), dd, moment, "decay_dephase"))
        moment += 1
        for a, b in pats[cyc % len(pats)]:
            for q in (a, b):
                ops.append(Op(GATE, (q,), [z_phase(rng.normal(0.0, zphase_sigma))], moment,
                              "z_phase"))
            ops.append(Op(GATE, (a, b), [SQRT_ISWAP], moment, "sqrt_iswap"))
            ops.append(Op(GATE, (a, b), [err], moment, "fsim_error"))
            if zz is not None:
                ops.append(Op(GATE, (a, b), [zz], moment, "u_zz"))
            for q in (a, b):
                ops.append(Op(GATE, (q,), [z_phase(rng.normal(0.0, zphase_sigma))], moment,
                              "z_phase"))
            ops.append(Op(CHANNEL, (a, b), dep2, moment, "depolarize2"))
        for q in range(n):
            ops.append(Op(CHANNEL, (q,), dd, moment, "decay_dephase"))
        moment += 1
    return Circuit(n, ops, f"approx_noise{rows}x{cols}")


# --------------------------------------------------------------------------
# Random matrices for tests.
# --------------------------------------------------------------------------


def random_unitary(k: int, rng: np.random.Generator) -> np.ndarray:
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return (q * ph).astype(np.complex128)


def random_matrix(k: int, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    d = 1 << k
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    return (scale * z / math.sqrt(2.0 * d)).astype(np.complex128)


# --------------------------------------------------------------------------
# Circuit layouts.
# --------------------------------------------------------------------------


def grid_coupler_patterns(rows: int, cols: int, qubit_of=None) -> List[List[Tuple[int, int]]]:
    """Four disjoint nearest-neighbour CZ patterns on a rows x cols grid.

    A: horizontal pairs starting at even columns, B: horizontal pairs at odd
    columns, C: vertical pairs at even rows, D: vertical pairs at odd rows.
    Every grid edge is in exactly one pattern (Section 5.1.4 describes the
    four-pattern cycle).  ``qubit_of(r, c)`` returns None for absent sites.
    """
    if qubit_of is None:
        def qubit_of(r, c):
            return cols * r + c
    pats: List[List[Tuple[int, int]]] = [[], [], [], []]
    for r in range(rows):
        for c in range(cols - 1):
            a, b = qubit_of(r, c), qubit_of(r, c + 1)
            if a is None or b is None:
                continue
            pats[0 if c % 2 == 0 else 1].append((a, b))
    for r in range(rows - 1):
        for c in range(cols):
            a, b = qubit_of(r, c), qubit_of(r + 1, c)
            if a is None or b is None:
                continue
            pats[2 if r % 2 == 0 else 3].append((a, b))
    return pats


def _one_qubit_layer(n: int, rng: np.random.Generator) -> List[Tuple[str, np.ndarray]]:
    picks = rng.integers(0, len(ONE_QUBIT_SET), size=n)
    return [ONE_QUBIT_SET[int(i)] for i in picks]


def _layered_circuit(
    n: int,
    cycles: int,
    pair_layers: Sequence[Sequence[Tuple[int, int]]],
    seed: int,
    p_dep: float | None,
    gamma: float | None,
    name: str,
) -> Circuit:
    """Cycle = a random 1-qubit layer then one CZ layer, both as moments.

    Noise placement (this project's reading of Sections 2 and 5.2): a
    1-qubit depolarizing channel after every gate on each qubit the gate
    touches, then amplitude damping on every qubit at the end of every
    moment ("after every gate or idle time").
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: List[Op] = []
    dep = depolarize(p_dep) if p_dep else None
    ad = amplitude_damp(gamma) if gamma else None
    moment = 0
    for cyc in range(cycles):
        # 1-qubit layer
        layer = _one_qubit_layer(n, rng)
        for q in range(n):
            nm, u = layer[q]
            ops.append(Op(GATE, (q,), [u], moment, nm))
        if dep is not None:
            for q in range(n):
                ops.append(Op(CHANNEL, (q,), dep, moment, "depolarize"))
        if ad is not None:
            for q in range(n):
                ops.append(Op(CHANNEL, (q,), ad, moment, "amplitude_damp"))
        moment += 1
        # 2-qubit layer
        pairs = pair_layers[cyc % len(pair_layers)]
        for a, b in pairs:
            ops.append(Op(GATE, (a, b), [CZ], moment, "cz"))
        if dep is not None:
            for a, b in pairs:
                ops.append(Op(CHANNEL, (a,), dep, moment, "depolarize"))
                ops.append(Op(CHANNEL, (b,), dep, moment, "depolarize"))
        if ad is not None:
            for q in range(n):
                ops.append(Op(CHANNEL, (q,), ad, moment, "amplitude_damp"))
        moment += 1
    return Circuit(n, ops, name)


def chain_circuit(n: int = 12, cycles: int = 20, p_dep: float | None = 1e-3, seed: int = 0,
                  gamma: float | None = None) -> Circuit:
    """1-D chain; CZ on (0,1),(2,3),... in even cycles and (1,2),(3,4),... in odd ones."""
    even = [(q, q + 1) for q in range(0, n - 1, 2)]
    odd = [(q, q + 1) for q in range(1, n - 1, 2)]
    return _layered_circuit(n, cycles, [even, odd], seed, p_dep, gamma, f"chain{n}")


def grid_circuit(rows: int, cols: int, cycles: int = 20, p_dep: float | None = None,
                 gamma: float | None = None, seed: int = 0) -> Circuit:
    """rows x cols grid, qubit q = cols*r + c, CZ patterns A, B, C, D cycled."""
    pats = grid_coupler_patterns(rows, cols)
    pats = [p for p in pats if p]
    return _layered_circuit(rows * cols, cycles, pats, seed, p_dep, gamma,
                            f"grid{rows}x{cols}")


def generic_grid_circuit(n: int, cycles: int, p_dep: float | None = None,
                         gamma: float | None = None, seed: int = 0) -> Circuit:
    """n qubits on R = floor(sqrt(n)) rows of C = ceil(n/R) sites, row-major,
    last row partial."""
    rows = max(1, int(math.isqrt(n)))
    cols = -(-n // rows)

    def qubit_of(r, c):
        q = cols * r + c
        return q if q < n else None

    pats = [p for p in grid_coupler_patterns(rows, cols, qubit_of) if p]
    if not pats:
        pats = [[]]
    return _layered_circuit(n, cycles, pats, seed, p_dep, gamma, f"ggrid{n}")


def random_gate_circuit(n: int, n_gates: int, seed: int, max_k: int = 2,
                        unitary: bool = True) -> Circuit:
    """Random dense gates on random distinct targets (tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops = []
    for i in range(n_gates):
        k = int(rng.integers(1, min(max_k, n) + 1))
        qs = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        m = random_unitary(k, rng) if unitary else random_matrix(k, rng)
        ops.append(Op(GATE, qs, [m], i, f"u{k}"))
    return Circuit(n, ops, f"rand{n}")


def random_noisy_circuit(n: int, n_layers: int, seed: int, p_dep: float = 0.05,
                         gamma: float = 0.05, lam: float = 0.0, p_flip: float = 0.0,
                         max_k: int = 2) -> Circuit:
    """Random unitary layers interleaved with 1-qubit channels (tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops = []
    for layer in range(n_layers):
        k = int(rng.integers(1, min(max_k, n) + 1))
        qs = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        ops.append(Op(GATE, qs, [random_unitary(k, rng)], layer, f"u{k}"))
        for q in qs:
            if p_dep:
                ops.append(Op(CHANNEL, (q,), depolarize(p_dep), layer, "depolarize"))
            if gamma:
                ops.append(Op(CHANNEL, (q,), amplitude_damp(gamma), layer, "amplitude_damp"))
            if lam:
                ops.append(Op(CHANNEL, (q,), phase_damp(lam), layer, "phase_damp"))
            if p_flip:
                ops.append(Op(CHANNEL, (q,), bit_flip(p_flip), layer, "bit_flip"))
    return Circuit(n, ops, f"noisy{n}")


def readout_arrays(n: int, p00: float, p11: float) -> Tuple[np.ndarray, np.ndarray]:
    """Per-qubit readout misidentification probabilities (Section 5.1.2):
    e0[q] = P(read 1 | state 0), e1[q] = P(read 0 | state 1)."""
    return np.full(n, float(p00)), np.full(n, float(p11))
