"""CPU oracle for the noisy quantum-trajectory method (arXiv 2111.02396).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only code allowed to import this
package.  The product path never calls it and shares no code with it.

The numeric core is ``qs_oracle.c`` (complex128, single thread, no fusion,
no deferral).  This module marshals circuits into it and computes the Kraus
lower bounds with a library eigenvalue routine (Section 3.5: pbar_i is the
smallest squared singular value of K_i, i.e. the smallest eigenvalue of
K_i^dag K_i).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DELAYED = 0
NAIVE = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        c_d, c_i, c_u32, c_u64, c_i64 = (ctypes.c_double, ctypes.c_int, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_int64)
        vp = ctypes.c_void_p
        L.or_philox4x32_10.argtypes = [vp, vp, vp]
        L.or_philox4x32_10.restype = None
        L.or_u53.argtypes = [c_u32, c_u32]
        L.or_u53.restype = c_d
        L.or_draw.argtypes = [c_u64, c_u32, c_u32, c_u32, c_u32]
        L.or_draw.restype = c_d
        L.or_apply_matrix.argtypes = [vp, c_i, c_i, vp, vp]
        L.or_apply_matrix.restype = None
        L.or_norm_sq.argtypes = [vp, c_i]
        L.or_norm_sq.restype = c_d
        L.or_expectation.argtypes = [vp, c_i, c_i, vp, vp, P(c_d), P(c_d)]
        L.or_expectation.restype = None
        L.or_select_branch.argtypes = [vp, c_i, c_i, vp, c_i, vp, vp, c_i, c_i, c_d,
                                       P(c_i), P(c_d), P(c_d)]
        L.or_select_branch.restype = c_i
        L.or_select_many.argtypes = [vp, c_i, c_i, vp, c_i, vp, vp, c_i, c_i, c_i64, vp, vp]
        L.or_select_many.restype = None
        L.or_apply_kraus_normalised.argtypes = [vp, c_i, c_i, vp, vp]
        L.or_apply_kraus_normalised.restype = c_i
        L.or_sample.argtypes = [vp, c_i, c_u64, c_u32, c_u32, c_i64, vp, vp, vp, vp]
        L.or_sample.restype = c_i
        L.or_run_trajectory.argtypes = [c_i, c_i, vp, vp, vp, vp, vp, vp, vp, vp, vp, c_i,
                                        c_u64, c_u32, c_u32, c_i64, vp, vp, vp, vp, vp, vp,
                                        vp, vp, vp]
        L.or_run_trajectory.restype = c_i
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c128(m) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(m, dtype=np.complex128))


# ---------------------------------------------------------------- RNG

def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(x) for x in out]


def u53(w0: int, w1: int) -> float:
    return float(lib().or_u53(w0, w1))


def draw(seed: int, index: int, traj: int, circ: int, stream: int) -> float:
    return float(lib().or_draw(seed, index, traj, circ, stream))


# ---------------------------------------------------------------- Kraus bounds

def kraus_bounds(kraus: Sequence[np.ndarray], mix_tol: float = 1e-12):
    """pbar_i = lambda_min(K_i^dag K_i) clamped at 0 (Section 3.5) and whether
    every K_i^dag K_i is a multiple of the identity (then sum pbar_i = 1)."""
    pbar = []
    mixture = True
    for K in kraus:
        K = _c128(K)
        G = K.conj().T @ K
        G = 0.5 * (G + G.conj().T)
        lam = float(np.linalg.eigvalsh(G)[0])
        pbar.append(max(lam, 0.0))
        c = float(np.real(np.trace(G))) / G.shape[0]
        if np.max(np.abs(G - c * np.eye(G.shape[0]))) > mix_tol:
            mixture = False
    return np.asarray(pbar, dtype=np.float64), mixture


# ---------------------------------------------------------------- state ops

def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def apply_matrix(psi: np.ndarray, targets: Sequence[int], U: np.ndarray) -> None:
    """In place: Algorithm 1 on a complex128 state."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    n = int(psi.size).bit_length() - 1
    t = np.asarray(targets, dtype=np.int32)
    U = _c128(U)
    assert U.shape == (1 << len(t), 1 << len(t))
    lib().or_apply_matrix(_ptr(psi), n, len(t), _ptr(t), _ptr(U))


def norm_sq(psi: np.ndarray) -> float:
    n = int(psi.size).bit_length() - 1
    return float(lib().or_norm_sq(_ptr(psi), n))


def expectation(psi: np.ndarray, targets: Sequence[int], M: np.ndarray) -> complex:
    n = int(psi.size).bit_length() - 1
    t = np.asarray(targets, dtype=np.int32)
    M = _c128(M)
    re, im = ctypes.c_double(), ctypes.c_double()
    lib().or_expectation(_ptr(psi), n, len(t), _ptr(t), _ptr(M), ctypes.byref(re),
                         ctypes.byref(im))
    return complex(re.value, im.value)


def z_expectations(psi: np.ndarray) -> np.ndarray:
    """<Z_q> = sum_x (-1)^{x_q} |psi_x|^2 / sum_x |psi_x|^2 for every qubit q:
    the per-trajectory expectation of Section 3.5 on the normalised state,
    written out from the definition (bit q of the index selects the sign)."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = int(psi.size).bit_length() - 1
    p = psi.real ** 2 + psi.imag ** 2
    N = p.sum()
    x = np.arange(psi.size, dtype=np.int64)
    return np.array([(p * (1 - 2 * ((x >> q) & 1))).sum() / N for q in range(n)])


def observable_expectation(psi: np.ndarray, targets: Sequence[int], O: np.ndarray) -> float:
    """<psi|O|psi> / <psi|psi> for a Hermitian O on the targets (matrix index
    bit j = targets[j])."""
    return float(expectation(psi, targets, O).real / norm_sq(psi))


def select_branch(psi: np.ndarray, targets: Sequence[int], kraus: Sequence[np.ndarray],
                  mode: int, r: float, pbar=None, mixture=None) -> Dict:
    n = int(psi.size).bit_length() - 1
    t = np.asarray(targets, dtype=np.int32)
    Ks = _c128(np.stack([_c128(K) for K in kraus]))
    if pbar is None:
        pbar, mixture = kraus_bounds(kraus)
    pbar = np.asarray(pbar, dtype=np.float64)
    path = ctypes.c_int()
    mf, ms = ctypes.c_double(), ctypes.c_double()
    c = lib().or_select_branch(_ptr(psi), n, len(t), _ptr(t), len(kraus), _ptr(Ks), _ptr(pbar),
                               int(bool(mixture)), mode, float(r), ctypes.byref(path),
                               ctypes.byref(mf), ctypes.byref(ms))
    return {"choice": int(c), "path": int(path.value), "margin_fast": mf.value,
            "margin_slow": ms.value}


def select_many(psi: np.ndarray, targets, kraus, mode: int, rs: np.ndarray) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    t = np.asarray(targets, dtype=np.int32)
    Ks = _c128(np.stack([_c128(K) for K in kraus]))
    pbar, mixture = kraus_bounds(kraus)
    rs = np.ascontiguousarray(rs, dtype=np.float64)
    out = np.zeros(rs.size, dtype=np.int8)
    lib().or_select_many(_ptr(psi), n, len(t), _ptr(t), len(kraus), _ptr(Ks), _ptr(pbar),
                         int(bool(mixture)), mode, rs.size, _ptr(rs), _ptr(out))
    return out


def apply_kraus_normalised(psi: np.ndarray, targets, K) -> None:
    n = int(psi.size).bit_length() - 1
    t = np.asarray(targets, dtype=np.int32)
    K = _c128(K)
    rc = lib().or_apply_kraus_normalised(_ptr(psi), n, len(t), _ptr(t), _ptr(K))
    if rc != 0:
        raise ZeroDivisionError("Kraus operator annihilated the state")


def sample(psi: np.ndarray, seed: int, traj: int, circ: int, n_samples: int,
           e0=None, e1=None):
    n = int(psi.size).bit_length() - 1
    out = np.zeros(n_samples, dtype=np.uint64)
    margins = np.zeros(n_samples, dtype=np.float64)
    e0 = None if e0 is None else np.ascontiguousarray(e0, dtype=np.float64)
    e1 = None if e1 is None else np.ascontiguousarray(e1, dtype=np.float64)
    rc = lib().or_sample(_ptr(psi), n, seed, traj, circ, n_samples, _ptr(e0), _ptr(e1),
                         _ptr(out), _ptr(margins))
    if rc != 0:
        raise MemoryError("oracle sampling failed")
    return out, margins


# ---------------------------------------------------------------- circuits

class Marshalled:
    """A circuit flattened into the oracle's op arrays."""

    def __init__(self, circuit):
        ops = circuit.ops
        self.n = circuit.n
        self.n_ops = len(ops)
        self.kinds = np.zeros(self.n_ops, dtype=np.int32)
        self.ks = np.zeros(self.n_ops, dtype=np.int32)
        self.targets = np.zeros(5 * self.n_ops, dtype=np.int32)
        self.n_mats = np.zeros(self.n_ops, dtype=np.int32)
        self.first_mat = np.zeros(self.n_ops, dtype=np.int64)
        self.mixture = np.zeros(self.n_ops, dtype=np.int32)
        offs, pbars, chunks = [], [], []
        pos = 0
        cache = {}
        for o, op in enumerate(ops):
            self.kinds[o] = op.kind
            self.ks[o] = op.k
            self.targets[5 * o:5 * o + op.k] = op.qubits
            self.n_mats[o] = len(op.mats)
            self.first_mat[o] = len(offs)
            if op.kind == 1:
                key = id(op.mats)
                if key not in cache:
                    cache[key] = kraus_bounds(op.mats)
                pb, mix = cache[key]
                self.mixture[o] = int(mix)
            else:
                pb = np.zeros(1)
            for i, m in enumerate(op.mats):
                m = _c128(m)
                offs.append(pos)
                pbars.append(float(pb[i]))
                chunks.append(m.ravel())
                pos += m.size
        self.mat_off = np.asarray(offs, dtype=np.int64)
        self.pbar = np.asarray(pbars, dtype=np.float64)
        self.pool = np.ascontiguousarray(np.concatenate(chunks) if chunks else
                                         np.zeros(1, np.complex128))
        self.n_channels = int(np.sum(self.kinds == 1))


def run_trajectory(circuit, traj: int, mode: int = DELAYED, seed: int = 0, circ: int = 0,
                   n_samples: int = 0, e0=None, e1=None, return_state: bool = False,
                   marshalled: Marshalled = None) -> Dict:
    m = marshalled if marshalled is not None else Marshalled(circuit)
    nch = m.n_channels
    choices = np.zeros(max(nch, 1), dtype=np.int8)
    paths = np.zeros(max(nch, 1), dtype=np.int8)
    mf = np.zeros(max(nch, 1), dtype=np.float64)
    ms = np.zeros(max(nch, 1), dtype=np.float64)
    samples = np.zeros(max(n_samples, 1), dtype=np.uint64)
    smargins = np.zeros(max(n_samples, 1), dtype=np.float64)
    psi = np.zeros(1 << m.n, dtype=np.complex128) if return_state else None
    e0 = None if e0 is None else np.ascontiguousarray(e0, dtype=np.float64)
    e1 = None if e1 is None else np.ascontiguousarray(e1, dtype=np.float64)
    rc = lib().or_run_trajectory(
        m.n, m.n_ops, _ptr(m.kinds), _ptr(m.ks), _ptr(m.targets), _ptr(m.n_mats),
        _ptr(m.first_mat), _ptr(m.mat_off), _ptr(m.pool), _ptr(m.pbar), _ptr(m.mixture),
        mode, seed, traj, circ, n_samples, _ptr(e0), _ptr(e1), _ptr(choices), _ptr(paths),
        _ptr(mf), _ptr(ms), _ptr(samples), _ptr(smargins), _ptr(psi))
    if rc != 0:
        raise RuntimeError(f"oracle trajectory failed (rc={rc})")
    return {
        "choices": choices[:nch], "paths": paths[:nch], "margin_fast": mf[:nch],
        "margin_slow": ms[:nch], "samples": samples[:n_samples],
        "sample_margins": smargins[:n_samples], "state": psi,
    }


def simulate(circuit, psi: Optional[np.ndarray] = None) -> np.ndarray:
    """Apply every gate of a channel-free circuit to |0...0> (or psi)."""
    if psi is None:
        psi = zero_state(circuit.n)
    for op in circuit.ops:
        if op.kind != 0:
            raise ValueError("simulate() takes a circuit without channels")
        apply_matrix(psi, op.qubits, op.mats[0])
    return psi
