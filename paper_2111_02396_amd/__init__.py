"""Python binding of libqs (include/qs.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python
objects to the C structures, calls the entry points of the same names, and
turns error codes into exceptions.  PyTorch, when used, only provides device
buffers and streams.  There is no fallback: if libqs.so is missing or fails
to load, every call raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs.so")
_lib = None

QS_OK = 0
QS_ERR_INVALID_ARGUMENT = -1
QS_ERR_OUT_OF_MEMORY = -2
QS_ERR_DEVICE = -3
QS_ERR_ZERO_NORM = -4
QS_ERR_NOT_SUPPORTED = -5

QS_KRAUS_DELAYED = 0
QS_KRAUS_NAIVE = 1
QS_KRAUS_CONVENTIONAL_INPLACE = 2
QS_OP_GATE = 0
QS_OP_CHANNEL = 1
QS_TRAJ_RETURN_STATE = 1
QS_TRAJ_TIME_KERNELS = 2
QS_TRAJ_NO_GRAPH = 4
QS_TRAJ_GRAPH = 8

_NAMES = {0: "QS_OK", -1: "QS_ERR_INVALID_ARGUMENT", -2: "QS_ERR_OUT_OF_MEMORY",
          -3: "QS_ERR_DEVICE", -4: "QS_ERR_ZERO_NORM", -5: "QS_ERR_NOT_SUPPORTED"}


class QsError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_NAMES.get(code, code)}: {message}")
        self.code = code


class QsOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32),
                ("targets", ctypes.c_int32 * 5), ("n_mats", ctypes.c_int32),
                ("mat_offset", ctypes.c_int64)]


class QsCircuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_ops", ctypes.c_int32),
                ("ops", ctypes.POINTER(QsOp)), ("mat_pool", ctypes.c_void_p),
                ("pool_len", ctypes.c_int64)]


class QsTrajParams(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_int64), ("traj_offset", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("circuit_id", ctypes.c_uint32),
                ("mode", ctypes.c_int32), ("max_fuse", ctypes.c_int32),
                ("tile_bits", ctypes.c_int32), ("n_samples", ctypes.c_int32), ("p0to1", ctypes.c_void_p),
                ("p1to0", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class QsTrajResult(ctypes.Structure):
    _fields_ = [("bitstrings", ctypes.c_void_p), ("kraus_choices", ctypes.c_void_p),
                ("kraus_paths", ctypes.c_void_p), ("n_slow", ctypes.c_void_p),
                ("final_state", ctypes.c_void_p), ("sweeps", ctypes.c_int64),
                ("gate_sweeps", ctypes.c_int64), ("host_seconds", ctypes.c_double),
                ("gate_kernel_ms", ctypes.c_double), ("gate_kernel_launches", ctypes.c_int64),
                ("gate_k_launches", ctypes.c_int64 * 6), ("zero_start_sweeps", ctypes.c_int64),
                ("z_expect", ctypes.c_void_p), ("max_fuse_used", ctypes.c_int32),
                ("tile_bits_used", ctypes.c_int32), ("tune_ms", ctypes.c_double),
                ("graph_replays", ctypes.c_int64)]


class QsBatchItem(ctypes.Structure):
    _fields_ = [("circuit", ctypes.c_void_p), ("n_traj", ctypes.c_int64),
                ("traj_offset", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("circuit_id", ctypes.c_uint32), ("n_samples", ctypes.c_int32),
                ("p0to1", ctypes.c_void_p), ("p1to0", ctypes.c_void_p),
                ("bitstrings", ctypes.c_void_p), ("kraus_choices", ctypes.c_void_p)]


class QsBatchParams(ctypes.Structure):
    _fields_ = [("max_fuse", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("hip_stream", ctypes.c_void_p)]


class QsBatchResult(ctypes.Structure):
    _fields_ = [("jobs", ctypes.c_int64), ("resident_jobs", ctypes.c_int64),
                ("gate_blocks", ctypes.c_int64), ("host_seconds", ctypes.c_double),
                ("plan_seconds", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("max_fuse_used", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("tune_ms", ctypes.c_double)]


def load():
    """Load libqs.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libqs.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, u64, i64, dbl = (ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_int64, ctypes.c_double)
    st = ctypes.c_int
    sig = {
        "qs_create_state": [i32, vp, ctypes.c_size_t, vp, vp],
        "qs_destroy_state": [vp],
        "qs_reset_state": [vp],
        "qs_state_device_ptr": [vp, vp],
        "qs_state_qubits": [vp, vp],
        "qs_flush": [vp],
        "qs_copy_state_to_host": [vp, vp, ctypes.c_size_t],
        "qs_load_state_from_host": [vp, vp, ctypes.c_size_t],
        "qs_copy_state": [vp, vp],
        "qs_apply_fused_gate": [vp, i32, vp, vp],
        "qs_apply_channel": [vp, i32, vp, i32, vp, u64, u32, u32, i32, vp, vp],
        "qs_norm": [vp, vp],
        "qs_expectation_z": [vp, vp],
        "qs_expectation": [vp, i32, vp, vp, vp],
        "qs_sample_measurements": [vp, u64, u32, i32, vp, vp, vp],
        "qs_sample_measurements_noalloc": [vp, u64, u32, i32, vp, vp, vp],
        "qs_run_trajectories": [vp, vp, vp, vp],
        "qs_run_trajectories_concurrent": [vp, i32, vp, vp, vp],
        "qs_kraus_bounds": [i32, i32, vp, vp, vp],
        "qs_fusion_plan": [vp, i32, vp, vp, vp, vp, vp],
        "qs_philox4x32_10": [vp, vp, vp],
        "qs_sweep_plan": [vp, i32, i32, vp, vp, vp, vp],
        "qs_run_batched": [vp, i32, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.qs_last_error_message.argtypes = []
    L.qs_last_error_message.restype = ctypes.c_char_p
    L.qs_version.argtypes = []
    L.qs_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(code: int):
    if code != QS_OK:
        msg = load().qs_last_error_message().decode(errors="replace")
        raise QsError(code, msg)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c128(m) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(m, dtype=np.complex128))


# ---------------------------------------------------------------- entry points

def qs_create_state(n_qubits: int, device_buf: Optional[int] = None, buf_bytes: int = 0,
                    hip_stream: Optional[int] = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().qs_create_state(n_qubits, device_buf, buf_bytes, hip_stream, ctypes.byref(h)))
    return h


def qs_destroy_state(s) -> None:
    _check(load().qs_destroy_state(s))


def qs_reset_state(s) -> None:
    _check(load().qs_reset_state(s))


def qs_state_device_ptr(s) -> int:
    p = ctypes.c_void_p()
    _check(load().qs_state_device_ptr(s, ctypes.byref(p)))
    return p.value


def qs_state_qubits(s) -> int:
    n = ctypes.c_int()
    _check(load().qs_state_qubits(s, ctypes.byref(n)))
    return n.value


def qs_flush(s) -> None:
    _check(load().qs_flush(s))


def qs_copy_state_to_host(s) -> np.ndarray:
    n = qs_state_qubits(s)
    out = np.empty(1 << n, dtype=np.complex64)
    _check(load().qs_copy_state_to_host(s, _p(out), out.nbytes))
    return out


def qs_load_state_from_host(s, amps) -> None:
    a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex64))
    _check(load().qs_load_state_from_host(s, _p(a), a.nbytes))


def qs_copy_state(dst, src) -> None:
    _check(load().qs_copy_state(dst, src))


def qs_apply_fused_gate(s, targets, matrix) -> None:
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    m = _c128(matrix)
    if m.shape != (1 << t.size, 1 << t.size):
        raise ValueError("matrix shape does not match the number of targets")
    _check(load().qs_apply_fused_gate(s, int(t.size), _p(t), _p(m)))


def qs_apply_channel(s, targets, kraus, seed: int, traj: int, channel_index: int,
                     mode: int = QS_KRAUS_DELAYED):
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    ks = _c128(np.stack([_c128(K) for K in kraus]))
    chosen, path = ctypes.c_int(-1), ctypes.c_int(-1)
    _check(load().qs_apply_channel(s, int(t.size), _p(t), len(kraus), _p(ks), seed, traj,
                                   channel_index, mode, ctypes.byref(chosen),
                                   ctypes.byref(path)))
    return chosen.value, path.value


def qs_norm(s) -> float:
    v = ctypes.c_double()
    _check(load().qs_norm(s, ctypes.byref(v)))
    return v.value


def qs_expectation_z(s) -> np.ndarray:
    z = np.zeros(qs_state_qubits(s), dtype=np.float64)
    _check(load().qs_expectation_z(s, _p(z)))
    return z


def qs_expectation(s, targets, observable) -> float:
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    o = _c128(observable)
    if o.shape != (1 << t.size, 1 << t.size):
        raise ValueError("observable shape does not match the number of targets")
    v = ctypes.c_double()
    _check(load().qs_expectation(s, int(t.size), _p(t), _p(o), ctypes.byref(v)))
    return v.value


def qs_sample_measurements(s, seed: int, traj: int, n_samples: int, p0to1=None, p1to0=None):
    out = np.zeros(max(n_samples, 1), dtype=np.uint64)
    e0 = None if p0to1 is None else np.ascontiguousarray(p0to1, dtype=np.float64)
    e1 = None if p1to0 is None else np.ascontiguousarray(p1to0, dtype=np.float64)
    _check(load().qs_sample_measurements(s, seed, traj, n_samples, _p(e0), _p(e1), _p(out)))
    return out[:n_samples]


def qs_sample_measurements_noalloc(s, seed: int, traj: int, n_samples: int, p0to1=None,
                                   p1to0=None):
    out = np.zeros(max(n_samples, 1), dtype=np.uint64)
    e0 = None if p0to1 is None else np.ascontiguousarray(p0to1, dtype=np.float64)
    e1 = None if p1to0 is None else np.ascontiguousarray(p1to0, dtype=np.float64)
    _check(load().qs_sample_measurements_noalloc(s, seed, traj, n_samples, _p(e0), _p(e1),
                                                 _p(out)))
    return out[:n_samples]


def qs_kraus_bounds(kraus):
    ks = _c128(np.stack([_c128(K) for K in kraus]))
    k = int(ks.shape[1]).bit_length() - 1
    pbar = np.zeros(len(kraus), dtype=np.float64)
    mix = ctypes.c_int()
    _check(load().qs_kraus_bounds(k, len(kraus), _p(ks), _p(pbar), ctypes.byref(mix)))
    return pbar, bool(mix.value)


def qs_philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _check(load().qs_philox4x32_10(_p(c), _p(k), _p(out)))
    return [int(x) for x in out]


class MarshalledCircuit:
    """A workload circuit as a qs_circuit (keeps its arrays alive)."""

    def __init__(self, circuit):
        ops = circuit.ops
        self.n = circuit.n
        self.ops = (QsOp * max(len(ops), 1))()
        chunks, pos = [], 0
        offsets = {}
        self.n_channels = 0
        for o, op in enumerate(ops):
            e = self.ops[o]
            e.kind = QS_OP_GATE if op.kind == 0 else QS_OP_CHANNEL
            e.k = op.k
            for j in range(5):
                e.targets[j] = op.qubits[j] if j < op.k else 0
            e.n_mats = len(op.mats)
            key = id(op.mats)
            if key not in offsets:
                offsets[key] = pos
                for m in op.mats:
                    m = _c128(m)
                    chunks.append(m.ravel())
                    pos += m.size
            e.mat_offset = offsets[key]
            if op.kind != 0:
                self.n_channels += 1
        self.pool = np.ascontiguousarray(np.concatenate(chunks) if chunks else
                                         np.zeros(1, np.complex128))
        self.c = QsCircuit(self.n, len(ops), self.ops, self.pool.ctypes.data_as(ctypes.c_void_p),
                           self.pool.size)


def qs_run_trajectories(s, circuit, n_traj: int, seed: int = 0, traj_offset: int = 0,
                        circuit_id: int = 0, mode: int = QS_KRAUS_DELAYED, max_fuse: int = 0,
                        tile_bits: int = 0,
                        n_samples: int = 0, p0to1=None, p1to0=None, return_state: bool = False,
                        record_choices: bool = True, time_kernels: bool = False,
                        z_expect: bool = False, graph: bool = False,
                        marshalled: Optional[MarshalledCircuit] = None) -> Dict:
    """Run trajectories traj_offset .. traj_offset + n_traj - 1 (qs_run_trajectories).
    `s` may also be a list of state handles: the range is then split over them
    and run at once (qs_run_trajectories_concurrent); the outputs are the same."""
    mc = marshalled if marshalled is not None else MarshalledCircuit(circuit)
    nch = mc.n_channels
    e0 = None if p0to1 is None else np.ascontiguousarray(p0to1, dtype=np.float64)
    e1 = None if p1to0 is None else np.ascontiguousarray(p1to0, dtype=np.float64)
    flags = (QS_TRAJ_RETURN_STATE if return_state else 0) | \
        (QS_TRAJ_TIME_KERNELS if time_kernels else 0) | (QS_TRAJ_GRAPH if graph else 0)
    params = QsTrajParams(n_traj, traj_offset, seed, circuit_id, mode, max_fuse, tile_bits,
                          n_samples, _p(e0), _p(e1), flags)
    bits = np.zeros(max(n_traj * n_samples, 1), dtype=np.uint64)
    choices = np.zeros(max(n_traj * nch, 1), dtype=np.int8) if record_choices else None
    paths = np.zeros(max(n_traj * nch, 1), dtype=np.int8) if record_choices else None
    nslow = np.zeros(max(n_traj, 1), dtype=np.int32)
    state = np.zeros(1 << mc.n, dtype=np.complex64) if return_state else None
    res = QsTrajResult()
    res.bitstrings, res.kraus_choices, res.kraus_paths = _p(bits), _p(choices), _p(paths)
    res.n_slow, res.final_state = _p(nslow), _p(state)
    zs = np.zeros((max(n_traj, 1), mc.n), dtype=np.float64) if z_expect else None
    res.z_expect = _p(zs)
    if isinstance(s, (list, tuple)):
        # several states at once (qs_run_trajectories_concurrent)
        hs = (ctypes.c_void_p * len(s))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                          for h in s])
        _check(load().qs_run_trajectories_concurrent(hs, len(s), ctypes.byref(mc.c),
                                                     ctypes.byref(params), ctypes.byref(res)))
    else:
        _check(load().qs_run_trajectories(s, ctypes.byref(mc.c), ctypes.byref(params),
                                          ctypes.byref(res)))
    out = {
        "samples": bits[:n_traj * n_samples].reshape(n_traj, n_samples),
        "n_slow": nslow[:n_traj],
        "state": state,
        "sweeps": res.sweeps,
        "gate_sweeps": res.gate_sweeps,
        "host_seconds": res.host_seconds,
        "gate_kernel_ms": res.gate_kernel_ms,
        "gate_kernel_launches": res.gate_kernel_launches,
        "gate_k_launches": [int(x) for x in res.gate_k_launches],
        "zero_start_sweeps": res.zero_start_sweeps,
        "max_fuse_used": res.max_fuse_used,
        "tile_bits_used": res.tile_bits_used,
        "tune_ms": res.tune_ms,
        "graph_replays": res.graph_replays,
    }
    if z_expect:
        out["z_expect"] = zs[:n_traj]
    if record_choices:
        out["choices"] = choices[:n_traj * nch].reshape(n_traj, nch)
        out["paths"] = paths[:n_traj * nch].reshape(n_traj, nch)
    return out


def _sample_buffer(n: int) -> Tuple[np.ndarray, object]:
    """A uint64 host array for n samples: pinned (page-locked) memory when a
    GPU is present, so that the library can transfer large sample sets into
    it directly, else ordinary memory.  Returns the array and its owner."""
    try:
        import torch

        if torch.cuda.is_available():
            t = torch.empty(max(n, 1), dtype=torch.int64, pin_memory=True)
            return t.numpy().view(np.uint64), t
    except (ImportError, RuntimeError):
        pass
    a = np.zeros(max(n, 1), dtype=np.uint64)
    return a, a


class PreparedBatch:
    """Workloads marshalled once for repeated qs_run_batched calls.  Each
    workload carries circuit, n_traj, seed, circuit_id, n_samples, e0, e1 and
    optionally traj_offset.  Sample buffers are pinned host memory when a GPU
    is present."""

    def __init__(self, workloads, record_choices: bool = True):
        self.keep = []
        self.items = (QsBatchItem * max(len(workloads), 1))()
        self.outs = []
        self.n = len(workloads)
        for i, w in enumerate(workloads):
            mc = MarshalledCircuit(w.circuit)
            e0 = None if w.e0 is None else np.ascontiguousarray(w.e0, dtype=np.float64)
            e1 = None if w.e1 is None else np.ascontiguousarray(w.e1, dtype=np.float64)
            bits, owner = _sample_buffer(w.n_traj * w.n_samples)
            self.keep.append(owner)
            ch = np.zeros(max(w.n_traj * mc.n_channels, 1), dtype=np.int8) if record_choices else None
            self.keep += [mc, e0, e1, bits, ch]
            it = self.items[i]
            it.circuit = ctypes.cast(ctypes.pointer(mc.c), ctypes.c_void_p)
            it.n_traj = w.n_traj
            it.traj_offset = getattr(w, "traj_offset", 0)
            it.seed = w.seed
            it.circuit_id = w.circuit_id
            it.n_samples = w.n_samples
            it.p0to1, it.p1to0 = _p(e0), _p(e1)
            it.bitstrings = _p(bits)
            it.kraus_choices = _p(ch)
            self.outs.append((bits, ch, mc.n_channels, w.n_traj, w.n_samples))


def qs_run_batched(workloads, max_fuse: int = 0, hip_stream: Optional[int] = None,
                   time_kernels: bool = False, record_choices: bool = True, copy: bool = True):
    """Run workloads (or a PreparedBatch) in one persistent launch; returns
    per-workload {"samples", "choices"} and launch statistics.  With
    copy=False the arrays are views of a PreparedBatch's own buffers, valid
    until its next call."""
    pb = workloads if isinstance(workloads, PreparedBatch) else PreparedBatch(workloads,
                                                                              record_choices)
    params = QsBatchParams(max_fuse, QS_TRAJ_TIME_KERNELS if time_kernels else 0, hip_stream)
    res = QsBatchResult()
    _check(load().qs_run_batched(pb.items, pb.n, ctypes.byref(params), ctypes.byref(res)))
    results = []
    own = (lambda a: a.copy()) if copy else (lambda a: a)
    for bits, ch, nch, n_traj, n_samples in pb.outs:
        d = {"samples": own(bits[:n_traj * n_samples].reshape(n_traj, n_samples))}
        if ch is not None:
            d["choices"] = own(ch[:n_traj * nch].reshape(n_traj, nch))
        results.append(d)
    stats = {"jobs": res.jobs, "resident_jobs": res.resident_jobs, "gate_blocks": res.gate_blocks,
             "host_seconds": res.host_seconds, "plan_seconds": res.plan_seconds,
             "kernel_ms": res.kernel_ms, "max_fuse_used": res.max_fuse_used,
             "tune_ms": res.tune_ms}
    return results, stats


def qs_fusion_plan(circuit, max_fuse: int):
    mc = MarshalledCircuit(circuit)
    n_ops = len(circuit.ops)
    nb = ctypes.c_int32()
    bk = np.zeros(max(n_ops, 1), dtype=np.int32)
    bt = np.zeros(5 * max(n_ops, 1), dtype=np.int32)
    bm = np.zeros(max(n_ops, 1) * 2048, dtype=np.float64)
    ob = np.zeros(max(n_ops, 1), dtype=np.int32)
    _check(load().qs_fusion_plan(ctypes.byref(mc.c), max_fuse, ctypes.byref(nb), _p(bk), _p(bt),
                                 _p(bm), _p(ob)))
    blocks = []
    for b in range(nb.value):
        k = int(bk[b])
        D = 1 << k
        m = bm[b * 2048:b * 2048 + 2 * D * D].view(np.complex128).reshape(D, D).copy()
        blocks.append((tuple(int(x) for x in bt[5 * b:5 * b + k]), m))
    return blocks, ob[:n_ops].copy()


def qs_sweep_plan(circuit, max_fuse: int, tile_bits: int = 0):
    mc = MarshalledCircuit(circuit)
    n_ops = max(len(circuit.ops), 1)
    ns = ctypes.c_int32()
    order = np.zeros(n_ops, dtype=np.int32)
    sw_of = np.zeros(n_ops, dtype=np.int32)
    bits = np.zeros(n_ops, dtype=np.uint64)
    _check(load().qs_sweep_plan(ctypes.byref(mc.c), max_fuse, tile_bits, ctypes.byref(ns),
                                _p(order), _p(sw_of), _p(bits)))
    n_blocks = len(qs_fusion_plan(circuit, max_fuse)[0])
    return ns.value, order[:n_blocks].copy(), sw_of[:n_blocks].copy(), bits[:ns.value].copy()


def qs_last_error_message() -> str:
    return load().qs_last_error_message().decode(errors="replace")


def qs_version() -> str:
    return load().qs_version().decode()


class State:
    """Owning wrapper around a qs_state handle."""

    def __init__(self, n_qubits: int, device_buf: Optional[int] = None, buf_bytes: int = 0,
                 hip_stream: Optional[int] = None):
        self.n = n_qubits
        self.h = qs_create_state(n_qubits, device_buf, buf_bytes, hip_stream)

    def close(self):
        if self.h is not None and self.h.value:
            qs_destroy_state(self.h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
