"""Allocation-free sampling entry point against qs_sample_measurements, both
through the C ABI: bit-identical bitstrings on two calls in a row (the
second on a smaller state with fewer samples), and refusal of sizes beyond
its fixed buffers."""

import ctypes

import torch  # noqa: F401  (imported at collection: the first import can be slow)

import numpy as np
import pytest

import workloads as W
from gpu_helpers import random_state

pytestmark = pytest.mark.gpu


def _pair(qs, n, n_samples, seed, traj, readout):
    rng = np.random.default_rng(100 + n)
    psi = random_state(n, rng)
    e0, e1 = W.readout_arrays(n, 0.03, 0.05) if readout else (None, None)
    with qs.State(n) as st:
        qs.qs_load_state_from_host(st.h, psi)
        ref = qs.qs_sample_measurements(st.h, seed, traj, n_samples, e0, e1)
        got = qs.qs_sample_measurements_noalloc(st.h, seed, traj, n_samples, e0, e1)
    return ref, got


def test_noalloc_sampling_matches_allocating_entry_point(qs):
    # first call: 2^20 amplitudes (1024 block sums), 3000 samples with readout
    ref, got = _pair(qs, 20, 3000, seed=11, traj=4, readout=True)
    assert got.dtype == np.uint64 and got.shape == (3000,)
    assert np.array_equal(got, ref)
    # second call, smaller: the array still holds the first call's larger
    # contents, and the smaller call must read only what it wrote
    ref, got = _pair(qs, 13, 257, seed=12, traj=0, readout=False)
    assert np.array_equal(got, ref)


def test_noalloc_sampling_sizes_and_errors(qs):
    # the largest sample count and a one-qubit state
    ref, got = _pair(qs, 1, 1 << 16, seed=3, traj=1, readout=True)
    assert np.array_equal(got, ref)
    with qs.State(12) as st:
        qs.qs_load_state_from_host(st.h, random_state(12, np.random.default_rng(1)))
        assert len(qs.qs_sample_measurements_noalloc(st.h, 1, 0, 0)) == 0
        with pytest.raises(qs.QsError) as e:
            qs.qs_sample_measurements_noalloc(st.h, 1, 0, (1 << 16) + 1)
        assert e.value.code == qs.QS_ERR_INVALID_ARGUMENT and "65536" in str(e.value)
        # deferred operations must be flushed first
        # p = 1: every pick is X, Y or Z, so an operation is deferred
        qs.qs_apply_channel(st.h, [3], W.depolarize(1.0), seed=1, traj=0, channel_index=0)
        with pytest.raises(qs.QsError) as e:
            qs.qs_sample_measurements_noalloc(st.h, 1, 0, 10)
        assert e.value.code == qs.QS_ERR_INVALID_ARGUMENT and "qs_flush" in str(e.value)
        qs.qs_flush(st.h)
        ref = qs.qs_sample_measurements(st.h, 5, 2, 100)
        assert np.array_equal(qs.qs_sample_measurements_noalloc(st.h, 5, 2, 100), ref)
    with qs.State(29) as st:
        with pytest.raises(qs.QsError) as e:
            qs.qs_sample_measurements_noalloc(st.h, 1, 0, 10)
        assert e.value.code == qs.QS_ERR_INVALID_ARGUMENT and "28 qubits" in str(e.value)
    # a zero state is refused (after the sampling kernels ran on it)
    with qs.State(10) as st:
        qs.qs_load_state_from_host(st.h, np.zeros(1 << 10, dtype=np.complex64))
        with pytest.raises(qs.QsError) as e:
            qs.qs_sample_measurements_noalloc(st.h, 1, 0, 10)
        assert e.value.code == qs.QS_ERR_ZERO_NORM


def test_noalloc_sampling_raw_c_abi(qs):
    """The entry point called through ctypes directly, with raw host arrays."""
    L = qs.load()
    n, ns = 16, 500
    psi = random_state(n, np.random.default_rng(9))
    with qs.State(n) as st:
        qs.qs_load_state_from_host(st.h, psi)
        out = (ctypes.c_uint64 * ns)()
        rc = L.qs_sample_measurements_noalloc(st.h, ctypes.c_uint64(77), ctypes.c_uint32(3), ns,
                                              None, None, ctypes.cast(out, ctypes.c_void_p))
        assert rc == 0
        ref = qs.qs_sample_measurements(st.h, 77, 3, ns)
    assert np.array_equal(np.frombuffer(out, dtype=np.uint64), ref)
