"""Parity at the benchmark's own sizes and launch shapes, through the C ABI.

* 24 qubits, the benchmark's launch configuration (Section 3.1 Algorithm 1,
  Section 3.5 Algorithm 2): the grid workload cut to its first two cycles,
  with amplitude damping raised to 0.05 so that several channels per
  trajectory need inner products, run with qs_run_trajectories_concurrent on
  two states and streams, fused blocks of at most 4 qubits in 13-bit tile
  sweeps (2048 tiles over 512 resident workgroups: every workgroup loops over
  several tiles), 200 samples per trajectory (the sampling prefix carries
  across two 8192-sum tiles); every output is compared with the oracle.
* 28 and 32 qubits (32 runs the 64-bit index kernels), with closed forms in
  place of an oracle run: GHZ (samples follow the u < 1/2 rule, norm 1,
  <Z_q> = 0), products of pair states (sampled amplitudes, samples against
  the bit-by-bit prefix, <Z_q>), and the 28-qubit grid followed by its
  inverse.
"""

from concurrent.futures import ThreadPoolExecutor

import torch

import numpy as np
import pytest

import workloads as W
from closed_forms import ghz_circuit, mirror_circuit, pair_amplitudes, pair_prefix, pair_product
from gpu_helpers import (AMP_TOL, SAMPLE_TIE, bracket_violations, compare_choices, rel_l2,
                         true_outcomes)

pytestmark = pytest.mark.gpu


def test_grid24_bench_launch_shape_against_oracle(qs, orc):
    c = W.grid_circuit(4, 6, 2, p_dep=1e-3, gamma=0.05, seed=0)
    e0, e1 = W.readout_arrays(24, 0.02, 0.02)
    seed, ns = 0, 200
    streams = [torch.cuda.Stream() for _ in range(2)]
    states = [qs.State(24, hip_stream=s.cuda_stream) for s in streams]
    try:
        got = qs.qs_run_trajectories([st.h for st in states], c, 2, seed=seed, n_samples=ns,
                                     p0to1=e0, p1to0=e1, max_fuse=4, tile_bits=13)
        # each state holds the last trajectory of its chunk: state j, trajectory j
        finals = [qs.qs_copy_state_to_host(st.h) for st in states]
    finally:
        for st in states:
            st.close()
    m = orc.Marshalled(c)

    def oracle_traj(t):
        return orc.run_trajectory(c, t, seed=seed, n_samples=ns, e0=e0, e1=e1, return_state=True,
                                  marshalled=m)

    with ThreadPoolExecutor(2) as ex:  # the oracle's C call releases the GIL
        refs = list(ex.map(oracle_traj, [0, 1]))
    compared = 0
    for t in range(2):
        ref = refs[t]
        assert int(np.sum(ref["paths"])) >= 1  # the inner-product path is exercised
        _, tie = compare_choices(got["choices"][t], ref)
        if tie:
            continue
        compared += 1
        assert np.array_equal(got["paths"][t], ref["paths"])
        assert got["n_slow"][t] == int(np.sum(ref["paths"]))
        assert rel_l2(finals[t], ref["state"]) < AMP_TOL
        mism = np.nonzero(got["samples"][t] != ref["samples"])[0]
        assert np.all(ref["sample_margins"][mism] < SAMPLE_TIE), mism
        # at 2^24 amplitudes every index carries less mass than the tie
        # width, so also require each sample's true outcome (readout flips
        # undone from their draws) to bracket its draw in the oracle's prefix
        C = np.cumsum(np.abs(ref["state"]) ** 2)
        C /= C[-1]
        outcomes = true_outcomes(got["samples"][t], 24, seed, t, 0, orc.draw, e0)
        bad = bracket_violations(outcomes, lambda x: (C[x - 1] if x else 0.0, C[x]), seed, t, 0,
                                 orc.draw)
        assert not bad, bad
    assert compared >= 1


def _device_state(qs, n):
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    st = qs.State(n, buf.data_ptr(), buf.numel() * 8, torch.cuda.current_stream().cuda_stream)
    return buf, st


@pytest.mark.parametrize("n", [28, 32])
def test_ghz_large(qs, orc, n):
    seed, ns = 7, 300
    buf, st = _device_state(qs, n)
    try:
        got = qs.qs_run_trajectories(st.h, ghz_circuit(n), 1, seed=seed, n_samples=ns,
                                     max_fuse=4, z_expect=True)
        N = qs.qs_norm(st.h)
        torch.cuda.synchronize()
        ends = buf[[0, (1 << n) - 1]].cpu().numpy()
    finally:
        st.close()
        del buf
    assert abs(N - 1.0) < 1e-6
    assert np.allclose(ends / np.sqrt(N), [2 ** -0.5, 2 ** -0.5], atol=1e-6)
    assert np.max(np.abs(got["z_expect"][0])) < 1e-5
    all_ones = (1 << n) - 1
    for s in range(ns):
        u = orc.draw(seed, s, 0, 0, 1)
        if abs(u - 0.5) < SAMPLE_TIE:
            continue
        assert int(got["samples"][0][s]) == (0 if u < 0.5 else all_ones), s


@pytest.mark.parametrize("n", [28, 32])
def test_pair_product_large(qs, orc, n):
    c, w = pair_product(n, seed=n)
    seed, ns = 13, 400
    rng = np.random.default_rng(n)
    idx = np.unique(rng.integers(0, 1 << n, size=4096, dtype=np.int64))
    buf, st = _device_state(qs, n)
    try:
        got = qs.qs_run_trajectories(st.h, c, 1, seed=seed, n_samples=ns, max_fuse=4,
                                     z_expect=True)
        N = qs.qs_norm(st.h)
        torch.cuda.synchronize()
        amps = buf[torch.from_numpy(idx).to("cuda")].cpu().numpy().astype(np.complex128)
    finally:
        st.close()
        del buf
    ref = pair_amplitudes(w, n, idx)
    err = np.linalg.norm(amps / np.sqrt(N) - ref) / np.linalg.norm(ref)
    assert err < AMP_TOL, err
    h = n // 2
    p = [np.abs(v) ** 2 / np.sum(np.abs(v) ** 2) for v in w]
    z = got["z_expect"][0]
    for q in range(h):
        assert abs(z[q] - (p[q][0] - p[q][1] + p[q][2] - p[q][3])) < 1e-5
        assert abs(z[q + h] - (p[q][0] + p[q][1] - p[q][2] - p[q][3])) < 1e-5
    # every sample brackets its draw in the exact prefix (each index holds
    # about 2^-n of the mass, far below the tie width, so bit-exact equality
    # with the exact inverse CDF is not expected)
    bad = bracket_violations(got["samples"][0], lambda x: pair_prefix(w, n, x), seed, 0, 0,
                             orc.draw)
    assert not bad, bad


def test_grid28_mirror_returns_to_zero(qs):
    """The 28-qubit benchmark grid (depth 20, blocks of at most 4 qubits)
    followed by its inverse is the identity."""
    n = 28
    c = mirror_circuit(W.grid28_workload().circuit)
    buf, st = _device_state(qs, n)
    try:
        got = qs.qs_run_trajectories(st.h, c, 1, seed=1, n_samples=100, max_fuse=4,
                                     z_expect=True)
        N = qs.qs_norm(st.h)
        torch.cuda.synchronize()
        a0 = complex(buf[0].cpu().numpy())
    finally:
        st.close()
        del buf
    err = np.sqrt(max(0.0, 2.0 - 2.0 * a0.real / np.sqrt(N)))
    assert err < AMP_TOL, err
    assert np.all(got["samples"][0] == 0)
    assert np.min(got["z_expect"][0]) > 1.0 - 1e-5


def _read_grid28_golden():
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grid28_oracle.txt")
    idx, amp, samples, margins = [], [], [], []
    with open(path) as f:
        for line in f:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "a":
                idx.append(int(p[1]))
                amp.append(complex(float(p[2]), float(p[3])))
            elif p[0] == "s":
                samples.append(int(p[1]))
                margins.append(float(p[2]))
    return (np.array(idx, dtype=np.int64), np.array(amp), np.array(samples, dtype=np.uint64),
            np.array(margins))


def test_grid28_against_stored_oracle_state(qs, orc):
    """The 28-qubit noiseless benchmark grid (4x7, depth 20, blocks of at
    most 4 qubits, 13-bit tile sweeps) against the oracle's final state at
    1024 stored indices (tests/golden/grid28_oracle.txt, written by the
    committed script beside it from the oracle alone), and its first 1000
    samples: every GPU sample and every stored oracle sample must bracket its
    draw in the prefix of the GPU's final state."""
    idx, ref_amp, ref_samples, ref_margins = _read_grid28_golden()
    w = W.grid28_workload()
    n, ns = 28, 1000
    buf, st = _device_state(qs, n)
    try:
        got = qs.qs_run_trajectories(st.h, w.circuit, 1, seed=w.seed, n_samples=ns, max_fuse=4,
                                     tile_bits=13)
        N = qs.qs_norm(st.h)
        torch.cuda.synchronize()
        amps = buf[torch.from_numpy(idx).to("cuda")].cpu().numpy().astype(np.complex128)
        p = buf.abs().double() ** 2
        C = torch.cumsum(p, 0)
        del p
        C /= C[-1].clone()

        def prefix(x):
            return (float(C[x - 1]) if x else 0.0, float(C[x]))

        bad_gpu = bracket_violations(got["samples"][0], prefix, w.seed, 0, 0, orc.draw)
        bad_ref = bracket_violations(ref_samples, prefix, w.seed, 0, 0, orc.draw)
        del C
    finally:
        st.close()
        del buf
    err = np.linalg.norm(amps / np.sqrt(N) - ref_amp) / np.linalg.norm(ref_amp)
    assert err < AMP_TOL, err
    assert not bad_gpu, bad_gpu
    assert not bad_ref, bad_ref
    mism = np.nonzero(got["samples"][0] != ref_samples)[0]
    assert np.all(ref_margins[mism] < SAMPLE_TIE)
