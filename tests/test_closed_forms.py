"""The closed forms the large-state GPU tests rely on, checked against the
oracle on small states (CPU only): amplitudes, the bit-by-bit inverse CDF
with readout flips, and <Z_q> of pair products; GHZ; mirror circuits."""

import math

import numpy as np
import pytest

import workloads as W
from closed_forms import (ghz_circuit, mirror_circuit, pair_amplitudes, pair_inverse_cdf,
                          pair_prefix, pair_product)


@pytest.mark.parametrize("n", [6, 10])
def test_pair_product_against_oracle(orc, n):
    c, w = pair_product(n, seed=n)
    psi = orc.simulate(c)
    ref = pair_amplitudes(w, n, np.arange(1 << n))
    assert np.max(np.abs(psi - ref)) < 1e-13
    seed, traj, ns = 13, 5, 400
    samples, _ = orc.sample(psi, seed, traj, 0, ns)
    for s in range(ns):
        x, margin = pair_inverse_cdf(w, n, orc.draw(seed, s, traj, 0, 1))
        assert x == int(samples[s]) or margin < 1e-12
    h = n // 2
    z = orc.z_expectations(psi)
    for q in range(h):
        p = np.abs(w[q]) ** 2
        assert abs(z[q] - (p[0] - p[1] + p[2] - p[3])) < 1e-12
        assert abs(z[q + h] - (p[0] + p[1] - p[2] - p[3])) < 1e-12


@pytest.mark.parametrize("n", [4, 8])
def test_pair_prefix_against_oracle(orc, n):
    """The bit-by-bit prefix of the pair-product state equals the running sum
    of the oracle's |psi_x|^2 at every index."""
    c, w = pair_product(n, seed=3 * n)
    psi = orc.simulate(c)
    C = np.cumsum(np.abs(psi) ** 2)
    for x in range(1 << n):
        lo, hi = pair_prefix(w, n, x)
        assert abs(hi - C[x]) < 1e-13
        assert abs(lo - (C[x - 1] if x else 0.0)) < 1e-13


def test_pair_inverse_cdf_margin_is_a_boundary_distance():
    """Draws placed on either side of an exact boundary of the prefix land on
    consecutive indices, and the reported margin is the distance to it."""
    _, w = pair_product(4, seed=1)
    p = np.abs(pair_amplitudes(w, 4, np.arange(16))) ** 2
    C = np.cumsum(p)
    for x in range(15):
        lo, m_lo = pair_inverse_cdf(w, 4, C[x] - 1e-9)
        hi, m_hi = pair_inverse_cdf(w, 4, C[x] + 1e-9)
        assert (lo, hi) == (x, x + 1)
        assert m_lo < 2e-9 and m_hi < 2e-9


@pytest.mark.parametrize("n", [2, 7])
def test_ghz_against_oracle(orc, n):
    psi = orc.simulate(ghz_circuit(n))
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = 1 / math.sqrt(2.0)
    assert np.max(np.abs(psi - ref)) < 1e-15


def test_mirror_is_identity(orc):
    psi = orc.simulate(mirror_circuit(W.grid_circuit(3, 3, 6, seed=0)))
    ref = orc.zero_state(9)
    assert np.linalg.norm(psi - ref) < 1e-13
