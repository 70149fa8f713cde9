"""Pins for the oracle's counter-based generator (Philox4x32-10, U53)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        assert orc.philox4x32_10(r[0:4], r[4:6]) == r[6:10]


def test_philox_matches_rocrand(orc, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "probe"
    subprocess.run([hipcc, "-O1", "-I/opt/rocm/include", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    cases[0] = 0
    cases[1, :4] = [5, 3, 0, 1]
    inp = "\n".join(" ".join(f"{int(v):08x}" for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    got = [[int(x, 16) for x in line.split()] for line in out.stdout.strip().splitlines()]
    assert len(got) == len(cases)
    for row, lib_words in zip(cases, got):
        assert orc.philox4x32_10([int(v) for v in row[:4]], [int(v) for v in row[4:]]) == lib_words


def test_u53_range_and_exactness(orc):
    assert orc.u53(0, 0) == 0.0
    top = orc.u53(0xFFFFFFFF, 0xFFFFFFFF)
    assert top < 1.0 and top == 1.0 - 2.0 ** -53
    # only the top 53 bits of (w1:w0) matter
    assert orc.u53(0x7FF, 0) == 0.0
    assert orc.u53(0x800, 0) == 2.0 ** -53
    assert orc.u53(0, 0x80000000) == 0.5


def test_draw_uses_counter_layout(orc):
    seed = (0x12345678 << 32) | 0x9ABCDEF0
    w = orc.philox4x32_10([11, 22, 33, 2], [0x9ABCDEF0, 0x12345678])
    assert orc.draw(seed, 11, 22, 33, 2) == orc.u53(w[0], w[1])


def test_draws_look_uniform(orc):
    xs = np.array([orc.draw(0, i, 3, 0, 0) for i in range(20000)])
    assert np.all((xs >= 0) & (xs < 1))
    hist, _ = np.histogram(xs, bins=20, range=(0, 1))
    chi2 = np.sum((hist - 1000.0) ** 2 / 1000.0)
    assert chi2 < 60.0  # 19 dof; p ~ 1e-6
