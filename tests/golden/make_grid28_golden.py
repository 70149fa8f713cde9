"""Writes grid28_oracle.txt: the oracle's final state of the 28-qubit
noiseless 4 x 7 grid (20 cycles, generator seed 0) at 1024 seeded indices,
and its first 1000 measurement samples (Philox seed 0, trajectory 0) with
each sample's distance to the nearest prefix boundary.

Calls only the oracle and the input builders.  About an hour on one core
and ~9 GiB of memory (the complex128 state twice).  Run from the repository
root: python tests/golden/make_grid28_golden.py
"""

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid28_oracle.txt")
N_AMPS = 1024
N_SAMPLES = 1000
INDEX_SEED = 2028


def sampled_indices(n):
    """The 1024 amplitude indices the file records (distinct, ascending)."""
    rng = np.random.default_rng(INDEX_SEED)
    return np.sort(rng.choice(1 << n, size=N_AMPS, replace=False))


def main():
    w = W.grid28_workload()
    c = w.circuit
    t0 = time.time()
    ref = oracle.run_trajectory(c, 0, seed=w.seed, n_samples=N_SAMPLES, return_state=True)
    dt = time.time() - t0
    psi = ref["state"]
    idx = sampled_indices(c.n)
    with open(OUT, "w") as f:
        f.write("# Oracle (complex128, single thread) on the 28-qubit 4x7 grid, 20 cycles,\n")
        f.write("# noiseless, circuit generator seed 0: written by make_grid28_golden.py\n")
        f.write(f"# in {dt:.0f} s.  norm^2 = {np.vdot(psi, psi).real:.17g}\n")
        f.write(f"# amplitudes: {N_AMPS} indices from numpy default_rng({INDEX_SEED})\n")
        f.write("# lines 'a index re im', then 's sample margin' (Philox seed 0, trajectory 0)\n")
        for i in idx:
            f.write(f"a {int(i)} {psi[i].real:.17g} {psi[i].imag:.17g}\n")
        for s, m in zip(ref["samples"], ref["sample_margins"]):
            f.write(f"s {int(s)} {float(m):.17g}\n")
    print(f"wrote {OUT} ({dt:.0f} s)")


if __name__ == "__main__":
    main()
