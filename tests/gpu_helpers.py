"""Comparison helpers for the GPU parity tests (no simulation arithmetic)."""

import numpy as np

# Amplitudes: relative L2 distance of the normalised states.
AMP_TOL = 1e-5
# Threshold ties (state-independent bound comparisons are FP64 on both sides).
FAST_TIE = 1e-12
# Ties on comparisons against inner products of a complex64 state.
SLOW_TIE = 1e-5
# Sampling ties: |u N - C(x)| / N below this counts as a tie.
SAMPLE_TIE = 1e-5


def rel_l2(gpu, ref) -> float:
    g = np.asarray(gpu, dtype=np.complex128)
    r = np.asarray(ref, dtype=np.complex128)
    g = g / np.linalg.norm(g)
    r = r / np.linalg.norm(r)
    return float(np.linalg.norm(g - r))


def random_state(n, rng):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    return v.astype(np.complex64)


def compare_choices(gpu_choices, orc_res):
    """Per-trajectory channel choices: equal up to the first threshold tie.
    Returns (compared, ties)."""
    oc = orc_res["choices"]
    mf = orc_res["margin_fast"]
    ms = orc_res["margin_slow"]
    compared = 0
    for j in range(len(oc)):
        if int(gpu_choices[j]) != int(oc[j]):
            tie = mf[j] < FAST_TIE or ms[j] < SLOW_TIE
            assert tie, (j, int(gpu_choices[j]), int(oc[j]), mf[j], ms[j])
            return compared, 1
        compared += 1
    return compared, 0


def true_outcomes(samples, n, seed, traj, circ, draw, e=None):
    """Undo symmetric readout flips (P(1|0) = P(0|1) = e[q]): qubit q of
    sample s was flipped iff its readout draw (stream 2, index s n + q) is
    below e[q], whatever the true bit, so the flips are known from the draws."""
    x = np.asarray(samples, dtype=np.uint64).copy()
    if e is None:
        return x
    for s in range(len(x)):
        for q in range(n):
            if draw(seed, s * n + q, traj, circ, 2) < e[q]:
                x[s] ^= np.uint64(1 << q)
    return x


def bracket_violations(outcomes, prefix, seed, traj, circ, draw, tol=SAMPLE_TIE):
    """Samples whose outcome x is not an inverse-CDF answer for their draw u
    within tol: the rule is C(x - 1) <= u < C(x) with C the normalised
    inclusive prefix of |psi|^2 in index order; prefix(x) returns
    (C(x - 1), C(x)).  Returns the indices of violating samples."""
    bad = []
    for s, x in enumerate(outcomes):
        u = draw(seed, s, traj, circ, 1)
        lo, hi = prefix(int(x))
        if not (lo - tol <= u < hi + tol):
            bad.append(s)
    return bad
