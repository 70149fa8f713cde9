"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package builds circuits and noise channels only: gate matrices, Kraus
lists, qubit layouts and the random choices that define a workload.  It holds
none of the simulation arithmetic (no gate application, no probabilities, no
Kraus bounds, no fusion, no sampling), so that the oracle and the HIP path stay
independent of each other while reading identical inputs.
"""

from .circuits import (  # noqa: F401
    GATE,
    CHANNEL,
    Op,
    Circuit,
    SQRT_X,
    SQRT_Y,
    SQRT_W,
    CZ,
    PAULI_I,
    PAULI_X,
    PAULI_Y,
    PAULI_Z,
    depolarize,
    depolarize2,
    amplitude_damp,
    phase_damp,
    bit_flip,
    decay_dephase,
    fsim,
    SQRT_ISWAP,
    z_phase,
    u_zz,
    approx_noise_grid_circuit,
    chain_circuit,
    grid_circuit,
    generic_grid_circuit,
    grid_coupler_patterns,
    random_unitary,
    random_matrix,
    random_gate_circuit,
    random_noisy_circuit,
    readout_arrays,
)
from .configs import (  # noqa: F401
    chain12_workload,
    grid28_workload,
    grid24_workload,
    noisy_grid_workload,
    batched_workload,
    serving_requests,
    TrajectoryWorkload,
)
