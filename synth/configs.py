"""The seeded workloads (sizes, seeds and knobs), one dict per configuration.

small        3x4 grid, 8 cycles, unsliced: 64 amplitudes (n_open = 0) and a sample mode
             with all 12 qubits open and 1000 samples.
sliced       5x6 grid, 14 cycles, 10 sliced bonds (1024 slices), largest intermediate
             2**26, one group of 12 open qubits (4096 amplitudes).
precision    the small and sliced networks in the split-precision forms.
serving      a Poisson request stream of circuits of 20..36 qubits and 10..16 cycles.
large        6x9 grid minus site (0,4) (53 qubits), 20 cycles, largest intermediate
             2**30, 2**14 groups x 6 open qubits (2**20 amplitudes), a fixed subset of
             256 slices.
"""

from __future__ import annotations

import copy

CONFIGS = {
    "small": {
        "name": "small",
        "circuit": {"rows": 3, "cols": 4, "cycles": 8, "seed": 1001},
        "amplitudes": {"count": 64, "seed": 1002},
        "samples": {"count": 1000, "seed": 1003},
        "sliced_labels": 0,
        "max_log2_size": 26,
        "path_seed": 1004,
    },
    "sliced": {
        "name": "sliced",
        "circuit": {"rows": 5, "cols": 6, "cycles": 14, "seed": 2001},
        "open_qubits": list(range(18, 30)),
        "groups": {"L": 1, "seed": 2002},
        "sliced_labels": 10,
        "max_log2_size": 26,
        "oracle_slices": {"count": 8, "seed": 2003},
        "samples": {"count": 1000, "seed": 2004},
        "path_seed": 2005,
        "plan_trials": 64,
        "reuse_batch": 64,        # head-reuse plan: steps above global labels once per 64
        "holes": 2,               # perturbed-network mode: drilled two-qubit gates (K = 4)
        # fidelity study of the approximations (holes, companion-edge cuts): the same circuit
        # with per-gate angles theta ~ pi/2 +- 0.1 (at pi/2 exactly a cut drops nothing)
        "fidelity_jitter": {"theta_jitter": 0.1, "jitter_seed": 3003},
    },
    "precision": {
        "name": "precision",
        "networks": ["small", "sliced"],
        "forms": ["fp16x3", "bf16x3", "fp16x3_3m", "bf16x3_3m"],
        "samples": {"count": 1024, "seed": 3001},
    },
    "serving": {
        "name": "serving",
        "rate_per_s": 20.0,
        "requests": 400,
        "warmup": 20,
        "seed": 4001,
        "qubits": [20, 36],
        "cycles": [10, 16],
    },
    "large": {
        "name": "large",
        "circuit": {"rows": 6, "cols": 9, "cycles": 20, "seed": 5001, "removed": [[0, 4]]},
        "open_qubits": [11, 19, 28, 29, 37, 44],
        "groups": {"L": 1 << 14, "seed": 5002},
        "max_log2_size": 30,
        "slice_subset": {"count": 256, "seed": 5003},
        "path_seed": 5004,
        "plan_trials": 1,
        "reuse_batch": 8,         # head-reuse mode: 32 subtasks x 8 local slices
        # parity twin: the same circuit with calibrated-like angles (theta ~ pi/2 +- 0.02 per
        # gate).  At pi/2 exactly fSim maps basis states to basis states and a slice that
        # fixes 98 bonds is mostly an exact zero (computed as rounding noise on any path).
        "parity_jitter": {"theta_jitter": 0.02, "jitter_seed": 5005},
    },
}


def config(name: str) -> dict:
    return copy.deepcopy(CONFIGS[name])
