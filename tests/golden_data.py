"""Readers of the stored full-size oracle values in tests/golden (written by
tests/golden/make_golden.py, which calls only the oracle and the seeded generators)."""

from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@dataclass
class SlicedSum:
    closed: int          # closed bits of the one group
    open_qubits: list
    amps: np.ndarray     # 4096 complex128, mu order (first open qubit = top bit)


@dataclass
class LargePair:
    pos: int             # position of the slice in the 256-slice subset
    group: int           # group index among the 2^14 groups
    slice_id: int
    closed: int
    amps: np.ndarray     # 64 complex128


def _path(name: str) -> str:
    p = os.path.join(GOLDEN, name)
    if not os.path.exists(p):
        import pytest
        pytest.fail(f"{p} missing: run python tests/golden/make_golden.py")
    return p


def sliced_full_sum() -> SlicedSum:
    p = _path("sliced_5x6_m14_full_sum.txt")
    closed, opn = None, None
    for line in open(p):
        if line.startswith("# group closed bits"):
            f = line.split()
            closed = int(f[4], 16)
            opn = [int(x) for x in line.split("open qubits")[1].split()]
    v = np.loadtxt(p, comments="#")
    return SlicedSum(closed, opn, v[:, 0] + 1j * v[:, 1])


def large_pairs():
    """(pairs, sliced bonds in slice-bit order, (theta_jitter, jitter_seed) of the circuit)."""
    p = _path("large_53q_m20_slice_group.txt")
    pairs, bonds, cur, jitter = [], None, None, None
    for line in open(p):
        if line.startswith("# sliced bonds"):
            bonds = [tuple(int(x) for x in b.split(",")) for b in line.split(":", 1)[1].split()]
        elif "theta_jitter" in line and line.startswith("#"):
            f = line.replace(",", " ").replace(".\n", " ").split()
            jitter = (float(f[f.index("theta_jitter") + 1]), int(f[f.index("jitter_seed") + 1].rstrip(".")))
        elif line.startswith("#"):
            continue
        elif line.startswith("pair"):
            f = line.split()
            cur = LargePair(int(f[1]), int(f[2]), int(f[3], 16), int(f[4], 16), [])
            pairs.append(cur)
        elif line.strip():
            re, im = map(float, line.split())
            cur.amps.append(complex(re, im))
    for q in pairs:
        q.amps = np.asarray(q.amps)
    return pairs, bonds, jitter


@dataclass
class FidelityRow:
    K: int               # broken edges (2 per hole)
    k: int               # companion-edge cuts
    f_est: float
    f: float
    xeb: float
    xeb_draws: float
    holes: list
    cuts: list           # [gate, pinned qubit]


def fidelity_table():
    """(rows, (theta_jitter, jitter_seed)) of tests/golden/fidelity_5x6_m14.txt."""
    p = _path("fidelity_5x6_m14.txt")
    rows, jitter = [], None
    for line in open(p):
        if line.startswith("#"):
            if "theta_jitter" in line:
                f = line.replace(",", " ").split()
                jitter = (float(f[f.index("theta_jitter") + 1]), int(f[f.index("jitter_seed") + 1]))
            continue
        f = line.split()
        holes = [] if f[6] == "-" else [int(x) for x in f[6].split(",")]
        cuts = [] if f[7] == "-" else [[int(a) for a in c.split(":")] for c in f[7:]]
        rows.append(FidelityRow(int(f[0]), int(f[1]), float(f[2]), float(f[3]), float(f[4]),
                                float(f[5]), holes, cuts))
    return rows, jitter


def sliced_cut_group():
    """(cuts, amplitudes) of tests/golden/sliced_5x6_m14_cut_group.txt: the 4096 oracle
    amplitudes of the sliced configuration's group on the jittered circuit with cuts."""
    p = _path("sliced_5x6_m14_cut_group.txt")
    cuts = None
    for line in open(p):
        if line.startswith("# and companion-edge cuts"):
            body = line.split("cuts", 1)[1].split("(")[0].split()
            cuts = [[int(a) for a in c.split(",")] for c in body]
    v = np.loadtxt(p, comments="#")
    return cuts, v[:, 0] + 1j * v[:, 1]
