"""Sycamore-like random circuits on a rectangular grid (seeded, structure only).

The paper works on Google's 53-qubit circuit files (Results paragraph), which are not
available; these circuits stand in for them with the same structure: a grid of qubits,
cycles made of one single-qubit gate per qubit followed by fSim gates on one of four
coupler patterns in the order ABCDCDAB, single-qubit gates drawn from {sqrtX, sqrtY,
sqrtW} without repeating the previous gate on a qubit.

Conventions (the paper is silent on them):
  * qubit ids are row-major over the sites that are present;
  * pattern A = horizontal couplers (r,c)-(r,c+1) with c even, B = horizontal with c
    odd, C = vertical (r,c)-(r+1,c) with r even, D = vertical with r odd; couplers that
    touch a removed site are dropped;
  * a coupler is stored as (qa, qb) with qa < qb;
  * cycle t = single-qubit layer, then the fSim layer of pattern sequence[t % len];
  * the single-qubit draw is cycle-major, then qubit id, from numpy PCG64(seed):
    cycle 0 picks uniformly among the three names, later cycles uniformly among the two
    names that differ from the qubit's previous gate.
"""

from __future__ import annotations

import math

import numpy as np

ONEQ_NAMES = ("sqrt_x", "sqrt_y", "sqrt_w")


def grid_sites(rows: int, cols: int, removed=()) -> list[tuple[int, int]]:
    """Present sites in row-major order; the list index is the qubit id."""
    gone = {tuple(s) for s in removed}
    return [(r, c) for r in range(rows) for c in range(cols) if (r, c) not in gone]


def pattern_couplers(sites, pattern: str) -> list[tuple[int, int]]:
    """Couplers of one pattern (a matching), sorted by (qa, qb)."""
    index = {s: i for i, s in enumerate(sites)}
    out = []
    for (r, c), qa in index.items():
        if pattern in "AB":
            if (c % 2 == 0) != (pattern == "A"):
                continue
            nb = (r, c + 1)
        elif pattern in "CD":
            if (r % 2 == 0) != (pattern == "C"):
                continue
            nb = (r + 1, c)
        else:
            raise ValueError(f"unknown coupler pattern {pattern!r}")
        qb = index.get(nb)
        if qb is not None:
            out.append((min(qa, qb), max(qa, qb)))
    return sorted(out)


def make_circuit(rows: int, cols: int, cycles: int, seed: int, removed=(),
                 theta: float = math.pi / 2, phi: float = math.pi / 6,
                 sequence: str = "ABCDCDAB", theta_jitter: float = 0.0,
                 jitter_seed: int | None = None) -> dict:
    """A seeded Sycamore-like circuit description (JSON-serialisable).

    theta_jitter > 0 gives every two-qubit gate its own angle theta + theta_jitter * z,
    z standard normal from PCG64(jitter_seed) in circuit order (cycle by cycle, coupler
    order), listed as circuit["fsim"]["thetas"]; the single-qubit draw is unchanged.  (The
    paper's gates have calibrated angles near, not at, pi/2; at pi/2 exactly fSim maps basis
    states to basis states, which makes heavily sliced networks mostly exact zeros.)"""
    sites = grid_sites(rows, cols, removed)
    n = len(sites)
    rng = np.random.Generator(np.random.PCG64(seed))
    prev = [None] * n
    layers = []
    for t in range(cycles):
        names = []
        for q in range(n):
            if prev[q] is None:
                k = int(rng.integers(0, 3))
                name = ONEQ_NAMES[k]
            else:
                others = [g for g in ONEQ_NAMES if g != prev[q]]
                name = others[int(rng.integers(0, 2))]
            prev[q] = name
            names.append(name)
        pat = sequence[t % len(sequence)]
        layers.append({"oneq": names, "pattern": pat,
                       "couplers": [list(c) for c in pattern_couplers(sites, pat)]})
    circ = {
        "kind": "sycamore_like_grid",
        "rows": rows, "cols": cols, "removed": [list(s) for s in removed],
        "n_qubits": n, "sites": [list(s) for s in sites],
        "cycles": cycles, "seed": seed, "sequence": sequence,
        "fsim": {"theta": float(theta), "phi": float(phi)},
        "layers": layers,
    }
    if theta_jitter > 0:
        circ = with_theta_jitter(circ, theta_jitter, seed if jitter_seed is None else jitter_seed)
    return circ


def with_theta_jitter(circuit: dict, theta_jitter: float, jitter_seed: int) -> dict:
    """Copy of a circuit whose two-qubit gates each get the angle theta + theta_jitter * z,
    z standard normal from PCG64(jitter_seed), in circuit order (cycle by cycle, coupler
    order), listed as circuit["fsim"]["thetas"]."""
    n2 = sum(len(l["couplers"]) for l in circuit["layers"])
    rng = np.random.Generator(np.random.PCG64(jitter_seed))
    theta = circuit["fsim"]["theta"]
    out = dict(circuit)
    out["fsim"] = dict(circuit["fsim"], theta_jitter=float(theta_jitter),
                       thetas=[float(theta + theta_jitter * z) for z in rng.standard_normal(n2)])
    return out


def circuit_from_config(cfg: dict) -> dict:
    c = cfg["circuit"]
    return make_circuit(c["rows"], c["cols"], c["cycles"], c["seed"],
                        removed=c.get("removed", ()),
                        theta=c.get("theta", math.pi / 2), phi=c.get("phi", math.pi / 6),
                        sequence=c.get("sequence", "ABCDCDAB"),
                        theta_jitter=c.get("theta_jitter", 0.0), jitter_seed=c.get("jitter_seed"))
