"""Write the full-size oracle fixtures of this directory (CPU only; run by hand).

    python tests/golden/make_golden.py sliced   # 30-qubit state vector, ~10 min, 16 GiB
    python tests/golden/make_golden.py large    # 53-qubit (slice, group) pairs, minutes each

Every stored amplitude comes from `oracle/` (complex128): the state-vector simulator for
the whole 1024-slice sum of the 5x6-grid, 14-cycle workload (the full slice set of a
sliced network is the exact amplitude <s|U|0^n>, Appendix B.2), and the pairwise
tensordot contractor for single (slice, group) pairs of the 53-qubit, 20-cycle share
(Appendix A groups, Appendix B.2 slices), on the circuit with per-gate angles jittered
around pi/2: at pi/2 exactly fSim maps basis states to basis states, and most slices that
fix 98 bonds are exact zeros, computed by any contraction order as rounding noise.  Each
pair is contracted along two orders, which must agree to rounding.

Inputs: circuits, targets and slice subsets come from `synth/` (seeded generators).  For
the 53-qubit share the sliced bonds and the slice ids are those of the package's seeded
plan of that workload - which bonds are cut is an input of the method, given to the
contraction under test in the same form - and the oracle builds its own network and its
own contraction path for them.  No value computed by the library's kernels enters a file.
"""

from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import contract, network, statevector  # noqa: E402

SLICED_FILE = os.path.join(HERE, "sliced_5x6_m14_full_sum.txt")
LARGE_FILE = os.path.join(HERE, "large_53q_m20_slice_group.txt")
# (position in the 256-slice subset, group index) pairs of the 53-qubit share: two spread
# pairs, and group 0 of the first four positions (one whole launch sequence of four slices)
LARGE_PAIRS = [(0, 0), (137, 9001), (1, 0), (2, 0), (3, 0)]
LARGE_PATH_SEED = 5101


def _write_amps(f, amps) -> None:
    for a in np.asarray(amps, dtype=np.complex128).ravel():
        f.write(f"{a.real:.17e} {a.imag:.17e}\n")


def make_sliced() -> None:
    cfg = synth.config("sliced")
    circ = synth.circuit_from_config(cfg)
    n = circ["n_qubits"]
    open_q = cfg["open_qubits"]
    closed = synth.group_targets(n, open_q, cfg["groups"]["L"], cfg["groups"]["seed"])
    t0 = time.time()
    psi = statevector.simulate(circ, backend="c")
    norm = float(np.vdot(psi, psi).real)
    amps = statevector.sparse_from_state(psi, n, open_q, closed)
    del psi
    dt = time.time() - t0
    with open(SLICED_FILE, "w") as f:
        f.write("# oracle amplitudes of the 5x6-grid, 14-cycle circuit (seed %d), all 1024 slices\n"
                % cfg["circuit"]["seed"])
        f.write("# = the exact amplitudes: oracle.statevector.simulate(backend='c'), complex128,\n")
        f.write("# norm of the whole state %.15f (%.0f s)\n" % (norm, dt))
        f.write("# group closed bits 0x%x (synth.group_targets, seed %d), open qubits %s\n"
                % (int(closed[0]), cfg["groups"]["seed"], " ".join(map(str, open_q))))
        f.write("# one line per open configuration mu (first open qubit = top bit): re im\n")
        _write_amps(f, amps[0])
    print(f"wrote {SLICED_FILE} ({dt:.0f} s, norm {norm:.15f})", flush=True)


def _pair(circ, w, bonds, sigma, cb, path_seed):
    n = circ["n_qubits"]
    closed = [q for q in range(n) if q not in set(w.open_qubits)]
    net = network.build_network(circ, {q: (cb >> (n - 1 - q)) & 1 for q in closed})
    fixed = {net.bond_label[tuple(b)]: (sigma >> bi) & 1 for bi, b in enumerate(bonds)}
    _, labels = net.sliced(fixed)
    path = contract.random_greedy_path(labels, path_seed)
    amps = contract.sparse_amplitudes(circ, w.open_qubits, [cb], sliced_bonds=bonds,
                                      slice_ids=[sigma], path=path)
    return amps[0], contract.peak_size(labels, path)


def make_large() -> None:
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("large")
    jit = synth.config("large")["parity_jitter"]
    # the same circuit with one angle per gate near pi/2 (at pi/2 exactly most slices of this
    # slicing are exact zeros, which any contraction order returns as rounding noise)
    circ = synth.with_theta_jitter(w.circuit, jit["theta_jitter"], jit["jitter_seed"])
    bonds = w.sliced_bonds
    lines = []
    for pos, grp in LARGE_PAIRS:
        sigma = int(w.slice_ids[pos])
        cb = int(w.closed_bits[grp])
        t0 = time.time()
        amps, peak = _pair(circ, w, bonds, sigma, cb, LARGE_PATH_SEED)
        dt = time.time() - t0
        # conditioning: a second contraction order must agree to rounding
        other, _ = _pair(circ, w, bonds, sigma, cb, LARGE_PATH_SEED + 1)
        cond = float(np.linalg.norm(amps - other) / np.linalg.norm(amps))
        print(f"pair (slice {pos}, group {grp}): peak 2^{int(np.log2(peak))}, {dt:.0f} s, "
              f"second path differs by {cond:.1e}", flush=True)
        if not cond < 1e-11:
            raise RuntimeError("the pair's amplitudes depend on the contraction order")
        lines.append((pos, grp, sigma, cb, int(np.log2(peak)), dt, cond, amps))
    with open(LARGE_FILE, "w") as f:
        f.write("# oracle amplitudes of single (slice, group) pairs of the 53-qubit, 20-cycle share\n")
        f.write("# (6x9 grid minus site (0,4), circuit seed %d; 2^14 groups x open qubits %s;\n"
                % (synth.config("large")["circuit"]["seed"], " ".join(map(str, w.open_qubits))))
        f.write("# 256-slice subset of %d sliced bonds), with the fSim angles jittered: theta_jitter "
                "%g, jitter_seed %d.\n" % (len(bonds), jit["theta_jitter"], jit["jitter_seed"]))
        f.write("# oracle.contract.sparse_amplitudes along oracle.contract.random_greedy_path(seed %d),\n"
                % LARGE_PATH_SEED)
        f.write("# complex128; 'path_diff' = relative difference from the order of seed %d.\n"
                % (LARGE_PATH_SEED + 1))
        f.write("# sliced bonds (q,j) in slice-bit order: %s\n"
                % " ".join(f"{q},{j}" for q, j in bonds))
        for pos, grp, sigma, cb, pk, dt, cond, amps in lines:
            f.write(f"pair {pos} {grp} {sigma:x} {cb:x} peak_log2 {pk} seconds {dt:.0f} "
                    f"path_diff {cond:.1e}\n")
            _write_amps(f, amps)
    print(f"wrote {LARGE_FILE}", flush=True)


if __name__ == "__main__":
    what = sys.argv[1:] or ["sliced", "large"]
    for w in what:
        {"sliced": make_sliced, "large": make_large}[w]()
