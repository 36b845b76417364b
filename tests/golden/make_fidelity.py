"""Fidelity of the approximated 30-qubit network (Method: holes and companion-edge cuts;
Appendix C; Appendix D), from oracle state vectors (CPU only; run by hand, about an hour and
40 GiB of memory):

    python tests/golden/make_fidelity.py

Circuit: the 5x6-grid, 14-cycle circuit of the sliced configuration with per-gate fSim
angles jittered around pi/2 (synth config "sliced", fidelity_jitter).  For each row the
script drills K/2 holes and applies k companion-edge cuts, simulates the approximated state
psi_hat with the oracle (complex128) and compares it with the exact psi:

    F_est   = 2^-K prod_i (1 + sin^2 theta_i) / 2   over the cut gates (Method)
    F       = |<psi|psi_hat>|^2 / (<psi|psi> <psi_hat|psi_hat>)
    XEB     = 2^n sum_s p_hat(s) p(s) - 1           (expected linear XEB, Appendix D)
    XEB_smp = 2^n mean p(s) - 1 over 2^14 draws s ~ p_hat (seeded)

with p, p_hat the normalised probabilities.  Inputs: which gates are drilled
(paper_2111_03011_amd.workload.choose_holes) and which bonds are sliced (the
configuration's plan), hence which gates are cut (workload.companion_cuts), are inputs of
the method; every stored number is computed from oracle state vectors.  The cut state of
the row without holes is also stored for the requested group (4096 amplitudes), the GPU
check of the 30-qubit cut network."""

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
from oracle import gates, statevector  # noqa: E402

TABLE_FILE = os.path.join(HERE, "fidelity_5x6_m14.txt")
CUT_FILE = os.path.join(HERE, "sliced_5x6_m14_cut_group.txt")
N_DRAWS = 1 << 14
DRAW_SEED = 3004
BLOCK = 1 << 20


def _chunks(n):
    for a in range(0, n, BLOCK):
        yield a, min(n, a + BLOCK)


def _compare(psi, hat, n, rng):
    nn = float(np.vdot(psi, psi).real)
    nh = float(np.vdot(hat, hat).real)
    f = abs(np.vdot(psi, hat)) ** 2 / (nn * nh)
    xeb, block_p = 0.0, []
    for a, b in _chunks(len(psi)):
        ph = np.abs(hat[a:b]) ** 2
        xeb += float(np.dot(ph, np.abs(psi[a:b]) ** 2))
        block_p.append(ph.sum())
    xeb = 2.0 ** n * xeb / (nn * nh) - 1.0
    # draws s ~ p_hat: a block by its weight, then a position inside it
    block_p = np.asarray(block_p) / nh
    blocks = rng.choice(len(block_p), size=N_DRAWS, p=block_p / block_p.sum())
    scores = []
    for blk in np.unique(blocks):
        a, b = blk * BLOCK, min(len(psi), (blk + 1) * BLOCK)
        cdf = np.cumsum(np.abs(hat[a:b]) ** 2)
        m = int(np.sum(blocks == blk))
        pos = np.searchsorted(cdf, rng.random(m) * cdf[-1], side="right")
        pos = np.minimum(pos, b - a - 1)
        scores.append(np.abs(psi[a + pos]) ** 2 / nn)
    xeb_s = 2.0 ** n * float(np.concatenate(scores).mean()) - 1.0
    return f, xeb, xeb_s


def main() -> None:
    from paper_2111_03011_amd.workload import choose_holes, companion_cuts, config_workload
    cfg = synth.config("sliced")
    jit = cfg["fidelity_jitter"]
    w = config_workload("sliced")
    circ = synth.with_theta_jitter(w.circuit, jit["theta_jitter"], jit["jitter_seed"])
    n = circ["n_qubits"]
    thetas = gates.gate_thetas(circ)
    t0 = time.time()
    holes = {0: [],
             1: choose_holes(circ, 1, w.open_qubits, w.closed_bits, max_log2=cfg["max_log2_size"],
                             n_sliced=cfg["sliced_labels"], seed=cfg["path_seed"]),
             2: choose_holes(circ, 2, w.open_qubits, w.closed_bits, max_log2=cfg["max_log2_size"],
                             n_sliced=cfg["sliced_labels"], seed=cfg["path_seed"])}
    print(f"holes {holes} ({time.time() - t0:.0f} s)", flush=True)
    psi = statevector.simulate(circ, backend="c")
    print(f"exact state ({time.time() - t0:.0f} s)", flush=True)
    rows = []
    for n_holes, with_cuts in ((0, True), (1, False), (1, True), (2, True)):
        c = dict(circ, holes=holes[n_holes])
        cuts = companion_cuts(c, w.sliced_bonds) if with_cuts else []
        c["cuts"] = cuts
        t1 = time.time()
        hat = statevector.simulate(c, backend="c")
        K = 2 * n_holes
        f_est = 2.0 ** -K * float(np.prod([(1 + np.sin(thetas[g]) ** 2) / 2 for g, _ in cuts]))
        f, xeb, xeb_s = _compare(psi, hat, n, np.random.Generator(np.random.PCG64(DRAW_SEED)))
        rows.append((K, len(cuts), holes[n_holes], cuts, f_est, f, xeb, xeb_s, time.time() - t1))
        print(f"K {K} k {len(cuts)}: F_est {f_est:.5f} F {f:.5f} XEB {xeb:.5f} "
              f"XEB({N_DRAWS} draws) {xeb_s:.4f} ({time.time() - t1:.0f} s)", flush=True)
        if n_holes == 0:
            amps = statevector.sparse_from_state(hat, n, w.open_qubits, w.closed_bits)
            with open(CUT_FILE, "w") as fh:
                fh.write("# oracle amplitudes of the 5x6-grid, 14-cycle circuit with per-gate angles "
                         "jittered (theta_jitter %g, jitter_seed %d)\n" % (jit["theta_jitter"],
                                                                           jit["jitter_seed"]))
                fh.write("# and companion-edge cuts %s (gate, pinned qubit)\n"
                         % " ".join(f"{g},{q}" for g, q in cuts))
                fh.write("# oracle.statevector.simulate(backend='c'), complex128; the group of the "
                         "sliced configuration (closed bits 0x%x), mu order\n" % int(w.closed_bits[0]))
                for a in amps[0]:
                    fh.write(f"{a.real:.17e} {a.imag:.17e}\n")
        del hat
    with open(TABLE_FILE, "w") as fh:
        fh.write("# fidelity of the approximated 5x6-grid, 14-cycle circuit (30 qubits), angles "
                 "jittered: theta_jitter %g, jitter_seed %d\n" % (jit["theta_jitter"], jit["jitter_seed"]))
        fh.write("# written by tests/golden/make_fidelity.py from oracle state vectors; "
                 "XEB_draws over %d draws (seed %d)\n" % (N_DRAWS, DRAW_SEED))
        fh.write("# K k F_est F XEB XEB_draws holes cuts\n")
        for K, k, hl, cuts, f_est, f, xeb, xeb_s, _ in rows:
            fh.write(f"{K} {k} {f_est:.6f} {f:.6f} {xeb:.6f} {xeb_s:.6f} "
                     f"{','.join(map(str, hl)) or '-'} "
                     f"{' '.join(f'{g}:{q}' for g, q in cuts) or '-'}\n")
    print(f"wrote {TABLE_FILE} and {CUT_FILE}", flush=True)


if __name__ == "__main__":
    main()
