"""The stored fidelity study of the approximations (Method: holes and companion-edge cuts,
F_est = 2^-K prod (1 + sin^2 theta_i) / 2; Appendix D: linear XEB), written from oracle
state vectors at 30 qubits by tests/golden/make_fidelity.py: its estimates follow from the
circuit's angles, its cut lists are the ones the library chooses, and the exact fidelity and
XEB follow the estimate."""

import numpy as np

import synth
from tests.golden_data import fidelity_table


def test_fidelity_table_follows_the_estimate():
    rows, (sigma, seed) = fidelity_table()
    cfg = synth.config("sliced")
    assert (sigma, seed) == (cfg["fidelity_jitter"]["theta_jitter"], cfg["fidelity_jitter"]["jitter_seed"])
    circ = synth.with_theta_jitter(synth.circuit_from_config(cfg), sigma, seed)
    thetas = circ["fsim"]["thetas"]
    assert len(rows) >= 4 and any(r.K == 0 and r.k > 0 for r in rows) and any(r.K > 0 and r.k == 0 for r in rows)
    for r in rows:
        assert r.K == 2 * len(r.holes) and r.k == len(r.cuts)
        f_est = 2.0 ** -r.K * np.prod([(1 + np.sin(thetas[g]) ** 2) / 2 for g, _ in r.cuts])
        assert abs(f_est - r.f_est) < 1e-6
        assert abs(r.f / r.f_est - 1) < 0.03            # exact fidelity follows the estimate
        assert abs(r.xeb - r.f) < 0.01 * max(r.f, 0.1)  # expected XEB tracks the fidelity
        assert abs(r.xeb_draws - r.xeb) < 0.05          # 2^14 draws: about 0.01 standard error
    cut_only = [r for r in rows if r.K == 0][0]
    assert cut_only.f < 1 - 0.01                        # the cuts lose a measurable share


def test_fidelity_table_cuts_are_the_library_choice():
    from paper_2111_03011_amd.workload import companion_cuts, config_workload
    rows, (sigma, seed) = fidelity_table()
    w = config_workload("sliced")
    circ = synth.with_theta_jitter(w.circuit, sigma, seed)
    for r in rows:
        if r.k:
            assert companion_cuts(dict(circ, holes=r.holes), w.sliced_bonds) == r.cuts
