"""Companion-edge cuts (Method, low-rank case (ii); Appendix C) through the library: each
cut's pinned bond and companion edge are sliced with one shared bit, and the GPU sum over
those slices matches the oracle's approximated state (the SVD rank-one approximation of
each pinned gate, applied in its state vector), with and without holes, in every form."""

import numpy as np
import pytest

import synth
from oracle import metrics, statevector
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu
TOLS = {0: 1e-5, 1: 1e-5, 2: 1e-3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _contraction(w, **kw):
    from paper_2111_03011_amd.contractor import Contraction
    return Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                       slice_ids=w.slice_ids, open_qubits=w.open_qubits,
                       closed_bits=w.closed_bits, **kw)


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("holes", [(), (9, 30)])
def test_cut_network_against_oracle(holes, precision):
    from paper_2111_03011_amd.workload import companion_cuts, companion_workload, make_workload
    circ = synth.make_circuit(4, 4, 12, 81, theta_jitter=0.2, jitter_seed=82)
    if holes:
        circ["holes"] = list(holes)
    open_q = [1, 6, 11, 14]
    closed = synth.group_targets(16, open_q, 32, 83)
    w = make_workload(circ, open_q, closed, max_log2=12, n_sliced=7, trials=4, seed=84)
    cuts = companion_cuts(circ, w.sliced_bonds)
    cw = companion_workload(w, cuts)
    log(f"holes {list(holes)}, precision {precision}: {len(cuts)} cuts {cuts}, "
        f"{len(cw.slice_ids)} slices of {len(cw.plan.sliced_labels)} sliced labels")
    assert len(cuts) >= 3
    c = _contraction(cw, max_batch_slices=16, precision=precision)
    c.contract()
    got = c.amps.cpu().numpy().copy()
    c.close()
    n = circ["n_qubits"]
    ref = statevector.sparse_from_state(statevector.simulate(cw.circuit), n, open_q, closed)
    uncut = statevector.sparse_from_state(statevector.simulate(circ), n, open_q, closed)
    err = metrics.rel_error(got, ref)
    log(f"  rel err vs oracle cut state {err:.3e}; the cuts move the amplitudes by "
        f"{metrics.rel_error(ref, uncut):.3e}")
    assert err <= TOLS[precision]
    assert metrics.rel_error(ref, uncut) > 10 * TOLS[precision]


def test_cut_network_30_qubits_against_stored_oracle():
    """The 30-qubit workload (5x6 grid, 14 cycles, all 1024 slices) on its circuit with
    jittered angles and the 8 companion-edge cuts of its plan's sliced bonds, against the
    oracle's state vector of the same approximated circuit (stored group of 4096
    amplitudes, tests/golden)."""
    from paper_2111_03011_amd.workload import (companion_cuts, companion_workload,
                                               config_workload, jittered_twin)
    from tests.golden_data import fidelity_table, sliced_cut_group
    _, (sigma, seed) = fidelity_table()
    cuts_ref, ref = sliced_cut_group()
    twin = jittered_twin(config_workload("sliced"), sigma, seed)
    cuts = companion_cuts(twin.circuit, twin.sliced_bonds)
    assert cuts == cuts_ref
    cw = companion_workload(twin, cuts)
    c = _contraction(cw, max_batch_slices=64)
    c.contract()
    got = c.amps.cpu().numpy()[0]
    c.close()
    err = metrics.rel_error(got, ref)
    log(f"30-qubit cut network ({len(cuts)} cuts, {len(cw.slice_ids)} slices): rel err {err:.3e}, "
        f"planned flops per slice {cw.plan.cost.flops_per_slice:.3e} "
        f"(uncut {twin.plan.cost.flops_per_slice:.3e})")
    assert err <= 1e-5
