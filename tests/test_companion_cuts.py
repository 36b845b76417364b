"""Companion-edge cuts (Method, low-rank case (ii); Appendix C) on the host: the package
realises a cut by slicing the pinned bond and its companion edge with one shared bit, after
folding the pinned bond's single-qubit gates into the earlier gate.  Checked here against
the oracle's own definition (the SVD rank-one approximation of each pinned slice, applied
in the state vector), by contracting the package's network slice by slice with the
oracle's pairwise contractor."""

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import metrics, statevector
from paper_2111_03011_amd.network import circuit_network
from paper_2111_03011_amd.workload import companion_cuts, companion_workload, make_workload


def _case():
    circ = synth.make_circuit(3, 4, 10, 71, theta_jitter=0.25, jitter_seed=72)
    open_q = list(range(12))
    w = make_workload(circ, open_q, np.zeros(1, np.uint64), max_log2=12, n_sliced=6, trials=4,
                      seed=74)
    return w


def _slice_sum(net, sliced, ids):
    """Sum over the given slice ids of the network's contraction (all legs open)."""
    path = ocontract.greedy_path([tuple(x for x in l if x not in sliced) for l in net.labels])
    total = 0
    for sid in ids:
        val = {x: (int(sid) >> b) & 1 for b, x in enumerate(sliced)}
        ts, ls = [], []
        for t, l in zip(net.tensors, net.labels):
            idx = tuple(val[x] if x in val else slice(None) for x in l)
            ts.append(np.asarray(t)[idx])
            ls.append(tuple(x for x in l if x not in val))
        total = total + ocontract.contract_path(ts, ls, path, net.out_label).reshape(-1)
    return total


def test_cut_selection_rules():
    w = _case()
    cuts = companion_cuts(w.circuit, w.sliced_bonds)
    assert cuts and len({g for g, _ in cuts}) == len(cuts)
    net = circuit_network(dict(w.circuit, cuts=cuts))
    assert len(net.cut_pairs) == len(cuts)
    sliced = set(w.plan.sliced_labels)
    for b, c in net.cut_pairs:
        assert b in sliced and c not in sliced
        assert c in net.bond_label.values() and b in net.bond_label.values()
    assert companion_cuts(w.circuit, w.sliced_bonds, max_cuts=1) == cuts[:1]


def test_cut_network_is_exact_and_tied_slices_equal_the_oracle_cut():
    w = _case()
    cuts = companion_cuts(w.circuit, w.sliced_bonds)
    cw = companion_workload(w, cuts)
    n = w.circuit["n_qubits"]
    assert len(cw.slice_ids) == len(w.slice_ids)
    # folding single-qubit gates elsewhere changes nothing: all slices of the pinned and
    # companion edges, bits independent, sum to the exact state
    k = len(cw.plan.sliced_labels)
    full = _slice_sum(cw.net, cw.plan.sliced_labels, range(1 << k))
    exact = statevector.simulate(w.circuit)
    assert np.allclose(full, exact, atol=1e-12)
    # the tied slices are the oracle's approximated state
    got = _slice_sum(cw.net, cw.plan.sliced_labels, cw.slice_ids)
    ref = statevector.simulate(cw.circuit)
    assert metrics.rel_error(got, ref) < 1e-12
    # ... which differs from the exact state by the dropped weight (angles jittered 0.25)
    f = abs(np.vdot(ref, exact)) ** 2 / (np.vdot(ref, ref).real * np.vdot(exact, exact).real)
    assert 0.5 < f < 0.9999
    assert cw.plan.cost.flops_per_slice <= w.plan.cost.flops_per_slice


def test_cut_network_rejects_bad_cuts():
    w = _case()
    c = w.circuit
    with pytest.raises(ValueError):
        circuit_network(dict(c, cuts=[[0, 0], [0, 1]]))        # the same gate twice
    qa, qb = c["layers"][0]["couplers"][0]
    with pytest.raises(ValueError):
        circuit_network(dict(c, cuts=[[0, qa]]))               # first gate: no bond to pin
    with pytest.raises(ValueError):
        circuit_network(dict(c, cuts=[[0, 99]]))
