"""Head-tail planning with the zigzag tail (Method, zigzag paragraph; Appendix E): the head
(gates before the tail's first cycle) becomes one tensor, then the tail's leaves are absorbed
one at a time in sweeps toward the final state and back."""

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import statevector
from paper_2111_03011_amd import planner
from paper_2111_03011_amd.network import circuit_network
from paper_2111_03011_amd.workload import make_zigzag_workload


def _absorbed_tail(net, path, tail_start):
    """Cycles of the tail leaves in the order the zigzag absorbs them, and the accumulator."""
    tail = {k for k, c in enumerate(net.cycle) if c >= tail_start}
    seq = [(i, j) for i, j in path if j in tail]
    accs = {i for i, _ in seq}
    return [net.cycle[j] for _, j in seq], accs


def test_cycles_tag_every_gate_and_follow_the_circuit():
    c = synth.make_circuit(3, 4, 8, 3)
    net = circuit_network(c)
    assert len(net.cycle) == len(net.tensors)
    assert set(net.cycle) <= set(range(-1, 8))
    # a gate's tensors sit in circuit order: cycles never decrease along the leaf list, apart
    # from the trailing final-state vectors (-1)
    gates = [x for x in net.cycle if x >= 0]
    assert gates == sorted(gates)


@pytest.mark.parametrize("tail_start", [3, 5, 7])
def test_zigzag_path_contracts_the_network_exactly(tail_start):
    """The order is a complete contraction: the oracle's pairwise contractor along it
    returns the state vector's amplitudes."""
    c = synth.make_circuit(3, 4, 8, 3)
    net = circuit_network(c)
    n = net.n_qubits
    prob = planner.make_problem(net.labels, net.out_label, n, list(range(n)), [0])
    path = planner.zigzag_path(prob, net.cycle, tail_start)
    assert len(planner.validate_path(len(net.tensors), path)) == 1
    res = ocontract.contract_path(net.tensors, net.labels, path, net.out_label).reshape(-1)
    assert np.allclose(res, statevector.simulate(c), atol=1e-12)


def test_zigzag_sweeps_out_and_back():
    """Tail leaves join one accumulator (the head's tensor), in runs of non-decreasing cycle
    (toward the final state) alternating with runs of non-increasing cycle (back toward
    the head), the first run starting at the interface."""
    c = synth.make_circuit(4, 4, 14, 44)
    net = circuit_network(c)
    n = net.n_qubits
    ts = 8
    prob = planner.make_problem(net.labels, net.out_label, n, list(range(n)), [0])
    path = planner.zigzag_path(prob, net.cycle, ts)
    cycles, accs = _absorbed_tail(net, path, ts)
    assert len(accs) == 1 and min(cycles) == ts and cycles[0] == ts
    runs, d = 1, 1
    for a, b in zip(cycles, cycles[1:]):
        if d * (b - a) < 0:
            d, runs = -d, runs + 1
    assert runs >= 3          # out, back and out again
    # every run is monotone by construction of the count above; the sweep reaches the
    # final cycle before it first turns around
    first_turn = next(k for k in range(1, len(cycles)) if cycles[k] < cycles[k - 1])
    assert max(cycles[:first_turn]) == max(net.cycle)


def test_zigzag_plan_meets_the_bound_and_keeps_base_slices():
    c = synth.make_circuit(4, 4, 14, 44)
    open_q = list(range(10, 16))
    closed = synth.group_targets(16, open_q, 4, 45)
    net = circuit_network(c)
    base = planner.find_plan(net, open_q, closed, max_log2=14, n_sliced=6, trials=2, seed=44)
    p = planner.zigzag_plan(net, open_q, closed, 10, 12, base_sliced=base.sliced_labels, trials=2)
    assert p.cost.peak_log2 <= 12 + 1e-9
    assert p.sliced_labels[:6] == list(base.sliced_labels)
    assert len(set(p.sliced_labels)) == len(p.sliced_labels)
    bonds = set(net.bond_label.values())
    assert set(p.sliced_labels) <= bonds
    # the plan's own figures agree with a recount along its path
    sp = planner.make_problem(net.labels, net.out_label, 16, open_q, closed, sliced=p.sliced_labels)
    leaves = {k for k, l in enumerate(net.labels) if any(x in p.sliced_labels for x in l)}
    again = planner.path_cost(sp, p.path, leaves)
    assert again.flops_per_slice == p.cost.flops_per_slice
    assert again.peak_log2 == p.cost.peak_log2


def test_zigzag_workload_with_head_reuse():
    c = synth.make_circuit(4, 4, 14, 44)
    open_q = list(range(10, 16))
    closed = synth.group_targets(16, open_q, 4, 45)
    w = make_zigzag_workload(c, open_q, closed, 10, 14, reuse_batch=8, seed=44)
    assert w.plan.cost.peak_log2 <= 14 + 1e-9
    assert w.plan.cost.flops_shared > 0 and len(w.slice_ids) == w.plan.n_slices
