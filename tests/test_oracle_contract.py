"""Pins of the oracle's pairwise contractor against the independent state-vector route,
path independence, slicing (Appendix B.2) and the sparse-state worked example
(Appendix A)."""

import itertools

import numpy as np

import synth
from oracle import contract, network, statevector


def test_all_open_equals_state_vector_small_config():
    c = synth.circuit_from_config(synth.config("small"))
    n = c["n_qubits"]
    amps = contract.sparse_amplitudes(c, list(range(n)), [0])
    psi = statevector.simulate(c)
    assert np.allclose(amps[0], psi, atol=1e-12, rtol=0)
    assert abs(np.sum(np.abs(amps) ** 2) - 1) < 1e-12


def test_amplitude_mode_matches_state_vector():
    cfg = synth.config("small")
    c = synth.circuit_from_config(cfg)
    n = c["n_qubits"]
    bits = synth.distinct_bitstrings(n, cfg["amplitudes"]["count"], cfg["amplitudes"]["seed"])
    amps = contract.sparse_amplitudes(c, [], bits)
    psi = statevector.simulate(c)
    assert amps.shape == (64, 1)
    assert np.allclose(amps[:, 0], psi[bits.astype(np.int64)], atol=1e-13, rtol=0)


def test_groups_with_open_qubits_match_state_vector():
    c = synth.make_circuit(3, 3, 7, 17)
    n = c["n_qubits"]
    open_q = [4, 1, 7]
    closed = synth.group_targets(n, open_q, 5, 99)
    amps = contract.sparse_amplitudes(c, open_q, closed)
    ref = statevector.sparse_from_state(statevector.simulate(c), n, open_q, closed)
    assert np.allclose(amps, ref, atol=1e-13, rtol=0)


def test_path_independence():
    c = synth.make_circuit(2, 3, 6, 3)
    n = c["n_qubits"]
    a = contract.sparse_amplitudes(c, list(range(n)), [0], path="greedy")
    b = contract.sparse_amplitudes(c, list(range(n)), [0], path="time")
    net = network.build_network(c, {})
    t, l = net.sliced({})
    p = contract.greedy_path(l, seed=5)
    d = contract.sparse_amplitudes(c, list(range(n)), [0], path=p)
    e = contract.sparse_amplitudes(c, list(range(n)), [0], path="random-greedy:7")
    assert np.allclose(a, b, atol=1e-13) and np.allclose(a, d, atol=1e-13)
    assert np.allclose(a, e, atol=1e-13)
    # the perturbed search is a different order, not a copy of the plain greedy one
    assert contract.random_greedy_path(l, 7, trials=1, temperature=4.0) != contract.greedy_path(l)


def test_slices_sum_to_unsliced_and_match_projected_state():
    c = synth.make_circuit(3, 3, 8, 23)
    n = c["n_qubits"]
    open_q = [0, 4, 8]
    closed = synth.group_targets(n, open_q, 3, 7)
    net = network.build_network(c, {})
    bonds = sorted(net.bond_label)[:: max(1, len(net.bond_label) // 4)][:4]
    per = contract.sparse_amplitudes(c, open_q, closed, sliced_bonds=bonds, per_slice=True)
    whole = contract.sparse_amplitudes(c, open_q, closed)
    assert per.shape[0] == 16
    assert np.allclose(per.sum(axis=0), whole, atol=1e-13)
    for sigma in (0, 5, 15):
        proj = {b: (sigma >> i) & 1 for i, b in enumerate(bonds)}
        psi_s = statevector.simulate(c, projectors=proj)
        ref = statevector.sparse_from_state(psi_s, n, open_q, closed)
        assert np.allclose(per[sigma], ref, atol=1e-13)
    # a subset of slices sums to the matching part only
    sub = contract.sparse_amplitudes(c, open_q, closed, sliced_bonds=bonds, slice_ids=[3, 9])
    assert np.allclose(sub, per[3] + per[9], atol=1e-13)


def test_bond_names_exclude_output_wires():
    c = synth.make_circuit(2, 2, 4, 1)
    net = network.build_network(c, {})
    for (q, j), lab in net.bond_label.items():
        assert lab != net.out_label[q]


def test_worked_example_three_qubits():
    # Appendix A: three qubits, targets {111, 010, 000} (qubit 1 is the leftmost bit).
    c = {"n_qubits": 3, "fsim": {"theta": 1.2, "phi": 0.3},
         "layers": [{"oneq": ["sqrt_x", "sqrt_y", "sqrt_w"], "couplers": [(0, 1)]},
                    {"oneq": ["sqrt_y", "sqrt_w", "sqrt_x"], "couplers": [(1, 2)]},
                    {"oneq": ["sqrt_w", "sqrt_x", "sqrt_y"], "couplers": [(0, 2)]}]}
    targets = [0b111, 0b010, 0b000]
    amps = contract.sparse_amplitudes(c, [], targets)
    psi = statevector.simulate(c)
    assert np.allclose(amps[:, 0], psi[targets], atol=1e-14)


def test_peak_size_counts_elements():
    labels = [("a", "b"), ("b", "c"), ("c", "d")]
    assert contract.peak_size(labels, [(0, 1), (0, 2)]) == 4
    assert contract.peak_size([("a",), ("b",)], [(0, 1)]) == 4


def test_jittered_angles_contractor_equals_state_vector():
    """Per-gate angles reach the contractor's network as they reach the simulator: the
    two routes agree on a jittered circuit, sliced and summed."""
    c = synth.make_circuit(3, 3, 8, 23, theta_jitter=0.03, jitter_seed=4)
    n = c["n_qubits"]
    open_q = [1, 5, 7]
    closed = synth.group_targets(n, open_q, 3, 8)
    bonds = [(1, 1), (4, 2), (3, 0)]
    amps = contract.sparse_amplitudes(c, open_q, closed, sliced_bonds=bonds)
    ref = statevector.sparse_from_state(statevector.simulate(c), n, open_q, closed)
    assert np.allclose(amps, ref, atol=1e-13)
