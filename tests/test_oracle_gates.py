"""Pins of the oracle's gate set: closed forms that Eq. (1), Appendix C and the reading
of the single-qubit gates fix, none of which re-types the oracle's own formulas."""

import numpy as np
import pytest

from oracle import gates


def test_single_qubit_gates_unitary_and_square_to_minus_i_pauli():
    paulis = {"sqrt_x": gates.PAULI_X, "sqrt_y": gates.PAULI_Y, "sqrt_w": gates.PAULI_W}
    for name, p in paulis.items():
        u = gates.ONEQ[name]
        assert np.allclose(u.conj().T @ u, np.eye(2), atol=1e-15)
        # sqrt(P)^2 = exp(-i pi/2 P) = -i P for an involutory P
        assert np.allclose(u @ u, -1j * p, atol=1e-15), name
        assert np.allclose(p @ p, np.eye(2), atol=1e-15)


def test_sqrt_w_explicit_entries():
    # W = (X + Y)/sqrt2 has off-diagonal entries e^{-i pi/4} (top right) and e^{i pi/4}
    w = gates.PAULI_W
    assert np.isclose(w[0, 1], np.exp(-1j * np.pi / 4))
    assert np.isclose(w[1, 0], np.exp(1j * np.pi / 4))
    u = gates.ONEQ["sqrt_w"] * np.sqrt(2)
    assert np.allclose(u, [[1, -np.exp(1j * np.pi / 4)], [np.exp(-1j * np.pi / 4), 1]])


@pytest.mark.parametrize("theta,phi", [(np.pi / 2, np.pi / 6), (0.3, 1.1), (1.4, -0.2)])
def test_fsim_unitary_symmetric(theta, phi):
    f = gates.fsim(theta, phi)
    assert np.allclose(f.conj().T @ f, np.eye(4), atol=1e-15)
    assert np.allclose(f, f.T)


def test_fsim_basis_maps_at_half_pi():
    phi = np.pi / 6
    f = gates.fsim(np.pi / 2, phi)
    e = np.eye(4)
    assert np.allclose(f @ e[0], e[0])                       # |00> -> |00>
    assert np.allclose(f @ e[1], -1j * e[2])                 # |01> -> -i|10>
    assert np.allclose(f @ e[2], -1j * e[1])                 # |10> -> -i|01>
    assert np.allclose(f @ e[3], np.exp(-1j * phi) * e[3])   # |11> -> e^{-i phi}|11>
    assert np.allclose(gates.fsim(0.0, 0.0), np.eye(4))


def test_fsim_tensor_indexing():
    g = gates.fsim_tensor(0.7, 0.4)
    f = gates.fsim(0.7, 0.4)
    for oa in range(2):
        for ob in range(2):
            for ia in range(2):
                for ib in range(2):
                    assert g[oa, ob, ia, ib] == f[2 * oa + ob, 2 * ia + ib]


def test_both_inputs_pinned_gives_rank_one():
    # Appendix C, first situation: (|0><0| x |0><0|) fSim is rank one and equals
    # (1,0) x (1,0) on the outputs.
    p0 = np.diag([1.0, 0.0])
    a = gates.fsim(1.3, 0.5) @ np.kron(p0, p0)
    assert np.linalg.matrix_rank(a) == 1
    assert np.allclose(a[:, 0], [1, 0, 0, 0])


@pytest.mark.parametrize("theta", [np.pi / 2, 1.2, 0.4])
def test_one_input_pinned_singular_values(theta):
    # Appendix C, second situation: with one input pinned, grouping (pinned input's
    # partner input, one output) against the other output gives squared singular values
    # (1 + sin^2 theta, cos^2 theta) in all four pinning cases.
    g = gates.fsim_tensor(theta, 0.9)           # [oa, ob, ia, ib]
    want = sorted([1 + np.sin(theta) ** 2, np.cos(theta) ** 2])
    for pinned_input in ("a", "b"):
        for v in (0, 1):
            t = g[:, :, v, :] if pinned_input == "a" else g[:, :, :, v]   # [oa, ob, free in]
            for companion in (0, 1):            # the output kept as the column index
                m = np.moveaxis(t, companion, -1).reshape(4, 2)
                s2 = sorted(np.linalg.svd(m, compute_uv=False) ** 2)
                if np.allclose(s2, want, atol=1e-12):
                    break
            else:
                pytest.fail(f"no grouping gives {want} for input {pinned_input}={v}")


@pytest.mark.parametrize("theta", [np.pi / 2, 1.45, 1.2, 0.9])
@pytest.mark.parametrize("pinned", [0, 1])
def test_companion_cut_keeps_the_dominant_column(theta, pinned):
    # Appendix C lists the four pinned matrices explicitly: for input value v their columns
    # (the companion output) are orthogonal, and the one of squared norm 1 + sin^2 theta is
    # the companion output equal to v.  So the rank-one cut keeps exactly the entries whose
    # other-qubit output equals the pinned input, and drops cos^2 theta per value.
    g = gates.fsim_tensor(theta, 0.7)                # [oa, ob, ia, ib]
    cut = gates.companion_cut(theta, 0.7, pinned)
    mask = np.zeros((2, 2, 2, 2))
    for oa in (0, 1):
        for ob in (0, 1):
            for ia in (0, 1):
                for ib in (0, 1):
                    pin_in, other_out = (ia, ob) if pinned == 0 else (ib, oa)
                    mask[oa, ob, ia, ib] = float(other_out == pin_in)
    assert np.allclose(cut, g * mask, atol=1e-12)
    assert np.isclose(np.sum(np.abs(g - cut) ** 2), 2 * np.cos(theta) ** 2)
    assert np.isclose(np.sum(np.abs(cut) ** 2), 2 * (1 + np.sin(theta) ** 2))
    if theta == np.pi / 2:                           # nothing is dropped at pi/2
        assert np.allclose(cut, g, atol=1e-15)


def test_companion_cut_in_the_state_vector():
    # one cut gate on a two-qubit register: the simulator applies the cut operator in place
    # of fSim (|psi> after the 1q layer, then G~), checked by hand here
    circ = {"n_qubits": 2, "fsim": {"theta": 1.1, "phi": 0.3},
            "layers": [{"oneq": ["sqrt_x", "sqrt_y"], "couplers": [[0, 1]]}], "cuts": [[0, 1]]}
    from oracle import statevector
    psi = statevector.simulate(circ)
    start = np.kron(gates.ONEQ["sqrt_x"][:, 0], gates.ONEQ["sqrt_y"][:, 0])
    want = gates.companion_cut(1.1, 0.3, 1).reshape(4, 4) @ start
    assert np.allclose(psi, want, atol=1e-14)
    assert not np.allclose(psi, gates.fsim(1.1, 0.3) @ start)
    with pytest.raises(ValueError):
        statevector.simulate(dict(circ, cuts=[[0, 5]]))


def test_edge_breaking_matrix():
    # Method: E = (1,0)^T (1,0) = I/2 + sigma_z/2
    e = np.outer([1, 0], [1, 0])
    assert np.allclose(e, 0.5 * gates.I2 + 0.5 * gates.PAULI_Z)
