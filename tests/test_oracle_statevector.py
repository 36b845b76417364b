"""Pins of the oracle's state-vector simulator: brute-force full unitaries on 1-3 qubits
built from Kronecker products and explicit basis loops, the norm, the empty circuit,
the Porter-Thomas collision ratio (main text, Fig. 3 discussion) and the projector form
of slicing (Appendix B.2: the slices sum to the whole)."""

import itertools
import math

import numpy as np
import pytest

import synth
from oracle import gates, statevector
from oracle.metrics import collision_ratio

BACKENDS = ("numpy", "c")


def _circuit(n, layers, theta=math.pi / 2, phi=math.pi / 6):
    return {"n_qubits": n, "fsim": {"theta": theta, "phi": phi},
            "layers": [{"oneq": o, "couplers": c} for o, c in layers]}


def _full_oneq_layer(names):
    m = np.eye(1)
    for nm in names:                      # qubit 0 is the leftmost (most significant) factor
        m = np.kron(m, gates.ONEQ[nm])
    return m


def _full_two_qubit(n, qa, qb, f):
    dim = 1 << n
    m = np.zeros((dim, dim), dtype=complex)
    for x in range(dim):                  # x = input basis state, y = output basis state
        for y in range(dim):
            same = all(((x >> (n - 1 - q)) & 1) == ((y >> (n - 1 - q)) & 1)
                       for q in range(n) if q not in (qa, qb))
            if not same:
                continue
            ai, bi = (x >> (n - 1 - qa)) & 1, (x >> (n - 1 - qb)) & 1
            ao, bo = (y >> (n - 1 - qa)) & 1, (y >> (n - 1 - qb)) & 1
            m[y, x] = f[2 * ao + bo, 2 * ai + bi]
    return m


def _brute(c):
    n = c["n_qubits"]
    n2 = sum(len(l["couplers"]) for l in c["layers"])
    thetas = c["fsim"].get("thetas", [c["fsim"]["theta"]] * n2)
    u = np.eye(1 << n, dtype=complex)
    gate = 0
    for layer in c["layers"]:
        u = _full_oneq_layer(layer["oneq"]) @ u
        for qa, qb in layer["couplers"]:
            f = gates.fsim(thetas[gate], c["fsim"]["phi"])
            u = _full_two_qubit(n, qa, qb, f) @ u
            gate += 1
    return u[:, 0]


@pytest.mark.parametrize("n,layers", [
    (1, [(["sqrt_x"], []), (["sqrt_w"], []), (["sqrt_y"], [])]),
    (2, [(["sqrt_x", "sqrt_y"], [(0, 1)]), (["sqrt_w", "sqrt_x"], [(0, 1)])]),
    (3, [(["sqrt_y", "sqrt_w", "sqrt_x"], [(0, 1)]), (["sqrt_x", "sqrt_y", "sqrt_w"], [(1, 2)]),
         (["sqrt_w", "sqrt_x", "sqrt_y"], [(0, 2)])]),
])
@pytest.mark.parametrize("backend", BACKENDS)
def test_statevector_matches_brute_force(n, layers, backend):
    c = _circuit(n, layers, theta=1.1, phi=0.7)
    assert np.allclose(statevector.simulate(c, backend=backend), _brute(c), atol=1e-14)


@pytest.mark.parametrize("backend", BACKENDS)
def test_four_qubit_gates_on_every_pair_match_brute_force(backend):
    """Two-qubit gates on every ordered pair position (adjacent, distant, the top and
    bottom bits) and with a non-symmetric four-way tensor: a wrong bit position, operand
    order or transposition in either backend changes the result."""
    n = 4
    layers = [(["sqrt_x", "sqrt_y", "sqrt_w", "sqrt_x"], [(0, 3), (1, 2)]),
              (["sqrt_w", "sqrt_x", "sqrt_y", "sqrt_w"], [(0, 1), (2, 3)]),
              (["sqrt_y", "sqrt_w", "sqrt_x", "sqrt_y"], [(1, 3)]),
              (["sqrt_x", "sqrt_x", "sqrt_w", "sqrt_y"], [(0, 2)])]
    c = _circuit(n, layers, theta=0.9, phi=1.3)
    assert np.allclose(statevector.simulate(c, backend=backend), _brute(c), atol=1e-14)
    # a general (non-symmetric, non-unitary) four-way tensor through the same primitive
    rng = np.random.default_rng(3)
    g = rng.normal(size=(2, 2, 2, 2)) + 1j * rng.normal(size=(2, 2, 2, 2))
    psi0 = rng.normal(size=16) + 1j * rng.normal(size=16)
    ref = _full_two_qubit(n, 1, 3, g.reshape(4, 4)) @ psi0
    if backend == "numpy":
        got = statevector.apply_2q(psi0.reshape((2,) * n), g, 1, 3).reshape(-1)
    else:
        st = statevector._CState(n)
        st.psi[:] = psi0
        st.apply_2q(g, 1, 3)
        got = st.flat()
    assert np.allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("backend", BACKENDS)
def test_per_gate_angles_match_brute_force(backend):
    """Calibrated gates (Results: angles near pi/2, one per gate): each two-qubit gate
    takes its own angle from the circuit's list, in circuit order; a swapped or shifted
    angle changes the state."""
    layers = [(["sqrt_y", "sqrt_w", "sqrt_x"], [(0, 1)]), (["sqrt_x", "sqrt_y", "sqrt_w"], [(1, 2)]),
              (["sqrt_w", "sqrt_x", "sqrt_y"], [(0, 2)])]
    c = _circuit(3, layers)
    c["fsim"]["thetas"] = [1.4, 1.6, 1.1]
    got = statevector.simulate(c, backend=backend)
    assert np.allclose(got, _brute(c), atol=1e-14)
    c2 = _circuit(3, layers)
    c2["fsim"]["thetas"] = [1.6, 1.4, 1.1]
    assert not np.allclose(got, statevector.simulate(c2, backend=backend), atol=1e-6)


@pytest.mark.parametrize("backend", BACKENDS)
def test_companion_cuts_match_brute_force(backend):
    """Companion-edge cuts (Appendix C): a cut gate is the fSim matrix with the entries whose
    other-qubit output differs from the pinned qubit's input set to zero (the explicit
    pinned matrices of Appendix C), written here as a basis loop."""
    layers = [(["sqrt_y", "sqrt_w", "sqrt_x"], [(0, 1)]), (["sqrt_x", "sqrt_y", "sqrt_w"], [(1, 2)]),
              (["sqrt_w", "sqrt_x", "sqrt_y"], [(0, 2)])]
    c = _circuit(3, layers)
    c["fsim"]["thetas"] = [1.3, 1.45, 1.1]
    c["cuts"] = [[0, 0], [2, 2]]
    n = 3
    u = np.eye(8, dtype=complex)
    gate = 0
    for oneq, couplers in layers:
        u = _full_oneq_layer(oneq) @ u
        for qa, qb in couplers:
            f = gates.fsim(c["fsim"]["thetas"][gate], c["fsim"]["phi"]).copy()
            pin = dict(c["cuts"]).get(gate)
            if pin is not None:
                for ao, bo, ai, bi in itertools.product((0, 1), repeat=4):
                    pin_in, other_out = (ai, bo) if pin == qa else (bi, ao)
                    if other_out != pin_in:
                        f[2 * ao + bo, 2 * ai + bi] = 0
            u = _full_two_qubit(n, qa, qb, f) @ u
            gate += 1
    got = statevector.simulate(c, backend=backend)
    assert np.allclose(got, u[:, 0], atol=1e-14)
    assert not np.allclose(got, _brute(c), atol=1e-3)


def test_jittered_circuit_angles():
    """The jitter flag draws one angle per two-qubit gate around theta (seeded, circuit
    order) and leaves the single-qubit gates as they were."""
    import math
    a = synth.make_circuit(3, 4, 8, 1001)
    b = synth.make_circuit(3, 4, 8, 1001, theta_jitter=0.02, jitter_seed=9)
    n2 = sum(len(l["couplers"]) for l in a["layers"])
    th = np.array(b["fsim"]["thetas"])
    assert len(th) == n2 and a["layers"] == b["layers"] and "thetas" not in a["fsim"]
    assert np.all(np.abs(th - math.pi / 2) < 0.2) and 0.005 < np.std(th) < 0.05
    assert synth.make_circuit(3, 4, 8, 1001, theta_jitter=0.02, jitter_seed=9)["fsim"] == b["fsim"]


@pytest.mark.parametrize("backend", BACKENDS)
def test_empty_circuit_is_all_zero_state(backend):
    c = _circuit(4, [])
    psi = statevector.simulate(c, backend=backend)
    assert psi[0] == 1 and np.count_nonzero(psi) == 1


@pytest.mark.parametrize("backend", BACKENDS)
def test_norm_and_porter_thomas(backend):
    psi = statevector.simulate(synth.make_circuit(3, 4, 8, 1001), backend=backend)
    assert abs(np.sum(np.abs(psi) ** 2) - 1.0) < 1e-12
    deep = statevector.simulate(synth.make_circuit(4, 4, 14, 11), backend=backend)
    # Porter-Thomas: 2^n sum p^2 -> 2 for deep random circuits
    assert abs(collision_ratio(np.abs(deep) ** 2) - 2.0) < 0.1


@pytest.mark.parametrize("backend", BACKENDS)
def test_projector_slices_sum_to_state(backend):
    c = synth.make_circuit(2, 3, 6, 5)
    full = statevector.simulate(c, backend=backend)
    bonds = [(0, 0), (2, 1), (4, 0)]
    acc = np.zeros_like(full)
    parts = []
    for vals in itertools.product((0, 1), repeat=len(bonds)):
        part = statevector.simulate(c, projectors=dict(zip(bonds, vals)), backend=backend)
        parts.append(part)
        acc += part
    assert np.allclose(acc, full, atol=1e-14)
    # slices are different pieces, not copies
    assert min(np.linalg.norm(p) for p in parts) < 0.9 * np.linalg.norm(full)


def test_sparse_from_state_bit_order():
    n = 3
    psi = np.arange(8, dtype=complex)
    # open qubit 2 (least significant); group closed bits 0b110 -> indices 6, 7
    out = statevector.sparse_from_state(psi, n, [2], [0b110])
    assert list(out[0]) == [6, 7]
    # open qubits [2, 0] (qubit 2 is the most significant bit of mu)
    out = statevector.sparse_from_state(psi, n, [2, 0], [0b010])
    # mu = (s2, s0): (0,0)->x=010=2, (0,1)->110=6, (1,0)->011=3, (1,1)->111=7
    assert list(out[0]) == [2, 6, 3, 7]


@pytest.mark.parametrize("backend", BACKENDS)
def test_drilled_gate_is_the_input_projector_pair(backend):
    """Hole drilling (Method): both input edges of a drilled fSim get E = |0><0|.  Eq. (1)
    has e0 as its first row and column, so fSim (P0 x P0) = (P0 x P0) fSim = |00><00| and
    the gate can be dropped; the simulator's drilled state equals the brute-force product
    with the projector pair in the gate's place (3 qubits, the middle gate drilled)."""
    for theta, phi in ((math.pi / 2, math.pi / 6), (0.7, 1.9)):
        f = gates.fsim(theta, phi)
        p00 = np.zeros((4, 4), dtype=complex)
        p00[0, 0] = 1.0
        assert np.allclose(f @ p00, p00) and np.allclose(p00 @ f, p00)
    layers = [(["sqrt_y", "sqrt_w", "sqrt_x"], [(0, 1)]), (["sqrt_x", "sqrt_y", "sqrt_w"], [(1, 2)]),
              (["sqrt_w", "sqrt_x", "sqrt_y"], [(0, 2)])]
    c = _circuit(3, layers)
    c["holes"] = [1]
    f = gates.fsim(c["fsim"]["theta"], c["fsim"]["phi"])
    proj = np.zeros((4, 4), dtype=complex)
    proj[0, 0] = 1.0
    u = np.eye(8, dtype=complex)
    gate = 0
    for oneq, couplers in layers:
        u = _full_oneq_layer(oneq) @ u
        for qa, qb in couplers:
            u = _full_two_qubit(3, qa, qb, proj if gate == 1 else f) @ u
            gate += 1
    assert np.allclose(statevector.simulate(c, backend=backend), u[:, 0], atol=1e-14)


def test_drilled_fidelity_follows_two_to_the_minus_k():
    """Each broken edge halves the fidelity (Method, F_K ~ 2^-K with K = 2 per hole): on a
    4x5-qubit, 14-cycle random circuit the mean of F / 2^-K over six random hole positions
    in the middle half of the gates is within 25% of 1 for one to three holes."""
    from oracle.metrics import fidelity
    circ = synth.make_circuit(4, 5, 14, 72)
    psi = statevector.simulate(circ)
    n2 = sum(len(l["couplers"]) for l in circ["layers"])
    rng = np.random.default_rng(72)
    for h in (1, 2, 3):
        ratios = []
        for _ in range(6):
            c = dict(circ)
            c["holes"] = sorted(rng.choice(range(n2 // 4, 3 * n2 // 4), size=h, replace=False).tolist())
            ratios.append(fidelity(statevector.simulate(c), psi) / 2.0 ** (-2 * h))
        assert 0.8 < np.mean(ratios) < 1.25, (h, ratios)


def test_drilled_network_contraction_equals_drilled_state():
    """The oracle's contractor on its drilled network (the |00><00| tensor in the gate's
    place) gives the simulator's drilled state, per group and summed over slices."""
    from oracle import contract as ocontract
    circ = synth.make_circuit(3, 3, 8, 5)
    circ["holes"] = [2, 9, 15]
    n = circ["n_qubits"]
    psi = statevector.simulate(circ)
    got = ocontract.sparse_amplitudes(circ, list(range(n)), [0])
    assert np.allclose(got.reshape(-1), psi, atol=1e-13)
    bonds = [(1, 1), (4, 2)]
    part = ocontract.sparse_amplitudes(circ, [0, 4, 8], [0b000110000], sliced_bonds=bonds,
                                       slice_ids=[0, 1, 2, 3])
    ref = statevector.sparse_from_state(psi, n, [0, 4, 8], [0b000110000])
    assert np.allclose(part, ref, atol=1e-13)
