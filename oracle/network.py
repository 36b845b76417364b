"""The circuit as a tensor network, built gate by gate (oracle; test infrastructure only).

Paper, "Method": single-qubit gates become matrices, two-qubit gates four-way tensors,
the initial product state a set of vectors (left boundary) and the final state the
right boundary.  Nothing is simplified here: every gate is its own tensor.

Labels are tuples:
  ("w", q, k)   the wire of qubit q after its k-th gate (k = 0 is the initial wire);
bond names for slicing are (q, j) = the wire right after the j-th two-qubit gate on q,
for every j except the last two-qubit gate on q, and `bond_label[(q, j)]` maps such a
name to its wire label.  A qubit's last wire is
its output leg `out_label[q]`.  The right boundary attaches a basis vector e_{s_q} to
the output leg of every closed qubit and leaves the open qubits' legs open.

Hole drilling (Method): a gate listed in `circuit["holes"]` (index in circuit order) has
both input edges broken by E = |0><0|, which turns the fSim tensor into |00><00|; here
that four-way tensor takes the gate's place (the wires stay connected).
"""

from __future__ import annotations

import numpy as np

from .gates import ONEQ, fsim_tensor, gate_thetas


class Network:
    def __init__(self):
        self.tensors: list[np.ndarray] = []
        self.labels: list[tuple] = []
        self.bond_label: dict[tuple[int, int], tuple] = {}
        self.out_label: dict[int, tuple] = {}

    def add(self, data: np.ndarray, labels) -> None:
        assert data.ndim == len(labels)
        self.tensors.append(np.asarray(data, dtype=np.complex128))
        self.labels.append(tuple(labels))

    def sliced(self, values: dict) -> tuple[list[np.ndarray], list[tuple]]:
        """Copy of the network with each label in `values` fixed to its value."""
        tensors, labels = [], []
        for t, lab in zip(self.tensors, self.labels):
            for l, v in values.items():
                if l in lab:
                    ax = lab.index(l)
                    t = np.take(t, v, axis=ax)
                    lab = lab[:ax] + lab[ax + 1:]
            tensors.append(t)
            labels.append(lab)
        return tensors, labels


def build_network(circuit: dict, closed_values: dict | None = None) -> Network:
    """Network of <s_closed| U |0^n>, open qubits left open.

    closed_values: {qubit: bit} for the projected (closed) qubits.
    """
    n = circuit["n_qubits"]
    closed_values = dict(closed_values or {})
    thetas = gate_thetas(circuit)
    phi = circuit["fsim"]["phi"]
    holes = set(int(h) for h in circuit.get("holes", ()))
    p00 = np.zeros((2, 2, 2, 2), dtype=np.complex128)
    p00[0, 0, 0, 0] = 1.0
    gate = 0
    net = Network()
    k = [0] * n
    n2q = [0] * n
    zero = np.array([1.0, 0.0], dtype=np.complex128)
    for q in range(n):
        net.add(zero, [("w", q, 0)])
    for layer in circuit["layers"]:
        for q, name in enumerate(layer["oneq"]):
            net.add(ONEQ[name], [("w", q, k[q] + 1), ("w", q, k[q])])
            k[q] += 1
        for qa, qb in layer["couplers"]:
            g = p00 if gate in holes else fsim_tensor(thetas[gate], phi)
            net.add(g, [("w", qa, k[qa] + 1), ("w", qb, k[qb] + 1),
                                                  ("w", qa, k[qa]), ("w", qb, k[qb])])
            gate += 1
            for q in (qa, qb):
                k[q] += 1
                net.bond_label[(q, n2q[q])] = ("w", q, k[q])
                n2q[q] += 1
    for q in range(n):
        net.out_label[q] = ("w", q, k[q])
    # A bond is the output of a two-qubit gate that feeds a later two-qubit gate on the
    # same qubit; the last two-qubit gate's output on a qubit only leads (through
    # single-qubit gates, if any) to the qubit's output leg and is not a bond.
    net.bond_label = {key: lab for key, lab in net.bond_label.items()
                      if key[1] + 1 < n2q[key[0]]}
    for q, v in closed_values.items():
        e = np.zeros(2, dtype=np.complex128)
        e[int(v)] = 1.0
        net.add(e, [net.out_label[q]])
    return net
