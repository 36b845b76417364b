"""Circuit -> simplified tensor network (host side of the library).

Paper, "Method": single-qubit gates are matrices, fSim gates (Eq. (1)) four-way
tensors, the initial product state is a set of vectors and the final state a boundary.
Results paragraph: the network is simplified by contracting order-one and order-two
tensors into their neighbours before planning.

The construction here never materialises a separate tensor for a single-qubit gate:
  * gates acting on a qubit before its first fSim are folded into that qubit's initial
    vector, which is then folded into the first fSim's input leg;
  * gates between two fSims on a qubit are folded forward into the later fSim's input;
  * gates after a qubit's last fSim are folded backward into that fSim's output leg,
    which becomes the qubit's output leg.
Afterwards any tensor of rank <= 2 (for example a first-cycle fSim whose two inputs were
both initial vectors) is contracted into a neighbour, repeatedly.

Labels are non-negative ints.  The output of the j-th two-qubit gate on qubit q that
feeds a later two-qubit gate on q is the bond named (q, j); `bond_label[(q, j)]` is its
label while it survives simplification.  `out_label[q]` is qubit q's output leg.
Tensor data are complex128, row-major in label order (first label slowest).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_S2 = 1.0 / math.sqrt(2.0)
# exp(-i pi/4 P) for P = X, Y, W = (X+Y)/sqrt2, written out entry by entry.
_ONEQ = {
    "sqrt_x": np.array([[_S2, -1j * _S2], [-1j * _S2, _S2]], dtype=np.complex128),
    "sqrt_y": np.array([[_S2, -_S2], [_S2, _S2]], dtype=np.complex128),
    "sqrt_w": np.array([[_S2, -_S2 * complex(_S2, _S2)],
                        [_S2 * complex(_S2, -_S2), _S2]], dtype=np.complex128),
}


def _fsim4(theta: float, phi: float) -> np.ndarray:
    """fSim as t[out_a, out_b, in_a, in_b]; the 4x4 of Eq. (1) is symmetric."""
    t = np.zeros((2, 2, 2, 2), dtype=np.complex128)
    t[0, 0, 0, 0] = 1.0
    t[0, 1, 0, 1] = math.cos(theta)
    t[1, 0, 1, 0] = math.cos(theta)
    t[0, 1, 1, 0] = -1j * math.sin(theta)
    t[1, 0, 0, 1] = -1j * math.sin(theta)
    t[1, 1, 1, 1] = complex(math.cos(phi), -math.sin(phi))
    return t


@dataclass
class TensorNetwork:
    n_qubits: int
    tensors: list = field(default_factory=list)      # complex128 arrays
    labels: list = field(default_factory=list)       # list[list[int]]
    out_label: list = field(default_factory=list)    # [n_qubits]
    bond_label: dict = field(default_factory=dict)   # (q, j) -> label
    cycle: list = field(default_factory=list)        # per tensor: cycle of its gate (-1: none)
    cut_pairs: list = field(default_factory=list)    # (sliced label, companion label) per cut

    def ranks(self):
        return [len(l) for l in self.labels]

    def flat_labels(self):
        return [x for l in self.labels for x in l]

    def flat_data(self):
        parts = [np.ascontiguousarray(t, dtype=np.complex128).reshape(-1) for t in self.tensors]
        return np.concatenate(parts) if parts else np.zeros(0, np.complex128)


def _apply_matrix(t: np.ndarray, labels: list, lab: int, m: np.ndarray, side: str) -> np.ndarray:
    """side 'in': t[..., a, ...] <- sum_b t[..., b, ...] m[b, a]   (m acts before t)
       side 'out': t[..., a, ...] <- sum_b m[a, b] t[..., b, ...]  (m acts after t)"""
    ax = labels.index(lab)
    mm = m if side == "in" else m.T
    out = np.tensordot(t, mm, axes=([ax], [0]))
    return np.moveaxis(out, -1, ax)


def circuit_network(circuit: dict, simplify: bool = True) -> TensorNetwork:
    """Tensor network of a circuit (Method).  `circuit["holes"]` (optional) lists two-qubit
    gates, by index in circuit order, whose two input edges are broken (hole drilling,
    Method): E = |0><0| on each input wire makes the fSim gate |00><00|, so the gate is
    dropped, the incoming wire is closed with <0| (after its pending single-qubit gates)
    and the outgoing wire starts again from |0>.  The perturbed network's amplitudes are
    those of psi_hat, with fidelity about 2^-K for K = 2 per hole.

    `circuit["cuts"]` (optional) lists companion-edge cuts [g, q] (Method, low-rank case
    (ii); Appendix C): the input edge of gate g on qubit q is sliced, and for each value v
    the gate's rank-one approximation keeps exactly the entries whose output on the other
    qubit equals v (the other singular vector, of weight cos^2 theta, is dropped).  Here the
    single-qubit gates between the previous two-qubit gate on q and g are folded into the
    previous gate's output instead of g's input, so that the bond (q, j) entering g is g's
    own input; the cut is then realised by slicing that bond and g's output bond on the
    other qubit (the companion edge) with one shared slice bit.  The pair of labels is kept
    in `cut_pairs`; the network itself stays exact (its full slice sum is the circuit's
    amplitude), the approximation is in summing only the slices where both bits agree."""
    n = circuit["n_qubits"]
    holes = set(int(h) for h in circuit.get("holes", ()))
    cuts = {}
    for g, q in circuit.get("cuts", ()):
        if int(g) in cuts or int(g) in holes:
            raise ValueError(f"gate {g} is cut twice or also drilled")
        cuts[int(g)] = int(q)
    cut_pairs, companions = [], set()
    n2 = sum(len(layer["couplers"]) for layer in circuit["layers"])
    # one angle for every gate, or calibrated per-gate angles ("thetas", circuit order)
    thetas = circuit["fsim"].get("thetas", [circuit["fsim"]["theta"]] * n2)
    if len(thetas) != n2:
        raise ValueError(f"fsim thetas lists {len(thetas)} angles for {n2} two-qubit gates")
    phi = circuit["fsim"]["phi"]
    if any(h < 0 or h >= n2 for h in holes) or any(g < 0 or g >= n2 for g in cuts):
        raise ValueError(f"hole and cut indices must name one of the {n2} two-qubit gates")
    gate = 0
    scale = complex(1.0)
    next_label = [0]

    def new_label():
        next_label[0] += 1
        return next_label[0] - 1

    tensors, labels, cycles = [], [], []
    head = [np.array([1.0, 0.0], dtype=np.complex128) for _ in range(n)]  # state before 1st fSim
    pending = [np.eye(2, dtype=np.complex128) for _ in range(n)]          # 1q gates since last fSim
    last = [None] * n          # (tensor index, output label) of the last fSim on q
    n2q = [0] * n
    bond_of = {}               # label -> (q, j)
    for cyc, layer in enumerate(circuit["layers"]):
        for q, name in enumerate(layer["oneq"]):
            u = _ONEQ[name]
            if last[q] is None:
                head[q] = u @ head[q]
            else:
                pending[q] = u @ pending[q]
        for qa, qb in layer["couplers"]:
            drilled = gate in holes
            theta = thetas[gate]
            gate += 1
            if drilled:
                for q in (qa, qb):
                    if last[q] is None:            # wire still a vector: <0|v is a number
                        scale *= complex(head[q][0])
                    else:                          # close the last fSim's output with <0|P
                        idx, o = last[q]
                        ax = labels[idx].index(o)
                        tensors[idx] = np.tensordot(tensors[idx], pending[q][0, :], axes=([ax], [0]))
                        labels[idx].remove(o)
                        bond_of.pop(o, None)
                    head[q] = np.array([1.0, 0.0], dtype=np.complex128)
                    pending[q] = np.eye(2, dtype=np.complex128)
                    last[q] = None
                    n2q[q] += 1
                continue
            t = _fsim4(theta, phi)
            oa, ob = new_label(), new_label()
            labs = [oa, ob, -1, -2]
            pin = cuts.get(gate - 1)
            if pin is not None:
                if pin not in (qa, qb):
                    raise ValueError(f"cut of gate {gate - 1} names qubit {pin}, not one of its own")
                if last[pin] is None:
                    raise ValueError(f"cut of gate {gate - 1}: no earlier two-qubit gate on qubit "
                                     f"{pin}, its input is not a bond")
                pidx, pout = last[pin]
                if pout in companions:
                    raise ValueError(f"cut of gate {gate - 1} pins the companion edge of another cut")
                # the pending single-qubit gates move to the previous gate's output
                tensors[pidx] = _apply_matrix(tensors[pidx], labels[pidx], pout, pending[pin], "out")
                pending[pin] = np.eye(2, dtype=np.complex128)
                comp = ob if pin == qa else oa
                cut_pairs.append((pout, comp))
                companions.add(comp)
            # fold the inputs: initial vectors or the pending gates of each wire
            for q, slot in ((qa, -1), (qb, -2)):
                if last[q] is None:
                    ax = labs.index(slot)
                    t = np.tensordot(t, head[q], axes=([ax], [0]))
                    labs.remove(slot)
                else:
                    prev_out = last[q][1]
                    t = _apply_matrix(t, labs, slot, pending[q], "in")
                    labs[labs.index(slot)] = prev_out
                    pending[q] = np.eye(2, dtype=np.complex128)
            tensors.append(t)
            labels.append(labs)
            cycles.append(cyc)
            idx = len(tensors) - 1
            for q, o in ((qa, oa), (qb, ob)):
                bond_of[o] = (q, n2q[q])
                n2q[q] += 1
                last[q] = (idx, o)
    out_label = [None] * n
    for q in range(n):
        if last[q] is None:
            o = new_label()
            tensors.append(head[q].copy())
            labels.append([o])
            cycles.append(-1)
            out_label[q] = o
        else:
            idx, o = last[q]
            tensors[idx] = _apply_matrix(tensors[idx], labels[idx], o, pending[q], "out")
            out_label[q] = o
            bond_of.pop(o, None)          # last output of a qubit is its leg, not a bond
    # tensors left without legs by closed wires are numbers: fold them into one tensor
    keep = [k for k in range(len(tensors)) if labels[k]]
    for k in range(len(tensors)):
        if not labels[k]:
            scale *= complex(np.asarray(tensors[k]).reshape(()))
    tensors = [tensors[k] for k in keep]
    labels = [labels[k] for k in keep]
    cycles = [cycles[k] for k in keep]
    if scale != 1.0:
        tensors[0] = tensors[0] * scale
    pinned = {b for b, _ in cut_pairs}
    for b, c in cut_pairs:
        if c not in bond_of:
            raise ValueError("a cut gate's other output must feed a later two-qubit gate")
        if c in pinned:
            raise ValueError("a cut's companion edge is the pinned edge of another cut")
    net = TensorNetwork(n_qubits=n, tensors=tensors, labels=labels, out_label=out_label,
                        bond_label={v: k for k, v in bond_of.items()}, cycle=cycles,
                        cut_pairs=cut_pairs)
    if simplify:
        simplify_low_rank(net)
        present = {x for l in net.labels for x in l}
        if any(b not in present or c not in present for b, c in cut_pairs):
            raise ValueError("simplification contracted a cut's edge away")
    return net


def simplify_low_rank(net: TensorNetwork) -> None:
    """Contract every tensor of rank <= 2 into a neighbour (one sharing a label),
    repeatedly; the neighbour's rank never grows."""
    changed = True
    while changed:
        changed = False
        holders = {}
        for i, l in enumerate(net.labels):
            for x in l or ():
                holders.setdefault(x, []).append(i)
        for i, l in enumerate(net.labels):
            if l is None or len(l) > 2:
                continue
            nbrs = sorted({j for x in l for j in holders[x] if j != i and net.labels[j] is not None})
            if not nbrs:
                continue
            j = min(nbrs, key=lambda k: (len(net.labels[k]), k))
            shared = [x for x in l if x in net.labels[j]]
            ai = [l.index(x) for x in shared]
            aj = [net.labels[j].index(x) for x in shared]
            res = np.tensordot(net.tensors[j], net.tensors[i], axes=(aj, ai))
            new = [x for x in net.labels[j] if x not in shared] + [x for x in l if x not in shared]
            net.tensors[j], net.labels[j] = res, new
            net.tensors[i], net.labels[i] = None, None
            for x in shared:
                for q_j, lab in list(net.bond_label.items()):
                    if lab == x:
                        del net.bond_label[q_j]
            changed = True
            break
    keep = [i for i, l in enumerate(net.labels) if l is not None]
    net.tensors = [net.tensors[i] for i in keep]
    net.labels = [list(net.labels[i]) for i in keep]
    if net.cycle:
        net.cycle = [net.cycle[i] for i in keep]
