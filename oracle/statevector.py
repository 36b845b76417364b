"""Gate-by-gate state-vector simulator (oracle; test infrastructure only).

The state of n qubits is a complex128 array of shape (2,)*n with axis q = qubit q, so
its C-order flattening has index x(s) = sum_q s_q 2^(n-1-q): qubit 0 is the most
significant bit.  One cycle applies the single-qubit layer, then the fSim gates of the
cycle's coupler pattern (paper, Results: sequence ABCDCDAB; Eq. (1) for fSim).

Slicing (Appendix B.2) fixes a bond of the network to one value.  A bond here is named
(q, j): the wire of qubit q right after the j-th two-qubit gate acting on q (j counts
from 0).  Fixing it to v is the same as inserting the projector |v><v| on that wire, so
`simulate(..., projectors={(q, j): v})` returns the unnormalised state of one slice,
<s|U_sigma|0^n> for every s.

Hole drilling (Method): a circuit may list `holes`, indices of two-qubit gates in circuit
order (cycle by cycle, coupler order).  Drilling gate g breaks its two input edges by
inserting E = |0><0| on each, right before the gate; since fSim|00> = |00>, the drilled
gate with both inputs projected is |00><00|, so the simulator applies the projector
|0><0| to both qubits in place of the gate.  The result is the unnormalised approximate
state psi_hat of the perturbed network.
"""

from __future__ import annotations

import numpy as np

from .gates import ONEQ, fsim_tensor


def apply_1q(psi: np.ndarray, u: np.ndarray, q: int) -> np.ndarray:
    out = np.tensordot(u, psi, axes=([1], [q]))
    return np.moveaxis(out, 0, q)


def apply_2q(psi: np.ndarray, g: np.ndarray, qa: int, qb: int) -> np.ndarray:
    """g[out_a, out_b, in_a, in_b] acting on qubits qa, qb."""
    out = np.tensordot(g, psi, axes=([2, 3], [qa, qb]))
    return np.moveaxis(out, [0, 1], [qa, qb])


def project(psi: np.ndarray, q: int, v: int) -> np.ndarray:
    p = np.zeros((2, 2), dtype=np.complex128)
    p[v, v] = 1.0
    return apply_1q(psi, p, q)


def simulate(circuit: dict, projectors: dict | None = None) -> np.ndarray:
    """Final state |psi> = U|0^n> (flattened, length 2^n), optionally one slice of it."""
    n = circuit["n_qubits"]
    projectors = dict(projectors or {})
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    g = fsim_tensor(circuit["fsim"]["theta"], circuit["fsim"]["phi"])
    holes = set(int(h) for h in circuit.get("holes", ()))
    n2q = [0] * n
    gate = 0
    for layer in circuit["layers"]:
        for q, name in enumerate(layer["oneq"]):
            psi = apply_1q(psi, ONEQ[name], q)
        for qa, qb in layer["couplers"]:
            if gate in holes:
                psi = project(project(psi, qa, 0), qb, 0)
            else:
                psi = apply_2q(psi, g, qa, qb)
            gate += 1
            for q in (qa, qb):
                key = (q, n2q[q])
                if key in projectors:
                    psi = project(psi, q, projectors[key])
                n2q[q] += 1
    return psi.reshape(-1)


def amplitude_index(bits: int, n: int) -> int:
    """State-vector index of a uint64 bitstring (bit n-1-q holds s_q): the same integer."""
    return int(bits) & ((1 << n) - 1)


def sparse_from_state(psi: np.ndarray, n: int, open_qubits, closed_bits) -> np.ndarray:
    """amps[i][mu] = psi(closed_bits[i] with the open qubits set from mu).

    mu = sum_t s_{open[t]} 2^(n_open-1-t): the first listed open qubit is the most
    significant bit of mu.
    """
    open_qubits = list(open_qubits)
    no = len(open_qubits)
    out = np.zeros((len(closed_bits), 1 << no), dtype=np.complex128)
    for i, cb in enumerate(closed_bits):
        for mu in range(1 << no):
            x = int(cb)
            for t, q in enumerate(open_qubits):
                bit = (mu >> (no - 1 - t)) & 1
                x &= ~(1 << (n - 1 - q))
                x |= bit << (n - 1 - q)
            out[i, mu] = psi[x]
    return out
