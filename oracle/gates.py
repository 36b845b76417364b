"""Gate matrices (oracle; test infrastructure only).

fSim(theta, phi) is Eq. (1) of the paper (also restated in Appendix C): in the basis
|q_a q_b> with index 2*a + b it is
    [[1, 0, 0, 0], [0, cos t, -i sin t, 0], [0, -i sin t, cos t, 0], [0, 0, 0, e^{-i phi}]].
The matrix is symmetric, so reading it as (output, input) or (input, output) gives the
same tensor.

The single-qubit gates sqrt(X), sqrt(Y), sqrt(W) are not defined in the paper (they come
from Google's circuits).  Reading used here: sqrt(P) = exp(-i pi/4 P) = (I - i P)/sqrt 2
for P in {X, Y, W}, W = (X + Y)/sqrt 2.
"""

from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI_W = (PAULI_X + PAULI_Y) / np.sqrt(2.0)


def sqrt_pauli(p: np.ndarray) -> np.ndarray:
    """exp(-i pi/4 P) for an involutory Pauli-type matrix P."""
    return (I2 - 1j * p) / np.sqrt(2.0)


ONEQ = {
    "sqrt_x": sqrt_pauli(PAULI_X),
    "sqrt_y": sqrt_pauli(PAULI_Y),
    "sqrt_w": sqrt_pauli(PAULI_W),
}


def fsim(theta: float, phi: float) -> np.ndarray:
    """Eq. (1): the 4x4 fSim matrix."""
    c, s = np.cos(theta), np.sin(theta)
    return np.array([
        [1, 0, 0, 0],
        [0, c, -1j * s, 0],
        [0, -1j * s, c, 0],
        [0, 0, 0, np.exp(-1j * phi)],
    ], dtype=np.complex128)


def fsim_tensor(theta: float, phi: float) -> np.ndarray:
    """fSim as a four-way tensor G[out_a, out_b, in_a, in_b] (q_a = lower qubit id)."""
    return fsim(theta, phi).reshape(2, 2, 2, 2)


def companion_cut(theta: float, phi: float, pinned: int) -> np.ndarray:
    """fSim with the companion-edge rank-one approximation (Method, low-rank case (ii);
    Appendix C), as a four-way tensor G[out_a, out_b, in_a, in_b].

    `pinned` (0 = q_a, 1 = q_b) is the input whose edge is fixed by slicing.  For each
    value v of that input the gate is a three-way tensor; grouping the pinned qubit's output
    with the other input against the other qubit's output (the companion edge) gives a 4 x 2
    matrix whose squared singular values are 1 + sin^2(theta) and cos^2(theta).  Each such
    matrix is replaced by its best rank-one approximation (largest singular triplet of its
    SVD), and the two slices are put back together."""
    g = fsim_tensor(theta, phi)
    other = 1 - pinned
    out = np.zeros_like(g)
    for v in (0, 1):
        t = g[:, :, v, :] if pinned == 0 else g[:, :, :, v]      # [out_a, out_b, in_other]
        # rows (out_pinned, in_other), columns out_other
        m = np.moveaxis(t, other, -1).reshape(4, 2)
        u, sv, vh = np.linalg.svd(m)
        r1 = sv[0] * np.outer(u[:, 0], vh[0, :])
        t1 = np.moveaxis(r1.reshape(2, 2, 2), -1, other)
        if pinned == 0:
            out[:, :, v, :] = t1
        else:
            out[:, :, :, v] = t1
    return out


def gate_thetas(circuit: dict) -> list:
    """The angle of every two-qubit gate in circuit order: the per-gate list
    circuit["fsim"]["thetas"] when present (calibrated gates: angles near, not at, one
    value), else the one angle circuit["fsim"]["theta"]."""
    f = circuit["fsim"]
    n2 = sum(len(l["couplers"]) for l in circuit["layers"])
    return list(f["thetas"]) if "thetas" in f else [f["theta"]] * n2
