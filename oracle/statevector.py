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

Companion-edge cuts (Method, low-rank case (ii); Appendix C): a circuit may list `cuts`,
pairs [g, q] naming a two-qubit gate g (circuit order) and one of its qubits q whose input
edge slicing fixes.  The gate is then replaced by gates.companion_cut: for each value of
that input, its best rank-one approximation across the other qubit's output (the
companion edge).  Summed over the fixed value, that is one 4 x 4 (non-unitary) operator in
place of fSim, so the simulator applies it like any gate; the result is the unnormalised
state of the approximated network.

The gate arithmetic has two interchangeable backends with the same pins: "numpy"
(tensordot per gate, new arrays) and "c" (sv.c: the same updates as in-place loops over
the amplitudes on every host core, for states of up to 30 qubits = 16 GiB).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .gates import ONEQ, companion_cut, fsim_tensor, gate_thetas

_HERE = os.path.dirname(os.path.abspath(__file__))
_SV_SRC = os.path.join(_HERE, "sv.c")
_SV_LIB = os.path.join(_HERE, "libsv.so")
_sv = None


def build_c(force: bool = False) -> str:
    """Compile sv.c into libsv.so next to it (gcc, OpenMP) unless it is up to date."""
    if force or not os.path.exists(_SV_LIB) or os.path.getmtime(_SV_LIB) < os.path.getmtime(_SV_SRC):
        tmp = _SV_LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SV_SRC], check=True)
        os.replace(tmp, _SV_LIB)
    return _SV_LIB


def _c_lib():
    global _sv
    if _sv is None:
        lib = ctypes.CDLL(build_c())
        p, i = ctypes.c_void_p, ctypes.c_int
        lib.sv_apply_1q.argtypes = [p, i, i, p]
        lib.sv_apply_2q.argtypes = [p, i, i, i, p]
        lib.sv_project.argtypes = [p, i, i, i]
        for f in (lib.sv_apply_1q, lib.sv_apply_2q, lib.sv_project):
            f.restype = None
        _sv = lib
    return _sv


class _CState:
    """Flat complex128 state updated in place by sv.c."""

    def __init__(self, n: int):
        self.n = n
        self.psi = np.zeros(1 << n, dtype=np.complex128)
        self.psi[0] = 1.0
        self.lib = _c_lib()

    def _ptr(self):
        return self.psi.ctypes.data_as(ctypes.c_void_p)

    def apply_1q(self, u: np.ndarray, q: int) -> None:
        m = np.ascontiguousarray(u, dtype=np.complex128)
        self.lib.sv_apply_1q(self._ptr(), self.n, q, m.ctypes.data_as(ctypes.c_void_p))

    def apply_2q(self, g: np.ndarray, qa: int, qb: int) -> None:
        m = np.ascontiguousarray(g, dtype=np.complex128).reshape(-1)
        self.lib.sv_apply_2q(self._ptr(), self.n, qa, qb, m.ctypes.data_as(ctypes.c_void_p))

    def project(self, q: int, v: int) -> None:
        self.lib.sv_project(self._ptr(), self.n, q, int(v))

    def flat(self) -> np.ndarray:
        return self.psi


class _NumpyState:
    """State of shape (2,)*n updated by the tensordot functions below."""

    def __init__(self, n: int):
        self.psi = np.zeros((2,) * n, dtype=np.complex128)
        self.psi[(0,) * n] = 1.0

    def apply_1q(self, u, q):
        self.psi = apply_1q(self.psi, u, q)

    def apply_2q(self, g, qa, qb):
        self.psi = apply_2q(self.psi, g, qa, qb)

    def project(self, q, v):
        self.psi = project(self.psi, q, v)

    def flat(self):
        return self.psi.reshape(-1)


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


def simulate(circuit: dict, projectors: dict | None = None, backend: str = "numpy") -> np.ndarray:
    """Final state |psi> = U|0^n> (flattened, length 2^n), optionally one slice of it."""
    n = circuit["n_qubits"]
    projectors = dict(projectors or {})
    if backend == "numpy":
        st = _NumpyState(n)
    elif backend == "c":
        st = _CState(n)
    else:
        raise ValueError(f"unknown backend {backend!r}")
    thetas = gate_thetas(circuit)
    phi = circuit["fsim"]["phi"]
    holes = set(int(h) for h in circuit.get("holes", ()))
    cuts = {int(g): int(q) for g, q in circuit.get("cuts", ())}
    n2q = [0] * n
    gate = 0
    for layer in circuit["layers"]:
        for q, name in enumerate(layer["oneq"]):
            st.apply_1q(ONEQ[name], q)
        for qa, qb in layer["couplers"]:
            if gate in holes:
                st.project(qa, 0)
                st.project(qb, 0)
            elif gate in cuts:
                if cuts[gate] not in (qa, qb):
                    raise ValueError(f"cut names qubit {cuts[gate]}, not one of gate {gate}'s")
                st.apply_2q(companion_cut(thetas[gate], phi, 0 if cuts[gate] == qa else 1), qa, qb)
            else:
                st.apply_2q(fsim_tensor(thetas[gate], phi), qa, qb)
            gate += 1
            for q in (qa, qb):
                key = (q, n2q[q])
                if key in projectors:
                    st.project(q, projectors[key])
                n2q[q] += 1
    return st.flat()


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
