"""Naive pairwise contraction of the circuit network (oracle; test infrastructure only).

Path format (Appendix E): a list of pairs (i, j); contracting tensors i and j puts the
result back at position i and retires j.  Every pair is one numpy.tensordot over the
labels the two tensors share.  Tensors still alive at the end are joined by outer
products in position order.

Sparse state (Appendix A): the oracle never uses sparse rows.  It loops over the
groups; for group i it projects every closed qubit's output leg onto that group's bit,
leaves the open legs open, contracts, and stores the 2^n_open results.

Slicing (Appendix B.2): for each slice id sigma, bit b of sigma is the value of the b-th
sliced bond; the network with those bonds fixed is contracted and the slice results are
summed in complex128 in the order the slice ids are given.
"""

from __future__ import annotations

import numpy as np

from .network import build_network


def _size(labels) -> int:
    return 1 << len(labels)


def greedy_path(labels: list[tuple], seed: int | None = None) -> list[tuple[int, int]]:
    """A simple greedy order: repeatedly contract the connected pair whose result
    grows memory the least (size(C) - size(A) - size(B)); ties go to the lowest index
    pair, or are broken by a seeded coin when `seed` is given."""
    rng = np.random.default_rng(seed) if seed is not None else None
    labs = {i: set(l) for i, l in enumerate(labels)}
    where: dict = {}
    for i, l in enumerate(labels):      # fixed label order: no dependence on string hashing
        for x in l:
            where.setdefault(x, set()).add(i)
    path = []
    while True:
        best, best_key = None, None
        for x, holders in where.items():
            if len(holders) != 2:
                continue
            i, j = sorted(holders)
            out = labs[i] ^ labs[j]
            cost = _size(out) - _size(labs[i]) - _size(labs[j])
            tie = rng.random() if rng is not None else 0.0
            key = (cost, tie, i, j)
            if best_key is None or key < best_key:
                best, best_key = (i, j), key
        if best is None:
            break
        i, j = best
        out = labs[i] ^ labs[j]
        for x in labs[j]:
            where[x].discard(j)
            if x in out:
                where[x].add(i)
        for x in labs[i] & labs[j]:
            where.pop(x, None)
        labs[i] = out
        del labs[j]
        path.append((i, j))
    return path


def random_greedy_path(labels: list[tuple], seed: int, trials: int = 20,
                       temperature: float = 0.5) -> list[tuple[int, int]]:
    """The greedy order of greedy_path with its cost perturbed: each candidate pair's
    memory growth gets temperature x (standard Gumbel noise) added, one pass per trial
    (seeded), and the pass with the smallest largest intermediate (then the fewest
    multiply-adds) is kept.  Any order gives the same contraction result; this one only
    keeps large networks within memory."""
    import math
    rng = np.random.default_rng(seed)
    best, best_key = None, None
    for _ in range(trials):
        labs = {i: set(l) for i, l in enumerate(labels)}
        where: dict = {}
        for i, l in enumerate(labels):  # fixed label order: the draws meet pairs in one order
            for x in l:
                where.setdefault(x, set()).add(i)
        path, peak, macs = [], 0, 0.0
        while True:
            pick, pick_key = None, None
            for x, holders in where.items():
                if len(holders) != 2:
                    continue
                i, j = sorted(holders)
                out = labs[i] ^ labs[j]
                cost = _size(out) - _size(labs[i]) - _size(labs[j])
                cost -= temperature * math.log(-math.log(rng.random()))
                if pick_key is None or cost < pick_key:
                    pick, pick_key = (i, j), cost
            if pick is None:
                break
            i, j = pick
            out = labs[i] ^ labs[j]
            macs += _size(labs[i] | labs[j])
            for x in labs[j]:
                where[x].discard(j)
                if x in out:
                    where[x].add(i)
            for x in labs[i] & labs[j]:
                where.pop(x, None)
            labs[i] = out
            del labs[j]
            peak = max(peak, len(out))
            path.append((i, j))
        key = (peak, macs)
        if best_key is None or key < best_key:
            best, best_key = path, key
    return best


def time_ordered_path(n_tensors: int) -> list[tuple[int, int]]:
    """Absorb the tensors one by one into tensor 0, in creation order."""
    return [(0, j) for j in range(1, n_tensors)]


def contract_path(tensors, labels, path, out_labels) -> np.ndarray:
    """Contract along `path`; return the result with axes in `out_labels` order."""
    ts = list(tensors)
    ls = [list(l) for l in labels]
    alive = [True] * len(ts)
    for i, j in path:
        if i == j or not (alive[i] and alive[j]):
            raise ValueError(f"invalid path step {(i, j)}")
        shared = [x for x in ls[i] if x in ls[j]]
        ai = [ls[i].index(x) for x in shared]
        aj = [ls[j].index(x) for x in shared]
        ts[i] = np.tensordot(ts[i], ts[j], axes=(ai, aj))
        ls[i] = [x for x in ls[i] if x not in shared] + [x for x in ls[j] if x not in shared]
        ts[j], alive[j] = None, False
    result, rl = None, []
    for k in range(len(ts)):
        if not alive[k]:
            continue
        if result is None:
            result, rl = ts[k], list(ls[k])
        else:
            result = np.tensordot(result, ts[k], axes=0)
            rl = rl + list(ls[k])
    if sorted(map(repr, rl)) != sorted(map(repr, out_labels)):
        raise ValueError(f"uncontracted labels {rl} differ from requested {list(out_labels)}")
    perm = [rl.index(x) for x in out_labels]
    return np.transpose(result, perm) if perm else result


def sparse_amplitudes(circuit: dict, open_qubits, closed_bits, sliced_bonds=(),
                      slice_ids=None, path: str | list = "greedy",
                      per_slice: bool = False) -> np.ndarray:
    """psi_hat[i][mu] for groups i (closed parts `closed_bits`, uint64 with bit n-1-q =
    s_q) and open configurations mu (first open qubit = most significant bit).

    sliced_bonds: bond names (q, j) whose values slice ids enumerate; slice_ids default
    to all 2^k.  With per_slice=True the result has a leading slice axis and nothing is
    summed.
    """
    n = circuit["n_qubits"]
    open_qubits = [int(q) for q in open_qubits]
    closed = [q for q in range(n) if q not in set(open_qubits)]
    k = len(sliced_bonds)
    if slice_ids is None:
        slice_ids = range(1 << k)
    slice_ids = [int(s) for s in slice_ids]
    no = len(open_qubits)
    shape = (len(slice_ids), len(closed_bits), 1 << no) if per_slice else (len(closed_bits), 1 << no)
    out = np.zeros(shape, dtype=np.complex128)
    cached_path = None
    for gi, cb in enumerate(closed_bits):
        values = {q: (int(cb) >> (n - 1 - q)) & 1 for q in closed}
        net = build_network(circuit, values)
        out_labels = [net.out_label[q] for q in open_qubits]
        for b in sliced_bonds:
            if tuple(b) not in net.bond_label:
                raise ValueError(f"{tuple(b)} is not a bond of this circuit")
        for si, sigma in enumerate(slice_ids):
            fixed = {net.bond_label[tuple(b)]: (sigma >> bi) & 1
                     for bi, b in enumerate(sliced_bonds)}
            tensors, labels = net.sliced(fixed)
            if isinstance(path, str):
                if cached_path is None:
                    if path == "greedy":
                        cached_path = greedy_path(labels)
                    elif path == "time":
                        cached_path = time_ordered_path(len(tensors))
                    elif path.startswith("random-greedy:"):
                        cached_path = random_greedy_path(labels, int(path.split(":")[1]))
                    else:
                        raise ValueError(path)
                p = cached_path
            else:
                p = path
            res = contract_path(tensors, labels, p, out_labels).reshape(-1)
            if per_slice:
                out[si, gi] = res
            else:
                out[gi] += res
    return out


def peak_size(labels, path) -> int:
    """Largest intermediate (elements) along a path - used to check a path is affordable."""
    ls = [set(l) for l in labels]
    peak = max((_size(l) for l in ls), default=1)
    for i, j in path:
        ls[i] = ls[i] ^ ls[j]
        ls[j] = set()
        peak = max(peak, _size(ls[i]))
    return peak
