"""Seeded target bitstrings and slice subsets.

Bit order: in a uint64 bitstring, bit (n-1-q) holds the value s_q of qubit q, so
qubit 0 is the most significant of the n bits.

Groups follow the sparse-state scheme of the supplement (section "Bitstrings choice"):
every group draws the bits of the closed qubits by coin flips and is joined with all
configurations of the open qubits.  Groups with an identical closed part are redrawn so
that all L*l requested bitstrings are distinct.
"""

from __future__ import annotations

import numpy as np


def bit_of(bits: int, n: int, q: int) -> int:
    return (int(bits) >> (n - 1 - q)) & 1


def bitstring_from_bits(values, n: int) -> int:
    out = 0
    for q, v in enumerate(values):
        if v:
            out |= 1 << (n - 1 - q)
    return out


def distinct_bitstrings(n: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct uniform n-bit strings (drawn without replacement), uint64."""
    if count > (1 << n):
        raise ValueError("more bitstrings requested than exist")
    rng = np.random.Generator(np.random.PCG64(seed))
    if n <= 24:
        pick = rng.choice(1 << n, size=count, replace=False)
        return np.asarray(pick, dtype=np.uint64)
    seen, out = set(), []
    while len(out) < count:
        v = int(rng.integers(0, 1 << n, dtype=np.uint64))
        if v not in seen:
            seen.add(v)
            out.append(v)
    return np.asarray(out, dtype=np.uint64)


def group_targets(n: int, open_qubits, L: int, seed: int) -> np.ndarray:
    """Closed parts of L groups (uint64; open-qubit bits are zero).

    Each closed qubit's bit is one coin flip, drawn in ascending qubit order; a group
    whose closed part repeats an earlier group is redrawn.
    """
    open_set = set(int(q) for q in open_qubits)
    closed = [q for q in range(n) if q not in open_set]
    if len(closed) < 63 and L > (1 << len(closed)):
        raise ValueError("more groups requested than closed configurations")
    rng = np.random.Generator(np.random.PCG64(seed))
    seen, out = set(), []
    while len(out) < L:
        flips = rng.integers(0, 2, size=len(closed))
        v = 0
        for q, f in zip(closed, flips):
            if f:
                v |= 1 << (n - 1 - q)
        if v not in seen:
            seen.add(v)
            out.append(v)
    return np.asarray(out, dtype=np.uint64)


def slice_subset(k: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct slice ids out of 2**k, uniform without replacement, ascending.

    For k > 62 every id is k coin flips (bit b = flip b), repeats redrawn, and the ids are
    returned as Python ints in an object array."""
    if k > 62:
        rng = np.random.Generator(np.random.PCG64(seed))
        seen = set()
        while len(seen) < count:
            flips = rng.integers(0, 2, size=k)
            seen.add(sum(int(f) << b for b, f in enumerate(flips)))
        return np.array(sorted(seen), dtype=object)
    total = 1 << k
    if count >= total:
        return np.arange(total, dtype=np.uint64)
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.choice(total, size=count, replace=False)
    return np.sort(np.asarray(pick, dtype=np.uint64))
