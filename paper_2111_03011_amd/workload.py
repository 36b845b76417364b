"""Seeded workloads: circuit -> network -> plan -> targets, for each configuration."""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import synth

from .network import TensorNetwork, circuit_network
from .planner import (Plan, find_plan, make_problem, merge_branches, order_for_reuse, path_cost,
                      zigzag_plan)


@dataclass
class Workload:
    name: str
    circuit: dict
    net: TensorNetwork
    open_qubits: list
    closed_bits: np.ndarray
    plan: Plan
    slice_ids: np.ndarray

    @property
    def sliced_bonds(self):
        """Sliced labels as bond names (q, j), in slice-bit order."""
        inv = {lab: key for key, lab in self.net.bond_label.items()}
        return [inv[x] for x in self.plan.sliced_labels]

    @property
    def n_amplitudes(self) -> int:
        return len(self.closed_bits) << len(self.open_qubits)


def make_workload(circuit: dict, open_qubits, closed_bits, max_log2: float = 26,
                  n_sliced=None, slice_ids=None, trials: int = 4, seed: int = 0,
                  name: str = "custom", reuse_batch: int = 1) -> Workload:
    net = circuit_network(circuit)
    plan = find_plan(net, open_qubits, closed_bits, max_log2=max_log2, n_sliced=n_sliced,
                     trials=trials, seed=seed, reuse_batch=reuse_batch)
    if slice_ids is None:
        if len(plan.sliced_labels) > 24:
            raise ValueError("too many slices to enumerate; pass a slice subset")
        slice_ids = np.arange(plan.n_slices, dtype=np.uint64)
    ids = (np.asarray(slice_ids, dtype=np.uint64) if len(plan.sliced_labels) <= 62
           else np.asarray(slice_ids, dtype=object))
    return Workload(name, circuit, net, list(open_qubits), np.asarray(closed_bits, np.uint64),
                    plan, ids)


def make_zigzag_workload(circuit: dict, open_qubits, closed_bits, tail_start: int,
                         max_log2: float = 26, reuse_batch: int = 1, trials: int = 4,
                         seed: int = 0, name: str = "zigzag") -> Workload:
    """Workload along a head-tail plan with the zigzag tail (planner.zigzag_plan), every
    slice id enumerated.  reuse_batch > 1 then orders its sliced labels for head reuse
    (order_for_reuse): the log2(reuse_batch) local labels on the low id bits, steps that
    do not depend on them computed once per batch."""
    net = circuit_network(circuit)
    plan = zigzag_plan(net, open_qubits, closed_bits, tail_start, max_log2, trials=trials,
                       seed=seed)
    if reuse_batch > 1:
        plan = order_for_reuse(net, plan, open_qubits, closed_bits, reuse_batch)
    if len(plan.sliced_labels) > 24:
        raise ValueError("too many slices to enumerate")
    return Workload(name, circuit, net, list(open_qubits), np.asarray(closed_bits, np.uint64),
                    plan, np.arange(plan.n_slices, dtype=np.uint64))


def choose_holes(circuit: dict, n_holes: int, open_qubits, closed_bits, max_log2: float = 26,
                 n_sliced=None, first_cycle: int | None = None, last_cycle: int | None = None,
                 seed: int = 0) -> list:
    """Hole positions for the perturbed network (Method: holes are placed so that the
    perturbed network is much cheaper to contract).  Greedy: each round drills the
    two-qubit gate, among those of cycles [first_cycle, last_cycle) (default: the middle
    third), whose network has the lowest planned total flops (one greedy path per
    candidate, same size bound and slice count)."""
    layers = circuit["layers"]
    m = len(layers)
    c0 = m // 3 if first_cycle is None else first_cycle
    c1 = (2 * m) // 3 if last_cycle is None else last_cycle
    starts = np.cumsum([0] + [len(l["couplers"]) for l in layers])
    cands = [g for c in range(c0, c1) for g in range(int(starts[c]), int(starts[c + 1]))]
    holes = []
    for _ in range(n_holes):
        best = None
        for g in cands:
            if g in holes:
                continue
            c = dict(circuit)
            c["holes"] = sorted(holes + [g])
            try:
                plan = find_plan(circuit_network(c), open_qubits, closed_bits, max_log2=max_log2,
                                 n_sliced=n_sliced, trials=1, seed=seed)
            except RuntimeError:
                continue
            if best is None or plan.total_flops < best[0]:
                best = (plan.total_flops, g)
        if best is None:
            break
        holes.append(best[1])
    return sorted(holes)


_CACHE = {}


def config_workload(name: str, mode: str = "default", trials: int | None = None) -> Workload:
    """name: small | sliced | large.  For small, mode 'amplitudes' (64 bitstrings, no open
    qubit) or 'samples' (all 12 qubits open, one group).  For large, mode 'reuse' keeps the
    plan's sliced bonds, puts the log2(reuse_batch) cheapest on the low id bits and draws
    the slice subset as subtasks of reuse_batch consecutive ids.  For sliced, mode 'reuse' plans
    for head reuse (bound-driven global slices, cheap local ones on the low slice-id bits,
    steps above global labels once per batch of the configuration's reuse_batch), and mode
    'holes' drills the configuration's number of holes (chosen by choose_holes) into the
    circuit, a perturbed network with fidelity about 2^-K (K = 2 per hole).  For sliced and
    large, mode 'branch' is the default plan with its path branch-merged (merge_branches;
    same sliced bonds and slices); large's 'reuse' mode starts from that merged path too.
    trials
    defaults to the configuration's plan_trials.  Plans are deterministic and memoised per
    process."""
    key = (name, mode, trials)
    if key not in _CACHE:
        _CACHE[key] = _config_workload(name, mode, trials)
    return _CACHE[key]


def _config_workload(name: str, mode: str, trials: int | None) -> Workload:
    cfg = synth.config(name)
    if trials is None:
        trials = cfg.get("plan_trials", 4)
    circuit = synth.circuit_from_config(cfg)
    n = circuit["n_qubits"]
    if name == "small":
        if mode == "samples":
            open_q, closed = list(range(n)), np.zeros(1, np.uint64)
        else:
            a = cfg["amplitudes"]
            open_q, closed = [], synth.distinct_bitstrings(n, a["count"], a["seed"])
        return make_workload(circuit, open_q, closed, max_log2=cfg["max_log2_size"],
                             n_sliced=None, trials=trials, seed=cfg["path_seed"], name=name)
    open_q = cfg["open_qubits"]
    g = cfg["groups"]
    closed = synth.group_targets(n, open_q, g["L"], g["seed"])
    if mode == "holes":
        circuit = dict(circuit)
        circuit["holes"] = choose_holes(circuit, cfg["holes"], open_q, closed,
                                        max_log2=cfg["max_log2_size"],
                                        n_sliced=cfg.get("sliced_labels"), seed=cfg["path_seed"])
    net = circuit_network(circuit)
    plan = find_plan(net, open_q, closed, max_log2=cfg["max_log2_size"],
                     n_sliced=cfg.get("sliced_labels"), trials=trials, seed=cfg["path_seed"],
                     reuse_batch=cfg.get("reuse_batch", 1) if mode == "reuse" else 1)
    if mode == "branch" or (mode == "reuse" and name == "large"):
        plan = merge_branches(net, plan, open_q, closed)
    k = len(plan.sliced_labels)
    if "slice_subset" in cfg and mode == "reuse":
        # subtasks (Method): count / B random assignments of the global labels, each with all
        # B values of the local labels, which sit on the low id bits
        b = cfg["reuse_batch"]
        plan = order_for_reuse(net, plan, open_q, closed, b)
        n_loc = b.bit_length() - 1
        sub = cfg["slice_subset"]
        glob = synth.slice_subset(k - n_loc, sub["count"] // b, sub["seed"])
        ids = [(int(g) << n_loc) | loc for g in glob for loc in range(b)]
    elif "slice_subset" in cfg:
        sub = cfg["slice_subset"]
        ids = synth.slice_subset(k, sub["count"], sub["seed"])
    else:
        ids = np.arange(plan.n_slices, dtype=np.uint64)
    ids = np.asarray(ids, dtype=np.uint64) if k <= 62 else np.asarray(ids, dtype=object)
    return Workload(name, circuit, net, list(open_q), np.asarray(closed, np.uint64), plan, ids)


def jittered_twin(w: Workload, theta_jitter: float, jitter_seed: int) -> Workload:
    """The same workload with one fSim angle per gate drawn around the circuit's angle (see
    synth.make_circuit): same network structure, hence the same path, slicing, slice ids
    and targets; only the gate entries differ."""
    import dataclasses
    c = synth.with_theta_jitter(w.circuit, theta_jitter, jitter_seed)
    net = circuit_network(c)
    if net.labels != w.net.labels:
        raise RuntimeError("the jittered network's structure differs from the workload's")
    return dataclasses.replace(w, circuit=c, net=net)


def zigzag_pair(w: Workload, tail_start: int, max_log2: float, count: int, seed: int,
                trials: int = 4):
    """A zigzag plan of the workload's network (planner.zigzag_plan) that slices the
    workload's bonds first (on the same low id bits) and further bonds as its own bound needs
    (on the bits above), and the workload's own path put on that same slicing, so that both
    sum the same slices.  Slice ids: the workload's ids with `count` seeded draws of the
    further bits.  Returns (zigzag workload, plain-path workload)."""
    import dataclasses
    base = list(w.plan.sliced_labels)
    zz = zigzag_plan(w.net, w.open_qubits, w.closed_bits, tail_start, max_log2,
                     base_sliced=base, trials=trials, seed=seed)
    sliced = zz.sliced_labels
    n_extra = len(sliced) - len(base)
    net = w.net
    sp = make_problem(net.labels, net.out_label, net.n_qubits, w.open_qubits, w.closed_bits,
                      sliced=sliced)
    leaves = {k for k, l in enumerate(net.labels) if any(x in sliced for x in l)}
    xs = synth.slice_subset(n_extra, count, seed)
    ids = [int(w.slice_ids[i % len(w.slice_ids)]) | (int(x) << len(base)) for i, x in enumerate(xs)]
    ids = np.asarray(ids, dtype=np.uint64 if len(sliced) <= 62 else object)
    plain = Plan(path=w.plan.path, sliced_labels=sliced, cost=path_cost(sp, w.plan.path, leaves),
                 n_slices=1 << len(sliced))
    if plain.cost.peak_log2 > max_log2 + 1e-9:
        raise RuntimeError("the workload's path exceeds the size bound on the zigzag slicing")
    return (dataclasses.replace(w, plan=zz, slice_ids=ids),
            dataclasses.replace(w, plan=plain, slice_ids=ids))


def companion_cuts(circuit: dict, sliced_bonds, max_cuts: int | None = None) -> list:
    """Companion-edge cuts [g, q] for sliced bonds (Method, low-rank case (ii)): a sliced
    bond (q, j) is the input on q of the next two-qubit gate g on q; its companion edge is
    g's output on the other qubit, which must be a bond (a later gate on that qubit) and not
    sliced itself.  Bonds are taken in the given order; a cut whose edges would collide with
    an earlier cut's (one's pinned edge the other's companion), or that simplification of
    the network would contract away, is skipped."""
    layers = circuit["layers"]
    holes = set(int(h) for h in circuit.get("holes", ()))
    on = {}                     # qubit -> gate indices in order
    pair = []
    g = 0
    for layer in layers:
        for qa, qb in layer["couplers"]:
            on.setdefault(qa, []).append(g)
            on.setdefault(qb, []).append(g)
            pair.append((qa, qb))
            g += 1
    sliced = {tuple(b) for b in sliced_bonds}
    cuts, pinned, comps = [], set(), set()
    for q, j in sliced_bonds:
        if max_cuts is not None and len(cuts) >= max_cuts:
            break
        if j + 1 >= len(on.get(q, ())):
            continue
        gate = on[q][j + 1]
        qa, qb = pair[gate]
        other = qb if q == qa else qa
        jo = on[other].index(gate)
        comp = (other, jo)
        if gate in holes or any(c[0] == gate for c in cuts) or jo + 1 >= len(on[other]):
            continue
        if comp in sliced or comp in pinned or (q, j) in comps:
            continue
        trial = cuts + [[gate, q]]
        try:
            circuit_network(dict(circuit, cuts=trial))
        except ValueError:
            continue
        cuts = trial
        pinned.add((q, j))
        comps.add(comp)
    return cuts


def companion_workload(w: Workload, cuts) -> Workload:
    """The workload with companion-edge cuts: the circuit lists `cuts`, the network folds
    the pinned bonds' single-qubit gates into the earlier gate, and each cut's companion
    label is sliced on a new high slice-id bit that copies its pinned bond's bit in every
    id (so each slice fixes both edges to the same value, and the slice set is the same
    size).  Same path; the planner's cost counts both edges as sliced."""
    import dataclasses
    circ = dict(w.circuit, cuts=[list(c) for c in cuts])
    net = circuit_network(circ)
    if net.labels != w.net.labels:
        raise RuntimeError("the cut network's structure differs from the workload's")
    base = list(w.plan.sliced_labels)
    pos = {x: i for i, x in enumerate(base)}
    if any(b not in pos for b, _ in net.cut_pairs):
        raise ValueError("every cut must pin one of the plan's sliced bonds")
    k = len(base)
    sliced = base + [c for _, c in net.cut_pairs]
    ids = []
    for sid in w.slice_ids:
        x = int(sid)
        for t, (b, _) in enumerate(net.cut_pairs):
            x |= ((x >> pos[b]) & 1) << (k + t)
        ids.append(x)
    ids = np.asarray(ids, dtype=np.uint64 if len(sliced) <= 62 else object)
    sp = make_problem(net.labels, net.out_label, net.n_qubits, w.open_qubits, w.closed_bits,
                      sliced=sliced)
    leaves = {i for i, l in enumerate(net.labels) if any(x in sliced for x in l)}
    plan = Plan(path=w.plan.path, sliced_labels=sliced, cost=path_cost(sp, w.plan.path, leaves),
                n_slices=len(ids))
    return dataclasses.replace(w, circuit=circ, net=net, plan=plan, slice_ids=ids)


def serving_template(seed: int, max_log2: float = 26, work_cap: float = 2e13,
                     max_tries: int = 50, branch_merge: bool = True):
    """One request of the serving stream, planned by the client ahead of time.

    Draws (seeded) n in [20, 36] qubits on a near-square grid (floor(sqrt n) rows, trailing
    sites of the last row removed), m in [10, 16] cycles, a kind (amplitudes: 2^[8, 16]
    bitstrings as groups of 64; samples: k in [1e3, 1e5], one group of 64 per sample) and
    2^[4, 12] slices; draws are repeated until a plan meets the size bound with that slice
    count and its total work stays below `work_cap` flops.  The accepted plan's path is then
    branch-merged (merge_branches; same slices), unless `branch_merge` is false, so the
    stream's requests do not depend on it.  Returns (Workload, n_samples).
    """
    import math
    rng = np.random.Generator(np.random.PCG64(seed))
    for attempt in range(max_tries):
        n = int(rng.integers(20, 37))
        m = int(rng.integers(10, 17))
        samples = bool(rng.random() < 0.5)
        if samples:
            k = int(10 ** rng.uniform(3, 5))
            L = k
        else:
            L = (1 << int(rng.integers(8, 17))) // 64
            k = 0
        ks = int(rng.integers(4, 13))
        r = math.isqrt(n)
        cols = -(-n // r)
        removed = [[r - 1, c] for c in range(cols) if (r - 1) * cols + c >= n]
        circ = synth.make_circuit(r, cols, m, seed * 100 + attempt, removed=removed)
        open_q = sorted(int(q) for q in rng.choice(n, 6, replace=False))
        closed = synth.group_targets(n, open_q, L, seed * 100 + attempt + 1)
        try:
            w = make_workload(circ, open_q, closed, max_log2=max_log2, n_sliced=ks, trials=2,
                              seed=seed, name=f"request-{seed}")
        except RuntimeError:
            continue
        if w.plan.total_flops <= work_cap:
            if branch_merge:
                import dataclasses
                w = dataclasses.replace(w, plan=merge_branches(w.net, w.plan, open_q, closed))
            return w, k
    raise RuntimeError("no request met the size bound and the work cap")
