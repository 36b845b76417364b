"""Contraction planning: path, sliced bonds and cost (host side of the library).

Paper, "Method" and Appendix B.2: the network is contracted pairwise along an order
found by a complexity-greedy search; slicing fixes chosen bonds so that the largest
intermediate fits the device, and every fixed assignment (a slice) is an independent
contraction whose results are summed.  Appendix A: tensors that carry final-state
qubits only keep the configurations that some requested bitstring needs.

Cost model.  A tensor carries dense labels (bond dimension 2 each) and a set Q of closed
final qubits.  Its row count is the number of distinct restrictions of the requested
closed parts to Q (1 when Q is empty), so its size in elements is rows(Q) * 2^|dense|.
Contracting A and B costs rows(Q_A | Q_B) * 2^|dense_A | dense_B| complex multiply-adds,
the paper's time complexity T_c (Table I); flops are 8 T_c.

Search.  Greedy: repeatedly contract the pair of tensors sharing a label that minimises
size(C) - size(A) - size(B); the randomised variant adds Gumbel noise scaled by a
temperature.  Slicing: bonds are added one at a time, each time the one that lowers the
largest intermediate while raising the total cost least, until the size bound (and,
when asked, an exact count) is met; the path is then searched again on the sliced
network.  Steps that touch no sliced leaf are the same in every slice; the objective
counts them once.

Head reuse (Method; Appendix B.2: the head is contracted once per subtask and reused by
all of its slices).  With `reuse_batch` = B > 1 the bonds the size bound needs are sliced
first (global labels); the remaining ones are local labels, chosen one at a time to
minimise the per-slice work when every step that depends on global labels only is
computed once per batch of B slices.  Local labels take the low bits of the slice id, so
consecutive slice ids differ only in them and the library shares those steps.

Branch merging (Results, the contraction of the 53-qubit circuits; Table I's two T_c
columns).  Along a stem (a chain of steps in which one large tensor absorbs smaller ones),
consecutive absorbed tensors are first contracted with each other into a branch, which
the stem then absorbs in one step (neighbouring absorptions may also trade places first).  The stem is read and written once per branch instead
of once per absorbed tensor, at the price of more flops (each merged step has larger K
and N): worth it where the separate steps are bound by memory bandwidth.  branch_merge
chooses the groups by dynamic programming over each stem against a roofline time model
of one step; the intermediates of the stem that remain are the original ones and branches
stay under their own size bound (by default the plan's peak), so the peak never grows.

Path format (Appendix E): pairs (i, j); the result is stored at position i.
"""

from __future__ import annotations

import heapq
import math
from dataclasses import dataclass, field

import numpy as np


def _popcount(x: int) -> int:
    return bin(x).count("1")


class RowCounter:
    """rows(Q): number of distinct closed-bit restrictions to the qubit mask Q.

    Counted exactly for up to `exact_limit` groups; above that the planner uses the bound
    min(L, 2^|Q|), which never underestimates, so a plan that meets the size bound with it
    also meets it with the library's exact row counts."""

    def __init__(self, n_qubits: int, closed_bits, exact_limit: int = 1 << 14):
        self.n = n_qubits
        self.bits = np.asarray(closed_bits, dtype=np.uint64)
        self.exact = self.bits.size <= exact_limit
        self.cache = {0: 1}

    def qmask(self, qubits) -> int:
        m = 0
        for q in qubits:
            m |= 1 << (self.n - 1 - q)
        return m

    def __call__(self, mask: int) -> int:
        r = self.cache.get(mask)
        if r is None:
            if self.bits.size <= 1:
                r = 1
            elif not self.exact:
                r = int(min(self.bits.size, 1 << min(62, _popcount(mask))))
            else:
                r = int(np.unique(self.bits & np.uint64(mask)).size)
            self.cache[mask] = r
        return r


@dataclass
class Problem:
    """Labels as bitsets; closed output legs turned into row masks; sliced labels dropped."""
    dense: list            # per leaf: int bitset of dense label ids
    qmask: list            # per leaf: int bit mask (bitstring positions) of closed qubits
    rows: RowCounter
    label_ids: list        # bit position -> original label

    def size(self, dense: int, q: int) -> int:
        return self.rows(q) << _popcount(dense)


def make_problem(labels, out_label, n_qubits, open_qubits, closed_bits, sliced=()) -> Problem:
    all_labels = sorted({x for l in labels for x in l})
    pos = {x: i for i, x in enumerate(all_labels)}
    open_set = set(int(q) for q in open_qubits)
    closed_leg = {out_label[q]: q for q in range(n_qubits) if q not in open_set}
    rows = RowCounter(n_qubits, closed_bits)
    sl = set(sliced)
    dense, qm = [], []
    for l in labels:
        d, m = 0, 0
        for x in l:
            if x in closed_leg:
                m |= 1 << (n_qubits - 1 - closed_leg[x])
            elif x not in sl:
                d |= 1 << pos[x]
        dense.append(d)
        qm.append(m)
    return Problem(dense=dense, qmask=qm, rows=rows, label_ids=all_labels)


@dataclass
class PathCost:
    flops_per_slice: float = 0.0     # 8 T_c of slice-dependent steps
    flops_invariant: float = 0.0     # 8 T_c of steps shared by all slices
    peak_log2: float = 0.0
    steps: list = field(default_factory=list)   # (i, j, rows, log2 dense A, B, C, macs, dep)
    flops_shared: float = 0.0        # part of flops_per_slice computed once per batch
    batch: int = 1                   # slices per batch the shared part is counted for

    def total(self, n_slices: int) -> float:
        n_batches = -(-n_slices // max(1, self.batch))
        return (self.flops_invariant + n_slices * (self.flops_per_slice - self.flops_shared)
                + n_batches * self.flops_shared)


def greedy_path(prob: Problem, temperature: float = 0.0, seed: int = 0):
    """Pairs (i, j) contracting every connected component; leftovers joined at the end."""
    rng = np.random.default_rng(seed)
    n = len(prob.dense)
    dense = list(prob.dense)
    qm = list(prob.qmask)
    alive = [True] * n
    holders = {}
    for i, d in enumerate(dense):
        x = d
        while x:
            b = x & -x
            holders.setdefault(b, set()).add(i)
            x ^= b
    # closed-qubit rows also link tensors (they must end in the same result)
    heap = []
    version = [0] * n

    def score(i, j):
        c = prob.size(dense[i] ^ dense[j], qm[i] | qm[j])
        s = c - prob.size(dense[i], qm[i]) - prob.size(dense[j], qm[j])
        if temperature > 0:
            g = -math.log(-math.log(rng.random() + 1e-300) + 1e-300)
            s = s - temperature * abs(s + 1) * g
        return s

    def push(i, j):
        if i > j:
            i, j = j, i
        heapq.heappush(heap, (score(i, j), i, j, version[i], version[j]))

    for b, hs in holders.items():
        hs = sorted(hs)
        if len(hs) == 2:
            push(hs[0], hs[1])
    path = []
    while heap:
        s, i, j, vi, vj = heapq.heappop(heap)
        if not (alive[i] and alive[j]) or vi != version[i] or vj != version[j]:
            continue
        shared = dense[i] & dense[j]
        new = dense[i] ^ dense[j]
        # move j's non-shared labels to i
        x = dense[j]
        while x:
            b = x & -x
            holders[b].discard(j)
            if not (b & shared):
                holders[b].add(i)
            x ^= b
        x = shared
        while x:
            b = x & -x
            holders[b].discard(i)
            x ^= b
        dense[i], qm[i] = new, qm[i] | qm[j]
        alive[j] = False
        version[i] += 1
        path.append((i, j))
        nbrs = set()
        x = new
        while x:
            b = x & -x
            nbrs |= holders[b]
            x ^= b
        nbrs.discard(i)
        for k in nbrs:
            if alive[k]:
                push(i, k)
    rest = [k for k in range(n) if alive[k]]
    # join what is left (disconnected pieces, row-only tensors): smallest first
    rest.sort(key=lambda k: prob.size(dense[k], qm[k]))
    while len(rest) > 1:
        i, j = rest[0], rest[1]
        dense[i] ^= dense[j]
        qm[i] |= qm[j]
        path.append((i, j))
        rest = [i] + rest[2:]
        rest.sort(key=lambda k: prob.size(dense[k], qm[k]))
    return path


def path_cost(prob: Problem, path, sliced_leaves=None) -> PathCost:
    """Cost of a path; `sliced_leaves` = leaf indices holding a sliced label (the steps
    above them differ between slices)."""
    dense = list(prob.dense)
    qm = list(prob.qmask)
    dep = [bool(sliced_leaves and k in sliced_leaves) for k in range(len(dense))]
    out = PathCost()
    peak = max((prob.size(d, q) for d, q in zip(dense, qm)), default=1)
    for i, j in path:
        union = dense[i] | dense[j]
        qc = qm[i] | qm[j]
        rows = prob.rows(qc)
        macs = float(rows) * float(1 << _popcount(union))
        d = dep[i] or dep[j]
        if d:
            out.flops_per_slice += 8.0 * macs
        else:
            out.flops_invariant += 8.0 * macs
        out.steps.append((i, j, rows, _popcount(dense[i]), _popcount(dense[j]),
                          _popcount(dense[i] ^ dense[j]), macs, d))
        dense[i] ^= dense[j]
        qm[i] = qc
        dep[i] = d
        peak = max(peak, prob.size(dense[i], qc))
    out.peak_log2 = math.log2(peak)
    return out


def _intermediates(prob: Problem, path):
    """(dense bitset, qmask) of every intermediate, leaves included."""
    dense = list(prob.dense)
    qm = list(prob.qmask)
    items = list(zip(dense, qm))
    for i, j in path:
        dense[i] ^= dense[j]
        qm[i] |= qm[j]
        items.append((dense[i], qm[i]))
    return items


def _step_operands(prob: Problem, path):
    """Per step: (dense A | dense B, q mask of C) -- what decides its cost."""
    dense = list(prob.dense)
    qm = list(prob.qmask)
    out = []
    for i, j in path:
        out.append((dense[i] | dense[j], qm[i] | qm[j], dense[i] ^ dense[j]))
        dense[i] ^= dense[j]
        qm[i] |= qm[j]
    return out


def choose_slices(prob: Problem, path, max_log2: float, exact: int | None = None,
                  forbidden: int = 0):
    """Bond bits to slice along a fixed path (greedy): returns a bitset of label bits.

    Each round adds the bond that, once sliced, gives the smallest largest intermediate
    (while the bound is not met) and then the smallest total cost over all slices.  Slicing
    bond b halves every intermediate and every step that carries b, so both figures are
    computed for all candidates at once from incidence matrices."""
    ops = _step_operands(prob, path)
    counts = {}
    for d in prob.dense:
        x = d
        while x:
            b = x & -x
            counts[b] = counts.get(b, 0) + 1
            x ^= b
    cands = [b for b, c in counts.items() if c == 2 and not (b & forbidden)]
    if not cands:
        return 0, max((math.log2(prob.rows(q)) + _popcount(d) for d, q in zip(prob.dense, prob.qmask)), default=0.0)
    inter = list(zip(prob.dense, prob.qmask)) + [(out, q) for _, q, out in ops]
    O = np.array([[bool(d & b) for b in cands] for d, _ in inter], dtype=np.float64)
    U = np.array([[bool(u & b) for b in cands] for u, _, _ in ops], dtype=np.float64)
    ls = np.array([math.log2(prob.rows(q)) + _popcount(d) for d, q in inter])
    lc = np.array([math.log2(prob.rows(q)) + _popcount(u) for u, q, _ in ops])
    taken = np.zeros(len(cands), dtype=bool)
    chosen, k = 0, 0
    cur_peak = float(ls.max())
    while True:
        need_more = cur_peak > max_log2 + 1e-9 or (exact is not None and k < exact)
        if not need_more or (exact is not None and k >= exact) or taken.all():
            break
        ct = np.exp2(lc)
        new_cost = (2.0 ** (k + 1)) * (ct.sum() - 0.5 * (ct @ U))
        new_peak = (ls[:, None] - O).max(axis=0)
        first = np.maximum(new_peak, max_log2) if cur_peak > max_log2 + 1e-9 else np.zeros_like(new_peak)
        first = np.where(taken, np.inf, first)
        order = np.lexsort((new_peak, new_cost, first))
        c = int(order[0])
        chosen |= cands[c]
        taken[c] = True
        ls = ls - O[:, c]
        lc = lc - U[:, c]
        k += 1
        cur_peak = float(ls.max())
    return chosen, cur_peak


def _subtree_labels(prob: Problem, path):
    """Per step: OR of the dense bitsets of the leaves under it (with sliced labels, when
    `prob` is the unsliced problem)."""
    acc = list(prob.dense)
    out = []
    for i, j in path:
        acc[i] |= acc[j]
        out.append(acc[i])
    return out


def choose_local_slices(prob: Problem, path, global_bits: int, n_local: int, batch: int,
                        max_log2: float, forbidden: int = 0):
    """Add n_local bonds (local labels) to the globally sliced set, one at a time, each the
    one that minimises the per-slice work when steps above global labels only are shared by
    a batch of min(batch, 2^(local labels so far)) slices, under the size bound.
    Returns the list of chosen bond bits in order, or None when the bound cannot be met."""
    ops = _step_operands(prob, path)
    sub = _subtree_labels(prob, path)
    counts = {}
    for d in prob.dense:
        x = d
        while x:
            b = x & -x
            counts[b] = counts.get(b, 0) + 1
            x ^= b
    cands = [b for b, c in counts.items() if c == 2 and not (b & forbidden) and not (b & global_bits)]
    if len(cands) < n_local:
        return None
    inter = list(zip(prob.dense, prob.qmask)) + [(out, q) for _, q, out in ops]
    O = np.array([[bool(d & b) for b in cands] for d, _ in inter], dtype=np.float64)
    U = np.array([[bool(u & b) for b in cands] for u, _, _ in ops], dtype=np.float64)
    Dl = np.array([[bool(t & b) for b in cands] for t in sub], dtype=bool)
    g_of = lambda x: _popcount(x & global_bits)
    ls = np.array([math.log2(prob.rows(q)) + _popcount(d) - g_of(d) for d, q in inter])
    lc = np.array([math.log2(prob.rows(q)) + _popcount(u) - g_of(u) for u, q, _ in ops])
    dep_g = np.array([bool(t & global_bits) for t in sub])
    local_dep = np.zeros(len(ops), dtype=bool)
    chosen = []
    taken = np.zeros(len(cands), dtype=bool)
    for k in range(n_local):
        share = float(min(batch, 2 ** (k + 1)))
        best = None
        macs_all = np.exp2(lc[:, None] - U)          # step cost with each candidate sliced
        peak_all = (ls[:, None] - O).max(axis=0)
        ldep = local_dep[:, None] | Dl                # steps that depend on a local label
        shared = (~ldep) & dep_g[:, None]
        eff = (macs_all * ldep).sum(axis=0) + (macs_all * shared).sum(axis=0) / share
        eff = np.where(taken | (peak_all > max_log2 + 1e-9), np.inf, eff)
        c = int(np.argmin(eff))
        if not np.isfinite(eff[c]):
            return None
        chosen.append(cands[c])
        taken[c] = True
        ls = ls - O[:, c]
        lc = lc - U[:, c]
        local_dep |= Dl[:, c]
    return chosen


def reuse_cost(prob_sliced: Problem, path, leaf_local, leaf_global, batch: int) -> PathCost:
    """PathCost with the steps that depend on global sliced leaves only marked as shared by
    a batch (leaf_local / leaf_global: leaves holding a local / global sliced label)."""
    cost = path_cost(prob_sliced, path, leaf_local | leaf_global)
    loc = [k in leaf_local for k in range(len(prob_sliced.dense))]
    for (i, j), st in zip(path, cost.steps):
        loc[i] = loc[i] or loc[j]
        if st[7] and not loc[i]:
            cost.flops_shared += 8.0 * st[6]
    cost.batch = batch
    return cost


@dataclass
class Plan:
    path: list
    sliced_labels: list
    cost: PathCost
    n_slices: int

    @property
    def total_flops(self) -> float:
        return self.cost.total(self.n_slices)


def find_plan(net, open_qubits, closed_bits, max_log2: float = 26.0,
              n_sliced: int | None = None, trials: int = 16, seed: int = 0,
              temperature: float = 0.05, rounds: int = 2, reuse_batch: int = 1) -> Plan:
    """Random-greedy search of (path, sliced bonds) under the size bound.

    n_sliced=None slices as few bonds as the bound needs; an int asks for exactly that
    many.  reuse_batch > 1 (with n_sliced) also tries head reuse: bound-driven global
    slices plus local ones (low slice-id bits), steps above global labels counted once per
    batch of reuse_batch slices.  Returns the plan with the lowest total flop count over
    the slices (steps shared by all slices counted once)."""
    n = net.n_qubits
    base = make_problem(net.labels, net.out_label, n, open_qubits, closed_bits)
    bond_bits = 0
    pos = {x: i for i, x in enumerate(base.label_ids)}
    bond_labels = set(net.bond_label.values())
    for x in base.label_ids:
        if x in bond_labels:
            bond_bits |= 1 << pos[x]
    forbidden = ((1 << len(base.label_ids)) - 1) & ~bond_bits
    best = None
    for t in range(trials):
        temp = 0.0 if t == 0 else temperature
        path = greedy_path(base, temperature=temp, seed=seed + 7919 * t)
        path0 = path
        sl = 0
        for _ in range(rounds):
            need_exact = n_sliced
            sl, pk = choose_slices(base, path, max_log2, exact=need_exact, forbidden=forbidden)
            sliced_prob = make_problem(net.labels, net.out_label, n, open_qubits, closed_bits,
                                       sliced=[base.label_ids[i] for i in range(len(base.label_ids))
                                               if (sl >> i) & 1])
            path2 = greedy_path(sliced_prob, temperature=temp, seed=seed + 104729 * t + 1)
            c1 = path_cost(sliced_prob, path)
            c2 = path_cost(sliced_prob, path2)
            if c2.peak_log2 <= max_log2 + 1e-9 and (c1.peak_log2 > max_log2 + 1e-9 or
                                                   c2.flops_per_slice < c1.flops_per_slice):
                path = path2
        sliced = [base.label_ids[i] for i in range(len(base.label_ids)) if (sl >> i) & 1]
        if n_sliced is not None and len(sliced) != n_sliced:
            continue
        sp = make_problem(net.labels, net.out_label, n, open_qubits, closed_bits, sliced=sliced)
        sliced_leaves = {k for k, l in enumerate(net.labels) if any(x in sliced for x in l)}
        cost = path_cost(sp, path, sliced_leaves)
        if cost.peak_log2 > max_log2 + 1e-9:
            continue
        cand = Plan(path=path, sliced_labels=sliced, cost=cost, n_slices=1 << len(sliced))
        if best is None or cand.total_flops < best.total_flops:
            best = cand
        if reuse_batch > 1 and n_sliced:
            for p in (path0, path):
                rc = _reuse_candidate(net, base, p, open_qubits, closed_bits, max_log2, n_sliced,
                                      reuse_batch, forbidden)
                if rc is not None and rc.total_flops < best.total_flops:
                    best = rc
    if best is None:
        raise RuntimeError("no plan met the size bound; raise trials or the bound")
    return best


def _reuse_candidate(net, base, path, open_qubits, closed_bits, max_log2, n_sliced, batch,
                     forbidden):
    g_bits, _ = choose_slices(base, path, max_log2, forbidden=forbidden)
    n_glob = _popcount(g_bits)
    # the low log2(batch) id bits vary inside every batch: they must all be local labels
    if n_sliced - n_glob < max(1, int(batch).bit_length() - 1):
        return None
    local = choose_local_slices(base, path, g_bits, n_sliced - n_glob, batch, max_log2, forbidden)
    if local is None:
        return None
    ids = lambda bits: [base.label_ids[i] for i in range(len(base.label_ids)) if (bits >> i) & 1]
    loc_labels = [ids(b)[0] for b in local]
    glob_labels = ids(g_bits)
    sliced = loc_labels + glob_labels                 # local labels on the low id bits
    n = net.n_qubits
    sp = make_problem(net.labels, net.out_label, n, open_qubits, closed_bits, sliced=sliced)
    leaf_loc = {k for k, l in enumerate(net.labels) if any(x in loc_labels for x in l)}
    leaf_glob = {k for k, l in enumerate(net.labels) if any(x in glob_labels for x in l)}
    cost = reuse_cost(sp, path, leaf_loc, leaf_glob, batch)
    if cost.peak_log2 > max_log2 + 1e-9:
        return None
    return Plan(path=path, sliced_labels=sliced, cost=cost, n_slices=1 << len(sliced))


def order_for_reuse(net, plan: Plan, open_qubits, closed_bits, batch: int) -> Plan:
    """Head reuse without extra slicing: of the plan's sliced labels, log2(batch) become
    local labels on the low slice-id bits, chosen one at a time to minimise the work of the
    steps that depend on them (every other slice-dependent step is then shared by a batch
    of `batch` consecutive ids); the path and the sliced set are unchanged."""
    n_loc = max(1, int(batch).bit_length() - 1)
    sl = list(plan.sliced_labels)
    deps = [set(x for x in lab if x in sl) for lab in net.labels]
    sets = []
    for i, j in plan.path:
        deps[i] = deps[i] | deps[j]
        sets.append(deps[i])
    macs = [st[6] for st in plan.cost.steps]
    local = []
    for _ in range(min(n_loc, len(sl))):
        best = None
        for x in sl:
            if x in local:
                continue
            chosen = set(local + [x])
            w = sum(m for m, st in zip(macs, sets) if st & chosen)
            if best is None or w < best[0]:
                best = (w, x)
        local.append(best[1])
    order = local + [x for x in sl if x not in local]
    sp = make_problem(net.labels, net.out_label, net.n_qubits, open_qubits, closed_bits, sliced=order)
    leaf_loc = {k for k, l in enumerate(net.labels) if any(x in local for x in l)}
    leaf_glob = {k for k, l in enumerate(net.labels) if any(x in sl and x not in local for x in l)}
    cost = reuse_cost(sp, plan.path, leaf_loc, leaf_glob, batch)
    return Plan(path=plan.path, sliced_labels=order, cost=cost, n_slices=plan.n_slices)


def zigzag_path(prob: Problem, cycles, tail_start: int, temperature: float = 0.0, seed: int = 0):
    """Head-tail order with the zigzag tail (Method, zigzag paragraph; Appendix E).

    Leaves of gates before cycle `tail_start` form the head, contracted by the greedy search
    into one tensor, whose legs toward the tail are the head-tail interface.  The tail's
    leaves are then absorbed into that tensor one at a time along chains of neighbouring
    gates: the sweep starts at the interface and moves to a neighbour (a leaf sharing a bond
    with the leaf absorbed last) at the same or a later cycle, complexity-greedily (fewest
    multiply-adds, then smallest result), until it reaches the final state; there it turns
    around and follows neighbours at earlier cycles back toward the interface, turns again,
    and so on.  Where the leaf absorbed last has no free neighbour in either direction the
    sweep restarts from the accumulator's cheapest neighbour; tail leaves joined to the
    accumulator by no bond are absorbed last, smallest first."""
    n = len(prob.dense)
    head = [k for k in range(n) if cycles[k] < tail_start]
    tail = [k for k in range(n) if cycles[k] >= tail_start]
    leaf_dense = list(prob.dense)
    dense, qm = list(prob.dense), list(prob.qmask)
    path = []
    acc = None
    if head:
        sub = Problem(dense=[dense[k] for k in head], qmask=[qm[k] for k in head], rows=prob.rows,
                      label_ids=prob.label_ids)
        for i, j in greedy_path(sub, temperature=temperature, seed=seed):
            a, b = head[i], head[j]
            path.append((a, b))
            dense[a] ^= dense[b]
            qm[a] |= qm[b]
        alive = set(head)
        for _, b in path:
            alive.discard(b)
        acc = min(alive)
    rest = set(tail)
    if acc is None:
        if not rest:
            return path
        acc = min(rest, key=lambda k: (cycles[k], k))
        rest.discard(acc)

    def cheapest(cands):
        def key(k):
            macs = prob.rows(qm[acc] | qm[k]) << _popcount(dense[acc] | dense[k])
            return (macs, prob.size(dense[acc] ^ dense[k], qm[acc] | qm[k]), k)
        return min(cands, key=key)

    direction, last = 1, None
    while rest:
        step = None
        if last is not None:
            for turn in (False, True):
                d = -direction if turn else direction
                nb = [k for k in rest if leaf_dense[k] & leaf_dense[last]
                      and d * (cycles[k] - cycles[last]) >= 0]
                if nb:
                    direction, step = d, cheapest(nb)
                    break
        if step is None:
            nb = [k for k in rest if dense[k] & dense[acc]]
            if nb:
                # (re)start at the interface side the sweep is heading from
                edge = min(direction * cycles[k] for k in nb)
                step = cheapest([k for k in nb if direction * cycles[k] == edge])
            else:
                step = min(rest, key=lambda k: (prob.size(dense[k], qm[k]), k))
        path.append((acc, step))
        dense[acc] ^= dense[step]
        qm[acc] |= qm[step]
        last = step
        rest.discard(step)
    return path


def zigzag_plan(net, open_qubits, closed_bits, tail_start: int, max_log2: float,
                base_sliced=(), trials: int = 4, seed: int = 0, temperature: float = 0.1,
                rounds: int = 3) -> Plan:
    """Head-tail plan with the zigzag tail (zigzag_path) under the size bound.

    The head becomes one tensor, whose legs include every unsliced bond crossing the
    head-tail interface, so the bound usually needs interface bonds sliced (the paper's
    global slicing of the interface, Appendix B.2).  Bonds in `base_sliced` are sliced
    first and keep the low slice-id bits (so a plan found by find_plan can be refined and
    its slices compared); further bonds are chosen along the zigzag path as in find_plan
    (choose_slices, then the path searched again on the sliced network) and take the
    following bits.  Returns the trial with the lowest total flop count."""
    n = net.n_qubits
    base_sliced = list(base_sliced)
    base = make_problem(net.labels, net.out_label, n, open_qubits, closed_bits, sliced=base_sliced)
    pos = {x: i for i, x in enumerate(base.label_ids)}
    bond_bits = 0
    for x in set(net.bond_label.values()):
        if x in pos:
            bond_bits |= 1 << pos[x]
    forbidden = ((1 << len(base.label_ids)) - 1) & ~bond_bits
    ids = lambda bits: [base.label_ids[i] for i in range(len(base.label_ids)) if (bits >> i) & 1]
    best = None
    for t in range(trials):
        temp, s = (0.0, seed) if t == 0 else (temperature, seed + 7919 * t)
        path = zigzag_path(base, net.cycle, tail_start, temperature=temp, seed=s)
        sliced = base_sliced
        for _ in range(rounds):
            extra, _ = choose_slices(base, path, max_log2, forbidden=forbidden)
            sliced = base_sliced + ids(extra)
            sp = make_problem(net.labels, net.out_label, n, open_qubits, closed_bits, sliced=sliced)
            path2 = zigzag_path(sp, net.cycle, tail_start, temperature=temp, seed=s + 1)
            c1, c2 = path_cost(sp, path), path_cost(sp, path2)
            if c2.peak_log2 <= max_log2 + 1e-9 and (c1.peak_log2 > max_log2 + 1e-9 or
                                                   c2.flops_per_slice < c1.flops_per_slice):
                path = path2
        sp = make_problem(net.labels, net.out_label, n, open_qubits, closed_bits, sliced=sliced)
        leaves = {k for k, l in enumerate(net.labels) if any(x in sliced for x in l)}
        cost = path_cost(sp, path, leaves)
        if cost.peak_log2 > max_log2 + 1e-9:
            continue
        cand = Plan(path=path, sliced_labels=list(sliced), cost=cost, n_slices=1 << len(sliced))
        if best is None or cand.total_flops < best.total_flops:
            best = cand
    if best is None:
        raise RuntimeError("no zigzag plan met the size bound")
    return best


@dataclass
class StepModel:
    """Roofline time of one step: the larger of its flops (8 per complex multiply-add) at
    the rate the matrix-core GEMM kernels reach and its complex64 bytes (A, B and C once
    each) at the rate the memory-bound kernels reach.  The flop rate falls with a short
    contraction: flop_rate * K / (K + k_half) for contracted dimension K (a tile's operand
    loads and result stores are amortised over K).  The defaults fit the per-launch table of
    the 53-qubit workload on one MI355X: about 120 TFLOP/s for long K, half that at K = 32,
    and 3.5 TB/s (of 8) averaged over the memory-bound steps."""
    flop_rate: float = 120e12
    byte_rate: float = 3.5e12
    k_half: float = 32.0

    def time(self, macs: float, elems: float, k: float = math.inf) -> float:
        rate = self.flop_rate if math.isinf(k) else self.flop_rate * k / (k + self.k_half)
        return max(8.0 * macs / rate, 8.0 * elems / self.byte_rate)


def branch_merge(prob: Problem, path, branch_log2: float, max_group: int = 6,
                 model: StepModel | None = None, reorder: bool = True):
    """Branch merging of a path (module docstring): returns the new path.

    The path is read as a tree.  A stem starts at a root or at the smaller operand of a
    step and follows the larger operand of each step down to a leaf; the smaller operands
    b_1 .. b_m it absorbs (bottom up) are themselves processed first.  With `reorder`, two
    neighbouring absorptions first trade places wherever that lowers the modelled time of
    their two steps and keeps the stem's intermediate between them at or below
    2^branch_log2 elements (passes until nothing moves).  Then consecutive b_s .. b_e (at
    most `max_group`) may be contracted into one branch (b_s (x) (b_s+1 (x) ... b_e)),
    every intermediate of which has at most 2^branch_log2 elements; the stem absorbs the
    branch in one step.  Groups are chosen by dynamic programming to minimise the modelled
    time of the stem's steps plus the branches' own; a group of one is the original step,
    so the path only changes where the model says it gains.  Each step of the new path
    keeps its larger operand at position i."""
    model = model or StepModel()
    n = len(prob.dense)
    alive = validate_path(n, path)
    dense = list(prob.dense)
    qm = list(prob.qmask)
    ch = []
    slot = list(range(n))
    for i, j in path:
        a, b = slot[i], slot[j]
        ch.append((a, b))
        dense.append(dense[a] ^ dense[b])
        qm.append(qm[a] | qm[b])
        slot[i] = n + len(ch) - 1
    roots = [slot[k] for k in alive]
    size = lambda d, q: prob.size(d, q)

    def step_time(da, qa, db, qb):
        q = qa | qb
        macs = float(prob.rows(q)) * float(1 << _popcount(da | db))
        return model.time(macs, size(da, qa) + size(db, qb) + size(da ^ db, q),
                          float(1 << _popcount(da & db)))

    def big_small(v):
        a, b = ch[v - n]
        return (a, b) if size(dense[a], qm[a]) >= size(dense[b], qm[b]) else (b, a)

    heads = set(roots) | {big_small(v)[1] for v in range(n, n + len(ch))}
    limit = 2.0 ** branch_log2
    new_id = {}
    nch = {}

    def make(a, b):
        v = len(dense)
        dense.append(dense[a] ^ dense[b])
        qm.append(qm[a] | qm[b])
        nch[v] = (a, b)
        return v

    # a head's absorbed operands are heads with smaller ids: increasing order sees them first
    for h in sorted(heads):
        if h < n:
            new_id[h] = h
            continue
        smalls = []
        u = h
        while u >= n:
            big, small = big_small(u)
            smalls.append(small)
            u = big
        smalls.reverse()
        bs = [new_id[b] for b in smalls]
        m = len(bs)
        moved, passes = reorder, 0
        while moved and passes < m:
            moved, passes = False, passes + 1
            d_, q_ = dense[u], qm[u]
            for k in range(m - 1):
                b1, b2 = bs[k], bs[k + 1]
                keep = (step_time(d_, q_, dense[b1], qm[b1]) +
                        step_time(d_ ^ dense[b1], q_ | qm[b1], dense[b2], qm[b2]))
                md, mq = d_ ^ dense[b2], q_ | qm[b2]
                swap = step_time(d_, q_, dense[b2], qm[b2]) + step_time(md, mq, dense[b1], qm[b1])
                if swap < keep * (1.0 - 1e-9) and size(md, mq) <= limit:
                    bs[k], bs[k + 1] = b2, b1
                    moved = True
                d_, q_ = d_ ^ dense[bs[k]], q_ | qm[bs[k]]
        sd, sq = [dense[u]], [qm[u]]
        for b in bs:
            sd.append(sd[-1] ^ dense[b])
            sq.append(sq[-1] | qm[b])
        best = [0.0] + [math.inf] * m
        arg = list(range(m + 1))
        for e in range(1, m + 1):
            bd, bq, build = 0, 0, 0.0
            for s_ in range(e, max(0, e - max_group), -1):
                b = bs[s_ - 1]
                if s_ < e:
                    build += step_time(dense[b], qm[b], bd, bq)
                bd, bq = bd ^ dense[b], bq | qm[b]
                if s_ < e and size(bd, bq) > limit:
                    break
                t = best[s_ - 1] + build + step_time(sd[s_ - 1], sq[s_ - 1], bd, bq)
                if t < best[e] * (1.0 - 1e-9) or s_ == e:
                    best[e], arg[e] = t, s_
        groups = []
        e = m
        while e > 0:
            groups.append((arg[e], e))
            e = arg[e] - 1
        cur = u
        for s_, e in reversed(groups):
            br = bs[e - 1]
            for t in range(e - 1, s_ - 1, -1):
                br = make(bs[t - 1], br)
            cur = make(cur, br)
        new_id[h] = cur
    pos = list(range(len(dense)))
    out = []
    for r in roots:
        stack = [(new_id[r], False)]
        while stack:
            v, done = stack.pop()
            if v < n:
                continue
            a, b = nch[v]
            if done:
                out.append((pos[a], pos[b]))
                pos[v] = pos[a]
            else:
                stack += [(v, True), (b, False), (a, False)]
    return out


def merge_branches(net, plan: Plan, open_qubits, closed_bits, branch_log2: float | None = None,
                   max_group: int = 6, model: StepModel | None = None,
                   reorder: bool = True, passes: int = 4) -> Plan:
    """The plan with its path branch-merged (branch_merge) on its sliced network; the
    sliced bonds are unchanged.  branch_log2 defaults to the plan's peak, so the merged plan
    keeps the space complexity of the original.  Each pass sees the stems the previous one
    left (a merged or reordered stem is a new chain); passes stop once one changes
    nothing."""
    sp = make_problem(net.labels, net.out_label, net.n_qubits, open_qubits, closed_bits,
                      sliced=plan.sliced_labels)
    if branch_log2 is None:
        branch_log2 = plan.cost.peak_log2
    path = plan.path
    for _ in range(passes):
        new = branch_merge(sp, path, branch_log2, max_group=max_group, model=model,
                           reorder=reorder)
        if new == path:
            break
        path = new
    leaves = {k for k, l in enumerate(net.labels) if any(x in plan.sliced_labels for x in l)}
    cost = path_cost(sp, path, leaves)
    return Plan(path=path, sliced_labels=list(plan.sliced_labels), cost=cost,
                n_slices=plan.n_slices)


def validate_path(n_tensors: int, pairs):
    """Check a path in the (i, j) -> i format (Appendix E) against n_tensors leaves: every
    pair names two distinct live tensors.  Returns the ids still alive at the end."""
    alive = [True] * n_tensors
    for step, (i, j) in enumerate(pairs):
        if not (0 <= i < n_tensors and 0 <= j < n_tensors) or i == j:
            raise ValueError(f"step {step}: invalid pair {(i, j)}")
        if not (alive[i] and alive[j]):
            raise ValueError(f"step {step}: pair {(i, j)} uses a retired tensor")
        alive[j] = False
    return [k for k in range(n_tensors) if alive[k]]
