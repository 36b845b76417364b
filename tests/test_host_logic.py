"""Host-side logic without a GPU: input generators, network builder, planner, path format
(Appendix E), sparse-state row sets (Appendix A), and the C ABI's validation and plan
compilation (no device call is made)."""

import math
import re

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import statevector
from paper_2111_03011_amd import planner, tnc
from paper_2111_03011_amd.network import circuit_network
from paper_2111_03011_amd.workload import make_workload

GOLDEN = __file__.rsplit("/", 1)[0] + "/golden/appendix_e_contraction_order.txt"


# ---------------------------------------------------------------- generators
def test_generator_counts_and_matchings():
    for name, n2, n1 in (("small", 34, 96), ("sliced", 171, 420), ("large", 450, 1060)):
        c = synth.circuit_from_config(synth.config(name))
        assert sum(len(l["couplers"]) for l in c["layers"]) == n2
        assert sum(len(l["oneq"]) for l in c["layers"]) == n1
        for l in c["layers"]:
            qs = [q for cp in l["couplers"] for q in cp]
            assert len(qs) == len(set(qs))               # each pattern is a matching
    c = synth.circuit_from_config(synth.config("large"))
    assert c["n_qubits"] == 53


def test_generator_never_repeats_a_gate_and_is_seeded():
    c = synth.make_circuit(4, 5, 12, 77)
    for a, b in zip(c["layers"], c["layers"][1:]):
        assert all(x != y for x, y in zip(a["oneq"], b["oneq"]))
    assert c == synth.make_circuit(4, 5, 12, 77)
    assert c != synth.make_circuit(4, 5, 12, 78)


def test_targets_distinct_and_bit_order():
    g = synth.group_targets(10, [2, 7], 100, 5)
    assert len(set(g.tolist())) == 100
    for x in g:
        assert synth.bit_of(int(x), 10, 2) == 0 and synth.bit_of(int(x), 10, 7) == 0
    assert synth.bitstring_from_bits([1, 0, 0], 3) == 0b100
    s = synth.slice_subset(10, 8, 3)
    assert len(s) == 8 and list(s) == sorted(s) and s.max() < 1024


# ---------------------------------------------------------------- network and planner
def test_network_builder_matches_oracle_state_vector():
    c = synth.make_circuit(3, 3, 9, 4)
    net = circuit_network(c)
    assert max(net.ranks()) <= 4
    p = ocontract.greedy_path(net.labels)
    res = ocontract.contract_path(net.tensors, net.labels, p, net.out_label).reshape(-1)
    assert np.allclose(res, statevector.simulate(c), atol=1e-13)


def test_network_builder_reads_per_gate_angles():
    """A jittered circuit (one angle per two-qubit gate) builds a network with the same
    labels as the plain one and the oracle's state vector."""
    c = synth.make_circuit(3, 3, 9, 4, theta_jitter=0.05, jitter_seed=2)
    net = circuit_network(c)
    assert net.labels == circuit_network(synth.make_circuit(3, 3, 9, 4)).labels
    p = ocontract.greedy_path(net.labels)
    res = ocontract.contract_path(net.tensors, net.labels, p, net.out_label).reshape(-1)
    assert np.allclose(res, statevector.simulate(c), atol=1e-13)


def _brute_macs(labels, out_set, closed_rows, path, sliced):
    """Recount complex multiply-adds step by step from plain label sets."""
    cur = [set(l) - set(sliced) for l in labels]
    q = [set() for _ in labels]
    for k, l in enumerate(cur):
        for x in list(l):
            if x in closed_rows:
                l.discard(x)
                q[k].add(x)
    total = 0
    for i, j in path:
        rows = closed_rows.rows(q[i] | q[j])
        total += rows * 2 ** len(cur[i] | cur[j])
        cur[i] = cur[i] ^ cur[j]
        q[i] = q[i] | q[j]
    return total


class _Rows(dict):
    def __init__(self, net, open_q, closed):
        super().__init__()
        n = net.n_qubits
        self.n, self.closed = n, closed
        for q in range(n):
            if q not in open_q:
                self[net.out_label[q]] = q

    def rows(self, legs):
        if not legs:
            return 1
        qs = [self[x] for x in legs]
        return len({tuple((int(c) >> (self.n - 1 - q)) & 1 for q in qs) for c in self.closed})


def test_planner_cost_equals_brute_recount_with_rows_and_slices():
    c = synth.make_circuit(4, 4, 10, 12)
    open_q = [2, 9, 13]
    closed = synth.group_targets(16, open_q, 24, 13)
    w = make_workload(c, open_q, closed, max_log2=9, trials=2, seed=12)
    assert w.plan.cost.peak_log2 <= 9
    rows = _Rows(w.net, open_q, closed)
    macs = _brute_macs(w.net.labels, None, rows, w.plan.path, w.plan.sliced_labels)
    total = w.plan.cost.flops_per_slice + w.plan.cost.flops_invariant
    assert math.isclose(8 * macs, total, rel_tol=1e-12)


def test_planner_exact_slice_count_and_seed_determinism():
    cfg = synth.config("small")
    c = synth.circuit_from_config(cfg)
    net = circuit_network(c)
    a = planner.find_plan(net, [0, 1, 2], [0], max_log2=8, n_sliced=4, trials=3, seed=9)
    b = planner.find_plan(net, [0, 1, 2], [0], max_log2=8, n_sliced=4, trials=3, seed=9)
    assert len(a.sliced_labels) == 4 and a.cost.peak_log2 <= 8
    assert a.path == b.path and a.sliced_labels == b.sliced_labels
    assert set(a.sliced_labels) <= set(net.bond_label.values())
    assert len(planner.validate_path(len(net.labels), a.path)) == 1


def test_worked_example_row_sets():
    # Appendix A: targets {111, 010, 000}; merging qubits 2 and 3 (ids 1, 2 here) needs
    # the configurations {11, 10, 00} only: 3 of 4; all three qubits: 3 rows.
    rc = planner.RowCounter(3, [0b111, 0b010, 0b000])
    assert rc(rc.qmask([1, 2])) == 3
    assert rc(rc.qmask([0, 1, 2])) == 3
    assert rc(rc.qmask([0])) == 2 and rc(rc.qmask([])) == 1


def test_appendix_e_path_format():
    pairs = [tuple(map(int, l.split())) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(pairs) == 448
    ids = {x for p in pairs for x in p}
    assert min(ids) == 0 and max(ids) == 454 and len(ids) == 449
    survivors = planner.validate_path(455, pairs)
    # the head ends at (192, 234); the open qubits' boundary tensors 402 + q are untouched
    head = pairs[: pairs.index((192, 234)) + 1]
    assert len(head) == 223
    assert set(survivors) == {192} | {402 + q for q in (11, 19, 28, 29, 37, 44)}
    tail = pairs[223:]
    assert all(402 <= p[1] <= 454 for p in tail[:47])
    with pytest.raises(ValueError):
        planner.validate_path(455, pairs + [(3, 70)])        # 70 was retired by (47, 70)


# ---------------------------------------------------------------- the C ABI on the host
HEADER = __file__.rsplit("/", 2)[0] + "/include/tnc.h"


def test_library_exports_every_declared_function():
    decl = re.findall(r"^(?:tnc_status|const char\*)\s+(tnc_\w+)\(", open(HEADER).read(), re.M)
    assert len(decl) >= 20
    l = tnc.lib()
    for name in decl:
        assert hasattr(l, name), name
    assert set(decl) == set(tnc.EXPORTS)


def _err(fn, *a):
    with pytest.raises(tnc.TncError) as e:
        fn(*a)
    return e.value.code


def test_network_validation():
    # label 5 held by three tensors
    assert _err(tnc.tnc_net_create, 0, 1, [1, 1, 1], [5, 5, 5], np.ones(6), [5]) == tnc.TNC_E_INVALID
    # dangling label (one holder, not an output)
    assert _err(tnc.tnc_net_create, 0, 1, [2], [1, 2], np.ones(4), [1]) == tnc.TNC_E_INVALID
    # output label held by two tensors
    assert _err(tnc.tnc_net_create, 0, 1, [1, 1], [3, 3], np.ones(4), [3]) == tnc.TNC_E_INVALID
    # repeated label inside one tensor
    assert _err(tnc.tnc_net_create, 0, 1, [2], [4, 4], np.ones(4), [4]) == tnc.TNC_E_INVALID
    h = tnc.tnc_net_create(0, 2, [2, 2], [0, 1, 1, 2], np.ones(8), [0, 2])
    assert _err(tnc.tnc_net_set_path, h, [(0, 0)]) == tnc.TNC_E_INVALID
    assert _err(tnc.tnc_net_set_path, h, []) == tnc.TNC_E_INVALID          # leaves two tensors
    tnc.tnc_net_set_path(h, [(1, 0)])
    assert _err(tnc.tnc_net_set_slices, h, [0], [0, 1]) == tnc.TNC_E_INVALID   # output leg
    assert _err(tnc.tnc_net_set_slices, h, [1], [2]) == tnc.TNC_E_INVALID      # id >= 2^k
    tnc.tnc_net_set_slices(h, [1], [0, 1])
    assert _err(tnc.tnc_plan_create, h) == tnc.TNC_E_INVALID                    # no targets
    assert _err(tnc.tnc_net_set_targets, h, [0, 0], [0]) == tnc.TNC_E_INVALID   # repeated open
    assert _err(tnc.tnc_net_set_targets, h, [], [1, 1]) == tnc.TNC_E_INVALID    # same groups
    tnc.tnc_net_set_targets(h, [0], [0, 1])
    assert _err(tnc.tnc_plan_create, h, tnc.TNC_BF16X3_3M) == tnc.TNC_E_UNSUPPORTED
    p = tnc.tnc_plan_create(h, tnc.TNC_C64, 4)
    ws = tnc.tnc_plan_workspace_bytes(p)
    assert ws > 0
    # workspace checks happen before any device call
    assert _err(tnc.tnc_contract, p, 0, ws, 0, 1 << 20) == tnc.TNC_E_INVALID
    assert _err(tnc.tnc_contract, p, 1 << 20, ws - 256, 0, 1 << 20) == tnc.TNC_E_OOM
    tnc.tnc_plan_destroy(p)
    tnc.tnc_net_destroy(h)


def test_plan_compile_matches_planner_and_rows():
    c = synth.make_circuit(3, 3, 8, 21)
    open_q = [4]
    closed = synth.group_targets(9, open_q, 20, 2)
    w = make_workload(c, open_q, closed, max_log2=7, trials=2, seed=3)
    h = tnc.tnc_net_create(0, 9, w.net.ranks(), w.net.flat_labels(), w.net.flat_data(), w.net.out_label)
    tnc.tnc_net_set_path(h, w.plan.path)
    tnc.tnc_net_set_slices(h, w.plan.sliced_labels, w.slice_ids)
    tnc.tnc_net_set_targets(h, open_q, closed)
    sizes = []
    for batch in (1, 4):
        p = tnc.tnc_plan_create(h, tnc.TNC_C64, batch)
        flops, _, steps = tnc.tnc_plan_stats(p)
        assert steps == len(w.plan.path)
        assert math.isclose(flops, w.plan.cost.flops_per_slice, rel_tol=1e-12)
        infos = [tnc.tnc_plan_launch_info(p, i) for i in range(tnc.tnc_plan_n_launches(p))]
        assert infos[-1].kind == 4 and infos[-1].rows == 20          # slice sum over 20 groups
        assert max(i.rows for i in infos) == 20
        assert not any(i.kind == 0 for i in infos)                   # no permutes
        sizes.append(tnc.tnc_plan_workspace_bytes(p))
        tnc.tnc_plan_destroy(p)
    assert sizes[1] > sizes[0]                                       # 4 slice copies
    tnc.tnc_net_destroy(h)


def test_automatic_batch_size():
    """max_batch_slices = 0: the smallest power of two whose batch carries 2.5e11 flops,
    capped at 256 and at the slice count; explicit sizes are capped at the slice count."""
    c = synth.make_circuit(3, 3, 8, 21)
    open_q = [4]
    closed = synth.group_targets(9, open_q, 20, 2)
    w = make_workload(c, open_q, closed, max_log2=7, trials=2, seed=3)
    n = len(w.slice_ids)
    h = tnc.tnc_net_create(0, 9, w.net.ranks(), w.net.flat_labels(), w.net.flat_data(), w.net.out_label)
    tnc.tnc_net_set_path(h, w.plan.path)
    tnc.tnc_net_set_slices(h, w.plan.sliced_labels, w.slice_ids)
    tnc.tnc_net_set_targets(h, open_q, closed)
    p = tnc.tnc_plan_create(h, tnc.TNC_C64, 0)
    assert tnc.tnc_plan_batch_slices(p) == min(256, n)              # tiny slices
    tnc.tnc_plan_destroy(p)
    p = tnc.tnc_plan_create(h, tnc.TNC_C64, 10 ** 6)
    assert tnc.tnc_plan_batch_slices(p) == n
    tnc.tnc_plan_destroy(p)
    with pytest.raises(tnc.TncError):
        tnc.tnc_plan_create(h, tnc.TNC_C64, -1)
    tnc.tnc_net_destroy(h)

    from paper_2111_03011_amd.workload import config_workload
    ws = config_workload("sliced")
    h = tnc.tnc_net_create(0, ws.net.n_qubits, ws.net.ranks(), ws.net.flat_labels(),
                           ws.net.flat_data(), ws.net.out_label)
    tnc.tnc_net_set_path(h, ws.plan.path)
    tnc.tnc_net_set_slices(h, ws.plan.sliced_labels, ws.slice_ids)
    tnc.tnc_net_set_targets(h, ws.open_qubits, ws.closed_bits)
    p = tnc.tnc_plan_create(h, tnc.TNC_C64, 0)
    flops = tnc.tnc_plan_stats(p)[0]
    b = tnc.tnc_plan_batch_slices(p)
    assert b == 1 << math.ceil(math.log2(2.5e11 / flops))
    tnc.tnc_plan_destroy(p)
    tnc.tnc_net_destroy(h)


def _grouped_pair_net(n_ca, n_oa, n_cb, n_ob, nk, L, seed):
    from paper_2111_03011_amd.network import TensorNetwork
    rng = np.random.default_rng(seed)
    k = list(range(nk))
    nxt = nk
    ca = list(range(nxt, nxt + n_ca)); nxt += n_ca
    oa = list(range(nxt, nxt + n_oa)); nxt += n_oa
    cb = list(range(nxt, nxt + n_cb)); nxt += n_cb
    ob = list(range(nxt, nxt + n_ob)); nxt += n_ob
    la, lb = ca + oa + k, k + cb + ob
    ta = rng.normal(size=(2,) * len(la)) + 0j
    tb = rng.normal(size=(2,) * len(lb)) + 0j
    outs = ca + oa + cb + ob
    n = len(outs)
    net = TensorNetwork(n_qubits=n, tensors=[ta, tb], labels=[la, lb], out_label=outs,
                        bond_label={})
    open_q = list(range(n_ca, n_ca + n_oa)) + list(range(n_ca + n_oa + n_cb, n))
    closed = synth.group_targets(n, open_q, L, seed + 1)
    return net, open_q, closed


@pytest.mark.parametrize("case,mode", [
    ((5, 2, 5, 2, 8, 1024), 2),   # 1024 rows share 32 rows of each operand: stacked
    ((1, 7, 1, 7, 8, 4), 0),      # M = N = 128 per row: plain per-row tiles
])
def test_sparse_row_gemm_plan(case, mode):
    """The compiled GEMM of a grouped pair network: per-row shape and algorithmic flops
    (rows x 8MNK) follow from the groups (Appendix A), and small per-row M with shared
    N-side rows is stacked (row mode 2)."""
    net, open_q, closed = _grouped_pair_net(*case, seed=17)
    h = tnc.tnc_net_create(0, net.n_qubits, net.ranks(), net.flat_labels(), net.flat_data(),
                           net.out_label)
    tnc.tnc_net_set_path(h, [(0, 1)])
    tnc.tnc_net_set_targets(h, open_q, closed)
    p = tnc.tnc_plan_create(h, tnc.TNC_C64, 1)
    infos = [tnc.tnc_plan_launch_info(p, i) for i in range(tnc.tnc_plan_n_launches(p))]
    g = [i for i in infos if i.kind == 1]
    assert len(g) == 1
    g = g[0]
    n_ca, n_oa, n_cb, n_ob, nk, L = case
    assert g.rows == L and g.k == 1 << nk
    assert {g.m, g.n} == {1 << n_oa, 1 << n_ob}
    assert math.isclose(g.flops, 8.0 * L * (1 << (n_oa + n_ob + nk)), rel_tol=1e-12)
    assert g.row_mode == mode
    tnc.tnc_plan_destroy(p)
    tnc.tnc_net_destroy(h)


def test_plan_log_lists_gemms():
    """TNC_PLAN_LOG prints one line per GEMM and stream launch of a compiled plan."""
    import subprocess
    import sys
    code = ("import synth\n"
            "from paper_2111_03011_amd import tnc\n"
            "from paper_2111_03011_amd.workload import make_workload\n"
            "c = synth.make_circuit(3, 3, 8, 21)\n"
            "closed = synth.group_targets(9, [4], 20, 2)\n"
            "w = make_workload(c, [4], closed, max_log2=7, trials=2, seed=3)\n"
            "h = tnc.tnc_net_create(0, 9, w.net.ranks(), w.net.flat_labels(), w.net.flat_data(), w.net.out_label)\n"
            "tnc.tnc_net_set_path(h, w.plan.path)\n"
            "tnc.tnc_net_set_slices(h, w.plan.sliced_labels, w.slice_ids)\n"
            "tnc.tnc_net_set_targets(h, [4], closed)\n"
            "p = tnc.tnc_plan_create(h, tnc.TNC_C64, 1)\n"
            "print(sum(1 for i in range(tnc.tnc_plan_n_launches(p)) if tnc.tnc_plan_launch_info(p, i).kind in (1, 2)))\n")
    root = __file__.rsplit("/", 2)[0]
    env = dict(__import__("os").environ, TNC_PLAN_LOG="1", PYTHONPATH=root)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         cwd=root, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    n = int(out.stdout.strip().splitlines()[-1])
    lines = [l for l in out.stderr.splitlines() if l.startswith("[tnc plan]")]
    assert len(lines) == n and n > 0


def _reuse_case(reuse_batch):
    circ = synth.make_circuit(4, 4, 14, 44)
    open_q = list(range(10, 16))
    closed = synth.group_targets(16, open_q, 4, 45)
    return make_workload(circ, open_q, closed, max_log2=14, n_sliced=6, trials=8, seed=44,
                         reuse_batch=reuse_batch)


def _plan_of(w, batch):
    h = tnc.tnc_net_create(0, w.net.n_qubits, w.net.ranks(), w.net.flat_labels(),
                           w.net.flat_data(), w.net.out_label)
    tnc.tnc_net_set_path(h, w.plan.path)
    tnc.tnc_net_set_slices(h, w.plan.sliced_labels, w.slice_ids)
    tnc.tnc_net_set_targets(h, w.open_qubits, w.closed_bits)
    p = tnc.tnc_plan_create(h, tnc.TNC_C64, batch)
    tnc.tnc_net_destroy(h)
    return p


def test_head_reuse_plan_and_its_work():
    """Head reuse (Method, Appendix B.2): with reuse_batch = 8 the planner slices the bonds
    the size bound needs, adds local bonds on the low slice-id bits, and counts the steps
    above global labels once per batch; the library shares exactly those steps, so its
    executed work equals the planner's total, also over a range that does not start on a
    batch boundary (runs are cut where a shared bit changes)."""
    import os
    w = _reuse_case(8)
    plain = _reuse_case(1)
    assert w.plan.cost.flops_shared > 0
    assert w.plan.total_flops < plain.plan.total_flops
    n = len(w.slice_ids)
    inv, ps, sh = w.plan.cost.flops_invariant, w.plan.cost.flops_per_slice, w.plan.cost.flops_shared
    p = _plan_of(w, 8)
    infos = [tnc.tnc_plan_launch_info(p, i) for i in range(tnc.tnc_plan_n_launches(p))]
    assert any(i.invariant == 2 for i in infos)
    assert math.isclose(tnc.tnc_plan_stats(p)[0], ps, rel_tol=1e-12)
    assert math.isclose(tnc.tnc_plan_work(p, 0, n), w.plan.total_flops, rel_tol=1e-12)
    # ids 3..15: runs 3..7 and 8..15
    want = inv + ((ps - sh) * 5 + sh) + ((ps - sh) * 8 + sh)
    assert math.isclose(tnc.tnc_plan_work(p, 3, 13), want, rel_tol=1e-12)
    assert tnc.tnc_plan_work(p, 0, 0) == 0.0
    with pytest.raises(tnc.TncError):
        tnc.tnc_plan_work(p, 60, 8)
    tnc.tnc_plan_destroy(p)
    os.environ["TNC_NO_SHARE"] = "1"
    try:
        q = _plan_of(w, 8)
    finally:
        os.environ.pop("TNC_NO_SHARE")
    infos = [tnc.tnc_plan_launch_info(q, i) for i in range(tnc.tnc_plan_n_launches(q))]
    assert not any(i.invariant == 2 for i in infos)
    assert math.isclose(tnc.tnc_plan_work(q, 0, n), inv + n * ps, rel_tol=1e-12)
    tnc.tnc_plan_destroy(q)


def test_drilled_network_builder_matches_oracle():
    """Hole drilling in the network builder (Method): the drilled gate is dropped, its
    incoming wires closed with <0| and its outgoing wires restarted from |0>.  The built
    network, contracted by the oracle's contractor, equals the oracle's drilled state
    (holes in the first cycle, adjacent ones, and one on the last gate of a qubit)."""
    circ = synth.make_circuit(3, 4, 8, 1001)
    n = circ["n_qubits"]
    n2 = sum(len(l["couplers"]) for l in circ["layers"])
    for holes in ([5], [0, 1, 2], [3, 4, 17], [n2 - 1, n2 - 2]):
        c = dict(circ)
        c["holes"] = holes
        net = circuit_network(c)
        plan = planner.find_plan(net, list(range(n)), np.zeros(1, np.uint64), trials=2)
        got = ocontract.contract_path(net.tensors, net.labels, plan.path, net.out_label)
        assert np.allclose(got.reshape(-1), statevector.simulate(c), atol=1e-12), holes
    bad = dict(circ)
    bad["holes"] = [n2]
    with pytest.raises(ValueError):
        circuit_network(bad)


def test_chosen_holes_lower_the_planned_cost():
    from paper_2111_03011_amd.workload import choose_holes
    circ = synth.make_circuit(4, 4, 10, 61)
    open_q = list(range(10, 16))
    closed = np.zeros(1, np.uint64)
    holes = choose_holes(circ, 2, open_q, closed, max_log2=26)
    assert len(holes) == 2
    plain = planner.find_plan(circuit_network(circ), open_q, closed, trials=1)
    c = dict(circ)
    c["holes"] = holes
    drilled = planner.find_plan(circuit_network(c), open_q, closed, trials=1)
    assert drilled.total_flops < plain.total_flops


def test_bench_timed_mode_and_traffic_record_keys():
    """bench.py times the 53-qubit share on its branch-merged path (unmerged with
    --plain-path, head reuse with --reuse), and reports committed counter traffic only for
    the kernel source, workload, path, precision, batch and launch program the record was
    taken for."""
    import argparse
    import bench
    a = lambda **kw: argparse.Namespace(**{"workload": "large", "precision": "c64",
                                            "reuse": False, "plain_path": False, **kw})
    assert bench.headline_mode(a()) == "branch"
    assert bench.headline_mode(a(plain_path=True)) == "default"
    assert bench.headline_mode(a(reuse=True)) == "reuse"
    assert bench.headline_mode(a(workload="sliced")) == "default"
    assert bench.headline_mode(a(workload="small")) == "samples"
    import json
    rec = json.load(open(bench.traffic_json("large", "c64")))
    assert bench.measured_traffic(a(plain_path=True), rec["batch"]) is None
    assert bench.measured_traffic(a(), rec["batch"] + 1) is None
    assert bench.measured_traffic(a(precision="bf16x3"), rec["batch"]) is None
    if rec["kernels_hip_sha256"] == bench.kernels_sha256() and rec["mode"] == "branch" and \
            rec.get("launch_shapes_sha256") == bench.launch_shapes_sha256(a(), rec["batch"]):
        assert bench.measured_traffic(a(), rec["batch"]) == rec["traffic_bytes_per_launch"]
    # the fingerprint follows the launch program: the unmerged path compiles other launches
    assert bench.launch_shapes_sha256(a(plain_path=True), 4) != bench.launch_shapes_sha256(a(), 4)
