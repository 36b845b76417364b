"""The 53-qubit share at full size (6x9 grid minus one site, 20 cycles, largest intermediate
2^30, 2^14 groups x 6 open qubits = 2^20 amplitudes, 98 sliced bonds).

Oracle parity at full size: stored oracle amplitudes of single (slice, group) pairs
(tests/golden, the oracle's own network for one group with the slice's bonds fixed,
contracted along its seeded random-greedy path, which keeps every intermediate <= 2^26)
against the same group inside the library's 2^14-group sparse state, contracted in the
launch configuration bench.py times (autotuned tiles; four slices per launch sequence on
the plain path, 64 on the branch-merged one): one slice at a time, and slices 0..3 in
one launch sequence through a captured graph, first and replayed pass, against the sum of
the four stored slices.
Properties that hold at any size complete it: a group inside the sparse state equals a
separate contraction with that group alone, and head reuse equals the plain plan."""

import numpy as np
import pytest

import synth
from oracle import metrics
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("form", [("c64", 0, 1e-5), ("bf16x3", 2, 1e-3), ("fp16x3", 1, 1e-5)],
                         ids=["c64", "bf16x3", "fp16x3"])
def test_large_pairs_match_stored_oracle(form):
    """On the jittered twin of the share (same structure, plan and slices; at theta = pi/2
    exactly most slices are exact zeros): each stored pair against its group inside the
    2^14-group sparse state.  The amplitudes lie far below FP32's normal range, reached
    through the per-slice scale records."""
    _pairs_against_stored_oracle("default", *form)


@pytest.mark.parametrize("form", [("c64", 0, 1e-5), ("bf16x3", 2, 1e-3), ("fp16x3", 1, 1e-5)],
                         ids=["c64", "bf16x3", "fp16x3"])
def test_large_branch_merged_pairs_match_stored_oracle(form):
    """The same stored pairs through the branch-merged path that bench.py times (same sliced
    bonds and slices, a different tree, intermediates in other label orders)."""
    _pairs_against_stored_oracle("branch", *form)


def _pairs_against_stored_oracle(mode, name, prec, tol):
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload, jittered_twin
    from tests.golden_data import large_pairs
    pairs, bonds, jitter = large_pairs()
    j = synth.config("large")["parity_jitter"]
    assert jitter == (j["theta_jitter"], j["jitter_seed"])
    w = jittered_twin(config_workload("large", mode=mode), *jitter)
    assert [tuple(b) for b in w.sliced_bonds] == bonds, "the stored pairs were made for another slicing"
    batch = 64 if mode == "branch" else 4      # slices per launch sequence, as bench.py takes
    c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels, slice_ids=w.slice_ids,
                    open_qubits=w.open_qubits, closed_bits=w.closed_bits, max_batch_slices=batch,
                    precision=prec)
    assert c.batch_slices == batch
    c.autotune(reps=1)
    for p in pairs:
        assert int(w.slice_ids[p.pos]) == p.slice_id and int(w.closed_bits[p.group]) == p.closed
        log(f"large {name} ({mode} path): slice position {p.pos}, group {p.group} of 2^14")
        c.contract_range(p.pos, 1)
        got = c.amps[p.group].cpu().numpy()
        err = metrics.rel_error(got, p.amps)
        mx = metrics.max_error_over_rms(got, p.amps)
        log(f"  rel err {err:.3e}, max err / rms {mx:.3e}, |amp| ~ {np.abs(p.amps).max():.1e}")
        assert err <= tol and mx <= 10 * tol
    # slice positions 0..3 in one launch sequence (the whole sequence at four slices per
    # launch, the first four of 64 otherwise), captured and replayed
    first = [p for p in pairs if p.group == 0 and p.pos < 4]
    assert sorted(p.pos for p in first) == [0, 1, 2, 3]
    ref = sum(p.amps for p in first)
    for rep in range(2):
        c.contract_range(0, 4)
        got = c.amps[0].cpu().numpy()
        err = metrics.rel_error(got, ref)
        log(f"  slices 0..3 as one launch sequence (pass {rep}): rel err {err:.3e}")
        assert err <= tol
    c.close()


def test_large_sparse_state_equals_single_groups():
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("large")
    assert w.n_amplitudes == 1 << 20 and w.plan.cost.peak_log2 <= 30
    ids = list(w.slice_ids[:2])
    log(f"large: {len(w.plan.sliced_labels)} sliced bonds, slices {[hex(int(i)) for i in ids]}")
    full = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels, slice_ids=ids,
                       open_qubits=w.open_qubits, closed_bits=w.closed_bits, max_batch_slices=1)
    full.contract()
    amps = full.amps.cpu().numpy()
    full.close()
    assert np.all(np.isfinite(amps))
    rng = np.random.default_rng(5)
    for g in sorted(rng.choice(len(w.closed_bits), size=3, replace=False)):
        one = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels, slice_ids=ids,
                          open_qubits=w.open_qubits, closed_bits=w.closed_bits[g:g + 1],
                          max_batch_slices=1)
        one.contract()
        got = one.amps.cpu().numpy()[0]
        one.close()
        err = metrics.rel_error(amps[g], got)
        log(f"  group {g}: sparse state vs alone rel diff {err:.2e}")
        assert err <= 1e-5


def test_large_head_reuse_equals_plain_plan():
    """Head reuse on the 53-qubit share: the reuse mode keeps the 98 sliced bonds, puts the
    log2(B) cheapest on the low slice-id bits and draws the subset as subtasks of B local
    slices; with batches of B, the steps above the other labels run once per subtask.
    Its sparse state over 32 of those slices equals the plain plan's over the same slices
    (ids translated to the plain label order), contracted one slice at a time."""
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload
    plain = config_workload("large")
    reuse = config_workload("large", mode="reuse")
    assert sorted(reuse.plan.sliced_labels) == sorted(plain.plan.sliced_labels)
    ids = [int(x) for x in reuse.slice_ids[:32]]
    pos = [plain.plan.sliced_labels.index(x) for x in reuse.plan.sliced_labels]
    plain_ids = [sum(((i >> b) & 1) << pos[b] for b in range(len(pos))) for i in ids]
    import synth
    b = synth.config("large")["reuse_batch"]
    r = Contraction(reuse.net, reuse.plan.path, sliced_labels=reuse.plan.sliced_labels,
                    slice_ids=ids, open_qubits=reuse.open_qubits, closed_bits=reuse.closed_bits,
                    max_batch_slices=b)
    shared = sum(l.flops for l in r.launches() if l.invariant == 2)
    r.contract()
    got = r.amps.cpu().numpy().copy()
    work = r.work()
    r.close()
    p = Contraction(plain.net, plain.plan.path, sliced_labels=plain.plan.sliced_labels,
                    slice_ids=plain_ids, open_qubits=plain.open_qubits,
                    closed_bits=plain.closed_bits, max_batch_slices=1)
    p.contract()
    ref = p.amps.cpu().numpy()
    plain_work = p.work()
    p.close()
    err = metrics.rel_error(got, ref)
    log(f"large head reuse: shared {shared:.3e} flops per batch, work {work:.3e} vs plain "
        f"{plain_work:.3e}; rel diff {err:.3e}")
    assert shared > 0 and work < 0.6 * plain_work
    assert err <= 1e-5


@pytest.mark.parametrize("precision,tol", [(2, 1e-3), (1, 1e-5)])
def test_large_head_reuse_split_precision(precision, tol):
    """The split-precision forms on the 53-qubit share with head reuse, against the complex64
    result of the same plan and slices (within each form's stated bound, 1 - F <= 1e-6)."""
    import synth
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("large", mode="reuse")
    b = synth.config("large")["reuse_batch"]
    ids = [int(x) for x in w.slice_ids[:16]]
    out = {}
    for prec in (0, precision):
        c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels, slice_ids=ids,
                        open_qubits=w.open_qubits, closed_bits=w.closed_bits,
                        max_batch_slices=b, precision=prec)
        c.contract()
        out[prec] = c.amps.cpu().numpy().copy()
        c.close()
    err = metrics.rel_error(out[precision], out[0])
    fid = metrics.fidelity(out[precision], out[0])
    log(f"large head reuse, precision {precision}: rel diff {err:.3e}, 1-F {1 - fid:.3e}")
    assert err <= tol and 1 - fid <= 1e-6
