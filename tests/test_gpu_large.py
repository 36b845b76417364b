"""The 53-qubit share at full size (6x9 grid minus one site, 20 cycles, largest intermediate
2^30, 2^14 groups x 6 open qubits = 2^20 amplitudes, 98 sliced bonds).

The oracle cannot contract this network (its own greedy path for a single group peaks at
2^26 to 2^33 elements depending on tie-breaks), so parity here is a property that holds at
any size: the amplitudes of a group computed inside the sparse state (rows of all 2^14
groups, gathered operand rows) equal those of a separate contraction with that group
alone (no rows at all) - the same slices, the same path."""

import numpy as np
import pytest

from oracle import metrics
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


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
