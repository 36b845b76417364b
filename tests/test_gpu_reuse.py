"""Head reuse (Method, Appendix B.2: the head is contracted once per subtask and shared by
its slices): steps whose sliced labels keep one value over a batch of consecutive slices
run once per batch.  Checked against the oracle on a small network planned for reuse (all
three precision forms, a range that does not start on a batch boundary), against the same
plan with sharing turned off, and at full size against the plain plan's 1024-slice sum."""

import os

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import metrics
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu
TOLS = {0: 1e-5, 1: 1e-5, 2: 1e-3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _contraction(w, **kw):
    from paper_2111_03011_amd.contractor import Contraction
    return Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                       slice_ids=w.slice_ids, open_qubits=w.open_qubits,
                       closed_bits=w.closed_bits, **kw)


def _reuse_case():
    from paper_2111_03011_amd.workload import make_workload
    circ = synth.make_circuit(4, 4, 14, 44)
    open_q = list(range(10, 16))
    closed = synth.group_targets(16, open_q, 4, 45)
    return make_workload(circ, open_q, closed, max_log2=14, n_sliced=6, trials=8, seed=44,
                         reuse_batch=8)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_head_reuse_small_against_oracle(precision):
    w = _reuse_case()
    assert w.plan.cost.flops_shared > 0
    log(f"head reuse, precision {precision}: sliced {w.plan.sliced_labels}")
    c = _contraction(w, max_batch_slices=8, precision=precision)
    assert any(l.invariant == 2 for l in c.launches())
    c.contract()
    got = c.amps.cpu().numpy().copy()
    ref = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits)
    err = metrics.rel_error(got, ref)
    log(f"  all 64 slices: rel err {err:.3e}")
    assert err <= TOLS[precision]
    ids = [int(x) for x in w.slice_ids[3:16]]
    c.contract_range(3, 13)
    part = c.amps.cpu().numpy().copy()
    c.close()
    ref_part = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                           sliced_bonds=w.sliced_bonds, slice_ids=ids)
    err = metrics.rel_error(part, ref_part)
    log(f"  slices 3..15 (runs 3..7, 8..15): rel err {err:.3e}")
    assert err <= TOLS[precision]
    if precision == 0:
        os.environ["TNC_NO_SHARE"] = "1"
        try:
            d = _contraction(w, max_batch_slices=8)
        finally:
            os.environ.pop("TNC_NO_SHARE")
        assert not any(l.invariant == 2 for l in d.launches())
        d.contract()
        err = metrics.rel_error(d.amps.cpu().numpy(), got)
        d.close()
        log(f"  shared against unshared: rel diff {err:.3e}")
        assert err <= 1e-6


def test_head_reuse_full_size_against_plain_plan():
    """The 1024-slice workload planned for head reuse (bound-driven global slices, local
    slices on the low id bits, batches of 64) sums to the plain plan's amplitudes; the plain
    plan's slices are checked against the oracle in test_gpu_parity."""
    from paper_2111_03011_amd.workload import config_workload
    plain_w = config_workload("sliced")
    reuse_w = config_workload("sliced", mode="reuse")
    c = _contraction(plain_w, max_batch_slices=64)
    c.contract()
    ref = c.amps.cpu().numpy().copy()
    c.close()
    r = _contraction(reuse_w, max_batch_slices=64)
    shared = sum(l.flops for l in r.launches() if l.invariant == 2)
    r.contract()
    got = r.amps.cpu().numpy()
    work = r.work()
    r.close()
    err, fid = metrics.rel_error(got, ref), metrics.fidelity(got, ref)
    log(f"head reuse full size: sliced {reuse_w.plan.sliced_labels}, shared flops per batch "
        f"{shared:.3e}, work {work:.3e} (plain {plain_w.plan.total_flops:.3e}); rel diff "
        f"{err:.3e}, 1-F {1 - fid:.3e}")
    assert shared > 0 and work < plain_w.plan.total_flops
    assert err <= 1e-5
