"""Zigzag tail order (Method, zigzag paragraph; Appendix E) through the library: a small
head-tail plan with head reuse against the oracle, and at full size the 53-qubit share's
zigzag path against the plain path on the same slices."""

import time

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


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_zigzag_with_head_reuse_small_against_oracle(precision):
    """4x4 grid, 14 cycles, tail from cycle 10, 64 slices as batches of 8 with the head
    shared inside each batch: every slice summed, and a range across a batch boundary."""
    from paper_2111_03011_amd.workload import make_zigzag_workload
    circ = synth.make_circuit(4, 4, 14, 44)
    open_q = list(range(10, 16))
    closed = synth.group_targets(16, open_q, 4, 45)
    w = make_zigzag_workload(circ, open_q, closed, 10, 14, reuse_batch=8, seed=44)
    log(f"zigzag + reuse, precision {precision}: {len(w.slice_ids)} slices, "
        f"sliced {w.plan.sliced_labels}")
    c = _contraction(w, max_batch_slices=8, precision=precision)
    assert any(l.invariant == 2 for l in c.launches())
    c.contract()
    got = c.amps.cpu().numpy().copy()
    ref = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits)
    err = metrics.rel_error(got, ref)
    log(f"  all slices: rel err {err:.3e}")
    assert err <= TOLS[precision]
    ids = [int(x) for x in w.slice_ids[5:19]]
    c.contract_range(5, 14)
    part = c.amps.cpu().numpy().copy()
    c.close()
    ref_part = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                           sliced_bonds=w.sliced_bonds, slice_ids=ids)
    err = metrics.rel_error(part, ref_part)
    log(f"  slices 5..18: rel err {err:.3e}")
    assert err <= TOLS[precision]


def test_zigzag_53q_matches_plain_path_on_same_slices():
    """A zigzag plan of the 53-qubit share (tail from cycle 19; the plain plan's 98 sliced
    bonds plus those its own 2^30 bound needs) and the plain plan's path on that same
    slicing, over four seeded slices of the circuit with jittered angles (at pi/2 exactly
    such slices are structural zeros): the two orders give the same sum."""
    import torch
    from paper_2111_03011_amd.workload import config_workload, jittered_twin, zigzag_pair
    jit = synth.config("large")["parity_jitter"]
    twin = jittered_twin(config_workload("large"), jit["theta_jitter"], jit["jitter_seed"])
    wz, wp = zigzag_pair(twin, 19, 30, 4, 1919)
    assert wz.plan.sliced_labels == wp.plan.sliced_labels
    log(f"53q zigzag: {len(wz.plan.sliced_labels)} sliced bonds, "
        f"peaks {wz.plan.cost.peak_log2:.1f} / {wp.plan.cost.peak_log2:.1f}")
    sums = []
    for tag, ww in (("zigzag", wz), ("plain path", wp)):
        c = _contraction(ww, max_batch_slices=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.contract()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sums.append(c.amps.cpu().numpy().copy())
        c.close()
        log(f"  {tag}: {1e3 * dt / len(ww.slice_ids):.1f} ms per slice (first pass), "
            f"|amp| max {np.abs(sums[-1]).max():.2e}")
        assert np.all(np.isfinite(sums[-1]))
    assert np.abs(sums[1]).max() > 0
    err = metrics.rel_error(sums[0], sums[1])
    log(f"  zigzag against plain path: rel diff {err:.3e}")
    assert err <= 5e-5
