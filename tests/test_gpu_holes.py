"""Perturbed network (Method: hole drilling): the GPU contracts the drilled network built by
the library and matches the oracle's drilled state (which the oracle computes with its own
projector form); at 20 qubits the fidelity of the GPU result to the exact state follows
F ~ 2^-K.  At full size, the drilled 1024-slice workload's fidelity to the plain sum over the
4096 requested amplitudes is reported beside the estimate."""

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import metrics, statevector
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _contraction(w, **kw):
    from paper_2111_03011_amd.contractor import Contraction
    return Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                       slice_ids=w.slice_ids, open_qubits=w.open_qubits,
                       closed_bits=w.closed_bits, **kw)


def test_drilled_full_state_and_fidelity():
    from paper_2111_03011_amd.workload import choose_holes, make_workload
    circ = synth.make_circuit(4, 5, 14, 72)
    n = circ["n_qubits"]
    open_q, closed = list(range(n)), np.zeros(1, np.uint64)
    psi = statevector.simulate(circ)
    for h in (1, 2):
        c = dict(circ)
        c["holes"] = choose_holes(circ, h, open_q, closed, max_log2=22)
        w = make_workload(c, open_q, closed, max_log2=22, trials=2, seed=3)
        g = _contraction(w, max_batch_slices=4)
        g.contract()
        got = g.amps.cpu().numpy()[0]
        g.close()
        ref = statevector.simulate(c)
        err = metrics.rel_error(got, ref)
        f = metrics.fidelity(got, psi)
        log(f"{h} hole(s) at {c['holes']}: rel err {err:.3e}, F {f:.4f} (2^-K = {2.0 ** (-2 * h):.4f})")
        assert err <= TOL
        assert 0.5 < f / 2.0 ** (-2 * h) < 2.0


def test_drilled_sliced_groups_against_oracle():
    from paper_2111_03011_amd.workload import make_workload
    circ = synth.make_circuit(4, 4, 10, 12)
    circ["holes"] = [7, 20, 31]
    open_q = [2, 9, 13]
    closed = synth.group_targets(16, open_q, 24, 13)
    w = make_workload(circ, open_q, closed, max_log2=9, trials=2, seed=12)
    log(f"drilled, {len(w.closed_bits)} groups, {len(w.plan.sliced_labels)} sliced bonds")
    g = _contraction(w, max_batch_slices=8)
    g.contract()
    got = g.amps.cpu().numpy()
    g.close()
    ref = ocontract.sparse_amplitudes(circ, open_q, closed, sliced_bonds=w.sliced_bonds,
                                      slice_ids=[int(x) for x in w.slice_ids])
    err = metrics.rel_error(got, ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL


def test_drilled_full_size_workload():
    from paper_2111_03011_amd.workload import config_workload
    plain_w = config_workload("sliced")
    w = config_workload("sliced", mode="holes")
    K = 2 * len(w.circuit["holes"])
    c = _contraction(plain_w, max_batch_slices=64)
    c.contract()
    ref = c.amps.cpu().numpy().copy()
    c.close()
    d = _contraction(w, max_batch_slices=64)
    d.contract()
    got = d.amps.cpu().numpy()
    work = d.work()
    d.close()
    f = metrics.fidelity(got, ref)
    log(f"drilled sliced workload: holes {w.circuit['holes']}, work {work:.3e} (plain "
        f"{plain_w.plan.total_flops:.3e}), F over 4096 amplitudes {f:.4f}, 2^-K {2.0 ** -K:.4f}")
    assert work < plain_w.plan.total_flops
    assert 0.25 < f / 2.0 ** -K < 4.0
