"""Serving (continuous batching) on the GPU: every request's amplitudes and samples are the
same when it runs alone as when it runs in a mix of concurrent requests (draws copied back
in several chunks included); admission waits for arena room; a request that can never fit
is refused at submission; a request whose launch fails fails alone."""

import os
import time

import numpy as np
import pytest

import synth
from oracle import metrics, statevector
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _requests():
    from paper_2111_03011_amd.workload import make_workload
    out = []
    specs = [  # rows, cols, cycles, seed, open qubits, groups, size bound, samples
        (3, 4, 8, 101, [0, 5, 11], 1, 7, 200),
        (4, 4, 10, 102, [2, 9, 13], 24, 9, 24),
        (3, 3, 9, 103, [], 40, 7, 0),
        (4, 5, 10, 104, [1, 7, 18], 8, 10, 8),
        (4, 4, 12, 105, [0, 15], 1, 8, 500),
        (3, 5, 10, 106, [4, 10], 16, 8, 0),
        (3, 4, 8, 107, [0, 3, 6, 9], 1, 7, 150000),   # draws in three chunks of <= 65536
    ]
    for r, c, m, seed, open_q, L, bound, k in specs:
        circ = synth.make_circuit(r, c, m, seed)
        n = circ["n_qubits"]
        closed = synth.group_targets(n, open_q, L, seed + 1)
        w = make_workload(circ, open_q, closed, max_log2=bound, trials=2, seed=seed)
        out.append((w, k, seed + 7))
    return out


def _alone(w, k, seed):
    from paper_2111_03011_amd.contractor import Contraction
    c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels, slice_ids=w.slice_ids,
                    open_qubits=w.open_qubits, closed_bits=w.closed_bits, max_batch_slices=8)
    c.contract()
    amps = c.amps.cpu().numpy().copy()
    bits = c.sample(seed, k) if k else None
    c.close()
    return amps, bits


def _submit(srv, w, k, seed):
    return srv.submit(w.net, w.plan.path, w.plan.sliced_labels, w.slice_ids, w.open_qubits,
                      w.closed_bits, n_samples=k, seed=seed, max_batch_slices=8)


def _wait(srv, ids, timeout=120):
    res, t0 = {}, time.time()
    while len(res) < len(ids):
        for rid in ids:
            if rid not in res:
                r = srv.poll(rid)
                if r is not None:
                    res[rid] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.002)
    return res


def test_results_same_alone_and_in_the_mix():
    from paper_2111_03011_amd.serving import Server
    reqs = _requests()
    alone = [_alone(*r) for r in reqs]
    srv = Server(arena_bytes=256 << 20, max_slots=3, chunk_batches=2)
    ids = [_submit(srv, *r) for r in reqs]
    res = _wait(srv, ids)
    for (w, k, seed), (a_amps, a_bits), rid in zip(reqs, alone, ids):
        r = res[rid]
        assert np.array_equal(r["amps"], a_amps), f"request {rid} differs in the mix"
        if k:
            assert np.array_equal(r["bits"], a_bits)
        psi = statevector.simulate(w.circuit)
        ref = statevector.sparse_from_state(psi, w.circuit["n_qubits"], w.open_qubits, w.closed_bits)
        err = metrics.rel_error(r["amps"], ref)
        log(f"  request {rid}: {r['slices']} slices, rel err vs state vector {err:.2e}, "
            f"latency {1e3 * (r['t_done'] - r['t_submit']):.1f} ms")
        assert err <= 1e-5
    # all six were submitted together; with three slots some ran concurrently
    admits = sorted(res[i]["t_admit"] for i in ids)
    dones = sorted(res[i]["t_done"] for i in ids)
    assert admits[1] < dones[0]
    srv.close()


def test_admission_waits_for_room_and_refuses_what_never_fits():
    from paper_2111_03011_amd import tnc
    from paper_2111_03011_amd.serving import Server
    reqs = _requests()[:3]
    foot = []
    probe = Server(arena_bytes=256 << 20, max_slots=1)
    for r in reqs:
        rid = _submit(probe, *r)
        foot.append(_wait(probe, [rid])[rid]["footprint"])
    probe.close()
    # room for the largest request only: requests run one at a time, all finish
    srv = Server(arena_bytes=int(max(foot)) + 256, max_slots=3, chunk_batches=1)
    ids = [_submit(srv, *r) for r in reqs]
    res = _wait(srv, ids)
    order = sorted(ids, key=lambda i: res[i]["t_admit"])
    for a, b in zip(order, order[1:]):
        if foot[ids.index(a)] + foot[ids.index(b)] > max(foot) + 256:
            assert res[b]["t_admit"] >= res[a]["t_done"]
    srv.close()
    small = Server(arena_bytes=4096, max_slots=1)
    with pytest.raises(tnc.TncError) as e:
        _submit(small, *reqs[0])
    assert e.value.code == tnc.TNC_E_OOM
    small.close()


def test_a_failed_launch_fails_one_request_and_spares_the_others():
    """TNC_FAULT=launch:N makes the N-th launch unit the server enqueues fail before it is
    enqueued (forced from the host; no kernel faults).  Exactly one request reports the
    failure; every other request of the mix returns the same bits as when run alone, and the
    server keeps serving afterwards."""
    from paper_2111_03011_amd import tnc
    from paper_2111_03011_amd.serving import Server
    reqs = _requests()
    alone = [_alone(*r) for r in reqs]
    os.environ["TNC_FAULT"] = "launch:4"
    try:
        srv = Server(arena_bytes=256 << 20, max_slots=3, chunk_batches=1)
    finally:
        os.environ.pop("TNC_FAULT")
    ids = [_submit(srv, *r) for r in reqs]
    failed, t0 = [], time.time()
    res = {}
    while len(res) + len(failed) < len(ids):
        for rid in ids:
            if rid in res or rid in failed:
                continue
            try:
                r = srv.poll(rid)
            except tnc.TncError as e:
                assert e.code == tnc.TNC_E_HIP and "TNC_FAULT" in str(e)
                failed.append(rid)
                continue
            if r is not None:
                res[rid] = r
        assert time.time() - t0 < 120, "requests did not finish"
        time.sleep(0.002)
    log(f"  failed: {failed}; finished: {sorted(res)}")
    assert len(failed) == 1
    for (w, k, seed), (a_amps, a_bits), rid in zip(reqs, alone, ids):
        if rid in failed:
            continue
        assert np.array_equal(res[rid]["amps"], a_amps), f"request {rid} differs"
        if k:
            assert np.array_equal(res[rid]["bits"], a_bits)
    # the failed request again, on the same server: it runs through
    k = ids.index(failed[0])
    rid = _submit(srv, *reqs[k])
    again = _wait(srv, [rid])[rid]
    assert np.array_equal(again["amps"], alone[k][0])
    srv.close()
