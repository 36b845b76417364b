"""tnc_sample_noalloc (the sampler for callers that cannot allocate: its buffers live in a
static device array inside the library) against tnc_sample (the same draws out of the
plan's workspace), bit for bit, through the C ABI: two calls in a row on each plan, the
second with a smaller input (fewer draws, or a plan with fewer groups), so that contents
the first call left in the shared static buffer cannot leak into the second."""

import numpy as np
import pytest

from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _draw_both(c, seed, n):
    from paper_2111_03011_amd import tnc
    stream = c._stream(None)
    want = c.sample(seed, n)
    got = tnc.tnc_sample_noalloc(c._plan, c.amps.data_ptr(), seed, n, stream)
    return want, got


def test_noalloc_matches_workspace_sampler_one_group():
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("small", mode="samples")
    c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels, slice_ids=w.slice_ids,
                    open_qubits=w.open_qubits, closed_bits=w.closed_bits)
    c.contract()
    for seed, n in ((1003, 5000), (77, 300), (5, 0)):
        log(f"noalloc one group (4096 amplitudes): seed {seed}, {n} draws")
        want, got = _draw_both(c, seed, n)
        assert got.shape == (n,) and np.array_equal(got, want)
    c.close()


def test_noalloc_matches_workspace_sampler_groups_then_fewer_groups():
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import make_workload
    import synth
    circ = synth.make_circuit(3, 4, 8, 1001)
    n = circ["n_qubits"]
    for L in (200, 24):
        closed = synth.group_targets(n, [1, 6, 10], L, 900 + L)
        w = make_workload(circ, [1, 6, 10], closed, max_log2=20, seed=3)
        c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                        slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits)
        c.contract()
        log(f"noalloc {L} groups of 8 amplitudes")
        want, got = _draw_both(c, 31 + L, L)
        assert np.array_equal(got, want)
        c.close()


def test_noalloc_rejects_plans_beyond_its_buffer():
    """One group of 2^22 amplitudes needs 32 MiB of running sums: more than the 16 MiB
    static buffer, so the call fails with TNC_E_INVALID before any device work."""
    from paper_2111_03011_amd import tnc
    from paper_2111_03011_amd.contractor import Contraction
    from tests.gpu_util import random_pair_network
    net = random_pair_network(14, 10, 1, seed=4)
    c = Contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)), closed_bits=[0])
    assert net.n_qubits == 22
    with pytest.raises(tnc.TncError) as e:
        tnc.tnc_sample_noalloc(c._plan, c.amps.data_ptr(), 1, 10, c._stream(None))
    assert e.value.code == tnc.TNC_E_INVALID and "scratch" in str(e.value)
    c.close()
