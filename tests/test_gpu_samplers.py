"""The paper's in-group samplers on the GPU (main text, sampling paragraph): Metropolis
chains and frugal rejection sampling through the C ABI, compared draw for draw with the
oracle on the same amplitudes and uniforms (bit-exact: both sides take every accept/reject
decision in FP64 with the same rounding), for one group (many draws, several chunks) and
for one draw per group."""

import numpy as np
import pytest

import synth
from oracle import sampling
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _contracted(w):
    from paper_2111_03011_amd.contractor import Contraction
    c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                    slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits)
    c.contract()
    return c, c.amps.cpu().numpy()


def _bits(w, draws):
    return sampling.bitstrings(draws, w.closed_bits, w.open_qubits, w.net.n_qubits)


@pytest.mark.parametrize("n,steps,trials", [(3000, 20, 64), (70000, 3, 6)])
def test_one_group_many_draws(n, steps, trials):
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("small", mode="samples")          # 12 open qubits, l = 4096
    log(f"one group: {n} draws, metropolis {steps} steps, frugal {trials} trials")
    c, amps = _contracted(w)
    got = c.sample_metropolis(7, n, steps)
    assert np.array_equal(got, _bits(w, sampling.metropolis(amps, 7, n, steps)))
    got = c.sample_frugal(8, n, 10.0, trials)
    assert np.array_equal(got, _bits(w, sampling.frugal(amps, 8, n, 10.0, trials)))
    c.close()


def test_one_draw_per_group():
    from paper_2111_03011_amd.workload import make_workload
    circ = synth.make_circuit(4, 4, 10, 21)
    closed = synth.group_targets(16, [1, 6, 11, 12], 50, 22)
    w = make_workload(circ, [1, 6, 11, 12], closed, max_log2=11, trials=2, seed=21)
    log(f"one draw per group: {len(w.closed_bits)} groups of 16")
    c, amps = _contracted(w)
    L = len(w.closed_bits)
    got = c.sample_metropolis(31, L, 40)
    assert np.array_equal(got, _bits(w, sampling.metropolis(amps, 31, L, 40)))
    got = c.sample_frugal(32, L, 4.0, 32)
    assert np.array_equal(got, _bits(w, sampling.frugal(amps, 32, L, 4.0, 32)))
    from paper_2111_03011_amd import tnc
    with pytest.raises(tnc.TncError):
        c.sample_metropolis(1, L + 1, 5)                   # one draw per group
    with pytest.raises(tnc.TncError):
        c.sample_metropolis(1, L, -1)
    with pytest.raises(tnc.TncError):
        c.sample_frugal(1, L, 0.0, 4)
    with pytest.raises(tnc.TncError):
        c.sample_frugal(1, L, 10.0, 0)
    c.close()
