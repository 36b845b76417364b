"""Split-precision form (BF16 hi+lo products, FP32 accumulation) against the oracle.

Bound stated for the split form: normwise relative amplitude error <= 1e-3 and
1 - fidelity <= 1e-6 on every case here (the per-product rounding is about 2^-16
relative; the errors measured on the GPU are printed)."""

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import metrics, statevector
from tests.gpu_util import log, random_pair_network, require_gpu

pytestmark = pytest.mark.gpu
SPLIT_TOL = 1e-3
SPLIT_INFIDELITY = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _contraction(net, path, **kw):
    from paper_2111_03011_amd.contractor import Contraction
    return Contraction(net, path, **kw)


@pytest.mark.parametrize("ra,rb,k", [(16, 14, 6), (20, 16, 12), (10, 17, 5), (14, 12, 5)])
def test_split_pair_gemm(ra, rb, k):
    from paper_2111_03011_amd import tnc
    net = random_pair_network(ra, rb, k, seed=ra * 7 + rb)
    c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)), closed_bits=[0],
                     precision=tnc.TNC_BF16X3)
    c.contract()
    got = c.amps.cpu().numpy()[0]
    c.close()
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    err = metrics.rel_error(got, ref)
    log(f"bf16x3 pair {ra},{rb},{k}: rel err {err:.3e}")
    assert err <= SPLIT_TOL


def test_split_small_amplitudes():
    from paper_2111_03011_amd import tnc
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("small", mode="samples")
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits,
                     precision=tnc.TNC_BF16X3)
    c.contract()
    got = c.amps.cpu().numpy()[0]
    c.close()
    psi = statevector.simulate(w.circuit)
    err, fid = metrics.rel_error(got, psi), metrics.fidelity(got, psi)
    log(f"bf16x3 small config: rel err {err:.3e}, 1-F {1 - fid:.3e}")
    assert err <= SPLIT_TOL and 1 - fid <= SPLIT_INFIDELITY


def test_split_sliced_config_one_slice_and_sum():
    """Full-size sliced workload: one seeded slice against the oracle, and the whole
    1024-slice sum against the complex64 path."""
    from paper_2111_03011_amd import tnc
    from paper_2111_03011_amd.workload import config_workload
    cfg = synth.config("sliced")
    w = config_workload("sliced")
    kw = dict(sliced_labels=w.plan.sliced_labels, slice_ids=w.slice_ids,
              open_qubits=w.open_qubits, closed_bits=w.closed_bits, max_batch_slices=64)
    cs = _contraction(w.net, w.plan.path, precision=tnc.TNC_BF16X3, **kw)
    sid = int(synth.slice_subset(len(w.plan.sliced_labels), cfg["oracle_slices"]["count"],
                                 cfg["oracle_slices"]["seed"])[0])
    cs.contract_range(int(np.nonzero(w.slice_ids == sid)[0][0]), 1)
    got = cs.amps.cpu().numpy()
    ref = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                      sliced_bonds=w.sliced_bonds, slice_ids=[sid])
    err = metrics.rel_error(got, ref)
    log(f"bf16x3 sliced config slice {sid}: rel err {err:.3e}")
    assert err <= SPLIT_TOL
    cs.contract()
    split = cs.amps.cpu().numpy().copy()
    cs.close()
    c64 = _contraction(w.net, w.plan.path, **kw)
    c64.contract()
    plain = c64.amps.cpu().numpy()
    c64.close()
    err, fid = metrics.rel_error(split, plain), metrics.fidelity(split, plain)
    log(f"bf16x3 vs complex64, 1024-slice sum: rel diff {err:.3e}, 1-F {1 - fid:.3e}")
    assert err <= SPLIT_TOL and 1 - fid <= SPLIT_INFIDELITY
