"""Split-precision forms (BF16 and FP16 hi+lo products, FP32 accumulation) against the
oracle.

Bounds stated for the split forms: normwise relative amplitude error <= 1e-3 for BF16x3
(about 16 significant bits per operand) and <= 1e-5 for FP16x3 (about 22 bits, operands
scaled by a power of two per slice), and 1 - fidelity <= 1e-6 on every case here; the
errors measured on the GPU are printed."""

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import metrics, statevector
from tests.gpu_util import log, random_pair_network, require_gpu

pytestmark = pytest.mark.gpu
SPLIT_TOL = 1e-3
SPLIT_INFIDELITY = 1e-6
FORMS = [("bf16x3", 2, 1e-3), ("fp16x3", 1, 1e-5)]   # (name, tnc precision, error bound)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _contraction(net, path, **kw):
    from paper_2111_03011_amd.contractor import Contraction
    return Contraction(net, path, **kw)


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
@pytest.mark.parametrize("ra,rb,k", [(16, 14, 6), (20, 16, 12), (10, 17, 5), (14, 12, 5)])
def test_split_pair_gemm(ra, rb, k, form):
    name, prec, tol = form
    net = random_pair_network(ra, rb, k, seed=ra * 7 + rb)
    c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)), closed_bits=[0],
                     precision=prec)
    c.contract()
    got = c.amps.cpu().numpy()[0]
    c.close()
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    err = metrics.rel_error(got, ref)
    log(f"{name} pair {ra},{rb},{k}: rel err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("scale_a,scale_b", [(2.0 ** -40, 2.0 ** 30), (2.0 ** 25, 2.0 ** 25),
                                             (2.0 ** -50, 2.0 ** -50)])
def test_fp16_scaling_keeps_range(scale_a, scale_b):
    """FP16 alone holds magnitudes between about 6e-8 and 65504; operands far outside that
    range (tiny, huge, and a product of both) still contract to the oracle's result within
    the FP16x3 bound, because each operand is scaled by a power of two per slice."""
    from paper_2111_03011_amd import tnc
    net = random_pair_network(15, 13, 7, seed=99)
    net.tensors[0] = net.tensors[0] * scale_a
    net.tensors[1] = net.tensors[1] * scale_b
    c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)), closed_bits=[0],
                     precision=tnc.TNC_FP16X3)
    c.contract()
    got = c.amps.cpu().numpy()[0]
    c.close()
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    err = metrics.rel_error(got, ref)
    log(f"fp16x3 operands scaled by {scale_a:.1e}, {scale_b:.1e}: rel err {err:.3e}")
    assert np.all(np.isfinite(got)) and err <= 1e-5


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
def test_split_small_amplitudes(form):
    from paper_2111_03011_amd.workload import config_workload
    name, prec, tol = form
    w = config_workload("small", mode="samples")
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits,
                     precision=prec)
    c.contract()
    got = c.amps.cpu().numpy()[0]
    c.close()
    psi = statevector.simulate(w.circuit)
    err, fid = metrics.rel_error(got, psi), metrics.fidelity(got, psi)
    log(f"{name} small config: rel err {err:.3e}, 1-F {1 - fid:.3e}")
    assert err <= tol and 1 - fid <= SPLIT_INFIDELITY


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
def test_split_sliced_config_one_slice_and_sum(form):
    """Full-size sliced workload: one seeded slice against the oracle, and the whole
    1024-slice sum against the complex64 path."""
    from paper_2111_03011_amd.workload import config_workload
    name, prec, tol = form
    cfg = synth.config("sliced")
    w = config_workload("sliced")
    kw = dict(sliced_labels=w.plan.sliced_labels, slice_ids=w.slice_ids,
              open_qubits=w.open_qubits, closed_bits=w.closed_bits, max_batch_slices=64)
    cs = _contraction(w.net, w.plan.path, precision=prec, **kw)
    sid = int(synth.slice_subset(len(w.plan.sliced_labels), cfg["oracle_slices"]["count"],
                                 cfg["oracle_slices"]["seed"])[0])
    cs.contract_range(int(np.nonzero(w.slice_ids == sid)[0][0]), 1)
    got = cs.amps.cpu().numpy()
    ref = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                      sliced_bonds=w.sliced_bonds, slice_ids=[sid])
    err = metrics.rel_error(got, ref)
    log(f"{name} sliced config slice {sid}: rel err {err:.3e}")
    assert err <= tol
    cs.contract()
    split = cs.amps.cpu().numpy().copy()
    cs.close()
    c64 = _contraction(w.net, w.plan.path, **kw)
    c64.contract()
    plain = c64.amps.cpu().numpy()
    c64.close()
    err, fid = metrics.rel_error(split, plain), metrics.fidelity(split, plain)
    log(f"{name} vs complex64, 1024-slice sum: rel diff {err:.3e}, 1-F {1 - fid:.3e}")
    assert err <= max(tol, 1e-5) and 1 - fid <= SPLIT_INFIDELITY


def _chain_network(seed, scales):
    """A -- B -- C with 12 labels shared by A and B, 8 by B and C, and 6, 2 and 6 open legs;
    contracted as (A B) C, so the second product reads the first one's output."""
    from paper_2111_03011_amd.network import TensorNetwork
    rng = np.random.default_rng(seed)
    k1, k2 = list(range(12)), list(range(12, 20))
    fa, fb, fc = list(range(20, 26)), list(range(26, 28)), list(range(28, 34))
    labels = [fa + k1, k1 + k2 + fb, k2 + fc]
    tensors = []
    for lab, s in zip(labels, scales):
        r = len(lab)
        t = (rng.normal(size=(2,) * r) + 1j * rng.normal(size=(2,) * r)) / np.sqrt(2)
        tensors.append(t * s)
    outs = fa + fb + fc
    return TensorNetwork(n_qubits=len(outs), tensors=tensors, labels=labels, out_label=outs,
                         bond_label={})


@pytest.mark.parametrize("blocks", ["1", "1000000"])
def test_fp16_scale_of_a_produced_operand(blocks):
    """The FP16 scale of an intermediate operand comes from its producer's epilogue (the
    GEMM, or the split-K reduction when the product is split along K; here 16 splits, the
    wide reduction).  Operand magnitudes far from 1 make a wrong or missing maximum show up
    as overflow or lost precision."""
    import os
    from paper_2111_03011_amd import tnc
    net = _chain_network(77, (2.0 ** 30, 2.0 ** 20, 2.0 ** -40))
    path = [(0, 1), (0, 2)]
    ref = ocontract.contract_path(net.tensors, net.labels, path, net.out_label).reshape(-1)
    os.environ["TNC_SPLITK_BLOCKS"] = blocks
    try:
        c = _contraction(net, path, open_qubits=list(range(net.n_qubits)), closed_bits=[0],
                         precision=tnc.TNC_FP16X3)
    finally:
        os.environ.pop("TNC_SPLITK_BLOCKS", None)
    g = [l for l in c.launches() if l.kind == 1]
    assert len(g) == 2
    if blocks != "1":
        assert g[0].k_splits >= 8, [l.k_splits for l in g]
    c.contract()
    got = c.amps.cpu().numpy()[0]
    c.close()
    err = metrics.rel_error(got, ref)
    log(f"fp16x3 chain, split-K {[l.k_splits for l in g]}: rel err {err:.3e}")
    assert np.all(np.isfinite(got)) and err <= 1e-5


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
@pytest.mark.parametrize("config", [0, 1, 3, 4])
@pytest.mark.parametrize("free_a", [7, 6])
def test_split_m_fast_operand_paired_loads(config, free_a, form):
    """An M-side operand whose fastest label is an m label is loaded two rows per 16-byte
    access in the 128-row tiles; full (M = 128) and partial (M = 64) tiles, split-K off and
    on, against the oracle."""
    import os
    name, prec, tol = form
    shared, free_b = 9, 5
    k = list(range(shared))
    fa = list(range(shared, shared + free_a))
    order_a = k + fa                                   # m labels last: m is A's fastest index
    net = random_pair_network(free_a + shared, free_b + shared, shared, 700 + free_a, order_a, None)
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    for blocks in ("1", "1000000"):
        os.environ["TNC_GEMM_CONFIG"] = str(config)
        os.environ["TNC_SPLITK_BLOCKS"] = blocks
        try:
            c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)),
                             closed_bits=[0], precision=prec)
        finally:
            os.environ.pop("TNC_GEMM_CONFIG", None)
            os.environ.pop("TNC_SPLITK_BLOCKS", None)
        g = [l for l in c.launches() if l.kind == 1]
        assert len(g) == 1 and g[0].m == 1 << free_a and g[0].config == config
        c.contract()
        err = metrics.rel_error(c.amps.cpu().numpy()[0], ref)
        c.close()
        log(f"{name} m-fast A, M {1 << free_a}, config {config}, split-K {g[0].k_splits}: rel err {err:.3e}")
        assert err <= tol
