"""Scale records: every form keeps values inside the range of its arithmetic.

A slice of a large sliced network can have amplitudes far below FP32's smallest normal
number (the 53-qubit share's slices sit near 1e-39), and operand products can leave
FP32's range in either direction.  Each tensor carries a power-of-two exponent per slice
and operands are rescaled exactly while loaded, so the results below match the oracle
(complex128) within each form's bound even though the true values lie outside FP32's
range.  Bounds: complex64 and FP16x3 1e-5, BF16x3 1e-3 (normwise)."""

import os

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import metrics, statevector
from tests.gpu_util import log, random_pair_network, require_gpu

pytestmark = pytest.mark.gpu
FORMS = [("c64", 0, 1e-5), ("bf16x3", 2, 1e-3), ("fp16x3", 1, 1e-5)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _contraction(net, path, **kw):
    from paper_2111_03011_amd.contractor import Contraction
    return Contraction(net, path, **kw)


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
@pytest.mark.parametrize("scale_a,scale_b,ra,rb,k", [
    (2.0 ** -75, 2.0 ** -70, 16, 14, 6),     # product ~2^-145: below FP32's subnormals
    (2.0 ** 70, 2.0 ** 68, 16, 14, 6),       # product ~2^138: above FP32's largest value
    (2.0 ** -80, 2.0 ** 5, 14, 4, 2),        # small-operand stream
])
def test_pair_outside_fp32_range(scale_a, scale_b, ra, rb, k, form):
    name, prec, tol = form
    net = random_pair_network(ra, rb, k, seed=ra * 31 + rb)
    net.tensors[0] = net.tensors[0] * scale_a
    net.tensors[1] = net.tensors[1] * scale_b
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)), closed_bits=[0],
                     precision=prec)
    c.contract()
    got = c.amps.cpu().numpy()[0]
    kinds = sorted({l.kind for l in c.launches()})
    c.close()
    err = metrics.rel_error(got, ref)
    log(f"{name} pair {ra},{rb},{k} scaled {scale_a:.1e} x {scale_b:.1e} (kinds {kinds}): "
        f"rel err {err:.3e}")
    assert np.all(np.isfinite(got)) and err <= tol


def _chain(seed, scales):
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


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
@pytest.mark.parametrize("blocks", ["1", "1000000"])
def test_chain_exponents_carry_through_split_k(blocks, form):
    """(A B) C with A B far below FP32's range: the second product reads an operand whose
    stored values were rescaled, its exponent comes from the first product (written by the
    GEMM, largest component folded in by the GEMM or, with 16 splits, by the reduction)."""
    name, prec, tol = form
    net = _chain(5, (2.0 ** -60, 2.0 ** -60, 2.0 ** -30))
    path = [(0, 1), (0, 2)]
    ref = ocontract.contract_path(net.tensors, net.labels, path, net.out_label).reshape(-1)
    os.environ["TNC_SPLITK_BLOCKS"] = blocks
    try:
        c = _contraction(net, path, open_qubits=list(range(net.n_qubits)), closed_bits=[0],
                         precision=prec)
    finally:
        os.environ.pop("TNC_SPLITK_BLOCKS", None)
    g = [l for l in c.launches() if l.kind == 1]
    c.contract()
    got = c.amps.cpu().numpy()[0]
    c.close()
    err = metrics.rel_error(got, ref)
    log(f"{name} chain, split-K {[l.k_splits for l in g]}: rel err {err:.3e}")
    assert np.all(np.isfinite(got)) and err <= tol


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
@pytest.mark.parametrize("mode", ["amplitudes", "samples"])
def test_scaled_circuit_network_through_every_step_kind(mode, form):
    """The 3x4 / 8-cycle network with every leaf multiplied by 2^-6: the amplitudes are
    2^(-6 x leaves) times the state vector's (about 2^-250, far below FP32), reached through
    streams with shared and per-row small operands, GEMMs, sparse rows and the FP64 sum."""
    from paper_2111_03011_amd.workload import config_workload
    name, prec, tol = form
    w = config_workload("small", mode=mode)
    net = w.net
    scaled = type(net)(n_qubits=net.n_qubits, tensors=[t * 2.0 ** -6 for t in net.tensors],
                       labels=net.labels, out_label=net.out_label, bond_label=net.bond_label)
    c = _contraction(scaled, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits,
                     precision=prec)
    c.contract()
    got = c.amps.cpu().numpy()
    kinds = sorted({l.kind for l in c.launches()})
    c.close()
    psi = statevector.simulate(w.circuit)
    if mode == "samples":
        ref = psi.reshape(1, -1)
    else:
        ref = psi[w.closed_bits.astype(np.int64)].reshape(-1, 1)
    ref = ref * 2.0 ** (-6 * len(net.tensors))
    err = metrics.rel_error(got, ref)
    log(f"{name} small config ({mode}), leaves x 2^-6 ({len(net.tensors)} leaves, kinds {kinds}): "
        f"rel err {err:.3e}, |amp| ~ {np.abs(ref).max():.1e}")
    assert np.all(np.isfinite(got)) and err <= tol


def test_sliced_slices_through_records_match_oracle():
    """One seeded slice of the 5x6 / 14-cycle workload per form, against the oracle (the
    records are on in every form; here they rescale nothing, the values stay near 1)."""
    from paper_2111_03011_amd.workload import config_workload
    cfg = synth.config("sliced")
    w = config_workload("sliced")
    sid = int(synth.slice_subset(len(w.plan.sliced_labels), cfg["oracle_slices"]["count"],
                                 cfg["oracle_slices"]["seed"])[3])
    ref = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                      sliced_bonds=w.sliced_bonds, slice_ids=[sid])
    pos = int(np.nonzero(w.slice_ids == sid)[0][0])
    for name, prec, tol in FORMS:
        c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                         slice_ids=w.slice_ids, open_qubits=w.open_qubits,
                         closed_bits=w.closed_bits, max_batch_slices=64, precision=prec)
        c.contract_range(pos, 1)
        err = metrics.rel_error(c.amps.cpu().numpy(), ref)
        c.close()
        log(f"{name} sliced slice {sid}: rel err {err:.3e}")
        assert err <= tol
