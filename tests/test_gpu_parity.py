"""GPU parity: libtnc (through its C ABI) against the CPU oracle on the same seeded
inputs.  Tolerance: normwise relative error <= 1e-5 for complex64 contraction with FP32
accumulation (the bound the target states); samples are compared exactly on identical
amplitudes and uniforms."""

import numpy as np
import pytest

import synth
from oracle import contract as ocontract
from oracle import metrics, sampling, statevector
from tests.gpu_util import log, random_pair_network, require_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _contraction(net, path, **kw):
    from paper_2111_03011_amd.contractor import Contraction
    return Contraction(net, path, **kw)


def _pair_case(rank_a, rank_b, shared, seed, order_a=None, order_b=None):
    net = random_pair_network(rank_a, rank_b, shared, seed, order_a, order_b)
    c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)), closed_bits=[0])
    c.contract()
    got = c.amps.cpu().numpy()[0]
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    kinds = sorted({l.kind for l in c.launches()})
    c.close()
    return metrics.rel_error(got, ref), kinds


@pytest.mark.parametrize("ra,rb,k", [(12, 7, 5), (13, 8, 6), (11, 6, 6)])
def test_stream_long_k(ra, rb, k):
    """The small-operand stream with K = 32 and 64 (taken by default only up to K = 16;
    TNC_STREAM_MAX_NK=6 moves the limit), against the oracle."""
    import os
    os.environ["TNC_STREAM_MAX_NK"] = "6"
    try:
        err, kinds = _pair_case(ra, rb, k, seed=ra * 100 + rb + k)
    finally:
        os.environ.pop("TNC_STREAM_MAX_NK", None)
    log(f"stream K 2^{k}: rel err {err:.3e} kinds {kinds}")
    assert 2 in kinds and 1 not in kinds
    assert err <= TOL


@pytest.mark.parametrize("ra,rb,k,oa,ob,want", [
    # fused small-operand stream: gate-like operand, K labels spread through the big one
    (14, 4, 2, [5, 0, 6, 7, 8, 9, 10, 11, 1, 12, 13, 2, 3, 4], None, 2),
    (12, 7, 4, None, None, 2),
    # GEMM, operands already grouped ([M][K] x [K][N])
    (16, 14, 6, None, None, 1),
    # GEMM, transposed operands ([K][M] x [N][K])
    (15, 13, 5, list(range(5)) + list(range(5, 15)), list(range(15, 23)) + list(range(5)), 1),
    # GEMM after permutes (labels interleaved)
    (14, 12, 5, [5, 0, 6, 1, 7, 2, 8, 3, 9, 4, 10, 11, 12, 13], None, 1),
    # N = 32 with M >= 128 (128 x 32 tiles)
    (14, 11, 6, None, None, 1),
    # N = 8 and N = 2 (128 x 8 tiles on 16x16x4 matrix instructions), ragged K order
    (18, 10, 7, None, None, 1),
    (16, 8, 7, None, [16, 0, 1, 2, 3, 4, 5, 6], 1),
    # narrow N (<= 16), small M (<= 64), long K with split-K
    (20, 16, 12, None, None, 1),
    (10, 17, 5, None, None, 1),
])
def test_pair_contractions(ra, rb, k, oa, ob, want):
    log(f"pair case ra={ra} rb={rb} k={k}")
    err, kinds = _pair_case(ra, rb, k, seed=ra * 100 + rb, order_a=oa, order_b=ob)
    log(f"  rel err {err:.3e} kinds {kinds}")
    assert want in kinds
    assert err <= TOL


def test_small_amplitudes_match_state_vector():
    from paper_2111_03011_amd.workload import config_workload
    log("small config, 64 amplitudes")
    w = config_workload("small", mode="amplitudes")
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits)
    c.contract()
    got = c.amps.cpu().numpy()[:, 0]
    psi = statevector.simulate(w.circuit)
    ref = psi[w.closed_bits.astype(np.int64)]
    err = metrics.rel_error(got, ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL
    c.close()


def test_small_samples_exact_on_same_amplitudes():
    from paper_2111_03011_amd.workload import config_workload
    cfg = synth.config("small")
    log("small config, all qubits open, 1000 samples")
    w = config_workload("small", mode="samples")
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits)
    norm = c.contract(norm=True)
    amps = c.amps.cpu().numpy()
    psi = statevector.simulate(w.circuit)
    assert metrics.rel_error(amps[0], psi) <= TOL
    assert abs(norm - np.sum(np.abs(amps) ** 2)) <= 1e-12 * max(norm, 1.0)
    seed, k = cfg["samples"]["seed"], cfg["samples"]["count"]
    bits = c.sample(seed, k)
    draws = sampling.sample(amps, seed, k)
    want = sampling.bitstrings(draws, w.closed_bits, w.open_qubits, w.net.n_qubits)
    assert np.array_equal(bits, want)
    # and the draws follow |psi|^2: chi-square over the 16 most likely outcomes + rest
    p = np.abs(psi) ** 2
    top = np.argsort(p)[::-1][:16]
    obs = np.array([np.sum(bits == t) for t in top] + [0])
    obs[-1] = k - obs[:-1].sum()
    exp = np.concatenate([p[top], [1 - p[top].sum()]]) * k
    chi2 = np.sum((obs - exp) ** 2 / exp)
    assert chi2 < 45      # 16 dof, p ~ 2e-4
    c.close()


def _sliced_workload(rows, cols, cycles, seed, open_q, L, max_log2, n_sliced=None):
    from paper_2111_03011_amd.workload import make_workload
    circ = synth.make_circuit(rows, cols, cycles, seed)
    n = circ["n_qubits"]
    closed = synth.group_targets(n, open_q, L, seed + 1)
    return make_workload(circ, open_q, closed, max_log2=max_log2, n_sliced=n_sliced,
                         trials=2, seed=seed)


@pytest.mark.parametrize("shape", [
    (3, 4, 8, 11, [0, 5, 11], 1, 7, 4),     # one group, forced slicing
    (4, 4, 10, 12, [2, 9, 13], 24, 9, None),  # sparse rows (24 groups) and slicing
    (3, 4, 8, 13, [], 40, 8, None),          # amplitude mode (no open qubit), sliced
])
def test_sliced_per_slice_and_sum(shape):
    r, cc, m, seed, open_q, L, max_log2, k = shape
    log(f"sliced case {shape}")
    w = _sliced_workload(r, cc, m, seed, open_q, L, max_log2, k)
    bonds = w.sliced_bonds
    log(f"  {len(bonds)} sliced bonds, {len(w.plan.path)} steps")
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits)
    per = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                      sliced_bonds=bonds, slice_ids=w.slice_ids, per_slice=True)
    for idx in sorted({0, len(w.slice_ids) // 2, len(w.slice_ids) - 1}):
        c.contract_range(idx, 1)
        got = c.amps.cpu().numpy()
        err = metrics.rel_error(got, per[idx])
        log(f"  slice {idx}: rel err {err:.3e}")
        assert err <= TOL
    c.contract()
    got = c.amps.cpu().numpy()
    psi = statevector.simulate(w.circuit)
    ref = statevector.sparse_from_state(psi, w.circuit["n_qubits"], w.open_qubits, w.closed_bits)
    err = metrics.rel_error(got, ref)
    log(f"  full sum rel err {err:.3e}")
    assert err <= TOL
    assert np.allclose(per.sum(axis=0), ref, atol=1e-12)
    c.close()


def test_group_sampling_one_per_group_exact():
    log("one draw per group")
    w = _sliced_workload(4, 4, 10, 21, [1, 6, 11, 12], 50, 11)
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits)
    c.contract()
    amps = c.amps.cpu().numpy()
    bits = c.sample(99, len(w.closed_bits))
    want = sampling.bitstrings(sampling.sample(amps, 99, len(w.closed_bits)), w.closed_bits,
                               w.open_qubits, w.circuit["n_qubits"])
    assert np.array_equal(bits, want)
    c.close()


def test_sliced_config_sampled_slices_full_size():
    """The 5x6 / 14-cycle workload at full size: two of the oracle's eight seeded slices
    compared element by element (one slice per call)."""
    from paper_2111_03011_amd.workload import config_workload
    cfg = synth.config("sliced")
    log("sliced config at full size, single slices")
    w = config_workload("sliced")
    assert len(w.slice_ids) == 1024 and w.plan.cost.peak_log2 <= 26
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits,
                     max_batch_slices=64)
    picks = synth.slice_subset(len(w.plan.sliced_labels), cfg["oracle_slices"]["count"],
                               cfg["oracle_slices"]["seed"])[:2]
    for sid in picks:
        pos = int(np.nonzero(w.slice_ids == sid)[0][0])
        c.contract_range(pos, 1)
        got = c.amps.cpu().numpy()
        ref = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                          sliced_bonds=w.sliced_bonds, slice_ids=[int(sid)])
        err = metrics.rel_error(got, ref)
        log(f"  slice {int(sid)}: rel err {err:.3e}")
        assert err <= TOL
    c.close()


# Largest |error| / rms of the reference over the 4096 amplitudes of a full sum: the
# normwise bound (1e-5) times the few-sigma excursion of the largest of 4096 errors.
MAX_OVER_RMS = 1e-4


def test_sliced_full_sum_matches_stored_oracle_in_the_benchmarked_launch_shape():
    """The whole 1024-slice sum of the 5x6 / 14-cycle workload, contracted as bench.py runs
    it (64 slices per launch sequence, autotuned tiles, one captured graph replayed per
    batch), against the oracle's exact amplitudes (the 30-qubit state vector; the full slice
    set is the unsliced network, Appendix B.2), element by element: normwise error <= 1e-5
    and max |error| / rms <= 1e-4, on the first (capturing) pass and on a replayed pass."""
    from paper_2111_03011_amd.workload import config_workload
    from tests.golden_data import sliced_full_sum
    exact = sliced_full_sum()
    log("sliced config, full 1024-slice sum against the stored oracle amplitudes")
    w = config_workload("sliced")
    assert w.closed_bits.tolist() == [exact.closed]
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits,
                     max_batch_slices=64)
    assert c.batch_slices == 64
    c.autotune(reps=1)
    for rep in range(2):
        norm = c.contract(norm=True)
        got = c.amps.cpu().numpy()[0]
        err = metrics.rel_error(got, exact.amps)
        mx = metrics.max_error_over_rms(got, exact.amps)
        log(f"  pass {rep}: rel err {err:.3e}, max err / rms {mx:.3e}, norm {norm:.6e}")
        assert err <= TOL and mx <= MAX_OVER_RMS
        assert abs(norm - np.sum(np.abs(exact.amps) ** 2)) <= 1e-4 * norm
    c.close()


def test_batches_and_graph_replays_are_bitwise_identical():
    """Slices contracted S at a time (one captured graph per batch) give exactly the
    amplitudes of one-at-a-time eager contraction: the FP64 sum is accumulated in slice
    order whatever the batch size.  The graph is replayed several times with eager work
    and synchronisations in between; every replay must match."""
    import os
    import torch
    log("batches and graph replays")
    w = _sliced_workload(4, 4, 10, 31, [3, 8], 12, 9)
    n = len(w.slice_ids)
    kw = dict(sliced_labels=w.plan.sliced_labels, slice_ids=w.slice_ids,
              open_qubits=w.open_qubits, closed_bits=w.closed_bits)
    os.environ["TNC_NO_GRAPH"] = "1"
    try:
        ref_c = _contraction(w.net, w.plan.path, max_batch_slices=1, **kw)
        ref_c.contract()
        ref = ref_c.amps.cpu().numpy().copy()
        ref_c.close()
    finally:
        os.environ.pop("TNC_NO_GRAPH", None)
    for S in (3, 8):
        c = _contraction(w.net, w.plan.path, max_batch_slices=S, **kw)
        for rep in range(3):
            c.contract()
            got = c.amps.cpu().numpy()
            assert np.array_equal(got, ref), (S, rep, metrics.rel_error(got, ref))
            junk = torch.randn(1 << 16, device="cuda").sum().item()   # eager work in between
            torch.cuda.synchronize()
            assert np.isfinite(junk)
        c.close()
    log(f"  {n} slices, batches 3 and 8 identical to eager one-by-one")


def test_autotuned_plan_matches_oracle_and_recaptures_graph():
    """After the autotuner has re-chosen tiles and split-K for every GEMM of the full-size
    5x6 / 14-cycle plan (batch of 64 slices, the configuration bench.py times), a seeded
    slice still matches the oracle element by element, and the captured graph is rebuilt:
    two graph replays of the whole sum agree bitwise with each other."""
    from paper_2111_03011_amd.workload import config_workload
    cfg = synth.config("sliced")
    log("autotuned sliced config")
    w = config_workload("sliced")
    c = _contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                     slice_ids=w.slice_ids, open_qubits=w.open_qubits,
                     closed_bits=w.closed_bits, max_batch_slices=64)
    c.contract_range(0, 64)
    changed = c.autotune(reps=1)
    log(f"  autotuner changed {changed} launches")
    sid = synth.slice_subset(len(w.plan.sliced_labels), cfg["oracle_slices"]["count"],
                             cfg["oracle_slices"]["seed"])[2]
    pos = int(np.nonzero(w.slice_ids == sid)[0][0])
    c.contract_range(pos, 1)
    got = c.amps.cpu().numpy()
    ref = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                      sliced_bonds=w.sliced_bonds, slice_ids=[int(sid)])
    err = metrics.rel_error(got, ref)
    log(f"  slice {int(sid)}: rel err {err:.3e}")
    assert err <= TOL
    c.contract_range(0, 192)
    a = c.amps.cpu().numpy().copy()
    c.contract_range(0, 192)
    assert np.array_equal(a, c.amps.cpu().numpy())
    c.close()


def _grouped_pair(n_ca, n_oa, n_cb, n_ob, nk, L, seed):
    """Two random tensors sharing nk labels; each carries closed and open output legs.
    Qubits: A's closed, A's open, B's closed, B's open.  L distinct closed parts."""
    from paper_2111_03011_amd.network import TensorNetwork
    rng = np.random.default_rng(seed)
    k = list(range(nk))
    nxt = nk
    ca = list(range(nxt, nxt + n_ca)); nxt += n_ca
    oa = list(range(nxt, nxt + n_oa)); nxt += n_oa
    cb = list(range(nxt, nxt + n_cb)); nxt += n_cb
    ob = list(range(nxt, nxt + n_ob)); nxt += n_ob
    la, lb = ca + oa + k, k + cb + ob
    ta = (rng.normal(size=(2,) * len(la)) + 1j * rng.normal(size=(2,) * len(la))) / np.sqrt(2)
    tb = (rng.normal(size=(2,) * len(lb)) + 1j * rng.normal(size=(2,) * len(lb))) / np.sqrt(2)
    outs = ca + oa + cb + ob
    n = len(outs)
    net = TensorNetwork(n_qubits=n, tensors=[ta, tb], labels=[la, lb], out_label=outs,
                        bond_label={})
    open_q = list(range(n_ca, n_ca + n_oa)) + list(range(n_ca + n_oa + n_cb, n))
    closed = synth.group_targets(n, open_q, L, seed + 1)
    return net, open_q, closed


def _grouped_reference(net, open_q, closed):
    full = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label)
    n = net.n_qubits
    full = full.reshape((2,) * n)
    ref = np.zeros((len(closed), 1 << len(open_q)), dtype=np.complex128)
    for i, cbits in enumerate(closed):
        for mu in range(1 << len(open_q)):
            idx = [(int(cbits) >> (n - 1 - q)) & 1 for q in range(n)]
            for t, q in enumerate(open_q):
                idx[q] = (mu >> (len(open_q) - 1 - t)) & 1
            ref[i, mu] = full[tuple(idx)]
    return ref


@pytest.mark.parametrize("case", [
    # (closed on A, open on A, closed on B, open on B, shared K labels, groups)
    (5, 2, 5, 2, 8, 1024),    # every closed configuration: 32 output rows per shared row
    (6, 3, 3, 4, 7, 300),     # ragged: groups of uneven size, partial 128-row blocks
    (4, 1, 2, 3, 9, 64),      # M = 2 per row, 64 rows per block
])
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_row_stacked_sparse_rows(case, precision):
    """Sparse-row GEMMs whose per-row M is below a tile: output rows sharing one N-side row
    are stacked along M (row mode 2).  Every group's amplitudes match the oracle's full
    pairwise contraction indexed at the group's bits."""
    net, open_q, closed = _grouped_pair(*case, seed=sum(case) + precision)
    log(f"stacked case {case} precision {precision}")
    ref = _grouped_reference(net, open_q, closed)
    tol = {0: TOL, 1: 1e-5, 2: 1e-3}[precision]
    c = _contraction(net, [(0, 1)], open_qubits=open_q, closed_bits=closed, precision=precision)
    modes = [l.row_mode for l in c.launches() if l.kind == 1]
    assert modes == [2], modes
    c.contract()
    err = metrics.rel_error(c.amps.cpu().numpy(), ref)
    c.close()
    log(f"  stacked: rel err {err:.3e}")
    assert err <= tol


def test_degenerate_cases():
    """Edge cases of the path: contracting zero slices leaves psi_hat at zero (norm 0); a
    group whose amplitudes are all zero draws mu = floor(u * l) exactly as the oracle does;
    a batch size that does not divide the slice count (ragged last batch) and a batch
    larger than the slice count give the one-at-a-time sum."""
    w = _sliced_workload(3, 4, 8, 11, [0, 5, 11], 6, 9, 4)   # 16 slices, 6 groups
    kw = dict(sliced_labels=w.plan.sliced_labels, slice_ids=w.slice_ids,
              open_qubits=w.open_qubits, closed_bits=w.closed_bits)
    n = len(w.slice_ids)
    log(f"degenerate cases: {n} slices, {len(w.closed_bits)} groups")
    c = _contraction(w.net, w.plan.path, **kw)
    c.contract_range(0, 0)
    zero = c.amps.cpu().numpy()
    assert not zero.any()
    bits = c.sample(5, len(w.closed_bits))
    want = sampling.bitstrings(sampling.sample(zero, 5, len(w.closed_bits)), w.closed_bits,
                               w.open_qubits, w.circuit["n_qubits"])
    assert np.array_equal(bits, want)
    c.contract()
    ref = c.amps.cpu().numpy().copy()
    c.close()
    for S in (3, 4 * n):
        c = _contraction(w.net, w.plan.path, max_batch_slices=S, **kw)
        c.contract()
        got = c.amps.cpu().numpy()
        assert metrics.rel_error(got, ref) <= 1e-6, (S, metrics.rel_error(got, ref))
        c.close()
    oref = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                       sliced_bonds=w.sliced_bonds,
                                       slice_ids=[int(x) for x in w.slice_ids])
    assert metrics.rel_error(ref, oref) <= TOL


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("config", [0, 1, 2, 3, 4, 5, 7, 8])
def test_every_tile_configuration(config, precision):
    """Each GEMM tile configuration (forced with TNC_GEMM_CONFIG), without and with split-K
    (TNC_SPLITK_BLOCKS), on a product whose M and N are smaller than some tiles (partial
    tiles) and whose operands are read in interleaved label orders.  The split-precision
    forms have no 128x8 tile and take 128x16 for it."""
    import os
    log(f"tile configuration {config}, precision {precision}")
    tol = {0: TOL, 1: 1e-5, 2: 1e-3}[precision]
    # A: 6 free labels interleaved with 10 shared; B: 4 free labels after the shared ones
    order_a = [10, 0, 11, 1, 12, 2, 13, 3, 14, 4, 15, 5, 6, 7, 8, 9]
    net = random_pair_network(16, 14, 10, 4242 + config, order_a, None)
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    for blocks in ("1", "1000000"):     # split-K off, then as many splits as allowed
        os.environ["TNC_GEMM_CONFIG"] = str(config)
        os.environ["TNC_SPLITK_BLOCKS"] = blocks
        try:
            c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)),
                             closed_bits=[0], precision=precision)
        finally:
            os.environ.pop("TNC_GEMM_CONFIG", None)
            os.environ.pop("TNC_SPLITK_BLOCKS", None)
        g = [l for l in c.launches() if l.kind == 1]
        assert len(g) == 1 and g[0].config == (1 if precision and config == 5 else config)
        assert (g[0].k_splits > 1) == (blocks != "1")
        c.contract()
        err = metrics.rel_error(c.amps.cpu().numpy()[0], ref)
        log(f"  split-K {g[0].k_splits}: rel err {err:.3e}")
        assert err <= tol
        c.close()


@pytest.mark.parametrize("precision", [0, 2, 1])
@pytest.mark.parametrize("rank_a,rank_b,shared,interleave", [
    (14, 16, 4, True),    # K = 16, N = 4096 wider than a workgroup's 512 columns
    (12, 13, 3, False),   # K = 8, N = 1024
    (11, 8, 1, True),     # K = 2, N = 128 (several output rows per pass)
    (9, 6, 0, False),     # K = 1: an outer product
    (8, 7, 2, True),      # K = 4, N = 32, M = 64 (one partial stage)
    (9, 12, 4, False),    # K = 16 on the matrix cores: M = 32 (one 32-row chunk), N = 256
    (13, 12, 4, True),    # K = 16 on the matrix cores: N = 256 (one column block), M = 512
    (10, 10, 4, True),    # K = 16, N = 64: below a 256-column block, vector ALUs
])
def test_short_k_vector_kernel(rank_a, rank_b, shared, interleave, precision):
    """Configuration 6 (products with K <= 16, chosen for wide outputs: on the vector ALUs,
    or on the FP32 matrix cores for K = 16 and N >= 256) forced on pair products of several
    shapes, operands read in interleaved label orders; every form computes it in FP32."""
    import os
    log(f"short-K kernel: ranks {rank_a}, {rank_b}, K 2^{shared}, precision {precision}")
    fa = rank_a - shared
    k = list(range(shared))
    free_a = list(range(shared, shared + fa))
    order_a = None
    if interleave and shared:
        order_a = []
        for i in range(max(fa, shared)):
            if i < fa:
                order_a.append(free_a[i])
            if i < shared:
                order_a.append(k[i])
    net = random_pair_network(rank_a, rank_b, shared, 900 + rank_a * 10 + rank_b, order_a, None)
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    os.environ["TNC_GEMM_CONFIG"] = "6"
    try:
        c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)), closed_bits=[0],
                         precision=precision)
    finally:
        os.environ.pop("TNC_GEMM_CONFIG", None)
    g = [l for l in c.launches() if l.kind == 1]
    if not g:
        c.close()
        pytest.skip("this product runs as a small-operand stream")
    assert len(g) == 1 and g[0].config == 6, [(l.config, l.m, l.n, l.k) for l in g]
    c.contract()
    err = metrics.rel_error(c.amps.cpu().numpy()[0], ref)
    c.close()
    log(f"  M {g[0].m} N {g[0].n} K {g[0].k}: rel err {err:.3e}")
    assert err <= TOL


def test_short_k_vector_kernel_rows_and_fold():
    """Configuration 6 on sparse-state steps: output rows with gathered operand rows, and
    rows folded into M, against the oracle's per-group contraction."""
    import os
    log("short-K kernel with rows")
    for case in [(3, 7, 1, 6, 3, 12), (3, 7, 0, 6, 3, 8), (3, 7, 1, 8, 4, 12), (3, 7, 0, 8, 4, 8)]:
        net, open_q, closed = _grouped_pair(*case, seed=77)
        ref = _grouped_reference(net, open_q, closed)
        os.environ["TNC_GEMM_CONFIG"] = "6"
        try:
            c = _contraction(net, [(0, 1)], open_qubits=open_q, closed_bits=closed)
        finally:
            os.environ.pop("TNC_GEMM_CONFIG", None)
        g = [l for l in c.launches() if l.kind == 1]
        if not g or g[0].config != 6:
            c.close()
            continue
        c.contract()
        err = metrics.rel_error(c.amps.cpu().numpy(), ref)
        log(f"  case {case}: rows {g[0].rows} M {g[0].m} N {g[0].n} K {g[0].k} mode {g[0].row_mode}: rel err {err:.3e}")
        c.close()
        assert err <= TOL


@pytest.mark.parametrize("case", [
    (3, 5, 2, 1, 9, 24),    # rows of M 32, N 2, K 512 (the 53-qubit share's narrow step)
    (3, 4, 2, 2, 7, 12),    # M 16, N 4, K 128
    (3, 3, 2, 0, 10, 12),   # M 8, N 1, K 1024
    (3, 6, 2, 1, 7, 16),    # M 64, N 2, K 128
    (2, 4, 3, 1, 11, 12),   # M 16, N 2, K 2048
])
@pytest.mark.parametrize("precision", [0, 2, 1])
def test_rows_of_narrow_long_k_products(case, precision):
    """Sparse-state steps whose rows are small products over a long contraction (one wave
    per row, k spread over the lanes and summed across them, in FP32 in every form), forced
    through configuration 5, against the oracle's per-group contraction."""
    import os
    net, open_q, closed = _grouped_pair(*case, seed=91)
    ref = _grouped_reference(net, open_q, closed)
    os.environ["TNC_GEMM_CONFIG"] = "5"
    # neither split-K nor row stacking: the narrow-row kernel takes the step
    os.environ["TNC_SPLITK_BLOCKS"] = "1"
    os.environ["TNC_NO_STACK"] = "1"
    try:
        c = _contraction(net, [(0, 1)], open_qubits=open_q, closed_bits=closed, precision=precision)
    finally:
        for k in ("TNC_GEMM_CONFIG", "TNC_SPLITK_BLOCKS", "TNC_NO_STACK"):
            os.environ.pop(k, None)
    g = [l for l in c.launches() if l.kind == 1]
    if not g or g[0].config != 5:
        c.close()
        pytest.skip("this product runs on another kernel in this form")
    assert g[0].k_splits == 1
    log(f"narrow rows {case}, precision {precision}: rows {g[0].rows} M {g[0].m} N {g[0].n} K {g[0].k}")
    c.contract()
    err = metrics.rel_error(c.amps.cpu().numpy(), ref)
    c.close()
    log(f"  rel err {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("config", [7, 8])
@pytest.mark.parametrize("precision", [0, 2, 1])
@pytest.mark.parametrize("order", ["plain", "interleaved"])
def test_split_big_tile_full_and_partial(config, precision, order):
    """The eight-wave tiles (7: 128 x 128, 8: 256 x 64 complex; complex64 and split
    precision) on products spanning several tiles in M and N, operands in plain and
    interleaved label orders, without and with split-K."""
    import os
    shared = 9
    free_a, free_b = 10, 9          # M = 1024, N = 512 with 10 and 9 free labels
    k = list(range(shared))
    fa = list(range(shared, shared + free_a))
    order_a = None
    if order == "interleaved":
        order_a = [x for pair in zip(fa, k) for x in pair] + fa[len(k):]
    net = random_pair_network(free_a + shared, free_b + shared, shared, 555 + precision, order_a, None)
    ref = ocontract.contract_path(net.tensors, net.labels, [(0, 1)], net.out_label).reshape(-1)
    tol = {0: 1e-5, 1: 1e-5, 2: 1e-3}[precision]
    for blocks in ("1", "1000000"):
        os.environ["TNC_GEMM_CONFIG"] = str(config)
        os.environ["TNC_SPLITK_BLOCKS"] = blocks
        try:
            c = _contraction(net, [(0, 1)], open_qubits=list(range(net.n_qubits)), closed_bits=[0],
                             precision=precision)
        finally:
            os.environ.pop("TNC_GEMM_CONFIG", None)
            os.environ.pop("TNC_SPLITK_BLOCKS", None)
        g = [l for l in c.launches() if l.kind == 1]
        assert len(g) == 1 and g[0].config == config
        c.contract()
        err = metrics.rel_error(c.amps.cpu().numpy()[0], ref)
        c.close()
        log(f"  tile {config}, precision {precision}, {order}, split-K {g[0].k_splits}: rel err {err:.3e}")
        assert err <= tol
