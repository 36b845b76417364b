"""The 53-qubit share at full size (6x9 grid minus one site, 20 cycles, largest intermediate
2^30, 2^14 groups x 6 open qubits = 2^20 amplitudes, 98 sliced bonds).

The oracle cannot contract this network (its own greedy path for a single group peaks at
2^26 to 2^33 elements depending on tie-breaks), so parity here is a property that holds at
any size: the amplitudes of a group computed inside the sparse state (rows of all 2^14
groups, gathered operand rows) equal those of a separate contraction with that group
alone (no rows at all) - the same slices, the same path."""

import numpy as np
import pytest

from oracle import metrics
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_large_sparse_state_equals_single_groups():
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("large")
    assert w.n_amplitudes == 1 << 20 and w.plan.cost.peak_log2 <= 30
    ids = list(w.slice_ids[:2])
    log(f"large: {len(w.plan.sliced_labels)} sliced bonds, slices {[hex(int(i)) for i in ids]}")
    full = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels, slice_ids=ids,
                       open_qubits=w.open_qubits, closed_bits=w.closed_bits, max_batch_slices=1)
    full.contract()
    amps = full.amps.cpu().numpy()
    full.close()
    assert np.all(np.isfinite(amps))
    rng = np.random.default_rng(5)
    for g in sorted(rng.choice(len(w.closed_bits), size=3, replace=False)):
        one = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels, slice_ids=ids,
                          open_qubits=w.open_qubits, closed_bits=w.closed_bits[g:g + 1],
                          max_batch_slices=1)
        one.contract()
        got = one.amps.cpu().numpy()[0]
        one.close()
        err = metrics.rel_error(amps[g], got)
        log(f"  group {g}: sparse state vs alone rel diff {err:.2e}")
        assert err <= 1e-5
