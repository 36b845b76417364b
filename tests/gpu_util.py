"""Helpers shared by the GPU tests (no arithmetic of the method here)."""

from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def require_gpu():
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def random_pair_network(rank_a, rank_b, shared, seed, order_a=None, order_b=None):
    """Two random complex tensors sharing `shared` labels; every other label is an open
    output leg.  order_* give each tensor's label order as lists of label ids."""
    from paper_2111_03011_amd.network import TensorNetwork
    rng = np.random.default_rng(seed)
    n_free_a, n_free_b = rank_a - shared, rank_b - shared
    k = list(range(shared))
    fa = list(range(shared, shared + n_free_a))
    fb = list(range(shared + n_free_a, shared + n_free_a + n_free_b))
    la = order_a if order_a is not None else fa + k
    lb = order_b if order_b is not None else k + fb
    ta = (rng.normal(size=(2,) * rank_a) + 1j * rng.normal(size=(2,) * rank_a)) / np.sqrt(2)
    tb = (rng.normal(size=(2,) * rank_b) + 1j * rng.normal(size=(2,) * rank_b)) / np.sqrt(2)
    outs = fa + fb
    return TensorNetwork(n_qubits=len(outs), tensors=[ta, tb], labels=[list(la), list(lb)],
                         out_label=outs, bond_label={})
