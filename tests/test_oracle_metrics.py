"""Pins of the metric formulas against the paper's printed numbers (Table I, Results,
Discussions) and against closed forms."""

import numpy as np

from oracle import metrics


def test_table_one_totals():
    # overall T_c = 2^16 x (head + tail), original and branch-merged columns
    assert abs(2 ** 16 * (2.3816e13 + 2.9425e13) / 3.489e18 - 1) < 1e-3
    assert abs(2 ** 16 * (6.967e13 + 8.796e13) / 1.033e19 - 1) < 1e-3
    # Discussions: 8 T_c flops without branch merging
    assert abs(8 * 3.489e18 / 2.79e19 - 1) < 1e-3


def test_table_one_efficiencies():
    peak = 15.7e12                        # V100 single-precision peak
    head = metrics.gpu_efficiency(6.967e13, peak, 112)
    tail = metrics.gpu_efficiency(8.796e13, peak, 315)
    total = metrics.gpu_efficiency(6.967e13 + 8.796e13, peak, 427)
    assert abs(head - 0.3176) < 0.002
    assert abs(tail - 0.1427) < 0.002
    assert abs(total - 0.1885) < 0.002


def test_fidelity_estimate_and_normalisation():
    assert abs(2 ** -8 * 0.9564714760983217 - 0.0037) < 1e-4
    assert metrics.full_space_normalisation(53, 2 ** 20, 64, 1.0) == 2.0 ** 27
    assert 2 ** 45 // 2 ** 16 == 2 ** 29 and 2 ** 20 * 2 ** 6 == 2 ** 26


def test_error_and_fidelity_closed_forms():
    ref = np.array([1, 1j, -1, 0.5])
    assert metrics.rel_error(ref, ref) == 0
    assert np.isclose(metrics.rel_error(1.1 * ref, ref), 0.1)
    assert np.isclose(metrics.fidelity(np.exp(0.3j) * 2 * ref, ref), 1.0)
    orth = np.array([1, 0, 0, 0]), np.array([0, 1, 0, 0])
    assert metrics.fidelity(*orth) == 0
    assert np.isclose(metrics.max_error_over_rms(ref + 0.01, ref), 0.01 / np.sqrt(np.mean(np.abs(ref) ** 2)))


def test_linear_xeb_limits():
    n = 10
    p = np.random.default_rng(1).exponential(size=1 << n)
    p /= p.sum()
    # uniform samples: expectation of 2^n P(s) is 1 -> XEB 0
    assert abs(metrics.linear_xeb(n, p) - 0.0) < 1e-12
    # exact samples from p: E[2^n P] = 2^n sum p^2 -> XEB = collision - 1 (~1 for PT)
    assert np.isclose(metrics.linear_xeb(n, [np.sum(p * p)]), metrics.collision_ratio(p) - 1)
