"""Pins of the oracle's sampler: SplitMix64's published output sequence for seed 0, exact
inverse-CDF decisions on hand-made weights, and draw frequencies against the exact law
(main text: one bitstring per group by |psi_hat|^2)."""

import numpy as np

from oracle import sampling


def test_splitmix64_published_sequence():
    # First outputs of SplitMix64 started from state 0 (reference implementation).
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [sampling.splitmix64_output(0, j) for j in range(3)] == want


def test_uniform_range_and_mean():
    u = np.array([sampling.uniform(1234, j) for j in range(20000)])
    assert u.min() >= 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 0.01
    hist = np.histogram(u, bins=10, range=(0, 1))[0]
    chi2 = np.sum((hist - 2000) ** 2 / 2000)
    assert chi2 < 30          # 9 degrees of freedom, p ~ 4e-4


def test_draw_index_hand_cases():
    assert sampling.draw_index(np.array([0.0, 1.0, 0.0]), 0.999) == 1
    assert sampling.draw_index(np.array([1.0, 1.0]), 0.25) == 0
    assert sampling.draw_index(np.array([1.0, 1.0]), 0.5) == 1   # c_0 = 1 is not > 1
    assert sampling.draw_index(np.array([1.0, 1.0]), 0.75) == 1
    assert sampling.draw_index(np.zeros(4), 0.6) == 2             # all-zero group: uniform


def test_frequencies_follow_squared_amplitudes():
    rng = np.random.default_rng(0)
    a = rng.normal(size=8) + 1j * rng.normal(size=8)
    p = np.abs(a) ** 2 / np.sum(np.abs(a) ** 2)
    draws = sampling.sample(a[None, :], seed=77, n_samples=20000)
    counts = np.bincount(draws[:, 1], minlength=8)
    chi2 = np.sum((counts - 20000 * p) ** 2 / (20000 * p))
    assert chi2 < 30          # 7 degrees of freedom


def test_one_draw_per_group_and_bitstrings():
    amps = np.array([[1, 0, 0, 0], [0, 0, 0, 1j], [0, 1, 0, 0]], dtype=complex)
    d = sampling.sample(amps, seed=3, n_samples=3)
    assert d[:, 0].tolist() == [0, 1, 2] and d[:, 1].tolist() == [0, 3, 1]
    # n = 4, open qubits [3, 0] (qubit 3 is the most significant bit of mu)
    bits = sampling.bitstrings(d, [0b0110, 0b0100, 0b0010], [3, 0], 4)
    assert bits.tolist() == [0b0110, 0b1101, 0b1010]
