"""Pins of the oracle's samplers: SplitMix64's published output sequence for seed 0, exact
inverse-CDF decisions on hand-made weights, draw frequencies against the exact law (main
text: one bitstring per group by |psi_hat|^2), the Metropolis chain against its transition
matrix raised to the step count, and frugal rejection sampling against the exact law when
m bounds the weight ratio."""

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


def _chain_law(w, steps):
    """Distribution after `steps` moves of the Metropolis chain with uniform proposals
    (the proposal may be the current state) and acceptance min(1, w_nu / w_mu), started
    uniform: the Markov-chain definition, as a matrix power."""
    l = len(w)
    P = np.zeros((l, l))
    for mu in range(l):
        for nu in range(l):
            if nu != mu:
                P[mu, nu] = min(1.0, w[nu] / w[mu]) / l
        P[mu, mu] = 1.0 - P[mu].sum()
    return np.full(l, 1.0 / l) @ np.linalg.matrix_power(P, steps)


def _chi2(counts, p):
    n = counts.sum()
    return float(np.sum((counts - n * p) ** 2 / (n * p)))


def test_metropolis_follows_the_chain_law_step_by_step():
    w = np.array([0.2, 1.0, 3.0, 8.0])
    a = np.sqrt(w)[None, :].astype(complex)
    draws = sampling.metropolis(a, seed=11, n_samples=40000, steps=3)
    counts = np.bincount(draws[:, 1], minlength=4)
    assert _chi2(counts, _chain_law(w, 3)) < 20          # 3 degrees of freedom
    # the test tells neighbouring step counts apart
    assert _chi2(counts, _chain_law(w, 2)) > 100 and _chi2(counts, _chain_law(w, 4)) > 100


def test_metropolis_reaches_the_squared_amplitude_law():
    rng = np.random.default_rng(5)
    w = rng.uniform(0.5, 1.5, size=16)
    a = (np.sqrt(w) * np.exp(1j * rng.uniform(0, 6.3, size=16)))[None, :]
    draws = sampling.metropolis(a, seed=12, n_samples=8000, steps=60)
    counts = np.bincount(draws[:, 1], minlength=16)
    assert _chi2(counts, w / w.sum()) < 45               # 15 degrees of freedom


def test_metropolis_special_cases():
    # no step: the uniform start; an all-zero group accepts every proposal (the last one)
    a = np.zeros((1, 8), dtype=complex)
    d0 = sampling.metropolis(a, seed=4, n_samples=3, steps=0)
    assert d0[:, 1].tolist() == [min(int(sampling.uniform(4, j) * 8), 7) for j in range(3)]
    d = sampling.metropolis(a, seed=4, n_samples=2, steps=5)
    for j in range(2):
        k0 = j * 11
        assert d[j, 1] == min(int(sampling.uniform(4, k0 + 9) * 8), 7)
    # one nonzero entry is absorbing once proposed; several groups: chain d on group d
    b = np.zeros((3, 4), dtype=complex)
    b[0, 2] = b[1, 0] = b[2, 3] = 1.0
    g = sampling.metropolis(b, seed=9, n_samples=3, steps=200)
    assert g.tolist() == [[0, 2], [1, 0], [2, 3]]


def test_frugal_is_exact_rejection_when_m_bounds_the_ratio():
    rng = np.random.default_rng(6)
    w = rng.uniform(0.1, 2.0, size=16)
    a = np.sqrt(w)[None, :].astype(complex)
    m = float(w.max() * 16 / w.sum())                     # m >= w_nu / mean w for every nu
    draws = sampling.frugal(a, seed=13, n_samples=20000, m=m, trials=1000)
    counts = np.bincount(draws[:, 1], minlength=16)
    assert _chi2(counts, w / w.sum()) < 45               # 15 degrees of freedom
    # a too small m flattens the law (acceptance saturates at 1)
    flat = sampling.frugal(a, seed=13, n_samples=20000, m=0.05, trials=1000)
    assert _chi2(np.bincount(flat[:, 1], minlength=16), w / w.sum()) > 200


def test_frugal_special_cases():
    # equal weights with m = 1: every first proposal is accepted
    a = np.ones((1, 8), dtype=complex)
    d = sampling.frugal(a, seed=21, n_samples=4, m=1.0, trials=5)
    assert d[:, 1].tolist() == [min(int(sampling.uniform(21, 10 * j) * 8), 7) for j in range(4)]
    # an all-zero group rejects everything and keeps the last proposal
    z = np.zeros((2, 8), dtype=complex)
    e = sampling.frugal(z, seed=22, n_samples=2, m=10.0, trials=3)
    assert e.tolist() == [[0, min(int(sampling.uniform(22, 4) * 8), 7)],
                          [1, min(int(sampling.uniform(22, 6 + 4) * 8), 7)]]
