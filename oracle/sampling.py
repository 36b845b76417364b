"""Sampling one bitstring per group by |psi_hat|^2 (oracle; test infrastructure only).

Main text, sampling paragraph: from each group of l correlated amplitudes one bitstring
is drawn with probability proportional to |psi_hat_i^mu|^2.  `sample` draws from that law
directly; `metropolis` runs the paper's in-group Markov chain (Metropolis algorithm) and
`frugal` the frugal rejection sampling the paper names as the faster alternative for
Porter-Thomas distributed groups.  With a single group, k bitstrings are drawn from it
(k independent draws or chains).

Uniforms come from SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) used as a counter-based generator: draw j uses the state
seed + (j+1)*gamma, i.e. the (j+1)-th output of the sequential generator started at
`seed`, and u_j = (output >> 11) * 2^-53.

Inverse CDF: with w_mu = re^2 + im^2 (each product and the sum rounded to float64),
c_mu = sum_{nu <= mu} w_nu (summed in mu order, float64) and
T = c_{l-1}, the draw is the smallest mu with c_mu > u * T.  A group whose amplitudes are
all zero draws mu = floor(u * l).
"""

from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_mix(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_output(seed: int, j: int) -> int:
    """The (j+1)-th output of SplitMix64 started from state `seed`."""
    return splitmix64_mix((int(seed) + (int(j) + 1) * GOLDEN_GAMMA) & MASK64)


def uniform(seed: int, j: int) -> float:
    return (splitmix64_output(seed, j) >> 11) * (2.0 ** -53)


def draw_index(weights: np.ndarray, u: float) -> int:
    c = 0.0
    cum = []
    for w in weights:
        c += float(w)
        cum.append(c)
    total = cum[-1]
    if total == 0.0:
        return min(int(u * len(weights)), len(weights) - 1)
    target = u * total
    for mu, cm in enumerate(cum):
        if cm > target:
            return mu
    return len(weights) - 1


def sample(amps: np.ndarray, seed: int, n_samples: int) -> np.ndarray:
    """amps: [L][l] complex.  L == 1: n_samples draws from the one group (u_j, j = 0..k-1).
    L > 1: n_samples must equal L, one draw per group (group i uses u_i).
    Returns (group index, mu) pairs as an int64 array of shape [n_samples, 2]."""
    amps = np.asarray(amps)
    L = amps.shape[0]
    a = amps.astype(np.complex128)
    w = a.real * a.real + a.imag * a.imag
    out = np.zeros((n_samples, 2), dtype=np.int64)
    if L == 1:
        for j in range(n_samples):
            out[j] = (0, draw_index(w[0], uniform(seed, j)))
    else:
        if n_samples != L:
            raise ValueError("with several groups, draw exactly one sample per group")
        for i in range(L):
            out[i] = (i, draw_index(w[i], uniform(seed, i)))
    return out


def _index(u: float, l: int) -> int:
    return min(int(u * l), l - 1)


def _groups_of_draws(amps, n_samples):
    L = amps.shape[0]
    if L > 1 and n_samples != L:
        raise ValueError("with several groups, draw exactly one sample per group")
    return [0] * n_samples if L == 1 else list(range(L))


def metropolis(amps: np.ndarray, seed: int, n_samples: int, steps: int) -> np.ndarray:
    """In-group Metropolis chains (main text, sampling paragraph).

    Draw d runs one chain on its group (group d, or the only group) over mu in [0, l):
    with k0 = d (2 steps + 1), the start is mu_0 = floor(u_k0 l); step t = 1..steps proposes
    nu = floor(u_(k0+2t-1) l) uniformly and moves there iff w_nu >= u_(k0+2t) w_mu (accepted
    with probability min(1, w_nu / w_mu)); the draw is mu_steps.  Returns (group, mu) pairs."""
    amps = np.asarray(amps).astype(np.complex128)
    w = amps.real * amps.real + amps.imag * amps.imag
    l = amps.shape[1]
    out = np.zeros((n_samples, 2), dtype=np.int64)
    for d, g in enumerate(_groups_of_draws(amps, n_samples)):
        k0 = d * (2 * steps + 1)
        mu = _index(uniform(seed, k0), l)
        for t in range(1, steps + 1):
            nu = _index(uniform(seed, k0 + 2 * t - 1), l)
            if float(w[g, nu]) >= uniform(seed, k0 + 2 * t) * float(w[g, mu]):
                mu = nu
        out[d] = (g, mu)
    return out


def frugal(amps: np.ndarray, seed: int, n_samples: int, m: float, trials: int) -> np.ndarray:
    """Frugal rejection sampling (main text, sampling paragraph; Markov et al. 2018).

    Draw d, with k0 = 2 d trials, proposes nu_t = floor(u_(k0+2t) l), t = 0..trials-1, and
    accepts the first with u_(k0+2t+1) (m S) < w_nu l, S = sum of w over the group in mu
    order (acceptance probability min(1, w_nu / (m mean w))); after `trials` rejections it
    keeps the last proposal.  Returns (group, mu) pairs."""
    amps = np.asarray(amps).astype(np.complex128)
    w = amps.real * amps.real + amps.imag * amps.imag
    l = amps.shape[1]
    totals = []
    for g in range(amps.shape[0]):
        c = 0.0
        for x in w[g]:
            c += float(x)
        totals.append(c)
    out = np.zeros((n_samples, 2), dtype=np.int64)
    for d, g in enumerate(_groups_of_draws(amps, n_samples)):
        k0 = 2 * d * trials
        ms = float(m) * totals[g]
        for t in range(trials):
            nu = _index(uniform(seed, k0 + 2 * t), l)
            if uniform(seed, k0 + 2 * t + 1) * ms < float(w[g, nu]) * float(l):
                break
        out[d] = (g, nu)
    return out


def bitstrings(draws: np.ndarray, closed_bits, open_qubits, n: int) -> np.ndarray:
    """Full uint64 bitstrings of (group, mu) draws."""
    open_qubits = list(open_qubits)
    no = len(open_qubits)
    out = []
    for gi, mu in draws:
        x = int(closed_bits[int(gi)])
        for t, q in enumerate(open_qubits):
            if (int(mu) >> (no - 1 - t)) & 1:
                x |= 1 << (n - 1 - q)
        out.append(x)
    return np.asarray(out, dtype=np.uint64)
