"""Error, fidelity, XEB and efficiency formulas (oracle; test infrastructure only)."""

from __future__ import annotations

import numpy as np


def rel_error(test, ref) -> float:
    """Normwise relative error ||test - ref||_2 / ||ref||_2 over all requested amplitudes."""
    test = np.asarray(test, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(test - ref) / den) if den > 0 else float(np.linalg.norm(test))


def max_error_over_rms(test, ref) -> float:
    test = np.asarray(test, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    return float(np.max(np.abs(test - ref)) / rms) if rms > 0 else float(np.max(np.abs(test)))


def fidelity(test, ref) -> float:
    """|<ref|test>|^2 / (||ref||^2 ||test||^2) (Appendix D compares full state vectors;
    here it is taken over whatever set of amplitudes is given)."""
    test = np.asarray(test, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    num = abs(np.vdot(ref, test)) ** 2
    den = np.vdot(ref, ref).real * np.vdot(test, test).real
    return float(num / den)


def linear_xeb(n: int, probs_of_samples) -> float:
    """Appendix D: F_XEB = 2^n / N_s * sum_i P(s_i) - 1, P the exact probabilities."""
    p = np.asarray(probs_of_samples, dtype=np.float64)
    return float((2.0 ** n) * p.mean() - 1.0)


def full_space_normalisation(n: int, L: int, l: int, norm: float) -> float:
    """Results: the 2^n-space normalisation estimated from the sparse norm; for n = 53
    and L*l = 2^26 this is 2^27 * N."""
    return (2.0 ** n) / (L * l) * norm


def gpu_efficiency(t_c: float, peak_flops: float, seconds: float) -> float:
    """Table I caption: 8 T_c / (P t), T_c counted in complex multiply-adds."""
    return 8.0 * t_c / (peak_flops * seconds)


def collision_ratio(probs) -> float:
    """2^n * sum p^2 for a full distribution: 2 for Porter-Thomas (deep random
    circuits), 1 for the uniform distribution."""
    p = np.asarray(probs, dtype=np.float64).ravel()
    return float(p.size * np.sum(p * p))
