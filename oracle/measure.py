"""Measurement in FP64: probabilities, marginals, diagonal expectation values."""
from __future__ import annotations

import numpy as np

from . import gates, sim


def probs(psi: np.ndarray) -> np.ndarray:
    """p_x = |psi_x|^2 over the full basis (Born rule)."""
    return np.abs(psi) ** 2


def marginal(psi: np.ndarray, D: int, n: int, qudits) -> np.ndarray:
    """Marginal distribution of the listed qudits: p(y) = sum over all x whose
    digits on ``qudits`` equal y of |psi_x|^2.  Bin index y = sum_i y_i D^(m-1-i)
    in the listed order (what the paper's measure(index=...) returns as p)."""
    qudits = list(qudits)
    p = probs(psi).reshape((D,) * n)
    others = [a for a in range(n) if a not in qudits]
    s = p.sum(axis=tuple(others)) if others else p
    # s has the measured axes in increasing qudit order; reorder to the listed order
    order = sorted(qudits)
    s = np.transpose(s, [order.index(q) for q in qudits])
    return np.ascontiguousarray(s).reshape(-1)


def sample_inverse_cdf(p: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Measurement outcomes for the uniforms u in [0, 1) by inversion of the
    cumulative distribution of p (the histogram the paper's measure(...,
    shots) returns, section "Code style"): outcome y is the first index with
    cumsum(p)[y] > u * sum(p), or the last bin of non-zero probability when
    no such index exists."""
    c = np.cumsum(np.asarray(p, dtype=np.float64))
    idx = np.searchsorted(c, np.asarray(u, dtype=np.float64) * c[-1], side="right")
    # a product u * sum(p) that reaches sum(p) has no bin above it: u = 1, a
    # subnormal sum (the product then rounds up to it), or a zero sum.  Such a
    # draw belongs to the last bin with non-zero probability (bin 0 for a zero sum)
    return np.where(idx >= len(c), np.searchsorted(c, c[-1], side="left"), idx)


def sample_counts(p: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Histogram of the outcomes sample_inverse_cdf(p, u)."""
    return np.bincount(sample_inverse_cdf(p, u), minlength=len(p))


def z_diag(D: int) -> np.ndarray:
    """Diagonal of the clock operator Z = diag(w^k)."""
    w = gates.omega(D)
    return np.array([w ** k for k in range(D)], dtype=np.complex128)


def term_table(D: int, term) -> np.ndarray:
    q, name = term
    if name == "z":
        return z_diag(D)
    return np.asarray(name, dtype=np.complex128)


def expect_diag(psi: np.ndarray, D: int, n: int, terms) -> complex:
    """<O> = <psi| O |psi> for O = sum_t d_t(x_{q_t}) diagonal:
    sum_x |psi_x|^2 sum_t d_t(x_{q_t})."""
    dig = sim.digits_of(D, n, np.arange(D ** n))
    f = np.zeros(D ** n, dtype=np.complex128)
    for t in terms:
        f += term_table(D, t)[dig[t[0]]]
    return complex(np.sum(probs(psi) * f))


def hermitian_part_diag(D: int, n: int, terms) -> np.ndarray:
    """Diagonal of (O + O^dagger)/2, so that Re<psi|O|psi> = <psi|H_O|psi>."""
    dig = sim.digits_of(D, n, np.arange(D ** n))
    f = np.zeros(D ** n, dtype=np.float64)
    for t in terms:
        f += term_table(D, t).real[dig[t[0]]]
    return f
