"""Gate matrices in FP64 (paper, Appendix "Matrix form of the quantum gates").

Levels are 0-indexed: the paper derives its formulas with levels 1..D and states
that the programmed version uses 0..D-1 (end of subsection "Generalized rotation
gate").
"""
from __future__ import annotations

import numpy as np


def omega(D: int) -> complex:
    """omega = exp(2 pi i / D) (subsection "Generalized phase-shift gate")."""
    return np.exp(2j * np.pi / D)


def shift(D: int, s: int = 1) -> np.ndarray:
    """Generalized NOT X_s: |x> -> |x + s mod D> (subsection "Generalized NOT gate").
    Column x holds a single 1 in row (x + s) mod D."""
    m = np.zeros((D, D), dtype=np.complex128)
    for x in range(D):
        m[(x + s) % D, x] = 1.0
    return m


def clock(D: int, a: int = 1) -> np.ndarray:
    """Phase-shift gate P = diag(1, w, ..., w^(D-1)) (subsection "Generalized
    phase-shift gate"); ``a`` raises it to the a-th power, diag(w^(a k))."""
    w = omega(D)
    return np.diag([w ** (a * k) for k in range(D)]).astype(np.complex128)


def fourier(D: int) -> np.ndarray:
    """Fourier / generalized Hadamard: H_mn = w^(m n) / sqrt(D) (subsection
    "Fourier gate")."""
    w = omega(D)
    return np.array([[w ** (m * n) for n in range(D)] for m in range(D)],
                    dtype=np.complex128) / np.sqrt(D)


def gm_sym(D: int, j: int, k: int) -> np.ndarray:
    """Symmetric generalized Gell-Mann matrix S_x^{jk} = |j><k| + |k><j|, j < k."""
    assert 0 <= j < k < D
    m = np.zeros((D, D), dtype=np.complex128)
    m[j, k] = 1.0
    m[k, j] = 1.0
    return m


def gm_asym(D: int, j: int, k: int) -> np.ndarray:
    """Antisymmetric generalized Gell-Mann matrix S_y^{jk} = -i|j><k| + i|k><j|, j < k."""
    assert 0 <= j < k < D
    m = np.zeros((D, D), dtype=np.complex128)
    m[j, k] = -1j
    m[k, j] = 1j
    return m


def gm_diag(D: int, j: int) -> np.ndarray:
    """Diagonal generalized Gell-Mann matrix S_z^j, j = 1..D-1.

    Reading of the garbled sum in the paper: with 0-indexed levels, levels
    0..j-1 carry +1, level j carries -j, all others 0, scaled by
    sqrt(2 / (j (j+1))).  This is the reading that reproduces the paper's D=2
    example diag(1, -1) and its R_z element formula (exponent (-j) on the
    level after the first j)."""
    assert 1 <= j < D
    d = np.zeros(D)
    d[:j] = 1.0
    d[j] = -float(j)
    return np.diag(d * np.sqrt(2.0 / (j * (j + 1)))).astype(np.complex128)


def expm_hermitian(S: np.ndarray, theta: float) -> np.ndarray:
    """exp(-i theta S / 2) for Hermitian S through its eigendecomposition
    S = V diag(lam) V^dagger (the rotation definition R = e^{-i theta S / 2},
    subsection "Generalized rotation gate")."""
    lam, V = np.linalg.eigh(S)
    return (V * np.exp(-0.5j * theta * lam)) @ V.conj().T


def rx(D: int, j: int, k: int, theta: float) -> np.ndarray:
    return expm_hermitian(gm_sym(D, j, k), theta)


def ry(D: int, j: int, k: int, theta: float) -> np.ndarray:
    return expm_hermitian(gm_asym(D, j, k), theta)


def rz(D: int, j: int, theta: float) -> np.ndarray:
    return expm_hermitian(gm_diag(D, j), theta)


def generator(op, D: int) -> np.ndarray:
    """The Hermitian generator S of a rotation descriptor, R = exp(-i theta S/2)."""
    kind = op[0]
    if kind == "rx":
        return gm_sym(D, op[2], op[3])
    if kind == "ry":
        return gm_asym(D, op[2], op[3])
    if kind == "rz":
        return gm_diag(D, op[2])
    raise ValueError(f"{kind} has no generator")


def crot_generator(op, D: int) -> np.ndarray:
    """Generator S of a controlled rotation descriptor ("crx", c, t, j, k, p),
    ("cry", c, t, j, k, p) or ("crz", c, t, j, p)."""
    kind = op[0]
    if kind == "crx":
        return gm_sym(D, op[3], op[4])
    if kind == "cry":
        return gm_asym(D, op[3], op[4])
    if kind == "crz":
        return gm_diag(D, op[3])
    raise ValueError(f"{kind} is not a controlled rotation")


def crot_mats(op, D: int, theta: np.ndarray) -> list:
    """The differentiable controlled rotation sum_m |m><m| (x) R(m theta)
    (Appendix, subsection "Controlled Rotation Gate"): the target matrix for
    each control level m, R(m theta) = exp(-i m theta S / 2)."""
    S = crot_generator(op, D)
    t = float(theta[op[-1]])
    return [expm_hermitian(S, m * t) for m in range(D)]


def op_matrix(op, D: int, theta: np.ndarray) -> np.ndarray:
    """Dense matrix of a one-qudit descriptor (or of a custom block)."""
    kind = op[0]
    if kind == "h":
        return fourier(D)
    if kind == "x":
        return shift(D, op[2])
    if kind == "clock":
        return clock(D, op[2])
    if kind in ("rx", "ry", "rz"):
        return expm_hermitian(generator(op, D), float(theta[op[-1]]))
    if kind == "u":
        return np.asarray(op[3], dtype=np.complex128)
    raise ValueError(f"{kind} is not a one-qudit matrix gate")
