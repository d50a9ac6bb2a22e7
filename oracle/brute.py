"""Full circuit unitaries for tiny registers (D^n <= 4096), a route independent of
``sim``: dense one-qudit operators are Kronecker products I x .. x U x .. x I in
qudit-0-first order, and permutation / diagonal gates are built from the paper's
sparse construction (enumerate every digit string, apply the digit rule, set the
single non-zero of each column)."""
from __future__ import annotations

import itertools

import numpy as np

from . import gates


def _index(D, digs):
    n = len(digs)
    return sum(d * D ** (n - 1 - k) for k, d in enumerate(digs))


def kron_1q(D: int, n: int, q: int, U: np.ndarray) -> np.ndarray:
    out = np.array([[1.0 + 0j]])
    for k in range(n):
        out = np.kron(out, U if k == q else np.eye(D))
    return out


def kron_block(D: int, n: int, q0: int, k: int, B: np.ndarray) -> np.ndarray:
    left = np.eye(D ** q0)
    right = np.eye(D ** (n - q0 - k))
    return np.kron(np.kron(left, B), right)


def sparse_perm(D: int, n: int, rule) -> np.ndarray:
    """Operator with <rule(k)|P|k> = 1 for every digit string k."""
    N = D ** n
    P = np.zeros((N, N), dtype=np.complex128)
    for digs in itertools.product(range(D), repeat=n):
        P[_index(D, rule(list(digs))), _index(D, digs)] = 1.0
    return P


def sparse_diag(D: int, n: int, phase) -> np.ndarray:
    N = D ** n
    P = np.zeros((N, N), dtype=np.complex128)
    for digs in itertools.product(range(D), repeat=n):
        i = _index(D, digs)
        P[i, i] = phase(digs)
    return P


def sparse_controlled_rotation(op, D: int, n: int, theta) -> np.ndarray:
    """The controlled rotation from the paper's sparse element rules
    (subsection "Controlled Rotation Gate"): with k_c the control digit, the
    two-level x- and y-type rotations put cos(k_c theta/2) on the j and k levels
    of the target and -i sin(k_c theta/2) (x) or -sin / +sin (y, the
    antisymmetric order of the plain R_y) between them; the z-type rotation puts
    exp(-i k_c theta/2 sqrt(2/(j(j+1))) (-j)^[level = j]) on target levels
    0..j; every other target level keeps its amplitude."""
    kind, c, t = op[0], op[1], op[2]
    th = float(theta[op[-1]])
    N = D ** n
    U = np.zeros((N, N), dtype=np.complex128)
    for digs in itertools.product(range(D), repeat=n):
        col = _index(D, digs)
        kc, kt = digs[c], digs[t]
        half = kc * th / 2
        if kind == "crz":
            j = op[3]
            a = np.sqrt(2.0 / (j * (j + 1)))
            ph = np.exp(-1j * half * a * ((-j) if kt == j else 1)) if kt <= j else 1.0
            U[col, col] = ph
            continue
        j, k = op[3], op[4]
        if kt not in (j, k):
            U[col, col] = 1.0
            continue
        other = list(digs)
        other[t] = k if kt == j else j
        row_other = _index(D, other)
        U[col, col] = np.cos(half)
        if kind == "crx":
            U[row_other, col] = -1j * np.sin(half)
        else:  # <j|R|k> = -sin, <k|R|j> = +sin
            U[row_other, col] = -np.sin(half) if kt == k else np.sin(half)
    return U


def op_unitary(op, D: int, n: int, theta) -> np.ndarray:
    kind = op[0]
    if kind in ("h", "clock", "rx", "ry", "rz"):
        return kron_1q(D, n, op[1], gates.op_matrix(op, D, theta))
    if kind == "x":
        q, s = op[1], op[2]
        return sparse_perm(D, n, lambda d: d[:q] + [(d[q] + s) % D] + d[q + 1:])
    if kind == "u":
        return kron_block(D, n, op[1], op[2], np.asarray(op[3], dtype=np.complex128))
    if kind == "csum":
        c, t = op[1], op[2]

        def rule(d):
            d[t] = (d[t] + d[c]) % D
            return d
        return sparse_perm(D, n, rule)
    if kind == "cshift":
        c, t, sh = op[1], op[2], op[3]

        def rule(d):
            d[t] = (d[t] + (sh[0] if c < 0 else sh[d[c]])) % D
            return d
        return sparse_perm(D, n, rule)
    if kind == "swap":
        a, b = op[1], op[2]

        def rule(d):
            d[a], d[b] = d[b], d[a]
            return d
        return sparse_perm(D, n, rule)
    if kind == "mcx":
        controls, t = list(op[1]), op[2]

        def rule(d):
            prod = 1
            for c in controls:
                prod *= d[c]
            d[t] = (d[t] + prod) % D
            return d
        return sparse_perm(D, n, rule)
    if kind == "cz":
        c, t = op[1], op[2]
        w = gates.omega(D)
        return sparse_diag(D, n, lambda d: w ** ((d[c] * d[t]) % D))
    if kind in ("crx", "cry", "crz"):
        return sparse_controlled_rotation(op, D, n, theta)
    raise ValueError(kind)


def circuit_unitary(circuit, theta=None) -> np.ndarray:
    D, n = circuit.dim, circuit.n
    assert D ** n <= 4096, "brute force is for tiny registers only"
    theta = circuit.theta if theta is None else theta
    U = np.eye(D ** n, dtype=np.complex128)
    for op in circuit.ops:
        U = op_unitary(op, D, n, theta) @ U
    return U
