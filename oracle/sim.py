"""State vectors and gate application in FP64 (plain definitions).

Basis index: for digits (x_0, ..., x_{n-1}) the decimal representation is
x = sum_k x_k D^(n-1-k), so qudit 0 is the most significant digit (subsection
"Generalized CNOT gate", decimal representation).  A state is a complex128
vector of D^n amplitudes in that order.
"""
from __future__ import annotations

import numpy as np

from . import gates


def index_of(D: int, digits) -> int:
    """Decimal representation j = sum_k j_k D^(n-1-k)."""
    n = len(digits)
    return int(sum(int(d) * D ** (n - 1 - k) for k, d in enumerate(digits)))


def digits_of(D: int, n: int, x):
    """Digits (x_0..x_{n-1}) of index/indices x, qudit 0 first."""
    x = np.asarray(x, dtype=np.int64)
    return [(x // D ** (n - 1 - k)) % D for k in range(n)]


def basis_state(D: int, n: int, digits=None) -> np.ndarray:
    """|j_0 j_1 ... j_{n-1}> as a dense vector (the paper's State('j0-j1-...'))."""
    psi = np.zeros(D ** n, dtype=np.complex128)
    psi[0 if digits is None else index_of(D, digits)] = 1.0
    return psi


def parse_state_string(s: str):
    """'0-1-3' -> [0, 1, 3] (digits joined by '-')."""
    return [int(t) for t in s.split("-")]


def apply_matrix(psi: np.ndarray, D: int, n: int, qudits, U: np.ndarray) -> np.ndarray:
    """psi'[x] = sum_y U[x_S, y_S] psi[x with the digits on S replaced by y_S],
    where S = qudits (in the listed order, first listed = most significant row
    digit of U).  This is the action of the operator that is U on the qudits S
    and the identity on the others."""
    qudits = list(qudits)
    k = len(qudits)
    t = psi.reshape((D,) * n)
    Ut = np.asarray(U, dtype=np.complex128).reshape((D,) * (2 * k))
    # contract U's input indices with the state's axes S
    out = np.tensordot(Ut, t, axes=(list(range(k, 2 * k)), qudits))
    # tensordot puts U's output indices first; move them back to the positions S
    out = np.moveaxis(out, list(range(k)), qudits)
    return np.ascontiguousarray(out).reshape(-1)


def apply_1q(psi, D, n, q, U):
    """One-qudit gate U on qudit q: psi[h, :, l] <- U psi[h, :, l] with the state
    viewed as [D^q][D][D^(n-1-q)]."""
    v = psi.reshape(D ** q, D, D ** (n - 1 - q))
    return np.einsum("ab,hbl->hal", U, v).reshape(-1)


def apply_digit_map(psi: np.ndarray, D: int, n: int, fn) -> np.ndarray:
    """Permutation gate given by a map of digit vectors: the amplitude of |x>
    moves to |fn(x)>.  ``fn`` takes the list of digit arrays and returns the new
    list.  This is the paper's sparse construction (enumerate every digit string,
    apply the digit rule, read off the target index)."""
    N = D ** n
    x = np.arange(N, dtype=np.int64)
    dig = digits_of(D, n, x)
    new = fn([d.copy() for d in dig])
    dest = np.zeros(N, dtype=np.int64)
    for k in range(n):
        dest += new[k] * D ** (n - 1 - k)
    out = np.zeros_like(psi)
    out[dest] = psi
    return out


def apply_cshift(psi, D, n, c, t, shifts):
    """x_t -> x_t + shifts[x_c] mod D (c = -1: unconditional shift shifts[0])."""
    shifts = np.asarray(shifts, dtype=np.int64)

    def fn(d):
        s = shifts[0] if c < 0 else shifts[d[c]]
        d[t] = (d[t] + s) % D
        return d
    return apply_digit_map(psi, D, n, fn)


def apply_csum(psi, D, n, c, t):
    """Generalized CNOT: |x_c, x_t> -> |x_c, x_t + x_c mod D> (the index rule of
    subsection "Generalized CNOT gate")."""
    def fn(d):
        d[t] = (d[t] + d[c]) % D
        return d
    return apply_digit_map(psi, D, n, fn)


def apply_shift(psi, D, n, q, s):
    """Generalized NOT X_s on qudit q: x_q -> x_q + s mod D."""
    def fn(d):
        d[q] = (d[q] + s) % D
        return d
    return apply_digit_map(psi, D, n, fn)


def apply_swap(psi, D, n, a, b):
    """SWAP of qudits a and b (subsection "Generalized SWAP Gate")."""
    def fn(d):
        d[a], d[b] = d[b], d[a]
        return d
    return apply_digit_map(psi, D, n, fn)


def apply_controlled_stack(psi, D, n, c, t, mats) -> np.ndarray:
    """sum_m |m><m|_c (x) mats[m]_t: on the slab where qudit c is at level m,
    every fibre along qudit t is multiplied by mats[m]."""
    v = np.array(psi, dtype=np.complex128).reshape((D,) * n)
    tt = t if t < c else t - 1  # the target's axis once axis c is indexed away
    for m in range(D):
        idx = [slice(None)] * n
        idx[c] = m
        sub = v[tuple(idx)]
        v[tuple(idx)] = np.moveaxis(np.tensordot(np.asarray(mats[m]), sub, axes=([1], [tt])), 0, tt)
    return v.reshape(-1)


def apply_mcx(psi, D, n, controls, t):
    """Multi-controlled shift: x_t -> x_t + prod_i x_{c_i} mod D.  The paper
    names the Toffoli and multi-controlled NOT gates without a formula; this
    is the generalization of its CNOT index rule (x_t -> x_t + x_c), equal to
    CSUM for one control and to the Toffoli / multi-controlled NOT for qubits."""
    controls = list(controls)

    def fn(d):
        prod = np.ones_like(d[t])
        for c in controls:
            prod = prod * d[c]
        d[t] = (d[t] + prod) % D
        return d
    return apply_digit_map(psi, D, n, fn)


def apply_phase(psi, D, n, phase_of_digits) -> np.ndarray:
    """Diagonal gate: psi_x <- phi(digits(x)) psi_x."""
    dig = digits_of(D, n, np.arange(D ** n))
    return psi * phase_of_digits(dig)


def apply_cz(psi, D, n, c, t):
    """Controlled phase |c, t> -> w^(c t) |c, t>."""
    w = gates.omega(D)
    return apply_phase(psi, D, n, lambda d: w ** ((d[c] * d[t]) % D))


def apply_op(psi: np.ndarray, D: int, n: int, op, theta) -> np.ndarray:
    """Apply one gate descriptor (see ``qf_inputs``)."""
    kind = op[0]
    if kind in ("h", "x", "clock", "rx", "ry", "rz"):
        return apply_1q(psi, D, n, op[1], gates.op_matrix(op, D, theta))
    if kind == "u":
        q0, k = op[1], op[2]
        return apply_matrix(psi, D, n, list(range(q0, q0 + k)), op[3])
    if kind == "csum":
        return apply_csum(psi, D, n, op[1], op[2])
    if kind == "cshift":
        return apply_cshift(psi, D, n, op[1], op[2], op[3])
    if kind == "cz":
        return apply_cz(psi, D, n, op[1], op[2])
    if kind == "swap":
        return apply_swap(psi, D, n, op[1], op[2])
    if kind == "mcx":
        return apply_mcx(psi, D, n, op[1], op[2])
    if kind == "mcx_inv":
        controls, t = op[1], op[2]

        def fn(d):
            prod = np.ones_like(d[t])
            for c in controls:
                prod = prod * d[c]
            d[t] = (d[t] - prod) % D
            return d
        return apply_digit_map(psi, D, n, fn)
    if kind in ("crx", "cry", "crz"):
        return apply_controlled_stack(psi, D, n, op[1], op[2], gates.crot_mats(op, D, theta))
    if kind == "cstack":
        return apply_controlled_stack(psi, D, n, op[1], op[2], op[3])
    raise ValueError(f"unknown gate kind {kind}")


def run(circuit, psi0=None, theta=None, batch_digits=None) -> np.ndarray:
    """Apply the circuit's gates one after another to psi0 (default |0...0>)."""
    D, n = circuit.dim, circuit.n
    theta = circuit.theta if theta is None else theta
    psi = basis_state(D, n, batch_digits) if psi0 is None else np.array(psi0, dtype=np.complex128)
    for op in circuit.ops:
        psi = apply_op(psi, D, n, op, theta)
    return psi


def inverse_op(op, D: int, theta):
    """The inverse of a descriptor, as a descriptor (used by the oracle adjoint and
    by un-apply tests).  Rotations invert by negating the angle, so the inverse is
    returned as a dense matrix gate."""
    kind = op[0]
    if kind in ("h", "x", "clock", "rx", "ry", "rz"):
        return ("u", op[1], 1, gates.op_matrix(op, D, theta).conj().T)
    if kind == "u":
        return ("u", op[1], op[2], np.asarray(op[3]).conj().T)
    if kind == "csum":
        return ("cshift", op[1], op[2], tuple((-v) % D for v in range(D)))
    if kind == "cshift":
        return ("cshift", op[1], op[2], tuple((-int(v)) % D for v in op[3]))
    if kind == "cz":
        return ("cz_inv", op[1], op[2])
    if kind == "swap":
        return op
    if kind == "mcx":
        return ("mcx_inv", op[1], op[2])
    if kind in ("crx", "cry", "crz"):
        return ("cstack", op[1], op[2], [m.conj().T for m in gates.crot_mats(op, D, theta)])
    raise ValueError(kind)


def apply_inverse(psi, D, n, op, theta):
    inv = inverse_op(op, D, theta)
    if inv[0] == "cz_inv":
        w = gates.omega(D)
        return apply_phase(psi, D, n, lambda d: w ** (-((d[inv[1]] * d[inv[2]]) % D)))
    return apply_op(psi, D, n, inv, theta)
