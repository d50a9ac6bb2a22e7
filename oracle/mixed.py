"""Registers whose qudits have different dimensions, dims = [d_0, ..., d_{n-1}]
(the multidimensional circuits of section "Related work", Table 1, and of the
example circuit of section "Code style", Circuit(dim=[2, 3, 4], ...)), in FP64.

Basis index: the mixed-radix form of the decimal representation, qudit 0 most
significant, x = sum_q x_q S_q with S_q = d_{q+1} ... d_{n-1}.

Gates on one qudit q use that qudit's dimension d_q (Fourier of size d_q,
shift mod d_q, clock with omega_{d_q}, Gell-Mann rotations of size d_q).  The
paper gives the two-qudit gates for one D only; across dimensions this oracle
reads them as:
  * CSUM (generalized CNOT) c -> t:  x_t -> (x_t + x_c) mod d_t,
  * controlled shift:                x_t -> (x_t + shifts[x_c]) mod d_t,
  * CZ:                              phase omega_{d_t}^(x_c x_t),
  * controlled rotation:             sum_{m < d_c} |m><m|_c (x) R(m theta) on d_t,
  * multi-controlled shift:          x_t -> (x_t + prod_i x_{c_i}) mod d_t,
  * SWAP only between qudits of equal dimension.
Every function here is test infrastructure: plain and slow.
"""
from __future__ import annotations

import numpy as np

from . import gates

ROTATIONS = ("rx", "ry", "rz", "crx", "cry", "crz")


def strides(dims) -> list:
    """S_q = product of the dimensions after q."""
    out = []
    for q in range(len(dims)):
        s = 1
        for d in dims[q + 1:]:
            s *= int(d)
        out.append(s)
    return out


def size(dims) -> int:
    s = 1
    for d in dims:
        s *= int(d)
    return s


def index_of(dims, digits) -> int:
    return int(sum(int(x) * s for x, s in zip(digits, strides(dims))))


def digits_of(dims, x):
    """Digit arrays (x_0, ..., x_{n-1}) of the index array x."""
    x = np.asarray(x, dtype=np.int64)
    return [(x // s) % int(d) for s, d in zip(strides(dims), dims)]


def basis_state(dims, digits=None) -> np.ndarray:
    psi = np.zeros(size(dims), dtype=np.complex128)
    psi[0 if digits is None else index_of(dims, digits)] = 1.0
    return psi


def apply_1q(psi, dims, q, U) -> np.ndarray:
    """U (d_q x d_q) on qudit q: contract U's column index with axis q."""
    t = np.asarray(psi, dtype=np.complex128).reshape([int(d) for d in dims])
    out = np.tensordot(np.asarray(U, dtype=np.complex128), t, axes=([1], [q]))
    return np.ascontiguousarray(np.moveaxis(out, 0, q)).reshape(-1)


def apply_block(psi, dims, q0, k, B) -> np.ndarray:
    """Dense block B on the adjacent qudits q0..q0+k-1, of size
    d_q0 ... d_{q0+k-1} (first qudit most significant)."""
    dims = [int(d) for d in dims]
    sub = dims[q0:q0 + k]
    t = np.asarray(psi, dtype=np.complex128).reshape(dims)
    Bt = np.asarray(B, dtype=np.complex128).reshape(sub + sub)
    out = np.tensordot(Bt, t, axes=(list(range(k, 2 * k)), list(range(q0, q0 + k))))
    out = np.moveaxis(out, list(range(k)), list(range(q0, q0 + k)))
    return np.ascontiguousarray(out).reshape(-1)


def apply_digit_map(psi, dims, fn) -> np.ndarray:
    """Permutation gate: the amplitude of |x> moves to |fn(x)> (digit lists)."""
    N = size(dims)
    dig = digits_of(dims, np.arange(N))
    new = fn([d.copy() for d in dig])
    dest = np.zeros(N, dtype=np.int64)
    for d, s in zip(new, strides(dims)):
        dest += d * s
    out = np.zeros_like(np.asarray(psi, dtype=np.complex128))
    out[dest] = psi
    return out


def apply_phase(psi, dims, phase_of_digits) -> np.ndarray:
    return np.asarray(psi, dtype=np.complex128) * phase_of_digits(digits_of(dims, np.arange(size(dims))))


def apply_controlled_stack(psi, dims, c, t, mats) -> np.ndarray:
    """sum_m |m><m|_c (x) mats[m]_t for m < d_c."""
    dims = [int(d) for d in dims]
    v = np.array(psi, dtype=np.complex128).reshape(dims)
    tt = t if t < c else t - 1
    for m in range(dims[c]):
        idx = [slice(None)] * len(dims)
        idx[c] = m
        sub = v[tuple(idx)]
        v[tuple(idx)] = np.moveaxis(np.tensordot(np.asarray(mats[m]), sub, axes=([1], [tt])), 0, tt)
    return v.reshape(-1)


def one_qudit_matrix(op, d: int, theta) -> np.ndarray:
    return gates.op_matrix(op, d, theta)


def crot_mats(op, dims, theta) -> list:
    """R(m theta) in the target's dimension for every control level m < d_c."""
    c, t = op[1], op[2]
    S = gates.crot_generator(op, int(dims[t]))
    th = float(theta[op[-1]])
    return [gates.expm_hermitian(S, m * th) for m in range(int(dims[c]))]


def _mcx_map(dims, controls, t, sign):
    def fn(d):
        prod = np.ones_like(d[t])
        for c in controls:
            prod = prod * d[c]
        d[t] = (d[t] + sign * prod) % int(dims[t])
        return d
    return fn


def apply_op(psi, dims, op, theta) -> np.ndarray:
    kind = op[0]
    if kind in ("h", "x", "clock", "rx", "ry", "rz"):
        return apply_1q(psi, dims, op[1], one_qudit_matrix(op, int(dims[op[1]]), theta))
    if kind == "u":
        return apply_block(psi, dims, op[1], op[2], op[3])
    if kind == "csum":
        c, t = op[1], op[2]

        def fn(d):
            d[t] = (d[t] + d[c]) % int(dims[t])
            return d
        return apply_digit_map(psi, dims, fn)
    if kind == "cshift":
        c, t, sh = op[1], op[2], np.asarray(op[3], dtype=np.int64)

        def fn(d):
            d[t] = (d[t] + (sh[0] if c < 0 else sh[d[c]])) % int(dims[t])
            return d
        return apply_digit_map(psi, dims, fn)
    if kind in ("cz", "cz_inv"):
        c, t = op[1], op[2]
        w = gates.omega(int(dims[t]))
        sgn = 1 if kind == "cz" else -1
        return apply_phase(psi, dims, lambda d: w ** (sgn * ((d[c] * d[t]) % int(dims[t]))))
    if kind == "swap":
        a, b = op[1], op[2]
        if int(dims[a]) != int(dims[b]):
            raise ValueError("SWAP needs qudits of equal dimension")

        def fn(d):
            d[a], d[b] = d[b], d[a]
            return d
        return apply_digit_map(psi, dims, fn)
    if kind == "mcx":
        return apply_digit_map(psi, dims, _mcx_map(dims, op[1], op[2], 1))
    if kind == "mcx_inv":
        return apply_digit_map(psi, dims, _mcx_map(dims, op[1], op[2], -1))
    if kind in ("crx", "cry", "crz"):
        return apply_controlled_stack(psi, dims, op[1], op[2], crot_mats(op, dims, theta))
    if kind == "cstack":
        return apply_controlled_stack(psi, dims, op[1], op[2], op[3])
    raise ValueError(f"unknown gate kind {kind}")


def inverse_op(op, dims, theta):
    kind = op[0]
    if kind in ("h", "x", "clock", "rx", "ry", "rz"):
        return ("u", op[1], 1, one_qudit_matrix(op, int(dims[op[1]]), theta).conj().T)
    if kind == "u":
        return ("u", op[1], op[2], np.asarray(op[3]).conj().T)
    if kind == "csum":
        dt = int(dims[op[2]])
        return ("cshift", op[1], op[2], tuple((-v) % dt for v in range(int(dims[op[1]]))))
    if kind == "cshift":
        dt = int(dims[op[2]])
        return ("cshift", op[1], op[2], tuple((-int(v)) % dt for v in op[3]))
    if kind == "cz":
        return ("cz_inv", op[1], op[2])
    if kind == "swap":
        return op
    if kind == "mcx":
        return ("mcx_inv", op[1], op[2])
    if kind in ("crx", "cry", "crz"):
        return ("cstack", op[1], op[2], [m.conj().T for m in crot_mats(op, dims, theta)])
    raise ValueError(kind)


def run(circuit, psi0=None, theta=None, digits=None) -> np.ndarray:
    """Apply the circuit's gates in order to psi0 (default |digits>, or |0...0>)."""
    theta = circuit.theta if theta is None else np.asarray(theta, dtype=np.float64)
    psi = basis_state(circuit.dims, digits) if psi0 is None else np.array(psi0, dtype=np.complex128)
    for op in circuit.ops:
        psi = apply_op(psi, circuit.dims, op, theta)
    return psi


# ---- measurement ----

def probs(psi) -> np.ndarray:
    return np.abs(np.asarray(psi)) ** 2


def marginal(psi, dims, qudits) -> np.ndarray:
    """p(y) for the listed qudits, y in mixed radix over their dimensions in the
    listed order (first listed most significant)."""
    dims = [int(d) for d in dims]
    qudits = list(qudits)
    p = probs(psi).reshape(dims)
    others = tuple(a for a in range(len(dims)) if a not in qudits)
    s = p.sum(axis=others) if others else p
    order = sorted(qudits)
    s = np.transpose(s, [order.index(q) for q in qudits])
    return np.ascontiguousarray(s).reshape(-1)


def term_table(dims, term) -> np.ndarray:
    """Diagonal of a one-qudit observable term (q, "z") or (q, table of d_q values)."""
    q, d = term
    if isinstance(d, str):
        if d != "z":
            raise ValueError(d)
        return gates.omega(int(dims[q])) ** np.arange(int(dims[q]))
    return np.asarray(d, dtype=np.complex128)


def observable_diag(dims, terms) -> np.ndarray:
    """f(x) = sum over terms of table_t[x_{q_t}] for every basis index x."""
    dig = digits_of(dims, np.arange(size(dims)))
    f = np.zeros(size(dims), dtype=np.complex128)
    for term in terms:
        f += term_table(dims, term)[dig[term[0]]]
    return f


def expect_diag(psi, dims, terms) -> complex:
    return complex(np.sum(probs(psi) * observable_diag(dims, terms)))


# ---- gradients (adjoint method, gate by gate; see oracle.grad for the derivation) ----

def _derivative_term(op, dims, psi, lam) -> float:
    """Im <lam| S |psi>; a controlled rotation's generator at control level m is m S."""
    if op[0] in ("rx", "ry", "rz"):
        Spsi = apply_1q(psi, dims, op[1], gates.generator(op, int(dims[op[1]])))
    else:
        S = gates.crot_generator(op, int(dims[op[2]]))
        Spsi = apply_controlled_stack(psi, dims, op[1], op[2], [m * S for m in range(int(dims[op[1]]))])
    return float(np.vdot(lam, Spsi).imag)


def loss(circuit, terms, theta=None) -> float:
    return float(expect_diag(run(circuit, theta=theta), circuit.dims, terms).real)


def adjoint(circuit, terms, theta=None) -> np.ndarray:
    """dL/dtheta for L = Re <psi| O |psi>: lam = H_O psi, then the reverse walk."""
    lam_of = lambda psi: observable_diag(circuit.dims, terms).real * psi  # noqa: E731
    return adjoint_seeded(circuit, None, theta=theta, lam_fn=lam_of)


def adjoint_seeded(circuit, lam_final, theta=None, lam_fn=None) -> np.ndarray:
    """Reverse walk from lam_final = dL/d(conj psi) at the final state (or from
    lam_fn(psi_final))."""
    theta = circuit.theta if theta is None else np.asarray(theta, dtype=np.float64)
    psi = run(circuit, theta=theta)
    lam = lam_fn(psi) if lam_fn is not None else np.array(lam_final, dtype=np.complex128)
    g = np.zeros(len(theta))
    for op in reversed(circuit.ops):
        if op[0] in ROTATIONS:
            g[op[-1]] += _derivative_term(op, circuit.dims, psi, lam)
        inv = inverse_op(op, circuit.dims, theta)
        psi = apply_op(psi, circuit.dims, inv, theta)
        lam = apply_op(lam, circuit.dims, inv, theta)
    return g


def finite_diff(circuit, terms, idx, h: float = 1e-6) -> np.ndarray:
    out = np.zeros(len(idx))
    for m, i in enumerate(idx):
        tp = circuit.theta.copy()
        tm = circuit.theta.copy()
        tp[i] += h
        tm[i] -= h
        out[m] = (loss(circuit, terms, tp) - loss(circuit, terms, tm)) / (2 * h)
    return out
