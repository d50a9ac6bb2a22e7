"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no gate arithmetic.  It only describes circuits as ordered
lists of gate descriptors (kind, qudits, levels, parameter slot) plus the
random numbers a workload draws: rotation angles, clock exponents, random
states and random unitaries.  Both the FP64 oracle and the HIP path interpret
these descriptors on their own.

Gate descriptors (tuples; levels are 0-indexed, qudit 0 is the most
significant digit of the basis index):

    ("h", q)                 Fourier gate on qudit q
    ("x", q, s)              shift x_q -> x_q + s mod D
    ("clock", q, a)          Z^a = diag(omega^(a k))
    ("rx", q, j, k, p)       two-level rotation with the symmetric generator
    ("ry", q, j, k, p)       two-level rotation with the antisymmetric generator
    ("rz", q, j, p)          rotation with the j-th diagonal generator, 1 <= j < D
    ("csum", c, t)           x_t -> x_t + x_c mod D
    ("cshift", c, t, shifts) x_t -> x_t + shifts[x_c] mod D (c = -1: shifts[0])
    ("cz", c, t)             phase omega^(x_c x_t)
    ("u", q0, k, mat)        dense D^k x D^k matrix on qudits q0..q0+k-1
    ("crx", c, t, j, k, p)   controlled rotation sum_m |m><m|_c (x) R_x^{jk}(m theta)_t
    ("cry", c, t, j, k, p)   the same with R_y^{jk}
    ("crz", c, t, j, p)      the same with R_z^{j}
    ("swap", a, b)           exchange the digits of qudits a and b
    ("mcx", (c1, ..), t)     x_t -> x_t + prod_i x_{c_i} mod D (Toffoli for two controls)

The angle of a rotation is ``theta[p]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

Op = Tuple


@dataclass
class Circuit:
    dim: int
    n: int
    ops: List[Op]
    theta: np.ndarray = field(default_factory=lambda: np.zeros(0))
    name: str = ""

    @property
    def nparams(self) -> int:
        return int(len(self.theta))

    @property
    def amps(self) -> int:
        return self.dim ** self.n


# ----------------------------------------------------------------------------
# Layer builders.  Inside one rotation layer the order is type-major
# (x, then y, then z), level-pair-major inside a type, qudits innermost;
# rotations on different qudits commute, so the qudit order does not change
# the result.  A level pair (l, l+1) of an R_z names the diagonal generator
# j = l + 1.
# ----------------------------------------------------------------------------

def _rot_layer(ops: list, n: int, types: Sequence[str], pairs: Sequence[Tuple[int, int]],
               pstart: int) -> int:
    p = pstart
    for t in types:
        for (j, k) in pairs:
            for q in range(n):
                if t == "z":
                    ops.append(("rz", q, k, p))
                else:
                    ops.append(("r" + t, q, j, k, p))
                p += 1
    return p


def csum_chain(n: int) -> List[Op]:
    return [("csum", i, i + 1) for i in range(n - 1)]


def csum_ring(n: int) -> List[Op]:
    return [("csum", i, (i + 1) % n) for i in range(n)]


def adjacent_pairs(D: int, count: int | None = None) -> List[Tuple[int, int]]:
    pairs = [(l, l + 1) for l in range(D - 1)]
    return pairs if count is None else pairs[:count]


def hea(D: int, n: int, layers: int, seed: int | np.random.Generator, pairs=None,
        types=("x", "y", "z"), clock=True, entangler="ring", cz_stride: int = 0,
        name: str = "") -> Circuit:
    """Hardware-efficient ansatz: per layer rotations, clock gates Z^a, CSUM ring
    (or chain), then optional CZ(i, i+cz_stride mod n).  Angles ~ U[-pi, pi] are
    drawn per layer in application order, then the layer's clock exponents."""
    rng = np.random.default_rng(seed) if not isinstance(seed, np.random.Generator) else seed
    pairs = adjacent_pairs(D, 2) if pairs is None else list(pairs)
    ops: List[Op] = []
    thetas = []
    p = 0
    for _ in range(layers):
        p0 = p
        p = _rot_layer(ops, n, types, pairs, p)
        thetas.append(rng.uniform(-np.pi, np.pi, size=p - p0))
        if clock:
            a = rng.integers(0, D, size=n)
            ops.extend(("clock", q, int(a[q])) for q in range(n))
        if entangler == "ring":
            ops.extend(csum_ring(n))
        elif entangler == "chain":
            ops.extend(csum_chain(n))
        if cz_stride:
            ops.extend(("cz", i, (i + cz_stride) % n) for i in range(n))
    theta = np.concatenate(thetas) if thetas else np.zeros(0)
    return Circuit(D, n, ops, theta, name)


# ----------------------------------------------------------------------------
# The five workloads.
# ----------------------------------------------------------------------------

def config1() -> Circuit:
    """Qutrits, n=4, complex128: H on all, CSUM chain, then 2 x [R_y on pairs
    (0,1),(1,2) of every qudit; CSUM chain].  16 angles, 29 gates.  Seed 0."""
    D, n = 3, 4
    rng = np.random.default_rng(0)
    ops: List[Op] = [("h", q) for q in range(n)] + csum_chain(n)
    thetas = []
    p = 0
    for _ in range(2):
        p0 = p
        p = _rot_layer(ops, n, ("y",), [(0, 1), (1, 2)], p)
        thetas.append(rng.uniform(-np.pi, np.pi, size=p - p0))
        ops.extend(csum_chain(n))
    return Circuit(D, n, ops, np.concatenate(thetas), "config1_d3_n4_c128")


def config2(n: int = 16, layers: int = 10) -> Circuit:
    """Qutrits, n=16, complex64: depth-10 HEA with R_x,R_y,R_z on pairs (0,1),(1,2),
    clock Z^a (a ~ U{0,1,2}), CSUM ring.  960 angles, 1280 gates.  Seed 1."""
    return hea(3, n, layers, 1, name=f"config2_d3_n{n}_l{layers}_c64")


def config3(n: int = 10, layers: int = 8) -> Circuit:
    """D=5, n=10: depth-8 HEA with R_x,R_y,R_z on the 4 adjacent pairs, CSUM ring,
    then CZ(i, i+2).  960 parameters, 1120 gates.  Seed 2."""
    return hea(5, n, layers, 2, pairs=adjacent_pairs(5), clock=False, cz_stride=2,
               name=f"config3_d5_n{n}_l{layers}_c64")


def config3_fd_params(c: Circuit, count: int = 16) -> np.ndarray:
    """Indices of the parameters checked by central finite differences
    (drawn after the angles from the same seed)."""
    rng = np.random.default_rng(2)
    rng.uniform(-np.pi, np.pi, size=c.nparams)
    return np.sort(rng.choice(c.nparams, size=count, replace=False))


def config4(count_d3: int = 768, count_d4: int = 256, layers: int = 6) -> List[Circuit]:
    """Ragged batch: 768 qutrit circuits (n ~ U{6..10}) and 256 ququart circuits
    (n ~ U{5..8}); each a depth-6 config-2 style HEA with its own angles.  Seed 3.
    The qudit counts are drawn first, then one child stream per circuit."""
    rng = np.random.default_rng(3)
    n3 = rng.integers(6, 11, size=count_d3)
    n4 = rng.integers(5, 9, size=count_d4)
    seeds = rng.integers(0, 2**63 - 1, size=count_d3 + count_d4)
    out = []
    for i, n in enumerate(n3):
        out.append(hea(3, int(n), layers, int(seeds[i]), name=f"c4_d3_{i}"))
    for i, n in enumerate(n4):
        out.append(hea(4, int(n), layers, int(seeds[count_d3 + i]), name=f"c4_d4_{i}"))
    return out


def config5(n: int = 8, layers: int = 12, D: int = 10) -> Circuit:
    """D=10, n=8: depth-12, per layer R_y on the 9 adjacent pairs of every qudit,
    then a CSUM ring.  864 parameters, 960 gates.  Seed 4.  Pair-major with qudits
    innermost, so qudit q sees R_y^{0,1} first and R_y^{8,9} last."""
    rng = np.random.default_rng(4)
    ops: List[Op] = []
    thetas = []
    p = 0
    for _ in range(layers):
        p0 = p
        for (j, k) in adjacent_pairs(D):
            for q in range(n):
                ops.append(("ry", q, j, k, p))
                p += 1
        thetas.append(rng.uniform(-np.pi, np.pi, size=p - p0))
        ops.extend(csum_ring(n))
    return Circuit(D, n, ops, np.concatenate(thetas), f"config5_d{D}_n{n}_l{layers}_c64")


# ----------------------------------------------------------------------------
# Observables (descriptors only): a sum of single-qudit diagonal terms,
# each term a (qudit, "z") pair meaning Z = diag(omega^k) on that qudit.
# ----------------------------------------------------------------------------

def z0_terms() -> List[Tuple[int, str]]:
    return [(0, "z")]


def zsum_terms(n: int) -> List[Tuple[int, str]]:
    return [(q, "z") for q in range(n)]


# ----------------------------------------------------------------------------
# Random states, unitaries and circuits for kernel-level tests.
# ----------------------------------------------------------------------------

def random_state(D: int, n: int, seed: int, batch: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    N = D ** n
    v = rng.standard_normal((batch, N)) + 1j * rng.standard_normal((batch, N))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.reshape(-1) if batch == 1 else v


def uniforms(count: int, seed: int) -> np.ndarray:
    """count seeded uniforms in [0, 1) (float64): the draws of measurement shots."""
    return np.random.default_rng(seed).random(count)


def sparse_state(D: int, n: int, seed: int, keep: float = 0.1) -> np.ndarray:
    """A normalised random state with most amplitudes exactly zero (about a
    fraction keep non-zero), so distributions have runs of empty bins."""
    rng = np.random.default_rng(seed)
    N = D ** n
    v = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * (rng.random(N) < keep)
    if not np.any(v):
        v[int(rng.integers(N))] = 1.0
    return v / np.linalg.norm(v)


def random_unitary(m: int, seed: int | np.random.Generator) -> np.ndarray:
    """Haar-random m x m unitary: QR of a complex Gaussian with the phases of
    R's diagonal moved into Q."""
    rng = np.random.default_rng(seed) if not isinstance(seed, np.random.Generator) else seed
    z = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def random_circuit(D: int, n: int, depth: int, seed: int, kinds=None) -> Circuit:
    """A random mix of every gate kind, for small-n parity and brute-force pins."""
    rng = np.random.default_rng(seed)
    kinds = kinds or ["h", "x", "clock", "rx", "ry", "rz", "csum", "cz", "cshift", "u1", "u2"]
    ops: List[Op] = []
    thetas: List[float] = []
    for _ in range(depth):
        kind = kinds[rng.integers(len(kinds))]
        q = int(rng.integers(n))
        if kind == "h":
            ops.append(("h", q))
        elif kind == "x":
            ops.append(("x", q, int(rng.integers(1, D))))
        elif kind == "clock":
            ops.append(("clock", q, int(rng.integers(1, D))))
        elif kind in ("rx", "ry"):
            j, k = sorted(rng.choice(D, size=2, replace=False).tolist())
            ops.append((kind, q, int(j), int(k), len(thetas)))
            thetas.append(float(rng.uniform(-np.pi, np.pi)))
        elif kind == "rz":
            ops.append(("rz", q, int(rng.integers(1, D)), len(thetas)))
            thetas.append(float(rng.uniform(-np.pi, np.pi)))
        elif kind in ("csum", "cz", "cshift") and n >= 2:
            c, t = rng.choice(n, size=2, replace=False).tolist()
            if kind == "cshift":
                ops.append(("cshift", int(c), int(t), tuple(int(v) for v in rng.integers(0, D, size=D))))
            else:
                ops.append((kind, int(c), int(t)))
        elif kind == "u1":
            ops.append(("u", q, 1, random_unitary(D, rng)))
        elif kind == "u2" and n >= 2:
            q0 = int(rng.integers(n - 1))
            ops.append(("u", q0, 2, random_unitary(D * D, rng)))
        elif kind == "swap" and n >= 2:
            a_, b_ = rng.choice(n, size=2, replace=False).tolist()
            ops.append(("swap", int(a_), int(b_)))
        elif kind == "mcx" and n >= 3:
            nc = int(rng.integers(1, min(4, n)))
            qs = rng.choice(n, size=nc + 1, replace=False).tolist()
            ops.append(("mcx", tuple(int(v) for v in qs[:nc]), int(qs[nc])))
        elif kind in ("crx", "cry", "crz") and n >= 2:
            c, t = rng.choice(n, size=2, replace=False).tolist()
            if kind == "crz":
                ops.append(("crz", int(c), int(t), int(rng.integers(1, D)), len(thetas)))
            else:
                j, k = sorted(rng.choice(D, size=2, replace=False).tolist())
                ops.append((kind, int(c), int(t), int(j), int(k), len(thetas)))
            thetas.append(float(rng.uniform(-np.pi, np.pi)))
    return Circuit(D, n, ops, np.asarray(thetas, dtype=np.float64), f"random_d{D}_n{n}_s{seed}")


def cr_ansatz(D: int, n: int, layers: int, seed: int) -> Circuit:
    """Ansatz with the paper's differentiable controlled rotations: per layer
    R_y on level pairs (0,1), (1,2) of every qudit, then controlled rotations
    i -> i+1 mod n cycling through the x, y and z types (x, y on levels (0,1),
    z with j = 1), each with its own angle.  Angles ~ U[-pi, pi] from the seed."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    p = 0
    for _ in range(layers):
        p = _rot_layer(ops, n, ("y",), adjacent_pairs(D, 2), p)
        for i in range(n):
            kind = ("crx", "cry", "crz")[i % 3]
            if kind == "crz":
                ops.append(("crz", i, (i + 1) % n, 1, p))
            else:
                ops.append((kind, i, (i + 1) % n, 0, 1, p))
            p += 1
    return Circuit(D, n, ops, rng.uniform(-np.pi, np.pi, size=p), f"cr_ansatz_d{D}_n{n}_l{layers}")


@dataclass
class MixedCircuit:
    """A circuit on qudits of different dimensions dims[q] (qudit 0 most
    significant).  Descriptors as above, every level and shift taken in the
    dimension of the qudit it acts on."""
    dims: List[int]
    ops: List[Op]
    theta: np.ndarray = field(default_factory=lambda: np.zeros(0))
    name: str = ""

    @property
    def n(self) -> int:
        return len(self.dims)

    @property
    def nparams(self) -> int:
        return int(len(self.theta))

    @property
    def amps(self) -> int:
        return int(np.prod(self.dims))


def paper_mixed_example() -> dict:
    """The example circuit of section "Code style": dims [2, 3, 4]; Fourier on
    every qudit, R_x(pi/2) on qudit 0 (levels 0, 1), CNOT (CSUM) from qudit 0 to
    qudit 2; initial state |0, 1, 3>; measure qudits [0, 1] with 1000 shots."""
    ops = [("h", 0), ("h", 1), ("h", 2), ("rx", 0, 0, 1, 0), ("csum", 0, 2)]
    return {"circuit": MixedCircuit([2, 3, 4], ops, np.array([np.pi / 2]), "paper_mixed_example"),
            "digits": (0, 1, 3), "measured": [0, 1], "shots": 1000}


def random_mixed_circuit(dims: Sequence[int], depth: int, seed: int, kinds=None) -> MixedCircuit:
    """A random mix of gate kinds on a register of per-qudit dimensions."""
    rng = np.random.default_rng(seed)
    dims = [int(d) for d in dims]
    n = len(dims)
    kinds = kinds or ["h", "x", "clock", "rx", "ry", "rz", "csum", "cz", "cshift", "u1", "u2", "crx", "cry", "crz",
                      "swap", "mcx"]
    ops: List[Op] = []
    thetas: List[float] = []
    for _ in range(depth):
        kind = kinds[rng.integers(len(kinds))]
        q = int(rng.integers(n))
        d = dims[q]
        if kind == "h":
            ops.append(("h", q))
        elif kind == "x":
            ops.append(("x", q, int(rng.integers(1, d))))
        elif kind == "clock":
            ops.append(("clock", q, int(rng.integers(1, d))))
        elif kind in ("rx", "ry"):
            j, k = sorted(rng.choice(d, size=2, replace=False).tolist())
            ops.append((kind, q, int(j), int(k), len(thetas)))
            thetas.append(float(rng.uniform(-np.pi, np.pi)))
        elif kind == "rz":
            ops.append(("rz", q, int(rng.integers(1, d)), len(thetas)))
            thetas.append(float(rng.uniform(-np.pi, np.pi)))
        elif kind in ("csum", "cz", "cshift") and n >= 2:
            c, t = rng.choice(n, size=2, replace=False).tolist()
            if kind == "cshift":
                ops.append(("cshift", int(c), int(t), tuple(int(v) for v in rng.integers(0, dims[t], size=dims[c]))))
            else:
                ops.append((kind, int(c), int(t)))
        elif kind == "u1":
            ops.append(("u", q, 1, random_unitary(d, rng)))
        elif kind == "u2" and n >= 2:
            q0 = int(rng.integers(n - 1))
            ops.append(("u", q0, 2, random_unitary(dims[q0] * dims[q0 + 1], rng)))
        elif kind in ("crx", "cry", "crz") and n >= 2:
            c, t = rng.choice(n, size=2, replace=False).tolist()
            if kind == "crz":
                ops.append(("crz", int(c), int(t), int(rng.integers(1, dims[t])), len(thetas)))
            else:
                j, k = sorted(rng.choice(dims[t], size=2, replace=False).tolist())
                ops.append((kind, int(c), int(t), int(j), int(k), len(thetas)))
            thetas.append(float(rng.uniform(-np.pi, np.pi)))
        elif kind == "swap":
            pairs = [(a_, b_) for a_ in range(n) for b_ in range(n) if a_ != b_ and dims[a_] == dims[b_]]
            if pairs:
                a_, b_ = pairs[int(rng.integers(len(pairs)))]
                ops.append(("swap", a_, b_))
        elif kind == "mcx" and n >= 3:
            nc = int(rng.integers(1, min(4, n)))
            qs = rng.choice(n, size=nc + 1, replace=False).tolist()
            ops.append(("mcx", tuple(int(v) for v in qs[:nc]), int(qs[nc])))
    return MixedCircuit(dims, ops, np.asarray(thetas, dtype=np.float64), f"random_mixed_{dims}_s{seed}")


def mixed_hea(dims: Sequence[int], layers: int, seed: int) -> MixedCircuit:
    """Ansatz on a mixed register: per layer R_x, R_y on levels (0, 1) and R_z
    (j = 1) of every qudit, then a CSUM ring; angles ~ U[-pi, pi]."""
    rng = np.random.default_rng(seed)
    dims = [int(d) for d in dims]
    n = len(dims)
    ops: List[Op] = []
    p = 0
    for _ in range(layers):
        for t in ("x", "y", "z"):
            for q in range(n):
                ops.append(("rz", q, 1, p) if t == "z" else ("r" + t, q, 0, 1, p))
                p += 1
        ops.extend(csum_ring(n))
    return MixedCircuit(dims, ops, rng.uniform(-np.pi, np.pi, size=p), f"mixed_hea_{dims}_l{layers}")


def grover_d3_n2_marker22() -> dict:
    """Inputs of the qutrit Grover example: two qutrits, marked basis state |2,2>."""
    return {"dim": 3, "n": 2, "marker": (2, 2)}


def deutsch_jozsa_d(D: int, mode: str) -> Circuit:
    """Qudit Deutsch-Jozsa on 4 qudits, initial state |0,0,0,D-1>: Fourier on all,
    oracle (constant: shift on the last qudit; balanced: CSUM 2->3), Fourier on the
    first three qudits.  The initial digits are returned in ``name``."""
    n = 4
    ops: List[Op] = [("h", q) for q in range(n)]
    ops.append(("x", n - 1, 1) if mode == "constant" else ("csum", 2, 3))
    ops.extend(("h", q) for q in range(n - 1))
    return Circuit(D, n, ops, np.zeros(0), f"dj_{mode}")
