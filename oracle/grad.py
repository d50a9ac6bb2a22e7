"""Gradients of L(theta) = Re<psi(theta)| O |psi(theta)> in FP64.

Two independent routes:

* ``adjoint`` - the adjoint method (Jones & Gacon 2020, arXiv:2009.02823), gate by
  gate with no fusion: lambda = H_O psi with H_O = (O + O^dagger)/2; walking the
  gates in reverse, for a rotation U = exp(-i theta S / 2) the derivative is
  dL/dtheta = 2 Re <lambda| dU/dtheta U^-1 |psi> = Im <lambda| S |psi>, evaluated
  with psi and lambda both taken just after the gate; then both are un-applied.
* ``finite_diff`` - central differences (L(theta + h e_i) - L(theta - h e_i)) / 2h.
"""
from __future__ import annotations

import numpy as np

from . import gates, measure, sim


def loss(circuit, terms, theta=None) -> float:
    psi = sim.run(circuit, theta=theta)
    return float(measure.expect_diag(psi, circuit.dim, circuit.n, terms).real)


def adjoint(circuit, terms, theta=None, psi_final=None) -> np.ndarray:
    D, n = circuit.dim, circuit.n
    theta = circuit.theta if theta is None else np.asarray(theta, dtype=np.float64)
    psi = sim.run(circuit, theta=theta) if psi_final is None else psi_final.copy()
    lam = measure.hermitian_part_diag(D, n, terms) * psi
    g = np.zeros(len(theta))
    for op in reversed(circuit.ops):
        if op[0] in ("rx", "ry", "rz"):
            S = gates.generator(op, D)
            Spsi = sim.apply_1q(psi, D, n, op[1], S)
            g[op[-1]] += float(np.vdot(lam, Spsi).imag)
        psi = sim.apply_inverse(psi, D, n, op, theta)
        lam = sim.apply_inverse(lam, D, n, op, theta)
    return g


def finite_diff(circuit, terms, idx, h: float = 1e-6, theta=None) -> np.ndarray:
    theta = circuit.theta if theta is None else np.asarray(theta, dtype=np.float64)
    out = np.zeros(len(idx))
    for m, i in enumerate(idx):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        out[m] = (loss(circuit, terms, tp) - loss(circuit, terms, tm)) / (2 * h)
    return out
