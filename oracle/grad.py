"""Gradients of L(theta) = Re<psi(theta)| O |psi(theta)> in FP64, and of any
real loss of the final state.

Two independent routes:

* ``adjoint`` - the adjoint method (Jones & Gacon 2020, arXiv:2009.02823), gate by
  gate with no fusion: lambda = H_O psi with H_O = (O + O^dagger)/2; walking the
  gates in reverse, for a rotation U = exp(-i theta S / 2) the derivative is
  dL/dtheta = 2 Re <lambda| dU/dtheta U^-1 |psi> = Im <lambda| S |psi>, evaluated
  with psi and lambda both taken just after the gate; then both are un-applied.
* ``finite_diff`` - central differences (L(theta + h e_i) - L(theta - h e_i)) / 2h.

For a real loss L(psi) of the final state (the paper's training losses, e.g.
abs(target - output).sum(), section "Code style"), ``adjoint_seeded`` runs the
same reverse walk from lam = dL/d(conj psi) instead of H_O psi (for a real L,
dL/dtheta = 2 Re <dL/d(conj psi) | d psi/d theta>, which the walk evaluates gate
by gate as Im <lam|S|psi>); ``finite_diff_state`` is the central-difference
route for such losses.
"""
from __future__ import annotations

import numpy as np

from . import gates, measure, sim


def _rotation_derivative_term(op, D, n, psi, lam) -> float:
    """Im <lam| S |psi> for a rotation exp(-i theta S / 2); for the controlled
    rotation sum_m |m><m| (x) exp(-i m theta S / 2) the generator of the slab at
    control level m is m S."""
    if op[0] in ("rx", "ry", "rz"):
        Spsi = sim.apply_1q(psi, D, n, op[1], gates.generator(op, D))
    else:
        S = gates.crot_generator(op, D)
        Spsi = sim.apply_controlled_stack(psi, D, n, op[1], op[2], [m * S for m in range(D)])
    return float(np.vdot(lam, Spsi).imag)


ROTATIONS = ("rx", "ry", "rz", "crx", "cry", "crz")


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
        if op[0] in ROTATIONS:
            g[op[-1]] += _rotation_derivative_term(op, D, n, psi, lam)
        psi = sim.apply_inverse(psi, D, n, op, theta)
        lam = sim.apply_inverse(lam, D, n, op, theta)
    return g


def adjoint_seeded(circuit, lam_final, theta=None, psi_final=None) -> np.ndarray:
    """Adjoint gradient of a real loss of the final state, given
    lam_final = dL/d(conj psi) at the final state."""
    D, n = circuit.dim, circuit.n
    theta = circuit.theta if theta is None else np.asarray(theta, dtype=np.float64)
    psi = sim.run(circuit, theta=theta) if psi_final is None else psi_final.copy()
    lam = np.array(lam_final, dtype=np.complex128)
    g = np.zeros(len(theta))
    for op in reversed(circuit.ops):
        if op[0] in ROTATIONS:
            g[op[-1]] += _rotation_derivative_term(op, D, n, psi, lam)
        psi = sim.apply_inverse(psi, D, n, op, theta)
        lam = sim.apply_inverse(lam, D, n, op, theta)
    return g


def finite_diff_state(circuit, loss_of_state, idx, h: float = 1e-6, theta=None) -> np.ndarray:
    """Central differences of loss_of_state(psi(theta)) for the parameters idx."""
    theta = circuit.theta if theta is None else np.asarray(theta, dtype=np.float64)
    out = np.zeros(len(idx))
    for m, i in enumerate(idx):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        out[m] = (loss_of_state(sim.run(circuit, theta=tp)) - loss_of_state(sim.run(circuit, theta=tm))) / (2 * h)
    return out


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
