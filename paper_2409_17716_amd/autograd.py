"""Differentiable circuits: torch.autograd.Function front ends over the
library's adjoint kernels.

A ``DeviceCircuit`` compiles a circuit once into a bound plan (gate matrices
built on the device from a device tensor of angles) and owns the final-state
and adjoint buffers.  Two calls are differentiable in the angles:

* ``expectation(theta, terms)`` - Re<psi(theta)| O |psi(theta)> per register for
  a diagonal observable O (a sum of one-qudit terms, e.g. sum_i Z_i);
* ``state(theta)`` - the final state itself, so any real loss torch builds on
  it (the paper's training losses, e.g. abs(target - state).sum(), section
  "Code style") backpropagates: torch's gradient of the state seeds the
  reverse walk (QF_SEED).

Both backward passes run ``qf_adjoint_grad_dev``: the reverse walk un-applies
the gates on the final state and on lam = dL/d(conj psi), taking every
rotation's derivative Im<lam|S|psi> on the way (adjoint method, Jones & Gacon,
arXiv:2009.02823), so no per-gate state is stored; a plan with checkpoints
keeps one state every ``ckpt_every`` gates.  Nothing synchronises the host.

Registers of per-qudit dimensions (a circuit with ``dims``) have no bound
plans; their DeviceCircuit runs the host-angle calls instead (``qf_plan_forward``
and ``qf_adjoint_grad``, the same kernels with the angles copied to the host,
which synchronises), with one angle vector shared by every register.

The final state lives in the DeviceCircuit, so a backward pass finds it only if
no later forward pass of the same DeviceCircuit overwrote it (and the reverse
walk consumes it).  Otherwise the backward pass first runs the forward pass
again from the angles saved for it.  The one torch operation of a backward
pass is the chain rule's product of the parameter gradient with the upstream
gradient of the expectation.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import Plan, QfError, QF_EINVAL, new_state, qf_expect, qf_state_init


def _torch():
    import torch
    return torch


class DeviceCircuit:
    """A circuit bound to device buffers for ``batch`` registers of n qudits.

    ``circuit``: any object with ``dim`` (or per-qudit ``dims``), ``n``, ``ops``
    (gate descriptors) and ``nparams``; or pass ``dim`` (an int or a list of
    per-qudit dimensions), ``n``, ``ops``, ``nparams`` directly.
    ``digits``: initial basis state (n digits, or batch x n), default |0...0>.
    Extra keyword arguments are plan options (``ckpt_every``, ``tile_digits`` ...).
    """

    def __init__(self, circuit=None, *, dim=None, n: Optional[int] = None,
                 ops: Optional[Sequence[tuple]] = None, nparams: Optional[int] = None, dtype: str = "c64",
                 batch: int = 1, digits=None, **plan_opts):
        torch = _torch()
        if circuit is not None:
            dim = list(circuit.dims) if hasattr(circuit, "dims") else circuit.dim
            n, ops, nparams = circuit.n, circuit.ops, circuit.nparams
        if dim is None or n is None or ops is None or nparams is None:
            raise QfError(QF_EINVAL, "DeviceCircuit needs a circuit or dim, n, ops and nparams")
        if not isinstance(dim, (int, np.integer)):
            dim = [int(d) for d in dim]
            if len(set(dim)) == 1:
                dim = dim[0]
        self.dim = dim if isinstance(dim, list) else int(dim)
        self.n, self.nparams, self.batch, self.dtype = int(n), int(nparams), int(batch), dtype
        self.digits = None if digits is None else np.asarray(digits, dtype=np.int32)
        self.plan = Plan(self.dim, self.n, ops, self.nparams, dtype, **plan_opts)
        # mixed dimensions: host-angle calls (no bound plans for them)
        self.host = isinstance(self.dim, list)
        if not self.host:
            self.plan.bind(self.batch)
        self.psi = new_state(self.n, self.dim, dtype, self.batch)
        self.lam = new_state(self.n, self.dim, dtype, self.batch)
        self.grad = torch.zeros((self.batch, max(1, self.nparams)), dtype=torch.float64, device="cuda")
        self._gen = 0      # forward passes run into self.psi so far
        self._held = 0     # the forward pass whose final state self.psi holds (0: none)

    # ---- plumbing shared by the Functions ----
    def _angles(self, theta):
        """theta as a contiguous FP64 device tensor and its per-register stride."""
        torch = _torch()
        if not theta.is_cuda:
            raise QfError(QF_EINVAL, "theta must be a device tensor")
        th = theta.detach()
        if th.dtype != torch.float64 or not th.is_contiguous():
            th = th.to(torch.float64).contiguous()
        if th.dim() == 1:
            if th.numel() != self.nparams:
                raise QfError(QF_EINVAL, f"theta has {th.numel()} angles, the circuit {self.nparams}")
            return th, 0
        if th.dim() == 2 and th.shape == (self.batch, self.nparams):
            if self.host:
                raise QfError(QF_EINVAL, "per-register angles need qudits of one dimension")
            return th, self.nparams
        raise QfError(QF_EINVAL, f"theta must have shape ({self.nparams},) or ({self.batch}, {self.nparams})")

    def _forward(self, th, stride: int) -> int:
        qf_state_init(self.psi, self.n, self.dim, self.digits)
        if self.host:
            self.plan.forward(self.psi, th.cpu().numpy())
        else:
            self.plan.forward_dev(self.psi, th, stride)
        self._gen += 1
        self._held = self._gen
        return self._gen

    def _adjoint(self, th, stride: int, terms, seed: bool = False) -> None:
        """Gradient of every register into self.grad (the reverse walk consumes self.psi)."""
        torch = _torch()
        if self.host:
            g = self.plan.adjoint_grad(self.psi, self.lam, th.cpu().numpy(), terms, seed=seed)
            g = torch.from_numpy(np.ascontiguousarray(np.asarray(g).reshape(self.batch, -1)))
            self.grad[:, :self.nparams].copy_(g)
        else:
            self.plan.adjoint_grad_dev(self.psi, self.lam, th, stride, terms, self.grad, seed=seed)

    def _final_state_for(self, th, stride: int, gen: int) -> None:
        """Make self.psi hold the final state of forward pass ``gen`` (re-running
        the forward pass if a later one overwrote it); the reverse walk that
        follows consumes it."""
        if self._held != gen:
            self._forward(th, stride)
        self._held = 0

    def _param_grad(self, theta, per_register_scale=None):
        torch = _torch()
        G = self.grad[:, :self.nparams]
        if per_register_scale is not None:
            G = G * per_register_scale.to(torch.float64).reshape(-1, 1)
        if theta.dim() == 1:
            G = G.sum(0)
        return G.to(theta.dtype)

    # ---- differentiable calls ----
    def expectation(self, theta, terms):
        """Re<O> per register (float64 tensor of shape (batch,)), differentiable in theta.
        terms: list of (qudit, "z") or (qudit, table of dim complex values)."""
        return _Expectation.apply(theta, self, list(terms))

    def state(self, theta):
        """The final state (a copy owned by the caller; shape (N,) for one
        register of N amplitudes, (batch, N) otherwise), differentiable in theta."""
        return _State.apply(theta, self)


def _function_base():
    return _torch().autograd.Function


class _Expectation(_function_base()):
    @staticmethod
    def forward(ctx, theta, dc: DeviceCircuit, terms):
        torch = _torch()
        th, stride = dc._angles(theta)
        gen = dc._forward(th, stride)
        out = qf_expect(dc.psi, dc.n, dc.dim, terms)
        ctx.dc, ctx.terms, ctx.gen = dc, terms, gen
        ctx.save_for_backward(theta)
        return out.view(dc.batch, 2)[:, 0].clone().to(torch.float64)

    @staticmethod
    def backward(ctx, gout):
        (theta,) = ctx.saved_tensors
        dc = ctx.dc
        th, stride = dc._angles(theta)
        dc._final_state_for(th, stride, ctx.gen)
        dc._adjoint(th, stride, ctx.terms)
        return dc._param_grad(theta, gout), None, None


class _State(_function_base()):
    @staticmethod
    def forward(ctx, theta, dc: DeviceCircuit):
        th, stride = dc._angles(theta)
        gen = dc._forward(th, stride)
        ctx.dc, ctx.gen = dc, gen
        ctx.save_for_backward(theta)
        out = dc.psi.clone()
        return out if dc.batch == 1 else out.view(dc.batch, -1)

    @staticmethod
    def backward(ctx, g):
        (theta,) = ctx.saved_tensors
        dc = ctx.dc
        th, stride = dc._angles(theta)
        dc._final_state_for(th, stride, ctx.gen)
        dc.lam.copy_(g.reshape(-1))
        dc._adjoint(th, stride, None, seed=True)
        return dc._param_grad(theta), None
