"""Ragged batches of variational circuits on one GPU.

Circuits are grouped by (D, n, gate layout); every group becomes one bound
stage plan over a batch of registers, with each register's angles (and clock
exponents) in a device array.  One training step (init, forward, <O> and the
adjoint gradient of every circuit) is then a fixed sequence of kernel launches
with no host work, captured once in a HIP graph and replayed per step; new
angles are written into the device arrays between replays.  The groups are
spread over a few streams (forked from and joined back into the capturing
stream) by longest-processing-time-first on their algorithmic bytes per step,
so the graph holds that many independent chains of about equal length (with
split=True a group with more than 1/streams of the amplitudes is first split
into batch chunks, each with its own plan; measured slower on the 1024-circuit
batch, whose largest group does not limit the step once the GPU is full) and the
groups' small launches overlap on the GPU (HIP maps streams onto a handful of
hardware queues, 4 by default, so more streams than that would share queues
unevenly).  With tune=True the autotuner picks
every group's schedule (tile size, register-group size: per-qudit D x D
matrices or two-qudit D^2 x D^2 blocks, stage kernel) by timing forward plus
adjoint in the device-parameter mode at the group's batch.

``plain_step`` runs the same circuits one at a time through the ordinary
per-circuit path (host-built matrices, host gradient) for comparison.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import Plan, new_state, qf_state_init


def _torch():
    import torch
    return torch


def default_terms(n: int):
    """sum_i Z_i (the loss Re<sum_i Z_i>)."""
    return [(q, "z") for q in range(n)]


def _layout(c) -> Tuple:
    """Gate layout of a circuit with angles and clock exponents abstracted."""
    key = []
    for op in c.ops:
        if op[0] == "clock":
            key.append(("clock", op[1]))
        elif op[0] in ("rx", "ry", "rz"):
            key.append(op[:-1] + (op[-1],))
        elif op[0] == "u":
            key.append(("u", op[1], op[2], np.asarray(op[3]).tobytes()))
        else:
            key.append(op)
    return (c.dim, c.n, tuple(key))


@dataclass
class _Group:
    idx: List[int]
    dim: int
    n: int
    nrot: int                      # rotation angles per circuit
    nclock: int                    # clock exponents per circuit (stored after the angles)
    plan: Plan = None
    theta: object = None           # device float64 [batch, nrot + nclock]
    psi: object = None
    lam: object = None
    grad: object = None            # device float64 [batch, nrot + nclock]
    loss: object = None            # device float64 [batch, 2]
    terms: list = field(default_factory=list)
    options: dict = field(default_factory=dict)  # the schedule options the plan was built with
    chain: int = 0                 # index of the stream the group's launches go to


class RaggedBatch:
    """A ragged batch of circuits (uneven n and D) stepped as one HIP graph."""

    def __init__(self, circuits: Sequence, dtype: str = "c64",
                 terms: Callable[[int], list] = default_terms, tune: bool = False, streams: int = 4,
                 split: bool = False):
        torch = _torch()
        self.circuits = list(circuits)
        self.dtype = dtype
        groups: Dict[Tuple, List[int]] = {}
        for i, c in enumerate(self.circuits):
            groups.setdefault(_layout(c), []).append(i)
        # a group holding more than a share of the amplitudes is split into
        # batch chunks, so that the chains can be balanced
        share = sum(c.dim ** c.n for c in self.circuits) / max(1, int(streams))
        chunks = []
        for key, idx in sorted(groups.items(), key=lambda kv: (kv[0][0], kv[0][1])):
            amps = len(idx) * self.circuits[idx[0]].dim ** self.circuits[idx[0]].n
            parts = min(len(idx), max(1, int(np.ceil(amps / share)))) if streams and split else 1
            for p in range(parts):
                chunks.append((key, idx[p * len(idx) // parts:(p + 1) * len(idx) // parts]))
        self.groups: List[_Group] = []
        for key, idx in chunks:
            c0 = self.circuits[idx[0]]
            ops, nclock = [], 0
            for op in c0.ops:
                if op[0] == "clock":
                    ops.append(("clockp", op[1], c0.nparams + nclock))
                    nclock += 1
                else:
                    ops.append(op)
            P = c0.nparams + nclock
            g = _Group(idx=idx, dim=c0.dim, n=c0.n, nrot=c0.nparams, nclock=nclock)
            g.plan = Plan(c0.dim, c0.n, ops, P, dtype)
            th = np.zeros((len(idx), P))
            for r, ci in enumerate(idx):
                c = self.circuits[ci]
                th[r, :c.nparams] = c.theta
                th[r, c.nparams:] = [op[2] for op in c.ops if op[0] == "clock"]
            g.theta = torch.tensor(th, dtype=torch.float64, device="cuda")
            g.psi = new_state(g.n, g.dim, dtype, batch=len(idx))
            g.lam = new_state(g.n, g.dim, dtype, batch=len(idx))
            if tune:
                qf_state_init(g.psi, g.n, g.dim, None)
                g.options = g.plan.autotune(g.psi, th[0], adjoint=True, bound=True)
            g.plan.bind(len(idx))
            g.grad = torch.zeros((len(idx), P), dtype=torch.float64, device="cuda")
            g.loss = torch.zeros((len(idx), 2), dtype=torch.float64, device="cuda")
            g.terms = terms(g.n)
            self.groups.append(g)
        # longest processing time first: each group, heaviest first, joins the
        # chain with the least work so far
        self.streams = [torch.cuda.Stream() for _ in range(min(int(streams), len(self.groups)))]
        load = [0.0] * max(1, len(self.streams))
        for g in sorted(self.groups, key=self.group_bytes, reverse=True):
            g.chain = int(np.argmin(load))
            load[g.chain] += self.group_bytes(g)
        self.chain_bytes = load
        self.graph = None

    @staticmethod
    def group_bytes(g: _Group) -> float:
        """Algorithmic HBM bytes of one step of a group: each forward pass reads
        and writes the batch's states once, each adjoint pass psi and lam."""
        state = g.psi.numel() * g.psi.element_size()
        return state * (2 * g.plan.num_stages + 4 * g.plan.num_adjoint_stages)

    @property
    def amplitudes(self) -> int:
        return sum(c.dim ** c.n for c in self.circuits)

    def _group_step(self, g: _Group) -> None:
        P = g.nrot + g.nclock
        qf_state_init(g.psi, g.n, g.dim, None)
        g.plan.forward_dev(g.psi, g.theta, P)
        g.plan.adjoint_grad_dev(g.psi, g.lam, g.theta, P, g.terms, g.grad, g.loss)

    def step(self) -> None:
        """Enqueue one training step of every circuit: each chain of groups on
        its stream, forked from and joined back into the current stream."""
        torch = _torch()
        cur = torch.cuda.current_stream()
        if not self.streams:
            for g in self.groups:
                self._group_step(g)
            return
        for si, s in enumerate(self.streams):
            s.wait_stream(cur)
            with torch.cuda.stream(s):
                for g in self.groups:
                    if g.chain == si:
                        self._group_step(g)
        for s in self.streams:
            cur.wait_stream(s)

    def schedules(self) -> List[dict]:
        """Per group: D, n, batch and the schedule options its plan was built with
        (those the autotuner chose when tune=True)."""
        keep = ("fuse", "tile_digits", "adj_tile_digits", "group_digits", "stage_kernel", "pipe_wgs")
        return [{"D": g.dim, "n": g.n, "batch": len(g.idx), "stages": g.plan.num_stages,
                 "adjoint_stages": g.plan.num_adjoint_stages, "stream": g.chain,
                 "step_bytes": int(self.group_bytes(g)), **{k: g.options.get(k, 0) for k in keep}}
                for g in self.groups]

    def capture(self) -> None:
        """Capture step() in a HIP graph (after one eager warm-up step)."""
        torch = _torch()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.step()
        torch.cuda.synchronize()

    def replay(self) -> None:
        self.graph.replay()

    def set_angles(self, i: int, theta: np.ndarray) -> None:
        """Write new rotation angles of circuit i into its group's device array."""
        torch = _torch()
        for g in self.groups:
            if i in g.idx:
                r = g.idx.index(i)
                g.theta[r, :g.nrot].copy_(torch.as_tensor(theta, dtype=torch.float64))
                return
        raise KeyError(i)

    def gradients(self) -> List[np.ndarray]:
        out: List[Optional[np.ndarray]] = [None] * len(self.circuits)
        for g in self.groups:
            gr = g.grad.cpu().numpy()
            for r, ci in enumerate(g.idx):
                out[ci] = gr[r, :g.nrot].copy()
        return out

    def losses(self) -> np.ndarray:
        out = np.zeros(len(self.circuits))
        for g in self.groups:
            lv = g.loss.cpu().numpy()
            for r, ci in enumerate(g.idx):
                out[ci] = lv[r, 0]
        return out


class PlainLoop:
    """The same circuits one at a time through the per-circuit path: a plan per
    circuit, host-built matrices, and the host-side gradient of qf_adjoint_grad."""

    def __init__(self, circuits: Sequence, dtype: str = "c64",
                 terms: Callable[[int], list] = default_terms):
        from . import plan_for
        self.circuits = list(circuits)
        self.plans = [plan_for(c, dtype) for c in self.circuits]
        self.psi = [new_state(c.n, c.dim, dtype) for c in self.circuits]
        self.lam = [new_state(c.n, c.dim, dtype) for c in self.circuits]
        self.terms = [terms(c.n) for c in self.circuits]
        self.grads: List[np.ndarray] = []

    def step(self) -> None:
        self.grads = []
        for c, p, psi, lam, t in zip(self.circuits, self.plans, self.psi, self.lam, self.terms):
            qf_state_init(psi, c.n, c.dim, None)
            p.forward(psi, c.theta)
            self.grads.append(p.adjoint_grad(psi, lam, c.theta, t))
