"""GPU parity of the device-parameter (bound) mode and of ragged batches stepped
as one HIP graph, against the FP64 oracle and the per-circuit path."""
import numpy as np
import pytest

import qf_inputs as qi
from oracle import grad, measure, sim
from tests.gpu_helpers import maxabs, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qf():
    import paper_2409_17716_amd as qf
    return qf


def _close(g, ref, rel=1e-4, floor=1e-2):
    f = floor * np.abs(ref).max()
    return np.all(np.abs(g - ref) <= rel * np.maximum(np.abs(ref), f))


@pytest.mark.parametrize("make,dt", [(lambda: qi.config3(n=5, layers=2), "c64"),
                                     (lambda: qi.random_circuit(3, 5, 120, 41), "c128"),
                                     (lambda: qi.config2(n=6, layers=3), "c64")])
def test_bound_mode_shared_theta(qf, make, dt):
    import torch
    c = make()
    terms = qi.zsum_terms(c.n)
    p = qf.plan_for(c, dt)
    p.bind(1)
    th = torch.tensor(c.theta, dtype=torch.float64, device="cuda")
    t = qf.new_state(c.n, c.dim, dt)
    lam = qf.new_state(c.n, c.dim, dt)
    g = torch.zeros(max(1, c.nparams), dtype=torch.float64, device="cuda")
    loss = torch.zeros(2, dtype=torch.float64, device="cuda")
    qf.qf_state_init(t, c.n, c.dim, None)
    p.forward_dev(t, th, 0)
    want = sim.run(c)
    tol = 2e-5 if dt == "c64" else 1e-12
    assert maxabs(to_np(t), want) <= tol
    p.adjoint_grad_dev(t, lam, th, 0, terms, g, loss)
    ref = grad.adjoint(c, terms)
    assert _close(to_np(g)[:c.nparams], ref, 1e-4 if dt == "c64" else 1e-9, 1e-2 if dt == "c64" else 1e-3)
    lv = to_np(loss)
    assert abs(lv[0] - measure.expect_diag(want, c.dim, c.n, terms).real) <= 1e-5


@pytest.mark.parametrize("kernel", [0, 2])
def test_bound_mode_per_register_theta_and_checkpoints(qf, kernel):
    import torch
    c = qi.config2(n=5, layers=3)
    terms = qi.zsum_terms(c.n)
    B = 3
    rng = np.random.default_rng(9)
    thetas = rng.uniform(-np.pi, np.pi, size=(B, c.nparams))
    p = qf.plan_for(c, "c64", ckpt_every=40, stage_kernel=kernel, tile_digits=3, pipe_wgs=1)
    p.bind(B)
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    t = qf.new_state(c.n, c.dim, "c64", batch=B)
    lam = qf.new_state(c.n, c.dim, "c64", batch=B)
    g = torch.zeros((B, c.nparams), dtype=torch.float64, device="cuda")
    qf.qf_state_init(t, c.n, c.dim, None)
    p.forward_dev(t, th, c.nparams)
    got = to_np(t).reshape(B, -1)
    for b in range(B):
        assert maxabs(got[b], sim.run(c, theta=thetas[b])) <= 2e-5
    p.adjoint_grad_dev(t, lam, th, c.nparams, terms, g)
    gg = to_np(g)
    for b in range(B):
        assert _close(gg[b], grad.adjoint(c, terms, theta=thetas[b]))


@pytest.mark.parametrize("tune,streams,split", [(False, 0, False), (False, 4, False), (True, 4, False),
                                                (False, 16, False), (False, 3, True)])
def test_ragged_batch_graph_replays(qf, tune, streams, split):
    """Ragged batch (D=3 and D=4 registers of uneven n) captured in one graph,
    on one stream or one stream per group, with default or autotuned
    schedules: every replay, with eager work and new angles between replays,
    matches the oracle and the per-circuit path."""
    import torch
    from paper_2409_17716_amd.batched import PlainLoop, RaggedBatch
    circuits = qi.config4(count_d3=5, count_d4=3, layers=2)
    circuits = [c for c in circuits if c.n <= 7]
    rb = RaggedBatch(circuits, tune=tune, streams=streams, split=split)
    for sch in rb.schedules():
        assert sch["fuse"] == 0 and sch["stages"] >= 1
    rb.capture()
    rng = np.random.default_rng(5)
    for rep in range(3):
        if rep:
            for i, c in enumerate(circuits):
                c.theta = rng.uniform(-np.pi, np.pi, size=c.nparams)
                rb.set_angles(i, c.theta)
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        rb.replay()
        torch.cuda.synchronize()
        grads = rb.gradients()
        losses = rb.losses()
        for i, c in enumerate(circuits):
            terms = qi.zsum_terms(c.n)
            ref = grad.adjoint(c, terms)
            assert _close(grads[i], ref), (rep, i)
            assert abs(losses[i] - grad.loss(c, terms)) <= 1e-5
    plain = PlainLoop(circuits)
    plain.step()
    for i in range(len(circuits)):
        assert _close(plain.grads[i], rb.gradients()[i])
