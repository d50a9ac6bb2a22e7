"""GPU checks at the full workload sizes, in the launch configuration bench.py
times (default plans).  The FP64 oracle cannot evaluate these circuits
(3^16, 5^10 and 10^8 amplitudes, hundreds of gates) amplitude by amplitude, so
the checks are properties that hold at any size:

* the default stage plan agrees with the independent one-kernel-per-gate plan
  (fuse=1: per-axis sweeps, permutation and diagonal kernels, each pinned to the
  oracle at small sizes) in the 2-norm of the difference;
* unitarity: the state keeps norm 1, and the inverse circuit (angles negated,
  order reversed, CSUM as the inverse shift, clock and CZ as their inverse
  powers) returns it to |0...0>;
* probabilities sum to 1 and <Z_0> from qf_expect equals the sum over the
  probabilities;
* gradients: the stage adjoint agrees with the per-gate adjoint; the ragged
  batch agrees with the per-circuit loop and, on sampled circuits, with the
  oracle adjoint.

Where the FP64 oracle can evaluate a full-size circuit in minutes on CPU cores,
its values were written once by tests/golden/make_fullsize_goldens.py (oracle
only) and are compared element by element: the D=5, n=10 loss and all 960
gradients (and 16 FP64 central differences), the D=3, n=16 <Z_0>, <sum Z_i>
and single-qudit marginals.
"""
import json
import os

import numpy as np
import pytest

import qf_inputs as qi
from oracle import grad
from tests.gpu_helpers import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qf():
    import paper_2409_17716_amd as qf
    return qf


def inverse_circuit(c):
    """The circuit's inverse as a descriptor list plus its angle vector (the
    rotation angles negated).  Inverses stay in descriptor form: H^-1 = H^3,
    (Z^a)^-1 = Z^(D-a), CSUM^-1 = shift by -x_c, CZ^-1 = CZ^(D-1)."""
    D = c.dim
    ops = []
    for op in reversed(c.ops):
        k = op[0]
        if k == "h":
            ops += [op] * 3
        elif k == "clock":
            ops.append(("clock", op[1], (-op[2]) % D))
        elif k == "csum":
            ops.append(("cshift", op[1], op[2], tuple((-v) % D for v in range(D))))
        elif k == "cz":
            ops += [op] * (D - 1)
        elif k in ("rx", "ry", "rz"):
            ops.append(op)
        else:
            raise ValueError(k)
    return qi.Circuit(dim=D, n=c.n, ops=ops, theta=-np.asarray(c.theta), name=c.name + "_inv")


def run(qf, c, **kw):
    p = qf.plan_for(c, "c64", **kw)
    t = qf.new_state(c.n, c.dim, "c64")
    qf.qf_state_init(t, c.n, c.dim, None)
    p.forward(t, c.theta)
    return p, t


def check_forward(qf, c):
    import torch
    _, ts = run(qf, c)
    _, tg = run(qf, c, fuse=1)
    diff = torch.linalg.vector_norm((ts - tg).to(torch.complex128)).item()
    norm = torch.linalg.vector_norm(ts.to(torch.complex128)).item()
    print(f"[fullsize] {c.name}: |stage - per-gate|_2 = {diff:.2e}, |psi| - 1 = {norm - 1:.2e}", flush=True)
    assert diff <= 1e-4
    assert abs(norm - 1) <= 1e-4
    # the inverse circuit returns the state to |0...0>
    ci = inverse_circuit(c)
    pi = qf.plan_for(ci, "c64")
    pi.forward(ts, ci.theta)
    a0 = abs(complex(ts[0].item()))
    print(f"[fullsize] {c.name}: |<0|C^-1 C|0>| = {a0:.7f}", flush=True)
    assert a0 >= 1 - 1e-4
    # probabilities and <Z_0> on the forward state
    probs = qf.qf_probs(tg, c.n, c.dim)
    total = probs.to(torch.float64).sum().item()
    assert abs(total - 1) <= 1e-4
    e = to_np(qf.qf_expect(tg, c.n, c.dim, qi.z0_terms()))
    N = c.dim ** c.n
    x0 = torch.arange(N, device="cuda", dtype=torch.int64) // (c.dim ** (c.n - 1))
    w = torch.exp(2j * np.pi * x0.to(torch.float64) / c.dim)
    ref = (probs.to(torch.float64) * w).sum().item()
    assert abs(complex(e[0], e[1]) - ref) <= 1e-6


def test_config2_full(qf):
    """D=3, n=16 (43,046,721 amplitudes), the benchmarked circuit."""
    check_forward(qf, qi.config2())


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _grad_close(g, ref, rel, floor_frac):
    floor = floor_frac * np.abs(ref).max()
    return np.all(np.abs(g - ref) <= rel * np.maximum(np.abs(ref), floor))


def _report(tag, g, ref):
    err = np.abs(g - ref)
    rel = err / np.maximum(np.abs(ref), 1e-300)
    print(f"[fullsize] {tag}: max|dg| = {err.max():.3e} (max|g| {np.abs(ref).max():.3e}), max|dg|/max|g| = "
          f"{err.max() / np.abs(ref).max():.3e}, relative error quantiles 50/90/99/100% = "
          f"{np.quantile(rel, 0.5):.2e} / {np.quantile(rel, 0.9):.2e} / {np.quantile(rel, 0.99):.2e} / "
          f"{rel.max():.2e}", flush=True)


def test_config3_full_and_gradient(qf):
    """D=5, n=10, 1120 gates in complex64 (the workload's precision): forward
    properties, then the default-plan stage adjoint against the FP64 oracle's
    loss and all 960 adjoint gradients, and the 16 FP64 central differences the
    workload names (tests/golden/config3_d5_n10_full.json, written by the oracle
    only).  Relative bound 1e-4 with the complex64 floor 1e-2 * max|g| (the
    relative bound alone is not reachable for near-zero entries in single
    precision; the observed distribution is printed)."""
    c = qi.config3()
    check_forward(qf, c)
    gold = _golden("config3_d5_n10_full.json")
    ref = np.array(gold["grad_adjoint"])
    fd = np.array(gold["grad_fd"])
    idx = np.array(gold["fd_params"])
    terms = qi.zsum_terms(c.n)
    p, t = run(qf, c)
    lam = qf.new_state(c.n, c.dim, "c64")
    loss = to_np(qf.qf_expect(t, c.n, c.dim, terms))[0]
    print(f"[fullsize] config3 c64 loss {loss!r} vs oracle {gold['loss']!r}", flush=True)
    assert abs(loss - gold["loss"]) <= 1e-7
    g = p.adjoint_grad(t, lam, c.theta, terms)
    _report("config3 c64 stage adjoint vs oracle adjoint", g, ref)
    _report("config3 c64 stage adjoint vs FP64 FD (16)", g[idx], fd)
    assert _grad_close(g, ref, 1e-4, 1e-2)
    assert _grad_close(g[idx], fd, 1e-4, 1e-2)


def test_config3_full_complex128_and_autograd(qf):
    """The same 960 gradients with a complex128 state (oracle adjoint to 1e-8
    relative, FD to 1e-4), and in complex64 through the autograd front end
    (loss.backward())."""
    import torch
    from paper_2409_17716_amd.autograd import DeviceCircuit
    c = qi.config3()
    gold = _golden("config3_d5_n10_full.json")
    ref = np.array(gold["grad_adjoint"])
    fd = np.array(gold["grad_fd"])
    idx = np.array(gold["fd_params"])
    terms = qi.zsum_terms(c.n)
    p = qf.plan_for(c, "c128")
    t = qf.new_state(c.n, c.dim, "c128")
    qf.qf_state_init(t, c.n, c.dim, None)
    p.forward(t, c.theta)
    lam = qf.new_state(c.n, c.dim, "c128")
    g = p.adjoint_grad(t, lam, c.theta, terms)
    _report("config3 c128 stage adjoint vs oracle adjoint", g, ref)
    assert _grad_close(g, ref, 1e-8, 1e-3)
    # the central differences carry about 6e-10 of their own error (h = 1e-6),
    # so the FD comparison uses the same floor in both precisions
    assert _grad_close(g[idx], fd, 1e-4, 1e-2)
    del t, lam
    dc = DeviceCircuit(c)
    theta = torch.tensor(c.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    L = dc.expectation(theta, terms)
    L.backward()
    ga = theta.grad.cpu().numpy()
    _report("config3 c64 autograd vs oracle adjoint", ga, ref)
    assert abs(L.item() - gold["loss"]) <= 1e-7
    assert _grad_close(ga, ref, 1e-4, 1e-2)
    assert _grad_close(ga[idx], fd, 1e-4, 1e-2)


def test_config2_full_against_oracle(qf):
    """D=3, n=16 (the benchmarked circuit, default plan): <Z_0>, Re and Im of
    <sum_i Z_i> and every single-qudit marginal against the FP64 oracle
    (tests/golden/config2_d3_n16_full.json).  A marginal p of a state with
    error dpsi moves by at most 2 sqrt(p) |dpsi|_2; with |dpsi|_2 about 1.4e-6
    (the measured distance between the stage and per-gate paths after 1280
    complex64 gates) that is 1.6e-6, so |dp| <= 2e-6.  The expectation values
    are held to 1e-8 absolute, far below their worst-case bound 2 |dpsi|_2 and
    about 100 times the observed error (rounding errors of the 3^16
    amplitudes largely cancel in the sums); the observed errors are printed."""
    c = qi.config2()
    gold = _golden("config2_d3_n16_full.json")
    _, t = run(qf, c)
    z0 = to_np(qf.qf_expect(t, c.n, c.dim, qi.z0_terms()))
    zs = to_np(qf.qf_expect(t, c.n, c.dim, qi.zsum_terms(c.n)))
    dz0 = abs(complex(z0[0], z0[1]) - complex(*gold["z0"]))
    dzs = abs(complex(zs[0], zs[1]) - complex(*gold["zsum"]))
    dm = 0.0
    for q in range(c.n):
        pm = to_np(qf.qf_probs(t, c.n, c.dim, [q]))
        dm = max(dm, float(np.abs(pm - np.array(gold["marginals"][q])).max()))
    print(f"[fullsize] config2: |d<Z_0>| = {dz0:.3e} (|<Z_0>| = {abs(complex(*gold['z0'])):.3e}), "
          f"|d<sum Z>| = {dzs:.3e}, max |d marginal| = {dm:.3e}", flush=True)
    assert dz0 <= 1e-8 and dzs <= 1e-8
    assert dm <= 2e-6


def test_config5_full(qf):
    """D=10, n=8 (10^8 amplitudes, 800 MB in complex64)."""
    check_forward(qf, qi.config5())


def test_config5_full_checkpointed_adjoint(qf):
    """D=10, n=8, 864 parameters: the adjoint with a checkpoint every 4 layers
    (320 gates, two saved states) against the checkpoint-free stage adjoint and
    the per-gate adjoint (one axis kernel per fused run)."""
    c = qi.config5()
    terms = qi.zsum_terms(c.n)
    grads = {}
    for name, kw in (("ckpt", dict(ckpt_every=320)), ("plain", {}), ("per_gate", dict(fuse=2))):
        p, t = run(qf, c, **kw)
        lam = qf.new_state(c.n, c.dim, "c64")
        grads[name] = p.adjoint_grad(t, lam, c.theta, terms)
        del p, t, lam
    ref = grads["per_gate"]
    _report("config5 checkpointed vs per-gate", grads["ckpt"], ref)
    _report("config5 plain vs per-gate", grads["plain"], ref)
    assert _grad_close(grads["ckpt"], ref, 1e-4, 1e-2)
    assert _grad_close(grads["plain"], ref, 1e-4, 1e-2)
    assert _grad_close(grads["ckpt"], grads["plain"], 1e-4, 1e-2)


def test_config4_full_batch(qf):
    """All 1024 ragged circuits in one graph replay against the per-circuit loop,
    and 8 sampled circuits against the oracle adjoint."""
    import torch
    from paper_2409_17716_amd.batched import PlainLoop, RaggedBatch
    circuits = qi.config4()
    rb = RaggedBatch(circuits)
    rb.capture()
    rb.replay()
    torch.cuda.synchronize()
    gb = rb.gradients()
    pl = PlainLoop(circuits)
    pl.step()
    rel = max(float(np.abs(gb[i] - pl.grads[i]).max() / np.abs(pl.grads[i]).max()) for i in range(len(circuits)))
    print(f"[fullsize] config4: max relative gradient difference batched vs loop = {rel:.2e}", flush=True)
    assert rel <= 1e-6
    rng = np.random.default_rng(11)
    for i in rng.choice(len(circuits), size=8, replace=False):
        c = circuits[int(i)]
        ref = grad.adjoint(c, qi.zsum_terms(c.n))
        assert _grad_close(gb[i], ref, 1e-4, 1e-2), (i, c.n)
