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
"""
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


def test_config3_full_and_gradient(qf):
    """D=5, n=10, 1120 gates: forward properties, then the stage adjoint against
    the per-gate adjoint (960 parameters)."""
    c = qi.config3()
    check_forward(qf, c)
    terms = qi.zsum_terms(c.n)
    grads = []
    for fuse in (0, 1):
        p, t = run(qf, c, fuse=fuse)
        lam = qf.new_state(c.n, c.dim, "c64")
        grads.append(p.adjoint_grad(t, lam, c.theta, terms))
    g0, g1 = grads
    err = np.abs(g0 - g1).max() / np.abs(g1).max()
    print(f"[fullsize] config3 gradient: max|stage - per-gate| / max|g| = {err:.2e}", flush=True)
    assert err <= 1e-3


def test_config5_full(qf):
    """D=10, n=8 (10^8 amplitudes, 800 MB in complex64)."""
    check_forward(qf, qi.config5())


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
        if c.n > 8:
            continue
        ref = grad.adjoint(c, qi.zsum_terms(c.n))
        assert np.abs(gb[i] - ref).max() <= 1e-4 * np.abs(ref).max()
