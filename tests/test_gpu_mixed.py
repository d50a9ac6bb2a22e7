"""GPU parity on registers of per-qudit dimensions against the FP64 mixed-radix
oracle: every per-gate entry point on every qudit or pair, probabilities,
marginals, expectations and shots, the paper's dim=[2, 3, 4] example, and
plans (both per-gate schedules) with their adjoint gradients."""
import itertools

import numpy as np
import pytest

import qf_inputs as qi
from oracle import gates, measure, mixed
from tests.gpu_helpers import TOL, maxabs, rounded, to_dev, to_np

pytestmark = pytest.mark.gpu

DIMS = [[2, 3, 4], [4, 3, 2, 5], [3, 2, 2, 3, 2], [5, 7, 2, 3]]


@pytest.fixture(scope="module")
def qf():
    import paper_2409_17716_amd as qf
    return qf


def _state(dims, seed, batch=1):
    rng = np.random.default_rng(seed)
    N = int(np.prod(dims))
    v = rng.standard_normal((batch, N)) + 1j * rng.standard_normal((batch, N))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.reshape(-1)


def _rows(a, batch):
    return a.reshape(batch, -1)


@pytest.mark.parametrize("dims", DIMS, ids=str)
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_one_qudit_gates_and_slab_rotations(qf, dims, dt):
    n, rng = len(dims), np.random.default_rng(len(dims))
    psi = rounded(_state(dims, 1, batch=2), dt)
    for q in range(n):
        U = qi.random_unitary(dims[q], rng)
        x = to_dev(psi, dt)
        qf.qf_apply_1q(x, n, dims, q, U)
        want = np.concatenate([mixed.apply_1q(r, dims, q, U) for r in _rows(psi, 2)])
        assert maxabs(to_np(x), want) <= TOL[dt], q
        for kind in ("rx", "ry", "rz"):
            th = float(rng.uniform(-np.pi, np.pi))
            if kind == "rz":
                j, k = int(rng.integers(1, dims[q])), 0
                op = ("rz", q, j, 0)
            else:
                j, k = (int(v) for v in sorted(rng.choice(dims[q], size=2, replace=False)))
                op = (kind, q, j, k, 0)
            x = to_dev(psi, dt)
            qf.qf_apply_rot(x, n, dims, kind, q, j, k, th)
            want = np.concatenate([mixed.apply_op(r, dims, op, np.array([th])) for r in _rows(psi, 2)])
            assert maxabs(to_np(x), want) <= TOL[dt], (q, kind)


@pytest.mark.parametrize("dims", DIMS, ids=str)
def test_permutations_bit_exact(qf, dims):
    """CSUM, controlled shifts, SWAP (equal dimensions) and MCX on every pair:
    amplitudes move unchanged."""
    n, dt = len(dims), "c64"
    rng = np.random.default_rng(3)
    psi = rounded(_state(dims, 2), dt)
    for c, t in itertools.permutations(range(n), 2):
        x = to_dev(psi, dt)
        qf.qf_apply_ctrl(x, n, dims, c, t, list(range(dims[c])))
        assert np.array_equal(to_np(x), mixed.apply_op(psi, dims, ("csum", c, t), None)), (c, t)
        sh = tuple(int(v) for v in rng.integers(-20, 20, size=dims[c]))
        x = to_dev(psi, dt)
        qf.qf_apply_ctrl(x, n, dims, c, t, sh)
        assert np.array_equal(to_np(x), mixed.apply_op(psi, dims, ("cshift", c, t, sh), None)), (c, t)
        if dims[c] == dims[t] and c < t:
            x = to_dev(psi, dt)
            qf.qf_apply_swap(x, n, dims, c, t)
            assert np.array_equal(to_np(x), mixed.apply_op(psi, dims, ("swap", c, t), None))
    for t in range(n):
        x = to_dev(psi, dt)
        qf.qf_apply_ctrl(x, n, dims, -1, t, [dims[t] - 1])
        assert np.array_equal(to_np(x), mixed.apply_op(psi, dims, ("x", t, dims[t] - 1), None))
    for t in range(n):
        others = [q for q in range(n) if q != t]
        ctrls = [int(v) for v in rng.choice(others, size=min(3, len(others)), replace=False)]
        x = to_dev(psi, dt)
        qf.qf_apply_mcx(x, n, dims, ctrls, t)
        assert np.array_equal(to_np(x), mixed.apply_op(psi, dims, ("mcx", tuple(ctrls), t), None)), (ctrls, t)


@pytest.mark.parametrize("dims", DIMS, ids=str)
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_diagonals_controlled_rotations_and_blocks(qf, dims, dt):
    import torch
    n = len(dims)
    rng = np.random.default_rng(4)
    psi = rounded(_state(dims, 3), dt)
    for c, t in itertools.permutations(range(n), 2):
        # controlled phase w_t^(x_c x_t) as a two-qudit diagonal table over (x_c, x_t)
        tab = np.exp(2j * np.pi / dims[t]) ** np.outer(np.arange(dims[c]), np.arange(dims[t])).reshape(-1)
        x = to_dev(psi, dt)
        qf.qf_apply_diag(x, n, dims, [c, t], tab)
        assert maxabs(to_np(x), mixed.apply_op(psi, dims, ("cz", c, t), None)) <= TOL[dt], (c, t)
        for kind in ("crx", "cry", "crz"):
            th = float(rng.uniform(-np.pi, np.pi))
            if kind == "crz":
                j, k = int(rng.integers(1, dims[t])), 0
                op = ("crz", c, t, j, 0)
            else:
                j, k = (int(v) for v in sorted(rng.choice(dims[t], size=2, replace=False)))
                op = (kind, c, t, j, k, 0)
            x = to_dev(psi, dt)
            qf.qf_apply_crot(x, n, dims, kind, c, t, j, k, th)
            assert maxabs(to_np(x), mixed.apply_op(psi, dims, op, np.array([th]))) <= TOL[dt], (c, t, kind)
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    for q0 in range(n - 1):
        for k in (1, 2):
            if q0 + k > n:
                continue
            K = int(np.prod(dims[q0:q0 + k]))
            B = qi.random_unitary(K, rng)
            x = to_dev(psi, dt)
            qf.qf_apply_fused(x, n, dims, q0, k, torch.tensor(B, dtype=tdt, device="cuda"))
            assert maxabs(to_np(x), mixed.apply_block(psi, dims, q0, k, rounded(B, dt))) <= 4 * TOL[dt], (q0, k)


# Registers whose expectation chunks span many rows of the lanes' span (span
# 18, chunk 36,864: 2,048 rows, so every element takes its varying digits
# itself) or a few (span 120, chunk 5,760: 48 rows in the workgroup's table).
WIDE = [[2, 16, 2, 2, 2, 16, 3, 3, 2], [2, 3, 16, 4, 5, 3, 2]]


@pytest.mark.parametrize("dims", WIDE, ids=str)
def test_expectation_chunk_rows(qf, dims):
    n, dt = len(dims), "c128"
    psi = _state(dims, 7, batch=2)
    x = to_dev(psi, dt)
    rows = _rows(psi, 2)
    terms = [(q, "z") for q in range(n)] + [(2, np.arange(dims[2]) * 0.25 - 0.5j)]
    got = to_np(qf.qf_expect(x, n, dims, terms)).reshape(2, 2)
    for b in range(2):
        w = mixed.expect_diag(rows[b], dims, terms)
        assert abs(got[b, 0] - w.real) <= 1e-12 and abs(got[b, 1] - w.imag) <= 1e-12, (b, got[b], w)


@pytest.mark.parametrize("dims", DIMS, ids=str)
def test_measurement(qf, dims):
    """Probabilities, marginals in any order, expectation of the Z sum and of a
    custom term, and shots, on two registers."""
    import torch
    n, dt = len(dims), "c128"
    psi = _state(dims, 5, batch=2)
    x = to_dev(psi, dt)
    rows = _rows(psi, 2)
    assert maxabs(to_np(qf.qf_probs(x, n, dims)), np.concatenate([mixed.probs(r) for r in rows])) <= 1e-15
    for qs in ([n - 1], [1, 0], list(range(n))[::-1], [n - 2, n - 1, 0]):
        got = to_np(qf.qf_probs(x, n, dims, qudits=qs))
        want = np.concatenate([mixed.marginal(r, dims, qs) for r in rows])
        assert maxabs(got, want) <= 1e-14, qs
    terms = [(q, "z") for q in range(n)] + [(1, np.arange(dims[1]) * 0.5 + 0.25j)]
    got = to_np(qf.qf_expect(x, n, dims, terms)).reshape(2, 2)
    for b in range(2):
        w = mixed.expect_diag(rows[b], dims, terms)
        assert abs(got[b, 0] - w.real) <= 1e-13 and abs(got[b, 1] - w.imag) <= 1e-13
    shots = 5000
    u = qi.uniforms(2 * shots, 6)
    counts, samples = qf.qf_sample(x, n, dims, shots, torch.from_numpy(u).cuda(), qudits=[n - 1, 0], samples=True)
    samples = samples.cpu().numpy().reshape(2, shots)
    K = dims[n - 1] * dims[0]
    for b in range(2):
        p = mixed.marginal(rows[b], dims, [n - 1, 0])
        want = measure.sample_inverse_cdf(p, u[b * shots:(b + 1) * shots])
        c = np.cumsum(p)
        xs = u[b * shots:(b + 1) * shots] * c[-1]
        near = np.min(np.abs(xs[:, None] - c[None, :]), axis=1) <= 1e-12
        assert np.array_equal(samples[b][~near], want[~near])
        assert np.array_equal(counts.cpu().numpy()[b * K:(b + 1) * K], np.bincount(samples[b], minlength=K))


def test_paper_example(qf):
    """Section "Code style": dims [2, 3, 4], |0, 1, 3>, Fourier on all, R_x(pi/2)
    on qudit 0, CNOT 0 -> 2; the measured pair (0, 1) is uniform, and 1000
    shots draw the oracle's outcomes."""
    import torch
    ex = qi.paper_mixed_example()
    c = ex["circuit"]
    for dt, fuse in (("c64", 1), ("c128", 2)):
        p = qf.plan_for(c, dt, fuse=fuse)
        t = qf.new_state(c.n, c.dims, dt)
        qf.qf_state_init(t, c.n, c.dims, list(ex["digits"]))
        p.forward(t, c.theta)
        want = mixed.run(c, digits=ex["digits"])
        assert maxabs(to_np(t), want) <= TOL[dt]
        prob = to_np(qf.qf_probs(t, c.n, c.dims, qudits=ex["measured"]))
        assert np.allclose(prob, 1 / 6, atol=1e-6 if dt == "c64" else 1e-14)
        u = qi.uniforms(ex["shots"], 3)
        counts, s = qf.qf_sample(t, c.n, c.dims, ex["shots"], torch.from_numpy(u).cuda(), qudits=ex["measured"],
                                 samples=True)
        ref = measure.sample_inverse_cdf(mixed.marginal(want, c.dims, ex["measured"]), u)
        edges = np.arange(1, 7) / 6
        near = np.min(np.abs(u[:, None] - edges[None, :]), axis=1) <= 1e-6
        assert np.array_equal(s.cpu().numpy()[~near], ref[~near])
        assert int(counts.sum().item()) == 1000


def _grad_close(g, ref, rel, dt):
    floor = (1e-2 if dt == "c64" else 1e-3) * np.abs(ref).max()
    return np.all(np.abs(g - ref) <= rel * np.maximum(np.abs(ref), floor))


CIRCS = [
    ("d234", lambda: qi.random_mixed_circuit([2, 3, 4], 120, 1), "c128"),
    ("d4325", lambda: qi.random_mixed_circuit([4, 3, 2, 5], 150, 2), "c64"),
    ("d32232", lambda: qi.random_mixed_circuit([3, 2, 2, 3, 2], 150, 3), "c128"),
    ("d5723_hea", lambda: qi.mixed_hea([5, 7, 2, 3], 3, 4), "c64"),
]


@pytest.mark.parametrize("name,make,dt", CIRCS, ids=[c[0] for c in CIRCS])
@pytest.mark.parametrize("fuse", [1, 2])
def test_plans_forward_and_adjoint(qf, name, make, dt, fuse):
    c = make()
    terms = [(q, "z") for q in range(c.n)]
    p = qf.plan_for(c, dt, fuse=fuse)
    t = qf.new_state(c.n, c.dims, dt)
    qf.qf_state_init(t, c.n, c.dims, None)
    p.forward(t, c.theta)
    want = mixed.run(c)
    assert maxabs(to_np(t), want) <= 4 * TOL[dt]
    lam = qf.new_state(c.n, c.dims, dt)
    g = p.adjoint_grad(t, lam, c.theta, terms)
    ref = mixed.adjoint(c, terms)
    assert _grad_close(g, ref, 1e-4 if dt == "c64" else 1e-9, dt), np.abs(g - ref).max()


def test_batched_plan_and_seeded_adjoint(qf):
    """Three registers from different basis states through one plan; the seeded
    adjoint (lam = dL/d conj psi of L = sum |psi|^4) against the oracle's."""
    import torch
    c = qi.random_mixed_circuit([3, 4, 2, 3], 100, 5, kinds=["h", "rx", "ry", "rz", "csum", "cz", "crx", "crz",
                                                               "mcx", "u1"])
    digs = [[0, 0, 0, 0], [2, 3, 1, 0], [1, 2, 0, 2]]
    p = qf.plan_for(c, "c128", fuse=2)
    t = qf.new_state(c.n, c.dims, "c128", batch=3)
    qf.qf_state_init(t, c.n, c.dims, np.array(digs))
    p.forward(t, c.theta)
    want = [mixed.run(c, digits=d) for d in digs]
    assert maxabs(to_np(t), np.concatenate(want)) <= 1e-12
    # L = sum |psi|^4: dL/d(conj psi) = 2 |psi|^2 psi; torch's gradient is twice that
    lam = torch.tensor(np.concatenate([4 * np.abs(w) ** 2 * w for w in want]), dtype=torch.complex128,
                       device="cuda")
    g = p.adjoint_grad(t, lam, c.theta, None, seed=True)
    for b in range(3):
        ref = mixed.adjoint_seeded(c, 2 * np.abs(want[b]) ** 2 * want[b])
        ref_psi = mixed.run(c, digits=digs[b])
        assert np.allclose(ref_psi, want[b])
        # the oracle's seeded walk starts from |0...0>; rerun it from this register's basis state
        lam0 = 2 * np.abs(want[b]) ** 2 * want[b]
        psi = want[b].copy()
        gb = np.zeros(c.nparams)
        for op in reversed(c.ops):
            if op[0] in mixed.ROTATIONS:
                gb[op[-1]] += mixed._derivative_term(op, c.dims, psi, lam0)
            inv = mixed.inverse_op(op, c.dims, c.theta)
            psi = mixed.apply_op(psi, c.dims, inv, c.theta)
            lam0 = mixed.apply_op(lam0, c.dims, inv, c.theta)
        if b == 0:
            assert np.allclose(gb, ref, atol=1e-12)
        assert _grad_close(g[b], gb, 1e-9, "c128")


def test_large_mixed_register(qf):
    """dims [2, 3, 4, 5] x 3 (1.7 million amplitudes), complex64: the mixed
    ansatz in both schedules against the oracle, with the gradient."""
    dims = [2, 3, 4, 5] * 3
    c = qi.mixed_hea(dims, 2, 6)
    terms = [(q, "z") for q in range(c.n)]
    want = mixed.run(c)
    ref = mixed.adjoint(c, terms)
    for fuse in (1, 2):
        p = qf.plan_for(c, "c64", fuse=fuse)
        t = qf.new_state(c.n, c.dims, "c64")
        qf.qf_state_init(t, c.n, c.dims, None)
        p.forward(t, c.theta)
        assert maxabs(to_np(t), want) <= 5e-6
        lam = qf.new_state(c.n, c.dims, "c64")
        g = p.adjoint_grad(t, lam, c.theta, terms)
        assert _grad_close(g, ref, 1e-4, "c64"), np.abs(g - ref).max()


def test_autograd_on_mixed_registers(qf):
    """loss.backward() through the torch.autograd.Functions on a mixed register
    (host-angle calls): the expectation over two registers and the paper's
    state loss sum |t - psi|, against the mixed oracle's adjoint."""
    import torch
    from paper_2409_17716_amd.autograd import DeviceCircuit
    c = qi.random_mixed_circuit([2, 3, 4, 3], 80, 7, kinds=["h", "rx", "ry", "rz", "csum", "cz", "crx", "cry",
                                                             "crz", "mcx"])
    terms = [(q, "z") for q in range(c.n)]
    dc = DeviceCircuit(c, dtype="c128", batch=2)
    assert dc.host
    th = torch.tensor(c.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    L = dc.expectation(th, terms).sum()
    L.backward()
    assert abs(L.item() - 2 * mixed.loss(c, terms)) <= 1e-12
    assert _grad_close(th.grad.cpu().numpy(), 2 * mixed.adjoint(c, terms), 1e-9, "c128")
    target = _state(c.dims, 9)
    dc2 = DeviceCircuit(c, dtype="c128")
    th2 = torch.tensor(c.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    psi = dc2.state(th2)
    loss = (torch.tensor(target, device="cuda") - psi).abs().sum()
    loss.backward()
    want = mixed.run(c)
    r = target - want
    ref = mixed.adjoint_seeded(c, -r / (2 * np.abs(r)))
    assert abs(loss.item() - np.abs(r).sum()) <= 1e-10
    assert _grad_close(th2.grad.cpu().numpy(), ref, 1e-9, "c128")
