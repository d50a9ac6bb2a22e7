"""GPU parity of planned circuits (forward) and of the adjoint gradient against the
FP64 oracle: full states at small sizes, the five workloads at reduced size, and
gradients against the oracle adjoint and central finite differences."""
import numpy as np
import pytest

import qf_inputs as qi
from oracle import grad, measure, sim
from tests.gpu_helpers import TOL, maxabs, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qf():
    import paper_2409_17716_amd as qf
    return qf


def run_gpu(qf, c, dtype, fuse=0, psi0=None, **kw):
    p = qf.plan_for(c, dtype, fuse=fuse, **kw)
    if psi0 is None:
        t = qf.new_state(c.n, c.dim, dtype)
        qf.qf_state_init(t, c.n, c.dim, None)
    else:
        t = to_dev(psi0, dtype)
    p.forward(t, c.theta)
    return p, t


CIRCUITS = [
    ("config1", lambda: qi.config1(), "c128"),
    ("config2_small", lambda: qi.config2(n=7, layers=3), "c64"),
    ("config3_small", lambda: qi.config3(n=5, layers=2), "c64"),
    ("config5_small", lambda: qi.config5(n=4, layers=2), "c64"),
    ("random_d3", lambda: qi.random_circuit(3, 6, 120, 1), "c128"),
    ("random_d4", lambda: qi.random_circuit(4, 5, 120, 2), "c64"),
    ("random_d7", lambda: qi.random_circuit(7, 3, 80, 3), "c128"),
]


@pytest.mark.parametrize("name,make,dt", CIRCUITS, ids=[c[0] for c in CIRCUITS])
@pytest.mark.parametrize("fuse,kernel", [(0, 0), (0, 1), (0, 2), (1, 0), (2, 0), (3, 0)])
def test_plan_forward_matches_oracle(qf, name, make, dt, fuse, kernel):
    c = make()
    _, t = run_gpu(qf, c, dt, fuse=fuse, stage_kernel=kernel)
    want = sim.run(c)
    assert maxabs(to_np(t), want) <= TOL[dt], name


PAIR_SHIFT = [
    ("config2_n10", lambda: qi.config2(n=10, layers=3), "c64"),
    ("config2_n11", lambda: qi.config2(n=11, layers=2), "c64"),
    ("hea_d4_n8", lambda: qi.hea(4, 8, 2, 31), "c64"),
    ("hea_d3_n10_chain", lambda: qi.hea(3, 10, 3, 32, entangler="chain"), "c64"),
    ("hea_d3_n10_c128", lambda: qi.hea(3, 10, 2, 35), "c128"),
    ("hea_d4_n7_c128", lambda: qi.hea(4, 7, 2, 36), "c128"),
]


@pytest.mark.parametrize("name,make,dt", PAIR_SHIFT, ids=[c[0] for c in PAIR_SHIFT])
@pytest.mark.parametrize("kernel", [0, 2])
def test_pair_rounds_with_shift_before(qf, name, make, dt, kernel):
    """Registers large enough that a tile spans several wavefronts: rounds that
    take U on a, the CSUM a+1 -> a+2 and U on a+1 read the CSUM's target from
    other lanes' sub-tiles (the round's loads all precede its stores)."""
    c = make()
    _, t = run_gpu(qf, c, dt, stage_kernel=kernel)
    assert maxabs(to_np(t), sim.run(c)) <= TOL[dt], name


TILES = [(3, 1), (3, 2), (4, 2), (5, 3), (2, 1)]


@pytest.mark.parametrize("tile,low", TILES)
@pytest.mark.parametrize("kernel,group", [(0, 0), (0, 1), (0, 2), (0, 9), (1, 0), (2, 0), (2, 1), (2, 9)])
def test_stage_tiles_small(qf, tile, low, kernel, group):
    """Small tiles force many passes, controls outside the tile and deferred gates;
    kernel 0 = register rounds (group 9 = the largest group compiled for D),
    1 = one LDS sweep per op.  The group sizes reach both builds of the round
    kernel (the 8-wave one for single-qudit groups of D = 5..11 in complex64,
    D = 3..5 in complex128, and D = 2 pairs)."""
    for c, dt in ((qi.config2(n=7, layers=3), "c64"), (qi.random_circuit(3, 6, 150, 21), "c128"),
                  (qi.config3(n=5, layers=2), "c64"), (qi.random_circuit(4, 5, 150, 22), "c64"),
                  (qi.random_circuit(2, 9, 200, 23), "c64"), (qi.random_circuit(7, 4, 100, 24), "c64"),
                  (qi.random_circuit(5, 4, 100, 25), "c128"), (qi.random_circuit(4, 4, 100, 26), "c128"),
                  (qi.random_circuit(2, 8, 150, 27), "c128")):
        gmax = {2: 5, 3: 3, 4: 2, 5: 2}.get(c.dim, 1)
        if kernel == 2:
            gmax = min(gmax, 3)
        p, t = run_gpu(qf, c, dt, tile_digits=min(tile, c.n), low_digits=low, stage_kernel=kernel,
                       group_digits=min(group, gmax))
        assert p.num_stages >= 1
        assert maxabs(to_np(t), sim.run(c)) <= TOL[dt], (c.name, tile, low)


def test_stage_batch_and_reuse(qf):
    """One plan applied to a batch of registers, twice with different angles."""
    c = qi.config2(n=6, layers=2)
    p = qf.plan_for(c, "c64")
    psi = qi.random_state(3, 6, 5, batch=3)
    for theta in (c.theta, -0.5 * c.theta):
        t = to_dev(psi.reshape(-1), "c64")
        p.forward(t, theta)
        got = to_np(t).reshape(3, -1)
        for b in range(3):
            assert maxabs(got[b], sim.run(c, psi[b], theta=theta)) <= 2e-5


def test_config1_outputs(qf):
    """D=3, n=4, complex128: state and basis probabilities within 1e-12."""
    c = qi.config1()
    _, t = run_gpu(qf, c, "c128")
    want = sim.run(c)
    assert maxabs(to_np(t), want) <= 1e-12
    p = to_np(qf.qf_probs(t, c.n, c.dim))
    assert maxabs(p, measure.probs(want)) <= 1e-12


def test_plan_batch_of_registers(qf):
    c = qi.config2(n=5, layers=2)
    psi = qi.random_state(3, 5, 2, batch=4)
    p = qf.plan_for(c, "c64")
    t = to_dev(psi.reshape(-1), "c64")
    p.forward(t, c.theta)
    got = to_np(t).reshape(4, -1)
    for b in range(4):
        assert maxabs(got[b], sim.run(c, psi[b])) <= 2e-5


ADJ = [
    ("random_d3_c128", lambda: qi.random_circuit(3, 4, 80, 11), "c128", 1e-9),
    ("random_d5_c128", lambda: qi.random_circuit(5, 3, 60, 12), "c128", 1e-9),
    ("config3_small", lambda: qi.config3(n=5, layers=2), "c64", 1e-4),
    ("config2_small", lambda: qi.config2(n=6, layers=2), "c64", 1e-4),
    ("config5_small", lambda: qi.config5(n=3, layers=2), "c64", 1e-4),
]


def _grad_close(g, ref, rel, dtype="c64"):
    """|g - ref| <= rel * max(|ref|, floor).  The floor covers entries whose exact
    value is (near) zero: with a complex64 state the per-amplitude rounding error
    (about 1e-6 after a few hundred gates) bounds the absolute gradient error at
    about 1e-2 * rel * max|ref|; complex128 keeps 1e-3."""
    floor = (1e-2 if dtype == "c64" else 1e-3) * np.abs(ref).max()
    return np.all(np.abs(g - ref) <= rel * np.maximum(np.abs(ref), floor))


@pytest.mark.parametrize("name,make,dt,rel", ADJ, ids=[a[0] for a in ADJ])
@pytest.mark.parametrize("fuse", [0, 2, 3])
def test_adjoint_matches_oracle_adjoint(qf, name, make, dt, rel, fuse):
    c = make()
    terms = qi.zsum_terms(c.n)
    p, t = run_gpu(qf, c, dt, fuse=fuse)
    lam = qf.new_state(c.n, c.dim, dt)
    g = p.adjoint_grad(t, lam, c.theta, terms)
    ref = grad.adjoint(c, terms)
    assert _grad_close(g, ref, rel, dt), (np.abs(g - ref).max(), np.abs(ref).max())


@pytest.mark.parametrize("tile,ckpt", [(3, 0), (4, 40), (0, 100), (3, 37)])
def test_adjoint_stage_tiles_and_checkpoints(qf, tile, ckpt):
    c = qi.config2(n=6, layers=3)
    terms = qi.zsum_terms(c.n)
    p, t = run_gpu(qf, c, "c64", adj_tile_digits=tile, ckpt_every=ckpt)
    lam = qf.new_state(c.n, c.dim, "c64")
    g = p.adjoint_grad(t, lam, c.theta, terms)
    ref = grad.adjoint(c, terms)
    assert _grad_close(g, ref, 1e-4, "c64"), (np.abs(g - ref).max(), np.abs(ref).max())


def test_adjoint_batch(qf):
    c = qi.config3(n=4, layers=2)
    terms = qi.zsum_terms(c.n)
    psi = qi.random_state(5, 4, 3, batch=2)
    p = qf.plan_for(c, "c128")
    t = to_dev(psi.reshape(-1), "c128")
    p.forward(t, c.theta)
    lam = qf.new_state(c.n, c.dim, "c128", batch=2)
    g = p.adjoint_grad(t, lam, c.theta, terms)
    for b in range(2):
        psi_f = sim.run(c, psi[b])
        ref = grad.adjoint(c, terms, psi_final=psi_f)
        assert _grad_close(g[b], ref, 1e-9, "c128")


def test_adjoint_vs_finite_differences(qf):
    """config-3 structure at n=5: GPU adjoint vs FP64 central differences
    (h = 1e-6) on 16 parameters, relative error <= 1e-4."""
    c = qi.config3(n=5, layers=2)
    terms = qi.zsum_terms(c.n)
    p, t = run_gpu(qf, c, "c64")
    lam = qf.new_state(c.n, c.dim, "c64")
    g = p.adjoint_grad(t, lam, c.theta, terms)
    idx = qi.config3_fd_params(c, 16)
    fd = grad.finite_diff(c, terms, idx, h=1e-6)
    assert _grad_close(g[idx], fd, 1e-4), np.abs(g[idx] - fd).max()


def test_pair_blocks_on_matrix_cores(qf):
    """Pair mode on D=10 (100 x 100 real blocks on the matrix cores) and D=7
    (49 x 49 complex blocks), against the oracle."""
    for c in (qi.config5(n=4, layers=3), qi.config5(n=5, layers=2), qi.random_circuit(7, 4, 120, 31)):
        p, t = run_gpu(qf, c, "c64", fuse=3)
        assert maxabs(to_np(t), sim.run(c)) <= 2e-5, c.name


def test_autotune_keeps_parity(qf):
    c = qi.config2(n=7, layers=3)
    p = qf.plan_for(c, "c64")
    scratch = qf.new_state(c.n, c.dim, "c64")
    qf.qf_state_init(scratch, c.n, c.dim, None)
    chosen = p.autotune(scratch, c.theta)
    assert chosen["fuse"] in (0, 2, 3)
    t = qf.new_state(c.n, c.dim, "c64")
    qf.qf_state_init(t, c.n, c.dim, None)
    p.forward(t, c.theta)
    assert maxabs(to_np(t), sim.run(c)) <= 2e-5
    lam = qf.new_state(c.n, c.dim, "c64")
    g = p.adjoint_grad(t, lam, c.theta, qi.zsum_terms(c.n))
    ref = grad.adjoint(c, qi.zsum_terms(c.n))
    assert _grad_close(g, ref, 1e-4, "c64")


@pytest.mark.parametrize("adjoint,bound", [(True, False), (True, True), (False, True)])
def test_autotune_flags_keep_parity(qf, adjoint, bound):
    """Tuning on forward + adjoint, and on device-parameter schedules only
    (timed bound to the batch): the rebuilt plan matches the oracle in both
    modes, and bound tuning chooses a stage plan."""
    import torch
    c = qi.config2(n=7, layers=2)
    terms = qi.zsum_terms(c.n)
    p = qf.plan_for(c, "c64")
    scratch = qf.new_state(c.n, c.dim, "c64", batch=3)
    qf.qf_state_init(scratch, c.n, c.dim, None)
    chosen = p.autotune(scratch, c.theta, adjoint=adjoint, bound=bound)
    if bound:
        assert chosen["fuse"] == 0
    want = sim.run(c)
    ref = grad.adjoint(c, terms)
    t = qf.new_state(c.n, c.dim, "c64")
    qf.qf_state_init(t, c.n, c.dim, None)
    p.forward(t, c.theta)
    assert maxabs(to_np(t), want) <= 2e-5
    lam = qf.new_state(c.n, c.dim, "c64")
    assert _grad_close(p.adjoint_grad(t, lam, c.theta, terms), ref, 1e-4, "c64")
    if bound:
        p.bind(3)
        th = torch.tensor(np.tile(c.theta, (3, 1)), dtype=torch.float64, device="cuda")
        psi = qf.new_state(c.n, c.dim, "c64", batch=3)
        lam = qf.new_state(c.n, c.dim, "c64", batch=3)
        g = torch.zeros((3, c.nparams), dtype=torch.float64, device="cuda")
        qf.qf_state_init(psi, c.n, c.dim, None)
        p.forward_dev(psi, th, c.nparams)
        p.adjoint_grad_dev(psi, lam, th, c.nparams, terms, g)
        for b in range(3):
            assert _grad_close(g.cpu().numpy()[b], ref, 1e-4, "c64")


def test_autotune_persistent_cache(qf, tmp_path, monkeypatch):
    """QF_TUNE_CACHE: the first tuning appends its choice to the file; after the
    in-memory cache is dropped, a new plan of the same circuit takes the choice
    from the file without timing again."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("QF_TUNE_CACHE", str(path))
    qf.qf_shutdown()
    c = qi.config2(n=6, layers=2)
    t = qf.new_state(c.n, c.dim, "c64")
    qf.qf_state_init(t, c.n, c.dim, None)
    first = qf.plan_for(c, "c64").autotune(t, c.theta, adjoint=True)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and len(lines[0].split()) == 11
    qf.qf_shutdown()
    again = qf.plan_for(c, "c64").autotune(t, c.theta, adjoint=True)
    assert again == first
    assert len(path.read_text().splitlines()) == 1
    monkeypatch.delenv("QF_TUNE_CACHE")
    qf.qf_shutdown()


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("kernel", [0, 1, 2])
def test_tile_order(qf, order, kernel):
    """Both tile orders (per-XCD ranges, plain dispatch order), short runs, a
    batch of registers: forward and adjoint against the oracle."""
    c = qi.config2(n=8, layers=3)
    psi0 = qi.random_state(3, 8, 31, batch=3)
    p = qf.plan_for(c, "c64", tile_digits=4, low_digits=1, stage_kernel=kernel, tile_order=order,
                    adj_tile_digits=4)
    t = to_dev(psi0.reshape(-1), "c64")
    p.forward(t, c.theta)
    got = to_np(t).reshape(3, -1)
    for b in range(3):
        assert maxabs(got[b], sim.run(c, psi0[b])) <= 2e-5
    terms = qi.zsum_terms(c.n)
    p1 = qf.plan_for(c, "c64", tile_digits=4, low_digits=1, stage_kernel=kernel, tile_order=order,
                     adj_tile_digits=4)
    psi = qf.new_state(c.n, c.dim, "c64")
    qf.qf_state_init(psi, c.n, c.dim, None)
    p1.forward(psi, c.theta)
    lam = qf.new_state(c.n, c.dim, "c64")
    g = p1.adjoint_grad(psi, lam, c.theta, terms)
    gref = grad.adjoint(c, terms)
    assert _grad_close(g, gref, 1e-4, "c64"), np.abs(g - gref).max()


@pytest.mark.parametrize("search", [1, 2])
def test_tile_search(qf, search):
    """Greedy tiles and swap-improved tiles (forced at this small size): forward
    and adjoint against the oracle, with tiles small enough that the two
    choices give different pass lists."""
    c = qi.config2(n=8, layers=3)
    p = qf.plan_for(c, "c64", tile_digits=4, low_digits=1, adj_tile_digits=4, tile_search=search)
    t = qf.new_state(c.n, c.dim, "c64")
    qf.qf_state_init(t, c.n, c.dim, None)
    p.forward(t, c.theta)
    assert maxabs(to_np(t), sim.run(c)) <= 2e-5
    terms = qi.zsum_terms(c.n)
    lam = qf.new_state(c.n, c.dim, "c64")
    g = p.adjoint_grad(t, lam, c.theta, terms)
    gref = grad.adjoint(c, terms)
    assert _grad_close(g, gref, 1e-4, "c64"), np.abs(g - gref).max()


@pytest.mark.parametrize("make", [lambda: qi.config2(n=10, layers=3), lambda: qi.config3(n=7, layers=2)],
                         ids=["config2_n10", "config3_n7"])
def test_default_tile_shapes_against_oracle(qf, make):
    """Registers large enough that the default plans use the full-size tile
    shapes (D=3: 7-qudit tiles with 2 low qudits and outer digits; D=5: 5-qudit
    forward and 4-qudit adjoint tiles with outer digits): forward state and
    adjoint gradient against the oracle."""
    c = make()
    terms = qi.zsum_terms(c.n)
    p, t = run_gpu(qf, c, "c64")
    want = sim.run(c)
    assert maxabs(to_np(t), want) <= 2e-5
    lam = qf.new_state(c.n, c.dim, "c64")
    g = p.adjoint_grad(t, lam, c.theta, terms)
    ref = grad.adjoint(c, terms, psi_final=want)
    assert _grad_close(g, ref, 1e-4, "c64"), np.abs(g - ref).max()


@pytest.mark.parametrize("fuse", [0, 1, 2, 3])
def test_single_qudit_register(qf, fuse):
    """n = 1: forward and adjoint of every schedule against the oracle."""
    c = qi.Circuit(5, 1, [("h", 0), ("rx", 0, 0, 3, 0), ("clock", 0, 2), ("ry", 0, 1, 4, 1), ("rz", 0, 3, 2),
                          ("x", 0, 3)], np.array([0.3, -1.1, 2.2]))
    terms = qi.zsum_terms(1)
    p, t = run_gpu(qf, c, "c128", fuse=fuse)
    assert maxabs(to_np(t), sim.run(c)) <= 1e-12
    lam = qf.new_state(1, 5, "c128")
    g = p.adjoint_grad(t, lam, c.theta, terms)
    assert _grad_close(g, grad.adjoint(c, terms), 1e-9, "c128")
