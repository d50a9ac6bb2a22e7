"""GPU parity of the per-gate entry points against the FP64 oracle.

Tolerances: max |d amplitude| <= 2e-5 (complex64) and <= 1e-12 (complex128);
permutations are compared bit for bit.  Sizes span several workgroups and a
ragged tail on every axis (both the coalesced-column and the LDS-row paths)."""
import numpy as np
import pytest

import qf_inputs as qi
from oracle import gates, measure, sim
from tests.gpu_helpers import TOL, maxabs, rounded, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qf():
    import paper_2409_17716_amd as qf
    return qf


AXIS_CASES = [(2, 13, "c64"), (3, 9, "c64"), (3, 8, "c128"), (4, 6, "c64"), (5, 5, "c128"), (5, 6, "c64"),
              (7, 4, "c64"), (10, 4, "c64"), (10, 3, "c128"), (11, 3, "c128"), (16, 3, "c64"), (6, 4, "c64")]


@pytest.mark.parametrize("D,n,dt", AXIS_CASES)
def test_apply_1q_every_axis(qf, D, n, dt):
    rng = np.random.default_rng(D * 100 + n)
    for batch in (1, 2):
        psi = qi.random_state(D, n, int(rng.integers(1 << 30)), batch=batch).reshape(-1)
        for q in range(n):
            U = qi.random_unitary(D, rng)
            t = to_dev(psi, dt)
            qf.qf_apply_1q(t, n, D, q, U)
            want = np.concatenate([sim.apply_1q(r, D, n, q, U) for r in rounded(psi, dt).reshape(batch, -1)])
            assert maxabs(to_np(t), want) <= TOL[dt], (D, n, q, batch)


@pytest.mark.parametrize("D,n,dt", [(3, 7, "c64"), (5, 4, "c128"), (2, 11, "c64"), (10, 3, "c64"), (4, 5, "c128")])
def test_apply_ctrl_bit_exact(qf, D, n, dt):
    rng = np.random.default_rng(7 + D)
    psi = rounded(qi.random_state(D, n, 3), dt)
    for c in list(range(n)) + [-1]:
        for tg in range(n):
            if c == tg:
                continue
            shifts = list(range(D)) if rng.random() < 0.5 else [int(v) for v in rng.integers(-D, 2 * D, size=D)]
            t = to_dev(psi, dt)
            qf.qf_apply_ctrl(t, n, D, c, tg, shifts)
            want = sim.apply_cshift(psi, D, n, c, tg, shifts)
            assert np.array_equal(to_np(t), want), (c, tg, shifts)


@pytest.mark.parametrize("D,n", [(3, 6), (5, 4), (2, 9)])
def test_csum_and_shift_on_basis_states(qf, D, n):
    """Permutations acting on basis states give the exact basis state."""
    rng = np.random.default_rng(D)
    for _ in range(6):
        digits = [int(v) for v in rng.integers(0, D, size=n)]
        c, tg = [int(v) for v in rng.choice(n, size=2, replace=False)]
        t = to_dev(np.zeros(D ** n), "c64")
        qf.qf_state_init(t, n, D, digits)
        qf.qf_apply_ctrl(t, n, D, c, tg, list(range(D)))
        qf.qf_apply_ctrl(t, n, D, -1, c, [1])
        want = list(digits)
        want[tg] = (want[tg] + want[c]) % D
        want[c] = (want[c] + 1) % D
        assert np.array_equal(to_np(t), sim.basis_state(D, n, want))


def test_state_init_batch(qf):
    D, n = 3, 4
    digs = np.array([[0, 1, 2, 0], [2, 2, 2, 2], [1, 0, 0, 1]])
    t = to_dev(np.zeros(3 * D ** n), "c128")
    qf.qf_state_init(t, n, D, digs)
    want = np.concatenate([sim.basis_state(D, n, d) for d in digs])
    assert np.array_equal(to_np(t), want)
    qf.qf_state_init(t, n, D, None)
    assert np.array_equal(to_np(t), np.concatenate([sim.basis_state(D, n)] * 3))


@pytest.mark.parametrize("D,n,dt", [(3, 8, "c64"), (5, 4, "c128"), (4, 6, "c64")])
def test_apply_diag(qf, D, n, dt):
    rng = np.random.default_rng(D)
    psi = qi.random_state(D, n, 5)
    w = gates.omega(D)
    for k in (1, 2, 3):
        qs = [int(v) for v in rng.choice(n, size=k, replace=False)]
        ph = np.exp(1j * rng.uniform(-np.pi, np.pi, size=D ** k))
        t = to_dev(psi, dt)
        qf.qf_apply_diag(t, n, D, qs, ph)
        dig = sim.digits_of(D, n, np.arange(D ** n))
        y = np.zeros(D ** n, dtype=np.int64)
        for q in qs:
            y = y * D + dig[q]
        want = rounded(psi, dt) * ph[y]
        assert maxabs(to_np(t), want) <= TOL[dt]
    # CZ table
    c, tg = 0, n - 1
    tab = np.array([w ** ((a * b) % D) for a in range(D) for b in range(D)])
    t = to_dev(psi, dt)
    qf.qf_apply_diag(t, n, D, [c, tg], tab)
    assert maxabs(to_np(t), sim.apply_cz(rounded(psi, dt), D, n, c, tg)) <= TOL[dt]


@pytest.mark.parametrize("D,n,k,dt", [(3, 6, 2, "c64"), (3, 5, 3, "c64"), (4, 5, 2, "c128"), (10, 4, 2, "c64"),
                                      (2, 10, 5, "c64"), (5, 3, 2, "c128")])
def test_apply_fused(qf, D, n, k, dt):
    import torch
    rng = np.random.default_rng(D * 10 + k)
    psi = qi.random_state(D, n, 9)
    for q0 in range(n - k + 1):
        B = qi.random_unitary(D ** k, rng)
        Bt = to_dev(B.reshape(-1), dt).reshape(D ** k, D ** k)
        t = to_dev(psi, dt)
        qf.qf_apply_fused(t, n, D, q0, k, Bt)
        want = sim.apply_matrix(rounded(psi, dt), D, n, list(range(q0, q0 + k)), B.astype(
            np.complex64 if dt == "c64" else np.complex128).astype(np.complex128))
        tol = TOL[dt] if dt == "c128" else 2e-5
        assert maxabs(to_np(t), want) <= tol, (q0,)


@pytest.mark.parametrize("D,n,k", [(2, 8, 5), (4, 5, 3), (3, 6, 4), (10, 4, 2), (5, 4, 3), (2, 9, 8), (10, 3, 2)])
def test_apply_fused_matrix_cores(qf, D, n, k):
    """complex64 blocks with D^k >= 32 run on the FP32 matrix cores (v_mfma_f32_16x16x4f32,
    rows padded to a multiple of 16); every admissible position, so both the
    L = 1 (contiguous fibres) and the strided staging paths are covered."""
    rng = np.random.default_rng(100 * D + k)
    psi = qi.random_state(D, n, 17, batch=2).reshape(-1)
    K = D ** k
    for q0 in range(n - k + 1):
        B = qi.random_unitary(K, rng)
        Bt = to_dev(B.reshape(-1), "c64").reshape(K, K)
        t = to_dev(psi, "c64")
        qf.qf_apply_fused(t, n, D, q0, k, Bt)
        Bq = B.astype(np.complex64).astype(np.complex128)
        want = np.concatenate([sim.apply_matrix(r, D, n, list(range(q0, q0 + k)), Bq)
                               for r in rounded(psi, "c64").reshape(2, -1)])
        assert maxabs(to_np(t), want) <= 2e-5, (q0, maxabs(to_np(t), want))


def test_grover_fused_block(qf):
    """One Grover iteration on two qutrits via two custom 9x9 blocks: marked
    amplitude 23/27, the others 5/27."""
    D, n = 3, 2
    s = np.full(9, 1 / 3, dtype=np.complex128)
    m = sim.basis_state(D, n, [2, 2])
    oracle_u = np.eye(9) - 2 * np.outer(m, m)
    diffusion = 2 * np.outer(s, s) - np.eye(9)
    for dt in ("c64", "c128"):
        t = to_dev(np.zeros(9), dt)
        qf.qf_state_init(t, n, D, None)
        H = gates.fourier(D)
        qf.qf_apply_1q(t, n, D, 0, H)
        qf.qf_apply_1q(t, n, D, 1, H)
        for U in (oracle_u, diffusion):
            qf.qf_apply_fused(t, n, D, 0, 2, to_dev(U.reshape(-1), dt).reshape(9, 9))
        want = np.full(9, 5 / 27)
        want[8] = 23 / 27
        assert maxabs(to_np(t), want) <= (1e-6 if dt == "c64" else 1e-14)


@pytest.mark.parametrize("D,n,dt", [(3, 7, "c64"), (5, 4, "c128"), (2, 12, "c64")])
def test_probs(qf, D, n, dt):
    batch = 2
    psi = qi.random_state(D, n, 4, batch=batch).reshape(-1)
    t = to_dev(psi, dt)
    ref = [rounded(r, dt) for r in psi.reshape(batch, -1)]
    p = to_np(qf.qf_probs(t, n, D))
    assert maxabs(p, np.concatenate([measure.probs(r) for r in ref])) <= (1e-6 if dt == "c64" else 1e-15)
    for qs in ([0], [n - 1], [1, 0], [n - 1, 0], list(range(n)), [2, n - 1, 0], [n - 2, 1]):
        pm = to_np(qf.qf_probs(t, n, D, qs))
        want = np.concatenate([measure.marginal(r, D, n, qs) for r in ref])
        assert maxabs(pm, want) <= (2e-6 if dt == "c64" else 1e-13), qs


@pytest.mark.parametrize("D,n,dt", [(3, 8, "c64"), (5, 5, "c128"), (10, 3, "c64")])
def test_expect(qf, D, n, dt):
    batch = 3
    psi = qi.random_state(D, n, 8, batch=batch).reshape(-1)
    t = to_dev(psi, dt)
    ref = [rounded(r, dt) for r in psi.reshape(batch, -1)]
    for terms in (qi.z0_terms(), qi.zsum_terms(n), [(n - 1, "z"), (1, "z"), (n - 1, "z")]):
        out = to_np(qf.qf_expect(t, n, D, terms)).reshape(batch, 2)
        for b in range(batch):
            want = measure.expect_diag(ref[b], D, n, terms)
            assert abs(complex(out[b, 0], out[b, 1]) - want) <= 1e-12


def test_expect_and_probs_are_bitwise_reproducible(qf):
    D, n = 3, 10
    t = to_dev(qi.random_state(D, n, 1), "c64")
    a = to_np(qf.qf_expect(t, n, D, qi.zsum_terms(n)))
    b = to_np(qf.qf_expect(t, n, D, qi.zsum_terms(n)))
    assert np.array_equal(a, b)
    pa = to_np(qf.qf_probs(t, n, D, [3, 1]))
    pb = to_np(qf.qf_probs(t, n, D, [3, 1]))
    assert np.array_equal(pa, pb)
