"""GPU measurement shots against the FP64 oracle, draw for draw on the same
uniforms: full registers and marginals (any order), several prefix-sum levels
and registers per launch, empty bins, the draws at the ends of [0, 1), zero
shots and a zero state."""
import numpy as np
import pytest

import qf_inputs as qi
from oracle import measure
from tests.gpu_helpers import rounded, to_dev

pytestmark = pytest.mark.gpu

# The GPU's prefix sum adds in another order than the oracle's running sum, so
# a draw whose u * total lies within both sums' rounding errors of a cumulative
# boundary may fall on either side.  The margin is measured: the oracle's
# deviation from an extended-precision running sum, plus a bound for the GPU's
# (per scan level a value passes through at most 4 additions in its thread, 6
# lane-shift steps, 3 wavefront totals and 1 block offset; three levels and
# the search's offset, each addition adding at most 2^-53 of the total).
GPU_ADDS = 48


@pytest.fixture(scope="module")
def qf():
    import paper_2409_17716_amd as qf
    return qf


def _oracle(psi_rows, D, n, qudits, u_rows):
    """Per register: the oracle's outcomes, the draws within rounding reach of a
    boundary, and a validity check for the GPU's outcome on those draws."""
    out = []
    for psi, u in zip(psi_rows, u_rows):
        p = measure.probs(psi) if qudits is None else measure.marginal(psi, D, n, qudits)
        c = np.cumsum(p)
        cx = np.cumsum(p.astype(np.longdouble))
        tot = float(cx[-1])
        delta = 2 * (float(np.max(np.abs(c - cx))) + GPU_ADDS * 2.0 ** -53 * tot)
        x = u * tot
        k = np.searchsorted(cx, x)
        d_up = np.abs(cx[np.minimum(k, len(c) - 1)] - x).astype(np.float64)
        d_dn = np.abs(cx[np.maximum(k - 1, 0)] - x).astype(np.float64)
        near = np.minimum(d_up, d_dn) <= delta

        def valid(g, xs, p=p, cx=cx, delta=delta):
            lo = np.where(g > 0, cx[np.maximum(g - 1, 0)], 0.0).astype(np.float64)
            return (p[g] > 0) & (lo - delta <= xs) & (xs <= cx[g].astype(np.float64) + delta)
        out.append((measure.sample_inverse_cdf(p, u), near, valid, x))
    return out


def _check(qf, psi, D, n, dt, qudits, shots, seed, batch):
    import torch
    t = to_dev(psi.reshape(-1), dt)
    u = qi.uniforms(batch * shots, seed)
    u[:2] = [0.0, np.nextafter(1.0, 0.0)]
    ud = torch.from_numpy(u).cuda()
    counts, samples = qf.qf_sample(t, n, D, shots, ud, qudits=qudits, samples=True)
    counts2 = qf.qf_sample(t, n, D, shots, ud, qudits=qudits)
    torch.cuda.synchronize()
    counts, samples, counts2 = counts.cpu().numpy(), samples.cpu().numpy(), counts2.cpu().numpy()
    K = D ** (n if qudits is None else len(qudits))
    rows = rounded(psi, dt).reshape(batch, -1)
    ref = _oracle(rows, D, n, qudits, u.reshape(batch, shots))
    for b, (want, near, valid, x) in enumerate(ref):
        got = samples[b * shots:(b + 1) * shots].astype(np.int64)
        ok = ~near
        assert near.sum() <= max(5, shots // 1000), near.sum()
        assert np.array_equal(got[ok], want[ok]), (b, np.flatnonzero(got[ok] != want[ok])[:5])
        # draws on a boundary: any outcome whose interval reaches the draw
        assert np.all(valid(got[near], x[near]))
        assert np.array_equal(counts[b * K:(b + 1) * K], np.bincount(got, minlength=K))
    assert np.array_equal(counts, counts2)
    return samples, ref[0][0]


# 3^13 and 3^11 hold more than 4096 outcomes (block-local sums searched by
# levels); their last 1024-element scan blocks hold 979 and 1019 elements, so
# the last 32-element sub-block is short (19 and 27 elements)
@pytest.mark.parametrize("D,n,dt,batch", [(3, 7, "c64", 2), (2, 12, "c128", 1), (5, 5, "c128", 3),
                                          (3, 13, "c64", 2), (3, 11, "c128", 3)])
def test_full_register(qf, D, n, dt, batch):
    """3^13 * 2 outcomes take three prefix-sum levels over two registers."""
    psi = qi.random_state(D, n, 11, batch=batch)
    _check(qf, psi, D, n, dt, None, 20000, 5, batch)


@pytest.mark.parametrize("D,n,dt,qudits", [(3, 8, "c64", [5]), (3, 8, "c128", [6, 1, 3]),
                                           (5, 5, "c64", [4, 0]), (4, 6, "c128", [0, 1, 2, 3, 4, 5]),
                                           (2, 14, "c64", [13, 0, 7, 2, 9])])
def test_marginals(qf, D, n, dt, qudits):
    psi = qi.random_state(D, n, 12, batch=2)
    _check(qf, psi, D, n, dt, qudits, 30000, 6, 2)


def test_empty_bins_and_ends(qf):
    """A state with most outcomes of zero probability: no draw lands on one,
    u = 0 gives the first non-empty outcome and u just below 1 the last one."""
    D, n = 3, 9
    psi = qi.sparse_state(D, n, 13, keep=0.05)
    samples, want = _check(qf, psi, D, n, "c128", None, 50000, 7, 1)
    p = measure.probs(psi)
    nz = np.flatnonzero(p)
    assert np.all(p[samples] > 0)
    assert samples[0] == nz[0] and samples[1] == nz[-1]


def test_zero_shots_and_zero_state(qf):
    import torch
    D, n = 3, 6
    t = to_dev(qi.random_state(D, n, 14), "c64")
    c = qf.qf_sample(t, n, D, 0, None)
    assert int(c.abs().sum().item()) == 0 and c.numel() == D ** n
    z = torch.zeros(2 * D ** n, dtype=torch.complex128, device="cuda")
    u = torch.from_numpy(qi.uniforms(2 * 100, 8)).cuda()
    c, s = qf.qf_sample(z, n, D, 100, u, qudits=[2, 4], samples=True)
    c = c.cpu().numpy().reshape(2, -1)
    assert np.all(c[:, 0] == 100) and c[:, 1:].sum() == 0 and int(s.abs().sum().item()) == 0


def test_draws_that_reach_the_total(qf):
    """A register whose probabilities are subnormal (amplitudes ~2e-162 in
    complex128): u just below 1 rounds up to the total and goes to the last
    outcome of non-zero probability, as does u = 1; the oracle agrees."""
    import torch
    D, n = 3, 3
    psi = np.zeros(D ** n, dtype=np.complex128)
    psi[[4, 11]] = 2.3e-162
    t = to_dev(psi, "c128")
    top = np.nextafter(1.0, 0.0)
    u = np.array([0.0, 0.3, top, 1.0])
    c, smp = qf.qf_sample(t, n, D, len(u), torch.from_numpy(u).cuda(), samples=True)
    got = smp.cpu().numpy()
    want = measure.sample_inverse_cdf(measure.probs(psi), u)
    assert list(got) == list(want)
    assert got[0] == 4 and got[2] == 11 and got[3] == 11  # never a trailing empty outcome


def test_draws_that_reach_the_total_many_outcomes(qf):
    """The same rule with 3^9 outcomes (the search over scan-block ends, then
    inside one block) and the non-zero outcomes in different scan blocks."""
    import torch
    D, n = 3, 9
    psi = np.zeros(D ** n, dtype=np.complex128)
    psi[[4, 5000, 15000]] = 2.3e-162
    t = to_dev(psi, "c128")
    top = np.nextafter(1.0, 0.0)
    u = np.array([0.0, 0.3, 0.6, top, 1.0])
    c, smp = qf.qf_sample(t, n, D, len(u), torch.from_numpy(u).cuda(), samples=True)
    got = smp.cpu().numpy()
    want = measure.sample_inverse_cdf(measure.probs(psi), u)
    assert list(got) == list(want)
    assert got[0] == 4 and got[3] == 15000 and got[4] == 15000


def test_full_size_marginal_and_register(qf):
    """The 3^16 register in complex64: 10^5 shots of the full distribution and
    of a two-qudit marginal."""
    D, n = 3, 16
    psi = qi.random_state(D, n, 15)
    _check(qf, psi, D, n, "c64", None, 100000, 9, 1)
    _check(qf, psi, D, n, "c64", [15, 0], 100000, 10, 1)
