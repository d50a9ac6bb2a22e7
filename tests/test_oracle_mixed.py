"""Pins of the mixed-dimension oracle (oracle.mixed) against what the paper and
the mathematics fix: the paper's own dim=[2, 3, 4] example in closed form,
Kronecker-product operators, permutations built digit by digit with numpy's
row-major multi-index, textbook identities across dimensions, brute-force
marginals, the uniform-register oracle as the special case of equal
dimensions, and finite differences for the gradient."""
import itertools

import numpy as np
import pytest
import scipy.linalg

import qf_inputs as qi
from oracle import gates, measure, mixed, sim


def _w(d):
    return np.exp(2j * np.pi / d)


def test_paper_example_closed_form():
    """Section "Code style" example.  By hand: Fourier on |0> and R_x(pi/2)
    give qudit 0 the amplitudes (1 - i)/2 on both levels; Fourier on |1> gives
    w_3^y / sqrt 3; Fourier on |3> gives w_4^(3 z) / 2; the CNOT moves
    z -> z + x_0 mod 4.  The measured pair (qudits 0, 1) is uniform, 1/6."""
    ex = qi.paper_mixed_example()
    c = ex["circuit"]
    psi = mixed.run(c, digits=ex["digits"])
    want = np.zeros(24, dtype=np.complex128)
    for x0, x1, x2 in itertools.product(range(2), range(3), range(4)):
        z = (x2 - x0) % 4
        want[np.ravel_multi_index((x0, x1, x2), (2, 3, 4))] = (1 - 1j) / 2 * _w(3) ** x1 / np.sqrt(3) * \
            _w(4) ** (3 * z) / 2
    assert np.allclose(psi, want, atol=1e-15)
    p = mixed.marginal(psi, c.dims, ex["measured"])
    assert np.allclose(p, np.full(6, 1 / 6), atol=1e-15)
    # the histogram of its 1000 shots: chi-square against the uniform 1/6
    counts = measure.sample_counts(p, qi.uniforms(ex["shots"], 3))
    chi2 = float(np.sum((counts - 1000 / 6) ** 2 / (1000 / 6)))
    assert counts.sum() == 1000 and chi2 < 20.5  # 5 degrees of freedom, p = 0.001


@pytest.mark.parametrize("dims", [[2, 3, 4], [3, 2, 5, 2], [4, 1 + 1, 3]])
def test_one_qudit_gate_is_the_kronecker_product(dims):
    rng = np.random.default_rng(len(dims))
    psi = rng.standard_normal(int(np.prod(dims))) + 1j * rng.standard_normal(int(np.prod(dims)))
    for q, d in enumerate(dims):
        U = qi.random_unitary(d, rng)
        full = np.kron(np.kron(np.eye(int(np.prod(dims[:q]))), U), np.eye(int(np.prod(dims[q + 1:]))))
        assert np.allclose(mixed.apply_1q(psi, dims, q, U), full @ psi, atol=1e-13)
    if len(dims) >= 2:
        B = qi.random_unitary(dims[0] * dims[1], rng)
        full = np.kron(B, np.eye(int(np.prod(dims[2:]))))
        assert np.allclose(mixed.apply_block(psi, dims, 0, 2, B), full @ psi, atol=1e-13)


def _perm_matrix(dims, rule):
    """Permutation operator from a rule on digit tuples, indices by numpy's
    row-major multi-index."""
    N = int(np.prod(dims))
    P = np.zeros((N, N))
    for dig in itertools.product(*[range(d) for d in dims]):
        P[np.ravel_multi_index(rule(list(dig)), dims), np.ravel_multi_index(dig, dims)] = 1
    return P


@pytest.mark.parametrize("dims", [[2, 3, 4], [4, 3, 2], [3, 5, 2, 2]])
def test_permutations_digit_by_digit(dims):
    rng = np.random.default_rng(sum(dims))
    N = int(np.prod(dims))
    psi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    n = len(dims)
    for c, t in itertools.permutations(range(n), 2):
        def csum(d, c=c, t=t):
            d[t] = (d[t] + d[c]) % dims[t]
            return d
        assert np.array_equal(mixed.apply_op(psi, dims, ("csum", c, t), None), _perm_matrix(dims, csum) @ psi)
        sh = tuple(int(v) for v in rng.integers(0, dims[t], size=dims[c]))

        def cshift(d, c=c, t=t, sh=sh):
            d[t] = (d[t] + sh[d[c]]) % dims[t]
            return d
        assert np.array_equal(mixed.apply_op(psi, dims, ("cshift", c, t, sh), None),
                              _perm_matrix(dims, cshift) @ psi)
    ctrls, t = (0, 1), n - 1

    def mcx(d):
        d[t] = (d[t] + d[0] * d[1]) % dims[t]
        return d
    assert np.array_equal(mixed.apply_op(psi, dims, ("mcx", ctrls, t), None), _perm_matrix(dims, mcx) @ psi)
    same = [(a, b) for a, b in itertools.combinations(range(n), 2) if dims[a] == dims[b]]
    for a, b in same:
        def swap(d, a=a, b=b):
            d[a], d[b] = d[b], d[a]
            return d
        assert np.array_equal(mixed.apply_op(psi, dims, ("swap", a, b), None), _perm_matrix(dims, swap) @ psi)


def test_swap_needs_equal_dimensions():
    with pytest.raises(ValueError):
        mixed.apply_op(np.ones(6), [2, 3], ("swap", 0, 1), None)


@pytest.mark.parametrize("dims,c,t", [([2, 3, 4], 0, 2), ([2, 3, 4], 2, 1), ([5, 3], 0, 1), ([3, 5], 1, 0)])
def test_fourier_conjugates_csum_into_cz(dims, c, t):
    """F_t^dagger X_t^m F_t = Z_t^(-m) in the target's dimension, so Fourier on
    t, CSUM c -> t, inverse Fourier on t is the inverse CZ: the CSUM and CZ
    readings across dimensions agree."""
    rng = np.random.default_rng(7)
    N = int(np.prod(dims))
    psi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    F = gates.fourier(dims[t])
    x = mixed.apply_1q(psi, dims, t, F)
    x = mixed.apply_op(x, dims, ("csum", c, t), None)
    x = mixed.apply_1q(x, dims, t, F.conj().T)
    assert np.allclose(x, mixed.apply_op(psi, dims, ("cz_inv", c, t), None), atol=1e-13)
    dig = np.array(list(itertools.product(*[range(d) for d in dims])))
    ph = _w(dims[t]) ** (dig[:, c] * dig[:, t])
    assert np.allclose(mixed.apply_op(psi, dims, ("cz", c, t), None), ph * psi, atol=1e-14)


@pytest.mark.parametrize("dims,c,t,op", [([2, 4], 0, 1, ("cry", 0, 1, 1, 3, 0)), ([3, 2, 4], 0, 2, ("crx", 0, 2, 0, 2, 0)),
                                         ([4, 3], 1, 0, ("crz", 1, 0, 3, 0)), ([2, 5, 3], 2, 1, ("crz", 2, 1, 2, 0))])
def test_controlled_rotation_block_diagonal(dims, c, t, op):
    """sum_m |m><m|_c (x) expm(-i m theta S / 2)_t built entry by entry with
    scipy's matrix exponential; a qubit control gives the textbook controlled
    rotation diag(I, R(theta))."""
    theta = np.array([0.83])
    S = gates.crot_generator(op, dims[t])
    N = int(np.prod(dims))
    M = np.zeros((N, N), dtype=np.complex128)
    for din in itertools.product(*[range(d) for d in dims]):
        R = scipy.linalg.expm(-0.5j * din[c] * theta[0] * S)
        for a in range(dims[t]):
            dout = list(din)
            dout[t] = a
            M[np.ravel_multi_index(dout, dims), np.ravel_multi_index(din, dims)] += R[a, din[t]]
    rng = np.random.default_rng(8)
    psi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    assert np.allclose(mixed.apply_op(psi, dims, op, theta), M @ psi, atol=1e-13)


def test_marginal_and_expectation_brute_force():
    dims = [3, 2, 4, 2]
    rng = np.random.default_rng(9)
    N = int(np.prod(dims))
    psi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    psi /= np.linalg.norm(psi)
    for qs in ([2], [3, 0], [1, 2, 0], [0, 1, 2, 3], [3, 2, 1, 0]):
        want = np.zeros(int(np.prod([dims[q] for q in qs])))
        for dig in itertools.product(*[range(d) for d in dims]):
            y = np.ravel_multi_index([dig[q] for q in qs], [dims[q] for q in qs])
            want[y] += abs(psi[np.ravel_multi_index(dig, dims)]) ** 2
        assert np.allclose(mixed.marginal(psi, dims, qs), want, atol=1e-15)
    terms = [(0, "z"), (2, "z"), (3, rng.standard_normal(2) + 1j * rng.standard_normal(2))]
    want = 0j
    for dig in itertools.product(*[range(d) for d in dims]):
        f = _w(3) ** dig[0] + _w(4) ** dig[2] + terms[2][1][dig[3]]
        want += abs(psi[np.ravel_multi_index(dig, dims)]) ** 2 * f
    assert abs(mixed.expect_diag(psi, dims, terms) - want) < 1e-14


def test_equal_dimensions_reduce_to_the_uniform_oracle():
    for D, n, seed in ((3, 4, 1), (2, 5, 2), (5, 3, 3)):
        c = qi.random_circuit(D, n, 60, seed, kinds=["h", "x", "clock", "rx", "ry", "rz", "csum", "cz", "cshift",
                                                     "u1", "u2", "crx", "cry", "crz", "swap", "mcx"])
        m = qi.MixedCircuit([D] * n, c.ops, c.theta)
        assert np.allclose(mixed.run(m), sim.run(c), atol=1e-13)


def test_adjoint_gradient_matches_finite_differences():
    c = qi.random_mixed_circuit([2, 3, 4, 3], 50, 4)
    terms = [(q, "z") for q in range(c.n)]
    g = mixed.adjoint(c, terms)
    fd = mixed.finite_diff(c, terms, list(range(c.nparams)))
    assert c.nparams > 5
    assert np.allclose(g, fd, atol=1e-7)


def test_adjoint_on_the_mixed_ansatz():
    c = qi.mixed_hea([2, 3, 4, 5], 2, 5)
    terms = [(q, "z") for q in range(c.n)]
    assert np.allclose(mixed.adjoint(c, terms), mixed.finite_diff(c, terms, list(range(c.nparams))), atol=1e-7)
