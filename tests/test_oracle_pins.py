"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics:
printed matrices, closed forms, invariants, textbook special cases and a
brute-force second route.  CPU only."""
import json
import os

import numpy as np
import pytest

import qf_inputs as qi
from oracle import brute, gates, grad, measure, sim

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-12


def _eval_entry(expr, theta):
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    env = {"c": c, "s": s, "i": 1j, "em": np.exp(-0.5j * theta), "ep": np.exp(0.5j * theta)}
    return complex(eval(expr, {"__builtins__": {}}, env))


def _eval_matrix(rows, theta=0.0):
    return np.array([[_eval_entry(e, theta) for e in r] for r in rows])


# ---------------------------------------------------------------- gate matrices

def test_printed_rotation_matrices():
    """The paper's printed D=2, D=3 and D=4 rotation matrices."""
    fx = json.load(open(os.path.join(GOLDEN, "paper_rotation_matrices.json")))
    for case in fx["cases"]:
        for theta in (0.3, -1.7, 2.9, np.pi):
            if case["gate"] == "rz":
                got = gates.rz(case["D"], case["j"], theta)
            else:
                got = getattr(gates, case["gate"])(case["D"], case["j"], case["k"], theta)
            want = _eval_matrix(case["matrix"], theta)
            assert np.abs(got - want).max() < TOL, case["name"]
    g = fx["generators_D2"]
    assert np.allclose(gates.gm_sym(2, 0, 1), _eval_matrix(g["sx"]))
    assert np.allclose(gates.gm_asym(2, 0, 1), _eval_matrix(g["sy"]))
    assert np.allclose(gates.gm_diag(2, 1), _eval_matrix(g["sz"]))


@pytest.mark.parametrize("D", range(2, 11))
def test_rotation_closed_forms(D):
    """The paper's general element formulas for R_x^{jk}, R_y^{jk} (two-level
    rotation, identity elsewhere) and R_z^j (diagonal phases) versus the oracle's
    eigendecomposition route."""
    rng = np.random.default_rng(D)
    for theta in rng.uniform(-np.pi, np.pi, size=3):
        c, s = np.cos(theta / 2), np.sin(theta / 2)
        for j in range(D):
            for k in range(j + 1, D):
                ex = np.eye(D, dtype=complex)
                ex[j, j] = ex[k, k] = c
                ex[j, k] = ex[k, j] = -1j * s
                assert np.abs(gates.rx(D, j, k, theta) - ex).max() < TOL
                ey = np.eye(D, dtype=complex)
                ey[j, j] = ey[k, k] = c
                ey[j, k] = -s
                ey[k, j] = s
                assert np.abs(gates.ry(D, j, k, theta) - ey).max() < TOL
        for j in range(1, D):
            # 1-indexed levels k = 1..j+1 carry the phase, exponent (-j) on k = j+1
            want = np.ones(D, dtype=complex)
            a = np.sqrt(2.0 / (j * (j + 1)))
            for k1 in range(1, j + 2):
                want[k1 - 1] = np.exp(-0.5j * theta * a * ((-j) if k1 == j + 1 else 1))
            assert np.abs(gates.rz(D, j, theta) - np.diag(want)).max() < TOL


@pytest.mark.parametrize("D", range(2, 11))
def test_gell_mann_orthonormal(D):
    """Generalized Gell-Mann matrices: Hermitian, traceless, Tr(S_a S_b) = 2 delta_ab,
    D^2 - 1 of them (fixes the diagonal family's normalisation and support)."""
    mats = []
    for j in range(D):
        for k in range(j + 1, D):
            mats += [gates.gm_sym(D, j, k), gates.gm_asym(D, j, k)]
    mats += [gates.gm_diag(D, j) for j in range(1, D)]
    assert len(mats) == D * D - 1
    G = np.array([[np.trace(a @ b) for b in mats] for a in mats])
    assert np.abs(G - 2 * np.eye(len(mats))).max() < TOL
    for m in mats:
        assert abs(np.trace(m)) < TOL
        assert np.abs(m - m.conj().T).max() < TOL


@pytest.mark.parametrize("D", [2, 3, 4, 5, 7, 10])
def test_fourier_shift_clock_identities(D):
    H, X, Z = gates.fourier(D), gates.shift(D, 1), gates.clock(D, 1)
    w = gates.omega(D)
    I = np.eye(D)
    # unitarity
    for U in (H, X, Z):
        assert np.abs(U.conj().T @ U - I).max() < TOL
    # H|0> is the equal superposition of all D levels
    assert np.allclose(H[:, 0], np.full(D, 1 / np.sqrt(D)))
    # X^D = Z^D = I, Weyl relation Z X = w X Z
    assert np.abs(np.linalg.matrix_power(X, D) - I).max() < TOL
    assert np.abs(np.linalg.matrix_power(Z, D) - I).max() < TOL
    assert np.abs(Z @ X - w * X @ Z).max() < TOL
    # H^2 is the parity permutation |j> -> |-j mod D>, H^4 = I
    P = np.zeros((D, D))
    for j in range(D):
        P[(-j) % D, j] = 1
    assert np.abs(H @ H - P).max() < TOL
    assert np.abs(np.linalg.matrix_power(H, 4) - I).max() < TOL
    # shift by s acts as |x> -> |x+s>
    for s in range(D):
        Xs = gates.shift(D, s)
        for x in range(D):
            assert Xs[(x + s) % D, x] == 1


def test_printed_fourier_and_phase_shift():
    """The paper's printed Fourier matrix H (entries w^(r c) / sqrt D, so
    H[1][1] = w / sqrt D and H[1][2] = w^2 / sqrt D) and phase-shift matrix
    P = diag(1, w, .., w^(D-1)), written out for D = 3, 4 (5 for P).  A conjugated
    Fourier gate (w^(-r c)) fails here."""
    fx = json.load(open(os.path.join(GOLDEN, "paper_fourier_phase.json")))
    for case in fx["fourier"]:
        D = case["D"]
        w = np.exp(2j * np.pi / D)
        want = w ** np.array(case["exponents"], dtype=float) / np.sqrt(D)
        assert np.abs(gates.fourier(D) - want).max() < TOL, D
    for case in fx["phase_shift"]:
        D = case["D"]
        w = np.exp(2j * np.pi / D)
        assert np.abs(gates.clock(D, 1) - np.diag(w ** np.array(case["exponents"], dtype=float))).max() < TOL


@pytest.mark.parametrize("D", [2, 3, 4, 5, 7])
def test_fourier_diagonalises_the_shift(D):
    """H maps the shift to the clock: H X = Z H, i.e. H X H^dagger = Z
    (column n+1 of H is column n times w^m in row m).  The conjugate H^dagger
    gives Z^dagger instead, so a sign flip of the exponent fails."""
    H, X, Z = gates.fourier(D), gates.shift(D, 1), gates.clock(D, 1)
    assert np.abs(H @ X - Z @ H).max() < TOL
    assert np.abs(H @ X @ H.conj().T - Z).max() < TOL
    if D > 2:
        assert np.abs(H.conj().T @ X @ H - Z).max() > 0.1


@pytest.mark.parametrize("D", [2, 3, 4, 5, 10])
def test_clock_power(D):
    """Z^a is the a-th power of the printed phase-shift matrix P for every a
    (a = 0 gives the identity, a = D wraps to the identity), and satisfies the
    Weyl relation Z^a X = w^a X Z^a.  A clock that ignores a fails for a != 1."""
    w = np.exp(2j * np.pi / D)
    P = np.diag(w ** np.arange(D, dtype=float))
    X = gates.shift(D, 1)
    for a in range(-1, 2 * D + 1):
        Za = gates.clock(D, a)
        assert np.abs(Za - np.linalg.matrix_power(P, a % D)).max() < 1e-12, a
        assert np.abs(Za @ X - w ** a * X @ Za).max() < 1e-12, a
    assert np.abs(gates.clock(D, 0) - np.eye(D)).max() < TOL
    assert np.abs(gates.clock(D, D) - np.eye(D)).max() < 1e-12


def test_clock_exponents_in_circuits():
    """A register run through clock gates of every exponent: qudit q at level
    x_q picks up w^(a_q x_q), checked on basis states against the power of the
    printed P (the workloads draw a in {0, .., D-1})."""
    D, n = 3, 3
    w = np.exp(2j * np.pi / D)
    for a in ([0, 1, 2], [2, 2, 0], [1, 0, 2]):
        c = qi.Circuit(D, n, [("clock", q, a[q]) for q in range(n)])
        for digs in ([0, 0, 0], [1, 2, 1], [2, 1, 2]):
            psi = sim.run(c, sim.basis_state(D, n, digs))
            want = np.prod([w ** (a[q] * digs[q]) for q in range(n)])
            assert abs(psi[sim.index_of(D, digs)] - want) < TOL
            assert abs(np.abs(psi).sum() - 1) < TOL


@pytest.mark.parametrize("D", [2, 3, 5])
def test_rotation_inverse_and_unitary(D):
    for j in range(D):
        for k in range(j + 1, D):
            for f in (gates.rx, gates.ry):
                R = f(D, j, k, 0.77)
                assert np.abs(R @ f(D, j, k, -0.77) - np.eye(D)).max() < TOL
                assert np.abs(R.conj().T @ R - np.eye(D)).max() < TOL


# ------------------------------------------------------------ index and states

def test_decimal_index_and_state_string():
    D = 4
    dig = sim.parse_state_string("0-1-3")
    assert dig == [0, 1, 3]
    assert sim.index_of(D, dig) == 0 * 16 + 1 * 4 + 3
    psi = sim.basis_state(D, 3, dig)
    assert psi[7] == 1 and np.count_nonzero(psi) == 1


@pytest.mark.parametrize("D,n", [(3, 4), (2, 5), (5, 3)])
def test_fourier_on_qudit0_is_most_significant(D, n):
    c = qi.Circuit(D, n, [("h", 0)])
    psi = sim.run(c)
    nz = np.flatnonzero(np.abs(psi) > 1e-14)
    assert list(nz) == [m * D ** (n - 1) for m in range(D)]
    assert np.allclose(np.abs(psi[nz]), 1 / np.sqrt(D))


@pytest.mark.parametrize("D,n", [(2, 6), (3, 5), (4, 4), (5, 3), (10, 3)])
def test_ghz(D, n):
    """H on qudit 0 then CSUM chain (0->1)...(n-2->n-1) gives (1/sqrt D) sum_j |j..j>."""
    c = qi.Circuit(D, n, [("h", 0)] + qi.csum_chain(n))
    psi = sim.run(c)
    want = np.zeros(D ** n, dtype=complex)
    for j in range(D):
        want[sim.index_of(D, [j] * n)] = 1 / np.sqrt(D)
    assert np.abs(psi - want).max() < TOL


@pytest.mark.parametrize("D,n", [(3, 4), (4, 3)])
def test_uniform_after_fourier_layer_and_chain(D, n):
    """H on every qudit gives amplitude D^(-n/2) everywhere; a CSUM chain permutes
    it, so the state stays uniform (first stage of the D=3, n=4 workload)."""
    c = qi.Circuit(D, n, [("h", q) for q in range(n)] + qi.csum_chain(n))
    psi = sim.run(c)
    assert np.abs(psi - D ** (-n / 2)).max() < TOL


def test_csum_on_basis_states():
    D, n = 3, 2
    for xc in range(D):
        for xt in range(D):
            psi = sim.apply_csum(sim.basis_state(D, n, [xc, xt]), D, n, 0, 1)
            assert psi[sim.index_of(D, [xc, (xt + xc) % D])] == 1
            psi = sim.apply_csum(sim.basis_state(D, n, [xc, xt]), D, n, 1, 0)
            assert psi[sim.index_of(D, [(xc + xt) % D, xt])] == 1


@pytest.mark.parametrize("D", [2, 3, 5])
def test_permutation_orders(D):
    n = 3
    psi = qi.random_state(D, n, 11)
    p = psi.copy()
    for _ in range(D):
        p = sim.apply_csum(p, D, n, 2, 0)
    assert np.abs(p - psi).max() < TOL
    p = psi.copy()
    for _ in range(D):
        p = sim.apply_shift(p, D, n, 1, 1)
    assert np.abs(p - psi).max() < TOL
    # shift via the digit map equals the shift matrix applied on the axis
    assert np.abs(sim.apply_shift(psi, D, n, 1, 2) - sim.apply_1q(psi, D, n, 1, gates.shift(D, 2))).max() < TOL


# ----------------------------------------------------------------- brute force

@pytest.mark.parametrize("D,n,seed", [(2, 4, 0), (3, 4, 1), (4, 3, 2), (5, 3, 3), (3, 3, 4), (6, 2, 5)])
def test_sim_matches_bruteforce_unitary(D, n, seed):
    c = qi.random_circuit(D, n, 40, seed)
    U = brute.circuit_unitary(c)
    assert np.abs(U.conj().T @ U - np.eye(D ** n)).max() < 1e-10
    psi0 = qi.random_state(D, n, seed + 100)
    assert np.abs(sim.run(c, psi0) - U @ psi0).max() < 1e-12


def test_config1_bruteforce():
    c = qi.config1()
    assert len(c.ops) == 29 and c.nparams == 16
    U = brute.circuit_unitary(c)
    assert np.abs(sim.run(c) - U[:, 0]).max() < 1e-12


def test_swap_bruteforce():
    D, n = 3, 3
    psi = qi.random_state(D, n, 3)
    U = brute.op_unitary(("swap", 0, 2), D, n, None)
    assert np.abs(sim.apply_swap(psi, D, n, 0, 2) - U @ psi).max() < TOL


# ------------------------------------------------------------------- invariants

@pytest.mark.parametrize("D,n", [(3, 5), (5, 3)])
def test_norm_and_unapply(D, n):
    c = qi.random_circuit(D, n, 60, 9)
    psi = sim.basis_state(D, n)
    for op in c.ops:
        psi = sim.apply_op(psi, D, n, op, c.theta)
        assert abs(np.linalg.norm(psi) - 1) < 1e-12
    for op in reversed(c.ops):
        psi = sim.apply_inverse(psi, D, n, op, c.theta)
    assert np.abs(psi - sim.basis_state(D, n)).max() < 1e-12


# ------------------------------------------------------------------ algorithms

@pytest.mark.parametrize("D", [2, 3, 4, 5])
def test_deutsch_jozsa(D):
    """Constant oracle: the register reads 0..0 with certainty.  Balanced oracle
    (CSUM 2->3 with the target in the Fourier state of |D-1>): the phase kickback
    w^{x_2} moves qudit 2 to level D-1, so p[0] = 0."""
    psi0 = sim.basis_state(D, 4, [0, 0, 0, D - 1])
    pc = measure.marginal(sim.run(qi.deutsch_jozsa_d(D, "constant"), psi0), D, 4, [0, 1, 2])
    assert abs(pc[0] - 1) < TOL
    pb = measure.marginal(sim.run(qi.deutsch_jozsa_d(D, "balanced"), psi0), D, 4, [0, 1, 2])
    assert abs(pb[0]) < TOL
    assert abs(pb[sim.index_of(D, [0, 0, D - 1])] - 1) < TOL


def test_grover_qutrits():
    """One Grover iteration on two qutrits marked |22>: the marked amplitude is
    23/27, all others 5/27 (oracle I - 2|m><m|, diffusion 2|s><s| - I)."""
    g = qi.grover_d3_n2_marker22()
    D, n = g["dim"], g["n"]
    s = sim.run(qi.Circuit(D, n, [("h", 0), ("h", 1)]))
    m = sim.basis_state(D, n, list(g["marker"]))
    oracle_u = np.eye(D ** n) - 2 * np.outer(m, m.conj())
    diffusion = 2 * np.outer(s, s.conj()) - np.eye(D ** n)
    c = qi.Circuit(D, n, [("u", 0, 2, oracle_u), ("u", 0, 2, diffusion)])
    out = sim.run(c, s)
    want = np.full(9, 5 / 27, dtype=complex)
    want[8] = 23 / 27
    assert np.abs(out - want).max() < TOL
    assert abs(measure.probs(out)[8] - 529 / 729) < TOL


# ------------------------------------------------------------------ measurement

def test_marginals_product_state():
    D, n = 3, 4
    rng = np.random.default_rng(5)
    singles = [qi.random_unitary(D, rng)[:, 0] for _ in range(n)]
    psi = singles[0]
    for v in singles[1:]:
        psi = np.kron(psi, v)
    for qs in ([0], [2], [1, 3], [3, 1], [0, 1, 2, 3], [2, 0, 3]):
        want = np.array([1.0])
        for q in qs:
            want = np.kron(want, np.abs(singles[q]) ** 2)
        assert np.abs(measure.marginal(psi, D, n, qs) - want).max() < TOL
    assert abs(measure.probs(psi).sum() - 1) < TOL


def test_expectation_special_cases():
    D, n = 5, 3
    w = gates.omega(D)
    for digs in ([0, 0, 0], [3, 1, 4], [2, 2, 2]):
        psi = sim.basis_state(D, n, digs)
        assert abs(measure.expect_diag(psi, D, n, qi.z0_terms()) - w ** digs[0]) < TOL
        want = sum(w ** d for d in digs)
        assert abs(measure.expect_diag(psi, D, n, qi.zsum_terms(n)) - want) < TOL
    # <Z> vanishes on the Fourier state of |0>
    psi = sim.run(qi.Circuit(D, n, [("h", 0)]))
    assert abs(measure.expect_diag(psi, D, n, qi.z0_terms())) < TOL


# -------------------------------------------------------------------- gradients

@pytest.mark.parametrize("D", [2, 3, 5, 10])
def test_gradient_closed_form_single_qudit(D):
    """R_y^{01}(theta)|0>, O = Z: Re<Z> = cos^2(t/2) + sin^2(t/2) cos(2 pi/D), so
    dL/dtheta = -sin(theta) (1 - cos(2 pi / D)) / 2."""
    for theta in (0.4, -2.1, 1.3):
        c = qi.Circuit(D, 1, [("ry", 0, 0, 1, 0)], np.array([theta]))
        L = grad.loss(c, qi.zsum_terms(1))
        assert abs(L - (np.cos(theta / 2) ** 2 + np.sin(theta / 2) ** 2 * np.cos(2 * np.pi / D))) < TOL
        g = grad.adjoint(c, qi.zsum_terms(1))
        assert abs(g[0] + 0.5 * np.sin(theta) * (1 - np.cos(2 * np.pi / D))) < 1e-12


@pytest.mark.parametrize("D,n,seed", [(3, 3, 1), (4, 2, 2), (5, 2, 3), (2, 4, 4)])
def test_adjoint_matches_finite_differences(D, n, seed):
    c = qi.random_circuit(D, n, 50, seed)
    terms = qi.zsum_terms(n)
    g = grad.adjoint(c, terms)
    idx = np.arange(c.nparams)
    fd = grad.finite_diff(c, terms, idx, h=1e-5)
    assert np.abs(g - fd).max() <= 1e-8 * max(1.0, np.abs(fd).max())


def test_adjoint_shared_parameter():
    """A parameter used by two gates gets the sum of both contributions."""
    D = 3
    c = qi.Circuit(D, 2, [("rx", 0, 0, 1, 0), ("csum", 0, 1), ("ry", 1, 1, 2, 0)], np.array([0.9]))
    g = grad.adjoint(c, qi.zsum_terms(2))
    fd = grad.finite_diff(c, qi.zsum_terms(2), [0], h=1e-5)
    assert abs(g[0] - fd[0]) < 1e-9


@pytest.mark.parametrize("D,n,seed", [(3, 3, 5), (4, 2, 6), (2, 4, 7)])
def test_seeded_adjoint_of_a_state_loss(D, n, seed):
    """The paper's training loss on the output state, L = sum_x |t_x - psi_x|
    (section "Code style"): the seeded adjoint from lam = dL/d(conj psi) =
    -(t - psi) / (2 |t - psi|) equals central differences of L, and the seed
    lam = H_O psi reproduces the expectation adjoint."""
    c = qi.random_circuit(D, n, 40, seed)
    target = qi.random_state(D, n, seed + 50)
    psi = sim.run(c)
    r = target - psi
    lam = -r / (2 * np.abs(r))
    g = grad.adjoint_seeded(c, lam, psi_final=psi)
    fd = grad.finite_diff_state(c, lambda p: float(np.abs(target - p).sum()), np.arange(c.nparams), h=1e-6)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())
    terms = qi.zsum_terms(n)
    lam_o = measure.hermitian_part_diag(D, n, terms) * psi
    assert np.abs(grad.adjoint_seeded(c, lam_o, psi_final=psi) - grad.adjoint(c, terms)).max() < 1e-12


# ---------------------------------------------------------- controlled rotation

def _cr_op(case, c=0, t=1, p=0):
    if case["gate"] == "crz":
        return ("crz", c, t, case["j"], p)
    return (case["gate"], c, t, case["j"], case["k"], p)


def test_controlled_rotation_is_the_textbook_gate_for_qubits():
    """D = 2: sum_m |m><m| (x) R(m theta) is |0><0| (x) I + |1><1| (x) R(theta),
    the textbook controlled rotation, for all three types."""
    fx = json.load(open(os.path.join(GOLDEN, "textbook_controlled_rotations.json")))
    for case in fx["cases"]:
        for theta in (0.4, -2.3, np.pi):
            c = qi.Circuit(2, 2, [_cr_op(case)], np.array([theta]))
            want = _eval_matrix(case["matrix"], theta)
            assert np.abs(brute.circuit_unitary(c) - want).max() < TOL, case["name"]
            assert np.abs(np.column_stack([sim.run(c, np.eye(4)[:, i]) for i in range(4)]) - want).max() < TOL


@pytest.mark.parametrize("D,n,seed", [(3, 3, 1), (4, 3, 2), (5, 2, 3), (2, 4, 4)])
def test_controlled_rotation_sparse_rules_match_definition(D, n, seed):
    """The paper's sparse element rules (brute route) against the definition as
    a control-indexed stack of rotations exp(-i m theta S / 2), on random
    circuits mixing controlled rotations of every type with the other gates."""
    c = qi.random_circuit(D, n, 40, seed, kinds=["h", "ry", "csum", "crx", "cry", "crz", "clock"])
    assert any(op[0].startswith("cr") for op in c.ops)
    U = brute.circuit_unitary(c)
    assert np.abs(U.conj().T @ U - np.eye(D ** n)).max() < 1e-10
    psi0 = qi.random_state(D, n, seed + 7)
    assert np.abs(sim.run(c, psi0) - U @ psi0).max() < 1e-12


@pytest.mark.parametrize("D", [3, 4, 6])
def test_controlled_rotation_identities(D):
    """theta = 0 is the identity; the control's level-0 slab never changes; on
    the slab at control level 1 the gate is the plain rotation R(theta), at level
    m it is R(m theta); angles add: C(a) C(b) = C(a + b)."""
    n = 2
    psi = qi.random_state(D, n, 3 + D)
    for kind, extra in (("crx", (0, D - 1)), ("cry", (1, 2)), ("crz", (D - 1,))):
        op = (kind, 0, 1) + extra + (0,)
        plain = ({"crx": "rx", "cry": "ry", "crz": "rz"}[kind], 1) + extra + (0,)
        out0 = sim.apply_op(psi, D, n, op, np.array([0.0]))
        assert np.abs(out0 - psi).max() < TOL
        th = np.array([0.83])
        out = sim.apply_op(psi, D, n, op, th)
        v, w = psi.reshape(D, D), out.reshape(D, D)
        assert np.abs(w[0] - v[0]).max() < TOL
        assert np.abs(w[1] - gates.op_matrix(plain, D, th) @ v[1]).max() < TOL
        assert np.abs(w[2] - gates.op_matrix(plain, D, 2 * th) @ v[2]).max() < TOL
        ab = sim.apply_op(sim.apply_op(psi, D, n, op, np.array([0.5])), D, n, op, np.array([-1.2]))
        assert np.abs(ab - sim.apply_op(psi, D, n, op, np.array([-0.7]))).max() < TOL


@pytest.mark.parametrize("D,n,seed", [(3, 3, 11), (4, 2, 12), (2, 4, 13)])
def test_controlled_rotation_adjoint_matches_finite_differences(D, n, seed):
    """The adjoint of the controlled rotation (slab generator m S) against
    central differences, alone and with shared angles."""
    c = qi.random_circuit(D, n, 40, seed, kinds=["h", "rx", "csum", "crx", "cry", "crz", "cz"])
    terms = qi.zsum_terms(n)
    g = grad.adjoint(c, terms)
    fd = grad.finite_diff(c, terms, np.arange(c.nparams), h=1e-5)
    assert np.abs(g - fd).max() <= 1e-8 * max(1.0, np.abs(fd).max())
    c2 = qi.cr_ansatz(D, n, 2, seed)
    g2 = grad.adjoint(c2, terms)
    fd2 = grad.finite_diff(c2, terms, np.arange(c2.nparams), h=1e-5)
    assert np.abs(g2 - fd2).max() <= 1e-8 * max(1.0, np.abs(fd2).max())


# ------------------------------------------------------------- SWAP and MCX

def test_swap_and_toffoli_textbook_qubits():
    """D = 2: SWAP and the two-control MCX are the textbook SWAP and Toffoli
    (basis permutations from the fixture)."""
    fx = json.load(open(os.path.join(GOLDEN, "textbook_swap_toffoli.json")))
    for x, y in enumerate(fx["swap_2q"]):
        psi = np.zeros(4, dtype=complex)
        psi[x] = 1
        assert sim.apply_swap(psi, 2, 2, 0, 1)[y] == 1
    for x, y in enumerate(fx["toffoli_3q_controls_0_1_target_2"]):
        psi = np.zeros(8, dtype=complex)
        psi[x] = 1
        assert sim.apply_mcx(psi, 2, 3, [0, 1], 2)[y] == 1


@pytest.mark.parametrize("D", [3, 4, 5])
def test_swap_exchanges_product_factors(D):
    """SWAP on a product state |u> (x) |v> (x) |w> gives |w> (x) |v> (x) |u>
    (built with Kronecker products), and SWAP^2 = I."""
    rng = np.random.default_rng(D)
    u, v, w = (qi.random_unitary(D, rng)[:, 0] for _ in range(3))
    psi = np.kron(np.kron(u, v), w)
    assert np.abs(sim.apply_swap(psi, D, 3, 0, 2) - np.kron(np.kron(w, v), u)).max() < TOL
    r = qi.random_state(D, 3, 4)
    assert np.abs(sim.apply_swap(sim.apply_swap(r, D, 3, 1, 2), D, 3, 1, 2) - r).max() < TOL


@pytest.mark.parametrize("D", [2, 3, 5])
def test_mcx_identities(D):
    """One control: the CSUM routine; a control at level 0 disables it; D
    applications give the identity; with controls at levels (a, b) the target
    moves by a b mod D."""
    n = 4
    r = qi.random_state(D, n, 9)
    assert np.abs(sim.apply_mcx(r, D, n, [2], 0) - sim.apply_csum(r, D, n, 2, 0)).max() < TOL
    p = r.copy()
    for _ in range(D):
        p = sim.apply_mcx(p, D, n, [0, 3], 1)
    assert np.abs(p - r).max() < TOL
    for a in range(D):
        for b in range(D):
            digs = [a, 0, b, 1]
            out = sim.apply_mcx(sim.basis_state(D, n, digs), D, n, [0, 2], 3)
            assert out[sim.index_of(D, [a, 0, b, (1 + a * b) % D])] == 1


@pytest.mark.parametrize("D,n,seed", [(3, 4, 1), (2, 5, 2), (4, 3, 3)])
def test_swap_mcx_bruteforce_and_adjoint(D, n, seed):
    """Circuits with SWAP and MCX: gate-by-gate runner vs the brute-force
    unitary, and the adjoint (un-applying both) vs central differences."""
    c = qi.random_circuit(D, n, 50, seed, kinds=["h", "ry", "rz", "swap", "mcx", "csum", "crx"])
    assert any(op[0] == "swap" for op in c.ops) and any(op[0] == "mcx" for op in c.ops)
    U = brute.circuit_unitary(c)
    psi0 = qi.random_state(D, n, seed + 3)
    assert np.abs(sim.run(c, psi0) - U @ psi0).max() < 1e-12
    terms = qi.zsum_terms(n)
    g = grad.adjoint(c, terms)
    fd = grad.finite_diff(c, terms, np.arange(c.nparams), h=1e-5)
    assert np.abs(g - fd).max() <= 1e-8 * max(1.0, np.abs(fd).max())


# ------------------------------------------------------------------ shots

def test_sampling_inverse_cdf_exact_cases():
    """Inverse-CDF sampling with given uniforms: a basis state gives its index
    for every uniform; a uniform distribution over K bins with the midpoint
    uniforms (i + 1/2) / K puts exactly one shot in each bin; a two-bin
    distribution (1/3, 2/3) sends u < 1/3 to bin 0 and u >= 1/3 to bin 1; the
    last bin of non-zero probability catches u -> 1 (never a zero-probability
    bin)."""
    D, n = 3, 3
    psi = sim.basis_state(D, n, [2, 0, 1])
    u = np.linspace(0, 0.999, 50)
    assert np.all(measure.sample_inverse_cdf(measure.probs(psi), u) == sim.index_of(D, [2, 0, 1]))
    K = 27
    counts = measure.sample_counts(np.full(K, 1.0 / K), (np.arange(K) + 0.5) / K)
    assert np.array_equal(counts, np.ones(K))
    p = np.array([1 / 3, 2 / 3])
    assert list(measure.sample_inverse_cdf(p, [0.0, 0.3333, 0.334, 0.9999999])) == [0, 0, 1, 1]
    top = np.nextafter(1.0, 0.0)
    assert measure.sample_inverse_cdf(np.array([0.5, 0.5, 0.0]), [top])[0] == 1
    assert measure.sample_inverse_cdf(np.array([0.1, 0.0, 0.7, 0.2, 0.0, 0.0]), [top, 0.0999, 0.1])[0] == 3
    assert list(measure.sample_inverse_cdf(np.array([0.1, 0.0, 0.7, 0.2, 0.0, 0.0]), [0.0999, 0.1, 0.85])) == [0, 2, 3]


def test_sampling_rule_when_the_draw_reaches_the_total():
    """For a normal total, u * total < total for every u < 1 (round to
    nearest), so the search always finds a bin.  The product reaches the total
    for u = 1, for a subnormal total (the product rounds up: 5e-324 * u with
    u = 1 - 2^-53 is 5e-324), and for a zero total; the draw then goes to the
    last bin of non-zero probability, never to a trailing empty bin, and a
    zero state gives bin 0."""
    top = np.nextafter(1.0, 0.0)
    assert top * 5e-324 == 5e-324
    sub = np.array([5e-324, 5e-324, 0.0, 0.0])
    assert list(measure.sample_inverse_cdf(sub, [0.0, top])) == [0, 1]
    assert measure.sample_inverse_cdf(np.array([0.25, 0.75, 0.0]), [1.0])[0] == 1
    assert list(measure.sample_inverse_cdf(np.zeros(5), [0.0, 0.5, top])) == [0, 0, 0]


def test_sampling_matches_distribution_statistically():
    """Many shots of a random state's marginal: the histogram agrees with the
    probabilities (chi-square statistic below the 1e-6 tail of its
    distribution; a statistical check of the sampling route)."""
    from scipy.stats import chi2
    D, n = 3, 4
    psi = qi.random_state(D, n, 21)
    p = measure.marginal(psi, D, n, [2, 0])
    shots = 200000
    u = np.random.default_rng(22).random(shots)
    counts = measure.sample_counts(p, u)
    assert counts.sum() == shots
    stat = float(np.sum((counts - shots * p) ** 2 / (shots * p)))
    assert stat < chi2.isf(1e-6, len(p) - 1)
