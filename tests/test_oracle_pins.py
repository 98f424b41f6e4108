"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute force over a dense
matrix, the order-parameter and complement reformulations (Sec. 2 eq. KuramotoReformulation,
eq. OrderParameter; Sec. 3 eq. KuramotoGraphApproach), closed forms (splay state, the two
oscillator Adler equation), invariants (Sec. 2 eq. 5c, Sec. 3 eq. KuramotoGraphConservation),
finite differences, and the qualitative synchronisation statements of Sec. 2.
"""
import math

import numpy as np
import pytest

import gen
import oracle

EPS = np.finfo(np.float64).eps


def _dense_rhs_brute(A, omega, K, theta, scale):
    """Pure-Python double loop over a dense 0/1 matrix (tiny inputs only)."""
    n = len(theta)
    out = []
    for m in range(n):
        acc = 0.0
        for l in range(n):
            if A[m][l]:
                acc += math.sin(theta[l] - theta[m])
        out.append(omega[m] + K * scale[m] * acc)
    return np.array(out)


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("n", [1, 2, 7, 12])
def test_rhs_matches_brute_force(n, symmetric):
    rng = np.random.default_rng(10 + n + 100 * symmetric)
    A = (rng.random((n, n)) < 0.6).astype(np.uint8)
    if symmetric:
        A = np.triu(A, 1)
        A = A + A.T
    np.fill_diagonal(A, 0)
    g = gen.from_dense(A)
    omega = rng.standard_normal(n)
    theta = rng.uniform(-10, 10, n)
    K = 2.5
    got = oracle.rhs(g, omega, K, theta)
    ref = _dense_rhs_brute(A.tolist(), omega, K, theta, [1.0 / n] * n)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14 * max(1.0, np.abs(ref).max()))
    # non-uniform scaling: 1/deg_m, zero rows give omega_m (Sec. 3, zero rows and scaling (ii))
    deg = A.sum(1)
    got = oracle.rhs(g, omega, K, theta, scaling=1)
    ref = _dense_rhs_brute(A.tolist(), omega, K, theta, [1.0 / d if d else 0.0 for d in deg])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14 * max(1.0, np.abs(ref).max()))
    assert np.all(got[deg == 0] == omega[deg == 0])


def test_complete_graph_brute_force():
    n = 9
    rng = np.random.default_rng(3)
    A = np.ones((n, n), np.uint8)
    np.fill_diagonal(A, 0)
    omega, theta = rng.standard_normal(n), rng.uniform(0, 2 * np.pi, n)
    got = oracle.rhs(gen.complete_graph(n), omega, 1.7, theta)
    ref = _dense_rhs_brute(A.tolist(), omega, 1.7, theta, [1.0 / n] * n)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_direct_sum_equals_order_parameter_form():
    """Addition theorem: (1/M) sum_l sin(theta_l - theta_m) = S_M cos theta_m - C_M sin theta_m
    (Sec. 2, eq. KuramotoReformulation) and = r sin(psi - theta_m) (Sec. 2, eq. OrderParameter)."""
    w = gen.all_to_all()
    n, K = w.graph.n, w.K
    got = oracle.rhs(w.graph, w.omega, K, w.theta0)
    S = math.fsum(np.sin(w.theta0)) / n
    C = math.fsum(np.cos(w.theta0)) / n
    op_form = w.omega + K * (S * np.cos(w.theta0) - C * np.sin(w.theta0))
    bound = 8 * EPS * K * (n + 2)  # summation bound of n unit-size terms
    np.testing.assert_allclose(got, op_form, rtol=0, atol=bound)
    r, psi = oracle.order_parameter(w.theta0)
    np.testing.assert_allclose(got, w.omega + K * r * np.sin(psi - w.theta0), rtol=0, atol=bound)
    assert abs(r - math.hypot(S, C)) < 1e-14


def test_complement_identity_dense_block():
    """Sec. 3, eq. KuramotoGraphApproach: sum_{A_ml=1} sin(theta_l-theta_m)
    = (S - sum_{A_ml=0} sin theta_l) cos theta_m - (C - sum_{A_ml=0} cos theta_l) sin theta_m,
    the zero set including the diagonal."""
    rng = np.random.default_rng(5)
    n = 300
    g = gen.random_dense(n, 0.9, rng)
    A = g.dense()
    theta = rng.uniform(0, 2 * np.pi, n)
    omega = np.zeros(n)
    got = oracle.rhs(g, omega, float(n), theta)  # K = N makes the factor K/N = 1
    s, c = np.sin(theta), np.cos(theta)
    S, C = math.fsum(s), math.fsum(c)
    ref = np.array([(S - math.fsum(s[A[m] == 0])) * c[m] - (C - math.fsum(c[A[m] == 0])) * s[m]
                    for m in range(n)])
    np.testing.assert_allclose(got, ref, rtol=0, atol=16 * EPS * 2 * n)


def test_splay_state_is_incoherent():
    """theta_m = 2 pi m / M gives S_M = C_M = 0 (sums of roots of unity), so F = omega on the
    complete graph and r = 0 (Sec. 2, special choices with the order-parameter form)."""
    for M in (16, 100, 512):
        th = gen.splay_theta(M)
        w = gen.special_omega(M, 2.0)
        F = oracle.rhs(gen.complete_graph(M), w, 3.0, th)
        np.testing.assert_allclose(F, w, rtol=0, atol=1e-13)
        r, _ = oracle.order_parameter(th)
        assert r < 1e-14


def test_special_choices_golden():
    """The paper's closed-form frequencies and phases for M = 4, omega0 = 2 (tests/golden)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "special_choices_M4.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    om = np.array([float(r[1]) for r in rows])
    th = np.array([float(r[2]) for r in rows])
    np.testing.assert_allclose(gen.special_omega(4, 2.0), om, rtol=0, atol=1e-15)
    np.testing.assert_allclose(gen.splay_theta(4), th, rtol=0, atol=1e-15)


def test_fixed_point_synchronised():
    """omega = 0 and equal phases: every sine term is sin(0) = 0, so F = 0 exactly."""
    w = gen.sbm_equal(n_comm=4, comm_size=64, steps=10)
    th = np.full(w.graph.n, 1.2345)
    F = oracle.rhs(w.graph, np.zeros(w.graph.n), w.K, th)
    assert np.all(F == 0.0)
    thT, _, _ = oracle.rk4(w.graph, np.zeros(w.graph.n), w.K, th, 0.01, 20)
    assert np.all(thT == th)


def test_conservation_symmetric_uniform():
    """Symmetric A with uniform scaling: sum_m F_m = sum_m omega_m (Sec. 3, eq.
    KuramotoGraphConservation); it fails for an asymmetric A or non-uniform scaling."""
    w = gen.sbm_equal(n_comm=8, comm_size=128, rho_in=0.8, p_out=0.01, steps=10)
    g = w.graph
    F = oracle.rhs(g, w.omega, w.K, w.theta0)
    terms = w.K / g.n * g.nnz
    assert abs(math.fsum(F) - math.fsum(w.omega)) < 16 * EPS * (terms + np.abs(w.omega).sum())
    # degree scaling on unequal degrees breaks it (Sec. 3, non-uniform scaling)
    F1 = oracle.rhs(g, w.omega, w.K, w.theta0, scaling=1)
    assert abs(math.fsum(F1) - math.fsum(w.omega)) > 1e-6
    # asymmetric A breaks it
    rng = np.random.default_rng(1)
    ga = gen.random_dense(64, 0.5, rng, symmetric=False)
    th = rng.uniform(0, 2 * np.pi, 64)
    Fa = oracle.rhs(ga, np.zeros(64), 64.0, th)
    assert abs(math.fsum(Fa)) > 1e-3


def test_rk4_linear_invariant_and_free_rotation():
    """RK methods preserve linear invariants: mean(theta(t) - theta(0) - t omega) = 0 (Sec. 2
    eq. 5c / Sec. 3 eq. KuramotoGraphConservation); with K = 0, theta(T) = theta0 + T omega."""
    w = gen.sbm_equal(n_comm=4, comm_size=64, rho_in=0.9, p_out=0.02, steps=50)
    thT, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, 50)
    T = 50 * w.dt
    dev = math.fsum(thT - w.theta0 - T * w.omega) / w.graph.n
    assert abs(dev) < 1e-13
    th0, _, _ = oracle.rk4(w.graph, w.omega, 0.0, w.theta0, w.dt, 50)
    np.testing.assert_allclose(th0, w.theta0 + T * w.omega, rtol=0, atol=1e-13)


def _adler_phi(t, a, K, phi0):
    """Closed form of phi' = a - K sin(phi), phi = theta_2 - theta_1 of the two-oscillator
    classical model, via u = tan(phi/2) (a Riccati equation with constant coefficients)."""
    u0 = math.tan(phi0 / 2)
    if a * a > K * K:
        w = math.sqrt(a * a - K * K)
        t0 = -2.0 * math.atan((a * u0 - K) / w) / w
        u = (K + w * math.tan(w * (t - t0) / 2)) / a
    else:
        q = math.sqrt(K * K - a * a)
        z = (K - a * u0) / q
        assert abs(z) < 1
        t0 = -2.0 * math.atanh(z) / q
        u = (K - q * math.tanh(q * (t - t0) / 2)) / a
    return 2 * math.atan(u)


@pytest.mark.parametrize("a,K,phi0,T", [(0.5, 1.0, 1.0, 3.0), (1.2, 1.0, -1.5, 1.0)])
def test_rk4_fourth_order_adler(a, K, phi0, T):
    """Two coupled oscillators reduce to the Adler equation: phi' = (omega2 - omega1) - K sin phi
    (K/M with M = 2, two terms). RK4 error against the closed form shrinks 16x per halving."""
    g = gen.complete_graph(2)
    omega = np.array([0.3, 0.3 + a])
    th0 = np.array([0.2, 0.2 + phi0])
    exact = _adler_phi(T, a, K, phi0)
    errs = []
    for dt in (0.04, 0.02, 0.01, 0.005):
        n = int(round(T / dt))
        thT, _, _ = oracle.rk4(g, omega, K, th0, dt, n)
        errs.append(abs((thT[1] - thT[0]) - exact))
        # theta_1 + theta_2 = const + (omega_1 + omega_2) t exactly
        assert abs((thT[0] + thT[1]) - (th0.sum() + T * omega.sum())) < 1e-13
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for rt in ratios:
        assert 16 * 0.85 < rt < 16 * 1.15, (errs, ratios)
    assert errs[-1] < 1e-8


def test_synchronisation_qualitative():
    """Sec. 2, numerical integration: omega0 = 2, M = 100; K = 1 shows no synchronisation while
    K = 5 gives an order-parameter modulus close to one."""
    M = 100
    g = gen.complete_graph(M)
    w, th = gen.special_omega(M, 2.0), gen.splay_theta(M)
    _, r1, _ = oracle.rk4(g, w, 1.0, th, 0.02, 2500, r_every=2500)
    _, r5, _ = oracle.rk4(g, w, 5.0, th, 0.02, 2500, r_every=2500)
    assert r1[-1] < 0.3
    assert r5[-1] > 0.9


def test_order_parameter_special_cases():
    th = np.full(37, 0.7)
    r, psi = oracle.order_parameter(th)
    assert abs(r - 1) < 1e-15 and abs(psi - 0.7) < 1e-15
    r, psi = oracle.order_parameter(np.array([0.0, np.pi / 2]))
    assert abs(r - math.sqrt(0.5)) < 1e-15 and abs(psi - np.pi / 4) < 1e-15


def _fd_jacobian(g, omega, K, theta, h=1e-6, scaling=0):
    n = len(theta)
    J = np.empty((n, n))
    for j in range(n):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        J[:, j] = (oracle.rhs(g, omega, K, tp, scaling) - oracle.rhs(g, omega, K, tm, scaling)) / (2 * h)
    return J


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("scaling", [0, 1])
def test_vjp_matches_finite_difference_jacobian(symmetric, scaling):
    rng = np.random.default_rng(7)
    g = gen.random_dense(10, 0.5, rng, symmetric=symmetric)
    omega, theta = rng.standard_normal(10), rng.uniform(0, 6, 10)
    lam = rng.standard_normal(10)
    J = _fd_jacobian(g, omega, 3.0, theta, scaling=scaling)
    np.testing.assert_allclose(oracle.vjp(g, 3.0, theta, lam, scaling), J.T @ lam, rtol=0, atol=1e-8)


def _loss(thT, target):
    return oracle.loss_and_seed(thT, target)[0]


@pytest.mark.parametrize("symmetric", [True, False])
def test_adjoint_matches_central_differences(symmetric):
    rng = np.random.default_rng(11)
    n, steps, dt, K = 8, 25, 0.05, 2.0
    g = gen.random_dense(n, 0.6, rng, symmetric=symmetric)
    omega, th0 = rng.standard_normal(n), rng.uniform(0, 2 * np.pi, n)
    target = rng.uniform(0, 2 * np.pi, n)
    thT, _, _ = oracle.rk4(g, omega, K, th0, dt, steps)
    L, seed = oracle.loss_and_seed(thT, target)
    gt, gw, gk = oracle.adjoint_rk4(g, omega, K, th0, dt, steps, seed)
    h = 1e-6

    def f(om, th, k):
        return _loss(oracle.rk4(g, om, k, th, dt, steps)[0], target)
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        fd_t = (f(omega, th0 + e, K) - f(omega, th0 - e, K)) / (2 * h)
        fd_w = (f(omega + e, th0, K) - f(omega - e, th0, K)) / (2 * h)
        assert abs(gt[j] - fd_t) < 1e-7 * max(1.0, abs(fd_t))
        assert abs(gw[j] - fd_w) < 1e-7 * max(1.0, abs(fd_w))
    fd_k = (f(omega, th0, K + h) - f(omega, th0, K - h)) / (2 * h)
    assert abs(gk - fd_k) < 1e-7 * max(1.0, abs(fd_k))


def test_loss_seed_matches_finite_differences():
    rng = np.random.default_rng(2)
    th, target = rng.uniform(0, 6, 16), rng.uniform(0, 6, 16)
    _, seed = oracle.loss_and_seed(th, target)
    h = 1e-6
    for j in range(16):
        e = np.zeros(16)
        e[j] = h
        fd = (_loss(th + e, target) - _loss(th - e, target)) / (2 * h)
        assert abs(seed[j] - fd) < 1e-8


def test_adjoint_exact_cases():
    """L = sum theta(T): the linear invariant gives dL/dtheta0 = 1, dL/domega = T, dL/dK = 0 for
    symmetric A with uniform scaling; K = 0 gives theta(T) = theta0 + T omega exactly."""
    w = gen.sbm_equal(n_comm=3, comm_size=20, rho_in=0.8, p_out=0.1, steps=30)
    n, steps, dt = w.graph.n, 30, 0.02
    ones = np.ones(n)
    gt, gw, gk = oracle.adjoint_rk4(w.graph, w.omega, w.K, w.theta0, dt, steps, ones)
    np.testing.assert_allclose(gt, ones, rtol=0, atol=1e-12)
    np.testing.assert_allclose(gw, steps * dt * ones, rtol=0, atol=1e-12)
    assert abs(gk) < 1e-12
    seed = np.random.default_rng(0).standard_normal(n)
    gt, gw, gk = oracle.adjoint_rk4(w.graph, w.omega, 0.0, w.theta0, dt, steps, seed)
    np.testing.assert_allclose(gt, seed, rtol=0, atol=1e-13)
    np.testing.assert_allclose(gw, steps * dt * seed, rtol=0, atol=1e-13)


def test_potential_gradient_and_decrease():
    """-grad V = F for symmetric A and uniform scaling, and V decreases along the flow (Sec. 3,
    eq. ExtendedPotentialConservation; Sec. 2, potential)."""
    rng = np.random.default_rng(4)
    g = gen.random_dense(12, 0.7, rng)
    omega, th = rng.standard_normal(12), rng.uniform(0, 6, 12)
    K, h = 2.0, 1e-6
    F = oracle.rhs(g, omega, K, th)
    for j in range(12):
        e = np.zeros(12)
        e[j] = h
        dV = (oracle.potential(g, omega, K, th + e) - oracle.potential(g, omega, K, th - e)) / (2 * h)
        assert abs(-dV - F[j]) < 1e-8
    w = gen.sbm_equal(n_comm=2, comm_size=32, rho_in=0.9, p_out=0.05, steps=10)
    th = w.theta0.copy()
    V = [oracle.potential(w.graph, w.omega, w.K, th)]
    for _ in range(20):
        th, _, _ = oracle.rk4(w.graph, w.omega, w.K, th, 0.01, 5)
        V.append(oracle.potential(w.graph, w.omega, w.K, th))
    assert np.all(np.diff(V) <= 1e-12)


@pytest.mark.parametrize("M", [1, 2, 5, 64, 300])
def test_potential_complete_graph_closed_form(M):
    """Classical model (Sec. 2, eq. Potential): the pair sum of 1 - cos over all l, m equals
    M^2 (1 - C^2 - S^2) with C, S the normalised order-parameter sums, so
    V = -omega^T theta + (K M / 2)(1 - C_M^2 - S_M^2). C, S come from numpy's exact sums."""
    rng = np.random.default_rng(40 + M)
    omega, th = rng.standard_normal(M), rng.uniform(-7, 7, M)
    K = 1.7
    C = math.fsum(np.cos(th)) / M
    S = math.fsum(np.sin(th)) / M
    ref = -math.fsum(omega * th) + 0.5 * K * M * (1.0 - C * C - S * S)
    got = oracle.potential(gen.complete_graph(M), omega, K, th)
    scale = math.fsum(np.abs(omega * th)) + K * M
    assert abs(got - ref) <= 1e-12 * scale, (got, ref)
    # with omega = 0 the potential is (K M / 2)(1 - r^2) >= 0; 0 only at synchrony
    r, _ = oracle.order_parameter(th)
    got0 = oracle.potential(gen.complete_graph(M), np.zeros(M), K, th)
    assert abs(got0 - 0.5 * K * M * (1.0 - r * r)) <= 1e-12 * K * M
    # the splay state has r = 0, hence V = K M / 2 for omega = 0 (M >= 2)
    if M >= 2:
        sp = gen.splay_theta(M)
        assert abs(oracle.potential(gen.complete_graph(M), np.zeros(M), K, sp) - 0.5 * K * M) <= 1e-12 * K * M


def _potential_dense(A, omega, K, th, scale):
    """-omega^T theta + K/2 (sum Ahat - cos^T Ahat cos - sin^T Ahat sin) with Ahat = diag(scale) A
    (Sec. 3, eq. ExtendedPotentialConservation, second form), by numpy products."""
    Ah = scale[:, None] * A.astype(np.float64)
    c, s = np.cos(th), np.sin(th)
    return -float(omega @ th) + 0.5 * K * (float(Ah.sum()) - float(c @ (Ah @ c)) - float(s @ (Ah @ s)))


@pytest.mark.parametrize("kind", ["sbm", "weighted", "asym"])
def test_potential_graph_closed_form_and_synchrony(kind):
    """Graph potential (Sec. 3, eq. ExtendedPotentialConservation): the term-by-term form equals
    the order-parameter form K/2 (sum Ahat - c^T Ahat c - s^T Ahat s) for symmetric, weighted and
    asymmetric A, uniform and degree scaling (the potential's definition stays valid for
    non-symmetric scaled matrices); and at equal phases with omega = 0 it is exactly 0, the
    constant of integration fixed by synchrony (Sec. 2, indicator for synchronisation)."""
    rng = np.random.default_rng(7)
    if kind == "sbm":
        g = gen.sbm_equal(n_comm=3, comm_size=40, rho_in=0.8, p_out=0.05, steps=1).graph
    elif kind == "weighted":
        g = gen.weighted_sbm([20, 30, 17], [3, 1, 2], 0.2, 4, 0.05, rng)
    else:
        g = gen.random_dense(45, 0.4, rng, symmetric=False)
    A = g.dense()
    n = g.n
    omega, th = rng.standard_normal(n), rng.uniform(-5, 5, n)
    K = 2.3
    for scaling in (0, 1):
        deg = A.sum(1).astype(np.float64)
        scale = np.full(n, 1.0 / n) if scaling == 0 else np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)
        ref = _potential_dense(A, omega, K, th, scale)
        got = oracle.potential(g, omega, K, th, scaling=scaling)
        bound = 1e-12 * (np.abs(omega * th).sum() + K * (np.abs(A) * scale[:, None]).sum())
        assert abs(got - ref) <= bound, (kind, scaling, got, ref)
        # synchrony: every 1 - cos(0) is exactly 0
        for c0 in (0.0, 2.1, -40.0):
            assert oracle.potential(g, np.zeros(n), K, np.full(n, c0), scaling=scaling) == 0.0
    # a constant shift of all phases changes V only through -omega^T theta
    d = 0.37
    v0 = oracle.potential(g, omega, K, th)
    v1 = oracle.potential(g, omega, K, th + d)
    assert abs((v1 - v0) + d * omega.sum()) <= 1e-11 * (1 + abs(v0))


def test_rhs_rows_subset_consistent():
    w = gen.sbm_equal(n_comm=4, comm_size=64, steps=10)
    F = oracle.rhs(w.graph, w.omega, w.K, w.theta0)
    rows = np.array([0, 5, 255, 17, 17])
    np.testing.assert_array_equal(oracle.rhs_rows(w.graph, w.omega, w.K, w.theta0, rows), F[rows])


# ---------------------------------------------------------------------------------------------
# implicit midpoint rule (the second-order geometric integrator of Sec. 2)

def _mid_setup(seed=31):
    rng = np.random.default_rng(seed)
    sizes = np.array([40, 25, 35])
    g = gen.sbm(sizes, np.array([0.8, 0.6, 0.9]), 0.05, key=555, uperm=rng.permutation(100).astype(np.int32))
    return g, rng.standard_normal(100), rng.uniform(0, 2 * np.pi, 100)


def test_midpoint_few_iterations_are_textbook_methods():
    """One iteration is explicit Euler, two are the explicit midpoint rule (both written out
    here from the right-hand side)."""
    g, om, th = _mid_setup()
    K, dt = 2.5, 0.05
    e1, _, _ = oracle.midpoint(g, om, K, th, dt, 1, 1)
    assert np.abs(e1 - (th + dt * oracle.rhs(g, om, K, th))).max() < 1e-14
    e2, _, _ = oracle.midpoint(g, om, K, th, dt, 1, 2)
    want = th + dt * oracle.rhs(g, om, K, th + 0.5 * dt * oracle.rhs(g, om, K, th))
    assert np.abs(e2 - want).max() < 1e-14


def test_midpoint_converged_solves_the_implicit_equation():
    g, om, th = _mid_setup(32)
    K, dt = 3.0, 0.05
    y1, _, _ = oracle.midpoint(g, om, K, th, dt, 1, 40)
    res = y1 - th - dt * oracle.rhs(g, om, K, 0.5 * (th + y1))
    assert np.abs(res).max() < 1e-13


def test_midpoint_is_symmetric_and_second_order():
    g, om, th = _mid_setup(33)
    K = 3.0
    # symmetry: a step of dt followed by a step of -dt returns to the start
    y1, _, _ = oracle.midpoint(g, om, K, th, 0.05, 1, 40)
    y0, _, _ = oracle.midpoint(g, om, K, y1, -0.05, 1, 40)
    assert np.abs(y0 - th).max() < 1e-13
    # order 2 against an RK4 reference at T = 0.8
    ref, _, _ = oracle.rk4(g, om, K, th, 0.8 / 400, 400)
    errs = []
    for nst in (20, 40, 80):
        y, _, _ = oracle.midpoint(g, om, K, th, 0.8 / nst, nst, 40)
        errs.append(np.abs(y - ref).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.4), ratios


def test_midpoint_conserves_the_mean():
    """Symmetric A, uniform scaling: (1/N) sum (theta - theta0 - t omega) stays 0 (eq.
    KuramotoGraphConservation), for any number of iterations."""
    g, om, th = _mid_setup(34)
    for iters in (1, 3, 8):
        y, _, _ = oracle.midpoint(g, om, 2.0, th, 0.03, 50, iters)
        assert abs(np.mean(y - th - 1.5 * om)) < 1e-13


# ---------------------------------------------------------------------------------------------
# variable-step embedded Runge-Kutta pair (the variable stepsize fourth-order method of Sec. 2)

def test_rkf45_tableau_order_conditions():
    """The propagated weights satisfy the 8 conditions of order 4, the estimating weights the
    17 of order 5 (rooted trees up to order 5), with c_i = sum_j a_ij."""
    a, b4, b5 = oracle.rkf45_tableau()
    c = a.sum(axis=1)
    ac = a @ c
    ac2 = a @ c ** 2
    aac = a @ ac
    o4 = [(np.ones(6), 1.0), (c, 1 / 2), (c ** 2, 1 / 3), (ac, 1 / 6), (c ** 3, 1 / 4), (c * ac, 1 / 8),
          (ac2, 1 / 12), (aac, 1 / 24)]
    o5 = o4 + [(c ** 4, 1 / 5), (c ** 2 * ac, 1 / 10), (c * ac2, 1 / 15), (c * aac, 1 / 30), (ac ** 2, 1 / 20),
               (a @ c ** 3, 1 / 20), (a @ (c * ac), 1 / 40), (a @ ac2, 1 / 60), (a @ aac, 1 / 120)]
    for vec, val in o4:
        assert abs(b4 @ vec - val) < 1e-14, val
    for vec, val in o5:
        assert abs(b5 @ vec - val) < 1e-14, val
    # b4 is not of order 5 (the estimate is a genuine one)
    assert abs(b4 @ c ** 4 - 1 / 5) > 1e-4
    assert np.all(np.triu(a) == 0)


def test_rkf45_exact_without_coupling_and_error_control():
    g, om, th = _mid_setup(35)
    # K = 0: theta(T) = theta0 + T omega exactly, with growing steps
    y, st = oracle.rkf45(g, om, 0.0, th, 2.0, 0.01, 1e-8)
    assert np.abs(y - (th + 2.0 * om)).max() < 1e-13 and st[0] == 2.0 and st[3] == 0 and st[2] < 10
    # tighter tolerance, smaller error against a fine RK4 reference; rejections occur from a
    # too large first step
    ref, _, _ = oracle.rk4(g, om, 3.0, th, 1.0 / 2000, 2000)
    errs = []
    for atol in (1e-4, 1e-7, 1e-10):
        y, st = oracle.rkf45(g, om, 3.0, th, 1.0, 0.5, atol)
        assert st[0] == 1.0 and (atol > 1e-9 or st[3] >= 1)
        errs.append(np.abs(y - ref).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-8
    # the linear invariant (symmetric A, uniform scaling)
    y, _ = oracle.rkf45(g, om, 3.0, th, 1.0, 0.5, 1e-6)
    assert abs(np.mean(y - th - om)) < 1e-13


# ---------------------------------------------------------------------------------------------
# integer-weighted adjacency (Introduction: coefficients in a finite set)

def test_weighted_rhs_brute_force_and_linearity():
    rng = np.random.default_rng(61)
    g = gen.weighted_sbm([30, 20, 25], [2, 0, 3], 0.2, 4, 0.05, rng, uperm=rng.permutation(75).astype(np.int32))
    A = g.dense().astype(np.float64)
    om, th = rng.standard_normal(75), rng.uniform(0, 2 * np.pi, 75)
    K = 1.7
    brute = om + K / 75 * (A * np.sin(th[None, :] - th[:, None])).sum(axis=1)
    assert np.abs(oracle.rhs(g, om, K, th) - brute).max() < 1e-13
    # degree scaling uses the weighted row sums
    deg = A.sum(axis=1)
    brute1 = om + K * np.where(deg > 0, 1 / np.maximum(deg, 1), 0) * (A * np.sin(th[None, :] - th[:, None])).sum(axis=1)
    assert np.abs(oracle.rhs(g, om, K, th, scaling=1) - brute1).max() < 1e-13
    # linear in A: F(A1 + A2) - omega = (F(A1) - omega) + (F(A2) - omega)
    A1 = np.minimum(A, 1).astype(np.int32)
    g1, g2 = gen.from_dense(A1, g.labels), gen.from_dense((A - A1).astype(np.int32), g.labels)
    lhs = oracle.rhs(g, om, K, th) - om
    rhs = (oracle.rhs(g1, om, K, th) - om) + (oracle.rhs(g2, om, K, th) - om)
    assert np.abs(lhs - rhs).max() < 1e-13
