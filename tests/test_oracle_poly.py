"""Pins of the polynomial-coupling oracle (App. A.3 difference form and the
Desai-Zwanzig model of App. A.5): the graph Laplacian for h(x) = x, the
paper's fast forms on the complete graph (first moment for Desai-Zwanzig,
binomial expansion over the moments w_k for general h), the odd-coupling
invariant, and the exact solution of the linear system."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.csgraph

import oracle


def random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    up = np.triu(rng.random((n, n)) < p, 1)
    A = (up | up.T).astype(np.float64)
    S = scipy.sparse.csr_matrix(A)
    S.sort_indices()
    return A, S.indptr.astype(np.int64), S.indices.astype(np.int32)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_linear_coupling_is_the_graph_laplacian():
    n, K = 80, 2.0
    A, rp, col = random_graph(n, 0.2, 1)
    x = np.random.default_rng(2).normal(size=n)
    got = oracle.poly_rhs(n, rp, col, None, K, [0.0, 1.0], None, x)
    L = scipy.sparse.csgraph.laplacian(A)
    assert rel(got, -K / n * (L @ x)) < 1e-13


def test_desai_zwanzig_mean_field_form():
    """App. A.5: x_m' = -V'(x_m) + (w_1 - x_m) on the complete graph (K = 1);
    the l = m pair contributes h(0) = 0.  V(x) = x^4/4 - x^2/2, -V'(x) = x - x^3."""
    n = 300
    x = np.random.default_rng(3).normal(size=n)
    got = oracle.poly_rhs(n, None, None, None, 1.0, [0.0, 1.0], [0.0, 1.0, 0.0, -1.0], x, complete=True)
    want = (x - x ** 3) + (x.mean() - x)
    assert rel(got, want) < 1e-13


@pytest.mark.parametrize("p", [2, 4, 6])
def test_binomial_moment_form(p):
    """eq. PolyDifferenceRHSfast: sum_l h(x_l - x_m) = sum_a h_a sum_k C(a,k) W_k (-x_m)^(a-k)
    with W_k = sum_l x_l^k (l = m included, so h(0) is removed for the
    complete graph without self loops)."""
    rng = np.random.default_rng(4 + p)
    n, K = 200, 1.5
    h = rng.normal(size=p + 1)
    x = rng.uniform(-1.2, 1.2, n)
    got = oracle.poly_rhs(n, None, None, None, K, h, None, x, complete=True)
    W = [np.sum(x ** k) for k in range(p + 1)]
    s = np.zeros(n)
    for a in range(p + 1):
        for k in range(a + 1):
            s += h[a] * math.comb(a, k) * W[k] * (-x) ** (a - k)
    want = K / n * (s - h[0])
    assert rel(got, want) < 1e-11


def test_odd_coupling_conserves_the_sum():
    n = 120
    A, rp, col = random_graph(n, 0.15, 5)
    x = np.random.default_rng(6).normal(size=n)
    c = oracle.poly_rhs(n, rp, col, None, 3.0, [0.0, 1.0, 0.0, 0.4, 0.0, -0.1], None, x)
    assert abs(c.sum()) < 1e-12 * np.abs(c).sum()


@pytest.mark.parametrize("stepper", ["rk4", "euler"])
def test_linear_system_exact_solution(stepper):
    """f(x) = -g x, h(x) = x: x' = -M x with M = g I + (K/N) L.  One step of
    the stepper is exactly the matrix polynomial R(-dt M) (Euler: I - dt M;
    RK4: the degree-4 Taylor polynomial of the exponential), so the trajectory
    is R^steps x0; RK4 also tracks expm(-t M) x0."""
    n, K, g = 40, 4.0, 0.3
    A, rp, col = random_graph(n, 0.3, 7)
    x0 = np.random.default_rng(8).normal(size=n)
    M = g * np.eye(n) + K / n * scipy.sparse.csgraph.laplacian(A)
    T, steps = 2.0, 400
    dt = T / steps
    got = oracle.poly_integrate(n, rp, col, None, K, [0.0, 1.0], [0.0, -g], x0, dt, steps, stepper=stepper)
    Z = -dt * M
    I = np.eye(n)
    Rm = I + Z if stepper == "euler" else I + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    assert rel(got, np.linalg.matrix_power(Rm, steps) @ x0) < 1e-12
    if stepper == "rk4":
        assert rel(got, scipy.linalg.expm(-T * M) @ x0) < 1e-10


def test_frequencies_and_local_term_add():
    n = 50
    A, rp, col = random_graph(n, 0.3, 9)
    rng = np.random.default_rng(10)
    x, om = rng.normal(size=n), rng.normal(size=n)
    f = [0.5, -1.0, 0.25]
    base = oracle.poly_rhs(n, rp, col, None, 2.0, [0.1, 1.0, 0.3], None, x)
    full = oracle.poly_rhs(n, rp, col, om, 2.0, [0.1, 1.0, 0.3], f, x)
    assert rel(full - base, om + f[0] + f[1] * x + f[2] * x * x) < 1e-13


def test_general_polynomial_reduces_to_the_difference_form():
    """h(x - y) = sum_a h_a (x - y)^a expands to c[i, j] = h_{i+j} C(i+j, i) (-1)^j."""
    rng = np.random.default_rng(30)
    n, p, K = 70, 3, 2.0
    A, rp, col = random_graph(n, 0.25, 31)
    h = rng.normal(size=p + 1)
    c = np.zeros((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1 - i):
            c[i, j] = h[i + j] * math.comb(i + j, i) * (-1) ** j
    x = rng.uniform(-1, 1, n)
    got = oracle.poly_rhs_general(n, rp, col, None, K, c, None, x)
    assert rel(got, oracle.poly_rhs(n, rp, col, None, K, h, None, x)) < 1e-12


def test_general_polynomial_moment_form():
    """App. A.3 eq. PolyRHS on the complete graph: sum_{l != m} g(x_l, x_m) =
    sum_{a,b} c[a, b] W_a x_m^b - g(x_m, x_m), W_a = sum_l x_l^a."""
    rng = np.random.default_rng(32)
    n, p, K = 200, 3, 1.5
    c = rng.normal(size=(p + 1, p + 1))
    x = rng.uniform(-1.2, 1.2, n)
    got = oracle.poly_rhs_general(n, None, None, None, K, c, None, x, complete=True)
    Wm = np.array([np.sum(x ** a) for a in range(p + 1)])
    V = np.vstack([x ** b for b in range(p + 1)])
    full = Wm @ c @ V
    own = np.einsum("an,ab,bn->n", V, c, V)
    assert rel(got, K / n * (full - own)) < 1e-11


def test_general_polynomial_separable_product():
    """g(x, y) = x^2 y: the coupling is x_m (A x^2)_m."""
    n = 90
    A, rp, col = random_graph(n, 0.3, 33)
    x = np.random.default_rng(34).normal(size=n)
    c = np.zeros((3, 3))
    c[2, 1] = 1.0
    got = oracle.poly_rhs_general(n, rp, col, None, 3.0, c, None, x)
    assert rel(got, 3.0 / n * x * (A @ x ** 2)) < 1e-12


def vdp_F(eps):
    """van der Pol in the paper's Table 1 form: f = (x2 - x1^3/3 + x1, -eps x1)."""
    F = np.zeros((2, 4, 4))
    F[0, 0, 1] = 1.0
    F[0, 3, 0] = -1.0 / 3.0
    F[0, 1, 0] = 1.0
    F[1, 1, 0] = -eps
    return F


def test_osc2_local_term_is_van_der_pol():
    n = 50
    rng = np.random.default_rng(60)
    x = rng.normal(size=(2, n))
    got = oracle.osc2_rhs(n, None, None, None, 0.0, [0.0, 1.0], vdp_F(0.3), x, complete=True)
    assert rel(got[0], x[1] - x[0] ** 3 / 3 + x[0]) < 1e-14 and rel(got[1], -0.3 * x[0]) < 1e-14


def test_osc2_coupling_is_the_laplacian_per_component():
    n, K = 80, 2.5
    A, rp, col = random_graph(n, 0.2, 61)
    x = np.random.default_rng(62).normal(size=(2, n))
    got = oracle.osc2_rhs(n, rp, col, None, K, [0.0, 1.0], np.zeros((2, 4, 4)), x)
    L = scipy.sparse.csgraph.laplacian(A)
    assert rel(got, -K / n * (L @ x.T).T) < 1e-13


def test_osc2_components_match_the_one_component_oracle():
    """Each component's coupling is the one-component polynomial oracle's."""
    n = 60
    A, rp, col = random_graph(n, 0.3, 63)
    rng = np.random.default_rng(64)
    x = rng.uniform(-1, 1, (2, n))
    h = [0.1, 1.0, 0.0, -0.3]
    got = oracle.osc2_rhs(n, rp, col, None, 3.0, h, np.zeros((2, 4, 4)), x)
    for d in range(2):
        assert rel(got[d], oracle.poly_rhs(n, rp, col, None, 3.0, h, None, x[d])) < 1e-13


@pytest.mark.parametrize("stepper", ["rk4", "euler"])
def test_osc2_integrate_is_the_stepper_map_of_the_harmonic_oscillator(stepper):
    """Uncoupled linear local terms f = (v, -u): every node follows x <- M x
    with M the stepper's matrix polynomial of dt A, A = [[0, 1], [-1, 0]]
    (RK4: the degree-4 Taylor polynomial; Euler: I + dt A)."""
    n, dt, steps = 5, 0.1, 30
    F = np.zeros((2, 4, 4))
    F[0, 0, 1] = 1.0
    F[1, 1, 0] = -1.0
    x0 = np.random.default_rng(65).normal(size=(2, n))
    got = oracle.osc2_integrate(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), None, 0.0, [0.0, 1.0], F, x0,
                                dt, steps, stepper=stepper)
    B = dt * np.array([[0.0, 1.0], [-1.0, 0.0]])
    M = np.eye(2) + B if stepper == "euler" else np.eye(2) + B + B @ B / 2 + B @ B @ B / 6 + B @ B @ B @ B / 24
    want = np.linalg.matrix_power(M, steps) @ x0
    assert rel(got, want) < 1e-13
