"""Pins of the oracle's time steppers and of the triadic hyperedge predicate.

The GPU trajectory tests of the triadic, ring / rank-one and Cucker-Smale
models compare against the oracle's own RK4 and Euler loops, so each loop is
fixed here by something other than itself:

* an independent integrator (scipy's DOP853 at tight tolerances) and the
  step-size convergence order (RK4: the end-point error falls 16x when dt
  halves; Euler: 2x),
* reductions to the phase-model stepper, which ``test_oracle_pins`` fixes by
  the Adler closed form (triadic with K2 = 0; the ring against its explicit
  CSR adjacency; rank one with unit weights against the complete graph),
* the exact result of one RK4 / Euler step on a linear system: for y' = M y a
  step multiplies y by the stepper's matrix polynomial, I + hM + (hM)^2/2 +
  (hM)^3/6 + (hM)^4/24 for RK4 and I + hM for Euler.  The Cucker-Smale model
  with beta = 0 is linear (s' = v, v' = -(K/N) L v, L the graph Laplacian).

The triadic right-hand side with 0 < p < 1 (App. A.7 on a hypergraph whose
intra-community triples are drawn by a hash predicate) is fixed by a NumPy
brute force over a dense incidence tensor B[m, j, k], built from a splitmix64
written here from its published definition (the test vectors of
``tests/golden/splitmix64.json`` pin it), and by the oracle's explicit
hyperedge-list path (pinned by the one-triangle golden file) on the list of
triples the predicate selects.

Every pin is paired with planted mistakes (a wrong stage weight, a wrong
stage argument, the predicate called with wrong ids or an unsorted key,
unordered pairs counted once) that it must reject.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.integrate import solve_ivp
from scipy.sparse.csgraph import laplacian

import oracle
import workloads as W
from conftest import load_golden

M64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# splitmix64 and the hyperedge predicate, written from their definitions
# ---------------------------------------------------------------------------

def splitmix64(x):
    """One output of splitmix64 for state x (Steele, Lea and Flood, 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_python_splitmix64_published_vectors():
    g = load_golden("splitmix64.json")
    for s, o in zip(g["states"], g["outputs"]):
        assert splitmix64(int(s, 16)) == int(o, 16)


def threshold(p):
    """floor(p * 2^64) on the FP64 value of p."""
    return int(math.ldexp(p, 64)) if p < 1.0 else M64


def present(seed, thr, a, b, c, sort=True):
    """Hyperedge predicate of the intra-community triple {a, b, c}: the hash
    of the sorted ids packed 21 bits apart, against the threshold."""
    x, y, z = sorted((a, b, c)) if sort else (a, b, c)
    key = x | (y << 21) | (z << 42)
    return splitmix64((seed ^ key) & M64) < thr


def incidence(n, labels, seed, p, tri, mistake=None):
    """Dense B[m, j, k] (ordered pairs j != k, both != m): intra-community
    triples through the predicate plus the listed cross triangles.  `mistake`
    plants one slip, for the checks below."""
    B = np.zeros((n, n, n))
    thr = threshold(p)
    for c in range(labels.max() + 1):
        mem = np.flatnonzero(labels == c)
        for m in mem:
            for j in mem:
                for k in mem:
                    if m == j or m == k or j == k:
                        continue
                    if mistake == "unordered_once" and j > k:
                        continue
                    if mistake == "unsorted_key":
                        hit = present(seed, thr, int(m), int(j), int(k), sort=False)
                    elif mistake == "wrong_ids":
                        hit = present(seed, thr, int(j), int(j), int(k))
                    else:
                        hit = present(seed, thr, int(m), int(j), int(k))
                    if hit:
                        B[m, j, k] = 1.0
    for t in tri:
        for m, j, k in ((t[0], t[1], t[2]), (t[1], t[0], t[2]), (t[2], t[0], t[1])):
            B[m, j, k] = B[m, k, j] = 1.0
    return B


def dense_triadic(A, B, omega, K1, K2, theta):
    """omega_m + (K1/N) sum_l A_ml sin(theta_l - theta_m)
    + (K2/N^2) sum_{j,k} B_mjk sin(theta_j + theta_k - 2 theta_m)."""
    n = len(theta)
    pair = (A * np.sin(theta[None, :] - theta[:, None])).sum(axis=1)
    arg = theta[None, :, None] + theta[None, None, :] - 2 * theta[:, None, None]
    tri = (B * np.sin(arg)).sum(axis=(1, 2))
    return omega + K1 / n * pair + K2 / n ** 2 * tri


def hyper_problem(seed=11, n=48):
    rng = np.random.default_rng(seed)
    sizes = [14, 11, 9, 8]
    labels = W.shuffled_labels(sizes, n, rng)          # 6 nodes in no community
    g = W.sbm(labels, len(sizes), 0.7, p_out=0.05, seed=seed)
    tri = W.cross_triangles(labels, 9, seed + 1)
    theta = rng.uniform(0, 2 * np.pi, n)
    omega = rng.normal(size=n)
    return g, tri, theta, omega


@pytest.mark.parametrize("p", [0.9, 0.5, 0.23])
def test_triadic_predicate_branch_matches_dense_bruteforce(p):
    """App. A.7 (lambda = (1,1,-2)) on a hypergraph with 0 < p < 1: the oracle's
    in-loop predicate against the dense tensor sum over ordered pairs."""
    g, tri, theta, omega = hyper_problem()
    seed, K1, K2 = 0xC0FFEE, 1.3, 2.9
    A = oracle.dense_from_csr(g.n, g.row_ptr, g.col)
    B = incidence(g.n, g.labels, seed, p, tri)
    assert 0 < B.sum() < np.count_nonzero(np.ones_like(B))
    want = dense_triadic(A, B, omega, K1, K2, theta)
    got = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, seed, p, tri, omega, K1, K2, theta)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_triadic_predicate_branch_equals_explicit_list_of_its_triples():
    """The triples the predicate selects, handed to the oracle as an explicit
    hyperedge list with no communities, give the same right-hand side: the
    predicate branch and the list branch agree term by term."""
    g, tri, theta, omega = hyper_problem(seed=5)
    seed, p = 987654321, 0.9
    thr = threshold(p)
    listed = [tuple(t) for t in tri]
    for c in range(g.labels.max() + 1):
        mem = np.flatnonzero(g.labels == c)
        for a in range(len(mem)):
            for b in range(a + 1, len(mem)):
                for d in range(b + 1, len(mem)):
                    if present(seed, thr, int(mem[a]), int(mem[b]), int(mem[d])):
                        listed.append((mem[a], mem[b], mem[d]))
    got = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, seed, p, tri, omega, 0.7, 1.9, theta)
    nolab = np.full(g.n, -1, dtype=np.int32)
    want = oracle.triadic_rhs(g.n, g.row_ptr, g.col, nolab, 0, 0.0, np.array(listed), omega, 0.7, 1.9, theta)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("mistake", ["unsorted_key", "wrong_ids", "unordered_once"])
def test_triadic_bruteforce_rejects_planted_predicate_mistakes(mistake):
    g, tri, theta, omega = hyper_problem()
    seed, p, K1, K2 = 0xC0FFEE, 0.9, 1.3, 2.9
    A = oracle.dense_from_csr(g.n, g.row_ptr, g.col)
    got = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, seed, p, tri, omega, K1, K2, theta)
    bad = dense_triadic(A, incidence(g.n, g.labels, seed, p, tri, mistake), omega, K1, K2, theta)
    assert np.abs(bad - got).max() > 1e-6


# ---------------------------------------------------------------------------
# steppers written with one slip each (pure Python over the oracle's RHS)
# ---------------------------------------------------------------------------

def stepper_with(rhs, y0, dt, steps, mistake):
    """Classical RK4 with one planted mistake: 'weights' (equal weights 1/4),
    'stage_arg' (third stage at y + dt k2), 'last_arg' (fourth stage at
    y + dt/2 k3), 'euler_half' (Euler with dt/2)."""
    y = np.array(y0, dtype=np.float64, copy=True)
    for _ in range(steps):
        k1 = rhs(y)
        if mistake == "euler_half":
            y = y + 0.5 * dt * k1
            continue
        k2 = rhs(y + 0.5 * dt * k1)
        k3 = rhs(y + (dt if mistake == "stage_arg" else 0.5 * dt) * k2)
        k4 = rhs(y + (0.5 * dt if mistake == "last_arg" else dt) * k3)
        if mistake == "weights":
            y = y + dt / 4.0 * (k1 + k2 + k3 + k4)
        else:
            y = y + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


RK4_SLIPS = ["weights", "stage_arg", "last_arg"]


def convergence_ok(errs, order):
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    return all(2 ** order * 0.8 < r < 2 ** order * 1.25 for r in ratios), ratios


# ---------------------------------------------------------------------------
# triadic integrator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("stepper", ["rk4", "euler"])
def test_triadic_integrate_with_k2_zero_is_the_phase_stepper(stepper):
    P = W.random_phase_problem(150, 4, seed=12)
    g = P.graph
    tri = W.cross_triangles(g.labels, 40, 3)
    th, r = oracle.triadic_integrate(g.n, g.row_ptr, g.col, g.labels, 9, 0.8, tri, P.omega, P.K, 0.0,
                                     P.theta0, 0.02, 30, stepper=stepper)
    want, wr = oracle.phase_integrate(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0], P.theta0, 0.02, 30,
                                      stepper=stepper)
    np.testing.assert_allclose(th, want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r, wr, rtol=0, atol=1e-13)


def three_node_hypergraph():
    """Nodes 0, 1, 2 on one triangle (as a listed hyperedge) and a path 0-1-2 of
    pairwise links."""
    rp = np.array([0, 1, 3, 4], dtype=np.int64)
    col = np.array([1, 0, 2, 1], dtype=np.int32)
    labels = np.full(3, -1, dtype=np.int32)
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    omega = np.array([0.4, -0.3, 1.1])
    theta0 = np.array([0.1, 2.0, 4.2])
    return rp, col, labels, tri, omega, theta0


def test_triadic_integrate_order_against_dop853():
    """RK4 on the triadic model converges to an independent high-order solution
    with error ratio 16 when dt halves; Euler with ratio 2; the r(t) trace is
    the order parameter of the states."""
    rp, col, labels, tri, omega, theta0 = three_node_hypergraph()
    K1, K2, T = 1.4, 5.0, 2.0
    f = lambda t, y: oracle.triadic_rhs(3, rp, col, labels, 0, 0.0, tri, omega, K1, K2, y)
    ref = solve_ivp(f, (0, T), theta0, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    for stepper, order, grid in (("rk4", 4, (20, 40, 80)), ("euler", 1, (400, 800, 1600))):
        errs = []
        for steps in grid:
            th, r = oracle.triadic_integrate(3, rp, col, labels, 0, 0.0, tri, omega, K1, K2, theta0, T / steps,
                                             steps, stepper=stepper)
            errs.append(np.abs(th - ref).max())
            assert abs(r[-1] - abs(np.exp(1j * th).mean())) < 1e-15
            assert abs(r[0] - abs(np.exp(1j * theta0).mean())) < 1e-15
        ok, ratios = convergence_ok(errs, order)
        assert ok, (stepper, errs, ratios)
    assert errs[-1] < 1e-2


@pytest.mark.parametrize("mistake", RK4_SLIPS)
def test_triadic_order_pin_rejects_planted_stepper_mistakes(mistake):
    rp, col, labels, tri, omega, theta0 = three_node_hypergraph()
    K1, K2, T = 1.4, 5.0, 2.0
    rhs = lambda y: oracle.triadic_rhs(3, rp, col, labels, 0, 0.0, tri, omega, K1, K2, y)
    ref = solve_ivp(lambda t, y: rhs(y), (0, T), theta0, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    errs = [np.abs(stepper_with(rhs, theta0, T / s, s, mistake) - ref).max() for s in (20, 40, 80)]
    ok, _ = convergence_ok(errs, 4)
    assert not ok


# ---------------------------------------------------------------------------
# ring and rank-one integrators (App. B)
# ---------------------------------------------------------------------------

def ring_csr(n, k):
    rows = [sorted({(m + d) % n for d in range(-k, k + 1)} - {m}) for m in range(n)]
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    return rp, np.array([c for r in rows for c in r], dtype=np.int32)


ODD_H = ([0.0, 1.0, -0.35, 0.2], [0.0, 0.0, 0.0, 0.0])   # odd h: h(0) = 0, so the self pair adds nothing


@pytest.mark.parametrize("stepper", ["rk4", "euler"])
@pytest.mark.parametrize("n,k", [(37, 3), (64, 10)])
def test_ring_integrate_equals_phase_stepper_on_explicit_ring(stepper, n, k):
    rng = np.random.default_rng(n + k)
    om, th0 = rng.normal(size=n), rng.uniform(0, 2 * np.pi, n)
    ds, dc = ODD_H
    got, gr = oracle.structured_integrate("ring", n, om, 3.0, ds, dc, th0, 0.03, 40, k=k, stepper=stepper)
    rp, col = ring_csr(n, k)
    want, wr = oracle.phase_integrate(n, rp, col, om, 3.0, ds, dc, th0, 0.03, 40, stepper=stepper)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)
    np.testing.assert_allclose(gr, wr, rtol=0, atol=1e-13)


@pytest.mark.parametrize("stepper", ["rk4", "euler"])
def test_rank1_integrate_with_unit_weights_is_the_complete_graph_stepper(stepper):
    n = 50
    rng = np.random.default_rng(4)
    om, th0 = rng.normal(size=n), rng.uniform(0, 2 * np.pi, n)
    ds, dc = ODD_H
    got, gr = oracle.structured_integrate("rank1", n, om, 2.0, ds, dc, th0, 0.05, 30, alpha=np.ones(n),
                                          beta=np.ones(n), stepper=stepper)
    want, wr = oracle.phase_integrate(n, None, None, om, 2.0, ds, dc, th0, 0.05, 30, stepper=stepper,
                                      complete=True)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)
    np.testing.assert_allclose(gr, wr, rtol=0, atol=1e-13)


def test_rank1_integrate_order_against_dop853():
    """Random alpha, beta and a series with a cosine part (so the self pair
    counts): RK4 ratio 16, Euler ratio 2 against DOP853."""
    n, T = 7, 1.5
    rng = np.random.default_rng(8)
    om, th0 = rng.normal(size=n), rng.uniform(0, 2 * np.pi, n)
    al, be = rng.uniform(-1, 2, n), rng.uniform(0.3, 1.5, n)
    ds, dc = [0.0, 1.0, 0.4], [0.2, -0.5, 0.3]
    f = lambda t, y: oracle.structured_rhs("rank1", n, om, 4.0, ds, dc, y, alpha=al, beta=be)
    ref = solve_ivp(f, (0, T), th0, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    for stepper, order, grid in (("rk4", 4, (40, 80, 160)), ("euler", 1, (600, 1200, 2400))):
        errs = [np.abs(oracle.structured_integrate("rank1", n, om, 4.0, ds, dc, th0, T / s, s, alpha=al, beta=be,
                                                   stepper=stepper)[0] - ref).max() for s in grid]
        ok, ratios = convergence_ok(errs, order)
        assert ok, (stepper, errs, ratios)


@pytest.mark.parametrize("mistake", RK4_SLIPS + ["euler_half"])
def test_ring_pin_rejects_planted_stepper_mistakes(mistake):
    n, k = 37, 3
    rng = np.random.default_rng(n + k)
    om, th0 = rng.normal(size=n), rng.uniform(0, 2 * np.pi, n)
    ds, dc = ODD_H
    rp, col = ring_csr(n, k)
    stepper = "euler" if mistake == "euler_half" else "rk4"
    want, _ = oracle.phase_integrate(n, rp, col, om, 3.0, ds, dc, th0, 0.03, 40, stepper=stepper)
    rhs = lambda y: oracle.structured_rhs("ring", n, om, 3.0, ds, dc, y, k=k)
    bad = stepper_with(rhs, th0, 0.03, 40, mistake)
    assert np.abs(bad - want).max() > 1e-9


# ---------------------------------------------------------------------------
# Cucker-Smale integrator
# ---------------------------------------------------------------------------

def cs_linear_problem(n=30, seed=6):
    P = W.random_phase_problem(n, 3, seed=seed)
    g = P.graph
    rng = np.random.default_rng(seed)
    s0, v0 = rng.uniform(0, 10, (3, g.n)), rng.standard_normal((3, g.n))
    return g, s0, v0


def cs_linear_exact(g, K, s0, v0, dt, steps, stepper):
    """beta = 0: y = (s, v) per coordinate obeys y' = M y with
    M = [[0, I], [0, -(K/N) L]].  A step multiplies y by the stepper's matrix
    polynomial of h M; `steps` steps by its power."""
    n = g.n
    L = laplacian(sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(n, n))).toarray()
    M = np.zeros((2 * n, 2 * n))
    M[:n, n:] = np.eye(n)
    M[n:, n:] = -(K / n) * L
    Z = dt * M
    I = np.eye(2 * n)
    R = I + Z if stepper == "euler" else I + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    Rn = np.linalg.matrix_power(R, steps)
    y = Rn @ np.concatenate([s0, v0], axis=1).T        # [2n, 3]
    return y[:n].T, y[n:].T


@pytest.mark.parametrize("stepper", ["rk4", "euler"])
def test_cs_integrate_is_the_steppers_matrix_polynomial_when_linear(stepper):
    g, s0, v0 = cs_linear_problem()
    K, dt, steps = 6.0, 0.07, 25
    s, v = oracle.cs_integrate(g.n, g.row_ptr, g.col, K, 1.0, 0.0, s0, v0, dt, steps, stepper=stepper)
    ws, wv = cs_linear_exact(g, K, s0, v0, dt, steps, stepper)
    np.testing.assert_allclose(s, ws, rtol=0, atol=1e-11)
    np.testing.assert_allclose(v, wv, rtol=0, atol=1e-12)


def cs_stepper_with(g, K, beta, s0, v0, dt, steps, mistake):
    """RK4 over the oracle's Cucker-Smale RHS with one planted mistake:
    'weights', 'stage_arg', 'last_arg' (as for the phase steppers),
    's_from_v_slope' (the position stages move along the velocity slope of the
    stage instead of the position slope), 'euler_half'."""
    n = g.n

    def rhs(s, v):
        return oracle.cs_rhs(n, g.row_ptr, g.col, K, 1.0, beta, s, v)

    s, v = s0.copy(), v0.copy()
    for _ in range(steps):
        ks, kv = [], []
        if mistake == "euler_half":
            a, b = rhs(s, v)
            s, v = s + 0.5 * dt * a, v + 0.5 * dt * b
            continue
        for q, c in enumerate((0.0, 0.5, 0.5, 1.0)):
            if mistake == "stage_arg" and q == 2:
                c = 1.0
            if mistake == "last_arg" and q == 3:
                c = 0.5
            if q == 0:
                ts, tv = s, v
            else:
                slope = kv[q - 1] if mistake == "s_from_v_slope" else ks[q - 1]
                ts, tv = s + c * dt * slope, v + c * dt * kv[q - 1]
            a, b = rhs(ts, tv)
            ks.append(a)
            kv.append(b)
        w = (0.25, 0.25, 0.25, 0.25) if mistake == "weights" else (1 / 6, 1 / 3, 1 / 3, 1 / 6)
        s = s + dt * sum(wi * k for wi, k in zip(w, ks))
        v = v + dt * sum(wi * k for wi, k in zip(w, kv))
    return s, v


@pytest.mark.parametrize("mistake", RK4_SLIPS + ["euler_half"])
def test_cs_linear_pin_rejects_planted_stepper_mistakes(mistake):
    g, s0, v0 = cs_linear_problem()
    K, dt, steps = 6.0, 0.07, 25
    stepper = "euler" if mistake == "euler_half" else "rk4"
    ws, wv = cs_linear_exact(g, K, s0, v0, dt, steps, stepper)
    bs, bv = cs_stepper_with(g, K, 0.0, s0, v0, dt, steps, mistake)
    assert max(np.abs(bs - ws).max(), np.abs(bv - wv).max()) > 1e-8


def cs_nonlinear_reference(n=12, seed=3, K=30.0, T=1.0):
    g, s0, v0 = cs_linear_problem(n=n, seed=seed)

    def f(t, y):
        s, v = y[:3 * g.n].reshape(3, g.n), y[3 * g.n:].reshape(3, g.n)
        sd, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, K, 1.0, 0.25, s, v)
        return np.concatenate([sd.ravel(), vd.ravel()])

    y0 = np.concatenate([s0.ravel(), v0.ravel()])
    ref = solve_ivp(f, (0, T), y0, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    return g, s0, v0, ref


def test_cs_integrate_order_against_dop853_when_nonlinear():
    """beta = 1/4 (the config-4 weight): RK4 ratio 16 and Euler ratio 2 against
    DOP853; here the position stages feed the velocity slopes."""
    K, T = 30.0, 1.0
    g, s0, v0, ref = cs_nonlinear_reference(K=K, T=T)
    n = g.n
    for stepper, order, grid in (("rk4", 4, (10, 20, 40)), ("euler", 1, (200, 400, 800))):
        errs = []
        for steps in grid:
            s, v = oracle.cs_integrate(n, g.row_ptr, g.col, K, 1.0, 0.25, s0, v0, T / steps, steps,
                                       stepper=stepper)
            errs.append(np.abs(np.concatenate([s.ravel(), v.ravel()]) - ref).max())
        ok, ratios = convergence_ok(errs, order)
        assert ok, (stepper, errs, ratios)


@pytest.mark.parametrize("mistake", RK4_SLIPS + ["s_from_v_slope"])
def test_cs_nonlinear_pin_rejects_planted_stepper_mistakes(mistake):
    """'s_from_v_slope' leaves the beta = 0 system unchanged (v' does not
    depend on positions there), so the nonlinear order pin is the one that
    must reject it."""
    K, T = 30.0, 1.0
    g, s0, v0, ref = cs_nonlinear_reference(K=K, T=T)
    errs = []
    for steps in (10, 20, 40):
        s, v = cs_stepper_with(g, K, 0.25, s0, v0, T / steps, steps, mistake)
        errs.append(np.abs(np.concatenate([s.ravel(), v.ravel()]) - ref).max())
    ok, _ = convergence_ok(errs, 4)
    assert not ok
