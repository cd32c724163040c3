"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
own formula: they use hand-derived golden values, closed-form solutions,
invariants, special cases that reduce to a library routine, and convergence
orders.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import laplacian

import oracle
import workloads as W
from conftest import ev, load_golden


def csr_from_edges(n, edges):
    rows = [[] for _ in range(n)]
    for a, b in edges:
        rows[a].append(b)
        rows[b].append(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = []
    for i in range(n):
        r = sorted(rows[i])
        col.extend(r)
        rp[i + 1] = rp[i] + len(r)
    return rp, np.asarray(col, dtype=np.int32)


def complete_csr(n):
    return csr_from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])


# ---------------------------------------------------------------------------
# phase model right-hand side
# ---------------------------------------------------------------------------

def test_phase_rhs_golden_path_graph():
    """eq. (2.2), App. A.2: hand-derived values on a path graph with an
    isolated node (global 1/N), for h = sin and for a mixed series with d0,
    a cosine term and a second harmonic."""
    g = load_golden("phase_path3.json")
    n = g["n"]
    rp, col = csr_from_edges(n, g["edges"])
    theta = np.array([ev(t) for t in g["theta"]])
    omega = np.array(g["omega"])
    for case in g["cases"]:
        out = oracle.phase_rhs(n, rp, col, omega, g["K"], case["d_sin"], case["d_cos"], theta)
        want = np.array([ev(e) for e in case["expect"]])
        np.testing.assert_allclose(out, want, rtol=0, atol=1e-14)


def test_phase_rhs_mean_field_identity():
    """App. A.4 eq. (Kuramotofast3): on the complete graph with h = sin,
    H_m = omega_m + K Im(r_1 exp(-i theta_m)) with r_1 = mean(exp(i theta))."""
    rng = np.random.default_rng(7)
    n = 300
    theta = rng.uniform(0, 2 * np.pi, n)
    omega = rng.standard_normal(n)
    K = 2.5
    r1 = np.mean(np.exp(1j * theta))
    want = omega + K * np.imag(r1 * np.exp(-1j * theta))
    got_c = oracle.phase_rhs(n, None, None, omega, K, [0, 1], [0, 0], theta, complete=True)
    rp, col = complete_csr(n)
    got_csr = oracle.phase_rhs(n, rp, col, omega, K, [0, 1], [0, 0], theta)
    np.testing.assert_allclose(got_c, want, atol=1e-12)
    np.testing.assert_allclose(got_csr, want, atol=1e-12)


def test_phase_rhs_antisymmetry_invariant():
    """Symmetric A and odd h (sine terms only): sum_m (H_m - omega_m) = 0."""
    P = W.random_phase_problem(400, 4, seed=3, p=3, unassigned=20)
    g = P.graph
    d_cos = np.zeros_like(P.d_cos)
    out = oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, P.d_sin, d_cos, P.theta0)
    coupling = out - P.omega
    assert abs(coupling.sum()) < 1e-11 * np.abs(coupling).sum()
    assert np.abs(coupling).max() > 1e-3


def test_phase_rhs_permutation_equivariant():
    """Relabelling nodes permutes H the same way (catches index mix-ups)."""
    P = W.random_phase_problem(200, 3, seed=11, p=2, unassigned=5)
    g = P.graph
    base = oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, P.d_sin, P.d_cos, P.theta0)
    perm = np.random.default_rng(1).permutation(g.n)   # new id of old node i is perm[i]
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    Pm = sp.csr_matrix((np.ones(g.n), (perm, np.arange(g.n))), shape=(g.n, g.n))
    B = (Pm @ A @ Pm.T).tocsr()
    B.sort_indices()
    th = np.empty(g.n); th[perm] = P.theta0
    om = np.empty(g.n); om[perm] = P.omega
    out = oracle.phase_rhs(g.n, B.indptr.astype(np.int64), B.indices.astype(np.int32), om, P.K,
                           P.d_sin, P.d_cos, th)
    np.testing.assert_allclose(out[perm], base, atol=1e-13)


def test_phase_rhs_rows_subset_matches_full():
    P = W.random_phase_problem(150, 2, seed=5, p=2)
    g = P.graph
    full = oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, P.d_sin, P.d_cos, P.theta0)
    rows = np.array([0, 17, 149, 3])
    sub = oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, P.d_sin, P.d_cos, P.theta0, rows=rows)
    np.testing.assert_array_equal(sub, full[rows])


def test_phase_rhs_matches_dense_bruteforce():
    """Independent NumPy dense evaluation of the same definition (tiny N)."""
    for seed in range(4):
        P = W.random_phase_problem(48, 3, seed=seed, p=1 + seed, unassigned=4)
        g = P.graph
        A = oracle.dense_from_csr(g.n, g.row_ptr, g.col)
        want = oracle.dense_phase_rhs(A, P.omega, P.K, P.d_sin, P.d_cos, P.theta0)
        got = oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, P.d_sin, P.d_cos, P.theta0)
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_order_parameter_special_cases():
    assert abs(oracle.order_parameter(np.full(17, 1.234)) - 1.0) < 1e-15
    assert oracle.order_parameter(np.arange(12) * 2 * np.pi / 12) < 1e-15
    th = np.random.default_rng(0).uniform(0, 6, 50)
    assert abs(oracle.order_parameter(th) - abs(np.mean(np.exp(1j * th)))) < 1e-15


# ---------------------------------------------------------------------------
# time stepping
# ---------------------------------------------------------------------------

def adler_phi(t, phi0, dw, K):
    """Closed form of phi' = dw - K sin(phi) for |dw| < K (Adler locking),
    via u = tan(phi/2): u(t) = (K - g f(g (t - t0)/2)) / dw, g = sqrt(K^2 - dw^2),
    f = tanh or coth depending on the start."""
    g = math.sqrt(K * K - dw * dw)
    u0 = math.tan(phi0 / 2)
    z = (K - dw * u0) / g
    if abs(z) < 1:
        t0 = -2 * math.atanh(z) / g
        u = (K - g * np.tanh(g * (t - t0) / 2)) / dw
    else:
        t0 = -2 * math.atanh(1 / z) / g
        u = (K - g / np.tanh(g * (t - t0) / 2)) / dw
    return 2 * np.arctan(u)


def two_oscillators(theta0, omega, K, dt, steps, stepper="rk4"):
    rp, col = csr_from_edges(2, [(0, 1)])
    th, _ = oracle.phase_integrate(2, rp, col, omega, K, [0, 1], [0, 0], theta0, dt, steps,
                                   stepper=stepper, trace=False)
    return th


def test_rk4_adler_locking_closed_form():
    """Two coupled oscillators (N = 2, so K/N = K/2 per link): phi = theta_1 - theta_0
    obeys phi' = dw - K sin(phi); compare with the closed-form locking solution."""
    K, w0, w1 = 1.5, 0.3, 1.0
    dw = w1 - w0
    for phi0 in (-1.2, 0.1, -0.6):
        T = 6.0
        # with N = 2 the pairwise term is (K/2) sin(.), so phi' = dw - K sin(phi)
        th = two_oscillators(np.array([0.2, 0.2 + phi0]), np.array([w0, w1]), K, 0.01, 600)
        phi = th[1] - th[0]
        assert abs(phi - adler_phi(T, phi0, dw, K)) < 1e-9
        # the common mode moves at the mean frequency
        assert abs((th[0] + th[1]) / 2 - (0.2 + phi0 / 2 + (w0 + w1) / 2 * T)) < 1e-9


def test_rk4_adler_drift_period():
    """Unlocked pair (|dw| > K): phi advances by exactly 2 pi per period
    2 pi / sqrt(dw^2 - K^2)."""
    K, dw = 1.0, 2.0
    T = 2 * math.pi / math.sqrt(dw * dw - K * K)
    steps = 4000
    th = two_oscillators(np.array([0.0, 0.0]), np.array([0.0, dw]), K, T / steps, steps)
    assert abs((th[1] - th[0]) - 2 * math.pi) < 1e-10


@pytest.mark.parametrize("stepper,order", [("rk4", 4), ("euler", 1)])
def test_stepper_convergence_order(stepper, order):
    """Halving dt divides the end-point error by 2^order (RK4: 16; Euler: 2)."""
    K, w0, w1, phi0, T = 1.5, 0.3, 1.0, -1.0, 2.0
    exact = adler_phi(T, phi0, w1 - w0, K)
    errs = []
    for steps in (20, 40, 80):
        th = two_oscillators(np.array([0.0, phi0]), np.array([w0, w1]), K, T / steps, steps, stepper)
        errs.append(abs((th[1] - th[0]) - exact))
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    for r in ratios:
        assert 2 ** order * 0.8 < r < 2 ** order * 1.25, (errs, ratios)


def test_synchrony_identical_frequencies():
    """Identical omega, all-to-all, K > 0: phases lock, r -> 1."""
    n = 64
    rng = np.random.default_rng(2)
    theta0 = rng.uniform(0, 2 * np.pi, n)
    th, r = oracle.phase_integrate(n, None, None, np.full(n, 0.7), 4.0, [0, 1], [0, 0], theta0,
                                   0.05, 1000, complete=True)
    assert 1 - r[-1] < 1e-6
    assert r[0] < 0.5


def test_ott_antonsen_all_to_all():
    """All-to-all Kuramoto with Lorentzian omega (half-width D): the
    Ott-Antonsen reduction gives r(t) = r_inf / sqrt(1 + (r_inf^2/r0^2 - 1) exp(-(K - 2D) t)),
    r_inf = sqrt(1 - 2D/K); finite-N fluctuations are O(1/sqrt(N))."""
    n, D, K, r0 = 3000, 0.5, 3.0, 0.2
    rng = np.random.default_rng(5)
    omega = W.lorentzian(n, D, rng)
    # wrapped Cauchy initial phases with mean resultant r0
    theta0 = 2 * np.arctan(np.tan(np.pi * (rng.random(n) - 0.5)) * (1 - r0) / (1 + r0))
    steps, dt = 100, 0.04
    _, r = oracle.phase_integrate(n, None, None, omega, K, [0, 1], [0, 0], theta0, dt, steps,
                                  complete=True)
    t = np.arange(steps + 1) * dt
    rinf = math.sqrt(1 - 2 * D / K)
    want = rinf / np.sqrt(1 + (rinf ** 2 / r0 ** 2 - 1) * np.exp(-(K - 2 * D) * t))
    assert np.max(np.abs(r - want)) < 5 / math.sqrt(n)


# ---------------------------------------------------------------------------
# triadic model
# ---------------------------------------------------------------------------

def test_splitmix64_published_vectors():
    g = load_golden("splitmix64.json")
    for s, o in zip(g["states"], g["outputs"]):
        assert oracle.splitmix64(int(s, 16)) == int(o, 16)


def test_triple_predicate_threshold_and_rate():
    assert oracle.triple_threshold(0.5) == 2 ** 63
    assert oracle.triple_threshold(0.0) == 0
    assert oracle.triple_threshold(1.0) == 2 ** 64 - 1
    # order of the three ids does not matter; the rate matches p
    hits, tot = 0, 0
    for a in range(30):
        for b in range(a + 1, 30):
            for c in range(b + 1, 30):
                x = oracle.triple_present(12345, 0.9, a, b, c)
                assert x == oracle.triple_present(12345, 0.9, c, a, b)
                hits += x
                tot += 1
    sd = math.sqrt(tot * 0.9 * 0.1)
    assert abs(hits - 0.9 * tot) < 5 * sd


def test_triadic_golden_single_triangle():
    g = load_golden("triadic_one_triangle.json")
    n = g["n"]
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(0, dtype=np.int32)
    theta = np.array([ev(t) for t in g["theta"]])
    labels = np.full(n, -1, dtype=np.int32)
    out = oracle.triadic_rhs(n, rp, col, labels, 0, 0.0, np.array(g["triangles"]), np.zeros(n),
                             0.0, g["K2"], theta)
    np.testing.assert_allclose(out, [ev(e) for e in g["expect"]], atol=1e-14)


def test_triadic_all_to_all_reduces_to_order_parameters():
    """App. A.7 eq. (HOKuramoto_fastRHS) with lambda = (1,1,-2), restricted to
    distinct j, k, m: sum_{j != k, both != m} exp(i(theta_j + theta_k))
    = (S1 - z_m)^2 - (S2 - z_m^2), S1 = sum z, S2 = sum z^2."""
    n = 40
    rng = np.random.default_rng(9)
    theta = rng.uniform(0, 2 * np.pi, n)
    labels = np.zeros(n, dtype=np.int32)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(0, dtype=np.int32)
    K2 = 2.0
    out = oracle.triadic_rhs(n, rp, col, labels, 77, 1.0, np.zeros((0, 3)), np.zeros(n), 0.0, K2, theta)
    z = np.exp(1j * theta)
    S1, S2 = z.sum(), (z ** 2).sum()
    want = K2 / n ** 2 * np.imag(np.conj(z) ** 2 * ((S1 - z) ** 2 - (S2 - z ** 2)))
    np.testing.assert_allclose(out, want, atol=1e-12)


def test_triadic_pairwise_part_is_kuramoto():
    P = W.random_phase_problem(120, 3, seed=4)
    g = P.graph
    out = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, 1, 0.0, np.zeros((0, 3)), P.omega, P.K,
                             0.0, P.theta0)
    want = oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0], P.theta0)
    np.testing.assert_allclose(out, want, atol=1e-13)


# ---------------------------------------------------------------------------
# Cucker-Smale
# ---------------------------------------------------------------------------

def test_cs_golden_two_birds():
    g = load_golden("cs_two_birds.json")
    rp, col = csr_from_edges(2, [(0, 1)])
    s, v = np.array(g["s"]), np.array(g["v"])
    sd, vd = oracle.cs_rhs(2, rp, col, g["K"], g["sigma"], g["beta"], s, v)
    np.testing.assert_array_equal(sd, v)
    np.testing.assert_allclose(vd, [[ev(e) for e in row] for row in g["expect_vdot"]], atol=1e-15)


def test_cs_beta_zero_is_laplacian_consensus():
    """beta = 0 makes the weight the constant K: v' = -(K/N) L v with L the
    graph Laplacian (scipy.sparse.csgraph)."""
    P = W.random_phase_problem(90, 3, seed=6)
    g = P.graph
    rng = np.random.default_rng(1)
    s, v = rng.uniform(0, 5, (3, g.n)), rng.standard_normal((3, g.n))
    K = 1.7
    _, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, K, 1.0, 0.0, s, v)
    L = laplacian(sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))).toarray()
    want = -(K / g.n) * (L @ v.T).T
    np.testing.assert_allclose(vd, want, atol=1e-13)


def test_cs_momentum_and_symmetries():
    """Symmetric A: sum_m v_m' = 0.  Translating positions changes nothing;
    rotating positions and velocities rotates v'."""
    P = W.random_phase_problem(80, 2, seed=8)
    g = P.graph
    rng = np.random.default_rng(3)
    s, v = rng.uniform(0, 10, (3, g.n)), rng.standard_normal((3, g.n))
    _, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s, v)
    assert np.abs(vd.sum(axis=1)).max() < 1e-13
    _, vd_t = oracle.cs_rhs(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s + np.array([[3.0], [-1.0], [2.0]]), v)
    np.testing.assert_allclose(vd_t, vd, atol=1e-13)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    _, vd_r = oracle.cs_rhs(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, Q @ s, Q @ v)
    np.testing.assert_allclose(vd_r, Q @ vd, atol=1e-13)


def test_cs_matches_dense_bruteforce_and_conserves_momentum_in_time():
    P = W.random_phase_problem(40, 2, seed=2)
    g = P.graph
    rng = np.random.default_rng(4)
    s, v = rng.uniform(0, 10, (3, g.n)), rng.standard_normal((3, g.n))
    A = oracle.dense_from_csr(g.n, g.row_ptr, g.col)
    _, want = oracle.dense_cs_rhs(A, 1.0, 1.0, 0.25, s, v)
    _, got = oracle.cs_rhs(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s, v)
    np.testing.assert_allclose(got, want, atol=1e-14)
    s1, v1 = oracle.cs_integrate(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s, v, 0.05, 50)
    np.testing.assert_allclose(v1.mean(axis=1), v.mean(axis=1), atol=1e-13)
    # velocity spread contracts (alignment)
    assert np.var(v1, axis=1).sum() < np.var(v, axis=1).sum()


# ---------------------------------------------------------------------------
# planted-mistake checks: each pin above must catch a plausible oracle slip
# ---------------------------------------------------------------------------

def _mutant_phase_rhs(kind, n, rp, col, omega, K, d_sin, d_cos, theta):
    """Re-implementations of the phase RHS with one deliberate mistake each,
    to show the pins are sharp enough (pure NumPy, CPU only)."""
    out = np.empty(n)
    for m in range(n):
        acc = 0.0
        for l in col[rp[m]:rp[m + 1]]:
            x = theta[l] - theta[m]
            if kind == "sign":
                x = -x
            hv = d_cos[0]
            for k in range(1, len(d_sin)):
                if kind == "drop_cos":
                    hv += d_sin[k] * math.sin(k * x)
                else:
                    hv += d_sin[k] * math.sin(k * x) + d_cos[k] * math.cos(k * x)
            acc += hv
        scale = K / (rp[m + 1] - rp[m] if kind == "local_n" and rp[m + 1] > rp[m] else n)
        out[m] = omega[m] + scale * acc
    return out


@pytest.mark.parametrize("kind", ["sign", "drop_cos", "local_n"])
def test_golden_catches_planted_mistakes(kind):
    g = load_golden("phase_path3.json")
    n = g["n"]
    rp, col = csr_from_edges(n, g["edges"])
    theta = np.array([ev(t) for t in g["theta"]])
    omega = np.array(g["omega"])
    caught = False
    for case in g["cases"]:
        out = _mutant_phase_rhs(kind, n, rp, col, omega, g["K"], case["d_sin"], case["d_cos"], theta)
        want = np.array([ev(e) for e in case["expect"]])
        caught |= not np.allclose(out, want, atol=1e-12)
    assert caught
