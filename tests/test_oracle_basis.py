"""Pins of the FP64 oracle's separable expansions of the Cucker-Smale weight
(App. A.6: truncated Fourier series on [-L, L]^3; the learned MLP basis and
its loss gradient).  Each pin checks the oracle against something other than
itself: exact quadrature of polynomials, closed-form Fourier coefficients,
the paper's fast right-hand side with complex order parameters, special cases
of the network, central finite differences, and conservation laws."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _fd_ok(params, R, lo, hi, a, b, t, grad, idx, h=1e-6):
    """central finite differences of the loss at the parameter indices idx"""
    worst = 0.0
    for k in idx:
        pp = params.copy()
        pp[k] += h
        lp, _ = oracle.mlp_loss_grad(pp, R, lo, hi, a, b, t)
        pp[k] -= 2 * h
        lm, _ = oracle.mlp_loss_grad(pp, R, lo, hi, a, b, t)
        fd = (lp - lm) / (2 * h)
        worst = max(worst, abs(fd - grad[k]) / (abs(fd) + 1e-3 * np.abs(grad).max()))
    return worst


def _random_mlp(R, seed, scale=0.6):
    rng = np.random.default_rng(seed)
    n = oracle.mlp_param_count(R)
    p = rng.normal(scale=scale, size=n)
    p[-R:] = np.where(np.arange(R) % 4 == 3, -1.0, 1.0)  # fixed signs
    return p


def test_gauss_legendre_exact_on_polynomials():
    for m in (3, 10, 40, 96):
        x, w = oracle.gauss_legendre(m)
        assert abs(w.sum() - 2.0) < 1e-13
        for k in range(0, 2 * m, 3):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs((w * x ** k).sum() - exact) < 1e-13, (m, k)


def test_fourier_coeffs_closed_forms():
    L, K, sig = 20.0, 1.5, 1.0
    # beta = 0: w = K constant -> only the zero mode
    c = oracle.cs_fourier_coeffs(K, sig, 0.0, L, 2)
    assert abs(c[0, 0, 0] - K) < 1e-12
    assert np.abs(c.ravel()[1:]).max() < 1e-12
    # beta = -1: w = K (sig^2 + |y|^2); the cosine coefficient of y^2 on [-L, L]
    # is 2 L^2 (-1)^a / (pi a)^2 and its mean L^2 / 3
    c = oracle.cs_fourier_coeffs(K, sig, -1.0, L, 3)
    assert abs(c[0, 0, 0] - K * (sig ** 2 + L ** 2)) < 1e-9
    for a in (1, 2, 3):
        want = K * 2 * L ** 2 * (-1) ** a / (math.pi * a) ** 2
        for idx in ((a, 0, 0), (0, a, 0), (0, 0, a)):
            assert abs(c[idx] - want) < 1e-9, (idx, c[idx], want)
    mixed = [c[i, j, k] for i in range(4) for j in range(4) for k in range(4) if (i > 0) + (j > 0) + (k > 0) >= 2]
    assert np.abs(mixed).max() < 1e-9


def test_fourier_series_converges_inside_cube():
    L = 20.0
    rng = np.random.default_rng(0)
    ys = rng.uniform(-10, 10, (40, 3))
    exact = (1.0 + (ys ** 2).sum(1)) ** -0.25
    errs = []
    for p in (1, 2, 4, 8):
        c = oracle.cs_fourier_coeffs(1.0, 1.0, 0.25, L, p, nq=64)
        approx = np.array([oracle.cs_fourier_weight(c, L, y) for y in ys])
        errs.append(np.abs(approx - exact).max())
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 0.2 * errs[0]


def test_fourier_rhs_equals_paper_fast_form_all_to_all():
    """One complete community: the pair sum with the truncated series equals
    the fast form v_m' = sum_alpha c_alpha e^{-i pi <alpha, s_m>/L} (h_alpha - u_alpha v_m)
    with the order parameters u_alpha, h_alpha (App. A.6)."""
    n, L, p = 40, 20.0, 2
    rng = np.random.default_rng(3)
    s = rng.uniform(0, 10, (3, n))
    v = rng.standard_normal((3, n))
    c = oracle.cs_fourier_coeffs(1.0, 1.0, 0.25, L, p, nq=64)
    _, vd = oracle.cs_rhs_separable(n, None, None, np.zeros(n), 1.0, 1.0, 0.25, s, v, "fourier",
                                    fourier=c, L=L, complete=True)
    fast = np.zeros((3, n), dtype=complex)
    rngp = range(-p, p + 1)
    for a1 in rngp:
        for a2 in rngp:
            for a3 in rngp:
                al = np.array([a1, a2, a3])
                e = np.exp(1j * math.pi * (al @ s) / L)       # [n]
                u = e.sum() / n
                h = (e[None, :] * v).sum(1) / n              # [3]
                fast += c[abs(a1), abs(a2), abs(a3)] * np.conj(e)[None, :] * (h[:, None] - u * v)
    assert np.abs(fast.imag).max() < 1e-13
    assert np.abs(fast.real - vd).max() < 1e-13 * max(1.0, np.abs(vd).max())


def test_separable_with_exact_communities_is_exact():
    g = W.sbm(np.repeat(np.arange(4), 30).astype(np.int32), 4, 0.7, p_out=0.05, seed=11)
    n = g.n
    rng = np.random.default_rng(5)
    s = rng.uniform(0, 10, (3, n))
    v = rng.standard_normal((3, n))
    _, ref = oracle.cs_rhs(n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s, v)
    c = oracle.cs_fourier_coeffs(1.0, 1.0, 0.25, 20.0, 1, nq=48)
    for labels, exact in ((g.labels, np.ones(4)), (np.full(n, -1), None)):
        _, vd = oracle.cs_rhs_separable(n, g.row_ptr, g.col, labels, 1.0, 1.0, 0.25, s, v, "fourier",
                                        fourier=c, L=20.0, exact_comm=exact)
        assert np.abs(vd - ref).max() < 1e-15
    # approximate communities do change the result
    _, vd = oracle.cs_rhs_separable(n, g.row_ptr, g.col, g.labels, 1.0, 1.0, 0.25, s, v, "fourier",
                                    fourier=c, L=20.0)
    assert np.abs(vd - ref).max() > 1e-4


@pytest.mark.parametrize("basis", ["fourier", "mlp"])
def test_separable_conserves_momentum(basis):
    g = W.sbm(np.repeat(np.arange(3), 40).astype(np.int32), 3, 0.8, p_out=0.05, seed=12)
    n = g.n
    rng = np.random.default_rng(6)
    s = rng.uniform(0, 10, (3, n))
    v = rng.standard_normal((3, n))
    kw = dict(fourier=oracle.cs_fourier_coeffs(1.0, 1.0, 0.25, 20.0, 1, nq=48), L=20.0) if basis == "fourier" \
        else dict(mlp=_random_mlp(8, 1), R=8, lo=np.zeros(3), hi=np.full(3, 10.0))
    _, vd = oracle.cs_rhs_separable(n, g.row_ptr, g.col, g.labels, 1.0, 1.0, 0.25, s, v, basis, **kw)
    assert np.abs(vd.sum(1)).max() < 1e-13 * np.abs(vd).sum()


def test_mlp_special_cases():
    R = 4
    lo, hi = np.array([0.0, -2.0, 1.0]), np.array([10.0, 2.0, 5.0])
    npar = oracle.mlp_param_count(R)
    assert npar == 64 * 3 + 64 + 64 * 64 + 64 + R * 64 + 2 * R
    x = np.array([[0.0, 5.0, 10.0], [-2.0, 0.0, 2.0], [1.0, 3.0, 5.0]])
    # only output biases: phi = b3 everywhere
    p = np.zeros(npar)
    p[-2 * R:-R] = [0.5, -1.0, 2.0, 0.0]
    assert np.abs(oracle.mlp_forward(p, R, lo, hi, x) - p[-2 * R:-R]).max() == 0.0
    # first layer off: h1 = silu(0) = 0, so phi = W3 silu(b2) + b3
    p = np.random.default_rng(0).normal(size=npar)
    p[: 64 * 3 + 64] = 0.0
    b2 = p[64 * 3 + 64 + 64 * 64: 64 * 3 + 64 + 64 * 64 + 64]
    W3 = p[64 * 3 + 64 + 64 * 64 + 64:][: R * 64].reshape(R, 64)
    b3 = p[-2 * R:-R]
    silu = lambda z: z / (1 + np.exp(-z))
    want = W3 @ silu(b2) + b3
    assert np.abs(oracle.mlp_forward(p, R, lo, hi, x) - want[None, :]).max() < 1e-13
    # a single chain u_y -> h1[0] -> h2[0] -> phi[1]: phi_1 = silu(silu(u_y)), u = box-scaled coordinate
    p = np.zeros(npar)
    p[0 * 3 + 1] = 1.0                       # W1[0][1]
    p[64 * 3 + 64 + 0] = 1.0                 # W2[0][0]
    p[64 * 3 + 64 + 64 * 64 + 64 + 1 * 64 + 0] = 1.0   # W3[1][0]
    u = np.array([-1.0, 0.0, 1.0])           # x_y = -2, 0, 2 in [-2, 2]
    phi = oracle.mlp_forward(p, R, lo, hi, x)
    assert np.abs(phi[:, 1] - silu(silu(u))).max() < 1e-15
    assert np.abs(phi[:, [0, 2, 3]]).max() == 0.0


def test_mlp_gradient_matches_finite_differences():
    R = 8
    p = _random_mlp(R, 7)
    lo, hi = np.zeros(3), np.full(3, 10.0)
    rng = np.random.default_rng(8)
    a = rng.uniform(0, 10, (25, 3))
    b = rng.uniform(0, 10, (25, 3))
    t = (1 + ((a - b) ** 2).sum(1)) ** -0.25
    loss, g = oracle.mlp_loss_grad(p, R, lo, hi, a, b, t)
    # the loss is the mean squared error of the separable form
    phi_a = oracle.mlp_forward(p, R, lo, hi, a.T)
    phi_b = oracle.mlp_forward(p, R, lo, hi, b.T)
    wt = (phi_a * phi_b * p[-R:]).sum(1)
    assert abs(loss - ((wt - t) ** 2).mean()) < 1e-13 * max(loss, 1.0)
    npar = len(p)
    idx = np.concatenate([rng.choice(np.arange(0, npar - R), 80, replace=False),
                          np.arange(npar - 2 * R, npar - R)])        # incl. every b3
    assert _fd_ok(p, R, lo, hi, a, b, t, g, idx) < 1e-6
    assert np.all(g[-R:] == 0.0)                                     # signs are not trained


@pytest.mark.parametrize("slip", ["half", "sign_of_w2", "transposed_w2", "no_second_point"])
def test_fd_pin_catches_planted_gradient_mistakes(slip):
    R = 6
    p = _random_mlp(R, 9)
    lo, hi = np.zeros(3), np.full(3, 10.0)
    rng = np.random.default_rng(10)
    a = rng.uniform(0, 10, (12, 3))
    b = rng.uniform(0, 10, (12, 3))
    t = (1 + ((a - b) ** 2).sum(1)) ** -0.25
    _, g = oracle.mlp_loss_grad(p, R, lo, hi, a, b, t)
    o2 = 64 * 3 + 64
    bad = g.copy()
    if slip == "half":
        bad *= 0.5
    elif slip == "sign_of_w2":
        bad[o2:o2 + 4096] *= -1
    elif slip == "transposed_w2":
        bad[o2:o2 + 4096] = bad[o2:o2 + 4096].reshape(64, 64).T.ravel()
    else:
        # only one endpoint of each pair backpropagated: its W3 share halves
        s3 = o2 + 4096 + 64
        bad[s3:s3 + R * 64] *= 0.5
    idx = np.concatenate([np.arange(0, o2, 7), o2 + rng.choice(4096, 150, replace=False),
                          np.arange(o2 + 4096, len(p) - R, 5)])
    assert _fd_ok(p, R, lo, hi, a, b, t, bad, idx) > 1e-3


def test_rank64_separable_floor_on_flock_communities():
    """What any rank-R separable basis w~(x, y) = sum_r s_r phi_r(x) phi_r(y)
    can reach on the flocking communities (400 x 500 points in [0, 10]^3,
    w(r) = (1 + r^2)^(-1/4)): by Eckart-Young the truncated SVD of each
    community's weight matrix is the best rank-R approximation in Frobenius
    and spectral norm, so its errors are a floor for every basis, learned or
    Fourier.  The diagonal keeps w(0), the smooth choice (it multiplies
    v_i - v_i = 0 in the coupling).  Measured on 20 communities with the
    workload's own velocities: the coupling error
    ||C~ - C||_inf / ||C||_inf of the community sum stays at or above 1e-3 on
    average at rank 64 and clearly above it at rank 32, and the largest
    per-pair relative weight error stays above 1e-1.  A per-pair judge at
    1e-3 therefore sends every community to the exact path at rank <= 64."""
    F = W.flock()
    g = F.graph
    cpl = {32: [], 64: [], 128: []}
    pair = {32: [], 64: [], 128: []}
    for c in range(0, 400, 20):
        m = np.flatnonzero(g.labels == c)
        X, V = F.x0[:, m].T, F.v0[:, m].T
        Wm = (1.0 + ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)) ** -0.25
        U, s, Vt = np.linalg.svd(Wm)
        C = Wm @ V - Wm.sum(1)[:, None] * V
        off = ~np.eye(len(m), dtype=bool)
        for R in cpl:
            E = (U[:, :R] * s[:R]) @ Vt[:R] - Wm
            Ce = E @ V - E.sum(1)[:, None] * V
            cpl[R].append(np.abs(Ce).max() / np.abs(C).max())
            pair[R].append((np.abs(E[off]) / Wm[off]).max())
    mean = {R: float(np.mean(v)) for R, v in cpl.items()}
    # the floor falls with rank (a sanity check of the measurement itself)
    assert mean[32] > mean[64] > mean[128]
    assert mean[32] > 1.5e-3 and mean[64] > 1.0e-3
    assert min(pair[64]) > 1e-1
    # rank 128 (outside the 16..64 range of the basis) would reach 1e-3
    assert mean[128] < 1e-3
