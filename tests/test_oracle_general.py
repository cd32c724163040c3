"""Pins of the general (non-difference) phase coupling of the oracle: the
real 2-D Fourier series of App. A.2 reduces to the difference-form oracle,
equals the paper's generalised-order-parameter form on the complete graph,
and matches a separable product computed as a matrix-vector product."""
import numpy as np
import scipy.sparse

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


def test_difference_form_is_a_special_case():
    """h(x - y) = sum_k dcos_k cos(k(x-y)) + dsin_k sin(k(x-y)) expands to
    c11 = c22 = dcos_k, c21 = dsin_k, c12 = -dsin_k on the diagonal (k, k)."""
    rng = np.random.default_rng(1)
    n, p, K = 90, 3, 2.0
    A, rp, col = random_graph(n, 0.2, 2)
    ds = np.concatenate([[0.0], rng.normal(size=p)])
    dc = rng.normal(size=p + 1)
    c11, c12, c21, c22 = (np.zeros((p + 1, p + 1)) for _ in range(4))
    for k in range(p + 1):
        c11[k, k] = dc[k]
        if k > 0:
            c22[k, k] = dc[k]
            c21[k, k] = ds[k]
            c12[k, k] = -ds[k]
    th = rng.uniform(0, 2 * np.pi, n)
    om = rng.normal(size=n)
    got = oracle.phase_rhs_general(n, rp, col, om, K, c11, c12, c21, c22, th)
    want = oracle.phase_rhs(n, rp, col, om, K, ds, dc, th)
    assert rel(got - om, want - om) < 1e-12


def test_generalised_order_parameter_form():
    """App. A.2: on the complete graph, sum_{l != m} g(theta_l, theta_m) =
    sum_{a,b} coefficients x (sums over l of cos/sin(a theta_l)) x cos/sin(b theta_m)
    minus the l = m term."""
    rng = np.random.default_rng(3)
    n, p, K = 250, 2, 1.5
    cs = [rng.normal(size=(p + 1, p + 1)) for _ in range(4)]
    th = rng.uniform(0, 2 * np.pi, n)
    got = oracle.phase_rhs_general(n, None, None, None, K, *cs, th, complete=True)
    C = np.array([np.cos(a * th).sum() for a in range(p + 1)])
    S = np.array([np.sin(a * th).sum() for a in range(p + 1)])
    cb = np.cos(np.outer(np.arange(p + 1), th))
    sb = np.sin(np.outer(np.arange(p + 1), th))
    full = (C @ cs[0]) @ cb + (C @ cs[1]) @ sb + (S @ cs[2]) @ cb + (S @ cs[3]) @ sb
    ca, sa = cb, sb
    self_term = np.einsum("an,ab,bn->n", ca, cs[0], cb) + np.einsum("an,ab,bn->n", ca, cs[1], sb) + \
        np.einsum("an,ab,bn->n", sa, cs[2], cb) + np.einsum("an,ab,bn->n", sa, cs[3], sb)
    assert rel(got, K / n * (full - self_term)) < 1e-11


def test_separable_product():
    """g(x, y) = cos(2x) sin(y): the coupling is sin(theta_m) (A cos(2 theta))_m."""
    rng = np.random.default_rng(4)
    n, K = 120, 3.0
    A, rp, col = random_graph(n, 0.25, 5)
    p = 2
    c11, c12, c21, c22 = (np.zeros((p + 1, p + 1)) for _ in range(4))
    c12[2, 1] = 1.0
    th = rng.uniform(0, 2 * np.pi, n)
    got = oracle.phase_rhs_general(n, rp, col, None, K, c11, c12, c21, c22, th)
    assert rel(got, K / n * np.sin(th) * (A @ np.cos(2 * th))) < 1e-12
