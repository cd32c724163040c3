"""Pins of the structured-adjacency oracle (App. B: rank-one coupling and the
k-nearest-neighbour ring).  Each check reaches the oracle's direct sums by an
independent route: the paper's factorised rank-one form, the paper's window
recurrence for the ring, the CSR phase oracle on an explicit ring adjacency,
the complete-graph phase oracle, reductions in k, linearity, an odd-coupling
invariant and synchrony."""
import numpy as np
import pytest

import oracle


def coeffs(rng, p):
    ds = np.concatenate([[0.0], rng.normal(size=p)])
    dc = np.concatenate([[rng.normal()], rng.normal(size=p)])
    return ds, dc


def h0(ds, dc):
    return dc.sum()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_rank1_factorised_form():
    """App. B.1: sum_l alpha_m beta_l h(theta_l - theta_m) equals alpha_m times
    the harmonics of R_k = sum_l beta_l e^{i k theta_l} against e^{-i k theta_m}
    (each harmonic on its own), computed here from complex sums."""
    rng = np.random.default_rng(1)
    n, p, K = 300, 3, 2.5
    ds, dc = coeffs(rng, p)
    th = rng.uniform(0, 2 * np.pi, n)
    al, be, om = rng.normal(size=n), rng.uniform(0.2, 2.0, n), rng.normal(size=n)
    got = oracle.structured_rhs("rank1", n, om, K, ds, dc, th, alpha=al, beta=be)
    s = dc[0] * be.sum() * np.ones(n)
    for k in range(1, p + 1):
        R = (be * np.exp(1j * k * th)).sum()
        w = R * np.exp(-1j * k * th)
        s += ds[k] * w.imag + dc[k] * w.real
    want = om + K / n * al * s
    assert rel(got - om, want - om) < 1e-12


def test_rank1_all_ones_is_the_complete_graph_plus_self_term():
    rng = np.random.default_rng(2)
    n, p, K = 200, 2, 1.7
    ds, dc = coeffs(rng, p)
    th = rng.uniform(0, 2 * np.pi, n)
    om = rng.normal(size=n)
    one = np.ones(n)
    got = oracle.structured_rhs("rank1", n, om, K, ds, dc, th, alpha=one, beta=one)
    comp = oracle.phase_rhs(n, np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32), om, K, ds, dc, th,
                            complete=True)
    assert rel(got - om, comp - om + K / n * h0(ds, dc)) < 1e-12


def test_rank1_linear_in_alpha_and_beta():
    rng = np.random.default_rng(3)
    n, p, K = 150, 2, 3.0
    ds, dc = coeffs(rng, p)
    th = rng.uniform(0, 2 * np.pi, n)
    al, be = rng.normal(size=n), rng.normal(size=n)
    base = oracle.structured_rhs("rank1", n, None, K, ds, dc, th, alpha=al, beta=be)
    sa = rng.uniform(0.5, 2.0, n)
    # scaling alpha_m scales row m; scaling every beta_l by c scales all rows by c
    assert rel(oracle.structured_rhs("rank1", n, None, K, ds, dc, th, alpha=sa * al, beta=be), sa * base) < 1e-12
    assert rel(oracle.structured_rhs("rank1", n, None, K, ds, dc, th, alpha=al, beta=-3.0 * be), -3.0 * base) < 1e-12


@pytest.mark.parametrize("n,k", [(500, 37), (64, 1), (101, 50)])
def test_ring_window_recurrence(n, k):
    """App. B.2: F_{m+1} = F_m - e^{i theta_{m-k}} + e^{i theta_{m+k+1}} (indices
    mod N), started from the direct window sum at m = 0; the ring sum of
    h = sin + c cos is Im + c Re of F_m e^{-i theta_m}."""
    rng = np.random.default_rng(4)
    th = rng.uniform(0, 2 * np.pi, n)
    c1, K = 0.7, 2.0
    z = np.exp(1j * th)
    F = np.empty(n, dtype=complex)
    F[0] = sum(z[l % n] for l in range(-k, k + 1))
    for m in range(n - 1):
        F[m + 1] = F[m] - z[(m - k) % n] + z[(m + k + 1) % n]
    w = F * np.exp(-1j * th)
    want = K / n * (w.imag + c1 * w.real)
    got = oracle.structured_rhs("ring", n, None, K, [0.0, 1.0], [0.0, c1], th, k=k)
    assert rel(got, want) < 1e-10


@pytest.mark.parametrize("n,k,p", [(300, 20, 2), (97, 3, 1), (50, 24, 3)])
def test_ring_equals_csr_oracle_on_explicit_ring(n, k, p):
    """The CSR phase oracle on the ring's adjacency built from the circular
    distance (no diagonal), plus the self term (K/N) h(0)."""
    rng = np.random.default_rng(5)
    ds, dc = coeffs(rng, p)
    th = rng.uniform(0, 2 * np.pi, n)
    om = rng.normal(size=n)
    K = 1.3
    rows = []
    for m in range(n):
        nb = sorted({(m + d) % n for d in range(-k, k + 1)} - {m})
        rows.append(nb)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c in r], dtype=np.int32)
    csr = oracle.phase_rhs(n, rp, col, om, K, ds, dc, th)
    got = oracle.structured_rhs("ring", n, om, K, ds, dc, th, k=k)
    assert rel(got - om, csr - om + K / n * h0(ds, dc)) < 1e-12


def test_ring_limits_of_k():
    rng = np.random.default_rng(6)
    n, p, K = 120, 2, 2.2
    ds, dc = coeffs(rng, p)
    th = rng.uniform(0, 2 * np.pi, n)
    om = rng.normal(size=n)
    one = np.ones(n)
    full = oracle.structured_rhs("rank1", n, om, K, ds, dc, th, alpha=one, beta=one)
    for k in (n // 2, n, 10 * n):
        assert rel(oracle.structured_rhs("ring", n, om, K, ds, dc, th, k=k) - om, full - om) < 1e-12
    # k = 0: only the self term
    got = oracle.structured_rhs("ring", n, om, K, ds, dc, th, k=0)
    assert np.allclose(got, om + K / n * h0(ds, dc), rtol=0, atol=1e-15)


def test_ring_odd_coupling_conserves_the_mean_frequency():
    """Symmetric adjacency and odd h: sum_m (H_m - omega_m) = 0."""
    rng = np.random.default_rng(7)
    n, K = 400, 3.0
    ds = np.array([0.0, 1.0, -0.4, 0.2])
    dc = np.zeros(4)
    th = rng.uniform(0, 2 * np.pi, n)
    c = oracle.structured_rhs("ring", n, None, K, ds, dc, th, k=33)
    assert abs(c.sum()) < 1e-12 * np.abs(c).sum()


def test_structured_synchrony_identical_frequencies():
    """Identical frequencies, all-to-all rank-one coupling with K > 0: the
    phases lock (r -> 1), and the ring of the same half-width agrees."""
    rng = np.random.default_rng(8)
    n = 60
    th0 = rng.uniform(0, 2 * np.pi, n)
    om = np.full(n, 0.3)
    one = np.ones(n)
    th, r = oracle.structured_integrate("rank1", n, om, 4.0, [0.0, 1.0], [0.0, 0.0], th0, 0.05, 400, alpha=one,
                                        beta=one)
    assert 1.0 - r[-1] < 1e-6
    th2, r2 = oracle.structured_integrate("ring", n, om, 4.0, [0.0, 1.0], [0.0, 0.0], th0, 0.05, 400, k=n // 2)
    assert np.abs(r2 - r).max() < 1e-12 and np.abs(th2 - th).max() < 1e-9
