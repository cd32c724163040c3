"""GPU parity of the polynomial difference coupling (App. A.3; the
Desai-Zwanzig model of App. A.5) against the FP64 oracle: single right-hand
sides on planted-community graphs (with nodes outside every community), both
methods and precisions, harmonics of h up to degree 8 with a local
polynomial f, trajectories, and sampled rows at N = 1e6."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

DZ_F = [0.0, 1.0, 0.0, -1.0]   # -V'(x) for the double well V = x^4/4 - x^2/2


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2203_16657_amd as cia
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cia.load()
    return cia, torch


def coupling_err(got, want, base):
    c = want - base
    return float(np.abs((got - base) - c).max() / max(np.abs(c).max(), 1e-300))


def gpu_rhs(env, plan, x, precision):
    cia, torch = env
    dt = torch.float64 if precision else torch.float32
    t = torch.as_tensor(x, dtype=dt, device="cuda")
    out = torch.empty_like(t)
    plan.rhs(t, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("graph", ["config1", "config2_scaled"])
@pytest.mark.parametrize("h", [[0.0, 1.0], [0.2, 1.0, -0.3, 0.5]])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_poly_rhs(env, graph, h, method, precision):
    cia, torch = env
    P = W.kuramoto_small() if graph == "config1" else W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    x = np.random.default_rng(1).uniform(-1.5, 1.5, g.n)
    K = 3.0
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=K, h=h, method=method, precision=precision)
    got, xr = gpu_rhs(env, plan, x, precision)
    want = oracle.poly_rhs(g.n, g.row_ptr, g.col, None, K, h, None, xr)
    err = coupling_err(got, want, 0.0)
    say(graph, "h", h, "method", method, "prec", precision, "coupling rel_inf", err, "n_unassigned",
        plan.info().n_unassigned)
    assert err < (1e-12 if precision else 1e-5)
    plan.close()


@pytest.mark.parametrize("p", [2, 5, 8])
def test_poly_degrees_with_local_term(env, p):
    cia, torch = env
    P = W.kuramoto_small()
    g = P.graph
    rng = np.random.default_rng(20 + p)
    h = rng.normal(size=p + 1) / np.arange(1, p + 2)
    x = rng.uniform(-1.0, 1.0, g.n)
    om = rng.normal(size=g.n)
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, om, K=2.0, h=h, f=DZ_F, precision=1)
    got, _ = gpu_rhs(env, plan, x, 1)
    want = oracle.poly_rhs(g.n, g.row_ptr, g.col, om, 2.0, h, DZ_F, x)
    base = om + x - x ** 3
    err = coupling_err(got, want, base)
    say("degree", p, "coupling rel_inf", err, "total rel", np.abs(got - want).max() / np.abs(want).max())
    assert err < 1e-11 and np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    plan.close()


def test_poly_complete_graph(env):
    """All-to-all Desai-Zwanzig, the paper's fast form (one community)."""
    cia, torch = env
    n = 3000
    x = np.random.default_rng(5).normal(size=n)
    plan = cia.Plan.poly(n, complete=True, K=1.0, h=[0.0, 1.0], f=DZ_F, precision=1)
    got, _ = gpu_rhs(env, plan, x, 1)
    want = (x - x ** 3) + (x.mean() - x)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    plan.close()


@pytest.mark.parametrize("stepper", [0, 1])
def test_poly_trajectory(env, stepper):
    cia, torch = env
    P = W.kuramoto_small()
    g = P.graph
    x0 = np.random.default_rng(7).uniform(-1.5, 1.5, g.n)
    om = 0.1 * np.random.default_rng(8).normal(size=g.n)
    steps, dt = 100, 0.01
    h = [0.0, 1.0, 0.0, 0.2]
    want = oracle.poly_integrate(g.n, g.row_ptr, g.col, om, 4.0, h, DZ_F, x0, dt, steps,
                                 stepper="rk4" if stepper == 0 else "euler")
    for precision in (1, 0):
        for method in (0, 1):
            plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, om, K=4.0, h=h, f=DZ_F, method=method,
                                 precision=precision, stepper=stepper)
            x = torch.as_tensor(x0, dtype=torch.float64 if precision else torch.float32, device="cuda")
            plan.integrate(x, dt, steps)
            d = np.abs(x.cpu().numpy().astype(np.float64) - want).max()
            say("stepper", stepper, "prec", precision, "method", method, "max |dx|", d)
            assert d < (1e-10 if precision else 1e-4)
            plan.close()


def test_poly_rejects_trace_and_bad_degree(env):
    cia, torch = env
    P = W.kuramoto_small()
    g = P.graph
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, h=[0.0, 1.0])
    x = torch.zeros(g.n, dtype=torch.float32, device="cuda")
    with pytest.raises(cia.CIAError):
        plan.integrate(x, 0.01, 2, np.zeros(3))
    plan.close()
    with pytest.raises(cia.CIAError):
        cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, h=np.zeros(10))   # degree 9


def test_poly_full_size_sampled_rows(env):
    """The N = 1e6 power-law community graph of the phase bench, Desai-Zwanzig
    coupling, FP32: sampled rows against the oracle."""
    cia, torch = env
    P = W.kuramoto_large()
    g = P.graph
    x = np.random.default_rng(9).uniform(-1.5, 1.5, g.n)
    for method in (0, 1):
        plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=3.0, h=[0.0, 1.0], method=method)
        got, xr = gpu_rhs(env, plan, x, 0)
        rows = np.sort(np.random.default_rng(10).choice(g.n, 2000, replace=False))
        want = oracle.poly_rhs(g.n, g.row_ptr, g.col, None, 3.0, [0.0, 1.0], None, xr, rows=rows)
        err = coupling_err(got[rows], want, 0.0)
        say("N = 1e6 method", method, "sampled coupling rel_inf", err)
        assert err < 1e-5
        plan.close()


@pytest.mark.parametrize("graph", ["config1", "config2_scaled"])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_general_polynomial_coupling(env, graph, method, precision):
    """g(x_l, x_m) = sum c[a, b] x_l^a x_m^b (App. A.3, eq. PolyApprox), order 3,
    with the Desai-Zwanzig local term."""
    cia, torch = env
    P = W.kuramoto_small() if graph == "config1" else W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    rng = np.random.default_rng(40 + method)
    c = rng.normal(size=(4, 4)) / 4.0
    x = rng.uniform(-1.2, 1.2, g.n)
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, g=c, f=DZ_F, method=method,
                         precision=precision)
    got, xr = gpu_rhs(env, plan, x, precision)
    want = oracle.poly_rhs_general(g.n, g.row_ptr, g.col, None, 2.0, c, DZ_F, xr)
    base = xr - xr ** 3
    err = coupling_err(got, want, base)
    say("general poly", graph, "method", method, "prec", precision, "coupling rel_inf", err)
    assert err < (1e-12 if precision else 1e-5)
    plan.close()


def test_general_polynomial_complete_graph(env):
    cia, torch = env
    n = 5000
    rng = np.random.default_rng(41)
    c = rng.normal(size=(3, 3)) / 3.0
    x = rng.uniform(-1, 1, n)
    plan = cia.Plan.poly(n, complete=True, K=1.0, g=c, precision=1)
    got, _ = gpu_rhs(env, plan, x, 1)
    want = oracle.poly_rhs_general(n, None, None, None, 1.0, c, None, x, complete=True)
    assert coupling_err(got, want, 0.0) < 1e-12
    plan.close()


def test_poly_graph_replay_and_autotune(env):
    """The replayed RK4 step graph gives bitwise the eager trajectory, and
    the autotuner's re-cut units keep the right-hand side."""
    cia, torch = env
    P = W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    x0 = np.random.default_rng(50).uniform(-1, 1, g.n).astype(np.float32)
    outs = []
    for flags in (0, cia.CIA_FLAG_HIPGRAPH):
        plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, h=[0.0, 1.0, 0.0, -0.2], f=DZ_F,
                             flags=flags)
        x = torch.as_tensor(x0, device="cuda")
        plan.integrate(x, 0.01, 15)
        plan.integrate(x, 0.01, 15)
        outs.append(x.cpu().numpy())
        plan.close()
    assert np.array_equal(outs[0], outs[1])
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, h=[0.0, 1.0], f=DZ_F)
    a, _ = gpu_rhs(env, plan, x0, 0)
    rep = plan.autotune()
    b, _ = gpu_rhs(env, plan, x0, 0)
    assert rep.best_us <= rep.default_us and np.abs(a - b).max() <= 1e-6 * np.abs(a).max()
    plan.close()


def clique(n):
    col = np.array([j for i in range(n) for j in range(n) if j != i], np.int32)
    return np.arange(n + 1, dtype=np.int64) * (n - 1), col


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_poly_edge_cases(env, method, precision):
    """A single node without edges (labelled or not), every node outside any
    community, and one clique that is a single community (E1 alone, empty
    S-neg and S-pos)."""
    cia, torch = env
    tol = 1e-12 if precision else 1e-5
    for labels in (np.zeros(1, np.int32), None):
        om = np.array([0.3])
        plan = cia.Plan.poly(1, np.zeros(2, np.int64), np.zeros(0, np.int32), labels, om, K=2.0, h=[0.1, 1.0],
                             f=DZ_F, method=method, precision=precision)
        x = np.array([0.7])
        got, xr = gpu_rhs(env, plan, x, precision)
        assert abs(got[0] - (0.3 + xr[0] - xr[0] ** 3)) < tol
        plan.close()
    P = W.random_phase_problem(800, 0, seed=4, p_out=0.02, unassigned=800)
    g = P.graph
    x = np.random.default_rng(60).uniform(-1, 1, g.n)
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, h=[0.0, 1.0, 0.0, -0.3], method=method,
                         precision=precision)
    assert plan.info().n_unassigned == g.n
    got, xr = gpu_rhs(env, plan, x, precision)
    want = oracle.poly_rhs(g.n, g.row_ptr, g.col, None, 2.0, [0.0, 1.0, 0.0, -0.3], None, xr)
    assert coupling_err(got, want, 0.0) < tol
    plan.close()
    n = 300
    rp, col = clique(n)
    x = np.random.default_rng(61).uniform(-1, 1, n)
    plan = cia.Plan.poly(n, rp, col, np.zeros(n, np.int32), None, K=1.5, h=[0.2, 1.0, 0.5], f=DZ_F, method=method,
                         precision=precision)
    info = plan.info()
    assert method == 1 or (info.nnz_neg == 0 and info.nnz_pos == 0 and info.ncomm == 1)
    got, xr = gpu_rhs(env, plan, x, precision)
    want = oracle.poly_rhs(n, rp, col, None, 1.5, [0.2, 1.0, 0.5], DZ_F, xr)
    assert coupling_err(got, want, xr - xr ** 3) < tol
    plan.close()
