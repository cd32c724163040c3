"""GPU parity of the two-component oscillators of the paper's Table 1 (van
der Pol / FitzHugh-Nagumo: f = (x2 - x1^3/3 + x1, -eps x1), h(xi) = xi on
each component) and of a general [2][4][4] local polynomial, against the FP64
oracle: single right-hand sides on planted-community graphs with nodes
outside every community, both methods and precisions, trajectories, graph
replay, the autotuner, and sampled rows at N = 1e6."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def vdp_F(eps):
    F = np.zeros((2, 4, 4))
    F[0, 0, 1] = 1.0
    F[0, 3, 0] = -1.0 / 3.0
    F[0, 1, 0] = 1.0
    F[1, 1, 0] = -eps
    return F


def fhn_F(eps, a, b, current):
    """FitzHugh-Nagumo: u' = u - u^3/3 - v + I, v' = eps (u + a - b v)."""
    F = np.zeros((2, 4, 4))
    F[0, 0, 0] = current
    F[0, 1, 0] = 1.0
    F[0, 3, 0] = -1.0 / 3.0
    F[0, 0, 1] = -1.0
    F[1, 0, 0] = eps * a
    F[1, 1, 0] = eps
    F[1, 0, 1] = -eps * b
    return F


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2203_16657_amd as cia
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cia.load()
    return cia, torch


def gpu_rhs(env, plan, x, precision):
    cia, torch = env
    dt = torch.float64 if precision else torch.float32
    t = torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    out = torch.empty_like(t)
    plan.rhs(t, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)


def coupling_err(got, want, base):
    c = want - base
    return float(np.abs((got - base) - c).max() / max(np.abs(c).max(), 1e-300))


def local_terms(F, x, omega):
    """f_d(u, v) + omega on component 0, for isolating the coupling error."""
    u, v = x[0], x[1]
    out = np.zeros_like(x)
    for d in range(2):
        for i in range(4):
            for j in range(4):
                out[d] += F[d, i, j] * u ** i * v ** j
    if omega is not None:
        out[0] += omega
    return out


@pytest.mark.parametrize("graph", ["config1", "config2_scaled"])
@pytest.mark.parametrize("model", ["vdp", "fhn", "random"])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_osc2_rhs(env, graph, model, method, precision):
    cia, torch = env
    P = W.kuramoto_small() if graph == "config1" else W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    rng = np.random.default_rng(70)
    x = rng.uniform(-1.5, 1.5, (2, g.n))
    om = 0.5 * rng.normal(size=g.n)
    if model == "vdp":
        F, h = vdp_F(0.3), [0.0, 1.0]
    elif model == "fhn":
        F, h = fhn_F(0.08, 0.7, 0.8, 0.5), [0.0, 1.0]
    else:
        F, h = rng.normal(size=(2, 4, 4)) / 4.0, [0.1, 1.0, -0.2, 0.3]
    K = 3.0
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, om, K=K, h=h, dim=2, f2=F, method=method,
                         precision=precision)
    got, xr = gpu_rhs(env, plan, x, precision)
    want = oracle.osc2_rhs(g.n, g.row_ptr, g.col, om, K, h, F, xr)
    err = coupling_err(got, want, local_terms(F, xr, om))
    tot = float(np.abs(got - want).max() / np.abs(want).max())
    say(graph, model, "method", method, "prec", precision, "coupling rel_inf", err, "total rel", tot)
    assert err < (1e-11 if precision else 1e-5)
    assert tot < (1e-12 if precision else 1e-6)
    plan.close()


@pytest.mark.parametrize("stepper", [0, 1])
def test_osc2_trajectory(env, stepper):
    """Coupled van der Pol oscillators, 100 steps of dt = 0.01."""
    cia, torch = env
    P = W.kuramoto_small()
    g = P.graph
    rng = np.random.default_rng(71)
    x0 = rng.uniform(-2.0, 2.0, (2, g.n))
    om = 0.1 * rng.normal(size=g.n)
    F, h, K, steps, dt = vdp_F(0.5), [0.0, 1.0], 4.0, 100, 0.01
    want = oracle.osc2_integrate(g.n, g.row_ptr, g.col, om, K, h, F, x0, dt, steps,
                                 stepper="rk4" if stepper == 0 else "euler")
    for precision in (1, 0):
        for method in (0, 1):
            plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, om, K=K, h=h, dim=2, f2=F, method=method,
                                 precision=precision, stepper=stepper)
            x = torch.as_tensor(x0, dtype=torch.float64 if precision else torch.float32, device="cuda")
            plan.integrate(x, dt, steps)
            d = np.abs(x.cpu().numpy().astype(np.float64) - want).max()
            say("stepper", stepper, "prec", precision, "method", method, "max |dx|", d)
            assert d < (1e-10 if precision else 2e-4)
            plan.close()


def test_osc2_graph_replay_and_autotune(env):
    cia, torch = env
    P = W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    x0 = np.random.default_rng(72).uniform(-1, 1, (2, g.n)).astype(np.float32)
    outs = []
    for flags in (0, cia.CIA_FLAG_HIPGRAPH):
        plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, h=[0.0, 1.0], dim=2, f2=vdp_F(0.3),
                             flags=flags)
        x = torch.as_tensor(x0, device="cuda")
        plan.integrate(x, 0.01, 15)
        plan.integrate(x, 0.01, 15)
        outs.append(x.cpu().numpy())
        plan.close()
    assert np.array_equal(outs[0], outs[1])
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, h=[0.0, 1.0], dim=2, f2=vdp_F(0.3))
    a, _ = gpu_rhs(env, plan, x0, 0)
    rep = plan.autotune()
    b, _ = gpu_rhs(env, plan, x0, 0)
    say("autotune", rep.default_us, rep.best_us)
    assert rep.best_us <= rep.default_us and np.abs(a - b).max() <= 1e-6 * np.abs(a).max()
    plan.close()


def test_osc2_rejects_unsupported(env):
    cia, torch = env
    g = W.kuramoto_small().graph
    with pytest.raises(cia.CIAError):
        cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, h=[0.0, 1.0], dim=2, f=[0.0, 1.0])
    with pytest.raises(cia.CIAError):
        cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, dim=2, g=np.eye(2))
    with pytest.raises(cia.CIAError):
        cia.Plan.poly(1000, complete=True, h=[0.0, 1.0], dim=2, method=1)   # all-to-all needs the CIA method
    with pytest.raises(cia.CIAError):
        cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, h=[0.0, 1.0], dim=3)


def test_osc2_full_size_sampled_rows(env):
    """The N = 1e6 power-law community graph, coupled van der Pol, FP32:
    sampled rows of both components against the oracle."""
    cia, torch = env
    g = W.kuramoto_large().graph
    x = np.random.default_rng(73).uniform(-1.5, 1.5, (2, g.n))
    F = vdp_F(0.3)
    rows = np.sort(np.random.default_rng(74).choice(g.n, 2000, replace=False))
    for method in (0, 1):
        plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=3.0, h=[0.0, 1.0], dim=2, f2=F,
                             method=method)
        got, xr = gpu_rhs(env, plan, x, 0)
        want = oracle.osc2_rhs(g.n, g.row_ptr, g.col, None, 3.0, [0.0, 1.0], F, xr, rows=rows)
        c = want - local_terms(F, xr[:, rows], None)
        err = np.abs(got[:, rows] - want)
        say("N = 1e6 method", method, "sampled coupling rel_inf", float(err.max() / np.abs(c).max()))
        # FP32 bound: the coupling to 1e-5 of its largest value, plus the
        # rounding of the stored right-hand side (a few units in the last place)
        assert np.all(err <= 1e-5 * np.abs(c).max() + 4 * 2.0 ** -24 * np.abs(want))
        plan.close()


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_osc2_edge_cases(env, method, precision):
    """A single node without edges, every node outside any community, and one
    clique that is a single community (E1 alone)."""
    cia, torch = env
    tol = 1e-11 if precision else 1e-5
    F = fhn_F(0.08, 0.7, 0.8, 0.5)
    for labels in (np.zeros(1, np.int32), None):
        plan = cia.Plan.poly(1, np.zeros(2, np.int64), np.zeros(0, np.int32), labels, np.array([0.2]), K=2.0,
                             h=[0.0, 1.0], dim=2, f2=F, method=method, precision=precision)
        got, xr = gpu_rhs(env, plan, np.array([[0.4], [-0.3]]), precision)
        want = local_terms(F, xr, np.array([0.2]))
        assert np.abs(got - want).max() < tol * max(1.0, np.abs(want).max())
        plan.close()
    P = W.random_phase_problem(800, 0, seed=4, p_out=0.02, unassigned=800)
    g = P.graph
    x = np.random.default_rng(75).uniform(-1, 1, (2, g.n))
    plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, h=[0.0, 1.0], dim=2, f2=F, method=method,
                         precision=precision)
    got, xr = gpu_rhs(env, plan, x, precision)
    want = oracle.osc2_rhs(g.n, g.row_ptr, g.col, None, 2.0, [0.0, 1.0], F, xr)
    assert coupling_err(got, want, local_terms(F, xr, None)) < tol
    plan.close()
    n = 300
    col = np.array([j for i in range(n) for j in range(n) if j != i], np.int32)
    rp = np.arange(n + 1, dtype=np.int64) * (n - 1)
    x = np.random.default_rng(76).uniform(-1, 1, (2, n))
    plan = cia.Plan.poly(n, rp, col, np.zeros(n, np.int32), None, K=1.5, h=[0.1, 1.0, 0.3], dim=2, f2=vdp_F(0.3),
                         method=method, precision=precision)
    got, xr = gpu_rhs(env, plan, x, precision)
    want = oracle.osc2_rhs(n, rp, col, None, 1.5, [0.1, 1.0, 0.3], vdp_F(0.3), xr)
    assert coupling_err(got, want, local_terms(vdp_F(0.3), xr, None)) < tol
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_osc2_complete_graph(env, precision):
    """All-to-all coupled van der Pol and FitzHugh-Nagumo oscillators (one
    community, E1 alone) against the oracle's pair sum, one RHS and an RK4
    trajectory."""
    cia, torch = env
    n = 3000
    rng = np.random.default_rng(77)
    x = rng.uniform(-2, 2, (2, n))
    om = 0.3 * rng.normal(size=n)
    for F, h in ((vdp_F(0.4), [0.0, 1.0]), (fhn_F(0.08, 0.7, 0.8, 0.5), [0.0, 1.0, 0.0, -0.1])):
        plan = cia.Plan.poly(n, complete=True, omega=om, K=1.5, h=h, dim=2, f2=F, precision=precision)
        got, xr = gpu_rhs(env, plan, x, precision)
        want = oracle.osc2_rhs(n, None, None, om, 1.5, h, F, xr, complete=True)
        err = coupling_err(got, want, local_terms(F, xr, om))
        say("complete prec", precision, "coupling rel_inf", err)
        assert err < (1e-12 if precision else 1e-5)
        plan.close()
    if precision:
        n = 400
        x0 = rng.uniform(-2, 2, (2, n))
        F = vdp_F(0.4)
        rp = np.arange(n + 1, dtype=np.int64) * (n - 1)
        col = np.array([j for i in range(n) for j in range(n) if j != i], np.int32)
        want = oracle.osc2_integrate(n, rp, col, None, 1.5, [0.0, 1.0], F, x0, 0.01, 50)
        plan = cia.Plan.poly(n, complete=True, K=1.5, h=[0.0, 1.0], dim=2, f2=F, precision=1)
        xt = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
        plan.integrate(xt, 0.01, 50)
        d = float(np.abs(xt.cpu().numpy() - want).max())
        say("complete trajectory max |dx|", d)
        assert d < 1e-11
        plan.close()
