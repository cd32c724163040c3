"""GPU parity of the general (non-difference) phase coupling g(theta_l,
theta_m), the real 2-D Fourier series of App. A.2, against the FP64 oracle:
community graphs with nodes outside every community, orders 1..8, both
methods and precisions, the complete graph (one community, also above 1e5
nodes on the FP64 observable path), the difference form as a special case,
and an RK4 trajectory."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


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


def coeffs(p, seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(p + 1, p + 1)) / (p + 1) for _ in range(4)]


def coupling_err(got, want):
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


def gpu_rhs(torch, plan, th, precision):
    t = torch.as_tensor(th, dtype=torch.float64 if precision else torch.float32, device="cuda")
    out = torch.empty_like(t)
    plan.rhs(t, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("graph", ["config1", "config2_scaled"])
@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_general_rhs(env, graph, p, method, precision):
    cia, torch = env
    P = W.kuramoto_small() if graph == "config1" else W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    cs = coeffs(p, 10 * p + method)
    th = np.random.default_rng(3).uniform(0, 2 * np.pi, g.n)
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, gen=cs, method=method, precision=precision)
    got, thr = gpu_rhs(torch, plan, th, precision)
    want = oracle.phase_rhs_general(g.n, g.row_ptr, g.col, None, 2.0, *cs, thr)
    err = coupling_err(got, want)
    say(graph, "p", p, "method", method, "prec", precision, "rel_inf", err)
    assert err < (1e-12 if precision else 1e-5)
    plan.close()


def test_difference_form_through_the_general_path(env):
    """The difference coupling given as a general one equals the difference plan."""
    cia, torch = env
    P = W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    ds, dc = [0.0, 1.0, -0.3], [0.2, 0.5, 0.1]
    p = 2
    c11, c12, c21, c22 = (np.zeros((p + 1, p + 1)) for _ in range(4))
    for k in range(p + 1):
        c11[k, k] = dc[k]
        if k:
            c22[k, k], c21[k, k], c12[k, k] = dc[k], ds[k], -ds[k]
    th = np.random.default_rng(4).uniform(0, 2 * np.pi, g.n)
    a = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, K=3.0, gen=(c11, c12, c21, c22), precision=1)
    b = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, K=3.0, d_sin=ds, d_cos=dc, precision=1)
    ga, _ = gpu_rhs(torch, a, th, 1)
    gb, _ = gpu_rhs(torch, b, th, 1)
    assert coupling_err(ga, gb) < 1e-12
    a.close()
    b.close()


@pytest.mark.parametrize("n", [4000, 150_000])
def test_general_complete_graph(env, n):
    """All-to-all (one community; above 1e5 nodes the FP32 plan sums the
    community observables in FP64), sampled rows against the oracle."""
    cia, torch = env
    cs = coeffs(2, 77)
    th = np.random.default_rng(5).uniform(0, 2 * np.pi, n)
    plan = cia.Plan.phase(n, complete=True, K=3.0, gen=cs)
    assert plan.info().wide_comms == (1 if n > 100_000 else 0)
    got, thr = gpu_rhs(torch, plan, th, 0)
    rows = np.random.default_rng(6).choice(n, 64, replace=False)
    want = oracle.phase_rhs_general(n, None, None, None, 3.0, *cs, thr, rows=rows, complete=True)
    err = coupling_err(got[rows], want)
    say("complete n", n, "rel_inf", err)
    assert err < 1e-5
    plan.close()


def test_general_trajectory(env):
    """FP64 RK4 against an RK4 loop over the oracle's general right-hand side."""
    cia, torch = env
    P = W.kuramoto_small()
    g = P.graph
    cs = coeffs(2, 88)
    om = P.omega
    th0 = P.theta0
    dt, steps = 0.01, 25

    def H(x):
        return oracle.phase_rhs_general(g.n, g.row_ptr, g.col, om, 4.0, *cs, x)

    x = th0.copy()
    for _ in range(steps):
        k1 = H(x)
        k2 = H(x + 0.5 * dt * k1)
        k3 = H(x + 0.5 * dt * k2)
        k4 = H(x + dt * k3)
        x = x + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    for method in (0, 1):
        plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, om, K=4.0, gen=cs, method=method, precision=1)
        t = torch.as_tensor(th0, dtype=torch.float64, device="cuda")
        plan.integrate(t, dt, steps)
        d = np.abs(np.angle(np.exp(1j * (t.cpu().numpy() - x)))).max()
        say("general trajectory method", method, "max circ", d)
        assert d < 1e-9
        plan.close()


def test_general_rejections(env):
    cia, torch = env
    P = W.kuramoto_small()
    g = P.graph
    with pytest.raises(cia.CIAError):
        cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, gen=coeffs(9, 1))      # order above 8
    with pytest.raises(cia.CIAError):
        cia.Plan.phase(1000, complete=True, gen=coeffs(1, 2), method=1)              # all-to-all direct kernel


def test_general_graph_replay(env):
    cia, torch = env
    P = W.kuramoto_small()
    g = P.graph
    cs = coeffs(2, 99)
    outs = []
    for flags in (0, cia.CIA_FLAG_HIPGRAPH):
        plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=4.0, gen=cs, flags=flags)
        t = torch.as_tensor(P.theta0.astype(np.float32), device="cuda")
        r = np.zeros(21)
        plan.integrate(t, 0.01, 20, r)
        outs.append((t.cpu().numpy(), r))
        plan.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
