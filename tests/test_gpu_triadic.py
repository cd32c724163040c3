"""GPU parity of the higher-order (triadic) Kuramoto path against the FP64
oracle (App. A.7 on a hypergraph: seeded intra-community triples plus listed
cross-community triples, pairwise sine coupling)."""
import sys

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


def rel_inf(got, want):
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


def plan_for(cia, T, method, precision=0, **kw):
    g = T.graph
    return cia.Plan.triadic(g.n, g.row_ptr, g.col, g.labels, None, K1=T.K1, K2=T.K2, tri_seed=T.tri_seed,
                            p_tri=T.p_tri, cross_tri=T.cross_tri, method=method, precision=precision, **kw)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_triadic_rhs_small(env, method, precision):
    cia, torch = env
    T = W.triadic(seed=31, n=1500, lo=60, hi=400, tri_per_node=1.0)
    g = T.graph
    say("triadic rhs n", g.n, "comms", g.ncomm, "method", method, "prec", precision)
    plan = plan_for(cia, T, method, precision)
    dt = torch.float64 if precision else torch.float32
    th = torch.as_tensor(T.theta0, dtype=dt, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    torch.cuda.synchronize()
    info = plan.info()
    th64 = th.cpu().numpy().astype(np.float64)
    got = out.cpu().numpy().astype(np.float64)
    want = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, T.tri_seed, T.p_tri, T.cross_tri, None,
                              T.K1, T.K2, th64)
    err = rel_inf(got, want)
    say("   rel_inf", err, "missing pairs", info.nnz_extra)
    assert err < (1e-12 if precision else 1e-5)
    if method == 0:
        assert info.nnz_extra > 0
    plan.close()


def test_triadic_p_tri_extremes(env):
    """p_tri = 1: no missing triples (E2 empty); p_tri = 0: no intra triples."""
    cia, torch = env
    for p in (1.0, 0.0):
        T = W.triadic(seed=7, n=900, lo=40, hi=200, p_tri=p, tri_per_node=0.5)
        g = T.graph
        plan = plan_for(cia, T, 0, 1)
        th = torch.as_tensor(T.theta0, dtype=torch.float64, device="cuda")
        out = torch.empty_like(th)
        plan.rhs(th, out)
        got = out.cpu().numpy()
        want = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, T.tri_seed, T.p_tri, T.cross_tri, None,
                                  T.K1, T.K2, T.theta0)
        say("p_tri", p, rel_inf(got, want), plan.info().nnz_extra)
        assert rel_inf(got, want) < 1e-12
        plan.close()


def test_triadic_trajectory(env):
    cia, torch = env
    T = W.triadic(seed=12, n=600, lo=40, hi=150, tri_per_node=1.0)
    g = T.graph
    steps = 60
    want_th, want_r = oracle.triadic_integrate(g.n, g.row_ptr, g.col, g.labels, T.tri_seed, T.p_tri,
                                               T.cross_tri, T.omega, T.K1, T.K2, T.theta0, T.dt, steps)
    for method in (0, 1):
        plan = cia.Plan.triadic(g.n, g.row_ptr, g.col, g.labels, T.omega, K1=T.K1, K2=T.K2,
                                tri_seed=T.tri_seed, p_tri=T.p_tri, cross_tri=T.cross_tri, method=method,
                                precision=1)
        th = torch.as_tensor(T.theta0, dtype=torch.float64, device="cuda")
        r = np.zeros(steps + 1)
        plan.integrate(th, T.dt, steps, r)
        circ = np.abs(np.angle(np.exp(1j * (th.cpu().numpy() - want_th))))
        say("triadic traj method", method, circ.max(), np.abs(r - want_r).max())
        assert circ.max() < 1e-9 and np.abs(r - want_r).max() < 1e-9
        plan.close()


def test_triadic_rejects_intra_listed_triangle(env):
    cia, torch = env
    T = W.triadic(seed=5, n=300, lo=40, hi=100, tri_per_node=0.2)
    g = T.graph
    lab = g.labels
    c0 = np.flatnonzero(lab == lab[lab >= 0][0])[:3]
    bad = np.vstack([T.cross_tri, np.sort(c0)[None, :]])
    with pytest.raises(cia.CIAError) as e:
        cia.Plan.triadic(g.n, g.row_ptr, g.col, g.labels, None, K1=1, K2=1, tri_seed=T.tri_seed, p_tri=T.p_tri,
                         cross_tri=bad)
    assert "inside one community" in cia.cia_last_error()


@pytest.mark.parametrize("precision", [0, 1])
def test_triadic_missing_pair_count(env, precision):
    """The missing-pair lists built on the device hold exactly three partner
    pairs per intra-community triple that is not a hyperedge (counted here
    with the oracle's predicate over every triple of every community)."""
    cia, torch = env
    T = W.triadic(seed=5, n=300, lo=40, hi=100, tri_per_node=0.2)
    g = T.graph
    plan = plan_for(cia, T, 0, precision)
    missing = 0
    for c in np.unique(g.labels[g.labels >= 0]):
        mem = [int(u) for u in np.flatnonzero(g.labels == c)]
        for a in range(len(mem)):
            for b in range(a + 1, len(mem)):
                for d in range(b + 1, len(mem)):
                    missing += not oracle.triple_present(T.tri_seed, T.p_tri, mem[a], mem[b], mem[d])
    say("missing triples", missing, "stored pairs", plan.info().nnz_extra)
    assert missing > 0 and plan.info().nnz_extra == 3 * missing
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_triadic_config3_community_sizes(env, precision):
    """The config-3 recipe (sizes U[200, 2000], pairwise p_in 0.9 and inter
    degree 3, intra triples with p = 0.9, 3 cross triples per node on
    average) at N = 6000; CIA against the oracle on sampled rows."""
    cia, torch = env
    T = W.triadic(seed=3, n=6000)
    g = T.graph
    say("config-3 sizes: n", g.n, "communities", g.ncomm, "precision", precision)
    plan = plan_for(cia, T, 0, precision)
    dt = torch.float64 if precision else torch.float32
    th = torch.as_tensor(T.theta0, dtype=dt, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(0).choice(g.n, 150, replace=False)
    want = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, T.tri_seed, T.p_tri, T.cross_tri, None, T.K1,
                              T.K2, th.cpu().numpy().astype(np.float64), rows=rows)
    err = rel_inf(got[rows], want)
    say("   missing pairs", plan.info().nnz_extra, "rel_inf", err)
    assert err < (1e-12 if precision else 1e-5)
    plan.close()


def test_triadic_full_size_direct(env):
    """Config 3 at full size (N = 1e5, 91 communities of U[200, 2000]): the
    direct method (present hyperedges enumerated on the GPU with the
    predicate) against the oracle on sampled rows."""
    cia, torch = env
    T = W.triadic(seed=3, n=100_000)
    g = T.graph
    say("config 3: n", g.n, "communities", g.ncomm, "pairwise nnz", g.nnz, "cross triples", len(T.cross_tri))
    plan = plan_for(cia, T, 1, 0)
    th = torch.as_tensor(T.theta0, dtype=torch.float32, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(1).choice(g.n, 60, replace=False)
    want = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, T.tri_seed, T.p_tri, T.cross_tri, None, T.K1,
                              T.K2, th.cpu().numpy().astype(np.float64), rows=rows)
    err = rel_inf(got[rows], want)
    say("   rel_inf", err)
    assert err < 1e-5
    plan.close()


def test_triadic_full_size_cia(env):
    """Config 3 at full size (N = 1e5, 91 communities of U[200, 2000], about
    1e10 stored missing pairs built on the device): CIA against the oracle on
    sampled rows, then RK4 steps stay finite."""
    cia, torch = env
    T = W.triadic(seed=3, n=100_000)
    g = T.graph
    plan = plan_for(cia, T, 0, 0)
    info = plan.info()
    say("config 3 CIA: n", g.n, "missing pairs", info.nnz_extra, "list GB", info.bytes_aux / 1e9)
    th = torch.as_tensor(T.theta0, dtype=torch.float32, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(2).choice(g.n, 60, replace=False)
    want = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, T.tri_seed, T.p_tri, T.cross_tri, None, T.K1,
                              T.K2, th.cpu().numpy().astype(np.float64), rows=rows)
    err = rel_inf(got[rows], want)
    say("   rel_inf", err)
    assert err < 1e-5
    plan.integrate(th, T.dt, 2)
    assert torch.isfinite(th).all().item()
    plan.close()


@pytest.mark.parametrize("precision,lam", [(0, 8191), (1, 4095)])
def test_triadic_largest_listed_community(env, precision, lam):
    """One community of the largest size whose missing-pair lists fit 16-bit
    LDS offsets (8191 nodes in FP32, 4095 in FP64), few missing triples:
    CIA against the oracle on sampled rows."""
    cia, torch = env
    T = W.triadic(seed=9, n=lam, lo=lam, hi=lam, p_tri=0.999, tri_per_node=0.0)
    g = T.graph
    assert g.ncomm == 1
    plan = plan_for(cia, T, 0, precision)
    info = plan.info()
    dt = torch.float64 if precision else torch.float32
    th = torch.as_tensor(T.theta0, dtype=dt, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(3).choice(g.n, 6, replace=False)
    want = oracle.triadic_rhs(g.n, g.row_ptr, g.col, g.labels, T.tri_seed, T.p_tri, T.cross_tri, None, T.K1,
                              T.K2, th.cpu().numpy().astype(np.float64), rows=rows)
    err = rel_inf(got[rows], want)
    say("community", lam, "precision", precision, "missing pairs", info.nnz_extra, "rel_inf", err)
    assert info.nnz_extra > 0
    assert err < (1e-12 if precision else 1e-5)
    plan.close()


@pytest.mark.parametrize("precision,lam", [(0, 8192), (1, 4096)])
def test_triadic_community_above_list_limit(env, precision, lam):
    cia, torch = env
    T = W.triadic(seed=9, n=lam, lo=lam, hi=lam, p_tri=0.999, tri_per_node=0.0)
    with pytest.raises(cia.CIAError):
        plan_for(cia, T, 0, precision)
    assert "communities of up to %d nodes" % (lam - 1) in cia.cia_last_error()


@pytest.mark.parametrize("method", [0, 1])
def test_triadic_graph_replay_matches_eager(env, method):
    """The replayed RK4 step graph (pair-sum and stage launches captured
    once) gives bitwise the eager result, over two integrate calls."""
    cia, torch = env
    T = W.triadic(seed=14, n=2500, lo=200, hi=600, tri_per_node=1.0)
    g = T.graph
    outs = []
    for flags in (0, cia.CIA_FLAG_HIPGRAPH):
        plan = cia.Plan.triadic(g.n, g.row_ptr, g.col, g.labels, T.omega, K1=T.K1, K2=T.K2, tri_seed=T.tri_seed,
                                p_tri=T.p_tri, cross_tri=T.cross_tri, method=method, flags=flags)
        th = torch.as_tensor(T.theta0, dtype=torch.float32, device="cuda")
        r = np.zeros(2 * 21)
        plan.integrate(th, T.dt, 20, r[:21])
        plan.integrate(th, T.dt, 20, r[21:])
        outs.append((th.cpu().numpy(), r))
        plan.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
