"""GPU parity of the Cucker-Smale path (App. A.6) against the FP64 oracle:
the exact fallback and the direct method against the plain sum, the Fourier
basis against the oracle's own Fourier coefficients, the learned basis (bf16
matrix-core features, forward and backward) against the oracle's FP64
perceptron, the judge, and trajectories."""
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


def coupling_err(got_v, want_v):
    """coupling-only max-norm error relative to the largest reference entry"""
    return float(np.abs(got_v - want_v).max() / max(np.abs(want_v).max(), 1e-300))


def small_flock(seed, n=3000, ncomm=None, sizes=None, p_in=0.8, inter_deg=4.0, unassigned=0, box=10.0):
    """Equal or given community sizes, p_in, uniform inter edges, a tail of
    unassigned nodes; positions U[0, box]^3, velocities N(0, 1)."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = np.full(ncomm, (n - unassigned) // ncomm, dtype=np.int64)
        sizes[: (n - unassigned) - int(sizes.sum())] += 1
    sizes = np.asarray(sizes, dtype=np.int64)
    labels = W.shuffled_labels(sizes, n, rng)
    g = W.sbm(labels, len(sizes), p_in, n_inter=int(round(inter_deg * n / 2)), seed=seed)
    x = rng.uniform(0.0, box, (3, n))
    v = rng.standard_normal((3, n))
    return g, x, v


def state_tensor(torch, x, v):
    return torch.as_tensor(np.concatenate([x, v]).astype(np.float32), device="cuda").contiguous()


def run_rhs(torch, plan, st):
    out = torch.empty_like(st)
    plan.rhs(st, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def random_mlp(R, seed, scale=0.5):
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=scale, size=oracle.mlp_param_count(R)).astype(np.float32)
    p[-R:] = 1.0
    return p


@pytest.mark.parametrize("method", [0, 1])
def test_flock_exact_rhs(env, method):
    cia, torch = env
    g, x, v = small_flock(41, n=3000, ncomm=12, unassigned=137)
    say("flock exact rhs n", g.n, "method", method)
    plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, method=method)
    st = state_tensor(torch, x, v)
    got = run_rhs(torch, plan, st)
    s64 = st.cpu().numpy().astype(np.float64)
    sd, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s64[:3], s64[3:])
    assert np.array_equal(got[:3], sd)
    err = coupling_err(got[3:], vd)
    say("   coupling rel_inf", err, "units", plan.info().nunits)
    assert err < 1e-5


@pytest.mark.parametrize("sigma,beta", [(1.0, 0.25), (1e-30, 0.25), (1e-20, 0.5), (0.01, 10.0)])
def test_flock_exact_kernel_paths(env, sigma, beta):
    """The exact-path kernel's cases: a community above the LDS staging cap
    (4500 members, read from global memory with per-row S-neg lists) beside
    staged ones whose sizes leave 1 to 3 members after the groups of four,
    rows of no community.  s2 = 1 takes the unclamped weight-sum loop; an s2
    that is 0 in FP32 (sigma = 1e-30), a denormal s2 (1e-40) and an
    s2^(-beta) beyond the FP32 range (1e-4 to the power -10) take the clamped
    loop with the self pair masked."""
    cia, torch = env
    g, x, v = small_flock(49, n=5131, sizes=[4500, 333, 250, 7], p_in=[0.8, 0.7, 0.9, 1.0], inter_deg=2.0,
                          unassigned=41)
    st = state_tensor(torch, x, v)
    s64 = st.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(3).choice(g.n, 1500, replace=False)
    _, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, 1.7, sigma, beta, s64[:3], s64[3:], rows=rows)
    plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, K=1.7, sigma=sigma, beta=beta)
    got = run_rhs(torch, plan, st)
    err = coupling_err(got[3:, rows], vd)
    say("exact kernel paths sigma", sigma, "beta", beta, "ncomm", plan.info().ncomm, "rel_inf", err)
    assert plan.info().ncomm == 4 and err < 1e-5


def test_flock_edge_cases(env):
    cia, torch = env
    # one community of a single node, one dissolved by the cost rule (p_in tiny),
    # and a graph with no edges at all
    sizes = [1, 40, 300, 5]
    g, x, v = small_flock(42, n=400, sizes=sizes, p_in=[0.9, 0.02, 0.8, 1.0], inter_deg=1.0)
    st = state_tensor(torch, x, v)
    s64 = st.cpu().numpy().astype(np.float64)
    _, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s64[:3], s64[3:])
    for basis in (0, 1):
        plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=basis, flags=0)
        got = run_rhs(torch, plan, st)
        say("edge basis", basis, "ncomm", plan.info().ncomm, "unassigned", plan.info().n_unassigned)
        # Fourier basis under the judge falls back wherever it is inaccurate
        assert coupling_err(got[3:], vd) < (1e-5 if basis == 0 else 1e-3)
    e_rp = np.zeros(401, dtype=np.int64)
    plan = cia.Plan.flock(400, e_rp, np.zeros(0, dtype=np.int32), g.labels)
    got = run_rhs(torch, plan, st)
    assert np.abs(got[3:]).max() == 0.0
    with pytest.raises(cia.CIAError):
        cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=2, rank=20)
    with pytest.raises(cia.CIAError):
        cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=1, p=3)


@pytest.mark.parametrize("p", [1, 2])
def test_flock_fourier_rhs(env, p):
    cia, torch = env
    g, x, v = small_flock(43, n=2500, ncomm=10, unassigned=50)
    L = 20.0
    plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=1, p=p, L=L, flags=cia.CIA_FLAG_NO_JUDGE)
    assert plan.info().ncomm == 10
    st = state_tensor(torch, x, v)
    got = run_rhs(torch, plan, st)
    s64 = st.cpu().numpy().astype(np.float64)
    c = oracle.cs_fourier_coeffs(1.0, 1.0, 0.25, L, p, nq=64)
    _, vd = oracle.cs_rhs_separable(g.n, g.row_ptr, g.col, g.labels, 1.0, 1.0, 0.25, s64[:3], s64[3:], "fourier",
                                    fourier=c, L=L)
    err = coupling_err(got[3:], vd)
    say("fourier p", p, "coupling rel_inf vs separable oracle", err)
    assert err < 1e-5
    # features of the basis itself
    xs = torch.as_tensor(x.astype(np.float32), device="cuda").contiguous()
    stride = ((2 * p + 1) ** 3 + 3) // 4 * 4
    F = torch.empty((g.n, stride), dtype=torch.float32, device="cuda")
    plan.basis_features(xs, F)
    torch.cuda.synchronize()
    Fh = F.cpu().numpy().astype(np.float64)
    assert np.all(Fh[:, 0] == 1.0) and np.all(Fh[:, (2 * p + 1) ** 3:] == 0.0)
    # the separable form reproduces the series at a few pairs
    rng = np.random.default_rng(0)
    xs64 = xs.cpu().numpy().astype(np.float64)
    for _ in range(20):
        a, b = rng.integers(0, g.n, 2)
        y = xs64[:, b] - xs64[:, a]
        series = oracle.cs_fourier_weight(c, L, y)
        # reconstruct coefficients of the real form from the oracle cube
        w = c[0, 0, 0]
        h = 0
        for a1 in range(-p, p + 1):
            for a2 in range(-p, p + 1):
                for a3 in range(-p, p + 1):
                    if not (a1 > 0 or (a1 == 0 and (a2 > 0 or (a2 == 0 and a3 > 0)))):
                        continue
                    cf = 2 * c[abs(a1), abs(a2), abs(a3)]
                    w += cf * (Fh[a, 1 + 2 * h] * Fh[b, 1 + 2 * h] + Fh[a, 2 + 2 * h] * Fh[b, 2 + 2 * h])
                    h += 1
        assert abs(w - series) < 1e-5


@pytest.mark.parametrize("R", [16, 32, 64])
def test_mlp_features_match_oracle(env, R):
    cia, torch = env
    g, x, v = small_flock(44, n=1000, ncomm=4)
    plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=2, rank=R, flags=cia.CIA_FLAG_NO_JUDGE)
    params = random_mlp(R, 5)
    lo, hi = np.zeros(3), np.full(3, 10.0)
    plan.basis_set_params(params, lo, hi)
    n = 1000 - 37   # ragged against the 64-point tiles
    xs = torch.as_tensor(x[:, :n].astype(np.float32), device="cuda").contiguous()
    F = torch.full((n, R), 7.0, dtype=torch.float32, device="cuda")
    plan.basis_features(xs, F)
    torch.cuda.synchronize()
    got = F.cpu().numpy().astype(np.float64)
    want = oracle.mlp_forward(params.astype(np.float64), R, lo, hi, xs.cpu().numpy().astype(np.float64))
    err = np.abs(got - want).max() / np.abs(want).max()
    say("mlp features R", R, "rel err", err)
    # bf16 operands (8-bit significands) in layers 2 and 3, FP32 accumulation
    assert err < 2e-2
    pr, lo2, hi2 = plan.basis_get_params(len(params))
    assert np.array_equal(pr, params) and np.array_equal(lo2, lo) and np.array_equal(hi2, hi)


@pytest.mark.parametrize("R,P", [(32, 1000), (16, 4096), (64, 77)])
def test_mlp_loss_grad_match_oracle(env, R, P):
    cia, torch = env
    g, x, v = small_flock(45, n=500, ncomm=2)
    plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=2, rank=R, flags=cia.CIA_FLAG_NO_JUDGE)
    params = random_mlp(R, 6, scale=0.4)
    lo, hi = np.zeros(3), np.full(3, 10.0)
    plan.basis_set_params(params, lo, hi)
    rng = np.random.default_rng(7)
    a = rng.uniform(0, 10, (P, 3)).astype(np.float32)
    b = rng.uniform(0, 10, (P, 3)).astype(np.float32)
    t = ((1 + ((a.astype(np.float64) - b) ** 2).sum(1)) ** -0.25).astype(np.float32)
    da, db, dtt = (torch.as_tensor(z, device="cuda").contiguous() for z in (a, b, t))
    grad = torch.full((len(params),), 3.0, dtype=torch.float32, device="cuda")
    loss = plan.basis_loss_grad(da, db, dtt, grad)
    gg = grad.cpu().numpy().astype(np.float64)
    lw, gw = oracle.mlp_loss_grad(params.astype(np.float64), R, lo, hi, a, b, t)
    say("loss grad R", R, "P", P, "loss", loss, lw)
    assert abs(loss - lw) < 2e-2 * lw
    assert np.all(gg[-R:] == 0.0)
    tot = np.linalg.norm(gg - gw) / np.linalg.norm(gw)
    say("   grad rel l2", tot)
    assert tot < 3e-2
    o = [0, 192, 256, 256 + 4096, 256 + 4096 + 64, 256 + 4096 + 64 + R * 64, 256 + 4096 + 64 + R * 64 + R]
    for k in range(6):
        blk = slice(o[k], o[k + 1])
        e = np.linalg.norm(gg[blk] - gw[blk]) / np.linalg.norm(gw[blk])
        say("   block", k, "rel l2", e)
        assert e < 6e-2


def test_flock_learned_rhs_matches_separable_oracle(env):
    cia, torch = env
    g, x, v = small_flock(46, n=2400, ncomm=8, unassigned=31)
    R = 32
    plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=2, rank=R, flags=cia.CIA_FLAG_NO_JUDGE)
    params = random_mlp(R, 8, scale=0.3)
    lo, hi = np.zeros(3), np.full(3, 10.0)
    plan.basis_set_params(params, lo, hi)
    st = state_tensor(torch, x, v)
    got = run_rhs(torch, plan, st)
    s64 = st.cpu().numpy().astype(np.float64)
    _, vd = oracle.cs_rhs_separable(g.n, g.row_ptr, g.col, g.labels, 1.0, 1.0, 0.25, s64[:3], s64[3:], "mlp",
                                    mlp=params.astype(np.float64), R=R, lo=lo, hi=hi)
    err = coupling_err(got[3:], vd)
    say("learned rhs vs separable oracle", err)
    assert err < 2e-2
    # momentum: the expanded weight is symmetric and the graph undirected
    mom = np.abs(got[3:].sum(1)).max() / np.abs(got[3:]).sum()
    say("   momentum residual", mom)
    assert mom < 1e-5


def test_flock_training_gain_and_judge(env):
    """Config-4 shape at 1/20 scale: 20 communities of 500, p_in 0.8, inter
    degree 4, x ~ U[0,10]^3.  The trained rank-32 basis beats the Fourier basis
    of the paper at comparable rank (p = 1: 27 features) and the judge sends
    every community whose sampled error exceeds the bound to the exact path."""
    cia, torch = env
    g, x, v = small_flock(47, n=10000, ncomm=20)
    st = state_tensor(torch, x, v)
    s64 = st.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(1).choice(g.n, 1500, replace=False)
    _, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s64[:3], s64[3:], rows=rows)
    plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=2, rank=32, flags=cia.CIA_FLAG_NO_JUDGE)
    lt = np.zeros(3000)
    plan.basis_train(st, 3000, seed=11, loss_trace=lt)
    say("train loss first/last", lt[:5].mean(), lt[-100:].mean())
    assert lt[-100:].mean() < 0.05 * lt[:5].mean()
    err_l = coupling_err(run_rhs(torch, plan, st)[3:, rows], vd)
    fplan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=1, p=1, flags=cia.CIA_FLAG_NO_JUDGE)
    err_f = coupling_err(run_rhs(torch, fplan, st)[3:, rows], vd)
    say("learned rank 32 err", err_l, "fourier p=1 err", err_f, "gain", err_f / err_l)
    assert err_l < 2e-2
    assert err_f > 5 * err_l
    # Eckart-Young: no rank-32 symmetric separable weight beats the truncated
    # eigendecomposition of a community's weight matrix
    members = np.flatnonzero(g.labels == 0)
    xm = s64[:3, members]
    Wc = (1.0 + ((xm[:, :, None] - xm[:, None, :]) ** 2).sum(0)) ** -0.25
    ev = np.linalg.eigvalsh(Wc)
    floor = np.sqrt(np.sort(ev ** 2)[:-32].sum())
    Fm = torch.empty((len(members), 32), dtype=torch.float32, device="cuda")
    plan.basis_features(torch.as_tensor(xm.astype(np.float32), device="cuda").contiguous(), Fm)
    torch.cuda.synchronize()
    Fh = Fm.cpu().numpy().astype(np.float64)
    learned_fro = np.linalg.norm(Fh @ Fh.T - Wc)
    say("community 0: rank-32 Eckart-Young floor", floor, "learned", learned_fro, "ratio", learned_fro / floor)
    assert learned_fro >= floor * (1 - 1e-9)
    # judge: an untrained basis fails everywhere, so every community takes the
    # exact path; the trained one fails a tight bound (rank 32 cannot reach
    # 1e-3 here) and passes a loose one
    params, lo, hi = plan.basis_get_params(oracle.mlp_param_count(32))
    cases = ((random_mlp(32, 9), 1e-3, "all"), (params, 1e-3, "most"), (params, 0.5, "none"))
    for prm, tol, want in cases:
        jp = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=2, rank=32, judge_tol=tol)
        jp.basis_set_params(prm, lo, hi)
        got = run_rhs(torch, jp, st)[3:, rows]
        fbk = jp.info().judge_fallbacks
        err = coupling_err(got, vd)
        say("judge tol", tol, "case", want, "fallbacks", fbk, "of", jp.info().ncomm, "err", err)
        if want == "all":
            assert fbk == 20 and err < 1e-5
        elif want == "most":
            assert fbk >= 15 and err < err_l
        else:
            assert fbk == 0 and abs(err - err_l) < 1e-6


@pytest.mark.parametrize("stepper", [0, 1])
def test_flock_trajectory(env, stepper):
    cia, torch = env
    g, x, v = small_flock(48, n=1500, ncomm=6, unassigned=20)
    steps, dt = 25, 0.01
    st = state_tensor(torch, x, v)
    s64 = st.cpu().numpy().astype(np.float64)
    want_s, want_v = oracle.cs_integrate(g.n, g.row_ptr, g.col, 1.0, 1.0, 0.25, s64[:3], s64[3:], dt, steps,
                                         stepper="euler" if stepper else "rk4")
    for method in (0, 1):
        plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, method=method, stepper=stepper)
        y = st.clone()
        plan.integrate(y, dt, steps)
        torch.cuda.synchronize()
        got = y.cpu().numpy().astype(np.float64)
        # positions are stored in FP32 and rounded at every step (up to
        # steps * 2^-24 * max|s| in all), so they are compared relative to max|s|
        es = np.abs(got[:3] - want_s).max() / np.abs(want_s).max()
        ev = np.abs(got[3:] - want_v).max() / np.abs(want_v).max()
        say("trajectory stepper", stepper, "method", method, "pos rel", es, "vel rel", ev)
        assert es < 1e-5 and ev < 1e-5


def test_flock_full_size_sampled_rows(env):
    """Config 4 at full size (N = 2e5, 400 x 500): exact fallback and direct
    method on sampled rows against the oracle."""
    cia, torch = env
    F = W.flock()
    g = F.graph
    st = state_tensor(torch, F.x0, F.v0)
    s64 = st.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(2).choice(g.n, 400, replace=False)
    _, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, F.K, F.sigma, F.beta, s64[:3], s64[3:], rows=rows)
    for method in (0, 1):
        plan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, method=method)
        got = run_rhs(torch, plan, st)
        err = coupling_err(got[3:, rows], vd)
        say("full size method", method, "err", err, "units", plan.info().nunits)
        assert err < 1e-5


def test_flock_learned_basis_full_size(env):
    """Config 4 at full size (N = 2e5, 400 x 500, rank 32): the basis trained
    on the GPU by the library's own kernels, without the judge, against the
    oracle on sampled rows (error below 2e-2, at least 5x below the Fourier
    basis p = 1 of comparable rank, momentum conserved by the symmetric
    expansion); with the judge at 1e-3 every community falls back (no rank-32
    separable basis reaches 1e-3 per pair here, see the Eckart-Young floor
    test) and the result matches the exact sum to 1e-5."""
    cia, torch = env
    F = W.flock()
    g = F.graph
    st = state_tensor(torch, F.x0, F.v0)
    s64 = st.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(3).choice(g.n, 600, replace=False)
    _, vd = oracle.cs_rhs(g.n, g.row_ptr, g.col, F.K, F.sigma, F.beta, s64[:3], s64[3:], rows=rows)
    free = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=2, rank=32, flags=cia.CIA_FLAG_NO_JUDGE)
    lt = np.zeros(3000)
    free.basis_train(st, 3000, seed=11, loss_trace=lt)
    say("full-size training loss first/last", lt[:5].mean(), lt[-100:].mean())
    assert lt[-100:].mean() < 0.05 * lt[:5].mean()
    got = run_rhs(torch, free, st)
    err_l = coupling_err(got[3:, rows], vd)
    mom = np.abs(got[3:].sum(1)).max() / np.abs(got[3:]).sum()
    fplan = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=1, p=1, flags=cia.CIA_FLAG_NO_JUDGE)
    err_f = coupling_err(run_rhs(torch, fplan, st)[3:, rows], vd)
    say("full size learned err", err_l, "fourier p=1 err", err_f, "gain", err_f / err_l, "momentum", mom)
    assert err_l < 2e-2 and err_f > 5 * err_l and mom < 1e-5
    params, lo, hi = free.basis_get_params(oracle.mlp_param_count(32))
    judged = cia.Plan.flock(g.n, g.row_ptr, g.col, g.labels, basis=2, rank=32, judge_tol=1e-3)
    judged.basis_set_params(params, lo, hi)
    err_j = coupling_err(run_rhs(torch, judged, st)[3:, rows], vd)
    fbk = judged.info().judge_fallbacks
    say("full size judged: fallbacks", fbk, "of", judged.info().ncomm, "err", err_j)
    assert fbk == 400 and err_j < 1e-5
