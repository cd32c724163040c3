"""Seeded sweep over random problem shapes: for each seed a random network
(size, number and sizes of communities, intra and inter densities, nodes
outside every community, Fourier order, unit size), method, precision and
model (phase difference form, general phase coupling, polynomial coupling
with one or two components), one right-hand side against the FP64 oracle.
The shapes cover single-slice and many-slice communities, ragged slice
tails, communities that P1's cost rule dissolves, and empty remainders."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

SEEDS = list(range(24))


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


def within(got, want, base, precision):
    """Coupling part C = want - base to a relative 1e-11 (FP64) or 1e-5
    (FP32) of its largest value, plus the rounding of the stored total: the
    kernel returns base + C in its own precision, and forming and storing that
    sum rounds it by a few units in the last place of |base + C| whatever the
    accuracy of C."""
    c = want - base
    e = np.abs((got - base) - c)
    tol, ulp = (1e-11, 2.0 ** -52) if precision else (1e-5, 2.0 ** -23)
    ok = bool(np.all(e <= tol * np.abs(c).max() + 4 * ulp * np.abs(want)))
    return ok, float(e.max() / max(np.abs(c).max(), 1e-300))


def problem(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(40, 6000))
    ncomm = int(rng.integers(0, 12))
    unassigned = int(rng.integers(0, n // 4 + 1)) if ncomm else n
    if ncomm > n - unassigned - 1:
        ncomm = max(0, n - unassigned - 1)
    p_in = float(rng.uniform(0.3, 1.0))
    p_out = float(rng.choice([0.0, 0.001, 0.01, 0.05]))
    P = W.random_phase_problem(n, ncomm, seed=2000 + seed, p_in=p_in, p_out=p_out, unassigned=unassigned)
    return rng, P


@pytest.mark.parametrize("seed", SEEDS)
def test_sweep(env, seed):
    cia, torch = env
    rng, P = problem(seed)
    g = P.graph
    method = int(rng.integers(0, 2))
    precision = int(rng.integers(0, 2))
    model = ["phase", "general", "poly", "osc2"][seed % 4]
    unit_work = int(rng.choice([0, 256, 4096, 65536]))
    dt = torch.float64 if precision else torch.float32
    # the kernels see omega in their own precision; so does the oracle here
    om = P.omega if precision else P.omega.astype(np.float32).astype(np.float64)
    say("seed", seed, "model", model, "n", g.n, "method", method, "prec", precision, "unit_work", unit_work)
    if model in ("phase", "general"):
        p = int(rng.integers(1, 5))
        th = rng.uniform(0, 2 * np.pi, g.n)
        if model == "phase":
            ds, dc = rng.normal(size=p + 1), rng.normal(size=p + 1)
            ds[0] = 0.0
            plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=2.5, d_sin=ds, d_cos=dc, method=method,
                                  precision=precision, unit_work=unit_work)
        else:
            cs = [rng.normal(size=(p + 1, p + 1)) / (p + 1) for _ in range(4)]
            plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=2.5, gen=cs, method=method,
                                  precision=precision, unit_work=unit_work)
        t = torch.as_tensor(th, dtype=dt, device="cuda")
        out = torch.empty_like(t)
        plan.rhs(t, out)
        torch.cuda.synchronize()
        got, thr = out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
        if model == "phase":
            want = oracle.phase_rhs(g.n, g.row_ptr, g.col, om, 2.5, ds, dc, thr)
        else:
            want = oracle.phase_rhs_general(g.n, g.row_ptr, g.col, om, 2.5, *cs, thr)
        ok, err = within(got, want, om, precision)
    elif model == "poly":
        p = int(rng.integers(1, 6))
        h = rng.normal(size=p + 1) / np.arange(1, p + 2)
        f = [0.0, 1.0, 0.0, -1.0]
        x = rng.uniform(-1.2, 1.2, g.n)
        plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, P.omega, K=2.5, h=h, f=f, method=method,
                             precision=precision, unit_work=unit_work)
        t = torch.as_tensor(x, dtype=dt, device="cuda")
        out = torch.empty_like(t)
        plan.rhs(t, out)
        torch.cuda.synchronize()
        got, xr = out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
        want = oracle.poly_rhs(g.n, g.row_ptr, g.col, om, 2.5, h, f, xr)
        ok, err = within(got, want, om + xr - xr ** 3, precision)
    else:
        h = [0.0, 1.0, 0.0, float(rng.uniform(-0.3, 0.3))]
        F = rng.normal(size=(2, 4, 4)) / 4.0
        x = rng.uniform(-1.2, 1.2, (2, g.n))
        plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, P.omega, K=2.5, h=h, dim=2, f2=F, method=method,
                             precision=precision, unit_work=unit_work)
        t = torch.as_tensor(x, dtype=dt, device="cuda")
        out = torch.empty_like(t)
        plan.rhs(t, out)
        torch.cuda.synchronize()
        got, xr = out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
        want = oracle.osc2_rhs(g.n, g.row_ptr, g.col, om, 2.5, h, F, xr)
        base = np.zeros_like(xr)
        for d in range(2):
            for i in range(4):
                for j in range(4):
                    base[d] += F[d, i, j] * xr[0] ** i * xr[1] ** j
        base[0] += om
        ok, err = within(got, want, base, precision)
    info = plan.info()
    say("   coupling rel_inf", err, "ncomm", info.ncomm, "unassigned", info.n_unassigned, "units", info.nunits)
    assert ok, (seed, err)
    plan.close()


@pytest.mark.parametrize("flags", [0x100, 0x200, 0x400, 0x600, 0x700])
@pytest.mark.parametrize("model", ["phase", "general", "poly", "osc2"])
def test_global_gather_paths(env, flags, model):
    """S-neg as int32 positions (FORCE_NEG32) and without LDS staging
    (NO_LDS): the global-gather paths that communities too large for LDS
    take, forced on a community graph, for every model on the stage kernels;
    with FORCE_WIDE the FP64-observable variants of the phase models (the
    polynomial models are FP64 in their moments anyway)."""
    cia, torch = env
    P = W.random_phase_problem(3000, 6, seed=3000 + flags, p_in=0.8, p_out=0.01, unassigned=40)
    g = P.graph
    rng = np.random.default_rng(flags)
    for precision in (0, 1):
        dt = torch.float64 if precision else torch.float32
        om = P.omega if precision else P.omega.astype(np.float32).astype(np.float64)
        if model in ("phase", "general"):
            th = rng.uniform(0, 2 * np.pi, g.n)
            if model == "phase":
                ds, dc = [0.0, 1.0, -0.4], [0.3, 0.2, 0.1]
                plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=2.0, d_sin=ds, d_cos=dc,
                                      precision=precision, flags=flags)
            else:
                cs = [rng.normal(size=(3, 3)) / 3 for _ in range(4)]
                plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=2.0, gen=cs,
                                      precision=precision, flags=flags)
            t = torch.as_tensor(th, dtype=dt, device="cuda")
            out = torch.empty_like(t)
            plan.rhs(t, out)
            torch.cuda.synchronize()
            got, thr = out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
            want = (oracle.phase_rhs(g.n, g.row_ptr, g.col, om, 2.0, ds, dc, thr) if model == "phase" else
                    oracle.phase_rhs_general(g.n, g.row_ptr, g.col, om, 2.0, *cs, thr))
            ok, err = within(got, want, om, precision)
        elif model == "poly":
            h = [0.1, 1.0, 0.0, -0.3]
            x = rng.uniform(-1, 1, g.n)
            plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, P.omega, K=2.0, h=h, precision=precision,
                                 flags=flags)
            t = torch.as_tensor(x, dtype=dt, device="cuda")
            out = torch.empty_like(t)
            plan.rhs(t, out)
            torch.cuda.synchronize()
            got, xr = out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
            want = oracle.poly_rhs(g.n, g.row_ptr, g.col, om, 2.0, h, None, xr)
            ok, err = within(got, want, om, precision)
        else:
            F = rng.normal(size=(2, 4, 4)) / 4.0
            x = rng.uniform(-1, 1, (2, g.n))
            plan = cia.Plan.poly(g.n, g.row_ptr, g.col, g.labels, P.omega, K=2.0, h=[0.0, 1.0], dim=2, f2=F,
                                 precision=precision, flags=flags)
            t = torch.as_tensor(x, dtype=dt, device="cuda")
            out = torch.empty_like(t)
            plan.rhs(t, out)
            torch.cuda.synchronize()
            got, xr = out.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
            want = oracle.osc2_rhs(g.n, g.row_ptr, g.col, om, 2.0, [0.0, 1.0], F, xr)
            base = np.zeros_like(xr)
            for d in range(2):
                for i in range(4):
                    for j in range(4):
                        base[d] += F[d, i, j] * xr[0] ** i * xr[1] ** j
            base[0] += om
            ok, err = within(got, want, base, precision)
        say("flags", hex(flags), model, "prec", precision, "coupling rel_inf", err, "ncomm", plan.info().ncomm)
        assert ok, (flags, model, precision, err)
        plan.close()
