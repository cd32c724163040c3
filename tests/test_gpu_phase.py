"""GPU parity of the phase-model path (CIA and direct) against the FP64 oracle.

Error metric for a single RHS: the coupling part C = H - omega, compared in
the infinity norm relative to the oracle's, with the oracle fed the same
FP32-rounded phases the GPU saw:  ||C_gpu - C_ref||_inf / ||C_ref||_inf.
Gates: 1e-5 for FP32 plans, 1e-12 for FP64 plans.  Phase trajectories are
compared by the circular difference, order parameters directly.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def gpu_rhs(env, P, method, precision, theta, omega=None, rows=None, **kw):
    cia, torch = env
    g = P.graph
    dt = torch.float64 if precision == cia.CIA_F64 else torch.float32
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, omega, K=P.K, d_sin=P.d_sin, d_cos=P.d_cos,
                          method=method, precision=precision, **kw)
    try:
        th = torch.as_tensor(theta, dtype=dt, device="cuda")
        out = torch.empty_like(th)
        plan.rhs(th, out)
        torch.cuda.synchronize()
        info = plan.info()
        return out.cpu().numpy().astype(np.float64), th.cpu().numpy().astype(np.float64), info
    finally:
        plan.close()


def check_rhs(env, P, method, precision, label, **kw):
    cia, torch = env
    g = P.graph
    say("case", label, "n", g.n, "method", method, "prec", precision, kw)
    theta = P.theta0
    got, th_used, info = gpu_rhs(env, P, method, precision, theta, omega=None, **kw)
    want = oracle.phase_rhs(g.n, g.row_ptr, g.col, None, P.K, P.d_sin, P.d_cos, th_used)
    err = rel_inf(got, want)
    tol = TOL64 if precision == cia.CIA_F64 else TOL32
    say("   rel_inf", err, "units", info.nunits, "ncomm", info.ncomm)
    assert err <= tol, (label, err)
    return info


@pytest.mark.parametrize("p", [1, 2, 4])
@pytest.mark.parametrize("method", [0, 1])
def test_rhs_random_small(env, p, method):
    cia, _ = env
    P = W.random_phase_problem(3000, 7, seed=100 + p, p_in=0.8, p_out=0.01, unassigned=53, p=p)
    for prec in (cia.CIA_F32, cia.CIA_F64):
        check_rhs(env, P, method, prec, "random p=%d" % p)


@pytest.mark.parametrize("flags", [0x100, 0x200, 0x400, 0x1])
def test_rhs_kernel_path_overrides(env, flags):
    """FP64-wide observables, int32 S-neg and global (non-LDS) gathers."""
    cia, _ = env
    P = W.random_phase_problem(2500, 5, seed=7, p_in=0.85, p_out=0.02, unassigned=11, p=2)
    check_rhs(env, P, cia.CIA_METHOD_CIA, cia.CIA_F32, "flags=%#x" % flags, flags=flags)


@pytest.mark.parametrize("unit_work,block", [(64, 256), (1000, 512), (1 << 20, 256)])
def test_rhs_unit_shapes(env, unit_work, block):
    """Ragged tails: many tiny units, large blocks, one unit per community."""
    cia, _ = env
    P = W.random_phase_problem(4100, 3, seed=17, p_in=0.9, p_out=0.005, unassigned=301, p=1)
    check_rhs(env, P, cia.CIA_METHOD_CIA, cia.CIA_F32, "units", unit_work=unit_work, block=block)


def test_rhs_adds_omega(env):
    cia, torch = env
    P = W.random_phase_problem(500, 3, seed=2, p=1)
    g = P.graph
    got, th, _ = gpu_rhs(env, P, cia.CIA_METHOD_CIA, cia.CIA_F64, P.theta0, omega=P.omega)
    want = oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, P.d_sin, P.d_cos, th)
    assert np.abs(got - want).max() < 1e-12


def test_edge_cases(env):
    cia, torch = env
    # single node, no edges
    for n, labels in ((1, np.zeros(1, np.int32)), (1, None), (5, np.full(5, -1, np.int32))):
        rp = np.zeros(n + 1, np.int64)
        col = np.zeros(0, np.int32)
        om = np.arange(n, dtype=np.float64) * 0.5
        for method in (0, 1):
            plan = cia.Plan.phase(n, rp, col, labels, om, K=2.0, method=method, precision=cia.CIA_F64)
            th = torch.zeros(n, dtype=torch.float64, device="cuda")
            out = torch.empty_like(th)
            plan.rhs(th, out)
            assert np.allclose(out.cpu().numpy(), om)
            r = np.zeros(3)
            plan.integrate(th, 0.1, 2, r)
            assert np.allclose(th.cpu().numpy(), np.mod(om * 0.2, 2 * np.pi))
            plan.close()
    # every node outside any community
    P = W.random_phase_problem(800, 0, seed=4, p_out=0.02, unassigned=800)
    check_rhs(env, P, cia.CIA_METHOD_CIA, cia.CIA_F32, "all unassigned")


def test_complete_graph_all_to_all(env):
    """CIA_GRAPH_COMPLETE: E1 alone (no remainder) vs the oracle's all-to-all sum."""
    cia, torch = env
    n = 3000
    rng = np.random.default_rng(3)
    theta = rng.uniform(0, 2 * np.pi, n)
    for method in (0, 1):
        for prec in (cia.CIA_F32, cia.CIA_F64):
            dt = torch.float64 if prec else torch.float32
            plan = cia.Plan.phase(n, complete=True, K=3.0, d_sin=[0, 1, 0.3], d_cos=[0.2, 0, 0.1],
                                  method=method, precision=prec)
            th = torch.as_tensor(theta, dtype=dt, device="cuda")
            out = torch.empty_like(th)
            plan.rhs(th, out)
            got = out.cpu().numpy().astype(np.float64)
            want = oracle.phase_rhs(n, None, None, None, 3.0, [0, 1, 0.3], [0.2, 0, 0.1],
                                    th.cpu().numpy().astype(np.float64), complete=True)
            err = rel_inf(got, want)
            say("complete", method, prec, err)
            assert err < (TOL64 if prec else TOL32)
            plan.close()


def test_wide_community_fp64_observables(env):
    """A community above 1e5 nodes takes the FP64 observable path; near
    synchrony the E1 terms cancel strongly, which FP32 sums could not hold."""
    cia, torch = env
    n = 150_000
    rng = np.random.default_rng(8)
    theta = 1.0 + 1e-3 * rng.standard_normal(n)
    plan = cia.Plan.phase(n, complete=True, K=3.0, precision=cia.CIA_F32)
    assert plan.info().wide_comms == 1
    th = torch.as_tensor(theta, dtype=torch.float32, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    got = out.cpu().numpy().astype(np.float64)
    rows = rng.choice(n, 64, replace=False)
    want = oracle.phase_rhs(n, None, None, None, 3.0, [0, 1], [0, 0],
                            th.cpu().numpy().astype(np.float64), rows=rows, complete=True)
    err = rel_inf(got[rows], want)
    say("wide rel_inf", err)
    assert err < TOL32
    plan.close()


@pytest.mark.parametrize("unit_work,block", [(64, 256), (0, 512)])
def test_rhs_merged_pos_slices(env, unit_work, block):
    """Dense links between communities (FP32, p = 1): slices whose +1 lists
    are stored as one partner-sorted list and summed per row in fixed point,
    beside slices that keep one row per lane (sparse rows); one RHS against
    the oracle, the same bits on a second plan, and an RK4 trajectory."""
    cia, torch = env
    rng = np.random.default_rng(31)
    sizes = [1800, 1200, 640, 333, 64, 7]
    n = sum(sizes) + 129
    labels = W.shuffled_labels(sizes, n, rng)
    g = W.sbm(labels, len(sizes), 0.8, p_out=0.04, seed=31)
    theta = rng.uniform(0.0, 2 * np.pi, n)
    omega = rng.standard_normal(n)
    kw = dict(unit_work=unit_work, block=block)
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, K=2.5, **kw)
    info = plan.info()
    th = torch.as_tensor(theta, dtype=torch.float32, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    out2 = torch.empty_like(th)
    plan2 = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, K=2.5, **kw)
    plan2.rhs(th, out2)
    torch.cuda.synchronize()
    plan.close()
    plan2.close()
    got = out.cpu().numpy().astype(np.float64)
    want = oracle.phase_rhs(g.n, g.row_ptr, g.col, None, 2.5, [0, 1], [0, 0], th.cpu().numpy().astype(np.float64))
    err = rel_inf(got, want)
    say("merged S-pos rhs: slices merged", info.merged_slices, "units", info.nunits, "rel_inf", err)
    assert info.merged_slices > 0
    assert err <= TOL32
    assert torch.equal(out, out2)

    steps = 100
    want_th, want_r = oracle.phase_integrate(g.n, g.row_ptr, g.col, omega, 2.5, [0, 1], [0, 0], theta, 0.01, steps)
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, omega, K=2.5, **kw)
    th = torch.as_tensor(theta, dtype=torch.float32, device="cuda")
    r = np.zeros(steps + 1)
    plan.integrate(th, 0.01, steps, r)
    plan.close()
    circ = np.abs(np.angle(np.exp(1j * (th.cpu().numpy().astype(np.float64) - want_th))))
    say("merged S-pos trajectory: max |dr|", np.abs(r - want_r).max(), "max circ", circ.max())
    assert np.abs(r - want_r).max() < 1e-4
    assert circ.max() < 1e-3


@pytest.mark.parametrize("flags", [0x100, 0x400, 0x20])
def test_rhs_merged_pos_slices_kernel_paths(env, flags):
    """Merged S-pos slices beside the other kernel paths: FP64-wide
    observables (the tiled/wide instantiation), no LDS staging (S-neg
    gathered from global memory), and units re-cut by the autotuner."""
    rng = np.random.default_rng(37)
    sizes = [1500, 900, 410, 65]
    n = sum(sizes) + 77
    labels = W.shuffled_labels(sizes, n, rng)
    g = W.sbm(labels, len(sizes), 0.75, p_out=0.05, seed=37)
    theta = rng.uniform(0.0, 2 * np.pi, n)
    cia, torch = env
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, K=2.0, flags=flags)
    try:
        th = torch.as_tensor(theta, dtype=torch.float32, device="cuda")
        out = torch.empty_like(th)
        plan.rhs(th, out)
        torch.cuda.synchronize()
        info = plan.info()
    finally:
        plan.close()
    got = out.cpu().numpy().astype(np.float64)
    th_used = th.cpu().numpy().astype(np.float64)
    want = oracle.phase_rhs(g.n, g.row_ptr, g.col, None, 2.0, [0, 1], [0, 0], th_used)
    err = rel_inf(got, want)
    say("merged S-pos, flags %#x: slices merged" % flags, info.merged_slices, "units", info.nunits, "rel_inf", err)
    assert info.merged_slices > 0
    assert err <= TOL32


def test_merged_pos_slices_graph_replay_bitwise(env):
    """A plan with merged S-pos slices integrated by replaying its captured
    RK4 step graph gives the bits of plain launches, over three calls with
    host work and synchronisation between them."""
    cia, torch = env
    rng = np.random.default_rng(41)
    sizes = [1200, 700, 300]
    n = sum(sizes) + 45
    labels = W.shuffled_labels(sizes, n, rng)
    g = W.sbm(labels, len(sizes), 0.8, p_out=0.05, seed=41)
    omega = rng.standard_normal(n)
    theta = rng.uniform(0.0, 2 * np.pi, n).astype(np.float32)
    runs = []
    for flags in (0, 0x8):
        plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, omega, K=2.0, flags=flags)
        assert plan.info().merged_slices > 0
        th = torch.as_tensor(theta, device="cuda")
        got = []
        for steps in (10, 15, 10):
            r = np.zeros(steps + 1)
            plan.integrate(th, 0.01, steps, r)
            torch.cuda.synchronize()
            got.append((th.cpu().numpy().copy(), r))
        plan.close()
        runs.append(got)
    for (a, ra), (b, rb) in zip(runs[0], runs[1]):
        assert np.array_equal(a, b) and np.array_equal(ra, rb)


def test_deterministic_bits(env):
    cia, torch = env
    P = W.random_phase_problem(5000, 6, seed=9, p=2)
    a, _, _ = gpu_rhs(env, P, 0, cia.CIA_F32, P.theta0)
    b, _, _ = gpu_rhs(env, P, 0, cia.CIA_F32, P.theta0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("stepper", [0, 1])
def test_trajectory_fp64_small_config(env, stepper):
    """N = 1000 planted SBM (5 x 200, p_in 0.9, p_out 0.01), K = 4, RK4 dt 0.01,
    200 steps, FP64 on the GPU: circular phase error and r(t) vs the oracle."""
    cia, torch = env
    P = W.kuramoto_small()
    g = P.graph
    steps = P.steps if stepper == 0 else 100
    want_th, want_r = oracle.phase_integrate(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0],
                                             P.theta0, P.dt, steps,
                                             stepper="rk4" if stepper == 0 else "euler")
    for method in (0, 1):
        plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K, method=method,
                              precision=cia.CIA_F64, stepper=stepper)
        th = torch.as_tensor(P.theta0, dtype=torch.float64, device="cuda")
        r = np.zeros(steps + 1)
        plan.integrate(th, P.dt, steps, r)
        got = th.cpu().numpy()
        circ = np.abs(np.angle(np.exp(1j * (got - want_th))))
        say("traj64 method", method, "stepper", stepper, "max circ", circ.max(), "max dr", np.abs(r - want_r).max())
        assert circ.max() < 1e-9
        assert np.abs(r - want_r).max() < 1e-9
        plan.close()


def test_trajectory_fp32_scaled_large_config(env):
    """Config-2 recipe at N = 20000 (power-law sizes, Cauchy omega), FP32 RK4,
    150 steps: r(t) within 1e-3 of the FP64 oracle; phases close on the circle."""
    cia, torch = env
    P = W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    steps = 150
    want_th, want_r = oracle.phase_integrate(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0],
                                             P.theta0, P.dt, steps)
    for method in (0, 1):
        plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K, method=method)
        th = torch.as_tensor(P.theta0, dtype=torch.float32, device="cuda")
        r = np.zeros(steps + 1)
        plan.integrate(th, P.dt, steps, r)
        got = th.cpu().numpy().astype(np.float64)
        circ = np.abs(np.angle(np.exp(1j * (got - want_th))))
        # FP32 phases lose ~ulp(|omega| t) for the heavy Cauchy tail; judge the bulk
        bulk = np.abs(P.omega) < 10
        say("traj32 method", method, "dr", np.abs(r - want_r).max(), "circ bulk max", circ[bulk].max(),
            "median", np.median(circ))
        assert np.abs(r - want_r).max() < 1e-3
        assert circ[bulk].max() < 1e-3
        plan.close()


@pytest.mark.parametrize("recipe", ["config1", "config2_scaled"])
def test_order_parameter_ten_time_units(env, recipe):
    """FP32 on the GPU, RK4 dt 0.01 for 1000 steps (10 time units): r(t)
    within 1e-3 of the FP64 oracle at every step, and every community's own
    order parameter r_c at the end (the global r stays near N^-1/2 at weak
    effective coupling, so r_c is the sharper check), for CIA and direct."""
    cia, torch = env
    P = W.kuramoto_small() if recipe == "config1" else W.scaled_kuramoto(3000, seed=21, hi=300)
    g = P.graph
    steps = 1000
    want_th, want_r = oracle.phase_integrate(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0], P.theta0,
                                             P.dt, steps)
    comms = [np.flatnonzero(g.labels == c) for c in np.unique(g.labels[g.labels >= 0])]

    def r_comm(th):
        return np.array([np.abs(np.exp(1j * th[m]).mean()) for m in comms])
    for method in (0, 1):
        plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K, method=method)
        th = torch.as_tensor(P.theta0, dtype=torch.float32, device="cuda")
        r = np.zeros(steps + 1)
        plan.integrate(th, P.dt, steps, r)
        dr = np.abs(r - want_r).max()
        drc = np.abs(r_comm(th.cpu().numpy().astype(np.float64)) - r_comm(want_th)).max()
        say("r(t) over 10 time units:", recipe, "n", g.n, "method", method, "max |dr|", dr,
            "communities", len(comms), "max |dr_c| at t=10", drc)
        assert dr < 1e-3 and drc < 1e-3
        plan.close()


def test_full_size_sampled_rows(env):
    """N = 1e6 power-law workload, the plans bench.py times: sampled rows of
    one RHS against the oracle computed row by row."""
    cia, torch = env
    P = W.kuramoto_large()
    g = P.graph
    rng = np.random.default_rng(99)
    rows = np.sort(rng.choice(g.n, 3000, replace=False))
    for method in (0, 1):
        say("full size method", method)
        got, th, info = gpu_rhs(env, P, method, cia.CIA_F32, P.theta0)
        want = oracle.phase_rhs(g.n, g.row_ptr, g.col, None, P.K, [0, 1], [0, 0], th, rows=rows)
        # infinity norm of the full oracle vector is not available; the sample's
        # maximum magnitude stands in (a lower bound makes the gate stricter)
        err = rel_inf(got[rows], want)
        say("   rel_inf", err, "nnz_neg", info.nnz_neg, "nnz_pos", info.nnz_pos, "units", info.nunits)
        assert err < TOL32
        if method == 0:
            # the remainder has the size the workload recipe implies
            assert 5.5e7 < info.nnz_neg < 7.5e7
            assert 4.5e6 < info.nnz_pos < 5.5e6


def test_plan_from_detected_communities(env):
    """Labels from cia_detect_communities (no planted labels used) give a CIA
    plan whose RHS matches the oracle."""
    cia, torch = env
    P = W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    lab, work = cia.detect_communities(g.n, g.row_ptr, g.col)
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, lab, None, K=P.K)
    th = torch.as_tensor(P.theta0.astype(np.float32), device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    torch.cuda.synchronize()
    want = oracle.phase_rhs(g.n, g.row_ptr, g.col, None, P.K, [0, 1], [0, 0], th.cpu().numpy().astype(np.float64))
    err = rel_inf(out.cpu().numpy().astype(np.float64), want)
    say("detected communities", plan.info().ncomm, "work", work, "rel_inf", err)
    assert plan.info().ncomm == len(np.unique(lab[lab >= 0])) and err < TOL32
    plan.close()


def test_order_parameter_ten_time_units_config2_sizes(env):
    """Power-law recipe at N = 30000 with communities up to 4929 nodes (LDS
    staged, several work units each), FP32 RK4 dt 0.01 for 1000 steps on the
    GPU, CIA and direct: r(t) within 1e-3 of the FP64 oracle at every step
    and every community's r_c within 1e-3 at t = 10.  The oracle trajectory
    is stored by tests/golden/make_order_parameter_config2.py (it takes a
    quarter of an hour on the host cores)."""
    from conftest import load_golden
    cia, torch = env
    ref = load_golden("order_parameter_config2_n30000.json")
    rc = ref["recipe"]
    P = W.scaled_kuramoto(rc["n"], seed=rc["seed"], hi=rc["hi"])
    g = P.graph
    # the stored trajectory belongs to exactly this input
    assert g.nnz == ref["check"]["nnz"] and g.ncomm == ref["check"]["ncomm"]
    assert abs(P.omega.sum() - ref["check"]["sum_omega"]) < 1e-6 * max(1.0, abs(ref["check"]["sum_omega"]))
    assert abs(P.theta0.sum() - ref["check"]["sum_theta0"]) < 1e-9 * abs(ref["check"]["sum_theta0"])
    steps = rc["steps"]
    want_r = np.array(ref["r"])
    want_rc = np.array(ref["r_c"])
    comms = [np.flatnonzero(g.labels == c) for c in ref["communities"]]
    assert max(len(m) for m in comms) > 4000
    for method in (0, 1):
        plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K, method=method)
        info = plan.info()
        if method == 0:
            assert info.nunits > info.ncomm   # large communities span several units
        th = torch.as_tensor(P.theta0, dtype=torch.float32, device="cuda")
        r = np.zeros(steps + 1)
        plan.integrate(th, P.dt, steps, r)
        got = th.cpu().numpy().astype(np.float64)
        got_rc = np.array([np.abs(np.exp(1j * got[m]).mean()) for m in comms])
        dr = np.abs(r - want_r).max()
        drc = np.abs(got_rc - want_rc).max()
        say("r(t) config-2 sizes: n", g.n, "method", method, "units", info.nunits, "max |dr|", dr,
            "max |dr_c| at t=10", drc, "largest community", max(len(m) for m in comms))
        assert dr <= 1e-3 and drc <= 1e-3
        plan.close()
