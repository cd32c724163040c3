"""Small networks integrated in one resident workgroup (every z of a stage in
LDS, stages separated by barriers, one launch per cia_integrate call):
trajectories and r(t) against the FP64 oracle, and against the
stage-by-stage launches of the same plan (CIA_FLAG_NO_RESIDENT) for both
precisions, Fourier orders 1 to 4, a nonzero d_0, nodes of no community,
int32 S-neg (CIA_FLAG_FORCE_NEG32), Euler, zero steps and tiny networks."""
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


def circ(a, b):
    return np.abs(np.remainder(a - b + np.pi, 2 * np.pi) - np.pi)


def run(env, P, prec, steps, flags=0, stepper=0, dt=0.01):
    cia, torch = env
    g = P.graph
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K, d_sin=P.d_sin, d_cos=P.d_cos,
                          precision=prec, flags=flags, stepper=stepper)
    res = plan.info().resident
    tdt = torch.float64 if prec == cia.CIA_F64 else torch.float32
    th = torch.as_tensor(P.theta0, dtype=tdt, device="cuda")
    r = np.zeros(steps + 1)
    plan.integrate(th, dt, steps, r)
    out = th.cpu().numpy().astype(np.float64)
    plan.close()
    return out, r, res


def test_config1_is_resident_and_matches_oracle(env):
    """The N = 1000 FP64 network (5 communities of 200) runs resident; 200
    RK4 steps against the oracle to 1e-9, with RK4 and Euler."""
    cia, _ = env
    P = W.kuramoto_small()
    g = P.graph
    for stepper in (cia.CIA_RK4, cia.CIA_EULER):
        th, r, res = run(env, P, cia.CIA_F64, 200, stepper=stepper)
        assert res == 1
        want_th, want_r = oracle.phase_integrate(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0], P.theta0,
                                                 P.dt, 200, stepper="rk4" if stepper == cia.CIA_RK4 else "euler")
        e = circ(th, want_th).max()
        say("resident config1 stepper", stepper, "max circ", e, "max dr", np.abs(r - want_r).max())
        assert e < 1e-9 and np.abs(r - want_r).max() < 1e-9


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", [0, 1])
def test_resident_equals_stagewise(env, p, prec):
    cia, _ = env
    P = W.random_phase_problem(1500 if prec == cia.CIA_F64 else 2000, 9, seed=300 + p, p_in=0.85, p_out=0.005,
                               unassigned=61, p=p)
    steps = 40
    a_th, a_r, a_res = run(env, P, prec, steps)
    b_th, b_r, b_res = run(env, P, prec, steps, flags=cia.CIA_FLAG_NO_RESIDENT)
    assert a_res == 1 and b_res == 0
    e, dr = circ(a_th, b_th).max(), np.abs(a_r - b_r).max()
    say("resident vs stagewise p", p, "prec", prec, "max circ", e, "max dr", dr)
    tol = 1e-11 if prec == cia.CIA_F64 else 2e-4
    assert e < tol and dr < tol


def test_resident_fp64_against_oracle_with_d0_and_outside_nodes(env):
    cia, _ = env
    P = W.random_phase_problem(1500, 6, seed=311, p_in=0.85, p_out=0.02, unassigned=40, p=2)
    P.d_cos = np.array([0.3, 0.1, -0.2])
    g = P.graph
    steps = 30
    th, r, res = run(env, P, cia.CIA_F64, steps)
    assert res == 1
    want_th, want_r = oracle.phase_integrate(g.n, g.row_ptr, g.col, P.omega, P.K, P.d_sin, P.d_cos, P.theta0,
                                             0.01, steps)
    e = circ(th, want_th).max()
    say("resident fp64 d0 outside: max circ", e, "max dr", np.abs(r - want_r).max())
    assert e < 1e-9 and np.abs(r - want_r).max() < 1e-9


def test_resident_int32_negatives_and_edges(env):
    """Int32 S-neg (every community unstaged), zero steps (state as given,
    r(t_0) only) and a 40-node network."""
    cia, torch = env
    P = W.random_phase_problem(1800, 5, seed=321, p_in=0.85, p_out=0.005, unassigned=25, p=1)
    a_th, a_r, a_res = run(env, P, cia.CIA_F32, 25, flags=cia.CIA_FLAG_FORCE_NEG32)
    b_th, b_r, _ = run(env, P, cia.CIA_F32, 25, flags=cia.CIA_FLAG_FORCE_NEG32 | cia.CIA_FLAG_NO_RESIDENT)
    assert a_res == 1
    assert circ(a_th, b_th).max() < 2e-4 and np.abs(a_r - b_r).max() < 2e-4
    th0, r0, _ = run(env, P, cia.CIA_F64, 0)
    assert np.array_equal(th0, P.theta0)
    assert abs(r0[0] - oracle.order_parameter(P.theta0)) < 1e-12
    T = W.random_phase_problem(40, 2, seed=5, p_in=0.9, p_out=0.05, unassigned=3, p=1)
    g = T.graph
    th, r, res = run(env, T, cia.CIA_F64, 50)
    assert res == 1
    want_th, want_r = oracle.phase_integrate(g.n, g.row_ptr, g.col, T.omega, T.K, T.d_sin, T.d_cos, T.theta0,
                                             0.01, 50)
    assert circ(th, want_th).max() < 1e-9 and np.abs(r - want_r).max() < 1e-9


def test_large_remainder_stays_stagewise(env):
    """Above 2^17 remainder entries one CU's LDS would serve every gather of
    a stage: such plans keep the stage-by-stage launches."""
    cia, _ = env
    P = W.random_phase_problem(5000, 6, seed=331, p_in=0.8, p_out=0.01, unassigned=10, p=1)
    g = P.graph
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K)
    info = plan.info()
    assert info.nnz_neg + info.nnz_pos > (1 << 17) and info.resident == 0
    plan.close()
