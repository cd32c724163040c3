"""GPU parity of communities above the LDS staging cap (8191 nodes for FP32
z values): their z values are staged one column tile at a time and S-neg is
gathered tile by tile from LDS.  Checked against the FP64 oracle for one RHS
(tile counts 2 to 3, a community exactly at the cap, one just above it,
small communities and nodes of no community beside them), against the int32
S-neg path of the same plan (CIA_FLAG_FORCE_NEG32) over an RK4 trajectory,
for other unit and block sizes, and after the autotuner re-cuts the units."""
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


def big_problem(sizes, p_in, seed, unassigned=97, p_out=2e-4):
    rng = np.random.default_rng(seed)
    n = int(sum(sizes)) + unassigned
    labels = W.shuffled_labels(sizes, n, rng)
    g = W.sbm(labels, len(sizes), p_in, p_out=p_out, seed=seed)
    omega = rng.standard_normal(n)
    theta0 = rng.uniform(0.0, 2 * np.pi, n)
    return g, omega, theta0


@pytest.fixture(scope="module")
def prob():
    # 20000 -> 3 tiles of 6667, 9000 -> 2 tiles of 4500, 8192 -> 2 of 4096,
    # 8191 staged whole, two small staged communities
    return big_problem([20000, 9000, 8192, 8191, 700, 300], 0.6, seed=41)


def rhs(env, g, theta, **kw):
    cia, torch = env
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, K=3.0, **kw)
    th = torch.as_tensor(theta, dtype=torch.float32, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    torch.cuda.synchronize()
    info = plan.info()
    plan.close()
    return out.cpu().numpy().astype(np.float64), th.cpu().numpy().astype(np.float64), info


@pytest.mark.parametrize("unit_work,block", [(0, 0), (4096, 0), (0, 512), (4096, 512)])
def test_tiled_rhs_against_oracle(env, prob, unit_work, block):
    cia, _ = env
    g, _, theta0 = prob
    got, th, info = rhs(env, g, theta0, unit_work=unit_work, block=block)
    say("tiled rhs unit_work", unit_work, "block", block, "units", info.nunits, "tiled", info.tiled_comms,
        "max_comm", info.max_comm)
    assert info.tiled_comms == 3 and info.ncomm == 6
    want = oracle.phase_rhs(g.n, g.row_ptr, g.col, None, 3.0, [0, 1], [0, 0], th)
    err = float(np.abs(got - want).max() / np.abs(want).max())
    say("   rel_inf", err)
    assert err <= 1e-5


def test_tiled_equals_int32_path_over_trajectory(env):
    """Tiled staging and the int32 global-gather path of the same graph give
    the same RK4 trajectory up to FP32 summation order."""
    cia, torch = env
    g, omega, theta0 = big_problem([12000, 600], 0.7, seed=43)
    steps = 60
    res = []
    for flags in (0, cia.CIA_FLAG_FORCE_NEG32):
        plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, omega, K=6.0, flags=flags)
        if flags == 0:
            assert plan.info().tiled_comms == 1
        th = torch.as_tensor(theta0, dtype=torch.float32, device="cuda")
        r = np.zeros(steps + 1)
        plan.integrate(th, 0.01, steps, r)
        res.append((th.cpu().numpy().astype(np.float64), r))
        plan.close()
    circ = np.abs(np.angle(np.exp(1j * (res[0][0] - res[1][0]))))
    dr = np.abs(res[0][1] - res[1][1]).max()
    say("tiled vs int32 path: max circ", circ.max(), "max |dr|", dr)
    assert circ.max() < 1e-4 and dr < 1e-6


def test_tiled_autotune_keeps_results(env, prob):
    cia, torch = env
    g, _, theta0 = prob
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, None, K=3.0)
    th = torch.as_tensor(theta0, dtype=torch.float32, device="cuda")
    out = torch.empty_like(th)
    plan.rhs(th, out)
    before = out.cpu().numpy().astype(np.float64)
    rep = plan.autotune()
    plan.rhs(th, out)
    after = out.cpu().numpy().astype(np.float64)
    say("autotune on tiled plan: unit_work", rep.unit_work, "block", rep.block)
    scale = np.abs(before).max()
    assert np.abs(after - before).max() <= 1e-5 * scale
    plan.close()


def test_tiled_with_merged_pos_slices(env):
    """A tiled community (9000 nodes, two tiles) whose rows also have dense
    links out (p_out 0.01): the tile-by-tile S-neg sums and the merged,
    partner-sorted S-pos sums of the same slices, against the oracle."""
    cia, _ = env
    g, _, theta = big_problem([9000, 700, 300], 0.6, seed=43, p_out=0.01)
    got, th_used, info = rhs(env, g, theta)
    want = oracle.phase_rhs(g.n, g.row_ptr, g.col, None, 3.0, [0, 1], [0, 0], th_used)
    err = float(np.abs(got - want).max() / np.abs(want).max())
    say("tiled + merged: tiled", info.tiled_comms, "merged slices", info.merged_slices, "rel_inf", err)
    assert info.tiled_comms == 1 and info.merged_slices > 0
    assert err <= 1e-5
