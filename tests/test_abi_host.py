"""C-ABI library checks that need no GPU: symbols, struct layouts, argument
errors, and the host-side pre-simulation step P1 (Sec. 3.1, App. A.1)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cia():
    import paper_2203_16657_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2203_16657_amd import build
        build.build()
    m.load()
    return m


def header_functions():
    text = open(os.path.join(ROOT, "include", "cia.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(cia_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol(cia):
    names = header_functions()
    assert "cia_build" in names and "cia_integrate" in names and "cia_rhs" in names
    lib = ctypes.CDLL(cia.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(cia.EXPORTS) <= set(names)


def test_struct_layouts_match(cia):
    for cls in (cia.cia_graph, cia.cia_hypergraph, cia.cia_coupling, cia.cia_options,
                cia.cia_plan_info, cia.cia_timing, cia.cia_tune_report):
        assert cia.cia_abi_sizeof(cls.__name__) == ctypes.sizeof(cls), cls.__name__
    assert cia.cia_abi_sizeof("nope") == 0


def test_defaults(cia):
    o = cia.cia_options_default()
    assert o.method == cia.CIA_METHOD_CIA and o.precision == cia.CIA_F32 and o.stepper == cia.CIA_RK4
    assert o.device == -1 and abs(o.judge_tol - 1e-3) < 1e-15
    c = cia.cia_coupling_default()
    assert c.model == cia.CIA_MODEL_PHASE and c.p == 1


def test_build_without_device_fails_cleanly(cia):
    """No GPU in this container: cia_build must report CIA_EHIP, not crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    P = W.random_phase_problem(50, 2, seed=1)
    g = P.graph
    with pytest.raises(cia.CIAError) as e:
        cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega)
    assert e.value.status == cia.CIA_EHIP
    assert "device" in cia.cia_last_error()


def test_null_and_bad_arguments(cia):
    lib = cia.load()
    assert lib.cia_rhs(None, None, None, None) == cia.CIA_EINVAL
    assert lib.cia_integrate(None, None, 0.1, 1, None, None) == cia.CIA_EINVAL
    assert lib.cia_destroy(None) == cia.CIA_OK
    out = ctypes.c_void_p()
    assert lib.cia_build(None, None, None, None, None, ctypes.byref(out)) == cia.CIA_EINVAL
    assert "NULL" in cia.cia_last_error()


@pytest.mark.parametrize("case", ["asym", "selfloop", "unsorted", "range", "label"])
def test_p1_validation_errors(cia, case):
    rp = np.array([0, 1, 3, 4], dtype=np.int64)
    col = np.array([1, 0, 2, 1], dtype=np.int32)
    labels = np.array([0, 0, 1], dtype=np.int32)
    if case == "asym":
        rp = np.array([0, 1, 2, 2], dtype=np.int64)
        col = np.array([1, 2], dtype=np.int32)
    elif case == "selfloop":
        col = np.array([1, 0, 1, 1], dtype=np.int32)
    elif case == "unsorted":
        col = np.array([1, 2, 0, 1], dtype=np.int32)
    elif case == "range":
        col = np.array([1, 0, 7, 1], dtype=np.int32)
    elif case == "label":
        labels = np.array([0, -2, 1], dtype=np.int32)
    with pytest.raises(cia.CIAError) as e:
        cia.cia_p1(3, rp, col, labels)
    assert e.value.status == cia.CIA_EINVAL
    msg = cia.cia_last_error()
    assert {"asym": "symmetric", "selfloop": "self-loop", "unsorted": "increasing",
            "range": "range", "label": "labels"}[case] in msg


def test_p1_zero_nodes(cia):
    with pytest.raises(cia.CIAError):
        cia.cia_p1(0, np.zeros(1, np.int64), np.zeros(0, np.int32))


def test_p1_structure_matches_definition(cia):
    """B = P A P^T = D + S (Sec. 3.1): entries of S-neg are exactly the
    missing intra-community pairs, S-pos exactly the remaining edges; the
    diagonal is in neither."""
    P = W.random_phase_problem(300, 5, seed=21, p_in=0.85, p_out=0.03, unassigned=17)
    g = P.graph
    o = cia.cia_options_default()
    o.flags = cia.CIA_FLAG_KEEP_LABELS
    r = cia.cia_p1(g.n, g.row_ptr, g.col, g.labels, o)
    n = g.n
    perm = r["perm"]
    assert sorted(perm.tolist()) == list(range(n))
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    A = oracle.dense_from_csr(n, g.row_ptr, g.col)
    B = A[np.ix_(perm, perm)]
    D = np.zeros((n, n))
    co = r["comm_off"]
    for c in range(r["ncomm"]):
        D[co[c]:co[c + 1], co[c]:co[c + 1]] = 1.0
    np.fill_diagonal(D, 0.0)
    S = np.zeros((n, n))
    for i in range(n):
        for e in range(r["negptr"][i], r["negptr"][i + 1]):
            S[i, r["neg"][e]] -= 1
        row = r["pos"][r["posptr"][i]:r["posptr"][i + 1]]
        assert np.all(np.diff(row) > 0)
        S[i, row] += 1
    np.testing.assert_array_equal(B, D + S)
    # communities contiguous with labels preserved, unassigned last
    lab = g.labels[perm]
    for c in range(r["ncomm"]):
        assert len(set(lab[co[c]:co[c + 1]].tolist())) == 1
    assert np.all(lab[co[-1]:] == -1)
    assert r["n_unassigned"] == 17


def test_p1_cost_rule_dissolves_sparse_communities(cia):
    """App. A.1: a community whose missing links outnumber its links (plus
    the per-node cost of its observables) is not worth treating as a block."""
    rng = np.random.default_rng(0)
    labels = W.shuffled_labels([60, 60, 60], 180, rng)
    pin = np.array([0.95, 0.3, 0.9])
    g = W.sbm(labels, 3, pin, p_out=0.01, seed=3)
    r = cia.cia_p1(g.n, g.row_ptr, g.col, g.labels)
    assert r["ncomm"] == 2
    assert r["n_unassigned"] == 60
    o = cia.cia_options_default()
    o.flags = cia.CIA_FLAG_KEEP_LABELS
    assert cia.cia_p1(g.n, g.row_ptr, g.col, g.labels, o)["ncomm"] == 3


@pytest.mark.parametrize("p", [1, 3])
def test_decomposition_identity_on_host(cia, p):
    """E1 + E2 with the exported S reproduces the oracle's direct sum
    (App. A.2 real difference series; the dense block includes l = m, whose
    h(0) is removed).  Pure NumPy on the host, FP64."""
    P = W.random_phase_problem(250, 4, seed=31 + p, p_in=0.8, p_out=0.05, unassigned=9, p=p)
    g = P.graph
    r = cia.cia_p1(g.n, g.row_ptr, g.col, g.labels)
    perm, co = r["perm"], r["comm_off"]
    phi = P.theta0[perm]
    om = P.omega[perm]
    n = g.n

    def h(x):
        v = np.full_like(x, P.d_cos[0])
        for k in range(1, p + 1):
            v = v + P.d_sin[k] * np.sin(k * x) + P.d_cos[k] * np.cos(k * x)
        return v

    H = np.zeros(n)
    for c in range(r["ncomm"]):
        sl = slice(co[c], co[c + 1])
        z = np.exp(1j * phi[sl])
        for m in range(co[c], co[c + 1]):
            tot = P.d_cos[0] * (co[c + 1] - co[c])
            for k in range(1, p + 1):
                B = np.sum(z ** k) * np.exp(-1j * k * phi[m])
                tot += P.d_cos[k] * B.real + P.d_sin[k] * B.imag
            H[m] = tot - h(np.array([0.0]))[0]
    for i in range(n):
        neg = r["neg"][r["negptr"][i]:r["negptr"][i + 1]]
        pos = r["pos"][r["posptr"][i]:r["posptr"][i + 1]]
        H[i] += h(phi[pos] - phi[i]).sum() - h(phi[neg] - phi[i]).sum()
    H = om + P.K / n * H
    want = oracle.phase_rhs(n, g.row_ptr, g.col, P.omega, P.K, P.d_sin, P.d_cos, P.theta0)[perm]
    np.testing.assert_allclose(H, want, atol=1e-11)


def test_fourier_coeffs_exact_for_trig_polynomial(cia):
    """P2 (Sec. 3.1): a trigonometric polynomial of degree <= p is recovered
    exactly from m >= 2p+1 samples."""
    m = 32
    x = 2 * np.pi * np.arange(m) / m
    f = 0.3 + 2 * np.sin(x) - 0.5 * np.cos(3 * x) + 0.25 * np.sin(3 * x)
    ds, dc = cia.cia_fourier_coeffs(f, 4)
    np.testing.assert_allclose(ds, [0, 2, 0, 0.25, 0], atol=1e-13)
    np.testing.assert_allclose(dc, [0.3, 0, 0, -0.5, 0], atol=1e-13)
    with pytest.raises(cia.CIAError):
        cia.cia_fourier_coeffs(f[:5], 4)


def test_fourier_coeffs_converge_for_smooth_coupling(cia):
    """A smooth periodic h (here exp(cos x) sin x) is approximated with
    errors decaying quickly in p."""
    m = 256
    x = 2 * np.pi * np.arange(m) / m
    f = np.exp(np.cos(x)) * np.sin(x)
    errs = []
    xs = np.linspace(0, 2 * np.pi, 101)
    for p in (2, 4, 8):
        ds, dc = cia.cia_fourier_coeffs(f, p)
        approx = dc[0] + sum(ds[k] * np.sin(k * xs) + dc[k] * np.cos(k * xs) for k in range(1, p + 1))
        errs.append(np.abs(approx - np.exp(np.cos(xs)) * np.sin(xs)).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6


def test_binding_rejects_wrong_lengths(cia):
    """The binding checks host array lengths before any call reads them."""
    rp = np.array([0, 1, 2], np.int64)
    col = np.array([1, 0], np.int32)
    with pytest.raises(ValueError):
        cia.Plan.phase(2, rp, col, np.zeros(3, np.int32))          # labels too long
    with pytest.raises(ValueError):
        cia.Plan.phase(2, rp, col, None, np.zeros(1))                # omega too short
    with pytest.raises(ValueError):
        cia.Plan.phase(3, rp, col)                                   # row_ptr of the wrong length
    with pytest.raises(ValueError):
        cia.Plan.poly(2, np.array([0, 1, 5], np.int64), col)         # row_ptr beyond col
    with pytest.raises(ValueError):
        cia.Plan.structured(4, "rank1", alpha=np.ones(4))            # beta missing
    with pytest.raises(ValueError):
        cia.Plan.structured(4, "rank1", alpha=np.ones(3), beta=np.ones(4))


def test_incremental_batch_host_checks(cia):
    """cia_batch_add runs P1 on the host, so its argument checks need no GPU:
    a mismatched coupling function, a non-CSR graph, a bad label or a
    non-finite frequency is refused with the instance number and the handle
    stays usable; abort releases it."""
    bb = cia.BatchBuilder()
    P = W.ensemble_member(3, n_lo=200, n_hi=600)
    g = P.graph
    bb.add(g.n, g.row_ptr, g.col, g.labels, P.omega, P.K)
    assert bb.count == 1 and bb.n == g.n
    lib = cia.load()
    # another coupling function (p = 2) is refused
    ds, dc = np.array([0.0, 1.0, 0.5]), np.zeros(3)
    c = cia.cia_coupling_default()
    c.p, c.d_sin, c.d_cos, c.K = 2, ds.ctypes.data_as(ctypes.c_void_p), dc.ctypes.data_as(ctypes.c_void_p), 1.0
    rp, cl = g.row_ptr, g.col
    gg = cia.cia_graph(n=g.n, kind=cia.CIA_GRAPH_CSR, reserved=0, row_ptr=rp.ctypes.data_as(ctypes.c_void_p),
                       col=cl.ctypes.data_as(ctypes.c_void_p))
    st = lib.cia_batch_add(bb.handle, ctypes.byref(gg), None, ctypes.byref(c), None)
    assert st == cia.CIA_EINVAL and "instance 1" in cia.cia_last_error()
    bad = g.labels.copy()
    bad[0] = -7
    with pytest.raises(cia.CIAError):
        bb.add(g.n, g.row_ptr, g.col, bad, None, 1.0)
    om = P.omega.copy()
    om[5] = np.nan
    with pytest.raises(cia.CIAError):
        bb.add(g.n, g.row_ptr, g.col, g.labels, om, 1.0)
    # the handle still takes a valid instance after the refusals
    bb.add(g.n, g.row_ptr, g.col, g.labels, None, 2.0)
    assert bb.count == 2
    bb.abort()
    with pytest.raises(ValueError):
        bb.add(g.n, g.row_ptr, g.col, g.labels, None, 2.0)
