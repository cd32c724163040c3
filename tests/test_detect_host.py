"""Community detection for unlabeled graphs (host only, no GPU): the work it
reports against P1's own S lists and an independent count, recovery of the
planted partitions of the phase workloads, optimality against exhaustive
search on tiny graphs, determinism, refinement and the cost rule's limits."""
import itertools

import numpy as np
import pytest
import scipy.sparse

import paper_2203_16657_amd as cia
import workloads as W


@pytest.fixture(scope="module")
def lib():
    cia.load()
    return cia


def csr(A):
    S = scipy.sparse.csr_matrix(A)
    S.sort_indices()
    return S.indptr.astype(np.int64), S.indices.astype(np.int32)


def work_of(A, labels, alpha):
    """nnz(S-neg) + nnz(S-pos) + alpha * members of communities, counted from
    the dense adjacency (communities of one node count as none)."""
    n = len(labels)
    lab = np.asarray(labels)
    total = 0.0
    inside = np.zeros_like(A, dtype=bool)
    for c in np.unique(lab[lab >= 0]):
        m = np.flatnonzero(lab == c)
        if len(m) < 2:
            continue
        sub = A[np.ix_(m, m)]
        total += len(m) * (len(m) - 1) - sub.sum() + alpha * len(m)
        inside[np.ix_(m, m)] = True
    total += A[~inside].sum()
    return total


def same_partition(a, b):
    pairs = set(zip(a.tolist(), b.tolist()))
    return len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


@pytest.mark.parametrize("which", ["config1", "config2_scaled"])
def test_recovers_planted_partition(lib, which):
    P = W.kuramoto_small() if which == "config1" else W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    lab, work = lib.detect_communities(g.n, g.row_ptr, g.col)
    assert same_partition(lab, g.labels)
    # the reported work is P1's: nnz(S-neg) + nnz(S-pos) + alpha * assigned
    p1 = lib.cia_p1(g.n, g.row_ptr, g.col, labels=lab)
    assert work == p1["nnz_neg"] + p1["nnz_pos"] + 2.0 * (g.n - p1["n_unassigned"])


def test_reported_work_matches_an_independent_count(lib):
    rng = np.random.default_rng(3)
    n = 150
    lab_true = rng.integers(0, 6, n)
    pin = np.where(lab_true[:, None] == lab_true[None, :], 0.7, 0.03)
    up = np.triu(rng.random((n, n)) < pin, 1)
    A = (up | up.T).astype(np.int64)
    rp, col = csr(A)
    for alpha in (0.0, 2.0, 7.5):
        lab, work = lib.detect_communities(n, rp, col, dense_alpha=alpha)
        assert work == pytest.approx(work_of(A, lab, alpha), rel=0, abs=1e-9)


def all_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in all_partitions(rest):
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]
        yield [[first]] + part


def brute_min(A, alpha):
    n = len(A)
    best = None
    for part in all_partitions(list(range(n))):
        lab = np.full(n, -1)
        for c, m in enumerate(part):
            lab[m] = c
        w = work_of(A, lab, alpha)
        best = w if best is None else min(best, w)
    return best


def graph_of(edges, n):
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in edges:
        A[a, b] = A[b, a] = 1
    return A


@pytest.mark.parametrize("case", ["two_k4_bridge", "k5_with_tail", "k4_k3"])
def test_optimal_on_small_graphs(lib, case):
    if case == "two_k4_bridge":
        e = [p for p in itertools.combinations(range(4), 2)] + [p for p in itertools.combinations(range(4, 8), 2)]
        A = graph_of(e + [(3, 4)], 8)
    elif case == "k5_with_tail":
        A = graph_of([p for p in itertools.combinations(range(5), 2)] + [(4, 5), (5, 6)], 7)
    else:
        e = [p for p in itertools.combinations(range(4), 2)] + [(4, 5), (5, 6), (4, 6), (0, 4)]
        A = graph_of(e, 7)
    rp, col = csr(A)
    for alpha in (0.0, 1.0):
        lab, work = lib.detect_communities(len(A), rp, col, dense_alpha=alpha)
        assert work == brute_min(A, alpha), (case, alpha, lab)


def test_never_worse_than_trivial_partitions(lib):
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        n = 7
        up = np.triu(rng.random((n, n)) < 0.55, 1)
        A = (up | up.T).astype(np.int64)
        rp, col = csr(A)
        lab, work = lib.detect_communities(n, rp, col)
        assert work == work_of(A, lab, 2.0)
        assert work <= work_of(A, np.full(n, -1), 2.0) and work <= work_of(A, np.zeros(n, int), 2.0)
        assert work >= brute_min(A, 2.0)


def test_deterministic_and_refinement(lib):
    P = W.scaled_kuramoto(20000, seed=12, hi=1000)
    g = P.graph
    a, wa = lib.detect_communities(g.n, g.row_ptr, g.col)
    b, wb = lib.detect_communities(g.n, g.row_ptr, g.col)
    assert np.array_equal(a, b) and wa == wb
    # refining a damaged partition (two planted communities merged) recovers the planted one
    lab = g.labels.copy()
    c0, c1 = np.unique(lab[lab >= 0])[:2]
    lab[lab == c1] = c0
    r, wr = lib.detect_communities(g.n, g.row_ptr, g.col, init_labels=lab)
    assert same_partition(r, g.labels) and wr == wa


def test_cost_rule_limits_and_errors(lib):
    P = W.kuramoto_small()
    g = P.graph
    lab, work = lib.detect_communities(g.n, g.row_ptr, g.col, dense_alpha=1e9)
    assert np.all(lab == -1) and work == g.row_ptr[-1]   # every edge in S-pos
    with pytest.raises(lib.CIAError):
        lib.detect_communities(g.n, g.row_ptr, g.col, init_labels=np.full(g.n, -2))
    with pytest.raises(lib.CIAError):
        lib.detect_communities(g.n, g.row_ptr, g.col, dense_alpha=-1.0)
