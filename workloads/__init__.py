"""Seeded synthetic workloads shared by the oracle and the HIP path.

Holds no community-integration arithmetic: it only draws planted-community
graphs (stochastic block models), intrinsic frequencies, initial states and
triangle lists.  Every draw is determined by the seed.

Graph recipe (the paper's synthetic community graphs, Sec. 4 and Fig. 2):
nodes are split into planted communities; intra pairs are edges with
probability p_in; cross pairs are either Bernoulli(p_out) or a fixed number
of uniform random distinct pairs.  The label sequence is a uniformly shuffled
multiset, so node ids carry no trace of the community order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcia_gen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the generator (plain C, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.gen_sbm_create.restype = ctypes.c_void_p
        lib.gen_sbm_create.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                       ctypes.c_uint64]
        lib.gen_sbm_nnz.restype = ctypes.c_int64
        lib.gen_sbm_nnz.argtypes = [ctypes.c_void_p]
        lib.gen_sbm_fill.restype = None
        lib.gen_sbm_fill.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.gen_sbm_free.restype = None
        lib.gen_sbm_free.argtypes = [ctypes.c_void_p]
        lib.gen_cross_triangles.restype = ctypes.c_int64
        lib.gen_cross_triangles.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_uint64, ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """Symmetric CSR adjacency (user node order) with planted labels."""
    n: int
    row_ptr: np.ndarray          # int64 [n+1]
    col: np.ndarray              # int32 [nnz], rows sorted, no self-loops
    labels: np.ndarray           # int32 [n], -1 = no community
    ncomm: int
    sizes: np.ndarray = field(default=None)   # planted community sizes

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def shuffled_labels(sizes, n: int, rng: np.random.Generator) -> np.ndarray:
    """Label multiset (communities 0..M-1 with the given sizes, the rest -1),
    uniformly shuffled."""
    sizes = np.asarray(sizes, dtype=np.int64)
    lab = np.full(n, -1, dtype=np.int32)
    lab[: int(sizes.sum())] = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    rng.shuffle(lab)
    return lab


def sbm(labels: np.ndarray, ncomm: int, p_in, p_out: float = 0.0, n_inter: int = 0,
        seed: int = 0) -> Graph:
    """Planted SBM on given labels.  p_in: scalar or [ncomm].  Cross pairs are
    Bernoulli(p_out) if p_out > 0, else exactly n_inter uniform distinct pairs."""
    lib = _load()
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    n = labels.shape[0]
    pin = np.ascontiguousarray(np.broadcast_to(np.asarray(p_in, dtype=np.float64), (max(ncomm, 1),)))
    h = lib.gen_sbm_create(n, _ptr(labels), ncomm, _ptr(pin), float(p_out), int(n_inter),
                           int(seed) & 0xFFFFFFFFFFFFFFFF)
    if not h:
        raise ValueError("gen_sbm_create rejected its arguments")
    try:
        nnz = lib.gen_sbm_nnz(h)
        row_ptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        lib.gen_sbm_fill(h, _ptr(row_ptr), _ptr(col))
    finally:
        lib.gen_sbm_free(h)
    sizes = np.bincount(labels[labels >= 0], minlength=ncomm).astype(np.int64)
    return Graph(n=n, row_ptr=row_ptr, col=col[:nnz], labels=labels, ncomm=ncomm, sizes=sizes)


def cross_triangles(labels: np.ndarray, count: int, seed: int) -> np.ndarray:
    """`count` distinct random triples not all inside one community: int32 [count,3],
    each row sorted ascending."""
    lib = _load()
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.empty((max(count, 1), 3), dtype=np.int32)
    got = lib.gen_cross_triangles(labels.shape[0], _ptr(labels), int(count), int(seed), _ptr(out))
    if got < 0:
        raise ValueError("too many nodes for the packed triangle generator")
    return out[:got]


# --------------------------------------------------------------------------
# Distributions used by the workloads
# --------------------------------------------------------------------------

def power_law_sizes(n: int, exponent: float, lo: int, hi: int, rng) -> np.ndarray:
    """Community sizes with pdf ~ s^-exponent on [lo, hi] (inverse CDF, rounded),
    drawn until the next one would exceed n; the rest of the nodes stay unassigned."""
    out = []
    total = 0
    while True:
        u = rng.random()
        if exponent == 1.0:
            s = lo * (hi / lo) ** u
        else:
            a = 1.0 - exponent
            s = (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
        s = int(round(s))
        if total + s > n:
            break
        out.append(s)
        total += s
    return np.asarray(out, dtype=np.int64)


def uniform_sizes(n: int, lo: int, hi: int, rng) -> np.ndarray:
    out, total = [], 0
    while True:
        s = int(rng.integers(lo, hi + 1))
        if total + s > n:
            break
        out.append(s)
        total += s
    return np.asarray(out, dtype=np.int64)


def lorentzian(n: int, gamma: float, rng) -> np.ndarray:
    """Cauchy(0, gamma) by inverse CDF."""
    u = rng.random(n)
    return gamma * np.tan(np.pi * (u - 0.5))


# --------------------------------------------------------------------------
# The workloads: phase-oscillator configurations
# --------------------------------------------------------------------------

@dataclass
class PhaseProblem:
    name: str
    graph: Graph
    omega: np.ndarray     # float64 [n]
    theta0: np.ndarray    # float64 [n] in [0, 2pi)
    K: float
    dt: float
    steps: int
    d_sin: np.ndarray = field(default_factory=lambda: np.array([0.0, 1.0]))
    d_cos: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0]))


def kuramoto_small(seed: int = 1) -> PhaseProblem:
    """N = 1000: 5 communities of 200, p_in 0.9, p_out 0.01 per pair,
    omega ~ N(0,1), theta0 ~ U[0,2pi), K = 4, RK4 dt 0.01, 200 steps."""
    rng = np.random.default_rng(seed)
    n = 1000
    labels = shuffled_labels([200] * 5, n, rng)
    g = sbm(labels, 5, 0.9, p_out=0.01, seed=seed)
    omega = rng.standard_normal(n)
    theta0 = rng.uniform(0.0, 2 * np.pi, n)
    return PhaseProblem("kuramoto_sbm_n1000", g, omega, theta0, K=4.0, dt=0.01, steps=200)


def kuramoto_large(seed: int = 2, n: int = 1_000_000) -> PhaseProblem:
    """N = 1e6: sizes pdf ~ s^-2 on [100,5000] (remainder unassigned), p_in 0.95,
    2.5 n inter pairs per 1e6 nodes (mean inter degree 5), omega ~ Cauchy(0, 0.5),
    theta0 ~ U[0,2pi), K = 3, RK4 dt 0.01, 1000 steps."""
    rng = np.random.default_rng(seed)
    sizes = power_law_sizes(n, 2.0, 100, 5000, rng)
    labels = shuffled_labels(sizes, n, rng)
    g = sbm(labels, len(sizes), 0.95, n_inter=int(round(2.5 * n)), seed=seed)
    omega = lorentzian(n, 0.5, rng)
    theta0 = rng.uniform(0.0, 2 * np.pi, n)
    return PhaseProblem("kuramoto_powerlaw_n%d" % n, g, omega, theta0, K=3.0, dt=0.01, steps=1000)


def scaled_kuramoto(n: int, seed: int = 2, lo: int = 100, hi: int = 5000) -> PhaseProblem:
    """Same recipe as kuramoto_large at a smaller n (community sizes capped to n)."""
    rng = np.random.default_rng(seed)
    hi = min(hi, max(lo, n // 4))
    sizes = power_law_sizes(n, 2.0, lo, hi, rng)
    labels = shuffled_labels(sizes, n, rng)
    g = sbm(labels, len(sizes), 0.95, n_inter=int(round(2.5 * n)), seed=seed)
    omega = lorentzian(n, 0.5, rng)
    theta0 = rng.uniform(0.0, 2 * np.pi, n)
    return PhaseProblem("kuramoto_powerlaw_n%d" % n, g, omega, theta0, K=3.0, dt=0.01, steps=1000)


def random_phase_problem(n: int, ncomm: int, seed: int, p_in=0.9, p_out=0.02,
                         unassigned: int = 0, p: int = 1) -> PhaseProblem:
    """Small random test problem with general Fourier order p."""
    rng = np.random.default_rng(seed)
    na = n - unassigned
    if ncomm > 0:
        cuts = np.sort(rng.choice(np.arange(1, na), size=ncomm - 1, replace=False)) if ncomm > 1 else np.array([], dtype=np.int64)
        sizes = np.diff(np.concatenate([[0], cuts, [na]])).astype(np.int64)
    else:
        sizes = np.zeros(0, dtype=np.int64)
    labels = shuffled_labels(sizes, n, rng)
    pin = rng.uniform(min(p_in, 0.999), 1.0, max(ncomm, 1)) if p_in < 1.0 else np.ones(max(ncomm, 1))
    g = sbm(labels, ncomm, pin[:max(ncomm, 1)], p_out=p_out, seed=seed)
    omega = rng.standard_normal(n)
    theta0 = rng.uniform(0.0, 2 * np.pi, n)
    d_sin = np.concatenate([[0.0], rng.standard_normal(p)])
    d_cos = rng.standard_normal(p + 1) * 0.5
    return PhaseProblem("random_n%d" % n, g, omega, theta0, K=float(rng.uniform(0.5, 4)),
                        dt=0.01, steps=10, d_sin=d_sin, d_cos=d_cos)


# --------------------------------------------------------------------------
# Triadic (higher-order) workload
# --------------------------------------------------------------------------

@dataclass
class TriadicProblem:
    name: str
    graph: Graph                # pairwise adjacency
    tri_seed: int               # seed of the intra-community hyperedge predicate
    p_tri: float                # probability of an intra-community triple
    cross_tri: np.ndarray       # int32 [m,3] hyperedges not inside one community
    omega: np.ndarray
    theta0: np.ndarray
    K1: float
    K2: float
    dt: float
    steps: int


def triadic(seed: int = 3, n: int = 100_000, lo: int = 200, hi: int = 2000,
            p_in: float = 0.9, inter_deg: float = 3.0, p_tri: float = 0.9,
            tri_per_node: float = 1.0) -> TriadicProblem:
    """Sizes U[lo,hi]; pairwise p_in 0.9 with mean inter degree 3; intra
    triples present with probability p_tri (hash predicate); n*tri_per_node
    cross triples, so each node sits in 3*tri_per_node of them on average."""
    rng = np.random.default_rng(seed)
    hi = min(hi, n)
    lo = min(lo, hi)
    sizes = uniform_sizes(n, lo, hi, rng)
    labels = shuffled_labels(sizes, n, rng)
    g = sbm(labels, len(sizes), p_in, n_inter=int(round(inter_deg * n / 2)), seed=seed)
    tri = cross_triangles(labels, int(round(tri_per_node * n)), seed + 17)
    omega = rng.standard_normal(n)
    theta0 = rng.uniform(0.0, 2 * np.pi, n)
    return TriadicProblem("triadic_n%d" % n, g, seed * 7919 + 11, p_tri, tri, omega, theta0,
                          K1=4.0, K2=4.0, dt=0.01, steps=200)


# --------------------------------------------------------------------------
# Cucker-Smale workload
# --------------------------------------------------------------------------

@dataclass
class FlockProblem:
    name: str
    graph: Graph
    x0: np.ndarray      # float64 [3, n]
    v0: np.ndarray      # float64 [3, n]
    K: float
    sigma: float
    beta: float
    dt: float
    steps: int


def flock(seed: int = 4, n: int = 200_000, ncomm: int = 400, p_in: float = 0.8,
          inter_deg: float = 4.0, box: float = 10.0) -> FlockProblem:
    """ncomm equal communities, p_in 0.8, mean inter degree 4, x ~ U[0,box]^3,
    v ~ N(0,1)^3, weight 1/(1+r^2)^(1/4)."""
    rng = np.random.default_rng(seed)
    sizes = np.full(ncomm, n // ncomm, dtype=np.int64)
    sizes[: n - int(sizes.sum())] += 1
    labels = shuffled_labels(sizes, n, rng)
    g = sbm(labels, ncomm, p_in, n_inter=int(round(inter_deg * n / 2)), seed=seed)
    x0 = rng.uniform(0.0, box, (3, n))
    v0 = rng.standard_normal((3, n))
    return FlockProblem("flock_n%d" % n, g, x0, v0, K=1.0, sigma=1.0, beta=0.25, dt=0.01, steps=200)


# --------------------------------------------------------------------------
# Batched ensemble
# --------------------------------------------------------------------------

def ensemble_member(b: int, n_lo: float = 1e3, n_hi: float = 2e5, count: int = 256) -> PhaseProblem:
    """Instance b of the ensemble: N log-uniform in [n_lo, n_hi], 4..500 equal
    communities, p_in ~ U[0.7,0.95], p_out log-uniform in [1e-4,1e-2],
    K = 6 b/(count-1), omega ~ N(0,1), seed 5000+b."""
    seed = 5000 + b
    rng = np.random.default_rng(seed)
    n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
    m = int(rng.integers(4, 501))
    m = max(1, min(m, n // 2))
    sizes = np.full(m, n // m, dtype=np.int64)
    sizes[: n - int(sizes.sum())] += 1
    labels = shuffled_labels(sizes, n, rng)
    p_in = float(rng.uniform(0.7, 0.95))
    p_out = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
    g = sbm(labels, m, p_in, p_out=p_out, seed=seed)
    omega = rng.standard_normal(n)
    theta0 = rng.uniform(0.0, 2 * np.pi, n)
    K = 6.0 * b / max(count - 1, 1)
    return PhaseProblem("ensemble_%d" % b, g, omega, theta0, K=K, dt=0.01, steps=1000)
