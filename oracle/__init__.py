"""FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

Two independent realisations of the same definitions:

* ``liboracle.so`` (oracle.c): plain FP64 direct sums over a CSR adjacency or
  hypergraph, libm, OpenMP over rows; classical RK4 / explicit Euler.
* the ``dense_*`` functions below: NumPy brute force over a dense adjacency
  matrix, for tiny N only.

Definitions followed: eq. (2.1)/(2.2) (general network model), the phase
model of Sec. 3 with the real difference Fourier series of App. A.2, the
higher-order Kuramoto model of App. A.7 (on a hypergraph), and the
Cucker-Smale model of App. A.6.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.c_void_p
_vp = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile the oracle: gcc -O2, no fast-math (libm sin/cos, IEEE FP64)."""
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "basis.c", "structured.c", "poly.c")]
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(os.path.getmtime(f) for f in srcs):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-shared", "-fPIC", "-std=c11", "-o", tmp] + srcs + ["-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        d, i32, i64, u64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        lib.oracle_phase_rhs.restype = None
        lib.oracle_phase_rhs.argtypes = [i64, _vp, _vp, ctypes.c_int, _vp, d, ctypes.c_int, _vp, _vp,
                                         _vp, _vp, i64, _vp]
        lib.oracle_order_parameter.restype = d
        lib.oracle_order_parameter.argtypes = [i64, _vp]
        lib.oracle_phase_integrate.restype = ctypes.c_int
        lib.oracle_phase_integrate.argtypes = [i64, _vp, _vp, ctypes.c_int, _vp, d, ctypes.c_int, _vp,
                                               _vp, _vp, d, i64, ctypes.c_int, _vp]
        lib.oracle_splitmix64.restype = u64
        lib.oracle_splitmix64.argtypes = [u64]
        lib.oracle_triple_present.restype = ctypes.c_int
        lib.oracle_triple_present.argtypes = [u64, u64, i32, i32, i32]
        lib.oracle_triple_threshold.restype = u64
        lib.oracle_triple_threshold.argtypes = [d]
        lib.oracle_triadic_rhs.restype = None
        lib.oracle_triadic_rhs.argtypes = [i64, _vp, _vp, _vp, u64, d, i64, _vp, _vp, d, d, _vp, _vp,
                                           i64, _vp]
        lib.oracle_triadic_integrate.restype = ctypes.c_int
        lib.oracle_triadic_integrate.argtypes = [i64, _vp, _vp, _vp, u64, d, i64, _vp, _vp, d, d, _vp,
                                                 d, i64, ctypes.c_int, _vp]
        lib.oracle_cs_rhs.restype = None
        lib.oracle_cs_rhs.argtypes = [i64, ctypes.c_int, _vp, _vp, ctypes.c_int, d, d, d, _vp, _vp,
                                      _vp, i64, _vp, _vp]
        lib.oracle_cs_integrate.restype = ctypes.c_int
        lib.oracle_cs_integrate.argtypes = [i64, ctypes.c_int, _vp, _vp, ctypes.c_int, d, d, d, _vp,
                                            _vp, d, i64, ctypes.c_int]
        lib.oracle_gauss_legendre.restype = None
        lib.oracle_gauss_legendre.argtypes = [ctypes.c_int, _vp, _vp]
        lib.oracle_cs_fourier_coeffs.restype = ctypes.c_int
        lib.oracle_cs_fourier_coeffs.argtypes = [d, d, d, d, ctypes.c_int, ctypes.c_int, _vp]
        lib.oracle_cs_fourier_weight.restype = d
        lib.oracle_cs_fourier_weight.argtypes = [_vp, ctypes.c_int, d, _vp]
        lib.oracle_mlp_param_count.restype = i64
        lib.oracle_mlp_param_count.argtypes = [ctypes.c_int]
        lib.oracle_mlp_forward.restype = None
        lib.oracle_mlp_forward.argtypes = [_vp, ctypes.c_int, _vp, _vp, i64, _vp, _vp]
        lib.oracle_mlp_loss_grad.restype = ctypes.c_int
        lib.oracle_mlp_loss_grad.argtypes = [_vp, ctypes.c_int, _vp, _vp, i64, _vp, _vp, _vp, _vp, _vp]
        lib.oracle_cs_rhs_separable.restype = ctypes.c_int
        lib.oracle_cs_rhs_separable.argtypes = [i64, _vp, _vp, ctypes.c_int, _vp, _vp, d, d, d,
                                                ctypes.c_int, _vp, ctypes.c_int, d, _vp, ctypes.c_int,
                                                _vp, _vp, _vp, _vp, _vp, i64, _vp, _vp]
        lib.oracle_structured_rhs.restype = None
        lib.oracle_structured_rhs.argtypes = [ctypes.c_int, i64, i64, _vp, _vp, _vp, d, ctypes.c_int, _vp,
                                              _vp, _vp, _vp, i64, _vp]
        lib.oracle_structured_integrate.restype = ctypes.c_int
        lib.oracle_structured_integrate.argtypes = [ctypes.c_int, i64, i64, _vp, _vp, _vp, d, ctypes.c_int,
                                                    _vp, _vp, _vp, d, i64, ctypes.c_int, _vp]
        lib.oracle_poly_rhs.restype = None
        lib.oracle_poly_rhs.argtypes = [i64, _vp, _vp, ctypes.c_int, _vp, d, ctypes.c_int, _vp, ctypes.c_int, _vp,
                                        _vp, _vp, i64, _vp]
        lib.oracle_poly_integrate.restype = ctypes.c_int
        lib.oracle_poly_integrate.argtypes = [i64, _vp, _vp, ctypes.c_int, _vp, d, ctypes.c_int, _vp, ctypes.c_int,
                                              _vp, _vp, d, i64, ctypes.c_int]
        lib.oracle_phase_rhs_general.restype = None
        lib.oracle_phase_rhs_general.argtypes = [i64, _vp, _vp, ctypes.c_int, _vp, d, ctypes.c_int, _vp, _vp,
                                                 _vp, _vp, _vp, _vp, i64, _vp]
        lib.oracle_poly_rhs_general.restype = None
        lib.oracle_poly_rhs_general.argtypes = [i64, _vp, _vp, ctypes.c_int, _vp, d, ctypes.c_int, _vp,
                                                ctypes.c_int, _vp, _vp, _vp, i64, _vp]
        lib.oracle_osc2_rhs.restype = None
        lib.oracle_osc2_rhs.argtypes = [i64, _vp, _vp, ctypes.c_int, _vp, d, ctypes.c_int, _vp, _vp, _vp, _vp, i64,
                                        _vp]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _csr(row_ptr, col):
    if row_ptr is None:
        return None, None
    return np.ascontiguousarray(row_ptr, dtype=np.int64), np.ascontiguousarray(col, dtype=np.int32)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


# ---------------------------------------------------------------------------
# phase model
# ---------------------------------------------------------------------------

def phase_rhs(n, row_ptr, col, omega, K, d_sin, d_cos, theta, rows=None, complete=False):
    """H_m = omega_m + (K/N) sum_l a_ml h(theta_l - theta_m)  (eq. 2.2 with
    f_m = omega_m; h as in App. A.2).  rows: optional int64 subset."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    d_sin, d_cos = _f64(d_sin), _f64(d_cos)
    p = len(d_sin) - 1
    assert len(d_cos) == p + 1
    theta, omega = _f64(theta), _f64(omega)
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    out = np.empty(cnt, dtype=np.float64)
    lib.oracle_phase_rhs(n, _p(rp), _p(cl), int(bool(complete)), _p(omega), float(K), p, _p(d_sin),
                         _p(d_cos), _p(theta), _p(rws), 0 if rws is None else len(rws), _p(out))
    return out


def phase_rhs_general(n, row_ptr, col, omega, K, c11, c12, c21, c22, theta, rows=None, complete=False):
    """H_m = omega_m + (K/N) sum_l a_ml g(theta_l, theta_m) with g the real
    2-D Fourier series of App. A.2 (eq. FourierRealExpansion); c.. are
    (p+1) x (p+1) arrays, row = partner harmonic, column = own harmonic."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    cs = [np.ascontiguousarray(c, dtype=np.float64) for c in (c11, c12, c21, c22)]
    p = cs[0].shape[0] - 1
    assert all(c.shape == (p + 1, p + 1) for c in cs)
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    out = np.empty(cnt, dtype=np.float64)
    lib.oracle_phase_rhs_general(int(n), _p(rp), _p(cl), int(bool(complete)), _p(_f64(omega)), float(K), p,
                                 *[_p(c) for c in cs], _p(_f64(theta)), _p(rws), 0 if rws is None else len(rws),
                                 _p(out))
    return out


def order_parameter(theta) -> float:
    theta = _f64(theta)
    return float(_load().oracle_order_parameter(len(theta), _p(theta)))


def phase_integrate(n, row_ptr, col, omega, K, d_sin, d_cos, theta0, dt, steps,
                    stepper="rk4", complete=False, trace=True):
    """Returns (theta_final, r_trace or None).  No phase wrapping."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    d_sin, d_cos = _f64(d_sin), _f64(d_cos)
    th = np.array(theta0, dtype=np.float64, copy=True)
    r = np.empty(steps + 1, dtype=np.float64) if trace else None
    rc = lib.oracle_phase_integrate(n, _p(rp), _p(cl), int(bool(complete)), _p(_f64(omega)), float(K),
                                    len(d_sin) - 1, _p(d_sin), _p(d_cos), _p(th), float(dt), int(steps),
                                    1 if stepper == "euler" else 0, _p(r))
    if rc != 0:
        raise MemoryError("oracle_phase_integrate")
    return th, r


# ---------------------------------------------------------------------------
# structured adjacency (App. B): rank one and the k-nearest-neighbour ring
# ---------------------------------------------------------------------------

def _structured_args(kind, n, k, alpha, beta):
    if kind == "rank1":
        alpha, beta = _f64(alpha), _f64(beta)
        assert len(alpha) == n and len(beta) == n
        return 0, 0, alpha, beta
    assert kind == "ring" and k >= 0
    return 1, int(k), None, None


def structured_rhs(kind, n, omega, K, d_sin, d_cos, theta, k=0, alpha=None, beta=None, rows=None):
    """H_m = omega_m + (K/N) sum_l a_ml h(theta_l - theta_m) with a_ml =
    alpha_m beta_l ("rank1", App. B.1) or a_ml = [c_N(m, l) <= k] ("ring",
    App. B.2); l = m included in both."""
    lib = _load()
    kd, kk, alpha, beta = _structured_args(kind, n, k, alpha, beta)
    d_sin, d_cos = _f64(d_sin), _f64(d_cos)
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    out = np.empty(cnt, dtype=np.float64)
    lib.oracle_structured_rhs(kd, int(n), kk, _p(alpha), _p(beta), _p(_f64(omega)), float(K), len(d_sin) - 1,
                              _p(d_sin), _p(d_cos), _p(_f64(theta)), _p(rws), 0 if rws is None else len(rws),
                              _p(out))
    return out


def structured_integrate(kind, n, omega, K, d_sin, d_cos, theta0, dt, steps, k=0, alpha=None, beta=None,
                         stepper="rk4"):
    """Returns (theta_final, r_trace).  No phase wrapping."""
    lib = _load()
    kd, kk, alpha, beta = _structured_args(kind, n, k, alpha, beta)
    d_sin, d_cos = _f64(d_sin), _f64(d_cos)
    th = np.array(theta0, dtype=np.float64, copy=True)
    r = np.empty(steps + 1, dtype=np.float64)
    rc = lib.oracle_structured_integrate(kd, int(n), kk, _p(alpha), _p(beta), _p(_f64(omega)), float(K),
                                         len(d_sin) - 1, _p(d_sin), _p(d_cos), _p(th), float(dt), int(steps),
                                         1 if stepper == "euler" else 0, _p(r))
    if rc != 0:
        raise MemoryError("oracle_structured_integrate")
    return th, r


# ---------------------------------------------------------------------------
# polynomial difference coupling (App. A.3 difference form; Desai-Zwanzig)
# ---------------------------------------------------------------------------

def poly_rhs(n, row_ptr, col, omega, K, h, f, x, rows=None, complete=False):
    """x_m' = omega_m + f(x_m) + (K/N) sum_l a_ml h(x_l - x_m), h and f given by
    their coefficients in increasing powers (f may be None)."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    h = _f64(h)
    fq = -1 if f is None else len(f) - 1
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    out = np.empty(cnt, dtype=np.float64)
    lib.oracle_poly_rhs(int(n), _p(rp), _p(cl), int(bool(complete)), _p(_f64(omega)), float(K), len(h) - 1, _p(h),
                        fq, _p(_f64(f)), _p(_f64(x)), _p(rws), 0 if rws is None else len(rws), _p(out))
    return out


def poly_rhs_general(n, row_ptr, col, omega, K, c, f, x, rows=None, complete=False):
    """x_m' = omega_m + f(x_m) + (K/N) sum_l a_ml g(x_l, x_m), g(x, y) =
    sum_{a,b} c[a, b] x^a y^b (App. A.3, eq. PolyApprox); c is (p+1) x (p+1)."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    c = np.ascontiguousarray(c, dtype=np.float64)
    p = c.shape[0] - 1
    assert c.shape == (p + 1, p + 1)
    fq = -1 if f is None else len(f) - 1
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    out = np.empty(cnt, dtype=np.float64)
    lib.oracle_poly_rhs_general(int(n), _p(rp), _p(cl), int(bool(complete)), _p(_f64(omega)), float(K), p, _p(c),
                                fq, _p(_f64(f)), _p(_f64(x)), _p(rws), 0 if rws is None else len(rws), _p(out))
    return out


def osc2_rhs(n, row_ptr, col, omega, K, h, F, x, rows=None, complete=False):
    """Two-component oscillators (the paper's Table 1, van der Pol /
    FitzHugh-Nagumo): x is [2, n]; F is [2, 4, 4] with f_d(u, v) =
    sum F[d, i, j] u^i v^j; omega (optional) drives component 0.  Returns
    [2, len(rows) or n]."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    h = _f64(h)
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(2, 4, 4)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(2, n)
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    out = np.empty((2, cnt), dtype=np.float64)
    lib.oracle_osc2_rhs(int(n), _p(rp), _p(cl), int(bool(complete)), _p(_f64(omega)), float(K), len(h) - 1, _p(h),
                        _p(F), _p(x), _p(rws), 0 if rws is None else len(rws), _p(out))
    return out


def osc2_integrate(n, row_ptr, col, omega, K, h, F, x0, dt, steps, stepper="rk4"):
    """The two-component system stepped by the classical RK4 (or explicit
    Euler) scheme, each stage one osc2_rhs evaluation."""
    x = np.array(x0, dtype=np.float64, copy=True).reshape(2, n)

    def rhs(y):
        return osc2_rhs(n, row_ptr, col, omega, K, h, F, y)

    for _ in range(int(steps)):
        if stepper == "euler":
            x = x + dt * rhs(x)
            continue
        k1 = rhs(x)
        k2 = rhs(x + 0.5 * dt * k1)
        k3 = rhs(x + 0.5 * dt * k2)
        k4 = rhs(x + dt * k3)
        x = x + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return x


def poly_integrate(n, row_ptr, col, omega, K, h, f, x0, dt, steps, stepper="rk4", complete=False):
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    h = _f64(h)
    fq = -1 if f is None else len(f) - 1
    x = np.array(x0, dtype=np.float64, copy=True)
    rc = lib.oracle_poly_integrate(int(n), _p(rp), _p(cl), int(bool(complete)), _p(_f64(omega)), float(K),
                                   len(h) - 1, _p(h), fq, _p(_f64(f)), _p(x), float(dt), int(steps),
                                   1 if stepper == "euler" else 0)
    if rc != 0:
        raise MemoryError("oracle_poly_integrate")
    return x


# ---------------------------------------------------------------------------
# triadic model
# ---------------------------------------------------------------------------

def splitmix64(x: int) -> int:
    return int(_load().oracle_splitmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def triple_threshold(p: float) -> int:
    return int(_load().oracle_triple_threshold(float(p)))


def triple_present(seed: int, p: float, a: int, b: int, c: int) -> bool:
    lib = _load()
    return bool(lib.oracle_triple_present(int(seed), lib.oracle_triple_threshold(float(p)), a, b, c))


def triadic_rhs(n, row_ptr, col, labels, tri_seed, p_tri, tri, omega, K1, K2, theta, rows=None):
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    out = np.empty(cnt, dtype=np.float64)
    lib.oracle_triadic_rhs(n, _p(rp), _p(cl), _p(labels), int(tri_seed), float(p_tri), len(tri),
                           _p(tri), _p(_f64(omega)), float(K1), float(K2), _p(_f64(theta)), _p(rws),
                           0 if rws is None else len(rws), _p(out))
    return out


def triadic_integrate(n, row_ptr, col, labels, tri_seed, p_tri, tri, omega, K1, K2, theta0, dt,
                      steps, stepper="rk4", trace=True):
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    th = np.array(theta0, dtype=np.float64, copy=True)
    r = np.empty(steps + 1, dtype=np.float64) if trace else None
    rc = lib.oracle_triadic_integrate(n, _p(rp), _p(cl), _p(labels), int(tri_seed), float(p_tri),
                                      len(tri), _p(tri), _p(_f64(omega)), float(K1), float(K2), _p(th),
                                      float(dt), int(steps), 1 if stepper == "euler" else 0, _p(r))
    if rc != 0:
        raise MemoryError("oracle_triadic_integrate")
    return th, r


# ---------------------------------------------------------------------------
# Cucker-Smale
# ---------------------------------------------------------------------------

def cs_rhs(n, row_ptr, col, K, sigma, beta, s, v, rows=None, complete=False):
    """s, v: [dim, n].  Returns (sdot, vdot), each [dim, len(rows) or n]."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    s = np.ascontiguousarray(s, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    dim = s.shape[0]
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    sd = np.empty((dim, cnt), dtype=np.float64)
    vd = np.empty((dim, cnt), dtype=np.float64)
    lib.oracle_cs_rhs(n, dim, _p(rp), _p(cl), int(bool(complete)), float(K), float(sigma), float(beta),
                      _p(s), _p(v), _p(rws), 0 if rws is None else len(rws), _p(sd), _p(vd))
    return sd, vd


def cs_integrate(n, row_ptr, col, K, sigma, beta, s0, v0, dt, steps, stepper="rk4", complete=False):
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    s = np.array(s0, dtype=np.float64, copy=True)
    v = np.array(v0, dtype=np.float64, copy=True)
    rc = lib.oracle_cs_integrate(n, s.shape[0], _p(rp), _p(cl), int(bool(complete)), float(K),
                                 float(sigma), float(beta), _p(s), _p(v), float(dt), int(steps),
                                 1 if stepper == "euler" else 0)
    if rc != 0:
        raise MemoryError("oracle_cs_integrate")
    return s, v


# ---------------------------------------------------------------------------
# NumPy brute force over a dense adjacency (tiny N)
# ---------------------------------------------------------------------------

def dense_from_csr(n, row_ptr, col) -> np.ndarray:
    A = np.zeros((n, n), dtype=np.float64)
    for m in range(n):
        A[m, col[row_ptr[m]:row_ptr[m + 1]]] = 1.0
    return A


def dense_phase_rhs(A, omega, K, d_sin, d_cos, theta):
    """Dense O(N^2) evaluation of eq. (2.2) for the phase model."""
    n = A.shape[0]
    diff = theta[None, :] - theta[:, None]          # diff[m, l] = theta_l - theta_m
    h = np.full_like(diff, d_cos[0])
    for k in range(1, len(d_sin)):
        h += d_sin[k] * np.sin(k * diff) + d_cos[k] * np.cos(k * diff)
    return omega + (K / n) * (A * h).sum(axis=1)


def dense_cs_rhs(A, K, sigma, beta, s, v):
    n = A.shape[0]
    ds = s[:, None, :] - s[:, :, None]               # ds[d, m, l] = s_l - s_m
    w = K / (sigma ** 2 + (ds ** 2).sum(axis=0)) ** beta
    dv = v[:, None, :] - v[:, :, None]
    return v.copy(), (A[None] * w[None] * dv).sum(axis=2) / n


# ---------------------------------------------------------------------------
# separable expansions of the Cucker-Smale weight (basis.c)
# ---------------------------------------------------------------------------

MLP_HIDDEN = 64


def gauss_legendre(m):
    x = np.empty(m)
    w = np.empty(m)
    _load().oracle_gauss_legendre(int(m), _p(x), _p(w))
    return x, w


def cs_fourier_coeffs(K, sigma, beta, L, p, nq=96):
    """c[a1, a2, a3] for |alpha| = (a1, a2, a3) in 0..p (App. A.6)."""
    c = np.empty((p + 1) ** 3)
    if _load().oracle_cs_fourier_coeffs(float(K), float(sigma), float(beta), float(L), int(p), int(nq), _p(c)):
        raise MemoryError("oracle_cs_fourier_coeffs")
    return c.reshape(p + 1, p + 1, p + 1)


def cs_fourier_weight(c, L, y):
    c = np.ascontiguousarray(c, dtype=np.float64)
    p = c.shape[0] - 1
    y = np.ascontiguousarray(y, dtype=np.float64)
    return float(_load().oracle_cs_fourier_weight(_p(c), p, float(L), _p(y)))


def mlp_param_count(R):
    return int(_load().oracle_mlp_param_count(int(R)))


def mlp_forward(params, R, lo, hi, x):
    """x: [3, n] planes -> phi [n, R]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[1]
    out = np.empty((n, R))
    _load().oracle_mlp_forward(_p(_f64(params)), int(R), _p(_f64(lo)), _p(_f64(hi)), n, _p(x), _p(out))
    return out


def mlp_loss_grad(params, R, lo, hi, a, b, t):
    """a, b: [P, 3] pair endpoints, t: [P] targets -> (loss, grad like params)."""
    params = _f64(params)
    a, b, t = _f64(a), _f64(b), _f64(t)
    g = np.empty_like(params)
    loss = np.zeros(1)
    if _load().oracle_mlp_loss_grad(_p(params), int(R), _p(_f64(lo)), _p(_f64(hi)), len(t), _p(a), _p(b),
                                    _p(t), _p(g), _p(loss)):
        raise MemoryError("oracle_mlp_loss_grad")
    return float(loss[0]), g


def cs_rhs_separable(n, row_ptr, col, labels, K, sigma, beta, s, v, basis, fourier=None, L=0.0, mlp=None,
                     R=0, lo=None, hi=None, exact_comm=None, rows=None, complete=False):
    """Cucker-Smale RHS with the expanded weight on intra-community present pairs.
    basis: "fourier" (fourier = coefficient cube, L) or "mlp" (mlp = params, R, lo, hi)."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    s = np.ascontiguousarray(s, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.int32)
    ex = None if exact_comm is None else np.ascontiguousarray(exact_comm, dtype=np.uint8)
    rws = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = n if rws is None else len(rws)
    sd = np.empty((3, cnt))
    vd = np.empty((3, cnt))
    kind = {"fourier": 1, "mlp": 2}[basis]
    c = _f64(fourier) if kind == 1 else None
    p = 0 if c is None else np.asarray(fourier).shape[0] - 1
    rc = lib.oracle_cs_rhs_separable(n, _p(rp), _p(cl), int(bool(complete)), _p(lab), _p(ex), float(K),
                                     float(sigma), float(beta), kind, _p(c), int(p), float(L),
                                     _p(_f64(mlp)), int(R), _p(_f64(lo)), _p(_f64(hi)), _p(s), _p(v),
                                     _p(rws), 0 if rws is None else len(rws), _p(sd), _p(vd))
    if rc:
        raise MemoryError("oracle_cs_rhs_separable")
    return sd, vd
