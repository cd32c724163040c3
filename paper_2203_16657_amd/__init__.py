"""Python binding of libcia (the C ABI in include/cia.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libcia.so.  Functions carry the C names (cia_build, cia_rhs,
cia_integrate, cia_destroy, ...); `Plan` is a small convenience wrapper.
Device memory and streams come from PyTorch tensors (data_ptr / cuda_stream).

The library must be built (``python -m paper_2203_16657_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcia.so")

# ---- constants (mirror of cia.h) ----
CIA_OK, CIA_EINVAL, CIA_ENOMEM, CIA_EHIP, CIA_EUNSUPPORTED, CIA_ENONFINITE = 0, -1, -2, -3, -4, -5
CIA_GRAPH_CSR, CIA_GRAPH_COMPLETE, CIA_GRAPH_RANK1, CIA_GRAPH_RING = 0, 1, 2, 3
CIA_MODEL_PHASE, CIA_MODEL_TRIADIC, CIA_MODEL_FLOCK, CIA_MODEL_POLY = 0, 1, 2, 3
CIA_METHOD_CIA, CIA_METHOD_DIRECT = 0, 1
CIA_F32, CIA_F64 = 0, 1
CIA_RK4, CIA_EULER = 0, 1
CIA_BASIS_EXACT, CIA_BASIS_FOURIER, CIA_BASIS_LEARNED = 0, 1, 2
CIA_FLAG_KEEP_LABELS, CIA_FLAG_TIMING, CIA_FLAG_NO_VALIDATE, CIA_FLAG_HIPGRAPH = 0x1, 0x2, 0x4, 0x8
CIA_FLAG_NO_JUDGE, CIA_FLAG_AUTOTUNE = 0x10, 0x20
CIA_FLAG_FORCE_WIDE, CIA_FLAG_FORCE_NEG32, CIA_FLAG_NO_LDS, CIA_FLAG_NO_RESIDENT = 0x100, 0x200, 0x400, 0x800

_c = ctypes
_vp = ctypes.c_void_p


class cia_graph(_c.Structure):
    _fields_ = [("n", _c.c_int64), ("kind", _c.c_int32), ("reserved", _c.c_int32),
                ("row_ptr", _vp), ("col", _vp), ("alpha", _vp), ("beta", _vp), ("ring_k", _c.c_int64)]


class cia_hypergraph(_c.Structure):
    _fields_ = [("seed", _c.c_uint64), ("p_intra", _c.c_double), ("ntri", _c.c_int64), ("tri", _vp)]


class cia_coupling(_c.Structure):
    _fields_ = [("model", _c.c_int32), ("p", _c.c_int32), ("d_sin", _vp), ("d_cos", _vp),
                ("K", _c.c_double), ("K2", _c.c_double), ("hyper", _vp),
                ("cs_K", _c.c_double), ("cs_sigma", _c.c_double), ("cs_beta", _c.c_double),
                ("cs_L", _c.c_double), ("cs_basis", _c.c_int32), ("rank", _c.c_int32),
                ("train_iters", _c.c_int32), ("reserved", _c.c_int32), ("poly_q", _c.c_int32),
                ("reserved2", _c.c_int32), ("poly_h", _vp), ("poly_f", _vp), ("gen_c11", _vp), ("gen_c12", _vp),
                ("gen_c21", _vp), ("gen_c22", _vp), ("poly_g", _vp),
                ("poly_dim", _c.c_int32), ("reserved3", _c.c_int32), ("poly_f2", _vp)]


class cia_options(_c.Structure):
    _fields_ = [("method", _c.c_int32), ("precision", _c.c_int32), ("stepper", _c.c_int32),
                ("flags", _c.c_uint32), ("dense_alpha", _c.c_double), ("unit_work", _c.c_int32),
                ("block", _c.c_int32), ("judge_tol", _c.c_double), ("device", _c.c_int32),
                ("reserved", _c.c_int32)]


class cia_plan_info(_c.Structure):
    _fields_ = [("n", _c.c_int64), ("nnz_graph", _c.c_int64), ("nnz_neg", _c.c_int64),
                ("nnz_pos", _c.c_int64), ("n_unassigned", _c.c_int64), ("ncomm", _c.c_int32),
                ("nunits", _c.c_int32), ("max_comm", _c.c_int32), ("wide_comms", _c.c_int32),
                ("method", _c.c_int32), ("precision", _c.c_int32), ("model", _c.c_int32),
                ("p", _c.c_int32), ("bytes_per_rhs", _c.c_double), ("bytes_per_stage", _c.c_double),
                ("nnz_extra", _c.c_int64), ("judge_fallbacks", _c.c_int32), ("tiled_comms", _c.c_int32),
                ("bytes_aux", _c.c_double), ("resident", _c.c_int32), ("merged_slices", _c.c_int32)]


class cia_tune_report(_c.Structure):
    _fields_ = [("unit_work", _c.c_int32), ("block", _c.c_int32), ("candidates", _c.c_int32),
                ("reserved", _c.c_int32), ("best_us", _c.c_double), ("default_us", _c.c_double)]


class cia_timing(_c.Structure):
    _fields_ = [("stage_ms", _c.c_double), ("stage_launches", _c.c_int64), ("prep_ms", _c.c_double),
                ("prep_launches", _c.c_int64), ("aux_ms", _c.c_double), ("aux_launches", _c.c_int64)]


EXPORTS = ["cia_build", "cia_rhs", "cia_integrate", "cia_destroy", "cia_last_error",
           "cia_options_default", "cia_coupling_default", "cia_plan_get_info", "cia_plan_get_timing",
           "cia_fourier_coeffs", "cia_p1_build", "cia_p1_sizes", "cia_p1_export", "cia_p1_free",
           "cia_abi_sizeof", "cia_basis_param_count", "cia_basis_set_params", "cia_basis_get_params",
           "cia_basis_train", "cia_basis_loss_grad", "cia_basis_features", "cia_build_batch",
           "cia_batch_offsets", "cia_autotune", "cia_plan_set_timing", "cia_detect_communities",
           "cia_batch_begin", "cia_batch_add", "cia_batch_finish", "cia_batch_abort", "cia_integrate_noalloc"]
CIA_NOALLOC_R_MAX = 1 << 17   # r(t) values the allocation-free entry point can return

_lib = None


class CIAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("cia status %d: %s" % (status, msg))
        self.status = status


def load():
    """Load libcia.so (no fallback: the HIP library is the only implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcia.so is not built (%s); run paper_2203_16657_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = _c.POINTER
    lib.cia_build.restype = _c.c_int
    lib.cia_build.argtypes = [P(cia_graph), _vp, P(cia_coupling), _vp, P(cia_options), P(_vp)]
    lib.cia_rhs.restype = _c.c_int
    lib.cia_rhs.argtypes = [_vp, _vp, _vp, _vp]
    lib.cia_integrate.restype = _c.c_int
    lib.cia_integrate.argtypes = [_vp, _vp, _c.c_double, _c.c_int64, _vp, _vp]
    lib.cia_integrate_noalloc.restype = _c.c_int
    lib.cia_integrate_noalloc.argtypes = [_vp, _vp, _c.c_double, _c.c_int64, _vp, _vp]
    lib.cia_destroy.restype = _c.c_int
    lib.cia_destroy.argtypes = [_vp]
    lib.cia_last_error.restype = _c.c_char_p
    lib.cia_last_error.argtypes = []
    lib.cia_options_default.restype = None
    lib.cia_options_default.argtypes = [P(cia_options)]
    lib.cia_coupling_default.restype = None
    lib.cia_coupling_default.argtypes = [P(cia_coupling)]
    lib.cia_plan_get_info.restype = _c.c_int
    lib.cia_plan_get_info.argtypes = [_vp, P(cia_plan_info)]
    lib.cia_plan_get_timing.restype = _c.c_int
    lib.cia_plan_get_timing.argtypes = [_vp, P(cia_timing), _c.c_int]
    lib.cia_fourier_coeffs.restype = _c.c_int
    lib.cia_fourier_coeffs.argtypes = [_vp, _c.c_int64, _c.c_int32, _vp, _vp]
    lib.cia_p1_build.restype = _c.c_int
    lib.cia_p1_build.argtypes = [P(cia_graph), _vp, P(cia_options), P(_vp)]
    lib.cia_detect_communities.restype = _c.c_int
    lib.cia_detect_communities.argtypes = [P(cia_graph), _vp, _c.c_double, _vp, P(_c.c_double)]
    lib.cia_p1_sizes.restype = _c.c_int
    lib.cia_p1_sizes.argtypes = [_vp, _vp]
    lib.cia_p1_export.restype = _c.c_int
    lib.cia_p1_export.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.cia_p1_free.restype = _c.c_int
    lib.cia_p1_free.argtypes = [_vp]
    lib.cia_abi_sizeof.restype = _c.c_size_t
    lib.cia_abi_sizeof.argtypes = [_c.c_char_p]
    lib.cia_basis_param_count.restype = _c.c_int
    lib.cia_basis_param_count.argtypes = [_c.c_int32, _vp]
    lib.cia_basis_set_params.restype = _c.c_int
    lib.cia_basis_set_params.argtypes = [_vp, _vp, _c.c_int64, _vp, _vp]
    lib.cia_basis_get_params.restype = _c.c_int
    lib.cia_basis_get_params.argtypes = [_vp, _vp, _c.c_int64, _vp, _vp]
    lib.cia_basis_train.restype = _c.c_int
    lib.cia_basis_train.argtypes = [_vp, _vp, _c.c_int32, _c.c_uint64, _vp, _vp]
    lib.cia_basis_loss_grad.restype = _c.c_int
    lib.cia_basis_loss_grad.argtypes = [_vp, _vp, _vp, _vp, _c.c_int64, _vp, _vp, _vp]
    lib.cia_basis_features.restype = _c.c_int
    lib.cia_basis_features.argtypes = [_vp, _vp, _c.c_int64, _vp, _vp]
    lib.cia_build_batch.restype = _c.c_int
    lib.cia_build_batch.argtypes = [_c.c_int32, _vp, _vp, _vp, _vp, P(cia_options), P(_vp)]
    lib.cia_batch_begin.restype = _c.c_int
    lib.cia_batch_begin.argtypes = [P(cia_options), P(_vp)]
    lib.cia_batch_add.restype = _c.c_int
    lib.cia_batch_add.argtypes = [_vp, P(cia_graph), _vp, P(cia_coupling), _vp]
    lib.cia_batch_finish.restype = _c.c_int
    lib.cia_batch_finish.argtypes = [_vp, P(_vp)]
    lib.cia_batch_abort.restype = None
    lib.cia_batch_abort.argtypes = [_vp]
    lib.cia_batch_offsets.restype = _c.c_int
    lib.cia_batch_offsets.argtypes = [_vp, _vp, _vp]
    lib.cia_plan_set_timing.restype = _c.c_int
    lib.cia_plan_set_timing.argtypes = [_vp, _c.c_int32]
    lib.cia_autotune.restype = _c.c_int
    lib.cia_autotune.argtypes = [_vp, _vp, P(cia_tune_report)]
    _lib = lib
    return lib


def _check(st):
    if st != CIA_OK:
        raise CIAError(st, cia_last_error())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(_vp)


def _dev_ptr(t):
    """Device pointer of a tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _need_len(name, a, n):
    """The C side reads exactly n entries of a host array: check before the call."""
    if a is not None and (a.ndim != 1 or a.shape[0] != n):
        raise ValueError("%s: expected %d entries, got shape %s" % (name, n, tuple(a.shape)))


def _check_csr(n, row_ptr, col):
    if row_ptr is None or col is None:
        raise ValueError("row_ptr and col are required for a CSR graph")
    _need_len("row_ptr", row_ptr, n + 1)
    if row_ptr[0] != 0 or (n and row_ptr[-1] > col.shape[0]):
        raise ValueError("row_ptr must start at 0 and end at most at len(col) = %d" % col.shape[0])


def _check_state(plan, t, name):
    """A device tensor of plan.n * plan.dim values in the plan's precision
    (the kernels read and write exactly that many)."""
    import torch
    if isinstance(t, int):
        return
    want = torch.float64 if plan.precision == CIA_F64 else torch.float32
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if t.dtype != want or not t.is_contiguous() or t.numel() != plan.n * plan.dim:
        raise ValueError("%s: expected a contiguous %s tensor of %d values, got %s with %d" % (
            name, want, plan.n * plan.dim, t.dtype, t.numel()))


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# the C functions, one to one
# ---------------------------------------------------------------------------

def cia_last_error() -> str:
    return load().cia_last_error().decode(errors="replace")


def cia_options_default() -> cia_options:
    o = cia_options()
    load().cia_options_default(_c.byref(o))
    return o


def cia_coupling_default() -> cia_coupling:
    c = cia_coupling()
    load().cia_coupling_default(_c.byref(c))
    return c


def cia_build(graph: cia_graph, labels, coupling: cia_coupling, omega, options: cia_options | None):
    """Returns the plan handle (int).  labels/omega: numpy arrays or None.
    The caller keeps the arrays referenced by `graph` / `coupling` alive for
    the duration of the call."""
    lib = load()
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.int32)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
    _need_len("labels", lab, graph.n)
    _need_len("omega", om, graph.n)
    out = _vp()
    st = lib.cia_build(_c.byref(graph), _np_ptr(lab), _c.byref(coupling), _np_ptr(om),
                       None if options is None else _c.byref(options), _c.byref(out))
    _check(st)
    return out.value


def cia_rhs(plan, state, dstate, stream=None) -> None:
    _check(load().cia_rhs(plan, _dev_ptr(state), _dev_ptr(dstate), _stream_ptr(stream)))


def _trace_ptr(plan, r_trace, steps: int):
    """Host pointer of an r(t) trace after checking it can hold what the
    library writes: (steps + 1) doubles per instance of the plan."""
    if r_trace is None:
        return None
    if not isinstance(r_trace, np.ndarray) or r_trace.dtype != np.float64:
        raise ValueError("r_trace must be a float64 numpy array")
    if not (r_trace.flags.c_contiguous and r_trace.flags.writeable):
        raise ValueError("r_trace must be C-contiguous and writeable")
    if int(steps) < 0:
        raise ValueError("steps must be >= 0")
    cnt = _c.c_int32(0)
    _check(load().cia_batch_offsets(plan, _c.byref(cnt), None))
    need = int(cnt.value) * (int(steps) + 1)
    if r_trace.size < need:
        raise ValueError("r_trace holds %d values; this plan writes %d (%d instance(s) x %d steps + 1)" % (
            r_trace.size, need, cnt.value, int(steps)))
    return _np_ptr(r_trace)


def cia_integrate(plan, state, dt: float, steps: int, r_trace=None, stream=None) -> None:
    rt = _trace_ptr(plan, r_trace, steps)
    _check(load().cia_integrate(plan, _dev_ptr(state), float(dt), int(steps), rt, _stream_ptr(stream)))


def cia_integrate_noalloc(plan, state, dt: float, steps: int, r_trace=None, stream=None) -> None:
    """cia_integrate without any device allocation (r(t) in the library's
    static scratch array of CIA_NOALLOC_R_MAX values)."""
    rt = _trace_ptr(plan, r_trace, steps)
    _check(load().cia_integrate_noalloc(plan, _dev_ptr(state), float(dt), int(steps), rt, _stream_ptr(stream)))


def cia_destroy(plan) -> None:
    if plan:
        _check(load().cia_destroy(plan))


def cia_plan_get_info(plan) -> cia_plan_info:
    info = cia_plan_info()
    _check(load().cia_plan_get_info(plan, _c.byref(info)))
    return info


def cia_plan_get_timing(plan, reset: bool = False) -> cia_timing:
    t = cia_timing()
    _check(load().cia_plan_get_timing(plan, _c.byref(t), int(bool(reset))))
    return t


def cia_fourier_coeffs(samples, p: int):
    s = np.ascontiguousarray(samples, dtype=np.float64)
    ds = np.zeros(p + 1)
    dc = np.zeros(p + 1)
    _check(load().cia_fourier_coeffs(_np_ptr(s), len(s), int(p), _np_ptr(ds), _np_ptr(dc)))
    return ds, dc


def cia_abi_sizeof(name: str) -> int:
    return int(load().cia_abi_sizeof(name.encode()))


def cia_p1(n, row_ptr, col, labels=None, options=None, complete=False):
    """Run P1 on the host and return a dict of numpy arrays (perm, comm_off,
    negptr, neg, posptr, pos) plus the sizes."""
    lib = load()
    rp = None if complete else np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = None if complete else np.ascontiguousarray(col, dtype=np.int32)
    g = cia_graph(n=n, kind=CIA_GRAPH_COMPLETE if complete else CIA_GRAPH_CSR, reserved=0,
                  row_ptr=_np_ptr(rp), col=_np_ptr(cl))
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.int32)
    h = _vp()
    _check(lib.cia_p1_build(_c.byref(g), _np_ptr(lab), None if options is None else _c.byref(options),
                            _c.byref(h)))
    try:
        sz = np.zeros(6, dtype=np.int64)
        _check(lib.cia_p1_sizes(h, _np_ptr(sz)))
        n_, ncomm, nneg, npos, nun, nnz = (int(x) for x in sz)
        out = dict(perm=np.empty(n_, np.int32), comm_off=np.empty(ncomm + 1, np.int32),
                   negptr=np.zeros(n_ + 1, np.int64), neg=np.empty(max(nneg, 1), np.int32),
                   posptr=np.zeros(n_ + 1, np.int64), pos=np.empty(max(npos, 1), np.int32))
        _check(lib.cia_p1_export(h, *[_np_ptr(out[k]) for k in
                                      ("perm", "comm_off", "negptr", "neg", "posptr", "pos")]))
        out["neg"] = out["neg"][:nneg]
        out["pos"] = out["pos"][:npos]
        out.update(n=n_, ncomm=ncomm, nnz_neg=nneg, nnz_pos=npos, n_unassigned=nun, nnz_graph=nnz)
        return out
    finally:
        lib.cia_p1_free(h)


def detect_communities(n, row_ptr, col, init_labels=None, dense_alpha=2.0):
    """Community labels minimising the work of one CIA right-hand side (host
    only).  Returns (labels int32 [n], -1 = no community; work)."""
    lib = load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    g = cia_graph(n=int(n), kind=CIA_GRAPH_CSR, reserved=0, row_ptr=_np_ptr(rp), col=_np_ptr(cl))
    init = None if init_labels is None else np.ascontiguousarray(init_labels, dtype=np.int32)
    labels = np.empty(int(n), dtype=np.int32)
    work = _c.c_double(0.0)
    _check(lib.cia_detect_communities(_c.byref(g), _np_ptr(init), float(dense_alpha), _np_ptr(labels),
                                      _c.byref(work)))
    return labels, float(work.value)


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

def cia_build_batch(graphs, labels, couplings, omegas, options: cia_options | None):
    """graphs: list of cia_graph; labels / omegas: lists of arrays or None."""
    lib = load()
    count = len(graphs)
    G = (cia_graph * count)(*graphs)
    C = (cia_coupling * count)(*couplings)
    keep = []
    lab_arr = None
    if labels is not None:
        lab_arr = (_vp * count)()
        for b, l in enumerate(labels):
            if l is not None:
                a = np.ascontiguousarray(l, dtype=np.int32)
                _need_len("labels[%d]" % b, a, graphs[b].n)
                keep.append(a)
                lab_arr[b] = a.ctypes.data
    om_arr = None
    if omegas is not None:
        om_arr = (_vp * count)()
        for b, w in enumerate(omegas):
            if w is not None:
                a = np.ascontiguousarray(w, dtype=np.float64)
                _need_len("omega[%d]" % b, a, graphs[b].n)
                keep.append(a)
                om_arr[b] = a.ctypes.data
    out = _vp()
    o = options if options is not None else cia_options_default()
    _check(lib.cia_build_batch(count, _c.cast(G, _vp), None if lab_arr is None else _c.cast(lab_arr, _vp),
                               _c.cast(C, _vp), None if om_arr is None else _c.cast(om_arr, _vp), _c.byref(o),
                               _c.byref(out)))
    return out.value


def cia_batch_offsets(plan):
    cnt = _c.c_int32(0)
    _check(load().cia_batch_offsets(plan, _c.byref(cnt), None))
    off = np.empty(cnt.value + 1, dtype=np.int64)
    _check(load().cia_batch_offsets(plan, _c.byref(cnt), _np_ptr(off)))
    return off


def cia_plan_set_timing(plan, every: int) -> None:
    _check(load().cia_plan_set_timing(plan, int(every)))


def cia_autotune(plan, stream=None) -> cia_tune_report:
    rep = cia_tune_report()
    _check(load().cia_autotune(plan, _stream_ptr(stream), _c.byref(rep)))
    return rep


def cia_basis_param_count(rank: int) -> int:
    cnt = _c.c_int64(0)
    _check(load().cia_basis_param_count(int(rank), _c.byref(cnt)))
    return int(cnt.value)


def cia_basis_set_params(plan, params, lo, hi) -> None:
    pr = np.ascontiguousarray(params, dtype=np.float32)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    _check(load().cia_basis_set_params(plan, _np_ptr(pr), len(pr), _np_ptr(lo), _np_ptr(hi)))


def cia_basis_get_params(plan, count: int):
    pr = np.empty(count, dtype=np.float32)
    lo = np.empty(3)
    hi = np.empty(3)
    _check(load().cia_basis_get_params(plan, _np_ptr(pr), count, _np_ptr(lo), _np_ptr(hi)))
    return pr, lo, hi


def cia_basis_train(plan, state, iters: int, seed: int = 1, loss_trace=None, stream=None) -> None:
    lt = None
    if loss_trace is not None:
        assert loss_trace.dtype == np.float64 and loss_trace.flags.c_contiguous and len(loss_trace) >= iters
        lt = _np_ptr(loss_trace)
    _check(load().cia_basis_train(plan, _dev_ptr(state), int(iters), int(seed) & 0xFFFFFFFFFFFFFFFF, lt,
                                  _stream_ptr(stream)))


def cia_basis_loss_grad(plan, a, b, t, grad, stream=None) -> float:
    loss = _c.c_double(0.0)
    _check(load().cia_basis_loss_grad(plan, _dev_ptr(a), _dev_ptr(b), _dev_ptr(t), int(t.numel()),
                                      _dev_ptr(grad), _c.byref(loss), _stream_ptr(stream)))
    return float(loss.value)


def cia_basis_features(plan, x, out, stream=None) -> None:
    _check(load().cia_basis_features(plan, _dev_ptr(x), int(x.shape[1]), _dev_ptr(out), _stream_ptr(stream)))


class BatchBuilder:
    """Incremental ensemble build (cia_batch_begin / _add / _finish): instances
    are added one at a time, each running P1 on its own graph, so the caller
    can generate an instance, add it and drop its graph before the next.
    finish() returns the same Plan that Plan.batch builds from the full list."""

    def __init__(self, method=CIA_METHOD_CIA, precision=CIA_F32, stepper=CIA_RK4, flags=0, unit_work=0,
                 block=0, device=-1):
        lib = load()
        o = cia_options_default()
        o.method, o.precision, o.stepper, o.flags = method, precision, stepper, flags
        o.unit_work, o.block, o.device = unit_work, block, device
        h = _vp()
        _check(lib.cia_batch_begin(_c.byref(o), _c.byref(h)))
        self.handle = h.value
        self.precision = precision
        self.n = 0
        self.count = 0
        self._ds = np.array([0.0, 1.0])
        self._dc = np.array([0.0, 0.0])

    def add(self, n, row_ptr, col, labels=None, omega=None, K=1.0):
        """Append one phase-model instance with h = sin (arrays borrowed for the call)."""
        if self.handle is None:
            raise ValueError("batch already finished or aborted")
        n = int(n)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        _check_csr(n, rp, cl)
        lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.int32)
        om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
        _need_len("labels", lab, n)
        _need_len("omega", om, n)
        g = cia_graph(n=n, kind=CIA_GRAPH_CSR, reserved=0, row_ptr=_np_ptr(rp), col=_np_ptr(cl))
        c = cia_coupling_default()
        c.model, c.p, c.d_sin, c.d_cos, c.K = CIA_MODEL_PHASE, 1, _np_ptr(self._ds), _np_ptr(self._dc), float(K)
        _check(load().cia_batch_add(self.handle, _c.byref(g), _np_ptr(lab), _c.byref(c), _np_ptr(om)))
        self.n += n
        self.count += 1

    def finish(self):
        if self.handle is None:
            raise ValueError("batch already finished or aborted")
        h, self.handle = self.handle, None
        out = _vp()
        _check(load().cia_batch_finish(h, _c.byref(out)))
        plan = Plan(out.value, self.n, self.precision, CIA_MODEL_PHASE)
        plan.offsets = cia_batch_offsets(out.value)
        return plan

    def abort(self):
        if self.handle is not None:
            load().cia_batch_abort(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.abort()
        except Exception:
            pass


class Plan:
    """Owns a cia_plan.  Build with Plan.phase(...) (more models below)."""

    def __init__(self, handle, n, precision, model, dim=1):
        self.handle = handle
        self.n = n
        self.precision = precision
        self.model = model
        self.dim = dim

    @classmethod
    def phase(cls, n, row_ptr=None, col=None, labels=None, omega=None, K=1.0, d_sin=(0.0, 1.0),
              d_cos=(0.0, 0.0), method=CIA_METHOD_CIA, precision=CIA_F32, stepper=CIA_RK4,
              flags=0, complete=False, unit_work=0, block=0, dense_alpha=2.0, device=-1, gen=None):
        """gen: optional (c11, c12, c21, c22), (p+1) x (p+1) arrays of a general
        coupling g(theta_l, theta_m) (App. A.2 real 2-D series); then d_sin and
        d_cos are not used."""
        load()
        rp = None if complete else np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = None if complete else np.ascontiguousarray(col, dtype=np.int32)
        if not complete:
            _check_csr(int(n), rp, cl)
        g = cia_graph(n=int(n), kind=CIA_GRAPH_COMPLETE if complete else CIA_GRAPH_CSR, reserved=0,
                      row_ptr=_np_ptr(rp), col=_np_ptr(cl))
        ds = np.ascontiguousarray(d_sin, dtype=np.float64)
        dc = np.ascontiguousarray(d_cos, dtype=np.float64)
        c = cia_coupling_default()
        c.model = CIA_MODEL_PHASE
        c.p = len(ds) - 1
        c.d_sin = _np_ptr(ds)
        c.d_cos = _np_ptr(dc)
        c.K = float(K)
        if gen is not None:
            gc = [np.ascontiguousarray(x, dtype=np.float64) for x in gen]
            c.p = gc[0].shape[0] - 1
            assert all(x.shape == (c.p + 1, c.p + 1) for x in gc)
            c.gen_c11, c.gen_c12, c.gen_c21, c.gen_c22 = (_np_ptr(x) for x in gc)
        o = cia_options_default()
        o.method, o.precision, o.stepper, o.flags = method, precision, stepper, flags
        o.unit_work, o.block, o.dense_alpha, o.device = unit_work, block, dense_alpha, device
        h = cia_build(g, labels, c, omega, o)
        return cls(h, int(n), precision, CIA_MODEL_PHASE)

    @classmethod
    def poly(cls, n, row_ptr=None, col=None, labels=None, omega=None, K=1.0, h=(0.0, 1.0), f=None,
             method=CIA_METHOD_CIA, precision=CIA_F32, stepper=CIA_RK4, flags=0, complete=False, unit_work=0,
             block=0, dense_alpha=2.0, device=-1, g=None, dim=1, f2=None):
        """Polynomial difference coupling (App. A.3; Desai-Zwanzig, App. A.5):
        x_m' = omega_m + f(x_m) + (K/N) sum_l a_ml h(x_l - x_m), h and f by
        their coefficients in increasing powers (f optional).  dim=2: two
        components per node (van der Pol / FitzHugh-Nagumo of Table 1), state
        [2, n], h on each component, local terms f2[d, i, j] u^i v^j (f2 a
        [2, 4, 4] array, optional; f and g not allowed), omega on component 0."""
        load()
        rp = None if complete else np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = None if complete else np.ascontiguousarray(col, dtype=np.int32)
        if not complete:
            _check_csr(int(n), rp, cl)
        graph = cia_graph(n=int(n), kind=CIA_GRAPH_COMPLETE if complete else CIA_GRAPH_CSR, reserved=0,
                          row_ptr=_np_ptr(rp), col=_np_ptr(cl))
        hc = np.ascontiguousarray(h, dtype=np.float64)
        fc = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        c = cia_coupling_default()
        c.model = CIA_MODEL_POLY
        c.p = len(hc) - 1
        c.poly_h = _np_ptr(hc)
        c.poly_q = -1 if fc is None else len(fc) - 1
        c.poly_f = _np_ptr(fc)
        if g is not None:
            # general coupling g(x_l, x_m) = sum c[a, b] x_l^a x_m^b replaces h
            gc = np.ascontiguousarray(g, dtype=np.float64)
            c.p = gc.shape[0] - 1
            assert gc.shape == (c.p + 1, c.p + 1)
            c.poly_g = _np_ptr(gc)
        c.poly_dim = int(dim)
        f2c = None
        if f2 is not None:
            f2c = np.ascontiguousarray(f2, dtype=np.float64)
            assert f2c.shape == (2, 4, 4)
            c.poly_f2 = _np_ptr(f2c)
        c.K = float(K)
        o = cia_options_default()
        o.method, o.precision, o.stepper, o.flags = method, precision, stepper, flags
        o.unit_work, o.block, o.dense_alpha, o.device = unit_work, block, dense_alpha, device
        h_ = cia_build(graph, labels, c, omega, o)
        return cls(h_, int(n), precision, CIA_MODEL_POLY, dim=max(1, int(dim)))

    @classmethod
    def structured(cls, n, kind, omega=None, K=1.0, d_sin=(0.0, 1.0), d_cos=(0.0, 0.0), alpha=None, beta=None,
                   ring_k=0, method=CIA_METHOD_CIA, precision=CIA_F32, stepper=CIA_RK4, flags=0, device=-1):
        """Phase model on a structured adjacency (App. B): kind "rank1"
        (a_ml = alpha_m beta_l) or "ring" (a_ml = 1 iff the circular distance
        of m and l is at most ring_k); l = m is coupled in both."""
        load()
        al = be = None
        if kind == "rank1":
            if alpha is None or beta is None:
                raise ValueError("rank1 needs alpha and beta")
            al = np.ascontiguousarray(alpha, dtype=np.float64)
            be = np.ascontiguousarray(beta, dtype=np.float64)
            _need_len("alpha", al, int(n))
            _need_len("beta", be, int(n))
            gk = CIA_GRAPH_RANK1
        elif kind == "ring":
            gk = CIA_GRAPH_RING
        else:
            raise ValueError("kind must be 'rank1' or 'ring'")
        g = cia_graph(n=int(n), kind=gk, reserved=0, row_ptr=None, col=None, alpha=_np_ptr(al), beta=_np_ptr(be),
                      ring_k=int(ring_k))
        ds = np.ascontiguousarray(d_sin, dtype=np.float64)
        dc = np.ascontiguousarray(d_cos, dtype=np.float64)
        c = cia_coupling_default()
        c.model = CIA_MODEL_PHASE
        c.p = len(ds) - 1
        c.d_sin = _np_ptr(ds)
        c.d_cos = _np_ptr(dc)
        c.K = float(K)
        o = cia_options_default()
        o.method, o.precision, o.stepper, o.flags, o.device = method, precision, stepper, flags, device
        h = cia_build(g, None, c, omega, o)
        return cls(h, int(n), precision, CIA_MODEL_PHASE)

    @classmethod
    def triadic(cls, n, row_ptr, col, labels, omega=None, K1=1.0, K2=1.0, tri_seed=0, p_tri=0.9,
                cross_tri=None, method=CIA_METHOD_CIA, precision=CIA_F32, stepper=CIA_RK4, flags=0,
                unit_work=0, block=0, device=-1):
        """Higher-order Kuramoto model on a hypergraph: pairwise sine coupling
        (K1/N) plus the triadic term (K2/N^2); intra-community triples by the
        seeded predicate with probability p_tri, cross triples listed."""
        load()
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        _check_csr(int(n), rp, cl)
        g = cia_graph(n=int(n), kind=CIA_GRAPH_CSR, reserved=0, row_ptr=_np_ptr(rp), col=_np_ptr(cl))
        tri = np.ascontiguousarray(np.zeros((0, 3)) if cross_tri is None else cross_tri, dtype=np.int32)
        h = cia_hypergraph(seed=int(tri_seed) & 0xFFFFFFFFFFFFFFFF, p_intra=float(p_tri), ntri=len(tri),
                           tri=_np_ptr(tri) if len(tri) else None)
        c = cia_coupling_default()
        c.model = CIA_MODEL_TRIADIC
        c.K = float(K1)
        c.K2 = float(K2)
        c.hyper = ctypes.cast(ctypes.pointer(h), _vp)
        o = cia_options_default()
        o.method, o.precision, o.stepper, o.flags = method, precision, stepper, flags
        o.unit_work, o.block, o.device = unit_work, block, device
        handle = cia_build(g, labels, c, omega, o)
        return cls(handle, int(n), precision, CIA_MODEL_TRIADIC)

    @classmethod
    def batch(cls, problems, method=CIA_METHOD_CIA, precision=CIA_F32, stepper=CIA_RK4, flags=0, unit_work=0,
              block=0, device=-1):
        """Ensemble of phase-model networks: problems is a list of
        (n, row_ptr, col, labels, omega, K); h = sin."""
        load()
        keep, graphs, coups = [], [], []
        ds = np.array([0.0, 1.0])
        dc = np.array([0.0, 0.0])
        for (n, row_ptr, col, labels, omega, K) in problems:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            _check_csr(int(n), rp, cl)
            keep += [rp, cl]
            graphs.append(cia_graph(n=int(n), kind=CIA_GRAPH_CSR, reserved=0, row_ptr=_np_ptr(rp), col=_np_ptr(cl)))
            c = cia_coupling_default()
            c.model, c.p, c.d_sin, c.d_cos, c.K = CIA_MODEL_PHASE, 1, _np_ptr(ds), _np_ptr(dc), float(K)
            coups.append(c)
        o = cia_options_default()
        o.method, o.precision, o.stepper, o.flags = method, precision, stepper, flags
        o.unit_work, o.block, o.device = unit_work, block, device
        h = cia_build_batch(graphs, [q[3] for q in problems], coups, [q[4] for q in problems], o)
        plan = cls(h, int(sum(q[0] for q in problems)), precision, CIA_MODEL_PHASE)
        plan.offsets = cia_batch_offsets(h)
        return plan

    def set_timing(self, every: int):
        cia_plan_set_timing(self.handle, every)

    def autotune(self, stream=None) -> cia_tune_report:
        return cia_autotune(self.handle, stream)

    @classmethod
    def flock(cls, n, row_ptr, col, labels=None, K=1.0, sigma=1.0, beta=0.25, basis=CIA_BASIS_EXACT, rank=32,
              p=1, L=20.0, train_iters=0, method=CIA_METHOD_CIA, stepper=CIA_RK4, flags=0, judge_tol=1e-3,
              dense_alpha=2.0, device=-1):
        """Cucker-Smale flocking in 3-D (state: 6 planes s_x, s_y, s_z, v_x, v_y, v_z)."""
        load()
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        _check_csr(int(n), rp, cl)
        g = cia_graph(n=int(n), kind=CIA_GRAPH_CSR, reserved=0, row_ptr=_np_ptr(rp), col=_np_ptr(cl))
        c = cia_coupling_default()
        c.model = CIA_MODEL_FLOCK
        c.p = int(p)
        c.cs_K, c.cs_sigma, c.cs_beta, c.cs_L = float(K), float(sigma), float(beta), float(L)
        c.cs_basis, c.rank, c.train_iters = int(basis), int(rank), int(train_iters)
        o = cia_options_default()
        o.method, o.precision, o.stepper, o.flags = method, CIA_F32, stepper, flags
        o.judge_tol, o.dense_alpha, o.device = float(judge_tol), dense_alpha, device
        handle = cia_build(g, labels, c, None, o)
        return cls(handle, int(n), CIA_F32, CIA_MODEL_FLOCK, dim=6)

    def basis_set_params(self, params, lo, hi):
        cia_basis_set_params(self.handle, params, lo, hi)

    def basis_get_params(self, count):
        return cia_basis_get_params(self.handle, count)

    def basis_train(self, state, iters, seed=1, loss_trace=None, stream=None):
        cia_basis_train(self.handle, state, iters, seed, loss_trace, stream)

    def basis_loss_grad(self, a, b, t, grad, stream=None):
        return cia_basis_loss_grad(self.handle, a, b, t, grad, stream)

    def basis_features(self, x, out, stream=None):
        cia_basis_features(self.handle, x, out, stream)

    @property
    def dtype_np(self):
        return np.float64 if self.precision == CIA_F64 else np.float32

    def rhs(self, state, dstate, stream=None):
        _check_state(self, state, "state")
        _check_state(self, dstate, "dstate")
        cia_rhs(self.handle, state, dstate, stream)

    def integrate(self, state, dt, steps, r_trace=None, stream=None):
        _check_state(self, state, "state")
        cia_integrate(self.handle, state, dt, steps, r_trace, stream)

    def info(self) -> cia_plan_info:
        return cia_plan_get_info(self.handle)

    def timing(self, reset=False) -> cia_timing:
        return cia_plan_get_timing(self.handle, reset)

    def close(self):
        if self.handle:
            cia_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
