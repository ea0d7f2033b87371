"""ctypes binding of libdicod.so (include/dicod.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
and torch device tensors into pointers and C structures and raises
``DicodError`` on a negative return code.  The library is loaded after torch,
so both share torch's HIP runtime (same SONAME); importing fails loudly when
the library has not been built.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdicod.so")

DICOD_OK = 0
DICOD_PENDING = 1
DICOD_EINVAL = -1
DICOD_ENOMEM = -2
DICOD_EDEVICE = -3
DICOD_ENOTCONV = -4
DICOD_ENOREQ = -5
DICOD_ENOTSUP = -6

DICOD_PREC_FP64 = 0
DICOD_PREC_FP32 = 1
DICOD_PREC_MIXED = 2
DICOD_SCHED_EVENODD = 0
DICOD_SCHED_DICOD = 1
DICOD_SCHED_ASYNC = 2

_CODES = {v: k for k, v in dict(globals()).items() if k.startswith("DICOD_E")}


class DicodError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{_CODES.get(code, code)}: {message}")
        self.code = code


class dicod_config(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("schedule", ctypes.c_int),
        ("update_cap", ctypes.c_int),
        ("max_phases", ctypes.c_int64),
        ("max_refresh", ctypes.c_int),
        ("phases_per_poll", ctypes.c_int),
        ("inner_eps_factor", ctypes.c_double),
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("max_inflight", ctypes.c_int),
        ("timing", ctypes.c_int),
        ("trace_capacity", ctypes.c_int64),
        ("state_in_lds", ctypes.c_int),
        ("fp64_polish_after", ctypes.c_int),
        ("colors", ctypes.c_int),
        ("verify_from_scratch", ctypes.c_int),
        ("reg_state", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("screen", ctypes.c_int),
    ]


class dicod_stats(ctypes.Structure):
    _fields_ = [
        ("n_updates", ctypes.c_int64),
        ("n_phases", ctypes.c_int64),
        ("n_phase_launches", ctypes.c_int64),
        ("n_segment_runs", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("n_seg", ctypes.c_int),
        ("seg_len", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("n_refresh", ctypes.c_int),
        ("lambda_", ctypes.c_double),
        ("lambda_max", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("objective", ctypes.c_double),
        ("max_dz", ctypes.c_double),
        ("kkt_on", ctypes.c_double),
        ("kkt_off", ctypes.c_double),
        ("max_abs_z", ctypes.c_double),
        ("t_init_ms", ctypes.c_double),
        ("t_cd_ms", ctypes.c_double),
        ("t_verify_ms", ctypes.c_double),
        ("t_total_ms", ctypes.c_double),
        ("t_lgcd_kernel_ms", ctypes.c_double),
        ("round_updates", ctypes.c_int64 * 4),
        ("round_phases", ctypes.c_int64 * 4),
        ("round_ms", ctypes.c_double * 4),
        ("round_kernel_ms", ctypes.c_double * 4),
        ("round_launches", ctypes.c_int64 * 4),
        ("round_state", ctypes.c_int * 4),
        ("state_in_hbm", ctypes.c_int),
        ("polished_fp64", ctypes.c_int),
        ("t_queue_ms", ctypes.c_double),
        ("t_latency_ms", ctypes.c_double),
        ("round_max_dz", ctypes.c_double * 4),
        ("colors", ctypes.c_int),
        ("update_cap", ctypes.c_int),
        ("tuned", ctypes.c_int),
        ("pad_", ctypes.c_int),
        ("duality_gap", ctypes.c_double),
        ("n_screened", ctypes.c_int64),
    ]

    def to_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, ctypes.Array) else v
        d["lambda"] = d.pop("lambda_")
        return d


class dicod_tune_entry(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int),
        ("P", ctypes.c_int),
        ("W", ctypes.c_int),
        ("bucket", ctypes.c_int),
        ("colors", ctypes.c_int),
        ("seg_len", ctypes.c_int),
        ("update_cap", ctypes.c_int),
        ("team_threads", ctypes.c_int),
        ("trials", ctypes.c_int),
        ("pad_", ctypes.c_int),
        ("ms", ctypes.c_double),
        ("ms_prior", ctypes.c_double),
    ]

    def to_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d.pop("pad_")
        return d

    @classmethod
    def from_dict(cls, d):
        e = cls()
        for name, _ in cls._fields_:
            if name in d:
                setattr(e, name, d[name])
        return e


TRACE_DTYPE = np.dtype([("phase", np.int32), ("seg", np.int32), ("k0", np.int32),
                        ("n_local", np.int32), ("t0", np.int64), ("delta", np.float64)])

_lib = None
_vp = ctypes.c_void_p


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
            "g.build()'` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    i64, ci, cd = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    pc = ctypes.POINTER(dicod_config)
    ps = ctypes.POINTER(dicod_stats)
    L.dicod_config_init.argtypes = [pc]
    L.dicod_init.argtypes = [ctypes.POINTER(_vp), pc]
    L.dicod_finalize.argtypes = [_vp]
    L.dicod_finalize.restype = None
    L.dicod_last_error.argtypes = [_vp]
    L.dicod_last_error.restype = ctypes.c_char_p
    L.dicod_set_dictionary.argtypes = [_vp, _vp, ci, ci, ci]
    L.dicod_solve.argtypes = [_vp, _vp, ci, i64, _vp, ci, ci, cd, cd, ci, _vp, ps]
    L.dicod_solve_device.argtypes = [_vp, _vp, i64, cd, cd, ci, _vp, ps, _vp]
    L.dicod_solve_device_noalloc.argtypes = [_vp, _vp, i64, cd, cd, ci, _vp, ps, _vp]
    L.dicod_solve_batch_device.argtypes = [_vp, ci, _vp, _vp, _vp, _vp, cd, _vp, _vp,
                                           _vp, _vp, _vp]
    L.dicod_correlate.argtypes = [_vp, _vp, i64, ci, _vp]
    L.dicod_get_s_table.argtypes = [_vp, _vp, _vp]
    L.dicod_get_trace.argtypes = [_vp, _vp, i64, ctypes.POINTER(i64)]
    L.dicod_submit.argtypes = [_vp, _vp, i64, cd, cd, ci, ctypes.POINTER(ctypes.c_uint64)]
    L.dicod_poll.argtypes = [_vp, ctypes.c_uint64, _vp, ps]
    pe = ctypes.POINTER(dicod_tune_entry)
    L.dicod_autotune_device.argtypes = [_vp, ci, _vp, _vp, _vp, _vp, cd, _vp, _vp, ci, pe]
    L.dicod_get_tuning.argtypes = [_vp, pe, ci, ctypes.POINTER(ci)]
    L.dicod_set_tuning.argtypes = [_vp, pe]
    L.dicod_check_h1.argtypes = [_vp, ctypes.POINTER(cd), ctypes.POINTER(ci)]
    for name in ("dicod_config_init", "dicod_init", "dicod_set_dictionary", "dicod_solve",
                 "dicod_solve_device", "dicod_solve_device_noalloc", "dicod_solve_batch_device",
                 "dicod_correlate", "dicod_get_s_table", "dicod_get_trace", "dicod_submit",
                 "dicod_poll", "dicod_autotune_device", "dicod_get_tuning", "dicod_set_tuning",
                 "dicod_check_h1"):
        getattr(L, name).restype = ci
    _lib = L
    return L


def _check(ctx, rc, allow=(DICOD_OK,)):
    if rc in allow:
        return rc
    msg = lib().dicod_last_error(ctx)
    raise DicodError(rc, msg.decode() if msg else "")


def _np_ptr(a):
    return a.ctypes.data_as(_vp)


# ---- same-name wrappers of the C entry points --------------------------------

def dicod_config_init(**overrides):
    cfg = dicod_config()
    lib().dicod_config_init(ctypes.byref(cfg))
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise TypeError(f"unknown config field {k}")
        setattr(cfg, k, v)
    return cfg


def dicod_init(cfg=None):
    h = _vp()
    rc = lib().dicod_init(ctypes.byref(h), ctypes.byref(cfg) if cfg is not None else None)
    _check(None, rc)
    return h


def dicod_finalize(ctx):
    lib().dicod_finalize(ctx)


def dicod_last_error(ctx):
    m = lib().dicod_last_error(ctx)
    return m.decode() if m else ""


def dicod_set_dictionary(ctx, D):
    D = np.ascontiguousarray(D, dtype=np.float32)
    K, P, W = D.shape
    _check(ctx, lib().dicod_set_dictionary(ctx, _np_ptr(D), K, P, W))


def dicod_solve(ctx, X, D, lam, eps, n_seg=0, K=None, W=None):
    """Host arrays in, (Z float64 [K, L], stats dict) out.

    D None uses the resident dictionary, whose K and W must then be given."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    P, T = X.shape
    if D is not None:
        D = np.ascontiguousarray(D, dtype=np.float32)
        K, _, W = D.shape
        dptr = _np_ptr(D)
    else:
        if K is None or W is None:
            raise DicodError(DICOD_EINVAL, "D is None: pass K and W of the resident dictionary")
        dptr = None
    Z = np.zeros((K, max(T - W + 1, 1)), dtype=np.float64)   # T < W: the library says EINVAL
    st = dicod_stats()
    rc = lib().dicod_solve(ctx, _np_ptr(X), P, T, dptr, K, W, float(lam), float(eps),
                           int(n_seg), _np_ptr(Z), ctypes.byref(st))
    try:
        _check(ctx, rc)
    except DicodError as e:
        if rc == DICOD_ENOTCONV:     # Z and the statistics are written
            e.Z, e.stats = Z, st.to_dict()
        raise
    return Z, st.to_dict()


def dicod_solve_device(ctx, X_dev, lam, eps, n_seg=0, Z_dev=None, K=None, W=None,
                       stream=None, check=True):
    """torch tensors on the GPU: X_dev float32 [P, T]; returns (Z_dev, stats)."""
    assert X_dev.is_cuda and X_dev.dtype == torch.float32 and X_dev.is_contiguous()
    T = X_dev.shape[1]
    if Z_dev is None:
        Z_dev = torch.empty((K, T - W + 1), dtype=torch.float64, device=X_dev.device)
    assert Z_dev.is_cuda and Z_dev.dtype == torch.float64 and Z_dev.is_contiguous()
    st = dicod_stats()
    s = stream if stream is not None else torch.cuda.current_stream(X_dev.device).cuda_stream
    rc = lib().dicod_solve_device(ctx, _vp(X_dev.data_ptr()), T, float(lam), float(eps),
                                  int(n_seg), _vp(Z_dev.data_ptr()), ctypes.byref(st),
                                  _vp(s))
    if check:
        _check(ctx, rc)
    return Z_dev, st.to_dict(), rc


def dicod_solve_device_noalloc(ctx, X_dev, lam, eps, n_seg, Z_dev, stream=None, check=True):
    """As dicod_solve_device with the workspace in the library's static device
    scratch (no allocation); Z_dev must be given.  Returns (Z_dev, stats, rc)."""
    assert X_dev.is_cuda and X_dev.dtype == torch.float32 and X_dev.is_contiguous()
    assert Z_dev.is_cuda and Z_dev.dtype == torch.float64 and Z_dev.is_contiguous()
    st = dicod_stats()
    s = stream if stream is not None else torch.cuda.current_stream(X_dev.device).cuda_stream
    rc = lib().dicod_solve_device_noalloc(ctx, _vp(X_dev.data_ptr()), X_dev.shape[1],
                                          float(lam), float(eps), int(n_seg),
                                          _vp(Z_dev.data_ptr()), ctypes.byref(st), _vp(s))
    if check:
        _check(ctx, rc)
    return Z_dev, st.to_dict(), rc


def dicod_solve_batch_device(ctx, X_dev, T, x_off, lam, eps, n_seg, Z_dev, z_off,
                             stream=None):
    """Packed signals on the device; returns a list of stats dicts."""
    n = len(T)
    T = np.ascontiguousarray(T, dtype=np.int64)
    x_off = np.ascontiguousarray(x_off, dtype=np.int64)
    z_off = np.ascontiguousarray(z_off, dtype=np.int64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    nseg = None if n_seg is None else np.ascontiguousarray(n_seg, dtype=np.int32)
    st = (dicod_stats * n)()
    s = stream if stream is not None else torch.cuda.current_stream(X_dev.device).cuda_stream
    rc = lib().dicod_solve_batch_device(
        ctx, n, _vp(X_dev.data_ptr()), _np_ptr(T), _np_ptr(x_off), _np_ptr(lam),
        float(eps), _np_ptr(nseg) if nseg is not None else None, _vp(Z_dev.data_ptr()),
        _np_ptr(z_off), st, _vp(s))
    _check(ctx, rc)
    return [st[i].to_dict() for i in range(n)]


def dicod_autotune_device(ctx, X_dev, T, x_off, lam, eps, Z_dev, z_off, max_trials=16):
    """Tunes the schedule on packed device signals (layout as the batch solve);
    returns the chosen entry as a dict.  Runs on the context's stream, after
    the current torch stream has finished writing X_dev."""
    n = len(T)
    T = np.ascontiguousarray(T, dtype=np.int64)
    x_off = np.ascontiguousarray(x_off, dtype=np.int64)
    z_off = np.ascontiguousarray(z_off, dtype=np.int64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    torch.cuda.current_stream(X_dev.device).synchronize()
    e = dicod_tune_entry()
    rc = lib().dicod_autotune_device(ctx, n, _vp(X_dev.data_ptr()), _np_ptr(T), _np_ptr(x_off),
                                     _np_ptr(lam), float(eps), _vp(Z_dev.data_ptr()),
                                     _np_ptr(z_off), int(max_trials), ctypes.byref(e))
    _check(ctx, rc)
    return e.to_dict()


def dicod_get_tuning(ctx):
    n = ctypes.c_int(0)
    _check(ctx, lib().dicod_get_tuning(ctx, None, 0, ctypes.byref(n)))
    arr = (dicod_tune_entry * max(n.value, 1))()
    _check(ctx, lib().dicod_get_tuning(ctx, arr, n.value, ctypes.byref(n)))
    return [arr[i].to_dict() for i in range(n.value)]


def dicod_set_tuning(ctx, entry):
    """entry: dict of dicod_tune_entry fields, or None to empty the table."""
    e = None if entry is None else ctypes.byref(dicod_tune_entry.from_dict(entry))
    _check(ctx, lib().dicod_set_tuning(ctx, e))


def dicod_check_h1(ctx):
    """(ratio, holds): the H1 quantity of the resident dictionary."""
    r, h = ctypes.c_double(0.0), ctypes.c_int(0)
    _check(ctx, lib().dicod_check_h1(ctx, ctypes.byref(r), ctypes.byref(h)))
    return r.value, bool(h.value)


def dicod_correlate(ctx, X, K, W, precision=DICOD_PREC_FP64):
    X = np.ascontiguousarray(X, dtype=np.float32)
    P, T = X.shape
    out = np.zeros((K, T - W + 1), dtype=np.float64)
    _check(ctx, lib().dicod_correlate(ctx, _np_ptr(X), T, int(precision), _np_ptr(out)))
    return out


def dicod_get_s_table(ctx, K, W):
    S = np.zeros((K, K, 2 * W - 1), dtype=np.float64)
    n2 = np.zeros(K, dtype=np.float64)
    _check(ctx, lib().dicod_get_s_table(ctx, _np_ptr(S), _np_ptr(n2)))
    return S, n2


def dicod_get_trace(ctx, cap):
    out = np.zeros(cap, dtype=TRACE_DTYPE)
    n = ctypes.c_int64(0)
    _check(ctx, lib().dicod_get_trace(ctx, _np_ptr(out), cap, ctypes.byref(n)))
    return out[:min(n.value, cap)]


def dicod_submit(ctx, X, lam, eps, n_seg=0):
    X = np.ascontiguousarray(X, dtype=np.float32)
    rid = ctypes.c_uint64(0)
    _check(ctx, lib().dicod_submit(ctx, _np_ptr(X), X.shape[1], float(lam), float(eps),
                                   int(n_seg), ctypes.byref(rid)))
    return rid.value


def dicod_poll(ctx, req_id, K, L, out=None):
    """Returns (done, Z or None, stats or None).  out: optional float64 buffer of
    at least K * L elements that receives Z (the returned array is a view)."""
    if out is None:
        Z = np.empty((K, L), dtype=np.float64)
    else:
        Z = out.reshape(-1)[:K * L].reshape(K, L)
        assert Z.dtype == np.float64 and Z.flags.c_contiguous
    st = dicod_stats()
    rc = lib().dicod_poll(ctx, ctypes.c_uint64(req_id), _np_ptr(Z), ctypes.byref(st))
    _check(ctx, rc, allow=(DICOD_OK, DICOD_PENDING))
    if rc == DICOD_PENDING:
        return False, None, None
    return True, Z, st.to_dict()


class Context:
    """Owns a dicod context; keeps the resident dictionary's shape."""

    def __init__(self, **cfg):
        self.cfg = dicod_config_init(**cfg)
        self.h = dicod_init(self.cfg)
        self.K = self.P = self.W = None

    def close(self):
        if self.h:
            dicod_finalize(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_dictionary(self, D):
        dicod_set_dictionary(self.h, D)
        self.K, self.P, self.W = np.asarray(D).shape

    def solve(self, X, lam, eps, n_seg=0, D=None):
        if D is not None:
            self.K, self.P, self.W = np.asarray(D).shape
        return dicod_solve(self.h, X, D, lam, eps, n_seg, self.K, self.W)

    def solve_device(self, X_dev, lam, eps, n_seg=0, Z_dev=None, stream=None, check=True):
        return dicod_solve_device(self.h, X_dev, lam, eps, n_seg, Z_dev, self.K, self.W,
                                  stream, check)

    def solve_device_noalloc(self, X_dev, lam, eps, n_seg, Z_dev, stream=None, check=True):
        return dicod_solve_device_noalloc(self.h, X_dev, lam, eps, n_seg, Z_dev, stream, check)

    def solve_batch_device(self, X_dev, T, x_off, lam, eps, n_seg, Z_dev, z_off, stream=None):
        return dicod_solve_batch_device(self.h, X_dev, T, x_off, lam, eps, n_seg, Z_dev,
                                        z_off, stream)

    def autotune_device(self, X_dev, T, x_off, lam, eps, Z_dev, z_off, max_trials=16):
        return dicod_autotune_device(self.h, X_dev, T, x_off, lam, eps, Z_dev, z_off,
                                     max_trials)

    def tuning(self):
        return dicod_get_tuning(self.h)

    def set_tuning(self, entry):
        dicod_set_tuning(self.h, entry)

    def save_tuning(self, path):
        """Writes the tuning table to a JSON file (the cache of chosen schedules)."""
        import json
        with open(path, "w") as f:
            json.dump(self.tuning(), f, indent=1)

    def load_tuning(self, path):
        """Loads a tuning table written by save_tuning into this context."""
        import json
        with open(path) as f:
            for e in json.load(f):
                self.set_tuning(e)

    def check_h1(self):
        return dicod_check_h1(self.h)

    def correlate(self, X, precision=DICOD_PREC_FP64):
        return dicod_correlate(self.h, X, self.K, self.W, precision)

    def s_table(self):
        return dicod_get_s_table(self.h, self.K, self.W)

    def trace(self, cap=None):
        return dicod_get_trace(self.h, cap or int(self.cfg.trace_capacity))

    def submit(self, X, lam, eps, n_seg=0):
        return dicod_submit(self.h, X, lam, eps, n_seg)

    def poll(self, req_id, T, out=None):
        return dicod_poll(self.h, req_id, self.K, T - self.W + 1, out)
