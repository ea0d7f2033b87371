"""FP64 CPU oracle for locally greedy convolutional coordinate descent.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may use it; the GPU product path never does.

Thin ctypes wrapper over ``dicod_oracle.c`` (plain C, double precision).  Each
function names the passage of Moreau, Oudre & Vayatis (ICML 2018) it follows;
the C file lists the readings taken where the paper is ambiguous.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

SCHED_EVENODD = 0
SCHED_SEQUENCE = 1
SCHED_DICOD = 2


class OracleStats(ctypes.Structure):
    _fields_ = [
        ("n_updates", ctypes.c_int64),
        ("n_steps", ctypes.c_int64),
        ("n_phases", ctypes.c_int64),
        ("n_full_checks", ctypes.c_int64),
        ("dE_sum", ctypes.c_double),
        ("dE_min", ctypes.c_double),
        ("lowerbound_gap_min", ctypes.c_double),
        ("converged", ctypes.c_int),
        ("n_messages", ctypes.c_int64),
        ("n_interf", ctypes.c_int64),
        ("n_adjacent", ctypes.c_int64),
        ("interf_sum", ctypes.c_double),
    ]


TRACE_DTYPE = np.dtype([
    ("step", np.int64), ("phase", np.int32), ("seg", np.int32),
    ("k0", np.int32), ("n_local", np.int32), ("t0", np.int64),
    ("z_old", np.float64), ("z_new", np.float64), ("dE", np.float64),
])


class OracleTraceRec(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("phase", ctypes.c_int32),
        ("seg", ctypes.c_int32), ("k0", ctypes.c_int32),
        ("n_local", ctypes.c_int32), ("t0", ctypes.c_int64),
        ("z_old", ctypes.c_double), ("z_new", ctypes.c_double),
        ("dE", ctypes.c_double),
    ]


assert ctypes.sizeof(OracleTraceRec) == TRACE_DTYPE.itemsize

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # ORACLE_LIB: a separately built copy (e.g. with sanitizers) instead of
    # the library built here
    other = os.environ.get("ORACLE_LIB")
    if other:
        _lib = load_library(other)
        return _lib
    src = os.path.join(_HERE, "dicod_oracle.c")
    if (not os.path.exists(_LIB_PATH)
            or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src)):
        _build.build()
    _lib = load_library(_LIB_PATH)
    return _lib


def use_library(lib):
    """Route every wrapper to ``lib`` (a library from ``load_library``); returns
    the previous one.  Used by the tests that plant mistakes in a copy of the
    oracle to show that the pins catch them."""
    global _lib
    prev = _lib
    _lib = lib
    return prev


def load_library(path):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    lib.oracle_soft_threshold.restype = ctypes.c_double
    lib.oracle_soft_threshold.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_norms.argtypes = [dp, ci, ci, ci, dp]
    lib.oracle_s_table.argtypes = [dp, ci, ci, ci, dp]
    lib.oracle_gap_safe.argtypes = [dp, dp, dp, ci, ci, ci, i64, ctypes.c_double, dp, dp,
                                    ctypes.c_void_p]
    lib.oracle_gap_safe.restype = i64
    lib.oracle_h1_ratio.argtypes = [dp, ci, ci, ci]
    lib.oracle_h1_ratio.restype = ctypes.c_double
    lib.oracle_correlate.argtypes = [dp, ci, ci, ci, dp, i64, dp]
    lib.oracle_reconstruct.argtypes = [dp, dp, ci, ci, ci, i64, dp]
    lib.oracle_objective.restype = ctypes.c_double
    lib.oracle_objective.argtypes = [dp, dp, dp, ci, ci, ci, i64, ctypes.c_double]
    lib.oracle_beta.restype = ci
    lib.oracle_beta.argtypes = [dp, dp, dp, ci, ci, ci, i64, dp]
    lib.oracle_max_dz.restype = ctypes.c_double
    lib.oracle_max_dz.argtypes = [dp, dp, dp, ci, ci, ci, i64, ctypes.c_double,
                                  ctypes.POINTER(ci), ctypes.POINTER(i64)]
    lib.oracle_beta_at.restype = ci
    lib.oracle_beta_at.argtypes = [dp, dp, dp, ci, ci, ci, i64,
                                   ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int64), i64, dp]
    lib.oracle_lgcd.restype = ci
    lib.oracle_lgcd.argtypes = [
        dp, dp, ci, ci, ci, i64, ctypes.c_double, ctypes.c_double, ci, ci,
        ctypes.POINTER(ctypes.c_int32), i64, ci, i64, dp,
        ctypes.POINTER(OracleStats), ctypes.c_void_p, i64, ci]
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def soft_threshold(u, lam):
    """Sh(u, lambda) = sign(u) max(|u| - lambda, 0)  (Sec. 2.1)."""
    return _load().oracle_soft_threshold(float(u), float(lam))


def norms(D):
    """||D_k||_2^2 for D of shape (K, P, W)."""
    D = _f64(D)
    K, P, W = D.shape
    out = np.empty(K)
    _load().oracle_norms(_ptr(D), K, P, W, _ptr(out))
    return out


def s_table(D):
    """S[k, l, d + W - 1] = S_{k,l}[d] = sum_tau <D_k[tau], D_l[tau+d]>  (eq. (3))."""
    D = _f64(D)
    K, P, W = D.shape
    out = np.empty((K, K, 2 * W - 1))
    _load().oracle_s_table(_ptr(D), K, P, W, _ptr(out))
    return out


def gap_safe(X, D, Z, lam):
    """(gap, radius, screened bool [K, L]) of the Gap Safe sphere rule at Z:
    screened coordinates are zero in every solution of (2)."""
    X, D, Z = _f64(X), _f64(D), _f64(Z)
    K, P, W = D.shape
    g, r = ctypes.c_double(0.0), ctypes.c_double(0.0)
    out = np.zeros(Z.shape, dtype=np.uint8)
    n = _load().oracle_gap_safe(_ptr(X), _ptr(D), _ptr(Z), K, P, W, X.shape[1], float(lam),
                                ctypes.byref(g), ctypes.byref(r), out.ctypes.data)
    if n < 0:
        raise MemoryError("oracle_gap_safe: out of memory")
    return g.value, r.value, out.astype(bool)


def h1_ratio(D):
    """max over atoms k, l and shifts d != 0 of |S_{k,l}[d]| / (|D_k| |D_l|):
    hypothesis H1 of Theorem 1 (Sec. 3) holds when it is below 1."""
    D = _f64(D)
    K, P, W = D.shape
    return float(_load().oracle_h1_ratio(_ptr(D), K, P, W))


def correlate(D, Y):
    """out[k, t] = sum_{p,tau} D[k,p,tau] Y[p, t+tau]; beta at Z = 0 (Algorithm 1 init)."""
    D, Y = _f64(D), _f64(Y)
    K, P, W = D.shape
    T = Y.shape[1]
    out = np.empty((K, T - W + 1))
    _load().oracle_correlate(_ptr(D), K, P, W, _ptr(Y), T, _ptr(out))
    return out


def reconstruct(D, Z, T):
    """sum_k Z_k * D_k, shape (P, T)  (model eq. (1) without noise)."""
    D, Z = _f64(D), _f64(Z)
    K, P, W = D.shape
    out = np.empty((P, T))
    _load().oracle_reconstruct(_ptr(D), _ptr(Z), K, P, W, T, _ptr(out))
    return out


def objective(X, D, Z, lam):
    """E(Z) of eq. (2)."""
    X, D, Z = _f64(X), _f64(D), _f64(Z)
    K, P, W = D.shape
    return _load().oracle_objective(_ptr(X), _ptr(D), _ptr(Z), K, P, W,
                                    X.shape[1], float(lam))


def beta(X, D, Z):
    """beta from its definition in Sec. 2.1, recomputed from scratch."""
    X, D, Z = _f64(X), _f64(D), _f64(Z)
    K, P, W = D.shape
    out = np.empty_like(Z)
    rc = _load().oracle_beta(_ptr(X), _ptr(D), _ptr(Z), K, P, W, X.shape[1],
                             _ptr(out))
    if rc != 0:
        raise MemoryError("oracle_beta failed")
    return out


def beta_at(X, D, Z, k, t):
    """beta_k[t] at the coordinates (k[i], t[i]) from the definition in Sec. 2.1,
    one at a time (for signals too long for a full recompute)."""
    X, D, Z = _f64(X), _f64(D), _f64(Z)
    K, P, W = D.shape
    k = np.ascontiguousarray(k, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int64)
    out = np.empty(k.shape[0])
    rc = _load().oracle_beta_at(_ptr(X), _ptr(D), _ptr(Z), K, P, W, X.shape[1],
                                k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                k.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError("oracle_beta_at: bad coordinate or out of memory")
    return out


def max_dz(X, D, Z, lam):
    """(||Delta Z||_inf, k, t) with beta recomputed from scratch (Algorithm 3 stop test)."""
    X, D, Z = _f64(X), _f64(D), _f64(Z)
    K, P, W = D.shape
    k = ctypes.c_int(-1)
    t = ctypes.c_int64(-1)
    v = _load().oracle_max_dz(_ptr(X), _ptr(D), _ptr(Z), K, P, W, X.shape[1],
                              float(lam), ctypes.byref(k), ctypes.byref(t))
    return v, k.value, t.value


def lgcd(X, D, lam, eps, M, schedule=SCHED_EVENODD, seq=None, cap=0,
         max_steps=10**9, trace_cap=0, colors=2):
    """Locally greedy CD: Algorithm 3 with coloured phases (SCHED_EVENODD,
    2 colours = even/odd) or a given segment order (SCHED_SEQUENCE), or
    Algorithm 2 with the cores in lockstep and messages delivered one phase
    later (SCHED_DICOD; the stats count interfering concurrent updates).

    Returns (Z, stats dict, trace array or None).  Raises on bad arguments;
    stats['converged'] tells whether the stop test was met.
    """
    X, D = _f64(X), _f64(D)
    K, P, W = D.shape
    T = X.shape[1]
    L = T - W + 1
    Z = np.zeros((K, L))
    st = OracleStats()
    if seq is None:
        seq_arr = np.zeros(1, dtype=np.int32)
        seq_len = 0 if schedule == SCHED_SEQUENCE else 1
    else:
        seq_arr = np.ascontiguousarray(seq, dtype=np.int32)
        seq_len = seq_arr.size
    trace = np.zeros(max(trace_cap, 0), dtype=TRACE_DTYPE)
    rc = _load().oracle_lgcd(
        _ptr(X), _ptr(D), K, P, W, T, float(lam), float(eps), int(M),
        int(schedule), seq_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        int(seq_len), int(cap), int(max_steps), _ptr(Z), ctypes.byref(st),
        trace.ctypes.data if trace_cap > 0 else None, int(trace_cap), int(colors))
    if rc < 0:
        raise ValueError(f"oracle_lgcd rejected its arguments (rc={rc})")
    stats = {name: getattr(st, name) for name, _ in OracleStats._fields_}
    n_tr = min(int(stats["n_updates"]), trace_cap)
    return Z, stats, (trace[:n_tr].copy() if trace_cap > 0 else None)


def lambda_max(X, D):
    """max |D^T X| : the smallest lambda for which Z = 0 is optimal (eq. (2))."""
    return float(np.max(np.abs(correlate(D, X))))
