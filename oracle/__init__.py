"""FP64 CPU oracle for OptNet's batched QP layer (Amos & Kolter 2017, Section 3).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``.  The product package never imports it.

The arithmetic lives in ``qp_oracle.c`` (plain C loops, FP64, unreduced LU
solves of the paper's own matrices); this module is a ctypes shim that builds
the shared object with gcc when it is missing and marshals numpy arrays.

Functions
---------
solve(Q, q, A, b, G, h, max_iter=20, tol=1e-8, replay=None)
    Primal-dual interior point forward (Section 3.1, eq. cvxgen:affine and
    eq. cvxgen:cc).  Returns a dict with z, s, lam, nu, iters, status.
backward(Q, A, G, h, z, lam, nu, g)
    Gradients of eq. grads through eq. eq-d-def.  Returns a dict with
    dQ, dq, dA, db, dG, dh and the adjoint vector d = (d_z, d_lam, d_nu).
solve_batch / backward_batch
    Loops of the above over a leading batch dimension, optionally on a
    thread pool (each QP is independent).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OPTIMAL, MAX_ITER, SINGULAR, NONFINITE = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile qp_oracle.c into liboracle.so (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            lib.oracle_qp_solve.restype = ctypes.c_int
            lib.oracle_qp_solve.argtypes = [ctypes.c_int] * 3 + [dp] * 6 + [
                ctypes.c_int, ctypes.c_double, ctypes.c_int] + [dp] * 4 + [ip]
            lib.oracle_qp_backward.restype = ctypes.c_int
            lib.oracle_qp_backward.argtypes = [ctypes.c_int] * 3 + [dp] * 8 + [dp] * 7
            _lib = lib
    return _lib


def _arr(x, shape):
    if x is None:
        x = np.zeros(shape)
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(shape))
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def solve(Q, q, A, b, G, h, max_iter: int = 20, tol: float = 1e-8, replay=None):
    lib = _load()
    Q = np.asarray(Q, dtype=np.float64)
    n = Q.shape[0]
    m = 0 if G is None else np.asarray(G).reshape(-1, n).shape[0]
    p = 0 if A is None else np.asarray(A).reshape(-1, n).shape[0]
    Q = _arr(Q, (n, n)); q = _arr(q, (n,))
    A = _arr(A, (p, n)); b = _arr(b, (p,))
    G = _arr(G, (m, n)); h = _arr(h, (m,))
    z = np.zeros(n); s = np.zeros(m); lam = np.zeros(m); nu = np.zeros(p)
    it = ctypes.c_int(0)
    st = lib.oracle_qp_solve(n, m, p, _ptr(Q), _ptr(q), _ptr(A), _ptr(b), _ptr(G), _ptr(h),
                             int(max_iter), float(tol), -1 if replay is None else int(replay),
                             _ptr(z), _ptr(s), _ptr(lam), _ptr(nu), ctypes.byref(it))
    if st < 0:
        raise ValueError("oracle_qp_solve: call error %d" % st)
    return {"z": z, "s": s, "lam": lam, "nu": nu, "iters": it.value, "status": st}


def backward(Q, A, G, h, z, lam, nu, g):
    lib = _load()
    Q = np.asarray(Q, dtype=np.float64)
    n = Q.shape[0]
    m = 0 if G is None else np.asarray(G).reshape(-1, n).shape[0]
    p = 0 if A is None else np.asarray(A).reshape(-1, n).shape[0]
    Q = _arr(Q, (n, n)); A = _arr(A, (p, n)); G = _arr(G, (m, n)); h = _arr(h, (m,))
    z = _arr(z, (n,)); lam = _arr(lam, (m,)); nu = _arr(nu, (p,)); g = _arr(g, (n,))
    dQ = np.zeros((n, n)); dq = np.zeros(n); dA = np.zeros((p, n)); db = np.zeros(p)
    dG = np.zeros((m, n)); dh = np.zeros(m); d = np.zeros(n + m + p)
    st = lib.oracle_qp_backward(n, m, p, _ptr(Q), _ptr(A), _ptr(G), _ptr(h), _ptr(z), _ptr(lam),
                                _ptr(nu), _ptr(g), _ptr(dQ), _ptr(dq), _ptr(dA), _ptr(db),
                                _ptr(dG), _ptr(dh), _ptr(d))
    if st < 0:
        raise ValueError("oracle_qp_backward: call error %d" % st)
    return {"dQ": dQ, "dq": dq, "dA": dA, "db": db, "dG": dG, "dh": dh,
            "d_z": d[:n], "d_lam": d[n:n + m], "d_nu": d[n + m:], "status": st}


def _take(x, i):
    if x is None:
        return None
    x = np.asarray(x)
    return x[i]


def solve_batch(Q, q, A, b, G, h, max_iter=20, tol=1e-8, replay=None, threads: int = 1):
    """Solve B independent QPs (leading batch axis on every array).  `replay`
    may be an int array of per-problem step counts."""
    B = np.asarray(q).shape[0]

    def one(i):
        r = None if replay is None else int(np.asarray(replay).reshape(-1)[i])
        return solve(_take(Q, i), _take(q, i), _take(A, i), _take(b, i), _take(G, i),
                     _take(h, i), max_iter=max_iter, tol=tol, replay=r)

    if threads > 1:
        with ThreadPoolExecutor(threads) as ex:
            outs = list(ex.map(one, range(B)))
    else:
        outs = [one(i) for i in range(B)]
    return {k: np.stack([o[k] for o in outs]) if k not in ("iters", "status")
            else np.array([o[k] for o in outs]) for k in outs[0]}


def backward_batch(Q, A, G, h, z, lam, nu, g, threads: int = 1):
    B = np.asarray(z).shape[0]

    def one(i):
        return backward(_take(Q, i), _take(A, i), _take(G, i), _take(h, i), _take(z, i),
                        _take(lam, i), _take(nu, i), _take(g, i))

    if threads > 1:
        with ThreadPoolExecutor(threads) as ex:
            outs = list(ex.map(one, range(B)))
    else:
        outs = [one(i) for i in range(B)]
    return {k: np.stack([o[k] for o in outs]) if k != "status"
            else np.array([o[k] for o in outs]) for k in outs[0]}
