"""Shared helpers for GPU-vs-oracle parity tests (no arithmetic of the method).

Tolerances (from the design targets):
  z:    |dz|_inf / (1 + |z|_inf) <= 1e-5 (FP64), 2e-3 (FP32)
  grad: |dg|_inf / |g|_inf <= 1e-4 (FP64), 5e-3 (FP32), where g is the whole gradient of one
        problem (dQ, dq, dA, db, dG, dh concatenated).  A per-tensor ratio would divide by ~0
        whenever z is pinned by nz - neq active constraints (then dQ, dq vanish).
The oracle replays each problem's Newton step count reported by the GPU
(same algorithm, same number of steps), so differences are rounding only.
"""
import numpy as np

import oracle

TOL_Z = {np.float64: 1e-5, np.float32: 2e-3}
TOL_G = {np.float64: 1e-4, np.float32: 5e-3}


def z_err(z, zref):
    return np.abs(z - zref).max(initial=0.0) / (1.0 + np.abs(zref).max(initial=0.0))


def g_err(g, gref, scale=None):
    if scale is None:
        scale = np.abs(gref).max(initial=0.0)
    return np.abs(g - gref).max(initial=0.0) / max(scale, 1e-300)


def grad_scale(gref, keys=("dQ", "dq", "dA", "db", "dG", "dh")):
    """|g|_inf of the concatenated gradient of one problem."""
    return max(np.abs(gref[k]).max(initial=0.0) for k in keys if gref.get(k) is not None)


def oracle_replay(P, iters, dtype):
    """Oracle forward with the GPU's step count on the (cast) inputs of one problem."""
    c = lambda x: None if x is None else np.asarray(x, dtype=dtype).astype(np.float64)
    return oracle.solve(c(P["Q"]), c(P["q"]), c(P.get("A")), c(P.get("b")), c(P.get("G")),
                        c(P.get("h")), replay=int(iters))


def oracle_grads(P, r, g, dtype):
    c = lambda x: None if x is None else np.asarray(x, dtype=dtype).astype(np.float64)
    return oracle.backward(c(P["Q"]), c(P.get("A")), c(P.get("G")), c(P.get("h")), r["z"], r["lam"],
                           r["nu"], c(g))
