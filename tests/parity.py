"""Shared helpers for GPU-vs-oracle parity tests (no arithmetic of the method).

The oracle replays each problem's Newton step count reported by the GPU (same
algorithm, same number of steps, same cast inputs), so differences are rounding
only.  Every problem output is compared element by element:

  z:        |dz|_inf / (1 + |z|_inf)            <= TOL_Z: 1e-5 (FP64), 2e-3 (FP32)
  lam, nu:  the same measure                    <= TOL_Z, where the multipliers are
            unique (LICQ at the replayed iterate: the rows of G that are active there,
            with those of A, are linearly independent; Section 3, KKT conditions);
  s:        |ds|_inf / (1 + |s|_inf)            <= TOL_Z * (1 + |G|_inf), since
            s = h - G z + r_s moves by at most |G|_inf |dz|_inf under a change dz of z
            (|G|_inf the largest row 1-norm);
  gradient: |dg|_inf / |g|_inf                  <= TOL_G: 1e-4 (FP64), 5e-3 (FP32)
            over the whole gradient of one problem (dQ, dq, dA, db, dG, dh
            concatenated), and per tensor with the tensor's own norm in the
            denominator, floored at 10% of the whole gradient's: when nz - neq
            inequalities are active z is pinned by the active set and dQ, dq vanish,
            so a purely per-tensor ratio would divide by ~0.  With the floor every
            tensor's absolute error is held to between 1x and 10x less than the
            whole-gradient criterion allows.

Set QPMI_PARITY_LOG=<path> to append every measured margin as a JSON line.
"""
import json
import os

import numpy as np

import oracle

TOL_Z = {np.float64: 1e-5, np.float32: 2e-3}
TOL_G = {np.float64: 1e-4, np.float32: 5e-3}
GRAD_KEYS = ("dQ", "dq", "dA", "db", "dG", "dh")
PER_TENSOR_FLOOR = 1e-1


def z_err(z, zref):
    return np.abs(z - zref).max(initial=0.0) / (1.0 + np.abs(zref).max(initial=0.0))


def g_err(g, gref, scale=None):
    if scale is None:
        scale = np.abs(gref).max(initial=0.0)
    return np.abs(g - gref).max(initial=0.0) / max(scale, 1e-300)


def grad_scale(gref, keys=GRAD_KEYS):
    """|g|_inf of the concatenated gradient of one problem."""
    return max(np.abs(gref[k]).max(initial=0.0) for k in keys if gref.get(k) is not None)


def per_tensor_errors(got, gref, keys=GRAD_KEYS):
    """{key: |d|_inf / max(|ref|_inf, 10% of the whole gradient's |g|_inf)}."""
    sc = grad_scale(gref, keys)
    out = {}
    for k in keys:
        if got.get(k) is None or gref.get(k) is None or np.asarray(gref[k]).size == 0:
            continue
        den = max(np.abs(gref[k]).max(initial=0.0), PER_TENSOR_FLOOR * sc, 1e-300)
        out[k] = float(np.abs(np.asarray(got[k], np.float64) - gref[k]).max(initial=0.0) / den)
    return out


def _c(x, dtype):
    return None if x is None else np.asarray(x, dtype=dtype).astype(np.float64)


def oracle_replay(P, iters, dtype):
    """Oracle forward with the GPU's step count on the (cast) inputs of one problem."""
    c = lambda x: _c(x, dtype)
    return oracle.solve(c(P["Q"]), c(P["q"]), c(P.get("A")), c(P.get("b")), c(P.get("G")),
                        c(P.get("h")), replay=int(iters))


def oracle_grads(P, r, g, dtype):
    c = lambda x: _c(x, dtype)
    return oracle.backward(c(P["Q"]), c(P.get("A")), c(P.get("G")), c(P.get("h")), r["z"], r["lam"],
                           r["nu"], c(g))


def licq(P, r, dtype, rel=1e-6):
    """True when the inequality rows active at the replayed iterate (slack below
    `rel` of its row's scale), stacked on the equality rows, have full row rank."""
    G = _c(P.get("G"), dtype)
    A = _c(P.get("A"), dtype)
    rows = []
    if G is not None and G.size:
        scale = 1.0 + np.abs(G).sum(axis=1) * (1.0 + np.abs(r["z"]).max(initial=0.0))
        rows.append(G[r["s"] < rel * scale])
    if A is not None and A.size:
        rows.append(A)
    if not rows:
        return True
    M = np.concatenate(rows, axis=0)
    if M.shape[0] == 0:
        return True
    if M.shape[0] > M.shape[1]:
        return False
    return np.linalg.matrix_rank(M) == M.shape[0]


def s_tol(P, dtype):
    G = _c(P.get("G"), dtype)
    gi = np.abs(G).sum(axis=1).max(initial=0.0) if G is not None and G.size else 0.0
    return TOL_Z[dtype] * (1.0 + gi)


def log_margins(tag, rec):
    path = os.environ.get("QPMI_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(dict(tag=tag, **rec)) + "\n")


def compare_problem(P, got, dtype, tag="", grads=True, g=None, gref=None, ref=None):
    """Compare one GPU problem result `got` (z, lam, nu, s, iters[, dQ..dh]) with the
    oracle replay; assert every tolerance; return the measured errors."""
    ref = ref if ref is not None else oracle_replay(P, got["iters"], dtype)
    rec = {"iters": int(got["iters"])}
    rec["z"] = float(z_err(np.asarray(got["z"], np.float64), ref["z"]))
    assert rec["z"] <= TOL_Z[dtype], (tag, "z", rec)
    m = ref["s"].size
    p = ref["nu"].size
    if m:
        rec["s"] = float(z_err(np.asarray(got["s"], np.float64), ref["s"]))
        rec["s_tol"] = float(s_tol(P, dtype))
        assert rec["s"] <= rec["s_tol"], (tag, "s", rec)
    rec["licq"] = bool(licq(P, ref, dtype))
    if rec["licq"]:
        if m:
            rec["lam"] = float(z_err(np.asarray(got["lam"], np.float64), ref["lam"]))
            assert rec["lam"] <= TOL_Z[dtype], (tag, "lam", rec)
        if p:
            rec["nu"] = float(z_err(np.asarray(got["nu"], np.float64), ref["nu"]))
            assert rec["nu"] <= TOL_Z[dtype], (tag, "nu", rec)
    if grads:
        gref = gref if gref is not None else oracle_grads(P, ref, P["g"] if g is None else g, dtype)
        sc = grad_scale(gref)
        rec["grad"] = float(max(g_err(np.asarray(got[k], np.float64), gref[k], sc)
                                for k in GRAD_KEYS if got.get(k) is not None and gref.get(k) is not None))
        pt = per_tensor_errors(got, gref)
        rec.update({"pt_" + k: v for k, v in pt.items()})
        assert rec["grad"] <= TOL_G[dtype], (tag, "grad", rec)
        for k, v in pt.items():
            assert v <= TOL_G[dtype], (tag, "grad " + k, rec)
    log_margins(tag, rec)
    return rec
