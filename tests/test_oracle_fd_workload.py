"""Central finite differences (step 1e-6, FP64) of the oracle forward at
tolerance 1e-12 on a random 1% of the entries of Q, q, A, b, G, h of one
problem of the differentiation workload (nz=200, nineq=200, neq=50), against
the oracle backward (eq. eq-d-def + eq. grads) at the same solution."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1703_00443_amd import synth


@pytest.mark.slow
def test_oracle_backward_vs_central_differences_differentiation_workload():
    b = synth.make_batch(**dict(synth.DIFF_SCALE, B=1))
    P = b.problem(0)
    keys = ("Q", "q", "A", "b", "G", "h")
    solve = lambda d: oracle.solve(d["Q"], d["q"], d["A"], d["b"], d["G"], d["h"], tol=1e-12,
                                   max_iter=100)
    r = solve(P)
    assert r["status"] == oracle.OPTIMAL
    gr = oracle.backward(P["Q"], P["A"], P["G"], P["h"], r["z"], r["lam"], r["nu"], P["g"])
    rng = np.random.default_rng(2024)
    picks = []
    for key in keys:
        x = P[key]
        k = max(1, int(round(0.01 * x.size)))
        for flat in rng.choice(x.size, k, replace=False):
            picks.append((key, np.unravel_index(flat, x.shape)))
    eps = 1e-6

    def fd(pick):
        key, idx = pick
        out = []
        for sgn in (+1, -1):
            d = dict(P)
            d[key] = P[key].copy()
            d[key][idx] += sgn * eps
            rr = solve(d)
            assert rr["status"] == oracle.OPTIMAL
            out.append(rr["z"])
        return P["g"] @ (out[0] - out[1]) / (2 * eps)

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        fdv = np.array(list(ex.map(fd, picks)))
    an = np.array([gr["d" + key][idx] for key, idx in picks])
    scale = max(np.abs(gr["d" + k]).max() for k in keys)
    assert len(picks) >= 900
    # near-degenerate constraints at this size (lambda_i and s_i both small at the
    # solution) make a few entries sensitive: bound the worst entry at 5e-4 and the
    # median at 1e-5 of the gradient scale (a dropped term or a sign error is O(1))
    err = np.abs(an - fdv) / scale
    assert err.max() <= 5e-4, err.max()
    assert np.median(err) <= 1e-5, np.median(err)
