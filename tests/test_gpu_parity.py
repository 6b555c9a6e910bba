"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Each problem's GPU step count is replayed by the oracle on the same (cast)
inputs; z, s, lambda, nu (lambda and nu where LICQ makes them unique) and every
gradient (whole and per tensor) are compared element by element at the
tolerances stated in tests/parity.py.
"""
import numpy as np
import pytest

from paper_1703_00443_amd import synth

from parity import TOL_Z, compare_problem, z_err

pytestmark = pytest.mark.gpu


def _run(batch, dtype, sample=None, need_grad=True, opts_over=None):
    import torch
    from paper_1703_00443_amd import binding as qb
    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x.astype(dtype))).to(dev)
    n, m, p = batch.dims
    prob = qb.make_problem(T(batch.Q), T(batch.q), T(batch.A) if p else None,
                           T(batch.b) if p else None, T(batch.G) if m else None,
                           T(batch.h) if m else None)
    opts = qb.default_opts(tdt, **(opts_over or {}))
    fw = qb.forward(prob, opts)
    gr = qb.backward(prob, fw, T(batch.g), opts) if need_grad else None
    torch.cuda.synchronize()
    out = {k: getattr(fw, k).cpu().numpy() for k in ("z", "lam", "nu", "s", "status", "iters")}
    if gr is not None:
        for k in ("dQ", "dq", "dA", "db", "dG", "dh"):
            v = getattr(gr, k)
            out[k] = None if v is None else v.cpu().numpy()
    return out


def _check(batch, out, dtype, idx, need_grad=True, tag=""):
    """compare_problem for every problem in idx (the oracle runs on a thread pool)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    idx = list(idx)
    for i in idx:
        assert int(out["status"][i]) in (0, 1, 4), "problem %d status %d" % (i, out["status"][i])

    def one(i):
        got = {k: (out[k][i] if out.get(k) is not None else None)
               for k in ("z", "lam", "nu", "s", "iters", "dQ", "dq", "dA", "db", "dG", "dh")}
        return compare_problem(batch.problem(i), got, dtype, tag="%s[%d]" % (tag, i), grads=need_grad)

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1, len(idx)))) as ex:
        return list(ex.map(one, idx))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_cpu_check_workload(dtype):
    """8 problems, n=10, 20 inequalities, 5 equalities (every problem checked)."""
    b = synth.make_batch(**synth.CPU_CHECK)
    out = _run(b, dtype)
    assert np.all(out["status"] == 0)
    _check(b, out, dtype, range(8), tag="cpu_check_%s" % np.dtype(dtype).name)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_paper_scale_every_problem(dtype):
    """The paper-scale batch (128 problems, n=100, 100 inequalities, no
    equalities, the launch configuration bench.py times): every problem."""
    b = synth.make_batch(**synth.PAPER_SCALE)
    out = _run(b, dtype)
    assert np.all(out["status"] == 0), np.bincount(out["status"])
    _check(b, out, dtype, range(128), tag="paper_scale_%s" % np.dtype(dtype).name)


@pytest.mark.parametrize("dims", [(17, 33, 3), (1, 2, 0), (5, 0, 2), (6, 0, 0), (33, 7, 0),
                                  (64, 130, 9)])
def test_ragged_and_degenerate_shapes(dims):
    n, m, p = dims
    b = synth.make_batch(seed=4242, B=3, n=n, m=m, p=p)
    out = _run(b, np.float64)
    _check(b, out, np.float64, range(3))
    if m == 0:
        assert np.all(out["iters"] == 0)


def test_empty_batch():
    import torch
    from paper_1703_00443_amd import binding as qb
    dev = torch.device("cuda:0")
    Q = torch.eye(3, dtype=torch.float64, device=dev).expand(0, 3, 3)
    prob = qb.make_problem(Q, torch.zeros(0, 3, dtype=torch.float64, device=dev))
    prob.batch = 0
    fw = qb.forward(prob)
    assert fw.z.shape == (0, 3)


def test_shared_parameters_stride0():
    """Q, G, A shared across the batch (stride 0), q, h, b per problem: every
    output and gradient of every problem against the oracle."""
    import torch
    from paper_1703_00443_amd import binding as qb
    b = synth.make_batch(seed=77, B=5, n=12, m=18, p=2)
    dev = torch.device("cuda:0")
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    prob = qb.make_problem(T(b.Q[0]), T(b.q), T(b.A[0]), T(b.b), T(b.G[0]), T(b.h))
    fw = qb.forward(prob)
    gr = qb.backward(prob, fw, T(b.g))
    torch.cuda.synchronize()
    for i in range(5):
        P = {"Q": b.Q[0], "q": b.q[i], "A": b.A[0], "b": b.b[i], "G": b.G[0], "h": b.h[i],
             "g": b.g[i]}
        got = {k: getattr(fw, k)[i].cpu().numpy() for k in ("z", "lam", "nu", "s")}
        got["iters"] = int(fw.iters[i].item())
        got.update({k: getattr(gr, k)[i].cpu().numpy() for k in ("dQ", "dq", "dA", "db", "dG", "dh")})
        compare_problem(P, got, np.float64, tag="stride0[%d]" % i)


def test_status_codes():
    import torch
    from paper_1703_00443_amd import binding as qb
    dev = torch.device("cuda:0")
    b = synth.make_batch(seed=9, B=3, n=6, m=8, p=1)
    Q = b.Q.copy()
    q = b.q.copy()
    q[1, 0] = np.nan            # problem 1: non-finite input
    Q[2] = -np.eye(6)           # problem 2: negative definite -> factorization breakdown
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    prob = qb.make_problem(T(Q), T(q), T(b.A), T(b.b), T(b.G), T(b.h))
    fw = qb.forward(prob)
    st = fw.status.cpu().numpy()
    assert st[0] == 0 and st[1] == 3 and st[2] == 2, st
    # no factor was stored for problems 1 and 2: their gradients are zero, and the
    # good problem's gradients match the same problem solved alone
    gr = qb.backward(prob, fw, T(b.g))
    one = qb.make_problem(T(Q[:1]), T(q[:1]), T(b.A[:1]), T(b.b[:1]), T(b.G[:1]), T(b.h[:1]))
    fw1 = qb.forward(one)
    gr1 = qb.backward(one, fw1, T(b.g[:1]))
    torch.cuda.synchronize()
    for k in ("dQ", "dq", "dA", "db", "dG", "dh"):
        g = getattr(gr, k).cpu().numpy()
        assert np.all(g[1:] == 0), k
        np.testing.assert_array_equal(g[0], getattr(gr1, k)[0].cpu().numpy(), err_msg=k)


def test_deterministic_rerun():
    b = synth.make_batch(**dict(synth.CPU_CHECK, B=4))
    o1 = _run(b, np.float64)
    o2 = _run(b, np.float64)
    for k in ("z", "lam", "nu", "dQ", "dG"):
        np.testing.assert_array_equal(o1[k], o2[k])


def test_generic_variant_matches_lds_variant_bitwise():
    """The factor-in-global-memory variant runs the same arithmetic in the same
    order as the LDS-resident one."""
    from paper_1703_00443_amd import binding as qb
    b = synth.make_batch(**dict(synth.CPU_CHECK, B=3))
    o1 = _run(b, np.float64, opts_over={"variant": qb.VARIANT_LDS})
    o2 = _run(b, np.float64, opts_over={"variant": qb.VARIANT_GENERIC})
    for k in ("z", "lam", "nu", "iters", "dQ", "dG", "dA"):
        np.testing.assert_array_equal(o1[k], o2[k])


@pytest.mark.parametrize("variant", ["auto", "generic"])
@pytest.mark.parametrize("dims", [(1, 3, 0), (15, 20, 0), (16, 16, 0), (17, 40, 0), (100, 100, 0),
                                  (128, 96, 0), (129, 64, 0), (129, 160, 0)])
def test_variants_across_tile_edges(variant, dims):
    """Sizes around the 16-wide tiles and the 128-variable limit of the tiled
    policy, with the per-problem plan (auto) and with the generic policy.

    FP32 gradients are compared at every shape: with fewer inequality rows than
    variables H = Qs + G^T D G keeps the small eigenvalues of Qs (down to 1e-3
    with this generator), which the FP32 backward's FP64 projected CG resolves
    (a working-precision refinement stopped near cond(K) eps32 there)."""
    from paper_1703_00443_amd import binding as qb
    n, m, p = dims
    b = synth.make_batch(seed=31337, B=2, n=n, m=m, p=p, row_normalize=True)
    over = {"variant": qb.VARIANT_GENERIC} if variant == "generic" else None
    for dtype in (np.float64, np.float32):
        out = _run(b, dtype, opts_over=over)
        _check(b, out, dtype, range(2), need_grad=True)


@pytest.mark.parametrize("dims", [(2, 3, 1), (10, 20, 5), (17, 33, 3), (64, 128, 16), (100, 50, 25),
                                  (128, 128, 32), (40, 0, 8)])
def test_tiled_policy_with_equalities(dims):
    """Equality rows on the tiled policy: Schur complement Wt = A U and
    S = Wt Wt^T as MFMA tiles, S factored in LDS (both precisions)."""
    from paper_1703_00443_amd import binding as qb
    n, m, p = dims
    b = synth.make_batch(seed=2024, B=2, n=n, m=m, p=p)
    for dtype in (np.float64, np.float32):
        out = _run(b, dtype, opts_over={"variant": qb.VARIANT_TILED})
        _check(b, out, dtype, range(2))


@pytest.mark.parametrize("dims,B", [((129, 64, 0), 2), ((144, 200, 10), 2), ((200, 200, 50), 2),
                                    ((255, 300, 7), 1), ((256, 512, 64), 1)])
def test_big_tiles_fp32(dims, B):
    """FP32 problems with 128 < nz <= 256 on the 16x16-tile-grid policy (G staged
    through LDS in chunks), ragged tails and the largest size."""
    from paper_1703_00443_amd import binding as qb
    n, m, p = dims
    b = synth.make_batch(seed=4096 + n, B=B, n=n, m=m, p=p, row_normalize=True)
    out = _run(b, np.float32, opts_over={"variant": qb.VARIANT_TILED})
    _check(b, out, np.float32, range(B))


@pytest.mark.parametrize("dims,dtypes", [
    ((1, 3, 0), "both"), ((16, 16, 0), "both"), ((17, 40, 3), "both"), ((100, 100, 0), "both"),
    ((130, 260, 10), "both"), ((200, 200, 50), "both"), ((300, 300, 20), "f32"),
    ((512, 600, 64), "f32"), ((200, 200, 150), "both"), ((256, 256, 200), "f32"),
    ((500, 500, 0), "both")])
def test_stream_policy(dims, dtypes):
    """The streamed-tile policy (factor in the state buffer, 16x16 MFMA tiles
    streamed through registers, G staged through LDS): tile edges, equality
    rows, sizes beyond the register-resident policies, Schur blocks too large
    for LDS (factored in the state: FP64 at neq=150, FP32 at neq=200), and the
    largest size of the paper's layer-timing experiment (nz = nineq = 500) in
    both precisions.  The library's plan query confirms the policy that ran."""
    import torch
    from paper_1703_00443_amd import binding as qb
    n, m, p = dims
    B = 1 if n >= 300 else 2
    b = synth.make_batch(seed=8080 + n, B=B, n=n, m=m, p=p, row_normalize=True)
    for dtype in ((np.float64, np.float32) if dtypes == "both" else (np.float32,)):
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        assert qb.plan(tdt, n, m, p, qb.VARIANT_STREAM)[0] == qb.VARIANT_STREAM, (dims, dtype)
        out = _run(b, dtype, opts_over={"variant": qb.VARIANT_STREAM})
        _check(b, out, dtype, range(B), need_grad=True)


def test_automatic_plan_by_size():
    """The automatic plan: register tiles up to nz = 128 (FP32: 256), streamed
    tiles beyond, in both precisions up to nz = nineq = 500."""
    import torch
    from paper_1703_00443_amd import binding as qb
    for tdt in (torch.float64, torch.float32):
        assert qb.plan(tdt, 100, 100, 0)[0] == qb.VARIANT_TILED
        assert qb.plan(tdt, 500, 500, 0)[0] == qb.VARIANT_STREAM
        assert qb.plan(tdt, 300, 300, 20)[0] == qb.VARIANT_STREAM
    assert qb.plan(torch.float32, 250, 400, 10)[0] == qb.VARIANT_TILED
    assert qb.plan(torch.float64, 250, 400, 10)[0] == qb.VARIANT_STREAM


@pytest.mark.parametrize("n", [10, 60, 100, 200])
def test_unit_row_flag_box_qp(n):
    """QP_FLAG_G_UNIT_ROWS on box QPs (G = [I; -I]): the register-tile policy forms
    G^T D G as a diagonal and applies G by gathers.  Against the oracle replay in
    both precisions (nz = 200 runs only in FP32, the other sizes where the
    register tiles take them), and close to the dense path's result."""
    import torch
    from paper_1703_00443_amd import binding as qb
    b = synth.box_batch(seed=2024 + n, B=3, n=n)
    for dtype in ((np.float32,) if n > 128 else (np.float64, np.float32)):
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        assert qb.plan(tdt, n, 2 * n, 0)[0] == qb.VARIANT_TILED
        fast = _run(b, dtype, opts_over={"flags": qb.FLAG_G_UNIT_ROWS})
        dense = _run(b, dtype)
        _check(b, fast, dtype, range(3))
        for i in range(3):
            if fast["iters"][i] == dense["iters"][i]:
                assert z_err(fast["z"][i], dense["z"][i]) <= TOL_Z[dtype]


@pytest.mark.parametrize("n", [300, 500])
def test_unit_row_flag_streamed_policy(n):
    """QP_FLAG_G_UNIT_ROWS on box QPs above the register-tile limits, where the
    streamed-tile policy runs: G^T D G as a diagonal, products with G as
    gathers.  z and lambda close to the dense path's result (where the step
    counts agree; FP64 and FP32 at nz = 300, FP32 at nz = 500), and at nz = 300
    every output and gradient of one problem against the oracle replay."""
    import torch
    from paper_1703_00443_amd import binding as qb
    b = synth.box_batch(seed=3030 + n, B=2, n=n)
    # FP64 at nz = 500 with 1000 rows: the driver's vectors alone leave no room
    # for the streamed layout, so the generic policy runs (no unit-row path)
    for dtype in ((np.float64, np.float32) if n <= 300 else (np.float32,)):
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        assert qb.plan(tdt, n, 2 * n, 0)[0] == qb.VARIANT_STREAM
        fast = _run(b, dtype, opts_over={"flags": qb.FLAG_G_UNIT_ROWS})
        dense = _run(b, dtype)
        assert np.all(np.isin(fast["status"], (0, 1, 4))), fast["status"]
        for i in range(2):
            if fast["iters"][i] == dense["iters"][i]:
                assert z_err(fast["z"][i], dense["z"][i]) <= TOL_Z[dtype]
                assert z_err(fast["lam"][i], dense["lam"][i]) <= TOL_Z[dtype] * 10
        if n == 300:
            _check(b, fast, dtype, range(1), tag="box_stream%d" % n)


def test_unit_row_flag_in_uneven_batch():
    """Box QPs of sizes from 20 to 300 in one uneven launch with the flag set
    (register-tile and streamed policies, the unit-row instantiation of the
    persistent kernel), next to a dense-G problem: each result bitwise equal to
    the same problem solved alone with the flag, z of every box problem within
    tolerance of the dense path's, and z of the smaller ones against the oracle."""
    import torch
    from paper_1703_00443_amd import binding as qb
    from paper_1703_00443_amd.varlen import VarlenBatch
    from parity import oracle_replay
    sizes = [20, 64, 150, 300, 90]
    probs = [synth.box_batch(seed=5050 + n, B=1, n=n).problem(0) for n in sizes]
    probs.append(synth.make_batch(seed=5051, B=1, n=40, m=60, p=3).problem(0))
    for dtype in (np.float32, np.float64):
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        ps = [{k: (None if v is None else np.asarray(v, dtype)) for k, v in P.items()} for P in probs]
        flag = qb.default_opts(tdt, flags=qb.FLAG_G_UNIT_ROWS)
        vb = VarlenBatch(ps, dtype=tdt)
        vb.forward(flag)
        dense = VarlenBatch(ps, dtype=tdt)
        dense.forward()
        torch.cuda.synchronize()
        for i, P in enumerate(ps):
            one = VarlenBatch([P], dtype=tdt)
            one.forward(flag)
            torch.cuda.synchronize()
            r, a, d = vb.result(i), one.result(0), dense.result(i)
            np.testing.assert_array_equal(r["z"], a["z"])
            assert int(r["status"]) in (0, 1, 4)
            if r["iters"] == d["iters"]:
                assert z_err(r["z"], d["z"]) <= TOL_Z[dtype]
            if P["Q"].shape[0] <= 90:
                ref = oracle_replay(probs[i], int(r["iters"]), dtype)
                assert z_err(r["z"], ref["z"]) <= TOL_Z[dtype], (dtype, i)


def test_unit_row_flag_falls_back_on_dense_g():
    """With the flag set but a G whose rows are not signed unit vectors, the
    kernel takes the dense path: bitwise the unflagged result."""
    from paper_1703_00443_amd import binding as qb
    b = synth.make_batch(seed=77, B=3, n=40, m=80, p=4, row_normalize=True)
    for dtype in (np.float64, np.float32):
        a = _run(b, dtype, opts_over={"flags": qb.FLAG_G_UNIT_ROWS})
        d = _run(b, dtype)
        for k in ("z", "lam", "nu", "s", "iters", "dQ", "dG"):
            np.testing.assert_array_equal(a[k], d[k], err_msg=k)


@pytest.mark.parametrize("n", [12, 90, 180])
def test_unit_row_flag_with_equality_rows(n):
    """The unit-row path with equality rows (Schur complement on A): QPs over the
    probability simplex, z >= 0 written as G = -I, h = 0, and 1^T z = 1 (the
    simplex layer of the paper's representational examples), against the oracle
    replay; nz = 180 runs in FP32 only (the 16x16 register-tile grid)."""
    import torch
    from paper_1703_00443_amd import binding as qb
    base = synth.make_batch(seed=4040 + n, B=3, n=n, m=0, p=0)
    G = np.broadcast_to(-np.eye(n), (3, n, n)).copy()
    b = synth.QPBatch(base.Q, 2.0 * base.q, np.ones((3, 1, n)), np.ones((3, 1)), G, np.zeros((3, n)),
                      base.g)
    for dtype in ((np.float32,) if n > 128 else (np.float64, np.float32)):
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        assert qb.plan(tdt, n, n, 1)[0] == qb.VARIANT_TILED
        out = _run(b, dtype, opts_over={"flags": qb.FLAG_G_UNIT_ROWS})
        _check(b, out, dtype, range(3))
        assert np.allclose(out["z"].sum(axis=1), 1.0, atol=1e-5 if dtype == np.float64 else 1e-3)


@pytest.mark.parametrize("tol", [1e-10, 1e-11])
def test_fp64_tight_tolerance(tol):
    """FP64 at a tolerance below the default 1e-8 (the tight-tolerance mode):
    the paper-scale batch reaches it (OPTIMAL, or STALLED where H loses
    definiteness first), every fourth problem matches the oracle replay, and
    the returned KKT error max(mu, residuals) of the OPTIMAL ones is within 10
    tol.  Gradients are compared at 1e-10; at 1e-11 mu reaches 1e-12 and
    cond(H) eps approaches 1 at the returned iterate, where the reduced
    backward cannot converge (measured: one problem off by 0.9), so only the
    forward is compared there."""
    import oracle
    b = synth.make_batch(**synth.PAPER_SCALE)
    out = _run(b, np.float64, opts_over={"tol": tol})
    st = out["status"]
    assert np.all((st == 0) | (st == 4)), np.bincount(st)
    assert np.mean(st == 0) >= 0.9, np.bincount(st)
    _check(b, out, np.float64, range(0, 128, 4), need_grad=tol >= 1e-10, tag="tight_tol_%g" % tol)
    for i in range(0, 128, 16):
        if st[i] != 0:
            continue
        P = b.problem(i)
        z, lam, s = out["z"][i], out["lam"][i], out["s"][i]
        rx = P["Q"] @ z + P["q"] + P["G"].T @ lam
        rs = P["G"] @ z + s - P["h"]
        err = max(float(s @ lam) / len(s), np.abs(rx).max(), np.abs(rs).max())
        assert err <= 10 * tol, (i, err)


# G streamed through LDS: the residual's G z and G^T lam come from the chunks of
# rows that the formation of H stages.  Row counts that end in a partial chunk,
# and one that is not a multiple of 4, with and without equality rows, in the
# register-tile policy (both tile grids) and the streamed-tile policy.
STREAMED_G = [(np.float64, 100, 301, 5, 3), (np.float32, 200, 403, 0, 3), (np.float32, 120, 290, 7, 3),
              (np.float64, 150, 157, 6, 4), (np.float32, 300, 45, 0, 4)]


@pytest.mark.parametrize("dtype,n,m,p,variant", STREAMED_G)
def test_residual_products_from_streamed_g(dtype, n, m, p, variant):
    import torch
    from paper_1703_00443_amd import binding as qb
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    pol, lds = qb.plan(tdt, n, m, p, variant)
    assert pol == variant, (pol, variant)
    if variant == qb.VARIANT_TILED:  # the streamed policy always stages G in chunks
        esz = np.dtype(dtype).itemsize
        assert lds < m * (16 * ((n + 15) // 16) + 1) * esz, "G would be LDS-resident at %s" % ((n, m, p),)
    b = synth.make_batch(seed=6100 + n + m + p, B=4, n=n, m=m, p=p)
    out = _run(b, dtype, opts_over={"variant": variant})
    _check(b, out, dtype, range(4), tag="streamed_g_%s%s" % (np.dtype(dtype).name, (n, m, p)))


@pytest.mark.parametrize("dtype,n,m,variant", [(np.float64, 100, 301, 3), (np.float32, 200, 403, 3),
                                               (np.float64, 150, 157, 4)])
def test_status_codes_with_streamed_g(dtype, n, m, variant):
    """Where G is streamed, each Newton step factors before its residual is
    tested: a non-finite input still ends NONFINITE, a negative definite Q
    BREAKDOWN, and the good problem of the batch is bitwise the same problem
    solved alone, with zero gradients for the other two."""
    import torch
    from paper_1703_00443_amd import binding as qb
    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    b = synth.make_batch(seed=77 + n, B=3, n=n, m=m, p=0)
    Q, q = b.Q.copy(), b.q.copy()
    q[1, 0] = np.nan             # problem 1: non-finite input
    Q[2] = -1e4 * np.eye(n)      # problem 2: Q + G^T D G negative definite -> breakdown
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x.astype(dtype))).to(dev)
    opts = qb.default_opts(tdt, variant=variant)
    prob = qb.make_problem(T(Q), T(q), None, None, T(b.G), T(b.h))
    fw = qb.forward(prob, opts)
    gr = qb.backward(prob, fw, T(b.g), opts)
    one = qb.make_problem(T(Q[:1]), T(q[:1]), None, None, T(b.G[:1]), T(b.h[:1]))
    fw1 = qb.forward(one, opts)
    gr1 = qb.backward(one, fw1, T(b.g[:1]), opts)
    torch.cuda.synchronize()
    st = fw.status.cpu().numpy()
    assert st[0] in (0, 4) and st[1] == 3 and st[2] == 2, st
    np.testing.assert_array_equal(fw.z[0].cpu().numpy(), fw1.z[0].cpu().numpy())
    for k in ("dQ", "dq", "dG", "dh"):
        g = getattr(gr, k).cpu().numpy()
        assert np.all(g[1:] == 0), k
        np.testing.assert_array_equal(g[0], getattr(gr1, k)[0].cpu().numpy(), err_msg=k)
