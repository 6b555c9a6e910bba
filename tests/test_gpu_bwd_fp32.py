"""QP_FLAG_BWD_FP32: the FP32 backward in FP32 only (reduced solve with the
stored FP32 factor plus iterative refinement in FP32), against the oracle's
backward at the returned iterate (eq. grads-system solved in FP64 with the
GPU's own z, lambda, nu and s), and against the default FP32 backward (FP64
projected CG).  Its accuracy is bounded by cond(H) eps32 at the returned
iterate; the measured errors are logged and the bounds below hold on these
workloads."""
import numpy as np
import pytest

from paper_1703_00443_amd import synth

from parity import g_err, grad_scale, log_margins

pytestmark = pytest.mark.gpu


def _run(b, flags):
    import torch
    from paper_1703_00443_amd import binding as qb
    dev = torch.device("cuda:0")
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x.astype(np.float32))).to(dev)
    n, m, p = b.dims
    prob = qb.make_problem(T(b.Q), T(b.q), T(b.A) if p else None, T(b.b) if p else None,
                           T(b.G) if m else None, T(b.h) if m else None)
    o = qb.default_opts(torch.float32, flags=flags)
    fw = qb.forward(prob, o)
    gr = qb.backward(prob, fw, T(b.g), o)
    torch.cuda.synchronize()
    out = {k: getattr(fw, k).cpu().numpy() for k in ("z", "lam", "nu", "s", "status", "iters")}
    for k in ("dQ", "dq", "dA", "db", "dG", "dh"):
        v = getattr(gr, k)
        out[k] = None if v is None else v.cpu().numpy()
    return out


KEYS = ("dQ", "dq", "dA", "db", "dG", "dh")


def _at_iterate(P, r):
    """The oracle's backward (FP64) at the GPU's returned iterate, h' = G z + s."""
    import oracle
    c = lambda x: None if x is None else np.asarray(x, dtype=np.float32).astype(np.float64)
    Q, A, G, g = c(P["Q"]), c(P.get("A")), c(P.get("G")), c(P["g"])
    z, lam, nu, s = (np.asarray(r[k], np.float64) for k in ("z", "lam", "nu", "s"))
    return oracle.backward(Q, A, G, G @ z + s, z, lam, nu, g)


@pytest.mark.parametrize("case", ["cpu_check", "paper_scale"])
def test_fp32_only_backward(case):
    from paper_1703_00443_amd import binding as qb
    cfg = synth.CPU_CHECK if case == "cpu_check" else synth.PAPER_SCALE
    b = synth.make_batch(**cfg)
    f32 = _run(b, qb.FLAG_BWD_FP32)
    mix = _run(b, 0)
    B = b.Q.shape[0]
    # the forward is the same launch with the same inputs: bitwise equal
    for k in ("z", "lam", "s", "iters"):
        np.testing.assert_array_equal(f32[k], mix[k])
    idx = range(B) if B <= 16 else range(0, B, 8)
    errs, errs_mix = [], []
    for i in idx:
        P = b.problem(i)
        r = {k: f32[k][i] for k in ("z", "lam", "nu", "s")}
        go = _at_iterate(P, r)
        sc = grad_scale(go)
        e = max(g_err(f32[k][i], go[k], sc) for k in KEYS if f32[k] is not None)
        em = max(g_err(mix[k][i], go[k], sc) for k in KEYS if mix[k] is not None)
        errs.append(e)
        errs_mix.append(em)
        log_margins("bwd_fp32_%s[%d]" % (case, i), {"grad_at_iterate": float(e), "default_backward": float(em)})
    errs = np.array(errs)
    # FP32 arithmetic against an FP64 reference at the same iterate
    assert np.median(errs) <= 5e-3, errs
    assert errs.max() <= 5e-2, errs


def test_fp32_only_backward_uneven_batch_equals_uniform():
    """QP_FLAG_BWD_FP32 through qp_backward_varlen: every problem's gradients
    equal, to FP32 rounding, to the same problem's through qp_backward_batched
    with the flag (the same per-problem code in another kernel), on problems of
    several sizes."""
    import torch
    from paper_1703_00443_amd import binding as qb
    from paper_1703_00443_amd.varlen import VarlenBatch
    dims = [(10, 20, 5), (40, 60, 0), (100, 100, 0), (64, 32, 8)]
    probs = synth.make_varlen(31, dims, dtype=np.float32)
    flag = qb.default_opts(torch.float32, flags=qb.FLAG_BWD_FP32)
    vb = VarlenBatch(probs, dtype=torch.float32)
    vb.forward(flag).backward(vb.pack_vectors([P["g"] for P in probs]), opts=flag)
    torch.cuda.synchronize()
    for i, P in enumerate(probs):
        n, m, p = dims[i]
        b = synth.QPBatch(*(np.asarray(P[k], np.float32)[None] if P.get(k) is not None else
                            np.zeros((1, 0, n) if k in ("A", "G") else (1, 0), np.float32)
                            for k in ("Q", "q", "A", "b", "G", "h", "g")))
        one = _run(b, qb.FLAG_BWD_FP32)
        r = vb.result(i)
        assert r["iters"] == one["iters"][0]
        np.testing.assert_allclose(r["z"], one["z"][0], rtol=1e-5, atol=1e-5 * np.abs(one["z"][0]).max())
        sc = max(np.abs(one[k][0]).max() for k in KEYS if one[k] is not None and one[k].size)
        for k in KEYS:
            if one[k] is not None and one[k].size:
                np.testing.assert_allclose(r[k], one[k][0], rtol=0, atol=1e-4 * sc, err_msg="%d %s" % (i, k))
