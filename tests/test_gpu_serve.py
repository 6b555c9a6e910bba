"""Serving on the GPU: a Poisson stream of 100 mixed-size requests (half with a
backward) through the continuous-batching server; every result must equal the
same request solved alone (same kernel variant => bitwise), and every tenth is
checked against the oracle."""
import time

import numpy as np
import pytest

from paper_1703_00443_amd import synth

from parity import TOL_Z, oracle_replay, z_err

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone_results():
    import torch
    from paper_1703_00443_amd.serve import Server
    from paper_1703_00443_amd.varlen import VarlenBatch
    dims = synth.serving_dims(55, 100, n_lo=16, n_hi=192)
    probs = synth.make_varlen(55, [d[:3] for d in dims], dtype=np.float32)
    srv = Server(dtype=torch.float32, hbm_budget=1 << 30, max_inflight=3)
    rng = np.random.default_rng(1)
    futs = []
    for P, d in zip(probs, dims):
        futs.append(srv.submit(P, need_backward=d[3], dl_dz=P["g"] if d[3] else None))
        time.sleep(rng.exponential(0.002))
    res = [f.result(timeout=120) for f in futs]
    srv.close()
    assert srv.stats["admitted"] == len(probs)
    assert srv.stats["launches"] > 1
    for i in range(len(probs)):
        P = probs[i]
        one = VarlenBatch([P], dtype=torch.float32, table=srv.backend.table)
        one.forward()
        if dims[i][3]:
            one.backward(one.pack_vectors([P["g"]]))
        torch.cuda.synchronize()
        a = one.result(0)
        np.testing.assert_array_equal(res[i]["z"], a["z"])
        np.testing.assert_array_equal(res[i]["lam"], a["lam"])
        if dims[i][3]:
            np.testing.assert_array_equal(res[i]["dG"], a["dG"])
            np.testing.assert_array_equal(res[i]["dQ"], a["dQ"])
        assert res[i]["latency"] > 0
        if i % 10 == 0:
            ref = oracle_replay(P, res[i]["iters"], np.float32)
            assert z_err(res[i]["z"], ref["z"]) <= TOL_Z[np.float32]


def test_served_fp64_results_equal_alone_results():
    """The same in FP64: 30 requests (nz up to 128), results bitwise equal to the
    request solved alone, and z against the oracle for every fifth."""
    import torch
    from paper_1703_00443_amd.serve import Server
    from paper_1703_00443_amd.varlen import VarlenBatch
    dims = synth.serving_dims(56, 30, n_lo=8, n_hi=128)
    probs = synth.make_varlen(56, [d[:3] for d in dims])
    srv = Server(dtype=torch.float64, hbm_budget=1 << 30)
    futs = [srv.submit(P, need_backward=d[3], dl_dz=P["g"] if d[3] else None) for P, d in zip(probs, dims)]
    res = [f.result(timeout=120) for f in futs]
    srv.close()
    assert srv.stats["admitted"] == len(probs)
    for i, P in enumerate(probs):
        one = VarlenBatch([P], dtype=torch.float64, table=srv.backend.table)
        one.forward()
        if dims[i][3]:
            one.backward(one.pack_vectors([P["g"]]))
        torch.cuda.synchronize()
        a = one.result(0)
        np.testing.assert_array_equal(res[i]["z"], a["z"])
        if dims[i][3]:
            np.testing.assert_array_equal(res[i]["dQ"], a["dQ"])
        if i % 5 == 0:
            ref = oracle_replay(P, res[i]["iters"], np.float64)
            assert z_err(res[i]["z"], ref["z"]) <= TOL_Z[np.float64]


def test_served_large_requests_equal_alone_results():
    """Requests with nz up to 512 (the streamed-tile policy above 256 in FP32)
    in the mix: 24 requests, half with a backward, each result bitwise equal to
    the request solved alone, and every output of three of them against the oracle."""
    import torch
    from paper_1703_00443_amd.serve import Server
    from paper_1703_00443_amd.varlen import VarlenBatch
    from paper_1703_00443_amd import binding as qb
    dims = synth.serving_dims(57, 24, n_lo=200, n_hi=512)
    assert max(d[0] for d in dims) > 256
    assert any(qb.plan(torch.float32, *d[:3])[0] == qb.VARIANT_STREAM for d in dims)
    probs = synth.make_varlen(57, [d[:3] for d in dims], dtype=np.float32)
    srv = Server(dtype=torch.float32, hbm_budget=1 << 30, max_inflight=4)
    futs = [srv.submit(P, need_backward=d[3], dl_dz=P["g"] if d[3] else None) for P, d in zip(probs, dims)]
    res = [f.result(timeout=300) for f in futs]
    srv.close()
    assert srv.stats["admitted"] == len(probs)
    for i, P in enumerate(probs):
        one = VarlenBatch([P], dtype=torch.float32, table=srv.backend.table)
        one.forward()
        if dims[i][3]:
            one.backward(one.pack_vectors([P["g"]]))
        torch.cuda.synchronize()
        a = one.result(0)
        for k in ("z", "lam", "nu", "s"):
            np.testing.assert_array_equal(res[i][k], a[k], err_msg="%d %s" % (i, k))
        if dims[i][3]:
            for k in ("dQ", "dG", "dh"):
                np.testing.assert_array_equal(res[i][k], a[k], err_msg="%d %s" % (i, k))
    # the oracle (unreduced LU of size nz + 2 nineq + neq) on the three smallest
    # requests, two of them with a backward
    from parity import compare_problem
    order = sorted(range(len(dims)), key=lambda i: dims[i][0] + 2 * dims[i][1])
    picked = [i for i in order if dims[i][3]][:2] + [i for i in order if not dims[i][3]][:1]
    for i in picked:
        compare_problem(probs[i], dict(res[i]), np.float32, tag="serve_large[%d]%s" % (i, dims[i][:3]),
                        grads=bool(dims[i][3]))
