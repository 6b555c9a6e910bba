"""qp_backward_batched_noalloc (the backward for callers that cannot allocate
device memory) against qp_backward_batched through the C ABI: the same kernels
on the same inputs, so the gradients must be bitwise equal.  Two calls in a row
share the library's static scratch array, the second with a smaller input; a
request larger than the array is refused on the host."""
import ctypes

import numpy as np
import pytest

from paper_1703_00443_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("dQ", "dq", "dA", "db", "dG", "dh")


def _case(batch, dtype):
    import torch
    from paper_1703_00443_amd import binding as qb
    dev = torch.device("cuda:0")
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x.astype(dtype))).to(dev)
    n, m, p = batch.dims
    prob = qb.make_problem(T(batch.Q), T(batch.q), T(batch.A) if p else None, T(batch.b) if p else None,
                           T(batch.G) if m else None, T(batch.h) if m else None)
    fw = qb.forward(prob)
    return prob, fw, T(batch.g)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_backward_equals_backward_on_two_calls(dtype):
    import torch
    from paper_1703_00443_amd import binding as qb
    cases = [synth.make_batch(**synth.PAPER_SCALE), synth.make_batch(**synth.CPU_CHECK)]
    for k, batch in enumerate(cases):  # the second call is the smaller one
        print("noalloc case", k, batch.dims, batch.q.shape[0], np.dtype(dtype).name, flush=True)
        prob, fw, g = _case(batch, dtype)
        ref = qb.backward(prob, fw, g)
        got = qb.backward_noalloc(prob, fw, g)
        torch.cuda.synchronize()
        for key in KEYS:
            a, b = getattr(ref, key), getattr(got, key)
            if a is None:
                assert b is None, key
                continue
            assert torch.equal(a, b), (k, key)


def test_noalloc_refuses_more_than_its_scratch():
    from paper_1703_00443_amd import binding as qb
    lib = qb.load_library()
    o = qb.default_opts(__import__("torch").float64)
    d = qb.qp_data()
    # 100000 FP64 problems of nz = nineq = 100 need 100000 * 256 * 8 bytes of adjoints
    rc = lib.qp_backward_batched_noalloc(qb.QP_F64, 100000, qb.qp_dims(100, 100, 0), ctypes.byref(d),
                                         ctypes.byref(o), *([None] * 12), None)
    assert rc == qb.QP_EWS
