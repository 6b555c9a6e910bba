"""ctypes binding of libqpmi.so (declared in include/qpmi.h).

Argument marshalling only: every step of the solve runs in the HIP library.
torch supplies device memory and the current stream.  There is no fallback:
if the library is missing or no GPU is present the calls raise.

Low-level names mirror the C ABI (qp_forward_batched, qp_backward_batched,
qp_forward_varlen, qp_backward_varlen, ...); ``forward`` / ``backward`` are
the tensor-level wrappers used by the autograd Function, the bench and tests.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqpmi.so")

QP_F32, QP_F64 = 0, 1
QP_OK, QP_EARG, QP_EWS, QP_EDTYPE, QP_EHIP, QP_ENODEV, QP_ETOOBIG = 0, -1, -2, -3, -4, -5, -6
STATUS_OPTIMAL, STATUS_MAX_ITER, STATUS_BREAKDOWN, STATUS_NONFINITE, STATUS_STALLED = 0, 1, 2, 3, 4
VARIANT_AUTO, VARIANT_GENERIC, VARIANT_LDS, VARIANT_TILED, VARIANT_STREAM, VARIANT_ELIM = 0, 1, 2, 3, 4, 5
FLAG_G_UNIT_ROWS = 1  # qp_opts.flags: every row of G is a signed unit vector
FLAG_BWD_FP32 = 2     # qp_opts.flags: the FP32 backward computes in FP32 only

_ERRNAMES = {QP_EARG: "QP_EARG", QP_EWS: "QP_EWS", QP_EDTYPE: "QP_EDTYPE", QP_EHIP: "QP_EHIP",
             QP_ENODEV: "QP_ENODEV", QP_ETOOBIG: "QP_ETOOBIG"}


class qp_dims(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nineq", ctypes.c_int32), ("neq", ctypes.c_int32)]


class qp_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("tol", ctypes.c_double), ("variant", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class qp_data(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("Q", "q", "A", "b", "G", "h")] + \
               [(k, ctypes.c_int64) for k in ("sQ", "sq", "sA", "sb", "sG", "sh")]


class qp_problem_desc(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nineq", ctypes.c_int32), ("neq", ctypes.c_int32),
                ("variant", ctypes.c_int32)] + \
               [(k, ctypes.c_int64) for k in ("Q", "q", "A", "b", "G", "h", "z", "lam", "nu",
                                              "state")]


EXPORTED = ("qp_default_opts", "qp_state_bytes", "qp_workspace_query", "qp_forward_batched",
            "qp_backward_batched", "qp_backward_batched_noalloc", "qp_varlen_workspace_query",
            "qp_forward_varlen", "qp_backward_varlen", "qp_plan", "qp_last_hip_error", "qp_version")
NOALLOC_SCRATCH_BYTES = 16 << 20  # QP_NOALLOC_SCRATCH_BYTES

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libqpmi.so and declare its signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libqpmi.so is not built (%s); run `python -m paper_1703_00443_amd.build`"
                           % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER
    lib.qp_default_opts.argtypes = [i32, P(qp_opts)]
    lib.qp_state_bytes.argtypes = [i32, qp_dims, P(sz)]
    lib.qp_workspace_query.argtypes = [i32, i32, qp_dims, P(qp_opts), P(sz), P(sz)]
    lib.qp_forward_batched.argtypes = [i32, i32, qp_dims, P(qp_data), P(qp_opts), vp, vp, vp, vp,
                                       vp, vp, vp, vp, sz, vp]
    lib.qp_backward_batched.argtypes = [i32, i32, qp_dims, P(qp_data), P(qp_opts), vp, vp, vp, vp,
                                        vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.qp_backward_batched_noalloc.argtypes = [i32, i32, qp_dims, P(qp_data), P(qp_opts), vp, vp, vp,
                                                vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.qp_varlen_workspace_query.argtypes = [i32, i32, vp, P(qp_opts), P(sz), P(sz), P(sz)]
    lib.qp_forward_varlen.argtypes = [i32, i32, vp, vp, vp, vp, P(qp_opts), vp, vp, vp, vp, vp, vp,
                                      vp, vp, sz, vp]
    lib.qp_backward_varlen.argtypes = [i32, i32, vp, vp, vp, vp, P(qp_opts), vp, vp, vp, vp, vp, vp,
                                       vp, vp, sz, vp]
    lib.qp_plan.argtypes = [i32, qp_dims, i32, P(i32), P(i32)]
    lib.qp_last_hip_error.argtypes = []
    lib.qp_version.argtypes = []
    for name in EXPORTED:
        getattr(lib, name).restype = i32
    if path == LIB_PATH:
        _lib = lib
    return lib


def _check(rc, what):
    if rc != QP_OK:
        extra = ""
        if rc == QP_EHIP:
            extra = " (hipError %d)" % load_library().qp_last_hip_error()
        raise RuntimeError("%s failed: %s%s" % (what, _ERRNAMES.get(rc, str(rc)), extra))


def dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float64:
        return QP_F64
    if dt == torch.float32:
        return QP_F32
    raise TypeError("qpmi supports float32 and float64, got %s" % dt)


def default_opts(dt: torch.dtype, **over) -> qp_opts:
    o = qp_opts()
    _check(load_library().qp_default_opts(dtype_code(dt), ctypes.byref(o)), "qp_default_opts")
    for k, v in over.items():
        if v is not None:
            setattr(o, k, v)
    return o


def state_bytes(dt: torch.dtype, n: int, m: int, p: int) -> int:
    v = ctypes.c_size_t(0)
    _check(load_library().qp_state_bytes(dtype_code(dt), qp_dims(n, m, p), ctypes.byref(v)),
           "qp_state_bytes")
    return int(v.value)


def plan(dt: torch.dtype, n: int, m: int, p: int, variant: int = 0):
    """(policy, lds_bytes): the factorization policy (a VARIANT_* code) the
    forward runs for one problem of these dims on the current device."""
    pol, lds = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load_library().qp_plan(dtype_code(dt), qp_dims(n, m, p), variant, ctypes.byref(pol),
                                  ctypes.byref(lds)), "qp_plan")
    return int(pol.value), int(lds.value)


def workspace_bytes(dt: torch.dtype, batch: int, n: int, m: int, p: int, opts=None):
    f, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    o = opts if opts is not None else default_opts(dt)
    _check(load_library().qp_workspace_query(dtype_code(dt), batch, qp_dims(n, m, p),
                                             ctypes.byref(o), ctypes.byref(f), ctypes.byref(b)),
           "qp_workspace_query")
    return int(f.value), int(b.value)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None or t.numel() == 0 else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_gpu(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise RuntimeError("qpmi runs on the GPU only: got a %s tensor" % t.device)


@dataclass
class Problem:
    """Batched problem data with per-tensor batch strides (0 = shared)."""
    Q: torch.Tensor
    q: torch.Tensor
    A: Optional[torch.Tensor]
    b: Optional[torch.Tensor]
    G: Optional[torch.Tensor]
    h: Optional[torch.Tensor]
    batch: int
    n: int
    m: int
    p: int

    def data(self) -> qp_data:
        d = qp_data()
        n, m, p = self.n, self.m, self.p
        for name, t, per in (("Q", self.Q, n * n), ("q", self.q, n), ("A", self.A, p * n),
                             ("b", self.b, p), ("G", self.G, m * n), ("h", self.h, m)):
            setattr(d, name, None if t is None or t.numel() == 0 else t.data_ptr())
            batched = t is not None and t.dim() == {"Q": 3, "q": 2, "A": 3, "b": 2, "G": 3, "h": 2}[name]
            setattr(d, "s" + name, per if (batched and t.shape[0] > 1) else 0)
        return d


def make_problem(Q, q, A=None, b=None, G=None, h=None) -> Problem:
    """Validate shapes and make every tensor contiguous with one dtype/device.
    Leading batch dims are optional per tensor (absent or size 1 = shared)."""
    _require_gpu(Q, q, A, b, G, h)
    dt = Q.dtype
    n = Q.shape[-1]
    if Q.shape[-2] != n:
        raise ValueError("Q must be square")
    m = 0 if G is None else G.shape[-2]
    p = 0 if A is None else A.shape[-2]
    if m == 0:
        G = h = None
    if p == 0:
        A = b = None
    sizes = []
    for t, nd in ((Q, 3), (q, 2), (A, 3), (b, 2), (G, 3), (h, 2)):
        if t is not None:
            if t.dtype != dt:
                raise TypeError("all problem tensors must share one dtype")
            if t.dim() == nd:
                sizes.append(t.shape[0])
    batch = max(sizes) if sizes else 1
    for s in sizes:
        if s not in (1, batch):
            raise ValueError("inconsistent batch sizes %s" % sizes)
    c = lambda t: None if t is None else t.contiguous()
    return Problem(c(Q), c(q), c(A), c(b), c(G), c(h), batch, n, m, p)


@dataclass
class ForwardResult:
    z: torch.Tensor
    lam: torch.Tensor
    nu: torch.Tensor
    s: torch.Tensor
    state: torch.Tensor
    status: torch.Tensor
    iters: torch.Tensor


def forward(prob: Problem, opts: Optional[qp_opts] = None, out: Optional[ForwardResult] = None
            ) -> ForwardResult:
    """qp_forward_batched on the current stream."""
    lib = load_library()
    dt = prob.Q.dtype
    B, n, m, p = prob.batch, prob.n, prob.m, prob.p
    o = opts if opts is not None else default_opts(dt)
    dev = prob.Q.device
    if out is None:
        sb = state_bytes(dt, n, m, p)
        out = ForwardResult(
            z=torch.empty(B, n, dtype=dt, device=dev), lam=torch.empty(B, m, dtype=dt, device=dev),
            nu=torch.empty(B, p, dtype=dt, device=dev), s=torch.empty(B, m, dtype=dt, device=dev),
            state=torch.empty(B * sb, dtype=torch.uint8, device=dev),
            status=torch.empty(B, dtype=torch.int32, device=dev),
            iters=torch.empty(B, dtype=torch.int32, device=dev))
    fws, _ = workspace_bytes(dt, B, n, m, p, o)
    ws = torch.empty(fws, dtype=torch.uint8, device=dev) if fws else None
    d = prob.data()
    rc = lib.qp_forward_batched(dtype_code(dt), B, qp_dims(n, m, p), ctypes.byref(d), ctypes.byref(o),
                                _ptr(out.z), _ptr(out.lam), _ptr(out.nu), _ptr(out.s),
                                _ptr(out.state), _ptr(out.status), _ptr(out.iters), _ptr(ws), fws,
                                _stream())
    _check(rc, "qp_forward_batched")
    return out


@dataclass
class Grads:
    dQ: Optional[torch.Tensor]
    dq: Optional[torch.Tensor]
    dA: Optional[torch.Tensor]
    db: Optional[torch.Tensor]
    dG: Optional[torch.Tensor]
    dh: Optional[torch.Tensor]


def backward(prob: Problem, fwd: ForwardResult, dl_dz: torch.Tensor, opts: Optional[qp_opts] = None,
             need=("Q", "q", "A", "b", "G", "h"), ws: Optional[torch.Tensor] = None) -> Grads:
    """qp_backward_batched on the current stream; gradients per problem [B, ...]."""
    lib = load_library()
    dt = prob.Q.dtype
    B, n, m, p = prob.batch, prob.n, prob.m, prob.p
    o = opts if opts is not None else default_opts(dt)
    dev = prob.Q.device
    dl_dz = dl_dz.to(dtype=dt).contiguous()
    if dl_dz.shape != (B, n):
        dl_dz = dl_dz.expand(B, n).contiguous()
    mk = lambda key, *shape: torch.empty(*shape, dtype=dt, device=dev) if key in need else None
    g = Grads(mk("Q", B, n, n), mk("q", B, n), mk("A", B, p, n) if p else None,
              mk("b", B, p) if p else None, mk("G", B, m, n) if m else None, mk("h", B, m) if m else None)
    _, bws = workspace_bytes(dt, B, n, m, p, o)
    if ws is None or ws.numel() < bws:
        ws = torch.empty(bws, dtype=torch.uint8, device=dev)
    d = prob.data()
    rc = lib.qp_backward_batched(dtype_code(dt), B, qp_dims(n, m, p), ctypes.byref(d), ctypes.byref(o),
                                 _ptr(fwd.z), _ptr(fwd.lam), _ptr(fwd.nu), _ptr(fwd.s), _ptr(fwd.state),
                                 _ptr(dl_dz), _ptr(g.dQ), _ptr(g.dq), _ptr(g.dA), _ptr(g.db), _ptr(g.dG),
                                 _ptr(g.dh), _ptr(ws), bws, _stream())
    _check(rc, "qp_backward_batched")
    return g


def backward_noalloc(prob: Problem, fwd: ForwardResult, dl_dz: torch.Tensor,
                     opts: Optional[qp_opts] = None, out: Optional[Grads] = None) -> Grads:
    """qp_backward_batched_noalloc on the current stream: the library allocates
    nothing (its adjoint workspace is a static device array).  The gradient
    tensors are the caller's: pass `out` to reuse them."""
    lib = load_library()
    dt = prob.Q.dtype
    B, n, m, p = prob.batch, prob.n, prob.m, prob.p
    o = opts if opts is not None else default_opts(dt)
    dev = prob.Q.device
    dl_dz = dl_dz.to(dtype=dt).contiguous()
    if out is None:
        mk = lambda *shape: torch.empty(*shape, dtype=dt, device=dev)
        out = Grads(mk(B, n, n), mk(B, n), mk(B, p, n) if p else None, mk(B, p) if p else None,
                    mk(B, m, n) if m else None, mk(B, m) if m else None)
    d = prob.data()
    g = out
    rc = lib.qp_backward_batched_noalloc(dtype_code(dt), B, qp_dims(n, m, p), ctypes.byref(d),
                                         ctypes.byref(o), _ptr(fwd.z), _ptr(fwd.lam), _ptr(fwd.nu),
                                         _ptr(fwd.s), _ptr(fwd.state), _ptr(dl_dz), _ptr(g.dQ),
                                         _ptr(g.dq), _ptr(g.dA), _ptr(g.db), _ptr(g.dG), _ptr(g.dh),
                                         _stream())
    _check(rc, "qp_backward_batched_noalloc")
    return g
