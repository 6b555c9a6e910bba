"""Uneven batches: many QPs of different sizes in one persistent launch.

    vb = VarlenBatch(problems, dtype=torch.float32)   # list of dicts Q,q,[A,b],[G,h]
    vb.forward()            # qp_forward_varlen: one launch over every problem
    vb.backward(dl_dz)      # qp_backward_varlen: gradients of the problems in `need`
    vb.result(i)            # per-problem views (z, lam, nu, s, status, iters, grads)

The packer lays all inputs out in one device buffer, builds the descriptor
table (qp_problem_desc per problem: dims, element offsets, state byte offset,
kernel variant) and a launch order with the most expensive problems first, so
that the kernel's work queue balances the launch.  Per-problem kernel variants
come from an autotune table keyed only by the problem's own size bucket, so a
problem is solved with the same arithmetic alone or inside any batch.

Argument marshalling only; the arithmetic runs in libqpmi.so.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import binding as qb

KEYS = ("Q", "q", "A", "b", "G", "h")


def cost_estimate(n: int, m: int, p: int) -> float:
    """Flops of one factorization (the dominant term of a Newton step)."""
    return n * (n + 1) * m + n ** 3 / 3.0 + n * n * p + p ** 3 / 3.0


def _to_device(t: torch.Tensor, dev: torch.device) -> torch.Tensor:
    """Host tensor to `dev` without blocking the host: a pageable copy would wait
    for all earlier work on the stream (e.g. the forward of the same batch)."""
    if t.device == dev:
        return t
    if dev.type == "cuda" and t.device.type == "cpu":
        return t.pin_memory().to(dev, non_blocking=True)
    return t.to(dev)


class VarlenBatch:
    def __init__(self, problems: Sequence[Dict], dtype: torch.dtype = torch.float32,
                 device: Optional[torch.device] = None, variants: Optional[Sequence[int]] = None,
                 table=None):
        dev = device or torch.device("cuda:0")
        self.dtype, self.device = dtype, dev
        self.count = len(problems)
        descs = (qb.qp_problem_desc * max(1, self.count))()
        self.dims = []
        off_in = 0
        off_z = off_l = off_n = 0
        off_state = 0
        arrays = []  # (offset, array or None, size) in packing order
        for i, P in enumerate(problems):
            Q = np.asarray(P["Q"])
            n = Q.shape[0]
            G = P.get("G")
            A = P.get("A")
            m = 0 if G is None else int(np.asarray(G).size // n)
            p = 0 if A is None else int(np.asarray(A).size // n)
            d = descs[i]
            d.nz, d.nineq, d.neq = n, m, p
            if variants is not None:
                d.variant = int(variants[i])
            elif table is not None:
                d.variant = int(table.variant_for(dtype, n, m, p))
            else:
                d.variant = 0
            for key, size in (("Q", n * n), ("q", n), ("A", p * n), ("b", p), ("G", m * n), ("h", m)):
                setattr(d, key, off_in)
                arrays.append((off_in, P.get(key), size))
                off_in += size
            d.z, d.lam, d.nu = off_z, off_l, off_n
            off_z += n; off_l += m; off_n += p
            d.state = off_state
            off_state += qb.state_bytes(dtype, n, m, p)
            self.dims.append((n, m, p))
        # one cast-and-copy per array into a (pinned, when the target is a GPU) staging
        # buffer of the target dtype, then one asynchronous copy to the device
        pinned = dev.type == "cuda"
        host_t = torch.empty(max(1, off_in), dtype=dtype, pin_memory=pinned)
        host = host_t.numpy()
        for off, v, size in arrays:
            if not size:
                continue
            if v is None:
                host[off:off + size] = 0
                continue
            a = np.asarray(v).reshape(-1)
            if a.size != size:
                raise ValueError("array of %d elements where the problem's dims need %d"
                                 % (a.size, size))
            np.copyto(host[off:off + size], a, casting="unsafe")
        self._host_in = host_t  # kept alive until the copy below has run
        self.base_in = host_t.to(dev, non_blocking=pinned)
        self.descs_host = descs
        raw = bytes(memoryview(descs))[: ctypes.sizeof(qb.qp_problem_desc) * self.count]
        self.descs_dev = _to_device(torch.frombuffer(bytearray(raw), dtype=torch.uint8), dev) if raw \
            else torch.zeros(1, dtype=torch.uint8, device=dev)
        order = sorted(range(self.count), key=lambda i: -cost_estimate(*self.dims[i]))
        self.order = _to_device(torch.tensor(order, dtype=torch.int32), dev)
        self.z = torch.zeros(max(1, off_z), dtype=dtype, device=dev)
        self.lam = torch.zeros(max(1, off_l), dtype=dtype, device=dev)
        self.s = torch.zeros(max(1, off_l), dtype=dtype, device=dev)
        self.nu = torch.zeros(max(1, off_n), dtype=dtype, device=dev)
        self.state = torch.zeros(max(1, off_state), dtype=torch.uint8, device=dev)
        self.status = torch.zeros(max(1, self.count), dtype=torch.int32, device=dev)
        self.iters = torch.zeros(max(1, self.count), dtype=torch.int32, device=dev)
        fws, bws, _ = self.workspace_bytes()
        self.fws = torch.zeros(max(1, fws), dtype=torch.uint8, device=dev)
        self._fws_bytes, self._bws_bytes = fws, bws
        # the gradient buffer (shaped like the inputs) and the adjoint workspace
        # are allocated by the first backward() only
        self.grad = None
        self.bws = None
        self.offsets = [(descs[i].Q, descs[i].z, descs[i].lam, descs[i].nu) for i in range(self.count)]

    def workspace_bytes(self, opts=None):
        o = opts if opts is not None else qb.default_opts(self.dtype)
        f, b, s = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
        qb._check(qb.load_library().qp_varlen_workspace_query(
            qb.dtype_code(self.dtype), self.count, ctypes.addressof(self.descs_host),
            ctypes.byref(o), ctypes.byref(f), ctypes.byref(b), ctypes.byref(s)),
            "qp_varlen_workspace_query")
        return int(f.value), int(b.value), int(s.value)

    def forward(self, opts=None):
        o = opts if opts is not None else qb.default_opts(self.dtype)
        P = qb._ptr
        rc = qb.load_library().qp_forward_varlen(
            qb.dtype_code(self.dtype), self.count, P(self.descs_dev), ctypes.addressof(self.descs_host),
            P(self.order), P(self.base_in), ctypes.byref(o), P(self.z), P(self.lam), P(self.nu), P(self.s),
            P(self.state), P(self.status), P(self.iters), P(self.fws), self._fws_bytes, qb._stream())
        qb._check(rc, "qp_forward_varlen")
        return self

    def backward_buffers(self):
        """Allocate the gradient buffer (shaped like the inputs) and the packed
        adjoint workspace, once."""
        if self.grad is None:
            self.grad = torch.zeros(self.base_in.shape, dtype=self.dtype, device=self.device)
            self.bws = torch.zeros(max(1, self._bws_bytes), dtype=torch.uint8, device=self.device)
        return self

    def backward(self, dl_dz: torch.Tensor, need: Optional[torch.Tensor] = None, opts=None):
        """dl_dz packed like z (concatenation of the problems' z); `need` an int32
        mask per problem (None = all).  Gradients land in self.grad, packed like
        the inputs."""
        o = opts if opts is not None else qb.default_opts(self.dtype)
        P = qb._ptr
        self.backward_buffers()
        g = _to_device(dl_dz.to(dtype=self.dtype).contiguous(), self.device)
        self._dl = g
        self._need = None if need is None else \
            _to_device(need.to(dtype=torch.int32).contiguous(), self.device)
        rc = qb.load_library().qp_backward_varlen(
            qb.dtype_code(self.dtype), self.count, P(self.descs_dev), ctypes.addressof(self.descs_host),
            P(self._need), P(self.base_in), ctypes.byref(o), P(self.z), P(self.lam), P(self.nu), P(self.s),
            P(self.state), P(g), P(self.grad), P(self.bws), self._bws_bytes, qb._stream())
        qb._check(rc, "qp_backward_varlen")
        return self

    # ---- unpacking --------------------------------------------------------------------------
    def views(self, i: int) -> Dict[str, torch.Tensor]:
        n, m, p = self.dims[i]
        oin, oz, ol, on = self.offsets[i]
        d = self.descs_host[i]
        out = {
            "z": self.z[oz:oz + n], "lam": self.lam[ol:ol + m], "s": self.s[ol:ol + m],
            "nu": self.nu[on:on + p], "status": self.status[i], "iters": self.iters[i],
        }
        g = self.grad
        if g is not None:
            out.update({
                "dQ": g[d.Q:d.Q + n * n].view(n, n), "dq": g[d.q:d.q + n],
                "dA": g[d.A:d.A + p * n].view(p, n), "db": g[d.b:d.b + p],
                "dG": g[d.G:d.G + m * n].view(m, n), "dh": g[d.h:d.h + m],
            })
        return out

    def result(self, i: int) -> Dict[str, np.ndarray]:
        return {k: (v.cpu().numpy() if v.dim() else int(v.item())) for k, v in self.views(i).items()}

    def pack_vectors(self, vecs: List[np.ndarray]) -> torch.Tensor:
        """Concatenate per-problem z-shaped vectors (e.g. dl/dz) in packing order."""
        pinned = self.device.type == "cuda"
        total = sum(n for n, _, _ in self.dims)
        host_t = torch.empty(max(1, total), dtype=self.dtype, pin_memory=pinned)
        host = host_t.numpy()
        off = 0
        for (n, _, _), v in zip(self.dims, vecs):
            a = np.asarray(v).reshape(-1)
            if a.size != n:
                raise ValueError("vector of %d elements for a problem with nz = %d" % (a.size, n))
            np.copyto(host[off:off + n], a, casting="unsafe")
            off += n
        self._host_vec = host_t  # kept alive until the copy below has run
        return host_t[:total].to(self.device, non_blocking=pinned)


def problem_device_bytes(n: int, m: int, p: int, dtype: torch.dtype, backward: bool) -> int:
    """Device bytes a VarlenBatch allocates for one problem of these dims: packed
    inputs, outputs (z, lam, s, nu), the factor state (qp_state_bytes), status and
    iters; with `backward` also its share of the gradient buffer (shaped like the
    inputs) and of the packed adjoint workspace (nz + nineq + neq).  The
    launch-wide forward workspace (one work-queue counter) is not included."""
    esz = torch.finfo(dtype).bits // 8
    inputs = n * n + n + p * n + p + m * n + m
    total = esz * (inputs + n + 2 * m + p) + qb.state_bytes(dtype, n, m, p) + 8
    if backward:
        total += esz * (inputs + n + m + p)
    return int(total)


def allocated_bytes(vb: "VarlenBatch") -> int:
    """Bytes of the device tensors a VarlenBatch holds now (inputs, outputs, state,
    status, iters, descriptors, order, workspaces, gradients)."""
    ts = [vb.base_in, vb.z, vb.lam, vb.s, vb.nu, vb.state, vb.status, vb.iters, vb.descs_dev,
          vb.order, vb.fws, vb.grad, vb.bws]
    return int(sum(t.numel() * t.element_size() for t in ts if t is not None))


def capture_graph(vb: VarlenBatch, dl_dz: torch.Tensor, need: Optional[torch.Tensor] = None,
                  opts=None):
    """Capture forward + backward of an uneven batch into a HIP graph (torch.cuda.CUDAGraph).
    The launches read the batch's device buffers, so refreshing the inputs in place
    (vb.base_in, the dl_dz tensor) and replaying the graph re-solves.  The graph
    holds kernel nodes only (the work-queue counter is cleared by a kernel).  A
    host-side `need` mask is copied to the device before the capture, and the copy
    is kept on `vb` for the graph's lifetime."""
    if need is not None and need.device != vb.device:
        need = need.to(dtype=torch.int32).contiguous().to(vb.device)
        torch.cuda.synchronize()
    vb._graph_need = need
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        vb.forward(opts)
        vb.backward(dl_dz, need, opts)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        vb.forward(opts)
        vb.backward(dl_dz, need, opts)
    return g
