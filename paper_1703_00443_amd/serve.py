"""Serving loop with continuous batching for QP layer requests.

    srv = Server(dtype=torch.float32, hbm_budget=4 << 30, max_inflight=8)
    fut = srv.submit({"Q":..., "q":..., "G":..., "h":..., "A":..., "b":...},
                     need_backward=True, dl_dz=g)
    res = fut.result()        # dict: z, lam, nu, s, status, iters, grads (if asked), latency
    srv.close()

Requests arrive at any time.  A scheduler thread admits waiting requests
whenever an in-flight slot (one HIP stream per slot, default priority) is free
and the HBM footprint of everything in flight stays within the budget; the
admitted requests go out as one uneven-batch launch (forward, then backward for
the requests that asked for one) while earlier launches are still running on
other streams, so their work overlaps on the device.  A request larger than the
whole budget is rejected at submission.  Each launch records an event; the
scheduler completes the futures of a launch when its event has fired.

A launch completes when its slowest problem does, so requests are split into
size classes by nz (`class_bounds`) and a launch holds one class only; each
class may occupy at most its share of the slots.  Small requests then never
wait behind a large one's solve, and a burst of large requests cannot take
every slot.

The device work sits behind a small backend interface (`launch`, `ready`,
`collect`) so that the scheduler can be exercised without a GPU.
"""
from __future__ import annotations

import bisect
import collections
import math
import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


class RejectedError(RuntimeError):
    """The request's HBM footprint exceeds the server's whole budget."""


@dataclass
class Request:
    problem: Dict
    need_backward: bool
    dl_dz: Optional[np.ndarray]
    footprint: int
    t_arrival: float
    future: Future = field(default_factory=Future)
    dims: tuple = ()
    cls: int = 0
    fwd_bytes: int = 0
    bwd_bytes: int = 0


def state_bytes_host(esz: int, n: int, m: int, p: int) -> int:
    """qp_state_bytes without the library: the validity word, then U (leading
    dimension nz rounded up to 16), D, Wt and US, each region 256-byte aligned.
    A CPU test checks it against the library's answer."""
    al = lambda v: (v + 255) // 256 * 256
    ld = (n + 15) & ~15
    return int(256 + al(ld * ld * esz) + al(max(m, 1) * esz) + al((p * n if p else 1) * esz)
               + al((p * p if p else 1) * esz))


def footprint_parts(n: int, m: int, p: int, esz: int):
    """(forward bytes, backward bytes) a request occupies in an uneven-batch
    launch: the forward part is its packed inputs, outputs (z, lam, s, nu), factor
    state, status and iters; the backward part is its share of the gradient buffer
    (shaped like the inputs) and of the packed adjoint workspace.  A launch
    allocates the backward part of EVERY request it holds as soon as one of them
    asks for a backward (the gradient buffer covers all inputs)."""
    inputs = n * n + n + p * n + p + m * n + m
    # + status, iters (8 bytes), descriptor (96) and launch-order entry (4)
    fwd = esz * (inputs + n + 2 * m + p) + state_bytes_host(esz, n, m, p) + 108
    bwd = esz * (inputs + n + m + p)
    return int(fwd), int(bwd)


# launch-wide device bytes beyond the requests' own: the work-queue counter and the
# caching allocator's rounding of each of a launch's tensors (512 bytes apiece)
LAUNCH_OVERHEAD = 16384


def footprint_bytes(n: int, m: int, p: int, esz: int, need_backward: bool) -> int:
    """Device bytes one request occupies when it is launched alone."""
    f, b = footprint_parts(n, m, p, esz)
    return f + (b if need_backward else 0) + LAUNCH_OVERHEAD


def batch_bytes(reqs) -> int:
    """Device bytes of one launch of these requests (see footprint_parts)."""
    total = LAUNCH_OVERHEAD + sum(r.fwd_bytes for r in reqs)
    if any(r.need_backward for r in reqs):
        total += sum(r.bwd_bytes for r in reqs)
    return total


_DEDICATED: Dict[int, list] = {}
_DEDICATED_LOCK = threading.Lock()


def dedicated_stream(device_index: int, k: int):
    """The k-th stream of a process-wide pool (per device) whose streams each get a
    hardware queue of their own.  Streams that share a hardware queue run in
    order, so a short launch would wait behind a long one on another slot; HIP
    gives a stream created with a CU mask its own queue, and the full mask used
    here leaves every compute unit to it.  Default priority.  The streams live
    until the process ends (the caching allocator keeps blocks recorded on
    them), so they are reused across servers."""
    import ctypes
    import os
    import warnings
    import torch
    with _DEDICATED_LOCK:
        pool = _DEDICATED.setdefault(device_index, [])
        while len(pool) <= k:
            with torch.cuda.device(device_index):
                torch.cuda.init()
                hip = _loaded_hip_runtime(ctypes, os)
                if hip is None:  # only the queue assignment is lost, not correctness
                    warnings.warn("HIP runtime not found among loaded libraries; serving slots use "
                                  "ordinary streams, which may share hardware queues")
                    pool.append(torch.cuda.Stream(device=torch.device("cuda", device_index)))
                    continue
                cus = torch.cuda.get_device_properties(device_index).multi_processor_count
                words = (cus + 31) // 32
                mask = (ctypes.c_uint32 * words)(*([0xFFFFFFFF] * words))
                s = ctypes.c_void_p()
                rc = hip.hipExtStreamCreateWithCUMask(ctypes.byref(s), ctypes.c_uint32(words), mask)
                if rc != 0:
                    raise RuntimeError("hipExtStreamCreateWithCUMask failed: %d" % rc)
                pool.append(torch.cuda.ExternalStream(s.value, device=torch.device("cuda", device_index)))
        return pool[k]


def _loaded_hip_runtime(ctypes, os):
    """The HIP runtime torch already loaded (never a second copy: RTLD_NOLOAD)."""
    for name in ("libamdhip64.so.7", "libamdhip64.so.6", "libamdhip64.so"):
        try:
            return ctypes.CDLL(name, mode=os.RTLD_NOLOAD | ctypes.RTLD_GLOBAL)
        except OSError:
            continue
    return None


class DeviceBackend:
    """Launches admitted requests on HIP streams through VarlenBatch."""

    def __init__(self, dtype, device=None, table=None, opts=None):
        import torch
        from .autotune import AutotuneTable
        self.torch = torch
        self.dtype = dtype
        self.device = device or torch.device("cuda:0")
        self.table = table if table is not None else AutotuneTable.load()
        self.opts = opts
        self.esz = 8 if dtype == torch.float64 else 4

    def new_slot(self):
        idx = self.device.index if self.device.index is not None else 0
        self._slots = getattr(self, "_slots", 0) + 1
        return dedicated_stream(idx, self._slots - 1)

    def launch(self, slot, reqs: List[Request]):
        torch = self.torch
        from .varlen import VarlenBatch
        torch.cuda.set_device(self.device)
        with torch.cuda.stream(slot):
            vb = VarlenBatch([r.problem for r in reqs], dtype=self.dtype, device=self.device,
                             table=self.table)
            vb.forward(self.opts)
            nb = [r.need_backward for r in reqs]
            if any(nb):
                dl = vb.pack_vectors([r.dl_dz if r.need_backward else np.zeros(r.dims[0]) for r in reqs])
                need = torch.tensor([1 if b else 0 for b in nb], dtype=torch.int32)
                vb.backward(dl, need=need, opts=self.opts)
            # results go to pinned host buffers asynchronously on the same stream
            host = {}
            for k in ("z", "lam", "nu", "s", "status", "iters") + (("grad",) if any(nb) else ()):
                src = getattr(vb, k)
                dst = torch.empty(src.shape, dtype=src.dtype, pin_memory=True)
                dst.copy_(src, non_blocking=True)
                host[k] = dst
            host.setdefault("grad", None)
            ev = torch.cuda.Event()
            ev.record(slot)
        return {"vb": vb, "host": host, "event": ev}

    def ready(self, handle) -> bool:
        return handle["event"].query()

    def collect(self, handle, reqs: List[Request]) -> List[Dict]:
        vb, host = handle["vb"], handle["host"]
        out = []
        for i, r in enumerate(reqs):
            n, m, p = vb.dims[i]
            _, oz, ol, on = vb.offsets[i]
            d = vb.descs_host[i]
            res = {"z": host["z"][oz:oz + n].numpy(), "lam": host["lam"][ol:ol + m].numpy(),
                   "s": host["s"][ol:ol + m].numpy(), "nu": host["nu"][on:on + p].numpy(),
                   "status": int(host["status"][i]), "iters": int(host["iters"][i])}
            if r.need_backward:
                g = host["grad"]
                res.update({"dQ": g[d.Q:d.Q + n * n].view(n, n).numpy(), "dq": g[d.q:d.q + n].numpy(),
                            "dA": g[d.A:d.A + p * n].view(p, n).numpy(), "db": g[d.b:d.b + p].numpy(),
                            "dG": g[d.G:d.G + m * n].view(m, n).numpy(), "dh": g[d.h:d.h + m].numpy()})
            out.append(res)
        return out


class Server:
    def __init__(self, backend=None, dtype=None, hbm_budget: int = 4 << 30, max_inflight: int = 8,
                 max_batch: int = 512, idle_sleep: float = 2e-4, class_bounds=(64, 128, 256)):
        if backend is None:
            import torch
            backend = DeviceBackend(dtype if dtype is not None else torch.float32)
        self.backend = backend
        self.esz = getattr(backend, "esz", 4)
        self.budget = int(hbm_budget)
        self.max_batch = max_batch
        self.idle_sleep = idle_sleep
        # class c holds requests with class_bounds[c-1] < nz <= class_bounds[c]
        self.class_bounds = tuple(sorted(int(b) for b in class_bounds))
        n_cls = len(self.class_bounds) + 1
        self.class_cap = max(1, max_inflight // n_cls)
        self.class_inflight = [0] * n_cls
        self.slots = [backend.new_slot() for _ in range(max_inflight)]
        self.free_slots = collections.deque(range(max_inflight))
        self.waiting: "collections.deque[Request]" = collections.deque()
        self.incoming: "queue.Queue[Request]" = queue.Queue()
        self.inflight: List = []  # (slot index, handle, requests, bytes, class)
        self.bytes_in_flight = 0
        self.stats = {"admitted": 0, "rejected": 0, "launches": 0, "max_bytes_in_flight": 0,
                      "max_concurrent_launches": 0, "max_queue": 0, "launch_host_s": 0.0,
                      "launches_per_class": [0] * n_cls}
        self.failed: Optional[BaseException] = None
        self._stop = threading.Event()
        self._lock = threading.Lock()
        self._thread = threading.Thread(target=self._loop, name="qp-server", daemon=True)
        self._thread.start()

    # ---- client side ---------------------------------------------------------------------
    def submit(self, problem: Dict, need_backward: bool = False, dl_dz=None) -> Future:
        Q = np.asarray(problem["Q"])
        n = Q.shape[0]
        m = 0 if problem.get("G") is None else int(np.asarray(problem["G"]).reshape(-1, n).shape[0])
        p = 0 if problem.get("A") is None else int(np.asarray(problem["A"]).reshape(-1, n).shape[0])
        fb, bb = footprint_parts(n, m, p, self.esz)
        fp = fb + (bb if need_backward else 0) + LAUNCH_OVERHEAD
        req = Request(problem, need_backward, None if dl_dz is None else np.asarray(dl_dz), fp,
                      time.perf_counter(), dims=(n, m, p),
                      cls=bisect.bisect_left(self.class_bounds, n), fwd_bytes=fb, bwd_bytes=bb)
        if self.failed is not None:
            req.future.set_exception(RuntimeError("server stopped after an error: %r" % (self.failed,)))
            return req.future
        if need_backward and req.dl_dz is None:
            req.future.set_exception(ValueError("need_backward requires dl_dz"))
            return req.future
        if fp > self.budget:
            with self._lock:
                self.stats["rejected"] += 1
            req.future.set_exception(RejectedError(
                "request needs %d bytes of HBM, the server budget is %d" % (fp, self.budget)))
            return req.future
        self.incoming.put(req)
        return req.future

    def close(self, timeout: float = 60.0):
        self._stop.set()
        self._thread.join(timeout)

    # ---- scheduler -----------------------------------------------------------------------
    def _drain_incoming(self):
        while True:
            try:
                self.waiting.append(self.incoming.get_nowait())
            except queue.Empty:
                break
        self.stats["max_queue"] = max(self.stats["max_queue"], len(self.waiting))

    def _complete(self):
        still = []
        for slot, handle, reqs, nbytes, cls in self.inflight:
            if self.backend.ready(handle):
                try:
                    results = self.backend.collect(handle, reqs)
                    now = time.perf_counter()
                    for r, res in zip(reqs, results):
                        res["latency"] = now - r.t_arrival
                        if not r.future.cancelled():
                            r.future.set_result(res)
                except Exception as e:  # surface device errors on every request of the launch
                    for r in reqs:
                        if not r.future.done():
                            r.future.set_exception(e)
                self.bytes_in_flight -= nbytes
                self.free_slots.append(slot)
                self.class_inflight[cls] -= 1
            else:
                still.append((slot, handle, reqs, nbytes, cls))
        self.inflight = still

    def _next_class(self) -> Optional[int]:
        """Class of the oldest waiting request whose class has a slot share left."""
        for r in self.waiting:
            if not r.future.cancelled() and self.class_inflight[r.cls] < self.class_cap:
                return r.cls
        return None

    def _admit_and_launch(self) -> bool:
        launched = False
        while self.waiting and self.free_slots:
            cls = self._next_class()
            if cls is None:
                break
            batch, nbytes = [], 0
            sum_f = sum_b = 0
            any_b = False
            kept = collections.deque()
            for r in self.waiting:
                if r.future.cancelled():
                    continue
                # the launch's bytes with r in it: a backward anywhere in the launch
                # allocates the backward part of every request it holds
                cand = (LAUNCH_OVERHEAD + sum_f + r.fwd_bytes
                        + ((sum_b + r.bwd_bytes) if (any_b or r.need_backward) else 0))
                if (r.cls == cls and len(batch) < self.max_batch
                        and self.bytes_in_flight + cand <= self.budget):
                    batch.append(r)
                    sum_f += r.fwd_bytes
                    sum_b += r.bwd_bytes
                    any_b = any_b or r.need_backward
                    nbytes = cand
                else:
                    kept.append(r)  # another class, or waits until memory frees up
            self.waiting = kept
            if not batch:
                break
            slot = self.free_slots.popleft()
            t0 = time.perf_counter()
            try:
                handle = self.backend.launch(self.slots[slot], batch)
            except Exception as e:
                for r in batch:
                    r.future.set_exception(e)
                self.free_slots.append(slot)
                launched = True
                continue
            st = self.stats
            st["launch_host_s"] += time.perf_counter() - t0
            self.inflight.append((slot, handle, batch, nbytes, cls))
            self.bytes_in_flight += nbytes
            self.class_inflight[cls] += 1
            st["admitted"] += len(batch)
            st["launches"] += 1
            st["launches_per_class"][cls] += 1
            st["max_bytes_in_flight"] = max(st["max_bytes_in_flight"], self.bytes_in_flight)
            st["max_concurrent_launches"] = max(st["max_concurrent_launches"], len(self.inflight))
            launched = True
        return launched

    def _fail_all(self, exc: BaseException):
        """An unexpected scheduler error: every request not yet completed gets
        the exception, and the server stops accepting work."""
        self.failed = exc
        for _, _, reqs, _, _ in self.inflight:
            for r in reqs:
                if not r.future.done():
                    r.future.set_exception(exc)
        self.inflight = []
        self._drain_incoming()
        for r in self.waiting:
            if not r.future.done():
                r.future.set_exception(exc)
        self.waiting = collections.deque()

    def _loop(self):
        while True:
            try:
                self._drain_incoming()
                self._complete()
                launched = self._admit_and_launch()
            except Exception as e:  # keep no future waiting on a dead scheduler
                self._fail_all(e)
                break
            if self._stop.is_set() and not self.inflight and not self.waiting and self.incoming.empty():
                break
            if not launched:
                time.sleep(self.idle_sleep)


def percentiles(latencies, qs=(50, 99)):
    a = np.sort(np.asarray(latencies))
    return {"p%d" % q: float(a[min(len(a) - 1, int(math.ceil(q / 100.0 * len(a))) - 1)]) for q in qs}
