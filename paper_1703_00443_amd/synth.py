"""Seeded synthetic QP generators (inputs only; none of the solver's arithmetic).

Shared by the tests (which feed the same arrays to the HIP path and to the
oracle), the bench and the serving demo.  The recipe follows the paper's timing
experiment (Section 4.1, its footnote: Q = U^T U + 1e-3 I, G normal, h = G z0 + s0
with z0 normal and s0 uniform so that every problem is feasible) and the MNIST
layer parametrisation (Appendix A: Q = L L^T + eps I, b = A z0, h = G z0 + s0):

    L ~ N(0,1) [n,n],  Q = L L^T / n + 1e-3 I,  q ~ N(0,1) [n],
    G ~ N(0,1) [m,n] (rows optionally scaled to unit 2-norm),  A ~ N(0,1) [p,n],
    z0 ~ N(0,1) [n],  s0 ~ U(0,1) [m],  h = G z0 + s0,  b = A z0,
    dl/dz ~ N(0,1) [n].

Problem i of a batch drawn with seed S uses ``numpy.random.default_rng([S, i])``
so that every problem regenerates alone, independent of its batch.
All arrays are generated in float64; FP32 runs cast the same arrays.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class QPBatch:
    Q: np.ndarray  # [B,n,n]
    q: np.ndarray  # [B,n]
    A: np.ndarray  # [B,p,n]
    b: np.ndarray  # [B,p]
    G: np.ndarray  # [B,m,n]
    h: np.ndarray  # [B,m]
    g: np.ndarray  # [B,n]  upstream gradient dl/dz

    @property
    def dims(self):
        return self.Q.shape[1], self.G.shape[1], self.A.shape[1]

    def astype(self, dtype):
        return QPBatch(*(np.ascontiguousarray(x.astype(dtype)) for x in
                         (self.Q, self.q, self.A, self.b, self.G, self.h, self.g)))

    def problem(self, i):
        return {k: getattr(self, k)[i] for k in ("Q", "q", "A", "b", "G", "h", "g")}


def one_problem(rng: np.random.Generator, n: int, m: int, p: int, row_normalize: bool = False):
    L = rng.standard_normal((n, n))
    Q = L @ L.T / n + 1e-3 * np.eye(n)
    q = rng.standard_normal(n)
    G = rng.standard_normal((m, n))
    A = rng.standard_normal((p, n))
    z0 = rng.standard_normal(n)
    s0 = rng.uniform(0.0, 1.0, m)
    if row_normalize and m > 0:
        G = G / np.linalg.norm(G, axis=1, keepdims=True)
    h = G @ z0 + s0
    b = A @ z0
    g = rng.standard_normal(n)
    return Q, q, A, b, G, h, g


def make_batch(seed: int, B: int, n: int, m: int, p: int, row_normalize: bool = False,
               dtype=np.float64) -> QPBatch:
    parts = [one_problem(np.random.default_rng([seed, i]), n, m, p, row_normalize)
             for i in range(B)]
    arrs = [np.stack([pp[k] for pp in parts]) if B > 0 else None for k in range(7)]
    if B == 0:
        arrs = [np.zeros((0, n, n)), np.zeros((0, n)), np.zeros((0, p, n)), np.zeros((0, p)),
                np.zeros((0, m, n)), np.zeros((0, m)), np.zeros((0, n))]
    return QPBatch(*arrs).astype(dtype)


def box_batch(seed: int, B: int, n: int, dtype=np.float64) -> QPBatch:
    """Box-constrained QPs l <= z <= u (the bound constraints of the paper's
    ReLU layer in the proof of Theorem 2, z >= 0, and box bounds): G = [I; -I], h = [u; -l] with
    u ~ U(0.5, 1.5), l ~ -U(0.5, 1.5); Q, q and dl/dz as above (q scaled by 3
    so that a good share of the bounds is active).  Problem i uses
    default_rng([seed, i])."""
    I = np.eye(n)
    G = np.concatenate([I, -I])
    parts = []
    for i in range(B):
        rng = np.random.default_rng([seed, i])
        L = rng.standard_normal((n, n))
        Q = L @ L.T / n + 1e-3 * np.eye(n)
        q = 3.0 * rng.standard_normal(n)
        u = rng.uniform(0.5, 1.5, n)
        lo = -rng.uniform(0.5, 1.5, n)
        g = rng.standard_normal(n)
        parts.append((Q, q, np.concatenate([u, -lo]), g))
    return QPBatch(np.stack([x[0] for x in parts]), np.stack([x[1] for x in parts]),
                   np.zeros((B, 0, n)), np.zeros((B, 0)), np.broadcast_to(G, (B, 2 * n, n)).copy(),
                   np.stack([x[2] for x in parts]), np.stack([x[3] for x in parts])).astype(dtype)


# Workload shapes (sizes from the paper's timing experiment and its extensions).
CPU_CHECK = dict(seed=1000, B=8, n=10, m=20, p=5, row_normalize=False)
PAPER_SCALE = dict(seed=1001, B=128, n=100, m=100, p=0, row_normalize=True)
DIFF_SCALE = dict(seed=1002, B=128, n=200, m=200, p=50, row_normalize=False)


def varlen_dims(seed: int, count: int, n_lo: int = 8, n_hi: int = 256):
    """Uneven batch: n ~ U{n_lo..n_hi}, m = 2n, p ~ U{0..n//4}."""
    rng = np.random.default_rng([seed, 0x7A11])
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ps = np.array([rng.integers(0, n // 4 + 1) for n in ns])
    return [(int(n), int(2 * n), int(pp)) for n, pp in zip(ns, ps)]


def serving_dims(seed: int, count: int, n_lo: int = 16, n_hi: int = 512):
    """Serving stream: n log-uniform in [n_lo, n_hi], m ~ U{n..2n}, p ~ U{0..n//8},
    half of the requests also ask for a backward pass."""
    rng = np.random.default_rng([seed, 0x5E12])
    out = []
    for _ in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        n = max(n_lo, min(n, n_hi))
        m = int(rng.integers(n, 2 * n + 1))
        p = int(rng.integers(0, n // 8 + 1))
        out.append((n, m, p, bool(rng.uniform() < 0.5)))
    return out


def make_varlen(seed: int, dims, row_normalize: bool = False, dtype=np.float64):
    """One problem per entry of `dims` ((n, m, p) tuples); problem i uses
    default_rng([seed, i]).  Returns a list of dicts."""
    out = []
    for i, d in enumerate(dims):
        n, m, p = d[:3]
        Q, q, A, b, G, h, g = one_problem(np.random.default_rng([seed, i]), n, m, p, row_normalize)
        out.append({k: np.ascontiguousarray(v.astype(dtype)) for k, v in
                    zip(("Q", "q", "A", "b", "G", "h", "g"), (Q, q, A, b, G, h, g))})
    return out
