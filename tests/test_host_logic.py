"""Host-side logic with no GPU: the seeded generators, the autotune table
lookup, the uneven-batch cost model, and the bench's algorithmic counts."""
import json
import os

import numpy as np

from paper_1703_00443_amd import synth
from paper_1703_00443_amd.autotune import BUCKETS, AutotuneTable, bucket_of, candidates, ratio_of


def test_problem_regenerates_alone():
    """Problem i of a batch is drawn from its own stream [seed, i], so it is the
    same alone and inside any batch (what the alone-vs-mix tests rely on)."""
    b = synth.make_batch(seed=321, B=5, n=7, m=9, p=2)
    one = synth.one_problem(np.random.default_rng([321, 3]), 7, 9, 2)
    for k, v in zip(("Q", "q", "A", "b", "G", "h", "g"), one):
        np.testing.assert_array_equal(getattr(b, k)[3], v)


def test_generator_is_feasible_and_convex():
    """h = G z0 + s0 with s0 > 0 and b = A z0: z0 is strictly feasible; Q is
    symmetric positive definite (smallest eigenvalue at least 1e-3)."""
    rng = np.random.default_rng([11, 0])
    Q, q, A, b, G, h, g = synth.one_problem(rng, 12, 30, 3, row_normalize=True)
    np.testing.assert_allclose(Q, Q.T)
    assert np.linalg.eigvalsh(Q).min() >= 1e-3 - 1e-12
    np.testing.assert_allclose(np.linalg.norm(G, axis=1), 1.0)
    rng = np.random.default_rng([11, 0])
    L = rng.standard_normal((12, 12)); rng.standard_normal(12); rng.standard_normal((30, 12))
    rng.standard_normal((3, 12)); z0 = rng.standard_normal(12)
    assert np.all(h - G @ z0 > 0)
    np.testing.assert_allclose(A @ z0, b)


def test_workload_shapes():
    dims = synth.varlen_dims(4096, 300)
    assert all(8 <= n <= 256 and m == 2 * n and 0 <= p <= n // 4 for n, m, p in dims)
    sd = synth.serving_dims(4, 300)
    assert all(16 <= n <= 512 and n <= m <= 2 * n and 0 <= p <= n // 8 for n, m, p, _ in sd)
    frac_bwd = np.mean([d[3] for d in sd])
    assert 0.35 < frac_bwd < 0.65


def test_autotune_buckets_and_lookup(tmp_path):
    assert bucket_of(1) == 0 and bucket_of(16) == 0 and bucket_of(17) == 1
    assert bucket_of(BUCKETS[-1][1]) == len(BUCKETS) - 1
    for i, (lo, hi) in enumerate(BUCKETS):
        assert bucket_of(lo) == i and bucket_of(hi) == i
    t = AutotuneTable({"f32": {"noeq": {"4": 3}, "eq": {"4": 4}}})
    assert t.variant_for("f32", 100, 200, 0) == 3
    assert t.variant_for("f32", 100, 200, 7) == 4
    assert t.variant_for("f64", 100, 200, 0) == 0       # no entry: automatic plan
    path = os.path.join(str(tmp_path), "t.json")
    t.save(path)
    assert AutotuneTable.load(path).data == json.load(open(path))
    # candidate variants: register tiles only within their size limits
    assert 3 in candidates(128, "f64") and 3 not in candidates(129, "f64")
    assert 3 in candidates(256, "f32") and 3 not in candidates(257, "f32")
    assert 4 in candidates(1000, "f64")
    # the elimination order: nz <= 128 and nineq <= nz rounded up to 16
    assert 5 in candidates(100, "f64", 25) and 5 in candidates(100, "f32", 112)
    assert 5 not in candidates(100, "f64", 113) and 5 in candidates(300, "f32", 30)
    assert 5 not in candidates(300, "f64", 129)
    assert 5 not in candidates(100, "f64")               # nineq not given
    # ratio classes: an entry of the class wins, else the class-less entry
    assert [ratio_of(100, m) for m in (25, 26, 50, 51, 100, 101)] == ["r0", "r1", "r1", "r2", "r2", "r3"]
    t = AutotuneTable({"f64": {"noeq": {"4": 3}, "noeq/r0": {"4": 5}}})
    assert t.variant_for("f64", 100, 20, 0) == 5
    assert t.variant_for("f64", 100, 60, 0) == 3
    assert t.variant_for("f64", 100, 20, 3) == 0


def test_committed_table_is_valid():
    """Keys are eq/noeq, optionally with a nineq/nz class; the elimination order
    (5) appears only in the classes with nineq <= nz."""
    t = AutotuneTable.load()
    classes = ("r0", "r1", "r2")
    for dk, per in t.data.items():
        assert dk in ("f32", "f64")
        for key, buckets in per.items():
            eq, _, rc = key.partition("/")
            assert eq in ("eq", "noeq") and rc in ("",) + classes, key
            for b, v in buckets.items():
                assert 0 <= int(b) < len(BUCKETS) and v in (1, 2, 3, 4, 5)
                if v == 5:
                    assert rc in classes, (key, b)


def test_algorithmic_flops_counts():
    """Counts of the bench's roofline at the paper-scale shape, by hand: one
    iterate costs n(n+1)m + n^3/3 (factor) + residual + 2 solves."""
    import bench
    n = m = 100
    fac = n * (n + 1) * m + n ** 3 / 3
    res = 2 * n * n + 4 * n * m
    sol = 4 * n * m + 2 * n * n
    assert abs(bench.algorithmic_flops(n, m, 0, [0]) - (2 * fac + res + sol)) < 1e-6
    assert abs(bench.algorithmic_flops(n, m, 0, [3]) - (5 * fac + 4 * res + 7 * sol)) < 1e-6
    per_iter = fac + res + 2 * sol
    assert abs(per_iter - 1.52e6) / 1.52e6 < 0.01   # 1.52 Mflop per iterate at this shape
    # backward bytes: read Q, G, z, lam, s, dl/dz and the factor (U, D); write
    # dQ, dq, dG, dh  ->  3 n^2 + 2 m n + 3 n + 4 m elements = 50700 at this shape
    assert bench.backward_bytes(n, m, 0, 8) == 8 * 50700


def test_box_batch_structure():
    """Box QPs: G = [I; -I] (rows are signed unit vectors), h = [u; -l] with
    l < 0 < u (z = 0 is strictly feasible), Q symmetric positive definite,
    and each problem regenerates alone."""
    b = synth.box_batch(seed=3, B=4, n=7)
    n, m, p = b.dims
    assert (n, m, p) == (7, 14, 0)
    for i in range(4):
        G = b.G[i]
        assert np.all((G != 0).sum(axis=1) == 1) and np.all(np.abs(G[G != 0]) == 1)
        assert np.array_equal(G[:n], np.eye(n)) and np.array_equal(G[n:], -np.eye(n))
        assert np.all(b.h[i] > 0)
        assert np.allclose(b.Q[i], b.Q[i].T) and np.linalg.eigvalsh(b.Q[i]).min() > 0
    one = synth.box_batch(seed=3, B=2, n=7)
    assert np.array_equal(one.Q[1], b.Q[1]) and np.array_equal(one.h[1], b.h[1])
