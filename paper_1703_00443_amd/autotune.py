"""Project-written autotuner: which forward kernel variant each size bucket uses.

A bucket is (dtype, whether the problem has equality rows, the class of
nineq / nz, nz range).  For each bucket the tuner draws a set of problems from
the seeded generator, times forward + backward of every candidate variant
(register-resident MFMA tiles where they apply, streamed MFMA tiles,
LDS-resident generic, global-memory generic, and the paper's elimination order
of Section 3.1.1 where nineq fits it) as one uneven launch and keeps the
fastest one whose results are all usable (no more problems short of OPTIMAL
than under the automatic plan).  The table is a JSON file; the
variant of a problem depends only on its own dims, so results do not depend on
what else shares a launch.  Entries without a ratio class (key "eq" / "noeq")
serve every class that has no entry of its own.

    python -m paper_1703_00443_amd.autotune --dtype f32 --out paper_1703_00443_amd/autotune_table.json
"""
from __future__ import annotations

import argparse
import json
import os
import time
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "autotune_table.json")

BUCKETS = [(1, 16), (17, 32), (33, 64), (65, 96), (97, 128), (129, 192), (193, 256), (257, 384),
           (385, 512), (513, 1024)]
VARIANT_NAMES = {0: "auto", 1: "generic", 2: "lds", 3: "tiled", 4: "stream", 5: "elim"}
# classes of nineq / nz: the elimination order factors an nineq x nineq matrix
# per Newton step, the other variants an nz x nz one
RATIOS = [("r0", 0.25), ("r1", 0.5), ("r2", 1.0), ("r3", None)]


def ratio_of(n: int, m: int) -> str:
    for name, hi in RATIOS:
        if hi is None or m <= hi * n:
            return name
    return RATIOS[-1][0]


def bucket_of(n: int) -> int:
    for i, (lo, hi) in enumerate(BUCKETS):
        if lo <= n <= hi:
            return i
    return len(BUCKETS) - 1


def _dkey(dtype) -> str:
    import torch
    return "f64" if dtype in (torch.float64, "f64", np.float64) else "f32"


class AutotuneTable:
    def __init__(self, data: Optional[Dict] = None):
        self.data = data or {}

    def variant_for(self, dtype, n: int, m: int, p: int) -> int:
        dd = self.data.get(_dkey(dtype), {})
        eq = "eq" if p > 0 else "noeq"
        b = str(bucket_of(n))
        for key in (eq + "/" + ratio_of(n, m), eq):
            if b in dd.get(key, {}):
                return int(dd[key][b])
        return 0

    @classmethod
    def load(cls, path: str = DEFAULT_TABLE) -> "AutotuneTable":
        if not os.path.exists(path):
            return cls()
        with open(path) as f:
            return cls(json.load(f))

    def save(self, path: str = DEFAULT_TABLE):
        with open(path, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)


def candidates(n: int, dtype: str, m: int = None):
    """Variants that apply to problems of up to n variables (and m inequality
    rows): generic, LDS, streamed tiles, the register-resident tiles (n <= 128;
    FP32 n <= 256), and the elimination order (m <= 128 and m <= n rounded up
    to 16; whether its LDS regions fit is the plan's to say)."""
    c = [1, 2, 4]
    if n <= 128 or (dtype == "f32" and n <= 256):
        c.append(3)
    if m is not None and m <= 128 and m <= (n + 15) // 16 * 16:
        c.append(5)
    return c


def tune(dtype="f32", samples: int = 24, seed: int = 7, reps: int = 3, buckets=None,
         table: Optional[AutotuneTable] = None, log=print, ratios=("r3",)) -> AutotuneTable:
    """Tune the given nz buckets for the given nineq / nz classes (r3, the
    default, is nineq = 2 nz as in the uneven workload)."""
    import torch
    from . import synth
    from .varlen import VarlenBatch

    tdt = torch.float64 if dtype == "f64" else torch.float32
    table = table or AutotuneTable()
    dk = _dkey(tdt)
    table.data.setdefault(dk, {})
    rng = np.random.default_rng(seed)
    frac = {"r0": (0.1, 0.25), "r1": (0.26, 0.5), "r2": (0.51, 1.0), "r3": (2.0, 2.0)}
    for bi, eq, rc in ((bi, eq, rc) for bi in (buckets if buckets is not None else range(len(BUCKETS)))
                       for eq in ("noeq", "eq") for rc in ratios):
            lo, hi = BUCKETS[bi]
            dims = []
            for _ in range(samples):
                n = int(rng.integers(lo, hi + 1))
                p = 0 if eq == "noeq" else int(rng.integers(1, max(1, n // 4) + 1)) if n > 1 else 0
                if eq == "eq" and p == 0:
                    continue
                m = max(1, int(round(n * rng.uniform(*frac[rc]))))
                dims.append((n, m, p))
            if not dims:
                continue
            probs = synth.make_varlen(seed * 1000 + bi, dims)
            g = [pr["g"] for pr in probs]
            best = None
            key = eq if rc == "r3" else eq + "/" + rc
            cands = candidates(max(d[0] for d in dims), dk)
            from . import binding as qb
            if all(5 in candidates(d[0], dk, d[1]) and qb.plan(tdt, d[0], d[1], d[2], 5)[0] == 5
                   for d in dims):
                cands = cands + [5]
            base_not_optimal = None
            for v in [0] + cands:
                vb = VarlenBatch(probs, dtype=tdt, variants=[v] * len(probs))
                dl = vb.pack_vectors(g)
                vb.forward(); vb.backward(dl)
                torch.cuda.synchronize()
                st = vb.status[:vb.count].cpu().numpy()
                if v == 0:
                    # the automatic plan's outcome: no candidate may end fewer problems OPTIMAL
                    base_not_optimal = int(np.sum(st != 0))
                    continue
                if not np.all((st == 0) | (st == 1) | (st == 4)) or int(np.sum(st != 0)) > base_not_optimal:
                    log("bucket %s %s variant %s: statuses %s" % (BUCKETS[bi], key, VARIANT_NAMES[v],
                                                                 np.bincount(st, minlength=5)))
                    continue
                ts = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    vb.forward(); vb.backward(dl)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                t = float(np.median(ts))
                log("bucket %-10s %-9s variant %-7s %8.3f ms" % (BUCKETS[bi], key, VARIANT_NAMES[v], t * 1e3))
                if best is None or t < best[1]:
                    best = (v, t)
            if best is not None:
                table.data[dk].setdefault(key, {})[str(bi)] = best[0]
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtype", choices=("f32", "f64"), default="f32")
    ap.add_argument("--samples", type=int, default=24)
    ap.add_argument("--max-bucket", type=int, default=len(BUCKETS) - 1)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--ratios", default="r3", help="nineq / nz classes to tune (r0,r1,r2,r3)")
    args = ap.parse_args()
    table = AutotuneTable.load(args.out)
    table = tune(args.dtype, samples=args.samples, buckets=range(args.max_bucket + 1), table=table,
                 ratios=tuple(args.ratios.split(",")))
    table.save(args.out)
    print(json.dumps(table.data))


if __name__ == "__main__":
    main()
