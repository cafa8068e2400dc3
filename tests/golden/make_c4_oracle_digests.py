"""Writes c4_oracle_digests.json: the CPU oracle's RREF(M) of a seeded subset
of the 256-matrix batch workload (rows log-uniform in [500, 20,000] over
F_65521), as SHA-256 digests of its canonical CSR arrays.

The subset is the smallest and the largest matrix of the batch plus six
drawn with a fixed seed.  Only the seeded input generator (flgen) and the
oracle are called; the largest matrix takes several minutes of CPU time,
which is why the GPU test compares against these stored digests instead of
running the oracle itself.

    python tests/golden/make_c4_oracle_digests.py [threads]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import flgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "c4_oracle_digests.json")
SUBSET_SEED = 404
EXTRA = 6


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    cfg = flgen.BATCH_CONFIGS["c4"]
    # sizes of every member, from the same draws the generator makes first
    rows = []
    seed = flgen.BASE_SEED + 4
    for i in range(cfg["count"]):
        rng = np.random.default_rng(seed ^ (i << 32))
        rows.append(int(round(np.exp(rng.uniform(np.log(cfg["m_lo"]), np.log(cfg["m_hi"]))))))
    rows = np.array(rows)
    small, large = int(np.argmin(rows)), int(np.argmax(rows))
    rest = [i for i in range(cfg["count"]) if i not in (small, large)]
    pick = np.random.default_rng(SUBSET_SEED).choice(rest, EXTRA, replace=False)
    subset = sorted({small, large, *map(int, pick)})
    out = {"workload": "c4: 256 matrices over F_65521, rows log-uniform in [500, 20000]",
           "generator_seed": seed, "smallest": small, "largest": large, "matrices": {}}
    for i in subset:
        t0 = time.perf_counter()
        g = flgen.config_batch_member("c4", i)
        r = oracle.fl_rref(g, keep=False, threads=threads)
        rp, ci, v = r["rref"]
        out["matrices"][str(i)] = dict(m=g["m"], n=g["n"], nnz_in=int(len(g["col"])), rank=int(r["rank"]),
                                       nnz=int(rp[-1]), row_ptr_sha256=digest(rp.astype(np.uint64)),
                                       col_sha256=digest(ci.astype(np.uint32)),
                                       val_sha256=digest(v.astype(np.uint16)))
        print(f"matrix {i}: {g['m']}x{g['n']} rank {r['rank']} in {time.perf_counter() - t0:.1f}s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
