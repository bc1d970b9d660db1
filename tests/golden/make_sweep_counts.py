"""Write the oracle's count vectors of the 4096-variant batched sweep
(matmul / stencil / transpose, main domains of 2^16..2^30 points, extents
off the tile multiples) to tests/golden/sweep4096_counts.npz.

Calls only oracle/ (simulated execution, Sec. 3.2 Alg. 1 and Alg. 2) and the
seeded variant generator of synth/; nothing from the HIP library.  Runs on
the CPU for tens of minutes:

    python tests/golden/make_sweep_counts.py [--workers 7] [--mem-gib 40]

Variants run in worker processes, largest first, while the oracle's memory
(a byte per array cell, and 8 bytes per cell of arrays with a strided
access) of the running ones stays under --mem-gib.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "sweep4096_counts.npz")


def variants_digest(vs) -> str:
    """Digest of the variant list, so a reader can tell the file still
    matches the generator."""
    return hashlib.sha256(json.dumps(vs, sort_keys=True).encode()).hexdigest()


def oracle_bytes(v) -> int:
    """Memory the oracle holds for one variant (its arrays' cell maps)."""
    f = v["family"]
    if f == "matmul":
        return v["n"] * v["m"] + v["m"] * v["l"] + v["n"] * v["l"]
    n = v["n"]
    if f == "stencil":
        return (n + 2) ** 2 + n * n
    strided = v["op"] != "tiled"
    return 2 * n * n + (8 * n * n if strided else 0)


def oracle_work(v) -> int:
    f = v["family"]
    if f == "matmul":
        return v["n"] * v["m"] * v["l"]
    return v["n"] * v["n"]


def _count(args):
    i, v = args
    from oracle import count as C
    names = [x for x in C.names() if not x.startswith("foot.")]
    t0 = time.time()
    c = C.count(v)
    return i, [c.get(k, 0) for k in names], time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=7)
    ap.add_argument("--mem-gib", type=float, default=40.0)
    ap.add_argument("--limit", type=int, default=0, help="first N variants only (trial)")
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()

    from oracle import count as C
    from synth import suite_batched
    vs = suite_batched(4096)
    idx = list(range(len(vs)))
    if a.limit:
        idx = idx[:a.limit]
    names = [x for x in C.names() if not x.startswith("foot.")]
    counts = np.zeros((len(vs), len(names)), dtype=np.int64)
    done = np.zeros(len(vs), dtype=bool)
    order = sorted(idx, key=lambda i: -oracle_work(vs[i]))
    cap = int(a.mem_gib * (1 << 30))
    held, running = 0, {}
    t0 = time.time()
    secs = 0.0
    with cf.ProcessPoolExecutor(max_workers=a.workers) as ex:
        pending = list(order)
        while pending or running:
            while pending and len(running) < a.workers:
                i = pending[0]
                need = oracle_bytes(vs[i])
                if running and held + need > cap:
                    break
                pending.pop(0)
                held += need
                running[ex.submit(_count, (i, vs[i]))] = need
            fin, _ = cf.wait(list(running), return_when=cf.FIRST_COMPLETED)
            for fu in fin:
                held -= running.pop(fu)
                i, row, dt = fu.result()
                counts[i] = row
                done[i] = True
                secs += dt
                k = int(done.sum())
                if k % 64 == 0 or k == len(idx):
                    print("%d/%d variants, %.0f s wall, %.0f s oracle" %
                          (k, len(idx), time.time() - t0, secs), flush=True)
    np.savez_compressed(a.out, names=np.array(names), counts=counts, done=done,
                        digest=np.array(variants_digest(vs)),
                        oracle_seconds=np.array(secs))
    print("wrote", a.out)


if __name__ == "__main__":
    main()
