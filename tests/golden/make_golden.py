"""Write the oracle's expected outputs for the large lattice workloads.

Calls only the CPU oracle (oracle/) and the seeded input generator; nothing
here touches the HIP library.  Each case is stored as JSON with T, X, x, Y,
F2, the counters and the SHA-256 of the final labels (uint32, little
endian).

Two cases hold many problems and run the oracle in parallel host
processes: ``batch1024`` (the 1,024 problems of the mixed batch, master seed
41) and ``serve8`` (the first 8 serving requests of master seed 51, each with
its path recovered by repeated solves, section 1 and section 5
"Termination"); where a request's whole chain would take hours on the host
only its first solves are stored, and ``serve8_pathK`` stores request K's
whole chain on its own.

    python tests/golden/make_golden.py [name ...] [--workers=K]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_1511_06441_amd import inputs as gen      # noqa: E402


def cases():
    out = {}
    for s in (1, 2, 3):
        out[f"square64_s{s}"] = lambda s=s: gen.square64(s)
    for s in (11, 12, 13):
        for M in (400, 700, 1000):
            out[f"cube128_s{s}_M{M}"] = lambda s=s, M=M: gen.cube128(s, M)
    out["cube256_s21"] = lambda: gen.cube256(21)
    out["cube256stress_s22"] = lambda: gen.cube256_stress(22)
    # the paper's own shape (section 8): water on the cube boundary, B the centre
    for n in (50, 75, 100, 125):
        out[f"paper{n}_s61"] = lambda n=n: gen.cube_boundary_to_center(n, 61, K=100, M=10000)
    return out


def labels_sha256(labels) -> str:
    return hashlib.sha256(labels.astype("<u4").tobytes()).hexdigest()


def make(name, builder):
    inst = builder()
    t0 = time.time()
    r = O.solve_instance(inst)
    dt = time.time() - t0
    rec = dict(name=name, d=inst.d, n=inst.n, M=inst.M, meta=inst.meta,
               T=r.T, X=r.X, x=r.x, Y=r.Y, F2=r.F2, counters=r.counters,
               labels_sha256=labels_sha256(r.labels), oracle_seconds=round(dt, 2))
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(name, r.tuple(), r.counters, f"{dt:.1f}s", flush=True)


def _batch_one(j):
    inst = gen.mixed_instance(41, j)
    t0 = time.time()
    r = O.solve_instance(inst)
    dt = time.time() - t0
    return dict(j=j, d=inst.d, n=inst.n, K=inst.meta["K"], M=inst.M, seed=inst.meta["seed"],
                T=r.T, X=r.X, x=r.x, Y=r.Y, F2=r.F2, counters=r.counters,
                labels_sha256=labels_sha256(r.labels), oracle_seconds=round(dt, 2))


# Above this many vertices the whole repeated-solve chain would keep one host
# core busy for hours (the 1016^2 request: about 68 s per solve and some
# 1,500 solves), so only its first SERVE_PREFIX_STEPS solves are stored; the
# stored rows are a prefix of the whole chain (the chain does not depend on
# where it stops).
SERVE_FULL_PATH_MAX_VERTICES = 300_000
SERVE_PREFIX_STEPS = 24


def _serve_one(k, full=False):
    inst = gen.mixed_instance(51, k, (64, 1024), (32, 256))
    t0 = time.time()
    r = O.solve_instance(inst)
    if full or inst.N <= SERVE_FULL_PATH_MAX_VERTICES:
        path, rp, steps = O.reconstruct(inst.d, inst.n, inst.f1, inst.f2, inst.A, inst.B, inst.M)
        complete = True
    else:
        path, rp, steps, complete = O.reconstruct_upto(inst.d, inst.n, inst.f1, inst.f2, inst.A,
                                                       inst.B, inst.M, SERVE_PREFIX_STEPS)
    dt = time.time() - t0
    assert rp.tuple() == r.tuple()
    return dict(k=k, d=inst.d, n=inst.n, K=inst.meta["K"], M=inst.M, seed=inst.meta["seed"],
                T=r.T, X=r.X, x=r.x, Y=r.Y, F2=r.F2, counters=r.counters,
                labels_sha256=labels_sha256(r.labels), path_complete=bool(complete),
                path=[int(v) for v in path],
                resolves=[[int(v) for v in row] for row in steps], oracle_seconds=round(dt, 2))


def serve8_whole_path(k):
    """The whole chain of one serving request, stored on its own."""
    t0 = time.time()
    rec = _serve_one(k, full=True)
    with open(os.path.join(HERE, f"serve8_s51_path{k}.json"), "w") as fh:
        json.dump(rec, fh, indent=0)
    print(f"serve8_s51_path{k}: {len(rec['path'])} vertices, {time.time() - t0:.0f} s", flush=True)


def make_many(name, fn, items, workers, desc):
    """Run fn over items in `workers` host processes, largest first, and store
    the records in input order."""
    import multiprocessing as mp
    t0 = time.time()
    out = {}
    with mp.get_context("fork").Pool(workers) as pool:
        for rec in pool.imap_unordered(fn, items):
            key = rec.get("j", rec.get("k"))
            out[key] = rec
            print(f"{name}: {len(out)}/{len(items)} (item {key}, {rec['oracle_seconds']} s, "
                  f"{time.time() - t0:.0f} s elapsed)", flush=True)
    recs = [out[k] for k in sorted(out)]
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(dict(name=name, desc=desc, problems=recs,
                       oracle_seconds=round(sum(r["oracle_seconds"] for r in recs), 2)), fh, indent=0)


def batch1024(workers):
    ps = gen.batch_params(1024, 41)
    order = sorted(range(1024), key=lambda j: -(ps[j][2] ** ps[j][1]) * ps[j][4])
    make_many("batch1024_s41", _batch_one, order, workers,
              "the 1,024 problems of the mixed batch (master seed 41), oracle solves with labels")


def serve8(workers):
    ps = gen.serving_params(8, 51)
    order = sorted(range(8), key=lambda k: -(ps[k][2] ** ps[k][1]) * ps[k][4])
    make_many("serve8_s51", _serve_one, order, workers,
              "the first 8 serving requests (master seed 51): solve and path by repeated solves")


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("--workers")]
    workers = 7
    for a in sys.argv[1:]:
        if a.startswith("--workers="):
            workers = int(a.split("=", 1)[1])
    all_cases = cases()
    names = args or list(all_cases)
    for nm in names:
        if nm == "batch1024":
            batch1024(workers)
        elif nm == "serve8":
            serve8(workers)
        elif nm.startswith("serve8_path"):
            serve8_whole_path(int(nm[len("serve8_path"):]))
        else:
            make(nm, all_cases[nm])
