#!/usr/bin/env python
"""Throughput of the water-flow constrained-shortest-path cycle on one MI355X.

One step = the whole hot path (input checks, the persistent cycle kernel,
result read-back) for every solve of one workload, with inputs already
resident in HBM.  Default workload: the 128^3 cube (d=3, f1, f2 i.i.d.
uniform on 1..10 from seed 11, A = face x=0, B = face x=127) solved for
M = 400, 700 and 1000, i.e. three solves per step.

Prints ONE JSON line.  ``value`` is active-edge relaxations per second
(flows delivered, summed over the step's solves, divided by wall time);
solves/s, the HBM roofline of the cycle kernel and the CPU oracle's rate on
a bounded sample ride along.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
LABEL_BYTES = 4                # label words are uint32
FLOW_BYTES = 8                 # (destination, quality|direction)

WORKLOADS = {
    "cube128": dict(desc="d=3 n=128 (2,097,152 vertices, 6,242,304 edges), f1,f2 iid U{1..10} "
                         "splitmix64 seed 11, A=face x=0, B=face x=127, M in {400,700,1000}",
                    build=lambda gen: [gen.cube128(11, M) for M in (400, 700, 1000)],
                    sample_index=2),
    "cube256": dict(desc="d=3 n=256 (16,777,216 vertices, 50,135,040 edges), f1,f2 iid U{1..100} "
                         "seed 21, A=face x=0, B=face x=255, M=10000",
                    build=lambda gen: [gen.cube256(21)], sample_index=None),
    "cube256stress": dict(desc="d=3 n=256, f1=1, f2 iid U{1..3} seed 22, faces x=0 -> x=255, M=10000",
                          build=lambda gen: [gen.cube256_stress(22)], sample_index=None),
    "square64": dict(desc="d=2 n=64, f1,f2 iid U{1..5} seed 1, columns x=0 -> x=63, M=200",
                     build=lambda gen: [gen.square64(1)], sample_index=0),
}


def algorithmic_bytes(N, c):
    """Bytes the method must move for one solve (label init, own label per
    improvement, f1+f2+neighbour label per test, one flow record written per
    send, one flow record read plus a label read-modify-write per delivery)."""
    L = LABEL_BYTES
    return (N * L + c["U"] * L + c["D"] * (2 + L) + c["E"] * FLOW_BYTES
            + c["R"] * (FLOW_BYTES + 2 * L))


def cpu_baseline(inst):
    from oracle import oracle as O
    t0 = time.perf_counter()
    r = O.solve_instance(inst, want_labels=False)
    dt = time.perf_counter() - t0
    return dict(value=r.counters["R"] / dt, unit="relaxations/s", cores=1, kind="oracle",
                sample=f"one solve of {inst.name} (single-threaded C oracle, -O2), "
                       f"{dt:.1f} s, R={r.counters['R']}",
                seconds=round(dt, 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the path does not shard "
              "across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_06441_amd import csp
    from paper_1511_06441_amd import inputs as gen

    wl = WORKLOADS[args.workload]
    insts = wl["build"](gen)
    dev = [csp.to_device(i) for i in insts]
    solver = csp.Solver(0)
    stream = torch.cuda.current_stream()

    def step():
        out = []
        for di in dev:
            res, cnt = solver.solve(di, stream=stream)
            out.append((res, cnt, csp.csp_last_kernel_ms(solver.ctx)))
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for _ in range(args.steps):
        runs.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    R_step = sum(c.R for _, c, _ in runs[0])
    solves = len(dev) * args.steps
    bytes_step = sum(algorithmic_bytes(i.N, c.asdict()) for i, (_, c, _) in zip(insts, runs[0]))
    kern_ms = [ms for st in runs for (_, _, ms) in st]
    kern_ms_step = sum(kern_ms) / args.steps
    achieved = bytes_step / (kern_ms_step * 1e-3) / 1e9
    line = {
        "metric": "active-edge relaxations/s",
        "value": R_step * args.steps / wall,
        "unit": "relaxations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded splitmix64 lattices)",
        "config": {"workload": args.workload, "desc": wl["desc"], "solves_per_step": len(dev),
                   "parallelism": "single GPU"},
        "solves_per_s": solves / wall,
        "results": [dict(T=r.T, X=r.X, x=r.x, Y=r.Y, F2=r.F2, **c.asdict()) for r, c, _ in runs[0]],
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_solve<{insts[0].d}>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel_ms_avg": sum(kern_ms) / len(kern_ms),
            "algorithmic_bytes_per_step": bytes_step,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline and wl["sample_index"] is not None:
        line["cpu_baseline"] = cpu_baseline(insts[wl["sample_index"]])
    print(json.dumps(line), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
