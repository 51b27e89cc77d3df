"""Fixed workload for rocprofv3 runs.

First a plain device copy of a known size (torch ``copy_`` of 1 GiB; its
FETCH_SIZE / WRITE_SIZE calibrate the counters to bytes), then ``--solves``
solves of one workload through libcsp on the current stream.

    rocprofv3 --kernel-trace --stats -d OUT -o run -- \
        python paper_1511_06441_amd/profile_run.py --workload cube128 --solves 3
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cube128",
                    choices=["cube128", "cube128set", "cube256", "cube256stress", "square64"])
    ap.add_argument("--M", type=int, default=700)
    ap.add_argument("--solves", type=int, default=3)
    ap.add_argument("--dense", type=int, default=-1,
                    help="dense threshold of the improved set (-1 automatic, 0 always, 4294967295 never)")
    ap.add_argument("--phases", action="store_true", help="also print the per-phase time of each solve")
    args = ap.parse_args()

    import torch
    from paper_1511_06441_amd import csp
    from paper_1511_06441_amd import inputs as gen

    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy {COPY_BYTES} bytes done", flush=True)
    del a, b

    insts = {"cube128": lambda: [gen.cube128(11, args.M)],
             "cube128set": lambda: [gen.cube128(11, M) for M in (400, 700, 1000)],
             "cube256": lambda: [gen.cube256(21)],
             "cube256stress": lambda: [gen.cube256_stress(22)],
             "square64": lambda: [gen.square64(1)]}[args.workload]()
    s = csp.Solver(0)
    csp.csp_set_dense_threshold(s.ctx, args.dense)
    if args.phases:
        csp.csp_set_phase_timing(s.ctx, 2)
    for inst in insts:
        di = csp.to_device(inst)
        for i in range(args.solves):
            res, cnt = s.solve(di)
            print(f"{inst.name} solve {i}: {res.tuple()} C={cnt.C} R={cnt.R} "
                  f"kernel_ms={csp.csp_last_kernel_ms(s.ctx):.3f}", flush=True)
            if args.phases:
                sp = csp.csp_last_phase_spread(s.ctx)
                C = max(cnt.C, 1)
                print("  phases, us per cycle (mean over workgroups / largest workgroup): " +
                      " ".join(f"{k}={a / C:.2f}/{b / C:.2f}" for k, (a, b) in sp.items()), flush=True)
    s.close()


if __name__ == "__main__":
    main()
