#!/usr/bin/env python
"""Throughput of the water-flow constrained-shortest-path cycle on one MI355X.

One step = the whole hot path (input checks, the persistent cycle kernel,
result read-back) for every solve of one workload, with inputs already
resident in HBM.  Default workload: the 256^3 cube (d=3, f1, f2 i.i.d.
uniform on 1..100 from seed 21, A = face x=0, B = face x=255, M = 10000),
one solve per step.  The 128^3 cube (three solves, M = 400, 700, 1000) and
the other workloads are options.

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
FLOW_BYTES = 8                 # (destination, quality|direction)

WORKLOADS = {
    "cube128": dict(desc="d=3 n=128 (2,097,152 vertices, 6,242,304 edges), f1,f2 iid U{1..10} "
                         "splitmix64 seed 11, A=face x=0, B=face x=127, M in {400,700,1000}",
                    build=lambda gen: [gen.cube128(11, M) for M in (400, 700, 1000)],
                    sample_index=2, label_bytes=2),
    "cube256": dict(desc="d=3 n=256 (16,777,216 vertices, 50,135,040 edges), f1,f2 iid U{1..100} "
                         "seed 21, A=face x=0, B=face x=255, M=10000",
                    build=lambda gen: [gen.cube256(21)], sample_index=0, sample_cycles=(300, 900),
                    label_bytes=4),
    "cube256stress": dict(desc="d=3 n=256, f1=1, f2 iid U{1..3} seed 22, faces x=0 -> x=255, M=10000",
                          build=lambda gen: [gen.cube256_stress(22)], sample_index=0, sample_cycles=(60, 180),
                          label_bytes=4),
    "square64": dict(desc="d=2 n=64, f1,f2 iid U{1..5} seed 1, columns x=0 -> x=63, M=200",
                     build=lambda gen: [gen.square64(1)], sample_index=0, label_bytes=2),
    "env7": dict(desc="the environments of section 7 on [-1024,1024] x [0,2048] (2049^2 vertices, passage times "
                      "in {1,2}, f2=f1, M above every path weight, water from the x-axis): Lemma 1's (the y-axis "
                      "fast), Theorem 2's construction at t=1024, and the random one with p=1/2 (seed 71)",
                 build=lambda gen: [gen.lemma1_environment(1024), gen.fractal_environment(10),
                                    gen.binary_environment(1024, 0.5, 71)],
                 sample_index=None, label_bytes=4),
    "paper_cubes": dict(desc="the paper's runs (section 8): d=3 cubes n=50,75,100,125, water on the cube "
                             "boundary, B the centre vertex, f1,f2 iid U{1..100} seed 61, M=10000",
                        build=lambda gen: [gen.cube_boundary_to_center(n, 61, K=100, M=10000)
                                           for n in (50, 75, 100, 125)],
                        sample_index=3, label_bytes=4),
}

BATCH_DESC = ("1,024 independent problems (master seed 41): d in {2,3}, side log-uniform in [32,512] (d=2) / "
              "[16,160] (d=3), f1,f2 iid U{1..K} with K in 3..50 per problem, A/B = faces x=0 / x=n-1, "
              "M = round((1.5..4) n (K+1)/2); 306,237,961 vertices in all")


def mixed_on_device(gen, csp, master, count, lo2=(32, 512), lo3=(16, 160)):
    """Problems of the mixed batch, drawn on the GPU with the seeded generator."""
    out = []
    for j in range(count):
        s, d, n, K, M = gen.mixed_params(master, j, lo2, lo3)
        f1, f2 = gen.lattice_edges_torch(d, n, s, K, K, device="cuda")
        A = gen.face_mask_torch(d, n, 0, 0, "cuda")
        B = gen.face_mask_torch(d, n, 0, n - 1, "cuda")
        out.append(csp.DeviceInstance(d, n, f1, f2, A, B, M))
    return out


def run_batch(args):
    import torch
    from paper_1511_06441_amd import csp
    from paper_1511_06441_amd import inputs as gen

    count = args.batch_count
    dev = mixed_on_device(gen, csp, 41, count)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # cold: the first batch on a fresh context (every problem starts from the
    # default wheel size; those that overflow run again in a later round)
    solver = csp.Solver(0)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    csp.csp_solve_batch(solver.ctx, dev, stream=stream)
    torch.cuda.synchronize()
    cold = time.perf_counter() - tc
    tuned = None
    if args.autotune:
        tgt, tms = csp.csp_autotune_batch(solver.ctx, dev, stream=stream)
        tuned = {"vertices_per_workgroup": tgt, "kernel_ms": round(tms, 3)}
    for _ in range(args.warmup):
        csp.csp_solve_batch(solver.ctx, dev, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = []
    res = cnt = None
    for _ in range(args.steps):
        res, cnt = csp.csp_solve_batch(solver.ctx, dev, stream=stream)
        kern.append(csp.csp_last_kernel_ms(solver.ctx))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    R = sum(c.R for c in cnt)
    bytes_step = sum(algorithmic_bytes(di.N, c.asdict()) for di, c in zip(dev, cnt))
    kms = sum(kern) / len(kern)
    achieved = bytes_step / (kms * 1e-3) / 1e9
    line = {
        "metric": "active-edge relaxations/s",
        "value": R * args.steps / wall,
        "unit": "relaxations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded splitmix64 lattices, drawn on the GPU)",
        "config": {"workload": "batch%d" % count, "desc": BATCH_DESC if count == 1024 else "first %d problems" % count,
                   "solves_per_step": count, "parallelism": "single GPU"},
        "solves_per_s": count * args.steps / wall,
        "cold": {"seconds": cold, "solves_per_s": count / cold,
                 "note": "first batch on a fresh context; the timed steps reuse the wheel sizes it grew to"},
        "roofline": {"bound": "hbm", "kernel": "k_batch<2>, k_batch<3>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel_ms_avg": kms, "algorithmic_bytes_per_step": bytes_step},
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_batch(),
    }
    if tuned:
        line["autotune"] = tuned
    if args.plain:
        # the same problems as sequential single-problem launches
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        same = True
        for di, r in zip(dev, res):
            rp, _ = solver.solve(di, stream=stream)
            same = same and rp.tuple() == r.tuple()
        torch.cuda.synchronize()
        pw = time.perf_counter() - t1
        line["plain"] = {"solves_per_s": count / pw, "seconds": pw, "results_equal": same,
                         "batched_speedup": (count * args.steps / wall) / (count / pw),
                         "batched_speedup_cold": (count / cold) / (count / pw)}
    print(json.dumps(line), flush=True)
    solver.close()


SERVE_DESC = ("Poisson arrivals (seed 52) of requests from master seed 51: d in {2,3}, sides log-uniform "
              "64..1024 (2-D) / 32..256 (3-D), f1,f2 iid U{1..K}, K in 3..50, faces x=0 -> x=n-1, "
              "M = round((1.5..4) n (K+1)/2); each request is a solve plus the full path reconstruction "
              "by repeated solves")


def run_serve(args):
    import numpy as np
    import torch
    from paper_1511_06441_amd import csp, serving
    from paper_1511_06441_amd import inputs as gen

    count = args.serve_count
    params = gen.serving_params(count, 51)
    dev = []
    for (s, d, n, K, M) in params:
        f1, f2 = gen.lattice_edges_torch(d, n, s, K, K, device="cuda")
        dev.append(csp.DeviceInstance(d, n, f1, f2, gen.face_mask_torch(d, n, 0, 0, "cuda"),
                                      gen.face_mask_torch(d, n, 0, n - 1, "cuda"), M))
    torch.cuda.synchronize()
    print(f"# serve: {count} requests, {sum(x.N for x in dev)} vertices in all", file=sys.stderr, flush=True)
    solver = csp.Solver(0)
    server = csp.Server(solver, arena_bytes=args.serve_arena_gb << 30, max_jobs=256)
    # warm-up: the smallest request
    small = min(range(count), key=lambda k: dev[k].N)
    serving.replay(server, [dev[small]])

    def report(done, submitted, secs):
        print(f"#   {done}/{submitted} done after {secs:.0f} s", file=sys.stderr, flush=True)

    sat = serving.replay(server, dev, progress=report)
    sat_rps = count / sat.makespan
    solves = sum(c.solves for c in sat.completions.values())
    R = sum(c.counters["R"] + c.chain_counters["R"] for c in sat.completions.values())
    print(f"# saturation: {sat_rps:.3f} requests/s over {sat.makespan:.2f} s", file=sys.stderr, flush=True)
    sweep = []
    for frac in args.serve_fracs:
        arr = gen.poisson_arrivals(count, frac * sat_rps, 52)
        tr = serving.replay(server, dev, arr, progress=report)
        same = all(tr.completions[k].res == sat.completions[k].res and
                   tr.completions[k].path == sat.completions[k].path for k in range(count))
        sweep.append({"qps": frac * sat_rps, "fraction_of_saturation": frac,
                      "p50_s": tr.percentile(50), "p99_s": tr.percentile(99),
                      "mean_s": float(tr.latency.mean()), "makespan_s": tr.makespan,
                      "requests_per_s": count / tr.makespan, "results_equal_saturated": same})
        print(f"# qps {frac:.2f}x: p50 {tr.percentile(50):.3f} s p99 {tr.percentile(99):.3f} s",
              file=sys.stderr, flush=True)
    line = {
        "metric": "active-edge relaxations/s", "value": R / sat.makespan, "unit": "relaxations/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": sat.makespan * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded splitmix64 lattices, drawn on the GPU)",
        "config": {"workload": f"serve{count}", "desc": SERVE_DESC, "requests": count,
                   "parallelism": "single GPU"},
        "saturation": {"requests_per_s": sat_rps, "solves_per_s": solves / sat.makespan,
                       "p50_s": sat.percentile(50), "p99_s": sat.percentile(99), "solves": solves},
        "sweep": sweep, "roofline": None, "cpu_baseline": None,
    }
    if args.plain:
        # the same requests one after another with plain launches (solve,
        # then the host-driven repeated-solve chain), in submission order,
        # until the time cap: the completed ones are compared with the
        # served ones, request by request
        t0 = time.perf_counter()
        same = True
        per = []
        for k, di in enumerate(dev):
            if time.perf_counter() - t0 > args.plain_cap_s:
                break
            print(f"#   plain request {k}", file=sys.stderr, flush=True)
            tk = time.perf_counter()
            scratch = torch.zeros(di.N, dtype=torch.uint8, device="cuda")
            path, res = solver.reconstruct(di, scratch)
            torch.cuda.synchronize()
            per.append(time.perf_counter() - tk)
            c = sat.completions[k]
            same = same and res.tuple() == c.res and path.tolist() == c.path
        pw = sum(per)
        done = len(per)
        line["plain"] = {"requests_done": done, "of": count, "cap_s": args.plain_cap_s, "seconds": pw,
                         "seconds_per_request": per, "requests_per_s": done / pw if pw else None,
                         "results_equal": same,
                         "served_speedup": sat_rps / (done / pw) if pw and done else None,
                         "note": ("requests are done in submission order until the cap; the rate is over the "
                                  "completed ones")}
    server.close()
    solver.close()
    print(json.dumps(line), flush=True)


RECON_DESC = ("path recovery on cube128 (seed 11, M=700) and a 2-D 1016^2 lattice (serving request 3 of master "
              "seed 51: f1,f2 U{1..10}, M=10989): repeated solves (host-driven, one csp_solve_dev per path edge) "
              "against one solve with the improvement log and a walk back")


GRAPH_DESC = ("the 128^3 cube (seed 11, M=700) given as a general graph: adjacency lists of its 6,242,304 edges "
              "(12,484,608 directed entries), solved by the graph kernel (labels in HBM)")


def run_graph(args):
    import numpy as np
    import torch
    from paper_1511_06441_amd import csp
    from paper_1511_06441_amd import inputs as gen

    inst = gen.cube128(11, 700)
    n, N = inst.n, inst.N
    us, vs, w1, w2, ids = [], [], [], [], []
    v_all = np.arange(N, dtype=np.int64)
    for k in range(3):
        c = (v_all // n ** k) % n
        u = v_all[c < n - 1]
        us.append(u)
        vs.append(u + n ** k)
        w1.append(inst.f1[k * N + u])
        w2.append(inst.f2[k * N + u])
        ids.append(k * N + u)
    g = csp.graph_to_device(gen.graph_csr(N, np.concatenate(us), np.concatenate(vs), np.concatenate(w1),
                                          np.concatenate(w2), np.concatenate(ids)))
    A = torch.from_numpy(inst.A).cuda()
    B = torch.from_numpy(inst.B).cuda()
    solver = csp.Solver(0)
    for _ in range(args.warmup):
        csp.csp_solve_graph_dev(solver.ctx, g, A, B, inst.M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = []
    for _ in range(args.steps):
        res, cnt = csp.csp_solve_graph_dev(solver.ctx, g, A, B, inst.M)
        kern.append(csp.csp_last_kernel_ms(solver.ctx))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    di = csp.to_device(inst)
    r2, c2 = solver.solve(di)
    lattice_ms = csp.csp_last_kernel_ms(solver.ctx)
    kms = sum(kern) / len(kern)
    b = algorithmic_bytes(N, cnt.asdict())
    line = {"metric": "active-edge relaxations/s", "value": cnt.R * args.steps / wall, "unit": "relaxations/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
            "data": "synthetic (seeded splitmix64 lattice as adjacency lists)",
            "config": {"workload": "graph128", "desc": GRAPH_DESC, "parallelism": "single GPU"},
            "results": dict(T=res.T, X=res.X, x=res.x, Y=res.Y, F2=res.F2, **cnt.asdict()),
            "equal_to_lattice_solve": res.tuple() == r2.tuple() and cnt.asdict() == c2.asdict(),
            "lattice_kernel_ms": lattice_ms,
            "roofline": {"bound": "hbm", "kernel": "k_graph", "achieved": b / (kms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": b / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "traffic": None, "kernel_ms_avg": kms, "algorithmic_bytes_per_step": b},
            "cpu_baseline": None}
    print(json.dumps(line), flush=True)
    solver.close()


def run_recon(args):
    import torch
    from paper_1511_06441_amd import csp
    from paper_1511_06441_amd import inputs as gen

    s, d, n, K, M = gen.serving_params(4, 51)[3]
    insts = [("cube128_s11_M700", csp.to_device(gen.cube128(11, 700))),
             (f"square{n}_s51_3", csp.DeviceInstance(d, n, *gen.lattice_edges_torch(d, n, s, K, K, device="cuda"),
                                                     gen.face_mask_torch(d, n, 0, 0, "cuda"),
                                                     gen.face_mask_torch(d, n, 0, n - 1, "cuda"), M))]
    torch.cuda.synchronize()
    solver = csp.Solver(0)
    out = []
    for name, di in insts:
        solver.reconstruct_log(di)                      # warm-up (sizes the log)
        scratch = torch.zeros(di.N, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p_rep, r_rep = solver.reconstruct(di, scratch)
        torch.cuda.synchronize()
        t_rep = time.perf_counter() - t0
        t0 = time.perf_counter()
        reps = max(1, args.steps)
        for _ in range(reps):
            p_log, r_log, c_log = solver.reconstruct_log(di)
        torch.cuda.synchronize()
        t_log = (time.perf_counter() - t0) / reps
        out.append({"instance": name, "path_vertices": len(p_log), "T": r_log.T, "F2": r_log.F2,
                    "repeated_solves_s": t_rep, "logged_s": t_log, "speedup": t_rep / t_log,
                    "paths_equal": p_rep.tolist() == p_log.tolist() and r_rep.tuple() == r_log.tuple(),
                    "log_records": c_log.U})
        print(f"# {name}: repeated {t_rep:.3f} s, logged {t_log * 1e3:.1f} ms, {len(p_log)} vertices",
              file=sys.stderr, flush=True)
    line = {"metric": "path recoveries/s", "value": len(out) / sum(o["logged_s"] for o in out),
            "unit": "recoveries/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": sum(o["logged_s"] for o in out) * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded splitmix64 lattices)",
            "config": {"workload": "recon", "desc": RECON_DESC, "parallelism": "single GPU"},
            "results": out, "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)
    solver.close()


def run_micro(args):
    """The device limits behind the cycle's shape: copy bandwidth, scattered
    atomicMax rate, scattered 16-byte loads (the sending step's edge
    records) and the two barriers (the cycle loop's, and the fully fenced
    one with dirty lines to write back)."""
    import torch
    from paper_1511_06441_amd import csp

    solver = csp.Solver(0)
    stream = torch.cuda.current_stream()
    mb = lambda *a: csp.csp_microbench(solver.ctx, *a, stream=stream)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    mb(csp.MB_COPY, 1 << 30, 1)
    out = {"copy_1GiB_GBps": mb(csp.MB_COPY, 1 << 30, 10)[0]}
    # smaller copies: 2 x 8 MiB stays in the L2s (4 MiB per XCD), 2 x 64 MiB
    # and 2 x 96 MiB in the 256 MiB Infinity Cache
    out["copy_GBps_by_size"] = {}
    for mib in (8, 64, 96, 256):
        mb(csp.MB_COPY, mib << 20, 2)
        out["copy_GBps_by_size"][f"{mib}MiB"] = mb(csp.MB_COPY, mib << 20, 200 if mib < 256 else 50)[0]
    mb(csp.MB_ATOMIC, 1 << 24, 1 << 24)
    out["atomicmax_scattered_Gps"] = {"64MiB": mb(csp.MB_ATOMIC, 1 << 28, 1 << 24)[0],
                                      "1GiB": mb(csp.MB_ATOMIC, 1 << 28, 1 << 28)[0]}
    out["record_loads"] = {}
    for nr in (1024, 3400, 6800):
        mb(csp.MB_LOADS, nr, 10)
        g, us = mb(csp.MB_LOADS, nr, 400)
        out["record_loads"][f"{nr}_per_cu"] = {"G_loads_per_s": g, "us_per_round": us}
    # 3,400 loads per CU and round from slabs of 2^lg records per CU: 16 MiB
    # in all (lg 12, in the L2s) up to 1 GiB (lg 18, beyond the Infinity Cache)
    out["record_loads_by_footprint"] = {}
    for lg in (12, 14, 15, 16, 18):
        mb(csp.MB_LOADS, 3400, 10, lg)
        g, us = mb(csp.MB_LOADS, 3400, 400, lg)
        out["record_loads_by_footprint"][f"{(cus << lg) * 16 >> 20}MiB"] = {"G_loads_per_s": g, "us_per_round": us}
    out["barrier_us"] = {}
    for dirty in (0, 64, 256):
        mb(csp.MB_BARRIER, 100, cus, dirty)
        a, b2 = mb(csp.MB_BARRIER, 2000, cus, dirty)
        out["barrier_us"][f"{cus}wg_dirty{dirty}KiB"] = {"cycle_loop": a, "fenced": b2}
    line = {"metric": "device micro-benchmarks", "value": out["copy_1GiB_GBps"], "unit": "GB/s (copy)",
            "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": True, "dtype": "u32",
            "data": "synthetic", "config": {"workload": "micro", "cus": cus}, "micro": out}
    print(json.dumps(line), flush=True)
    solver.close()


def algorithmic_bytes(N, c, L=4):
    """Bytes the method must move for one solve with L-byte labels (label
    init, own label per improvement, f1+f2+neighbour label per test, one flow
    record written per send, one flow record read plus a label
    read-modify-write per delivery)."""
    return (N * L + c["U"] * L + c["D"] * (2 + L) + c["E"] * FLOW_BYTES
            + c["R"] * (FLOW_BYTES + 2 * L))


def trace_summary(csp, solver, torch, di, points=16):
    """Active set |I_t| and water in transit against t for one solve (outside
    the timed region), sampled at `points` evenly spaced rows."""
    cap = 1 << 20
    tr = torch.zeros((cap, 4), dtype=torch.int64, device="cuda")
    csp.csp_set_trace(solver.ctx, tr)
    try:
        res, cnt = solver.solve(di)
        rows = min(csp.csp_last_trace_rows(solver.ctx), cap)
    finally:
        csp.csp_set_trace(solver.ctx, None)
    a = tr[:rows].cpu().numpy()
    sent0 = cnt.E - int(a[:, 3].sum())
    transit = sent0 + (a[:, 3] - a[:, 1]).cumsum()
    idx = sorted(set(int(round(k * (rows - 1) / (points - 1))) for k in range(points)))
    return {"rows": rows, "T": res.T, "max_active": int(a[:, 2].max()), "t_max_active": int(a[a[:, 2].argmax(), 0]),
            "max_transit": int(max(sent0, transit.max())),
            "samples": [[int(a[k, 0]), int(a[k, 2]), int(transit[k])] for k in idx]}


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, when it was taken on the current kernel source; else None."""
    import hashlib
    import re
    summary = os.path.join(ROOT, "profiles", f"k_ranges3_{workload}_traffic.md")
    src = os.path.join(ROOT, "paper_1511_06441_amd", "csrc", "csp.hip")
    if not os.path.exists(summary):
        return None
    text = open(summary).read()
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    m_h = re.search(r"csp_hip_sha256:\s*([0-9a-f]{64})", text)
    if not (m_b and m_h):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_h.group(1):
        return None
    return float(m_b.group(1))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_run(inst, max_cycles):
    from oracle import oracle as O
    t0 = time.perf_counter()
    r = O.solve_instance(inst, want_labels=False, max_cycles=max_cycles)
    return r.counters["R"], time.perf_counter() - t0


def _oracle_window(args):
    """Relaxations/s of the oracle over cycles k1+1..k2 of one instance (two
    prefix runs; the difference removes set-up and the small first cycles)."""
    wl, k1, k2 = args
    inst = WORKLOADS[wl]["build"](_gen())[WORKLOADS[wl]["sample_index"]]
    R1, t1 = _oracle_run(inst, k1)
    R2, t2 = _oracle_run(inst, k2)
    return (R2 - R1) / (t2 - t1), R2 - R1, t2 - t1


def _gen():
    from paper_1511_06441_amd import inputs as gen
    return gen


def _oracle_mixed(j):
    """Oracle solve of problem j of the 1,024-problem batch: (R, seconds)."""
    inst = _gen().mixed_instance(41, j)
    return _oracle_run(inst, 0)


def cpu_baseline_batch(step=64):
    """The oracle on every step-th problem of the batch, instance-parallel over
    the host's processes (at most 16), each process timing its own solves."""
    import multiprocessing as mp
    gen = _gen()
    nproc = len(os.sched_getaffinity(0))
    procs = max(1, min(16, nproc))
    js = list(range(0, 1024, step))
    verts = sum(n ** d for (_, d, n, _, _) in (gen.mixed_params(41, j) for j in js))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        runs = pool.map(_oracle_mixed, js, chunksize=1)
    wall = time.perf_counter() - t0
    R = sum(r for r, _ in runs)
    cpu_s = sum(t for _, t in runs)
    return dict(value=R / cpu_s, unit="relaxations/s", cores=1, kind="oracle",
                sample=(f"problems 0, {step}, ..., {js[-1]} of the batch ({len(js)} problems, {verts:,} vertices), "
                        f"single-threaded C oracle (-O2): R={R} in {cpu_s:.1f} s of solve time"),
                seconds=round(cpu_s, 2), cpu_model=_cpu_model(), nproc=nproc,
                solves_per_s=len(js) / cpu_s,
                parallel={"value": R / wall, "processes": procs, "solves_per_s": len(js) / wall,
                          "seconds": round(wall, 2),
                          "how": "instance-parallel: the sample's problems spread over a pool of processes"})


def cpu_baseline(workload, inst):
    """The oracle timed on this host: one thread, and the same sample run in
    as many concurrent processes as the host gives this job (at most 16)."""
    import multiprocessing as mp
    wl = WORKLOADS[workload]
    nproc = len(os.sched_getaffinity(0))
    procs = max(1, min(16, nproc))
    if "sample_cycles" in wl:
        k1, k2 = wl["sample_cycles"]
        v, R, dt = _oracle_window((workload, k1, k2))
        with mp.get_context("fork").Pool(procs) as pool:
            par = pool.map(_oracle_window, [(workload, k1, k2)] * procs)
        sample = (f"cycles {k1 + 1}..{k2} of {inst.name} (difference of two prefix runs of the single-threaded "
                  f"C oracle, -O2): R={R} in {dt:.1f} s")
        par_v = sum(x[0] for x in par)
    else:
        R, dt = _oracle_run(inst, 0)
        v = R / dt
        with mp.get_context("fork").Pool(procs) as pool:
            par = pool.starmap(_oracle_run, [(inst, 0)] * procs)
        sample = f"one whole solve of {inst.name} (single-threaded C oracle, -O2), {dt:.1f} s, R={R}"
        par_v = sum(r / t for r, t in par)
    return dict(value=v, unit="relaxations/s", cores=1, kind="oracle", sample=sample, seconds=round(dt, 2),
                cpu_model=_cpu_model(), nproc=nproc,
                parallel={"value": par_v, "processes": procs,
                          "how": "the same sample in concurrent processes, one instance each; sum of their rates"})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube256",
                    choices=sorted(WORKLOADS) + ["batch1024", "serve", "recon", "graph128", "micro"])
    ap.add_argument("--batch-count", type=int, default=1024)
    ap.add_argument("--plain", action="store_true", help="batch workload: also time sequential plain launches")
    ap.add_argument("--serve-count", type=int, default=8)
    ap.add_argument("--serve-arena-gb", type=int, default=64)
    ap.add_argument("--serve-fracs", type=float, nargs="*", default=[0.25, 0.5, 0.8])
    ap.add_argument("--plain-cap-s", type=float, default=300.0,
                    help="serve workload with --plain: stop the sequential plain leg after this many seconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="lattice workloads: autotune each lattice shape before timing (traffic reported "
                         "null); batch1024: autotune the gang size")
    ap.add_argument("--path", type=int, default=0,
                    help="lattice workloads: 0 automatic, 1 contiguous ranges, 2 global labels, 3 x-pencil ranges (d=3)")
    ap.add_argument("--dense-sweep", type=int, nargs="*", default=None,
                    help="lattice workloads: also time each solve with these dense thresholds (flows delivered "
                         "to a range in a cycle; -1 never), untimed by the step")
    ap.add_argument("--trace", action="store_true",
                    help="also report |I_t| and water in transit against t (one extra solve each, untimed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the path does not shard "
              "across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch1024":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "recon":
        run_recon(args)
        return
    if args.workload == "graph128":
        run_graph(args)
        return
    if args.workload == "micro":
        run_micro(args)
        return

    import torch
    from paper_1511_06441_amd import csp
    from paper_1511_06441_amd import inputs as gen

    wl = WORKLOADS[args.workload]
    insts = wl["build"](gen)
    dev = [csp.to_device(i) for i in insts]
    solver = csp.Solver(0)
    stream = torch.cuda.current_stream()
    if args.path:
        csp.csp_set_path(solver.ctx, args.path)

    tuned = []
    if args.autotune:
        seen = set()
        for di in dev:
            if (di.d, di.n) not in seen:
                seen.add((di.d, di.n))
                b, pth, ms = solver.autotune(di, stream=stream)
                tuned.append({"d": di.d, "n": di.n, "blocks": b, "path": pth, "kernel_ms": round(ms, 3)})

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
    bytes_step = sum(algorithmic_bytes(i.N, c.asdict(), wl["label_bytes"]) for i, (_, c, _) in zip(insts, runs[0]))
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
        "dtype": "u16" if wl["label_bytes"] == 2 else "u32",
        "data": "synthetic (seeded splitmix64 lattices)",
        "config": {"workload": args.workload, "desc": wl["desc"], "solves_per_step": len(dev),
                   "parallelism": "single GPU"},
        "solves_per_s": solves / wall,
        "results": [dict(T=r.T, X=r.X, x=r.x, Y=r.Y, F2=r.F2, **c.asdict()) for r, c, _ in runs[0]],
        "kernel_ms_per_solve": [round(sum(st[k][2] for st in runs) / len(runs), 3) for k in range(len(dev))],
        "roofline": {
            "bound": "hbm",
            "kernel": (f"k_ranges<{insts[0].d}>" if csp.csp_last_path(solver.ctx) == 1
                       else f"k_solve<{insts[0].d}>"),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            # the counter summaries were taken with the automatic configuration
            "traffic": None if args.autotune else measured_traffic(args.workload),
            "kernel_ms_avg": sum(kern_ms) / len(kern_ms),
            "algorithmic_bytes_per_step": bytes_step,
        },
        "cpu_baseline": None,
    }
    if tuned:
        line["autotune"] = tuned
    if args.trace:
        line["trace"] = [trace_summary(csp, solver, torch, di) for di in dev]
    if args.dense_sweep is not None:
        sweep = []
        for thr in args.dense_sweep:
            csp.csp_set_dense_threshold(solver.ctx, (1 << 32) - 1 if thr < 0 else thr)
            ms = []
            for di in dev:
                solver.solve(di, stream=stream)
                reps = []
                for _ in range(3):
                    solver.solve(di, stream=stream)
                    reps.append(csp.csp_last_kernel_ms(solver.ctx))
                ms.append(round(min(reps), 3))
            sweep.append({"dense_threshold": thr, "kernel_ms": ms})
        csp.csp_set_dense_threshold(solver.ctx, -1)
        line["dense_sweep"] = sweep
    if not args.no_cpu_baseline and wl["sample_index"] is not None:
        line["cpu_baseline"] = cpu_baseline(args.workload, insts[wl["sample_index"]])
    print(json.dumps(line), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
