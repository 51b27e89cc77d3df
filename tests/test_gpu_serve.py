"""Serving with continuous batching: requests submitted while others run
give the oracle's result and path, and the same completion alone and in the
mix."""
import sys
import time

import numpy as np
import pytest

from paper_1511_06441_amd import inputs as gen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def solver(torch):
    from paper_1511_06441_amd import csp
    s = csp.Solver(0)
    yield s
    s.close()


@pytest.fixture
def server(solver):
    from paper_1511_06441_amd import csp
    srv = csp.Server(solver, arena_bytes=4 << 30, max_jobs=64)
    yield srv
    srv.close()


def _oracle_request(inst):
    from oracle import oracle as O
    ref = O.solve_instance(inst, want_labels=False)
    path, res, _ = O.reconstruct(inst.d, inst.n, inst.f1, inst.f2, inst.A, inst.B, inst.M)
    assert res.tuple() == ref.tuple()
    return ref, [int(v) for v in path]


def _key(c):
    return (c.status, c.res, tuple(sorted(c.counters.items())), c.solves, tuple(c.path))


def _run_all(server, devs, recon=True, stagger=0):
    """Submit every request (every `stagger`-th one after a poll, so later
    requests arrive while earlier ones run) and collect the completions."""
    done = {}
    for k, di in enumerate(devs):
        server.submit(di, reconstruct=recon, tag=k)
        if stagger and k % stagger == stagger - 1:
            for c in server.poll():
                done[c.tag] = c
    for c in server.drain():
        done[c.tag] = c
    assert sorted(done) == list(range(len(devs)))
    return done


def test_serve_small_vs_oracle(server, torch):
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(51, j, lo2=(8, 48), lo3=(4, 16)) for j in range(24)]
    devs = [csp.to_device(i) for i in insts]
    _say("serving 24 small requests")
    done = _run_all(server, devs, stagger=5)
    for k, inst in enumerate(insts):
        ref, path = _oracle_request(inst)
        c = done[k]
        assert c.status == 0, (inst.name, c.status)
        assert c.res == ref.tuple(), inst.name
        assert c.counters == ref.counters, inst.name
        assert c.path == path, inst.name
        assert c.solves == (max(len(path) - 1, 1) if ref.T >= 0 else 1)


def test_serve_gangs_vs_plain(server, solver, torch):
    """Requests that need gangs of workgroups, mixed with small ones: each
    completion equals the plain solve and reconstruction of the request."""
    from paper_1511_06441_amd import csp
    insts = [gen.opposite_faces(2, 420, 3, 9, 9, 3000), gen.square64(1),
             gen.opposite_faces(3, 52, 4, 12, 12, 600), gen.square64(2),
             gen.opposite_faces(2, 300, 5, 4, 4, 1200), gen.opposite_faces(3, 20, 6, 7, 7, 160)]
    devs = [csp.to_device(i) for i in insts]
    _say("serving gang requests")
    done = _run_all(server, devs, stagger=2)
    for k, (inst, di) in enumerate(zip(insts, devs)):
        r1, c1 = solver.solve(di)
        scratch = torch.zeros(inst.N, dtype=torch.uint8, device="cuda")
        path, res = solver.reconstruct(di, scratch)
        c = done[k]
        assert c.status == 0, (k, c.status)
        assert c.res == r1.tuple() == res.tuple(), k
        assert c.counters == c1.asdict(), k
        assert c.path == path.tolist(), k


def test_serve_alone_equals_mix(server, torch):
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(51, j, lo2=(16, 160), lo3=(8, 32)) for j in range(16)]
    devs = [csp.to_device(i) for i in insts]
    alone = {}
    for k, di in enumerate(devs):
        server.submit(di, reconstruct=True, tag=k)
        for c in server.drain():
            alone[c.tag] = c
    mixed = _run_all(server, devs, stagger=3)
    for k in range(len(devs)):
        assert _key(alone[k]) == _key(mixed[k]), insts[k].name


def test_serve_dimensions_one_and_four(server, torch):
    """1-d and 4-d requests (one of them needing a gang) with their paths."""
    from paper_1511_06441_amd import csp
    insts = [gen.opposite_faces(1, 300, 61, 9, 9, 900), gen.opposite_faces(4, 7, 62, 5, 5, 60),
             gen.opposite_faces(4, 20, 63, 6, 6, 300), gen.opposite_faces(1, 9, 64, 4, 4, 2)]
    done = _run_all(server, [csp.to_device(i) for i in insts], stagger=2)
    for k, inst in enumerate(insts):
        ref, path = _oracle_request(inst)
        c = done[k]
        assert c.status == 0, (k, c.status)
        assert c.res == ref.tuple() and c.counters == ref.counters, k
        assert c.path == path, k


def test_serve_without_reconstruction(server, torch):
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(53, j, lo2=(8, 64), lo3=(4, 20)) for j in range(12)]
    done = _run_all(server, [csp.to_device(i) for i in insts], recon=False)
    for k, inst in enumerate(insts):
        ref = O.solve_instance(inst, want_labels=False)
        assert done[k].res == ref.tuple() and done[k].counters == ref.counters
        assert done[k].path == [] and done[k].solves == 1


def test_serve_overflow_retry(solver, torch):
    """A one-flow starting wheel forces re-admission with larger pools."""
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(7, j, lo2=(8, 64), lo3=(4, 20)) for j in range(8)]
    csp.csp_set_pool_hint(solver.ctx, 1)
    try:
        srv = csp.Server(solver, arena_bytes=1 << 30, max_jobs=16)
        try:
            done = _run_all(srv, [csp.to_device(i) for i in insts])
        finally:
            srv.close()
    finally:
        csp.csp_set_pool_hint(solver.ctx, 0)
    for k, inst in enumerate(insts):
        ref, path = _oracle_request(inst)
        assert done[k].status == 0 and done[k].res == ref.tuple() and done[k].path == path


def test_serve_errors_come_back_per_request(server, torch):
    from paper_1511_06441_amd import csp
    ok = gen.square64(3)
    bad = gen.square64(3)
    bad.B = bad.B.copy()
    bad.B[0] = 1                      # vertex 0 is in A too
    zero = gen.square64(3)
    zero.f1 = zero.f1.copy()
    zero.f1[5] = 0                    # a real edge with f1 = 0
    done = _run_all(server, [csp.to_device(i) for i in (ok, bad, zero)])
    assert done[0].status == csp.CSP_OK
    assert done[1].status == csp.CSP_EINVAL
    assert done[2].status == csp.CSP_EINVAL
    with pytest.raises(csp.CspError):
        server.submit(csp.DeviceInstance(2, 1, ok_t := torch.zeros(4, dtype=torch.uint8, device="cuda"),
                                         ok_t, ok_t, ok_t, 10))


def test_serve_idle_then_again(server, torch):
    """Workers leave when the server idles; the next request starts them again."""
    from paper_1511_06441_amd import csp
    inst = gen.square64(1)
    ref, path = _oracle_request(inst)
    di = csp.to_device(inst)
    for rep in range(3):
        server.submit(di, tag=rep)
        (c,) = server.drain()
        assert c.res == ref.tuple() and c.path == path
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.05:
            server.poll()
            time.sleep(0.005)


def _submit_watching(srv, devs, recon):
    """Submit every request without polling in between; the largest number
    seen waiting for admission."""
    most = 0
    for k, di in enumerate(devs):
        srv.submit(di, reconstruct=recon, tag=k)
        most = max(most, srv.pending()[0])
    return most


def _collect(srv, count):
    done = {}
    for c in srv.drain():
        done[c.tag] = c
    assert sorted(done) == list(range(count))
    return done


@pytest.mark.parametrize("limit", ["job_slots", "arena", "workers"])
def test_serve_requests_wait_for_admission(solver, torch, limit):
    """Requests that cannot all be on the GPU at once wait until a job slot
    (max_jobs = 1), arena memory (12 MiB for 2-4 MB requests) or workers (gangs
    of 16 workgroups, 24 requests against one workgroup per CU) free up; every
    result, path included, equals the oracle's."""
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    if limit == "workers":
        # M above 65,535 keeps 32-bit labels in LDS: ranges of 32K vertices,
        # so an 80^3 request takes a gang of 16 workgroups
        base = [gen.opposite_faces(3, 80, 71, 10, 10, 70000), gen.opposite_faces(3, 80, 72, 10, 10, 70001)]
        insts = [base[k % 2] for k in range(24)]
        srv = csp.Server(solver, arena_bytes=16 << 30, max_jobs=64)
        recon = False
    else:
        base = [gen.opposite_faces(2, 120, 73, 6, 6, 500), gen.opposite_faces(2, 100, 74, 6, 6, 400),
                gen.opposite_faces(3, 30, 75, 8, 8, 300)]
        insts = [base[k % 3] for k in range(9)]
        srv = csp.Server(solver, arena_bytes=(1 << 30) if limit == "job_slots" else (12 << 20),
                         max_jobs=1 if limit == "job_slots" else 64)
        recon = True
    try:
        devs = [csp.to_device(i) for i in insts]
        torch.cuda.synchronize()
        _say("serving", len(devs), "requests, limited by", limit)
        most = _submit_watching(srv, devs, recon)
        done = _collect(srv, len(devs))
    finally:
        srv.close()
    assert most >= 1, "no request had to wait"
    refs = {}
    for k, inst in enumerate(insts):
        key = id(inst)
        if key not in refs:
            if recon:
                refs[key] = _oracle_request(inst)
            else:
                refs[key] = (O.solve_instance(inst, want_labels=False), [])
        ref, path = refs[key]
        c = done[k]
        assert c.status == 0, (k, c.status)
        assert c.res == ref.tuple() and c.counters == ref.counters, (k, inst.name)
        assert c.path == path, (k, inst.name)


def test_config5_requests_vs_stored_oracle(solver, torch):
    """The first 8 serving requests of master seed 51 (2-D sides 64..1024,
    3-D sides 32..256, up to 1,032,256 vertices), submitted at once to one
    server: result, counters of the first solve and the whole path recovered
    by repeated solves equal the oracle's stored outputs."""
    import json
    import os
    from paper_1511_06441_amd import csp
    with open(os.path.join(os.path.dirname(__file__), "golden", "serve8_s51.json")) as fh:
        rec = json.load(fh)["problems"]
    assert len(rec) == 8
    devs = []
    for k, g in enumerate(rec):
        s, d, n, K, M = gen.serving_params(8, 51)[k]
        assert (d, n, K, M, s) == (g["d"], g["n"], g["K"], g["M"], g["seed"])
        f1, f2 = gen.lattice_edges_torch(d, n, s, K, K, device="cuda")
        devs.append(csp.DeviceInstance(d, n, f1, f2, gen.face_mask_torch(d, n, 0, 0, "cuda"),
                                       gen.face_mask_torch(d, n, 0, n - 1, "cuda"), M))
    torch.cuda.synchronize()
    srv = csp.Server(solver, arena_bytes=16 << 30, max_jobs=64)
    try:
        _say("config-5: 8 requests with paths")
        t0 = time.perf_counter()
        done = _run_all(srv, devs, stagger=0)
        _say("  served in %.1f s" % (time.perf_counter() - t0))
    finally:
        srv.close()
    for k, g in enumerate(rec):
        c = done[k]
        assert c.status == 0, (k, c.status)
        assert c.res == (g["T"], g["X"], g["x"], g["Y"], g["F2"]), k
        assert c.counters == g["counters"], k
        if g["path_complete"]:
            assert c.path == g["path"], k
            assert c.solves == max(len(g["path"]) - 1, 1)
        else:
            # the oracle stored the first solves of the chain: the path's last
            # vertices are the ones those solves named; the rest must be a
            # lattice path from A whose edges sum to (T, F2)
            tail = g["path"]
            assert c.path[-len(tail):] == tail, k
            assert c.solves == len(c.path) - 1 and c.solves >= len(g["resolves"])
            s, d, n, K, M = gen.serving_params(8, 51)[k]
            _check_lattice_path(d, n, s, K, M, c.path, g["T"], g["F2"])


def _check_lattice_path(d, n, seed, K, M, path, T, F2):
    """path runs from the face x = 0 to its last vertex along lattice edges,
    visits no vertex twice, and its edges' f1 and f2 sum to T and F2 < M."""
    f1, f2 = gen.lattice_edges(d, n, seed, K, K)
    N = n ** d
    assert path[0] % n == 0 and len(set(path)) == len(path)
    s1 = s2 = 0
    for u, v in zip(path[:-1], path[1:]):
        lo, delta = min(u, v), abs(u - v)
        k = next(j for j in range(d) if n ** j == delta)
        assert (lo // n ** k) % n < n - 1            # the two ends are lattice neighbours
        s1 += int(f1[k * N + lo])
        s2 += int(f2[k * N + lo])
    assert (s1, s2) == (T, F2) and F2 < M
