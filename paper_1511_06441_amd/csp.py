"""Thin ctypes binding of libcsp (include/csp.h).  Argument marshalling only:
every step of a solve runs in the HIP library.  PyTorch supplies device
memory and streams.

Importing this module loads ``libcsp.so`` from this package directory and
raises if it is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsp.so")

CSP_OK = 0
CSP_EINVAL = -1
CSP_ENOMEM = -2
CSP_EDEVICE = -3
CSP_EOVERFLOW = -4
CSP_ECANCELED = -5
CSP_MAX_M = 0x0FFFFFFF
CSP_SCRATCH_BYTES = 256 << 20

EXPORTED = (
    "csp_create", "csp_destroy", "csp_last_error", "csp_solve_dev", "csp_solve",
    "csp_reconstruct_dev", "csp_last_kernel_ms", "csp_set_pool_hint",
    "csp_set_blocks", "csp_set_phase_timing", "csp_last_phase_us", "csp_set_path",
    "csp_last_path", "csp_solve_batch", "csp_serve_open", "csp_serve_submit",
    "csp_serve_poll", "csp_serve_pending", "csp_serve_close", "csp_set_trace", "csp_last_trace_rows",
    "csp_reconstruct_log_dev", "csp_solve_graph_dev", "csp_autotune", "csp_autotune_clear",
    "csp_set_batch_target", "csp_autotune_batch", "csp_reconstruct",
    "csp_set_dense_threshold", "csp_tuned_dense_threshold", "csp_last_phase_spread", "csp_set_wait_limit",
    "csp_solve_dev_noalloc", "csp_microbench",
)


class csp_result(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int64), ("X", ctypes.c_int64), ("x", ctypes.c_int64),
                ("Y", ctypes.c_int64), ("F2", ctypes.c_int64)]

    def tuple(self):
        return (self.T, self.X, self.x, self.Y, self.F2)


class csp_problem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int64), ("f1", ctypes.c_void_p),
                ("f2", ctypes.c_void_p), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("M", ctypes.c_uint32), ("labels", ctypes.c_void_p)]


class csp_counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("C", "U", "D", "E", "R", "P", "I")]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class csp_request(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int64), ("f1", ctypes.c_void_p),
                ("f2", ctypes.c_void_p), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("M", ctypes.c_uint32), ("reconstruct", ctypes.c_int), ("tag", ctypes.c_uint64)]


class csp_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("res", csp_result),
                ("cnt", csp_counters), ("cnt_chain", csp_counters), ("solves", ctypes.c_int64),
                ("path_len", ctypes.c_int64), ("path", ctypes.POINTER(ctypes.c_int64))]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libcsp.so not built ({LIB_PATH}); run python -m paper_1511_06441_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    p, i64, u32, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int
    lib.csp_create.argtypes = [i32, ctypes.POINTER(p)]
    lib.csp_create.restype = i32
    lib.csp_destroy.argtypes = [p]
    lib.csp_destroy.restype = None
    lib.csp_last_error.argtypes = [p]
    lib.csp_last_error.restype = ctypes.c_char_p
    lib.csp_solve_dev.argtypes = [p, i32, i64, p, p, p, p, u32, p, ctypes.POINTER(csp_result),
                                  ctypes.POINTER(csp_counters), i64, p]
    lib.csp_solve_dev.restype = i32
    lib.csp_solve_dev_noalloc.argtypes = lib.csp_solve_dev.argtypes
    lib.csp_solve_dev_noalloc.restype = i32
    lib.csp_microbench.argtypes = [p, i32, i64, i64, i64, ctypes.POINTER(ctypes.c_double), p]
    lib.csp_microbench.restype = i32
    lib.csp_solve.argtypes = [p, i32, i64, p, p, p, p, u32, p, ctypes.POINTER(csp_result),
                              ctypes.POINTER(csp_counters)]
    lib.csp_solve.restype = i32
    lib.csp_reconstruct_dev.argtypes = [p, i32, i64, p, p, p, p, u32, p, p, i64,
                                        ctypes.POINTER(i64), ctypes.POINTER(csp_result), p]
    lib.csp_reconstruct_dev.restype = i32
    lib.csp_last_kernel_ms.argtypes = [p, ctypes.POINTER(ctypes.c_float)]
    lib.csp_last_kernel_ms.restype = i32
    lib.csp_set_pool_hint.argtypes = [p, ctypes.c_uint64]
    lib.csp_set_pool_hint.restype = i32
    lib.csp_set_blocks.argtypes = [p, i32]
    lib.csp_set_blocks.restype = i32
    lib.csp_solve_batch.argtypes = [p, i32, p, p, p, p]
    lib.csp_solve_batch.restype = i32
    lib.csp_set_path.argtypes = [p, i32]
    lib.csp_set_path.restype = i32
    lib.csp_last_path.argtypes = [p]
    lib.csp_last_path.restype = i32
    lib.csp_autotune.argtypes = [p, i32, i64, p, p, p, p, u32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                 ctypes.POINTER(ctypes.c_float), p]
    lib.csp_autotune.restype = i32
    lib.csp_autotune_clear.argtypes = [p]
    lib.csp_autotune_clear.restype = i32
    lib.csp_reconstruct.argtypes = [p, i32, i64, p, p, p, p, u32, p, i64, ctypes.POINTER(i64),
                                    ctypes.POINTER(csp_result)]
    lib.csp_reconstruct.restype = i32
    lib.csp_set_batch_target.argtypes = [p, i64]
    lib.csp_set_batch_target.restype = i32
    lib.csp_autotune_batch.argtypes = [p, i32, p, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_float), p]
    lib.csp_autotune_batch.restype = i32
    lib.csp_set_phase_timing.argtypes = [p, i32]
    lib.csp_set_phase_timing.restype = i32
    lib.csp_last_phase_us.argtypes = [p, ctypes.POINTER(ctypes.c_double)]
    lib.csp_last_phase_us.restype = i32
    lib.csp_reconstruct_log_dev.argtypes = [p, i32, i64, p, p, p, p, u32, p, i64, ctypes.POINTER(i64),
                                            ctypes.POINTER(csp_result), ctypes.POINTER(csp_counters), p]
    lib.csp_reconstruct_log_dev.restype = i32
    lib.csp_solve_graph_dev.argtypes = [p, i64, p, p, p, p, p, p, p, u32, p, ctypes.POINTER(csp_result),
                                        ctypes.POINTER(csp_counters), i64, p]
    lib.csp_solve_graph_dev.restype = i32
    lib.csp_set_trace.argtypes = [p, p, i64]
    lib.csp_set_trace.restype = i32
    lib.csp_last_trace_rows.argtypes = [p, ctypes.POINTER(i64)]
    lib.csp_last_trace_rows.restype = i32
    lib.csp_last_phase_spread.argtypes = [p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.csp_last_phase_spread.restype = i32
    lib.csp_set_wait_limit.argtypes = [p, i64]
    lib.csp_set_wait_limit.restype = i32
    lib.csp_set_dense_threshold.argtypes = [p, i64]
    lib.csp_set_dense_threshold.restype = i32
    lib.csp_tuned_dense_threshold.argtypes = [p, i32, i64, ctypes.POINTER(i64)]
    lib.csp_tuned_dense_threshold.restype = i32
    lib.csp_serve_open.argtypes = [p, ctypes.c_uint64, i32, ctypes.POINTER(p)]
    lib.csp_serve_open.restype = i32
    lib.csp_serve_submit.argtypes = [p, ctypes.POINTER(csp_request)]
    lib.csp_serve_submit.restype = i32
    lib.csp_serve_poll.argtypes = [p, ctypes.POINTER(csp_completion), i32, ctypes.POINTER(i32)]
    lib.csp_serve_poll.restype = i32
    lib.csp_serve_pending.argtypes = [p, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.csp_serve_pending.restype = i32
    lib.csp_serve_close.argtypes = [p]
    lib.csp_serve_close.restype = i32
    return lib


lib = _load()


class CspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libcsp error {code}: {msg}")
        self.code = code


def _check(ctx, rc):
    if rc != CSP_OK:
        msg = lib.csp_last_error(ctx).decode() if ctx else ""
        raise CspError(rc, msg)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# --- the C entry points, same names ---------------------------------------

def csp_create(device: int = 0):
    h = ctypes.c_void_p()
    _check(None, lib.csp_create(device, ctypes.byref(h)))
    return h


def csp_destroy(ctx):
    lib.csp_destroy(ctx)


def csp_last_error(ctx) -> str:
    return lib.csp_last_error(ctx).decode()


def csp_solve_dev(ctx, d, n, f1, f2, A, B, M, labels=None, counters=True, max_cycles=0,
                  stream=None):
    """Device tensors (uint8 f1/f2 [d*N], A/B [N]; int32/uint32 labels [N])."""
    res = csp_result()
    cnt = csp_counters()
    rc = lib.csp_solve_dev(ctx, d, n, _ptr(f1), _ptr(f2), _ptr(A), _ptr(B), M, _ptr(labels),
                           ctypes.byref(res), ctypes.byref(cnt) if counters else None,
                           max_cycles, _stream(stream))
    _check(ctx, rc)
    return res, (cnt if counters else None)


def csp_solve_dev_noalloc(ctx, d, n, f1, f2, A, B, M, labels=None, counters=True, max_cycles=0,
                          stream=None):
    """As csp_solve_dev; the solve's device state lives in the library's
    static per-GPU scratch (CSP_SCRATCH_BYTES), so the call allocates nothing."""
    res = csp_result()
    cnt = csp_counters()
    rc = lib.csp_solve_dev_noalloc(ctx, d, n, _ptr(f1), _ptr(f2), _ptr(A), _ptr(B), M, _ptr(labels),
                                   ctypes.byref(res), ctypes.byref(cnt) if counters else None,
                                   max_cycles, _stream(stream))
    _check(ctx, rc)
    return res, (cnt if counters else None)


MB_COPY, MB_ATOMIC, MB_LOADS, MB_BARRIER = 0, 1, 2, 3


def csp_microbench(ctx, kind, p0, p1, p2=0, stream=None):
    """Device micro-benchmark (include/csp.h): returns its two result slots."""
    r = (ctypes.c_double * 2)()
    _check(ctx, lib.csp_microbench(ctx, kind, p0, p1, p2, r, _stream(stream)))
    return r[0], r[1]


def csp_solve(ctx, d, n, f1, f2, A, B, M, labels=None):
    """Host numpy arrays; labels (numpy uint32 [N]) is filled if given."""
    res = csp_result()
    cnt = csp_counters()
    addr = lambda a: ctypes.c_void_p(a.ctypes.data) if a is not None else None
    rc = lib.csp_solve(ctx, d, n, addr(f1), addr(f2), addr(A), addr(B), M, addr(labels),
                       ctypes.byref(res), ctypes.byref(cnt))
    _check(ctx, rc)
    return res, cnt


def csp_reconstruct(ctx, d, n, f1, f2, A, B, M, cap):
    """Host numpy inputs; returns (path int64 array A -> X, result)."""
    import numpy as np
    path = np.zeros(max(int(cap), 1), dtype=np.int64)
    ln = ctypes.c_int64()
    res = csp_result()
    addr = lambda a: ctypes.c_void_p(a.ctypes.data)
    rc = lib.csp_reconstruct(ctx, d, n, addr(f1), addr(f2), addr(A), addr(B), M, addr(path), int(cap),
                             ctypes.byref(ln), ctypes.byref(res))
    _check(ctx, rc)
    return path[:ln.value].copy(), res


def csp_reconstruct_dev(ctx, d, n, f1, f2, A, B, M, scratch_mask, cap, stream=None):
    import numpy as np
    path = np.zeros(max(cap, 1), dtype=np.int64)
    ln = ctypes.c_int64()
    res = csp_result()
    rc = lib.csp_reconstruct_dev(ctx, d, n, _ptr(f1), _ptr(f2), _ptr(A), _ptr(B), M,
                                 _ptr(scratch_mask), ctypes.c_void_p(path.ctypes.data), cap,
                                 ctypes.byref(ln), ctypes.byref(res), _stream(stream))
    _check(ctx, rc)
    return path[:ln.value].copy(), res


def _problems(instances, labels=None):
    probs = (csp_problem * len(instances))()
    for i, di in enumerate(instances):
        probs[i] = csp_problem(di.d, di.n, di.f1.data_ptr(), di.f2.data_ptr(), di.A.data_ptr(),
                               di.B.data_ptr(), di.M,
                               labels[i].data_ptr() if labels is not None and labels[i] is not None else None)
    return probs


def csp_solve_batch(ctx, instances, labels=None, counters=True, stream=None):
    """instances: list of DeviceInstance; labels: optional list of device int32 tensors (or None)."""
    k = len(instances)
    probs = _problems(instances, labels)
    res = (csp_result * k)()
    cnt = (csp_counters * k)() if counters else None
    rc = lib.csp_solve_batch(ctx, k, ctypes.cast(probs, ctypes.c_void_p), ctypes.cast(res, ctypes.c_void_p),
                             ctypes.cast(cnt, ctypes.c_void_p) if counters else None, _stream(stream))
    _check(ctx, rc)
    return list(res), (list(cnt) if counters else None)


def csp_last_kernel_ms(ctx) -> float:
    ms = ctypes.c_float()
    _check(ctx, lib.csp_last_kernel_ms(ctx, ctypes.byref(ms)))
    return ms.value


def csp_set_pool_hint(ctx, flows_per_bucket: int):
    _check(ctx, lib.csp_set_pool_hint(ctx, flows_per_bucket))


def csp_set_blocks(ctx, blocks: int):
    _check(ctx, lib.csp_set_blocks(ctx, blocks))


def csp_set_path(ctx, path: int):
    _check(ctx, lib.csp_set_path(ctx, path))


def csp_last_path(ctx) -> int:
    return lib.csp_last_path(ctx)


def csp_autotune(ctx, d, n, f1, f2, A, B, M, stream=None):
    """Time the candidate configurations for this lattice shape and record
    the fastest on ctx; returns (blocks, path, kernel ms)."""
    b, pth, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    _check(ctx, lib.csp_autotune(ctx, d, n, _ptr(f1), _ptr(f2), _ptr(A), _ptr(B), M, ctypes.byref(b),
                                 ctypes.byref(pth), ctypes.byref(ms), _stream(stream)))
    return b.value, pth.value, ms.value


def csp_set_wait_limit(ctx, microseconds: int):
    """Barrier wait limit of later single solves (-1: the default, 20 s)."""
    _check(ctx, lib.csp_set_wait_limit(ctx, microseconds))


def csp_set_dense_threshold(ctx, flows: int):
    _check(ctx, lib.csp_set_dense_threshold(ctx, flows))


def csp_tuned_dense_threshold(ctx, d: int, n: int) -> int:
    v = ctypes.c_int64()
    _check(ctx, lib.csp_tuned_dense_threshold(ctx, d, n, ctypes.byref(v)))
    return v.value


def csp_autotune_clear(ctx):
    _check(ctx, lib.csp_autotune_clear(ctx))


def csp_set_batch_target(ctx, vertices_per_workgroup: int):
    _check(ctx, lib.csp_set_batch_target(ctx, vertices_per_workgroup))


def csp_autotune_batch(ctx, instances, stream=None):
    """Time the batch gang-size candidates on these problems and keep the
    fastest on ctx; returns (vertices per workgroup, kernel ms)."""
    probs = _problems(instances)
    tgt, ms = ctypes.c_int64(), ctypes.c_float()
    _check(ctx, lib.csp_autotune_batch(ctx, len(instances), ctypes.cast(probs, ctypes.c_void_p),
                                       ctypes.byref(tgt), ctypes.byref(ms), _stream(stream)))
    return tgt.value, ms.value


PHASES = ("departure", "barrier_after_departure", "next_time", "arrival",
          "barrier_after_arrival", "frontier_gather")


def csp_set_phase_timing(ctx, on):
    """False/0 off, True/1 workgroup 0, 2 every workgroup (csp_last_phase_spread)."""
    _check(ctx, lib.csp_set_phase_timing(ctx, int(on)))


def csp_reconstruct_log_dev(ctx, d, n, f1, f2, A, B, M, cap, stream=None):
    """Path A -> X from one logged solve; returns (path int64 array, result, counters)."""
    import numpy as np
    path = np.zeros(max(int(cap), 1), dtype=np.int64)
    ln = ctypes.c_int64()
    res = csp_result()
    cnt = csp_counters()
    rc = lib.csp_reconstruct_log_dev(ctx, d, n, _ptr(f1), _ptr(f2), _ptr(A), _ptr(B), M,
                                     path.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(ln),
                                     ctypes.byref(res), ctypes.byref(cnt), _stream(stream))
    _check(ctx, rc)
    return path[:ln.value].copy(), res, cnt


@dataclass
class DeviceGraph:
    """A general graph's adjacency arrays in device memory (torch tensors)."""
    nv: int
    off: object      # int64 [nv+1]
    nbr: object      # int32 [m]
    f1: object       # uint8 [m]
    f2: object       # uint8 [m]
    eid: object      # int64 [m]


def graph_to_device(csr, device="cuda"):
    import torch
    off, nbr, f1, f2, eid = csr
    t = lambda a: torch.from_numpy(a).to(device)
    return DeviceGraph(int(off.size - 1), t(off), t(nbr), t(f1), t(f2), t(eid))


def csp_solve_graph_dev(ctx, g: DeviceGraph, A, B, M, labels=None, max_cycles=0, counters=True, stream=None):
    res = csp_result()
    cnt = csp_counters() if counters else None
    rc = lib.csp_solve_graph_dev(ctx, g.nv, _ptr(g.off), _ptr(g.nbr), _ptr(g.f1), _ptr(g.f2), _ptr(g.eid),
                                 _ptr(A), _ptr(B), M, _ptr(labels), ctypes.byref(res),
                                 ctypes.byref(cnt) if counters else None, max_cycles, _stream(stream))
    _check(ctx, rc)
    return res, cnt


def csp_set_trace(ctx, trace=None):
    """trace: device int64 tensor of shape (cap, 4), or None to switch the trace off."""
    if trace is None:
        _check(ctx, lib.csp_set_trace(ctx, None, 0))
    else:
        assert trace.dim() == 2 and trace.shape[1] == 4 and trace.is_contiguous()
        _check(ctx, lib.csp_set_trace(ctx, ctypes.c_void_p(trace.data_ptr()), trace.shape[0]))


def csp_last_trace_rows(ctx) -> int:
    rows = ctypes.c_int64()
    _check(ctx, lib.csp_last_trace_rows(ctx, ctypes.byref(rows)))
    return rows.value


def csp_last_phase_us(ctx) -> dict:
    us = (ctypes.c_double * 6)()
    _check(ctx, lib.csp_last_phase_us(ctx, us))
    return dict(zip(PHASES, list(us)))


SPREAD_PHASES = ("send", "publish", "candidates", "deliver", "wait")


def csp_last_phase_spread(ctx) -> dict:
    """Per phase of the range-owned kernel: (mean over workgroups, largest
    workgroup) in microseconds, after a solve with phase timing 2."""
    mean, mx = (ctypes.c_double * 6)(), (ctypes.c_double * 6)()
    _check(ctx, lib.csp_last_phase_spread(ctx, mean, mx))
    slots = {"send": 0, "publish": 1, "candidates": 2, "deliver": 3, "wait": 4}
    return {k: (mean[i], mx[i]) for k, i in slots.items()}


# --- convenience ------------------------------------------------------------

@dataclass
class DeviceInstance:
    """An instance resident in device memory (torch uint8 tensors)."""
    d: int
    n: int
    f1: object
    f2: object
    A: object
    B: object
    M: int

    @property
    def N(self):
        return self.n ** self.d


def to_device(inst, device="cuda"):
    import torch
    t = lambda a: torch.from_numpy(a).to(device)
    return DeviceInstance(inst.d, inst.n, t(inst.f1), t(inst.f2), t(inst.A), t(inst.B), int(inst.M))


class Solver:
    """Owns one libcsp context on a device."""

    def __init__(self, device: int = 0):
        self.ctx = csp_create(device)
        self.device = device

    def close(self):
        if self.ctx:
            csp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, di: DeviceInstance, labels=None, M=None, max_cycles=0, stream=None):
        return csp_solve_dev(self.ctx, di.d, di.n, di.f1, di.f2, di.A, di.B,
                             di.M if M is None else M, labels=labels,
                             max_cycles=max_cycles, stream=stream)

    def autotune(self, di: DeviceInstance, stream=None):
        return csp_autotune(self.ctx, di.d, di.n, di.f1, di.f2, di.A, di.B, di.M, stream=stream)

    def reconstruct_log(self, di: DeviceInstance, cap=None, stream=None):
        cap = cap if cap is not None else min(di.M, di.N) + 1
        return csp_reconstruct_log_dev(self.ctx, di.d, di.n, di.f1, di.f2, di.A, di.B, di.M, cap, stream=stream)

    def reconstruct(self, di: DeviceInstance, scratch_mask, cap=None, stream=None):
        cap = cap if cap is not None else di.N + 1
        return csp_reconstruct_dev(self.ctx, di.d, di.n, di.f1, di.f2, di.A, di.B, di.M,
                                   scratch_mask, cap, stream=stream)


# --- serving -----------------------------------------------------------------

def csp_serve_open(ctx, arena_bytes: int, max_jobs: int):
    srv = ctypes.c_void_p()
    _check(ctx, lib.csp_serve_open(ctx, arena_bytes, max_jobs, ctypes.byref(srv)))
    return srv


def csp_serve_submit(ctx, srv, di: DeviceInstance, reconstruct=True, tag=0, M=None):
    q = csp_request(di.d, di.n, di.f1.data_ptr(), di.f2.data_ptr(), di.A.data_ptr(), di.B.data_ptr(),
                    di.M if M is None else M, 1 if reconstruct else 0, tag)
    _check(ctx, lib.csp_serve_submit(srv, ctypes.byref(q)))


@dataclass
class Completion:
    tag: int
    status: int
    res: tuple
    counters: dict
    chain_counters: dict
    solves: int
    path: list


def csp_serve_poll(ctx, srv, cap=64):
    buf = (csp_completion * cap)()
    n = ctypes.c_int()
    _check(ctx, lib.csp_serve_poll(srv, buf, cap, ctypes.byref(n)))
    out = []
    for k in range(n.value):
        c = buf[k]
        path = [c.path[i] for i in range(c.path_len)] if c.path_len > 0 else []
        out.append(Completion(c.tag, c.status, c.res.tuple(), c.cnt.asdict(), c.cnt_chain.asdict(),
                              c.solves, path))
    return out


def csp_serve_pending(srv):
    q, r = ctypes.c_int(), ctypes.c_int()
    _check(None, lib.csp_serve_pending(srv, ctypes.byref(q), ctypes.byref(r)))
    return q.value, r.value


def csp_serve_close(srv):
    _check(None, lib.csp_serve_close(srv))


class Server:
    """Continuous-batching server on one libcsp context: submit requests while
    others run, poll for completions."""

    def __init__(self, solver: Solver, arena_bytes: int = 8 << 30, max_jobs: int = 256):
        self.solver = solver
        self.srv = csp_serve_open(solver.ctx, arena_bytes, max_jobs)

    def submit(self, di: DeviceInstance, reconstruct=True, tag=0):
        csp_serve_submit(self.solver.ctx, self.srv, di, reconstruct=reconstruct, tag=tag)

    def poll(self, cap=64):
        return csp_serve_poll(self.solver.ctx, self.srv, cap)

    def pending(self):
        return csp_serve_pending(self.srv)

    def drain(self, timeout_s=120.0):
        """Poll until nothing is queued or running; returns the completions."""
        import time
        out = []
        t0 = time.perf_counter()
        while True:
            out.extend(self.poll())
            q, r = self.pending()
            if q == 0 and r == 0:
                return out
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"serving did not drain in {timeout_s} s ({q} queued, {r} running)")
            time.sleep(0.0002)

    def close(self):
        if self.srv:
            csp_serve_close(self.srv)
            self.srv = None
