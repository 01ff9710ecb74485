"""Python front end of the contact library: torch tensors in, C ABI calls out.

Tensors are device tensors in the library's layout: x, v of shape (3, n),
C of shape (9, n), m of shape (n,) -- float64 for the FP64 path, float32
for the mixed path -- and body ids as an (n,) int16/uint16 tensor whose bits
are the uint16 ids.  PyTorch supplies memory and the current stream; all
arithmetic runs in libapic.so.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check, lib, make_grid


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _prec_of_dtype(dtype) -> int:
    if dtype in (torch.float64, "float64") or getattr(dtype, "__name__", "") == "float64":
        return _lib.FP64
    if dtype in (torch.float32, "float32") or getattr(dtype, "__name__", "") == "float32":
        return _lib.FP32_MIXED
    raise TypeError(f"unsupported dtype {dtype}")


def precision_of(x: torch.Tensor) -> int:
    if x.dtype == torch.float64:
        return _lib.FP64
    if x.dtype == torch.float32:
        return _lib.FP32_MIXED
    raise TypeError(f"unsupported dtype {x.dtype}")


def _check_tensors(x, v, C, m, body):
    n = x.shape[1]
    dt = x.dtype
    for name, t, shape in (("x", x, (3, n)), ("v", v, (3, n)), ("C", C, (9, n)), ("m", m, (n,))):
        if tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name}: expected contiguous {dt} cuda tensor of shape {shape}")
    if tuple(body.shape) != (n,) or body.element_size() != 2 or not body.is_contiguous():
        raise ValueError("body: expected contiguous 16-bit tensor of shape (n,)")
    return n


class Context:
    """One library context (workspace arena) on a device."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self._h = ctypes.c_void_p()
        check(lib().apic_create(ctypes.byref(self._h), int(device), int(budget_bytes)),
              "apic_create")
        self.device = device

    def close(self):
        if self._h:
            lib().apic_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def contact_step(self, x, v, C, m, body, h, origin=(0.0, 0.0, 0.0), dims=(0, 0, 0),
                     mu=0.0, n_iter=1, report=True):
        """Overwrite v and C with the preferred generalized velocity S(v, C)."""
        n = _check_tensors(x, v, C, m, body)
        g = make_grid(h, origin, dims)
        rep = _lib.Report()
        rc = lib().apic_contact_step(self._h, _stream(), ctypes.byref(g), n, _ptr(x), _ptr(v),
                                     _ptr(C), _ptr(m), _ptr(body), float(mu), int(n_iter),
                                     precision_of(x), ctypes.byref(rep) if report else None)
        check(rc, "apic_contact_step")
        return _lib.report_dict(rep) if report else None

    def contact_step_noalloc(self, x, v, C, m, body, h, origin=(0.0, 0.0, 0.0),
                             dims=(0, 0, 0), mu=0.0, n_iter=1, report=True):
        """contact_step through the allocation-free entry point (the library's
        fixed per-GPU scratch; no device allocation by the call)."""
        n = _check_tensors(x, v, C, m, body)
        g = make_grid(h, origin, dims)
        rep = _lib.Report()
        rc = lib().apic_contact_step_noalloc(self._h, _stream(), ctypes.byref(g), n, _ptr(x),
                                             _ptr(v), _ptr(C), _ptr(m), _ptr(body), float(mu),
                                             int(n_iter), precision_of(x),
                                             ctypes.byref(rep) if report else None)
        check(rc, "apic_contact_step_noalloc")
        return _lib.report_dict(rep) if report else None

    def contact_step_batched(self, scenes, x, v, C, m, body, normals=None, report=True):
        """scenes: list of dicts with offset, count, h, origin, dims, mu, n_iter,
        n_bodies and optionally flags, accel, x_ref (see scene_table).
        normals: optional (3, n) tensor of the caller's particle normals."""
        n = _check_tensors(x, v, C, m, body)
        if normals is not None and (tuple(normals.shape) != (3, n) or normals.dtype != x.dtype
                                    or not normals.is_contiguous()):
            raise ValueError("normals: expected a contiguous (3, n) tensor of x's dtype")
        arr = scene_table(scenes)
        reps = (_lib.Report * len(scenes))()
        rc = lib().apic_contact_step_batched(self._h, _stream(), arr, len(scenes), n, _ptr(x),
                                             _ptr(v), _ptr(C), _ptr(m), _ptr(body),
                                             _ptr(normals), precision_of(x),
                                             reps if report else None)
        check(rc, "apic_contact_step_batched")
        return [_lib.report_dict(r) for r in reps] if report else None

    # ---- launch tuning --------------------------------------------------
    def get_tuning(self, dtype, n: int) -> dict:
        t = _lib.Tuning()
        check(lib().apic_get_tuning(self._h, _prec_of_dtype(dtype), int(n), ctypes.byref(t)),
              "apic_get_tuning")
        return _lib.tuning_dict(t)

    def set_tuning(self, dtype, n: int, tuning: dict):
        t = _lib.make_tuning(tuning)
        check(lib().apic_set_tuning(self._h, _prec_of_dtype(dtype), int(n), ctypes.byref(t)),
              "apic_set_tuning")

    def autotune(self, scenes, x, v, C, m, body, reps: int = 2):
        """Time every candidate launch tuning on this batch (inputs are only
        read) and keep the fastest for its (precision, size bucket).  Returns
        (best, [(candidate, ms per step), ...])."""
        n = _check_tensors(x, v, C, m, body)
        arr = scene_table(scenes)
        cap = 64
        cands = (_lib.Tuning * cap)()
        times = (ctypes.c_double * cap)()
        best = _lib.Tuning()
        ntried = ctypes.c_int32()
        check(lib().apic_autotune(self._h, _stream(), arr, len(scenes), n, _ptr(x), _ptr(v),
                                  _ptr(C), _ptr(m), _ptr(body), precision_of(x), int(reps),
                                  ctypes.byref(best), cands, times, cap, ctypes.byref(ntried)),
              "apic_autotune")
        k = min(ntried.value, cap)
        return (_lib.tuning_dict(best),
                [(_lib.tuning_dict(cands[i]), times[i]) for i in range(k)])

    def sort_keys(self, scenes, x, body):
        """(sorted keys, permutation) as int64 cuda tensors."""
        n = x.shape[1]
        arr = scene_table(scenes)
        keys = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
        rc = lib().apic_sort_keys(self._h, _stream(), arr, len(scenes), n, _ptr(x), _ptr(body),
                                  precision_of(x), _ptr(keys), _ptr(perm))
        check(rc, "apic_sort_keys")
        mask = (1 << 32) - 1
        return (keys[:n].to(torch.int64) & mask), (perm[:n].to(torch.int64) & mask)


def scene_table(scenes):
    """The ABI scene table of a list of dicts: offset, count, h, n_bodies and
    optionally origin, dims, mu, n_iter, flags (PIC | RULE_SEPARATE), accel
    (the resident driver's mechanical acceleration) and x_ref (reference
    point of the reported L; default the grid origin)."""
    arr = (_lib.Scene * len(scenes))()
    for i, s in enumerate(scenes):
        origin = s.get("origin", (0, 0, 0))
        arr[i].offset = int(s["offset"])
        arr[i].count = int(s["count"])
        arr[i].grid = make_grid(s["h"], origin, s.get("dims", (0, 0, 0)))
        arr[i].mu = float(s.get("mu", 0.0))
        arr[i].n_iter = int(s.get("n_iter", 0))
        arr[i].n_bodies = int(s["n_bodies"])
        arr[i].flags = int(s.get("flags", 0))
        arr[i].reserved = 0
        arr[i].accel[:] = [float(a) for a in s.get("accel", (0.0, 0.0, 0.0))]
        arr[i].x_ref[:] = [float(a) for a in s.get("x_ref", origin)]
    return arr


class Plan:
    """A planned contact step (apic_plan_*): the batch is measured once, then
    step() only enqueues on the current stream (no host synchronisation), so
    it can be captured into a CUDA/HIP graph."""

    def __init__(self, ctx: Context, scenes, x, body, headroom: float = 1.5):
        self.n = x.shape[1]
        self.ns = len(scenes)
        self.dtype = x.dtype
        self._ctx = ctx
        self._h = ctypes.c_void_p()
        arr = scene_table(scenes)
        check(lib().apic_plan_create(ctx._h, _stream(), arr, self.ns, self.n, _ptr(x), _ptr(body),
                                     precision_of(x), float(headroom), ctypes.byref(self._h)),
              "apic_plan_create")

    def step(self, x, v, C, m, body, normals=None, scenes_dev=None, reports_dev=None,
             status_dev=None):
        """Enqueue one step.  scenes_dev: optional uint8 device tensor holding
        an ABI scene table; reports_dev: optional uint8 device tensor of
        n_scenes reports; status_dev: optional int32 device tensor."""
        if _check_tensors(x, v, C, m, body) != self.n or x.dtype != self.dtype:
            raise ValueError("tensors do not match the plan")
        check(lib().apic_plan_step(self._h, _stream(), _ptr(scenes_dev), _ptr(x), _ptr(v),
                                   _ptr(C), _ptr(m), _ptr(body), _ptr(normals),
                                   _ptr(reports_dev), _ptr(status_dev)), "apic_plan_step")

    def close(self):
        if self._h:
            lib().apic_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reports_from_bytes(buf, ns):
    """Report dicts from the bytes of n_scenes device reports (a uint8 CPU
    tensor or bytes)."""
    raw = bytes(buf.numpy().tobytes() if hasattr(buf, "numpy") else buf)
    arr = (_lib.Report * ns).from_buffer_copy(raw[:ctypes.sizeof(_lib.Report) * ns])
    return [_lib.report_dict(r) for r in arr]


def scene_table_bytes(scenes) -> bytes:
    """The ABI scene table as bytes (to upload as a device table)."""
    arr = scene_table(scenes)
    return bytes(memoryview(arr).cast("B"))


class Sim:
    """Resident time stepping of a packed batch (apic_sim_*): each step sets
    V <- S(V) and then x <- x + dt v, with state kept in HBM."""

    def __init__(self, ctx: Context, scenes, dt, x, v, C, m, body):
        n = _check_tensors(x, v, C, m, body)
        self.n = n
        self.ns = len(scenes)
        self.dtype = x.dtype
        self.device = x.device
        arr = scene_table(scenes)
        dts = (ctypes.c_double * self.ns)(*[float(d) for d in dt])
        self._h = ctypes.c_void_p()
        self._ctx = ctx
        check(lib().apic_sim_create(ctx._h, _stream(), arr, self.ns, n, dts, _ptr(x), _ptr(v),
                                    _ptr(C), _ptr(m), _ptr(body), precision_of(x),
                                    ctypes.byref(self._h)), "apic_sim_create")

    def step(self, n_steps: int = 1, graph: bool = False):
        check(lib().apic_sim_step(self._h, _stream(), int(n_steps), int(bool(graph))),
              "apic_sim_step")

    def read(self):
        x = torch.empty((3, self.n), dtype=self.dtype, device=self.device)
        v = torch.empty((3, self.n), dtype=self.dtype, device=self.device)
        C = torch.empty((9, self.n), dtype=self.dtype, device=self.device)
        check(lib().apic_sim_read(self._h, _stream(), _ptr(x), _ptr(v), _ptr(C)), "apic_sim_read")
        return x, v, C

    def report(self):
        reps = (_lib.Report * self.ns)()
        drift = (ctypes.c_double * (2 * self.ns))()
        steps = ctypes.c_int64()
        check(lib().apic_sim_report(self._h, reps, ctypes.cast(drift, ctypes.c_void_p),
                                    ctypes.byref(steps)), "apic_sim_report")
        return ([_lib.report_dict(r) for r in reps],
                [(drift[2 * s], drift[2 * s + 1]) for s in range(self.ns)], steps.value)

    def profiling(self, on: bool):
        check(lib().apic_sim_set_profiling(self._h, int(bool(on))), "apic_sim_set_profiling")

    def kernel_times(self):
        """{class: (total ms, launches)} since the last call."""
        ms = (ctypes.c_double * len(_lib.KERNEL_CLASSES))()
        cnt = (ctypes.c_int64 * len(_lib.KERNEL_CLASSES))()
        check(lib().apic_sim_kernel_times(self._h, ctypes.cast(ms, ctypes.c_void_p),
                                          ctypes.cast(cnt, ctypes.c_void_p)),
              "apic_sim_kernel_times")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KERNEL_CLASSES)}

    def info(self):
        out = (ctypes.c_int64 * 8)()
        check(lib().apic_sim_info(self._h, ctypes.cast(out, ctypes.c_void_p)), "apic_sim_info")
        return {"n": out[0], "shared_blocks": out[1], "body_blocks": out[2], "segments": out[3],
                "items": out[4], "sort_bits": out[5], "bytes": out[6]}

    def close(self):
        if self._h:
            lib().apic_sim_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(n: int, h: float = 1.0, origin=(0.0, 0.0, 0.0), dims=(0, 0, 0),
              precision: int = _lib.FP32_MIXED) -> int:
    g = make_grid(h, origin, dims)
    return int(lib().apic_scene_footprint(int(n), ctypes.byref(g), int(precision)))


class Server:
    """Continuous-batching request loop (apic_server_*): requests join as
    arena room, scene slots and the footprint budget allow, all resident
    requests advance one driver step per tick, and finished ones are copied
    to their output tensors."""

    def __init__(self, ctx: Context, dtype, max_particles: int, max_scenes: int,
                 budget_bytes: int = 0):
        self._h = ctypes.c_void_p()
        self._ctx = ctx
        self.prec = _prec_of_dtype(dtype)
        self._keep = {}  # tag -> tensors that must outlive the request
        check(lib().apic_server_create(ctx._h, self.prec, int(max_particles), int(max_scenes),
                                       int(budget_bytes), ctypes.byref(self._h)),
              "apic_server_create")
        self._done = (ctypes.c_int64 * 4096)()
        self._status = (ctypes.c_int32 * 4096)()
        self.failed = {}  # tag -> status of requests retired with an error

    def submit(self, tag: int, scene: dict, dt: float, steps: int, x, v, C, m, body,
               x_out, v_out, C_out):
        n = _check_tensors(x, v, C, m, body)
        for name, t, shape in (("x_out", x_out, (3, n)), ("v_out", v_out, (3, n)),
                               ("C_out", C_out, (9, n))):
            if tuple(t.shape) != shape or t.dtype != x.dtype or not t.is_contiguous():
                raise ValueError(f"{name}: expected contiguous {x.dtype} tensor {shape}")
        if precision_of(x) != self.prec:
            raise TypeError("request dtype differs from the server's")
        sc = scene_table([dict(scene, offset=0, count=n)])
        rc = lib().apic_server_submit(self._h, int(tag), sc, float(dt), int(steps), _ptr(x),
                                      _ptr(v), _ptr(C), _ptr(m), _ptr(body), _ptr(x_out),
                                      _ptr(v_out), _ptr(C_out))
        check(rc, "apic_server_submit")
        self._keep[int(tag)] = (x, v, C, m, body, x_out, v_out, C_out)

    def tick(self):
        """One tick; returns (info dict, [completed tags]).  Requests retired
        with an error are recorded in self.failed (tag -> status)."""
        t = _lib.Tick()
        check(lib().apic_server_tick(self._h, _stream(), ctypes.byref(t), self._done,
                                     self._status, len(self._done)), "apic_server_tick")
        done = []
        for i in range(min(t.completed + t.failed, len(self._done))):
            tag, st = int(self._done[i]), int(self._status[i])
            self._keep.pop(tag, None)
            if st == _lib.OK:
                done.append(tag)
            else:
                self.failed[tag] = st
        info = {"resident": t.resident, "admitted": t.admitted, "completed": t.completed,
                "queued": t.queued, "deferred": t.deferred, "failed": t.failed,
                "replayed": t.replayed, "particles": t.particles, "footprint": t.footprint}
        return info, done

    def cancel(self, tag: int):
        check(lib().apic_server_cancel(self._h, int(tag)), "apic_server_cancel")
        self._keep.pop(int(tag), None)

    def close(self):
        if self._h:
            lib().apic_server_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
