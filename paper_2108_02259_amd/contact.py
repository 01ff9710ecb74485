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

    def contact_step_batched(self, scenes, x, v, C, m, body, report=True):
        """scenes: list of dicts with offset, count, h, origin, dims, mu, n_iter, n_bodies."""
        n = _check_tensors(x, v, C, m, body)
        arr = (_lib.Scene * len(scenes))()
        for i, s in enumerate(scenes):
            arr[i].offset = int(s["offset"])
            arr[i].count = int(s["count"])
            arr[i].grid = make_grid(s["h"], s.get("origin", (0, 0, 0)), s.get("dims", (0, 0, 0)))
            arr[i].mu = float(s["mu"])
            arr[i].n_iter = int(s["n_iter"])
            arr[i].n_bodies = int(s["n_bodies"])
        reps = (_lib.Report * len(scenes))()
        rc = lib().apic_contact_step_batched(self._h, _stream(), arr, len(scenes), n, _ptr(x),
                                             _ptr(v), _ptr(C), _ptr(m), _ptr(body),
                                             precision_of(x), reps if report else None)
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
        arr = (_lib.Scene * len(scenes))()
        for i, s in enumerate(scenes):
            arr[i].offset = int(s["offset"])
            arr[i].count = int(s["count"])
            arr[i].grid = make_grid(s["h"], s.get("origin", (0, 0, 0)), s.get("dims", (0, 0, 0)))
            arr[i].mu = float(s.get("mu", 0.0))
            arr[i].n_iter = int(s.get("n_iter", 0))
            arr[i].n_bodies = int(s["n_bodies"])
        keys = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)
        rc = lib().apic_sort_keys(self._h, _stream(), arr, len(scenes), n, _ptr(x), _ptr(body),
                                  precision_of(x), _ptr(keys), _ptr(perm))
        check(rc, "apic_sort_keys")
        mask = (1 << 32) - 1
        return (keys[:n].to(torch.int64) & mask), (perm[:n].to(torch.int64) & mask)


def scene_table(scenes):
    arr = (_lib.Scene * len(scenes))()
    for i, s in enumerate(scenes):
        arr[i].offset = int(s["offset"])
        arr[i].count = int(s["count"])
        arr[i].grid = make_grid(s["h"], s.get("origin", (0, 0, 0)), s.get("dims", (0, 0, 0)))
        arr[i].mu = float(s.get("mu", 0.0))
        arr[i].n_iter = int(s.get("n_iter", 0))
        arr[i].n_bodies = int(s["n_bodies"])
    return arr


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


def footprint(n: int, blocks_hint: int = 0, precision: int = _lib.FP32_MIXED) -> int:
    return int(lib().apic_scene_footprint(int(n), int(blocks_hint), int(precision)))


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
        """One tick; returns (info dict, [completed tags])."""
        t = _lib.Tick()
        check(lib().apic_server_tick(self._h, _stream(), ctypes.byref(t), self._done,
                                     len(self._done)), "apic_server_tick")
        done = [int(self._done[i]) for i in range(min(t.completed, len(self._done)))]
        for tag in done:
            self._keep.pop(tag, None)
        info = {"resident": t.resident, "admitted": t.admitted, "completed": t.completed,
                "queued": t.queued, "particles": t.particles, "footprint": t.footprint}
        return info, done

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
