"""ctypes binding of libapic.so (the C ABI in include/apic_contact.h).

Argument marshalling only: every step of the contact path runs in the HIP
library.  Importing this module on a machine without the built library
raises immediately; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapic.so")

OK = 0
E_INVALID = -1
E_NOMEM = -2
E_OUT_OF_GRID = -3
E_DEVICE = -4
E_BUDGET = -5
E_KEY_OVERFLOW = -6
E_BODY = -7
E_SCRATCH = -8
E_RESIZE = -9
E_TABLE = -10
NOALLOC_SCRATCH_BYTES = 64 << 20

# scene flags
PIC = 1
RULE_SEPARATE = 2

FP64 = 0
FP32_MIXED = 1


class Grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("h", ctypes.c_double),
                ("dims", ctypes.c_int32 * 3)]


class Report(ctypes.Structure):
    _fields_ = [("P_before", ctypes.c_double * 3), ("P_after", ctypes.c_double * 3),
                ("L_before", ctypes.c_double * 3), ("L_after", ctypes.c_double * 3),
                ("E_before", ctypes.c_double), ("E_after", ctypes.c_double),
                ("P_scale", ctypes.c_double), ("L_scale", ctypes.c_double),
                ("n_particles", ctypes.c_int64), ("n_unconstrained", ctypes.c_int64),
                ("grid_blocks", ctypes.c_int64), ("max_bodies_per_node", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Scene(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("count", ctypes.c_int64), ("grid", Grid),
                ("mu", ctypes.c_double), ("n_iter", ctypes.c_int32),
                ("n_bodies", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("accel", ctypes.c_double * 3),
                ("x_ref", ctypes.c_double * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [("item_waves_per_cu", ctypes.c_int32), ("node_wg_per_cu", ctypes.c_int32),
                ("xcd_split", ctypes.c_int32), ("p2g_group", ctypes.c_int32),
                ("p2g_pairs", ctypes.c_int32)]


class Tick(ctypes.Structure):
    _fields_ = [("resident", ctypes.c_int32), ("admitted", ctypes.c_int32),
                ("completed", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("deferred", ctypes.c_int32), ("failed", ctypes.c_int32),
                ("replayed", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("particles", ctypes.c_int64), ("footprint", ctypes.c_int64)]


# (name, restype, argtypes) of every exported entry point
P = ctypes.c_void_p
SIGNATURES = {
    "apic_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, ctypes.c_size_t]),
    "apic_destroy": (None, [P]),
    "apic_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "apic_contact_step": (ctypes.c_int, [P, P, ctypes.POINTER(Grid), ctypes.c_int64, P, P, P, P,
                                         P, ctypes.c_double, ctypes.c_int32, ctypes.c_int,
                                         ctypes.POINTER(Report)]),
    "apic_contact_step_noalloc": (ctypes.c_int, [P, P, ctypes.POINTER(Grid), ctypes.c_int64, P, P,
                                                 P, P, P, ctypes.c_double, ctypes.c_int32,
                                                 ctypes.c_int, ctypes.POINTER(Report)]),
    "apic_contact_step_batched": (ctypes.c_int, [P, P, ctypes.POINTER(Scene), ctypes.c_int32,
                                                 ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int,
                                                 ctypes.POINTER(Report)]),
    "apic_plan_create": (ctypes.c_int, [P, P, ctypes.POINTER(Scene), ctypes.c_int32,
                                        ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_double,
                                        ctypes.POINTER(P)]),
    "apic_plan_step": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, P, P]),
    "apic_plan_destroy": (None, [P]),
    "apic_sort_keys": (ctypes.c_int, [P, P, ctypes.POINTER(Scene), ctypes.c_int32,
                                      ctypes.c_int64, P, P, ctypes.c_int, P, P]),
    "apic_scene_footprint": (ctypes.c_int64, [ctypes.c_int64, ctypes.POINTER(Grid), ctypes.c_int]),
    "apic_sim_create": (ctypes.c_int, [P, P, ctypes.POINTER(Scene), ctypes.c_int32,
                                       ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int,
                                       ctypes.POINTER(P)]),
    "apic_sim_step": (ctypes.c_int, [P, P, ctypes.c_int32, ctypes.c_int32]),
    "apic_sim_read": (ctypes.c_int, [P, P, P, P, P]),
    "apic_sim_report": (ctypes.c_int, [P, ctypes.POINTER(Report), P, ctypes.POINTER(ctypes.c_int64)]),
    "apic_sim_set_profiling": (ctypes.c_int, [P, ctypes.c_int32]),
    "apic_sim_kernel_times": (ctypes.c_int, [P, P, P]),
    "apic_sim_info": (ctypes.c_int, [P, P]),
    "apic_sim_destroy": (None, [P]),
    "apic_server_create": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int64, ctypes.POINTER(P)]),
    "apic_server_submit": (ctypes.c_int, [P, ctypes.c_int64, ctypes.POINTER(Scene), ctypes.c_double,
                                          ctypes.c_int32, P, P, P, P, P, P, P, P]),
    "apic_server_tick": (ctypes.c_int, [P, P, ctypes.POINTER(Tick),
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "apic_server_cancel": (ctypes.c_int, [P, ctypes.c_int64]),
    "apic_server_destroy": (None, [P]),
    "apic_get_tuning": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(Tuning)]),
    "apic_set_tuning": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(Tuning)]),
    "apic_autotune": (ctypes.c_int, [P, P, ctypes.POINTER(Scene), ctypes.c_int32, ctypes.c_int64,
                                     P, P, P, P, P, ctypes.c_int, ctypes.c_int32,
                                     ctypes.POINTER(Tuning), ctypes.POINTER(Tuning),
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)]),
}

# kernel classes reported by apic_sim_kernel_times
KERNEL_CLASSES = ["layout", "sort", "gather", "segments", "mass", "p2g0", "gridvel", "round1",
                  "round", "final", "after"]

_lib = None


class ApicError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        msg = lib().apic_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


def lib():
    """Load libapic.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int, where: str):
    if rc != OK:
        raise ApicError(rc, where)


def make_grid(h: float, origin=(0.0, 0.0, 0.0), dims=(0, 0, 0)) -> Grid:
    g = Grid()
    g.origin[:] = [float(o) for o in origin]
    g.h = float(h)
    g.dims[:] = [int(d) for d in dims]
    return g


def report_dict(r: Report) -> dict:
    return {"P_before": list(r.P_before), "P_after": list(r.P_after),
            "L_before": list(r.L_before), "L_after": list(r.L_after),
            "E_before": r.E_before, "E_after": r.E_after, "P_scale": r.P_scale,
            "L_scale": r.L_scale, "n_particles": r.n_particles,
            "n_unconstrained": r.n_unconstrained, "grid_blocks": r.grid_blocks,
            "max_bodies_per_node": r.max_bodies_per_node}


def tuning_dict(t: Tuning) -> dict:
    return {"item_waves_per_cu": t.item_waves_per_cu, "node_wg_per_cu": t.node_wg_per_cu,
            "xcd_split": t.xcd_split, "p2g_group": t.p2g_group, "p2g_pairs": t.p2g_pairs}


def make_tuning(d: dict) -> Tuning:
    t = Tuning()
    for k in ("item_waves_per_cu", "node_wg_per_cu", "xcd_split", "p2g_group"):
        setattr(t, k, int(d[k]))
    t.p2g_pairs = int(d.get("p2g_pairs", 0))  # absent from tunings recorded before the knob
    return t
