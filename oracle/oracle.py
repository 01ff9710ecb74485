"""ctypes binding of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

The oracle (``apic_oracle.c``) is a plain, slow FP64 CPU implementation of
the APIC augury contact step (arXiv 2108.02259, Sections 2.1.2-2.4 and
Appendices A-B).  It is the reference every GPU result is checked against.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the GPU library never does, and this
module imports nothing from the GPU package.

Array conventions: float64, structure-of-arrays, shape (3, n) for positions
and velocities, (9, n) for the affine matrix C (row-major C_ab per particle),
(n,) for masses and uint16 body ids.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
E_INVALID = -1
E_NOMEM = -2
E_OUT_OF_GRID = -3
E_KEY_OVERFLOW = -6

KERNEL_QUAD = 0
KERNEL_LINEAR = 1
TRANSFER_APIC = 0
TRANSFER_PIC = 1
RULE_COULOMB = 0
RULE_SEPARATE = 1


def build() -> str:
    """Compile the oracle with gcc (plain C11, -O2)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("transfer", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("h", ctypes.c_double),
                ("dims", ctypes.c_int32 * 3)]


@dataclass
class Grid:
    """Background grid: node j sits at origin + h*j; dims > 0 means dense."""
    h: float
    origin: tuple = (0.0, 0.0, 0.0)
    dims: tuple = (0, 0, 0)
    dim: int = 3
    kernel: int = KERNEL_QUAD
    transfer: int = TRANSFER_APIC
    rule: int = RULE_COULOMB

    def c(self) -> _Grid:
        g = _Grid()
        g.dim, g.kernel, g.transfer, g.rule = self.dim, self.kernel, self.transfer, self.rule
        g.origin[:] = [float(o) for o in self.origin]
        g.h = float(self.h)
        g.dims[:] = [int(d) for d in self.dims]
        return g


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.ora_shape_1d.argtypes = [ctypes.c_int32, ctypes.c_double, P, P, P]
        L.ora_inertia.argtypes = [P, P, P]
        L.ora_apply_H.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P]
        L.ora_normals.argtypes = [P, ctypes.c_int64, P, P, P, P, P]
        L.ora_undesirable.argtypes = [ctypes.c_int32, P, P, ctypes.c_double, P]
        L.ora_contact_step.argtypes = [P, ctypes.c_int64, P, P, P, P, P,
                                       ctypes.c_double, ctypes.c_int32, P, P, P, P]
        L.ora_momentum.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, P, P]
        L.ora_cell_keys.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32, P,
                                    ctypes.c_int64, P, P, P]
        for f in ("ora_shape_1d", "ora_inertia", "ora_apply_H", "ora_normals",
                  "ora_undesirable", "ora_contact_step", "ora_momentum", "ora_cell_keys"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned status {code}")
        self.code = code


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check(rc: int):
    if rc != OK:
        raise OracleError(rc)


def shape_1d(kernel: int, xi: float):
    """(first node, weights, d weights / d xi) of the 1-D basis at xi."""
    first = ctypes.c_int64()
    w = np.zeros(4)
    dw = np.zeros(4)
    cnt = lib().ora_shape_1d(kernel, float(xi), ctypes.byref(first), _ptr(w), _ptr(dw))
    return first.value, w[:cnt].copy(), dw[:cnt].copy()


def inertia(grid: Grid, xp) -> np.ndarray:
    """D_p from its definition, as a 3x3 matrix."""
    g = grid.c()
    xp = _f64(xp, (3,))
    D = np.zeros(9)
    _check(lib().ora_inertia(ctypes.byref(g), _ptr(xp), _ptr(D)))
    return D.reshape(3, 3)


def apply_H(grid: Grid, x, m, u, E):
    """One application of the transfer operator H to U = {u, E}."""
    x = _f64(x)
    n = x.shape[1]
    m, u, E = _f64(m, (n,)), _f64(u, (3, n)), _f64(E, (9, n))
    uo = np.zeros((3, n))
    Eo = np.zeros((9, n))
    g = grid.c()
    _check(lib().ora_apply_H(ctypes.byref(g), n, _ptr(x), _ptr(m), _ptr(u), _ptr(E),
                             _ptr(uo), _ptr(Eo)))
    return uo, Eo


def normals(grid: Grid, x, m, body):
    x = _f64(x)
    n = x.shape[1]
    m = _f64(m, (n,))
    body = np.ascontiguousarray(body, dtype=np.uint16)
    nrm = np.zeros((3, n))
    unc = np.zeros(n, dtype=np.int32)
    g = grid.c()
    _check(lib().ora_normals(ctypes.byref(g), n, _ptr(x), _ptr(m), _ptr(body),
                             _ptr(nrm), _ptr(unc)))
    return nrm, unc


def undesirable(rule: int, d, nrm, mu: float) -> np.ndarray:
    d = _f64(d, (3,))
    nrm = _f64(nrm, (3,))
    out = np.zeros(3)
    _check(lib().ora_undesirable(rule, _ptr(d), _ptr(nrm), float(mu), _ptr(out)))
    return out


def contact_step(grid: Grid, x, v, C, m, body, mu: float, n_iter: int,
                 want_normals=False, want_w1=False, normals_in=None):
    """The contact step S: returns dict(v, C[, normals, unconstrained][, w1]).
    normals_in (3, n), optional: the caller's particle normals (zero =
    unconstrained) instead of the body-mass-gradient normals."""
    x = _f64(x)
    n = x.shape[1]
    nin = None if normals_in is None else _f64(normals_in, (3, n))
    v = _f64(v, (3, n)).copy()
    C = _f64(C, (9, n)).copy()
    m = _f64(m, (n,))
    body = np.ascontiguousarray(body, dtype=np.uint16)
    nrm = np.zeros((3, n)) if want_normals else None
    unc = np.zeros(n, dtype=np.int32) if want_normals else None
    w1 = np.zeros((12, n)) if want_w1 else None
    g = grid.c()
    _check(lib().ora_contact_step(ctypes.byref(g), n, _ptr(x), _ptr(v), _ptr(C), _ptr(m),
                                  _ptr(body), float(mu), int(n_iter), _ptr(nin), _ptr(nrm),
                                  _ptr(w1), _ptr(unc)))
    out = {"v": v, "C": C}
    if want_normals:
        out["normals"] = nrm
        out["unconstrained"] = unc
    if want_w1:
        out["w1"] = w1
    return out


def momentum(x, v, C, m, h: float, xref=(0.0, 0.0, 0.0)):
    """dict(P, L, E, P_scale, L_scale) with the affine spin term in L and E."""
    x = _f64(x)
    n = x.shape[1]
    v, C, m = _f64(v, (3, n)), _f64(C, (9, n)), _f64(m, (n,))
    xr = _f64(xref, (3,))
    out = np.zeros(9)
    _check(lib().ora_momentum(n, _ptr(x), _ptr(v), _ptr(C), _ptr(m), float(h), _ptr(xr),
                              _ptr(out)))
    return {"P": out[0:3].copy(), "L": out[3:6].copy(), "E": float(out[6]),
            "P_scale": float(out[7]), "L_scale": float(out[8])}


@dataclass
class Scene:
    """One scene of a packed batch: particles [offset, offset+count)."""
    offset: int
    count: int
    grid: Grid
    n_bodies: int
    extra: dict = field(default_factory=dict)


def cell_keys(scenes, x, body):
    """Cell keys (input order) and the stable sorting permutation."""
    x = _f64(x)
    n = x.shape[1]
    body = np.ascontiguousarray(body, dtype=np.uint16)
    ns = len(scenes)
    grids = (_Grid * max(ns, 1))()
    for i, s in enumerate(scenes):
        grids[i] = s.grid.c()
    offs = np.array([s.offset for s in scenes], dtype=np.int64)
    cnts = np.array([s.count for s in scenes], dtype=np.int64)
    bases = np.zeros(max(ns, 1), dtype=np.int32)
    tot = 0
    for i, s in enumerate(scenes):
        bases[i] = tot
        tot += s.n_bodies
    keys = np.zeros(n, dtype=np.uint32)
    perm = np.zeros(n, dtype=np.uint32)
    _check(lib().ora_cell_keys(ns, grids, _ptr(offs), _ptr(cnts), _ptr(bases), tot,
                               _ptr(x), n, _ptr(body), _ptr(keys), _ptr(perm)))
    return keys, perm
