"""Seeded synthetic scenes for the contact step.

This module only builds inputs: particle positions, velocities, affine
matrices, masses, body ids and grid specifications.  It contains none of
the contact method's arithmetic, so the GPU path and the CPU oracle can both
be fed from it.

The paper's experiments use finite-element meshes that are not available;
the scenes below are lattice-sampled solids of the same kind (boundary and
interior nodes treated as particles), with the shapes and sizes of the
workloads this library is measured on:

* ``two_cubes``      -- two 12^3-particle unit cubes colliding head-on
                        (dense grid, FP64, mu = 0, 3 iterations);
* ``slab_block``     -- a 64x64x16 block sliding on a 256x256x16 slab
                        (1,114,112 particles, sparse grid, 4 iterations);
* ``spheres``        -- 256 lattice spheres of radius 8h with random
                        translation and spin (about 5.5e5 particles);
* ``batch_scenes``   -- many independent two-body scenes of log-uniform size;
* ``request_stream`` -- Poisson arrivals of two- or three-body scenes.

Every generator takes a seed and uses ``numpy.random.default_rng``.  All
arrays are float64 structure-of-arrays: x, v of shape (3, n), C of shape
(9, n) (row-major C_ab per particle), m of shape (n,), body of shape (n,)
uint16.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2108_02259


@dataclass
class Scene:
    x: np.ndarray
    v: np.ndarray
    C: np.ndarray
    m: np.ndarray
    body: np.ndarray
    h: float
    origin: tuple = (0.0, 0.0, 0.0)
    dims: tuple = (0, 0, 0)
    mu: float = 0.0
    n_iter: int = 4
    dt: float = 0.0
    steps: int = 1
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_bodies(self) -> int:
        return int(self.body.max()) + 1 if self.n else 0

    def copy(self) -> "Scene":
        return Scene(self.x.copy(), self.v.copy(), self.C.copy(), self.m.copy(),
                     self.body.copy(), self.h, tuple(self.origin), tuple(self.dims),
                     self.mu, self.n_iter, self.dt, self.steps, self.name, dict(self.meta))


def lattice_box(nx: int, ny: int, nz: int, spacing: float, corner, rng, jitter: float):
    """Points corner + spacing*(i, j, k), i < nx ..., plus uniform jitter."""
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([i.ravel(), j.ravel(), k.ravel()]).astype(np.float64) * spacing
    pts += np.asarray(corner, dtype=np.float64).reshape(3, 1)
    if jitter > 0:
        pts += rng.uniform(-jitter, jitter, size=pts.shape)
    return pts


def lattice_ball(radius: float, spacing: float, centre, rng, jitter: float):
    """Lattice points centre + spacing*(i, j, k) within `radius`, plus jitter."""
    r = int(math.floor(radius / spacing))
    g = np.arange(-r, r + 1)
    i, j, k = np.meshgrid(g, g, g, indexing="ij")
    off = np.stack([i.ravel(), j.ravel(), k.ravel()]).astype(np.float64) * spacing
    keep = (off ** 2).sum(0) <= radius * radius + 1e-12
    pts = off[:, keep] + np.asarray(centre, dtype=np.float64).reshape(3, 1)
    if jitter > 0:
        pts += rng.uniform(-jitter, jitter, size=pts.shape)
    return pts


def skew(w) -> np.ndarray:
    """Row-major 3x3 matrix [w]_x (the velocity gradient of a rigid spin)."""
    wx, wy, wz = w
    return np.array([0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0])


def _assemble(parts, h, **kw) -> Scene:
    xs, vs, Cs, ms, bs = zip(*parts)
    return Scene(np.concatenate(xs, 1), np.concatenate(vs, 1), np.concatenate(Cs, 1),
                 np.concatenate(ms), np.concatenate(bs).astype(np.uint16), h, **kw)


def _body(pts, vel, Cmat, mass, bid):
    n = pts.shape[1]
    v = np.repeat(np.asarray(vel, dtype=np.float64).reshape(3, 1), n, 1)
    C = np.repeat(np.asarray(Cmat, dtype=np.float64).reshape(9, 1), n, 1)
    return pts, v, C, np.full(n, float(mass)), np.full(n, bid, dtype=np.uint16)


def snap_dense_grid(x: np.ndarray, h: float, halo: int = 3):
    """Dense grid spec covering the particles' box plus `halo` nodes per side,
    with the origin on the h-lattice (so cell keys do not shift)."""
    lo = np.floor(x.min(1) / h) - halo
    hi = np.floor(x.max(1) / h) + halo + 1
    origin = tuple(float(v) for v in lo * h)
    dims = tuple(int(v) for v in (hi - lo + 1))
    return origin, dims


def two_cubes(seed: int = SEED_BASE + 1, n_side: int = 12, jitter_frac: float = 0.1) -> Scene:
    """Two unit cubes, each an n_side^3 lattice spanning [0, 1]^3, uniform
    density 1 (mass 1/n_side^3 each), closing head-on at +-1 along x with the
    facing particle planes half a grid cell apart.  Grid h = 1/16, dense,
    snapped to the particles' box plus a 3-node halo."""
    rng = np.random.default_rng(seed)
    h = 1.0 / 16.0
    sp = 1.0 / (n_side - 1)
    jit = jitter_frac * h
    a = lattice_box(n_side, n_side, n_side, sp, (0.0, 0.0, 0.0), rng, jit)
    b = lattice_box(n_side, n_side, n_side, sp, (1.0 + 0.5 * h, 0.0, 0.0), rng, jit)
    mass = 1.0 / n_side ** 3
    sc = _assemble([_body(a, (1, 0, 0), np.zeros(9), mass, 0),
                    _body(b, (-1, 0, 0), np.zeros(9), mass, 1)], h,
                   mu=0.0, n_iter=3, dt=0.2 * h, steps=200, name="two_cubes")
    sc.origin, sc.dims = snap_dense_grid(sc.x, h)
    return sc


def slab_block(seed: int = SEED_BASE + 2, mu: float = 0.3, slab=(256, 256, 16),
               block=(64, 64, 16), jitter_frac: float = 0.1, n_iter: int = 4) -> Scene:
    """A block of block[0] x block[1] x block[2] particles on a slab of
    slab[0] x slab[1] x slab[2] particles, lattice spacing h = 1 at cell
    centres, density 1 (m = h^3).  The block is centred over the slab with
    its bottom particle plane 0.5 h above the slab's top plane and moves at
    (2, 0, -0.5); the slab is at rest.  Sparse grid, origin 0."""
    rng = np.random.default_rng(seed)
    h = 1.0
    jit = jitter_frac * h
    s = lattice_box(*slab, h, (0.5, 0.5, 0.5), rng, jit)
    bx = 0.5 + (slab[0] - block[0]) // 2
    by = 0.5 + (slab[1] - block[1]) // 2
    bz = 0.5 + (slab[2] - 1) + 0.5         # 0.5 h above the slab's top plane
    b = lattice_box(*block, h, (bx, by, bz), rng, jit)
    vb = np.array([2.0, 0.0, -0.5])
    sc = _assemble([_body(s, (0, 0, 0), np.zeros(9), h ** 3, 0),
                    _body(b, vb, np.zeros(9), h ** 3, 1)], h,
                   mu=mu, n_iter=n_iter, dt=0.2 * h / float(np.linalg.norm(vb)),
                   steps=1000, name="slab_block")
    return sc


def spheres(seed: int = SEED_BASE + 3, n_spheres: int = 256, radius_cells: float = 8.0,
            box_cells: float = 256.0, jitter_frac: float = 0.1) -> Scene:
    """n_spheres lattice balls of radius 8h placed by random sequential
    packing in a box of 256 h with surface gaps of at least h; centre
    velocities ~ N(0, 1)^3, spins ~ N(0, 0.5^2)^3, so v_p = v_c + w x (x_p - c)
    and C_p = [w]_x.  Body ids 0..n_spheres-1, mu = 0.4, 6 iterations."""
    rng = np.random.default_rng(seed)
    h = 1.0
    r = radius_cells * h
    centres = []
    lo, hi = r + h, box_cells * h - r - h
    tries = 0
    while len(centres) < n_spheres:
        c = rng.uniform(lo, hi, size=3)
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("sphere packing did not converge")
        if all(np.linalg.norm(c - o) >= 2 * r + h for o in centres):
            centres.append(c)
    parts = []
    vmax = 0.0
    for bid, c in enumerate(centres):
        pts = lattice_ball(r, h, c, rng, jitter_frac * h)
        vc = rng.normal(0.0, 1.0, size=3)
        w = rng.normal(0.0, 0.5, size=3)
        rel = pts - c.reshape(3, 1)
        v = vc.reshape(3, 1) + np.cross(np.broadcast_to(w, rel.T.shape), rel.T).T
        n = pts.shape[1]
        vmax = max(vmax, float(np.sqrt((v ** 2).sum(0)).max()))
        parts.append((pts, v, np.repeat(skew(w).reshape(9, 1), n, 1), np.full(n, h ** 3),
                      np.full(n, bid, dtype=np.uint16)))
    return _assemble(parts, h, mu=0.4, n_iter=6, dt=0.2 * h / vmax, steps=200,
                     name="spheres")


def _shape_points(kind: str, n_target: int, h: float, centre, rng, jitter: float):
    if kind == "cube":
        s = max(2, int(round(n_target ** (1.0 / 3.0))))
        corner = np.asarray(centre) - 0.5 * (s - 1) * h
        return lattice_box(s, s, s, h, corner, rng, jitter)
    r = max(1.5 * h, (3.0 * n_target / (4.0 * math.pi)) ** (1.0 / 3.0) * h)
    return lattice_ball(r, h, centre, rng, jitter)


def two_body_scene(rng, n_total: int, h: float = 1.0, jitter_frac: float = 0.1,
                   n_iter: int = 4, n_bodies: int = 2, mu=None, steps: int = 50) -> Scene:
    """Two (or three) lattice solids, cube or ball at random, with particle
    counts summing to about n_total, approaching each other along a random
    direction with a relative speed ~ U[0.5, 3]; mu ~ U[0, 0.8]."""
    split = rng.uniform(0.3, 0.7)
    if n_bodies == 2:
        counts = [max(8, int(n_total * split)), max(8, n_total - int(n_total * split))]
    else:
        f = rng.dirichlet([1.0] * n_bodies)
        counts = [max(8, int(n_total * fi)) for fi in f]
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    speed = rng.uniform(0.5, 3.0)
    parts = []
    pos = np.zeros(3)
    prev_extent = 0.0
    for bid, cnt in enumerate(counts):
        kind = "cube" if rng.uniform() < 0.5 else "ball"
        pts0 = _shape_points(kind, cnt, h, (0.0, 0.0, 0.0), rng, jitter_frac * h)
        ext = float(np.sqrt((pts0 ** 2).sum(0)).max())
        if bid > 0:
            pos = pos + d * (prev_extent + ext + 0.5 * h)
        pts = pts0 + pos.reshape(3, 1)
        prev_extent = ext
        sgn = 1.0 if bid % 2 == 0 else -1.0
        vel = sgn * 0.5 * speed * d
        parts.append(_body(pts, vel, np.zeros(9), h ** 3, bid))
    sc = _assemble(parts, h, mu=float(rng.uniform(0.0, 0.8)) if mu is None else mu,
                   n_iter=n_iter, dt=0.2 * h / (0.5 * speed), steps=steps, name="two_body")
    # keep positions small and positive-ish: translate so the box starts near 4h
    shift = -np.floor(sc.x.min(1) / h) * h + 4 * h
    sc.x += shift.reshape(3, 1)
    return sc


def batch_scenes(seed: int = SEED_BASE + 4, n_scenes: int = 1024, pmin: float = 1e3,
                 pmax: float = 2e5, n_iter: int = 4):
    """n_scenes independent two-body scenes with log-uniform particle counts."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_scenes):
        p = int(round(math.exp(rng.uniform(math.log(pmin), math.log(pmax)))))
        out.append(two_body_scene(rng, p, n_iter=n_iter))
    return out


@dataclass
class Request:
    arrival: float
    scene: Scene
    steps: int


def request_stream(lam: float, duration: float, seed: int = SEED_BASE + 5,
                   pmin: float = 2e3, pmax: float = 5e5, steps: int = 50, n_iter: int = 4,
                   max_requests: int | None = None):
    """Poisson arrivals at rate lam over `duration` seconds; each request is a
    seeded two- or three-body scene of log-uniform size asking for `steps`."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / lam)
        if t > duration or (max_requests is not None and len(out) >= max_requests):
            break
        p = int(round(math.exp(rng.uniform(math.log(pmin), math.log(pmax)))))
        nb = 2 if rng.uniform() < 0.5 else 3
        out.append(Request(t, two_body_scene(rng, p, n_iter=n_iter, n_bodies=nb,
                                             steps=steps), steps))
    return out


def box_face_normals(nx: int, ny: int, nz: int) -> np.ndarray:
    """Particle normals of an nx x ny x nz lattice box (the ordering of
    lattice_box) as a finite-element mesh would give them: the lattice is read
    as a hexahedral mesh whose nodes are the particles, and each boundary node
    gets the area-weighted sum of the outward normals of the boundary faces
    around it, normalised.  On a regular lattice the faces around a node have
    equal area, so a face node gets its face's normal, an edge node the
    normalised sum of its two faces' normals and a corner node that of three.
    Interior nodes touch no boundary face and get a zero normal.  (Mesh
    geometry only: this is an input the caller supplies, not part of the
    contact method.)"""
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    idx = (i.ravel(), j.ravel(), k.ravel())
    nrm = np.zeros((3, nx * ny * nz))
    for d, (q, hi) in enumerate(zip(idx, (nx, ny, nz))):
        nrm[d] -= (q == 0)
        nrm[d] += (q == hi - 1)
    length = np.sqrt((nrm ** 2).sum(0))
    on = length > 0
    nrm[:, on] /= length[on]
    return nrm


def random_blobs(seed: int, n_bodies: int = 2, side: int = 5, h: float = 1.0,
                 jitter_frac: float = 0.1, spacing_frac: float = 1.0, gap_frac: float = 0.5,
                 random_fields: bool = True, cell_offset: float = 0.5,
                 uniform_mass: bool = False) -> Scene:
    """Small test scenes: n_bodies lattice cubes of side^3 particles in a row
    along x, touching (gap_frac*h between facing planes), with random
    velocities and affine matrices (or zero C when random_fields is False),
    random masses in [0.5, 1.5] (or, with uniform_mass, one mass per body from
    {1, 0.75, 0.5, 1.25}, exact binary fractions)."""
    rng = np.random.default_rng(seed)
    sp = spacing_frac * h
    parts = []
    x0 = cell_offset * h
    for bid in range(n_bodies):
        pts = lattice_box(side, side, side, sp, (x0, cell_offset * h, cell_offset * h), rng,
                          jitter_frac * h)
        n = pts.shape[1]
        x0 += (side - 1) * sp + gap_frac * h
        if random_fields:
            v = rng.normal(size=(3, n)) + rng.normal(size=(3, 1)) * 2.0
            C = rng.normal(size=(9, n)) / h
        else:
            v = np.repeat(rng.normal(size=(3, 1)), n, 1)
            C = np.zeros((9, n))
        mass = (np.full(n, (1.0, 0.75, 0.5, 1.25)[bid % 4]) if uniform_mass
                else rng.uniform(0.5, 1.5, size=n))
        parts.append((pts, v, C, mass, np.full(n, bid, dtype=np.uint16)))
    return _assemble(parts, h, name="blobs")


def pack(scs, dtype=np.float32):
    """Concatenate scenes into packed SoA arrays (x, v, C, m, body) of the
    given float type, with the scene table (list of dicts) and per-scene dt.
    Pure data movement: the values are the scenes' own, rounded to dtype."""
    n = sum(sc.n for sc in scs)
    x = np.empty((3, n), dtype)
    v = np.empty((3, n), dtype)
    C = np.empty((9, n), dtype)
    m = np.empty(n, dtype)
    body = np.empty(n, np.uint16)
    table, dts = [], []
    off = 0
    for sc in scs:
        sl = slice(off, off + sc.n)
        x[:, sl] = sc.x
        v[:, sl] = sc.v
        C[:, sl] = sc.C
        m[sl] = sc.m
        body[sl] = sc.body
        table.append(dict(offset=off, count=sc.n, h=sc.h, origin=sc.origin, dims=sc.dims,
                          mu=sc.mu, n_iter=sc.n_iter, n_bodies=sc.n_bodies))
        dts.append(sc.dt)
        off += sc.n
    return x, v, C, m, body, table, dts
