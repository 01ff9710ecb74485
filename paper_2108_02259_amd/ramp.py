"""The reduced ramp: a validation driver around the library's contact step.

The paper's frictional-sliding example (Section 3.3) lets an elastic block
slide down a fixed ramp tilted by 30 degrees under gravity.  Without the
finite-element solver, this driver reduces it to what the contact step
needs, in the ramp's own frame:

* the ramp is a heavy lattice slab (mass ratio 1e6) whose velocity is held
  at zero after every step (its bottom face is fixed in the paper);
* gravity is tilted instead of the ramp: a = g (sin theta, 0, -cos theta)
  acts on the block only;
* the block's missing stiffness is stood in for by a rigid-body projection
  after every contact step: the block's velocity field is replaced by the
  rigid motion with the same linear momentum and the same angular momentum
  (with the APIC spin term), C = [w]_x -- the infinitely stiff limit.

Each driver step: v <- v + dt a, (v, C) <- S(v, C) (the library's contact
step), ramp velocity <- 0, block <- rigid projection, x <- x + dt v.  The
driver's own arithmetic (prediction, projection, drift) runs as torch ops on
the device; the contact step is the library's.
"""
from __future__ import annotations

import math

import numpy as np

from . import scenes

THETA = math.radians(30.0)


def ramp_scene(block_side: int = 6, plane=(20, 10, 3), gap: float = 1.0, h: float = 1.0):
    """The ramp (body 0, heavy) and the block (body 1), jitter-free lattices
    of spacing 1 at cell centres; the block's bottom plane `gap` above the
    ramp's top plane."""
    rng = np.random.default_rng(0)
    ramp = scenes.lattice_box(*plane, 1.0, (0.5, 0.5, 0.5), rng, 0.0)
    top = 0.5 + plane[2] - 1
    block = scenes.lattice_box(block_side, block_side, block_side, 1.0,
                               (2.5, 2.5, top + gap), rng, 0.0)
    n_r, n_b = ramp.shape[1], block.shape[1]
    x = np.concatenate([ramp, block], 1)
    m = np.concatenate([np.full(n_r, 1e6), np.ones(n_b)])
    body = np.concatenate([np.zeros(n_r, np.uint16), np.ones(n_b, np.uint16)])
    sc = scenes.Scene(x, np.zeros_like(x), np.zeros((9, x.shape[1])), m, body, h, mu=0.0,
                      n_iter=4, name="ramp")
    return sc, n_r


def gravity(g: float = 10.0):
    return np.array([g * math.sin(THETA), 0.0, -g * math.cos(THETA)])


def rigid_projection(x, v, C, m, h):
    """The rigid motion (v = V + w x r, C = [w]_x) with the same linear and
    angular momentum (orbital plus the APIC spin (h^2/2) axial(C - C^T)) as
    the given field, on torch tensors of one body."""
    import torch
    M = m.sum()
    xc = (m * x).sum(1) / M
    P = (m * v).sum(1)
    r = x - xc[:, None]
    spin = torch.stack([C[7] - C[5], C[2] - C[6], C[3] - C[1]])
    L = (m * torch.linalg.cross(r.T, v.T).T).sum(1) + 0.5 * h * h * (m * spin).sum(1)
    rr = (r * r).sum(0)
    eye = torch.eye(3, dtype=x.dtype, device=x.device)
    inertia = ((m * (rr + h * h)).sum() * eye - (m * r) @ r.T)
    w = torch.linalg.solve(inertia, L)
    v_new = P[:, None] / M + torch.linalg.cross(w.expand(r.shape[1], 3), r.T).T
    zero = torch.zeros_like(w[0])
    wx = torch.stack([zero, -w[2], w[1], w[2], zero, -w[0], -w[1], w[0], zero])
    return v_new, wx[:, None].expand(9, r.shape[1]).contiguous()


def run(ctx, mu: float, steps: int, dt: float = 2e-3, g: float = 10.0, n_iter: int = 4,
        dtype=np.float64, h: float = 1.0, gap: float = 1.0, trace_every: int = 0,
        block_side: int = 6):
    """Drive the reduced ramp on the GPU; returns (times, block centre-of-mass
    displacements (3, k), final state)."""
    import torch
    sc, n_r = ramp_scene(block_side=block_side, gap=gap, h=h)
    dev = torch.device("cuda:0")
    x, v, C, m = (torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).to(dev)
                  for a in (sc.x, sc.v, sc.C, sc.m))
    body = torch.from_numpy(sc.body.view(np.int16).copy()).to(dev)
    a = torch.zeros_like(x)
    a[:, n_r:] = torch.from_numpy(gravity(g).astype(dtype)).to(dev)[:, None]
    row = [dict(offset=0, count=sc.n, h=h, mu=mu, n_iter=n_iter, n_bodies=2)]
    blk = slice(n_r, sc.n)
    c0 = x[:, blk].mean(1).clone()
    times, disp = [], []
    for s in range(steps):
        v += dt * a
        ctx.contact_step_batched(row, x, v, C, m, body, report=False)
        v[:, :n_r] = 0.0
        C[:, :n_r] = 0.0
        v[:, blk], C[:, blk] = rigid_projection(x[:, blk], v[:, blk], C[:, blk], m[blk], h)
        x += dt * v
        if trace_every and (s + 1) % trace_every == 0:
            times.append((s + 1) * dt)
            disp.append((x[:, blk].mean(1) - c0).cpu().numpy())
    return times, np.array(disp).T if disp else None, (x, v, C, m, body)


def analytic_slide(t, mu: float, g: float = 10.0):
    """Distance slid along the ramp by a rigid block from rest:
    1/2 g t^2 (sin theta - mu cos theta), zero when mu >= tan theta."""
    return 0.5 * g * np.asarray(t) ** 2 * max(0.0, math.sin(THETA) - mu * math.cos(THETA))
