"""GPU tests of the reduced ramp (the paper's frictional-sliding example of
Section 3.3 without its finite-element solver, see paper_2108_02259_amd/ramp.py):
the one-step stick/slip threshold at mu = tan 30 degrees against the oracle,
the driver against the same driver around the oracle's contact step, and
the ordering of the slide with friction."""
import math
import sys

import numpy as np
import pytest

from helpers import FP64_TOL, parity_error
from oracle import oracle as ora
from paper_2108_02259_amd import ramp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2108_02259_amd.contact import Context
    c = Context(0)
    yield c
    c.close()


def test_one_step_threshold_at_tan_theta(ctx):
    """Block at rest on the ramp, one step of tilted gravity: Vbar = dt g on
    the block.  At the centre of its bottom face the normal is -e_z exactly
    and dv is along -Vbar, so |dv_t| / (-dv.n) = tan 30 degrees: the first
    series field keeps the tangential change (stick) iff mu >= tan 30.  The
    GPU step follows the oracle on both sides of the threshold, and the two
    sides differ."""
    import torch
    sc, n_r = ramp.ramp_scene(block_side=5)
    dt = 2e-3
    v = np.zeros_like(sc.x)
    v[:, n_r:] = dt * ramp.gravity()[:, None]
    blk = sc.x[:, n_r:]
    c = n_r + int(np.flatnonzero((np.abs(blk[0] - 4.5) < 1e-12) & (np.abs(blk[1] - 4.5) < 1e-12)
                                 & (np.abs(blk[2] - blk[2].min()) < 1e-12))[0])
    mu_star = math.tan(ramp.THETA)
    outs = {}
    for mu in (mu_star * (1 - 1e-6), mu_star * (1 + 1e-6)):
        ref = ora.contact_step(ora.Grid(h=sc.h), sc.x, v, sc.C, sc.m, sc.body, mu, 4,
                               want_w1=True, want_normals=True)
        np.testing.assert_allclose(ref["normals"][:, c], [0.0, 0.0, -1.0], atol=1e-14)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        vt, Ct = d(v), d(sc.C)
        ctx.contact_step_batched([dict(offset=0, count=sc.n, h=sc.h, mu=mu, n_iter=4,
                                       n_bodies=2)], d(sc.x), vt, Ct, d(sc.m),
                                 torch.from_numpy(sc.body.view(np.int16).copy()).cuda())
        vg, Cg = vt.cpu().numpy(), Ct.cpu().numpy()
        err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
        w1t = ref["w1"][:2, c]
        say(f"  mu {mu:.9f}: parity {err:.2e}, first series field (tangential) {w1t}")
        assert err <= FP64_TOL
        outs[mu] = (vg, w1t)
    (v_slip, w_slip), (v_stick, w_stick) = outs.values()
    assert np.all(w_stick == 0.0) and abs(w_slip[0]) > 0.0
    assert np.abs(v_slip - v_stick).max() > 1e-9


def test_ramp_driver_follows_the_oracle_driver(ctx):
    """Three driver steps (gravity, contact, fixed ramp, rigid block, drift) on
    the GPU against the same driver around the oracle's contact step,
    teacher-forced step by step."""
    import torch
    from paper_2108_02259_amd.ramp import rigid_projection
    dt, mu = 2e-3, 0.3
    sc, n_r = ramp.ramp_scene(block_side=5)
    g = ramp.gravity()
    x, v, C = sc.x.copy(), sc.v.copy(), sc.C.copy()
    for step in range(3):
        vbar = v.copy()
        vbar[:, n_r:] += dt * g[:, None]
        ref = ora.contact_step(ora.Grid(h=sc.h), x, vbar, C, sc.m, sc.body, mu, 4)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        vt, Ct = d(vbar), d(C)
        ctx.contact_step_batched([dict(offset=0, count=sc.n, h=sc.h, mu=mu, n_iter=4,
                                       n_bodies=2)], d(x), vt, Ct, d(sc.m),
                                 torch.from_numpy(sc.body.view(np.int16).copy()).cuda())
        err = parity_error(vt.cpu().numpy(), Ct.cpu().numpy(), ref["v"], ref["C"], sc.h)
        say(f"  step {step}: parity {err:.2e}")
        assert err <= FP64_TOL
        # the driver's own arithmetic on the GPU result
        vt[:, :n_r] = 0.0
        Ct[:, :n_r] = 0.0
        b = slice(n_r, sc.n)
        vt[:, b], Ct[:, b] = rigid_projection(d(x)[:, b], vt[:, b], Ct[:, b], d(sc.m)[b], sc.h)
        v, C = vt.cpu().numpy(), Ct.cpu().numpy()
        x = x + dt * v
    # the rigid block keeps its shape: all its particles move alike (up to a
    # small rotation)
    assert np.abs(v[:, n_r:] - v[:, n_r:].mean(1, keepdims=True)).max() < 0.05 * np.abs(v).max()


def test_ramp_slides_less_with_more_friction(ctx):
    """150 driver steps: the block slides down-slope, less the more friction
    there is, and stays above the ramp."""
    slid = {}
    for mu in (0.0, 0.3, 0.8):
        _, disp, _ = ramp.run(ctx, mu, 150, trace_every=150)
        slid[mu] = disp[:, -1]
        say(f"  mu {mu}: centre of mass moved {disp[:, -1]}, analytic slide "
            f"{ramp.analytic_slide(0.3, mu):.3f}")
    assert slid[0.0][0] > slid[0.3][0] > slid[0.8][0] > 0.0
    assert all(d[2] > -0.5 for d in slid.values())
