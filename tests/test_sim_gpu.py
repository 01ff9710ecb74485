"""GPU tests of the resident driver (apic_sim_*): one step equals the
stateless contact step plus drift, graph replay equals eager stepping, a few
FP64 steps follow the oracle-driven trajectory, momentum drift stays at
round-off, and a plan that outgrows its capacity re-sizes without changing
results."""
import sys

import numpy as np
import pytest

from helpers import FP32_TOL, FP64_TOL, cast_inputs, oracle_step, parity_error
from paper_2108_02259_amd import scenes

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


def to_dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def body_dev(body):
    import torch
    return torch.from_numpy(body.view(np.int16).copy()).cuda()


def table_of(sc):
    return [dict(offset=0, count=sc.n, h=sc.h, origin=sc.origin, dims=sc.dims, mu=sc.mu,
                 n_iter=sc.n_iter, n_bodies=sc.n_bodies)]


def make_sim(ctx, sc, dtype, dt):
    from paper_2108_02259_amd.contact import Sim
    x, v, C, m = cast_inputs(sc, dtype)
    xt, vt, Ct, mt = to_dev(x, v, C, m)
    return Sim(ctx, table_of(sc), [dt], xt, vt, Ct, mt, body_dev(sc.body))


@pytest.mark.parametrize("dtype,tol", [(np.float64, FP64_TOL), (np.float32, FP32_TOL)],
                         ids=["fp64", "fp32"])
@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_one_step_matches_oracle(ctx, dtype, tol, graph):
    say("sim one step", dtype.__name__, graph)
    sc = scenes.random_blobs(31, n_bodies=2, side=7, h=0.5)
    sc.mu, sc.n_iter = 0.4, 3
    dt = 0.01
    sim = make_sim(ctx, sc, dtype, dt)
    sim.step(1, graph=graph)
    x1, v1, C1 = (a.cpu().numpy() for a in sim.read())
    x, v, C, m = cast_inputs(sc, dtype)
    ref = oracle_step(sc, x, v, C, m, sc.mu, sc.n_iter)
    assert parity_error(v1, C1, ref["v"], ref["C"], sc.h) <= tol
    xref = x.astype(np.float64) + dt * ref["v"]
    assert np.abs(x1 - xref).max() <= tol * max(1.0, np.abs(xref).max())
    _, drift, steps = sim.report()
    assert steps == 1
    sim.close()


def test_graph_replay_equals_eager(ctx):
    say("graph vs eager")
    sc = scenes.random_blobs(32, n_bodies=3, side=6, h=0.5)
    sc.mu, sc.n_iter = 0.2, 2
    a = make_sim(ctx, sc, np.float64, 0.02)
    b = make_sim(ctx, sc, np.float64, 0.02)
    a.step(7, graph=False)
    b.step(7, graph=True)
    xa, va, Ca = (t.cpu().numpy() for t in a.read())
    xb, vb, Cb = (t.cpu().numpy() for t in b.read())
    assert parity_error(vb, Cb, va, Ca, sc.h) <= 1e-9
    assert np.abs(xa - xb).max() <= 1e-9 * np.abs(xa).max()
    # replays on an eager-touched graph keep working: interleave
    a.step(2, graph=True)
    b.step(2, graph=False)
    xa, va, Ca = (t.cpu().numpy() for t in a.read())
    xb, vb, Cb = (t.cpu().numpy() for t in b.read())
    assert parity_error(vb, Cb, va, Ca, sc.h) <= 1e-9
    a.close()
    b.close()


def test_fp64_trajectory_follows_oracle_driver(ctx):
    """Four driver steps (contact step, then x += dt v) against the oracle
    driven the same way; FP64 round-off is amplified only mildly in 4 steps."""
    say("trajectory")
    from oracle import oracle as ora
    sc = scenes.two_cubes()
    dt = sc.dt
    sim = make_sim(ctx, sc, np.float64, dt)
    x, v, C = sc.x.copy(), sc.v.copy(), sc.C.copy()
    for _ in range(4):
        out = ora.contact_step(ora.Grid(h=sc.h, origin=sc.origin), x, v, C, sc.m, sc.body,
                               sc.mu, sc.n_iter)
        v, C = out["v"], out["C"]
        x = x + dt * v
    sim.step(4, graph=True)
    xs, vs, Cs = (t.cpu().numpy() for t in sim.read())
    assert parity_error(vs, Cs, v, C, sc.h) <= 1e-9
    assert np.abs(xs - x).max() <= 1e-12
    sim.close()


@pytest.mark.parametrize("dtype,bound", [(np.float64, 1e-12), (np.float32, 1e-5)],
                         ids=["fp64", "fp32"])
def test_momentum_drift_over_steps(ctx, dtype, bound):
    say("drift", dtype.__name__)
    sc = scenes.slab_block(slab=(40, 40, 6), block=(12, 12, 6))
    sim = make_sim(ctx, sc, dtype, sc.dt)
    sim.step(30, graph=True)
    reps, drift, steps = sim.report()
    say(f"  max drift P {drift[0][0]:.2e} L {drift[0][1]:.2e}")
    assert steps == 30
    assert drift[0][0] <= bound and drift[0][1] <= bound
    sim.close()


def test_plan_grows_when_bodies_spread(ctx):
    """Two bodies flying apart enlarge the scene's block box far beyond the
    initial headroom: the sim re-plans and matches stateless stepping."""
    say("resize")
    import torch
    sc = scenes.random_blobs(33, n_bodies=2, side=5, h=1.0, random_fields=False)
    sc.v[:, sc.body == 0] = np.array([[-6.0], [0.0], [0.0]])
    sc.v[:, sc.body == 1] = np.array([[6.0], [1.0], [0.0]])
    sc.mu, sc.n_iter = 0.0, 1
    dt = 1.0
    sim = make_sim(ctx, sc, np.float64, dt)
    sim.step(6, graph=True)
    xs, vs, Cs = (t.cpu().numpy() for t in sim.read())
    _, _, steps = sim.report()
    assert steps == 6
    info = sim.info()
    # reference: stateless steps on the host-driven state
    x, v, C, m = (a.copy() for a in cast_inputs(sc, np.float64))
    xt, vt, Ct, mt = to_dev(x, v, C, m)
    bt = body_dev(sc.body)
    for _ in range(6):
        ctx.contact_step(xt, vt, Ct, mt, bt, sc.h, mu=sc.mu, n_iter=sc.n_iter)
        xt += dt * vt
    torch.cuda.synchronize()
    assert parity_error(vs, Cs, vt.cpu().numpy(), Ct.cpu().numpy(), sc.h) <= 1e-9
    assert np.abs(xs - xt.cpu().numpy()).max() <= 1e-9
    say("  info", info)
    sim.close()
