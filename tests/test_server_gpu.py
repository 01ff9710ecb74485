"""GPU tests of the serving loop (apic_server_*): a request's result is the
same alone and in a continuously batched mix, the loop follows the oracle
driven step by step, admission respects the footprint budget and the scene
slots, and requests that can never fit are refused."""
import sys

import numpy as np
import pytest

from helpers import FP32_TOL, FP64_TOL, cast_inputs, parity_error
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


def requests(seed, k, pmin=200, pmax=3000):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        n = int(round(np.exp(rng.uniform(np.log(pmin), np.log(pmax)))))
        sc = scenes.two_body_scene(rng, n, n_iter=int(rng.integers(1, 5)),
                                   n_bodies=2 if i % 2 else 3)
        out.append((sc, int(rng.integers(2, 6))))
    return out


def table_row(sc):
    return dict(h=sc.h, origin=sc.origin, dims=sc.dims, mu=sc.mu, n_iter=sc.n_iter,
                n_bodies=sc.n_bodies)


def tensors(sc, dtype):
    import torch
    x, v, C, m = cast_inputs(sc, dtype)
    dev = torch.device("cuda:0")
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (x, v, C, m)]
    body = torch.from_numpy(sc.body.view(np.int16).copy()).to(dev)
    outs = [torch.empty_like(ins[0]), torch.empty_like(ins[1]), torch.empty_like(ins[2])]
    return ins, body, outs


def run(srv, reqs, dtype, stagger=0, max_ticks=200, check=None):
    """Submit (all at once, or `stagger` per tick) and tick until every
    request is done; returns {tag: (x, v, C)} as numpy arrays."""
    held = {}
    pending = list(range(len(reqs)))
    done = set()
    ticks = 0
    while len(done) < len(reqs):
        take = pending if stagger == 0 else pending[:stagger]
        for tag in take:
            sc, steps = reqs[tag]
            ins, body, outs = tensors(sc, dtype)
            srv.submit(tag, table_row(sc), sc.dt, steps, *ins, body, *outs)
            held[tag] = outs
        pending = pending[len(take):]
        info, fin = srv.tick()
        if check:
            check(info)
        done.update(fin)
        ticks += 1
        assert ticks < max_ticks
    return {t: tuple(o.cpu().numpy() for o in held[t]) for t in held}


@pytest.mark.parametrize("dtype,tol", [(np.float64, FP64_TOL), (np.float32, FP32_TOL)],
                         ids=["fp64", "fp32"])
def test_result_same_alone_and_in_the_mix(ctx, dtype, tol):
    from paper_2108_02259_amd.contact import Server
    reqs = requests(7, 6)
    say("requests", [(sc.n, st) for sc, st in reqs])
    alone = {}
    for tag, r in enumerate(reqs):
        srv = Server(ctx, dtype, max_particles=200_000, max_scenes=8)
        alone[tag] = run(srv, [r], dtype)[0]
        srv.close()
    srv = Server(ctx, dtype, max_particles=200_000, max_scenes=8)
    mix = run(srv, reqs, dtype, stagger=2)
    srv.close()
    for tag, (sc, _) in enumerate(reqs):
        xa, va, Ca = alone[tag]
        xm, vm, Cm = mix[tag]
        err = parity_error(vm, Cm, va, Ca, sc.h)
        ex = np.abs(xm - xa).max() / max(1.0, np.abs(xa).max())
        say(f"  request {tag}: n={sc.n} v/C {err:.2e} x {ex:.2e}")
        assert err <= tol and ex <= tol


def test_server_follows_the_oracle_driver(ctx):
    """FP64: three driver steps of one request against the oracle's contact
    step followed by x += dt v."""
    from oracle import oracle as ora
    from paper_2108_02259_amd.contact import Server
    sc = scenes.random_blobs(51, n_bodies=3, side=6, h=0.5)
    sc.mu, sc.n_iter, sc.dt = 0.25, 2, 0.01
    x, v, C = sc.x.copy(), sc.v.copy(), sc.C.copy()
    for _ in range(3):
        out = ora.contact_step(ora.Grid(h=sc.h), x, v, C, sc.m, sc.body, sc.mu, sc.n_iter)
        v, C = out["v"], out["C"]
        x = x + sc.dt * v
    srv = Server(ctx, np.float64, max_particles=10_000, max_scenes=2)
    got = run(srv, [(sc, 3)], np.float64)[0]
    srv.close()
    assert parity_error(got[1], got[2], v, C, sc.h) <= 1e-9
    assert np.abs(got[0] - x).max() <= 1e-12


def test_admission_respects_budget_and_slots(ctx):
    from paper_2108_02259_amd._lib import FP32_MIXED, lib
    from paper_2108_02259_amd.contact import Server
    reqs = requests(8, 7, pmin=500, pmax=4000)
    fps = [lib().apic_scene_footprint(sc.n, None, FP32_MIXED) for sc, _ in reqs]
    budget = int(max(fps) * 1.6)
    srv = Server(ctx, np.float32, max_particles=200_000, max_scenes=3, budget_bytes=budget)
    seen = []

    def check(info):
        assert info["footprint"] <= budget
        assert info["resident"] <= 3
        seen.append(info)

    mixed = run(srv, reqs, np.float32, stagger=0, check=check)
    srv.close()
    assert max(i["queued"] for i in seen) > 0   # the budget made requests wait
    assert sum(i["completed"] for i in seen) == len(reqs)
    solo = Server(ctx, np.float32, max_particles=200_000, max_scenes=3)
    for tag in (0, 3, 6):
        a = run(solo, [reqs[tag]], np.float32)[0]
        sc = reqs[tag][0]
        assert parity_error(mixed[tag][1], mixed[tag][2], a[1], a[2], sc.h) <= FP32_TOL
    solo.close()


def test_request_that_never_fits_is_refused(ctx):
    from paper_2108_02259_amd._lib import ApicError, E_BUDGET
    from paper_2108_02259_amd.contact import Server
    sc, _ = requests(9, 1, pmin=2000, pmax=2001)[0]
    srv = Server(ctx, np.float32, max_particles=1000, max_scenes=2)
    ins, body, outs = tensors(sc, np.float32)
    with pytest.raises(ApicError) as e:
        srv.submit(0, table_row(sc), sc.dt, 2, *ins, body, *outs)
    assert e.value.code == E_BUDGET
    srv.close()


def test_failing_request_is_retired_and_the_rest_complete(ctx):
    """A dense-grid request that drifts out of its grid at its second step and
    a request with a non-finite velocity are retired with their errors; the
    healthy requests stepped with them complete with their alone results."""
    import torch
    from paper_2108_02259_amd._lib import E_INVALID, E_OUT_OF_GRID
    from paper_2108_02259_amd.contact import Server
    healthy = requests(11, 3, pmin=400, pmax=1500)
    alone = {}
    for tag, r in enumerate(healthy):
        srv = Server(ctx, np.float32, max_particles=100_000, max_scenes=8)
        alone[tag] = run(srv, [r], np.float32)[0]
        srv.close()
    # leaves its dense grid: fast along +x, the grid ends just past the body
    out = scenes.random_blobs(12, n_bodies=2, side=4, h=0.5)
    out.v[:] = 0.0
    out.v[0] = 40.0
    origin, dims = scenes.snap_dense_grid(out.x, out.h, halo=3)
    out.origin, out.dims, out.dt, out.n_iter, out.mu = origin, dims, 0.01, 1, 0.2
    bad = scenes.random_blobs(13, n_bodies=2, side=4, h=0.5)
    bad.v[2, 5] = np.nan
    bad.n_iter, bad.mu, bad.dt = 2, 0.3, 0.01
    srv = Server(ctx, np.float32, max_particles=100_000, max_scenes=8)
    held = {}
    for tag, (sc, steps) in list(enumerate(healthy)) + [(10, (out, 5)), (11, (bad, 3))]:
        ins, body, outs = tensors(sc, np.float32)
        srv.submit(tag, table_row(sc), sc.dt, steps, *ins, body, *outs)
        held[tag] = outs
    done = set()
    for _ in range(40):
        _, fin = srv.tick()
        done.update(fin)
        if len(done) == len(healthy) and len(srv.failed) == 2:
            break
    say(f"  failed {srv.failed}")
    assert srv.failed == {10: E_OUT_OF_GRID, 11: E_INVALID}
    assert done == set(range(len(healthy)))
    for tag, (sc, _) in enumerate(healthy):
        xm, vm, Cm = (o.cpu().numpy() for o in held[tag])
        xa, va, Ca = alone[tag]
        assert parity_error(vm, Cm, va, Ca, sc.h) <= FP32_TOL
        assert np.abs(xm - xa).max() <= FP32_TOL * max(1.0, np.abs(xa).max())
    srv.close()
    del torch


def test_cancel_queued_and_resident_requests(ctx):
    from paper_2108_02259_amd._lib import ApicError
    from paper_2108_02259_amd.contact import Server
    reqs = requests(14, 3, pmin=300, pmax=800)
    srv = Server(ctx, np.float32, max_particles=100_000, max_scenes=1)
    held = {}
    for tag, (sc, _) in enumerate(reqs):
        ins, body, outs = tensors(sc, np.float32)
        for o in outs:
            o.fill_(7.0)
        srv.submit(tag, table_row(sc), sc.dt, 4, *ins, body, *outs)
        held[tag] = outs
    info, _ = srv.tick()               # request 0 resident, 1 and 2 queued
    assert info["resident"] == 1 and info["deferred"] == 2
    srv.cancel(2)                      # queued
    srv.cancel(0)                      # resident: leaves at the next tick
    with pytest.raises(ApicError):
        srv.cancel(99)
    done = set()
    for _ in range(10):
        _, fin = srv.tick()
        done.update(fin)
    assert done == {1}
    for tag in (0, 2):
        assert all(np.all(o.cpu().numpy() == 7.0) for o in held[tag])
    srv.close()


def test_server_acceleration_matches_the_resident_driver(ctx):
    """A request with a mechanical acceleration follows the resident driver
    (Vbar = V + dt {a, 0} each step) with the same acceleration."""
    from paper_2108_02259_amd.contact import Server, Sim
    sc = scenes.random_blobs(15, n_bodies=2, side=5, h=0.5)
    sc.mu, sc.n_iter, sc.dt = 0.3, 2, 0.01
    row = dict(table_row(sc), accel=(0.0, -9.81, 2.0))
    srv = Server(ctx, np.float64, max_particles=10_000, max_scenes=2)
    ins, body, outs = tensors(sc, np.float64)
    srv.submit(0, row, sc.dt, 3, *ins, body, *outs)
    for _ in range(3):
        srv.tick()
    xs, vs, Cs = (o.cpu().numpy() for o in outs)
    srv.close()
    ins2, body2, _ = tensors(sc, np.float64)
    sim = Sim(ctx, [dict(row, offset=0, count=sc.n)], [sc.dt], *ins2, body2)
    sim.step(3)
    xg, vg, Cg = (t.cpu().numpy() for t in sim.read())
    sim.close()
    assert parity_error(vs, Cs, vg, Cg, sc.h) <= FP64_TOL
    assert np.abs(xs - xg).max() <= 1e-12 * max(1.0, np.abs(xg).max())
    assert np.abs(vs - sc.v).max() > 0.05   # the acceleration acted


@pytest.mark.parametrize("dtype,tol", [(np.float64, FP64_TOL), (np.float32, FP32_TOL)],
                         ids=["fp64", "fp32"])
def test_replayed_ticks_match_the_resident_driver(ctx, dtype, tol):
    """A resident set that stays unchanged is captured into a graph after a
    few ticks and replayed: two requests of 24 steps each follow the resident
    driver stepping the same two scenes, and some of their ticks report a
    replayed graph."""
    from paper_2108_02259_amd.contact import Server, Sim
    scs = [scenes.random_blobs(61, n_bodies=2, side=5, h=0.5),
           scenes.random_blobs(62, n_bodies=3, side=4, h=0.5)]
    for i, sc in enumerate(scs):
        sc.mu, sc.n_iter, sc.dt = 0.2 + 0.2 * i, 1 + i, 0.01
    steps = 24
    srv = Server(ctx, dtype, max_particles=20_000, max_scenes=4)
    held = []
    for tag, sc in enumerate(scs):
        ins, body, outs = tensors(sc, dtype)
        srv.submit(tag, dict(table_row(sc), accel=(0.0, 0.0, -1.0)), sc.dt, steps, *ins, body,
                   *outs)
        held.append(outs)
    replayed = 0
    for _ in range(steps):
        info, _ = srv.tick()
        replayed += info["replayed"]
    srv.close()
    say(f"  {replayed} of {steps} ticks replayed a graph")
    assert replayed >= steps // 4
    for tag, sc in enumerate(scs):
        ins2, body2, _ = tensors(sc, dtype)
        row = dict(table_row(sc), accel=(0.0, 0.0, -1.0), offset=0, count=sc.n)
        sim = Sim(ctx, [row], [sc.dt], *ins2, body2)
        sim.step(steps)
        xg, vg, Cg = (t.cpu().numpy() for t in sim.read())
        sim.close()
        xs, vs, Cs = (o.cpu().numpy() for o in held[tag])
        err = parity_error(vs, Cs, vg, Cg, sc.h)
        ex = np.abs(xs - xg).max() / max(1.0, np.abs(xg).max())
        say(f"  request {tag}: v/C {err:.2e} x {ex:.2e}")
        assert err <= tol and ex <= tol
