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
    fps = [lib().apic_scene_footprint(sc.n, 0, FP32_MIXED) for sc, _ in reqs]
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
