"""GPU tests of the batched form at its full size: 1,024 independent two-body
scenes (log-uniform 1e3..2e5 particles, about 3.8e7 in total) stepped together
by the resident driver in one set of launches per phase, in the same launch
configuration the benchmark times (FP32-mixed, graph replay).  Sampled
scenes are checked against the oracle, and against the same scene stepped
alone."""
import sys

import numpy as np
import pytest

from helpers import FP32_TOL, FP64_TOL, oracle_step, parity_error
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


def dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def body_dev(body):
    import torch
    return torch.from_numpy(body.view(np.int16).copy()).cuda()


def sim_of(ctx, scs, dtype):
    from paper_2108_02259_amd.contact import Sim
    x, v, C, m, body, table, dts = scenes.pack(scs, dtype)
    xt, vt, Ct, mt = dev(x, v, C, m)
    return Sim(ctx, table, dts, xt, vt, Ct, mt, body_dev(body)), table


def sampled(scs, rng, k_small=4, k_mid=2, mid_cap=30000, k_large=2, large_min=100000):
    """The smallest scenes, random mid-size ones and random large ones
    (1e5..2e5 particles)."""
    order = np.argsort([sc.n for sc in scs])
    small = list(order[:k_small])
    mids = [i for i in order if scs[i].n <= mid_cap and i not in small]
    large = [i for i in order if scs[i].n >= large_min]
    return (small + list(rng.choice(mids, size=k_mid, replace=False))
            + list(rng.choice(large, size=k_large, replace=False)))


@pytest.mark.parametrize("pairs", [0, 1], ids=["plain", "paired"])
def test_full_batch_sampled_scenes_match_oracle_and_alone(ctx, pairs):
    """The full batch in the launch shape the benchmark uses for it (one
    wave per workgroup, 40 waves per CU), with the plain and the paired
    scatter: sampled scenes against the oracle and against themselves run
    alone."""
    say("building 1,024-scene batch", "paired" if pairs else "plain")
    scs = scenes.batch_scenes()
    ntot = sum(sc.n for sc in scs)
    say(f"  {len(scs)} scenes, {ntot} particles")
    assert len(scs) == 1024 and ntot > 3e7
    tuning = dict(item_waves_per_cu=40, node_wg_per_cu=16, xcd_split=0, p2g_group=1,
                  p2g_pairs=pairs)
    for bucket in range(8, 27):
        ctx.set_tuning(np.float32, 1 << bucket, tuning)
    sim, table = sim_of(ctx, scs, np.float32)
    sim.step(1, graph=True)
    xg, vg, Cg = (t.cpu().numpy() for t in sim.read())
    _, drift, steps = sim.report()
    assert steps == 1
    sim.close()
    picks = sampled(scs, np.random.default_rng(4))
    for i in picks:
        sc, row = scs[i], table[i]
        sl = slice(row["offset"], row["offset"] + row["count"])
        x32, v32, C32, m32 = (a.astype(np.float32) for a in (sc.x, sc.v, sc.C, sc.m))
        ref = oracle_step(sc, x32, v32, C32, m32, sc.mu, sc.n_iter)
        err = parity_error(vg[:, sl], Cg[:, sl], ref["v"], ref["C"], sc.h)
        xref = x32.astype(np.float64) + np.float32(sc.dt) * ref["v"]
        ex = np.abs(xg[:, sl] - xref).max() / max(1.0, np.abs(xref).max())
        # the same scene alone
        alone, _ = sim_of(ctx, [sc], np.float32)
        alone.step(1, graph=True)
        xa, va, Ca = (t.cpu().numpy() for t in alone.read())
        alone.close()
        ea = parity_error(vg[:, sl], Cg[:, sl], va, Ca, sc.h)
        say(f"  scene {i}: n={sc.n} mu={sc.mu:.2f} oracle {err:.2e} x {ex:.2e} alone {ea:.2e}")
        assert err <= FP32_TOL and ex <= FP32_TOL and ea <= FP32_TOL
        assert np.abs(xg[:, sl] - xa).max() <= FP32_TOL * max(1.0, np.abs(xa).max())
    say(f"  max drift P {max(d[0] for d in drift):.2e} L {max(d[1] for d in drift):.2e}")
    default = dict(item_waves_per_cu=32, node_wg_per_cu=8, xcd_split=0, p2g_group=4)
    for bucket in range(8, 27):
        ctx.set_tuning(np.float32, 1 << bucket, default)


def test_batch_fp64_alone_vs_mix_over_steps(ctx):
    """Forty mixed-size scenes over 5 driver steps in FP64: each scene's
    trajectory in the batch equals the scene stepped alone to 1e-10."""
    say("fp64 alone vs mix")
    scs = scenes.batch_scenes(n_scenes=40, pmin=200, pmax=6000)
    sim, table = sim_of(ctx, scs, np.float64)
    sim.step(5, graph=True)
    xg, vg, Cg = (t.cpu().numpy() for t in sim.read())
    sim.close()
    for i in (0, 7, 19, 33):
        sc, row = scs[i], table[i]
        sl = slice(row["offset"], row["offset"] + row["count"])
        alone, _ = sim_of(ctx, [sc], np.float64)
        alone.step(5, graph=False)
        xa, va, Ca = (t.cpu().numpy() for t in alone.read())
        alone.close()
        ea = parity_error(vg[:, sl], Cg[:, sl], va, Ca, sc.h)
        say(f"  scene {i}: n={sc.n} err {ea:.2e}")
        assert ea <= FP64_TOL
        assert np.abs(xg[:, sl] - xa).max() <= FP64_TOL * max(1.0, np.abs(xa).max())
