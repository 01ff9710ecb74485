"""GPU parity: the HIP contact step against the FP64 CPU oracle on identical
seeded inputs.  Bars: cell keys and permutation bit-exact; FP64 path within
1e-10 and FP32-mixed path within 2e-5 of |v|_inf (velocity and h-scaled
affine part, normwise per step)."""
import sys

import numpy as np
import pytest

from helpers import FP32_TOL, FP64_TOL, cast_inputs, gpu_step, oracle_step, parity_error
from oracle import oracle as ora
from paper_2108_02259_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2108_02259_amd.contact import Context
    c = Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ---------------------------------------------------------------------------
# keys and order: bit-exact
# ---------------------------------------------------------------------------

def _keys_case(ctx, x, body, grids, counts, nbodies, dtype):
    import torch
    xs = x.astype(dtype)
    sc = []
    off = 0
    for g, c, nb in zip(grids, counts, nbodies):
        sc.append(dict(offset=off, count=c, h=g.h, origin=g.origin, dims=(0, 0, 0),
                       n_bodies=nb))
        off += c
    xt = torch.from_numpy(np.ascontiguousarray(xs)).cuda()
    bt = torch.from_numpy(body.view(np.int16).copy()).cuda()
    kg, pg = ctx.sort_keys(sc, xt, bt)
    osc = []
    off = 0
    for g, c, nb in zip(grids, counts, nbodies):
        osc.append(ora.Scene(off, c, g, nb))
        off += c
    keys, perm = ora.cell_keys(osc, xs.astype(np.float64), body)
    np.testing.assert_array_equal(pg.cpu().numpy(), perm.astype(np.int64))
    np.testing.assert_array_equal(kg.cpu().numpy(), keys[perm].astype(np.int64))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("seed", [1, 2])
def test_sort_keys_bit_exact_single(ctx, dtype, seed):
    say("keys single", dtype.__name__, seed)
    sc = scenes.random_blobs(seed, n_bodies=3, side=9, h=0.37, jitter_frac=0.45)
    g = ora.Grid(h=sc.h, origin=(-2.1, 0.3, -0.77))
    _keys_case(ctx, sc.x, sc.body, [g], [sc.n], [3], dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sort_keys_bit_exact_batched(ctx, dtype):
    say("keys batched", dtype.__name__)
    rng = np.random.default_rng(7)
    parts, bodies, grids, counts, nbs = [], [], [], [], []
    for s in range(5):
        sc = scenes.random_blobs(100 + s, n_bodies=2 + s % 2, side=4 + 3 * s, h=1.0)
        parts.append(sc.x - rng.uniform(0, 30, size=(3, 1)))  # negative cells too
        bodies.append(sc.body)
        grids.append(ora.Grid(h=0.5 + 0.25 * s, origin=tuple(rng.uniform(-3, 3, 3))))
        counts.append(sc.n)
        nbs.append(int(sc.body.max()) + 1)
    x = np.concatenate(parts, 1)
    body = np.concatenate(bodies)
    _keys_case(ctx, x, body, grids, counts, nbs, dtype)


def test_sort_keys_large_many_ties(ctx):
    """Full-size slab+block: 1.1M keys, several radix passes."""
    say("keys slab_block")
    sc = scenes.slab_block()
    _keys_case(ctx, sc.x, sc.body, [ora.Grid(h=sc.h)], [sc.n], [2], np.float32)


# ---------------------------------------------------------------------------
# contact step parity
# ---------------------------------------------------------------------------

CASES = [
    # name, builder, mu, n_iter
    ("blobs2_N0", lambda: scenes.random_blobs(11, n_bodies=2, side=6, h=0.5), 0.3, 0),
    ("blobs2_N1", lambda: scenes.random_blobs(12, n_bodies=2, side=6, h=0.5), 0.3, 1),
    ("blobs3_N4_mu0", lambda: scenes.random_blobs(13, n_bodies=3, side=7, h=0.5), 0.0, 4),
    ("blobs2_N3_mu1", lambda: scenes.random_blobs(14, n_bodies=2, side=9, h=1.0,
                                                  spacing_frac=0.4), 1.0, 3),
    ("dense_cells", lambda: scenes.random_blobs(15, n_bodies=2, side=12, h=1.0,
                                                spacing_frac=0.3), 0.5, 2),
    # friction far beyond any tangential change: the rule's sticking limit
    ("blobs2_N2_mu1e3", lambda: scenes.random_blobs(16, n_bodies=2, side=6, h=0.5), 1e3, 2),
    # rigid translations, no affine part: contact between uniform fields
    ("rigid2_N3", lambda: scenes.random_blobs(17, n_bodies=2, side=7, h=0.5,
                                              random_fields=False), 0.4, 3),
    # one body: every node is single-body, the rule still acts on its own normals
    ("single_body_N3", lambda: scenes.random_blobs(18, n_bodies=1, side=8, h=0.5), 0.3, 3),
    # four bodies in a row, six series rounds
    ("blobs4_N6", lambda: scenes.random_blobs(19, n_bodies=4, side=5, h=0.5), 0.4, 6),
]


@pytest.mark.parametrize("name,build,mu,n_iter", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype,tol", [(np.float64, FP64_TOL), (np.float32, FP32_TOL)],
                         ids=["fp64", "fp32"])
def test_contact_step_parity(ctx, name, build, mu, n_iter, dtype, tol):
    say("step", name, dtype.__name__)
    sc = build()
    x, v, C, m = cast_inputs(sc, dtype)
    ref = oracle_step(sc, x, v, C, m, mu, n_iter)
    vg, Cg, rep = gpu_step(ctx, sc, x, v, C, m, mu, n_iter)
    err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
    say(f"  parity error {err:.3e}")
    assert err <= tol
    drift_P = np.abs(np.array(rep["P_after"]) - rep["P_before"]).max() / rep["P_scale"]
    drift_L = np.abs(np.array(rep["L_after"]) - rep["L_before"]).max() / rep["L_scale"]
    say(f"  drift P {drift_P:.2e} L {drift_L:.2e}")
    assert drift_P <= (1e-12 if dtype == np.float64 else 1e-5)
    assert drift_L <= (1e-12 if dtype == np.float64 else 1e-5)
    assert rep["n_particles"] == sc.n
    # the reported momenta are the device's wave reductions of m v over the
    # step's inputs and outputs; the host sums the same values in FP64
    m64 = m.astype(np.float64)
    P_in = (m64 * v.astype(np.float64)).sum(axis=1)
    P_out = (m64 * vg.astype(np.float64)).sum(axis=1)
    scale = rep["P_scale"]
    assert np.abs(np.array(rep["P_before"]) - P_in).max() <= 1e-12 * scale
    assert np.abs(np.array(rep["P_after"]) - P_out).max() <= 1e-12 * scale
    check_report_sums(rep, x, v, C, m, vg, Cg, sc.h)


def check_report_sums(rep, x, v, C, m, vg, Cg, h, origin=(0.0, 0.0, 0.0)):
    """The reported L (about the grid origin, with the affine spin) and E
    (with the affine term) equal host FP64 sums over the step's inputs and
    outputs (summation order aside)."""
    f = lambda a: np.asarray(a, dtype=np.float64)
    before = ora.momentum(f(x), f(v), f(C), f(m), h, origin)
    after = ora.momentum(f(x), f(vg), f(Cg), f(m), h, origin)
    for key, ref in (("before", before), ("after", after)):
        assert np.abs(np.array(rep[f"L_{key}"]) - ref["L"]).max() <= 1e-12 * ref["L_scale"]
        assert rep[f"E_{key}"] == pytest.approx(ref["E"], rel=1e-12)
    assert rep["P_scale"] == pytest.approx(before["P_scale"], rel=1e-12)
    assert rep["L_scale"] == pytest.approx(before["L_scale"], rel=1e-12)


@pytest.mark.parametrize("dtype,tol", [(np.float64, FP64_TOL), (np.float32, FP32_TOL)],
                         ids=["fp64", "fp32"])
def test_dense_grid_two_cubes(ctx, dtype, tol):
    """Two cubes head-on (dense grid, mu = 0, 3 iterations)."""
    say("two cubes dense", dtype.__name__)
    sc = scenes.two_cubes()
    x, v, C, m = cast_inputs(sc, dtype)
    ref = oracle_step(sc, x, v, C, m, sc.mu, sc.n_iter, sc.origin, sc.dims)
    vg, Cg, _ = gpu_step(ctx, sc, x, v, C, m, sc.mu, sc.n_iter, sc.origin, sc.dims)
    err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
    say(f"  parity error {err:.3e}")
    assert err <= tol


def test_two_cubes_all_200_steps_follow_the_oracle_driver(ctx):
    """The small configuration run to its end in FP64: 200 driver steps
    (contact step on a dense grid re-snapped to the particles, then
    x += dt v), the GPU's stateless calls against the oracle driven the same
    way.  The cubes collide within the run (inelastically: they slow from
    1 to about 0.26 each and do not rebound; no elastic forces here).  The
    bound allows for round-off growth along the trajectory: on the CPU a
    relative perturbation of 1e-15 in the initial positions grows to 1.8e-9
    in v after 200 oracle steps, and the GPU's per-step FP64 results differ
    from the oracle's by summation order."""
    say("two cubes 200 steps")
    sc = scenes.two_cubes()
    xo, vo, Co = sc.x.copy(), sc.v.copy(), sc.C.copy()
    xg, vg, Cg = sc.x.copy(), sc.v.copy(), sc.C.copy()
    worst = 0.0
    for k in range(sc.steps):
        origin, dims = scenes.snap_dense_grid(xo, sc.h)
        ref = oracle_step(sc, xo, vo, Co, sc.m, sc.mu, sc.n_iter, origin, dims)
        vo, Co = ref["v"], ref["C"]
        xo = xo + sc.dt * vo
        origin_g, dims_g = scenes.snap_dense_grid(xg, sc.h)
        vg, Cg, _ = gpu_step(ctx, sc, xg, vg, Cg, sc.m, sc.mu, sc.n_iter, origin_g, dims_g)
        xg = xg + sc.dt * vg
        worst = max(worst, parity_error(vg, Cg, vo, Co, sc.h))
        if k % 50 == 49:
            say(f"  step {k + 1}: max parity error so far {worst:.2e}")
    assert worst <= 1e-8          # measured 3.4e-11 on MI355X
    assert np.abs(xg - xo).max() <= 1e-8
    # the cubes met: each body's mean approach speed has dropped from 1
    for b, sign in ((0, 1.0), (1, -1.0)):
        assert 0.0 < sign * vo[0, sc.body == b].mean() < 0.5


def test_out_of_dense_grid_is_reported_and_leaves_inputs(ctx):
    say("out of grid")
    from paper_2108_02259_amd._lib import ApicError, E_OUT_OF_GRID
    sc = scenes.two_cubes()
    dims = (sc.dims[0] - 4, sc.dims[1], sc.dims[2])
    v0 = sc.v.copy()
    with pytest.raises(ApicError) as e:
        gpu_step(ctx, sc, sc.x, v0, sc.C, sc.m, 0.0, 1, sc.origin, dims)
    assert e.value.code == E_OUT_OF_GRID


def test_empty_and_single_particle(ctx):
    say("empty/single")
    import torch
    x = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    v = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    C = torch.zeros((9, 0), dtype=torch.float64, device="cuda")
    m = torch.zeros((0,), dtype=torch.float64, device="cuda")
    b = torch.zeros((0,), dtype=torch.int16, device="cuda")
    ctx.contact_step(x, v, C, m, b, 1.0, mu=0.2, n_iter=2)
    sc = scenes.random_blobs(3, n_bodies=1, side=1, h=1.0)
    ref = oracle_step(sc, sc.x, sc.v, sc.C, sc.m, 0.2, 2)
    vg, Cg, _ = gpu_step(ctx, sc, sc.x, sc.v, sc.C, sc.m, 0.2, 2)
    assert parity_error(vg, Cg, ref["v"], ref["C"], sc.h) <= FP64_TOL


def test_crowded_cells_split_work_items(ctx):
    """Cell blocks with far more than 64 particles (ragged work items)."""
    say("crowded")
    sc = scenes.random_blobs(21, n_bodies=2, side=14, h=2.0, spacing_frac=0.1, jitter_frac=0.2)
    ref = oracle_step(sc, sc.x, sc.v, sc.C, sc.m, 0.4, 2)
    vg, Cg, _ = gpu_step(ctx, sc, sc.x, sc.v, sc.C, sc.m, 0.4, 2)
    assert parity_error(vg, Cg, ref["v"], ref["C"], sc.h) <= FP64_TOL


def test_many_bodies(ctx):
    say("many bodies")
    parts = []
    rng = np.random.default_rng(5)
    sc = scenes.spheres(n_spheres=12, box_cells=40.0, radius_cells=4.0)
    for dtype, tol in ((np.float64, FP64_TOL), (np.float32, FP32_TOL)):
        x, v, C, m = cast_inputs(sc, dtype)
        ref = oracle_step(sc, x, v, C, m, 0.4, 3)
        vg, Cg, _ = gpu_step(ctx, sc, x, v, C, m, 0.4, 3)
        assert parity_error(vg, Cg, ref["v"], ref["C"], sc.h) <= tol
    del parts, rng


def test_batched_matches_oracle_per_scene(ctx):
    say("batched")
    import torch
    rng = np.random.default_rng(9)
    scs = [scenes.two_body_scene(rng, int(n), n_iter=k) for n, k in
           ((300, 2), (50, 0), (1200, 4), (700, 1))]
    for dtype, tol in ((np.float64, FP64_TOL), (np.float32, FP32_TOL)):
        xs, vs, Cs, ms, bs, table = [], [], [], [], [], []
        off = 0
        for sc in scs:
            x, v, C, m = cast_inputs(sc, dtype)
            xs.append(x); vs.append(v); Cs.append(C); ms.append(m); bs.append(sc.body)
            table.append(dict(offset=off, count=sc.n, h=sc.h, mu=sc.mu, n_iter=sc.n_iter,
                              n_bodies=sc.n_bodies))
            off += sc.n
        cat = lambda a: torch.from_numpy(np.ascontiguousarray(np.concatenate(a, -1))).cuda()
        xt, vt, Ct, mt = cat(xs), cat(vs), cat(Cs), cat(ms)
        bt = torch.from_numpy(np.concatenate(bs).view(np.int16).copy()).cuda()
        reps = ctx.contact_step_batched(table, xt, vt, Ct, mt, bt)
        vg, Cg = vt.cpu().numpy(), Ct.cpu().numpy()
        for sc, row, x, v, C, m, rep in zip(scs, table, xs, vs, Cs, ms, reps):
            ref = oracle_step(sc, x, v, C, m, sc.mu, sc.n_iter)
            sl = slice(row["offset"], row["offset"] + row["count"])
            err = parity_error(vg[:, sl], Cg[:, sl], ref["v"], ref["C"], sc.h)
            say(f"  scene n={sc.n} N={sc.n_iter} err {err:.2e}")
            assert err <= tol
            assert rep["n_particles"] == sc.n


@pytest.mark.parametrize("mu", [0.0, 0.3, 1.0])
@pytest.mark.parametrize("dtype,tol", [(np.float32, FP32_TOL), (np.float64, FP64_TOL)],
                         ids=["fp32", "fp64"])
def test_full_size_slab_block(ctx, dtype, tol, mu):
    """The 1,114,112-particle slab + block at each of its friction
    coefficients, 4 iterations: every particle compared with the oracle, and
    the reported momenta and energy with host sums."""
    say("full slab_block", dtype.__name__, "mu", mu)
    sc = scenes.slab_block(mu=mu)
    x, v, C, m = cast_inputs(sc, dtype)
    vg, Cg, rep = gpu_step(ctx, sc, x, v, C, m, sc.mu, sc.n_iter)
    ref = oracle_step(sc, x, v, C, m, sc.mu, sc.n_iter)
    err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
    say(f"  parity error {err:.3e}, blocks {rep['grid_blocks']}")
    assert err <= tol
    check_report_sums(rep, x, v, C, m, vg, Cg, sc.h)


@pytest.mark.parametrize("dtype,tol", [(np.float32, FP32_TOL), (np.float64, FP64_TOL)],
                         ids=["fp32", "fp64"])
def test_full_size_spheres(ctx, dtype, tol):
    """The 256-sphere scene (539,904 particles, 256 bodies, mu 0.4, 6
    iterations): every particle compared with the oracle, the reported sums
    with host sums, and the most bodies at one node as the bodies' grids
    overlap."""
    say("full spheres", dtype.__name__)
    sc = scenes.spheres()
    x, v, C, m = cast_inputs(sc, dtype)
    vg, Cg, rep = gpu_step(ctx, sc, x, v, C, m, sc.mu, sc.n_iter)
    ref = oracle_step(sc, x, v, C, m, sc.mu, sc.n_iter)
    err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
    say(f"  n={sc.n} parity error {err:.3e}, bodies per node {rep['max_bodies_per_node']}")
    assert err <= tol
    assert rep["max_bodies_per_node"] >= 2
    check_report_sums(rep, x, v, C, m, vg, Cg, sc.h)


# ---------------------------------------------------------------------------
# unconstrained particles (zero own-body mass gradient): W = 0, full series
# rows kept for their work items
# ---------------------------------------------------------------------------

def unconstrained_scene(seed, side=9, n_lone=3):
    """Jitter-free lattice cubes at cell centres with one exact mass per body
    (every weight and mass sum is an exact binary fraction, so a zero
    gradient is exactly zero in any summation order), random velocities and
    affine fields, plus lone particles at cell centres as bodies of their
    own.  Interior particles (3 cells from every face) and the lone ones have
    no normal."""
    sc = scenes.random_blobs(seed, n_bodies=2, side=side, h=1.0, jitter_frac=0.0,
                             gap_frac=1.0, uniform_mass=True)
    rng = np.random.default_rng(seed + 1)
    nb = sc.n_bodies
    xs = [sc.x]
    for k in range(n_lone):
        xs.append(np.array([[3.5 + 11.0 * k], [30.5], [3.5]]))
    x = np.concatenate(xs, 1)
    v = np.concatenate([sc.v, rng.normal(size=(3, n_lone))], 1)
    C = np.concatenate([sc.C, rng.normal(size=(9, n_lone))], 1)
    m = np.concatenate([sc.m, np.full(n_lone, 0.5)])
    body = np.concatenate([sc.body, np.arange(nb, nb + n_lone, dtype=np.uint16)])
    return scenes.Scene(x, v, C, m, body, 1.0, name="unconstrained")


@pytest.mark.parametrize("n_iter", [0, 1, 4])
@pytest.mark.parametrize("dtype,tol", [(np.float64, FP64_TOL), (np.float32, FP32_TOL)],
                         ids=["fp64", "fp32"])
def test_unconstrained_particles(ctx, dtype, tol, n_iter):
    say("unconstrained", dtype.__name__, n_iter)
    sc = unconstrained_scene(160 + n_iter)
    x, v, C, m = cast_inputs(sc, dtype)
    g = ora.Grid(h=sc.h)
    ref = ora.contact_step(g, *(a.astype(np.float64) for a in (x, v, C, m)), sc.body, 0.4,
                           n_iter, want_normals=True)
    n_unc = int(ref["unconstrained"].sum())
    assert n_unc == 2 * 27 + 3
    vg, Cg, rep = gpu_step(ctx, sc, x, v, C, m, 0.4, n_iter)
    err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
    say(f"  parity error {err:.3e}, unconstrained {rep['n_unconstrained']} (oracle {n_unc})")
    assert err <= tol
    # N = 0 has no series, so no normals are formed and none is counted
    assert rep["n_unconstrained"] == (n_unc if n_iter > 0 else 0)
    check_report_sums(rep, x, v, C, m, vg, Cg, sc.h)
    # the unconstrained particles' affine rows are carried through the series
    unc = ref["unconstrained"].astype(bool)
    assert np.abs(Cg[:, unc]).max() > 0.1


TUNINGS = [dict(item_waves_per_cu=w, node_wg_per_cu=nw, xcd_split=x, p2g_group=g, p2g_pairs=p)
           for (w, nw, x, g, p) in ((16, 8, 0, 1, 0), (16, 8, 1, 1, 0), (16, 8, 0, 4, 0),
                                    (24, 4, 1, 4, 0), (16, 8, 0, 8, 0), (8, 32, 1, 8, 0),
                                    (1, 1, 0, 8, 0), (16, 8, 0, 1, 1), (24, 4, 1, 4, 1),
                                    (8, 32, 1, 8, 1))]


@pytest.mark.parametrize("dtype,tol", [(np.float64, FP64_TOL), (np.float32, FP32_TOL)],
                         ids=["fp64", "fp32"])
def test_every_launch_tuning_matches_oracle(ctx, dtype, tol):
    """Each launch tuning (waves per CU, XCD split, 1/4/8 work items merged per
    workgroup, paired or plain scatter) gives the oracle's result; crowded and
    sparse cell blocks mix so that runs of many items and single-item runs
    both occur, and cells hold up to a dozen particles (runs of both parities
    for the paired scatter)."""
    say("tunings", dtype.__name__)
    sc = scenes.random_blobs(41, n_bodies=3, side=9, h=0.5, spacing_frac=0.45, jitter_frac=0.3)
    x, v, C, m = cast_inputs(sc, dtype)
    ref = oracle_step(sc, x, v, C, m, 0.35, 3)
    for t in TUNINGS:
        ctx.set_tuning(dtype, sc.n, t)
        vg, Cg, _ = gpu_step(ctx, sc, x, v, C, m, 0.35, 3)
        err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
        say(f"  {t}: {err:.2e}")
        assert err <= tol
    ctx.set_tuning(dtype, sc.n, dict(item_waves_per_cu=16, node_wg_per_cu=8, xcd_split=0,
                                     p2g_group=4))


def test_set_tuning_rejects_bad_values(ctx):
    from paper_2108_02259_amd._lib import ApicError
    for bad in (dict(item_waves_per_cu=0, node_wg_per_cu=8, xcd_split=0, p2g_group=8),
                dict(item_waves_per_cu=16, node_wg_per_cu=8, xcd_split=2, p2g_group=8),
                dict(item_waves_per_cu=16, node_wg_per_cu=8, xcd_split=0, p2g_group=3),
                dict(item_waves_per_cu=16, node_wg_per_cu=8, xcd_split=0, p2g_group=4,
                     p2g_pairs=2)):
        with pytest.raises(ApicError):
            ctx.set_tuning(np.float32, 1000, bad)


def test_autotune_reads_inputs_only_and_keeps_best(ctx):
    say("autotune")
    import torch
    sc = scenes.random_blobs(42, n_bodies=2, side=12, h=1.0)
    x, v, C, m = cast_inputs(sc, np.float32)
    dev = torch.device("cuda:0")
    xt, vt, Ct, mt = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (x, v, C, m))
    bt = torch.from_numpy(sc.body.view(np.int16).copy()).to(dev)
    table = [dict(offset=0, count=sc.n, h=sc.h, mu=0.3, n_iter=2, n_bodies=sc.n_bodies)]
    best, tried = ctx.autotune(table, xt, vt, Ct, mt, bt, reps=1)
    torch.cuda.synchronize()
    assert np.array_equal(vt.cpu().numpy(), v) and np.array_equal(Ct.cpu().numpy(), C)
    assert len(tried) >= 20 and all(ms > 0 for _, ms in tried)
    assert any(t["p2g_pairs"] == 1 for t, _ in tried)  # the FP32 paired-scatter candidate
    times = [ms for _, ms in tried]
    assert tried[int(np.argmin(times))][0] == best
    assert ctx.get_tuning(np.float32, sc.n) == best
    ref = oracle_step(sc, x, v, C, m, 0.3, 2)
    vg, Cg, _ = gpu_step(ctx, sc, x, v, C, m, 0.3, 2)
    assert parity_error(vg, Cg, ref["v"], ref["C"], sc.h) <= FP32_TOL
