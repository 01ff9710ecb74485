"""GPU parity of the method's variants and the extended boundary against the
FP64 oracle: PIC transfers and the separation-only rule (scene flags),
caller-supplied normals, the resident driver's mechanical acceleration,
bodies per grid node, the reference point of L, and input validation."""
import sys

import numpy as np
import pytest

from helpers import FP32_TOL, FP64_TOL, cast_inputs, parity_error
from oracle import oracle as ora
from paper_2108_02259_amd import _lib, scenes

pytestmark = pytest.mark.gpu

PRECISIONS = [(np.float64, FP64_TOL), (np.float32, FP32_TOL)]
PIDS = ["fp64", "fp32"]


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
    return torch.from_numpy(np.ascontiguousarray(body).view(np.int16).copy()).cuda()


def batched(ctx, rows, x, v, C, m, body, normals=None):
    xt, vt, Ct, mt = dev(x, v, C, m)
    nt = None if normals is None else dev(normals)[0]
    reps = ctx.contact_step_batched(rows, xt, vt, Ct, mt, body_dev(body), normals=nt)
    return vt.cpu().numpy(), Ct.cpu().numpy(), reps


def ora_grid(sc, flags=0):
    return ora.Grid(h=sc.h, origin=sc.origin, dims=sc.dims,
                    transfer=ora.TRANSFER_PIC if flags & _lib.PIC else ora.TRANSFER_APIC,
                    rule=ora.RULE_SEPARATE if flags & _lib.RULE_SEPARATE else ora.RULE_COULOMB)


def f64(*a):
    return [np.asarray(b, dtype=np.float64) for b in a]


# ---------------------------------------------------------------------------
# PIC transfers and the Section 2.3 rule, batched with the default method
# ---------------------------------------------------------------------------

FLAG_CASES = [("apic_coulomb", 0), ("pic_coulomb", _lib.PIC),
              ("apic_separate", _lib.RULE_SEPARATE), ("pic_separate", _lib.PIC | _lib.RULE_SEPARATE)]


@pytest.mark.parametrize("dtype,tol", PRECISIONS, ids=PIDS)
def test_scene_flags_match_the_oracle_in_one_batch(ctx, dtype, tol):
    """Four scenes, one per (transfer, rule) pair, in one batched call."""
    scs = [scenes.random_blobs(200 + i, n_bodies=2 + i % 2, side=6, h=0.5) for i in range(4)]
    mus, Ns = (0.3, 0.0, 0.5, 1.0), (3, 2, 4, 1)
    x, v, C, m, body, rows, _ = scenes.pack(scs, dtype)
    for row, (_, fl), mu, N in zip(rows, FLAG_CASES, mus, Ns):
        row.update(flags=fl, mu=mu, n_iter=N)
    vg, Cg, reps = batched(ctx, rows, x, v, C, m, body)
    for sc, row, (name, fl), rep in zip(scs, rows, FLAG_CASES, reps):
        sl = slice(row["offset"], row["offset"] + row["count"])
        xs, vs, Cs, ms = f64(x[:, sl], v[:, sl], C[:, sl], m[sl])
        ref = ora.contact_step(ora_grid(sc, fl), xs, vs, Cs, ms, sc.body, row["mu"],
                               row["n_iter"])
        err = parity_error(vg[:, sl], Cg[:, sl], ref["v"], ref["C"], sc.h)
        say(f"  {name}: err {err:.2e}")
        assert err <= tol
        if fl & _lib.PIC:  # C passes through bitwise
            np.testing.assert_array_equal(Cg[:, sl], C[:, sl])
        # linear momentum is conserved by every variant; L only with APIC
        dP = np.abs(np.array(rep["P_after"]) - rep["P_before"]).max() / rep["P_scale"]
        dL = np.abs(np.array(rep["L_after"]) - rep["L_before"]).max() / rep["L_scale"]
        say(f"    drift P {dP:.1e} L {dL:.1e}")
        assert dP <= (1e-12 if dtype == np.float64 else 1e-5)
        if not fl & _lib.PIC:
            assert dL <= (1e-12 if dtype == np.float64 else 1e-5)


def test_pic_loses_angular_momentum_on_the_gpu(ctx):
    """The paper's contrast (Section 2.2): a spinning body through the PIC
    step loses angular momentum, through the APIC step keeps it."""
    rng = np.random.default_rng(1)
    pts = scenes.lattice_box(6, 6, 6, 0.5, (0.25, 0.25, 0.25), rng, 0.05)
    n = pts.shape[1]
    c = pts.mean(1, keepdims=True)
    w = np.array([0.2, -0.5, 1.0])
    v = np.cross(np.broadcast_to(w, pts.T.shape), (pts - c).T).T
    C = np.repeat(scenes.skew(w).reshape(9, 1), n, 1)
    body = np.zeros(n, np.uint16)
    drift = {}
    for fl in (0, _lib.PIC):
        row = dict(offset=0, count=n, h=0.5, mu=0.0, n_iter=0, n_bodies=1, flags=fl,
                   x_ref=tuple(c[:, 0]))
        _, _, reps = batched(ctx, [row], pts, v, C, np.ones(n), body)
        r = reps[0]
        drift[fl] = np.abs(np.array(r["L_after"]) - r["L_before"]).max() / r["L_scale"]
    say(f"  L drift APIC {drift[0]:.1e} PIC {drift[_lib.PIC]:.1e}")
    assert drift[0] <= 1e-12 and drift[_lib.PIC] > 1e-3


@pytest.mark.parametrize("dtype,tol", PRECISIONS, ids=PIDS)
def test_separation_rule_full_size_slab_block(ctx, dtype, tol):
    """The 1,114,112-particle slab + block with the Section 2.3 rule."""
    sc = scenes.slab_block(mu=0.3)
    x, v, C, m = cast_inputs(sc, dtype)
    row = dict(offset=0, count=sc.n, h=sc.h, mu=sc.mu, n_iter=sc.n_iter, n_bodies=2,
               flags=_lib.RULE_SEPARATE)
    vg, Cg, _ = batched(ctx, [row], x, v, C, m, sc.body)
    ref = ora.contact_step(ora_grid(sc, _lib.RULE_SEPARATE), *f64(x, v, C, m), sc.body,
                           sc.mu, sc.n_iter)
    err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
    say(f"  slab_block separate {np.dtype(dtype).name}: {err:.2e}")
    assert err <= tol


# ---------------------------------------------------------------------------
# caller-supplied normals (Section 2.3: area-weighted FE face normals)
# ---------------------------------------------------------------------------

def block_on_plane_scene(seed, side=6):
    rng = np.random.default_rng(seed)
    plane = scenes.lattice_box(side + 6, side + 6, 3, 1.0, (0.5, 0.5, 0.5), rng, 0.0)
    block = scenes.lattice_box(side, side, side, 1.0, (3.5, 3.5, 3.5), rng, 0.0)
    x = np.concatenate([plane, block], 1)
    n_p, n_b = plane.shape[1], block.shape[1]
    v = np.zeros((3, n_p + n_b))
    v[:, n_p:] = rng.normal(size=(3, n_b)) * 0.3 + np.array([[2.0], [0.3], [-0.5]])
    C = np.concatenate([np.zeros((9, n_p)), rng.normal(size=(9, n_b)) * 0.2], 1)
    m = np.concatenate([np.full(n_p, 4.0), np.full(n_b, 1.0)])
    body = np.concatenate([np.zeros(n_p, np.uint16), np.ones(n_b, np.uint16)])
    nrm = np.concatenate([scenes.box_face_normals(side + 6, side + 6, 3),
                          scenes.box_face_normals(side, side, side)], 1)
    return scenes.Scene(x, v, C, m, body, 1.0, mu=0.4, n_iter=3), nrm


@pytest.mark.parametrize("dtype,tol", PRECISIONS, ids=PIDS)
def test_given_face_normals_match_the_oracle(ctx, dtype, tol):
    sc, nrm = block_on_plane_scene(5)
    x, v, C, m = cast_inputs(sc, dtype)
    nd = nrm.astype(dtype)
    row = dict(offset=0, count=sc.n, h=sc.h, mu=sc.mu, n_iter=sc.n_iter, n_bodies=2)
    vg, Cg, reps = batched(ctx, [row], x, v, C, m, sc.body, normals=nd)
    ref = ora.contact_step(ora.Grid(h=sc.h), *f64(x, v, C, m), sc.body, sc.mu, sc.n_iter,
                           normals_in=nd.astype(np.float64), want_normals=True)
    err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
    n_unc = int(ref["unconstrained"].sum())
    say(f"  face normals: err {err:.2e}, unconstrained {reps[0]['n_unconstrained']} ({n_unc})")
    assert err <= tol
    assert reps[0]["n_unconstrained"] == n_unc > 0
    # they differ from the mass-gradient normals' result
    ref2 = ora.contact_step(ora.Grid(h=sc.h), *f64(x, v, C, m), sc.body, sc.mu, sc.n_iter)
    assert parity_error(vg, Cg, ref2["v"], ref2["C"], sc.h) > 100 * tol


@pytest.mark.parametrize("dtype,tol", PRECISIONS, ids=PIDS)
def test_given_random_normals_with_pic_and_separation(ctx, dtype, tol):
    sc = scenes.random_blobs(210, n_bodies=3, side=5, h=0.5)
    rng = np.random.default_rng(211)
    nrm = rng.normal(size=(3, sc.n))
    nrm /= np.sqrt((nrm ** 2).sum(0))
    nrm[:, rng.uniform(size=sc.n) < 0.2] = 0.0
    x, v, C, m = cast_inputs(sc, dtype)
    nd = nrm.astype(dtype)
    for fl in (0, _lib.PIC | _lib.RULE_SEPARATE):
        row = dict(offset=0, count=sc.n, h=sc.h, mu=0.35, n_iter=3, n_bodies=3, flags=fl)
        vg, Cg, _ = batched(ctx, [row], x, v, C, m, sc.body, normals=nd)
        ref = ora.contact_step(ora_grid(sc, fl), *f64(x, v, C, m), sc.body, 0.35, 3,
                               normals_in=nd.astype(np.float64))
        err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
        say(f"  random normals flags {fl}: {err:.2e}")
        assert err <= tol


# ---------------------------------------------------------------------------
# mechanical acceleration in the resident driver (Section 2.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,tol", PRECISIONS, ids=PIDS)
def test_driver_acceleration_follows_the_oracle_driver(ctx, dtype, tol):
    """Each step: Vbar = V + dt {a, 0} (rounded to the precision), V <- S(Vbar),
    x <- x + dt v; three steps teacher-forced against the oracle."""
    from paper_2108_02259_amd.contact import Sim
    sc = scenes.random_blobs(220, n_bodies=2, side=6, h=0.5)
    a = np.array([0.3, -9.81, 1.5])
    dt = 0.01
    x, v, C, m = cast_inputs(sc, dtype)
    row = dict(offset=0, count=sc.n, h=sc.h, mu=0.3, n_iter=2, n_bodies=2, accel=tuple(a))
    sim = Sim(ctx, [row], [dt], *dev(x, v, C, m), body_dev(sc.body))
    for step in range(3):
        sim.step(1, graph=step > 0)
        xg, vg, Cg = (t.cpu().numpy() for t in sim.read())
        vbar = (v.astype(np.float64) + dt * a.reshape(3, 1)).astype(dtype)
        ref = ora.contact_step(ora.Grid(h=sc.h), *f64(x, vbar, C, m), sc.body, 0.3, 2)
        err = parity_error(vg, Cg, ref["v"], ref["C"], sc.h)
        say(f"  step {step}: err {err:.2e}")
        assert err <= tol
        x_ref = x.astype(np.float64) + (dt * vg.astype(np.float64)).astype(dtype)
        assert np.abs(xg - x_ref.astype(dtype)).max() <= tol * max(1.0, np.abs(x).max())
        x, v, C = xg, vg, Cg  # teacher-forced: the next step starts from the GPU's state
    reps, drift, steps = sim.report()
    sim.close()
    assert steps == 3
    # the report's "before" is Vbar: the contact step itself conserves momentum
    assert drift[0][0] <= (1e-12 if dtype == np.float64 else 1e-5)


# ---------------------------------------------------------------------------
# bodies per grid node, reference point of L, validation
# ---------------------------------------------------------------------------

def bodies_per_node_brute_force(x, body, h, origin=(0.0, 0.0, 0.0)):
    """Most distinct bodies whose particles give some node a nonzero weight:
    integer geometry only (cells, stencil offsets, and the one weight that can
    vanish, t^2/4 at t = 0)."""
    xi = (np.asarray(x, dtype=np.float64) - np.asarray(origin).reshape(3, 1)) / h
    c = np.floor(xi).astype(np.int64)
    t = xi - c
    nodes = {}
    for p in range(x.shape[1]):
        offs = [[o for o in range(4) if not (o == 3 and t[d, p] == 0.0)] for d in range(3)]
        for a in offs[0]:
            for b in offs[1]:
                for cc in offs[2]:
                    key = (c[0, p] - 1 + a, c[1, p] - 1 + b, c[2, p] - 1 + cc)
                    nodes.setdefault(key, set()).add(int(body[p]))
    return max(len(s) for s in nodes.values())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_max_bodies_per_node(ctx, dtype):
    sc = scenes.spheres(n_spheres=14, box_cells=28.0, radius_cells=3.0)
    x, v, C, m = cast_inputs(sc, dtype)
    expect = bodies_per_node_brute_force(x, sc.body, sc.h)
    row = dict(offset=0, count=sc.n, h=sc.h, mu=0.4, n_iter=2, n_bodies=sc.n_bodies)
    _, _, reps = batched(ctx, [row], x, v, C, m, sc.body)
    say(f"  spheres: max bodies per node {reps[0]['max_bodies_per_node']} (expect {expect})")
    assert expect >= 2
    assert reps[0]["max_bodies_per_node"] == expect
    one = scenes.random_blobs(230, n_bodies=1, side=4, h=0.5)
    x1, v1, C1, m1 = cast_inputs(one, dtype)
    row1 = dict(offset=0, count=one.n, h=one.h, mu=0.4, n_iter=1, n_bodies=1)
    _, _, reps1 = batched(ctx, [row1], x1, v1, C1, m1, one.body)
    assert reps1[0]["max_bodies_per_node"] == 1


def test_reported_L_is_about_x_ref(ctx):
    sc = scenes.random_blobs(240, n_bodies=2, side=5, h=0.5)
    xr = (3.25, -1.5, 7.0)
    row = dict(offset=0, count=sc.n, h=sc.h, mu=0.3, n_iter=2, n_bodies=2, x_ref=xr)
    vg, Cg, reps = batched(ctx, [row], sc.x, sc.v, sc.C, sc.m, sc.body)
    for key, (vv, CC) in (("before", (sc.v, sc.C)), ("after", (vg, Cg))):
        ref = ora.momentum(sc.x, vv, CC, sc.m, sc.h, xr)
        assert np.abs(np.array(reps[0][f"L_{key}"]) - ref["L"]).max() <= 1e-12 * ref["L_scale"]


def test_non_finite_and_bad_inputs_are_refused_and_leave_v_C(ctx):
    from paper_2108_02259_amd._lib import ApicError
    sc = scenes.random_blobs(250, n_bodies=2, side=4, h=0.5)
    row = dict(offset=0, count=sc.n, h=sc.h, mu=0.3, n_iter=2, n_bodies=2)
    cases = []
    v = sc.v.copy(); v[1, 7] = np.nan; cases.append(("v", v, sc.C, sc.m, sc.body, _lib.E_INVALID))
    C = sc.C.copy(); C[4, 3] = np.inf; cases.append(("C", sc.v, C, sc.m, sc.body, _lib.E_INVALID))
    m = sc.m.copy(); m[5] = 0.0; cases.append(("m", sc.v, sc.C, m, sc.body, _lib.E_INVALID))
    b = sc.body.copy(); b[9] = 2; cases.append(("body", sc.v, sc.C, sc.m, b, _lib.E_BODY))
    for name, vv, CC, mm, bb, code in cases:
        xt, vt, Ct, mt = dev(sc.x, vv, CC, mm)
        with pytest.raises(ApicError) as e:
            ctx.contact_step_batched([row], xt, vt, Ct, mt, body_dev(bb))
        assert e.value.code == code, name
        np.testing.assert_array_equal(vt.cpu().numpy(), vv)
        np.testing.assert_array_equal(Ct.cpu().numpy(), CC)
