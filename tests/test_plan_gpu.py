"""GPU tests of the planned contact step (apic_plan_*): the step is enqueued
with no host synchronisation on a torch stream, captured into a graph and
replayed, each replay matching the oracle; a device scene table and device
reports; a table that does not match the plan and a batch that outgrows it
are reported through the device status with v and C untouched."""
import sys

import numpy as np
import pytest

from helpers import FP32_TOL, FP64_TOL, cast_inputs, parity_error
from oracle import oracle as ora
from paper_2108_02259_amd import _lib, scenes

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


def batch(dtype, seeds=(300, 301, 302)):
    scs = [scenes.random_blobs(s, n_bodies=2 + s % 2, side=5 + s % 3, h=0.5) for s in seeds]
    x, v, C, m, body, rows, _ = scenes.pack(scs, dtype)
    for i, row in enumerate(rows):
        row.update(mu=0.2 + 0.3 * i, n_iter=1 + i)
    return scs, x, v, C, m, body, rows


def oracle_rows(scs, rows, x, v, C, m, flags=None):
    out_v, out_C = np.zeros(v.shape), np.zeros(C.shape)
    for k, (sc, row) in enumerate(zip(scs, rows)):
        sl = slice(row["offset"], row["offset"] + row["count"])
        fl = (flags or [0] * len(rows))[k]
        g = ora.Grid(h=sc.h, transfer=ora.TRANSFER_PIC if fl & _lib.PIC else ora.TRANSFER_APIC,
                     rule=ora.RULE_SEPARATE if fl & _lib.RULE_SEPARATE else ora.RULE_COULOMB)
        f = lambda a: np.asarray(a, dtype=np.float64)
        r = ora.contact_step(g, f(x[:, sl]), f(v[:, sl]), f(C[:, sl]), f(m[sl]), sc.body,
                             row["mu"], row["n_iter"])
        out_v[:, sl], out_C[:, sl] = r["v"], r["C"]
    return out_v, out_C


def check_rows(scs, rows, vg, Cg, ref_v, ref_C, tol):
    for sc, row in zip(scs, rows):
        sl = slice(row["offset"], row["offset"] + row["count"])
        err = parity_error(vg[:, sl], Cg[:, sl], ref_v[:, sl], ref_C[:, sl], sc.h)
        assert err <= tol, err


@pytest.mark.parametrize("dtype,tol", [(np.float64, FP64_TOL), (np.float32, FP32_TOL)],
                         ids=["fp64", "fp32"])
def test_planned_step_captured_in_a_graph_and_replayed(ctx, dtype, tol):
    import torch
    from paper_2108_02259_amd.contact import Plan, reports_from_bytes
    scs, x, v, C, m, body, rows = batch(dtype)
    ref_v, ref_C = oracle_rows(scs, rows, x, v, C, m)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xt, vt, Ct, mt = d(x), d(v), d(C), d(m)
    bt = torch.from_numpy(body.view(np.int16).copy()).cuda()
    v0, C0 = vt.clone(), Ct.clone()
    rep_dev = torch.zeros(len(rows) * 160, dtype=torch.uint8, device="cuda")
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = Plan(ctx, rows, xt, bt)
        plan.step(xt, vt, Ct, mt, bt, reports_dev=rep_dev, status_dev=status)  # eager
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    check_rows(scs, rows, vt.cpu().numpy(), Ct.cpu().numpy(), ref_v, ref_C, tol)
    g = torch.cuda.CUDAGraph()
    vt.copy_(v0)
    Ct.copy_(C0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.step(xt, vt, Ct, mt, bt, reports_dev=rep_dev, status_dev=status)
    for k in range(3):
        vt.copy_(v0)               # eager work between the replays
        Ct.copy_(C0)
        status.fill_(12345)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        vg, Cg = vt.cpu().numpy(), Ct.cpu().numpy()
        say(f"  replay {k}: status {int(status.item())}")
        assert int(status.item()) == 0
        check_rows(scs, rows, vg, Cg, ref_v, ref_C, tol)
        reps = reports_from_bytes(rep_dev.cpu(), len(rows))
        for row, rep in zip(rows, reps):
            sl = slice(row["offset"], row["offset"] + row["count"])
            P_out = (m[sl].astype(np.float64) * vg[:, sl].astype(np.float64)).sum(1)
            assert rep["n_particles"] == row["count"]
            assert np.abs(np.array(rep["P_after"]) - P_out).max() <= 1e-12 * rep["P_scale"]
            assert rep["max_bodies_per_node"] >= 2
    del g
    plan.close()


def test_device_scene_table_changes_mu_and_flags(ctx):
    import torch
    from paper_2108_02259_amd.contact import Plan, scene_table_bytes
    scs, x, v, C, m, body, rows = batch(np.float64)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xt, mt = d(x), d(m)
    bt = torch.from_numpy(body.view(np.int16).copy()).cuda()
    plan = Plan(ctx, rows, xt, bt)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    rows2 = [dict(r) for r in rows]
    flags = [_lib.PIC, _lib.RULE_SEPARATE, 0]
    for r, fl in zip(rows2, flags):
        r.update(mu=r["mu"] * 0.5, flags=fl, n_iter=max(0, r["n_iter"] - 1))
    tab = torch.frombuffer(bytearray(scene_table_bytes(rows2)), dtype=torch.uint8).cuda()
    vt, Ct = d(v), d(C)
    plan.step(xt, vt, Ct, mt, bt, scenes_dev=tab, status_dev=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    ref_v, ref_C = oracle_rows(scs, rows2, x, v, C, m, flags)
    check_rows(scs, rows2, vt.cpu().numpy(), Ct.cpu().numpy(), ref_v, ref_C, FP64_TOL)
    # a table that does not match the plan: nothing written, E_TABLE
    bad = [dict(r) for r in rows]
    bad[1]["n_iter"] = 40
    tab = torch.frombuffer(bytearray(scene_table_bytes(bad)), dtype=torch.uint8).cuda()
    vt, Ct = d(v), d(C)
    plan.step(xt, vt, Ct, mt, bt, scenes_dev=tab, status_dev=status)
    torch.cuda.synchronize()
    assert int(status.item()) == _lib.E_TABLE
    np.testing.assert_array_equal(vt.cpu().numpy(), v)
    np.testing.assert_array_equal(Ct.cpu().numpy(), C)
    plan.close()


def test_planned_step_that_outgrows_its_plan_reports_resize(ctx):
    import torch
    from paper_2108_02259_amd.contact import Plan
    scs, x, v, C, m, body, rows = batch(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    bt = torch.from_numpy(body.view(np.int16).copy()).cuda()
    plan = Plan(ctx, rows, d(x), bt, headroom=1.2)
    x2 = x.copy()
    sl = slice(rows[0]["offset"], rows[0]["offset"] + rows[0]["count"])
    x2[:, sl][:, scs[0].body == 1] += 300.0     # spread one scene far apart
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    vt, Ct = d(v), d(C)
    plan.step(d(x2), vt, Ct, d(m), bt, status_dev=status)
    torch.cuda.synchronize()
    assert int(status.item()) == _lib.E_RESIZE
    np.testing.assert_array_equal(vt.cpu().numpy(), v)
    np.testing.assert_array_equal(Ct.cpu().numpy(), C)
    # the unchanged batch still steps
    plan.step(d(x), vt, Ct, d(m), bt, status_dev=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    ref_v, ref_C = oracle_rows(scs, rows, x, v, C, m)
    check_rows(scs, rows, vt.cpu().numpy(), Ct.cpu().numpy(), ref_v, ref_C, FP32_TOL)
    plan.close()
