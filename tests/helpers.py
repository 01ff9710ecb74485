"""Shared test helpers: run a scene through the GPU library and through the
oracle on identical inputs, and measure the normwise parity error."""
from __future__ import annotations

import numpy as np

from oracle import oracle as ora

FP64_TOL = 1e-10
FP32_TOL = 2e-5


def cast_inputs(sc, dtype):
    """The scene's arrays rounded to dtype (so both sides see the same values)."""
    return (sc.x.astype(dtype), sc.v.astype(dtype), sc.C.astype(dtype), sc.m.astype(dtype))


def parity_error(v_gpu, C_gpu, v_ref, C_ref, h):
    """max(|dv|_inf, h |dC|_inf) / |v_ref|_inf (both velocity and affine part)."""
    scale = max(np.abs(v_ref).max(), 1e-300)
    ev = np.abs(v_gpu - v_ref).max() / scale
    eC = h * np.abs(C_gpu - C_ref).max() / scale
    return max(ev, eC)


def oracle_step(sc, x, v, C, m, mu, n_iter, origin=(0, 0, 0), dims=(0, 0, 0)):
    g = ora.Grid(h=sc.h, origin=origin, dims=dims)
    return ora.contact_step(g, x.astype(np.float64), v.astype(np.float64), C.astype(np.float64),
                            m.astype(np.float64), sc.body, mu, n_iter)


def gpu_step(ctx, sc, x, v, C, m, mu, n_iter, origin=(0, 0, 0), dims=(0, 0, 0)):
    import torch
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    vt = torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    Ct = torch.from_numpy(np.ascontiguousarray(C)).to(dev)
    mt = torch.from_numpy(np.ascontiguousarray(m)).to(dev)
    bt = torch.from_numpy(sc.body.view(np.int16).copy()).to(dev)
    rep = ctx.contact_step(xt, vt, Ct, mt, bt, sc.h, origin, dims, mu, n_iter)
    torch.cuda.synchronize()
    return vt.cpu().numpy(), Ct.cpu().numpy(), rep
