"""Helpers shared by the GPU parity tests: build a problem on the device from a seeded spec and
bring device results back in the oracle's block layout."""
from __future__ import annotations

import numpy as np

from inputs import configs, feature_params
from inputs.problems import grid_points


def torch_mod():
    import torch
    return torch


def dev(a, dtype=None):
    torch = torch_mod()
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda").contiguous()


def build(spec, store_prec="fp64", f=None):
    """Define and assemble spec on the GPU; returns (problem, W, b, f)."""
    from paper_2409_01949_amd import Problem
    W, b = feature_params(spec)
    P = Problem.from_spec(spec, W, b, store_prec)
    if f is None:
        f = configs.forcing(spec)
    P.assemble(dev(f))
    return P, W, b, f


def device_blocks(P, K, store_prec="fp64"):
    """[(table_row, M_j [n_j, K] float64)] from the device block storage."""
    torch = torch_mod()
    nnz = P.sizes["nnz"]
    dt = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.bfloat16}[store_prec]
    buf = torch.empty(nnz, dtype=dt, device="cuda")
    table = P.copy_blocks(buf, prec=store_prec)
    torch.cuda.synchronize()
    host = buf.float().double().cpu().numpy() if store_prec == "bf16" else \
        buf.double().cpu().numpy()
    out = []
    for row in table:
        lvl, jx, jy, ix0, nx, iy0, ny, off = [int(v) for v in row]
        n = nx * ny
        out.append((row, host[off:off + n * K].reshape(K, n).T.copy()))
    return out


def block_rows(row, n_y):
    lvl, jx, jy, ix0, nx, iy0, ny, off = [int(v) for v in row]
    ix = np.arange(ix0, ix0 + nx)
    iy = np.arange(iy0, iy0 + ny)
    return (ix[:, None] * n_y + iy[None, :]).ravel()


def n_y(spec):
    return spec.n_points[1] if spec.dim == 2 else 1
