"""Problem specifications and the seeded draws of the random feature parameters.

A ProblemSpec fixes everything a caller decides before the method runs: the
domain box, the regular collocation grid, the decomposition sizes per level,
the width ratio, the number of random features per subdomain and the ranges
and seed of their uniform initialisation (Sec. 4.1, "Neural network
architecture and weight initialisation").
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


@dataclass(frozen=True)
class ProblemSpec:
    name: str
    dim: int                      # 1 or 2
    op: str                       # "d1" (d/dx, dim 1) | "neg_laplace" (-Laplacian, dim 2) | "identity"
    ansatz: str                   # "none" | "tanh_origin" | "tanh_box"
    ansatz_omega: float           # sharpness of the hard-constraint factor
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    n_points: Tuple[int, ...]     # regular grid, endpoints included, per axis
    levels: Tuple[Tuple[int, ...], ...]   # subdomains per axis, per level (coarse first)
    delta: float                  # width ratio
    K: int                        # random features per subdomain
    w_range: Tuple[float, float] = (-1.0, 1.0)
    b_range: Tuple[float, float] = (-1.0, 1.0)
    seed: int = 0
    meta: dict = field(default_factory=dict, compare=False, hash=False)
    # "box": the whole box [lo, hi]; "l_shape" (dim 2): the box without its upper-right quarter
    # [mid_x, hi_x] x [mid_y, hi_y], mid = (lo + hi)/2 (Sec. 4.4 eq. helmholtz_problem)
    domain: str = "box"
    # feature inputs: "local" xbar = (x - mu_j)/sigma_l (the default reading), "global" xbar = x
    input_norm: str = "local"

    @property
    def n_levels(self) -> int:
        return len(self.levels)

    @property
    def n_rows(self) -> int:
        return int(np.prod(self.n_points))

    def n_subdomains(self) -> int:
        return int(sum(int(np.prod(J)) for J in self.levels))


def n_phi(spec: ProblemSpec) -> int:
    """Random-feature parameters drawn for a problem: K for every subdomain of every level's full
    J_x x J_y grid (N_Phi = sum_l J_l K on a box; on an L-shaped domain the draw also covers the
    subdomains the method discards, whose parameters are then not used)."""
    return spec.n_subdomains() * spec.K


def feature_params(spec: ProblemSpec):
    """Seeded uniform draws of the fixed hidden weights W [N_Phi, dim] and biases b [N_Phi].

    Rows follow the global column order q (level, then subdomain j in x-major
    order, then feature k) of each level's full subdomain grid.  W is drawn first, then b, from
    one PCG64 stream.
    """
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    n = n_phi(spec)
    W = rng.uniform(spec.w_range[0], spec.w_range[1], size=(n, spec.dim))
    b = rng.uniform(spec.b_range[0], spec.b_range[1], size=n)
    return np.ascontiguousarray(W, dtype=np.float64), np.ascontiguousarray(b, dtype=np.float64)


def grid_axes(spec: ProblemSpec, n_points=None):
    """Per-axis coordinates of the regular grid: x_m = lo + m*step, last point = hi.

    step = (hi - lo)/(n - 1), each operation rounded separately (no fused
    multiply-add), so that every implementation reproduces the same doubles.
    """
    n_points = spec.n_points if n_points is None else n_points
    axes = []
    for a in range(spec.dim):
        n = int(n_points[a])
        lo, hi = float(spec.lo[a]), float(spec.hi[a])
        if n == 1:
            axes.append(np.array([lo]))
            continue
        step = (hi - lo) / (n - 1)
        m = np.arange(n, dtype=np.float64)
        x = m * step
        x = x + lo
        x[-1] = hi
        axes.append(x)
    return axes


def grid_points(spec: ProblemSpec, n_points=None) -> np.ndarray:
    """All grid points [N, dim], x-major order (row n = ix*ny + iy)."""
    axes = grid_axes(spec, n_points)
    if spec.dim == 1:
        return axes[0][:, None].copy()
    X, Y = np.meshgrid(axes[0], axes[1], indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def mlp_init(dims, seed):
    """Flat FP32 parameters [W_0, b_0, W_1, b_1, ...] of a tanh network: W_l ~ U(-a, a) with
    a = 1/sqrt(fan_in) (LeCun-uniform scale), b_l = 0; W_l [dims[l+1], dims[l]] row-major."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for n_in, n_out in zip(dims[:-1], dims[1:]):
        a = 1.0 / np.sqrt(n_in)
        parts.append(rng.uniform(-a, a, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)


def l_shape_boundary(spec: ProblemSpec, per_unit: int):
    """Boundary collocation points of the L-shaped domain (Sec. 4.4 baseline: points spread
    evenly along each boundary segment, 80 on the long segments and 40 on the short ones of the
    unit square's L): the six segments counter-clockwise from (lo_x, lo_y), each of length s
    holding round(per_unit s) points at the centres of equal sub-intervals (so no corner is
    taken twice and every segment has the same spacing).  Returns [N_B, 2]."""
    lo, hi = np.asarray(spec.lo, float), np.asarray(spec.hi, float)
    mid = 0.5 * (lo + hi)
    corners = [(lo[0], lo[1]), (hi[0], lo[1]), (hi[0], mid[1]), (mid[0], mid[1]),
               (mid[0], hi[1]), (lo[0], hi[1]), (lo[0], lo[1])]
    out = []
    for (x0, y0), (x1, y1) in zip(corners[:-1], corners[1:]):
        length = abs(x1 - x0) + abs(y1 - y0)
        n = int(round(per_unit * length))
        t = (np.arange(n, dtype=np.float64) + 0.5) / n
        out.append(np.stack([x0 + t * (x1 - x0), y0 + t * (y1 - y0)], axis=1))
    return np.concatenate(out)
