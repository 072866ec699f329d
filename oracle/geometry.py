"""Geometry of the multilevel decomposition (Sec. 3 "Problem and model definition",
Sec. 4.1 "Domain decomposition", Sec. 3 "Multilevel domain-decomposition structure").

A problem is described by any object with the attributes of a problem
specification: dim, lo, hi, n_points, levels, delta, K.

Readings of the paper used here:
  * grid: x_m = lo + m*step, step = (hi-lo)/(n-1), last point = hi, x-major row order
    (row n = ix*ny + iy); each operation rounded on its own;
  * centres equally spaced with the endpoints included: mu_j = lo + j*h, h = (hi-lo)/(J-1);
  * every subdomain, the two end ones included, has half-width sigma = delta*h/2
    (bounds mu -/+ (delta/2)*h, sigma = half their distance); supports are cut at the
    domain boundary;
  * a single subdomain along an axis (J = 1) is the whole axis: mu = midpoint,
    sigma = (hi-lo)/2, and its window factor along that axis is identically one;
  * a point belongs to the support I_j when |x_i - mu_i| < sigma_i on every axis (strict);
  * an L-shaped domain (Sec. 4.4 eq. helmholtz_problem) is the box without its upper-right
    quarter Q = (mid_x, hi_x] x (mid_y, hi_y], mid = (lo + hi)/2: its collocation points are the
    grid points not in Q (x > mid_x and y > mid_y both strict), and a subdomain is discarded
    when its centre lies in Q (Sec. 4.1: the rectangular subdomains outside the L are dropped;
    16 x 16 keeps 192, 8 x 8 keeps 48 as the paper counts them); the kept subdomains are
    numbered in the same level-then-x-major order.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np


def axis_coords(lo: float, hi: float, n: int) -> np.ndarray:
    if n == 1:
        return np.array([float(lo)])
    step = (float(hi) - float(lo)) / (n - 1)
    out = np.empty(n)
    for m in range(n):               # plain loop: one multiply, one add, each rounded
        out[m] = float(m) * step + float(lo)
    out[-1] = float(hi)
    return out


def is_l_shape(prob) -> bool:
    return getattr(prob, "domain", "box") == "l_shape"


def in_removed_quarter(prob, x) -> np.ndarray:
    """Points (rows of x [N, 2]) strictly inside the quarter an L-shaped domain removes."""
    mx = 0.5 * (float(prob.lo[0]) + float(prob.hi[0]))
    my = 0.5 * (float(prob.lo[1]) + float(prob.hi[1]))
    return (np.real(x[:, 0]) > mx) & (np.real(x[:, 1]) > my)


def grid(prob, n_points=None) -> np.ndarray:
    """Every point of the regular grid [N_grid, dim] in x-major order."""
    n_points = prob.n_points if n_points is None else n_points
    ax = [axis_coords(prob.lo[a], prob.hi[a], int(n_points[a])) for a in range(prob.dim)]
    if prob.dim == 1:
        return ax[0][:, None]
    X, Y = np.meshgrid(ax[0], ax[1], indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def points(prob, n_points=None) -> np.ndarray:
    """Collocation points [N, dim] in x-major order: the grid points of the domain."""
    x = grid(prob, n_points)
    if is_l_shape(prob):
        x = x[~in_removed_quarter(prob, x)]
    return x


def axis_centres(lo: float, hi: float, J: int, delta: float):
    """Centres and half-width of the J subdomains along one axis (Sec. 4.1 subdomain bounds)."""
    if J == 1:
        return np.array([0.5 * (float(lo) + float(hi))]), 0.5 * (float(hi) - float(lo))
    h = (float(hi) - float(lo)) / (J - 1)
    mu = np.array([float(j) * h + float(lo) for j in range(J)])
    sigma = delta * h / 2.0
    return mu, sigma


@dataclass
class Subdomain:
    level: int            # 0-based level index l
    j: int                # flat index within the level (x-major over (jx, jy))
    jj: tuple             # per-axis indices
    mu: np.ndarray        # centre [dim]
    sigma: np.ndarray     # half-width [dim]
    q0: int               # first global column: sum_{m<l} J_m K + j K
    single: bool          # level with a single subdomain (window == 1)
    single_axes: tuple = ()   # per axis: the level has one subdomain along that axis
    pidx: int = -1        # index among all subdomains of the full per-level grids (parameters)


def subdomains(prob) -> List[Subdomain]:
    """All subdomains in global column order q = sum_{m<l} J_m K + j K + k."""
    out = []
    q0 = 0
    pidx = 0
    lshape = is_l_shape(prob)
    for l, J in enumerate(prob.levels):
        per_axis = [axis_centres(prob.lo[a], prob.hi[a], int(J[a]), prob.delta)
                    for a in range(prob.dim)]
        single = all(int(J[a]) == 1 for a in range(prob.dim))
        j = 0
        for jj in np.ndindex(*[int(J[a]) for a in range(prob.dim)]):
            mu = np.array([per_axis[a][0][jj[a]] for a in range(prob.dim)])
            sig = np.array([per_axis[a][1] for a in range(prob.dim)])
            pidx += 1
            if lshape and in_removed_quarter(prob, mu[None, :])[0]:
                continue
            out.append(Subdomain(l, j, tuple(int(v) for v in jj), mu, sig, q0, single,
                                 tuple(int(J[a]) == 1 for a in range(prob.dim)), pidx - 1))
            q0 += prob.K
            j += 1
    return out


def kept_parameters(prob, W, b):
    """The random-feature parameters of the kept subdomains in column order, from a draw over
    every subdomain of the full per-level grids (the identity on a box)."""
    K = prob.K
    idx = np.concatenate([np.arange(sd.pidx * K, sd.pidx * K + K) for sd in subdomains(prob)])
    return np.ascontiguousarray(W[idx]), np.ascontiguousarray(b[idx])


def in_support(x: np.ndarray, sd: Subdomain) -> np.ndarray:
    """Boolean mask over points x [N, dim]: omega_j(x) != 0."""
    m = np.ones(x.shape[0], dtype=bool)
    for a in range(x.shape[1]):
        if sd.single_axes and sd.single_axes[a]:
            continue                   # one subdomain along this axis: it covers the whole axis
        m &= np.abs(x[:, a] - sd.mu[a]) < sd.sigma[a]
    return m


def support_rows(prob, x=None):
    """I_j for every subdomain: sorted global row indices (Sec. 3 index sets)."""
    x = points(prob) if x is None else x
    return [np.nonzero(in_support(x, sd))[0] for sd in subdomains(prob)]


def overlap_pairs(prob, rows=None):
    """All pairs (i <= j) of subdomains, across all levels, whose supports share a row."""
    rows = support_rows(prob) if rows is None else rows
    n = len(rows)
    sets = [set(r.tolist()) for r in rows]
    pairs = []
    for i in range(n):
        for j in range(i, n):
            if sets[i] & sets[j]:
                pairs.append((i, j))
    return pairs
