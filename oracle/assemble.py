"""Assembly of the least-squares system min ||M a - h|| (Sec. 3, eq. multilevel_ls).

Entries (Sec. 3 "Definition of the system matrices"):
    M_{n,q} = Op[omega_j phi_q C](x_n) / (sqrt(N_I) L),     h_n = f(x_n) / sqrt(N_I)
with all grid points taken as interior rows (the hard-constraint ansatz carries the
boundary condition, Sec. 4.3).  The block form follows eq. multilevel_domain_decomp:
M = sum_l sum_j V_j^T M_j W_j, with M_j = M restricted to I_j x K_j.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import basis
from . import geometry as geo


@dataclass
class Block:
    sd: geo.Subdomain
    rows: np.ndarray      # I_j: sorted global row indices
    M: np.ndarray         # M_j [len(rows), K]


def assemble_blocks(prob, W, b, x=None):
    """All blocks M_j of the system matrix.  W [N_Phi, d], b [N_Phi] in global column order."""
    x = geo.points(prob) if x is None else x
    N = x.shape[0]
    L = len(prob.levels)
    scale = 1.0 / (np.sqrt(float(N)) * L)
    subs = geo.subdomains(prob)
    ans = basis.ansatz(x, prob)
    blocks = []
    for l in range(L):
        level = [sd for sd in subs if sd.level == l]
        sums = basis.level_sum(x, level)
        for sd in level:
            rows = np.nonzero(geo.in_support(x, sd))[0]
            xs = x[rows]
            sums_r = tuple(s[rows] for s in sums)
            ans_r = tuple(a[rows] for a in ans)
            q = slice(sd.q0, sd.q0 + prob.K)
            val, grad, lap = basis.localized_function(xs, prob, sd, W[q], b[q], sums_r, ans_r)
            blocks.append(Block(sd, rows, basis.apply_operator(prob, val, grad, lap) * scale))
    return blocks


def rhs(prob, f, g=None):
    """h = f(x_n) / sqrt(N_I) over the collocation points, followed by the soft-constraint rows'
    right-hand sides: sqrt(lambda_b) g_b of the 1D conditions, or on an L-shaped domain
    sqrt(lambda_bc / N_B) g(x_b) at the N_B boundary points (g given there)."""
    N = geo.points(prob).shape[0]
    h = np.asarray(f, dtype=np.float64) / np.sqrt(float(N))
    bcs = prob.meta.get("bc", ())
    if bcs:
        h = np.concatenate([h, [wgt * val for (_, _, wgt, val) in bcs]])
    if g is not None:
        g = np.asarray(g, dtype=np.float64)
        h = np.concatenate([h, dirichlet_weight(prob, g.size) * g])
    return h


def dirichlet_weight(prob, n_b):
    """Row weight of the boundary term lambda_bc (1/N_B) sum_b (u(x_b) - g_b)^2 of the
    Helmholtz loss (Sec. 4.4): sqrt(lambda_bc / N_B)."""
    return float(np.sqrt(prob.meta["lambda_bc"] / n_b))


def dirichlet_rows(prob, W, b, xb):
    """The boundary rows B [N_B, N_Phi] of the Helmholtz loss (Sec. 3 matrix B, Sec. 4.4 with
    lambda_bc): B_{p,q} = sqrt(lambda_bc / N_B) (1/L) omega_j(x_p) phi_q(x_p), each subdomain's
    window normalised over the kept subdomains of its level at x_p."""
    xb = np.asarray(xb, dtype=np.float64)
    subs = geo.subdomains(prob)
    L = len(prob.levels)
    wgt = dirichlet_weight(prob, xb.shape[0])
    B = np.zeros((xb.shape[0], len(subs) * prob.K))
    ans = basis.ansatz(xb, prob)
    for l in range(L):
        level = [sd for sd in subs if sd.level == l]
        sums = basis.level_sum(xb, level)
        for sd in level:
            m = geo.in_support(xb, sd)
            if not m.any():
                continue
            q = slice(sd.q0, sd.q0 + prob.K)
            val, _, _ = basis.localized_function(xb[m], prob, sd, W[q], b[q],
                                                 tuple(s[m] for s in sums),
                                                 tuple(a[m] for a in ans))
            B[m, q] = wgt / L * val
    return B


def bc_rows(prob, W, b):
    """The soft-constraint rows B (Sec. 3 "Definition of the system matrices"), dense [N_B, N_Phi]:
    B_{p,q} = sqrt(lambda_b / N_B^(b)) (1/L) B_b[omega_j phi_q C](x_p) with one point per
    condition (N_B^(b) = 1), B_b the value (order 0) or the first derivative (order 1) at x_p,
    and weight sqrt(lambda_b) given per condition.  Zero rows when there are none."""
    bcs = prob.meta.get("bc", ())
    subs = geo.subdomains(prob)
    L = len(prob.levels)
    B = np.zeros((len(bcs), len(subs) * prob.K))
    for i, (xb, order, wgt, _) in enumerate(bcs):
        x = np.array([[float(xb)]])
        ans = basis.ansatz(x, prob)
        for l in range(L):
            level = [sd for sd in subs if sd.level == l]
            sums = basis.level_sum(x, level)
            for sd in level:
                if not geo.in_support(x, sd)[0]:
                    continue
                q = slice(sd.q0, sd.q0 + prob.K)
                val, grad, _ = basis.localized_function(x, prob, sd, W[q], b[q], sums, ans)
                B[i, q] = wgt / L * (val[0] if order == 0 else grad[0, :, 0])
    return B


def dense_from_blocks(blocks, n_rows, n_cols):
    M = np.zeros((n_rows, n_cols))
    for blk in blocks:
        K = blk.M.shape[1]
        M[np.ix_(blk.rows, np.arange(blk.sd.q0, blk.sd.q0 + K))] = blk.M
    return M


def assemble_dense(prob, W, b, x=None):
    """M as a dense array, each entry computed directly at every point (no block loop): the
    localised function of every subdomain is evaluated at all N points, where it is zero off
    the support."""
    x = geo.points(prob) if x is None else x
    N = x.shape[0]
    L = len(prob.levels)
    scale = 1.0 / (np.sqrt(float(N)) * L)
    subs = geo.subdomains(prob)
    M = np.zeros((N, len(subs) * prob.K))
    for l in range(L):
        level = [sd for sd in subs if sd.level == l]
        sums = basis.level_sum(x, level)
        safe = tuple(np.where(np.abs(s) > 0, s, 1.0) if i == 0 else s
                     for i, s in enumerate(sums))
        for sd in level:
            q = slice(sd.q0, sd.q0 + prob.K)
            val, grad, lap = basis.localized_function(x, prob, sd, W[q], b[q], safe)
            ent = basis.apply_operator(prob, val, grad, lap) * scale
            ent[~geo.in_support(x, sd)] = 0.0
            M[:, q] = ent
    return M


def matvec(blocks, v, n_rows):
    """y = M v = sum_j V_j^T (M_j (W_j v))."""
    y = np.zeros(n_rows)
    for blk in blocks:
        K = blk.M.shape[1]
        y[blk.rows] += blk.M @ v[blk.sd.q0:blk.sd.q0 + K]
    return y


def rmatvec(blocks, u, n_cols):
    """x = M^T u = sum_j W_j^T (M_j^T (V_j u))."""
    x = np.zeros(n_cols)
    for blk in blocks:
        K = blk.M.shape[1]
        x[blk.sd.q0:blk.sd.q0 + K] += blk.M.T @ u[blk.rows]
    return x
