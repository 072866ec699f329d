"""Least-squares solvers for min ||M a - h|| (Sec. 3 eq. multilevel_ls; Sec. 4.1 "Optimisation
and solvers": the method solves it with the LSQR algorithm).

  * householder_lstsq  dense Householder QR and back substitution (tiny full-rank systems)
  * lsqr               Paige & Saunders (1982), damp = 0, stopping tests on ||r|| and ||A^T r||
  * cgls               conjugate gradients on the normal equations in factored form (CGLS)
  * gram_blocks        G_ij = M_i^T M_j over the shared rows I_i and I_j, for overlapping pairs
  * normal_cg          CG on G a = M^T h with G held as its upper blocks
  * refine             FP64 residual refinement around a low-precision normal-equation solve

The matrix enters through callables matvec(v) -> M v and rmatvec(u) -> M^T u.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


# ---------------------------------------------------------------- dense QR

def householder_lstsq(M: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Minimiser of ||M a - h|| for full column rank M via Householder QR."""
    A = np.array(M, dtype=np.float64, copy=True)
    y = np.array(h, dtype=np.float64, copy=True)
    m, n = A.shape
    if m < n:
        raise ValueError("householder_lstsq needs rows >= cols")
    for k in range(n):
        col = A[k:, k]
        alpha = np.linalg.norm(col)
        if alpha == 0.0:
            continue
        sign = 1.0 if col[0] >= 0 else -1.0
        vk = col.copy()
        vk[0] += sign * alpha
        vk /= np.linalg.norm(vk)
        A[k:, k:] -= 2.0 * np.outer(vk, vk @ A[k:, k:])
        y[k:] -= 2.0 * vk * (vk @ y[k:])
    R = np.triu(A[:n, :n])
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


# ---------------------------------------------------------------- LSQR

@dataclass
class LsqrResult:
    x: np.ndarray
    istop: int
    itn: int
    rnorm: float
    arnorm: float
    anorm: float
    xnorm: float
    snapshots: Dict[int, np.ndarray] = field(default_factory=dict)
    history: List[tuple] = field(default_factory=list)
    # (alpha_{i+1}, beta_{i+1}) of the bidiagonalisation: entry 0 from the start, entry i after
    # step i
    bidiag: List[tuple] = field(default_factory=list)


def lsqr(matvec: Callable, rmatvec: Callable, h: np.ndarray, n: int, atol=1e-8, btol=1e-8,
         iter_lim=15000, x0: Optional[np.ndarray] = None, snapshot_at=(), callback=None,
         record=False) -> LsqrResult:
    """Paige-Saunders LSQR with damp = 0 and no condition-number limit.

    Golub-Kahan bidiagonalisation
        beta_1 u_1 = h - M x0,  alpha_1 v_1 = M^T u_1,
        beta_{i+1} u_{i+1} = M v_i - alpha_i u_i,  alpha_{i+1} v_{i+1} = M^T u_{i+1} - beta_{i+1} v_i,
    a plane rotation per step, x_i = x_{i-1} + (phi_i/rho_i) w_i, w_{i+1} = v_{i+1} - (theta_{i+1}/rho_i) w_i.
    Stop codes: 0 x0 solves exactly, 1 ||r|| <= btol ||h|| + atol ||A|| ||x||,
    2 ||A^T r|| <= atol ||A|| ||r||, 4/5 the same tests at machine precision, 7 iteration limit.
    """
    eps = np.finfo(np.float64).eps
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    u = np.array(h, dtype=np.float64, copy=True)
    bnorm = np.linalg.norm(u)
    if x0 is not None:
        u = u - matvec(x)
    beta = np.linalg.norm(u)
    snaps = {}
    hist = []
    if beta > 0:
        u = u / beta
        v = rmatvec(u)
        alpha = np.linalg.norm(v)
    else:
        v = np.zeros(n)
        alpha = 0.0
    if alpha > 0:
        v = v / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    anorm = 0.0
    rnorm, arnorm = beta, alpha * beta
    bidiag = [(alpha, beta)]
    if arnorm == 0.0:
        return LsqrResult(x, 0, 0, rnorm, arnorm, anorm, float(np.linalg.norm(x)), snaps, hist,
                          bidiag)
    if bnorm == 0.0:
        bnorm = beta
    istop, itn = 0, 0
    while itn < iter_lim:
        itn += 1
        u = matvec(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0:
            u = u / beta
            anorm = np.sqrt(anorm * anorm + alpha * alpha + beta * beta)
            v = rmatvec(u) - beta * v
            alpha = np.linalg.norm(v)
            if alpha > 0:
                v = v / alpha
        bidiag.append((alpha, beta))
        rho = np.sqrt(rhobar * rhobar + beta * beta)
        c = rhobar / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        xnorm = float(np.linalg.norm(x))
        rnorm = phibar
        arnorm = alpha * abs(c) * phibar
        test1 = rnorm / bnorm
        test2 = arnorm / (anorm * rnorm + eps)
        t1 = test1 / (1.0 + anorm * xnorm / bnorm)
        rtol = btol + atol * anorm * xnorm / bnorm
        if record:
            hist.append((itn, rnorm, arnorm, anorm, xnorm))
        if itn in snapshot_at:
            snaps[itn] = x.copy()
        if callback is not None and callback(itn, x):
            istop = 8
            break
        if 1.0 + test2 <= 1.0:
            istop = 5
        if 1.0 + t1 <= 1.0:
            istop = 4
        if test2 <= atol:
            istop = 2
        if test1 <= rtol:
            istop = 1
        if istop != 0:
            break
    else:
        istop = 7
    return LsqrResult(x, istop, itn, rnorm, arnorm, anorm, float(np.linalg.norm(x)), snaps, hist,
                      bidiag)


def bidiag_singular_values(bidiag, k):
    """Singular values (descending) of the (k+1) x k lower bidiagonal B_k of the Golub-Kahan
    process: alpha_1 .. alpha_k on the diagonal, beta_2 .. beta_{k+1} below it.  B_k = U^T M V
    with orthonormal U (k+1 columns) and V (k columns), so its singular values lie between the
    extreme singular values of M, and equal them once the process has spanned M's row space."""
    B = np.zeros((k + 1, k))
    for i in range(k):
        B[i, i] = bidiag[i][0]
        B[i + 1, i] = bidiag[i + 1][1]
    return np.linalg.svd(B, compute_uv=False)


def bidiag_extreme_singular_values(bidiag, k):
    """(sigma_max, sigma_min) of the same B_k without forming it, for long runs (k in the
    thousands, where the dense SVD costs O(k^3)).  The symmetric matrix [0 B_k; B_k^T 0] of
    order 2k+1 has eigenvalues +-sigma_i and one 0 (Golub and Kahan 1965); reordering its rows
    and columns as (e_1, f_1, e_2, f_2, ..., e_{k+1}) makes it tridiagonal with zero diagonal and
    off-diagonal alpha_1, beta_2, alpha_2, beta_3, ..., alpha_k, beta_{k+1}.  Its largest
    eigenvalue is sigma_max and its (k+1)-th smallest (index k+1 from 0, after the k negative
    ones and the zero) is sigma_min, found by LAPACK bisection (stebz) with the tightest
    absolute tolerance."""
    from scipy.linalg import eigvalsh_tridiagonal
    e = np.empty(2 * k)
    for i in range(k):
        e[2 * i] = bidiag[i][0]
        e[2 * i + 1] = bidiag[i + 1][1]
    d = np.zeros(2 * k + 1)
    tol = 2.0 * np.finfo(np.float64).tiny
    top = eigvalsh_tridiagonal(d, e, select="i", select_range=(2 * k, 2 * k), tol=tol,
                               lapack_driver="stebz")
    low = eigvalsh_tridiagonal(d, e, select="i", select_range=(k + 1, k + 1), tol=tol,
                               lapack_driver="stebz")
    return float(top[0]), float(low[0])


# ---------------------------------------------------------------- CGLS

@dataclass
class CglsResult:
    x: np.ndarray
    istop: int
    itn: int
    rnorm: float
    snorm: float
    snapshots: Dict[int, np.ndarray] = field(default_factory=dict)


def cgls(matvec, rmatvec, h, n, anorm_f, atol=1e-8, btol=1e-8, iter_lim=15000, x0=None,
         snapshot_at=(), callback=None) -> CglsResult:
    """CGLS (Bjorck, Numerical Methods for Least Squares Problems, sec. 7.4):
        r = h - M x, s = M^T r, p = s, gamma = ||s||^2;
        t = M p, a = gamma/||t||^2, x += a p, r -= a t, s = M^T r, p = s + (||s||^2/gamma) p.
    Stop: 1 if ||r|| <= btol ||h||, 2 if ||s|| <= atol ||M||_F ||r||, 7 at the iteration limit."""
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = np.array(h, dtype=np.float64, copy=True)
    bnorm = np.linalg.norm(r)
    if x0 is not None:
        r = r - matvec(x)
    s = rmatvec(r)
    p = s.copy()
    gamma = float(s @ s)
    snaps = {}
    istop, itn = 0, 0
    rnorm = float(np.linalg.norm(r))
    if gamma == 0.0:
        return CglsResult(x, 0, 0, rnorm, 0.0, snaps)
    while itn < iter_lim:
        itn += 1
        t = matvec(p)
        a = gamma / float(t @ t)
        x = x + a * p
        r = r - a * t
        s = rmatvec(r)
        gnew = float(s @ s)
        p = s + (gnew / gamma) * p
        gamma = gnew
        rnorm = float(np.linalg.norm(r))
        if itn in snapshot_at:
            snaps[itn] = x.copy()
        if callback is not None and callback(itn, x):
            istop = 8
            break
        if np.sqrt(gamma) <= atol * anorm_f * rnorm:
            istop = 2
        if rnorm <= btol * bnorm:
            istop = 1
        if istop:
            break
    else:
        istop = 7
    return CglsResult(x, istop, itn, rnorm, float(np.sqrt(gamma)), snaps)


# ---------------------------------------------------------------- Gram blocks

def gram_blocks(blocks, pairs=None, entry_map=None):
    """{(i, j): M_i^T M_j over rows in I_i and I_j} for i <= j with a shared row.

    entry_map, if given, is applied to every block's entries first (e.g. rounding to a lower
    precision); the products are then formed in float64."""
    mats = [blk.M if entry_map is None else entry_map(blk.M) for blk in blocks]
    G = {}
    n = len(blocks)
    if pairs is None:
        pairs = [(i, j) for i in range(n) for j in range(i, n)]
    for i, j in pairs:
        shared, ii, jj = np.intersect1d(blocks[i].rows, blocks[j].rows, assume_unique=True,
                                        return_indices=True)
        if shared.size == 0:
            continue
        G[(i, j)] = mats[i][ii].T @ mats[j][jj]
    return G


def gram_apply(G, blocks, p, dtype=np.float64):
    """y = G p with G given by its upper blocks (i <= j): y_i += G_ij p_j, y_j += G_ij^T p_i."""
    y = np.zeros(p.shape, dtype=dtype)
    for (i, j), g in G.items():
        qi = slice(blocks[i].sd.q0, blocks[i].sd.q0 + g.shape[0])
        qj = slice(blocks[j].sd.q0, blocks[j].sd.q0 + g.shape[1])
        y[qi] += (g @ p[qj]).astype(dtype)
        if i != j:
            y[qj] += (g.T @ p[qi]).astype(dtype)
    return y


def normal_cg(apply_G, g, n_iter, dtype=np.float64):
    """Hestenes-Stiefel CG on G d = g from d = 0 for n_iter steps, vectors and scalars in dtype."""
    d = np.zeros(g.shape, dtype=dtype)
    r = np.array(g, dtype=dtype, copy=True)
    p = r.copy()
    rr = r @ r
    for _ in range(n_iter):
        if rr == 0:
            break
        q = np.asarray(apply_G(p), dtype=dtype)
        pq = p @ q
        if not pq > 0:
            break
        a = rr / pq
        d = d + a * p
        r = r - a * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return d


def normal_pcg(apply_G, g, n_iter, apply_Minv=None, x0=None):
    """Preconditioned conjugate gradients (Hestenes-Stiefel, with a symmetric positive definite
    preconditioner M) on G d = g for n_iter steps from x0 (or zero), float64 throughout:
        r = g - G d, z = M^{-1} r, p = z;
        each step: q = G p, a = (r.z)/(p.q), d += a p, r -= a q, z = M^{-1} r,
                   p = z + ((r.z)_new / (r.z)) p.
    apply_Minv None means M = I (plain CG).  Stops early when r.z = 0 or p.q <= 0."""
    d = np.zeros(g.shape) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = np.array(g, dtype=np.float64, copy=True) - (apply_G(d) if x0 is not None else 0.0)
    z = r.copy() if apply_Minv is None else np.asarray(apply_Minv(r), dtype=np.float64)
    p = z.copy()
    rz = r @ z
    for _ in range(n_iter):
        if rz == 0:
            break
        q = np.asarray(apply_G(p), dtype=np.float64)
        pq = p @ q
        if not pq > 0:
            break
        a = rz / pq
        d = d + a * p
        r = r - a * q
        z = r.copy() if apply_Minv is None else np.asarray(apply_Minv(r), dtype=np.float64)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return d


def block_jacobi_inverse_apply(blocks, factors, r):
    """z = (R^T R)^{-1} r per block (R upper, R^T R = G_jj + lambda I): the block-Jacobi
    preconditioner of the normal equations, by two triangular solves per block."""
    z = np.zeros_like(r)
    for blk, R in zip(blocks, factors):
        K = R.shape[0]
        sl = slice(blk.sd.q0, blk.sd.q0 + K)
        z[sl] = np.linalg.solve(R, np.linalg.solve(R.T, r[sl]))
    return z


def refine(matvec, rmatvec, h, n, apply_G_lo, n_outer, n_inner, x0=None, lo_dtype=np.float32,
           callback=None):
    """Iterative refinement (BJ-style mixed precision): per outer step
         r = h - M c (float64), g = M^T r (float64), d ~ G_lo^{-1} g by n_inner CG steps in lo_dtype,
         c = c + d (float64)."""
    c = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    hist = []
    for it in range(n_outer):
        r = h - matvec(c)
        g = rmatvec(r)
        hist.append((float(np.linalg.norm(r)), float(np.linalg.norm(g))))
        d = normal_cg(apply_G_lo, g.astype(lo_dtype), n_inner, dtype=lo_dtype)
        c = c + d.astype(np.float64)
        if callback is not None and callback(it, c):
            break
    return c, hist


# ---------------------------------------------------------------- block-Jacobi preconditioning

def block_jacobi_factors(blocks, shift):
    """Per subdomain the upper Cholesky factor R_j of G_jj + lambda_j I, lambda_j =
    shift * trace(G_jj)/K (G_jj = M_j^T M_j).  A factorisation that fails is retried with 100x
    the shift up to 8 times, then R_j = I; an all-zero block gets R_j = I."""
    out = []
    for blk in blocks:
        K = blk.M.shape[1]
        G = blk.M.T @ blk.M
        lam = shift * np.trace(G) / K
        R = np.eye(K)
        if lam > 0:
            for _ in range(8):
                try:
                    R = np.linalg.cholesky(G + lam * np.eye(K)).T
                    break
                except np.linalg.LinAlgError:
                    lam *= 100.0
            else:
                R = np.eye(K)
        out.append(R)
    return out


def block_apply(blocks, factors, v, transpose=False, inverse=True):
    """Apply blockdiag(R_j)^{-1} (or its transpose) to a coefficient vector."""
    y = np.zeros_like(v)
    for blk, R in zip(blocks, factors):
        K = R.shape[0]
        q = slice(blk.sd.q0, blk.sd.q0 + K)
        if inverse:
            y[q] = np.linalg.solve(R.T, v[q]) if transpose else np.linalg.solve(R, v[q])
        else:
            y[q] = (R.T @ v[q]) if transpose else (R @ v[q])
    return y


def fold_blocks(blocks, factors):
    """The right-preconditioned blocks M_j R_j^{-1} (same rows), formed once; LSQR on them is
    LSQR on M R^{-1}, and a coefficient vector y of the folded system maps back as R^{-1} y."""
    out = []
    for blk, R in zip(blocks, factors):
        out.append(dataclasses.replace(blk, M=np.linalg.solve(R.T, blk.M.T).T))
    return out


# ---------------------------------------------------------------- block-Jacobi over patches
#
# The redundancy that makes M ill-conditioned (Sec. 5 "Conditioning and redundancy") is not only
# within one subdomain: neighbouring subdomains of a level overlap and their features describe
# nearly the same functions on the shared points.  Taking P^d neighbouring subdomains of a level
# as one block of the block-Jacobi preconditioner (a patch) orthonormalises their columns
# together.  A patch block holds every column of its members on the union of their supports
# (zero where a member's window vanishes); the preconditioner is then exactly the block-Jacobi
# one above applied to the patch blocks, and P = 1 is the per-subdomain preconditioner.


@dataclass
class PatchBlock:
    level: int
    index: tuple            # patch index per axis (j // P for the members' per-axis indices j)
    members: list           # the member subdomain blocks, per-axis indices in lexicographic order
    rows: np.ndarray        # union of the members' rows, sorted
    cols: np.ndarray        # global columns, member by member (features in order)
    M: np.ndarray           # [len(rows), len(cols)], zero outside each member's rows


def patch_blocks(blocks, P):
    """Group the subdomain blocks of every level into patches of P consecutive subdomains per
    axis (the last patch along an axis keeps what is left); patches in order of level, then
    patch index (x-major), which is also the column order of the preconditioned system."""
    groups = {}
    for blk in blocks:
        key = (blk.sd.level,) + tuple(int(j) // P for j in blk.sd.jj)
        groups.setdefault(key, []).append(blk)
    out = []
    for key in sorted(groups):
        mem = sorted(groups[key], key=lambda b: tuple(b.sd.jj))
        rows = np.unique(np.concatenate([np.asarray(b.rows) for b in mem]))
        cols = np.concatenate([np.arange(b.sd.q0, b.sd.q0 + b.M.shape[1]) for b in mem])
        M = np.zeros((rows.size, cols.size))
        c = 0
        for b in mem:
            M[np.searchsorted(rows, b.rows), c:c + b.M.shape[1]] = b.M
            c += b.M.shape[1]
        out.append(PatchBlock(key[0], key[1:], mem, rows, cols, M))
    return out


def patch_order(pblocks):
    """Column permutation of the patch system: position i holds original column perm[i]."""
    return np.concatenate([pb.cols for pb in pblocks])


def patch_matvec(pblocks, y, n_rows):
    """sum over patches of M_p y_p, y in patch column order."""
    out = np.zeros(n_rows)
    o = 0
    for pb in pblocks:
        k = pb.M.shape[1]
        out[pb.rows] += pb.M @ y[o:o + k]
        o += k
    return out


def patch_rmatvec(pblocks, u):
    """(M_p^T u) for every patch, concatenated in patch column order."""
    return np.concatenate([pb.M.T @ u[pb.rows] for pb in pblocks])


def patch_recover(pblocks, factors, y):
    """x = R^{-1} y patch by patch, returned in the original column order."""
    x = np.zeros(y.size)
    o = 0
    for pb, R in zip(pblocks, factors):
        k = pb.M.shape[1]
        x[pb.cols] = np.linalg.solve(R, y[o:o + k])
        o += k
    return x


def preconditioned_lsqr(matvec, rmatvec, blocks, factors, h, n, x0=None, **kw):
    """LSQR on M R^{-1} (right block-Jacobi preconditioning); returns (x, result) with
    x = x0 + R^{-1} y, y the LSQR solution for the residual h - M x0."""
    rhs = h if x0 is None else h - matvec(x0)
    res = lsqr(lambda y: matvec(block_apply(blocks, factors, y)),
               lambda u: block_apply(blocks, factors, rmatvec(u), transpose=True), rhs, n, **kw)
    x = block_apply(blocks, factors, res.x)
    if x0 is not None:
        x = x + x0
    return x, res


def refine_lsqr(matvec, rmatvec, matvec_lo, rmatvec_lo, h, n, n_outer, n_inner, blocks=None,
                factors=None, x0=None, callback=None):
    """FP64 iterative refinement around inner LSQR on a low-precision copy of the matrix:
    per outer step r = h - M c (float64), d = n_inner LSQR steps on M_lo d = r (float64 vectors,
    optionally right block-Jacobi preconditioned), c = c + d."""
    c = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    hist = []
    for it in range(n_outer):
        r = h - matvec(c)
        hist.append(float(np.linalg.norm(r)))
        if factors is None:
            d = lsqr(matvec_lo, rmatvec_lo, r, n, atol=0, btol=0, iter_lim=n_inner).x
        else:
            d, _ = preconditioned_lsqr(matvec_lo, rmatvec_lo, blocks, factors, r, n, atol=0,
                                       btol=0, iter_lim=n_inner)
        c = c + d
        if callback is not None and callback(it, c):
            break
    return c, hist
