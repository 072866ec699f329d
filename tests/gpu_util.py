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


def device_blocks(P, K, store_prec="fp64", folded=False):
    """[(table_row, M_j [n_j, K] float64)] from the device block storage (folded: the
    block-Jacobi-folded M R^-1)."""
    torch = torch_mod()
    nnz = P.sizes["nnz"]
    dt = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.bfloat16,
          "fp16": torch.float16}[store_prec]
    buf = torch.empty(nnz, dtype=dt, device="cuda")
    table = P.copy_blocks(buf, prec=store_prec, folded=folded)
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


def fold_tolerance(M_hat, K, shift):
    """Entry tolerance between two FP64 evaluations of the folded block M_j R_j^{-1}: the Gram
    block G + lambda I (lambda = shift trace(G)/K) has condition number up to about K/shift, so
    rounding differences of the Gram products change R_j, and M_j R_j^{-1} with it, by a small
    multiple of K eps / shift relative to the block's largest entry (measured: up to 0.8 of it
    on the test problems; the factor 4 is the margin)."""
    return 4.0 * K * np.finfo(np.float64).eps / shift * np.abs(M_hat).max()


def n_ambiguous(ref, rounding, tol):
    """Entries of ref that lie within tol of a rounding boundary of `rounding`."""
    r = rounding(ref)
    return int(np.sum((rounding(ref - tol) != r) | (rounding(ref + tol) != r)))


def check_rounded_fold(got, ref, rounding, tol):
    """The low-precision folded copy `got` is the rounding of an FP64 product within tol of the
    oracle's `ref`: rounding is monotone, so got lies between the roundings of ref - tol and
    ref + tol, and equals the rounding of ref wherever no boundary lies that close.  Returns
    (mismatches, ambiguous entries)."""
    r = rounding(ref)
    lo, hi = rounding(ref - tol), rounding(ref + tol)
    ambiguous = (lo != r) | (hi != r)
    mism = got != r
    assert not np.any(mism & ~ambiguous)
    assert np.all((got >= lo) & (got <= hi))
    return int(mism.sum()), int(ambiguous.sum())


def rounded_variants(folded_blocks, rounding, K, shift, limit=4):
    """Every low-precision folded matrix the device may hold: the oracle's rounding of its
    M_j R_j^{-1}, with each entry that lies within fold_tolerance of a rounding boundary taking
    either neighbour (at most `limit` such entries, so 2^limit variants)."""
    base = [rounding(b.M) for b in folded_blocks]
    amb = []
    for bi, b in enumerate(folded_blocks):
        tol = fold_tolerance(b.M, K, shift)
        lo, hi = rounding(b.M - tol), rounding(b.M + tol)
        r = base[bi]
        for idx in zip(*np.nonzero((lo != r) | (hi != r))):
            amb.append((bi, idx, lo[idx] if lo[idx] != r[idx] else hi[idx]))
    assert len(amb) <= limit, f"{len(amb)} entries lie within the fold tolerance of a boundary"
    out = []
    for mask in range(2 ** len(amb)):
        Ms = list(base)
        for t, (bi, idx, alt) in enumerate(amb):
            if mask >> t & 1:
                if Ms[bi] is base[bi]:
                    Ms[bi] = base[bi].copy()
                Ms[bi][idx] = alt
        out.append(Ms)
    return out


# ---------------------------------------------------------------- converged-solve tolerances
#
# Two correct LSQR implementations that sum in different orders drift apart once the Golub-Kahan
# vectors lose orthogonality, so a converged solve cannot be compared with the oracle's to a
# fixed precision.  The yardstick is the oracle against itself: the same LSQR on row-permuted
# copies of the system (the same computation in exact arithmetic, other rounding).  A GPU result
# must lie within ITERATE_MULTIPLE times the oracle's largest deviation under those permutations
# (u on the test points, ||r||, the extreme singular values of the recorded bidiagonal), as the
# matched-iterate tests require; a step count, a single integer whose spread over three
# permutations is a few percent, within COUNT_MULTIPLE times its spread plus COUNT_SLACK steps
# (50x its spread would admit any count).

ITERATE_MULTIPLE = 50.0
COUNT_MULTIPLE = 3.0
COUNT_SLACK = 2


class OracleSpread:
    """The oracle's LSQR on M and on `seeds` row-permuted copies, to the same stopping test.

    ref: the unpermuted run; u_ref: evaluate(ref.x); sigma_ref: (sigma_max, sigma_min) of its
    bidiagonal; itn, u, rnorm, sigma_max, sigma_min, err: the largest deviation of the permuted
    runs from ref (absolute in steps, relative otherwise; err: |error vs exact| when `exact` is
    given, absolute)."""

    def __init__(self, M, h, n, evaluate, exact=None, error=None, seeds=3, x_map=None,
                 **lsqr_kw):
        from oracle import evaluate as ev
        from oracle import linalg
        x_map = x_map or (lambda x: x)

        def run(A, rhs):
            r = linalg.lsqr(lambda v: A @ v, lambda u: A.T @ u, rhs, n, **lsqr_kw)
            k = r.itn
            s = linalg.bidiag_extreme_singular_values(r.bidiag, k) if k > 0 else (0.0, 0.0)
            return r, evaluate(x_map(r.x)), s

        error = error or (lambda u, ue: ev.rel_l2(u, ue))
        self.ref, self.u_ref, self.sigma_ref = run(M, h)
        self.err_ref = error(self.u_ref, exact) if exact is not None else None
        self.itn = self.u = self.rnorm = self.sigma_max = self.sigma_min = self.err = 0.0
        self.runs = []
        for seed in range(seeds):
            perm = np.random.default_rng(seed).permutation(M.shape[0])
            r, u, s = run(M[perm], h[perm])
            self.runs.append(r)
            self.itn = max(self.itn, abs(r.itn - self.ref.itn))
            self.u = max(self.u, ev.rel_l2(u, self.u_ref))
            self.rnorm = max(self.rnorm, abs(r.rnorm - self.ref.rnorm) / max(self.ref.rnorm, 1e-300))
            if self.sigma_ref[0] > 0:
                self.sigma_max = max(self.sigma_max, abs(s[0] - self.sigma_ref[0]) / self.sigma_ref[0])
                self.sigma_min = max(self.sigma_min, abs(s[1] - self.sigma_ref[1]) / self.sigma_ref[1])
            if exact is not None:
                self.err = max(self.err, abs(error(u, exact) - self.err_ref))

    def tol(self, spread, floor=1e-10):
        return max(floor, ITERATE_MULTIPLE * spread)

    def count_tol(self):
        return COUNT_MULTIPLE * self.itn + COUNT_SLACK

    def describe(self):
        return (f"oracle {self.ref.itn} steps (istop {self.ref.istop}), spreads: steps {self.itn}, "
                f"u {self.u:.1e}, ||r|| {self.rnorm:.1e}, sigma_max {self.sigma_max:.1e}, "
                f"sigma_min {self.sigma_min:.1e}" +
                (f", error {self.err:.1e}" if self.err_ref is not None else ""))
