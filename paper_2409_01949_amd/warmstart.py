"""Learned warm start for batched solves of a parameterised problem family.

A tanh MLP (libelmfb's elmfb_mlp: bfloat16 products, FP32 master weights, Adam) is trained on
coefficient vectors that the batched solver itself produced, and maps the problem parameters
plus a subdomain's position to that subdomain's K coefficients; its prediction is the x0 of
later batched solves.  Coefficients are taken in block-Jacobi coordinates y_j = R_j x_j (the
subdomain's features orthonormalised over its support): there they are of the size of the
local solution, whereas the raw coefficients of the redundant random features carry large,
cancelling components that no regression reproduces.  This module only prepares inputs and
standardises targets on the host; solves, training and inference run in the library.

The solution of each family is linear in the source coefficients c, so the network's output is
modulated: it maps (parameters, one-hot subdomain index) to N_MOD K-vectors G_i and the
prediction is sum_i f_i G_i with per-sample weights f that are linear in c (the library's
modulated MLP output).  The subdomains have their own random features, so each needs its own
function of the parameters: the one-hot index lets the first layer hold them.

1D family: du/dx = sum_{m=1..3} c_m cos(m omega x / 3) on [-2 pi, 2 pi] with the hard constraint
tanh(omega x) (u(0) = 0), J subdomains of K features.  Near a centre mu_j each mode is a
combination of sin and cos of its phase phi_m = m omega mu_j / 3, so the weights are
f = (c_m sin phi_m, c_m cos phi_m), m = 1..3, and the inputs (omega / 50, one-hot j).

2D family: -Lap u = f on [0, 1]^2, u = sum_{m=1..3} c_m sin(n_m pi x) sin(n_m pi y) with
n_m = max(1, round(m omega / 15)) and the hard constraint tanh(omega s) tanh(omega (1 - s)) per
axis, 16 x 16 subdomains of K features.  Each mode's contribution is one function G(omega, n, j)
of the frequency, the mode number and the subdomain, the same for every m: the network is not
modulated but learns G from inputs (omega / 50, n / 10, one-hot j), and the prediction is
sum_u c'_u G(omega, u, j) over the distinct mode numbers u (c'_u the sum of the c_m with
n_m = u).  Its targets come from the training solves themselves: the 8 right-hand sides of an
omega share the matrix, so their coefficient blocks are, up to the solves' accuracy, the same
combinations of the per-mode blocks, which a least-squares fit per omega recovers.
"""
from __future__ import annotations

import time

import numpy as np

from .elmfb import MLP, Batch

N_MOD = 6


def _n_sub(spec):
    n = 1
    for v in spec.levels[0]:
        n *= int(v)
    return n


def subdomain_inputs(spec, omega, coeffs):
    """Network inputs [J, 1 + J] and modulation weights [J, 6] of one instance of the 1D family
    (single level) for one coefficient vector."""
    lo, hi = spec.lo[0], spec.hi[0]
    J = spec.levels[0][0]
    mu = lo + (hi - lo) * np.arange(J) / (J - 1) if J > 1 else np.array([(lo + hi) / 2])
    c = np.asarray(coeffs, dtype=np.float64)
    X = np.concatenate([np.full((J, 1), omega / 50.0), np.eye(J)], axis=1)
    F = np.empty((J, N_MOD))
    for m in range(3):
        ph = (m + 1) * omega * mu / 3.0
        F[:, 2 * m] = c[m] * np.sin(ph)
        F[:, 2 * m + 1] = c[m] * np.cos(ph)
    return X, F


def subdomain_inputs_2d(spec, omega, coeffs):
    """Network inputs [J, 4 + J] and modulation weights [J, 3] of one instance of the 2D family
    (J = Jx Jy subdomains of one level) for one coefficient vector."""
    J = _n_sub(spec)
    modes = np.asarray(spec.meta["freqs"], dtype=np.float64)
    head = np.concatenate([[omega / 50.0], modes / 10.0])
    X = np.concatenate([np.tile(head, (J, 1)), np.eye(J)], axis=1)
    F = np.tile(np.asarray(coeffs, dtype=np.float64), (J, 1))
    return X, F


def distinct_modes(spec, C):
    """Distinct mode numbers u of a 2D instance and the coefficient of each, c'_u = sum of the
    c_m with n_m = u, for every coefficient vector in C: (modes, [len(C), len(modes)])."""
    freqs = list(spec.meta["freqs"])
    um = sorted(set(freqs))
    A = np.array([[sum(c[m] for m in range(len(freqs)) if freqs[m] == u) for u in um]
                  for c in np.atleast_2d(C)])
    return um, A


def mode_inputs(spec, omega, n):
    """Network inputs [J, 2 + J] of the per-mode model: (omega / 50, n / 10, one-hot j)."""
    J = _n_sub(spec)
    return np.concatenate([np.tile([omega / 50.0, n / 10.0], (J, 1)), np.eye(J)], axis=1)


def mode_targets(specs, omegas, C, Y):
    """Per-mode training set of the 2D family: for each omega, the blocks G_u [J, K] of every
    distinct mode from a least-squares fit of its right-hand sides' blocks Y_r = sum_u A_ru G_u;
    returns (inputs, targets) with one row per (omega, mode, subdomain)."""
    X, T = [], []
    o = 0
    for s, om, Cg in zip(specs, omegas, C):
        J, R = _n_sub(s), Cg.shape[0]
        Yg = Y[o:o + R * J].reshape(R, J * s.K)
        o += R * J
        um, A = distinct_modes(s, Cg)
        G = np.linalg.lstsq(A, Yg, rcond=None)[0]
        for i, u in enumerate(um):
            X.append(mode_inputs(s, om, u))
            T.append(G[i].reshape(J, s.K))
    return np.concatenate(X), np.concatenate(T)


def training_set(specs, omegas, C, Y):
    """(inputs, modulation weights or None, targets) of the family's model from the training
    solves' coefficient blocks Y [(instance, rhs, subdomain), K]."""
    if specs[0].dim == 2:
        X, T = mode_targets(specs, omegas, C, Y)
        return X, None, T
    X, F = family_inputs(specs, omegas, C)
    return X, F, Y


def predict(model, specs, omegas, C):
    """Predicted coefficient blocks [(instance, rhs, subdomain), K] for every pair."""
    if specs[0].dim != 2:
        return model.predict(*family_inputs(specs, omegas, C))
    rows, combos = [], []
    for s, om, Cg in zip(specs, omegas, C):
        um, A = distinct_modes(s, Cg)
        rows += [mode_inputs(s, om, u) for u in um]
        combos.append((A, _n_sub(s), len(um)))
    G = model.predict(np.concatenate(rows))
    out, o = [], 0
    for A, J, U in combos:
        Gi = G[o:o + U * J].reshape(U, J, -1)
        o += U * J
        out.append(np.einsum("ru,ujk->rjk", A, Gi).reshape(-1, Gi.shape[2]))
    return np.concatenate(out)


def family_inputs(specs, omegas, C):
    """(X, F) for every (instance, rhs, subdomain), in the coefficient order of a batch solve."""
    fn = subdomain_inputs_2d if specs[0].dim == 2 else subdomain_inputs
    parts = [fn(s, om, c) for s, om, Cg in zip(specs, omegas, C) for c in Cg]
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def coef_blocks(coef, specs, n_rhs):
    """Batch coefficients (per instance [n_rhs][J K]) as [(instance, rhs, subdomain), K]."""
    out, o = [], 0
    for s in specs:
        n = _n_sub(s) * s.K
        out.append(coef[o:o + n_rhs * n].reshape(n_rhs * _n_sub(s), s.K))
        o += n_rhs * n
    return np.concatenate(out)


class WarmStart:
    """Modulated MLP from subdomain inputs to coefficient blocks (targets scaled per column)."""

    def __init__(self, n_in, K, hidden=512, depth=3, max_batch=4096, seed=0, n_mod=N_MOD):
        from inputs import mlp_init

        self.dims = [n_in] + [hidden] * depth + [n_mod * K]
        self.net = MLP(self.dims, max_batch, n_mod=n_mod)
        self.net.set_params(mlp_init(self.dims, seed))
        self.max_batch = max_batch
        self.scale = np.ones(K)

    def fit(self, X, F, Y, epochs, lr=1e-3, seed=0, log=None):
        """Adam on the mean-squared error of the scaled targets (scaling only, so the model stays
        linear in F); returns the loss history (the last mini-batch's loss of every epoch).  The
        samples are copied to the device once; each epoch visits them in a seeded random order."""
        import torch

        self.scale = Y.std(axis=0) + 1e-12
        xs = torch.as_tensor(X.astype(np.float32)).cuda()
        fs = None if F is None else torch.as_tensor(F.astype(np.float32)).cuda()
        ts = torch.as_tensor((Y / self.scale).astype(np.float32)).cuda()
        rng = np.random.default_rng(seed)
        hist = []
        bs = min(self.max_batch, len(X))
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(len(X))).cuda()
            nb = len(X) // bs
            loss = None
            for b in range(nb):
                idx = perm[b * bs:(b + 1) * bs]
                loss = self.net.train_step(xs[idx], ts[idx], f=None if fs is None else fs[idx],
                                           lr=lr, want_loss=b == nb - 1)
            hist.append(loss)
            if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
                log(f"epoch {ep}: loss {loss:.4e} ({time.perf_counter() - t0:.1f} s)")
        return hist

    def predict(self, X, F=None):
        import torch

        out = []
        for o in range(0, len(X), self.max_batch):
            xd = torch.as_tensor(X[o:o + self.max_batch].astype(np.float32)).cuda()
            fd = (None if F is None else
                  torch.as_tensor(F[o:o + self.max_batch].astype(np.float32)).cuda())
            out.append(self.net.forward(xd, fd).cpu().numpy().astype(np.float64))
        return np.concatenate(out) * self.scale

    def destroy(self):
        self.net.destroy()


def family_batch(omegas, C, store_prec="fp32", dim=1):
    """Batch of warm-family instances of the 1D or 2D family (one per omega, its rows of C as
    right-hand sides), assembled, with their specs and per-pair ||h||."""
    import torch

    from inputs import configs, feature_params

    make = configs.warm_family_2d if dim == 2 else configs.warm_family_1d
    specs = [make(om, Cg[0]) for om, Cg in zip(omegas, C)]
    feats = [feature_params(s) for s in specs]
    R = C.shape[1]
    B = Batch(specs, [w for w, _ in feats], [b for _, b in feats], R, store_prec=store_prec)
    f = np.concatenate([configs.warm_batch_forcing(s, Cg).ravel() for s, Cg in zip(specs, C)])
    B.assemble(torch.as_tensor(f).cuda())
    hn = np.concatenate([np.linalg.norm(configs.warm_batch_forcing(s, Cg), axis=1)
                         / np.sqrt(s.n_rows) for s, Cg in zip(specs, C)])
    return B, specs, hn


def solve_batch(B, x0=None, btol=1e-4, inner=1000, outer=8, shift=1e-12, precondition=True,
                atol=0.0):
    """Refined block-Jacobi solve of every pair to ||h - M c|| <= btol ||h|| (or, with atol > 0,
    to least-squares optimality ||M^T r|| <= atol ||M|| ||r||), coefficients in block-Jacobi
    coordinates (x0 and result); returns (coefficients on the host, infos, seconds)."""
    import torch

    if precondition:
        B.precondition(shift)
    B.set_coords(True)
    coef = torch.empty(B.n_rhs * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = B.solve(coef, method="mixed_ir", inner_iters=inner, outer_lim=outer, atol=atol,
                    btol=btol, check_every=50, precond=True, x0=x0)
    torch.cuda.synchronize()
    return coef.cpu().numpy(), infos, time.perf_counter() - t0
