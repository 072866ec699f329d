"""Evaluation of the fitted solution and the error metrics.

u_tilde(x) = C(x) * (1/L) sum_l sum_j omega_j(x) sum_k a_q phi_q(x)
(Sec. 3 eq. multilevel_solution times the hard-constraint factor of Sec. 4.3), at arbitrary
points; rel-L2 = ||u - u_ref|| / ||u_ref||; e_L1 = mean |u - u_exact| / std(u_exact) with the
population standard deviation (Sec. 4.1 eq. l1_error).
"""
from __future__ import annotations

import numpy as np

from . import basis
from . import geometry as geo


def evaluate(prob, W, b, coef, x):
    """u_tilde at points x [M, d] for coefficient vector(s) coef [N_Phi] or [R, N_Phi]."""
    x = np.asarray(x, dtype=np.float64)
    coef = np.asarray(coef, dtype=np.float64)
    single = coef.ndim == 1
    C2 = coef[None, :] if single else coef
    L = len(prob.levels)
    subs = geo.subdomains(prob)
    C, _, _ = basis.ansatz(x, prob)
    out = np.zeros((C2.shape[0], x.shape[0]))
    for l in range(L):
        level = [sd for sd in subs if sd.level == l]
        S, _, _ = basis.level_sum(x, level)
        for sd in level:
            m = geo.in_support(x, sd)
            if not m.any():
                continue
            xs = x[m]
            if sd.single:
                w = np.ones(xs.shape[0])
            else:
                v, _, _ = basis.window_hat(xs, sd)
                w = v / S[m]
            q = slice(sd.q0, sd.q0 + prob.K)
            phi, _, _ = basis.features(xs, sd, W[q], b[q], basis.global_inputs(prob))
            out[:, m] += w[None, :] * (C2[:, q] @ phi.T)
    out = out * C[None, :] / L
    return out[0] if single else out


def rel_l2(u, ref):
    return float(np.linalg.norm(np.ravel(u) - np.ravel(ref)) / np.linalg.norm(np.ravel(ref)))


def e_l1(u, u_exact):
    u_exact = np.ravel(u_exact)
    return float(np.mean(np.abs(np.ravel(u) - u_exact)) / np.std(u_exact))
