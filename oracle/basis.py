"""Windows, random features, hard-constraint ansatz and operator rows.

  * window (Sec. 4.1, eq. window_func): omega_hat_j(x) = prod_i [1 + cos(pi (x_i - mu_i)/sigma_i)]^2
    on the support and zero outside, normalised per level by the sum over all subdomains of that
    level, so sum_j omega_j = 1 (Sec. 3 "Problem and model definition");
  * random features (Sec. 3, the shallow network with h = 1; Sec. 4.1 initialisation):
    phi_q(x) = tanh(W_q . xbar + b_q), xbar = (x - mu_j)/sigma_l (subdomain-local inputs, the
    default reading); with a problem's input_norm "global" the raw coordinates, xbar = x;
  * hard-constraint ansatz (Sec. 4.3 "Hard boundary constraints"):
    C(x) = prod_i tanh(w (x_i - lo_i)) tanh(w (hi_i - x_i)); for the 1D ODE C = tanh(w x);
  * operator rows (Sec. 3 "Definition of the system matrices"):
    N_{n,q} = Op[C omega_j phi_q](x_n) / (sqrt(N_I) L), h_n = f(x_n)/sqrt(N_I).

All functions accept complex arguments where the formulas allow it, so that the
complex-step method can check first derivatives.
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo


# ---------------------------------------------------------------- raw window per axis

def raw_window(t):
    """(1 + cos(pi t))^2 for |t| < 1, else 0, with t = (x - mu)/sigma."""
    w = (1.0 + np.cos(np.pi * t)) ** 2
    return np.where(np.abs(np.real(t)) < 1.0, w, 0.0)


def raw_window_dt(t):
    """d/dt (1 + cos(pi t))^2 = -2 pi sin(pi t)(1 + cos(pi t))."""
    d = -2.0 * np.pi * np.sin(np.pi * t) * (1.0 + np.cos(np.pi * t))
    return np.where(np.abs(np.real(t)) < 1.0, d, 0.0)


def raw_window_dtt(t):
    """d2/dt2 (1 + cos(pi t))^2 = 2 pi^2 (sin^2(pi t) - cos(pi t)(1 + cos(pi t)))."""
    s, c = np.sin(np.pi * t), np.cos(np.pi * t)
    d = 2.0 * np.pi ** 2 * (s * s - c * (1.0 + c))
    return np.where(np.abs(np.real(t)) < 1.0, d, 0.0)


def window_hat(x, sd: geo.Subdomain):
    """Unnormalised window, its gradient [N,d] and its Laplacian at points x [N,d]."""
    N, d = x.shape
    t = [(x[:, a] - sd.mu[a]) / sd.sigma[a] for a in range(d)]
    f = [raw_window(t[a]) for a in range(d)]
    f1 = [raw_window_dt(t[a]) / sd.sigma[a] for a in range(d)]
    f2 = [raw_window_dtt(t[a]) / sd.sigma[a] ** 2 for a in range(d)]
    for a in range(d):
        if sd.single_axes and sd.single_axes[a]:
            # one subdomain along this axis: factor 1 (its normalisation would be 0/0 at the ends)
            f[a] = np.ones(N, dtype=np.result_type(x, float))
            f1[a] = np.zeros(N, dtype=f[a].dtype)
            f2[a] = np.zeros(N, dtype=f[a].dtype)
    val = np.ones(N, dtype=np.result_type(x, float))
    for a in range(d):
        val = val * f[a]
    grad = np.zeros((N, d), dtype=val.dtype)
    lap = np.zeros(N, dtype=val.dtype)
    for a in range(d):
        g = f1[a]
        h = f2[a]
        for b in range(d):
            if b != a:
                g = g * f[b]
                h = h * f[b]
        grad[:, a] = g
        lap = lap + h
    return val, grad, lap


def level_sum(x, subs_of_level):
    """S = sum_j omega_hat_j, its gradient and Laplacian, summed over every subdomain of a level."""
    N, d = x.shape
    S = np.zeros(N, dtype=np.result_type(x, float))
    gS = np.zeros((N, d), dtype=S.dtype)
    lS = np.zeros(N, dtype=S.dtype)
    for sd in subs_of_level:
        v, g, l = window_hat(x, sd)
        S = S + v
        gS = gS + g
        lS = lS + l
    return S, gS, lS


def window(x, sd: geo.Subdomain, level_sums):
    """Normalised window omega_j = omega_hat_j / S with gradient and Laplacian (quotient rule).

    Along an axis with a single subdomain the factor is 1, so a level with one subdomain has
    omega == 1."""
    N, d = x.shape
    if sd.single:
        return np.ones(N), np.zeros((N, d)), np.zeros(N)
    S, gS, lS = level_sums
    v, g, l = window_hat(x, sd)
    w = v / S
    gw = np.zeros_like(g)
    for a in range(d):
        gw[:, a] = (g[:, a] - w * gS[:, a]) / S
    # sum over axes of d2/da2 (v/S) = (v_aa - 2 w_a S_a - w S_aa)/S
    lw = (l - 2.0 * np.sum(gw * gS, axis=1) - w * lS) / S
    return w, gw, lw


# ---------------------------------------------------------------- random features

def global_inputs(prob) -> bool:
    return getattr(prob, "input_norm", "local") == "global"


def features(x, sd: geo.Subdomain, W, b, global_in=False):
    """phi, grad phi [N,K,d] and Laplacian of phi [N,K] for the K features of one subdomain.

    W [K, d] and b [K] are the subdomain's fixed hidden parameters; global_in: xbar = x."""
    N, d = x.shape
    if global_in:
        xbar = x
        c = W                                     # d xbar / dx = 1
    else:
        xbar = (x - sd.mu[None, :]) / sd.sigma[None, :]
        c = W / sd.sigma[None, :]                 # chain rule factor W_i / sigma_i, [K, d]
    z = xbar @ W.T + b[None, :]
    phi = np.tanh(z)
    s = 1.0 - phi * phi
    grad = s[:, :, None] * c[None, :, :]
    lap = -2.0 * phi * s * np.sum(c * c, axis=1)[None, :]
    return phi, grad, lap


# ---------------------------------------------------------------- hard-constraint ansatz

def ansatz(x, prob):
    """C, grad C [N,d], Laplacian of C."""
    N, d = x.shape
    kind = prob.ansatz
    w = float(prob.ansatz_omega)
    if kind == "none":
        return np.ones(N), np.zeros((N, d)), np.zeros(N)
    if kind == "tanh_origin":
        C = np.tanh(w * x[:, 0])
        g = (w * (1.0 - C * C))[:, None]
        l = -2.0 * w * w * C * (1.0 - C * C)
        return C, g, l
    if kind == "tanh_box":
        # per coordinate: a(s) = tanh(w (s - lo)) tanh(w (hi - s))
        fa, fa1, fa2 = [], [], []
        for a in range(d):
            p = np.tanh(w * (x[:, a] - prob.lo[a]))
            r = np.tanh(w * (prob.hi[a] - x[:, a]))
            dp = w * (1.0 - p * p)               # d/ds p
            dr = -w * (1.0 - r * r)              # d/ds r
            ddp = -2.0 * w * p * dp              # d2/ds2 p
            ddr = 2.0 * w * r * dr               # d2/ds2 r: d/ds(-w(1-r^2)) = 2 w r dr
            fa.append(p * r)
            fa1.append(dp * r + p * dr)
            fa2.append(ddp * r + 2.0 * dp * dr + p * ddr)
        C = np.ones(N, dtype=fa[0].dtype)
        for a in range(d):
            C = C * fa[a]
        g = np.zeros((N, d), dtype=C.dtype)
        l = np.zeros(N, dtype=C.dtype)
        for a in range(d):
            ga = fa1[a]
            la = fa2[a]
            for bb in range(d):
                if bb != a:
                    ga = ga * fa[bb]
                    la = la * fa[bb]
            g[:, a] = ga
            l = l + la
        return C, g, l
    raise ValueError(kind)


# ---------------------------------------------------------------- operator rows

def localized_function(x, prob, sd, W, b, level_sums, ans=None):
    """Value, gradient and Laplacian of psi_q = C omega_j phi_q for the K features of sd."""
    C, gC, lC = ansatz(x, prob) if ans is None else ans
    w, gw, lw = window(x, sd, level_sums)
    P = C * w
    gP = gC * w[:, None] + C[:, None] * gw
    lP = lC * w + 2.0 * np.sum(gC * gw, axis=1) + C * lw
    phi, gphi, lphi = features(x, sd, W, b, global_inputs(prob))
    val = P[:, None] * phi
    grad = gP[:, None, :] * phi[:, :, None] + P[:, None, None] * gphi
    lap = lP[:, None] * phi + 2.0 * np.einsum("nd,nkd->nk", gP, gphi) + P[:, None] * lphi
    return val, grad, lap


def apply_operator(prob, val, grad, lap):
    """Op[psi] for the operators of the workloads."""
    if prob.op == "d1":
        return grad[:, :, 0]
    if prob.op == "neg_laplace":
        return -lap
    if prob.op == "identity":
        return val
    if prob.op == "helmholtz":
        # Lap u + k^2 u (Sec. 4.4 eq. helmholtz_problem)
        k = float(prob.meta["k"])
        return lap + k * k * val
    if prob.op == "oscillator":
        # m u'' + mu u' + k u in 1D (Sec. 4.2 eq. harm_oscillator): lap is the second derivative
        m, mu, k = prob.meta["osc"]
        return m * lap + mu * grad[:, :, 0] + k * val
    raise ValueError(prob.op)
