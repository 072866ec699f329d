"""Reference MLP for the learned warm start: a fully connected tanh network mapping problem
parameters (plus a subdomain's position) to that subdomain's coefficient block, trained with
mean-squared error and Adam (Kingma & Ba 2015) with the method's learning rate 1e-3 (Sec. 4.1
"Optimisation and solvers").

Test infrastructure only: nothing in the library imports this module.

Layers l = 1..L:  z_l = a_{l-1} W_l^T + b_l,  a_l = tanh(z_l) (hidden), y = z_L (output);
optionally modulated: with per-sample weights f [batch, n_mod] the last layer has n_mod K outputs
and the model output is y[k] = sum_i f_i z_L[i K + k] (a network whose output is linear in f);
W_l [n_l, n_{l-1}], row-major samples [batch, features].  Loss = mean over batch and outputs of
(y - t)^2.  Arithmetic is float64.  With bf16=True the operands of every product are rounded to
bfloat16 (round to nearest even) where a low-precision implementation stores them: the input,
the weights, each hidden activation a_l, and each back-propagated gradient g_l (of the output
and of every hidden pre-activation); sums are float64.  db_l sums the rounded g_l.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .lowprec import to_bf16

Params = List[Tuple[np.ndarray, np.ndarray]]


def _r(x, bf16):
    return to_bf16(x) if bf16 else np.asarray(x, dtype=np.float64)


def forward(params: Params, X: np.ndarray, bf16=False):
    """Returns (y, acts) with acts[l] = the (rounded) input of layer l+1."""
    a = _r(X, bf16)
    acts = [a]
    L = len(params)
    y = None
    for l, (W, b) in enumerate(params):
        z = a @ _r(W, bf16).T + b
        if l < L - 1:
            a = _r(np.tanh(z), bf16)
            acts.append(a)
        else:
            y = z
    return y, acts


def modulate(z: np.ndarray, f: np.ndarray) -> np.ndarray:
    """y[b, k] = sum_i f[b, i] z[b, i K + k]."""
    B, n_mod = f.shape
    K = z.shape[1] // n_mod
    return np.einsum("bi,bik->bk", f, z.reshape(B, n_mod, K))


def demodulate_grad(dy: np.ndarray, f: np.ndarray, bf16=False) -> np.ndarray:
    """dL/dz for y = modulate(z, f): dz[b, i K + k] = f[b, i] dy[b, k] (rounded like g_L)."""
    g = (f[:, :, None] * dy[:, None, :]).reshape(dy.shape[0], -1)
    return _r(g, bf16)


def mse(y: np.ndarray, t: np.ndarray):
    """(loss, dL/dy)."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params: Params, acts, dy: np.ndarray, bf16=False, f=None):
    """Gradients [(dW_l, db_l)] of the loss whose output gradient is dy (of the modulated
    output when f is given)."""
    L = len(params)
    grads = [None] * L
    g = demodulate_grad(dy, f, bf16) if f is not None else _r(dy, bf16)
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        grads[l] = (g.T @ acts[l], g.sum(axis=0))
        if l > 0:
            a = acts[l]
            g = _r((g @ _r(W, bf16)) * (1.0 - a * a), bf16)
    return grads


def adam(params: Params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step.  state = (t, m, v) with m, v lists like params (None to start).  Returns
    (new params, new state)."""
    t, m, v = state if state is not None else (0, None, None)
    if m is None:
        m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    t += 1
    out, m2, v2 = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        new = []
        mm, vv = [], []
        for p, g, mp, vp in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mp = b1 * mp + (1 - b1) * g
            vp = b2 * vp + (1 - b2) * g * g
            mh = mp / (1 - b1 ** t)
            vh = vp / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
            mm.append(mp)
            vv.append(vp)
        out.append((new[0], new[1]))
        m2.append((mm[0], mm[1]))
        v2.append((vv[0], vv[1]))
    return out, (t, m2, v2)


def flatten(params: Params) -> np.ndarray:
    """[W_1 row-major, b_1, W_2, b_2, ...] as one vector."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(vec: np.ndarray, dims) -> Params:
    out, o = [], 0
    for n_in, n_out in zip(dims[:-1], dims[1:]):
        W = vec[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = vec[o:o + n_out]
        o += n_out
        out.append((np.array(W, dtype=np.float64), np.array(b, dtype=np.float64)))
    return out
