"""Manufactured problems: exact solutions and forcing terms.

These are problem statements, not the method: the caller evaluates the forcing
term f at the collocation points and hands the values to the solver.
"""
from __future__ import annotations

import numpy as np


def ode_cos_exact(x: np.ndarray, omega: float = 15.0) -> np.ndarray:
    """du/dx = cos(omega x), u(0) = 0  =>  u = sin(omega x)/omega."""
    return np.sin(omega * x[..., 0]) / omega


def ode_cos_forcing(x: np.ndarray, omega: float = 15.0) -> np.ndarray:
    return np.cos(omega * x[..., 0])


def ode_modes_forcing(x: np.ndarray, freqs, amps) -> np.ndarray:
    """du/dx = sum_m c_m cos(w_m x)."""
    s = np.zeros(x.shape[0])
    for w, c in zip(freqs, amps):
        s = s + c * np.cos(w * x[:, 0])
    return s


def ode_modes_exact(x: np.ndarray, freqs, amps) -> np.ndarray:
    s = np.zeros(x.shape[0])
    for w, c in zip(freqs, amps):
        s = s + c * np.sin(w * x[:, 0]) / w
    return s


def sines_exact(x: np.ndarray, freqs, amps) -> np.ndarray:
    """u = sum_m a_m sin(k_m pi x) sin(k_m pi y)  (Sec. 4.3, multiscale Laplace family)."""
    u = np.zeros(x.shape[0])
    for k, a in zip(freqs, amps):
        u = u + a * np.sin(k * np.pi * x[:, 0]) * np.sin(k * np.pi * x[:, 1])
    return u


def sines_forcing(x: np.ndarray, freqs, amps) -> np.ndarray:
    """f = -Laplace(u) = sum_m a_m 2 (k_m pi)^2 sin(k_m pi x) sin(k_m pi y)."""
    f = np.zeros(x.shape[0])
    for k, a in zip(freqs, amps):
        kp = k * np.pi
        f = f + a * 2.0 * kp * kp * np.sin(kp * x[:, 0]) * np.sin(kp * x[:, 1])
    return f


def oscillator_exact(t: np.ndarray, omega0: float, mu: float = 4.0, m: float = 1.0,
                     u0: float = 1.0, v0: float = 0.0) -> np.ndarray:
    """Under-damped m u'' + mu u' + k u = 0, k = m omega0^2, u(0) = u0, u'(0) = v0:
    u = exp(-d t) 2A cos(phi + w t), d = mu/(2m), w = sqrt(omega0^2 - d^2),
    phi = arctan(-(v0/u0 + d)/w), A = u0/(2 cos phi)."""
    d = mu / (2.0 * m)
    w = np.sqrt(omega0 ** 2 - d ** 2)
    phi = np.arctan(-(v0 / u0 + d) / w)
    A = u0 / (2.0 * np.cos(phi))
    return np.exp(-d * t) * 2.0 * A * np.cos(phi + w * t)



def helmholtz_exact(x: np.ndarray, omega: float) -> np.ndarray:
    """u = sin(w pi x) sin(2 w pi y) + sin(3 w pi x y) (Sec. 4.4 eq. helmholtz_exact)."""
    wp = omega * np.pi
    return np.sin(wp * x[:, 0]) * np.sin(2 * wp * x[:, 1]) + np.sin(3 * wp * x[:, 0] * x[:, 1])


def helmholtz_forcing(x: np.ndarray, omega: float, k: float) -> np.ndarray:
    """f = Lap u + k^2 u for that u (Sec. 4.4 eq. helmholtz_f)."""
    wp = omega * np.pi
    a = np.sin(wp * x[:, 0]) * np.sin(2 * wp * x[:, 1])
    c = np.sin(3 * wp * x[:, 0] * x[:, 1])
    return (-5.0 * wp * wp * a - 9.0 * wp * wp * (x[:, 0] ** 2 + x[:, 1] ** 2) * c
            + k * k * (a + c))
