"""The workloads: seeded synthetic problems with the shapes of the method's test cases.

Sizes follow the 1D first-order ODE, the multilevel 2D Poisson problems, the
batched ragged Poisson instances and the parameterised warm-start families.
Every random draw is seeded here; nothing in this module evaluates the method.
"""
from __future__ import annotations

import math

import numpy as np

from .problems import ProblemSpec, grid_points, l_shape_boundary
from . import families as fam


# ---------------------------------------------------------------- single problems

def ode1d() -> ProblemSpec:
    """du/dx = cos(15x) on [-2pi, 2pi], u(0)=0; 20 subdomains, width ratio 1.3, K=64, 2000 points."""
    return ProblemSpec(
        name="ode1d", dim=1, op="d1", ansatz="tanh_origin", ansatz_omega=15.0,
        lo=(-2 * math.pi,), hi=(2 * math.pi,), n_points=(2000,), levels=((20,),),
        delta=1.3, K=64, w_range=(-1.0, 1.0), b_range=(-1.0, 1.0), seed=0,
        meta={"family": "ode_cos", "omega": 15.0, "n_test": (1000,)},
    )


def poisson3l() -> ProblemSpec:
    """-Lap u = f on [0,1]^2, u = sum_{k in 1,4,16} sin(k pi x) sin(k pi y)/k; levels 1,4,16; K=96; 400^2."""
    return ProblemSpec(
        name="poisson3l", dim=2, op="neg_laplace", ansatz="tanh_box", ansatz_omega=16.0,
        lo=(0.0, 0.0), hi=(1.0, 1.0), n_points=(400, 400),
        levels=((1, 1), (4, 4), (16, 16)), delta=2.9, K=96,
        w_range=(-2.0, 2.0), b_range=(-1.0, 1.0), seed=0,
        meta={"family": "sines", "freqs": (1.0, 4.0, 16.0), "amps": (1.0, 0.25, 1.0 / 16.0),
              "n_test": (480, 480), "n_check": (128, 128)},
    )


def poisson5l() -> ProblemSpec:
    """u = sum_{k=1..5} sin(2^k pi x) sin(2^k pi y); levels 1,8,16,32,64; K=256; 1024^2 points."""
    return ProblemSpec(
        name="poisson5l", dim=2, op="neg_laplace", ansatz="tanh_box", ansatz_omega=32.0,
        lo=(0.0, 0.0), hi=(1.0, 1.0), n_points=(1024, 1024),
        levels=((1, 1), (8, 8), (16, 16), (32, 32), (64, 64)), delta=2.9, K=256,
        w_range=(-2.0, 2.0), b_range=(-1.0, 1.0), seed=0,
        meta={"family": "sines", "freqs": tuple(float(2 ** k) for k in range(1, 6)),
              "amps": (1.0,) * 5, "n_test": (1228, 1228), "n_check": (256, 256)},
    )


def laplace_baseline(levels=((16, 16),), seed=0) -> ProblemSpec:
    """The method's 2D multiscale Laplace baseline: n_omega=4 (4,8,12,16), K=16, 80^2 points, R=1."""
    a = 1.0 / math.sqrt(2.0)          # LeCun uniform bound R*sqrt(1/dim(z)) with R=1, dim(z)=2
    return ProblemSpec(
        name="laplace_baseline", dim=2, op="neg_laplace", ansatz="tanh_box", ansatz_omega=16.0,
        lo=(0.0, 0.0), hi=(1.0, 1.0), n_points=(80, 80), levels=tuple(levels), delta=2.9, K=16,
        w_range=(-a, a), b_range=(-a, a), seed=seed,
        meta={"family": "sines", "freqs": (4.0, 8.0, 12.0, 16.0), "amps": (0.25,) * 4,
              "n_test": (96, 96)},
    )


def helmholtz(omega: float = 8.0, levels=((16, 16),), K: int = 16, n: int = 80, k: float = 1.0,
              seed: int = 0) -> ProblemSpec:
    """Lap u + k^2 u = f on the L-shaped domain [0,1]^2 without [0.5,1]^2, u = g on the boundary
    (Sec. 4.4): the manufactured solution of eq. helmholtz_exact, k = 1; the baseline has
    omega = 8, one level of 16 x 16 subdomains (those outside the L discarded), K = 16, width
    ratio 2.9, R = 1 (W, b ~ U(-1/sqrt(2), 1/sqrt(2))), the 80 x 80 grid's points inside the L as
    interior rows, 80 boundary points per unit length with lambda_bc = 25 omega^4, and the
    96 x 96 grid's points inside the L as test points."""
    a = 1.0 / math.sqrt(2.0)
    return ProblemSpec(
        name=f"helmholtz{int(omega)}_L{len(levels)}", dim=2, op="helmholtz", ansatz="none",
        ansatz_omega=0.0, lo=(0.0, 0.0), hi=(1.0, 1.0), n_points=(n, n), levels=tuple(levels),
        delta=2.9, K=K, w_range=(-a, a), b_range=(-a, a), seed=seed, domain="l_shape",
        meta={"family": "helmholtz", "omega": float(omega), "k": float(k), "n_test": (96, 96),
              "bc_per_unit": 80, "lambda_bc": 25.0 * float(omega) ** 4},
    )


# ---------------------------------------------------------------- small parity cases

def tiny1d(K=4, J=3, n=50, delta=1.5, seed=1) -> ProblemSpec:
    return ProblemSpec(
        name="tiny1d", dim=1, op="d1", ansatz="tanh_origin", ansatz_omega=3.0,
        lo=(-1.0,), hi=(1.0,), n_points=(n,), levels=((J,),), delta=delta, K=K,
        w_range=(-1.0, 1.0), b_range=(-1.0, 1.0), seed=seed,
        meta={"family": "ode_cos", "omega": 3.0, "n_test": (97,)},
    )


def small1d_multilevel(seed=2) -> ProblemSpec:
    return ProblemSpec(
        name="small1d_ml", dim=1, op="d1", ansatz="tanh_origin", ansatz_omega=6.0,
        lo=(-2.0,), hi=(3.0,), n_points=(301,), levels=((1,), (4,), (9,)), delta=2.2, K=12,
        w_range=(-1.0, 1.0), b_range=(-1.0, 1.0), seed=seed,
        meta={"family": "ode_cos", "omega": 6.0, "n_test": (333,)},
    )


def small2d(seed=4) -> ProblemSpec:
    """Several tiles and ragged tails: 3 levels, non-square grid, K not a multiple of 16."""
    return ProblemSpec(
        name="small2d", dim=2, op="neg_laplace", ansatz="tanh_box", ansatz_omega=6.0,
        lo=(0.0, 0.0), hi=(1.0, 1.5), n_points=(61, 83), levels=((1, 1), (2, 3), (5, 6)),
        delta=2.9, K=20, w_range=(-2.0, 2.0), b_range=(-1.0, 1.0), seed=seed,
        meta={"family": "sines", "freqs": (1.0, 3.0), "amps": (1.0, 0.3), "n_test": (71, 77)},
    )


def oscillator(omega0: float = 80.0, J: int = 20, K: int = 12, n: int = 260, delta: float = 2.9,
               levels=None, seed: int = 7) -> ProblemSpec:
    """m u'' + mu u' + k u = 0 on [0, 1] with m = 1, mu = 4, k = omega0^2, u(0) = 1, u'(0) = 0
    imposed by two soft-constraint rows with weights sqrt(lambda_u0) = omega0^2 and
    sqrt(lambda_v0) = omega0; no hard-constraint factor; one level of J subdomains."""
    k = omega0 ** 2
    return ProblemSpec(
        name=f"osc{int(omega0)}", dim=1, op="oscillator", ansatz="none", ansatz_omega=0.0,
        lo=(0.0,), hi=(1.0,), n_points=(n,), levels=levels or ((J,),), delta=delta, K=K,
        w_range=(-1.0, 1.0), b_range=(-1.0, 1.0), seed=seed,
        meta={"family": "oscillator", "omega0": omega0, "osc": (1.0, 4.0, k),
              # (x, derivative order, weight sqrt(lambda), value): u(0) = 1, u'(0) = 0
              "bc": ((0.0, 0, k, 1.0), (0.0, 1, omega0, 0.0)), "n_test": (1000,)},
    )


def wide2d(K: int, seed: int = 6) -> ProblemSpec:
    """A small 2D problem with many features per subdomain (K up to 256): 3 levels, non-square
    grid, so every block is wider than it is tall in points at the finest level."""
    return ProblemSpec(
        name=f"wide2d_K{K}", dim=2, op="neg_laplace", ansatz="tanh_box", ansatz_omega=6.0,
        lo=(0.0, 0.0), hi=(1.0, 1.2), n_points=(45, 52), levels=((1, 1), (2, 2), (3, 2)),
        delta=2.9, K=K, w_range=(-2.0, 2.0), b_range=(-1.0, 1.0), seed=seed + K,
        meta={"family": "sines", "freqs": (1.0, 2.0), "amps": (1.0, 0.5), "n_test": (53, 59)},
    )


def medium2d(seed=5) -> ProblemSpec:
    """A multilevel case big enough to span many workgroups, small enough for the oracle."""
    return ProblemSpec(
        name="medium2d", dim=2, op="neg_laplace", ansatz="tanh_box", ansatz_omega=8.0,
        lo=(0.0, 0.0), hi=(1.0, 1.0), n_points=(150, 150), levels=((1, 1), (4, 4), (8, 8)),
        delta=2.9, K=48, w_range=(-2.0, 2.0), b_range=(-1.0, 1.0), seed=seed,
        meta={"family": "sines", "freqs": (1.0, 4.0, 8.0), "amps": (1.0, 0.25, 0.125),
              "n_test": (180, 180), "n_check": (64, 64)},
    )


# ---------------------------------------------------------------- problem data

def forcing(spec: ProblemSpec, pts=None) -> np.ndarray:
    pts = grid_points(spec) if pts is None else pts
    m = spec.meta
    if m["family"] == "ode_cos":
        return fam.ode_cos_forcing(pts, m["omega"])
    if m["family"] == "ode_modes":
        return fam.ode_modes_forcing(pts, m["freqs"], m["amps"])
    if m["family"] == "sines":
        return fam.sines_forcing(pts, m["freqs"], m["amps"])
    if m["family"] == "oscillator":   # homogeneous equation
        return np.zeros(len(pts))
    if m["family"] == "helmholtz":
        return fam.helmholtz_forcing(pts, m["omega"], m["k"])
    raise ValueError(m["family"])


def exact(spec: ProblemSpec, pts) -> np.ndarray:
    m = spec.meta
    if m["family"] == "ode_cos":
        return fam.ode_cos_exact(pts, m["omega"])
    if m["family"] == "ode_modes":
        return fam.ode_modes_exact(pts, m["freqs"], m["amps"])
    if m["family"] == "oscillator":
        return fam.oscillator_exact(np.asarray(pts)[:, 0], m["omega0"])
    if m["family"] == "sines":
        return fam.sines_exact(pts, m["freqs"], m["amps"])
    if m["family"] == "helmholtz":
        return fam.helmholtz_exact(np.asarray(pts), m["omega"])
    raise ValueError(m["family"])


def test_grid(spec: ProblemSpec, which="n_test") -> np.ndarray:
    return grid_points(spec, spec.meta[which])


# ---------------------------------------------------------------- batched ragged instances

def batch_instances(n=512, seed=3, n_rhs=8, J_range=(4, 24), K_range=(64, 128),
                    p_range=(20.0, 60.0)):
    """Ragged 2D Poisson instances: J~U{4..24} square, K~U{64..128}, 20..60 grid points per
    subdomain cell, 3 integer modes k~U{1..20}, per-RHS amplitudes N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs, amps = [], []
    for i in range(n):
        J = int(rng.integers(J_range[0], J_range[1] + 1))
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        p = float(rng.uniform(p_range[0], p_range[1]))
        g = int(round(J * math.sqrt(p)))
        ks = tuple(float(v) for v in rng.integers(1, 21, size=3))
        A = rng.standard_normal((n_rhs, 3))
        specs.append(ProblemSpec(
            name=f"batch{i}", dim=2, op="neg_laplace", ansatz="tanh_box", ansatz_omega=max(ks),
            lo=(0.0, 0.0), hi=(1.0, 1.0), n_points=(g, g), levels=((J, J),), delta=2.9, K=K,
            w_range=(-2.0, 2.0), b_range=(-1.0, 1.0), seed=10_000 + i,
            meta={"family": "sines", "freqs": ks, "amps": tuple(A[0]), "rhs_amps": A},
        ))
        amps.append(A)
    return specs, amps


def batch_forcing(spec: ProblemSpec) -> np.ndarray:
    """[n_rhs, N] forcing for every right-hand side of one batched instance."""
    pts = grid_points(spec)
    A = spec.meta["rhs_amps"]
    return np.stack([fam.sines_forcing(pts, spec.meta["freqs"], A[r]) for r in range(A.shape[0])])


# ---------------------------------------------------------------- warm-start families

def warm_family_1d(omega: float, coeffs) -> ProblemSpec:
    """du/dx = sum_{m=1..3} c_m cos(m omega x/3) on [-2pi,2pi], ansatz tanh(omega x); J=64, K=32."""
    freqs = tuple(m * omega / 3.0 for m in (1, 2, 3))
    return ProblemSpec(
        name="warm1d", dim=1, op="d1", ansatz="tanh_origin", ansatz_omega=float(omega),
        lo=(-2 * math.pi,), hi=(2 * math.pi,), n_points=(6000,), levels=((64,),), delta=2.9,
        K=32, w_range=(-1.0, 1.0), b_range=(-1.0, 1.0), seed=0,
        meta={"family": "ode_modes", "freqs": freqs, "amps": tuple(coeffs), "n_test": (1000,)},
    )


def warm_modes_2d(omega: float):
    """Mode numbers of the 2D warm-start family: n_m = max(1, round(m omega / 15)), m = 1..3
    (halves rounded up)."""
    return tuple(max(1, int(math.floor(m * float(omega) / 15.0 + 0.5))) for m in (1, 2, 3))


def warm_family_2d(omega: float, coeffs=(1.0, 1.0, 1.0), n: int = 200, J: int = 16,
                   K: int = 48) -> ProblemSpec:
    """-Lap u = f on [0,1]^2, u = sum_{m=1..3} c_m sin(n_m pi x) sin(n_m pi y) with
    n_m = max(1, round(m omega / 15)); hard constraint tanh(omega s) tanh(omega (1 - s)) per axis;
    one level of 16 x 16 subdomains, K = 48, width ratio 2.9, 200^2 points."""
    return ProblemSpec(
        name="warm2d", dim=2, op="neg_laplace", ansatz="tanh_box", ansatz_omega=float(omega),
        lo=(0.0, 0.0), hi=(1.0, 1.0), n_points=(n, n), levels=((J, J),), delta=2.9, K=K,
        w_range=(-1.0, 1.0), b_range=(-1.0, 1.0), seed=0,
        meta={"family": "sines", "freqs": tuple(float(v) for v in warm_modes_2d(omega)),
              "amps": tuple(coeffs), "n_test": (240, 240)},
    )


def warm_draws(n, seed):
    """Problem parameters (omega ~ U[5,50], c ~ N(0,1)^3) for n instances."""
    rng = np.random.Generator(np.random.PCG64(seed))
    om = rng.uniform(5.0, 50.0, size=n)
    c = rng.standard_normal((n, 3))
    return om, c


def warm_groups(n_groups, seed, n_rhs=8):
    """Parameters of the 1D warm-start family in groups that share omega (one matrix, n_rhs
    source-coefficient vectors): omega ~ U[5, 50], c ~ N(0, 1)^3 per right-hand side."""
    rng = np.random.Generator(np.random.PCG64(seed))
    om = rng.uniform(5.0, 50.0, size=n_groups)
    C = rng.standard_normal((n_groups, n_rhs, 3))
    return om, C


def warm_batch_forcing(spec: ProblemSpec, C) -> np.ndarray:
    """[n_rhs, N] forcing of one warm-family instance (1D or 2D) for each coefficient vector
    C[r]."""
    pts = grid_points(spec)
    f = fam.sines_forcing if spec.dim == 2 else fam.ode_modes_forcing
    return np.stack([f(pts, spec.meta["freqs"], c) for c in C])


def warm_exact(spec: ProblemSpec, c, pts) -> np.ndarray:
    """Exact solution of a warm-family instance with coefficient vector c at points pts."""
    f = fam.sines_exact if spec.dim == 2 else fam.ode_modes_exact
    return f(np.asarray(pts), spec.meta["freqs"], c)


def boundary_points(spec: ProblemSpec) -> np.ndarray:
    """Boundary collocation points of an L-shaped problem [N_B, 2]."""
    return l_shape_boundary(spec, spec.meta["bc_per_unit"])


def in_l_shape(spec: ProblemSpec, pts) -> np.ndarray:
    """Points of a grid that belong to the L-shaped domain (not strictly inside the removed
    upper-right quarter): the problem's domain, used to pick test points."""
    pts = np.asarray(pts)
    mid = 0.5 * (np.asarray(spec.lo) + np.asarray(spec.hi))
    return ~((pts[:, 0] > mid[0]) & (pts[:, 1] > mid[1]))
