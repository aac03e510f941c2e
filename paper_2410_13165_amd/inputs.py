"""Seeded synthetic inputs shared by the tests, the benchmark and the examples.

Only parameter draws live here (field amplitudes, wave vectors, phases,
velocities, noise); nothing of the lattice Boltzmann method itself.  Each
workload returns plain dicts that both the GPU binding and the CPU oracle
accept.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

TWO_PI = 2.0 * math.pi


def plane_sine(d: int, u: Sequence[float], R: float = 0.0) -> dict:
    """phi0 = prod_i sin(2 pi x_i) written as a sum of cosines (exact in 1-3D)."""
    if d == 1:
        modes = [(1.0, [TWO_PI], -math.pi / 2)]
    elif d == 2:
        # sin a sin b = (cos(a - b) - cos(a + b)) / 2
        modes = [(0.5, [TWO_PI, -TWO_PI], 0.0), (-0.5, [TWO_PI, TWO_PI], 0.0)]
    elif d == 3:
        # sin a sin b sin c = (sin(a+b-c) + sin(a-b+c) + sin(-a+b+c) - sin(a+b+c)) / 4
        modes = []
        for sgn, amp in (((1, 1, -1), 0.25), ((1, -1, 1), 0.25), ((-1, 1, 1), 0.25),
                         ((1, 1, 1), -0.25)):
            modes.append((amp, [TWO_PI * s for s in sgn], -math.pi / 2))
    else:
        raise ValueError("plane_sine is defined for d <= 3")
    return {"kind": "cos_sum", "amps": [m[0] for m in modes], "kvecs": [m[1] for m in modes],
            "phases": [m[2] for m in modes], "u": list(u), "R": R}


def diagonal_sine(d: int, u: Sequence[float], k: float = math.pi) -> dict:
    """Example 3: phi* = sin[pi (sum_i x_i - u_i t)]."""
    return {"kind": "cos_sum", "amps": [1.0], "kvecs": [[k] * d], "phases": [-math.pi / 2],
            "u": list(u), "R": 0.0}


def example1(u: Sequence[float], R: float = 5.0) -> dict:
    """Example 1: exp[-(x1 - u1 t) - (x2 - u2 t)] + R t."""
    return {"kind": "exp_sum", "amps": [1.0], "kvecs": [[-1.0, -1.0]], "phases": [0.0],
            "u": list(u), "R": R}


def tanh_bubble(d: int, u: Sequence[float]) -> dict:
    """Example 2: 1/2 - 1/2 tanh((Rr - |x - u t|)/(2W)), Rr = 1/(5(d-1)), W = (5-d)/75."""
    return {"kind": "tanh_bubble", "Rr": 1.0 / (5.0 * (d - 1)), "W": (5.0 - d) / 75.0,
            "center": [0.0] * d, "u": list(u), "R": 0.0}


def random_cosines(d: int, u: Sequence[float], R: float, seed: int, n_modes: int = 4,
                   kmax: float = 3.0) -> dict:
    """Sum of n random-wavevector cosines: a_j ~ N(0,1), kappa_j = 2 pi U(-kmax, kmax)^d,
    theta_j ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    amps = rng.normal(size=n_modes)
    kv = TWO_PI * rng.uniform(-kmax, kmax, size=(n_modes, d))
    ph = rng.uniform(0.0, TWO_PI, size=n_modes)
    return {"kind": "cos_sum", "amps": amps.tolist(), "kvecs": kv.tolist(),
            "phases": ph.tolist(), "u": list(u), "R": R}


def tau_draw(seed: int, lo: float, hi: float) -> float:
    return float(np.random.default_rng(seed).uniform(lo, hi))


def noise(shape: Sequence[int], seed: int, std: float = 1e-3) -> np.ndarray:
    """i.i.d. N(0, std^2) values, float64, C order of the given shape."""
    return np.random.default_rng(seed).normal(0.0, std, size=tuple(shape))


def gaussian_random_field(n: int, d: int, seed: int, corr: float = 0.1) -> np.ndarray:
    """Periodic Gaussian random field on [0,1)^d with n nodes per axis: white
    noise filtered by sqrt(exp(-|k|^2 corr^2 / 2)) in Fourier space, scaled to unit
    variance.  Returned in C order of shape (n,)*d (any axis order: isotropic)."""
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(n,) * d)
    W = np.fft.rfftn(w)
    k1 = 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n)
    kr = 2.0 * np.pi * np.fft.rfftfreq(n, d=1.0 / n)
    grids = np.meshgrid(*([k1] * (d - 1) + [kr]), indexing="ij", sparse=True)
    k2 = sum(g * g for g in grids)
    W *= np.sqrt(np.exp(-0.5 * k2 * corr * corr))
    f = np.fft.irfftn(W, s=(n,) * d, axes=tuple(range(d)))
    f -= f.mean()
    return f / f.std()


# Gradient workload: D3Q19 on the periodic unit cube with 256 nodes per axis,
# u = (0.05, 0.1, 0.08), tau = 1/2, R = 0, 1000 float32 steps from a Gaussian
# random field (correlation length 0.1, seed 5), misfit to another field (seed 6),
# checkpoints every 32 steps.
ADJOINT_D3Q19 = {"d": 3, "n": 256, "u": [0.05, 0.1, 0.08], "steps": 1000, "every": 32,
                 "seed_init": 5, "seed_target": 6, "corr": 0.1}


# Stability sweep: 512 independent periodic D2Q9 lattices, sizes drawn from
# {64^2, 128^2, 256^2, 512^2}, tau ~ U(0.5, 2.0), sigma ~ U(-0.75, 0.75)^2
# (straddling the |sigma| < 1/2 region), R = 0, K = 1, noise of standard deviation
# 1e-3, 4000 steps.
SWEEP_D2Q9 = {"count": 512, "sizes": [64, 128, 256, 512], "tau": (0.5, 2.0),
              "sigma": (-0.75, 0.75), "std": 1e-3, "steps": 4000, "seed": 4}


def sweep_specs(count=None, seed=None):
    w = SWEEP_D2Q9
    rng = np.random.default_rng(w["seed"] if seed is None else seed)
    specs = []
    for _ in range(count or w["count"]):
        n = int(w["sizes"][rng.integers(0, len(w["sizes"]))])
        specs.append({"dims": (n, n), "tau": float(rng.uniform(*w["tau"])),
                      "u": rng.uniform(*w["sigma"], size=2).tolist(), "dx": 1.0 / n, "K": 1})
    return specs


def sweep_phi0(specs, seed=None):
    w = SWEEP_D2Q9
    rng = np.random.default_rng((w["seed"] if seed is None else seed) + 1000)
    return np.concatenate([rng.normal(0.0, w["std"], size=int(np.prod(sp["dims"])))
                           for sp in specs])


# Workload of the benchmark: D3Q19 on the unit cube, 512 nodes per axis,
# full-way Dirichlet walls on all six faces with data from four random cosines
# (seed 3), u = (0.05, 0.1, 0.08) (Table 3), R = 1, K = 3, P = 4.
BENCH_D3Q19 = {
    "d": 3, "n": 512, "u": [0.05, 0.1, 0.08], "R": 1.0, "seed": 3, "steps": 2000,
}


def bench_field() -> dict:
    w = BENCH_D3Q19
    return random_cosines(3, w["u"], w["R"], w["seed"])
