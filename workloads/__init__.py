"""Seeded synthetic inputs for the parareal-with-splitting workloads.

This module only draws and samples input data (initial states, coefficient
fields, partition-of-unity weights, perturbation directions). It holds none of
the method's arithmetic, so the oracle and the HIP path can both be fed from
it. All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).

Grid convention: n interior nodes per direction, h = 1/(n+1), interior node i
(0-based) at x = (i+1) h; "extended" grids add the two boundary nodes
(x = 0 and x = 1). Faces f = 0..n of a line sit at x = (f + 1/2) h.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.fft

__all__ = [
    "smooth_field_1d", "smooth_field_2d", "sine_modes_2d", "sine_series_1d",
    "linear_pou_1d", "Workload", "config1", "config2", "config3", "config4", "config5",
    "small_dim2", "small_dd1", "strip_pou_2d", "small_dd2", "dd2_manufactured",
]


def _cos_sin_table(x, K):
    k = np.arange(-K, K + 1)[:, None]
    arg = 2.0 * np.pi * k * x[None, :]
    return np.cos(arg), np.sin(arg)


def smooth_field_1d(n_ext: int, ell: float, K: int, seed: int) -> np.ndarray:
    """Stationary Gaussian field g(x) = sum_k sqrt(S_k)(xi_k cos 2pi k x + eta_k sin 2pi k x),
    |k| <= K, spectral weight S_k = exp(-2 pi^2 ell^2 k^2), scaled to unit variance,
    sampled on the n_ext nodes of the extended grid of [0, 1]."""
    rng = np.random.default_rng(seed)
    ks = np.arange(-K, K + 1)
    S = np.exp(-2.0 * np.pi ** 2 * ell ** 2 * ks.astype(float) ** 2)
    S = S / S.sum()
    xi = rng.standard_normal(ks.size)
    eta = rng.standard_normal(ks.size)
    x = np.arange(n_ext) / (n_ext - 1)
    Cx, Sx = _cos_sin_table(x, K)
    w = np.sqrt(S)
    return (w * xi) @ Cx + (w * eta) @ Sx


def smooth_field_2d(nx_ext: int, ny_ext: int, ell: float, K: int, seed: int) -> np.ndarray:
    """2D version of :func:`smooth_field_1d` on the extended (ny_ext, nx_ext) grid,
    wave vectors k in [-K, K]^2, S_k = exp(-2 pi^2 ell^2 |k|^2)."""
    rng = np.random.default_rng(seed)
    ks = np.arange(-K, K + 1).astype(float)
    S = np.exp(-2.0 * np.pi ** 2 * ell ** 2 * (ks[:, None] ** 2 + ks[None, :] ** 2))  # [k2, k1]
    S = S / S.sum()
    w = np.sqrt(S)
    xi = rng.standard_normal(S.shape) * w
    eta = rng.standard_normal(S.shape) * w
    x = np.arange(nx_ext) / (nx_ext - 1)
    y = np.arange(ny_ext) / (ny_ext - 1)
    Cx, Sx = _cos_sin_table(x, K)  # [k1, x]
    Cy, Sy = _cos_sin_table(y, K)  # [k2, y]
    # cos(a+b) = CaCb - SaSb ; sin(a+b) = SaCb + CaSb with a = 2pi k1 x, b = 2pi k2 y
    g = Cy.T @ xi @ Cx - Sy.T @ xi @ Sx + Cy.T @ eta @ Sx + Sy.T @ eta @ Cx
    return g  # [y, x]


def sine_modes_2d(nx: int, ny: int, seed: int, kmax: int = 4) -> np.ndarray:
    """u0 = sum_{k1,k2=1..kmax} c_k sin(k1 pi x) sin(k2 pi y), c_k ~ N(0,1)/(k1^2+k2^2),
    on the interior nodes, shape (ny, nx)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((kmax, kmax))  # [k2-1, k1-1]
    k = np.arange(1, kmax + 1)
    c = c / (k[:, None] ** 2 + k[None, :] ** 2)
    x = np.arange(1, nx + 1) / (nx + 1)
    y = np.arange(1, ny + 1) / (ny + 1)
    Sx = np.sin(np.pi * k[:, None] * x[None, :])
    Sy = np.sin(np.pi * k[:, None] * y[None, :])
    return Sy.T @ c @ Sx


def sine_series_1d(n: int, seed: int, kmax: int = 4096) -> np.ndarray:
    """u0 = sum_{k=1..kmax} xi_k / k sin(k pi x), xi ~ N(0,1), on n interior nodes
    (a type-I discrete sine transform of the coefficient vector)."""
    rng = np.random.default_rng(seed)
    kmax = min(kmax, n)
    coef = np.zeros(n)
    coef[:kmax] = rng.standard_normal(kmax) / np.arange(1, kmax + 1)
    return scipy.fft.dst(coef, type=1) / 2.0


def linear_pou_1d(n: int, n_cores: int, overlap: int, n_colors: int) -> np.ndarray:
    """Partition-of-unity face weights rho[color, f], f = 0..n, for n interior nodes split
    into n_cores equal cores; core k has colour k % n_colors. Across each core boundary
    (face c) the weight ramps linearly over the `overlap` faces c-overlap/2 .. c+overlap/2-1,
    taking the values (2m+1)/(2*overlap), m = 0..overlap-1; weights sum to 1 on every face."""
    assert n % n_cores == 0 and overlap % 2 == 0
    core = n // n_cores
    half = overlap // 2
    assert half < core // 2
    f = np.arange(n + 1)
    chi = np.zeros((n_cores, n + 1))
    for k in range(n_cores):
        lo, hi = k * core, (k + 1) * core
        left = np.ones(n + 1) if k == 0 else np.clip((2 * (f - (lo - half)) + 1) / (2 * overlap), 0, 1)
        right = np.ones(n + 1) if k == n_cores - 1 else np.clip(1 - (2 * (f - (hi - half)) + 1) / (2 * overlap), 0, 1)
        chi[k] = np.minimum(left, right)
    rho = np.zeros((n_colors, n + 1))
    for k in range(n_cores):
        rho[k % n_colors] += chi[k]
    return rho


def strip_pou_2d(n: int, q: int, beta: float, n_colors: int = 2) -> np.ndarray:
    """Partition of unity of the 2D domain decomposition into vertical strips:
    n_colors * q equal cores of [0, 1] in x, core k of colour k % n_colors; across
    each interior core boundary b the left core's weight falls from 1 to 0 over
    [b - beta/2, b + beta/2] as cos^2(pi/2 (x - b + beta/2)/beta) and the right
    core's rises as one minus it, so every colour's support is q strips, each
    overlapping its neighbours by beta. Sampled on the half grid of x:
    rho[k, m] at x = (m + 1) h / 2, m = 0..2n (m = 2f: x-face f, m = 2i+1: node i);
    weights are exactly 0 or 1 outside the overlaps and sum to 1 everywhere."""
    n_cores = n_colors * q
    assert 0.0 < beta < 1.0 / n_cores
    x = (np.arange(2 * n + 1) + 1) * (0.5 / (n + 1))
    chi = np.zeros((n_cores, 2 * n + 1))
    for k in range(n_cores):
        left = np.ones_like(x)
        right = np.ones_like(x)
        if k > 0:
            a = k / n_cores - beta / 2
            t = np.clip((x - a) / beta, 0.0, 1.0)
            left = 1.0 - np.cos(0.5 * np.pi * t) ** 2
            left[x <= a] = 0.0
            left[x >= a + beta] = 1.0
        if k < n_cores - 1:
            a = (k + 1) / n_cores - beta / 2
            t = np.clip((x - a) / beta, 0.0, 1.0)
            right = np.cos(0.5 * np.pi * t) ** 2
            right[x <= a] = 1.0
            right[x >= a + beta] = 0.0
        chi[k] = np.minimum(left, right)
    # make each overlap's pair sum to exactly one (the right weight is 1 - left)
    for k in range(n_cores - 1):
        a = (k + 1) / n_cores - beta / 2
        m = (x > a) & (x < a + beta)
        chi[k + 1, m] = 1.0 - chi[k, m]
    rho = np.zeros((n_colors, 2 * n + 1))
    for k in range(n_cores):
        rho[k % n_colors] += chi[k]
    return rho


@dataclass
class Workload:
    """One problem instance: shapes, times and input arrays (all float64 numpy)."""
    name: str
    dim: int
    nx: int
    ny: int
    T: float
    n_slices: int
    fine_steps: int
    coarse_steps: int = 1
    split: str = "dim"          # "dim" or "dd"
    fine: str = "fie"           # "fie" or "dr"
    c: float = 0.0
    ax: Optional[np.ndarray] = None      # faces, (ny, nx+1)
    ay: Optional[np.ndarray] = None      # faces, (ny+1, nx)
    theta: Optional[np.ndarray] = None   # nodal log-coefficient on the extended grid
    rho: Optional[np.ndarray] = None     # (M, nx+1) in 1D, (M, 2nx+1) in 2D
    u0: Optional[np.ndarray] = None
    k_max: int = 0
    tol: float = 0.0
    # source F(t) = sum_m g_m(t) S_m: (S (m, ny, nx), g at the fine step ends
    # (m, N*s), g at the coarse step ends (m, N*cs)), or None
    forcing: Optional[tuple] = None
    extra: dict = field(default_factory=dict)

    @property
    def npts(self):
        return self.nx * self.ny

    @property
    def point_updates_per_iteration(self):
        return self.npts * self.fine_steps * self.n_slices


def _face_coords(n):
    h = 1.0 / (n + 1)
    return (np.arange(n + 1) + 0.5) * h, np.arange(1, n + 1) * h


def config1() -> Workload:
    """2D heat u_t = Lap u, 32x32 interior, u0 = sin(pi x) sin(pi y), T = 0.1,
    N = 8 slices, s = 16 fine steps, one coarse step, K = 8 iterations."""
    n = 32
    x = np.arange(1, n + 1) / (n + 1)
    u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    return Workload("heat2d_32_N8_s16", 2, n, n, 0.1, 8, 16, ax=np.ones((n, n + 1)),
                    ay=np.ones((n + 1, n)), u0=u0, k_max=8, tol=0.0)


def variable_faces_2d(nx, ny):
    """a(x, y) = 1 + 0.5 sin(2 pi x) cos(2 pi y) sampled at face midpoints."""
    xf, xn = _face_coords(nx)
    yf, yn = _face_coords(ny)
    ax = 1.0 + 0.5 * np.sin(2 * np.pi * xf)[None, :] * np.cos(2 * np.pi * yn)[:, None]
    ay = 1.0 + 0.5 * np.sin(2 * np.pi * xn)[None, :] * np.cos(2 * np.pi * yf)[:, None]
    return ax, ay


def config2(n: int = 1023, n_slices: int = 64, fine_steps: int = 64) -> Workload:
    """2D u_t = div(a grad u), a = 1 + 0.5 sin(2 pi x) cos(2 pi y), 1023^2 interior,
    u0 = 16 seeded sine modes (seed 2), T = 0.05, N = 64, s = 64, stop at increment < 1e-8."""
    ax, ay = variable_faces_2d(n, n)
    return Workload(f"varcoef2d_{n}_N{n_slices}_s{fine_steps}", 2, n, n, 0.05, n_slices, fine_steps,
                    ax=ax, ay=ay, u0=sine_modes_2d(n, n, seed=2), k_max=n_slices, tol=1e-8)


def config3(n: int = 1 << 20, n_cores: int = 8, n_colors: int = 2, overlap: int = 32,
            n_slices: int = 32, fine_steps: int = 128, T: float = 2.0 ** -22) -> Workload:
    """1D u_t = (a u_x)_x with domain-decomposition splitting: 2^20 interior nodes,
    8 overlapping cores (overlap 32 cells), linear partition of unity, a = exp(0.3 g) with g
    a smooth Gaussian field (correlation length 0.05, seed 3), u0 a random sine series
    (seed 13), N = 32, s = 128."""
    theta = 0.3 * smooth_field_1d(n + 2, ell=0.05, K=40, seed=3)
    rho = linear_pou_1d(n, n_cores, overlap, n_colors)
    return Workload(f"dd1d_{n}_M{n_colors}_N{n_slices}_s{fine_steps}", 1, n, 1, T, n_slices,
                    fine_steps, split="dd", theta=theta, rho=rho, u0=sine_series_1d(n, seed=13),
                    k_max=n_slices, tol=1e-8)


def config4(n_instances: int = 256, sizes=(63, 127, 255, 511), slices=(16, 32, 64),
            fine_steps: int = 32, seed: int = 4) -> list:
    """Batch of independent 2D instances with n ~ U(sizes), N ~ U(slices),
    a = exp(0.5 g) (g smooth Gaussian field, correlation length 0.1, seed 4+i),
    u0 as config 2 (seed 1000+i), T = 0.05, s = 32, tolerance 1e-8 per instance."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=n_instances)
    Ns = rng.choice(np.asarray(slices), size=n_instances)
    return [batch_instance(i, int(ns[i]), int(Ns[i]), fine_steps) for i in range(n_instances)]


def batch_instance(i: int, n: int, n_slices: int, fine_steps: int = 32) -> Workload:
    """Instance i of the batch workload at grid n and N slices: a = exp(0.5 g) (g smooth
    Gaussian field, correlation length 0.1, seed 4+i), u0 as config 2 (seed 1000+i),
    T = 0.05, tolerance 1e-8."""
    theta = 0.5 * smooth_field_2d(n + 2, n + 2, ell=0.1, K=20, seed=4 + i)
    return Workload(f"batch{i}_{n}_N{n_slices}", 2, n, n, 0.05, n_slices, fine_steps, theta=theta,
                    u0=sine_modes_2d(n, n, seed=1000 + i), k_max=n_slices, tol=1e-8)


def config5(n: int = 511, n_slices: int = 32, fine_steps: int = 32, n_dirs: int = 20) -> Workload:
    """Differentiation workload: 511^2, a = exp(theta); hidden theta* = 0.5 g (seed 5),
    evaluation theta = 0.5 g (seed 6), u0 as config 2 (seed 7), 20 smooth perturbation
    directions (seeds 100..119) in (u0, theta), T = 0.05, N = 32, s = 32."""
    theta_star = 0.5 * smooth_field_2d(n + 2, n + 2, ell=0.1, K=20, seed=5)
    theta = 0.5 * smooth_field_2d(n + 2, n + 2, ell=0.1, K=20, seed=6)
    dirs = []
    for d in range(n_dirs):
        du = sine_modes_2d(n, n, seed=100 + d)
        dth = smooth_field_2d(n + 2, n + 2, ell=0.1, K=20, seed=100 + d)
        du /= np.abs(du).max()
        dth /= np.abs(dth).max()
        dirs.append((du, dth))
    return Workload(f"adjoint2d_{n}_N{n_slices}_s{fine_steps}", 2, n, n, 0.05, n_slices, fine_steps,
                    theta=theta, u0=sine_modes_2d(n, n, seed=7), k_max=n_slices,
                    extra={"theta_star": theta_star, "dirs": dirs})


def small_dim2(nx: int, ny: int, n_slices: int, fine_steps: int, seed: int = 0, T: float = 0.05,
               variable: bool = True, c: float = 0.0) -> Workload:
    """Small 2D dimensional-splitting case for tests: log-normal coefficient field
    (theta = 0.5 g) or a = 1, seeded sine-mode u0 plus small white noise."""
    rng = np.random.default_rng(seed + 7919)
    theta = (0.5 * smooth_field_2d(nx + 2, ny + 2, ell=0.2, K=6, seed=seed)
             if variable else np.zeros((ny + 2, nx + 2)))
    u0 = sine_modes_2d(nx, ny, seed=seed + 1) + 0.01 * rng.standard_normal((ny, nx))
    return Workload(f"small2d_{nx}x{ny}_N{n_slices}_s{fine_steps}", 2, nx, ny, T, n_slices,
                    fine_steps, theta=theta, u0=u0, c=c, k_max=n_slices, tol=0.0)


def small_dd1(n: int, n_cores: int, n_colors: int, overlap: int, n_slices: int, fine_steps: int,
              seed: int = 0, T: float = 1e-3) -> Workload:
    """Small 1D domain-decomposition case for tests."""
    theta = 0.3 * smooth_field_1d(n + 2, ell=0.1, K=8, seed=seed)
    rho = linear_pou_1d(n, n_cores, overlap, n_colors)
    return Workload(f"smalldd_{n}_M{n_colors}_q{n_cores // n_colors}", 1, n, 1, T, n_slices,
                    fine_steps, split="dd", theta=theta, rho=rho,
                    u0=sine_series_1d(n, seed=seed + 1, kmax=min(n, 64)), k_max=n_slices, tol=0.0)


def small_dd2(nx: int, ny: int, q: int, beta: float, n_slices: int, fine_steps: int,
              seed: int = 0, T: float = 0.01, n_colors: int = 2, variable: bool = True,
              c: float = 0.0) -> Workload:
    """Small 2D domain-decomposition case (vertical strips) for tests: log-normal
    coefficient field (or a = 1), seeded sine-mode u0 plus small white noise."""
    w = small_dim2(nx, ny, n_slices, fine_steps, seed=seed, T=T, variable=variable, c=c)
    w.name = f"smalldd2_{nx}x{ny}_M{n_colors}_q{q}_N{n_slices}_s{fine_steps}"
    w.split = "dd"
    w.rho = strip_pou_2d(nx, q, beta, n_colors)
    return w


def dd2_manufactured(n: int = 999, n_slices: int = 20, fine_steps: int = 20, q: int = 2,
                     beta: float = 1.0 / 16, coarse_steps: int = 1) -> Workload:
    """The paper's 2D domain-decomposition runs (section 5, constant diagonal D):
    the manufactured test problem split into two subdomains of q vertical strips
    each with overlap beta, for both propagators. Defaults: h = 1e-3, DT = 0.05,
    dt = 2.5e-3, q = 2, beta = 1/16."""
    w = manufactured2d(n, n_slices, fine_steps, coarse_steps=coarse_steps)
    w.name = f"dd2d_{n}_M2_q{q}_N{n_slices}_s{fine_steps}"
    w.split = "dd"
    w.rho = strip_pou_2d(n, q, beta, 2)
    return w


def step_end_times(T: float, n_slices: int, steps: int) -> np.ndarray:
    """End times of the steps of every slice: t = n*DT + (j+1)*DT/steps, ordered
    slice-major (the layout of the source time tables)."""
    DT = T / n_slices
    n = np.repeat(np.arange(n_slices), steps)
    j = np.tile(np.arange(steps), n_slices)
    return n * DT + (j + 1) * (DT / steps)


def manufactured2d(n: int, n_slices: int, fine_steps: int, coarse_steps: int = 1,
                   T: float = 1.0) -> Workload:
    """The paper's test problem (section 5): heat equation on the unit square with
    D = I, homogeneous Dirichlet data, u0 = 0 and the source f for which
    u = sin(2 pi t) sin(2 pi x) sin(2 pi y) is the exact solution:
    f = u_t - Lap u = (2 pi cos 2 pi t + 8 pi^2 sin 2 pi t) sin(2 pi x) sin(2 pi y),
    sampled at the interior nodes (one separable source term). The paper's run:
    h = 1e-3 (n = 999), DT = 0.05 (N = 20), dt = 2.5e-3 (s = 20), T = 1."""
    x = np.arange(1, n + 1) / (n + 1)
    S = np.outer(np.sin(2 * np.pi * x), np.sin(2 * np.pi * x))[None]
    g = lambda t: (2 * np.pi * np.cos(2 * np.pi * t) + 8 * np.pi ** 2 * np.sin(2 * np.pi * t))[None]
    w = Workload(f"manufactured2d_{n}_N{n_slices}_s{fine_steps}", 2, n, n, T, n_slices, fine_steps,
                 coarse_steps=coarse_steps, theta=np.zeros((n + 2, n + 2)), u0=np.zeros((n, n)),
                 forcing=(S, g(step_end_times(T, n_slices, fine_steps)),
                          g(step_end_times(T, n_slices, coarse_steps))),
                 k_max=n_slices, tol=1e-6)
    w.extra["exact_space"] = S[0]
    return w
