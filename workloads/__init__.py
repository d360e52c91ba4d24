"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds only input generation: box and method parameters of the named
workloads, and seeded random charge sets. It contains none of the method's
arithmetic, so the CPU oracle and the HIP path can both consume it without
sharing any computation.

Recipe (the paper's performance and accuracy tests place uniform random charges
of alternating sign in a slab, Sec. 6.2, 6.3 and 7.4):
  * ``numpy.random.default_rng(seed)`` (PCG64);
  * draw x ~ U[0, Lx), y ~ U[0, Ly), z ~ U(z_lo, z_hi) as whole vectors, in that order;
  * charges: the first ``n_pos`` entries get +q_pos, the rest -q_neg, then a seeded
    permutation is applied (``rng.permutation``), so the set is exactly neutral.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np


@dataclasses.dataclass
class SlabParams:
    """Box, permittivities and method parameters of one slab system.

    Lengths share one unit; the Poisson equation is eps*Lap(phi) = -rho, so a
    point charge q at distance r in a uniform medium has potential q/(4*pi*eps*r).
    ``n_g = 0`` means the support is derived as 2*ceil(4.3*g_t/h).
    ``uniform_fast`` selects the solver for equal permittivities inside and
    outside (no wall group, no images, no correction, z domain [-H_E, H+H_E]);
    ``one_jump`` the solver for a jump at one wall only (every charge imaged
    across it, then the free-space solve on the span of charges and images);
    ``triply`` the triply periodic variant (z periodic with period H, uniform
    z grid of Nz nodes). ``deterministic`` asks the HIP path for
    bitwise-reproducible solves (no effect on what is computed).
    """

    Lx: float
    Ly: float
    H: float
    eps: float
    eps_b: float
    eps_t: float
    xi: float
    Nx: int
    Ny: int
    Nz: int
    r_cut: float
    g_w: float = 0.0
    n_g: int = 0
    gauge: bool = True
    kmax_gt: bool = False
    uniform_fast: bool = False
    one_jump: bool = False
    triply: bool = False
    deterministic: bool = False

    def copy(self, **kw) -> "SlabParams":
        return dataclasses.replace(self, **kw)


def charges(seed: int, n_pos: int, n_neg: int, Lx: float, Ly: float,
            z_lo: float, z_hi: float, q_pos: float = 1.0,
            q_neg: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Uniform random charges in [0,Lx) x [0,Ly) x (z_lo, z_hi), exactly neutral
    when n_pos*q_pos == n_neg*q_neg. Returns (pos[N,3] float64, q[N] float64)."""
    n = n_pos + n_neg
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, Lx, n)
    y = rng.uniform(0.0, Ly, n)
    z = rng.uniform(z_lo, z_hi, n)
    q = np.concatenate([np.full(n_pos, q_pos), np.full(n_neg, -q_neg)])
    q = q[rng.permutation(n)]
    pos = np.stack([x, y, z], axis=1)
    return np.ascontiguousarray(pos), np.ascontiguousarray(q)


# --- the named workloads ---------------------------------------------------

def config_small(seed: int = 0):
    """N=64 (32 of +1, 32 of -1) in Lx=Ly=16, H=16, 0.5<z<15.5; uniform
    permittivity 1; xi=0.5; grid 32x32x33; near cutoff 4.0."""
    p = SlabParams(Lx=16.0, Ly=16.0, H=16.0, eps=1.0, eps_b=1.0, eps_t=1.0,
                   xi=0.5, Nx=32, Ny=32, Nz=33, r_cut=4.0)
    pos, q = charges(seed, 32, 32, 16.0, 16.0, 0.5, 15.5)
    return p, pos, q


def config_jump(seed: int = 0):
    """N=16384 monovalent ions in Lx=Ly=64, H=32, 0.5<z<31.5; eps=1 inside,
    eps_b=eps_t=0.05; xi=1.0; grid 256x256x129; near cutoff 3.0."""
    p = SlabParams(Lx=64.0, Ly=64.0, H=32.0, eps=1.0, eps_b=0.05, eps_t=0.05,
                   xi=1.0, Nx=256, Ny=256, Nz=129, r_cut=3.0)
    pos, q = charges(seed, 8192, 8192, 64.0, 64.0, 0.5, 31.5)
    return p, pos, q


def config_large(seed: int = 0, divalent: bool = False):
    """N=1,048,576 ions (+1/-1), or the +2/-1 variant with N=1,048,575
    (349,525 of +2 and 699,050 of -1), in Lx=Ly=256, H=64, 0.5<z<63.5;
    eps=1, eps_b=0.05, eps_t=20; xi=1.5; grid 1024x1024x257; cutoff 2.0."""
    p = SlabParams(Lx=256.0, Ly=256.0, H=64.0, eps=1.0, eps_b=0.05, eps_t=20.0,
                   xi=1.5, Nx=1024, Ny=1024, Nz=257, r_cut=2.0)
    if divalent:
        pos, q = charges(seed, 349525, 699050, 256.0, 256.0, 0.5, 63.5,
                         q_pos=2.0, q_neg=1.0)
    else:
        pos, q = charges(seed, 524288, 524288, 256.0, 256.0, 0.5, 63.5)
    return p, pos, q


def scaled_jump(seed: int, L: float, H: float, n_pairs: int, eps_b: float = 0.05,
                eps_t: float = 0.05, xi: float = 1.0, h: float = 0.25,
                r_cut: float = 3.0, Nz: int | None = None):
    """A smaller system with the jump workload's resolution (h, xi) and
    density family: Lx=Ly=L, grid L/h per side, Nz = H/h + 1 unless given."""
    n = int(round(L / h))
    nz = Nz if Nz is not None else int(round(H / h)) + 1
    p = SlabParams(Lx=L, Ly=L, H=H, eps=1.0, eps_b=eps_b, eps_t=eps_t, xi=xi,
                   Nx=n, Ny=n, Nz=nz, r_cut=r_cut)
    pos, q = charges(seed, n_pairs, n_pairs, L, L, 0.5, H - 0.5)
    return p, pos, q


def gaussian_walls(p: SlabParams, s: float, sign_b: float = 1.0, sign_t: float = -1.0,
                   center: Tuple[float, float] | None = None) -> Tuple[np.ndarray, np.ndarray]:
    """Wall charge densities sampled at the x,y grid points [Ny, Nx]: a
    Gaussian of standard deviation s and unit total charge times sign on each
    wall, sigma = sign/(2 pi s^2) exp(-r^2/(2 s^2)) with r the periodic
    distance to ``center`` (the box centre by default). The charged-wall test
    of the paper takes +-1/2 of that on the two walls."""
    h = p.Lx / p.Nx
    cx, cy = center if center is not None else (0.5 * p.Lx, 0.5 * p.Ly)
    dx = np.arange(p.Nx) * h - cx
    dy = np.arange(p.Ny) * h - cy
    dx -= p.Lx * np.round(dx / p.Lx)
    dy -= p.Ly * np.round(dy / p.Ly)
    g = np.exp(-(dy[:, None] ** 2 + dx[None, :] ** 2) / (2.0 * s * s)) / (2.0 * math.pi * s * s)
    return sign_b * g, sign_t * g


def config_charged_walls(seed: int = 0, g_w: float = 1e-2, n: int = 10, Nx: int = 32, Nz: int = 129):
    """The charged-wall energy test: box 2 x 2 x 1, eps = 1, eps_b = 1/20,
    eps_t = 1/50, xi = 6.8, n unit charges of alternating sign uniform in
    [0,2)^2 x [4.5 g_w, 1 - 4.5 g_w], Gaussian wall densities of s = 0.2 and
    total charge +1/2 (bottom) and -1/2 (top) at the box centre, r_cut = 0.53.
    Returns (params, pos, q, sigma_b, sigma_t)."""
    p = SlabParams(Lx=2.0, Ly=2.0, H=1.0, eps=1.0, eps_b=1.0 / 20.0, eps_t=1.0 / 50.0, xi=6.8,
                   Nx=Nx, Ny=Nx, Nz=Nz, r_cut=0.53, g_w=g_w)
    pos, q = charges(seed, n // 2, n // 2, 2.0, 2.0, 4.5 * g_w, 1.0 - 4.5 * g_w)
    sb, st = gaussian_walls(p, 0.2)
    return p, pos, q, 0.5 * sb, 0.5 * st


def config_triply(seed: int = 0):
    """The triply periodic performance workload of Sec. 7.4: 2 x 10^4 charges
    of alternating sign uniform in a 185 x 185 x 100 box (Lz = 2H of the slab
    test), point charges, 64^2 x 32 grid (the paper's optimum is 70^2; a power
    of two here), g_t = 1.2 h (the 3-digit setting), r_cut = 20.7 (xi r_cut = 3,
    as in the slab workloads)."""
    h = 185.0 / 64
    xi = 1.0 / (2.0 * 1.2 * h)
    p = SlabParams(Lx=185.0, Ly=185.0, H=100.0, eps=1.0, eps_b=1.0, eps_t=1.0, xi=xi, Nx=64, Ny=64, Nz=32,
                   r_cut=20.7, triply=True)
    pos, q = charges(seed, 10000, 10000, 185.0, 185.0, 0.0, 100.0)
    return p, pos, q


def batch_systems(n_sys: int = 64, seed0: int = 1000) -> List[Tuple[SlabParams, np.ndarray, np.ndarray]]:
    """Uneven independent slabs: N log-uniform in [1024, 65536] (even, +-1),
    L in {32,64,128}, H in {16,32,64}, eps_b, eps_t drawn from {0.05,1,20}
    with eps=1 inside; xi=1.5, h=0.25, Nz=H/h+1, cutoff 2.0."""
    out = []
    for s in range(n_sys):
        rng = np.random.default_rng(seed0 + s)
        n = int(round(math.exp(rng.uniform(math.log(1024), math.log(65536)))))
        n -= n % 2
        L = float(rng.choice([32.0, 64.0, 128.0]))
        H = float(rng.choice([16.0, 32.0, 64.0]))
        eb = float(rng.choice([0.05, 1.0, 20.0]))
        et = float(rng.choice([0.05, 1.0, 20.0]))
        nxy = int(round(L / 0.25))
        p = SlabParams(Lx=L, Ly=L, H=H, eps=1.0, eps_b=eb, eps_t=et, xi=1.5,
                       Nx=nxy, Ny=nxy, Nz=int(round(H / 0.25)) + 1, r_cut=2.0)
        pos, q = charges(seed0 + 7919 * (s + 1), n // 2, n // 2, L, L, 0.5, H - 0.5)
        out.append((p, pos, q))
    return out


def perturb(pos: np.ndarray, rng: np.random.Generator, std: float,
            Lx: float, Ly: float, H: float, margin: float = 0.5) -> np.ndarray:
    """Gaussian steps of the given std per axis; wrap in x,y, reflect z into
    [margin, H-margin]. Used as a Brownian-like request stream."""
    p = pos + rng.normal(0.0, std, pos.shape)
    p[:, 0] %= Lx
    p[:, 1] %= Ly
    lo, hi = margin, H - margin
    z = p[:, 2]
    z = np.where(z < lo, 2 * lo - z, z)
    z = np.where(z > hi, 2 * hi - z, z)
    p[:, 2] = np.clip(z, lo, hi)
    return np.ascontiguousarray(p)


def serving_trajectories(n_traj: int = 256, seed0: int = 3000) -> List[Tuple[SlabParams, np.ndarray, np.ndarray]]:
    """Independent Brownian-like trajectories for a serving stream: N
    log-uniform in [512, 262144] (even, +-1), box and permittivities drawn as
    in batch_systems and fixed per trajectory; returns the initial state."""
    out = []
    for t in range(n_traj):
        rng = np.random.default_rng(seed0 + t)
        n = int(round(math.exp(rng.uniform(math.log(512), math.log(262144)))))
        n -= n % 2
        L = float(rng.choice([32.0, 64.0, 128.0]))
        H = float(rng.choice([16.0, 32.0, 64.0]))
        eb = float(rng.choice([0.05, 1.0, 20.0]))
        et = float(rng.choice([0.05, 1.0, 20.0]))
        nxy = int(round(L / 0.25))
        p = SlabParams(Lx=L, Ly=L, H=H, eps=1.0, eps_b=eb, eps_t=et, xi=1.5,
                       Nx=nxy, Ny=nxy, Nz=int(round(H / 0.25)) + 1, r_cut=2.0)
        pos, q = charges(seed0 + 104729 * (t + 1), n // 2, n // 2, L, L, 0.5, H - 0.5)
        out.append((p, pos, q))
    return out


def poisson_arrivals(rate: float, duration: float, n_traj: int, seed: int = 2000) -> Tuple[np.ndarray, np.ndarray]:
    """Arrival times (s) of a Poisson stream of the given rate over
    [0, duration) and the trajectory of each request (uniform)."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration * 1.5) + 64
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, n))])
    t = t[t < duration]
    traj = rng.integers(0, n_traj, len(t))
    return t, traj


NAMED: Dict[str, object] = {
    "small": config_small,
    "jump": config_jump,
    "large": config_large,
}
