"""Pins of the Brownian-dynamics step reference (Sec. 7, eq. leimkuhler) and
of the far-field reuse reference, against closed forms and the full solve."""
import math

import numpy as np

from oracle import bd
from oracle import dpse_oracle as O
from workloads import SlabParams, charges


def _chain(k_spring, h, kT, n_steps, n_chains, seed, mu=1.0):
    """n_chains independent 1D walkers in the harmonic force -k z, stepped by
    eq. leimkuhler; returns their positions after n_steps."""
    rng = np.random.default_rng(seed)
    x = np.zeros((n_chains, 3))
    w_prev = rng.standard_normal((n_chains, 3))
    for _ in range(n_steps):
        w_next = rng.standard_normal((n_chains, 3))
        x, _ = bd.leimkuhler_step(x, -k_spring * x, w_prev, w_next, mu, h, kT, z_lo=-np.inf)
        w_prev = w_next
    return x


def test_harmonic_stationary_variance_is_exact():
    """For a harmonic force the scheme's stationary variance is kT/k exactly
    for any stable step (the recurrence X' = (1 - h k) X + s (W + W') with
    s^2 = kT h / 2 and Cov(X, W) = s gives V = 2 s^2 / (h k)); plain
    Euler-Maruyama would give kT / (k (1 - h k / 2)), 33 % more at h k = 0.5."""
    kT, k = 0.7, 2.0
    for h in (0.05, 0.25):
        x = _chain(k, h, kT, 400, 20000, seed=int(100 * h))
        v = x.var(axis=0)
        se = kT / k * math.sqrt(2.0 / x.shape[0])        # standard error of a variance
        assert np.all(np.abs(v - kT / k) < 5 * se), (h, v)


def test_free_diffusion_displacement_variance():
    """With no force the n-step displacement is s (W_0 + 2 W_1 + ... + 2 W_{n-1} + W_n):
    variance s^2 (4 n - 2) = 2 kT mu n h - kT mu h, the diffusive 2 D t less one step."""
    kT, mu, h, n = 1.3, 0.8, 0.1, 50
    rng = np.random.default_rng(3)
    m = 40000
    x = np.zeros((m, 3))
    w_prev = rng.standard_normal((m, 3))
    for _ in range(n):
        w_next = rng.standard_normal((m, 3))
        x, _ = bd.leimkuhler_step(x, np.zeros_like(x), w_prev, w_next, mu, h, kT, z_lo=-np.inf)
        w_prev = w_next
    expect = 2 * kT * mu * n * h - kT * mu * h
    se = expect * math.sqrt(2.0 / m)
    assert np.all(np.abs(x.var(axis=0) - expect) < 5 * se)


def test_step_rejects_charges_leaving_the_slab():
    pos = np.array([[1.0, 1.0, 0.05], [2.0, 2.0, 0.5]])
    F = np.zeros_like(pos)
    w = np.zeros_like(pos)
    w2 = w.copy()
    w2[0, 2] = -1.0
    _, bad = bd.leimkuhler_step(pos, F, w, w2, 1.0, 0.01, 1.0, z_lo=0.0, z_hi=1.0)
    assert bad
    _, bad = bd.leimkuhler_step(pos, F, w, w, 1.0, 0.01, 1.0, z_lo=0.0, z_hi=1.0)
    assert not bad


def test_near_reuse_is_the_full_solve_at_the_same_positions():
    """Reusing a full solve's far field at the very positions of that solve
    reproduces its outputs; after a small move the reuse differs from a new
    full solve by the change of the far field only."""
    p = SlabParams(Lx=16.0, Ly=16.0, H=8.0, eps=1.0, eps_b=0.05, eps_t=20.0, xi=1.0, Nx=64, Ny=64, Nz=33,
                   r_cut=3.0)
    pos, q = charges(2, 60, 60, 16.0, 16.0, 0.5, 7.5)
    U, phi, F, I = O.solve(p, pos, q)
    Ur, phir, Fr = bd.near_reuse(p, pos, q, I)
    assert abs(Ur - U) < 1e-12 * abs(U) and np.abs(Fr - F).max() < 1e-12 * np.abs(F).max()
    assert np.abs(phir - phi).max() < 1e-12 * np.abs(phi).max()
    moved = pos + np.random.default_rng(4).normal(0.0, 0.02, pos.shape)
    U2, phi2, F2, I2 = O.solve(p, moved, q)
    Ur2, phir2, Fr2 = bd.near_reuse(p, moved, q, I)
    # the difference is exactly the change of the far field (near parts agree)
    dfar = q[:, None] * (I2["far"][:, 1:] - I["far"][:, 1:])
    assert np.abs((F2 - Fr2) - dfar).max() < 1e-12 * np.abs(F2).max()
    assert 1e-6 < np.sqrt(((F2 - Fr2) ** 2).sum() / (F2 ** 2).sum()) < 5e-2
