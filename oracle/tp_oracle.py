"""TEST INFRASTRUCTURE ONLY -- FP64 CPU oracle of the triply periodic variant.

The paper notes that its method carries over to a box periodic in all three
directions (Sec. 7 and the performance comparison of Sec. 7.4): the far
field of the Ewald split (Sec. 3.2) is then a plain Fourier solve on a
uniform grid, with no images, correction or boundary value problem. Written
here step by step in plain NumPy, with the same Ewald split, kernel S-bar,
near field and self term as the slab oracle:

  1. spread f = sum_k q_k S-bar(g - z_k) on the uniform grid x_i = i h,
     y_j = j h, z_c = c h_z (h_z = Lz/Nz), over x,y index windows as in the
     slab and the z nodes within H_E of the charge in periodic distance;
  2. F(k) = (1/(Nx Ny Nz)) sum f e^{-i k.x} (``numpy.fft.rfftn``);
  3. psi^(k) = F(k) / (eps |k|^2), psi^(0) = 0 (the neutral set's mean);
  4. E^ = -i k psi^ (multipliers 0 on Nyquist indices), inverse transforms;
  5. S-bar averages at the charges with weights h^2 h_z;
  6. near field over pairs with minimal-image distance r < r_cut in all three
     directions; phi-bar = far + near - self term; F = q E-bar; U = 1/2 sum q phi-bar.

Readings: the z period is the ``H`` of the parameters; no gauge constant (the
k = 0 mode is zero); the windows need Lz >= 4 H_E.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import dpse_oracle as O


def derive_tp(p):
    h = p.Lx / p.Nx
    if abs(p.Ly / p.Ny - h) > 1e-12 * h:
        raise ValueError("the x and y grid spacings must be equal")
    g_t = math.sqrt(1.0 / (4.0 * p.xi ** 2) + p.g_w ** 2)
    n_g = p.n_g if p.n_g else 2 * math.ceil(4.3 * g_t / h)
    H_E = n_g * h / 2.0
    if p.H < 4.0 * H_E:
        raise ValueError("the z period must be at least 4 H_E")
    hz = p.H / p.Nz
    xi_e = 1.0 / math.sqrt(4.0 * p.g_w ** 2 + 1.0 / p.xi ** 2)
    return dict(h=h, hz=hz, g_t=g_t, n_g=n_g, H_E=H_E, z=np.arange(p.Nz) * hz, xi_e=xi_e)


def _window(p, d, x, y, z):
    ix, dx = O._xwin(x, d["h"], d["n_g"], p.Nx)
    iy, dy = O._xwin(y, d["h"], d["n_g"], p.Ny)
    dzall = d["z"] - z
    dzall -= p.H * np.round(dzall / p.H)
    iz = np.nonzero(np.abs(dzall) <= d["H_E"])[0]
    dz = dzall[iz]
    r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    return iz, iy, ix, r2


def _wrap(pos, p):
    pos = np.array(pos, dtype=np.float64)
    pos[:, 0] -= p.Lx * np.floor(pos[:, 0] / p.Lx)
    pos[:, 1] -= p.Ly * np.floor(pos[:, 1] / p.Ly)
    pos[:, 2] -= p.H * np.floor(pos[:, 2] / p.H)
    return pos


def _sbar(d, r2):
    g = d["g_t"]
    return (2.0 * math.pi * g * g) ** -1.5 * np.exp(-r2 / (2.0 * g * g))


def wavenumbers(p):
    """k_x [nkx], k_y [Ny], k_z [Nz] of numpy's rfftn layout over (z, y, x),
    and the derivative multipliers with the Nyquist entries set to 0."""
    kx = 2.0 * np.pi * np.fft.rfftfreq(p.Nx, d=1.0 / p.Nx) / p.Lx
    ky = 2.0 * np.pi * np.fft.fftfreq(p.Ny, d=1.0 / p.Ny) / p.Ly
    kz = 2.0 * np.pi * np.fft.fftfreq(p.Nz, d=1.0 / p.Nz) / p.H
    dkx, dky, dkz = kx.copy(), ky.copy(), kz.copy()
    dkx[-1] = 0.0                 # Nyquist of the half spectrum (Nx even)
    dky[p.Ny // 2] = 0.0
    dkz[p.Nz // 2] = 0.0
    return kx, ky, kz, dkx, dky, dkz


def near_tp(p, d, pos, q, targets=None):
    """Near field [n, 4] with the minimal image in x, y and z, no walls
    (only the rows of ``targets`` when given: sampled checks of large sets)."""
    tt = np.arange(len(q)) if targets is None else np.asarray(targets)
    n = len(tt)
    out = np.zeros((n, 4))
    dx = pos[tt, None, 0] - pos[None, :, 0]
    dy = pos[tt, None, 1] - pos[None, :, 1]
    dz = pos[tt, None, 2] - pos[None, :, 2]
    dx -= p.Lx * np.round(dx / p.Lx)
    dy -= p.Ly * np.round(dy / p.Ly)
    dz -= p.H * np.round(dz / p.H)
    r2 = dx * dx + dy * dy + dz * dz
    m = r2 < p.r_cut ** 2
    m[np.arange(n), tt] = False
    ti, sj = np.nonzero(m)
    r = np.sqrt(r2[ti, sj])
    G, e = O.near_kernel(r, p, d["xi_e"])
    np.add.at(out[:, 0], ti, q[sj] * G)
    np.add.at(out[:, 1], ti, q[sj] * e * dx[ti, sj])
    np.add.at(out[:, 2], ti, q[sj] * e * dy[ti, sj])
    np.add.at(out[:, 3], ti, q[sj] * e * dz[ti, sj])
    return out / (O.FOUR_PI * p.eps)


def solve_tp(p, pos, q, near_targets=None):
    """Returns (U, phi, F, intermediates) of the triply periodic solve; with
    ``near_targets`` the near field (and so phi, F) only for those charges
    (U is then not formed)."""
    d = derive_tp(p)
    pos = _wrap(pos, p)
    q = np.asarray(q, dtype=np.float64)
    f = np.zeros((p.Nz, p.Ny, p.Nx))
    for k in range(len(q)):
        iz, iy, ix, r2 = _window(p, d, *pos[k])
        f[np.ix_(iz, iy, ix)] += q[k] * _sbar(d, r2)
    Fk = np.fft.rfftn(f, axes=(0, 1, 2)) / (p.Nx * p.Ny * p.Nz)
    kx, ky, kz, dkx, dky, dkz = wavenumbers(p)
    K2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        psi = np.where(K2 > 0.0, Fk / (p.eps * K2), 0.0)
    fields = [psi, -1j * dkx[None, None, :] * psi, -1j * dky[None, :, None] * psi, -1j * dkz[:, None, None] * psi]
    grids = np.stack([np.fft.irfftn(a * (p.Nx * p.Ny * p.Nz), s=(p.Nz, p.Ny, p.Nx), axes=(0, 1, 2))
                      for a in fields])
    far = np.zeros((len(q), 4))
    w = d["h"] ** 2 * d["hz"]
    for k in range(len(q)):
        iz, iy, ix, r2 = _window(p, d, *pos[k])
        wgt = _sbar(d, r2) * w
        far[k] = np.tensordot(grids[np.ix_(np.arange(4), iz, iy, ix)], wgt, axes=([1, 2, 3], [0, 1, 2]))
    near = near_tp(p, d, pos, q, targets=near_targets)
    tt = np.arange(len(q)) if near_targets is None else np.asarray(near_targets)
    self_c = 2.0 * d["xi_e"] / (O.FOUR_PI * p.eps * O.SQRT_PI)
    phi = far[tt, 0] + near[:, 0] - q[tt] * self_c
    F = q[tt, None] * (far[tt, 1:] + near[:, 1:])
    U = 0.5 * float(np.sum(q * phi)) if near_targets is None else None
    return U, phi, F, dict(f=f, grids=grids, far=far, near=near, derived=d)
