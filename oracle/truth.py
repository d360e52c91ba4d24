"""TEST INFRASTRUCTURE ONLY -- independent physical reference for slab electrostatics.

Point charges (g_w = 0) in a box periodic in x,y, permittivity eps for
0 < z < H, eps_b below and eps_t above. Inside the slab the potential equals
that of the charges plus the classical infinite image series (Sec. 4.1
eq. ims, applied at both walls) in a uniform medium eps. Each image family is
summed with the standard two-dimensional Ewald formula (real-space erfc sum,
reciprocal sum with erfc factors in z, and the k = 0 term z erf + Gaussian),
which is exact for any splitting parameter alpha; alpha-independence is itself
a check of this module.

Image families of a charge q at height z0 (gamma_X = (eps - eps_X)/(eps + eps_X)):
  z0 + 2mH   (m != 0)  strength (gamma_b gamma_t)^|m| q
  2mH - z0   (m <= 0)  strength gamma_b^(|m|+1) gamma_t^|m| q
  2mH - z0   (m >= 1)  strength gamma_t^m gamma_b^(m-1) q
Every family of a neutral set is neutral.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special

SQRT_PI = math.sqrt(math.pi)


def image_sources(pos, q, H, eps, eps_b, eps_t, tol=1e-17):
    """Returns (src_pos[M,3], src_q[M], src_orig[M]) where src_orig is the index
    of the generating charge for the original family and -1 for images."""
    gb = (eps - eps_b) / (eps + eps_b)
    gt = (eps - eps_t) / (eps + eps_t)
    P, Q, O = [pos], [q], [np.arange(len(q))]
    g2 = abs(gb * gt)
    if gb == 0.0 and gt == 0.0:
        return pos, q, O[0]
    m_max = 1 if g2 == 0.0 else max(1, int(math.ceil(math.log(tol) / math.log(g2))) + 1)
    x, y, z0 = pos[:, 0], pos[:, 1], pos[:, 2]
    none = -np.ones(len(q), dtype=int)
    for m in range(1, m_max + 1):
        for sgn in (+1, -1):
            s = (gb * gt) ** m
            if s != 0.0:
                P.append(np.stack([x, y, z0 + sgn * 2 * m * H], 1)); Q.append(s * q); O.append(none)
    for m in range(-m_max, m_max + 1):
        if m <= 0:
            s = gb ** (abs(m) + 1) * gt ** abs(m)
        else:
            s = gt ** m * gb ** (m - 1)
        if s != 0.0:
            P.append(np.stack([x, y, 2 * m * H - z0], 1)); Q.append(s * q); O.append(none)
    return np.concatenate(P), np.concatenate(Q), np.concatenate(O)


def _ef(kz, u):
    """e^{kz} erfc(u), overflow-safe."""
    out = np.empty_like(u)
    pos = u > 0
    out[pos] = scipy.special.erfcx(u[pos]) * np.exp(kz[pos] - u[pos] ** 2)
    out[~pos] = np.exp(kz[~pos]) * scipy.special.erfc(u[~pos])
    return out


def ewald2d(Lx, Ly, H, eps, eps_b, eps_t, pos, q, alpha=None, n_real=None, k_cut=None,
            probes=None):
    """Potential phi[N] and field E[N,3] at every charge (its own direct term
    excluded, the self Ewald constant removed, its images included), plus the
    energy U = 1/2 sum q phi. Units: eps Lap phi = -rho.

    With ``probes`` (points in 0 <= z <= H) also returns the pointwise potential
    and field there: (U, phi, E, phi_probe, E_probe)."""
    pos = np.asarray(pos, float)
    q = np.asarray(q, float)
    n_chg = len(q)
    if probes is not None:
        probes = np.asarray(probes, float).reshape(-1, 3)
        tpos = np.concatenate([pos, probes])
    else:
        tpos = pos
    A = Lx * Ly
    if alpha is None:
        alpha = 2.5 / min(Lx, Ly)
    sp, sq, so = image_sources(pos, q, H, eps, eps_b, eps_t)
    rc = 6.2 / alpha
    nr = n_real if n_real is not None else int(math.ceil(rc / min(Lx, Ly))) + 1
    kc = k_cut if k_cut is not None else 2.0 * alpha * 6.2
    mx = int(math.ceil(kc * Lx / (2 * math.pi)))
    my = int(math.ceil(kc * Ly / (2 * math.pi)))
    kv = []
    for i in range(-mx, mx + 1):
        for j in range(-my, my + 1):
            if i == 0 and j == 0:
                continue
            kx, ky = 2 * math.pi * i / Lx, 2 * math.pi * j / Ly
            if math.hypot(kx, ky) <= kc:
                kv.append((kx, ky))
    kv = np.array(kv)
    kn = np.sqrt((kv ** 2).sum(1))
    n = len(tpos)
    phi = np.zeros(n)
    E = np.zeros((n, 3))
    for t in range(n):
        rx = tpos[t, 0] - sp[:, 0]
        ry = tpos[t, 1] - sp[:, 1]
        rz = tpos[t, 2] - sp[:, 2]
        # real space
        for a in range(-nr, nr + 1):
            for b in range(-nr, nr + 1):
                dx = rx + a * Lx
                dy = ry + b * Ly
                r = np.sqrt(dx * dx + dy * dy + rz * rz)
                m = r < rc
                if a == 0 and b == 0:
                    m &= ~(so == t)
                rr = r[m]
                s = sq[m]
                ec = scipy.special.erfc(alpha * rr)
                phi[t] += np.sum(s * ec / rr)
                fac = s * (ec / rr ** 2 + 2 * alpha / SQRT_PI * np.exp(-(alpha * rr) ** 2) / rr) / rr
                E[t, 0] += np.sum(fac * dx[m])
                E[t, 1] += np.sum(fac * dy[m])
                E[t, 2] += np.sum(fac * rz[m])
        # reciprocal space (k != 0): only sources whose terms are not negligible
        near = np.abs(rz) * kn.min() < 60.0
        if np.any(near):
            zz = rz[near][:, None]
            cph = (kv[:, 0][None] * rx[near][:, None] + kv[:, 1][None] * ry[near][:, None])
            k = kn[None]
            u1 = alpha * zz + k / (2 * alpha)
            u2 = -alpha * zz + k / (2 * alpha)
            kz = k * zz
            t1 = _ef(kz, u1)
            t2 = _ef(-kz, u2)
            s = sq[near][:, None]
            phi[t] += (math.pi / A) * np.sum(s * np.cos(cph) / k * (t1 + t2))
            fs = (math.pi / A) * s * np.sin(cph) / k * (t1 + t2)
            E[t, 0] += np.sum(fs * kv[:, 0][None])
            E[t, 1] += np.sum(fs * kv[:, 1][None])
            E[t, 2] += -(math.pi / A) * np.sum(s * np.cos(cph) * (t1 - t2))
        # k = 0 term
        zz = rz
        phi[t] += -(2 * math.pi / A) * np.sum(
            sq * (zz * scipy.special.erf(alpha * zz) + np.exp(-(alpha * zz) ** 2) / (alpha * SQRT_PI)))
        E[t, 2] += (2 * math.pi / A) * np.sum(sq * scipy.special.erf(alpha * zz))
        if t < n_chg:
            phi[t] -= 2 * alpha / SQRT_PI * q[t]
    phi /= 4 * math.pi * eps
    E /= 4 * math.pi * eps
    U = 0.5 * float(np.sum(q * phi[:n_chg]))
    if probes is not None:
        return U, phi[:n_chg], E[:n_chg], phi[n_chg:], E[n_chg:]
    return U, phi, E


def ewald3d(L, pos, q, eps=1.0, alpha=None, n_real=None, k_cut=None):
    """Classical Ewald sum of point charges in a box L = (Lx, Ly, Lz)
    periodic in all three directions, tin-foil boundary (no dipole term):
    real-space erfc(alpha r)/r over images within n_real boxes, reciprocal
    sum exp(-k^2/(4 alpha^2))/k^2 over |n_i| <= k_cut, self term -2 alpha/sqrt(pi).
    Returns (U, phi[N], E[N,3]), each charge's own direct term excluded."""
    L = np.asarray(L, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    n = len(q)
    alpha = alpha or 5.0 / float(L.min())
    n_real = n_real if n_real is not None else 2
    k_cut = k_cut if k_cut is not None else 14
    phi = np.zeros(n)
    E = np.zeros((n, 3))
    rng = range(-n_real, n_real + 1)
    for a in rng:
        for b in rng:
            for c in rng:
                sh = np.array([a, b, c]) * L
                d = pos[:, None, :] - pos[None, :, :] + sh
                r = np.linalg.norm(d, axis=2)
                if a == 0 and b == 0 and c == 0:
                    np.fill_diagonal(r, np.inf)
                er = scipy.special.erfc(alpha * r) / r
                phi += er @ q
                g = (er + 2.0 * alpha / SQRT_PI * np.exp(-(alpha * r) ** 2)) / r ** 2
                E += np.einsum("ij,ijk->ik", g * q[None, :], d)
    V = float(np.prod(L))
    ks = np.arange(-k_cut, k_cut + 1)
    KX, KY, KZ = np.meshgrid(2 * math.pi * ks / L[0], 2 * math.pi * ks / L[1], 2 * math.pi * ks / L[2],
                             indexing="ij")
    K = np.stack([KX.ravel(), KY.ravel(), KZ.ravel()], 1)
    K2 = (K ** 2).sum(1)
    K, K2 = K[K2 > 0], K2[K2 > 0]
    A = 4 * math.pi / V * np.exp(-K2 / (4 * alpha ** 2)) / K2
    phase = pos @ K.T                                   # [N, M]
    S = np.exp(1j * phase).T @ q                        # structure factor, [M]
    phi += np.real(np.exp(-1j * phase) @ (A * S))
    E += np.real((1j * np.exp(-1j * phase) * (A * S)[None, :]) @ K)
    phi -= 2 * alpha / SQRT_PI * q
    phi /= 4 * math.pi * eps
    E /= 4 * math.pi * eps
    return 0.5 * float(np.sum(q * phi)), phi, E
