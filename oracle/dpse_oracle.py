"""TEST INFRASTRUCTURE ONLY -- FP64 CPU oracle of the DP-SE far+near solve.

Plain, slow, direct NumPy code following the paper's algorithm step by step
(Maxian et al., arXiv 2101.07088, Sec. 4-5 and App. A). Library primitives
serve as single steps: ``numpy.fft`` for the x,y Fourier transform,
``scipy.fft.dct`` (type 1) for the Chebyshev transform, ``numpy.linalg.solve``
for the per-mode dense systems, ``numpy.polynomial.chebyshev`` for series
evaluation and differentiation. There is no blocking or fusion: each stage
returns a full array, and every intermediate is kept for per-stage parity.

Readings of points the paper leaves open (the HIP path takes the same ones):
  * point charges: g_w may be 0; the self potential is removed as in Sec. 6.3;
  * support n_g = 2*ceil(4.3*g_t/h) unless given (Sec. 5.1 uses n_sigma ~ 4.2-4.3);
  * z grid: Gauss-Lobatto Chebyshev nodes z_j = c + R cos(pi j/(Nz-1)) on
    [-3H_E, H+3H_E] (Sec. 5.2.2), coefficients without a halved first term (App. A);
  * truncation: x,y windows are the n_g grid indices floor(x/h)-n_g/2+1 ..
    floor(x/h)+n_g/2; z nodes with |z_c - z| <= H_E are kept (Sec. 5.1);
  * interpolation quadrature: h^2 times Clenshaw-Curtis weights;
  * z derivative: exact derivative of the degree Nz-1 Chebyshev series;
  * Nyquist modes: derivative multipliers are 0 there, the potential keeps them;
  * correction cap: modes with |k| <= pi/h (integer test), optionally also
    |k| <= 4.2/g_t; correction evaluated at nodes with -H_E <= z_c <= H+H_E;
  * groups: C_o = {z < 2H_E or z > H-2H_E} (strict); bottom image for
    z < 2H_E, top image for z > H-2H_E; zero-strength images skipped;
  * near field: strict r < r_cut, minimal image in x,y, one image per wall for
    every charge (its own included);
  * A_i(0) is the mean of its two formulas; gauge constant added to phi directly;
  * one dielectric jump (``one_jump``): every charge is imaged across that
    wall and the free-space solve of the uniform case runs on the span of
    charges and images, [-H - H_E, H + H_E] or [-H_E, 2H + H_E];
  * wall charges: sigma_b, sigma_t are given by their values at the x,y grid
    points and enter only the correction (eqs. mm2, mm4) and A_i (eqs. ai1,
    ai2); the wall integral of eq. Ufinal is taken by reciprocity: with
    phi_s the potential of the walls alone (the correction with m_phi = 0 and
    m_E = +sigma_b, -sigma_t, plus its k = 0 slope) and B_i the gauge constant,
    int sigma phi = sum_k q_k phi_s(z_k) + int sigma phi_s + B_i int sigma,
    where phi_s(z_k) is the S-bar average of phi_s on the grid (phi_s is
    harmonic, so the average is the point value) and int sigma phi_s is the
    trapezoid sum over the wall grid points. ``wall_energy_literal`` takes the
    integral as written instead (pins only).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np
import scipy.fft
import scipy.special
from numpy.polynomial import chebyshev as npcheb

FOUR_PI = 4.0 * math.pi
SQRT_PI = math.sqrt(math.pi)


# ---------------------------------------------------------------------------
# Derived quantities (Sec. 3.2 eq. gt; Sec. 5.1 eq. He; Sec. 5.2.2 domain)
# ---------------------------------------------------------------------------

def cc_weights(n: int) -> np.ndarray:
    """Clenshaw-Curtis weights on [-1,1] for the nodes s_j = cos(pi j/(n-1)).

    Defined by exactness on T_0..T_{n-1}: sum_j w_j T_m(s_j) = int_{-1}^{1} T_m,
    which is 2/(1-m^2) for even m and 0 for odd m. Solved directly.
    """
    j = np.arange(n)
    m = np.arange(n)
    T = np.cos(np.pi * np.outer(m, j) / (n - 1))  # T[m, j] = T_m(s_j)
    mom = np.zeros(n)
    even = (m % 2 == 0)
    mom[even] = 2.0 / (1.0 - m[even].astype(float) ** 2)
    return np.linalg.solve(T, mom)


def derive(p) -> Dict[str, object]:
    """All plan quantities of one system, from the paper's definitions."""
    h = p.Lx / p.Nx
    hy = p.Ly / p.Ny
    if abs(hy - h) > 1e-12 * h:
        raise ValueError("the x and y grid spacings must be equal (Sec. 5.1)")
    g_t = math.sqrt(1.0 / (4.0 * p.xi ** 2) + p.g_w ** 2)          # eq. gt
    n_g = p.n_g if p.n_g else 2 * math.ceil(4.3 * g_t / h)
    H_E = n_g * h / 2.0                                             # eq. He
    uniform = getattr(p, "uniform_fast", False)
    one = getattr(p, "one_jump", False)
    if uniform and one:
        raise ValueError("the uniform and the one-jump solvers exclude each other")
    if uniform and not (p.eps_b == p.eps == p.eps_t):
        raise ValueError("the uniform-permittivity solver needs eps_b == eps == eps_t")
    jump_b, jump_t = p.eps_b != p.eps, p.eps_t != p.eps
    if one and jump_b == jump_t:
        raise ValueError("the one-jump solver needs a jump at exactly one wall")
    # free-space solve of Sec. 3.1.1 (no wall group, no correction) for no
    # jump, and for one jump after imaging every charge across that wall
    # (Sec. 4, opening; Sec. 1): the sources (Gaussians of support H_E) and
    # images fill [-H_E, H + H_E], [-H - H_E, H + H_E] (bottom jump) or
    # [-H_E, 2H + H_E] (top jump); with two jumps the domain is
    # [-3 H_E, H + 3 H_E] (Sec. 5.2.2)
    fast = uniform or one
    one_side = ("b" if jump_b else "t") if one else None
    if uniform:
        a, b = -H_E, p.H + H_E
    elif one_side == "b":
        a, b = -p.H - H_E, p.H + H_E
    elif one_side == "t":
        a, b = -H_E, 2.0 * p.H + H_E
    else:
        a, b = -3.0 * H_E, p.H + 3.0 * H_E
    c = 0.5 * (a + b)
    R = 0.5 * (b - a)
    N = p.Nz
    s = np.cos(np.pi * np.arange(N) / (N - 1))
    z = c + R * s
    w = R * cc_weights(N)
    gamma_b = (p.eps - p.eps_b) / (p.eps + p.eps_b)   # image strength ratio, eq. ims
    gamma_t = (p.eps - p.eps_t) / (p.eps + p.eps_t)
    tau_b = 2.0 * p.eps / (p.eps_b + p.eps)            # eq. phibst
    tau_t = 2.0 * p.eps / (p.eps_t + p.eps)            # eq. phitst
    xi_e = 1.0 / math.sqrt(4.0 * p.g_w ** 2 + 1.0 / p.xi ** 2)
    # wave numbers, n in [-N/2, N/2): rfft column Nx/2 is n_x = -Nx/2
    nkx = p.Nx // 2 + 1
    nx = np.arange(nkx)
    nx[-1] = -(p.Nx // 2)
    ny = np.fft.fftfreq(p.Ny, d=1.0 / p.Ny).astype(int)
    ny[p.Ny // 2] = -(p.Ny // 2)
    kx = 2.0 * np.pi * nx / p.Lx
    ky = 2.0 * np.pi * ny / p.Ly
    KX, KY = np.meshgrid(kx, ky)          # [Ny, nkx]
    NXI, NYI = np.meshgrid(nx, ny)
    kabs = np.sqrt(KX ** 2 + KY ** 2)
    # correction cap k <= pi/h as an integer test (Sec. 5.2.2 step 4)
    keep = 4 * (NXI.astype(np.int64) ** 2 * p.Ny ** 2 + NYI.astype(np.int64) ** 2 * p.Nx ** 2) \
        <= (p.Nx * p.Ny) ** 2
    if p.kmax_gt:
        keep &= kabs <= 4.2 / g_t
    # derivative multipliers vanish on Nyquist indices
    dkx = np.where(NXI == -(p.Nx // 2), 0.0, KX)
    dky = np.where(NYI == -(p.Ny // 2), 0.0, KY)
    return dict(h=h, g_t=g_t, n_g=n_g, H_E=H_E, a=a, b=b, c=c, R=R, s=s, z=z, fast=fast, one_side=one_side,
                w=w, gamma_b=gamma_b, gamma_t=gamma_t, tau_b=tau_b, tau_t=tau_t,
                xi_e=xi_e, kx=KX, ky=KY, kabs=kabs, keep=keep, dkx=dkx, dky=dky)


# ---------------------------------------------------------------------------
# Groups and images (Sec. 4.1 eq. ims; Sec. 5.2.2 step 1)
# ---------------------------------------------------------------------------

def groups_and_images(p, d, pos, q):
    z = pos[:, 2]
    H_E = d["H_E"]
    low = z < 2.0 * H_E
    high = z > p.H - 2.0 * H_E
    if d["fast"]:  # no walls to correct for: one group
        low = np.zeros_like(low)
        high = np.zeros_like(high)
    c_o = low | high
    img_b, img_t = low, high
    if d["one_side"] is not None:  # one jump: every charge imaged across that wall
        img_b = np.full_like(low, d["one_side"] == "b")
        img_t = np.full_like(high, d["one_side"] == "t")
    ipos, iq = [], []
    if d["gamma_b"] != 0.0:
        sel = np.nonzero(img_b)[0]
        ipos.append(np.stack([pos[sel, 0], pos[sel, 1], -z[sel]], axis=1))
        iq.append(d["gamma_b"] * q[sel])
    if d["gamma_t"] != 0.0:
        sel = np.nonzero(img_t)[0]
        ipos.append(np.stack([pos[sel, 0], pos[sel, 1], 2.0 * p.H - z[sel]], axis=1))
        iq.append(d["gamma_t"] * q[sel])
    if ipos:
        ipos = np.concatenate(ipos, axis=0)
        iq = np.concatenate(iq)
    else:
        ipos = np.zeros((0, 3))
        iq = np.zeros(0)
    return c_o, ipos, iq


# ---------------------------------------------------------------------------
# Spreading and interpolation with the truncated Gaussian S-bar
# (Sec. 3.2 eq. spreadkernelEw; Sec. 5.1 truncation; Sec. 5.2.2 steps 2,3,7)
# ---------------------------------------------------------------------------

def _xwin(x, h, n_g, n):
    i0 = math.floor(x / h)
    idx = i0 + np.arange(-n_g // 2 + 1, n_g // 2 + 1)
    return idx % n, idx * h - x


def _windows(p, d, x, y, zc):
    ix, dx = _xwin(x, d["h"], d["n_g"], p.Nx)
    iy, dy = _xwin(y, d["h"], d["n_g"], p.Ny)
    iz = np.nonzero(np.abs(d["z"] - zc) <= d["H_E"])[0]
    dz = d["z"][iz] - zc
    r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    return iz, iy, ix, r2


def sbar(d, r2):
    g = d["g_t"]
    return (2.0 * math.pi * g * g) ** -1.5 * np.exp(-r2 / (2.0 * g * g))


def spread(p, d, pos, q) -> np.ndarray:
    """f(x_i, y_j, z_c) = sum_k q_k S-bar(grid point - z_k), truncated."""
    f = np.zeros((p.Nz, p.Ny, p.Nx))
    for k in range(len(q)):
        iz, iy, ix, r2 = _windows(p, d, pos[k, 0], pos[k, 1], pos[k, 2])
        f[np.ix_(iz, iy, ix)] += q[k] * sbar(d, r2)
    return f


def interp(p, d, fields, pos, kernel_r2=None) -> np.ndarray:
    """Averages sum_window h^2 w_c S-bar(g - z_k) u(g) of each field u.

    fields: array [nf, Nz, Ny, Nx]. Returns [n, nf]."""
    nf = fields.shape[0]
    out = np.zeros((len(pos), nf))
    hh = d["h"] ** 2
    for k in range(len(pos)):
        iz, iy, ix, r2 = _windows(p, d, pos[k, 0], pos[k, 1], pos[k, 2])
        wgt = (kernel_r2 or (lambda rr: sbar(d, rr)))(r2) * (hh * d["w"][iz])[:, None, None]
        blk = fields[np.ix_(np.arange(nf), iz, iy, ix)]
        out[k] = np.tensordot(blk, wgt, axes=([1, 2, 3], [0, 1, 2]))
    return out


# ---------------------------------------------------------------------------
# Fourier-Chebyshev transforms (Sec. 5.2.1 steps 2 and 5; App. A)
# ---------------------------------------------------------------------------

def fft_xy(f, p):
    """F(k, z_c) = (1/(Nx Ny)) sum_ij f e^{-i(kx x_i + ky y_j)}; half spectrum in x."""
    return np.fft.rfft2(f, axes=(1, 2)) / (p.Nx * p.Ny)


def ifft_xy(F, p):
    """u(x_i, y_j) = sum_k F e^{+i k.x} (the inverse of fft_xy)."""
    return np.fft.irfft2(F * (p.Nx * p.Ny), s=(p.Ny, p.Nx), axes=(1, 2))


def cheb_coeffs(V):
    """Chebyshev coefficients along axis 0 of values at the Gauss-Lobatto nodes:
    V(s_j) = sum_n c_n T_n(s_j), no halving of c_0 (App. A)."""
    n = V.shape[0]
    def dct(x):
        return scipy.fft.dct(x, type=1, axis=0)
    if np.iscomplexobj(V):
        y = dct(V.real) + 1j * dct(V.imag)
    else:
        y = dct(V)
    y = y / (n - 1)
    y[0] *= 0.5
    y[-1] *= 0.5
    return y


def cheb_eval_nodes(C, n_nodes):
    """Values sum_n C_n T_n(s_j) at the Gauss-Lobatto nodes, by direct sums."""
    n = C.shape[0]
    T = np.cos(np.pi * np.outer(np.arange(n_nodes), np.arange(n)) / (n_nodes - 1))
    return np.tensordot(T, C, axes=([1], [0]))


# ---------------------------------------------------------------------------
# Per-mode Chebyshev BVP: Greengard's integral formulation (App. A)
# ---------------------------------------------------------------------------

def bvp_operators(N):
    """Linear maps from u = (y''_0..y''_{N-1}, y_0, y'_0) to the coefficients
    y'_0..y'_{N-1} (eq. ds) and y_0..y_{N-1} (eq. cs), with y''_n = 0 for n>N-1
    and y'_N = 0 when forming y_{N-1} (App. A truncation)."""
    nu = N + 2
    P = np.zeros((N, nu))      # y'_n
    P[0, N + 1] = 1.0
    P[1, 0] = 1.0
    if N > 2:
        P[1, 2] = -0.5
    for n in range(2, N):
        P[n, n - 1] = 1.0 / (2 * n)
        if n + 1 <= N - 1:
            P[n, n + 1] = -1.0 / (2 * n)
    Y = np.zeros((N, nu))      # y_n
    Y[0, N] = 1.0
    Y[1] = P[0] - (0.5 * P[2] if N > 2 else 0.0)
    for n in range(2, N):
        nxt = P[n + 1] if n + 1 <= N - 1 else 0.0
        Y[n] = (P[n - 1] - nxt) / (2 * n)
    return P, Y


def bvp_matrix(N, kappa, dirichlet, ops=None):
    """Dense (N+2)x(N+2) system: mode equations y''_n - kappa^2 y_n = g_n
    (eq. modes/BVPH), then the top and bottom boundary rows: Robin
    sum(y'_n + kappa y_n) = 0, sum (-1)^n (y'_n - kappa y_n) = 0 (eq. BCs) for
    k != 0, homogeneous Dirichlet sum y_n = 0, sum (-1)^n y_n = 0 (eq. BCs0)."""
    P, Y = ops if ops is not None else bvp_operators(N)
    M = np.zeros((N + 2, N + 2))
    M[:N, :N] = np.eye(N)
    M[:N] -= kappa ** 2 * Y
    sgn = (-1.0) ** np.arange(N)
    if dirichlet:
        M[N] = Y.sum(axis=0)
        M[N + 1] = (sgn[:, None] * Y).sum(axis=0)
    else:
        M[N] = (P + kappa * Y).sum(axis=0)
        M[N + 1] = (sgn[:, None] * (P - kappa * Y)).sum(axis=0)
    return M


def solve_modes(p, d, fhat_list, chunk=512):
    """Solve eps*(psi'' - k^2 psi) = -f for every mode and every RHS in
    fhat_list (arrays [Nz, Ny, nkx] of Chebyshev coefficients).

    In s = (z-c)/R: y'' - (kR)^2 y = -R^2 f/eps, Robin BCs for k != 0 and
    homogeneous Dirichlet at z = a, b for k = 0 (Sec. 5.2.2 steps 2-3).
    Returns the solution coefficient arrays, same shapes."""
    N = p.Nz
    R = d["R"]
    ops = bvp_operators(N)
    kap = (d["kabs"] * R).ravel()
    nm = kap.size
    rhs = [(-R * R / p.eps) * fh.reshape(N, nm) for fh in fhat_list]
    outs = [np.zeros((N, nm), dtype=complex) for _ in fhat_list]
    P, Y = ops
    for s0 in range(0, nm, chunk):
        sl = slice(s0, min(nm, s0 + chunk))
        Ms = np.stack([bvp_matrix(N, kk, kk == 0.0, ops) for kk in kap[sl]])
        cols = []
        for r in rhs:
            cols.append(r[:, sl].real.T)
            cols.append(r[:, sl].imag.T)
        B = np.zeros((Ms.shape[0], N + 2, len(cols)))
        for ci, col in enumerate(cols):
            B[:, :N, ci] = col
        U = np.linalg.solve(Ms, B)                 # [m, N+2, ncols]
        yc = np.einsum("nu,muc->mnc", Y, U)        # coefficients y_n
        for ri in range(len(rhs)):
            outs[ri][:, sl] = (yc[:, :, 2 * ri] + 1j * yc[:, :, 2 * ri + 1]).T
    return [o.reshape(N, p.Ny, -1) for o in outs]


def series_at(Cf, s):
    """Value of sum_n C_n T_n(s) for every mode (C: [N, ...])."""
    return npcheb.chebval(s, Cf)


def series_dz_at(Cf, s, R):
    """z-derivative of the series at s: (1/R) d/ds sum_n C_n T_n(s)."""
    return npcheb.chebval(s, npcheb.chebder(Cf, axis=0)) / R


# ---------------------------------------------------------------------------
# Harmonic correction (Sec. 3.1.2 eqs. harmeq, harmbc1-4; Sec. 4.3.3 eqs. mm1-mm4)
# ---------------------------------------------------------------------------

def correction_coeffs(p, k, mphi_b, mE_b, mphi_t, mE_t):
    """Solve the four jump conditions for psi_c = A e^{kz} + B e^{-kz} (slab),
    A_b e^{kz} (below), B_t e^{-kz} (above), per mode with k > 0.

    Unknowns are scaled as (alpha, beta, a_b, b_t) = (A e^{kH}, B, A_b, B_t e^{-kH})
    so no entry exceeds 1 in magnitude; the interior correction is then
    alpha e^{k(z-H)} + beta e^{-kz}. Returns complex (alpha, beta)."""
    E = np.exp(-k * p.H)
    one = np.ones_like(k)
    zero = np.zeros_like(k)
    # rows: harmbc1, harmbc2, harmbc3, harmbc4; columns: alpha, beta, a_b, b_t
    M = np.stack([
        np.stack([E, one, -one, zero], axis=-1),
        np.stack([p.eps * k * E, -p.eps * k, -p.eps_b * k, zero], axis=-1),
        np.stack([one, E, zero, -one], axis=-1),
        np.stack([p.eps * k, -p.eps * k * E, zero, p.eps_t * k], axis=-1),
    ], axis=-2)
    rhs = -np.stack([mphi_b, mE_b, mphi_t, mE_t], axis=-1)
    B = np.concatenate([rhs.real[..., None], rhs.imag[..., None]], axis=-1)
    X = np.linalg.solve(M, B)
    sol = X[..., 0] + 1j * X[..., 1]
    return sol[..., 0], sol[..., 1], M, sol


# ---------------------------------------------------------------------------
# Near field (Sec. 3.2 eqs. GnearK, EnearK; Sec. 4.2; Sec. 5.2.2)
# ---------------------------------------------------------------------------

def near_kernel(r, p, xi_e):
    """Averaged near-field potential kernel G-bar(r) (without 1/(4 pi eps)) and
    the radial factor e(r) with field = q e(r) r_vec: e = -(dG/dr)/r."""
    if p.g_w > 0.0:
        a1 = 1.0 / (2.0 * p.g_w)
        G = (scipy.special.erf(a1 * r) - scipy.special.erf(xi_e * r)) / r
        dG = (2.0 / SQRT_PI) * (a1 * np.exp(-(a1 * r) ** 2) - xi_e * np.exp(-(xi_e * r) ** 2)) / r - G / r
        small = r < 1e-3 * p.g_w
        if np.any(small):
            rs = r[small]
            # Taylor series of [erf(a r) - erf(b r)]/r at r = 0
            c0 = (2.0 / SQRT_PI) * (a1 - xi_e)
            c2 = -(2.0 / SQRT_PI) * (a1 ** 3 - xi_e ** 3) / 3.0
            c4 = (2.0 / SQRT_PI) * (a1 ** 5 - xi_e ** 5) / 10.0
            G[small] = c0 + c2 * rs ** 2 + c4 * rs ** 4
            dG[small] = 2 * c2 * rs + 4 * c4 * rs ** 3
    else:
        G = scipy.special.erfc(xi_e * r) / r
        dG = -(2.0 / SQRT_PI) * xi_e * np.exp(-(xi_e * r) ** 2) / r - G / r
    return G, -dG / r


def near_field(p, d, pos, q, chunk=1024, rows=None, targets=None):
    """For each charge k: sum over charges j != k and over the bottom/top
    images of all j (strengths gamma_b q_j, gamma_t q_j, at (x,y,-z) and
    (x,y,2H-z)) with minimal-image distance r < r_cut. Returns [n, 4].
    ``rows`` (a slice step) restricts the targets to every rows-th chunk of
    ``chunk`` charges (the others stay 0); used only to time a sample.
    ``targets`` (an index array) computes only those charges and returns
    [len(targets), 4] (sampled checks of large systems)."""
    if targets is not None:
        targets = np.asarray(targets)
        out = np.zeros((len(targets), 4))
        for t0 in range(0, len(targets), 32):
            tt = targets[t0:t0 + 32]
            out[t0:t0 + 32] = _near_targets(p, d, pos, q, tt)
        return out / (FOUR_PI * p.eps)
    n = len(q)
    out = np.zeros((n, 4))
    srcs = [(pos, q, True)]
    if d["gamma_b"] != 0.0:
        srcs.append((np.stack([pos[:, 0], pos[:, 1], -pos[:, 2]], 1), d["gamma_b"] * q, False))
    if d["gamma_t"] != 0.0:
        srcs.append((np.stack([pos[:, 0], pos[:, 1], 2 * p.H - pos[:, 2]], 1), d["gamma_t"] * q, False))
    for t0 in range(0, n, chunk * (rows or 1)):
        ts = slice(t0, min(n, t0 + chunk))
        tp = pos[ts]
        for sp, sq, exclude_self in srcs:
            dx = tp[:, None, 0] - sp[None, :, 0]
            dy = tp[:, None, 1] - sp[None, :, 1]
            dz = tp[:, None, 2] - sp[None, :, 2]
            dx -= p.Lx * np.round(dx / p.Lx)
            dy -= p.Ly * np.round(dy / p.Ly)
            r2 = dx * dx + dy * dy + dz * dz
            m = r2 < p.r_cut ** 2
            if exclude_self:
                ii = np.arange(ts.start, ts.stop)
                m[ii - t0, ii] = False
            ti, sj = np.nonzero(m)
            r = np.sqrt(r2[ti, sj])
            G, e = near_kernel(r, p, d["xi_e"])
            qs = sq[sj]
            np.add.at(out[:, 0], ti + t0, qs * G)
            np.add.at(out[:, 1], ti + t0, qs * e * dx[ti, sj])
            np.add.at(out[:, 2], ti + t0, qs * e * dy[ti, sj])
            np.add.at(out[:, 3], ti + t0, qs * e * dz[ti, sj])
    return out / (FOUR_PI * p.eps)


def _near_targets(p, d, pos, q, tt):
    """Unscaled near sums (times 4 pi eps) for the charges with indices tt."""
    out = np.zeros((len(tt), 4))
    srcs = [(pos, q, True)]
    if d["gamma_b"] != 0.0:
        srcs.append((np.stack([pos[:, 0], pos[:, 1], -pos[:, 2]], 1), d["gamma_b"] * q, False))
    if d["gamma_t"] != 0.0:
        srcs.append((np.stack([pos[:, 0], pos[:, 1], 2 * p.H - pos[:, 2]], 1), d["gamma_t"] * q, False))
    tp = pos[tt]
    for sp, sq, exclude_self in srcs:
        dx = tp[:, None, 0] - sp[None, :, 0]
        dy = tp[:, None, 1] - sp[None, :, 1]
        dz = tp[:, None, 2] - sp[None, :, 2]
        dx -= p.Lx * np.round(dx / p.Lx)
        dy -= p.Ly * np.round(dy / p.Ly)
        r2 = dx * dx + dy * dy + dz * dz
        m = r2 < p.r_cut ** 2
        if exclude_self:
            m[np.arange(len(tt)), tt] = False
        ti, sj = np.nonzero(m)
        r = np.sqrt(r2[ti, sj])
        G, e = near_kernel(r, p, d["xi_e"])
        qs = sq[sj]
        np.add.at(out[:, 0], ti, qs * G)
        np.add.at(out[:, 1], ti, qs * e * dx[ti, sj])
        np.add.at(out[:, 2], ti, qs * e * dy[ti, sj])
        np.add.at(out[:, 3], ti, qs * e * dz[ti, sj])
    return out


def near_at_points(p, d, pos, q, pts):
    """Pointwise near-field potential at the points pts [m, 3] (Sec. 5.2.2,
    gauge paragraph): kernel G^(n)(r; g_w, xi) of eq. Gnear over the charges
    and their first images, truncated at r_cut, minimal image in x, y."""
    xi_p = 1.0 / math.sqrt(2.0 * p.g_w ** 2 + 1.0 / p.xi ** 2)
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    tot = np.zeros(len(pts))
    srcs = [(pos[:, 2], q)]
    if d["gamma_b"] != 0.0:
        srcs.append((-pos[:, 2], d["gamma_b"] * q))
    if d["gamma_t"] != 0.0:
        srcs.append((2 * p.H - pos[:, 2], d["gamma_t"] * q))
    dx = pts[:, None, 0] - pos[None, :, 0]
    dy = pts[:, None, 1] - pos[None, :, 1]
    dx -= p.Lx * np.round(dx / p.Lx)
    dy -= p.Ly * np.round(dy / p.Ly)
    for zs, qs in srcs:
        dz = pts[:, None, 2] - zs[None, :]
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        ti, sj = np.nonzero(r < p.r_cut)
        rr = r[ti, sj]
        if p.g_w > 0.0:
            G = (scipy.special.erf(rr / (math.sqrt(2.0) * p.g_w)) - scipy.special.erf(xi_p * rr)) / rr
        else:
            G = scipy.special.erfc(xi_p * rr) / rr
        np.add.at(tot, ti, qs[sj] * G)
    return tot / (FOUR_PI * p.eps)


def near_at_origin(p, d, pos, q):
    """Pointwise near-field potential at x = 0 (the gauge point)."""
    return float(near_at_points(p, d, pos, q, np.zeros((1, 3)))[0])


def gamma_half(p, r2):
    """The kernel gamma^{1/2} of eq. lapsplit (std 1/(2 xi)): averaging the
    far-field grid with it gives the pointwise far-field potential."""
    xi = p.xi
    return (8.0 * xi ** 3 / (2.0 * math.pi) ** 1.5) * np.exp(-2.0 * xi * xi * r2)


# ---------------------------------------------------------------------------
# Wall charges (Sec. 2 eqs. rho, cbc2, cbc4; Sec. 4.3.3 eqs. mm2, mm4;
# Sec. 4.3.4 eqs. ai1, ai2; eq. Ufinal)
# ---------------------------------------------------------------------------

def wall_densities(p, sigma_b, sigma_t):
    """The wall densities at the x,y grid points [Ny, Nx] (None: no charge)
    and their Fourier coefficients with the normalisation of fft_xy."""
    sb = np.zeros((p.Ny, p.Nx)) if sigma_b is None else np.asarray(sigma_b, dtype=np.float64)
    st = np.zeros((p.Ny, p.Nx)) if sigma_t is None else np.asarray(sigma_t, dtype=np.float64)
    if sb.shape != (p.Ny, p.Nx) or st.shape != (p.Ny, p.Nx):
        raise ValueError("wall densities are sampled on the Ny x Nx grid points")
    return sb, st, np.fft.rfft2(sb) / (p.Nx * p.Ny), np.fft.rfft2(st) / (p.Nx * p.Ny)


def wall_energy_literal(p, pos, q, phi, sigma_b, sigma_t, inter):
    """U of eq. Ufinal with the wall integrals as written: the pointwise
    potential at every wall grid point is the gamma^{1/2} average of the
    far-field grid, plus the pointwise near field of the charges and their
    images, plus B_i; the integrals are trapezoid sums h^2 sum sigma phi."""
    d = inter["derived"]
    sb, st, _, _ = wall_densities(p, sigma_b, sigma_t)
    X, Y = np.meshgrid(np.arange(p.Nx) * d["h"], np.arange(p.Ny) * d["h"])
    wall = 0.0
    for zw, sig in ((0.0, sb), (p.H, st)):
        pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, zw)], axis=1)
        far = interp(p, d, inter["grids"][:1], pts, kernel_r2=lambda rr: gamma_half(p, rr))[:, 0]
        near = near_at_points(p, d, pos, q, pts)
        wall += d["h"] ** 2 * float(np.sum(sig.ravel() * (far + near + inter["B_i"])))
    return 0.5 * float(np.sum(q * phi)) + 0.5 * wall


# ---------------------------------------------------------------------------
# The whole solve (Sec. 5.2.2 steps 1-7, field paragraph, gauge paragraph)
# ---------------------------------------------------------------------------

def solve(p, pos, q, timings=None, near_rows=None, sigma_b=None, sigma_t=None
          ) -> Tuple[float, np.ndarray, np.ndarray, Dict[str, np.ndarray]]:
    """The whole solve. ``timings`` (a dict) receives wall seconds of the far
    and near parts; ``near_rows`` is passed to near_field (timing samples only);
    ``sigma_b``, ``sigma_t`` are wall charge densities at the x,y grid points."""
    import time
    t_start = time.perf_counter()
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    d = derive(p)
    walls = sigma_b is not None or sigma_t is not None
    if walls and d["fast"]:
        raise ValueError("wall charges need the correction solve; the uniform-permittivity solver has none")
    sb, st, sbh, sth = wall_densities(p, sigma_b, sigma_t)
    N = p.Nz
    R = d["R"]
    # step 1: groups and images
    c_o, ipos, iq = groups_and_images(p, d, pos, q)
    # steps 2-3: spread C_o alone, and all charges plus the images
    f_o = spread(p, d, pos[c_o], q[c_o])
    f_i = spread(p, d, np.concatenate([pos, ipos]), np.concatenate([q, iq]))
    # forward Fourier-Chebyshev transforms
    F_o = fft_xy(f_o, p)
    F_i = fft_xy(f_i, p)
    fh_o = cheb_coeffs(F_o)
    fh_i = cheb_coeffs(F_i)
    # per-mode BVPs for psi_o* and psi_i*
    y_o, y_i = solve_modes(p, d, [fh_o, fh_i])
    s0 = (0.0 - d["c"]) / R
    sH = (p.H - d["c"]) / R
    v_o0, v_oH = series_at(y_o, s0), series_at(y_o, sH)
    d_o0, d_oH = series_dz_at(y_o, s0, R), series_dz_at(y_o, sH, R)
    v_i0, v_iH = series_at(y_i, s0), series_at(y_i, sH)
    d_i0, d_iH = series_dz_at(y_i, s0, R), series_dz_at(y_i, sH, R)
    # step 4: mismatches (eqs. mm1-mm4 with psi_b* = tau_b psi_o*, psi_t* = tau_t psi_o*)
    tb, tt = d["tau_b"], d["tau_t"]
    mphi_b = v_i0 - tb * v_o0
    mE_b = p.eps * d_i0 - p.eps_b * tb * d_o0 + sbh     # eq. mm2
    mphi_t = v_iH - tt * v_oH
    mE_t = p.eps * d_iH - p.eps_t * tt * d_oH - sth     # eq. mm4
    kabs = d["kabs"]
    act = d["keep"] & (kabs > 0.0)
    alpha = np.zeros_like(v_i0)
    beta = np.zeros_like(v_i0)
    if np.any(act):
        al, be, _, _ = correction_coeffs(p, kabs[act], mphi_b[act], mE_b[act],
                                         mphi_t[act], mE_t[act])
        alpha[act] = al
        beta[act] = be
    z = d["z"]
    win = (z >= -d["H_E"]) & (z <= p.H + d["H_E"])
    kk = kabs[None]
    zz = z[:, None, None]
    with np.errstate(over="ignore", invalid="ignore"):
        e1 = np.where(win[:, None, None], np.exp(kk * (zz - p.H)), 0.0)
        e2 = np.where(win[:, None, None], np.exp(-kk * zz), 0.0)
    psi_c = alpha[None] * e1 + beta[None] * e2
    dpsi_c = kk * (alpha[None] * e1 - beta[None] * e2)
    psi_c[:, ~act] = 0.0
    dpsi_c[:, ~act] = 0.0
    if d["fast"]:
        # no jumps: the Robin BVPs on [-H_E, H + H_E] are the free-space
        # solutions (Sec. 3.1.1), there is nothing to correct; at k = 0 the
        # field of the neutral set vanishes outside the sources, so the slope
        # A_i cancels psi_i*' at both ends of the domain (mean of the two)
        alpha[:] = 0.0
        beta[:] = 0.0
        psi_c[:] = 0.0
        dpsi_c[:] = 0.0
        A_i1 = -series_dz_at(y_i[:, 0, 0], -1.0, R)
        A_i2 = -series_dz_at(y_i[:, 0, 0], 1.0, R)
        A_i = 0.5 * (A_i1 + A_i2)
    else:
        # step 5: k = 0 linear mode (eqs. CE, ai1, ai2; mean of the two)
        dk0_oa = series_dz_at(y_o[:, 0, 0], -1.0, R)
        dk0_ob = series_dz_at(y_o[:, 0, 0], 1.0, R)
        A_b = -tb * dk0_oa
        A_t = -tt * dk0_ob
        A_i1 = (p.eps_b * (tb * d_o0[0, 0] + A_b) - p.eps * d_i0[0, 0] - sbh[0, 0].real) / p.eps
        A_i2 = (p.eps_t * (tt * d_oH[0, 0] + A_t) - p.eps * d_iH[0, 0] + sth[0, 0].real) / p.eps
        A_i = 0.5 * (A_i1 + A_i2)
    # step 6: potential and z-derivative at the nodes (series plus correction)
    Psi = cheb_eval_nodes(y_i, N) + psi_c
    Psi_z = cheb_eval_nodes(npcheb.chebder(y_i, axis=0), N) / R + dpsi_c
    Psi[:, 0, 0] += A_i.real * z
    Psi_z[:, 0, 0] += A_i.real
    # fields: E = -grad psi (Sec. 5.2.1 step 4; field paragraph of Sec. 5.2.2)
    Ex_h = -1j * d["dkx"][None] * Psi
    Ey_h = -1j * d["dky"][None] * Psi
    Ez_h = -Psi_z
    grids = np.stack([ifft_xy(Psi, p), ifft_xy(Ex_h, p), ifft_xy(Ey_h, p), ifft_xy(Ez_h, p)])
    # step 7: interpolate (average) at the charges
    far = interp(p, d, grids, pos)
    t_near = time.perf_counter()
    near = near_field(p, d, pos, q, rows=near_rows)
    t_near = time.perf_counter() - t_near
    # gauge phi(0) = 0 (Sec. 5.2.2): pointwise near + gamma^{1/2}-averaged far at the origin
    if p.gauge:
        far0 = interp(p, d, grids[:1], np.zeros((1, 3)), kernel_r2=lambda rr: gamma_half(p, rr))[0, 0]
        near0 = near_at_origin(p, d, pos, q)
        B_i = -(far0 + near0)
    else:
        far0 = near0 = 0.0
        B_i = 0.0
    # outputs: self term of Sec. 6.3, F = q E-bar, U = 1/2 sum q phi-bar (eq. Ufinal)
    self_c = 2.0 * d["xi_e"] / (FOUR_PI * p.eps * SQRT_PI)
    phi = far[:, 0] + near[:, 0] + B_i - q * self_c
    E = far[:, 1:] + near[:, 1:]
    F = q[:, None] * E
    U = 0.5 * float(np.sum(q * phi))
    wall_terms = {}
    if walls:
        # the walls alone: the correction with m_phi = 0, m_E = +sigma_b, -sigma_t
        # and the k = 0 slope of eqs. ai1, ai2 without charges (mean of the two)
        al_s = np.zeros_like(alpha)
        be_s = np.zeros_like(beta)
        if np.any(act):
            zk = np.zeros(int(np.count_nonzero(act)), dtype=complex)
            a_, b_, _, _ = correction_coeffs(p, kabs[act], zk, sbh[act], zk, -sth[act])
            al_s[act] = a_
            be_s[act] = b_
        A_s = (sth[0, 0].real - sbh[0, 0].real) / (2.0 * p.eps)
        Psi_s = al_s[None] * e1 + be_s[None] * e2
        Psi_s[:, ~act] = 0.0
        Psi_s[:, 0, 0] += A_s * z
        phi_s = ifft_xy(Psi_s, p)
        phi_s_q = interp(p, d, phi_s[None], pos)[:, 0]
        Eh = np.exp(-kabs * p.H)
        on_b = np.where(act, al_s * Eh + be_s, 0.0)
        on_t = np.where(act, al_s + be_s * Eh, 0.0)
        on_t[0, 0] = A_s * p.H
        phi_s_b = ifft_xy(on_b[None], p)[0]
        phi_s_t = ifft_xy(on_t[None], p)[0]
        hh = d["h"] ** 2
        W_ss = hh * float(np.sum(sb * phi_s_b + st * phi_s_t))
        Q_s = hh * float(np.sum(sb + st))
        E_qs = float(np.sum(q * phi_s_q))
        U += 0.5 * (E_qs + W_ss + B_i * Q_s)
        wall_terms = dict(sigma_b_hat=sbh, sigma_t_hat=sth, alpha_s=al_s, beta_s=be_s, A_s=A_s,
                          phi_s=phi_s, phi_s_q=phi_s_q, phi_s_b=phi_s_b, phi_s_t=phi_s_t,
                          E_qs=E_qs, W_ss=W_ss, Q_s=Q_s)
    if timings is not None:
        timings["near"] = t_near
        timings["far"] = time.perf_counter() - t_start - t_near
    inter = dict(f_o=f_o, f_i=f_i, F_o=F_o, F_i=F_i, fh_o=fh_o, fh_i=fh_i,
                 y_o=y_o, y_i=y_i, mphi_b=mphi_b, mE_b=mE_b, mphi_t=mphi_t, mE_t=mE_t,
                 alpha=alpha, beta=beta, A_i=A_i, A_i1=A_i1, A_i2=A_i2, Psi=Psi,
                 Psi_z=Psi_z, grids=grids, far=far, near=near, B_i=B_i, far0=far0,
                 near0=near0, c_o=c_o, img_pos=ipos, img_q=iq, derived=d, **wall_terms)
    return U, phi, F, inter
