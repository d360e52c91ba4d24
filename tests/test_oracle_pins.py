"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Nothing here retypes an oracle formula: each test compares the oracle with an
independent route -- printed values of the paper (tests/golden), a brute-force
loop, a library routine the oracle does not use for that step, a closed-form
continuum solution, the Ewald2D + image-series reference, or an exact
invariance of the discrete method.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate
from numpy.polynomial import chebyshev as npcheb

from oracle import dpse_oracle as O
from oracle import truth
from oracle.planner import paper_rule, r_nf
from workloads import SlabParams, charges

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


# --- planner rules vs printed parameters (Sec. 5.1, 5.3, 6) -----------------

def test_planner_reproduces_ewnoparam_table():
    for n, xi, nz, he, rnf in _rows("ewnoparam.txt"):
        d = paper_rule(2.0, int(n), 0.75, 0.025, four_digits=False)
        assert abs(d["xi"] - float(xi)) < 5e-3 * float(xi) + 0.05
        assert d["Nz"] == int(nz)
        assert abs(d["H_E"] - float(he)) < 0.006
        assert abs(r_nf(0.025, d["xi"], 5e-4) - float(rnf)) < 0.011


def test_planner_reproduces_sec6_parameters():
    for name, L, n, H, gw, gt, xi, he, rnf, nz, *_ in _rows("paper_params.txt"):
        d = paper_rule(float(L), int(n), float(H), float(gw), four_digits=True)
        assert abs(d["g_t"] - float(gt)) < 0.005, name
        assert abs(d["xi"] - float(xi)) < 0.06, name
        assert abs(d["H_E"] - float(he)) < 0.006, name
        assert d["Nz"] == int(nz), name
        assert abs(r_nf(float(gw), d["xi"], 1e-4) - float(rnf)) < 0.006, name


def test_near_constraint_alpha():
    for delta, alpha in _rows("constraints.txt"):
        # point charges: r_nf = alpha/xi for any xi
        for xi in (0.5, 3.0):
            assert abs(r_nf(0.0, xi, float(delta)) * xi - float(alpha)) < 0.006


# --- transforms ---------------------------------------------------------------

def test_fft_xy_matches_explicit_dft():
    rng = np.random.default_rng(1)
    p = SlabParams(Lx=4.0, Ly=3.0, H=1, eps=1, eps_b=1, eps_t=1, xi=1, Nx=8, Ny=6, Nz=3, r_cut=1)
    f = rng.standard_normal((3, 6, 8))
    F = O.fft_xy(f, p)
    ref = np.zeros((3, 6, 5), complex)
    for c in range(3):
        for jy in range(6):
            for jx in range(5):
                acc = 0j
                for y in range(6):
                    for x in range(8):
                        acc += f[c, y, x] * np.exp(-2j * np.pi * (jx * x / 8 + jy * y / 6))
                ref[c, jy, jx] = acc / 48
    assert np.abs(F - ref).max() < 1e-14
    assert np.abs(O.ifft_xy(F, p) - f).max() < 1e-13


def test_chebyshev_transform_interpolates_and_is_exact_on_polynomials():
    rng = np.random.default_rng(2)
    n = 17
    s = np.cos(np.pi * np.arange(n) / (n - 1))
    V = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    C = O.cheb_coeffs(V)
    back = np.array([[sum(C[m, col] * math.cos(m * math.acos(max(-1, min(1, sj)))) for m in range(n))
                      for col in range(3)] for sj in s])
    assert np.abs(back - V).max() < 1e-13
    # a polynomial of degree < n: 3 T_0 - 2 T_5 + T_16
    vals = npcheb.chebval(s, [3, 0, 0, 0, 0, -2] + [0] * 10 + [1])
    Cp = O.cheb_coeffs(vals)
    want = np.zeros(n); want[0] = 3; want[5] = -2; want[16] = 1
    assert np.abs(Cp - want).max() < 1e-14


def test_clenshaw_curtis_weights_integrate():
    w = O.cc_weights(21)
    s = np.cos(np.pi * np.arange(21) / 20)
    assert abs(w @ np.exp(s) - (math.e - 1 / math.e)) < 1e-14
    w5 = O.cc_weights(5)
    s5 = np.cos(np.pi * np.arange(5) / 4)
    assert abs(w5 @ s5 ** 4 - 0.4) < 1e-15


# --- per-mode BVP (App. A) ----------------------------------------------------

@pytest.mark.parametrize("kappa", [0.0, 0.3, 3.7, 40.0])
def test_bvp_recovers_manufactured_polynomial(kappa):
    rng = np.random.default_rng(3)
    N = 12
    c = rng.standard_normal(N)
    c[-1] = 0.0  # keep degree <= N-2 so y' has degree <= N-3 (truncation exact)
    # enforce the BCs by adjusting c0 and c1 (linear in them)
    def bc(cc):
        d1 = npcheb.chebder(cc)
        if kappa == 0.0:
            return np.array([npcheb.chebval(1, cc), npcheb.chebval(-1, cc)])
        return np.array([npcheb.chebval(1, d1) + kappa * npcheb.chebval(1, cc),
                         npcheb.chebval(-1, d1) - kappa * npcheb.chebval(-1, cc)])
    base = bc(c)
    J = np.zeros((2, 2))
    for i in range(2):
        e = np.zeros(N); e[i] = 1.0
        J[:, i] = bc(c + e) - base
    c[:2] -= np.linalg.solve(J, base)
    g = npcheb.chebder(c, 2)
    g = np.concatenate([g, np.zeros(N - len(g))]) - kappa ** 2 * c
    P, Y = O.bvp_operators(N)
    M = O.bvp_matrix(N, kappa, kappa == 0.0, (P, Y))
    u = np.linalg.solve(M, np.concatenate([g, [0.0, 0.0]]))
    assert np.abs(Y @ u - c).max() < 1e-13 * np.abs(u).max()


def test_bvp_converges_to_free_space_green_function():
    """y'' - k^2 y = g with the DtN (Robin) conditions equals the free-space
    convolution -(1/2k) int e^{-k|s-t|} g(t) dt for g supported inside (-1,1)."""
    kappa, N = 2.5, 110
    g = lambda t: np.exp(-((t - 0.2) ** 2) / (2 * 0.08 ** 2))
    s = np.cos(np.pi * np.arange(N) / (N - 1))
    gc = O.cheb_coeffs(g(s))
    P, Y = O.bvp_operators(N)
    u = np.linalg.solve(O.bvp_matrix(N, kappa, False, (P, Y)), np.concatenate([gc, [0, 0]]))
    yc = Y @ u
    for x in (-0.7, 0.1, 0.25, 0.9):
        exact = -scipy.integrate.quad(lambda t: np.exp(-kappa * abs(x - t)) * g(t), -1, 1,
                                      points=[x, 0.2], limit=200, epsabs=1e-14)[0] / (2 * kappa)
        assert abs(npcheb.chebval(x, yc) - exact) < 1e-10


# --- harmonic correction (Sec. 3.1.2) -----------------------------------------

def test_correction_satisfies_jump_conditions():
    rng = np.random.default_rng(4)
    p = SlabParams(Lx=1, Ly=1, H=1.7, eps=2.0, eps_b=0.1, eps_t=30.0, xi=1, Nx=2, Ny=2, Nz=3, r_cut=1)
    k = np.array([0.1, 1.0, 7.0, 25.0])
    m = [rng.standard_normal(4) + 1j * rng.standard_normal(4) for _ in range(4)]
    al, be, _, sol = O.correction_coeffs(p, k, *m)
    ab, bt = sol[:, 2], sol[:, 3]
    E = np.exp(-k * p.H)
    psi_i = lambda z: al * np.exp(k * (z - p.H)) + be * np.exp(-k * z)
    dpsi_i = lambda z: k * al * np.exp(k * (z - p.H)) - k * be * np.exp(-k * z)
    A_b = ab                      # psi_b = A_b e^{kz}
    B_t = bt / E                  # psi_t = B_t e^{-kz}
    assert np.abs(psi_i(0.0) - A_b - (-m[0])).max() < 1e-12
    assert np.abs(p.eps * dpsi_i(0.0) - p.eps_b * k * A_b - (-m[1])).max() < 1e-11
    assert np.abs(psi_i(p.H) - B_t * E - (-m[2])).max() < 1e-12
    assert np.abs(p.eps * dpsi_i(p.H) + p.eps_t * k * B_t * E - (-m[3])).max() < 1e-10


# --- brute-force spreading and near field -------------------------------------

def test_spread_matches_pointwise_loop():
    p = SlabParams(Lx=3.0, Ly=3.0, H=2.0, eps=1, eps_b=1, eps_t=1, xi=2.0, Nx=12, Ny=12, Nz=11, r_cut=1.0, n_g=8)
    d = O.derive(p)
    pos = np.array([[0.1, 2.95, 0.7], [1.53, 1.0, 1.9]])
    q = np.array([1.5, -0.5])
    f = O.spread(p, d, pos, q)
    ref = np.zeros_like(f)
    g = d["g_t"]
    for k in range(2):
        for c in range(p.Nz):
            dz = d["z"][c] - pos[k, 2]
            if abs(dz) > d["H_E"]:
                continue
            for j in range(p.Ny):
                dy = (j * d["h"] - pos[k, 1] + 1.5) % 3.0 - 1.5
                if not (-d["H_E"] < dy <= d["H_E"] + 1e-12):
                    continue
                for i in range(p.Nx):
                    dx = (i * d["h"] - pos[k, 0] + 1.5) % 3.0 - 1.5
                    if not (-d["H_E"] < dx <= d["H_E"] + 1e-12):
                        continue
                    ref[c, j, i] += q[k] * math.exp(-(dx * dx + dy * dy + dz * dz) / (2 * g * g)) / (2 * math.pi * g * g) ** 1.5
    assert np.abs(f - ref).max() < 1e-13 * np.abs(ref).max()


def test_near_field_matches_pair_loop():
    p = SlabParams(Lx=3.0, Ly=2.5, H=2.0, eps=1.3, eps_b=0.2, eps_t=5.0, xi=2.0, Nx=12, Ny=10, Nz=11, r_cut=1.1)
    d = O.derive(p)
    pos, q = charges(5, 4, 4, 3.0, 2.5, 0.05, 1.95)
    out = O.near_field(p, d, pos, q)
    gb, gt = d["gamma_b"], d["gamma_t"]
    ref = np.zeros((8, 4))
    for t in range(8):
        for s in range(8):
            for (zs, st, skip_self) in ((pos[s, 2], q[s], True), (-pos[s, 2], gb * q[s], False),
                                        (2 * p.H - pos[s, 2], gt * q[s], False)):
                for a in (-1, 0, 1):
                    for b in (-1, 0, 1):
                        if skip_self and s == t and a == 0 and b == 0:
                            continue
                        rx = pos[t, 0] - pos[s, 0] + a * p.Lx
                        ry = pos[t, 1] - pos[s, 1] + b * p.Ly
                        rz = pos[t, 2] - zs
                        r = math.sqrt(rx * rx + ry * ry + rz * rz)
                        if r >= p.r_cut:
                            continue
                        G = math.erfc(p.xi * r) / r
                        e = (math.erfc(p.xi * r) / r ** 2 + 2 * p.xi / math.sqrt(math.pi) * math.exp(-(p.xi * r) ** 2) / r) / r
                        ref[t] += st * np.array([G, e * rx, e * ry, e * rz]) / (4 * math.pi * p.eps)
    assert np.abs(out - ref).max() < 1e-13
    # the sampled-target form gives the same rows
    tt = np.array([6, 1, 3])
    assert np.abs(O.near_field(p, d, pos, q, targets=tt) - ref[tt]).max() < 1e-13


# --- the whole oracle against the Ewald2D + image-series reference ------------

def _paper_grid(L, H, eb, et, nxy=32, nz=None):
    d = paper_rule(L, nxy, H, 0.0, four_digits=True)
    return SlabParams(Lx=L, Ly=L, H=H, eps=1.0, eps_b=eb, eps_t=et, xi=d["xi"], Nx=nxy, Ny=nxy,
                      Nz=nz or d["Nz"], r_cut=r_nf(0.0, d["xi"], 1e-4), n_g=d["n_g"])


@pytest.mark.parametrize("eb,et", [(1.0, 1.0), (0.05, 0.05), (0.5, 0.2), (0.05, 20.0), (1.0, 0.02)])
def test_oracle_matches_ewald2d_images(eb, et):
    pos, q = charges(3, 4, 4, 4.0, 4.0, 0.3, 1.7)
    p = _paper_grid(4.0, 2.0, eb, et)
    U, phi, F, I = O.solve(p, pos, q)
    Ut, pt, Et, p0, _ = truth.ewald2d(4.0, 4.0, 2.0, 1.0, eb, et, pos, q, probes=[[0, 0, 0]])
    Ft = q[:, None] * Et
    assert np.sqrt(((F - Ft) ** 2).sum() / (Ft ** 2).sum()) < 3e-4
    assert abs(U - Ut) < 5e-4 * 0.5 * np.sum(np.abs(q * pt))
    # gauge phi(0) = 0: the oracle's potentials are the truth's minus its value at the origin
    assert np.abs(phi - (pt - p0[0])).max() < 2e-3 * np.abs(pt - p0[0]).mean()
    # the two discrete formulas for A_i(0) agree to about 3 digits (Sec. 5.2.2 step 5)
    assert abs(I["A_i1"] - I["A_i2"]) < 1e-2 * abs(I["A_i"]) + 1e-6


def test_oracle_spectral_convergence_in_z():
    pos, q = charges(7, 4, 4, 4.0, 4.0, 0.3, 1.7)
    errs = []
    for nz in (30, 45, 82):
        p = _paper_grid(4.0, 2.0, 0.1, 0.3, nz=nz)
        _, _, F, _ = O.solve(p, pos, q)
        _, _, Et = truth.ewald2d(4.0, 4.0, 2.0, 1.0, 0.1, 0.3, pos, q)
        Ft = q[:, None] * Et
        errs.append(np.sqrt(((F - Ft) ** 2).sum() / (Ft ** 2).sum()))
    assert errs[0] > 5 * errs[1] > 5 * errs[2] / 5 and errs[2] < 3e-4


def test_energy_force_consistency_finite_difference():
    """W1 (finite difference of U) vs W2 = sum F.dX, eqs. w1, w2 of Sec. 6.3."""
    pos, q = charges(11, 5, 5, 4.0, 4.0, 0.3, 1.7)
    p = _paper_grid(4.0, 2.0, 1 / 20, 1 / 50)
    rng = np.random.default_rng(0)
    dX = rng.standard_normal(pos.shape)
    dX /= np.linalg.norm(dX, axis=1, keepdims=True)
    d0 = 1e-4
    Up = O.solve(p, pos + 0.5 * d0 * dX, q)[0]
    Um = O.solve(p, pos - 0.5 * d0 * dX, q)[0]
    _, _, F, _ = O.solve(p, pos, q)
    W1 = -(Up - Um) / d0
    W2 = float(np.sum(F * dX))
    assert abs(W1 - W2) < 2e-3 * abs(W1)


# --- exact invariances of the discrete method ---------------------------------

def _small(eb=0.2, et=5.0, gauge=True):
    p = SlabParams(Lx=6.0, Ly=6.0, H=4.0, eps=1.0, eps_b=eb, eps_t=et, xi=1.5, Nx=24, Ny=24, Nz=25,
                   r_cut=2.0, gauge=gauge)
    pos, q = charges(21, 6, 6, 6.0, 6.0, 0.3, 3.7)
    return p, pos, q


def test_linearity_and_sign_flip():
    p, pos, q = _small()
    U, phi, F, _ = O.solve(p, pos, q)
    U2, phi2, F2, _ = O.solve(p, pos, 2 * q)
    Um, phim, Fm, _ = O.solve(p, pos, -q)
    assert abs(U2 - 4 * U) < 1e-12 * abs(U)
    assert np.abs(F2 - 4 * F).max() < 1e-12 * np.abs(F).max()
    assert np.abs(Fm - F).max() < 1e-12 * np.abs(F).max()
    assert np.abs(phim + phi).max() < 1e-12 * np.abs(phi).max()


def test_mirror_symmetry_swaps_walls():
    p, pos, q = _small(gauge=False)
    U, phi, F, I = O.solve(p, pos, q)
    pm = pos.copy(); pm[:, 2] = p.H - pos[:, 2]
    Um, phim, Fm, Im = O.solve(p.copy(eps_b=p.eps_t, eps_t=p.eps_b), pm, q)
    # forces are exactly mirror-symmetric; the potential only up to the constant
    # part A_i H of the linear k=0 mode, which the discrete interpolation does
    # not reproduce as an exact constant on a coarse z grid
    assert np.abs(Fm[:, :2] - F[:, :2]).max() < 1e-12 * np.abs(F).max()
    assert np.abs(Fm[:, 2] + F[:, 2]).max() < 1e-12 * np.abs(F).max()
    g, gm = I["grids"], Im["grids"][:, ::-1]
    assert np.abs(g[0] - gm[0] - (I["A_i"].real * p.H)).max() < 1e-11 * np.abs(g[0]).max()
    assert np.abs(g[1:3] - gm[1:3]).max() < 1e-11 * np.abs(g[1:]).max()
    assert np.abs(g[3] + gm[3]).max() < 1e-11 * np.abs(g[1:]).max()


def test_grid_translation_and_axis_swap_and_permutation():
    p, pos, q = _small()
    U, phi, F, _ = O.solve(p, pos, q)
    h = p.Lx / p.Nx
    pt = pos.copy(); pt[:, 0] = (pt[:, 0] + 3 * h) % p.Lx
    Ut, _, Ft, _ = O.solve(p, pt, q)
    assert abs(Ut - U) < 1e-11 * abs(U) and np.abs(Ft - F).max() < 1e-10 * np.abs(F).max()
    ps = pos[:, [1, 0, 2]]
    Us, _, Fs, _ = O.solve(p, ps, q)
    assert abs(Us - U) < 1e-11 * abs(U) and np.abs(Fs[:, [1, 0, 2]] - F).max() < 1e-10 * np.abs(F).max()
    perm = np.random.default_rng(0).permutation(len(q))
    Up, php, Fp, _ = O.solve(p, pos[perm], q[perm])
    assert abs(Up - U) < 1e-12 * abs(U) and np.abs(Fp - F[perm]).max() < 1e-12 * np.abs(F).max()
    assert np.abs(php - phi[perm]).max() < 1e-12 * np.abs(phi).max()


def test_permittivity_scaling():
    p, pos, q = _small()
    U, phi, F, _ = O.solve(p, pos, q)
    U3, phi3, F3, _ = O.solve(p.copy(eps=3.0, eps_b=3 * p.eps_b, eps_t=3 * p.eps_t), pos, q)
    assert abs(3 * U3 - U) < 1e-12 * abs(U)
    assert np.abs(3 * F3 - F).max() < 1e-12 * np.abs(F).max()


# --- the uniform-permittivity solver (no wall group, no images, no correction) ---

def _fast_grid(L, H, nz=None):
    p = _paper_grid(L, H, 1.0, 1.0)
    d = O.derive(p)
    # the z rule of Sec. 5.1 on the smaller domain [-H_E, H + H_E]
    nz = nz or int(math.ceil(math.pi * (H + 2 * d["H_E"]) / (2 * d["h"])))
    return p.copy(uniform_fast=True, Nz=nz)


def test_fast_uniform_matches_ewald2d():
    pos, q = charges(3, 4, 4, 4.0, 4.0, 0.3, 1.7)
    p = _fast_grid(4.0, 2.0)
    d = O.derive(p)
    assert abs(d["a"] + d["H_E"]) < 1e-15 and abs(d["b"] - (2.0 + d["H_E"])) < 1e-15
    U, phi, F, I = O.solve(p, pos, q)
    Ut, pt, Et, p0, _ = truth.ewald2d(4.0, 4.0, 2.0, 1.0, 1.0, 1.0, pos, q, probes=[[0, 0, 0]])
    Ft = q[:, None] * Et
    assert np.sqrt(((F - Ft) ** 2).sum() / (Ft ** 2).sum()) < 3e-4
    assert abs(U - Ut) < 5e-4 * 0.5 * np.sum(np.abs(q * pt))
    assert np.abs(phi - (pt - p0[0])).max() < 2e-3 * np.abs(pt - p0[0]).mean()
    # nothing corrected, one group
    assert not np.any(I["c_o"]) and np.all(I["alpha"] == 0) and len(I["img_q"]) == 0
    # the field of the neutral set vanishes at both ends: the two end slopes agree
    assert abs(I["A_i1"] - I["A_i2"]) < 1e-3 * abs(I["A_i"]) + 1e-8
    # and the general algorithm on its own domain reaches the same answer
    Ug, phig, Fg, _ = O.solve(_paper_grid(4.0, 2.0, 1.0, 1.0), pos, q)
    assert np.sqrt(((F - Fg) ** 2).sum() / (Fg ** 2).sum()) < 5e-4


def test_fast_uniform_spectral_convergence_and_energy():
    pos, q = charges(7, 4, 4, 4.0, 4.0, 0.3, 1.7)
    _, _, Et = truth.ewald2d(4.0, 4.0, 2.0, 1.0, 1.0, 1.0, pos, q)
    Ft = q[:, None] * Et
    errs = []
    for nz in (17, 25, 41):
        _, _, F, _ = O.solve(_fast_grid(4.0, 2.0, nz=nz), pos, q)
        errs.append(np.sqrt(((F - Ft) ** 2).sum() / (Ft ** 2).sum()))
    assert errs[0] > 3 * errs[1] and errs[1] > errs[2] and errs[2] < 3e-4
    # energy/force consistency (eqs. w1, w2)
    p = _fast_grid(4.0, 2.0)
    rng = np.random.default_rng(1)
    dX = rng.standard_normal(pos.shape)
    dX /= np.linalg.norm(dX, axis=1, keepdims=True)
    d0 = 1e-4
    Up = O.solve(p, pos + 0.5 * d0 * dX, q)[0]
    Um = O.solve(p, pos - 0.5 * d0 * dX, q)[0]
    W1 = -(Up - Um) / d0
    W2 = float(np.sum(O.solve(p, pos, q)[2] * dX))
    assert abs(W1 - W2) < 5e-4 * abs(W1)


def test_fast_uniform_needs_equal_permittivities():
    with pytest.raises(ValueError):
        O.derive(_paper_grid(4.0, 2.0, 0.5, 1.0).copy(uniform_fast=True))


# --- wall charges (Sec. 2 eqs. cbc2, cbc4; Sec. 4.3.3 eqs. mm2, mm4; ai1, ai2; eq. Ufinal)

def _wall_box(eps_b, eps_t, eps=1.0, N=32, Nz=33, L=8.0, H=4.0):
    p = SlabParams(Lx=L, Ly=L, H=H, eps=eps, eps_b=eps_b, eps_t=eps_t, xi=1.0, Nx=N, Ny=N, Nz=Nz, r_cut=2.0)
    pos, q = charges(1, 4, 4, L, L, 1.0, H - 1.0)
    h = L / N
    X, Y = np.meshgrid(np.arange(N) * h, np.arange(N) * h)
    return p, pos, q, X, Y


@pytest.mark.parametrize("eps_side", [1.0, 0.05, 20.0])
def test_wall_sheet_matches_textbook_single_interface(eps_side):
    """A sheet s cos(k x) on the bottom wall with no jump at the top: inside the
    slab the potential is s/(k (eps + eps_b)) e^{-k z} cos(k x), the textbook
    field of a charged interface between two half-spaces; mirrored for a sheet
    on the top wall (potential s/(k (eps + eps_t)) e^{-k (H - z)} cos(k x))."""
    k = 2.0 * math.pi * 2 / 8.0
    s = 0.3
    p, pos, q, X, Y = _wall_box(eps_side, 1.0)
    _, _, _, I = O.solve(p, pos, q, sigma_b=s * np.cos(k * X))
    z = I["derived"]["z"]
    ins = (z >= 0) & (z <= p.H)
    ref = s / ((p.eps + eps_side) * k) * np.exp(-k * z)[:, None, None] * np.cos(k * X)[None]
    assert np.abs(I["phi_s"][ins] - ref[ins]).max() < 1e-12
    p, pos, q, X, Y = _wall_box(1.0, eps_side)
    _, _, _, I = O.solve(p, pos, q, sigma_t=s * np.cos(k * Y))
    ref = s / ((p.eps + eps_side) * k) * np.exp(-k * (p.H - z))[:, None, None] * np.cos(k * Y)[None]
    assert np.abs(I["phi_s"][ins] - ref[ins]).max() < 1e-12


@pytest.mark.parametrize("eps_b,eps_t", [(0.05, 20.0), (1.0, 1.0), (20.0, 0.05)])
def test_wall_capacitor_field(eps_b, eps_t):
    """Uniform +s on the bottom wall and -s on the top: the field inside is the
    parallel-plate field s/eps along +z whatever the outer permittivities, and
    every charge's force changes by exactly q s / eps along z (up to the
    truncation of the interpolation kernel)."""
    s = 0.2
    p, pos, q, X, Y = _wall_box(eps_b, eps_t, eps=2.0, Nz=65)   # nodes fine enough for the kernel's mass
    N = p.Nx
    _, _, F0, _ = O.solve(p, pos, q)
    _, _, F1, I = O.solve(p, pos, q, sigma_b=np.full((N, N), s), sigma_t=np.full((N, N), -s))
    assert abs(I["A_s"] - (-s / p.eps)) < 1e-14
    dF = F1 - F0
    assert np.abs(dF[:, :2]).max() < 1e-10
    assert np.allclose(dF[:, 2], q * s / p.eps, rtol=1e-4, atol=0)


def test_wall_energy_reciprocity_matches_literal_integral():
    """The energy with wall charges by reciprocity (the oracle's route) equals
    eq. Ufinal with the wall integrals taken as written: the pointwise
    potential (gamma^{1/2} average of the far field, pointwise near field of
    the charges and their images, gauge constant) summed over the wall grid
    points. The wall part is about a third of U here."""
    import workloads as W
    p, pos, q, sb, st = W.config_charged_walls(0, g_w=1e-2)
    U, phi, F, I = O.solve(p, pos, q, sigma_b=sb, sigma_t=st)
    Ul = O.wall_energy_literal(p, pos, q, phi, sb, st, I)
    wall = 0.5 * (I["E_qs"] + I["W_ss"] + I["B_i"] * I["Q_s"])
    assert abs(wall) > 0.2 * abs(U)
    assert abs(U - Ul) < 1e-5 * abs(U)


def _rate_of_work(p, pos, q, sb, st, seed=7, d0=1e-4, walls=True):
    rng = np.random.default_rng(seed)
    dX = rng.normal(size=pos.shape)
    dX /= np.linalg.norm(dX, axis=1)[:, None]
    kw = dict(sigma_b=sb, sigma_t=st)
    U, phi, F, _ = O.solve(p, pos, q, **kw)
    up = O.solve(p, pos + 0.5 * d0 * dX, q, **kw)
    um = O.solve(p, pos - 0.5 * d0 * dX, q, **kw)
    if walls:
        W1 = -(up[0] - um[0]) / d0
    else:  # the particle term of eq. Ufinal alone
        W1 = -(0.5 * np.sum(q * up[1]) - 0.5 * np.sum(q * um[1])) / d0
    W2 = float(np.sum(F * dX))
    return W1, W2


def test_wall_energy_is_the_potential_of_the_forces():
    """The charged-wall energy test of Sec. 6.3 (eqs. w1, w2): the rate of work
    of the forces equals the finite-difference rate of work of the energy at
    least as closely as the paper's own table (tests/golden/energslabEw.txt),
    and leaving out the wall integral of eq. Ufinal breaks it."""
    import workloads as W
    for gw, printed in _rows("energslabEw.txt"):
        gw, printed = float(gw), float(printed)
        if gw not in (1e-2, 1e-10):
            continue
        p, pos, q, sb, st = W.config_charged_walls(0, g_w=gw)
        W1, W2 = _rate_of_work(p, pos, q, sb, st)
        assert abs(W1 - W2) <= printed * abs(W1), (gw, W1, W2)
    p, pos, q, sb, st = W.config_charged_walls(0, g_w=1e-2)
    W1, W2 = _rate_of_work(p, pos, q, sb, st, walls=False)
    assert abs(W1 - W2) > 1e-2 * abs(W2)


def test_walls_rejected_by_the_uniform_solver():
    p, pos, q, X, Y = _wall_box(1.0, 1.0)
    with pytest.raises(ValueError):
        O.solve(p.copy(uniform_fast=True), pos, q, sigma_b=np.zeros((p.Ny, p.Nx)))


# --- one dielectric jump: images of every charge, then the free-space solve (Sec. 4 opening)

def _one_jump(eps_b, eps_t, nz=65):
    return SlabParams(Lx=4.0, Ly=4.0, H=2.0, eps=1.0, eps_b=eps_b, eps_t=eps_t, xi=2.0, Nx=32, Ny=32, Nz=nz,
                      r_cut=1.5, one_jump=True)


@pytest.mark.parametrize("eps_b,eps_t", [(0.05, 1.0), (1.0, 0.05), (20.0, 1.0)])
def test_one_jump_matches_image_series(eps_b, eps_t):
    """With a jump at one wall the exact solution is the charges plus one
    image each (the image series of the Ewald2D reference has nothing else);
    the one-jump solver reaches it to the method's accuracy, on the span of
    charges and images, with every charge imaged and nothing corrected."""
    pos, q = charges(3, 4, 4, 4.0, 4.0, 0.3, 1.7)
    p = _one_jump(eps_b, eps_t)
    d = O.derive(p)
    if eps_b != 1.0:
        assert abs(d["a"] + p.H + d["H_E"]) < 1e-14 and abs(d["b"] - p.H - d["H_E"]) < 1e-14
    else:
        assert abs(d["a"] + d["H_E"]) < 1e-14 and abs(d["b"] - 2 * p.H - d["H_E"]) < 1e-14
    U, phi, F, I = O.solve(p, pos, q)
    _, _, Et = truth.ewald2d(4.0, 4.0, 2.0, 1.0, eps_b, eps_t, pos, q)
    Ft = q[:, None] * Et
    assert np.sqrt(((F - Ft) ** 2).sum() / (Ft ** 2).sum()) < 2e-4
    assert len(I["img_q"]) == len(q) and not np.any(I["c_o"]) and np.all(I["alpha"] == 0)


def test_one_jump_top_is_the_mirror_of_bottom():
    """Reflecting the charges (z -> H - z) and swapping the outer permittivities
    maps the bottom-jump solve onto the top-jump one exactly: the two domains
    and their Chebyshev nodes are mirror images."""
    pos, q = charges(5, 5, 5, 4.0, 4.0, 0.3, 1.7)
    U1, phi1, F1, _ = O.solve(_one_jump(0.05, 1.0), pos, q)
    pm = pos.copy()
    pm[:, 2] = 2.0 - pm[:, 2]
    U2, phi2, F2, _ = O.solve(_one_jump(1.0, 0.05), pm, q)
    Fm = F2.copy()
    Fm[:, 2] *= -1
    assert np.abs(Fm - F1).max() < 1e-10 * np.abs(F1).max()
    # phi differs by the gauge point (the origin sits on the other wall) and by
    # A_i H times the interpolation kernel's discrete mass, which the mirror
    # turns the k = 0 slope's A_i z into (it varies at the truncation level)
    assert np.abs((phi2 - phi2.mean()) - (phi1 - phi1.mean())).max() < 1e-6 * np.abs(phi1).max()


def test_one_jump_needs_exactly_one_jump():
    for eb, et in ((1.0, 1.0), (0.05, 20.0)):
        with pytest.raises(ValueError):
            O.derive(_one_jump(eb, et))
    with pytest.raises(ValueError):
        O.derive(_one_jump(0.05, 1.0).copy(uniform_fast=True))
