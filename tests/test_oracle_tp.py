"""Pins of the triply periodic oracle (Sec. 7's TP variant of the method)
against the classical three-dimensional Ewald sum of point charges, and
exact invariances of the discrete method."""
import numpy as np
import pytest

from oracle import tp_oracle as T
from oracle import truth
from workloads import SlabParams, charges


def _tp(N, xi, L=16.0):
    return SlabParams(Lx=L, Ly=L, H=L, eps=1.0, eps_b=1.0, eps_t=1.0, xi=xi, Nx=N, Ny=N, Nz=N, r_cut=3.5)


def rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def test_tp_matches_ewald3d():
    """Forces, potentials and energy of point charges agree with the classical
    Ewald sum (tin-foil boundary, alpha-independent to 2e-16 itself) to the
    accuracy of the Gaussian truncation."""
    pos, q = charges(1, 20, 20, 16.0, 16.0, 0.0, 16.0)
    Ut, pt, Et = truth.ewald3d((16.0, 16.0, 16.0), pos, q, alpha=0.35, n_real=2, k_cut=14)
    Ut2, _, Et2 = truth.ewald3d((16.0, 16.0, 16.0), pos, q, alpha=0.5, n_real=2, k_cut=18)
    assert abs(Ut - Ut2) < 1e-12 * abs(Ut) and np.abs(Et - Et2).max() < 1e-12 * np.abs(Et).max()
    for N, xi, tol in ((32, 1.0, 5e-5), (64, 1.4, 2e-5)):
        U, phi, F, _ = T.solve_tp(_tp(N, xi), pos, q)
        assert rel(F, q[:, None] * Et) < tol
        assert abs(U - Ut) < 10 * tol * abs(Ut)
        assert np.abs(phi - pt).max() < 5 * tol * np.abs(pt).max()


def test_tp_shift_by_grid_cells_and_wrap_are_exact():
    """Moving every charge by whole grid cells (z included) or by a period
    leaves the discrete solve unchanged up to rounding; a generic shift only
    at the method's accuracy."""
    p = _tp(32, 1.0)
    pos, q = charges(2, 15, 15, 16.0, 16.0, 0.0, 16.0)
    U, phi, F, _ = T.solve_tp(p, pos, q)
    h = 0.5
    for sh in ((3 * h, 0.0, 5 * h), (0.0, -2 * h, -7 * h), (16.0, 0.0, -32.0)):
        U2, phi2, F2, _ = T.solve_tp(p, pos + np.array(sh), q)
        assert abs(U2 - U) < 1e-12 * abs(U) and np.abs(F2 - F).max() < 1e-11 * np.abs(F).max()
        assert np.abs(phi2 - phi).max() < 1e-11 * np.abs(phi).max()
    U3, _, F3, _ = T.solve_tp(p, pos + np.array([0.123, 0.377, 0.211]), q)
    assert 1e-9 < rel(F3, F) < 1e-4


def test_tp_needs_four_support_radii_per_period():
    with pytest.raises(ValueError):
        T.derive_tp(_tp(16, 1.0, L=8.0))
