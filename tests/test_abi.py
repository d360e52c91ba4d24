"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/dpse.h declares, and its host-only parameter derivation follows
the paper's rules (validated against printed values, not against the oracle)."""
import ctypes
import math
import os
import re

import pytest

import paper_2101_07088_amd as dp
from paper_2101_07088_amd import native
from workloads import SlabParams, config_jump, config_large, config_small

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "dpse.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpse_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(dp.library_path())
    syms = declared_symbols()
    assert "dpse_solve" in syms and "dpse_plan_create" in syms and len(syms) >= 9
    for s in syms:
        assert hasattr(lib, s), s


def test_derive_named_workloads():
    for cfg, ng, he in ((config_small, 18, 4.5), (config_jump, 18, 2.25), (config_large, 12, 1.5)):
        p = cfg()[0] if cfg is not config_large else SlabParams(
            Lx=256.0, Ly=256.0, H=64.0, eps=1.0, eps_b=0.05, eps_t=20.0, xi=1.5, Nx=1024, Ny=1024, Nz=257,
            r_cut=2.0)
        info = dp.derive(p)
        assert info["support"] == ng
        assert abs(info["H_E"] - he) < 1e-12
        assert abs(info["g_t"] - 1.0 / (2 * p.xi)) < 1e-12
        assert info["z_lo"] == -3 * he and abs(info["z_hi"] - (p.H + 3 * he)) < 1e-12
        assert info["n_modes"] == p.Ny * (p.Nx // 2 + 1)


def test_derived_cutoff_reproduces_printed_rnf():
    # r_cut = 0 asks the library for eq. rnf; g_w > 0 adds n_sigma g_w = 4 g_w
    rows = [l.split() for l in open(os.path.join(GOLDEN, "ewnoparam.txt")) if l.strip() and not l.startswith("#")]
    for n, xi, nz, he, rnf in rows:
        g_t = 1.2 * 2.0 / int(n)  # 3-digit rule h = g_t/1.2 on a box of side 2
        xi_v = 1.0 / (2.0 * math.sqrt(g_t * g_t - 0.025 ** 2))
        # the cutoff does not depend on the grid; any valid grid will do
        q = SlabParams(Lx=2.0, Ly=2.0, H=2.0, eps=1, eps_b=1, eps_t=1, xi=xi_v, Nx=64, Ny=64, Nz=33, r_cut=0.0,
                       g_w=0.025, n_g=2)
        prm = native._params(q, delta=5e-4)
        inf = native._Info()
        assert native._lib().dpse_derive(ctypes.byref(prm), ctypes.byref(inf)) == 0
        assert abs((inf.r_cut - 4 * 0.025) - float(rnf)) < 0.011


@pytest.mark.parametrize("change", [
    dict(Nz=34), dict(Nx=48), dict(Nx=2048, Lx=512.0, Ly=512.0, Ny=2048), dict(Ly=32.0),
    dict(eps=0.0), dict(xi=-1.0), dict(r_cut=9.0), dict(n_g=17), dict(g_w=-1.0), dict(H=2.0),
])
def test_derive_rejects_invalid_parameters(change):
    p = config_small()[0].copy(**change)
    with pytest.raises(dp.DpseError) as e:
        dp.derive(p)
    assert e.value.status == 1


def test_uniform_fast_flag_validation():
    """The uniform-permittivity solver needs equal permittivities and uses the
    domain [-H_E, H + H_E]."""
    p, _, _ = config_small(0)
    info = dp.derive(p.copy(uniform_fast=True))
    assert abs(info["z_lo"] + info["H_E"]) < 1e-12 and abs(info["z_hi"] - (p.H + info["H_E"])) < 1e-12
    with pytest.raises(dp.DpseError):
        dp.derive(p.copy(uniform_fast=True, eps_b=0.5))


def test_set_walls_rejects_a_null_plan():
    """dpse_plan_set_walls validates its plan on the host (no GPU needed)."""
    import ctypes
    from paper_2101_07088_amd.native import _lib
    assert _lib().dpse_plan_set_walls(None, None, None) == 1


def test_one_jump_flag_validation():
    """The one-jump solver needs a jump at exactly one wall, excludes the
    uniform solver, and spans the charges and their images."""
    p, _, _ = config_small(0)
    pb = p.copy(one_jump=True, eps_b=0.05, eps_t=p.eps)
    info = dp.derive(pb)
    assert abs(info["z_lo"] + p.H + info["H_E"]) < 1e-12 and abs(info["z_hi"] - (p.H + info["H_E"])) < 1e-12
    info = dp.derive(p.copy(one_jump=True, eps_b=p.eps, eps_t=20.0))
    assert abs(info["z_lo"] + info["H_E"]) < 1e-12 and abs(info["z_hi"] - (2 * p.H + info["H_E"])) < 1e-12
    for bad in (p.copy(one_jump=True, eps_b=p.eps, eps_t=p.eps), p.copy(one_jump=True, eps_b=0.05, eps_t=20.0),
                pb.copy(uniform_fast=True)):
        with pytest.raises(dp.DpseError):
            dp.derive(bad)


def test_triply_flag_validation():
    """The triply periodic variant: equal permittivities, Nz a power of two,
    a period of at least 4 H_E, r_cut below half of it, no other solver flag."""
    from workloads import SlabParams
    p = SlabParams(Lx=16.0, Ly=16.0, H=16.0, eps=1.0, eps_b=1.0, eps_t=1.0, xi=1.0, Nx=64, Ny=64, Nz=64,
                   r_cut=3.0, triply=True)
    info = dp.derive(p)
    assert info["z_lo"] == 0.0 and abs(info["z_hi"] - (16.0 - 0.25)) < 1e-12
    for bad in (p.copy(Nz=65), p.copy(eps_b=0.5), p.copy(H=8.0), p.copy(uniform_fast=True),
                p.copy(one_jump=True), p.copy(H=5.5, r_cut=3.0)):
        with pytest.raises(dp.DpseError):
            dp.derive(bad)


def test_solve_static_rejects_a_null_plan():
    """dpse_solve_static validates its plan on the host (no GPU needed)."""
    from paper_2101_07088_amd.native import _lib
    assert _lib().dpse_solve_static(None, None, 1, None, None, None, None, None) == 1
