"""GPU checks at the full size of the large workload (N = 2^20 ions, 256 x 256
x 64 slab, eps_b = 0.05, eps_t = 20, xi = 1.5, grid 1024 x 1024 x 257), in
the launch configuration the benchmark uses. The oracle cannot run the whole
solve at this size, so the checks are:
  * sampled outputs the oracle computes one by one: the near field at 96
    charges, and the spread grids f_i, f_o on an 8 x 8 column of grid points
    (from the oracle's spread of every charge that can reach it);
  * properties that hold at any size: the mixed path against the FP64 path
    (<= 1e-5 relative RMS force), the mirror z -> H - z with eps_b <-> eps_t,
    translation by whole grid cells, and the +2/-1 valence variant."""
import numpy as np
import pytest

import workloads as W
from oracle import dpse_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def solve(p, pos, q, precision, stages=()):
    import paper_2101_07088_amd as dp
    plan = dp.Plan(p, max_n=len(q), precision=precision)
    tp = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    U, phi, F = plan.solve(tp, tq)
    st = plan.sync_status()
    out = dict(status=st, U=float(U.cpu()[0]), phi=phi.cpu().numpy(), F=F.cpu().numpy())
    for s in stages:
        out[s] = plan.debug(s)
    plan.close()
    del tp, tq, U, phi, F
    torch.cuda.empty_cache()
    return out


@pytest.fixture(scope="module")
def large():
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = W.config_large(0)
    print(f"[large] N={len(q)} grid {p.Nx}x{p.Ny}x{p.Nz}: FP64 solve", flush=True)
    r64 = solve(p, pos, q, dp.DPSE_FP64, stages=(dp.Stage.NEAR, dp.Stage.FAR))
    assert r64["status"] == 0
    return p, pos, q, r64


def test_large_mixed_against_fp64(large):
    import paper_2101_07088_amd as dp
    p, pos, q, r64 = large
    rm = solve(p, pos, q, dp.DPSE_MIXED, stages=(dp.Stage.FAR,))
    assert rm["status"] == 0
    eF = rel_rms(rm["F"], r64["F"])
    far64 = q[:, None] * r64[dp.Stage.FAR][: len(q), 1:]
    farm = q[:, None] * rm[dp.Stage.FAR][: len(q), 1:]
    efar = rel_rms(farm, far64)
    # U = 1/2 sum q phi cancels strongly over a million charges: its error is
    # measured against the scale 1/2 sum |q phi| of its terms
    eU = abs(rm["U"] - r64["U"]) / (0.5 * np.sum(np.abs(q * r64["phi"])))
    ephi = rel_rms(rm["phi"], r64["phi"])
    print(f"[large] mixed vs FP64: relRMS F {eF:.2e}, far-field F {efar:.2e}, phi {ephi:.2e}, U {eU:.2e} "
          f"(relative to U itself {abs(rm['U'] - r64['U']) / abs(r64['U']):.2e})", flush=True)
    assert eF <= 1e-5 and efar <= 1e-5 and ephi <= 1e-5 and eU <= 1e-5


def test_large_mixed_every_spread_shape(large):
    """Every spreading shape the autotuner may choose on this grid (scatter,
    gather, and the gather form with its sums on the matrix cores), in the
    mixed path, against the FP64 path at the mixed bar; one plan, so the
    kernels run after one another on LDS that earlier kernels wrote."""
    import paper_2101_07088_amd as dp
    p, pos, q, r64 = large
    plan = dp.Plan(p, max_n=len(q), precision=dp.DPSE_MIXED)
    tp = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    tried = []
    for i in range(16):
        try:
            plan.set_tiles([i, -1, -1])
        except dp.DpseError:
            continue
        U, phi, F = plan.solve(tp, tq)
        assert plan.sync_status() == 0
        eF = rel_rms(F.cpu().numpy(), r64["F"])
        print(f"[large] spread shape {i}: mixed vs FP64 relRMS F {eF:.2e}", flush=True)
        assert eF <= 1e-5, i
        tried.append(i)
    assert len(tried) >= 8
    plan.close()
    del tp, tq
    torch.cuda.empty_cache()


def test_large_fp64_gather_and_matrix_core_spreading(large):
    """The FP64 path with the thread-per-column gather spreading and with its
    matrix-core form, against the default FP64 solve (the same sums in
    another order: 1e-12)."""
    import paper_2101_07088_amd as dp
    p, pos, q, r64 = large
    plan = dp.Plan(p, max_n=len(q), precision=dp.DPSE_FP64)
    tp = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    for i in (6, 12):
        plan.set_tiles([i, -1, -1])
        U, phi, F = plan.solve(tp, tq)
        assert plan.sync_status() == 0
        eF, ep = rel_rms(F.cpu().numpy(), r64["F"]), rel_rms(phi.cpu().numpy(), r64["phi"])
        print(f"[large] FP64 spread shape {i}: relRMS F {eF:.2e} phi {ep:.2e} vs the default", flush=True)
        assert eF <= 1e-12 and ep <= 1e-12, i
    plan.close()
    del tp, tq
    torch.cuda.empty_cache()


def test_large_near_field_sampled(large):
    import paper_2101_07088_amd as dp
    p, pos, q, r64 = large
    d = O.derive(p)
    rng = np.random.default_rng(1)
    tt = np.sort(rng.choice(len(q), 96, replace=False))
    ref = O.near_field(p, d, pos, q, targets=tt)
    got = r64[dp.Stage.NEAR][tt]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"[large] near field at 96 charges: max rel err {err:.2e}", flush=True)
    assert err < 1e-12


def test_large_spread_sampled(large):
    """f_i and f_o on the grid columns x in [i0, i0+8), y in [j0, j0+8), all z,
    against the oracle's spread of every charge within reach of them."""
    import paper_2101_07088_amd as dp
    p, pos, q, _ = large
    d = O.derive(p)
    h, HE = d["h"], d["H_E"]
    i0, j0 = 517, 203
    x0, y0 = i0 * h, j0 * h
    reach = 8 * h + 2 * HE
    dx = (pos[:, 0] - x0 + 0.5 * p.Lx) % p.Lx - 0.5 * p.Lx
    dy = (pos[:, 1] - y0 + 0.5 * p.Ly) % p.Ly - 0.5 * p.Ly
    sel = (np.abs(dx) <= reach) & (np.abs(dy) <= reach)
    ps, qs = pos[sel], q[sel]
    c_o, ipos, iq = O.groups_and_images(p, d, ps, qs)
    print(f"[large] spread sample: {sel.sum()} charges, {len(iq)} images", flush=True)
    f_i = O.spread(p, d, np.concatenate([ps, ipos]), np.concatenate([qs, iq]))[:, j0:j0 + 8, i0:i0 + 8]
    f_o = O.spread(p, d, ps[c_o], qs[c_o])[:, j0:j0 + 8, i0:i0 + 8]
    r = solve(p, pos, q, dp.DPSE_FP64, stages=(dp.Stage.F_I, dp.Stage.F_O))
    g_i = r[dp.Stage.F_I][:, j0:j0 + 8, i0:i0 + 8]
    g_o = r[dp.Stage.F_O][:, j0:j0 + 8, i0:i0 + 8]
    ei = np.abs(g_i - f_i).max() / np.abs(f_i).max()
    eo = np.abs(g_o - f_o).max() / max(np.abs(f_o).max(), 1e-300)
    print(f"[large] spread sample: f_i max rel err {ei:.2e}, f_o {eo:.2e}", flush=True)
    assert ei < 1e-12 and eo < 1e-12


def test_large_mirror_and_translation(large):
    """Exact invariances of the discrete method: z -> H - z with eps_b <-> eps_t
    flips F_z and keeps F_x, F_y; a shift by whole grid cells in x and y keeps
    F and U (phi moves by the gauge constant only)."""
    import paper_2101_07088_amd as dp
    p, pos, q, r64 = large
    pm = p.copy(eps_b=p.eps_t, eps_t=p.eps_b)
    posm = pos.copy()
    posm[:, 2] = p.H - pos[:, 2]
    rm = solve(pm, posm, q, dp.DPSE_FP64)
    assert rm["status"] == 0
    Fm = rm["F"] * np.array([1.0, 1.0, -1.0])
    e_mirror = rel_rms(Fm, r64["F"])
    h = p.Lx / p.Nx
    post = pos.copy()
    post[:, 0] = (pos[:, 0] + 3 * h) % p.Lx
    post[:, 1] = (pos[:, 1] + 5 * h) % p.Ly
    rt = solve(p, post, q, dp.DPSE_FP64)
    assert rt["status"] == 0
    e_tr = rel_rms(rt["F"], r64["F"])
    dphi = rt["phi"] - r64["phi"]
    print(f"[large] mirror F {e_mirror:.2e}; translation F {e_tr:.2e}, U {abs(rt['U'] - r64['U']) / abs(r64['U']):.2e}, "
          f"phi spread {np.ptp(dphi):.2e}", flush=True)
    assert e_mirror < 1e-10 and e_tr < 1e-10
    assert abs(rt["U"] - r64["U"]) < 1e-10 * abs(r64["U"])
    assert np.ptp(dphi) < 1e-9 * np.abs(r64["phi"]).max()


def test_large_divalent_mixed():
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = W.config_large(0, divalent=True)
    print(f"[large] divalent N={len(q)}", flush=True)
    r64 = solve(p, pos, q, dp.DPSE_FP64)
    rm = solve(p, pos, q, dp.DPSE_MIXED)
    assert r64["status"] == 0 and rm["status"] == 0
    eF = rel_rms(rm["F"], r64["F"])
    print(f"[large] divalent mixed vs FP64: relRMS F {eF:.2e}", flush=True)
    assert eF <= 1e-5
