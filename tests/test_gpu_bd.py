"""GPU tests of the Brownian-dynamics pieces against the oracle: the step
kernel of eq. leimkuhler (Sec. 7), the near-field-only solve that reuses the
last full solve's far field, and a short driven trajectory replayed on the
CPU with the same noise."""
import numpy as np
import pytest

import workloads as W
from oracle import bd as OB
from oracle import dpse_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def system(seed=8, n_pairs=80):
    p = W.SlabParams(Lx=16.0, Ly=16.0, H=8.0, eps=1.0, eps_b=0.05, eps_t=20.0, xi=1.0, Nx=64, Ny=64, Nz=33,
                     r_cut=3.0, g_w=0.1)
    pos, q = W.charges(seed, n_pairs, n_pairs, 16.0, 16.0, 1.0, 7.0)
    return p, pos, q


def test_bd_step_matches_oracle():
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = system()
    plan = dp.Plan(p, max_n=len(q))
    rng = np.random.default_rng(1)
    F = rng.normal(size=pos.shape)
    wp, wn = rng.normal(size=pos.shape), rng.normal(size=pos.shape)
    out = torch.empty((len(q), 3), dtype=torch.float64, device="cuda")
    esc = torch.zeros(1, dtype=torch.int32, device="cuda")
    for mu_dt, noise in ((1e-3, 0.02), (0.5, 2.0)):   # the second pushes charges out of the slab
        tp = dev(pos)
        plan.bd_step(tp, dev(F), dev(wp), dev(wn), mu_dt, noise, out, esc)
        torch.cuda.synchronize()
        new, bad = OB.leimkuhler_step(pos, F, wp, wn, 1.0, mu_dt, 2.0 * noise ** 2 / mu_dt,
                                      z_lo=4 * p.g_w, z_hi=p.H - 4 * p.g_w)
        assert np.abs(out.cpu().numpy() - new).max() < 1e-14 * np.abs(new).max()
        n_out = int(np.sum(~((new[:, 2] > 4 * p.g_w) & (new[:, 2] < p.H - 4 * p.g_w))))
        assert int(esc.item()) == n_out and bad == (n_out > 0)
        print(f"[case] bd step mu_dt={mu_dt}: escaped {n_out}", flush=True)
    with pytest.raises(dp.DpseError):   # pos_out must not alias pos
        plan.bd_step(tp, dev(F), dev(wp), dev(wn), 1e-3, 0.02, tp, esc)
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-5)])
def test_solve_near_reuses_the_last_far_field(precision, tol):
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = system(seed=9)
    plan = dp.Plan(p, max_n=len(q), precision=precision)
    tq = dev(q)
    with pytest.raises(dp.DpseError):     # nothing to reuse yet
        plan.solve_near(dev(pos), tq)
    plan.solve(dev(pos), tq)
    assert plan.sync_status() == 0
    _, _, _, I = O.solve(p, pos, q)
    moved = pos + np.random.default_rng(2).normal(0.0, 0.03, pos.shape)
    U, phi, F = plan.solve_near(dev(moved), tq)
    assert plan.sync_status() == 0
    U0, phi0, F0 = OB.near_reuse(p, moved, q, I)
    eF, ep = rel_rms(F.cpu().numpy(), F0), rel_rms(phi.cpu().numpy(), phi0)
    eU = abs(float(U.cpu()[0]) - U0) / (0.5 * np.sum(np.abs(q * phi0)))
    print(f"[case] solve_near prec={precision}: F {eF:.2e} phi {ep:.2e} U {eU:.2e}", flush=True)
    assert eF < tol and ep < tol and eU < tol
    # a second reuse from the same full solve, and refusals
    U2, _, F2 = plan.solve_near(dev(pos), tq)
    assert plan.sync_status() == 0
    Uf, _, Ff, _ = O.solve(p, pos, q)
    assert rel_rms(F2.cpu().numpy(), Ff) < tol
    with pytest.raises(dp.DpseError):     # another n
        plan.solve_near(dev(pos[:-2]), dev(q[:-2]))
    sb, st = W.gaussian_walls(p, 2.0)
    plan.set_walls(dev(sb), dev(st))
    with pytest.raises(dp.DpseError):     # the walls changed the far field
        plan.solve_near(dev(pos), tq)
    plan.close()


def test_driven_trajectory_matches_oracle_replay():
    """Seven steps with a full solve every third step: the driver's positions
    equal a CPU replay (oracle forces, oracle step) with the same noise."""
    _need_gpu()
    import paper_2101_07088_amd as dp
    from paper_2101_07088_amd.bd import BrownianDynamics
    p, pos, q = system(seed=10, n_pairs=40)
    plan = dp.Plan(p, max_n=len(q))
    mu, kT, dt = 1.0, 1.0, 2e-3
    drv = BrownianDynamics(plan, dev(pos), dev(q), mu, kT, dt, far_every=3, seed=5)
    noise = [drv.w_prev.cpu().numpy()]
    for _ in range(7):
        drv.step()
        noise.append(drv.w_prev.cpu().numpy())
    gpu_pos = drv.pos.cpu().numpy()
    x = pos.copy()
    last = None
    for s in range(7):
        if s % 3 == 0:
            _, _, F, last = O.solve(p, x, q)
        else:
            _, _, F = OB.near_reuse(p, x, q, last)
        x, bad = OB.leimkuhler_step(x, F, noise[s], noise[s + 1], mu, dt, kT, z_lo=4 * p.g_w,
                                    z_hi=p.H - 4 * p.g_w)
        assert not bad
    err = np.abs(gpu_pos - x).max()
    print(f"[case] bd trajectory: 7 steps, {drv.full_solves} full solves, {drv.retries} retries, "
          f"max |dx| {err:.2e}", flush=True)
    assert drv.full_solves == 3 and err < 1e-10
    plan.close()
