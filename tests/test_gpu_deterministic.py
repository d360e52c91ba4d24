"""DPSE_DETERMINISTIC: bitwise-reproducible solves through the C ABI.

Two solves of the same inputs (on one plan, on two plans, and with other
solves running on the device between and beside them) give identical output
bits, in FP64 and mixed precision, for the slab solver (with and without wall
charges), the small grid where only the scatter forms fit otherwise, and the
triply periodic variant; the deterministic path also matches the FP64 oracle
at the parity bar, stage by stage where the stage is a plain definition."""
import numpy as np
import pytest

import workloads as W
from oracle import dpse_oracle as O
from oracle import tp_oracle as TPO

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_rms(a, b):
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def jump(seed, n_pairs, L=16.0, H=8.0, eb=0.05, et=20.0, Nz=33):
    p = W.SlabParams(Lx=L, Ly=L, H=H, eps=1.0, eps_b=eb, eps_t=et, xi=1.0, Nx=int(L / 0.25), Ny=int(L / 0.25),
                     Nz=Nz, r_cut=3.0, deterministic=True)
    pos, q = W.charges(seed, n_pairs, n_pairs, L, L, 0.5, H - 0.5)
    return p, pos, q


def triply(seed=3):
    p = W.SlabParams(Lx=16.0, Ly=16.0, H=16.0, eps=1.0, eps_b=1.0, eps_t=1.0, xi=1.0, Nx=64, Ny=64, Nz=64,
                     r_cut=3.0, triply=True, deterministic=True)
    pos, q = W.charges(seed, 150, 150, 16.0, 16.0, 0.0, 16.0)
    pos[:4, 2] = [0.05, 15.97, 0.6, 15.4]   # charges near both ends of the period
    return p, pos, q


CASES = {
    "jump": lambda: jump(31, 300),
    "small": lambda: (W.config_small(0)[0].copy(deterministic=True),) + W.config_small(0)[1:],
    "triply": triply,
}


def _solve(plan, pos, q, stages=()):
    import paper_2101_07088_amd as dp
    U, phi, F = plan.solve(dev(pos), dev(q))
    assert plan.sync_status() == 0
    out = [float(U.cpu()[0]), phi.cpu().numpy(), F.cpu().numpy()]
    out.append({s: plan.debug(s) for s in stages})
    return out


def _same(a, b):
    return a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_bitwise_repeatable(name, precision):
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = CASES[name]()
    print(f"[det] case={name} prec={precision} N={len(q)} grid={p.Nx}x{p.Ny}x{p.Nz}", flush=True)
    plan_a = dp.Plan(p, max_n=len(q), precision=precision)
    r1 = _solve(plan_a, pos, q, stages=(dp.Stage.F_I, dp.Stage.FAR, dp.Stage.NEAR))
    # other work on the device: a different system solved on another stream,
    # concurrently with the next solve
    other_p, other_pos, other_q = jump(32, 500, L=32.0, H=12.0, eb=1.0, et=0.05, Nz=65)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan_o = dp.Plan(other_p.copy(deterministic=False), max_n=len(other_q), precision=precision)
        for _ in range(3):
            plan_o.solve(dev(other_pos), dev(other_q))
    r2 = _solve(plan_a, pos, q, stages=(dp.Stage.F_I, dp.Stage.FAR, dp.Stage.NEAR))
    side.synchronize()
    assert plan_o.sync_status() == 0
    plan_b = dp.Plan(p, max_n=len(q) + 7, precision=precision)
    r3 = _solve(plan_b, pos, q, stages=(dp.Stage.F_I, dp.Stage.FAR, dp.Stage.NEAR))
    assert _same(r1, r2) and _same(r1, r3)
    for s in r1[3]:
        assert np.array_equal(r1[3][s], r2[3][s]) and np.array_equal(r1[3][s], r3[3][s]), s
    # and the deterministic path is the method: parity with the oracle
    if name == "triply":
        U0, phi0, F0, _ = TPO.solve_tp(p, pos, q)
    else:
        U0, phi0, F0, _ = O.solve(p, pos, q)
    bar = 1e-9 if precision == 0 else 1e-5
    eF = rel_rms(r1[2], F0)
    print(f"[det] {name} prec={precision}: relRMS F vs oracle {eF:.2e}", flush=True)
    assert eF < bar and rel_rms(r1[1], phi0) < bar
    assert abs(r1[0] - U0) < bar * 0.5 * np.sum(np.abs(q * phi0))
    for pl in (plan_a, plan_b, plan_o):
        pl.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_bitwise_repeatable_with_walls(precision):
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = jump(33, 200)
    sb, st = W.gaussian_walls(p, 2.0)
    walls = (dev(3.0 * sb), dev(3.0 * st))   # +3 on the bottom wall, -3 on the top
    plans = [dp.Plan(p, max_n=len(q), precision=precision) for _ in range(2)]
    res = []
    for pl in plans:
        pl.set_walls(*walls)
        res.append(_solve(pl, pos, q))
        res.append(_solve(pl, pos, q))
    assert all(_same(res[0], r) for r in res[1:])
    U0, phi0, F0, _ = O.solve(p, pos, q, sigma_b=3.0 * sb, sigma_t=3.0 * st)
    bar = 1e-9 if precision == 0 else 1e-5
    assert rel_rms(res[0][2], F0) < bar
    assert abs(res[0][0] - U0) < bar * 0.5 * np.sum(np.abs(q * phi0))
    for pl in plans:
        pl.close()


def test_deterministic_matches_default_path():
    """Same method, other summation order: FP64 results agree to rounding,
    and the spread grid (a plain sum) and the near field stage match the
    oracle's at 1e-12."""
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = jump(34, 250)
    r_det = _solve(dp.Plan(p, max_n=len(q)), pos, q, stages=(dp.Stage.F_I, dp.Stage.NEAR, dp.Stage.FAR))
    r_def = _solve(dp.Plan(p.copy(deterministic=False), max_n=len(q)), pos, q)
    assert rel_rms(r_det[2], r_def[2]) < 1e-13
    _, _, _, inter = O.solve(p, pos, q)
    assert rel_max(r_det[3][dp.Stage.F_I], inter["f_i"]) < 1e-12
    assert rel_max(r_det[3][dp.Stage.NEAR][: len(q)], inter["near"]) < 1e-12
    assert rel_max(r_det[3][dp.Stage.FAR][: len(q)], inter["far"]) < 1e-11
