"""dpse_solve_static (the solve with its workspace in the library's static
device array, for callers that cannot allocate) against dpse_solve, both
through the C ABI: two calls in a row on one plan, the second with fewer
charges, for FP64 and mixed precision slabs and the triply periodic variant
(the array keeps each call's contents, so the second call also checks that
everything a solve reads is cleared or rewritten); bitwise equality with
DPSE_DETERMINISTIC; and the refusals (a plan that owns its workspace, a
workspace larger than the array)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def neutral_subset(pos, q, k):
    """The first k positive and the first k negative unit charges."""
    idx = np.concatenate([np.flatnonzero(q > 0)[:k], np.flatnonzero(q < 0)[:k]])
    assert abs(q[idx].sum()) < 1e-12
    return np.ascontiguousarray(pos[idx]), np.ascontiguousarray(q[idx])


def slab(seed, n_pairs, L=16.0, H=8.0, eb=0.05, et=20.0, Nz=33, **kw):
    p = W.SlabParams(Lx=L, Ly=L, H=H, eps=1.0, eps_b=eb, eps_t=et, xi=1.0, Nx=int(L / 0.25), Ny=int(L / 0.25),
                     Nz=Nz, r_cut=3.0, **kw)
    pos, q = W.charges(seed, n_pairs, n_pairs, L, L, 0.5, H - 0.5)
    return p, pos, q


def triply(seed=3, **kw):
    p = W.SlabParams(Lx=16.0, Ly=16.0, H=16.0, eps=1.0, eps_b=1.0, eps_t=1.0, xi=1.0, Nx=64, Ny=64, Nz=64,
                     r_cut=3.0, triply=True, **kw)
    pos, q = W.charges(seed, 150, 150, 16.0, 16.0, 0.0, 16.0)
    return p, pos, q


# (inputs, precision index: 0 FP64, 1 mixed, charges per sign of the second call)
CASES = {
    "small_fp64": (lambda: W.config_small(0), 0, 20),
    "slab_mixed": (lambda: slab(41, 300), 1, 170),
    "slab_fp64": (lambda: slab(42, 300), 0, 110),
    "triply_mixed": (lambda: triply(), 1, 90),
}


def _reference(p, precision, pos, q):
    """The existing entry point, dpse_solve, on a plan with its own workspace."""
    import paper_2101_07088_amd as dp
    plan = dp.Plan(p, max_n=len(q), precision=precision)
    U, phi, F = plan.solve(dev(pos), dev(q))
    st = plan.sync_status()
    out = (st, float(U.cpu()[0]), phi.cpu().numpy(), F.cpu().numpy())
    plan.close()
    return out


def _static(plan, pos, q):
    n = len(q)
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    PH = torch.empty(n, dtype=torch.float64, device="cuda")
    F = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    plan.solve_static(dev(pos), dev(q), E, PH, F)
    st = plan.sync_status()
    return st, float(E.cpu()[0]), PH.cpu().numpy(), F.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_static_matches_solve_twice(name):
    """Two calls in a row, the second with a smaller neutral subset: each
    agrees with dpse_solve on the same inputs (FP64 1e-12, mixed 1e-6: the
    same kernels, up to the order of atomic sums)."""
    _need_gpu()
    import paper_2101_07088_amd as dp
    make, prec_i, k2 = CASES[name]
    p, pos, q = make()
    prec = (dp.DPSE_FP64, dp.DPSE_MIXED)[prec_i]
    bar = 1e-12 if prec == dp.DPSE_FP64 else 1e-6
    plan = dp.Plan(p, max_n=len(q), precision=prec, own_workspace=False)
    assert plan.info["workspace_bytes"] <= dp.native.STATIC_SCRATCH_BYTES
    calls = [(pos, q), neutral_subset(pos, q, k2)]
    assert len(calls[1][1]) < len(calls[0][1])
    for i, (ps, qs) in enumerate(calls):
        print(f"[no_alloc] {name} call {i}: n={len(qs)}", flush=True)
        st, U, phi, F = _static(plan, ps, qs)
        st0, U0, phi0, F0 = _reference(p, prec, ps, qs)
        assert st == 0 and st0 == 0, (st, st0)
        ef, ep = rel_rms(F, F0), rel_rms(phi, phi0)
        eu = abs(U - U0) / (0.5 * float(np.sum(np.abs(qs * phi0))))
        print(f"[no_alloc] {name} call {i}: force {ef:.2e} phi {ep:.2e} energy {eu:.2e}", flush=True)
        assert ef <= bar and ep <= bar and eu <= bar, (ef, ep, eu)
    plan.close()


def test_static_bitwise_deterministic():
    """With DPSE_DETERMINISTIC both entry points give the same output bits,
    on two calls in a row (the second smaller)."""
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = slab(43, 300, deterministic=True)
    for prec in (dp.DPSE_FP64, dp.DPSE_MIXED):
        plan = dp.Plan(p, max_n=len(q), precision=prec, own_workspace=False)
        for ps, qs in ((pos, q), neutral_subset(pos, q, 120)):
            st, U, phi, F = _static(plan, ps, qs)
            st0, U0, phi0, F0 = _reference(p, prec, ps, qs)
            assert st == 0 and st0 == 0
            assert U == U0 and np.array_equal(phi, phi0) and np.array_equal(F, F0)
        plan.close()


def test_static_refusals():
    """A plan owning its workspace, and a workspace beyond the static array
    (the 16384-ion jump workload: 426 MB), are refused before any launch."""
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = W.config_small(0)
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    PH = torch.empty(len(q), dtype=torch.float64, device="cuda")
    F = torch.empty((len(q), 3), dtype=torch.float64, device="cuda")
    own = dp.Plan(p, max_n=len(q))
    with pytest.raises(dp.DpseError) as ex:
        own.solve_static(dev(pos), dev(q), E, PH, F)
    assert ex.value.status == 1
    own.close()
    pj, posj, qj = W.config_jump(0)
    big = dp.Plan(pj, max_n=len(qj), precision=dp.DPSE_MIXED, own_workspace=False)
    assert big.info["workspace_bytes"] > dp.native.STATIC_SCRATCH_BYTES
    Ej = torch.empty(1, dtype=torch.float64, device="cuda")
    PHj = torch.empty(len(qj), dtype=torch.float64, device="cuda")
    Fj = torch.empty((len(qj), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(dp.DpseError) as ex:
        big.solve_static(dev(posj), dev(qj), Ej, PHj, Fj)
    assert ex.value.status == dp.native.DPSE_ESCRATCH
    big.close()
