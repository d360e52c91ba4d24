"""GPU parity of the triply periodic variant (DPSE_TRIPLY) with its FP64
oracle: a cubic box and one with a different z spacing, charges near both
ends of the z period (the periodic copies), heights given outside the period
(wrapped), FP64 at 1e-9 and mixed at 1e-5; and the paper's triply periodic
performance workload at full size on sampled charges."""
import numpy as np
import pytest

import workloads as W
from oracle import tp_oracle as T

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def gpu(p, pos, q, precision):
    import paper_2101_07088_amd as dp
    plan = dp.Plan(p, max_n=len(q), precision=precision)
    U, phi, F = plan.solve(dev(pos), dev(q))
    st = plan.sync_status()
    plan.close()
    return st, float(U.cpu()[0]), phi.cpu().numpy(), F.cpu().numpy()


def boxes():
    out = []
    p = W.SlabParams(Lx=16.0, Ly=16.0, H=16.0, eps=1.0, eps_b=1.0, eps_t=1.0, xi=1.4, Nx=64, Ny=64, Nz=64,
                     r_cut=3.0, triply=True)
    pos, q = W.charges(21, 200, 200, 16.0, 16.0, 0.0, 16.0)
    pos[:20, 2] = np.linspace(0.0, 0.6, 20)          # near z = 0: copies at z + Lz
    pos[20:40, 2] = np.linspace(15.4, 15.999, 20)    # near z = Lz: copies at z - Lz
    out.append(("cubic 64^3", p, pos, q))
    p2 = p.copy(H=24.0, Nz=64, eps=2.5, eps_b=2.5, eps_t=2.5)   # h_z = 0.375, h = 0.25
    pos2, q2 = W.charges(22, 150, 150, 16.0, 16.0, 0.0, 24.0)
    out.append(("64^2 x 64, h_z 0.375", p2, pos2, q2))
    return out


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-5)])
def test_triply_matches_oracle(precision, tol):
    _need_gpu()
    for label, p, pos, q in boxes():
        U0, phi0, F0, _ = T.solve_tp(p, pos, q)
        st, U, phi, F = gpu(p, pos, q, precision)
        assert st == 0
        eF, ep = rel_rms(F, F0), rel_rms(phi, phi0)
        eU = abs(U - U0) / (0.5 * np.sum(np.abs(q * phi0)))
        print(f"[case] triply {label} prec={precision}: F {eF:.2e} phi {ep:.2e} U {eU:.2e}", flush=True)
        assert eF < tol and ep < tol and eU < tol
        # heights outside the period are wrapped
        shifted = pos + np.array([0.0, 0.0, 3.0 * p.H])
        shifted[::2, 2] -= 5.0 * p.H
        st2, U2, phi2, F2 = gpu(p, shifted, q, precision)
        assert st2 == 0 and rel_rms(F2, F) < 1e-12 + (0 if precision == 0 else 1e-6)


def test_triply_paper_workload_sampled():
    """N = 2 x 10^4 in 185 x 185 x 100, 64^2 x 32, mixed and FP64: the far
    field of every charge and the near field of every 40th charge against the
    oracle."""
    _need_gpu()
    import paper_2101_07088_amd as dp
    p, pos, q = W.config_triply(0)
    sel = np.arange(0, len(q), 40)
    _, phi0, F0, I = T.solve_tp(p, pos, q, near_targets=sel)
    for precision, tol in ((0, 1e-9), (1, 1e-5)):
        plan = dp.Plan(p, max_n=len(q), precision=precision)
        U, phi, F = plan.solve(dev(pos), dev(q))
        assert plan.sync_status() == 0
        far = plan.debug(dp.Stage.FAR)[: len(q)]
        ef = rel_rms(far[:, 1:], I["far"][:, 1:])
        eF = rel_rms(F.cpu().numpy()[sel], F0)
        ep = rel_rms(phi.cpu().numpy()[sel], phi0)
        print(f"[case] triply paper workload prec={precision}: far field {ef:.2e}, sampled F {eF:.2e} phi {ep:.2e}",
              flush=True)
        assert ef < tol and eF < tol and ep < tol
        plan.close()
