"""Benchmark: charge-force evaluations per second of the DP-SE far+near solve.

One step = one complete solve (all stages: validation and binning, spreading,
forward transforms, the per-mode column solve with the harmonic correction,
inverse transforms, interpolation, near field, gauge and energy) of the large
slab workload: N = 1,048,576 monovalent ions in Lx = Ly = 256, H = 64, eps = 1
inside, eps_b = 0.05 below, eps_t = 20 above, xi = 1.5, grid 1024 x 1024 x 257,
near cutoff 2. Positions and charges are resident in HBM before the timed
region.

The headline path is the mixed-precision one (FP32 grid stages, FP64
per-mode solves and per-charge sums) when its relative RMS force error
against the FP64 path on the same charges is <= 1e-5; otherwise the FP64
path. Secondary lines: the 16,384-ion jump workload (256 x 256 x 129) in
both precisions (accuracy over seeds 0-4), the 64-charge small workload
(eager against graph launches), and the optional variant, batch and serving
measurements. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def stage_bytes(p, beta, s):
    """Algorithmic HBM bytes per launch of each grid stage: every stage-boundary
    array read once and written once (G grid points, C half-spectrum reals,
    beta the fraction of Chebyshev nodes where the wall-group grid can be
    non-zero, s bytes per real)."""
    G = p.Nz * p.Ny * p.Nx
    Cr = 2 * p.Nz * p.Ny * (p.Nx // 2 + 1)
    return {
        "spread": (1 + beta) * G * s,
        "fft_forward": (1 + beta) * (G + Cr) * s,
        "column": (3 + beta) * Cr * s,
        "fft_inverse": (2 * Cr + 4 * G) * s,
        "interp": 4 * G * s,
    }


SPREAD_SHAPES = [(32, 4), (32, 8), (16, 4), (16, 8), (32, 2), (16, 2), (16, 8), (16, 4), (32, 8), (32, 4), (16, 16),
                 (32, 16)]
INTERP_SHAPES = [(16, 4), (16, 8), (32, 2), (32, 4), (16, 2), (16, 8), (16, 4), (0, 0)]
COLUMN_SHAPES = [(2048, 256), (1024, 256), (4096, 256), (2048, 512), (4096, 512), (2048, 256)]  # (KE, threads)


def kernel_name(stage, tiles, mixed, p, support):
    """Name (as rocprofv3 prints it, spaces removed) of the single kernel of a
    grid stage for the tuned launch shapes, or None for multi-kernel stages."""
    r = "float" if mixed else "double"
    if stage == "spread":
        i = tiles[0]
        t, pz = SPREAD_SHAPES[i]
        return f"k_spread{'_gather' if i >= 6 else ''}<{r},{t},{pz}>"
    if stage == "interp":
        i = tiles[1]
        if i == 7:   # one wave per charge in bin order (columns in 4 passes of 64 lanes for n_g <= 16)
            c, gn = (4, 4 if mixed else 2) if support * support <= 256 else (16, 1)
            return f"k_interp_wave<{r},{c},{gn}>"
        t, pz = INTERP_SHAPES[i]
        # the gather shapes carry the wall-term switch (off on this workload)
        return f"k_interp_gather<{r},{t},{pz},false>" if i >= 5 else f"k_interp<{r},{t},{pz}>"
    if stage == "column":
        if tiles[2] == 5:   # the segmented-scan kernel of the grids with Nz <= 257
            return f"k_column_scan<{r},{int(math.log2((p.Nz - 1) // 8))}>"
        ke, nt = COLUMN_SHAPES[tiles[2]]
        return f"k_column<{r},{ke},{nt}>"
    return None


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload, or None when there is none or a kernel source
    has changed since the counters were taken."""
    import glob
    import hashlib
    if kernel is None:
        return None
    files = glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_large_*.txt"))
    if not files:
        return None
    src = os.path.join(ROOT, "paper_2101_07088_amd", "csrc")
    found = None
    for line in open(files[0]):
        f = line.split()
        if len(f) == 3 and f[0] == "source_sha256":
            if hashlib.sha256(open(os.path.join(src, f[1]), "rb").read()).hexdigest()[:16] != f[2]:
                return None
        elif len(f) >= 10 and f[0] == "kernel" and f[1] == kernel:
            found = float(f[9])
    return found


def band_fraction(p, info):
    """Fraction of the Chebyshev nodes in the wall bands, where the spread of
    the wall group can be non-zero: H - 3 H_E < z <= H + H_E and
    -H_E <= z < 3 H_E (charges of the group lie within 2 H_E of a wall and
    reach nodes within H_E of them)."""
    z = [0.5 * (info["z_lo"] + info["z_hi"]) + 0.5 * (info["z_hi"] - info["z_lo"]) * math.cos(math.pi * j / (p.Nz - 1))
         for j in range(p.Nz)]
    he = info["H_E"]
    if getattr(p, "uniform_fast", False) or getattr(p, "one_jump", False) or getattr(p, "triply", False):
        return 0.0
    return sum(1 for zz in z if (p.H - 3 * he < zz <= p.H + he) or (-he <= zz < 3 * he)) / p.Nz


def time_path(dp, torch, p, tpos, tq, precision, steps, warmup, walls=None, live_stages=False, latency_solves=0):
    """Plan, autotune (outside the timed region), warm up, then time `steps`
    solves back to back. With live_stages the library's per-stage HIP events
    are recorded on the plan's stream during the timed region itself (their
    cost is negligible next to a solve of the large workload); otherwise in a
    separate pass of the same solves. latency_solves > 0 adds a pass of that
    many solves, each bracketed by its own events (p50/p99)."""
    plan = dp.Plan(p, max_n=len(tq), precision=precision)
    if walls is not None:
        plan.set_walls(*walls)
    tiles, tile_ms = plan.autotune(tpos, tq, reps=3)   # plan-time tuning, outside the timed region
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    PH = torch.empty(len(tq), dtype=torch.float64, device="cuda")
    F = torch.empty((len(tq), 3), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        plan.solve(tpos, tq, E, PH, F)
    plan.sync()
    if live_stages:
        plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        plan.solve(tpos, tq, E, PH, F)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = plan.sync_status()
    if live_stages:
        stages, _ = plan.stage_times()
        plan.set_timing(False)
    else:
        plan.set_timing(True)
        for _ in range(steps):
            plan.solve(tpos, tq, E, PH, F)
        stages, _ = plan.stage_times()
        plan.set_timing(False)
    # per-solve latency with events on the plan's (= current) stream
    nl = latency_solves or steps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nl)]
    torch.cuda.synchronize()
    for k in range(nl):
        evs[k][0].record()
        plan.solve(tpos, tq, E, PH, F)
        evs[k][1].record()
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    plan.sync()
    out = dict(wall_s=wall, lat_ms=lat, stages=stages, status=st, U=float(E.cpu()[0]), tiles=tiles, tile_ms=tile_ms,
               phi=PH.cpu().numpy(), F=F.cpu().numpy(), far=plan.debug(dp.Stage.FAR)[: len(tq)], info=plan.info,
               workspace_bytes=plan.info["workspace_bytes"])
    plan.close()
    del E, PH, F
    torch.cuda.empty_cache()
    return out


def cpu_baseline(p, pos, q, seed=0):
    """The FP64 CPU oracle (as written, untuned) timed on bounded samples of
    the same workload, each stage's cost scaled to the whole solve:
      * groups and images of every charge (whole);
      * spreading and interpolation: the per-charge cost from two sample
        sizes (the difference cancels the fixed cost of the full grids),
        times the charges each stage visits, plus the one-time grid clear;
      * the x,y transforms on a slab of z planes, times the planes of the
        two forward and four inverse transforms;
      * the z transforms, the per-mode dense solves, the wall values, the
        correction and the node evaluations on one block of 512 modes, times
        the blocks;
      * the near field on 64 targets (all pairs with every charge and image),
        times N / 64.
    Returns the estimated evaluations per second of a full solve."""
    from oracle import dpse_oracle as O
    rng = np.random.default_rng(seed)
    n = len(q)
    d = O.derive(p)
    tm = {}
    T0 = time.perf_counter()
    t0 = time.perf_counter()
    c_o, ipos, iq = O.groups_and_images(p, d, pos, q)
    tm["groups"] = time.perf_counter() - t0

    def per_item(fn, m1, m2):
        a = time.perf_counter(); fn(m1); t1 = time.perf_counter() - a
        a = time.perf_counter(); fn(m2); t2 = time.perf_counter() - a
        return max(t2 - t1, 0.0) / (m2 - m1), max(t1 - (t2 - t1) * m1 / (m2 - m1), 0.0)

    sel = rng.choice(n, 2000, replace=False)
    c_spread, fix_spread = per_item(lambda m: O.spread(p, d, pos[sel[:m]], q[sel[:m]]), 400, 2000)
    tm["spread"] = 2 * fix_spread + c_spread * (int(np.count_nonzero(c_o)) + n + len(iq))
    grids = np.zeros((4, p.Nz, p.Ny, p.Nx))   # lazily zeroed pages; only the windows are touched
    c_interp, _ = per_item(lambda m: O.interp(p, d, grids, pos[sel[:m]]), 200, 1000)
    tm["interp"] = c_interp * n
    del grids
    planes = 8
    f = rng.standard_normal((planes, p.Ny, p.Nx))
    a = time.perf_counter(); F = O.fft_xy(f, p); t = time.perf_counter() - a
    a = time.perf_counter(); O.ifft_xy(F, p); ti = time.perf_counter() - a
    tm["fft_xy"] = (2 * t + 4 * ti) * p.Nz / planes
    nm_all = p.Ny * (p.Nx // 2 + 1)
    blk = 512
    ms = rng.choice(nm_all, blk, replace=False)
    Fi = (rng.standard_normal((p.Nz, 1, blk)) + 1j * rng.standard_normal((p.Nz, 1, blk)))
    a = time.perf_counter()
    fh_i = O.cheb_coeffs(Fi)
    fh_o = O.cheb_coeffs(Fi)
    tm["cheb"] = (time.perf_counter() - a) * nm_all / blk
    sub = dict(d)
    sub["kabs"] = d["kabs"].ravel()[ms].reshape(1, blk)
    pb = p.copy(Ny=1, Nx=2 * (blk - 1))   # the shape solve_modes reshapes to: [Nz, 1, blk]
    a = time.perf_counter()
    y_o, y_i = O.solve_modes(pb, sub, [fh_o, fh_i])
    tm["bvp"] = (time.perf_counter() - a) * nm_all / blk
    a = time.perf_counter()
    R = d["R"]
    s0, sH = (0.0 - d["c"]) / R, (p.H - d["c"]) / R
    vals = [O.series_at(y, s) for y in (y_o, y_i) for s in (s0, sH)]
    ders = [O.series_dz_at(y, s, R) for y in (y_o, y_i) for s in (s0, sH)]
    kk = sub["kabs"][0]
    pos_k = kk > 0.0
    O.correction_coeffs(p, kk[pos_k], (vals[2][0] - vals[0][0])[pos_k], (ders[2][0] - ders[0][0])[pos_k],
                        (vals[3][0] - vals[1][0])[pos_k], (ders[3][0] - ders[1][0])[pos_k])
    from numpy.polynomial import chebyshev as npcheb
    O.cheb_eval_nodes(y_i, p.Nz)
    O.cheb_eval_nodes(npcheb.chebder(y_i, axis=0), p.Nz)
    tm["modes_rest"] = (time.perf_counter() - a) * nm_all / blk
    tt = rng.choice(n, 64, replace=False)
    a = time.perf_counter()
    O.near_field(p, d, pos, q, targets=tt)
    tm["near"] = (time.perf_counter() - a) * n / len(tt)
    sampled = time.perf_counter() - T0
    total = sum(tm.values())
    try:
        import threadpoolctl
        blas = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except Exception:
        blas = 1
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n / total, "unit": "charge-force evals/s", "cores": int(blas), "kind": "oracle",
            "cpu_model": cpu, "host_cpus": os.cpu_count(),
            "sample": (f"FP64 oracle on samples of the large workload ({sampled:.1f} s of CPU work): spreading of "
                       f"400 and 2000 charges and interpolation of 200 and 1000 (per-charge cost from the "
                       f"difference), x,y "
                       f"transforms of {planes} planes, z transforms + dense per-mode solves + correction + node "
                       f"evaluation of {blk} modes, near field of 64 targets; each scaled to the whole solve "
                       f"(estimated {total:.0f} s per solve; BLAS threads {blas}, FFT and loops single-threaded)"),
            "stage_estimate_s": {k: round(v, 2) for k, v in tm.items()}}


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def bench_batch(dp, torch, steps, n_sys=64, n_branches=8):
    """Uneven batch: 64 independent slabs (N log-uniform in [1024, 65536],
    L in {32,64,128}, H in {16,32,64}, eps_b, eps_t in {0.05,1,20}, xi=1.5,
    h=0.25, r_cut=2), mixed precision, one graph launch per step; against
    the same 64 solves one after another on one stream without a graph, in
    mixed precision and in FP64 (the plain single-system path)."""
    import workloads as W
    from paper_2101_07088_amd.batch import BatchRunner
    systems = W.batch_systems(n_sys)
    tens = [(p, torch.tensor(pos, dtype=torch.float64, device="cuda"),
             torch.tensor(q, dtype=torch.float64, device="cuda")) for p, pos, q in systems]
    n_total = sum(len(q) for _, _, q in systems)
    out = {"systems": n_sys, "charges": n_total, "branches": n_branches}

    def timed(runner, k):
        runner.run()
        torch.cuda.synchronize()
        st = runner.statuses()
        assert all(x == 0 for x in st), st
        t0 = time.perf_counter()
        for _ in range(k):
            runner.run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    seq = BatchRunner(tens, precision=dp.DPSE_MIXED, n_branches=1, use_graph=False)
    t_seq = timed(seq, max(2, steps // 4))
    seq.close()
    del seq
    seq64 = BatchRunner(tens, precision=dp.DPSE_FP64, n_branches=1, use_graph=False)
    t_seq64 = timed(seq64, max(2, steps // 4))
    seq64.close()
    del seq64
    out.update({"sequential_fp64_evals_per_s": n_total / t_seq64, "sequential_fp64_ms": 1e3 * t_seq64})
    br = BatchRunner(tens, precision=dp.DPSE_MIXED, n_branches=n_branches, use_graph=True)
    t_b = timed(br, steps)
    grid_points = sum(p.Nx * p.Ny * p.Nz for p, _, _ in systems)
    out.update({"grid_points": grid_points, "grid_points_per_s": grid_points / t_b,
                "evals_per_s": n_total / t_b, "ms_per_batch": 1e3 * t_b,
                "sequential_evals_per_s": n_total / t_seq, "sequential_ms": 1e3 * t_seq,
                "speedup_vs_sequential": t_seq / t_b, "speedup_vs_sequential_fp64": t_seq64 / t_b,
                "arena_bytes": br.workspace_bytes})
    # accuracy of the mixed batch against FP64 single solves on a sample of systems
    errs = []
    for k in range(0, n_sys, 16):
        p, tp, tq = tens[k]
        pl = dp.Plan(p, max_n=int(tq.shape[0]), precision=dp.DPSE_FP64)
        U, phi, F = pl.solve(tp, tq)
        pl.sync()
        errs.append(rel_rms(br.force[k].cpu().numpy(), F.cpu().numpy()))
        pl.close()
    out["mixed_vs_fp64_rel_rms_force_max"] = max(errs)
    out["accuracy_sample"] = f"systems {list(range(0, n_sys, 16))}"
    br.close()
    return out


def bench_uniform(dp, torch, steps):
    """The jump workload's charges and box with equal permittivities (eps_b =
    eps_t = eps = 1), mixed precision: the general solver on 256^2 x 129
    against the uniform-permittivity solver on 256^2 x 65 (its smaller z
    domain needs about half the nodes for the same accuracy) and on 256^2 x
    129; the force difference between them is the method error."""
    import workloads as W
    p, pos, q = W.config_jump(0)
    pu = p.copy(eps_b=1.0, eps_t=1.0)
    tpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    out = {}
    forces = {}
    for name, prm in (("general_Nz129", pu), ("fast_Nz65", pu.copy(uniform_fast=True, Nz=65)),
                      ("fast_Nz129", pu.copy(uniform_fast=True))):
        r = time_path(dp, torch, prm, tpos, tq, dp.DPSE_MIXED, steps, 3)
        out[name] = {"ms": 1e3 * r["wall_s"] / steps, "evals_per_s": len(q) / (r["wall_s"] / steps)}
        forces[name] = r["F"]
    ref = forces["general_Nz129"]
    for name in ("fast_Nz65", "fast_Nz129"):
        out[name]["rel_rms_force_vs_general"] = rel_rms(forces[name], ref)
    out["speedup_fast_Nz65"] = out["general_Nz129"]["ms"] / out["fast_Nz65"]["ms"]
    return out


def bench_one_jump(dp, torch, steps):
    """A thin slab with a jump at the bottom wall only: the jump workload's
    density and grid spacing in a 64 x 64 x 5 box (N = 2560, eps_b = 0.05,
    eps_t = eps = 1), mixed precision. The general solver on [-3 H_E, H + 3 H_E]
    (length 18.5) and the one-jump solver on [-H - H_E, H + H_E] (length 14.5)
    at N_z = 33 and 65, against the general solver at N_z = 129 in FP64 (the
    converged reference)."""
    import workloads as W
    p, pos, q = W.scaled_jump(0, 64.0, 5.0, 1280, eps_b=0.05, eps_t=1.0, Nz=65)
    tpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    ref = time_path(dp, torch, p.copy(Nz=129), tpos, tq, dp.DPSE_FP64, 3, 1)["F"]
    out = {"n": len(q)}
    for nz in (33, 65):
        for name, prm in ((f"general_Nz{nz}", p.copy(Nz=nz)), (f"one_jump_Nz{nz}", p.copy(Nz=nz, one_jump=True))):
            r = time_path(dp, torch, prm, tpos, tq, dp.DPSE_MIXED, steps, 3)
            out[name] = {"ms": 1e3 * r["wall_s"] / steps, "evals_per_s": len(q) / (r["wall_s"] / steps),
                         "rel_rms_force_vs_reference": rel_rms(r["F"], ref),
                         "z_domain": [r["info"]["z_lo"], r["info"]["z_hi"]]}
    return out


def bench_bd(dp, torch, steps):
    """Brownian dynamics (Sec. 7, eq. leimkuhler) of the jump workload's
    charges, mixed precision, kT = mu = 1, dt = 1e-3 (about 0.045 per axis
    per step): steps per second (forces, step kernel, the host's check for
    charges leaving the slab) with a full solve every step and with the far
    field reused between full solves every 4 and 16 steps; and the force
    error of the reuse steps against full solves at the same positions."""
    import workloads as W
    from paper_2101_07088_amd.bd import BrownianDynamics
    p, pos, q = W.config_jump(0)
    tpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    out = {"n": len(q), "dt": 1e-3}
    plan = dp.Plan(p, max_n=len(q), precision=dp.DPSE_MIXED)
    plan.autotune(tpos, tq, reps=3)
    for K in (1, 4, 16):
        drv = BrownianDynamics(plan, tpos, tq, 1.0, 1.0, 1e-3, far_every=K, seed=11)
        for _ in range(4):
            drv.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            drv.step()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        out[f"far_every_{K}"] = {"ms_per_step": 1e3 * t, "steps_per_s": 1.0 / t,
                                 "evals_per_s": len(q) / t, "retries": drv.retries}
    # accuracy of the reuse steps
    ref = dp.Plan(p, max_n=len(q), precision=dp.DPSE_MIXED)
    drv = BrownianDynamics(plan, tpos, tq, 1.0, 1.0, 1e-3, far_every=16, seed=12)
    errs = []
    for s in range(32):
        before = drv.pos.clone()
        drv.step()
        if s % 16:
            _, _, Ff = ref.solve(before, tq)
            ref.sync()
            errs.append(rel_rms(drv.force.cpu().numpy(), Ff.cpu().numpy()))
    ref.close()
    plan.close()
    out["reuse_rel_rms_force_vs_full"] = {"mean": float(np.mean(errs)), "max": float(np.max(errs)),
                                          "after_1_step": errs[0], "after_15_steps": errs[14]}
    return out


def bench_triply(dp, torch, steps):
    """The triply periodic performance workload of Sec. 7.4 (2 x 10^4
    charges, 185 x 185 x 100, 64^2 x 32, point charges, g_t = 1.2 h): solve
    time in mixed precision and FP64 with the per-stage split. The paper
    quotes 0.84 ms for this comparison (single precision, 70^2 grid, RTX
    2080 Ti); another machine's figure, context only."""
    import workloads as W
    p, pos, q = W.config_triply(0)
    tpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    out = {"n": len(q), "grid": [p.Nx, p.Ny, p.Nz], "paper_ms_rtx2080ti": 0.84}
    forces = {}
    for name, prec in (("mixed", dp.DPSE_MIXED), ("fp64", dp.DPSE_FP64)):
        r = time_path(dp, torch, p, tpos, tq, prec, steps, 3)
        out[name] = {"ms": 1e3 * r["wall_s"] / steps, "evals_per_s": len(q) / (r["wall_s"] / steps),
                     "p50_ms": float(np.percentile(r["lat_ms"], 50)),
                     "stages_ms": {k: round(v, 4) for k, v in r["stages"].items()}}
        forces[name] = r["F"]
    out["mixed_vs_fp64_rel_rms_force"] = rel_rms(forces["mixed"], forces["fp64"])
    return out


def bench_walls(dp, torch, steps):
    """The jump workload with fixed charge densities on both walls (Sec. 2
    eq. rho): Gaussians of s = 4 centred in the box with total charge +64
    (bottom) and -64 (top), mixed precision, energy requested: the solve with
    the walls against the same solve without them, the one-time cost of
    dpse_plan_set_walls, the force change the walls make and the mixed
    path's force difference from the FP64 path with the walls."""
    import workloads as W
    p, pos, q = W.config_jump(0)
    sb, st = W.gaussian_walls(p, 4.0)
    walls = (torch.tensor(64.0 * sb, device="cuda"), torch.tensor(64.0 * st, device="cuda"))
    tpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    r0 = time_path(dp, torch, p, tpos, tq, dp.DPSE_MIXED, steps, 3)
    rw = time_path(dp, torch, p, tpos, tq, dp.DPSE_MIXED, steps, 3, walls=walls)
    r64 = time_path(dp, torch, p, tpos, tq, dp.DPSE_FP64, steps, 3, walls=walls)
    plan = dp.Plan(p, max_n=len(q), precision=dp.DPSE_MIXED)
    plan.set_walls(*walls)
    plan.sync()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.set_walls(*walls)
    plan.sync()
    t_set = (time.perf_counter() - t0) / reps
    plan.close()
    n = len(q)
    return {"ms_no_walls": 1e3 * r0["wall_s"] / steps, "ms_walls": 1e3 * rw["wall_s"] / steps,
            "evals_per_s_walls": n / (rw["wall_s"] / steps), "finalize_stage_ms_walls": rw["stages"]["finalize"],
            "finalize_stage_ms_no_walls": r0["stages"]["finalize"], "set_walls_ms": 1e3 * t_set,
            "status": rw["status"], "rel_rms_force_change_by_walls": rel_rms(rw["F"], r0["F"]),
            "mixed_vs_fp64_rel_rms_force": rel_rms(rw["F"], r64["F"]),
            "mixed_vs_fp64_rel_energy": abs(rw["U"] - r64["U"]) / abs(r64["U"])}


def bench_serve(dp, torch, rate, duration, warm, n_traj=256, budget_gb=16.0, n_slots=4, max_queue=256):
    """Serving stream: Poisson arrivals of solves from n_traj Brownian-like
    trajectories (N log-uniform in [512, 262144], box and permittivities
    fixed per trajectory, each request moves every charge by N(0, 0.05^2)
    per axis on the device). Latency is arrival to result on the host; the
    first `warm` seconds are not counted."""
    import workloads as W
    from paper_2101_07088_amd.serve import Overloaded, Server
    trajs = W.serving_trajectories(n_traj)
    srv = Server(budget_bytes=int(budget_gb * 2 ** 30), n_slots=n_slots, precision=dp.DPSE_MIXED,
                 max_queue=max_queue)
    state = []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2000)
    for t, (p, pos, q) in enumerate(trajs):
        srv.register(t, p, 1 << int(math.ceil(math.log2(len(q)))))
        state.append([p, torch.tensor(pos, dtype=torch.float64, device="cuda"),
                      torch.tensor(q, dtype=torch.float64, device="cuda")])
    times, which = W.poisson_arrivals(rate, duration, n_traj)

    def step_positions(st):
        p, pos, _ = st
        x = pos + 0.05 * torch.randn(pos.shape, dtype=torch.float64, device="cuda", generator=gen)
        x[:, 0].remainder_(p.Lx)
        x[:, 1].remainder_(p.Ly)
        lo, hi = 0.5, p.H - 0.5
        z = x[:, 2]
        z = torch.where(z < lo, 2 * lo - z, z)
        z = torch.where(z > hi, 2 * hi - z, z)
        x[:, 2] = z.clamp(lo, hi)
        st[1] = x
        return x

    done = []
    shed = 0
    sample = {}
    i = 0
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while i < len(times) and times[i] <= now:
            st = state[which[i]]
            x = step_positions(st)
            ev = torch.cuda.Event()
            ev.record()
            try:
                r = srv.submit(int(which[i]), x, st[2], ready_event=ev, arrival=t0 + times[i])
                r.callbacks.append(done.append)
                if i % 997 == 0 and len(sample) < 4:
                    sample[i] = (int(which[i]), x.clone(), r)
            except Overloaded:
                shed += times[i] >= warm
            i += 1
        srv.step()
        if i >= len(times) and not srv.pending():
            break
    wall = time.perf_counter() - t0
    torch.cuda.synchronize()
    counted = [r for r in done if r.arrival - t0 >= warm]
    lat = np.array([r.latency for r in counted]) * 1e3
    evals = sum(r.n for r in counted)
    offered = int(np.sum(times >= warm))
    span = max(r.finished for r in counted) - (t0 + warm) if counted else float("nan")
    out = {"rate_offered_req_s": rate, "duration_s": duration, "warmup_s": warm, "trajectories": n_traj,
           "requests_offered": offered, "requests_served": len(counted), "requests_shed": int(shed),
           "served_req_s": len(counted) / span, "evals_per_s": evals / span,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "slots": n_slots, "budget_bytes": srv.budget, "peak_bytes": srv.stats["peak_bytes"],
           "peak_active": srv.stats["peak_active"], "failed": srv.stats["failed"], "wall_s": wall}
    errs = []
    for k, (t, x, r) in sample.items():
        if not r.done():
            continue
        p, _, q = state[t]
        pl = dp.Plan(p, max_n=len(q), precision=dp.DPSE_FP64)
        U, phi, F = pl.solve(x, q)
        pl.sync()
        errs.append(rel_rms(r.result[2].cpu().numpy(), F.cpu().numpy()))
        pl.close()
    out["mixed_vs_fp64_rel_rms_force_max"] = max(errs) if errs else None
    srv.close()
    return out


def bench_small(dp, torch, steps):
    """The 64-charge small workload (32 x 32 x 33, FP64): per-solve time of
    eager launches (about 20 kernels) against one graph launch of the
    captured solve, and the launch overhead that the graph removes."""
    import workloads as W
    p, pos, q = W.config_small(0)
    tpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    plan = dp.Plan(p, max_n=len(q))
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    PH = torch.empty(len(q), dtype=torch.float64, device="cuda")
    F = torch.empty((len(q), 3), dtype=torch.float64, device="cuda")
    out = {"n": len(q), "grid": [p.Nx, p.Ny, p.Nz]}
    k = max(200, 10 * steps)
    for name, fn in (("eager", plan.solve), ("graph", plan.solve_graph)):
        for _ in range(10):
            fn(tpos, tq, E, PH, F)
        plan.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn(tpos, tq, E, PH, F)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / k
        out[name] = {"us_per_solve": 1e6 * t, "evals_per_s": len(q) / t}
    plan.set_timing(True)
    for _ in range(20):
        plan.solve(tpos, tq, E, PH, F)
    stages, _ = plan.stage_times()
    plan.set_timing(False)
    out["gpu_busy_us_eager"] = 1e3 * sum(stages.values())
    out["launch_overhead_us_removed_by_graph"] = out["eager"]["us_per_solve"] - out["graph"]["us_per_solve"]
    plan.close()
    return out


def bench_jump(dp, torch, steps, warmup, seeds=(1, 2, 3, 4)):
    """The jump workload (N = 16384, 256 x 256 x 129): both precisions at seed
    0 (time, p50/p99, stages), and the mixed path's force error against the
    FP64 path at seeds 0-4."""
    import workloads as W
    out = {"workload": "jump: N=16384 +-1 ions, Lx=Ly=64, H=32, eps=1, eps_b=eps_t=0.05, xi=1.0, "
                       "grid 256x256x129, r_cut=3.0"}
    p, pos, q = W.config_jump(0)
    tpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    res = {}
    for prec, name in ((dp.DPSE_FP64, "fp64"), (dp.DPSE_MIXED, "mixed")):
        r = time_path(dp, torch, p, tpos, tq, prec, steps, warmup, latency_solves=200)
        res[name] = r
        out[name] = {"ms": 1e3 * r["wall_s"] / steps, "evals_per_s": len(q) / (r["wall_s"] / steps),
                     "p50_ms": float(np.percentile(r["lat_ms"], 50)), "p99_ms": float(np.percentile(r["lat_ms"], 99)),
                     "latency_solves": len(r["lat_ms"]), "stages_ms": {k: round(v, 5) for k, v in r["stages"].items()},
                     "tiles": list(r["tiles"])}
        print(f"[bench] jump {name}: {out[name]['ms']:.3f} ms/solve", file=sys.stderr, flush=True)
    errs = {0: rel_rms(res["mixed"]["F"], res["fp64"]["F"])}
    for sd in seeds:
        p, pos, q = W.config_jump(sd)
        tp_ = torch.tensor(pos, dtype=torch.float64, device="cuda")
        tq_ = torch.tensor(q, dtype=torch.float64, device="cuda")
        Fs = {}
        for prec in (dp.DPSE_FP64, dp.DPSE_MIXED):
            pl = dp.Plan(p, max_n=len(q), precision=prec)
            _, _, F = pl.solve(tp_, tq_)
            assert pl.sync_status() == 0
            Fs[prec] = F.cpu().numpy()
            pl.close()
        errs[sd] = rel_rms(Fs[dp.DPSE_MIXED], Fs[dp.DPSE_FP64])
    out["mixed_vs_fp64_rel_rms_force_by_seed"] = {str(k): v for k, v in errs.items()}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--latency-solves", type=int, default=200,
                    help="solves of the separate per-solve latency pass (p50/p99)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["auto", "fp64", "mixed"], default="auto")
    ap.add_argument("--jump", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the 16384-ion jump workload (both precisions, accuracy over seeds 0-4)")
    ap.add_argument("--small", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the 64-charge workload, eager against graph launches")
    ap.add_argument("--batch", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the 64-system uneven batch")
    ap.add_argument("--serve", action=argparse.BooleanOptionalAction, default=True,
                    help="also run the serving stream")
    ap.add_argument("--batch-branches", type=int, default=8)
    ap.add_argument("--uniform", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the uniform-permittivity and one-jump solvers against the general one")
    ap.add_argument("--triply", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the triply periodic variant on the paper's TP workload")
    ap.add_argument("--bd", action=argparse.BooleanOptionalAction, default=True,
                    help="also time Brownian-dynamics steps with and without far-field reuse")
    ap.add_argument("--walls", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the solve with charged walls against the plain one")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-duration", type=float, default=10.0)
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    ap.add_argument("--serve-slots", type=int, default=4,
                    help="concurrent requests of the serving stream (execution slots, one stream each)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (calibrates HBM byte counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the sharding "
              "is a design, not code); run with --gpus 1", file=sys.stderr)
        return 2
    import torch
    import paper_2101_07088_amd as dp
    import workloads as W

    if a.copy_probe_mb:
        src = torch.ones(a.copy_probe_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p, pos, q = W.config_large(a.seed)
    tpos = torch.tensor(pos, dtype=torch.float64, device="cuda")
    tq = torch.tensor(q, dtype=torch.float64, device="cuda")
    n = len(q)
    res = {}
    for prec in (["mixed", "fp64"] if a.precision == "auto" else [a.precision]):
        # the headline path gets the full step count, live stage events and the latency pass
        head_pass = prec == "mixed" or a.precision == "fp64"
        steps = a.steps if head_pass else max(3, a.steps // 4)
        res[prec] = time_path(dp, torch, p, tpos, tq, dp.DPSE_FP64 if prec == "fp64" else dp.DPSE_MIXED,
                              steps, a.warmup, live_stages=True,
                              latency_solves=a.latency_solves if head_pass else steps)
        res[prec]["steps"] = steps
        print(f"[bench] large {prec}: {1e3 * res[prec]['wall_s'] / steps:.3f} ms/solve, stages "
              + ", ".join(f"{k}={v:.3f}" for k, v in res[prec]["stages"].items()), file=sys.stderr, flush=True)
    acc = {}
    head = "fp64" if "fp64" in res else "mixed"
    if "fp64" in res and "mixed" in res:
        F64, Fm = res["fp64"]["F"], res["mixed"]["F"]
        err = rel_rms(Fm, F64)
        ffar64 = q[:, None] * res["fp64"]["far"][:, 1:]
        ffarm = q[:, None] * res["mixed"]["far"][:, 1:]
        acc = {"mixed_vs_fp64_rel_rms_force": err, "mixed_vs_fp64_rel_rms_far_force": rel_rms(ffarm, ffar64),
               "mixed_vs_fp64_rel_rms_phi": rel_rms(res["mixed"]["phi"], res["fp64"]["phi"]),
               # U = 1/2 sum q phi cancels strongly over a million charges: its
               # error is measured against the scale 1/2 sum |q phi| of its terms
               "mixed_vs_fp64_energy_err_rel_to_sum_abs": abs(res["mixed"]["U"] - res["fp64"]["U"])
               / (0.5 * float(np.sum(np.abs(q * res["fp64"]["phi"]))))}
        head = "mixed" if err <= 1e-5 else "fp64"
    elif "mixed" in res:
        head = "mixed"
    r = res[head]
    steps = r["steps"]
    ms = 1e3 * r["wall_s"] / steps
    value = n / (r["wall_s"] / steps)
    s_bytes = 4 if head == "mixed" else 8
    beta = band_fraction(p, r["info"])
    sb = stage_bytes(p, beta, s_bytes)
    single = ("spread", "column", "interp")   # stages of one kernel each
    dom = max(single, key=lambda k: r["stages"][k])
    t_dom = r["stages"][dom] * 1e-3
    achieved = sb[dom] / t_dom / 1e9
    dom_kernel = kernel_name(dom, r["tiles"], head == "mixed", p, r["info"]["support"])
    traffic = profiled_traffic(dom_kernel)
    line = {
        "metric": "charge-force evals/s at <=1e-5 rel RMS force err vs FP64; p50/p99 solve ms",
        "value": value, "unit": "charge-force evals/s", "n_gpus": 1, "steps": steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "none (one GPU)", "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": "large slab: N=1048576 +-1 ions, Lx=Ly=256, H=64, eps=1, eps_b=0.05, eps_t=20, "
                               "xi=1.5, grid 1024x1024x257, r_cut=2.0, seed %d" % a.seed,
                   "precision": head, "parallelism": "single GPU"},
        "p50_ms": float(np.percentile(r["lat_ms"], 50)), "p99_ms": float(np.percentile(r["lat_ms"], 99)),
        "latency_solves": int(len(r["lat_ms"])),
        "stages_ms": {k: round(v, 5) for k, v in r["stages"].items()},
        "tiles": {"spread": r["tiles"][0], "interp": r["tiles"][1], "column": r["tiles"][2]},
        # the autotuner's timings of the candidate launch shapes that apply (ms per solve)
        "tile_ms": {name: {i: round(float(v), 4) for (st, i), v in sorted(r["tile_ms"].items()) if st == s}
                    for s, name in enumerate(("spread", "interp", "column"))},
        "accuracy": acc,
        "roofline": {"bound": "hbm", "kernel": dom_kernel or dom, "stage": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes": sb[dom], "beta": beta,
                     "launch_ms": r["stages"][dom],
                     "all_stages": {k: {"algorithmic_bytes": v, "ms": r["stages"][k],
                                        "frac": v / (r["stages"][k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                                    for k, v in sb.items()}},
        "workspace_bytes": r["workspace_bytes"],
        # grid points solved per second: the batch line's figure of the same kind
        # tells whether its 64 small systems keep the chip as busy as one large one
        "grid_points_per_s": p.Nx * p.Ny * p.Nz / (r["wall_s"] / steps),
    }
    for prec, rr in res.items():
        line[f"{prec}_evals_per_s"] = n / (rr["wall_s"] / rr["steps"])
        line[f"{prec}_ms"] = 1e3 * rr["wall_s"] / rr["steps"]
        line[f"{prec}_p50_ms"] = float(np.percentile(rr["lat_ms"], 50))
        line[f"{prec}_p99_ms"] = float(np.percentile(rr["lat_ms"], 99))
    del res
    torch.cuda.empty_cache()
    if a.jump:
        line["jump"] = bench_jump(dp, torch, a.steps, a.warmup)
    if a.small:
        line["small"] = bench_small(dp, torch, a.steps)
        print(f"[bench] small: {line['small']}", file=sys.stderr, flush=True)
    if a.uniform:
        line["uniform_eps"] = bench_uniform(dp, torch, a.steps)
        print(f"[bench] uniform eps: {line['uniform_eps']}", file=sys.stderr, flush=True)
        line["one_jump"] = bench_one_jump(dp, torch, a.steps)
        print(f"[bench] one jump: {line['one_jump']}", file=sys.stderr, flush=True)
    if a.triply:
        line["triply_periodic"] = bench_triply(dp, torch, a.steps)
        print(f"[bench] triply periodic: {line['triply_periodic']}", file=sys.stderr, flush=True)
    if a.bd:
        line["brownian_dynamics"] = bench_bd(dp, torch, a.steps)
        print(f"[bench] brownian dynamics: {line['brownian_dynamics']}", file=sys.stderr, flush=True)
    if a.walls:
        line["charged_walls"] = bench_walls(dp, torch, a.steps)
        print(f"[bench] charged walls: {line['charged_walls']}", file=sys.stderr, flush=True)
    if a.batch:
        line["batch"] = bench_batch(dp, torch, a.steps, n_branches=a.batch_branches)
        print(f"[bench] batch: {line['batch']}", file=sys.stderr, flush=True)
    if a.serve:
        line["serving"] = bench_serve(dp, torch, a.serve_rate, a.serve_duration, a.serve_warmup, n_slots=a.serve_slots)
        print(f"[bench] serving: {line['serving']}", file=sys.stderr, flush=True)
        cap = line["serving"]["served_req_s"]
        if a.serve_rate > 0.8 * cap:
            # the offered stream exceeds what one GPU serves: also report latency at 70% of that capacity
            line["serving_at_70pct_capacity"] = bench_serve(dp, torch, 0.7 * cap, a.serve_duration / 2,
                                                            a.serve_warmup, n_slots=a.serve_slots)
            print(f"[bench] serving at 70%: {line['serving_at_70pct_capacity']}", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, pos, q)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
