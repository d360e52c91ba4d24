"""Batched solves of uneven independent slab systems as one graph launch.

The systems are spread over a few concurrent branches (longest-first greedy
on an estimated cost, so that branches finish together); the systems of a
branch run one after another and share one workspace arena sized for the
largest of them, so device memory grows with the number of branches, not the
number of systems. The whole batch is captured once by
dpse_batch_graph_create and then run with one dpse_graph_launch per step,
which removes the per-kernel launch cost between the many small kernels of
the small systems. The systems' positions and charges live in caller tensors
that the graph reads on every launch.
"""
from __future__ import annotations

import math
from typing import List, Sequence

from . import native


def solve_cost(params, n: int) -> float:
    """Relative cost of one solve: grid points (spread/FFT/column/interp
    passes) plus per-charge stencil work; only used to balance branches."""
    G = params.Nx * params.Ny * params.Nz
    return G * (1.0 + math.log2(params.Nx * params.Ny) / 16.0) + 3000.0 * n


def assign_branches(costs: Sequence[float], n_branches: int) -> List[int]:
    """Longest-processing-time-first assignment of systems to branches."""
    order = sorted(range(len(costs)), key=lambda i: -costs[i])
    load = [0.0] * n_branches
    out = [0] * len(costs)
    for i in order:
        b = min(range(n_branches), key=lambda k: load[k])
        out[i] = b
        load[b] += costs[i]
    return out


class BatchRunner:
    """Plans, per-branch arenas and the captured graph of one batch.

    systems: sequence of (params, pos, q) with pos, q float64 device tensors
    ([n,3] and [n]); they stay referenced and are read on every run()."""

    def __init__(self, systems, precision: int = native.DPSE_MIXED, n_branches: int = 8, use_graph: bool = True,
                 autotune: bool = True):
        import torch
        self.torch = torch
        self.n_branches = max(1, min(n_branches, len(systems)))
        self.systems = list(systems)
        dev = self.systems[0][1].device
        self.plans = [native.Plan(p, max_n=int(q.shape[0]), precision=precision, own_workspace=False)
                      for p, _, q in self.systems]
        costs = [solve_cost(p, int(q.shape[0])) for p, _, q in self.systems]
        self.branch = assign_branches(costs, self.n_branches)
        self.arena_bytes = [0] * self.n_branches
        for i, pl in enumerate(self.plans):
            b = self.branch[i]
            self.arena_bytes[b] = max(self.arena_bytes[b], pl.info["workspace_bytes"])
        self.arenas = [torch.empty(max(nb, 256), dtype=torch.uint8, device=dev) for nb in self.arena_bytes]
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(self.n_branches)]
        for i, pl in enumerate(self.plans):
            pl.bind(self.arenas[self.branch[i]], self.streams[self.branch[i]])
        self.tiles = {}
        if autotune:
            torch.cuda.synchronize()
            # one tuning run per distinct grid shape, on its first system; the
            # others of that shape reuse the choice
            for i, pl in enumerate(self.plans):
                p, pos, q = self.systems[i]
                key = (p.Nx, p.Ny, p.Nz, pl.info["support"])
                if key not in self.tiles:
                    self.tiles[key], _ = pl.autotune(pos, q, reps=2)
                else:
                    pl.set_tiles(self.tiles[key])
            torch.cuda.synchronize()
        self.energy = [torch.empty(1, dtype=torch.float64, device=dev) for _ in self.systems]
        self.phi = [torch.empty(int(q.shape[0]), dtype=torch.float64, device=dev) for _, _, q in self.systems]
        self.force = [torch.empty((int(q.shape[0]), 3), dtype=torch.float64, device=dev) for _, _, q in self.systems]
        self.graph = None
        if use_graph:
            self.graph = native.BatchGraph(self.plans, [s[1] for s in self.systems], [s[2] for s in self.systems],
                                           self.energy, self.phi, self.force, branch=self.branch,
                                           n_branches=self.n_branches)

    @property
    def workspace_bytes(self) -> int:
        return sum(self.arena_bytes)

    def run(self, stream=None):
        """Enqueues one solve of every system (one graph launch, or eager
        launches on the branch streams when use_graph is False) ordered
        after the work already on `stream` (default: the current stream)."""
        torch = self.torch
        if stream is None:
            stream = torch.cuda.current_stream()
        if self.graph is not None:
            self.graph.launch(stream)
            return
        for s in self.streams:
            s.wait_stream(stream)
        for i, pl in enumerate(self.plans):
            _, pos, q = self.systems[i]
            pl.solve(pos, q, self.energy[i], self.phi[i], self.force[i])
        for s in self.streams:
            stream.wait_stream(s)

    def statuses(self) -> List[int]:
        """Device statuses since the last call, one per branch arena (plans of
        a branch share their status word); waits for the branch streams."""
        torch = self.torch
        torch.cuda.synchronize()
        seen = {}
        for i, pl in enumerate(self.plans):
            b = self.branch[i]
            if b not in seen:
                seen[b] = pl.sync_status()
        return [seen[b] for b in sorted(seen)]

    def close(self):
        if self.graph is not None:
            self.graph.close()
            self.graph = None
        for pl in self.plans:
            pl.close()
        self.plans = []
