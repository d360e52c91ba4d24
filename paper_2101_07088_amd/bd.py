"""Brownian dynamics of the charges (Sec. 7): the non-Markovian
Euler-Maruyama scheme of Leimkuhler and Matthews (eq. leimkuhler) driven by
the solver's forces, with the far field reused between full solves.

Every ``far_every`` steps the forces come from a full solve; in between from
dpse_solve_near (the near field at the new positions, the far field of the
last full solve held fixed). A step that takes a charge out of the slab is
discarded and retried with new noise (Sec. 7), up to ``max_retries`` times.
Steric forces are not included. Noise comes from a seeded torch generator on
the device and enters the step kernel as input.
"""
from __future__ import annotations

import math

from .native import DpseError


class BrownianDynamics:
    def __init__(self, plan, pos, q, mu: float, kT: float, dt: float, far_every: int = 1, seed: int = 0,
                 max_retries: int = 20):
        torch = plan._torch
        self.torch = torch
        self.plan = plan
        self.q = q
        self.pos = pos.clone()
        self.tmp = torch.empty_like(pos)
        self.mu_dt = mu * dt
        self.noise = math.sqrt(kT * mu * dt / 2.0)
        self.far_every = max(1, int(far_every))
        self.max_retries = int(max_retries)
        self.gen = torch.Generator(device=pos.device)
        self.gen.manual_seed(seed)
        self.w_prev = torch.randn(pos.shape, generator=self.gen, dtype=torch.float64, device=pos.device)
        self.w_next = torch.empty_like(self.w_prev)
        n = int(q.shape[0])
        self.energy = torch.empty(1, dtype=torch.float64, device=pos.device)
        self.phi = torch.empty(n, dtype=torch.float64, device=pos.device)
        self.force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        self.escaped = torch.zeros(1, dtype=torch.int32, device=pos.device)
        self.steps = 0
        self.retries = 0
        self.full_solves = 0

    def forces(self):
        """Forces at the current positions (full solve or far-field reuse)."""
        if self.steps % self.far_every == 0:
            self.plan.solve(self.pos, self.q, self.energy, self.phi, self.force)
            self.full_solves += 1
        else:
            self.plan.solve_near(self.pos, self.q, self.energy, self.phi, self.force)

    def step(self):
        """One step; raises DpseError for a device-detected error of the solve
        and RuntimeError when no retry keeps the charges in the slab."""
        self.forces()
        st = self.plan.sync_status()
        if st != 0:
            raise DpseError(st, "dpse_solve" if self.steps % self.far_every == 0 else "dpse_solve_near")
        for attempt in range(self.max_retries + 1):
            self.w_next.normal_(generator=self.gen)
            self.plan.bd_step(self.pos, self.force, self.w_prev, self.w_next, self.mu_dt, self.noise, self.tmp,
                              self.escaped)
            if int(self.escaped.item()) == 0:
                break
            self.retries += 1
        else:
            raise RuntimeError("no admissible Brownian step after %d retries" % self.max_retries)
        self.pos, self.tmp = self.tmp, self.pos
        self.w_prev, self.w_next = self.w_next, self.w_prev
        self.steps += 1
