"""TEST INFRASTRUCTURE ONLY -- plain CPU reference of the Brownian-dynamics
step and of the far-field reuse between steps.

Only ``tests/`` and ``bench.py``'s baseline leg may import this module; the
product path never does.

The step is the non-Markovian Euler-Maruyama scheme of Leimkuhler and
Matthews that the paper integrates its Brownian dynamics with (Sec. 7, eq.
leimkuhler), without the steric forces (out of scope here):

    z^{n+1} = z^n + mu F(z^n) dt + sqrt(kT mu dt / 2) (W^n + W^{n+1}),

W^n independent standard normal vectors, drawn by the caller and passed in.
A step that would take any charge out of the admissible heights is rejected
as a whole (the paper retries it with new noise).

Far-field reuse (the paper's closing remark on reusing far-field work
between steps; the reading taken here): between full solves every K steps,
each charge keeps the far-field average (potential and field) and the gauge
constant of the last full solve, and only the near field is recomputed at
the new positions.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import dpse_oracle as O


def leimkuhler_step(pos, F, w_prev, w_next, mu, dt, kT, z_lo=0.0, z_hi=None):
    """One step of eq. leimkuhler. Returns (new positions, rejected?) where
    rejected means some new height is outside (z_lo, z_hi)."""
    pos = np.asarray(pos, dtype=np.float64)
    new = pos + mu * dt * np.asarray(F) + math.sqrt(kT * mu * dt / 2.0) * (np.asarray(w_prev) + np.asarray(w_next))
    z = new[:, 2]
    bad = bool(np.any(~(z > z_lo)) or (z_hi is not None and np.any(~(z < z_hi))))
    return new, bad


def near_reuse(p, pos, q, inter_last):
    """Outputs with the far field of a previous full solve held fixed: the
    near field at pos, plus the far averages and the gauge constant of
    ``inter_last`` (the intermediates of that solve, same charges in the same
    order). Returns (U, phi, F) as ``dpse_oracle.solve`` does."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    d = O.derive(p)
    near = O.near_field(p, d, pos, q)
    far = inter_last["far"]
    self_c = 2.0 * d["xi_e"] / (O.FOUR_PI * p.eps * O.SQRT_PI)
    phi = far[:, 0] + near[:, 0] + inter_last["B_i"] - q * self_c
    F = q[:, None] * (far[:, 1:] + near[:, 1:])
    return 0.5 * float(np.sum(q * phi)), phi, F
