"""Static relaxation with the FP64 oracle's energies and forces.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; never by the product
package.  FIRE, the fast inertial relaxation engine of Bitzek, Koskinen,
Gaehler, Moseler and Gumbsch (Phys. Rev. Lett. 97, 170201, 2006), with its
published default parameters: damped dynamics of unit mass that mixes the
velocity towards the force direction while the power F.v stays positive,
lengthens the time step after five such steps, and stops and shortens the
step as soon as the power turns negative.  It gives the 0 K reference of a
relaxed defect (a free surface) against which finite-temperature free
energies are checked.
"""
from __future__ import annotations

import numpy as np


def fire(pot, x, L, fmax=1e-6, dt=0.02, dt_max=0.2, max_steps=20000):
    """Relax positions ``x`` [N, 3] in the box ``L`` until every force
    component is below ``fmax`` (eV/A).  Returns (x, U, steps); raises if the
    force criterion is not met within ``max_steps``."""
    n_min, f_inc, f_dec, a_start, f_a = 5, 1.1, 0.5, 0.1, 0.99
    x = np.array(x, dtype=np.float64, copy=True)
    v = np.zeros_like(x)
    r = pot.eam(x, L)
    f, U = r["f"], r["U"]
    a, since_neg = a_start, 0
    for step in range(max_steps):
        if np.abs(f).max() < fmax:
            return x, U, step
        power = float(np.sum(f * v))
        if power > 0.0:
            v = (1.0 - a) * v + a * np.linalg.norm(v) * f / np.linalg.norm(f)
            since_neg += 1
            if since_neg > n_min:
                dt = min(dt * f_inc, dt_max)
                a *= f_a
        else:
            v[:] = 0.0
            dt *= f_dec
            a, since_neg = a_start, 0
        v = v + dt * f
        x = x + dt * v
        r = pot.eam(x, L)
        f, U = r["f"], r["U"]
    raise RuntimeError(f"fire: max |f| {np.abs(f).max():.3g} after {max_steps} steps")
