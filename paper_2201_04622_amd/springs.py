"""Spring constants of the Einstein reference crystal from the mean-squared
displacement (Eq. msd): equipartition gives k = 3 kB T / <(dr)^2>, with the
displacements taken from the lattice sites and the centre-of-mass
displacement removed, averaged over an equilibrium run of the real system
(H0, lambda = 0) at the size and temperature of the switching runs.

The dynamics, the displacement sums and k run in the library (run_switching
over the equilibration stretch of a protocol, eamfe_msd after each stretch,
eamfe_spring_constant); this module sequences the stretches and forms the
averages.
"""
from __future__ import annotations

import numpy as np

from . import eamfe as E

def spring_constants(ctx, replicas, x, v, n_steps, every, mode="fl", skin=0.3, dt=0.001, damp=0.1,
                     discard=0):
    """Run ``n_steps`` steps of the lambda = 0 Hamiltonian of ``mode`` (H0 for
    "fl"; the first Einstein crystal for "hh") from positions x and
    velocities v (device SoA, updated in place), sample the per-replica MSD
    every ``every`` steps after the first ``discard`` steps, and return
    (k per replica in eV/A^2, mean MSD per replica in A^2, samples)."""
    if every < 1 or n_steps < every:
        raise ValueError("spring_constants: need n_steps >= every >= 1")
    p = E.protocol(mode, n_steps, 1, 0, 0, skin=skin, dt=dt, damp=damp)
    acc = np.zeros(len(replicas))
    samples = 0
    for s in range(0, n_steps - n_steps % every, every):
        ctx.run_switching(p, x, v, s, s + every)
        if s + every > discard:
            acc += ctx.msd(x)
            samples += 1
    msd = acc / max(samples, 1)
    k = np.array([E.spring_constant(m, r.T) for m, r in zip(msd, replicas)])
    return k, msd, samples
