"""torch.autograd.Function over the HIP engine: U_r(theta, x) per replica.

theta is the [3, n] tensor of knot values (phi, rho, F) of the tabulated EAM;
forward sets the engine's tables from it and evaluates the energies (and
forces) with the EAM kernels; backward returns dL/dtheta from the adjoint
kernels (sum_r gU_r dU_r/dtheta, reduced on the device) and dL/dx = -gU_r f.
By Eq. dFdL with theta in the role of lambda, averaging dU/dtheta over the H0
ensemble gives dF/dtheta; the engine can accumulate that during a switching
run (Context.set_adjoint_sampling).
"""
from __future__ import annotations

import numpy as np
import torch

from . import eamfe as E


class _Knots:
    def __init__(self, theta: np.ndarray, r_cut: float, rho_max: float):
        self.phi, self.rho, self.embed = (np.ascontiguousarray(theta[k], dtype=np.float64) for k in range(3))
        self.r_cut, self.rho_max = float(r_cut), float(rho_max)


class EAMEnergy(torch.autograd.Function):
    """U = EAMEnergy.apply(theta, x, ctx, r_cut, rho_max) -> [n_rep] float64.

    ctx is an eamfe.Context whose system is set up; x is the device SoA
    [3, N_tot] float64 position tensor."""

    @staticmethod
    def forward(fctx, theta, x, ctx, r_cut, rho_max):
        th = theta.detach().to("cpu", torch.float64).numpy()
        knots = _Knots(th, r_cut, rho_max)
        ctx.eam_setup(knots)
        U = torch.zeros(ctx.n_rep, dtype=torch.float64, device=x.device)
        f = torch.zeros_like(x)
        ctx.eam_forces(x.detach().contiguous(), f, U)
        fctx.save_for_backward(x, f)
        fctx.ctx, fctx.theta_device = ctx, theta.device
        # dU/dtheta depends on theta itself (through F'(rho_i) and rho_i), so
        # backward needs this node's tables even if a later forward replaced them
        fctx.knots, fctx.version = knots, ctx.table_version
        fctx.n = th.shape[1]
        return U

    @staticmethod
    def backward(fctx, gU):
        x, f = fctx.saved_tensors
        ctx = fctx.ctx
        dtheta = None
        if fctx.needs_input_grad[0]:
            d = torch.zeros(3, fctx.n, dtype=torch.float64, device=x.device)
            current = ctx.knots if ctx.table_version != fctx.version else None
            if current is not None:
                ctx.eam_setup(fctx.knots)      # this node's theta
            try:
                ctx.adjoint_theta(x.detach().contiguous(), d, weights=gU.detach().cpu().numpy(), reduce=True)
            finally:
                if current is not None:
                    ctx.eam_setup(current)     # the context keeps the tables it had
            dtheta = d.to(fctx.theta_device)
        dx = None
        if fctx.needs_input_grad[1]:
            # dU_r/dx_i = -f_i for atoms of replica r
            w = torch.repeat_interleave(gU, torch.as_tensor(np.diff(ctx.offsets), device=gU.device))
            dx = -f * w[None, :]
        return dtheta, dx, None, None, None
