"""torch.autograd.Function around the lattice and its adjoint.

Forward: set the initial field, run `steps` steps with a checkpoint tape,
return phi^N.  Backward: one lbm_tape_gradient call (hand-written adjoint
kernels with segment replays) gives dL/dphi0 and dL/dtau from dL/dphi^N.
"""
from __future__ import annotations

import torch

from .lbm import Lattice


class Evolve(torch.autograd.Function):
    """phi^N = Evolve.apply(phi0, tau, lattice_kwargs, steps, every).

    phi0: float64 tensor shaped (N_d, ..., N_1) on the GPU; tau: 0-d tensor;
    lattice_kwargs: keyword arguments of Lattice without tau (d, dims, dx, u, ...).
    """

    @staticmethod
    def forward(ctx, phi0, tau, lattice_kwargs, steps, every):
        kw = dict(lattice_kwargs)
        d, dims = kw.pop("d"), kw.pop("dims")
        lat = Lattice(d, dims, float(tau), **kw)
        lat.set_initial(phi0.detach().reshape(-1))
        lat.tape_begin(int(every))
        lat.step(int(steps))
        ctx.lat = lat
        ctx.tau_dtype = tau.dtype if torch.is_tensor(tau) else torch.float64
        return lat.phi().clone()

    @staticmethod
    def backward(ctx, grad_out):
        lat = ctx.lat
        want_phi0 = ctx.needs_input_grad[0]
        want_tau = ctx.needs_input_grad[1]
        out = lat.tape_gradient(grad_out.contiguous(), want_phi0=want_phi0, want_tau=want_tau)
        g_phi0 = out.get("phi0").clone() if want_phi0 else None
        g_tau = (torch.tensor(out["tau"], dtype=ctx.tau_dtype, device=grad_out.device)
                 if want_tau else None)
        lat.close()
        ctx.lat = None
        return g_phi0, g_tau, None, None, None
