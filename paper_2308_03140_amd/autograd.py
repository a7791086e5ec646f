"""torch.autograd.Function over the C ABI.

MBDEnergy.apply(coords, alpha0, omega, rvdw, lattice, context, beta, a, q_frac, kgrid) -> E

The forward pass calls mbd_evaluate once with the gradient outputs requested
for the inputs that need them (the adjoint contraction of the paper's
eq:mbd-gradient, read as (1/4) Tr(Q^{-1/2} dQ/dX), runs in the library's HIP
kernels); the backward pass only scales the stored gradients by grad_output.
Double backward is not supported: the backward is marked once-differentiable,
so asking for a second derivative raises instead of treating the stored
gradients as constants.
"""
import ctypes

import torch

from . import _abi as A
from . import torch_api as T


class MBDEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coords, alpha0, omega, rvdw, lattice, context, beta=0.83, a=6.0, q_frac=None, kgrid=None):
        context.sync_stream()
        dev = context.device
        need = ctx.needs_input_grad
        periodic = lattice is not None
        s, keep = T.make_system(coords.detach(), alpha0.detach(), omega.detach(), rvdw.detach(), beta, a,
                                lattice.detach().cpu() if periodic else None, q_frac, kgrid, device=dev)
        N = s.n_atoms
        r = A.MbdResult()
        E = torch.empty(1, dtype=torch.float64, device=dev)
        r.energy = E.data_ptr()
        want = A.MBD_WANT_ENERGY
        grads = {}

        def out(name, shape, bit, field):
            nonlocal want
            g = torch.empty(*shape, dtype=torch.float64, device=dev)
            setattr(r, field, g.data_ptr())
            want |= bit
            grads[name] = g

        if need[0]:
            out("coords", (N, 3), A.MBD_WANT_GRAD_COORDS, "grad_coords")
        if need[1]:
            out("alpha0", (N,), A.MBD_WANT_GRAD_ALPHA0, "grad_alpha0")
        if need[2]:
            out("omega", (N,), A.MBD_WANT_GRAD_OMEGA, "grad_omega_or_c6")
        if need[3]:
            out("rvdw", (N,), A.MBD_WANT_GRAD_RVDW, "grad_rvdw")
        if periodic and need[4]:
            out("lattice", (3, 3), A.MBD_WANT_GRAD_LATTICE, "grad_lattice")
        code = A.mbd_evaluate(context.handle, s, want, r)
        if code != A.MBD_OK:
            T._raise(context, code)
        ctx.grads = grads
        ctx.lattice_device = lattice.device if periodic else None
        return E[0].clone()

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gE):
        g = ctx.grads

        def scaled(name, dev=None):
            if name not in g:
                return None
            v = gE * g[name]
            return v.to(dev) if dev is not None else v

        return (scaled("coords"), scaled("alpha0"), scaled("omega"), scaled("rvdw"),
                scaled("lattice", ctx.lattice_device), None, None, None, None, None)


def mbd_energy(coords, alpha0, omega, rvdw, context, lattice=None, beta=0.83, a=6.0, q_frac=None, kgrid=None):
    """Differentiable MBD energy (Ha) of one finite or periodic system."""
    return MBDEnergy.apply(coords, alpha0, omega, rvdw, lattice, context, beta, a, q_frac, kgrid)
