"""Gradients of a scalar misfit of the final concentration with respect to the per-node
diffusion-tensor field and the initial state, through the library's checkpointed adjoint
sweep (argument marshalling only).

elbm_forward_record runs the N steps, recording per node and step the entropic amplitude
lambda and the fallback branch and checkpointing the state every K steps, all into one
device workspace. elbm_gradient runs the reverse sweep: for each segment, newest first, the
K forward states are recomputed from the checkpoint and K adjoint steps run in reverse,
accumulating dL/dT per node; elbm_tensor_gradient maps it to dL/dD or dL/dL (log field).
"""
from __future__ import annotations

from typing import Optional

import torch

from .lattice import Lattice


class AdjointRun:
    """Checkpointed forward run of `steps` steps on a lattice with a tensor field.

    The lattice must already hold its tensor field (set_diffusion with a field), velocity,
    source and initial state. ckpt_every = K."""

    def __init__(self, lat: Lattice, steps: int, ckpt_every: int):
        if steps < 1 or ckpt_every < 1:
            raise ValueError("steps and ckpt_every must be >= 1")
        self.lat = lat
        self.steps = steps
        self.K = ckpt_every
        nbytes = lat.gradient_workspace_bytes(steps, ckpt_every)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=lat.device)
        self.dphi0 = None
        self.dj0 = None

    def forward(self) -> torch.Tensor:
        """Run the N steps; returns phi at the final time (FP64, (nz, ny, nx))."""
        self.lat.forward_record(self.steps, self.K, self.ws)
        phi, _ = self.lat.moments()
        return phi

    def backward(self, grad_phi: torch.Tensor) -> torch.Tensor:
        """dL/dT accumulated over all steps (working precision, (n, 6) node-major) for
        dL/dphi_N = grad_phi; also keeps dL/dphi0 and dL/dj0 of the equilibrium start. The
        lattice is left at the final state."""
        lat = self.lat
        g = grad_phi.to(device=lat.device, dtype=torch.float64).contiguous()
        if g.numel() != lat.n:
            raise ValueError("grad_phi must hold one value per node")
        t_grad = torch.zeros((lat.n, 6), dtype=lat.real, device=lat.device)  # node-major
        self.dphi0 = torch.empty(lat.shape, dtype=torch.float64, device=lat.device)
        self.dj0 = torch.empty((3,) + lat.shape, dtype=torch.float64, device=lat.device)
        lat.gradient(self.steps, self.K, self.ws, g, t_grad, self.dphi0, self.dj0)
        return t_grad

    def initial_gradient(self, with_flux: bool = False):
        """dL/dphi0 (and dL/dj0) of the equilibrium start, after backward()."""
        if self.dphi0 is None:
            raise RuntimeError("backward() has not run")
        return (self.dphi0, self.dj0) if with_flux else self.dphi0


class TensorFieldLoss(torch.autograd.Function):
    """phi_N = F(field): forward runs the lattice from its current initial state with the
    tensor field `field` (D, or L with D = expm(L) if the lattice was set up with a log
    field); backward returns dL/dfield through the adjoint kernels."""

    @staticmethod
    def forward(ctx, field: torch.Tensor, lat: Lattice, steps: int, ckpt_every: int,
                init: Optional[tuple] = None):
        is_log = getattr(lat, "is_log", False)
        lat.set_diffusion(field.detach(), is_log=is_log)
        if init is not None:
            lat.load_state(*init)
        run = AdjointRun(lat, steps, ckpt_every)
        phi = run.forward()
        ctx.run = run
        return phi

    @staticmethod
    def backward(ctx, grad_phi):
        run = ctx.run
        t_grad = run.backward(grad_phi)
        return run.lat.tensor_gradient(t_grad), None, None, None, None
