"""Gradients of a scalar misfit of the final concentration with respect to the per-node
diffusion-tensor field, through the hand-written adjoint step kernel of the HIP library.

Forward: N steps of the step kernel recording, per node and step, the entropic amplitude
lambda and the fallback branch (elbm_step_record); the raw state is checkpointed every K
steps. Backward: for each segment, newest first, the checkpoint is restored, the K forward
states are recomputed and kept, and K adjoint steps (elbm_adjoint_step) run in reverse,
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
        n = lat.n
        self.lam = torch.empty(steps * n, dtype=lat.real, device=lat.device)
        self.branch = torch.empty(steps * n, dtype=torch.uint8, device=lat.device)
        self.ckpts = []

    def forward(self) -> torch.Tensor:
        """Run the N steps; returns phi at the final time (FP64, (nz, ny, nx))."""
        lat, n = self.lat, self.lat.n
        self.ckpts = []
        s = 0
        while s < self.steps:
            self.ckpts.append(lat.save_state())
            m = min(self.K, self.steps - s)
            lat.step_record(m, self.lam[s * n:(s + m) * n], self.branch[s * n:(s + m) * n])
            s += m
        phi, _ = lat.moments()
        return phi

    def backward(self, grad_phi: torch.Tensor) -> torch.Tensor:
        """dL/dT accumulated over all steps (working precision, (n, 6) node-major) for
        dL/dphi_N = grad_phi; the lattice is left at the final state."""
        lat, n = self.lat, self.lat.n
        shape = lat.shape
        adj = grad_phi.to(device=lat.device, dtype=lat.real).reshape((1,) + shape).expand((lat.q,) + shape).contiguous()
        adj_next = torch.empty_like(adj)
        t_grad = torch.zeros((lat.n, 6), dtype=lat.real, device=lat.device)  # node-major
        states = []
        for seg in range(len(self.ckpts) - 1, -1, -1):
            buf, step0, pending0 = self.ckpts[seg]
            m = min(self.K, self.steps - seg * self.K)
            # recompute the segment's forward states straight into their buffers; the
            # checkpoint itself is the first one
            while len(states) < m - 1:
                states.append(torch.empty(lat.pop_bytes, dtype=torch.uint8, device=lat.device))
            seg_states = [buf] + states[:m - 1]
            has_src = lat.has_source
            pend = [pending0] + [1 if has_src else 0] * (m - 1)
            for j in range(m - 1):
                lat.step_buffers(seg_states[j], pend[j], seg_states[j + 1])
            for j in range(m - 1, -1, -1):
                s = seg * self.K + j
                lat.adjoint_step(seg_states[j], pend[j], self.lam[s * n:(s + 1) * n],
                                 self.branch[s * n:(s + 1) * n], adj, adj_next, t_grad)
                adj, adj_next = adj_next, adj
        self.adj0 = adj
        return t_grad

    def initial_gradient(self, with_flux: bool = False):
        """dL/dphi0 (and dL/dj0) of the equilibrium start, after backward()."""
        return self.lat.initial_gradient(self.adj0, with_flux)


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
