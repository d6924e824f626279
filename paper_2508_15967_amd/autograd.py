"""torch.autograd integration: gradients of any torch loss on ray endpoints
with respect to launch states and medium parameters, through the library's
checkpointed discrete adjoint (rg_trace_rays_adjoint)."""
from __future__ import annotations

import torch

from . import media
from . import raygraph as rgb


class _RayTraceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tracer, x0, k0, omega, *params):
        x0, k0, omega = x0.detach().contiguous(), k0.detach().contiguous(), omega.detach().contiguous()
        params = [p.detach().contiguous() for p in params]
        # with store_checkpoints=False the forward keeps no checkpoints: the
        # adjoint reruns it inside its own call (checkpoints = NULL), trading
        # one more forward for the checkpoint memory until backward
        ce = tracer.checkpoint_every if tracer.store_checkpoints else 0
        out = tracer.prog.trace(x0, k0, omega, params, dt=tracer.dt, n_steps=tracer.n_steps,
                                checkpoint_every=ce, **tracer.launch)
        if not tracer.store_checkpoints:
            out["_desc"].checkpoint_every = tracer.checkpoint_every  # checkpoints stay NULL
        ctx.tracer = tracer
        ctx.keep = (out, x0, k0, omega, params)  # device buffers the descriptor points to
        return out["x"], out["k"]

    @staticmethod
    def backward(ctx, gx, gk):
        out, x0, k0, omega, params = ctx.keep
        prog = ctx.tracer.prog
        gx = torch.zeros_like(out["x"]) if gx is None else gx.contiguous()
        gk = None if gk is None else gk.contiguous()
        need = ctx.needs_input_grad
        gx0 = torch.empty_like(x0) if need[1] else None
        gk0 = torch.empty_like(k0) if need[2] else None
        gps = [torch.empty_like(p) if need[4 + i] else None for i, p in enumerate(params)]
        prog.adjoint_desc(out["_desc"], gx, gk, gx0, gk0, gps)
        return (None, gx0, gk0, None, *gps)


class RayTracer:
    """Callable ray tracer for a medium: (x0, k0, omega, *params) -> (x_end, k_end),
    differentiable in x0, k0 and the parameter arrays.  store_checkpoints=False
    keeps no forward checkpoints between forward and backward (the adjoint
    reruns the forward)."""

    def __init__(self, medium, dt: float, n_steps: int, checkpoint_every: int = 100,
                 store_checkpoints: bool = True, **launch):
        g, D, params = media.build(medium)
        self.graph, self.D = g, D
        self.prog = g.compile(D, want_adjoint=True)
        self.default_params = params
        self.dt, self.n_steps, self.checkpoint_every = dt, n_steps, checkpoint_every
        self.store_checkpoints = store_checkpoints
        self.launch = launch

    def __call__(self, x0, k0, omega, *params):
        return _RayTraceFn.apply(self, x0, k0, omega, *params)
