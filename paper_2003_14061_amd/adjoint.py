"""Gradients of trajectory observables through torch.autograd.

``TrajectoryObservables`` runs a leapfrog trajectory of the MD method
(libmd's md_traj_forward, with checkpoints) and returns its observables:
the mean potential energy per atom over the steps and the soft radial
distribution g(r) of the last positions.  Its backward is libmd's
md_traj_backward: the hand-written reverse pass that recomputes each
checkpointed segment and walks it backwards (force Jacobian products, the
parameter derivatives of the forces, the drift adjoint), all in HIP
kernels.  A loss is then any torch expression of the observables.

The potential parameters (eps, sigma) are inputs like the initial state;
the cutoff moves with sigma (r_cut = r_cut_over_sigma * sigma).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import md


@dataclass(frozen=True)
class TrajectorySpec:
    """Everything about the trajectory except (x0, v0, eps, sigma)."""
    L: float
    n_steps: int
    dt: float
    r_cut_over_sigma: float = 2.5
    skin: float = 0.3
    mass: float = 1.0
    shifted: bool = True
    precision: str = "fp64"
    checkpoint_every: int = 20
    n_bins: int = 0
    gr_rmax: float = 2.5
    gr_width: float | None = None
    nl_capacity: int = 0

    def simulation(self, x0, v0, eps: float, sigma: float) -> md.Simulation:
        return md.Simulation(x0, v0, self.L, r_cut=self.r_cut_over_sigma * sigma, dt=self.dt,
                             skin=self.skin, eps=eps, sigma=sigma, mass=self.mass,
                             shifted=self.shifted, precision=self.precision,
                             neighbor_list=True, reorder=False, nl_capacity=self.nl_capacity)


class TrajectoryObservables(torch.autograd.Function):
    """(x0 [n,3], v0 [n,3], eps, sigma) -> (ubar, g [n_bins]).

    ubar = (1/S) sum_{s=1..S} U(x_s) / N; g is the soft g(r) of x_S."""

    @staticmethod
    def forward(ctx, x0, v0, eps, sigma, spec: TrajectorySpec):
        sim = spec.simulation(x0, v0, float(eps), float(sigma))
        obs = sim.traj_forward(spec.n_steps, spec.checkpoint_every, spec.n_bins, spec.gr_rmax,
                               spec.gr_width)
        ctx.sim = sim
        ctx.like = tuple((t.device, t.dtype, t.shape) if isinstance(t, torch.Tensor) else None
                         for t in (x0, v0, eps, sigma))
        return obs[0].clone(), obs[1:].clone()

    @staticmethod
    def backward(ctx, g_ubar, g_g):
        gobs = torch.cat([g_ubar.reshape(1), g_g.reshape(-1)]).to(torch.float64)
        gx, gv, gth = ctx.sim.traj_backward(gobs)
        ctx.sim = None

        def like(g, meta):
            if meta is None:
                return None
            device, dtype, shape = meta
            return g.to(device=device, dtype=dtype).reshape(shape)

        mx, mv, me, ms = ctx.like
        return like(gx, mx), like(gv, mv), like(gth[0], me), like(gth[1], ms), None


def trajectory_observables(x0, v0, eps, sigma, spec: TrajectorySpec):
    """Differentiable (ubar, g) of the trajectory described by spec."""
    return TrajectoryObservables.apply(x0, v0, eps, sigma, spec)
