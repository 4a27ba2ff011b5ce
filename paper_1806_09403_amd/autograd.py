"""The force history of a BTDF-IB-LBM run as a differentiable torch function.

``rollout(spec, populations, inflow, body_force, marker_xy, marker_uv,
centres)`` runs ``spec.steps`` steps on the GPU and returns the per-step
force history [steps, n_bodies, 3] (Fx, Fy, Tz of eq 27). Its backward is
the library's reverse sweep (``btdf_adjoint``): given dJ/d(history) it
returns dJ/d(initial populations, inflow velocity, body force, marker
positions, marker velocities, body centres), so any torch expression of the
history -- a mean drag coefficient, a lift target -- can be differentiated
with respect to the flow and the geometry, including through torch-side
parametrisations of the inputs (an initial state built from the inflow
speed, markers placed around a centre).

All tensors are float64 on the host; the arithmetic runs in the library's
kernels. The backward rebuilds the run from the saved inputs and lets
``btdf_adjoint`` take it forward again before sweeping back (one extra
forward run, no device state held between forward and backward).
"""
from dataclasses import dataclass
from typing import Tuple

import numpy as np
import torch

from ._lib import COS4, PERIODIC
from .sim import Sim


@dataclass(frozen=True)
class RolloutSpec:
    nx: int
    ny: int
    tau: float
    steps: int
    body_sizes: Tuple[int, ...]          # markers of each body, in order
    body_ds: Tuple[float, ...]           # arc length per marker of each body
    delta_kind: int = COS4
    thickening: float = 2.6
    bc: Tuple[int, int, int, int] = (PERIODIC,) * 4
    precision: int = 8
    checkpoint_every: int = 0            # 0: ceil(sqrt(steps)); >= steps: keep every state
    reference_velocity: Tuple[float, float] = (0.0, 0.0)  # storage reference of the populations


def _build(spec, populations, inflow, body_force, marker_xy, marker_uv, centres):
    s = Sim(spec.nx, spec.ny, spec.tau, spec.delta_kind, spec.thickening, spec.bc,
            tuple(float(v) for v in inflow), tuple(float(v) for v in body_force),
            (1.0, spec.reference_velocity[0], spec.reference_velocity[1]), spec.precision,
            history_capacity=spec.steps)
    at = 0
    for b, (n, ds) in enumerate(zip(spec.body_sizes, spec.body_ds)):
        s.add_body(marker_xy[at:at + n], marker_uv[at:at + n], float(centres[b, 0]), float(centres[b, 1]),
                   float(ds))
        at += n
    s.set_populations(populations)
    return s


class BtdfRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, spec, populations, inflow, body_force, marker_xy, marker_uv, centres):
        arrs = [t.detach().cpu().numpy().astype(np.float64) for t in
                (populations, inflow, body_force, marker_xy, marker_uv, centres)]
        s = _build(spec, *arrs)
        try:
            s.step(spec.steps)
            hist = s.force_history(spec.steps)
        finally:
            s.close()
        ctx.spec = spec
        ctx.arrs = arrs
        return torch.from_numpy(np.ascontiguousarray(hist))

    @staticmethod
    def backward(ctx, grad_hist):
        spec = ctx.spec
        s = _build(spec, *ctx.arrs)
        try:
            g, _ = s.adjoint(spec.steps, grad_hist.detach().cpu().numpy().astype(np.float64),
                             checkpoint_every=spec.checkpoint_every)
        finally:
            s.close()
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
        return (None, t(g["populations"]), t(g["inflow"]), t(g["body_force"]), t(g["marker_xy"]),
                t(g["marker_uv"]), t(g["centres"]))


def rollout(spec, populations, inflow, body_force, marker_xy, marker_uv, centres):
    """Force history [steps, n_bodies, 3] of the run; differentiable in every tensor input."""
    return BtdfRollout.apply(spec, populations, inflow, body_force, marker_xy, marker_uv, centres)

