"""torch.autograd bridge of the hand-written adjoint (gg_adjoint).

``chamber_misfit(c_in, D, R_patch, ...)`` returns the scalar
L = 1/2 sum_x weight(x) (C(x, T) - target(x))^2 of a gradient-generator run
and back-propagates into the inlet concentrations, the diffusion
coefficient and the source values on a patch. Forward and backward both run
in the HIP library: the forward call performs the run and the adjoint sweep
together and keeps the gradients for backward.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np
import torch

from .lattice import Lattice
from .workloads import Phase, Workload


def _with_parameters(wl: Workload, c_in: np.ndarray, D: float) -> Workload:
    """Copy of the workload with new inlet concentrations (segment defaults
    and every per-phase override) and diffusion coefficient."""
    segs = []
    inlets = [s for s in wl.segments if s.kind == "inlet"]
    cmap = {s.id: float(c_in[k]) for k, s in enumerate(inlets)}
    for s in wl.segments:
        segs.append(dataclasses.replace(s, c_in=cmap.get(s.id, s.c_in)))
    sched = None
    if wl.schedule:
        sched = [Phase(p.duration, p.open, tuple((sid, cmap.get(sid, v)) for sid, v in p.c_in))
                 for p in wl.schedule]
    out = dataclasses.replace(wl, segments=segs, schedule=sched, D=float(D))
    for attr in ("layout", "peclet"):
        if hasattr(wl, attr):
            setattr(out, attr, getattr(wl, attr))
    return out


class ChamberMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c_in, D, R_patch, wl, n_steps, weight, target, r_box, storage, ckpt_every):
        wl2 = _with_parameters(wl, c_in.detach().cpu().double().numpy(), float(D.detach().cpu()))
        lat = Lattice.from_workload(wl2, storage=storage)
        R = np.zeros(wl.mask.shape)
        x0, y0, w, h = r_box
        R[y0:y0 + h, x0:x0 + w] = R_patch.detach().cpu().double().numpy()
        if np.any(R != 0.0):
            lat.set_source(R)
        res = lat.adjoint(n_steps, weight, target, r_box=r_box, ckpt_every=ckpt_every)
        lat.close()
        inlets = [s.id for s in wl.segments if s.kind == "inlet"]
        g_cin = torch.tensor([res["d_c_in"][sid - 2] for sid in inlets], dtype=c_in.dtype)
        ctx.save_for_backward(g_cin.to(c_in.device),
                              torch.tensor(res["d_D"], dtype=D.dtype, device=D.device),
                              torch.from_numpy(res["d_R"]).to(R_patch.dtype).to(R_patch.device))
        return torch.tensor(res["loss"], dtype=torch.float64, device=c_in.device)

    @staticmethod
    def backward(ctx, gout):
        g_cin, g_D, g_R = ctx.saved_tensors
        return (gout * g_cin, gout * g_D, gout * g_R) + (None,) * 7


def chamber_misfit(c_in: torch.Tensor, D: torch.Tensor, R_patch: torch.Tensor, wl: Workload,
                   n_steps: int, weight: np.ndarray, target: np.ndarray,
                   r_box: Sequence[int], storage: str = "f32",
                   ckpt_every: int = 0) -> torch.Tensor:
    """Differentiable chamber misfit of a gradient-generator run.

    c_in: inlet concentrations, one per inlet segment in workload order;
    D: diffusion coefficient (0-d tensor); R_patch: source values on r_box
    (h x w). Returns a 0-d float64 tensor.
    """
    return ChamberMisfit.apply(c_in, D, R_patch, wl, int(n_steps), weight, target,
                               tuple(int(v) for v in r_box), storage, int(ckpt_every))
