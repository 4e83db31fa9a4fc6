"""The film-energy loss as a differentiable PyTorch function.

L(H0, eps, f) = dt * sum over steps n = loss_from+1 .. nsteps of the EM
energy of one film at integer time n (the film-energy probe's sum), for the
simulation a caller-supplied ``make_sim(H0, eps, f)`` builds at step 0, with
its gradients from the discrete adjoint of the coupled scheme (``mpx_adjoint``:
the transposed E step, H/M half steps and trapezoidal LLG solve, with the
CPML recursions; arXiv:2510.22221, Methods, "Numerical Model").

Parameters:
  * H0   -- the uniform bias (3,), A/m;
  * eps  -- eps_r of the cells of ``eps_box`` (nk, nj, ni), or one scalar for
            all of them (its gradient is then the sum over the box);
  * f    -- the film-thickness fraction: the cells of ``top_box`` (the film's
            top layer) carry Ms = ms_top * f, so dL/df = ms_top * sum of dL/dMs
            over them (through the LLG solve and the initial M = Ms u).

``make_sim`` must realise the parameters it is given (for a per-cell eps, one
material per distinct value: the material table holds at most 254 ids).  The
forward call runs the simulation and its adjoint once; backward only scales
the stored gradients.  Everything runs in the HIP library; the tensors here
carry parameters and results only.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Sequence

import numpy as np
import torch

from . import mpx


@dataclass
class FilmEnergySpec:
    make_sim: Callable[[tuple, np.ndarray, float], "mpx.Sim"]
    nsteps: int
    loss_from: int
    eps_box: Sequence[int]
    top_box: Sequence[int]
    ms_top: float
    film: int = 0
    checkpoint_every: int = 0


class FilmEnergyLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H0: torch.Tensor, eps: torch.Tensor, f: torch.Tensor, spec: FilmEnergySpec):
        h0 = tuple(float(v) for v in H0.detach().to("cpu", torch.float64).reshape(3))
        e = eps.detach().to("cpu", torch.float64).numpy()
        fv = float(f.detach().to("cpu", torch.float64))
        sim = spec.make_sim(h0, e, fv)
        try:
            res = sim.adjoint(spec.nsteps, spec.loss_from, film=spec.film, checkpoint_every=spec.checkpoint_every,
                              eps_box=tuple(spec.eps_box), ms_box=tuple(spec.top_box))
        finally:
            sim.close()
        deps = res["deps"] if eps.dim() > 0 else np.array(res["deps"].sum())
        df = spec.ms_top * float(res["dMs"].sum())
        ctx.save_for_backward(torch.as_tensor(res["dH0"], dtype=H0.dtype, device=H0.device).reshape(H0.shape),
                              torch.as_tensor(deps, dtype=eps.dtype, device=eps.device).reshape(eps.shape),
                              torch.as_tensor(df, dtype=f.dtype, device=f.device).reshape(f.shape))
        return torch.tensor(res["loss"], dtype=torch.float64, device=H0.device)

    @staticmethod
    def backward(ctx, g):
        gH0, geps, gf = ctx.saved_tensors
        return g * gH0, g * geps, g * gf, None


def film_energy_loss(H0: torch.Tensor, eps: torch.Tensor, f: torch.Tensor, spec: FilmEnergySpec) -> torch.Tensor:
    """L(H0, eps, f) with gradients by the discrete adjoint (see the module
    docstring)."""
    return FilmEnergyLoss.apply(H0, eps, f, spec)
