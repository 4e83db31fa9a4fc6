"""Losses of the coupled simulation as differentiable PyTorch functions.

1. The film-energy loss.

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

2. A functional F(trace) of one E component's probe record (trace[i] the
value after step i+1), e.g. the splitting of the two hybrid modes of the
anti-crossing (Results, "Numerically Predicted Strong Magnon-Photon
Coupling Phenomena") estimated from the trace's spectrum.  With the same
parameters (H0, eps, f), dF/dp = sum_i dF/dtrace_i dtrace_i/dp: one forward
run records the trace, torch differentiates F with respect to it, and
``mpx_adjoint_probe`` gives the gradient of the weighted trace
sum_i w_i trace_i with w = dF/dtrace on a second simulation built with the
same parameters (the trace is then recomputed there; both runs are the same
kernels on the same inputs, so the two records are equal).
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


@dataclass
class ProbeTraceSpec:
    make_sim: Callable[[tuple, np.ndarray, float], "mpx.Sim"]
    nsteps: int
    field: int  # 0, 1, 2: E_x, E_y, E_z
    ijk: Sequence[int]
    eps_box: Sequence[int]
    top_box: Sequence[int]
    ms_top: float
    checkpoint_every: int = 0


def _params(H0, eps, f):
    return (tuple(float(v) for v in H0.detach().to("cpu", torch.float64).reshape(3)),
            eps.detach().to("cpu", torch.float64).numpy(), float(f.detach().to("cpu", torch.float64)))


def record_trace(spec: ProbeTraceSpec, H0: torch.Tensor, eps: torch.Tensor, f: torch.Tensor) -> np.ndarray:
    """The probe record of the simulation make_sim builds (nsteps values)."""
    sim = spec.make_sim(*_params(H0, eps, f))
    try:
        pid = sim.add_probe(mpx.PROBE_FIELD, field=spec.field, ijk=tuple(spec.ijk), cap=spec.nsteps)
        sim.step(spec.nsteps)
        return np.asarray(sim.read_probe(pid, 1), dtype=np.float64).reshape(-1)[:spec.nsteps].copy()
    finally:
        sim.close()


class ProbeFunctionalLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H0: torch.Tensor, eps: torch.Tensor, f: torch.Tensor, spec: ProbeTraceSpec,
                fn: Callable[[torch.Tensor], torch.Tensor]):
        trace = record_trace(spec, H0, eps, f)
        with torch.enable_grad():
            tr = torch.tensor(trace, dtype=torch.float64, requires_grad=True)
            F = fn(tr)
            (w,) = torch.autograd.grad(F, tr)
        sim = spec.make_sim(*_params(H0, eps, f))
        try:
            res = sim.adjoint_probe(spec.nsteps, spec.field, tuple(spec.ijk), w.numpy(),
                                    checkpoint_every=spec.checkpoint_every, eps_box=tuple(spec.eps_box),
                                    ms_box=tuple(spec.top_box))
        finally:
            sim.close()
        deps = res["deps"] if eps.dim() > 0 else np.array(res["deps"].sum())
        df = spec.ms_top * float(res["dMs"].sum())
        ctx.save_for_backward(torch.as_tensor(res["dH0"], dtype=H0.dtype, device=H0.device).reshape(H0.shape),
                              torch.as_tensor(deps, dtype=eps.dtype, device=eps.device).reshape(eps.shape),
                              torch.as_tensor(df, dtype=f.dtype, device=f.device).reshape(f.shape))
        return F.detach().to(device=H0.device)

    @staticmethod
    def backward(ctx, g):
        gH0, geps, gf = ctx.saved_tensors
        return g * gH0, g * geps, g * gf, None, None


def probe_functional(H0: torch.Tensor, eps: torch.Tensor, f: torch.Tensor, spec: ProbeTraceSpec,
                     fn: Callable[[torch.Tensor], torch.Tensor]) -> torch.Tensor:
    """F(trace(H0, eps, f)) for a scalar torch function fn of the probe record,
    with gradients by the discrete adjoint of the weighted trace (see the
    module docstring)."""
    return ProbeFunctionalLoss.apply(H0, eps, f, spec, fn)


def band_centroid_splitting(trace: torch.Tensor, dt: float, f_mid: float, half_band: float,
                            pad: int = 4) -> torch.Tensor:
    """A smooth estimate of the frequency splitting of two modes on either
    side of f_mid: the power-weighted mean frequency of the Hann-windowed,
    mean-removed spectrum over (f_mid, f_mid + half_band] minus the one over
    [f_mid - half_band, f_mid].  Differentiable in the trace (its peaks'
    bin-refined positions are not: they jump between bins)."""
    x = trace - trace.mean()
    n = x.numel()
    win = torch.hann_window(n, periodic=False, dtype=x.dtype, device=x.device)
    nfft = max(n, int(pad) * n)
    P = torch.fft.rfft(x * win, nfft).abs() ** 2
    fr = torch.fft.rfftfreq(nfft, dt, dtype=x.dtype, device=x.device)
    lo = (fr >= f_mid - half_band) & (fr <= f_mid)
    hi = (fr > f_mid) & (fr <= f_mid + half_band)
    if not bool(lo.any()) or not bool(hi.any()):
        raise ValueError("a band holds no frequency bin")
    c_lo = (P[lo] * fr[lo]).sum() / P[lo].sum()
    c_hi = (P[hi] * fr[hi]).sum() / P[hi].sum()
    return c_hi - c_lo
