"""torch.autograd.Function around the library's hand-written adjoint.

``chi_energy_fraction(phi, chi, pi_phi, pi_chi, q, ...)`` evolves the two-field
lattice (V = lambda/4 phi^4 + q/2 phi^2 chi^2, velocity-Verlet) for ``nsteps``
and returns O = (E_K^chi + E_G^chi)/rho as a 0-dim float64 tensor.
``energy_fraction(..., field)`` returns that fraction for either field, and
``spectrum_bin(..., field, bin)`` returns Delta(bin) of field ``field``
at the final time (eq. discretePS).

Background (sec. 4.5.2): ``expansion="none"`` (a = 1, the default),
``"fixed"`` (the power law of eq. ScaleFactorPowerLaw with ``w_eos``, ``H0``,
``t_ref``, ``a0``, starting at time ``t0``) or ``"self"`` (self-consistent
expansion with ``kappa2``, from ``a0`` and ``b0`` = a' at the start; b0 must be
given, and both may be tensors that require a gradient).  ``alpha`` is the
alpha-time exponent.

When a gradient is wanted the forward call runs ``lattice_grad`` (reverse
integration with checkpoints) and keeps dO/d(phi, chi, pi_phi, pi_chi) at the
initial time, dO/dq and, with self-consistent expansion, dO/da0 and dO/db0 for
the backward.  Under ``torch.no_grad()``, or when no input requires a gradient,
only the forward steps and the observable run.  The inputs are copied; they
are not modified.
"""
from __future__ import annotations

import math

import torch

from .lattice import Lattice

_OBS = ("chi_fraction", "energy_fraction", "spectrum_bin")


def _lattice(fields, N, dx, dt, lam, q, bg):
    return Lattice(fields[:2], fields[2:], N=N, dx=dx, dt=dt, integrator="vv2", potential="phi4_chi2",
                   lam=lam, q=float(q), **bg)


def _copies(phi, chi, pi_phi, pi_chi):
    return [t.detach().reshape(-1).to(torch.float64).contiguous().clone() for t in (phi, chi, pi_phi, pi_chi)]


def _forward_value(fields, N, dx, dt, nsteps, lam, q, bg, observable, field, bin):
    """O after nsteps steps without the adjoint (library steps, then the energies
    or the spectrum of the final state)."""
    lat = _lattice(fields, N, dx, dt, lam, q, bg)
    try:
        lat.step(nsteps)
        if observable == "spectrum_bin":
            return float(lat.spectrum(field, "phi", nbins=bin + 1)["delta"][bin])
        s = 1 if observable == "chi_fraction" else field
        e = lat.energy()
        return (e["EK"][s] + e["EG"][s]) / e["rho"]
    finally:
        lat.close()


class _LatticeObservable(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, chi, pi_phi, pi_chi, q, a0, b0, N, dx, dt, nsteps, lam, stride, observable, field, bin,
                bg):
        fields = _copies(phi, chi, pi_phi, pi_chi)
        bg = dict(bg)
        if bg.get("expansion") == "self":
            bg.update(a0=float(a0), b0=float(b0))
        dev = phi.device
        if not any(ctx.needs_input_grad[:7]):
            ctx.grads = None
            v = _forward_value(fields, N, dx, dt, nsteps, lam, q, bg, observable, field, bin)
            return torch.tensor(v, dtype=torch.float64, device=dev)
        lat = _lattice(fields, N, dx, dt, lam, q, bg)
        try:
            r = lat.grad(nsteps, stride=stride, observable=observable, field=field, bin=bin)
        finally:
            lat.close()
        shape = phi.shape
        f64 = dict(dtype=torch.float64, device=dev)
        ctx.save_for_backward(r["dO_dphi"][0].reshape(shape), r["dO_dphi"][1].reshape(shape),
                              r["dO_dpi"][0].reshape(shape), r["dO_dpi"][1].reshape(shape),
                              torch.tensor(r["dO_dq"], **f64), torch.tensor(r["dO_da0"], **f64),
                              torch.tensor(r["dO_db0"], **f64))
        return torch.tensor(r["value"], **f64)

    @staticmethod
    def backward(ctx, g):
        gphi, gchi, gpp, gpc, gq, ga, gb = ctx.saved_tensors
        return (g * gphi, g * gchi, g * gpp, g * gpc, g * gq, g * ga, g * gb) + (None,) * 10


def _scalar(x):
    return x if torch.is_tensor(x) else torch.tensor(float(x), dtype=torch.float64)


def _apply(phi, chi, pi_phi, pi_chi, q, N, dx, dt, nsteps, lam, stride, observable, field, bin, expansion, alpha,
           a0, b0, kappa2, w_eos, H0, t0, t_ref):
    if observable not in _OBS:
        raise ValueError(f"unknown observable {observable!r}")
    if expansion not in ("none", "fixed", "self"):
        raise ValueError(f"unknown expansion {expansion!r}")
    bg = dict(expansion=expansion, alpha=float(alpha))
    if expansion == "fixed":
        if torch.is_tensor(a0) and a0.requires_grad:
            raise ValueError("a0 of a fixed background is a constant of the background, not a differentiable input")
        bg.update(a0=float(a0), w_eos=float(w_eos), H0=float(H0), t0=float(t0), t_ref=float(t_ref))
    elif expansion == "self":
        if b0 is None or not math.isfinite(float(b0)):
            raise ValueError("self-consistent expansion needs b0 = a' at the start as an input (its derivative "
                             "dO/db0 is returned for it)")
        bg.update(kappa2=float(kappa2), t0=float(t0))
    else:
        bg.update(t0=float(t0))
    a0t, b0t = _scalar(a0), _scalar(0.0 if b0 is None else b0)
    ins = (phi, chi, pi_phi, pi_chi, _scalar(q), a0t, b0t)
    if not torch.is_grad_enabled() or not any(t.requires_grad for t in ins):
        bgv = dict(bg)
        if expansion == "self":
            bgv.update(a0=float(a0), b0=float(b0))
        v = _forward_value(_copies(phi, chi, pi_phi, pi_chi), N, dx, dt, nsteps, lam, float(q), bgv, observable,
                           field, bin)
        return torch.tensor(v, dtype=torch.float64, device=phi.device)
    return _LatticeObservable.apply(*ins, N, dx, dt, nsteps, lam, stride, observable, field, bin, bg)


def chi_energy_fraction(phi, chi, pi_phi, pi_chi, q, *, N, dx, dt, nsteps, lam=1.0, stride=0, expansion="none",
                        alpha=1.0, a0=1.0, b0=None, kappa2=0.25, w_eos=1.0 / 3.0, H0=0.0, t0=0.0, t_ref=0.0):
    return _apply(phi, chi, pi_phi, pi_chi, q, N, dx, dt, nsteps, lam, stride, "chi_fraction", 0, 0, expansion,
                  alpha, a0, b0, kappa2, w_eos, H0, t0, t_ref)


def energy_fraction(phi, chi, pi_phi, pi_chi, q, *, N, dx, dt, nsteps, field, lam=1.0, stride=0, expansion="none",
                    alpha=1.0, a0=1.0, b0=None, kappa2=0.25, w_eos=1.0 / 3.0, H0=0.0, t0=0.0, t_ref=0.0):
    return _apply(phi, chi, pi_phi, pi_chi, q, N, dx, dt, nsteps, lam, stride, "energy_fraction", int(field), 0,
                  expansion, alpha, a0, b0, kappa2, w_eos, H0, t0, t_ref)


def spectrum_bin(phi, chi, pi_phi, pi_chi, q, *, N, dx, dt, nsteps, field, bin, lam=1.0, stride=0, expansion="none",
                 alpha=1.0, a0=1.0, b0=None, kappa2=0.25, w_eos=1.0 / 3.0, H0=0.0, t0=0.0, t_ref=0.0):
    return _apply(phi, chi, pi_phi, pi_chi, q, N, dx, dt, nsteps, lam, stride, "spectrum_bin", int(field), int(bin),
                  expansion, alpha, a0, b0, kappa2, w_eos, H0, t0, t_ref)
