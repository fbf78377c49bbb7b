"""torch.autograd.Function around the library's hand-written adjoint.

``chi_energy_fraction(phi, chi, pi_phi, pi_chi, q, ...)`` evolves the two-field
lattice (V = lambda/4 phi^4 + q/2 phi^2 chi^2, velocity-Verlet, a = 1) for
``nsteps`` and returns O = (E_K^chi + E_G^chi)/rho as a 0-dim float64 tensor.
``energy_fraction(..., field)`` returns that fraction for either field, and
``spectrum_bin(..., field, bin)`` returns Delta(bin) of field ``field``
at the final time (eq. discretePS).  The backward returns dO/d(phi, chi,
pi_phi, pi_chi) at the initial time and dO/dq, all computed by
``lattice_grad`` (reverse integration with checkpoints) during the forward
call.  The inputs are copied; they are not modified.
"""
from __future__ import annotations

import torch

from .lattice import Lattice


class _LatticeObservable(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, chi, pi_phi, pi_chi, q, N, dx, dt, nsteps, lam, stride, observable, field, bin):
        fields = [t.detach().reshape(-1).to(torch.float64).contiguous().clone() for t in (phi, chi, pi_phi, pi_chi)]
        lat = Lattice(fields[:2], fields[2:], N=N, dx=dx, dt=dt, integrator="vv2", expansion="none",
                      potential="phi4_chi2", lam=lam, q=float(q))
        try:
            r = lat.grad(nsteps, stride=stride, observable=observable, field=field, bin=bin)
        finally:
            lat.close()
        shape = phi.shape
        ctx.save_for_backward(r["dO_dphi"][0].reshape(shape), r["dO_dphi"][1].reshape(shape),
                              r["dO_dpi"][0].reshape(shape), r["dO_dpi"][1].reshape(shape),
                              torch.tensor(r["dO_dq"], dtype=torch.float64, device=phi.device))
        return torch.tensor(r["value"], dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, g):
        gphi, gchi, gpp, gpc, gq = ctx.saved_tensors
        return (g * gphi, g * gchi, g * gpp, g * gpc, g * gq) + (None,) * 9


def _q(q):
    return q if torch.is_tensor(q) else torch.tensor(float(q), dtype=torch.float64)


def chi_energy_fraction(phi, chi, pi_phi, pi_chi, q, *, N, dx, dt, nsteps, lam=1.0, stride=0):
    return _LatticeObservable.apply(phi, chi, pi_phi, pi_chi, _q(q), N, dx, dt, nsteps, lam, stride,
                                    "chi_fraction", 0, 0)


def energy_fraction(phi, chi, pi_phi, pi_chi, q, *, N, dx, dt, nsteps, field, lam=1.0, stride=0):
    return _LatticeObservable.apply(phi, chi, pi_phi, pi_chi, _q(q), N, dx, dt, nsteps, lam, stride,
                                    "energy_fraction", int(field), 0)


def spectrum_bin(phi, chi, pi_phi, pi_chi, q, *, N, dx, dt, nsteps, field, bin, lam=1.0, stride=0):
    return _LatticeObservable.apply(phi, chi, pi_phi, pi_chi, _q(q), N, dx, dt, nsteps, lam, stride,
                                    "spectrum_bin", int(field), int(bin))
