"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare."""
from __future__ import annotations

import math
import os
import sys
from contextlib import contextmanager

import numpy as np

import oracle

INTEG = {"lf": oracle.LF, "vv2": oracle.VV2, "vv4": oracle.VV4, "vv6": oracle.VV6, "vv8": oracle.VV8,
         "vv10": oracle.VV10}
EXPN = {"none": oracle.NONE, "fixed": oracle.FIXED, "self": oracle.SELF}
POT = {"phi4": oracle.PHI4, "phi4_chi2": oracle.PHI4_CHI2}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@contextmanager
def tile_env(spec, var="LATTICE_TILE"):
    """Set a launch-shape override (LATTICE_TILE, LATTICE_U1_TILE) for the
    lattices created inside the block."""
    old = os.environ.get(var)
    if spec is None:
        os.environ.pop(var, None)
    else:
        os.environ[var] = spec
    try:
        yield
    finally:
        if old is None:
            os.environ.pop(var, None)
        else:
            os.environ[var] = old


def scalar_kwargs(wl, N=None, **over):
    kw = dict(N=wl.N if N is None else N, dx=wl.dx, dt=wl.dt, integrator=wl.integrator, expansion=wl.expansion,
              potential=wl.potential, lam=wl.lam, q=wl.q, alpha=wl.alpha, kappa2=wl.kappa2, w_eos=wl.w_eos,
              H0=wl.H0, a0=wl.a0, t_ref=0.0, t0=0.0)
    kw.update(over)
    return kw


def oracle_model(kw):
    nf = 1 if kw["potential"] == "phi4" else 2
    return oracle.ScalarModel(N=kw["N"], dx=kw["dx"], dt=kw["dt"], nfields=nf, potential=POT[kw["potential"]],
                              expansion=EXPN[kw["expansion"]], integrator=INTEG[kw["integrator"]],
                              lam=kw.get("lam", 1.0), q=kw.get("q", 0.0), alpha=kw.get("alpha", 1.0),
                              kappa2=kw.get("kappa2", 0.25), w_eos=kw.get("w_eos", 1 / 3), H0=kw.get("H0", 0.0),
                              t0=kw.get("t_ref", 0.0), a0=kw.get("a0", 1.0))


def to_dev(arrs, dtype):
    import torch
    return [torch.tensor(np.ascontiguousarray(a).reshape(-1), device="cuda", dtype=dtype) for a in arrs]


def rel_maxdiff(g, o):
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    o = np.asarray(o, dtype=np.float64).reshape(-1)
    return float(np.max(np.abs(g - o)) / max(np.max(np.abs(o)), 1e-300))


def gpu_scalar(kw, phi, pi, steps_list, precision="f64"):
    """Run the HIP path; returns (lattice, phi tensors, pi tensors) after all steps."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    dt = torch.float32 if precision == "f32" else torch.float64
    tp, tq = to_dev(phi, dt), to_dev(pi, dt)
    lat = Lattice(tp, tq, precision=precision, **kw)
    for n in steps_list:
        lat.step(n)
    torch.cuda.synchronize()
    return lat, tp, tq


def compare_state(tp, tq, st, tol, what=""):
    worst = 0.0
    for s in range(len(tp)):
        e1 = rel_maxdiff(tp[s].cpu().numpy(), st.phi[s])
        e2 = rel_maxdiff(tq[s].cpu().numpy(), st.pi[s])
        worst = max(worst, e1, e2)
        assert e1 <= tol, f"{what} phi[{s}] rel err {e1:.3e} > {tol}"
        assert e2 <= tol, f"{what} pi[{s}] rel err {e2:.3e} > {tol}"
    return worst


def compare_energy(eg, eo, tol, what=""):
    for k in ("EK", "EG", "EV"):
        for i in range(2):
            o = eo[k][i]
            g = eg[k][i]
            if o == 0.0:
                assert abs(g) <= 1e-300 + tol * abs(eo["rho"]), (what, k, i, g)
            else:
                assert abs(g - o) <= tol * abs(o), f"{what} {k}[{i}] {g} vs {o}"
    assert abs(eg["rho"] - eo["rho"]) <= tol * abs(eo["rho"]), (what, eg["rho"], eo["rho"])
    assert abs(eg["a"] - eo["a"]) <= tol * abs(eo["a"]), (what, eg["a"], eo["a"])
    assert abs(eg["b"] - eo["b"]) <= tol * max(abs(eo["b"]), 1e-300), (what, eg["b"], eo["b"])
    assert abs(eg["t"] - eo["t"]) <= 1e-13 * max(1.0, abs(eo["t"]))
