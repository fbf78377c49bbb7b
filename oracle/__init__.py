"""Plain FP64 CPU oracle for the lattice step (test infrastructure only).

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` import this package.  The product path (``paper_2102_01031_amd``)
never does.  The numerics live in ``lattice_oracle.c`` (compiled with gcc by
``oracle/build.py``); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

PHI4, PHI4_CHI2 = 0, 1
NONE, FIXED, SELF = 0, 1, 2
LF, VV2, VV4, VV6, VV8, VV10 = 0, 1, 2, 3, 4, 5


class Params(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("nfields", C.c_int32), ("potential", C.c_int32),
        ("expansion", C.c_int32), ("integrator", C.c_int32), ("pad", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double), ("lam", C.c_double), ("q", C.c_double),
        ("alpha", C.c_double), ("kappa2", C.c_double), ("w_eos", C.c_double),
        ("H0", C.c_double), ("t0", C.c_double), ("a0", C.c_double),
    ]


class Clock(C.Structure):
    _fields_ = [("t", C.c_double), ("a", C.c_double), ("b", C.c_double),
                ("lf_stag", C.c_int32), ("pad", C.c_int32)]


class U1Params(C.Structure):
    _fields_ = [("N", C.c_int32), ("expansion", C.c_int32), ("dx", C.c_double), ("dt", C.c_double),
                ("lam", C.c_double), ("v", C.c_double), ("e", C.c_double),
                ("kappa_g", C.c_double), ("alpha", C.c_double), ("kappa2", C.c_double),
                ("w_eos", C.c_double), ("H0", C.c_double), ("t0", C.c_double), ("a0", C.c_double)]


class SU2Params(C.Structure):
    _fields_ = [("N", C.c_int32), ("expansion", C.c_int32), ("dx", C.c_double), ("dt", C.c_double),
                ("lam", C.c_double), ("v", C.c_double), ("g", C.c_double),
                ("alpha", C.c_double), ("kappa2", C.c_double),
                ("w_eos", C.c_double), ("H0", C.c_double), ("t0", C.c_double), ("a0", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB") or _build.library_path()
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(dp)
        L.orc_laplacian.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_grad2_sum.argtypes = [C.c_int, C.c_double, dp]
        L.orc_grad2_sum.restype = C.c_double
        L.orc_kernel.argtypes = [C.POINTER(Params), C.c_double, pp, C.c_int, dp]
        L.orc_energy.argtypes = [C.POINTER(Params), pp, pp, C.POINTER(Clock), dp]
        L.orc_fixed_background.argtypes = [C.POINTER(Params), C.c_double, dp, dp]
        L.orc_hubble_b0.argtypes = [C.POINTER(Params), pp, pp, C.c_double, dp]
        L.orc_run.argtypes = [C.POINTER(Params), pp, pp, C.POINTER(Clock), C.c_long]
        L.orc_lf_sync.argtypes = [C.POINTER(Params), pp, pp, C.POINTER(Clock)]
        L.orc_yoshida4.argtypes = [dp, dp]
        L.orc_triple_jump.argtypes = [C.c_int, dp, dp]
        L.orc_spectrum.argtypes = [C.c_int, C.c_double, dp, C.c_int, dp, dp, C.POINTER(C.c_long)]
        L.orc_occupation.argtypes = [C.POINTER(Params), C.c_double, C.c_double, pp, pp, C.c_int, C.c_double, C.c_int,
                                     dp, C.POINTER(C.c_long)]
        L.orc_vv2_tangent.argtypes = [C.POINTER(Params), C.c_double, pp, pp, pp, pp, C.c_double]
        L.orc_vv2_adjoint_step.argtypes = [C.POINTER(Params), C.c_double, pp, pp, pp, pp, dp]
        L.orc_observable.argtypes = [C.POINTER(Params), pp, pp, dp, pp, pp, dp]
        L.orc_adjoint_vv2.argtypes = [C.POINTER(Params), pp, pp, C.c_long, dp, pp, pp, dp]
        L.orc_observable_kind.argtypes = [C.POINTER(Params), C.c_double, C.c_int, C.c_int, C.c_int, pp, pp, dp, pp,
                                          pp, dp]
        L.orc_adjoint_vv2_kind.argtypes = [C.POINTER(Params), C.c_double, C.c_int, C.c_int, C.c_int, pp, pp,
                                           C.c_long, dp, pp, pp, dp]
        L.orc_adjoint_vv2_self.argtypes = [C.POINTER(Params), C.c_int, C.c_int, C.c_int, pp, pp, C.c_double,
                                           C.c_double, C.c_long, dp, pp, pp, dp, dp, dp]
        L.orc_u1_forces.argtypes = [C.POINTER(U1Params), pp, pp, pp, pp]
        L.orc_u1_energy.argtypes = [C.POINTER(U1Params), pp, pp, pp, pp, C.POINTER(Clock), dp]
        L.orc_u1_gauss.argtypes = [C.POINTER(U1Params), pp, pp, pp, pp, dp]
        L.orc_u1_run_lf.argtypes = [C.POINTER(U1Params), pp, pp, pp, pp, C.POINTER(Clock), C.c_long]
        L.orc_u1_lf_sync.argtypes = [C.POINTER(U1Params), pp, pp, pp, pp, C.POINTER(Clock)]
        L.orc_su2_forces.argtypes = [C.POINTER(SU2Params), pp, pp, pp, pp]
        L.orc_su2_energy.argtypes = [C.POINTER(SU2Params), pp, pp, pp, pp, C.POINTER(Clock), dp]
        L.orc_su2_gauss.argtypes = [C.POINTER(SU2Params), pp, pp, pp, pp, dp]
        L.orc_su2_run_lf.argtypes = [C.POINTER(SU2Params), pp, pp, pp, pp, C.POINTER(Clock), C.c_long]
        L.orc_su2_lf_sync.argtypes = [C.POINTER(SU2Params), pp, pp, pp, pp, C.POINTER(Clock)]
        L.orc_gauss_solve.argtypes = [C.c_int, C.c_double, dp, pp]
        L.orc_su2_run_vv.argtypes = [C.POINTER(SU2Params), pp, pp, pp, pp, C.POINTER(Clock), C.c_long, C.c_int]
        L.orc_u1_run_vv.argtypes = [C.POINTER(U1Params), pp, pp, pp, pp, C.POINTER(Clock), C.c_long, C.c_int]
        L.orc_u1_fixed_background.argtypes = [C.POINTER(U1Params), C.c_double, dp, dp]
        L.orc_u1_forces_at.argtypes = [C.POINTER(U1Params), C.c_double, pp, pp, pp, pp]
        L.orc_u1_hubble_b0.argtypes = [C.POINTER(U1Params), pp, pp, pp, pp, C.c_double, dp]
        L.orc_su2_gauss_init.argtypes = [C.POINTER(SU2Params), pp, pp, pp, pp, dp]
        L.orc_su2_fixed_background.argtypes = [C.POINTER(SU2Params), C.c_double, dp, dp]
        L.orc_su2_forces_at.argtypes = [C.POINTER(SU2Params), C.c_double, pp, pp, pp, pp]
        L.orc_su2_hubble_b0.argtypes = [C.POINTER(SU2Params), pp, pp, pp, pp, C.c_double, dp]
        L.orc_u1_gauss_init.argtypes = [C.POINTER(U1Params), pp, pp, pp, dp]
        L.orc_vv_stages.argtypes = [C.c_int, dp]
        L.orc_vv_stages.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's per-site loops (n > 0 sets them; returns the
    count in use).  Results do not depend on it: volume sums are serial."""
    return lib().orc_set_threads(int(n))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pp(arrs):
    arr = (C.POINTER(C.c_double) * len(arrs))(*[_dp(a) for a in arrs])
    return C.cast(arr, C.POINTER(C.POINTER(C.c_double)))


def _chk(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


# ----------------------------------------------------------------------------
# scalar sector
# ----------------------------------------------------------------------------

@dataclass
class ScalarModel:
    """Run parameters of a real-scalar lattice (program units)."""
    N: int
    dx: float
    dt: float
    nfields: int = 1
    potential: int = PHI4
    expansion: int = NONE
    integrator: int = LF
    lam: float = 1.0
    q: float = 0.0
    alpha: float = 1.0
    kappa2: float = 0.25
    w_eos: float = 1.0 / 3.0
    H0: float = 0.0
    t0: float = 0.0
    a0: float = 1.0

    def cparams(self) -> Params:
        return Params(self.N, self.nfields, self.potential, self.expansion, self.integrator, 0,
                      self.dx, self.dt, self.lam, self.q, self.alpha, self.kappa2, self.w_eos,
                      self.H0, self.t0, self.a0)


class ScalarState:
    """Oracle-side copy of a scalar lattice state (phi, pi per field + clock)."""

    def __init__(self, model: ScalarModel, phi, pi, t=0.0, a=None, b=None, lf_stag=0):
        self.m = model
        self.phi = [np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1)) .copy() for f in phi]
        self.pi = [np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1)).copy() for f in pi]
        assert len(self.phi) == model.nfields and len(self.pi) == model.nfields
        self._p = model.cparams()
        if model.expansion == FIXED:
            aa, bb = fixed_background(model, t)
            a = aa if a is None else a
            b = bb if b is None else b
        elif model.expansion == NONE:
            a, b = 1.0, 0.0
        else:
            a = model.a0 if a is None else a
            if b is None:
                b = hubble_b0(model, self.phi, self.pi, a)
        self.clock = Clock(t, a, b, lf_stag, 0)

    def _arrs(self):
        phi = self.phi + [self.phi[0]] * (2 - len(self.phi))
        pi = self.pi + [self.pi[0]] * (2 - len(self.pi))
        return phi, pi

    def run(self, nsteps: int):
        phi, pi = self._arrs()
        _chk(lib().orc_run(C.byref(self._p), _pp(phi), _pp(pi), C.byref(self.clock), int(nsteps)), "run")
        return self

    def sync(self):
        phi, pi = self._arrs()
        _chk(lib().orc_lf_sync(C.byref(self._p), _pp(phi), _pp(pi), C.byref(self.clock)), "sync")
        return self

    def energy(self) -> dict:
        phi, pi = self._arrs()
        out = np.zeros(12)
        _chk(lib().orc_energy(C.byref(self._p), _pp(phi), _pp(pi), C.byref(self.clock), _dp(out)), "energy")
        return dict(EK=out[0:2].copy(), EG=out[2:4].copy(), EV=out[4:6].copy(), rho=out[6],
                    hubble_lhs=out[7], hubble_rhs=out[8], hubble_res=out[9], a=out[10],
                    b=out[11], t=self.clock.t)

    @property
    def t(self):
        return self.clock.t

    @property
    def a(self):
        return self.clock.a

    @property
    def b(self):
        return self.clock.b


def _side(f: np.ndarray) -> int:
    N = int(round(f.size ** (1.0 / 3.0)))
    assert N ** 3 == f.size, "field size must be N^3"
    return N


def laplacian(f: np.ndarray, dx: float) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    N = _side(f)
    out = np.empty_like(f)
    _chk(lib().orc_laplacian(N, dx, _dp(f), _dp(out)), "laplacian")
    return out


def grad2_sum(f: np.ndarray, dx: float) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_grad2_sum(_side(f), dx, _dp(f))


def kernel(model: ScalarModel, a: float, phi, s: int) -> np.ndarray:
    phi = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in phi]
    phi2 = phi + [phi[0]] * (2 - len(phi))
    out = np.empty_like(phi[0])
    p = model.cparams()
    _chk(lib().orc_kernel(C.byref(p), a, _pp(phi2), s, _dp(out)), "kernel")
    return out


def fixed_background(model: ScalarModel, t: float):
    a, b = C.c_double(), C.c_double()
    p = model.cparams()
    _chk(lib().orc_fixed_background(C.byref(p), t, C.byref(a), C.byref(b)), "fixed_background")
    return a.value, b.value


def hubble_b0(model: ScalarModel, phi, pi, a: float) -> float:
    phi = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in phi]
    pi = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in pi]
    phi2 = phi + [phi[0]] * (2 - len(phi))
    pi2 = pi + [pi[0]] * (2 - len(pi))
    b0 = C.c_double()
    p = model.cparams()
    _chk(lib().orc_hubble_b0(C.byref(p), _pp(phi2), _pp(pi2), a, C.byref(b0)), "hubble_b0")
    return b0.value


def yoshida4():
    w1, w0 = C.c_double(), C.c_double()
    lib().orc_yoshida4(C.byref(w1), C.byref(w0))
    return w1.value, w0.value


def vv_stages(order):
    """Weights (in units of h) of the second-order maps of one velocity-Verlet
    step of the given order (2 ... 10)."""
    w = np.zeros(45)
    n = lib().orc_vv_stages(int(order), _dp(w))
    if n <= 0:
        raise RuntimeError(f"no velocity-Verlet step of order {order}")
    return w[:n].copy()


def triple_jump(n):
    """Weights (x1, x0) raising a symmetric map of order n to order n + 2."""
    x1, x0 = C.c_double(), C.c_double()
    lib().orc_triple_jump(int(n), C.byref(x1), C.byref(x0))
    return x1.value, x0.value


# ----------------------------------------------------------------------------
# adjoint (two fields, VV2, a = 1)
# ----------------------------------------------------------------------------

def vv2_tangent(model: ScalarModel, phi, pi, dphi, dpi, dq=0.0, t=0.0):
    """Advance (phi, pi) and the tangent (dphi, dpi) by one VV2 step from time t in place."""
    p = model.cparams()
    _chk(lib().orc_vv2_tangent(C.byref(p), float(t), _pp(phi), _pp(pi), _pp(dphi), _pp(dpi), dq), "tangent")


def vv2_adjoint_step(model: ScalarModel, phi_n, pi_n, lphi, lpi, t=0.0) -> float:
    """Pull (lphi, lpi) back through one VV2 step from state (phi_n, pi_n) at
    time t; returns dq."""
    p = model.cparams()
    dq = C.c_double(0.0)
    _chk(lib().orc_vv2_adjoint_step(C.byref(p), float(t), _pp(phi_n), _pp(pi_n), _pp(lphi), _pp(lpi),
                                    C.byref(dq)), "adjoint_step")
    return dq.value


# Observables of the adjoint, of field `field`: its energy fraction (0; field
# 1 is the chi fraction) and one bin `bin` >= 1 of its power spectrum of eq.
# discretePS (1).
OBS_ENERGY_FRACTION = 0
OBS_SPECTRUM_BIN = 1


def observable(model: ScalarModel, phi, pi, with_grad=False, kind=OBS_ENERGY_FRACTION, field=1, bin=0, a=1.0):
    """Observable `kind` of the state at scale factor a (and its gradient)."""
    p = model.cparams()
    O = C.c_double()
    if not with_grad:
        null = C.cast(None, C.POINTER(C.POINTER(C.c_double)))
        _chk(lib().orc_observable_kind(C.byref(p), float(a), kind, field, bin, _pp(phi), _pp(pi), C.byref(O), null,
                                       null, None), "obs")
        return O.value
    g = [np.zeros_like(phi[0]) for _ in range(2)]
    gp = [np.zeros_like(phi[0]) for _ in range(2)]
    dq = C.c_double()
    _chk(lib().orc_observable_kind(C.byref(p), float(a), kind, field, bin, _pp(phi), _pp(pi), C.byref(O), _pp(g),
                                   _pp(gp), C.byref(dq)), "obs")
    return O.value, g, gp, dq.value


def adjoint_vv2(model: ScalarModel, phi0, pi0, nsteps: int, kind=OBS_ENERGY_FRACTION, field=1, bin=0, t=0.0):
    """O(final), dO/dphi(0) per field, dO/dpi(0) per field, dO/dq, for nsteps
    VV2 steps from time t (a = 1, or the fixed background a(t))."""
    phi0 = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in phi0]
    pi0 = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in pi0]
    g = [np.zeros_like(phi0[0]) for _ in range(2)]
    gp = [np.zeros_like(phi0[0]) for _ in range(2)]
    O, dq = C.c_double(), C.c_double()
    p = model.cparams()
    _chk(lib().orc_adjoint_vv2_kind(C.byref(p), float(t), kind, field, bin, _pp(phi0), _pp(pi0), int(nsteps),
                                    C.byref(O), _pp(g), _pp(gp), C.byref(dq)), "adjoint_vv2")
    return O.value, g, gp, dq.value


def adjoint_vv2_self(model: ScalarModel, phi0, pi0, a0, b0, nsteps: int, kind=OBS_ENERGY_FRACTION, field=1,
                     bin=0):
    """Self-consistent expansion: O(final), dO/dphi(0), dO/dpi(0) per field,
    dO/dq, dO/da0, dO/db0 (b0 taken as an independent input)."""
    phi0 = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in phi0]
    pi0 = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in pi0]
    g = [np.zeros_like(phi0[0]) for _ in range(2)]
    gp = [np.zeros_like(phi0[0]) for _ in range(2)]
    O, dq, da, db = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    p = model.cparams()
    _chk(lib().orc_adjoint_vv2_self(C.byref(p), kind, field, bin, _pp(phi0), _pp(pi0), float(a0), float(b0),
                                    int(nsteps), C.byref(O), _pp(g), _pp(gp), C.byref(dq), C.byref(da),
                                    C.byref(db)), "adjoint_vv2_self")
    return O.value, g, gp, dq.value, da.value, db.value


# ----------------------------------------------------------------------------
# U(1) sector (a = 1, leapfrog)
# ----------------------------------------------------------------------------

@dataclass
class U1Model:
    N: int
    dx: float
    dt: float
    lam: float = 1.0
    v: float = 1.0
    e: float = 0.5
    kappa_g: float = 1.0
    expansion: int = NONE
    alpha: float = 1.0
    kappa2: float = 0.25
    w_eos: float = 1.0 / 3.0
    H0: float = 0.0
    t0: float = 0.0
    a0: float = 1.0

    def cparams(self) -> U1Params:
        return U1Params(self.N, self.expansion, self.dx, self.dt, self.lam, self.v, self.e, self.kappa_g,
                        self.alpha, self.kappa2, self.w_eos, self.H0, self.t0, self.a0)


class U1State:
    """phi: 2 real components, pi: 2, A: 3 link fields, piA: 3 (each N^3).
    With expansion the clock holds a and b = a' (fixed background: the closed
    form at t; self-consistent: a0 and b from the Hubble constraint unless given)."""

    def __init__(self, model: U1Model, phi, pi, A, piA, t=0.0, lf_stag=0, a=None, b=None):
        self.m = model
        cp = lambda L: [np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1)).copy() for f in L]
        self.phi, self.pi, self.A, self.piA = cp(phi), cp(pi), cp(A), cp(piA)
        self._p = model.cparams()
        if model.expansion == FIXED:
            aa, bb = C.c_double(), C.c_double()
            _chk(lib().orc_u1_fixed_background(C.byref(self._p), float(t), C.byref(aa), C.byref(bb)), "u1 fixed")
            a = aa.value if a is None else a
            b = bb.value if b is None else b
        elif model.expansion == SELF:
            a = model.a0 if a is None else a
            if b is None:
                bb = C.c_double()
                _chk(lib().orc_u1_hubble_b0(C.byref(self._p), *self._args(), float(a), C.byref(bb)), "u1 b0")
                b = bb.value
        else:
            a, b = 1.0, 0.0
        self.clock = Clock(t, a, b, lf_stag, 0)

    @property
    def a(self):
        return self.clock.a

    @property
    def b(self):
        return self.clock.b

    @property
    def t(self):
        return self.clock.t

    def _args(self):
        return _pp(self.phi), _pp(self.pi), _pp(self.A), _pp(self.piA)

    def run(self, nsteps: int):
        _chk(lib().orc_u1_run_lf(C.byref(self._p), *self._args(), C.byref(self.clock), int(nsteps)), "u1 run")
        return self

    def sync(self):
        _chk(lib().orc_u1_lf_sync(C.byref(self._p), *self._args(), C.byref(self.clock)), "u1 sync")
        return self

    def energy(self) -> dict:
        out = np.zeros(17)
        _chk(lib().orc_u1_energy(C.byref(self._p), *self._args(), C.byref(self.clock), _dp(out)), "u1 energy")
        d = _u1_dict(out)
        d.update(a=out[12], b=out[13], hubble_lhs=out[14], hubble_rhs=out[15], hubble_res=out[16],
                 t=self.clock.t)
        return d

    def gauss(self) -> dict:
        out = np.zeros(12)
        _chk(lib().orc_u1_gauss(C.byref(self._p), *self._args(), _dp(out)), "u1 gauss")
        return _u1_dict(out)

    def run_vv(self, nsteps: int, order: int = 2):
        """nsteps of the velocity-Verlet map of the given order (2 ... 10)."""
        _chk(lib().orc_u1_run_vv(C.byref(self._p), *self._args(), C.byref(self.clock), int(nsteps), int(order)),
             "u1 run vv")
        return self

    def gauss_init(self):
        """pi_A from the lattice Gauss law; returns <rho>."""
        mean = np.zeros(1)
        _chk(lib().orc_u1_gauss_init(C.byref(self._p), _pp(self.phi), _pp(self.pi), _pp(self.piA), _dp(mean)),
             "u1 gauss init")
        return mean

    def forces_at(self, a):
        """Forces (kicks per unit time) at scale factor a."""
        F = [np.zeros_like(self.phi[0]) for _ in range(5)]
        _chk(lib().orc_u1_forces_at(C.byref(self._p), float(a), _pp(self.phi), _pp(self.A), _pp(F[:2]), _pp(F[2:])),
             "u1 forces at a")
        return F[:2], F[2:]

    def forces(self):
        F = [np.zeros_like(self.phi[0]) for _ in range(5)]
        _chk(lib().orc_u1_forces(C.byref(self._p), _pp(self.phi), _pp(self.A), _pp(F[:2]), _pp(F[2:])), "u1 forces")
        return F[:2], F[2:]


def _u1_dict(out):
    return dict(EK_phi=out[0], EG_phi=out[1], EV=out[2], EK_A=out[3], EG_A=out[4], rho=out[5],
                gauss_max=out[6], div_max=out[7], charge_max=out[8], gauss_mean=out[9],
                gauss_sum_mean=out[10], gauss_abs_mean=out[11])


# ----------------------------------------------------------------------------
# SU(2) sector (doublet + SU(2) links, a = 1)
# ----------------------------------------------------------------------------

@dataclass
class SU2Model:
    N: int
    dx: float
    dt: float
    lam: float = 1.0
    v: float = 1.0
    g: float = 0.5
    expansion: int = NONE
    alpha: float = 1.0
    kappa2: float = 0.25
    w_eos: float = 1.0 / 3.0
    H0: float = 0.0
    t0: float = 0.0
    a0: float = 1.0

    def cparams(self) -> SU2Params:
        return SU2Params(self.N, self.expansion, self.dx, self.dt, self.lam, self.v, self.g, self.alpha,
                         self.kappa2, self.w_eos, self.H0, self.t0, self.a0)


class SU2State:
    """phi: 4 real doublet components, pi: 4, U: 12 link arrays (link i, quaternion
    component k at index 4 i + k), E: 9 electric arrays (link i, colour a at 3 i + a).
    With expansion the clock holds a and b = a' (fixed background: the closed
    form at t; self-consistent: a0 and b from the Hubble constraint unless given)."""

    def __init__(self, model: SU2Model, phi, pi, U, E, t=0.0, lf_stag=0, a=None, b=None):
        self.m = model
        cp = lambda L: [np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1)).copy() for f in L]
        self.phi, self.pi, self.U, self.E = cp(phi), cp(pi), cp(U), cp(E)
        assert len(self.phi) == 4 and len(self.pi) == 4 and len(self.U) == 12 and len(self.E) == 9
        self._p = model.cparams()
        if model.expansion == FIXED:
            aa, bb = C.c_double(), C.c_double()
            _chk(lib().orc_su2_fixed_background(C.byref(self._p), float(t), C.byref(aa), C.byref(bb)), "su2 fixed")
            a = aa.value if a is None else a
            b = bb.value if b is None else b
        elif model.expansion == SELF:
            a = model.a0 if a is None else a
            if b is None:
                bb = C.c_double()
                _chk(lib().orc_su2_hubble_b0(C.byref(self._p), *self._args(), float(a), C.byref(bb)), "su2 b0")
                b = bb.value
        else:
            a, b = 1.0, 0.0
        self.clock = Clock(t, a, b, lf_stag, 0)

    @property
    def a(self):
        return self.clock.a

    @property
    def b(self):
        return self.clock.b

    @property
    def t(self):
        return self.clock.t

    def _args(self):
        return _pp(self.phi), _pp(self.pi), _pp(self.U), _pp(self.E)

    def run(self, nsteps: int):
        _chk(lib().orc_su2_run_lf(C.byref(self._p), *self._args(), C.byref(self.clock), int(nsteps)), "su2 run")
        return self

    def sync(self):
        _chk(lib().orc_su2_lf_sync(C.byref(self._p), *self._args(), C.byref(self.clock)), "su2 sync")
        return self

    def energy(self) -> dict:
        out = np.zeros(17)
        _chk(lib().orc_su2_energy(C.byref(self._p), *self._args(), C.byref(self.clock), _dp(out)), "su2 energy")
        d = _su2_dict(out)
        d.update(a=out[12], b=out[13], hubble_lhs=out[14], hubble_rhs=out[15], hubble_res=out[16],
                 t=self.clock.t)
        return d

    def forces_at(self, a):
        """Forces (kicks per unit time) at scale factor a."""
        F = [np.zeros_like(self.phi[0]) for _ in range(13)]
        _chk(lib().orc_su2_forces_at(C.byref(self._p), float(a), _pp(self.phi), _pp(self.U), _pp(F[:4]),
                                     _pp(F[4:])), "su2 forces at a")
        return F[:4], F[4:]

    def gauss(self) -> dict:
        out = np.zeros(12)
        _chk(lib().orc_su2_gauss(C.byref(self._p), *self._args(), _dp(out)), "su2 gauss")
        return _su2_dict(out)

    def run_vv(self, nsteps: int, order: int = 2):
        """nsteps of the velocity-Verlet map of the given order (2 ... 10)."""
        _chk(lib().orc_su2_run_vv(C.byref(self._p), *self._args(), C.byref(self.clock), int(nsteps), int(order)),
             "su2 run vv")
        return self

    def gauss_init(self):
        """E from the lattice Gauss law (links at the identity); returns <rho^a>."""
        mean = np.zeros(3)
        _chk(lib().orc_su2_gauss_init(C.byref(self._p), *self._args(), _dp(mean)), "su2 gauss init")
        return mean

    def forces(self):
        F = [np.zeros_like(self.phi[0]) for _ in range(13)]
        _chk(lib().orc_su2_forces(C.byref(self._p), _pp(self.phi), _pp(self.U), _pp(F[:4]), _pp(F[4:])),
             "su2 forces")
        return F[:4], F[4:]


def _su2_dict(out):
    return dict(EK_phi=out[0], EG_phi=out[1], EV=out[2], EK_B=out[3], EG_B=out[4], rho=out[5],
                gauss_max=out[6], div_max=out[7], charge_max=out[8], gauss_mean=out[9],
                gauss_sum_mean=out[10], gauss_abs_mean=out[11])


def gauss_solve(rho, dx):
    """E_i = grad+_i Lap^-1 (rho - <rho>) of a real N^3 array (the oracle's own DFT)."""
    rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(-1))
    N = _side(rho)
    E = [np.zeros_like(rho) for _ in range(3)]
    _chk(lib().orc_gauss_solve(N, dx, _dp(rho), _pp(E)), "gauss solve")
    return E


def spectrum_bins(N):
    """Number of radial bins that hold every mode of an N^3 lattice."""
    h = N // 2
    return int(math.isqrt(3 * h * h)) + 1


def spectrum(f, dx, nbins=None):
    """Power spectrum of one field (eq. discretePS): per radial bin b (modes with
    b <= |n| < b + 1) the sum of |f~|^2 of the unnormalised DFT, the discrete
    spectrum Delta(b) and the number of modes."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    N = int(round(len(f) ** (1 / 3)))
    assert N ** 3 == len(f)
    nb = spectrum_bins(N) if nbins is None else int(nbins)
    s, d, c = np.zeros(nb), np.zeros(nb), np.zeros(nb, dtype=np.int64)
    r = lib().orc_spectrum(N, dx, f.ctypes.data_as(C.POINTER(C.c_double)), nb,
                           s.ctypes.data_as(C.POINTER(C.c_double)), d.ctypes.data_as(C.POINTER(C.c_double)),
                           c.ctypes.data_as(C.POINTER(C.c_long)))
    if r < 0:
        raise RuntimeError("orc_spectrum failed")
    return s, d, c


def occupation(model: ScalarModel, a, bdot, phi, pi, field, fstar2=1.0, nbins=None):
    """Lattice occupation number of field `field` per radial bin (eq.
    OccuppationNum) for fields and momenta at the same time, scale factor a and
    its derivative bdot; returns (n, count)."""
    phi = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in phi]
    pi = [np.ascontiguousarray(f, dtype=np.float64).reshape(-1) for f in pi]
    N = model.N
    nb = spectrum_bins(N) if nbins is None else int(nbins)
    n, c = np.zeros(nb), np.zeros(nb, dtype=np.int64)
    p = model.cparams()
    r = lib().orc_occupation(C.byref(p), float(a), float(bdot), _pp(phi), _pp(pi), int(field), float(fstar2), nb,
                             n.ctypes.data_as(C.POINTER(C.c_double)), c.ctypes.data_as(C.POINTER(C.c_long)))
    if r < 0:
        raise RuntimeError("orc_occupation failed")
    return n, c
