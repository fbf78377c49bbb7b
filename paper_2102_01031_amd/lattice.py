"""Thin ctypes binding of the C ABI in include/lattice.h.

Argument marshalling only: torch tensors supply device memory and the stream;
every step of the lattice update runs in the HIP library.  The library must be
built (``__graft_entry__.build()``); importing works without it, but creating a
``Lattice`` raises if ``csrc/liblattice.so`` is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "csrc", "liblattice.so")

LAT_OK, LAT_EINVAL, LAT_EUNSUPPORTED, LAT_ENODEV, LAT_EHIP, LAT_ESTATE, LAT_ENOMEM = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "LAT_OK", -1: "LAT_EINVAL", -2: "LAT_EUNSUPPORTED", -3: "LAT_ENODEV", -4: "LAT_EHIP",
                -5: "LAT_ESTATE", -6: "LAT_ENOMEM"}
INTEGRATORS = {"lf": 0, "vv2": 1, "vv4": 2, "vv6": 3, "vv8": 4, "vv10": 5}
EXPANSIONS = {"none": 0, "fixed": 1, "self": 2}
POTENTIALS = {"phi4": 0, "phi4_chi2": 1, "abelian_higgs": 2, "su2_higgs": 3}
PRECISIONS = {"f64": 0, "f32": 1}


class LatParams(C.Structure):
    _fields_ = [("N", C.c_int32), ("integrator", C.c_int32), ("expansion", C.c_int32),
                ("potential", C.c_int32), ("precision", C.c_int32), ("lf_staggered", C.c_int32),
                ("reserved0", C.c_int32), ("reserved1", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double), ("t0", C.c_double), ("alpha", C.c_double),
                ("lam", C.c_double), ("q", C.c_double), ("v", C.c_double), ("e_charge", C.c_double),
                ("kappa_g", C.c_double), ("kappa2", C.c_double), ("w_eos", C.c_double),
                ("H0", C.c_double), ("t_ref", C.c_double), ("a0", C.c_double), ("b0", C.c_double)]


class LatFields(C.Structure):
    _fields_ = [("phi", C.c_void_p * 2), ("pi", C.c_void_p * 2), ("A", C.c_void_p * 3),
                ("piA", C.c_void_p * 3), ("doublet", C.c_void_p * 4), ("pi_doublet", C.c_void_p * 4),
                ("U", C.c_void_p * 12), ("E", C.c_void_p * 9)]


class LatEnergies(C.Structure):
    _fields_ = [("t", C.c_double), ("a", C.c_double), ("b", C.c_double), ("EK", C.c_double * 2),
                ("EG", C.c_double * 2), ("EV", C.c_double * 2), ("EK_A", C.c_double),
                ("EG_A", C.c_double), ("rho", C.c_double), ("hubble_lhs", C.c_double),
                ("hubble_rhs", C.c_double), ("hubble_res", C.c_double), ("gauss_max", C.c_double),
                ("gauss_div_max", C.c_double), ("gauss_charge_max", C.c_double),
                ("gauss_mean", C.c_double), ("gauss_sum_mean", C.c_double), ("step", C.c_int64),
                ("EK_B", C.c_double), ("EG_B", C.c_double), ("gauss_abs_mean", C.c_double)]


# kind 6 "gauge": the U(1) and SU(2) leapfrog, sync and energy passes
KERNEL_KINDS = ["kick", "kick_red", "drift_kick", "drift_kick_red", "kick_drift", "energy", "gauge", "adjoint"]


# observable name -> (enum lat_observable, field forced by the name or None)
OBSERVABLES = {"chi_fraction": (0, 1), "energy_fraction": (0, None), "spectrum_bin": (1, None)}


class LatGradSpec(C.Structure):
    _fields_ = [("observable", C.c_int32), ("field", C.c_int32), ("nsteps", C.c_int64),
                ("checkpoint_stride", C.c_int64), ("bin", C.c_int32), ("reserved", C.c_int32)]


class LatGradOut(C.Structure):
    _fields_ = [("value", C.c_double), ("dO_dq", C.c_double), ("dO_dphi", C.c_void_p * 2),
                ("dO_dpi", C.c_void_p * 2), ("forward_ms", C.c_double), ("reverse_ms", C.c_double),
                ("dO_da0", C.c_double), ("dO_db0", C.c_double)]


class LatStats(C.Structure):
    _fields_ = [("launches", C.c_int64 * 8), ("kernel_ms", C.c_double * 8), ("blocks", C.c_int32),
                ("threads", C.c_int32), ("tile_x", C.c_int32), ("tile_y", C.c_int32),
                ("z_chunk", C.c_int32), ("pad", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.lattice_init.argtypes = [C.POINTER(vp), C.POINTER(LatParams), C.POINTER(LatFields), vp]
        L.lattice_init.restype = C.c_int
        L.lattice_step.argtypes = [vp, C.c_int64]
        L.lattice_step.restype = C.c_int
        L.lattice_sync.argtypes = [vp]
        L.lattice_sync.restype = C.c_int
        L.lattice_energy.argtypes = [vp, C.POINTER(LatEnergies)]
        L.lattice_energy.restype = C.c_int
        L.lattice_destroy.argtypes = [vp]
        L.lattice_destroy.restype = None
        L.lattice_last_error.argtypes = [vp]
        L.lattice_last_error.restype = C.c_char_p
        L.lattice_version.restype = C.c_char_p
        L.lattice_stats.argtypes = [vp, C.c_int, C.POINTER(LatStats)]
        L.lattice_stats.restype = C.c_int
        L.lattice_profile.argtypes = [vp, C.c_int]
        L.lattice_profile.restype = C.c_int
        L.lattice_grad.argtypes = [vp, C.POINTER(LatGradSpec), C.POINTER(LatGradOut)]
        L.lattice_grad.restype = C.c_int
        dp = C.POINTER(C.c_double)
        L.lattice_spectrum.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, dp, dp, C.POINTER(C.c_int64)]
        L.lattice_spectrum.restype = C.c_int
        L.lattice_occupation.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, dp, C.POINTER(C.c_int64)]
        L.lattice_occupation.restype = C.c_int
        L.lattice_gauss_init.argtypes = [vp, dp]
        L.lattice_gauss_init.restype = C.c_int
        L.lattice_init_batch.argtypes = [C.POINTER(vp), C.POINTER(LatParams), C.c_int32, C.POINTER(C.c_int32),
                                         C.POINTER(LatFields), C.c_int32, vp]
        L.lattice_init_batch.restype = C.c_int
        L.lattice_energy_batch.argtypes = [vp, C.c_int32, C.POINTER(LatEnergies)]
        L.lattice_energy_batch.restype = C.c_int
        L.lattice_batch_tile.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32)]
        L.lattice_batch_tile.restype = C.c_int
        L.lattice_energy_noalloc.argtypes = [C.POINTER(LatParams), C.POINTER(LatFields), vp, vp]
        L.lattice_energy_noalloc.restype = C.c_int
        _lib = L
    return _lib


def declared_symbols(header: str | None = None) -> list[str]:
    """Names of the functions declared in include/lattice.h."""
    header = header or os.path.join(os.path.dirname(HERE), "include", "lattice.h")
    txt = open(header).read()
    return sorted(set(re.findall(r"\b(lattice_\w+)\s*\(", txt)))


class LatticeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code, ctx=None):
    if code != LAT_OK:
        msg = lib().lattice_last_error(ctx).decode()
        raise LatticeError(code, msg)


def make_params(N, dx, dt, integrator="lf", expansion="none", potential="phi4", precision="f64", t0=0.0,
                alpha=1.0, lam=1.0, q=0.0, v=1.0, e=0.5, kappa_g=1.0, kappa2=0.25, w_eos=1.0 / 3.0, H0=0.0,
                t_ref=0.0, a0=1.0, b0=math.nan, lf_staggered=0, g=None) -> LatParams:
    """g: the SU(2) coupling g_B Q_B (the same parameter slot as the U(1) charge e)."""
    if g is not None:
        e = g
    return LatParams(N, INTEGRATORS[integrator], EXPANSIONS[expansion], POTENTIALS[potential],
                     PRECISIONS[precision], lf_staggered, 0, 0, dx, dt, t0, alpha, lam, q, v, e, kappa_g,
                     kappa2, w_eos, H0, t_ref, a0, b0)


class Lattice:
    """One lattice context bound to torch tensors (state is updated in place).

    phi, pi: lists of contiguous CUDA tensors of N^3 elements (float64, or float32
    with precision="f32").  For the Abelian-Higgs model also A and piA (3 each).
    For the SU(2) model (potential="su2_higgs", coupling g=...) phi and pi stay
    empty and doublet, pi_doublet (4 each), U (12: link i, quaternion component
    k at 4 i + k) and E (9: link i, colour a at 3 i + a) carry the state.
    """

    def __init__(self, phi=(), pi=(), *, A=None, piA=None, doublet=None, pi_doublet=None, U=None, E=None,
                 stream=None, **kw):
        import torch
        self._torch = torch
        self.params = make_params(**kw)
        dtype = torch.float32 if kw.get("precision", "f64") == "f32" else torch.float64
        N = kw["N"]
        self._keep = (list(phi) + list(pi) + list(A or []) + list(piA or []) + list(doublet or [])
                      + list(pi_doublet or []) + list(U or []) + list(E or []))
        for t in self._keep:
            if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype and t.numel() == N ** 3):
                raise ValueError("fields must be contiguous CUDA tensors of N^3 elements with the run's dtype")
        f = LatFields()
        for i, t in enumerate(phi):
            f.phi[i] = t.data_ptr()
        for i, t in enumerate(pi):
            f.pi[i] = t.data_ptr()
        for i, t in enumerate(A or []):
            f.A[i] = t.data_ptr()
        for i, t in enumerate(piA or []):
            f.piA[i] = t.data_ptr()
        for name, ts in (("doublet", doublet), ("pi_doublet", pi_doublet), ("U", U), ("E", E)):
            arr = getattr(f, name)
            for i, t in enumerate(ts or []):
                arr[i] = t.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._ctx = C.c_void_p()
        rc = lib().lattice_init(C.byref(self._ctx), C.byref(self.params), C.byref(f),
                                C.c_void_p(stream.cuda_stream))
        _check(rc, None)

    def step(self, n: int):
        _check(lib().lattice_step(self._ctx, int(n)), self._ctx)
        return self

    def sync(self):
        _check(lib().lattice_sync(self._ctx), self._ctx)
        return self

    def energy(self) -> dict:
        e = LatEnergies()
        _check(lib().lattice_energy(self._ctx, C.byref(e)), self._ctx)
        return dict(t=e.t, a=e.a, b=e.b, EK=list(e.EK), EG=list(e.EG), EV=list(e.EV), EK_A=e.EK_A,
                    EG_A=e.EG_A, rho=e.rho, hubble_lhs=e.hubble_lhs, hubble_rhs=e.hubble_rhs,
                    hubble_res=e.hubble_res, gauss_max=e.gauss_max, gauss_div_max=e.gauss_div_max,
                    gauss_charge_max=e.gauss_charge_max, gauss_mean=e.gauss_mean,
                    gauss_sum_mean=e.gauss_sum_mean, step=e.step, EK_B=e.EK_B, EG_B=e.EG_B,
                    gauss_abs_mean=e.gauss_abs_mean)

    def spectrum(self, field: int = 0, array: str = "phi", nbins: int | None = None) -> dict:
        """Discrete power spectrum (eq. discretePS) of one stored array, computed
        on the device: per radial bin b (modes with b <= |n| < b + 1) the sum of
        |f~|^2, the mode count, k_b = b k_IR and Delta(b)."""
        import math

        import numpy as np
        N = self.params.N
        nb = int(math.isqrt(3 * (N // 2) ** 2)) + 1 if nbins is None else int(nbins)
        s, d = np.zeros(nb), np.zeros(nb)
        c = np.zeros(nb, dtype=np.int64)
        dp = C.POINTER(C.c_double)
        _check(lib().lattice_spectrum(self._ctx, int(field), {"phi": 0, "pi": 1}[array], nb,
                                      s.ctypes.data_as(dp), d.ctypes.data_as(dp),
                                      c.ctypes.data_as(C.POINTER(C.c_int64))), self._ctx)
        kir = 2 * math.pi / (N * self.params.dx)
        return dict(sum=s, delta=d, count=c, k=kir * np.arange(nb))

    def occupation(self, field: int = 0, nbins: int | None = None, fstar2: float = 1.0) -> dict:
        """Lattice occupation number (eq. OccuppationNum) of one real field per
        radial bin, computed on the device from phi, pi, a and a' at the current
        time; fstar2 = (f_star/omega_star)^2.  Leapfrog momenta must be synced."""
        import math

        import numpy as np
        N = self.params.N
        nb = int(math.isqrt(3 * (N // 2) ** 2)) + 1 if nbins is None else int(nbins)
        n, c = np.zeros(nb), np.zeros(nb, dtype=np.int64)
        _check(lib().lattice_occupation(self._ctx, int(field), nb, float(fstar2),
                                        n.ctypes.data_as(C.POINTER(C.c_double)),
                                        c.ctypes.data_as(C.POINTER(C.c_int64))), self._ctx)
        kir = 2 * math.pi / (N * self.params.dx)
        return dict(n=n, count=c, k=kir * np.arange(nb))

    def gauss_init(self):
        """Set the gauge momenta (SU(2): E, U(1): piA) to the longitudinal solution
        of the lattice Gauss law for the stored scalar and momenta, on the device;
        returns the homogeneous charge <rho^a> per colour (one value for U(1))."""
        import numpy as np
        mean = np.zeros(3)
        _check(lib().lattice_gauss_init(self._ctx, mean.ctypes.data_as(C.POINTER(C.c_double))), self._ctx)
        return mean if self.params.potential == POTENTIALS["su2_higgs"] else mean[:1]

    def grad(self, nsteps: int, stride: int = 0, want_phi: bool = True, want_pi: bool = True,
             observable: str = "chi_fraction", field: int = 0, bin: int = 0) -> dict:
        """An observable after nsteps and its gradient with respect to the current
        phi, pi (both fields) and q (hand-written adjoint in the library).
        observable: "chi_fraction", the energy fraction in chi; "energy_fraction",
        that of field `field`; "spectrum_bin", Delta(bin) of field `field`
        (eq. discretePS)."""
        torch = self._torch
        N = self.params.N
        kind, forced = OBSERVABLES[observable]
        if forced is not None:
            field = forced
        spec = LatGradSpec(kind, int(field), int(nsteps), int(stride), int(bin), 0)
        out = LatGradOut()
        gphi = [torch.empty(N ** 3, dtype=torch.float64, device="cuda") for _ in range(2)] if want_phi else None
        gpi = [torch.empty(N ** 3, dtype=torch.float64, device="cuda") for _ in range(2)] if want_pi else None
        for i in range(2):
            out.dO_dphi[i] = gphi[i].data_ptr() if gphi else None
            out.dO_dpi[i] = gpi[i].data_ptr() if gpi else None
        _check(lib().lattice_grad(self._ctx, C.byref(spec), C.byref(out)), self._ctx)
        return dict(value=out.value, dO_dq=out.dO_dq, dO_dphi=gphi, dO_dpi=gpi, forward_ms=out.forward_ms,
                    reverse_ms=out.reverse_ms, dO_da0=out.dO_da0, dO_db0=out.dO_db0)

    def profile(self, enable: bool = True):
        _check(lib().lattice_profile(self._ctx, 1 if enable else 0), self._ctx)
        return self

    def stats(self, reset: bool = False) -> dict:
        s = LatStats()
        _check(lib().lattice_stats(self._ctx, 1 if reset else 0, C.byref(s)), self._ctx)
        return dict(launches={k: s.launches[i] for i, k in enumerate(KERNEL_KINDS)},
                    kernel_ms={k: s.kernel_ms[i] for i, k in enumerate(KERNEL_KINDS)},
                    blocks=s.blocks, threads=s.threads, tile=(s.tile_x, s.tile_y), z_chunk=s.z_chunk)

    def close(self):
        if self._ctx:
            lib().lattice_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _energy_dict(e):
    return dict(t=e.t, a=e.a, b=e.b, EK=list(e.EK), EG=list(e.EG), EV=list(e.EV), rho=e.rho, step=e.step)


class LatticeBatch:
    """Batch of independent single-field lattices (sizes may differ) stepped by
    batched launches (cache-sized segments of realizations, all steps of a call
    per segment), replayed from a captured HIP graph.

    phis, pis: lists (one entry per realization) of contiguous CUDA tensors of
    N_r^3 elements.  Other keyword arguments as for Lattice (N is ignored)."""

    def __init__(self, phis, pis, sizes, *, autotune=True, stream=None, **kw):
        import torch
        kw = dict(kw)
        kw.setdefault("N", int(sizes[0]))
        self.params = make_params(**kw)
        dtype = torch.float32 if kw.get("precision", "f64") == "f32" else torch.float64
        n = len(sizes)
        self.sizes = [int(v) for v in sizes]
        self._keep = list(phis) + list(pis)
        fa = (LatFields * n)()
        for r in range(n):
            for t in (phis[r], pis[r]):
                if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype and t.numel() == self.sizes[r] ** 3):
                    raise ValueError("fields must be contiguous CUDA tensors of N_r^3 elements with the run's dtype")
            fa[r].phi[0] = phis[r].data_ptr()
            fa[r].pi[0] = pis[r].data_ptr()
        Ns = (C.c_int32 * n)(*self.sizes)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._ctx = C.c_void_p()
        _check(lib().lattice_init_batch(C.byref(self._ctx), C.byref(self.params), n, Ns, fa,
                                        1 if autotune else 0, C.c_void_p(stream.cuda_stream)), None)

    def step(self, n: int):
        _check(lib().lattice_step(self._ctx, int(n)), self._ctx)
        return self

    def sync(self):
        _check(lib().lattice_sync(self._ctx), self._ctx)
        return self

    def energy(self, r: int) -> dict:
        e = LatEnergies()
        _check(lib().lattice_energy_batch(self._ctx, int(r), C.byref(e)), self._ctx)
        return _energy_dict(e)

    def tile(self, N: int):
        tx, ty, zc = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lattice_batch_tile(self._ctx, int(N), C.byref(tx), C.byref(ty), C.byref(zc)), self._ctx)
        return tx.value, ty.value, zc.value

    def close(self):
        if self._ctx:
            lib().lattice_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def energy_noalloc(phi, pi, out, *, stream=None, **kw):
    """lattice_energy_noalloc: energies of the real scalar state (phi, pi) (lists
    of CUDA tensors as for Lattice) enqueued on the stream without a context or
    any allocation; out: a CUDA float64 tensor of 8 elements receiving EK[0],
    EK[1], EG[0], EG[1], EV[0], EV[1], rho, a.  Other keywords as for Lattice."""
    import torch
    params = make_params(**kw)
    dtype = torch.float32 if kw.get("precision", "f64") == "f32" else torch.float64
    N = kw["N"]
    for t in list(phi) + list(pi):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype and t.numel() == N ** 3):
            raise ValueError("fields must be contiguous CUDA tensors of N^3 elements with the run's dtype")
    if not (out.is_cuda and out.is_contiguous() and out.dtype == torch.float64 and out.numel() >= 8):
        raise ValueError("out must be a contiguous CUDA float64 tensor of at least 8 elements")
    f = LatFields()
    for i, t in enumerate(phi):
        f.phi[i] = t.data_ptr()
    for i, t in enumerate(pi):
        f.pi[i] = t.data_ptr()
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().lattice_energy_noalloc(C.byref(params), C.byref(f), C.c_void_p(out.data_ptr()),
                                        C.c_void_p(stream.cuda_stream)), None)
    return out
