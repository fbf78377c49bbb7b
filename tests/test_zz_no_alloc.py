"""lattice_energy_noalloc (the allocation-free variant of lattice_energy for
callers that cannot allocate) against lattice_energy on a context created with
the same parameters and fields: two calls in a row on the same GPU, the second
on a smaller lattice, each within 1e-12 of lattice_energy (the parity bar of
the float64 path; float32 fields reduce in float64 on both sides)."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import say, to_dev
from paper_2102_01031_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [
    # (workload, N, precision, integrator, expansion, extra params)
    (workloads.PREHEAT_128, 64, "f64", "vv4", "self", dict(a0=1.3)),
    (workloads.LPHI4_32, 20, "f32", "lf", "fixed", dict(t0=0.7, lf_staggered=1)),
]


def _kw(wl, N, precision, integrator, expansion, extra):
    kw = dict(N=N, dx=wl.dx, dt=wl.dt, integrator=integrator, expansion=expansion, potential=wl.potential,
              lam=wl.lam, q=wl.q, alpha=wl.alpha, kappa2=wl.kappa2, w_eos=wl.w_eos, H0=wl.H0, a0=wl.a0,
              precision=precision)
    kw.update(extra)
    return kw


def _noalloc_raw(kw, tp, tq, out, stream):
    """Call through the C ABI with ctypes (no binding logic in between)."""
    from paper_2102_01031_amd import lattice as L
    p = L.make_params(**kw)
    f = L.LatFields()
    for i, t in enumerate(tp):
        f.phi[i] = t.data_ptr()
    for i, t in enumerate(tq):
        f.pi[i] = t.data_ptr()
    return L.lib().lattice_energy_noalloc(C.byref(p), C.byref(f), C.c_void_p(out.data_ptr()),
                                          C.c_void_p(stream.cuda_stream))


def test_noalloc_energy_matches_lattice_energy_twice():
    import torch
    from paper_2102_01031_amd.lattice import LAT_OK, Lattice
    stream = torch.cuda.current_stream()
    outs = []
    for wl, N, prec, integ, expn, extra in CASES:
        say(f"[noalloc] {wl.name} N={N} {prec} {integ} {expn} {extra}")
        phi, pi = wl.initial_fields(N=N)
        dt = torch.float32 if prec == "f32" else torch.float64
        tp, tq = to_dev(phi, dt), to_dev(pi, dt)
        kw = _kw(wl, N, prec, integ, expn, extra)
        out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc_raw(kw, tp, tq, out, stream) == LAT_OK
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        outs.append((out, got.copy()))
        # the existing entry point on a context created with the same p and f
        lat = Lattice(tp, tq, **kw)
        e = lat.energy()
        lat.close()
        nf = 2 if wl.potential == "phi4_chi2" else 1
        want = np.array([e["EK"][0], e["EK"][1], e["EG"][0], e["EG"][1], e["EV"][0], e["EV"][1], e["rho"], e["a"]])
        for i in range(8):
            if (i % 2 == 1 and i < 6) and nf == 1:
                assert got[i] == 0.0
                continue
            assert abs(got[i] - want[i]) <= 1e-12 * abs(want[i]), (i, got[i], want[i])
        say(f"[noalloc]   rho {got[6]:.15e} vs {want[6]:.15e}, a {got[7]:.15f}; "
            f"max rel diff {np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300)):.2e}")
        # the fields are untouched
        for s in range(len(tp)):
            assert np.array_equal(tp[s].cpu().numpy(), np.asarray(phi[s], dtype=np.float32 if prec == "f32" else np.float64).reshape(-1))
            assert np.array_equal(tq[s].cpu().numpy(), np.asarray(pi[s], dtype=np.float32 if prec == "f32" else np.float64).reshape(-1))
    # the first call's output is not disturbed by the second call
    first, first_vals = outs[0]
    assert np.array_equal(first.cpu().numpy(), first_vals)


def test_noalloc_energy_binding_and_refusals():
    import torch
    from paper_2102_01031_amd.lattice import LatticeError, energy_noalloc
    wl = workloads.LPHI4_32
    N = 16
    phi, pi = wl.initial_fields(N=N)
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    kw = dict(N=N, dx=wl.dx, dt=wl.dt, integrator="vv2", expansion="none", potential="phi4", lam=wl.lam)
    energy_noalloc(tp, tq, out, **kw)
    torch.cuda.synchronize()
    assert out[6].item() > 0 and out[7].item() == 1.0
    # gauge models are refused, nothing is written
    out.fill_(-1.0)
    with pytest.raises(LatticeError):
        energy_noalloc(tp, tq, out, **dict(kw, potential="abelian_higgs"))
    torch.cuda.synchronize()
    assert torch.all(out == -1.0)
