"""GPU checks of the hand-written adjoint (lattice_grad) of the two-field
velocity-Verlet run at a = 1:
  - against the oracle's adjoint (segment recomputation, no reverse
    integration) at small ragged sizes, 1e-10 relative;
  - at the full differentiable workload (64^3, 2000 steps) against central
    finite differences of the GPU forward along 8 random unit directions of
    (initial delta-phi field, q) plus the pure q direction, 1e-6 relative;
  - through the torch.autograd.Function, and gradcheck at a tiny size;
  - the fields hold their initial values after the call."""
import numpy as np
import pytest

import oracle
from gpu_util import rel_maxdiff, say, to_dev
from paper_2102_01031_amd import inputs, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def kw_of(wl, N, q=None):
    return dict(N=N, dx=wl.dx, dt=wl.dt, integrator="vv2", expansion="none", potential="phi4_chi2",
                lam=wl.lam, q=wl.q if q is None else q)


def gpu_grad(wl, N, phi, pi, T, q=None, stride=0):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_of(wl, N, q))
    r = lat.grad(T, stride=stride)
    return lat, tp, tq, r


def gpu_observable(wl, N, phi, pi, T, q):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_of(wl, N, q))
    lat.step(T)
    e = lat.energy()
    lat.close()
    return (e["EK"][1] + e["EG"][1]) / e["rho"]


@pytest.mark.parametrize("N,T,stride", [(16, 40, 0), (24, 33, 5), (13, 20, 1), (64, 25, 0)])
def test_grad_matches_oracle_adjoint(N, T, stride):
    wl = workloads.ADJ_64
    phi, pi = wl.initial_fields(N=N)
    say(f"[adj] oracle parity N={N} T={T} stride={stride}")
    lat, tp, tq, r = gpu_grad(wl, N, phi, pi, T, stride=stride)
    m = oracle.ScalarModel(N=N, dx=wl.dx, dt=wl.dt, nfields=2, potential=oracle.PHI4_CHI2, expansion=oracle.NONE,
                           integrator=oracle.VV2, lam=wl.lam, q=wl.q)
    O, g, gp, dq = oracle.adjoint_vv2(m, phi, pi, T)
    assert abs(r["value"] - O) <= 1e-12 * abs(O)
    for s in range(2):
        assert rel_maxdiff(r["dO_dphi"][s].cpu().numpy(), g[s]) <= 1e-10
        assert rel_maxdiff(r["dO_dpi"][s].cpu().numpy(), gp[s]) <= 1e-10
    assert abs(r["dO_dq"] - dq) <= 1e-10 * abs(dq)
    # the fields hold the initial state again
    for s in range(2):
        assert np.array_equal(tp[s].cpu().numpy(), phi[s].reshape(-1))
        assert np.array_equal(tq[s].cpu().numpy(), pi[s].reshape(-1))
    lat.close()


def test_grad_full_workload_vs_finite_differences():
    wl = workloads.ADJ_64
    N, T = wl.N, wl.steps
    phi, pi = wl.initial_fields()
    lat, tp, tq, r = gpu_grad(wl, N, phi, pi, T)
    g = r["dO_dphi"][0].cpu().numpy().reshape(N, N, N)
    dq = r["dO_dq"]
    O0 = r["value"]
    say(f"[adj] full workload: O={O0:.6e} dO/dq={dq:.6e} forward {r['forward_ms']:.1f} ms reverse "
        f"{r['reverse_ms']:.1f} ms")
    lat.close()
    assert abs(gpu_observable(wl, N, phi, pi, T, wl.q) - O0) <= 1e-12 * abs(O0)
    dirs = inputs.random_directions(8, N, seed=7) + [(np.zeros((N, N, N)), 1.0)]
    worst = 0.0
    for k, (v, vq) in enumerate(dirs):
        ad = float(np.sum(g * v) + dq * vq)

        def fd(eps):
            fp = gpu_observable(wl, N, [phi[0] + eps * v, phi[1]], pi, T, wl.q + eps * vq)
            fm = gpu_observable(wl, N, [phi[0] - eps * v, phi[1]], pi, T, wl.q - eps * vq)
            return (fp - fm) / (2 * eps)

        e = 2e-3 if vq == 1.0 else 4e-3
        d1, d2 = fd(e), fd(e / 2)
        rich = (4 * d2 - d1) / 3
        rel = abs(rich - ad) / abs(ad)
        worst = max(worst, rel)
        say(f"[adj] dir {k}: adjoint {ad:.10e} fd {rich:.10e} (raw {d2:.10e}) rel {rel:.2e}")
        assert rel <= 1e-6
    say(f"[adj] worst relative deviation from finite differences: {worst:.2e}")


def test_autograd_function_and_gradcheck():
    import torch
    from paper_2102_01031_amd.autograd import chi_energy_fraction
    wl = workloads.ADJ_64
    N, T = 12, 15
    phi, pi = wl.initial_fields(N=N)
    ts = [torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True) for a in (phi[0], phi[1], pi[0], pi[1])]
    q = torch.tensor(wl.q, dtype=torch.float64, requires_grad=True)
    O = chi_energy_fraction(*ts, q, N=N, dx=wl.dx, dt=wl.dt, nsteps=T, lam=wl.lam)
    O.backward()
    lat, tp, tq, r = gpu_grad(wl, N, phi, pi, T)
    assert abs(O.item() - r["value"]) < 1e-15 * abs(r["value"]) + 1e-300
    assert torch.equal(ts[0].grad.reshape(-1), r["dO_dphi"][0])
    assert torch.equal(ts[3].grad.reshape(-1), r["dO_dpi"][1])
    assert abs(q.grad.item() - r["dO_dq"]) <= 1e-15 * abs(r["dO_dq"])
    lat.close()
    # gradcheck of the Function at a tiny lattice
    n4 = 4
    ph4, pi4 = wl.initial_fields(N=n4)
    xs = [torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True) for a in (ph4[0], ph4[1], pi4[0], pi4[1])]
    q4 = torch.tensor(wl.q, dtype=torch.float64, requires_grad=True)
    f = lambda a, b, c, d, qq: chi_energy_fraction(a, b, c, d, qq, N=n4, dx=wl.dx, dt=wl.dt, nsteps=6, lam=wl.lam)
    assert torch.autograd.gradcheck(f, (*xs, q4), eps=1e-6, atol=1e-9, rtol=1e-5)


# Spectrum-bin observable: O = Delta(b) of one field after T steps (eq. discretePS)

def gpu_spectrum_observable(wl, N, phi, pi, T, q, field, b):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_of(wl, N, q))
    lat.step(T)
    d = lat.spectrum(field, "phi", nbins=b + 1)["delta"][b]
    lat.close()
    return d


@pytest.mark.parametrize("N,T,stride,field,b", [(16, 20, 0, 0, 1), (24, 15, 4, 1, 3), (13, 10, 1, 0, 10),
                                                 (64, 12, 0, 1, 5)])
def test_spectrum_bin_grad_matches_oracle_adjoint(N, T, stride, field, b):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    wl = workloads.ADJ_64
    phi, pi = wl.initial_fields(N=N)
    say(f"[adj] spectrum-bin oracle parity N={N} T={T} stride={stride} field={field} bin={b}")
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_of(wl, N))
    r = lat.grad(T, stride=stride, observable="spectrum_bin", field=field, bin=b)
    m = oracle.ScalarModel(N=N, dx=wl.dx, dt=wl.dt, nfields=2, potential=oracle.PHI4_CHI2, expansion=oracle.NONE,
                           integrator=oracle.VV2, lam=wl.lam, q=wl.q)
    O, g, gp, dq = oracle.adjoint_vv2(m, phi, pi, T, kind=oracle.OBS_SPECTRUM_BIN, field=field, bin=b)
    say(f"[adj]   O={r['value']:.6e} (oracle {O:.6e}) dO/dq={r['dO_dq']:.6e} (oracle {dq:.6e})")
    assert abs(r["value"] - O) <= 1e-12 * abs(O)
    for s in range(2):
        assert rel_maxdiff(r["dO_dphi"][s].cpu().numpy(), g[s]) <= 1e-10
        assert rel_maxdiff(r["dO_dpi"][s].cpu().numpy(), gp[s]) <= 1e-10
    assert abs(r["dO_dq"] - dq) <= 1e-10 * abs(dq)
    for s in range(2):
        assert np.array_equal(tp[s].cpu().numpy(), phi[s].reshape(-1))
        assert np.array_equal(tq[s].cpu().numpy(), pi[s].reshape(-1))
    # the value is the same bin as lattice_spectrum's after T steps
    assert abs(gpu_spectrum_observable(wl, N, phi, pi, T, wl.q, field, b) - O) <= 1e-12 * abs(O)
    lat.close()


def test_spectrum_bin_grad_full_workload_vs_finite_differences():
    wl = workloads.ADJ_64
    N, T, field, b = wl.N, wl.steps, 1, 4
    phi, pi = wl.initial_fields()
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_of(wl, N))
    r = lat.grad(T, observable="spectrum_bin", field=field, bin=b)
    g = r["dO_dphi"][0].cpu().numpy().reshape(N, N, N)
    dq = r["dO_dq"]
    O0 = r["value"]
    say(f"[adj] spectrum bin {b} of field {field}, full workload: O={O0:.6e} dO/dq={dq:.6e} forward "
        f"{r['forward_ms']:.1f} ms reverse {r['reverse_ms']:.1f} ms")
    lat.close()
    assert abs(gpu_spectrum_observable(wl, N, phi, pi, T, wl.q, field, b) - O0) <= 1e-12 * abs(O0)
    dirs = inputs.random_directions(4, N, seed=11) + [(np.zeros((N, N, N)), 1.0)]
    for k, (v, vq) in enumerate(dirs):
        ad = float(np.sum(g * v) + dq * vq)

        def fd(eps):
            fp = gpu_spectrum_observable(wl, N, [phi[0] + eps * v, phi[1]], pi, T, wl.q + eps * vq, field, b)
            fm = gpu_spectrum_observable(wl, N, [phi[0] - eps * v, phi[1]], pi, T, wl.q - eps * vq, field, b)
            return (fp - fm) / (2 * eps)

        e = 2e-3 if vq == 1.0 else 4e-3
        d1, d2 = fd(e), fd(e / 2)
        rich = (4 * d2 - d1) / 3
        rel = abs(rich - ad) / abs(ad)
        say(f"[adj] spectrum dir {k}: adjoint {ad:.10e} fd {rich:.10e} (raw {d2:.10e}) rel {rel:.2e}")
        assert rel <= 1e-6


def test_spectrum_bin_autograd_and_bad_selection():
    import torch
    from paper_2102_01031_amd.autograd import spectrum_bin
    from paper_2102_01031_amd.lattice import Lattice, LatticeError
    wl = workloads.ADJ_64
    N, T = 12, 9
    phi, pi = wl.initial_fields(N=N)
    ts = [torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True) for a in (phi[0], phi[1], pi[0], pi[1])]
    q = torch.tensor(wl.q, dtype=torch.float64, requires_grad=True)
    O = spectrum_bin(*ts, q, N=N, dx=wl.dx, dt=wl.dt, nsteps=T, field=0, bin=2, lam=wl.lam)
    O.backward()
    m = oracle.ScalarModel(N=N, dx=wl.dx, dt=wl.dt, nfields=2, potential=oracle.PHI4_CHI2, expansion=oracle.NONE,
                           integrator=oracle.VV2, lam=wl.lam, q=wl.q)
    Oo, g, gp, dq = oracle.adjoint_vv2(m, phi, pi, T, kind=oracle.OBS_SPECTRUM_BIN, field=0, bin=2)
    assert abs(O.item() - Oo) <= 1e-12 * abs(Oo)
    assert rel_maxdiff(ts[1].grad.cpu().numpy(), g[1]) <= 1e-10
    assert rel_maxdiff(ts[2].grad.cpu().numpy(), gp[0]) <= 1e-10
    assert abs(q.grad.item() - dq) <= 1e-10 * abs(dq)
    # out-of-range selections are rejected before any work
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_of(wl, N))
    bmax = int(np.floor(np.sqrt(3 * (N // 2) ** 2)))
    for field, b in ((2, 1), (-1, 1), (0, 0), (0, bmax + 1)):
        with pytest.raises(LatticeError):
            lat.grad(T, observable="spectrum_bin", field=field, bin=b)
    for bad in (dict(field=2), dict(field=0, bin=3)):
        with pytest.raises(LatticeError):
            lat.grad(T, observable="energy_fraction", **bad)
    r = lat.grad(T, observable="spectrum_bin", field=1, bin=bmax)   # the outermost shell is valid
    assert np.isfinite(r["value"]) and r["value"] >= 0.0
    lat.close()


# Fixed power-law background (radiation, H0 = 2): kicks at a(t_p), drifts at a(t_p + h/2)

def kw_fixed(wl, N, alpha=1.0, t0=0.25, q=None):
    kw = kw_of(wl, N, q)
    kw.update(expansion="fixed", w_eos=1 / 3, H0=2.0, t_ref=0.0, a0=1.0, t0=t0, alpha=alpha)
    return kw


def oracle_fixed(wl, N, alpha=1.0):
    return oracle.ScalarModel(N=N, dx=wl.dx, dt=wl.dt, nfields=2, potential=oracle.PHI4_CHI2,
                              expansion=oracle.FIXED, integrator=oracle.VV2, lam=wl.lam, q=wl.q, alpha=alpha,
                              w_eos=1 / 3, H0=2.0, t0=0.0, a0=1.0)


@pytest.mark.parametrize("N,T,stride,alpha,obs", [(16, 40, 0, 1.0, "chi_fraction"), (24, 33, 5, 0.5, "chi_fraction"),
                                                  (13, 20, 1, 1.0, "spectrum_bin"), (64, 25, 0, 0.5, "spectrum_bin")])
def test_grad_fixed_background_matches_oracle_adjoint(N, T, stride, alpha, obs):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    wl = workloads.ADJ_64
    phi, pi = wl.initial_fields(N=N)
    t0 = 0.25
    say(f"[adj] fixed background oracle parity N={N} T={T} stride={stride} alpha={alpha} {obs}")
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_fixed(wl, N, alpha, t0))
    sel = dict(field=1, bin=3) if obs == "spectrum_bin" else {}
    r = lat.grad(T, stride=stride, observable=obs, **sel)
    kind = oracle.OBS_SPECTRUM_BIN if obs == "spectrum_bin" else oracle.OBS_ENERGY_FRACTION
    O, g, gp, dq = oracle.adjoint_vv2(oracle_fixed(wl, N, alpha), phi, pi, T, kind=kind, t=t0, **sel)
    say(f"[adj]   O={r['value']:.6e} (oracle {O:.6e}) dO/dq={r['dO_dq']:.6e} (oracle {dq:.6e})")
    assert abs(r["value"] - O) <= 1e-12 * abs(O)
    for s in range(2):
        assert rel_maxdiff(r["dO_dphi"][s].cpu().numpy(), g[s]) <= 1e-10
        assert rel_maxdiff(r["dO_dpi"][s].cpu().numpy(), gp[s]) <= 1e-10
    assert abs(r["dO_dq"] - dq) <= 1e-10 * abs(dq)
    for s in range(2):
        assert np.array_equal(tp[s].cpu().numpy(), phi[s].reshape(-1))
        assert np.array_equal(tq[s].cpu().numpy(), pi[s].reshape(-1))
    lat.close()


def test_grad_fixed_background_full_workload_vs_finite_differences():
    """64^3 x 2000 VV2 steps on the fixed background, chi energy fraction at
    the final a, against differences of the library's own forward run."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    wl = workloads.ADJ_64
    N, T = wl.N, wl.steps
    phi, pi = wl.initial_fields()
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_fixed(wl, N))
    r = lat.grad(T)
    g = r["dO_dphi"][0].cpu().numpy().reshape(N, N, N)
    dq, O0 = r["dO_dq"], r["value"]
    say(f"[adj] fixed background full workload: O={O0:.6e} dO/dq={dq:.6e} forward {r['forward_ms']:.1f} ms "
        f"reverse {r['reverse_ms']:.1f} ms")
    lat.close()

    def O_fwd(phi_, q_):
        tp_, tq_ = to_dev(phi_, torch.float64), to_dev(pi, torch.float64)
        lt = Lattice(tp_, tq_, **kw_fixed(wl, N, q=q_))
        lt.step(T)
        e = lt.energy()
        lt.close()
        return (e["EK"][1] + e["EG"][1]) / e["rho"]

    assert abs(O_fwd(phi, wl.q) - O0) <= 1e-12 * abs(O0)
    dirs = inputs.random_directions(4, N, seed=23) + [(np.zeros((N, N, N)), 1.0)]
    for k, (v, vq) in enumerate(dirs):
        ad = float(np.sum(g * v) + dq * vq)

        def fd(eps):
            return (O_fwd([phi[0] + eps * v, phi[1]], wl.q + eps * vq)
                    - O_fwd([phi[0] - eps * v, phi[1]], wl.q - eps * vq)) / (2 * eps)

        e = 2e-3 if vq == 1.0 else 4e-3
        d1, d2 = fd(e), fd(e / 2)
        rich = (4 * d2 - d1) / 3
        rel = abs(rich - ad) / abs(ad)
        say(f"[adj] fixed dir {k}: adjoint {ad:.10e} fd {rich:.10e} rel {rel:.2e}")
        assert rel <= 1e-6


@pytest.mark.parametrize("N,T,expansion", [(16, 20, "none"), (24, 17, "fixed")])
def test_energy_fraction_of_phi_matches_oracle(N, T, expansion):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    wl = workloads.ADJ_64
    phi, pi = wl.initial_fields(N=N)
    say(f"[adj] energy fraction of phi N={N} T={T} {expansion}")
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    fixed = expansion == "fixed"
    lat = Lattice(tp, tq, **(kw_fixed(wl, N) if fixed else kw_of(wl, N)))
    r = lat.grad(T, observable="energy_fraction", field=0)
    m = oracle_fixed(wl, N) if fixed else oracle.ScalarModel(
        N=N, dx=wl.dx, dt=wl.dt, nfields=2, potential=oracle.PHI4_CHI2, expansion=oracle.NONE,
        integrator=oracle.VV2, lam=wl.lam, q=wl.q)
    O, g, gp, dq = oracle.adjoint_vv2(m, phi, pi, T, field=0, t=0.25 if fixed else 0.0)
    say(f"[adj]   O={r['value']:.6e} (oracle {O:.6e}) dO/dq={r['dO_dq']:.6e} (oracle {dq:.6e})")
    assert abs(r["value"] - O) <= 1e-12 * abs(O)
    for s in range(2):
        assert rel_maxdiff(r["dO_dphi"][s].cpu().numpy(), g[s]) <= 1e-10
        assert rel_maxdiff(r["dO_dpi"][s].cpu().numpy(), gp[s]) <= 1e-10
    assert abs(r["dO_dq"] - dq) <= 1e-10 * abs(dq)
    with pytest.raises(Exception):
        lat.grad(T, observable="energy_fraction", field=0, bin=2)
    lat.close()


# Self-consistent expansion: the library's own VV2 step with a and a' evolving;
# a' at the start is an independent input (passed explicitly, here from the
# oracle's Hubble constraint).

def kw_self(wl, N, alpha=1.0, kappa2=4.0, b0=None, q=None):
    kw = kw_of(wl, N, q)
    kw.update(expansion="self", kappa2=kappa2, a0=1.0, alpha=alpha)
    if b0 is not None:
        kw["b0"] = b0
    return kw


def oracle_self(wl, N, alpha=1.0, kappa2=4.0, q=None):
    return oracle.ScalarModel(N=N, dx=wl.dx, dt=wl.dt, nfields=2, potential=oracle.PHI4_CHI2,
                              expansion=oracle.SELF, integrator=oracle.VV2, lam=wl.lam, q=wl.q if q is None else q,
                              alpha=alpha, kappa2=kappa2)


@pytest.mark.parametrize("N,T,stride,alpha,obs,field,b", [(12, 10, 0, 1.0, "energy_fraction", 1, 0),
                                                           (16, 15, 4, 0.5, "energy_fraction", 0, 0),
                                                           (13, 8, 1, 1.0, "spectrum_bin", 1, 2)])
def test_grad_self_consistent_matches_oracle_adjoint(N, T, stride, alpha, obs, field, b):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    wl = workloads.ADJ_64
    phi, pi = wl.initial_fields(N=N)
    m = oracle_self(wl, N, alpha)
    b0 = oracle.hubble_b0(m, phi, pi, 1.0)
    say(f"[adj] self-consistent oracle parity N={N} T={T} stride={stride} alpha={alpha} {obs} field={field}")
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_self(wl, N, alpha, b0=b0))
    e0 = lat.energy()
    r = lat.grad(T, stride=stride, observable=obs, field=field, bin=b)
    kind = oracle.OBS_SPECTRUM_BIN if obs == "spectrum_bin" else oracle.OBS_ENERGY_FRACTION
    O, g, gp, dq, da0, db0 = oracle.adjoint_vv2_self(m, phi, pi, 1.0, b0, T, kind=kind, field=field, bin=b)
    say(f"[adj]   O={r['value']:.6e} (oracle {O:.6e}) dO/dq={r['dO_dq']:.6e} ({dq:.6e}) "
        f"dO/da0={r['dO_da0']:.6e} ({da0:.6e}) dO/db0={r['dO_db0']:.6e} ({db0:.6e})")
    assert abs(r["value"] - O) <= 1e-12 * abs(O)
    for s in range(2):
        assert rel_maxdiff(r["dO_dphi"][s].cpu().numpy(), g[s]) <= 1e-10
        assert rel_maxdiff(r["dO_dpi"][s].cpu().numpy(), gp[s]) <= 1e-10
    assert abs(r["dO_dq"] - dq) <= 1e-10 * abs(dq)
    assert abs(r["dO_da0"] - da0) <= 1e-10 * abs(da0)
    assert abs(r["dO_db0"] - db0) <= 1e-10 * abs(db0)
    # state, scale factor, time and step count as before the call
    for s in range(2):
        assert np.array_equal(tp[s].cpu().numpy(), phi[s].reshape(-1))
        assert np.array_equal(tq[s].cpu().numpy(), pi[s].reshape(-1))
    e1 = lat.energy()
    assert (e1["a"], e1["b"], e1["t"], e1["step"]) == (e0["a"], e0["b"], e0["t"], e0["step"])
    lat.close()


def test_grad_self_consistent_full_workload_vs_finite_differences():
    """64^3 x 2000 VV2 steps with the self-consistent expansion (kappa^2 of the
    preheating runs), chi energy fraction at the final a, against differences
    of the library's own forward run in (delta phi, q, a0, a'0)."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    wl = workloads.ADJ_64
    N, T = wl.N, wl.steps
    phi, pi = wl.initial_fields()
    kap = 0.25
    b0 = oracle.hubble_b0(oracle_self(wl, N, kappa2=kap), phi, pi, 1.0)
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **kw_self(wl, N, kappa2=kap, b0=b0))
    r = lat.grad(T)
    g = r["dO_dphi"][0].cpu().numpy().reshape(N, N, N)
    O0 = r["value"]
    say(f"[adj] self-consistent full workload: O={O0:.6e} dO/dq={r['dO_dq']:.6e} dO/da0={r['dO_da0']:.6e} "
        f"dO/db0={r['dO_db0']:.6e} forward {r['forward_ms']:.1f} ms reverse {r['reverse_ms']:.1f} ms")
    lat.close()

    def O_fwd(phi_, q_, a_, b_):
        tp_, tq_ = to_dev(phi_, torch.float64), to_dev(pi, torch.float64)
        kw = kw_self(wl, N, kappa2=kap, b0=b_, q=q_)
        kw["a0"] = a_
        lt = Lattice(tp_, tq_, **kw)
        lt.step(T)
        e = lt.energy()
        lt.close()
        return (e["EK"][1] + e["EG"][1]) / e["rho"]

    assert abs(O_fwd(phi, wl.q, 1.0, b0) - O0) <= 1e-12 * abs(O0)
    rng = np.random.default_rng(37)
    dirs = inputs.random_directions(3, N, seed=31)
    for k, (v, _) in enumerate(dirs):
        w = rng.standard_normal(3)
        w *= 0.5 / np.linalg.norm(w)
        ad = float(np.sum(g * v) + r["dO_dq"] * w[0] + r["dO_da0"] * w[1] + r["dO_db0"] * w[2])

        def fd(eps):
            return (O_fwd([phi[0] + eps * v, phi[1]], wl.q + eps * w[0], 1.0 + eps * w[1], b0 + eps * w[2])
                    - O_fwd([phi[0] - eps * v, phi[1]], wl.q - eps * w[0], 1.0 - eps * w[1], b0 - eps * w[2])) / (2 * eps)

        # steps smaller than the other workloads': a0 and a'0 move the whole run
        d1, d2 = fd(1e-3), fd(5e-4)
        rich = (4 * d2 - d1) / 3
        rel = abs(rich - ad) / abs(ad)
        say(f"[adj] self-consistent dir {k}: adjoint {ad:.10e} fd {rich:.10e} rel {rel:.2e}")
        assert rel <= 1e-6


@pytest.mark.parametrize("expansion,alpha", [("fixed", 0.5), ("self", 1.0)])
def test_autograd_with_expansion_and_forward_only_path(expansion, alpha):
    """The autograd wrapper with a fixed or self-consistent background gives
    the gradients lattice_grad gives for the same context (bitwise), dO/da0
    and dO/da'0 for the self-consistent one, and passes gradcheck at a tiny
    lattice.  Without a wanted gradient (no_grad, or no input requiring one)
    it runs the forward steps only, with the same value."""
    import torch
    from paper_2102_01031_amd.autograd import chi_energy_fraction, energy_fraction
    from paper_2102_01031_amd.lattice import Lattice
    wl = workloads.ADJ_64
    N, T = 12, 11
    phi, pi = wl.initial_fields(N=N)
    if expansion == "fixed":
        bgk = dict(expansion="fixed", alpha=alpha, a0=1.0, w_eos=1 / 3, H0=2.0, t0=0.25, t_ref=0.0)
        ctx_kw = kw_fixed(wl, N, alpha=alpha)
    else:
        kap = 4.0
        b0 = oracle.hubble_b0(oracle_self(wl, N, alpha, kappa2=kap), phi, pi, 1.0)
        bgk = dict(expansion="self", alpha=alpha, kappa2=kap)
        ctx_kw = kw_self(wl, N, alpha, kappa2=kap, b0=b0)
    say(f"[adj] autograd {expansion} alpha={alpha} N={N} T={T}")
    ts = [torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True) for a in (phi[0], phi[1], pi[0], pi[1])]
    q = torch.tensor(wl.q, dtype=torch.float64, requires_grad=True)
    extra = {}
    if expansion == "self":
        a0t = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
        b0t = torch.tensor(b0, dtype=torch.float64, requires_grad=True)
        extra = dict(a0=a0t, b0=b0t)
    O = energy_fraction(*ts, q, N=N, dx=wl.dx, dt=wl.dt, nsteps=T, field=0, lam=wl.lam, **bgk, **extra)
    O.backward()
    tp, tq = to_dev(phi, torch.float64), to_dev(pi, torch.float64)
    lat = Lattice(tp, tq, **ctx_kw)
    r = lat.grad(T, observable="energy_fraction", field=0)
    lat.close()
    assert O.item() == r["value"]
    assert torch.equal(ts[0].grad.reshape(-1), r["dO_dphi"][0])
    assert torch.equal(ts[1].grad.reshape(-1), r["dO_dphi"][1])
    assert torch.equal(ts[2].grad.reshape(-1), r["dO_dpi"][0])
    assert torch.equal(ts[3].grad.reshape(-1), r["dO_dpi"][1])
    assert q.grad.item() == r["dO_dq"]
    if expansion == "self":
        assert a0t.grad.item() == r["dO_da0"] and b0t.grad.item() == r["dO_db0"]
    # forward only: under no_grad and with plain inputs
    with torch.no_grad():
        O1 = energy_fraction(*ts, q, N=N, dx=wl.dx, dt=wl.dt, nsteps=T, field=0, lam=wl.lam, **bgk, **extra)
    plain = [t.detach() for t in ts]
    O2 = energy_fraction(*plain, wl.q, N=N, dx=wl.dx, dt=wl.dt, nsteps=T, field=0, lam=wl.lam, **bgk,
                         **({k: float(v) for k, v in extra.items()}))
    assert not O1.requires_grad and not O2.requires_grad
    for v in (O1.item(), O2.item()):
        assert abs(v - r["value"]) <= 1e-13 * abs(r["value"]), (v, r["value"])
    # gradcheck at a tiny lattice, through every differentiable input
    n4 = 4
    ph4, pi4 = wl.initial_fields(N=n4)
    xs = [torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True) for a in (ph4[0], ph4[1], pi4[0], pi4[1])]
    q4 = torch.tensor(wl.q, dtype=torch.float64, requires_grad=True)
    if expansion == "self":
        b04 = oracle.hubble_b0(oracle_self(wl, n4, alpha, kappa2=kap), ph4, pi4, 1.0)
        sc = [torch.tensor(1.0, dtype=torch.float64, requires_grad=True),
              torch.tensor(b04, dtype=torch.float64, requires_grad=True)]
        f = lambda a, b, c, d, qq, aa, bb: chi_energy_fraction(a, b, c, d, qq, N=n4, dx=wl.dx, dt=wl.dt, nsteps=6,
                                                               lam=wl.lam, a0=aa, b0=bb, **bgk)
        assert torch.autograd.gradcheck(f, (*xs, q4, *sc), eps=1e-6, atol=1e-9, rtol=1e-5)
    else:
        f = lambda a, b, c, d, qq: chi_energy_fraction(a, b, c, d, qq, N=n4, dx=wl.dx, dt=wl.dt, nsteps=6,
                                                       lam=wl.lam, **bgk)
        assert torch.autograd.gradcheck(f, (*xs, q4), eps=1e-6, atol=1e-9, rtol=1e-5)



@pytest.mark.parametrize("N,T", [(64, 40), (20, 17)])
def test_grad_dq_slots_vs_ticketed(N, T):
    """The reverse sweep adds each block's partial of dO/dq to the block's own
    slot and sums the slots after the sweep, instead of a ticketed last block
    adding each pass's sum: dO/dq agrees with the per-pass sums
    (LATTICE_ENERGY_DEFER=0) to rounding, and the adjoint arrays, which do not
    depend on it, bit for bit."""
    from gpu_util import tile_env
    wl = workloads.ADJ_64
    phi, pi = wl.initial_fields(N=N)
    rs = []
    for spec in (None, "0"):
        with tile_env(spec, "LATTICE_ENERGY_DEFER"):
            say(f"[adj] dq slots N={N} T={T} LATTICE_ENERGY_DEFER={spec}")
            lat, tp, tq, r = gpu_grad(wl, N, phi, pi, T)
            rs.append((r["value"], r["dO_dq"], [a.cpu().numpy() for a in r["dO_dphi"] + r["dO_dpi"]]))
            lat.close()
    (v1, q1, g1), (v0, q0, g0) = rs
    assert v1 == v0
    assert abs(q1 - q0) <= 1e-13 * abs(q0), (q1, q0)
    for a, b in zip(g1, g0):
        assert np.array_equal(a, b)
