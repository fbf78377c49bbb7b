"""GPU parity of the U(1) (Abelian-Higgs, compact links, leapfrog, a = 1) HIP
path against the FP64 oracle, the Gauss constraint held to roundoff on the
GPU, and reversibility."""
import numpy as np
import pytest

import oracle
from gpu_util import rel_maxdiff, say, tile_env, to_dev
from paper_2102_01031_amd import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def u1_kwargs(wl, N):
    return dict(N=N, dx=wl.dx, dt=wl.dt, integrator="lf", expansion="none", potential="abelian_higgs",
                lam=wl.lam, v=wl.v, e=wl.e, kappa_g=wl.kappa_g)


def gpu_u1(kw, fields, steps_list):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    phi, pi, A, piA = [to_dev(f, torch.float64) for f in fields]
    lat = Lattice(phi, pi, A=A, piA=piA, **kw)
    for n in steps_list:
        if n == "sync":
            lat.sync()
        else:
            lat.step(n)
    torch.cuda.synchronize()
    return lat, (phi, pi, A, piA)


def oracle_u1(kw, fields):
    m = oracle.U1Model(N=kw["N"], dx=kw["dx"], dt=kw["dt"], lam=kw["lam"], v=kw["v"], e=kw["e"],
                       kappa_g=kw["kappa_g"])
    return oracle.U1State(m, *fields)


def compare_u1(gt, st, tol, what):
    names = ("phi", "pi", "A", "piA")
    for k, (gl, ol) in enumerate(zip(gt, (st.phi, st.pi, st.A, st.piA))):
        for i, (g, o) in enumerate(zip(gl, ol)):
            if np.max(np.abs(o)) == 0:
                assert np.max(np.abs(g.cpu().numpy())) == 0
                continue
            e = rel_maxdiff(g.cpu().numpy(), o)
            assert e <= tol, f"{what} {names[k]}[{i}] rel err {e:.3e}"


def compare_u1_energy(eg, eo, tol, what):
    pairs = (("EK_phi", eg["EK"][0]), ("EG_phi", eg["EG"][0]), ("EV", eg["EV"][0]), ("EK_A", eg["EK_A"]),
             ("EG_A", eg["EG_A"]), ("rho", eg["rho"]))
    for k, g in pairs:
        o = eo[k]
        assert abs(g - o) <= tol * max(abs(o), 1e-300), f"{what} {k}: {g} vs {o}"


@pytest.mark.parametrize("N,steps", [(5, 9), (16, 25), (24, 40), (70, 6)])
def test_u1_parity_small(N, steps):
    wl = workloads.ABELIAN_HIGGS_128
    kw = u1_kwargs(wl, N)
    fields = wl.initial_fields(N=N)
    say(f"[u1] N={N} steps={steps}")
    lat, gt = gpu_u1(kw, fields, [steps])
    eg = lat.energy()
    st = oracle_u1(kw, fields).run(steps)
    compare_u1(gt, st, TOL, f"u1-{N}")
    compare_u1_energy(eg, st.energy(), TOL, f"u1-{N}")
    go = st.gauss()
    assert abs(eg["gauss_div_max"] - go["div_max"]) <= 1e-12 * go["div_max"]
    assert abs(eg["gauss_charge_max"] - go["charge_max"]) <= 1e-12 * go["charge_max"]
    scale = max(go["div_max"], go["charge_max"])
    assert eg["gauss_max"] <= 1e-12 * scale and go["gauss_max"] <= 1e-12 * scale
    lat.close()


@pytest.mark.parametrize("N,spec,steps", [(64, "4,4", 8), (64, "8,24", 8), (64, "4,64", 5), (64, "8,1", 4),
                                           (64, "tile", 5), (128, "4,40", 2), (128, "2,8", 2), (128, "2,128", 2)])
def test_u1_rows_kernel_parity(N, spec, steps):
    """The whole-row leapfrog kernel (N = 64, 128) over its launch shapes: 2, 4 or
    8 rows per block, z chunks that divide N, leave a ragged last chunk (24, 40),
    are one plane (1) or the whole lattice (64); 'tile' forces the per-plane
    kernel at the same size."""
    wl = workloads.ABELIAN_HIGGS_128
    kw = u1_kwargs(wl, N)
    fields = wl.initial_fields(N=N)
    say(f"[u1] rows kernel N={N} shape={spec} steps={steps}")
    with tile_env(spec, "LATTICE_U1_TILE"):
        lat, gt = gpu_u1(kw, fields, [steps])
    eg = lat.energy()
    st = oracle_u1(kw, fields).run(steps)
    compare_u1(gt, st, TOL, f"u1-rows-{N}-{spec}")
    compare_u1_energy(eg, st.energy(), TOL, f"u1-rows-{N}-{spec}")
    go = st.gauss()
    scale = max(go["div_max"], go["charge_max"])
    assert eg["gauss_max"] <= 1e-12 * scale
    lat.close()


def test_u1_parity_full_size():
    """The Abelian-Higgs workload's whole run (128^3, 50 leapfrog steps) against
    the oracle at 1e-12: every array, the energies, and the two terms of the
    Gauss residual on the stored pairing, after 10 steps and after 50."""
    wl = workloads.ABELIAN_HIGGS_128
    N = wl.N
    kw = u1_kwargs(wl, N)
    fields = wl.initial_fields()
    say(f"[u1] full size N={N} steps={wl.steps}")
    lat, gt = gpu_u1(kw, fields, [])
    st = oracle_u1(kw, fields)
    done = 0
    for n in (10, wl.steps - 10):
        lat.step(n)
        st.run(n)
        done += n
        eg = lat.energy()
        compare_u1(gt, st, TOL, f"u1-128 after {done}")
        compare_u1_energy(eg, st.energy(), TOL, f"u1-128 after {done}")
        go = st.gauss()
        for k, ko in (("gauss_div_max", "div_max"), ("gauss_charge_max", "charge_max")):
            assert abs(eg[k] - go[ko]) <= TOL * go[ko], (k, eg[k], go[ko])
        scale = max(go["div_max"], go["charge_max"])
        assert eg["gauss_max"] <= 1e-12 * scale and go["gauss_max"] <= 1e-12 * scale
        say(f"[u1]   {done} steps: rho {eg['rho']:.12e}, Gauss {eg['gauss_max'] / scale:.2e} of its terms")
    assert done == 50
    lat.close()


def test_u1_gauss_long_run_on_gpu():
    wl = workloads.ABELIAN_HIGGS_128
    N = 32
    kw = u1_kwargs(wl, N)
    lat, gt = gpu_u1(kw, wl.initial_fields(N=N), [])
    rho0 = lat.energy()["rho"]
    worst = 0.0
    for _ in range(10):
        lat.step(100)
        e = lat.energy()
        scale = max(e["gauss_div_max"], e["gauss_charge_max"])
        assert scale > 0
        worst = max(worst, e["gauss_max"] / scale)
    say(f"[u1] 1000 steps: max |G| / scale = {worst:.2e}, 1 - rho/rho0 = {1 - e['rho'] / rho0:.2e}")
    assert worst <= 1e-12
    assert abs(1 - e["rho"] / rho0) < 1e-2
    lat.close()


@pytest.mark.parametrize("N,integ,order,steps", [(12, "vv2", 2, 6), (16, "vv4", 4, 4), (13, "vv6", 6, 2),
                                                  (64, "vv4", 4, 2)])
def test_u1_vv_parity(N, integ, order, steps):
    """The velocity-Verlet family on the U(1) system (the row kernel at N = 64)."""
    wl = workloads.ABELIAN_HIGGS_128
    kw = u1_kwargs(wl, N)
    kw["integrator"] = integ
    rng = np.random.default_rng(90 + order)
    sh = (N, N, N)
    fields = ([0.5 * rng.standard_normal(sh) for _ in range(2)], [0.3 * rng.standard_normal(sh) for _ in range(2)],
              [0.8 * rng.standard_normal(sh) for _ in range(3)], [0.3 * rng.standard_normal(sh) for _ in range(3)])
    say(f"[u1] {integ} N={N} steps={steps}")
    lat, gt = gpu_u1(kw, fields, [steps])
    st = oracle_u1(kw, fields).run_vv(steps, order)
    compare_u1(gt, st, TOL, f"u1-{integ}-{N}")
    compare_u1_energy(lat.energy(), st.energy(), TOL, f"u1-{integ}-{N}")
    lat.close()


def test_u1_sync_and_reverse():
    wl = workloads.ABELIAN_HIGGS_128
    N = 20
    kw = u1_kwargs(wl, N)
    fields = wl.initial_fields(N=N)
    lat, gt = gpu_u1(kw, fields, [30, "sync"])
    st = oracle_u1(kw, fields).run(30).sync()
    compare_u1(gt, st, TOL, "u1-sync")
    lat.step(-30).sync()
    for gl, ol in zip(gt, fields):
        for g, o in zip(gl, ol):
            assert np.max(np.abs(g.cpu().numpy() - o.reshape(-1))) < 1e-12
    lat.close()
