"""GPU parity of the SU(2) (doublet + SU(2) links, leapfrog, a = 1) HIP path
against the FP64 oracle on the same seeded inputs, the Gauss constraint held
to roundoff on the GPU, link unitarity, and reversibility."""
import numpy as np
import pytest

import oracle
from gpu_util import rel_maxdiff, say, tile_env, to_dev
from paper_2102_01031_amd import inputs, workloads

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def su2_kwargs(wl, N):
    return dict(N=N, dx=wl.dx, dt=wl.dt, integrator="lf", expansion="none", potential="su2_higgs",
                lam=wl.lam, v=wl.v, g=wl.g)


def gpu_su2(kw, fields, steps_list):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    phi, pi, U, E = [to_dev(f, torch.float64) for f in fields]
    lat = Lattice(doublet=phi, pi_doublet=pi, U=U, E=E, **kw)
    for n in steps_list:
        if n == "sync":
            lat.sync()
        else:
            lat.step(n)
    torch.cuda.synchronize()
    return lat, (phi, pi, U, E)


def oracle_su2(kw, fields):
    m = oracle.SU2Model(N=kw["N"], dx=kw["dx"], dt=kw["dt"], lam=kw["lam"], v=kw["v"], g=kw["g"])
    return oracle.SU2State(m, *fields)


def compare_su2(gt, st, tol, what):
    names = ("doublet", "pi_doublet", "U", "E")
    worst = 0.0
    for k, (gl, ol) in enumerate(zip(gt, (st.phi, st.pi, st.U, st.E))):
        for i, (g, o) in enumerate(zip(gl, ol)):
            gn = g.cpu().numpy()
            if np.max(np.abs(o)) == 0:
                assert np.max(np.abs(gn)) == 0, f"{what} {names[k]}[{i}] should stay zero"
                continue
            e = rel_maxdiff(gn, o)
            worst = max(worst, e)
            assert e <= tol, f"{what} {names[k]}[{i}] rel err {e:.3e}"
    return worst


def compare_su2_energy(eg, eo, tol, what):
    pairs = (("EK_phi", eg["EK"][0]), ("EG_phi", eg["EG"][0]), ("EV", eg["EV"][0]), ("EK_B", eg["EK_B"]),
             ("EG_B", eg["EG_B"]), ("rho", eg["rho"]))
    for k, g in pairs:
        o = eo[k]
        if o == 0.0:
            assert abs(g) <= tol * abs(eo["rho"]), f"{what} {k}: {g} vs 0"
        else:
            assert abs(g - o) <= tol * abs(o), f"{what} {k}: {g} vs {o}"


@pytest.mark.parametrize("layout", ["records", "soa"])
@pytest.mark.parametrize("N,steps,seed", [(5, 9, 1), (16, 25, 2), (24, 30, 3), (70, 3, 4)])
def test_su2_parity_generic_state(N, steps, seed, layout):
    """A generic seeded state (random links, electric fields, doublet and
    momenta, no constraint): several 64 x 4 tiles, ragged tails in x (70) and
    y (5, 70), and odd sizes; the step on per-site records of the doublet and
    links (default for calls of 4 or more passes) and on the SoA arrays."""
    wl = workloads.SU2_HIGGS_128
    kw = su2_kwargs(wl, N)
    fields = inputs.random_su2_state(N, seed)
    say(f"[su2] generic state N={N} steps={steps} seed={seed} layout={layout}")
    with tile_env("0" if layout == "soa" else None, "LATTICE_SU2_AOS"):
        lat, gt = gpu_su2(kw, fields, [steps])
    eg = lat.energy()
    st = oracle_su2(kw, fields).run(steps)
    worst = compare_su2(gt, st, TOL, f"su2-{N}")
    compare_su2_energy(eg, st.energy(), TOL, f"su2-{N}")
    go = st.gauss()
    for kg, ko in (("gauss_mean", "gauss_mean"), ("gauss_div_max", "div_max"), ("gauss_charge_max", "charge_max"),
                   ("gauss_max", "gauss_max"), ("gauss_abs_mean", "gauss_abs_mean")):
        assert abs(eg[kg] - go[ko]) <= 1e-11 * go[ko], (kg, eg[kg], go[ko])
    say(f"[su2]   state rel err {worst:.2e}, rho {eg['rho']:.9e} (oracle {st.energy()['rho']:.9e})")
    lat.close()


@pytest.mark.parametrize("N,zc,steps", [(24, 5, 7), (24, 24, 4), (70, 3, 2), (16, 1, 6)])
def test_su2_parity_z_columns(N, zc, steps):
    """Blocks that march z columns of zc planes: a ragged last column (24 / 5,
    70 / 3), one column over the whole lattice (24) and one plane (1)."""
    wl = workloads.SU2_HIGGS_128
    kw = su2_kwargs(wl, N)
    fields = inputs.random_su2_state(N, 40 + N)
    say(f"[su2] z columns N={N} zc={zc} steps={steps}")
    with tile_env(str(zc), "LATTICE_SU2_ZC"):
        lat, gt = gpu_su2(kw, fields, [steps])
    eg = lat.energy()
    st = oracle_su2(kw, fields).run(steps)
    compare_su2(gt, st, TOL, f"su2-zc-{N}-{zc}")
    compare_su2_energy(eg, st.energy(), TOL, f"su2-zc-{N}-{zc}")
    go = st.gauss()
    assert abs(eg["gauss_max"] - go["gauss_max"]) <= 1e-11 * go["gauss_max"]
    lat.close()


@pytest.mark.parametrize("layout", ["records", "soa"])
@pytest.mark.parametrize("N,zc,steps", [(24, 5, 7), (70, 3, 4), (32, 16, 5)])
def test_su2_alternating_march(N, zc, steps, layout):
    """Leapfrog passes that alternate the z march direction of every column
    (LATTICE_SU2_ALT=1): against the oracle, and every field bitwise equal to
    upward marches only (each site's update is independent of the order)."""
    import torch
    wl = workloads.SU2_HIGGS_128
    kw = su2_kwargs(wl, N)
    fields = inputs.random_su2_state(N, 70 + N)
    say(f"[su2] alternating march N={N} zc={zc} steps={steps} layout={layout}")
    out = []
    for alt in ("1", "0"):
        with tile_env(alt, "LATTICE_SU2_ALT"), tile_env(str(zc), "LATTICE_SU2_ZC"), \
                tile_env("0" if layout == "soa" else None, "LATTICE_SU2_AOS"):
            lat, gt = gpu_su2(kw, fields, [steps])
        out.append([t.cpu() for group in gt for t in (group if isinstance(group, (list, tuple)) else [group])])
        if alt == "1":
            st = oracle_su2(kw, fields).run(steps)
            compare_su2(gt, st, TOL, f"su2-alt-{N}")
        lat.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("layout", ["records", "soa"])
@pytest.mark.parametrize("N,zc,steps", [(32, None, 5), (64, None, 4), (64, 3, 3)])
def test_su2_band_order(N, zc, steps, layout):
    """Blocks dealt to the XCDs in y bands over all planes (the default where
    N is a multiple of 32; with a ragged last z chunk at 64 / 3) with the
    momenta and output records non-temporal (the default), marches
    alternating: against the oracle, and every field bitwise equal to the
    plane-wide order (LATTICE_SU2_BAND=0) and to cached streams
    (LATTICE_SU2_NT=0)."""
    import torch
    wl = workloads.SU2_HIGGS_128
    kw = su2_kwargs(wl, N)
    fields = inputs.random_su2_state(N, 90 + N)
    say(f"[su2] band order N={N} zc={zc} steps={steps} layout={layout}")
    out = []
    for band, nt in ((None, None), ("0", None), (None, "0")):
        with tile_env(band, "LATTICE_SU2_BAND"), tile_env(nt, "LATTICE_SU2_NT"), \
                tile_env(None if zc is None else str(zc), "LATTICE_SU2_ZC"), \
                tile_env("0" if layout == "soa" else None, "LATTICE_SU2_AOS"):
            lat, gt = gpu_su2(kw, fields, [steps])
        out.append([t.cpu() for group in gt for t in (group if isinstance(group, (list, tuple)) else [group])])
        if band is None and nt is None:
            eg = lat.energy()
            st = oracle_su2(kw, fields).run(steps)
            compare_su2(gt, st, TOL, f"su2-band-{N}")
            compare_su2_energy(eg, st.energy(), TOL, f"su2-band-{N}")
        lat.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert torch.equal(a, b)


@pytest.mark.parametrize("N,steps", [(12, 40), (32, 10)])
def test_su2_parity_workload_state(N, steps):
    """The bench workload's initial state (white-noise doublet direction, unit
    links, no electric field) at small sizes."""
    wl = workloads.SU2_HIGGS_128
    kw = su2_kwargs(wl, N)
    fields = wl.initial_fields(N=N)
    say(f"[su2] workload state N={N} steps={steps}")
    lat, gt = gpu_su2(kw, fields, [steps])
    eg = lat.energy()
    st = oracle_su2(kw, fields).run(steps)
    compare_su2(gt, st, TOL, f"su2-wl-{N}")
    compare_su2_energy(eg, st.energy(), TOL, f"su2-wl-{N}")
    lat.close()


@pytest.mark.parametrize("N,integ,order,steps", [(12, "vv2", 2, 6), (12, "vv4", 4, 4), (13, "vv6", 6, 2),
                                                  (64, "vv4", 4, 1)])
def test_su2_vv_parity(N, integ, order, steps):
    """The velocity-Verlet family on the SU(2) system (merged half kicks on the
    device, plain composition in the oracle)."""
    wl = workloads.SU2_HIGGS_128
    kw = su2_kwargs(wl, N)
    kw["integrator"] = integ
    fields = inputs.random_su2_state(N, 80 + order)
    say(f"[su2] {integ} N={N} steps={steps}")
    lat, gt = gpu_su2(kw, fields, [steps])
    st = oracle_su2(kw, fields).run_vv(steps, order)
    worst = compare_su2(gt, st, TOL, f"su2-{integ}-{N}")
    compare_su2_energy(lat.energy(), st.energy(), TOL, f"su2-{integ}-{N}")
    say(f"[su2]   state rel err {worst:.2e}")
    lat.step(-steps)
    for gl, ol in zip(gt, fields):
        for g, o in zip(gl, ol):
            assert np.max(np.abs(g.cpu().numpy() - np.asarray(o).reshape(-1))) < 1e-12
    lat.close()


def test_su2_parity_full_size():
    wl = workloads.SU2_HIGGS_128
    N, steps = wl.N, 2
    kw = su2_kwargs(wl, N)
    fields = wl.initial_fields()
    say(f"[su2] full size N={N} steps={steps}")
    lat, gt = gpu_su2(kw, fields, [steps])
    eg = lat.energy()
    st = oracle_su2(kw, fields).run(steps)
    compare_su2(gt, st, TOL, "su2-128")
    compare_su2_energy(eg, st.energy(), TOL, "su2-128")
    lat.close()


def test_su2_gauss_and_unitarity_long_run_on_gpu():
    wl = workloads.SU2_HIGGS_128
    N = 32
    kw = su2_kwargs(wl, N)
    fields = wl.initial_fields(N=N)
    # a charge-free kinetic start (pi proportional to phi per site) so that
    # both sides of the Gauss law grow quickly
    w = 2.0 * np.random.default_rng(77).standard_normal((N, N, N))
    fields = (fields[0], [w * f for f in fields[0]], fields[2], fields[3])
    lat, gt = gpu_su2(kw, fields, [])
    rho0 = lat.energy()["rho"]
    worst = 0.0
    for _ in range(10):
        lat.step(100)
        e = lat.energy()
        scale = max(e["gauss_div_max"], e["gauss_charge_max"])
        assert scale > 0
        worst = max(worst, e["gauss_max"] / scale)
    U = [u.cpu().numpy() for u in gt[2]]
    unit = max(np.abs(sum(U[4 * i + k] ** 2 for k in range(4)) - 1).max() for i in range(3))
    say(f"[su2] 1000 steps: max |G| / scale = {worst:.2e}, 1 - rho/rho0 = {1 - e['rho'] / rho0:.2e}, "
        f"EK_B {e['EK_B']:.3e}, EG_B {e['EG_B']:.3e}, max ||U|^2 - 1| = {unit:.2e}")
    assert worst <= 1e-12
    assert unit <= 1e-13
    assert e["EK_B"] > 0 and e["EG_B"] > 0
    assert abs(1 - e["rho"] / rho0) < 1e-2
    lat.close()


def test_su2_layout_transitions():
    """Calls below and above the per-site-record threshold in turn (SoA for 1
    and 2 passes, records for 5 and 7), leapfrog and VV4, against the oracle."""
    wl = workloads.SU2_HIGGS_128
    N = 18
    fields = inputs.random_su2_state(N, 140)
    kw = su2_kwargs(wl, N)
    lat, gt = gpu_su2(kw, fields, [1, 5, 2, 7, 1])
    st = oracle_su2(kw, fields).run(16)
    compare_su2(gt, st, TOL, "su2-layouts-lf")
    lat.close()
    kw["integrator"] = "vv4"
    lat, gt = gpu_su2(kw, fields, [1, 2, 1])          # 3, 6, 3 passes
    st = oracle_su2(kw, fields).run_vv(4, 4)
    compare_su2(gt, st, TOL, "su2-layouts-vv4")
    lat.close()


def test_su2_sync_and_reverse():
    wl = workloads.SU2_HIGGS_128
    N = 20
    kw = su2_kwargs(wl, N)
    fields = inputs.random_su2_state(N, 8)
    lat, gt = gpu_su2(kw, fields, [30, "sync"])
    st = oracle_su2(kw, fields).run(30).sync()
    compare_su2(gt, st, TOL, "su2-sync")
    compare_su2_energy(lat.energy(), st.energy(), TOL, "su2-sync")
    lat.step(-30).sync()
    for gl, ol in zip(gt, fields):
        for g, o in zip(gl, ol):
            assert np.max(np.abs(g.cpu().numpy() - np.asarray(o).reshape(-1))) < 1e-12
    lat.close()


def test_su2_rejects_unsupported():
    import torch
    from paper_2102_01031_amd.lattice import Lattice, LatticeError
    wl = workloads.SU2_HIGGS_128
    N = 8
    phi, pi, U, E = [to_dev(f, torch.float64) for f in wl.initial_fields(N=N)]
    kw = su2_kwargs(wl, N)
    kw.update(precision="f32")
    f32 = [[t.float() for t in ts] for ts in (phi, pi, U, E)]
    with pytest.raises(LatticeError, match="UNSUPPORTED"):
        Lattice(doublet=f32[0], pi_doublet=f32[1], U=f32[2], E=f32[3], **kw)
    lat = Lattice(doublet=phi, pi_doublet=pi, U=U, E=E, **su2_kwargs(wl, N))
    with pytest.raises(LatticeError, match="UNSUPPORTED"):
        lat.occupation(0)
    with pytest.raises(LatticeError, match="EINVAL"):
        lat.spectrum(4)
    lat.close()


@pytest.mark.parametrize("N", [16, 27])
def test_su2_doublet_component_spectra(N):
    """Power spectra of the doublet's components and momenta (eq. discretePS)
    after a few steps, against the oracle's own-DFT spectrum of the same
    arrays (its state after the same steps)."""
    import math
    wl = workloads.SU2_HIGGS_128
    kw = su2_kwargs(wl, N)
    fields = inputs.random_su2_state(N, 120 + N)
    lat, gt = gpu_su2(kw, fields, [5, "sync"])
    st = oracle_su2(kw, fields).run(5).sync()
    for which, arrs in ((0, st.phi), (1, st.pi)):
        for c in range(4):
            sp = lat.spectrum(c, "phi" if which == 0 else "pi")
            s, d, cnt = oracle.spectrum(arrs[c], wl.dx, nbins=len(sp["sum"]))
            assert np.array_equal(sp["count"], cnt)
            rel = np.max(np.abs(sp["sum"] - s)) / s.max()
            assert rel <= 1e-12, (which, c, rel)
            kir = 2 * math.pi / (N * wl.dx)
            lhs = sum(kir / (b * kir) * sp["delta"][b] for b in range(1, len(sp["delta"])))
            f = arrs[c]
            assert abs(lhs - (np.mean(f * f) - np.mean(f) ** 2)) <= 1e-10 * np.mean(f * f)
    lat.close()
