"""GPU parity of the SU(2) model in an expanding background (sec. 5.5.2)
against the oracle at 1e-12: fixed power-law background (alpha = 1 and 0.5)
and self-consistent expansion (leapfrog, reading A3; velocity-Verlet family,
reading R1), on ragged tiles and at N = 64 (where calls of four or more passes
run on the per-site records), with energies, a, b and the Hubble residual,
the Gauss law, sync and reversal."""
import numpy as np
import pytest

import oracle
from gpu_util import rel_maxdiff, say, to_dev
from paper_2102_01031_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


EXP = {"fixed": oracle.FIXED, "self": oracle.SELF}
ORDER = {"vv2": 2, "vv4": 4, "vv6": 6}


def kw_of(N, integ, expansion, alpha):
    return dict(N=N, dx=0.5, dt=0.03, integrator=integ, expansion=expansion, potential="su2_higgs", lam=1.0,
                v=0.7, g=1.0, alpha=alpha, kappa2=0.5, w_eos=1 / 3, H0=0.6, t_ref=0.0, a0=1.0, t0=0.1)


def oracle_state(kw, fields):
    m = oracle.SU2Model(N=kw["N"], dx=kw["dx"], dt=kw["dt"], lam=kw["lam"], v=kw["v"], g=kw["g"],
                        expansion=EXP[kw["expansion"]], alpha=kw["alpha"], kappa2=kw["kappa2"], w_eos=kw["w_eos"],
                        H0=kw["H0"], t0=kw["t_ref"], a0=kw["a0"])
    return oracle.SU2State(m, *fields, t=kw["t0"])


def compare(gt, st, what):
    for name, gl, ol in zip(("doublet", "pi_doublet", "U", "E"), gt, (st.phi, st.pi, st.U, st.E)):
        for i, (g, o) in enumerate(zip(gl, ol)):
            e = rel_maxdiff(g.cpu().numpy(), o)
            assert e <= TOL, f"{what} {name}[{i}] rel err {e:.3e}"


def compare_energy(eg, eo, what):
    for kg, ko in (("rho", "rho"), ("EK_B", "EK_B"), ("EG_B", "EG_B"), ("a", "a"), ("b", "b")):
        assert abs(eg[kg] - eo[ko]) <= TOL * abs(eo[ko]), (what, kg, eg[kg], eo[ko])
    assert abs(eg["EK"][0] - eo["EK_phi"]) <= TOL * abs(eo["EK_phi"]), what
    assert abs(eg["EG"][0] - eo["EG_phi"]) <= TOL * abs(eo["EG_phi"]), what
    assert abs(eg["hubble_res"] - eo["hubble_res"]) <= 1e-11, (what, eg["hubble_res"], eo["hubble_res"])


def run_oracle(st, integ, n):
    return st.run(n) if integ == "lf" else st.run_vv(n, ORDER[integ])


@pytest.mark.parametrize("N,integ,expansion,alpha,calls", [
    (12, "lf", "fixed", 1.0, [5]), (13, "lf", "fixed", 0.5, [2, 3]), (64, "lf", "fixed", 0.5, [4]),
    (12, "lf", "self", 1.0, [3, 2]), (13, "lf", "self", 0.5, [4]), (64, "lf", "self", 0.5, [2]),
    (12, "vv2", "fixed", 0.5, [3]), (13, "vv4", "fixed", 1.0, [2]), (64, "vv4", "fixed", 0.5, [2]),
    (12, "vv2", "self", 0.5, [2, 1]), (13, "vv4", "self", 1.0, [1]), (12, "vv6", "self", 0.5, [1])])
def test_su2_expanding_matches_oracle(N, integ, expansion, alpha, calls):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    kw = kw_of(N, integ, expansion, alpha)
    fields = inputs.random_su2_state(N, 41)
    say(f"[su2-exp] N={N} {integ} {expansion} alpha={alpha} calls={calls}")
    phi, pi, U, E = [to_dev(f, torch.float64) for f in fields]
    lat = Lattice(doublet=phi, pi_doublet=pi, U=U, E=E, **kw)
    st = oracle_state(kw, fields)
    compare_energy(lat.energy(), st.energy(), "start")
    for n in calls:
        lat.step(n)
        run_oracle(st, integ, n)
        torch.cuda.synchronize()
        compare((phi, pi, U, E), st, f"+{n}")
        eg, eo = lat.energy(), st.energy()
        compare_energy(eg, eo, f"+{n}")
        say(f"[su2-exp]   +{n}: a={eg['a']:.10f} b={eg['b']:.6e} r_H={eg['hubble_res']:.2e}")
    assert eg["a"] != 1.0
    if integ == "lf":
        lat.sync()
        st.sync()
        compare((phi, pi, U, E), st, "synced")
        compare_energy(lat.energy(), st.energy(), "synced")
    lat.close()


@pytest.mark.parametrize("integ,expansion", [("lf", "self"), ("vv4", "self"), ("lf", "fixed")])
def test_su2_expanding_reversal_and_gauss(integ, expansion):
    """A run, back to the start (fields, a and b), with the Gauss residual of a
    Gauss-free start held to rounding along the way."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    N = 16
    phi0, _, U0, E0 = inputs.random_direction_su2(N, 0.8, 13)
    w = 0.5 * np.random.default_rng(14).standard_normal((N, N, N))
    fields = (phi0, [w * f for f in phi0], U0, E0)   # a charge-free kinetic start
    kw = kw_of(N, integ, expansion, 0.5)
    phi, pi, U, E = [to_dev(f, torch.float64) for f in fields]
    lat = Lattice(doublet=phi, pi_doublet=pi, U=U, E=E, **kw)
    e0 = lat.energy()
    lat.step(12)
    e1 = lat.energy()
    scale = max(e1["gauss_div_max"], e1["gauss_charge_max"])
    assert scale > 1e-3 and e1["gauss_max"] <= 1e-12 * scale
    if integ == "lf":
        lat.sync()
    lat.step(-12)
    if integ == "lf":
        lat.sync()
    e2 = lat.energy()
    assert abs(e2["a"] - e0["a"]) <= 1e-13 and abs(e2["b"] - e0["b"]) <= 1e-11 * abs(e0["b"])
    for gl, ol in zip((phi, pi, U, E), fields):
        for g, o in zip(gl, ol):
            assert np.max(np.abs(g.cpu().numpy() - np.asarray(o).reshape(-1))) <= 1e-11
    lat.close()


@pytest.mark.parametrize("N", [13, 64])
def test_su2_self_carry_bitwise(N):
    """Self-consistent leapfrog steps after a call's first take the sums before
    the kick from the passes around them: fields, a and b equal, bit for bit,
    those of a run that measures them in an energy pass on every step
    (LATTICE_SELF_CARRY=0)."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    from gpu_util import tile_env
    kw = kw_of(N, "lf", "self", 0.5)
    fields = inputs.random_su2_state(N, 41)
    runs = []
    for spec in (None, "0"):
        with tile_env(spec, "LATTICE_SELF_CARRY"):
            say(f"[su2-carry] N={N} LATTICE_SELF_CARRY={spec}")
            t = [to_dev(f, torch.float64) for f in fields]
            lat = Lattice(doublet=t[0], pi_doublet=t[1], U=t[2], E=t[3], **kw)
            lat.step(1)
            lat.step(5)
            lat.sync()
            lat.step(-3)
            e = lat.energy()
            torch.cuda.synchronize()
            runs.append(([g.cpu().numpy() for grp in t for g in grp], e["a"], e["b"]))
            lat.close()
    (f1, a1, b1), (f0, a0, b0) = runs
    assert a1 == a0 and b1 == b0, (a1, a0, b1, b0)
    for g1, g0 in zip(f1, f0):
        assert np.array_equal(g1, g0)


@pytest.mark.parametrize("N,integ", [(13, "lf"), (64, "lf"), (13, "vv4")])
def test_su2_self_drift_only(N, integ):
    """The self-consistent steps' shortcuts: the drift (zero kick weight) runs
    alone (su2_drift) in place of a step pass, and the kick pass also forms the
    volume sums of the kicked state (in the energy pass's launch shape) in
    place of a separate energy pass.  The same expressions, which the compiler
    may contract into fused multiply-adds differently in different kernels, so
    fields, a, b and rho agree with a run without the shortcuts
    (LATTICE_U1_FUSE=0) to rounding (1e-14)."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    from gpu_util import tile_env
    kw = kw_of(N, integ, "self", 0.5)
    fields = inputs.random_su2_state(N, 41)
    runs = []
    for spec in (None, "0"):
        with tile_env(spec, "LATTICE_U1_FUSE"):
            say(f"[su2-drift] N={N} {integ} LATTICE_U1_FUSE={spec}")
            t = [to_dev(f, torch.float64) for f in fields]
            lat = Lattice(doublet=t[0], pi_doublet=t[1], U=t[2], E=t[3], **kw)
            lat.step(3)
            lat.step(2)
            e = lat.energy()
            torch.cuda.synchronize()
            runs.append(([g.cpu().numpy() for grp in t for g in grp], e["a"], e["b"], e["rho"]))
            lat.close()
    (f1, a1, b1, r1), (f0, a0, b0, r0) = runs
    for v1, v0 in ((a1, a0), (b1, b0), (r1, r0)):
        assert abs(v1 - v0) <= 1e-14 * abs(v0), (v1, v0)
    for g1, g0 in zip(f1, f0):
        assert rel_maxdiff(g1, g0) <= 1e-14


@pytest.mark.parametrize("N,integ,expansion", [(13, "lf", "self"), (64, "lf", "none")])
def test_su2_deferred_sums_bitwise(N, integ, expansion):
    """The summing passes (energy; kick and sums) leave their block partials to
    a one-block kernel after them instead of a ticketed last block: energies,
    Gauss maxima, fields, a and b equal, bit for bit, those of the ticketed
    passes (LATTICE_ENERGY_DEFER=0)."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    from gpu_util import tile_env
    kw = kw_of(N, integ, expansion, 0.5)
    fields = inputs.random_su2_state(N, 41)
    runs = []
    for spec in (None, "0"):
        with tile_env(spec, "LATTICE_ENERGY_DEFER"):
            say(f"[su2-defer] N={N} {integ} {expansion} LATTICE_ENERGY_DEFER={spec}")
            t = [to_dev(f, torch.float64) for f in fields]
            lat = Lattice(doublet=t[0], pi_doublet=t[1], U=t[2], E=t[3], **kw)
            lat.step(4)
            e = lat.energy()
            torch.cuda.synchronize()
            runs.append(([g.cpu().numpy() for grp in t for g in grp], e))
            lat.close()
    (f1, e1), (f0, e0) = runs
    for k in ("rho", "EK_B", "EG_B", "a", "b", "gauss_max", "gauss_div_max", "gauss_charge_max", "gauss_mean"):
        assert e1[k] == e0[k], (k, e1[k], e0[k])
    for g1, g0 in zip(f1, f0):
        assert np.array_equal(g1, g0)
