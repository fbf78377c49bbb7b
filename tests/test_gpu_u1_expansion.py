"""GPU parity of the U(1) model in an expanding background (sec. 5.5.2) against
the oracle at 1e-12: fixed power-law background (alpha = 1 and 0.5) and
self-consistent expansion (leapfrog, reading A3; velocity-Verlet family,
reading R1), on the tiled kernel and on the whole-row kernel (N = 64), with
energies, a, b and the Hubble residual, the Gauss law, sync and reversal."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import rel_maxdiff, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


EXP = {"fixed": oracle.FIXED, "self": oracle.SELF}
ORDER = {"vv2": 2, "vv4": 4, "vv6": 6}


def fields_of(N, seed=7, mom=0.3):
    rng = np.random.default_rng(seed)
    V = N ** 3
    th = rng.uniform(0, 2 * np.pi, V)
    r = 0.4 * (1 + 0.3 * rng.standard_normal(V))
    phi = [math.sqrt(2) * r * np.cos(th), math.sqrt(2) * r * np.sin(th)]
    pi = [mom * rng.standard_normal(V) for _ in range(2)]
    A = [0.4 * rng.standard_normal(V) for _ in range(3)]
    piA = [mom * rng.standard_normal(V) for _ in range(3)]
    return phi, pi, A, piA


def kw_of(N, integ, expansion, alpha):
    return dict(N=N, dx=0.4, dt=0.02, integrator=integ, expansion=expansion, potential="abelian_higgs", lam=1.0,
                v=1.0, e=0.7, kappa_g=0.8, alpha=alpha, kappa2=0.5, w_eos=1 / 3, H0=0.6, t_ref=0.0, a0=1.0, t0=0.1)


def oracle_state(kw, fields):
    m = oracle.U1Model(N=kw["N"], dx=kw["dx"], dt=kw["dt"], lam=kw["lam"], v=kw["v"], e=kw["e"],
                       kappa_g=kw["kappa_g"], expansion=EXP[kw["expansion"]], alpha=kw["alpha"],
                       kappa2=kw["kappa2"], w_eos=kw["w_eos"], H0=kw["H0"], t0=kw["t_ref"], a0=kw["a0"])
    return oracle.U1State(m, *fields, t=kw["t0"])


def compare(gt, st, what):
    for name, gl, ol in zip(("phi", "pi", "A", "piA"), gt, (st.phi, st.pi, st.A, st.piA)):
        for i, (g, o) in enumerate(zip(gl, ol)):
            e = rel_maxdiff(g.cpu().numpy(), o)
            assert e <= TOL, f"{what} {name}[{i}] rel err {e:.3e}"


def compare_energy(eg, eo, what):
    for kg, ko in (("rho", "rho"), ("EK_A", "EK_A"), ("EG_A", "EG_A"), ("a", "a"), ("b", "b")):
        assert abs(eg[kg] - eo[ko]) <= TOL * abs(eo[ko]), (what, kg, eg[kg], eo[ko])
    assert abs(eg["EK"][0] - eo["EK_phi"]) <= TOL * abs(eo["EK_phi"]), what
    assert abs(eg["EG"][0] - eo["EG_phi"]) <= TOL * abs(eo["EG_phi"]), what
    assert abs(eg["hubble_res"] - eo["hubble_res"]) <= 1e-11, (what, eg["hubble_res"], eo["hubble_res"])


def run_oracle(st, integ, n):
    return st.run(n) if integ == "lf" else st.run_vv(n, ORDER[integ])


@pytest.mark.parametrize("N,integ,expansion,alpha,calls", [
    (12, "lf", "fixed", 1.0, [9]), (13, "lf", "fixed", 0.5, [5, 6]), (64, "lf", "fixed", 0.5, [4]),
    (12, "lf", "self", 1.0, [5, 4]), (13, "lf", "self", 0.5, [7]), (64, "lf", "self", 0.5, [3]),
    (12, "vv2", "fixed", 0.5, [4]), (13, "vv4", "fixed", 1.0, [3]), (64, "vv4", "fixed", 0.5, [2]),
    (12, "vv2", "self", 0.5, [3, 2]), (13, "vv4", "self", 1.0, [2]), (16, "vv6", "self", 0.5, [1])])
def test_u1_expanding_matches_oracle(N, integ, expansion, alpha, calls):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    kw = kw_of(N, integ, expansion, alpha)
    fields = fields_of(N)
    say(f"[u1-exp] N={N} {integ} {expansion} alpha={alpha} calls={calls}")
    phi, pi, A, piA = [to_dev(f, torch.float64) for f in fields]
    lat = Lattice(phi, pi, A=A, piA=piA, **kw)
    st = oracle_state(kw, fields)
    compare_energy(lat.energy(), st.energy(), "start")
    for n in calls:
        lat.step(n)
        run_oracle(st, integ, n)
        torch.cuda.synchronize()
        compare((phi, pi, A, piA), st, f"+{n}")
        eg, eo = lat.energy(), st.energy()
        compare_energy(eg, eo, f"+{n}")
        g = st.gauss()
        assert abs(eg["gauss_max"] - g["gauss_max"]) <= TOL * max(g["div_max"], g["charge_max"])
        say(f"[u1-exp]   +{n}: a={eg['a']:.10f} b={eg['b']:.6e} r_H={eg['hubble_res']:.2e}")
    assert eg["a"] != 1.0
    if integ == "lf":
        lat.sync()
        st.sync()
        compare((phi, pi, A, piA), st, "synced")
        compare_energy(lat.energy(), st.energy(), "synced")
    lat.close()


@pytest.mark.parametrize("integ,expansion", [("lf", "self"), ("vv4", "self"), ("lf", "fixed")])
def test_u1_expanding_reversal_and_gauss(integ, expansion):
    """A run, back to the start (fields, a and b), with the Gauss residual of a
    Gauss-free start held to rounding along the way."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    N = 16
    fields = fields_of(N, mom=0.0)
    kw = kw_of(N, integ, expansion, 0.5)
    phi, pi, A, piA = [to_dev(f, torch.float64) for f in fields]
    lat = Lattice(phi, pi, A=A, piA=piA, **kw)
    e0 = lat.energy()
    lat.step(20)
    e1 = lat.energy()
    scale = max(e1["gauss_div_max"], e1["gauss_charge_max"])
    assert scale > 0 and e1["gauss_max"] <= 1e-12 * scale
    if integ == "lf":
        lat.sync()
    lat.step(-20)
    if integ == "lf":
        lat.sync()
    e2 = lat.energy()
    assert abs(e2["a"] - e0["a"]) <= 1e-13 and abs(e2["b"] - e0["b"]) <= 1e-11 * abs(e0["b"])
    for g, o in zip(phi + pi + A + piA, fields[0] + fields[1] + fields[2] + fields[3]):
        assert np.max(np.abs(g.cpu().numpy() - o.reshape(-1))) <= 1e-11
    lat.close()


@pytest.mark.parametrize("N", [13, 64])
def test_u1_self_carry_bitwise(N):
    """Self-consistent leapfrog steps after a call's first take the sums before
    the kick from the passes around them: fields, a and b equal, bit for bit,
    those of a run that measures them in an energy pass on every step
    (LATTICE_SELF_CARRY=0)."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    from gpu_util import tile_env
    kw = kw_of(N, "lf", "self", 0.5)
    fields = fields_of(N)
    runs = []
    for spec in (None, "0"):
        with tile_env(spec, "LATTICE_SELF_CARRY"):
            say(f"[u1-carry] N={N} LATTICE_SELF_CARRY={spec}")
            t = [to_dev(f, torch.float64) for f in fields]
            lat = Lattice(t[0], t[1], A=t[2], piA=t[3], **kw)
            lat.step(1)
            lat.step(6)
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


@pytest.mark.parametrize("N,spec", [(13, "5"), (64, None), (64, "64")])
def test_u1_energy_columns(N, spec):
    """The energy pass in columns of z planes per block (the default, about 256
    blocks; or LATTICE_U1_ENERGY_ZC, with a ragged last column at N = 13)
    against one plane per block: the same site terms summed in another order."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    from gpu_util import tile_env
    kw = kw_of(N, "lf", "none", 1.0)
    fields = fields_of(N)
    es = []
    for s in (spec, "1"):
        with tile_env(s, "LATTICE_U1_ENERGY_ZC"):
            t = [to_dev(f, torch.float64) for f in fields]
            lat = Lattice(t[0], t[1], A=t[2], piA=t[3], **kw)
            lat.step(2)
            es.append(lat.energy())
            lat.close()
    for k in ("rho", "EK_A", "EG_A"):
        assert abs(es[0][k] - es[1][k]) <= 1e-13 * abs(es[1][k]), (k, es[0][k], es[1][k])
    for k in ("gauss_max", "gauss_div_max", "gauss_charge_max"):
        assert es[0][k] == es[1][k], k


@pytest.mark.parametrize("N,integ", [(64, "lf"), (64, "vv4"), (13, "lf")])
def test_u1_self_fused_kick_sums_bitwise(N, integ):
    """The self-consistent steps' shortcuts: on the whole-row kernel (N = 64) the
    kick pass also forms the volume sums of the kicked state that the b kick
    needs, and at every N the drift runs alone (u1_drift) in place of a step
    pass with zero kick weight.  Fields, a and b equal, bit for bit, those of a
    run with a separate energy pass after each kick and full step passes
    (LATTICE_U1_FUSE=0)."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    from gpu_util import tile_env
    kw = kw_of(N, integ, "self", 0.5)
    fields = fields_of(N)
    runs = []
    for spec in (None, "0"):
        with tile_env(spec, "LATTICE_U1_FUSE"):
            say(f"[u1-fuse] N={N} {integ} LATTICE_U1_FUSE={spec}")
            t = [to_dev(f, torch.float64) for f in fields]
            lat = Lattice(t[0], t[1], A=t[2], piA=t[3], **kw)
            lat.step(3)
            lat.step(2)
            e = lat.energy()
            torch.cuda.synchronize()
            runs.append(([g.cpu().numpy() for grp in t for g in grp], e["a"], e["b"], e["rho"]))
            lat.close()
    (f1, a1, b1, r1), (f0, a0, b0, r0) = runs
    assert a1 == a0 and b1 == b0 and r1 == r0, (a1, a0, b1, b0, r1, r0)
    for g1, g0 in zip(f1, f0):
        assert np.array_equal(g1, g0)


@pytest.mark.parametrize("N,integ,expansion", [(64, "lf", "self"), (13, "lf", "self"), (64, "vv4", "none"),
                                               (13, "lf", "none")])
def test_u1_deferred_sums_bitwise(N, integ, expansion):
    """The summing passes (energy; kick and sums) leave their block partials to
    a one-block kernel after them instead of a ticketed last block: energies,
    Gauss maxima, fields, a and b equal, bit for bit, those of the ticketed
    passes (LATTICE_ENERGY_DEFER=0), on the whole-row kernel (64) and the
    per-site kernel (13)."""
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    from gpu_util import tile_env
    kw = kw_of(N, integ, expansion, 0.5)
    fields = fields_of(N)
    runs = []
    for spec in (None, "0"):
        with tile_env(spec, "LATTICE_ENERGY_DEFER"):
            say(f"[u1-defer] N={N} {integ} {expansion} LATTICE_ENERGY_DEFER={spec}")
            t = [to_dev(f, torch.float64) for f in fields]
            lat = Lattice(t[0], t[1], A=t[2], piA=t[3], **kw)
            lat.step(4)
            e = lat.energy()
            torch.cuda.synchronize()
            runs.append(([g.cpu().numpy() for grp in t for g in grp], e))
            lat.close()
    (f1, e1), (f0, e0) = runs
    for k in ("rho", "EK_A", "EG_A", "a", "b", "gauss_max", "gauss_div_max", "gauss_charge_max", "gauss_mean"):
        assert e1[k] == e0[k], (k, e1[k], e0[k])
    for g1, g0 in zip(f1, f0):
        assert np.array_equal(g1, g0)
