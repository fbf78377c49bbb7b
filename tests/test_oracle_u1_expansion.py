"""Pins of the U(1) oracle in an expanding background (sec. 5.5.2: momenta
pi = a^{3-alpha} phi', pi_A = a^{1-alpha} F_0i, the kernels of eq.
kernelcomplexscalar and the one after it, and the b' equation with the gauge
energies weighted by alpha - 1), fixed (eq. ScaleFactorPowerLaw) and
self-consistent, with leapfrog and the velocity-Verlet family.

What fixes it, independently of its own formulas:
  - a neutral, real complex field with v = 0 and no gauge field is one real
    scalar with V = (lambda/4) phi^4 / 4: it must follow the scalar oracle (its
    own expansion code) step by step, scale factor included;
  - at alpha = 1 a pure gauge field is conformal (eq. U1eom loses every power
    of a), so its evolution must not see the background at all;
  - the Gauss law (eq. GaussU1-eom, which in these variables carries no power
    of a) holds to rounding along expanding runs;
  - the kicks are minus the gradient of a^{3+alpha} L^3 rho_pot, rho_pot the
    potential-type energies the oracle reports at a (the Hamiltonian form);
  - reversibility with a and b; the Hubble constraint (eq. FriedmannHubble)
    violated only at the integrator's order with sizeable gauge energy at
    alpha = 0.5, where the gauge energies enter the b kernel."""
import math

import numpy as np
import pytest


def rand_u1(N, seed=5, amp=0.4, Aamp=0.3, mom=0.2, pmom=0.2):
    rng = np.random.default_rng(seed)
    V = N ** 3
    th = rng.uniform(0, 2 * np.pi, V)
    r = amp * (1 + 0.3 * rng.standard_normal(V))
    phi = [math.sqrt(2) * r * np.cos(th), math.sqrt(2) * r * np.sin(th)]
    A = [Aamp * rng.standard_normal(V) for _ in range(3)]
    pi = [pmom * rng.standard_normal(V) for _ in range(2)]
    piA = [mom * rng.standard_normal(V) for _ in range(3)]
    return phi, pi, A, piA


def u1_model(orc, N=5, **kw):
    d = dict(N=N, dx=0.4, dt=0.02, lam=1.0, v=1.0, e=0.5, kappa_g=1.0)
    d.update(kw)
    return orc.U1Model(**d)


def run(st, integ, n):
    if integ == "LF":
        return st.run(n)
    return st.run_vv(n, {"VV2": 2, "VV4": 4, "VV6": 6}[integ])


@pytest.mark.parametrize("integ,expansion,alpha", [("LF", "FIXED", 1.0), ("LF", "FIXED", 0.5), ("LF", "SELF", 1.0),
                                                   ("VV2", "SELF", 0.5), ("VV4", "FIXED", 0.5),
                                                   ("VV4", "SELF", 1.0)])
def test_real_neutral_field_is_the_scalar_oracle(orc, integ, expansion, alpha):
    N, lam, dt = 5, 1.6, 0.02
    exp_ = getattr(orc, expansion)
    kw = dict(expansion=exp_, alpha=alpha, kappa2=3.0, w_eos=1 / 3, H0=0.6, t0=0.0, a0=1.0)
    rng = np.random.default_rng(3)
    V = N ** 3
    f = 0.8 + 0.2 * rng.standard_normal(V)
    p = 0.3 * rng.standard_normal(V)
    z = np.zeros(V)
    um = u1_model(orc, N, lam=lam, v=0.0, dt=dt, **kw)
    u = orc.U1State(um, [f, z], [p, z], [z, z, z], [z, z, z], t=0.1)
    sm = orc.ScalarModel(N=N, dx=um.dx, dt=dt, nfields=1, potential=orc.PHI4, lam=lam / 4,
                         integrator={"LF": orc.LF, "VV2": orc.VV2, "VV4": orc.VV4}[integ], **kw)
    s = orc.ScalarState(sm, [f], [p], t=0.1)
    assert abs(u.a - s.a) <= 1e-15 and abs(u.b - s.b) <= 1e-15 * abs(s.b)
    for _ in range(3):
        run(u, integ, 7)
        s.run(7)
        assert np.max(np.abs(u.phi[0] - s.phi[0])) <= 1e-13
        assert np.max(np.abs(u.pi[0] - s.pi[0])) <= 1e-13
        assert np.max(np.abs(u.phi[1])) == 0 and np.max(np.abs(u.A[0])) == 0
        assert abs(u.a - s.a) <= 1e-14 * s.a and abs(u.b - s.b) <= 1e-13 * abs(s.b)
        eu, es = u.energy(), s.energy()
        assert abs(eu["rho"] - es["rho"]) <= 1e-13 * es["rho"]
        assert abs(eu["b"] - es["b"]) <= 1e-13 * abs(es["b"])
    assert u.a > 1.02


@pytest.mark.parametrize("integ", ["LF", "VV4"])
@pytest.mark.parametrize("expansion", ["FIXED", "SELF"])
def test_pure_gauge_field_is_conformal_at_alpha_1(orc, integ, expansion):
    N = 5
    _, _, A, piA = rand_u1(N, mom=0.3)
    z = [np.zeros(N ** 3)] * 2
    flat = orc.U1State(u1_model(orc, N), z, z, A, piA)
    exp_ = getattr(orc, expansion)
    bg = orc.U1State(u1_model(orc, N, expansion=exp_, alpha=1.0, kappa2=2.0, w_eos=1 / 3, H0=0.9), z, z, A, piA)
    run(flat, integ, 20)
    run(bg, integ, 20)
    assert bg.a > 1.1
    for i in range(3):
        assert np.array_equal(bg.A[i], flat.A[i]) and np.array_equal(bg.piA[i], flat.piA[i])


@pytest.mark.parametrize("integ,expansion,alpha", [("LF", "FIXED", 0.5), ("LF", "SELF", 0.5), ("VV4", "SELF", 1.0),
                                                   ("VV2", "FIXED", 1.0)])
def test_gauss_law_with_expansion(orc, integ, expansion, alpha):
    # zero momenta: G = 0 at the start; the run creates charges and currents
    N = 6
    phi, pi, A, piA = rand_u1(N, mom=0.0, pmom=0.0)
    m = u1_model(orc, N, e=0.9, kappa_g=0.7, expansion=getattr(orc, expansion), alpha=alpha, kappa2=0.1, H0=0.5)
    st = orc.U1State(m, phi, pi, A, piA)
    worst = 0.0
    for _ in range(5):
        run(st, integ, 20)
        g = st.gauss()
        worst = max(worst, g["gauss_max"] / max(g["div_max"], g["charge_max"]))
    assert st.a > 1.05
    assert worst <= 1e-12, worst


@pytest.mark.parametrize("a,alpha", [(1.0, 1.0), (1.7, 1.0), (1.4, 0.5), (0.8, 0.0)])
def test_kicks_are_minus_gradient_of_the_expanding_hamiltonian(orc, a, alpha):
    N, kg = 4, 0.7
    m = u1_model(orc, N, e=0.8, kappa_g=kg, expansion=orc.SELF, alpha=alpha)
    phi, pi, A, piA = rand_u1(N, Aamp=0.6)
    st = orc.U1State(m, phi, pi, A, piA, a=a, b=0.0)
    Fphi, FA = st.forces_at(a)
    z2 = [np.zeros(N ** 3)] * 2
    z3 = [np.zeros(N ** 3)] * 3

    def H(ph, AA):   # a^{3+alpha} L^3 rho at zero momenta, L^3 in units of dx^3: N^3
        return a ** (3 + alpha) * orc.U1State(m, ph, z2, AA, z3, a=a, b=0.0).energy()["rho"] * N ** 3

    eps = 1e-5
    for site in (0, 21, 63):
        for c in range(2):
            pp = [f.copy() for f in phi]
            pm = [f.copy() for f in phi]
            pp[c][site] += eps
            pm[c][site] -= eps
            fd = -(H(pp, A) - H(pm, A)) / (2 * eps)
            assert abs(fd - Fphi[c][site]) < 1e-7 * max(1, abs(fd))
        for i in range(3):
            ap = [f.copy() for f in A]
            am = [f.copy() for f in A]
            ap[i][site] += eps
            am[i][site] -= eps
            fd = -kg * (H(phi, ap) - H(phi, am)) / (2 * eps)
            assert abs(fd - FA[i][site]) < 1e-7 * max(1, abs(fd))


@pytest.mark.parametrize("integ,expansion", [("LF", "FIXED"), ("LF", "SELF"), ("VV4", "SELF")])
def test_reversibility_with_expansion(orc, integ, expansion):
    N = 5
    phi, pi, A, piA = rand_u1(N)
    m = u1_model(orc, N, expansion=getattr(orc, expansion), alpha=0.5, kappa2=2.0, H0=0.5)
    st = orc.U1State(m, phi, pi, A, piA)
    a0, b0 = st.a, st.b
    if integ == "LF":
        st.run(15).sync().run(-15).sync()
    else:
        st.run_vv(15, 4).run_vv(-15, 4)
    assert abs(st.a - a0) <= 1e-14 and abs(st.b - b0) <= 1e-12 * abs(b0)
    for got, want in ((st.phi, phi), (st.pi, pi), (st.A, A), (st.piA, piA)):
        for g, w in zip(got, want):
            assert np.max(np.abs(g - w)) <= 1e-12 * max(1.0, np.max(np.abs(w)))


@pytest.mark.parametrize("integ,p", [("LF", 2), ("VV2", 2), ("VV4", 4)])
def test_hubble_constraint_order_with_gauge_energy(orc, integ, p):
    """alpha = 0.5: the gauge energies enter the b kernel with weight -1/2; a
    wrong power of a in them, or a missing gauge term, breaks the constraint at
    first order in time instead of at the integrator's order."""
    res = []
    for h in (0.02, 0.01):
        N = 4
        phi, pi, A, piA = rand_u1(N, mom=0.6, Aamp=0.5)
        m = u1_model(orc, N, dt=h, expansion=orc.SELF, alpha=0.5, kappa2=4.0)
        st = orc.U1State(m, phi, pi, A, piA)
        e0 = st.energy()
        assert abs(e0["hubble_res"]) < 1e-15
        assert e0["EK_A"] + e0["EG_A"] > 0.2 * e0["rho"]
        worst = 0.0
        for _ in range(6):
            run(st, integ, int(round(0.1 / h)))
            worst = max(worst, abs(st.energy()["hubble_res"]))
        assert st.a > 1.05
        res.append(worst)
    assert abs(math.log2(res[0] / res[1]) - p) < 0.4, res
