"""Pins of the oracle's leapfrog with self-consistent expansion (reading A3 of
the oracle header: sec. 6.1 keeps the kicks' momentum averages and the
drifts' field averages for the scale factor; the companion paper with the
discrete formulas is absent).

What fixes the scheme, independently of its own formulas:
  - kappa^2 = 0 switches gravity off, so b stays constant and a grows
    linearly; a linear a(t) is the power-law background of eq.
    ScaleFactorPowerLaw with exponent p = 1 (w = (2 alpha - 1)/3), and the
    fields must then follow the fixed-background leapfrog step for step;
  - time reversibility (run, sync, run backward, sync) of fields, momenta,
    a and b;
  - the trajectory does not depend on when it is synchronised;
  - second-order convergence towards the fourth-order velocity-Verlet
    solution of the same system, and the Hubble constraint violated only at
    order h^2 (convergence and constraint orders are also in
    test_oracle_scalar.py)."""
import math

import numpy as np
import pytest


def model(orc, integ, dt=0.01, kappa2=0.25, alpha=1.0, N=6, q=100.0, expansion=None, w_eos=1 / 3, H0=0.1443):
    return orc.ScalarModel(N=N, dx=0.4, dt=dt, nfields=2, potential=orc.PHI4_CHI2, lam=1.0, q=q,
                           expansion=orc.SELF if expansion is None else expansion, integrator=integ, alpha=alpha,
                           kappa2=kappa2, w_eos=w_eos, H0=H0, a0=1.0)


def state(orc, m, seed=11, amp=0.05):
    rng = np.random.default_rng(seed)
    V = m.N ** 3
    phi = [1.0 + amp * rng.standard_normal(V), amp * rng.standard_normal(V)]
    pi = [amp * rng.standard_normal(V), amp * rng.standard_normal(V)]
    return phi, pi


@pytest.mark.parametrize("alpha,w", [(1.0, 1 / 3), (0.5, 0.0)])
def test_no_gravity_is_the_linear_fixed_background(orc, alpha, w):
    H0 = 0.7
    ms = model(orc, orc.LF, kappa2=0.0, alpha=alpha)
    mf = model(orc, orc.LF, alpha=alpha, expansion=orc.FIXED, w_eos=w, H0=H0)
    phi, pi = state(orc, ms)
    a = orc.ScalarState(ms, phi, pi, a=1.0, b=H0)
    b = orc.ScalarState(mf, phi, pi)
    assert abs(b.a - 1.0) < 1e-15 and abs(b.b - H0) < 1e-15
    for _ in range(4):
        a.run(9)
        b.run(9)
        assert abs(a.a - b.a) <= 1e-13 * b.a and abs(a.b - H0) <= 1e-15
        for s in range(2):
            assert np.max(np.abs(a.phi[s] - b.phi[s])) <= 1e-13
            assert np.max(np.abs(a.pi[s] - b.pi[s])) <= 1e-12 * np.max(np.abs(b.pi[s]))
    a.sync()
    b.sync()
    for s in range(2):
        assert np.max(np.abs(a.pi[s] - b.pi[s])) <= 1e-12 * np.max(np.abs(b.pi[s]))


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_reversibility(orc, alpha):
    m = model(orc, orc.LF, alpha=alpha, kappa2=1.0)
    phi, pi = state(orc, m)
    st = orc.ScalarState(m, phi, pi)
    a0, b0 = st.a, st.b
    st.run(25)
    assert st.a > 1.001
    st.sync().run(-25).sync()
    assert abs(st.a - a0) <= 1e-14 and abs(st.b - b0) <= 1e-13 * abs(b0)
    for s in range(2):
        assert np.max(np.abs(st.phi[s] - phi[s])) <= 1e-13
        assert np.max(np.abs(st.pi[s] - pi[s])) <= 1e-12 * np.max(np.abs(pi[s]))


def test_trajectory_independent_of_sync_cadence(orc):
    m = model(orc, orc.LF, kappa2=1.0)
    phi, pi = state(orc, m)
    one = orc.ScalarState(m, phi, pi).run(20).sync()
    many = orc.ScalarState(m, phi, pi).run(7).sync().run(6).sync().run(1).sync().run(6).sync()
    assert abs(one.a - many.a) <= 1e-14 * one.a and abs(one.b - many.b) <= 1e-13 * abs(one.b)
    assert one.t == many.t
    for s in range(2):
        assert np.max(np.abs(one.phi[s] - many.phi[s])) <= 1e-13
        assert np.max(np.abs(one.pi[s] - many.pi[s])) <= 1e-12 * np.max(np.abs(one.pi[s]))


def test_converges_to_the_vv4_solution_at_second_order(orc):
    """Against VV4 on the same self-consistent system at a small step (its
    error is far below the leapfrog's), the leapfrog error falls by 4 when h
    halves: the scheme approximates the right equations, not only itself."""
    T = 0.8
    ref = model(orc, orc.VV4, dt=0.0025, kappa2=4.0, N=4, q=20.0)
    phi, pi = state(orc, ref, amp=0.2)
    r = orc.ScalarState(ref, phi, pi).run(int(round(T / 0.0025)))
    errs = []
    for h in (0.02, 0.01):
        m = model(orc, orc.LF, dt=h, kappa2=4.0, N=4, q=20.0)
        st = orc.ScalarState(m, phi, pi).run(int(round(T / h))).sync()
        assert abs(st.t - r.t) < 1e-12
        e = max(max(np.max(np.abs(st.phi[s] - r.phi[s])) for s in range(2)),
                max(np.max(np.abs(st.pi[s] - r.pi[s])) for s in range(2)),
                abs(st.a - r.a), abs(st.b - r.b))
        errs.append(e)
    assert r.a > 1.05
    assert abs(math.log2(errs[0] / errs[1]) - 2) < 0.2, errs


def test_energy_reports_synchronised_b(orc):
    """lattice-style measurement on a staggered state: b at integer time is
    the half-kicked b (not the stored half-step value), and the measurement
    leaves the state alone."""
    m = model(orc, orc.LF, kappa2=1.0)
    phi, pi = state(orc, m)
    st = orc.ScalarState(m, phi, pi).run(5)
    b_half = st.b
    e = st.energy()
    assert st.b == b_half
    synced = orc.ScalarState(m, phi, pi).run(5).sync()
    assert abs(e["b"] - synced.b) <= 1e-15 * abs(synced.b)
    assert abs(e["b"] - b_half) > 1e-8 * abs(b_half)
    assert abs(e["hubble_lhs"] - synced.b ** 2) <= 1e-14 * synced.b ** 2
    assert abs(e["rho"] - synced.energy()["rho"]) <= 1e-14 * e["rho"]
