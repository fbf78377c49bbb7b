"""Pins of the oracle's velocity-Verlet family for the gauge models (U(1) and
SU(2) at a = 1): VV2 equals the (separately pinned) leapfrog followed by its
sync; VV2 / VV4 / VV6 converge at orders 2 / 4 / 6; reversibility; the Gauss
law held along VV4 from Gauss-consistent charged initial conditions."""
import numpy as np
import pytest

import oracle as O
from paper_2102_01031_amd import inputs


def su2(N=4, dt=0.04, seed=3, **kw):
    m = O.SU2Model(N=N, dx=0.5, dt=dt, lam=1.0, v=0.7, g=1.0)
    return O.SU2State(m, *inputs.random_su2_state(N, seed, **kw))


def u1(N=4, dt=0.04, seed=4):
    m = O.U1Model(N=N, dx=0.5, dt=dt, lam=1.0, v=0.7, e=0.6, kappa_g=1.0)
    rng = np.random.default_rng(seed)
    sh = (N, N, N)
    f = lambda s: [s * rng.standard_normal(sh) for _ in range(2)]
    g = lambda s: [s * rng.standard_normal(sh) for _ in range(3)]
    return O.U1State(m, f(0.3), f(0.2), g(0.4), g(0.3))


def _copy(st):
    if isinstance(st, O.SU2State):
        return O.SU2State(st.m, st.phi, st.pi, st.U, st.E)
    return O.U1State(st.m, st.phi, st.pi, st.A, st.piA)


def _arrays(st):
    if isinstance(st, O.SU2State):
        return st.phi + st.pi + st.U + st.E
    return st.phi + st.pi + st.A + st.piA


@pytest.mark.parametrize("make", [su2, u1])
def test_vv2_is_leapfrog_with_sync(make):
    a = make()
    b = _copy(a)
    a.run_vv(7, 2)
    b.run(7).sync()
    for x, y in zip(_arrays(a), _arrays(b)):
        np.testing.assert_allclose(x, y, atol=1e-13)


@pytest.mark.parametrize("make", [su2, u1])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_convergence_order(make, order):
    T = 0.48
    ref = make(dt=T / 96)
    ref.run_vv(96, 8)
    errs = []
    for n in (4, 8):
        st = make(dt=T / n)
        st.run_vv(n, order)
        errs.append(max(np.abs(x - y).max() for x, y in zip(_arrays(st), _arrays(ref))))
    rate = np.log2(errs[0] / errs[1])
    assert rate == pytest.approx(order, abs=0.35), (errs, rate)


@pytest.mark.parametrize("make", [su2, u1])
def test_vv4_reversible(make):
    a = make()
    b = _copy(a)
    a.run_vv(9, 4)
    assert max(np.abs(x - y).max() for x, y in zip(_arrays(a), _arrays(b))) > 1e-3
    a.run_vv(-9, 4)
    for x, y in zip(_arrays(a), _arrays(b)):
        np.testing.assert_allclose(x, y, atol=1e-12)


def test_su2_vv4_keeps_gauss_law():
    N = 8
    m = O.SU2Model(N=N, dx=0.4, dt=0.02, lam=1.0, v=1.0, g=0.8)
    phi, pi = inputs.charged_fluctuations(N, m.dx, 4, 0.5, 2e-2, 0.5, 9)
    z = np.zeros((N, N, N))
    U = []
    for _ in range(3):
        U += [np.ones((N, N, N)), z, z, z]
    st = O.SU2State(m, phi, pi, U, [z] * 9)
    st.gauss_init()
    st.run_vv(20, 4)
    g = st.gauss()
    assert g["gauss_max"] < 1e-13 * max(g["div_max"], g["charge_max"])
