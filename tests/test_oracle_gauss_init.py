"""Pins of the oracle's Gauss-consistent initial gauge momenta (sec. 5.5.1, eqs.
kAi1 and GaugeCurrentFluc on the lattice) and of the charged-fluctuation
generator (eqs. fpr_influct3, fpr_influct4 with InConstr:1, InConstr:2):

- the solver's field satisfies the lattice Gauss law div- E = rho - <rho>
  exactly (to rounding) for any rho, and is curl-free (a lattice gradient);
- a plane-wave charge gives the closed-form field;
- after the SU(2) / U(1) init on charged fluctuations the oracle's own Gauss
  residual (a separate, covariant computation) vanishes to rounding, and stays
  there along the leapfrog evolution;
- the generator's charge has no homogeneous part, and each mode's momenta are
  a real multiple of its fields, the same for every component."""
import numpy as np
import pytest

import oracle as O
from paper_2102_01031_amd import inputs


def div_minus(E, dx, N):
    E = [e.reshape(N, N, N) for e in E]
    return sum((E[i] - np.roll(E[i], 1, axis=2 - i)) / dx for i in range(3))


@pytest.mark.parametrize("N", [5, 8, 12])
def test_solver_satisfies_lattice_gauss_law(N):
    dx = 0.37
    rho = np.random.default_rng(N).standard_normal((N, N, N))
    E = O.gauss_solve(rho, dx)
    res = div_minus(E, dx, N) - (rho - rho.mean())
    assert np.abs(res).max() < 1e-12 * np.abs(rho).max()
    Ez = [e.reshape(N, N, N) for e in E]
    for i in range(3):
        for j in range(3):
            if i == j:
                continue
            curl = (np.roll(Ez[j], -1, axis=2 - i) - Ez[j]) - (np.roll(Ez[i], -1, axis=2 - j) - Ez[i])
            assert np.abs(curl).max() < 1e-12 * np.abs(Ez[i]).max()


def test_solver_plane_wave_closed_form():
    N, dx = 8, 0.5
    m = (1, 2, 3)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    th = 2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / N
    rho = np.cos(th)
    lam = 4 / dx ** 2 * sum(np.sin(np.pi * mi / N) ** 2 for mi in m)
    E = O.gauss_solve(rho, dx)
    for i in range(3):
        ref = -(np.cos(th + 2 * np.pi * m[i] / N) - np.cos(th)) / (lam * dx)
        np.testing.assert_allclose(E[i].reshape(N, N, N), ref, atol=1e-13)


def test_generator_charge_free_and_mode_proportional():
    N = 12
    for ncomp in (2, 4):
        phi, pi = inputs.charged_fluctuations(N, 0.4, ncomp, 0.3, 1e-3, 0.7, 11 + ncomp)
        ft = [np.fft.fftn(f - f.mean()) for f in phi]
        fp = [np.fft.fftn(p) for p in pi]
        mask = np.abs(ft[0]) > 1e-12 * np.abs(ft[0]).max()
        c0 = (fp[0][mask] / ft[0][mask])
        assert np.abs(c0.imag).max() < 1e-8 * np.abs(c0.real).max()
        for n in range(1, ncomp):
            np.testing.assert_allclose(fp[n][mask] / ft[n][mask], c0, rtol=1e-8, atol=1e-10)
        if ncomp == 2:
            rho = phi[0] * pi[1] - phi[1] * pi[0]
            assert abs(rho.sum()) < 1e-12 * np.abs(rho).sum()
        else:
            psi = (phi[0] + 1j * phi[1], phi[2] + 1j * phi[3])
            pp = (pi[0] + 1j * pi[1], pi[2] + 1j * pi[3])
            S = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]])
            for a in range(3):
                rho = sum(np.conj(psi[r]) * 0.5 * S[a][r, q] * pp[q] for r in range(2) for q in range(2)).imag
                assert abs(rho.sum()) < 1e-12 * np.abs(rho).sum()


def _su2_charged(N, seed):
    m = O.SU2Model(N=N, dx=0.4, dt=0.02, lam=1.0, v=1.0, g=0.8)
    phi, pi = inputs.charged_fluctuations(N, m.dx, 4, 0.5, 2e-2, 0.5, seed)
    z = np.zeros((N, N, N))
    U = []
    for _ in range(3):
        U += [np.ones((N, N, N)), z, z, z]
    return O.SU2State(m, phi, pi, U, [z] * 9)


def test_su2_init_satisfies_covariant_gauss_law_and_keeps_it():
    st = _su2_charged(10, 21)
    before = st.gauss()
    assert before["gauss_max"] > 1e-3                      # the charged start violates it
    mean = st.gauss_init()
    assert np.abs(mean).max() < 1e-15
    g0 = st.gauss()
    assert g0["charge_max"] > 1e-3
    assert g0["gauss_max"] < 1e-13 * max(g0["div_max"], g0["charge_max"])
    st.run(40)
    g1 = st.gauss()
    assert g1["gauss_max"] < 1e-13 * max(g1["div_max"], g1["charge_max"])
    assert st.energy()["EG_B"] > 0


def test_su2_init_refuses_links_off_the_identity():
    st = _su2_charged(6, 3)
    st.U[1][5] = 1e-3
    with pytest.raises(RuntimeError):
        st.gauss_init()


def test_u1_init_satisfies_gauss_law_and_keeps_it():
    N = 10
    m = O.U1Model(N=N, dx=0.4, dt=0.02, lam=1.0, v=1.0, e=0.5, kappa_g=1.0)
    phi, pi = inputs.charged_fluctuations(N, m.dx, 2, 0.5, 2e-2, 0.5, 5)
    rng = np.random.default_rng(2)
    A = [0.5 * rng.standard_normal((N, N, N)) for _ in range(3)]   # the Abelian law does not see the links
    st = O.U1State(m, phi, pi, A, [np.zeros((N, N, N))] * 3)
    assert st.gauss()["gauss_max"] > 1e-3
    mean = st.gauss_init()
    assert abs(mean[0]) < 1e-15
    g0 = st.gauss()
    assert g0["gauss_max"] < 1e-13 * max(g0["div_max"], g0["charge_max"])
    st.run(40)
    g1 = st.gauss()
    assert g1["gauss_max"] < 1e-13 * max(g1["div_max"], g1["charge_max"])
