"""Pins of the U(1) (Abelian-Higgs) oracle: Gauss law, gauge invariance,
forces as energy gradients, brute-force covariant Laplacian, energy
conservation.  Sec. 3.2 (U(1) toolkit), sec. 5.2 (equations of motion and
Gauss constraint eq. GaussU1-eom), sec. 5.5.2 (kernels)."""
import math

import numpy as np
import pytest


def rand_u1(orc, N, seed=5, amp=0.4, Aamp=0.6, mom=False):
    rng = np.random.default_rng(seed)
    V = N ** 3
    th = rng.uniform(0, 2 * np.pi, V)
    r = amp * (1 + 0.3 * rng.standard_normal(V))
    phi = [math.sqrt(2) * r * np.cos(th), math.sqrt(2) * r * np.sin(th)]
    A = [Aamp * rng.standard_normal(V) for _ in range(3)]
    pi = [0.2 * rng.standard_normal(V) for _ in range(2)] if mom else [np.zeros(V), np.zeros(V)]
    piA = [0.2 * rng.standard_normal(V) for _ in range(3)] if mom else [np.zeros(V) for _ in range(3)]
    return phi, pi, A, piA


def model(orc, N=5, **kw):
    d = dict(N=N, dx=0.4, dt=0.02, lam=1.0, v=1.0, e=0.5, kappa_g=1.0)
    d.update(kw)
    return orc.U1Model(**d)


# --- T5: Gauss constraint preserved to roundoff by the leapfrog ----------------
@pytest.mark.parametrize("e,kg", [(0.5, 1.0), (1.3, 0.6)])
def test_gauss_constraint(orc, e, kg):
    m = model(orc, 5, e=e, kappa_g=kg)
    st = orc.U1State(m, *rand_u1(orc, 5))
    assert st.gauss()["gauss_max"] == 0.0
    for _ in range(10):
        st.run(20)
        g = st.gauss()
        scale = max(g["div_max"], g["charge_max"])
        assert scale > 1e-3
        assert g["gauss_max"] <= 1e-12 * scale
    st.sync()
    g = st.gauss()
    assert g["gauss_max"] <= 1e-12 * max(g["div_max"], g["charge_max"])


# --- T6: gauge invariance (transformation pair under which D+ is covariant) ----
def gauge_transform(orc, N, dx, e, state, alpha):
    phi, pi, A, piA = state
    ang = e * alpha

    def rot(c):
        return [np.cos(ang) * c[0] - np.sin(ang) * c[1], np.sin(ang) * c[0] + np.cos(ang) * c[1]]

    a3 = alpha.reshape(N, N, N)
    grad = [(np.roll(a3, -1, axis=2) - a3).reshape(-1) / dx,   # x fastest (last numpy axis)
            (np.roll(a3, -1, axis=1) - a3).reshape(-1) / dx,
            (np.roll(a3, -1, axis=0) - a3).reshape(-1) / dx]
    return rot(phi), rot(pi), [A[i] + grad[i] for i in range(3)], [p.copy() for p in piA]


def test_gauge_invariance(orc):
    N = 5
    m = model(orc, N, e=0.9)
    s0 = rand_u1(orc, N, mom=True)
    alpha = np.random.default_rng(9).uniform(-3, 3, N ** 3)
    s1 = gauge_transform(orc, N, m.dx, m.e, s0, alpha)
    E0 = orc.U1State(m, *s0).energy()
    E1 = orc.U1State(m, *s1).energy()
    for k in ("EK_phi", "EG_phi", "EV", "EK_A", "EG_A", "rho"):
        assert abs(E0[k] - E1[k]) <= 1e-13 * abs(E0["rho"]), k
    # evolution commutes with the transformation
    a = orc.U1State(m, *s0).run(15)
    b = orc.U1State(m, *s1).run(15)
    ta = gauge_transform(orc, N, m.dx, m.e, (a.phi, a.pi, a.A, a.piA), alpha)
    for x, y in zip(ta[0] + ta[1] + ta[2] + ta[3], b.phi + b.pi + b.A + b.piA):
        assert np.max(np.abs(x - y)) < 1e-12


# --- T7: forces are minus the gradient of the lattice energy --------------------
def test_forces_are_energy_gradients(orc):
    N = 4
    kg = 0.7
    m = model(orc, N, e=0.8, kappa_g=kg)
    phi, pi, A, piA = rand_u1(orc, N, mom=True)
    st = orc.U1State(m, phi, pi, A, piA)
    Fphi, FA = st.forces()

    def H(ph, AA):   # total energy N^3 rho with momenta zeroed (potential part)
        z2 = [np.zeros_like(ph[0])] * 2
        z3 = [np.zeros_like(ph[0])] * 3
        return orc.U1State(m, ph, z2, AA, z3).energy()["rho"] * N ** 3

    eps = 1e-5
    for site in (0, 21, 63):
        for c in range(2):
            pp = [f.copy() for f in phi]; pm = [f.copy() for f in phi]
            pp[c][site] += eps; pm[c][site] -= eps
            fd = -(H(pp, A) - H(pm, A)) / (2 * eps)
            assert abs(fd - Fphi[c][site]) < 1e-7 * max(1, abs(fd))
        for i in range(3):
            ap = [f.copy() for f in A]; am = [f.copy() for f in A]
            ap[i][site] += eps; am[i][site] -= eps
            fd = -kg * (H(phi, ap) - H(phi, am)) / (2 * eps)
            assert abs(fd - FA[i][site]) < 1e-7 * max(1, abs(fd))


# --- T13 (U(1)): covariant Laplacian against a dense Hermitian operator ----------
def test_covariant_laplacian_dense(orc):
    N, dx, e = 3, 0.4, 0.7
    m = model(orc, N, dx=dx, e=e, lam=0.0)
    phi, pi, A, piA = rand_u1(orc, N)
    idx = lambda x, y, z: x % N + N * ((y % N) + N * (z % N))
    M = np.zeros((N ** 3, N ** 3), dtype=complex)
    for z in range(N):
        for y in range(N):
            for x in range(N):
                n = idx(x, y, z)
                M[n, n] += -6 / dx ** 2
                for i, (ox, oy, oz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    M[n, idx(x + ox, y + oy, z + oz)] += np.exp(-1j * e * dx * A[i][n]) / dx ** 2
                    nm = idx(x - ox, y - oy, z - oz)
                    M[n, nm] += np.exp(1j * e * dx * A[i][nm]) / dx ** 2
    assert np.allclose(M, M.conj().T, atol=1e-14)
    psi = phi[0] + 1j * phi[1]
    D2 = M @ psi
    Fphi, _ = orc.U1State(m, phi, pi, A, piA).forces()
    assert np.max(np.abs(Fphi[0] - D2.real)) < 1e-12
    assert np.max(np.abs(Fphi[1] - D2.imag)) < 1e-12


def test_zero_links_reduce_to_scalar_laplacian(orc):
    N = 5
    m = model(orc, N, lam=0.0)
    phi, pi, A, piA = rand_u1(orc, N, Aamp=0.0)
    Fphi, FA = orc.U1State(m, phi, pi, A, piA).forces()
    for c in range(2):
        assert np.max(np.abs(Fphi[c] - orc.laplacian(phi[c], m.dx))) < 1e-12


# --- energy conservation at second order (a = 1) --------------------------------
def test_u1_energy_conservation_order(orc):
    errs = []
    for h in (0.02, 0.01):
        m = model(orc, 5, dt=h, e=0.9)
        st = orc.U1State(m, *rand_u1(orc, 5, mom=True))
        rho0 = st.energy()["rho"]
        worst = 0.0
        for _ in range(8):
            st.run(int(round(0.2 / h)))
            worst = max(worst, abs(1 - st.energy()["rho"] / rho0))
        errs.append(worst)
    assert abs(math.log2(errs[0] / errs[1]) - 2) < 0.3, errs


def test_u1_reversibility(orc):
    m = model(orc, 4, e=0.9)
    s0 = rand_u1(orc, 4, mom=True)
    st = orc.U1State(m, *s0).run(30).sync().run(-30).sync()
    for x, y in zip(st.phi + st.pi + st.A + st.piA, s0[0] + s0[1] + s0[2] + s0[3]):
        assert np.max(np.abs(x - y)) < 1e-12


def test_magnetic_energy_small_angle_limit(orc):
    """For small plaquette angles the compact magnetic energy tends to the
    non-compact sum of 1/2 (grad+_i A_j - grad+_j A_i)^2 (U(1) toolkit expressions),
    with no loss of digits from cancellation."""
    N = 5
    m = model(orc, N, e=0.7, kappa_g=1.0)
    phi, pi, A, piA = rand_u1(orc, N, Aamp=1e-5)
    E = orc.U1State(m, phi, pi, A, piA).energy()["EG_A"]
    a3 = [a.reshape(N, N, N) for a in A]
    d = lambda f, ax: (np.roll(f, -1, axis=2 - ax) - f) / m.dx     # forward difference along x/y/z
    F2 = 0.0
    for i in range(3):
        for j in range(i + 1, 3):
            F2 += np.sum((d(a3[j], i) - d(a3[i], j)) ** 2) / 2
    noncompact = F2 / N ** 3
    assert abs(E - noncompact) <= 1e-8 * noncompact
