"""Pins of the scalar-sector oracle against facts the paper and mathematics fix.

Each test names the passage it rests on.  None of them retypes the oracle's
own formulas: they use closed forms, spectral identities, exact discrete
solutions, invariants (reversibility, summation by parts, energy), special
cases solved by library routines (Jacobi elliptic functions) and convergence
orders.
"""
import math

import numpy as np
import pytest
from scipy.special import ellipj, ellipk


def plane_wave(N, n):
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    return np.cos(2 * np.pi * (n[0] * x + n[1] * y + n[2] * z) / N)


def lattice_w2(N, dx, n):
    # eq. ForwardBackwardMomentum: k_lat = 2 sin(pi n/N)/dx, so Lap -> -sum k_lat^2
    return sum((2.0 * math.sin(math.pi * ni / N) / dx) ** 2 for ni in n)


# --- T1: lattice dispersion ---------------------------------------------------
@pytest.mark.parametrize("N,n", [(8, (1, 0, 0)), (8, (3, 2, 1)), (8, (4, 4, 4)), (6, (1, 2, 3)),
                                 (5, (2, 1, 0)), (7, (3, 3, 1))])
def test_laplacian_plane_wave_eigenvalue(orc, N, n):
    dx = 0.37
    f = plane_wave(N, n)
    lap = orc.laplacian(f.reshape(-1), dx).reshape(N, N, N)
    expect = -lattice_w2(N, dx, n) * f
    assert np.max(np.abs(lap - expect)) <= 1e-12 * lattice_w2(N, dx, n) + 1e-13


# --- T13: brute force against a dense operator built from Kronecker products ---
@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_laplacian_dense_matrix(orc, N):
    dx = 0.7
    C = -2.0 * np.eye(N) + np.roll(np.eye(N), 1, axis=1) + np.roll(np.eye(N), -1, axis=1)
    if N == 2:
        C = np.array([[-2.0, 2.0], [2.0, -2.0]])
    I = np.eye(N)
    L = (np.kron(np.kron(I, I), C) + np.kron(np.kron(I, C), I) + np.kron(np.kron(C, I), I)) / dx ** 2
    rng = np.random.default_rng(3)
    f = rng.standard_normal(N ** 3)
    assert np.allclose(orc.laplacian(f, dx), L @ f, rtol=0, atol=1e-12)


# --- T12: summation by parts, sum (grad+ f)^2 = - sum f Lap f -----------------
def test_summation_by_parts(orc):
    N, dx = 9, 0.3
    f = np.random.default_rng(4).standard_normal(N ** 3)
    g2 = orc.grad2_sum(f, dx)
    fl = -np.dot(f, orc.laplacian(f, dx))
    assert abs(g2 - fl) <= 1e-13 * abs(g2)


# --- Yoshida weights: consistency and 4th-order conditions ---------------------
def test_yoshida_weights(orc):
    w1, w0 = orc.yoshida4()
    assert abs(2 * w1 + w0 - 1) < 1e-15
    assert abs(2 * w1 ** 3 + w0 ** 3) < 1e-14
    assert abs(w1 - 1.3512071919596578) < 1e-15


def free_model(orc, N, integ, dt=0.05, dx=0.5):
    return orc.ScalarModel(N=N, dx=dx, dt=dt, nfields=1, potential=orc.PHI4, lam=0.0,
                           expansion=orc.NONE, integrator=integ)


# --- T2: exact discrete free-field solution ------------------------------------
@pytest.mark.parametrize("integ", ["LF", "VV2"])
def test_free_field_exact_discrete(orc, integ):
    N, dx, h = 8, 0.5, 0.05
    n = (1, 2, 0)
    m = free_model(orc, N, getattr(orc, integ), h, dx)
    f0 = plane_wave(N, n).reshape(-1)
    st = orc.ScalarState(m, [f0], [np.zeros_like(f0)])
    wl = math.sqrt(lattice_w2(N, dx, n))
    Om = math.acos(1.0 - (wl * h) ** 2 / 2.0) / h      # cos(Om h) = 1 - (w h)^2 / 2
    for k in range(1, 41):
        st.run(1)
        amp = math.cos(k * Om * h)
        assert np.max(np.abs(st.phi[0] - amp * f0)) < 1e-13
    # the discrete frequency tends to the lattice frequency at second order
    assert abs(Om - wl) / wl < (wl * h) ** 2


def test_free_field_vv4_transfer_matrix(orc):
    N, dx, h = 8, 0.5, 0.05
    n = (2, 1, 1)
    m = free_model(orc, N, orc.VV4, h, dx)
    f0 = plane_wave(N, n).reshape(-1)
    st = orc.ScalarState(m, [f0], [0.3 * f0])
    w2 = lattice_w2(N, dx, n)

    def vv2_matrix(s):   # one VV2 map of a harmonic oscillator of frequency^2 w2
        return np.array([[1 - s * s * w2 / 2, s], [-s * w2 * (1 - s * s * w2 / 4), 1 - s * s * w2 / 2]])

    c = 2 ** (1 / 3)
    w1, w0 = 1 / (2 - c), -c / (2 - c)
    M = vv2_matrix(w1 * h) @ vv2_matrix(w0 * h) @ vv2_matrix(w1 * h)
    v = np.array([1.0, 0.3])
    for _ in range(30):
        st.run(1)
        v = M @ v
        assert np.max(np.abs(st.phi[0] - v[0] * f0)) < 1e-13
        assert np.max(np.abs(st.pi[0] - v[1] * f0)) < 1e-13
    # 4th order: the VV4 map approximates exp(h L) to O(h^5) per step
    th = math.sqrt(w2) * h
    exact = np.array([[math.cos(th), math.sin(th) / math.sqrt(w2)], [-math.sqrt(w2) * math.sin(th), math.cos(th)]])
    assert np.max(np.abs(M - exact)) < 10 * th ** 5


# --- higher orders: VV6, VV8, VV10 ------------------------------------------------
@pytest.mark.parametrize("n", [2, 4, 6, 8])
def test_triple_jump_identities(orc, n):
    """x1, x0 raise a symmetric order-n map to order n + 2 exactly when
    2 x1 + x0 = 1 (consistency) and 2 x1^(n+1) + x0^(n+1) = 0 (the order-(n+1)
    error term cancels); closed form x1 = 1/(2 - 2^(1/(n+1)))."""
    x1, x0 = orc.triple_jump(n)
    assert abs(2 * x1 + x0 - 1) < 1e-15
    assert abs(2 * x1 ** (n + 1) + x0 ** (n + 1)) < 1e-13 * abs(x0) ** (n + 1)
    assert abs(x1 - 1 / (2 - 2 ** (1 / (n + 1)))) < 1e-15
    if n == 2:
        assert (x1, x0) == orc.yoshida4()


def vv2_matrix(s, w2):
    """One VV2 map of size s of a harmonic mode of frequency^2 w2."""
    return np.array([[1 - s * s * w2 / 2, s], [-s * w2 * (1 - s * s * w2 / 4), 1 - s * s * w2 / 2]])


def composed_matrix(weights, s, w2):
    """Transfer matrix of the maps of sizes w s in order (the first applied first)."""
    M = np.eye(2)
    for w in weights:
        M = vv2_matrix(w * s, w2) @ M
    return M


@pytest.mark.parametrize("order,stages", [(2, 1), (4, 3), (6, 7), (8, 15), (10, 45)])
def test_vv_stage_weights(orc, order, stages):
    """The published compositions (Yoshida 1990: triple jump, solutions A and
    D; the order-10 triple jump of D): symmetric, consistent (weights add up
    to 1), and of the stated order: on a harmonic mode their product of VV2
    maps matches the exact rotation with a local error that falls by
    2^(order+1) when the step halves (the order conditions of the linear
    problem, checked from the weights alone)."""
    w = orc.vv_stages(order)
    assert len(w) == stages
    assert np.array_equal(w, w[::-1])
    assert abs(np.sum(w) - 1.0) < 1e-14
    if order == 4:
        assert np.allclose(w, [orc.yoshida4()[0], orc.yoshida4()[1], orc.yoshida4()[0]], rtol=0, atol=0)
    if order >= 4:
        # odd power sums vanish up to the order (the linear order conditions)
        for k in range(3, order, 2):
            assert abs(np.sum(w ** k)) < 1e-12 * np.sum(np.abs(w) ** k), (k, np.sum(w ** k))

    def err(th):
        exact = np.array([[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]])
        return np.max(np.abs(composed_matrix(w, th, 1.0) - exact))

    th = 0.2 if order < 10 else 0.4
    r = math.log2(err(th) / err(th / 2))
    assert abs(r - (order + 1)) < 0.25, r


@pytest.mark.parametrize("integ,order", [("VV6", 6), ("VV8", 8), ("VV10", 10)])
def test_free_field_high_order_transfer_matrix(orc, integ, order):
    """The oracle's VV6/VV8/VV10 step on a single plane wave equals the product
    of VV2 transfer matrices with its stage weights (pinned above), and that
    product approximates the exact rotation to order h^(order+1) per step."""
    N, dx, h = 8, 0.5, 0.05
    n = (2, 1, 1)
    m = free_model(orc, N, getattr(orc, integ), h, dx)
    f0 = plane_wave(N, n).reshape(-1)
    st = orc.ScalarState(m, [f0], [0.3 * f0])
    w2 = lattice_w2(N, dx, n)
    weights = orc.vv_stages(order)
    M = composed_matrix(weights, h, w2)
    v = np.array([1.0, 0.3])
    for _ in range(20):
        st.run(1)
        v = M @ v
        assert np.max(np.abs(st.phi[0] - v[0] * f0)) < 1e-13
        assert np.max(np.abs(st.pi[0] - v[1] * f0)) < 1e-13
    # local error against exp(h L): halving the step divides it by ~2^(order+1)
    def err(th):
        exact = np.array([[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]])
        return np.max(np.abs(composed_matrix(weights, th, 1.0) - exact))
    th = 0.2 if order < 10 else 0.4   # asymptotic, errors still above roundoff
    r = math.log2(err(th) / err(th / 2))
    assert abs(r - (order + 1)) < 0.25, r


def rand_state(orc, m, seed=11, amp=0.05):
    rng = np.random.default_rng(seed)
    V = m.N ** 3
    phi = [1.0 + amp * rng.standard_normal(V)]
    pi = [amp * rng.standard_normal(V)]
    if m.nfields == 2:
        phi.append(amp * rng.standard_normal(V))
        pi.append(amp * rng.standard_normal(V))
    return phi, pi


def two_field_model(orc, N, integ, exp_, dt=0.01, dx=0.4):
    return orc.ScalarModel(N=N, dx=dx, dt=dt, nfields=2, potential=orc.PHI4_CHI2, lam=1.0, q=100.0,
                           expansion=exp_, integrator=integ, alpha=1.0, kappa2=0.25, w_eos=1 / 3,
                           H0=0.1443, a0=1.0)


# --- T3: time reversibility -----------------------------------------------------
@pytest.mark.parametrize("integ", ["VV2", "VV4"])
@pytest.mark.parametrize("exp_", ["NONE", "FIXED", "SELF"])
def test_reversibility_vv(orc, integ, exp_):
    m = two_field_model(orc, 6, getattr(orc, integ), getattr(orc, exp_))
    phi, pi = rand_state(orc, m)
    st = orc.ScalarState(m, phi, pi)
    a0, b0 = st.a, st.b
    st.run(25).run(-25)
    for s in range(2):
        assert np.max(np.abs(st.phi[s] - phi[s])) <= 1e-13 * np.max(np.abs(phi[s])) + 1e-14
        assert np.max(np.abs(st.pi[s] - pi[s])) <= 1e-12 * np.max(np.abs(pi[s])) + 1e-14
    assert abs(st.a - a0) < 1e-14 and abs(st.b - b0) < 1e-14 and abs(st.t) < 1e-14


@pytest.mark.parametrize("exp_", ["NONE", "FIXED"])
def test_reversibility_lf(orc, exp_):
    m = two_field_model(orc, 6, orc.LF, getattr(orc, exp_))
    phi, pi = rand_state(orc, m)
    st = orc.ScalarState(m, phi, pi)
    st.run(25).sync().run(-25).sync()
    for s in range(2):
        assert np.max(np.abs(st.phi[s] - phi[s])) <= 1e-13
        assert np.max(np.abs(st.pi[s] - pi[s])) <= 1e-12 * np.max(np.abs(pi[s]))


def test_lf_rejects_wrong_direction(orc):
    m = two_field_model(orc, 4, orc.LF, orc.NONE)
    phi, pi = rand_state(orc, m)
    st = orc.ScalarState(m, phi, pi).run(2)
    with pytest.raises(RuntimeError):
        st.run(-1)


# --- T4: convergence order under dt halving ------------------------------------
@pytest.mark.parametrize("integ,exp_,p", [("LF", "FIXED", 2), ("VV2", "SELF", 2), ("VV4", "SELF", 4),
                                          ("VV2", "FIXED", 2), ("VV4", "NONE", 4), ("LF", "SELF", 2)])
def test_convergence_order(orc, integ, exp_, p):
    T = 0.8
    res = []
    for h in (0.04, 0.02, 0.01, 0.005):
        m = two_field_model(orc, 4, getattr(orc, integ), getattr(orc, exp_), dt=h, dx=0.5)
        m.q = 20.0
        phi, pi = rand_state(orc, m, amp=0.2)
        st = orc.ScalarState(m, phi, pi)
        st.run(int(round(T / h)))
        if integ == "LF":
            st.sync()
        res.append(np.concatenate([st.phi[0], st.phi[1], st.pi[0], st.pi[1], [st.a]]))
    e1 = np.max(np.abs(res[0] - res[1]))
    e2 = np.max(np.abs(res[1] - res[2]))
    e3 = np.max(np.abs(res[2] - res[3]))
    for r in (e1 / e2, e2 / e3):
        assert abs(math.log2(r) - p) < 0.15, (e1, e2, e3)


@pytest.mark.parametrize("integ,exp_,hs,p", [
    ("VV6", "SELF", (0.04, 0.02, 0.01, 0.005), 6), ("VV6", "NONE", (0.04, 0.02, 0.01, 0.005), 6),
    ("VV8", "SELF", (0.04, 0.02, 0.01, 0.005), 8), ("VV10", "SELF", (0.08, 0.04, 0.02, 0.01), 10),
    ("VV10", "FIXED", (0.08, 0.04, 0.02, 0.01), 10)])
def test_convergence_order_high(orc, integ, exp_, hs, p):
    """VV6/VV8/VV10 on the nonlinear two-field system (with the scale factor
    where expanding): the error under dt halving falls as h^p on the smallest
    steps (the larger ones are not yet asymptotic for VV8)."""
    T = 0.8
    res = []
    for h in hs:
        m = two_field_model(orc, 4, getattr(orc, integ), getattr(orc, exp_), dt=h, dx=0.5)
        m.q = 20.0
        phi, pi = rand_state(orc, m, amp=0.2)
        st = orc.ScalarState(m, phi, pi)
        st.run(int(round(T / h)))
        res.append(np.concatenate([st.phi[0], st.phi[1], st.pi[0], st.pi[1], [st.a]]))
    es = [np.max(np.abs(res[i] - res[i + 1])) for i in range(len(res) - 1)]
    assert es[0] > es[1] > es[2]
    assert abs(math.log2(es[1] / es[2]) - p) < 0.15, es


# --- T9: homogeneous limit = Jacobi cn ------------------------------------------
@pytest.mark.parametrize("integ,tol", [("VV4", 1e-7), ("VV2", 2e-4), ("LF", 2e-4)])
def test_homogeneous_cn(orc, integ, tol):
    N, h, phi0 = 4, 0.01, 1.3
    m = orc.ScalarModel(N=N, dx=0.5, dt=h, nfields=1, potential=orc.PHI4, lam=1.0,
                        expansion=orc.NONE, integrator=getattr(orc, integ))
    st = orc.ScalarState(m, [np.full(N ** 3, phi0)], [np.zeros(N ** 3)])
    period = 4 * ellipk(0.5) / phi0
    assert abs(period * phi0 - 7.416298709205487) < 1e-12
    nsteps = int(period / h)
    for chunk in range(4):
        st.run(nsteps // 4)
        t = (chunk + 1) * (nsteps // 4) * h
        sn, cn, dn, _ = ellipj(phi0 * t, 0.5)
        assert np.max(np.abs(st.phi[0] - phi0 * cn)) < tol
        if integ != "LF":
            assert np.max(np.abs(st.pi[0] + phi0 ** 2 * sn * dn)) < 4 * tol


# --- T8: energy conservation without expansion, error ~ h^p ---------------------
@pytest.mark.parametrize("integ,p", [("VV2", 2), ("VV4", 4), ("LF", 2)])
def test_energy_conservation_order(orc, integ, p):
    errs = []
    for h in (0.02, 0.01):
        m = two_field_model(orc, 6, getattr(orc, integ), orc.NONE, dt=h, dx=0.5)
        m.q = 20.0
        phi, pi = rand_state(orc, m, amp=0.2)
        st = orc.ScalarState(m, phi, pi)
        rho0 = st.energy()["rho"]
        worst = 0.0
        for _ in range(10):
            st.run(int(round(0.1 / h)))
            worst = max(worst, abs(1 - st.energy()["rho"] / rho0))
        errs.append(worst)
    assert errs[0] < 1e-2 and errs[1] < errs[0]
    assert abs(math.log2(errs[0] / errs[1]) - p) < 0.3, errs


def test_lf_energy_uses_synced_momenta(orc):
    m = two_field_model(orc, 5, orc.LF, orc.FIXED)
    phi, pi = rand_state(orc, m)
    st = orc.ScalarState(m, phi, pi).run(7)
    e_stag = st.energy()
    pis = [p.copy() for p in st.pi]
    st.sync()
    e_sync = st.energy()
    assert st.clock.lf_stag == 0
    assert abs(e_stag["rho"] - e_sync["rho"]) <= 1e-15 * abs(e_sync["rho"])
    assert max(np.max(np.abs(a - b)) for a, b in zip(pis, st.pi)) > 0


# --- T10: fixed background a(eta) closed form for radiation with alpha = 1 ------
def test_fixed_background_radiation(orc):
    H = 0.14433756729740643
    m = orc.ScalarModel(N=4, dx=0.5, dt=0.01, expansion=orc.FIXED, integrator=orc.LF,
                        alpha=1.0, w_eos=1.0 / 3.0, H0=H)
    for t in (0.0, 0.5, 3.0, 10.0):
        a, b = orc.fixed_background(m, t)
        assert abs(a - (1 + H * t)) < 1e-14 * a and abs(b - H) < 1e-15
    # matter domination, cosmic time alpha = 0: a ~ (1 + 3/2 H t)^(2/3)  (eq. aFixed)
    m2 = orc.ScalarModel(N=4, dx=0.5, dt=0.01, expansion=orc.FIXED, alpha=0.0, w_eos=0.0, H0=0.7)
    a, b = orc.fixed_background(m2, 2.0)
    assert abs(a - (1 + 1.5 * 0.7 * 2.0) ** (2 / 3)) < 1e-14
    # the state follows the closed form step by step
    f = [np.full(64, 1.0)]
    st = orc.ScalarState(m, f, [np.zeros(64)])
    for k in range(1, 6):
        st.run(3)
        assert abs(st.a - (1 + H * 0.03 * k)) < 1e-14 and abs(st.t - 0.03 * k) < 1e-15


# --- T11: Hubble constraint: zero at start, violation shrinks as h^p ------------
@pytest.mark.parametrize("integ,p", [("VV2", 2), ("VV4", 4), ("LF", 2)])
def test_hubble_constraint(orc, integ, p):
    res = []
    for h in (0.04, 0.02):
        m = two_field_model(orc, 4, getattr(orc, integ), orc.SELF, dt=h, dx=0.5)
        m.q = 20.0
        m.kappa2 = 1.0
        phi, pi = rand_state(orc, m, amp=0.2)
        st = orc.ScalarState(m, phi, pi)
        assert abs(st.energy()["hubble_res"]) < 1e-15
        worst = 0.0
        for _ in range(8):
            st.run(int(round(0.2 / h)))
            worst = max(worst, abs(st.energy()["hubble_res"]))
        assert st.a > 1.05
        res.append(worst)
    assert abs(math.log2(res[0] / res[1]) - p) < 0.35, res


# --- T7: kernel is minus the derivative of the field energy -----------------------
def test_kernel_is_energy_gradient(orc):
    N, dx, a, al = 4, 0.45, 1.3, 1.0
    m = orc.ScalarModel(N=N, dx=dx, dt=0.01, nfields=2, potential=orc.PHI4_CHI2, lam=0.8, q=7.0,
                        expansion=orc.SELF, alpha=al)
    phi, pi = rand_state(orc, m, amp=0.3)

    def H(ph):   # potential part of the Hamiltonian, a^{1+al} grad energy + a^{3+al} potential
        st = orc.ScalarState(m, ph, pi, a=a, b=0.0)
        e = st.energy()
        V = N ** 3
        return a ** (1 + al) * (e["EG"].sum() * 2 * a * a) * V / 2 + a ** (3 + al) * e["EV"].sum() * V

    for s in range(2):
        K = orc.kernel(m, a, phi, s)
        for site in (0, 17, 40, 63):
            eps = 1e-5
            pp = [f.copy() for f in phi]
            pm = [f.copy() for f in phi]
            pp[s][site] += eps
            pm[s][site] -= eps
            fd = -(H(pp) - H(pm)) / (2 * eps)
            assert abs(fd - K[site]) < 1e-7 * max(1.0, abs(K[site]))
