"""Pins of the oracle's adjoint of the velocity-Verlet step (two fields, a = 1):
dot-product identity against the tangent-linear step, tangent against central
differences of the nonlinear step, and the full reverse sweep against central
differences of the final observable (energy fraction in chi)."""
import numpy as np
import pytest


def model(orc, N=5, dt=0.01, q=30.0):
    return orc.ScalarModel(N=N, dx=0.4, dt=dt, nfields=2, potential=orc.PHI4_CHI2, lam=1.0, q=q,
                           expansion=orc.NONE, integrator=orc.VV2)


def state(N, seed=21):
    rng = np.random.default_rng(seed)
    V = N ** 3
    phi = [1.0 + 0.1 * rng.standard_normal(V), 0.05 * rng.standard_normal(V)]
    pi = [0.1 * rng.standard_normal(V), 0.05 * rng.standard_normal(V)]
    return phi, pi


def test_dot_product_identity(orc):
    N = 5
    m = model(orc, N)
    phi, pi = state(N)
    rng = np.random.default_rng(1)
    v = [rng.standard_normal(N ** 3) for _ in range(4)]
    dq = 0.37
    w = [rng.standard_normal(N ** 3) for _ in range(4)]
    # tangent: J v
    ph, pp = [f.copy() for f in phi], [f.copy() for f in pi]
    dph, dpp = [v[0].copy(), v[1].copy()], [v[2].copy(), v[3].copy()]
    orc.vv2_tangent(m, ph, pp, dph, dpp, dq)
    lhs = sum(np.dot(a, b) for a, b in zip(dph + dpp, w))
    # adjoint: J^T w
    lph, lpp = [w[0].copy(), w[1].copy()], [w[2].copy(), w[3].copy()]
    gq = orc.vv2_adjoint_step(m, phi, pi, lph, lpp)
    rhs = sum(np.dot(a, b) for a, b in zip(lph + lpp, v)) + dq * gq
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_tangent_matches_central_differences(orc):
    N = 4
    m = model(orc, N)
    phi, pi = state(N, 3)
    rng = np.random.default_rng(2)
    v = [rng.standard_normal(N ** 3) for _ in range(4)]
    dq = 0.5
    ph, pp = [f.copy() for f in phi], [f.copy() for f in pi]
    dph, dpp = [v[0].copy(), v[1].copy()], [v[2].copy(), v[3].copy()]
    orc.vv2_tangent(m, ph, pp, dph, dpp, dq)
    eps = 1e-6

    def step(sign):
        mm = model(orc, N, q=m.q + sign * eps * dq)
        st = orc.ScalarState(mm, [phi[0] + sign * eps * v[0], phi[1] + sign * eps * v[1]],
                             [pi[0] + sign * eps * v[2], pi[1] + sign * eps * v[3]])
        st.run(1)
        return st.phi + st.pi

    fp, fm = step(1), step(-1)
    for a, b, c in zip(fp, fm, dph + dpp):
        fd = (a - b) / (2 * eps)
        assert np.max(np.abs(fd - c)) < 1e-6 * max(1, np.max(np.abs(c)))


def test_observable_gradient_seed(orc):
    N = 4
    m = model(orc, N)
    phi, pi = state(N, 5)
    O, g, gp, dq = orc.observable(m, phi, pi, with_grad=True)
    assert 0 < O < 1
    eps = 1e-6
    for s in range(2):
        for site in (0, 13, 63):
            for arr, grad in ((phi, g), (pi, gp)):
                p_ = [f.copy() for f in arr]; m_ = [f.copy() for f in arr]
                p_[s][site] += eps; m_[s][site] -= eps
                if arr is phi:
                    fd = (orc.observable(m, p_, pi) - orc.observable(m, m_, pi)) / (2 * eps)
                else:
                    fd = (orc.observable(m, phi, p_) - orc.observable(m, phi, m_)) / (2 * eps)
                assert abs(fd - grad[s][site]) < 1e-8 * max(1e-3, abs(fd))
    fd = (orc.observable(model(orc, N, q=m.q + 1e-5), phi, pi)
          - orc.observable(model(orc, N, q=m.q - 1e-5), phi, pi)) / 2e-5
    assert abs(fd - dq) < 1e-7 * max(1e-3, abs(fd))


@pytest.mark.parametrize("nsteps", [1, 7, 30])
def test_reverse_sweep_vs_finite_differences(orc, nsteps):
    N = 5
    m = model(orc, N, dt=0.02)
    phi, pi = state(N, 8)
    O, g, gp, dq = orc.adjoint_vv2(m, phi, pi, nsteps)

    def O_of(phi_, pi_, q_):
        st = orc.ScalarState(model(orc, N, dt=0.02, q=q_), phi_, pi_)
        st.run(nsteps)
        return orc.observable(model(orc, N, dt=0.02, q=q_), st.phi, st.pi)

    assert abs(O - O_of(phi, pi, m.q)) < 1e-14
    rng = np.random.default_rng(7)
    for _ in range(4):
        v = [rng.standard_normal(N ** 3) for _ in range(4)]
        vq = rng.standard_normal()
        nrm = np.sqrt(sum(np.dot(a, a) for a in v) + vq * vq)
        v = [a / nrm for a in v]
        vq /= nrm
        eps = 1e-5
        fp = O_of([phi[0] + eps * v[0], phi[1] + eps * v[1]], [pi[0] + eps * v[2], pi[1] + eps * v[3]], m.q + eps * vq)
        fm = O_of([phi[0] - eps * v[0], phi[1] - eps * v[1]], [pi[0] - eps * v[2], pi[1] - eps * v[3]], m.q - eps * vq)
        fd = (fp - fm) / (2 * eps)
        ad = np.dot(g[0], v[0]) + np.dot(g[1], v[1]) + np.dot(gp[0], v[2]) + np.dot(gp[1], v[3]) + dq * vq
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-12


# Spectrum-bin observable: O = Delta(b) of one field (eq. discretePS).

def test_spectrum_bin_observable_value_and_seed(orc):
    N = 6
    m = model(orc, N)
    phi, pi = state(N, 11)
    for field, b in ((0, 1), (1, 2), (0, 3)):
        O, g, gp, dq = orc.observable(m, phi, pi, with_grad=True, kind=orc.OBS_SPECTRUM_BIN, field=field, bin=b)
        # the value is the same bin of the oracle's (separately pinned) spectrum
        ref = orc.spectrum(phi[field], m.dx, 5)[1][b]
        assert abs(O - ref) <= 1e-13 * abs(ref)
        # only phi of the chosen field enters; no explicit q dependence
        assert dq == 0.0
        assert not np.any(g[1 - field]) and not np.any(gp[0]) and not np.any(gp[1])
        # Delta(b) is a quadratic form in phi: phi . grad = 2 Delta(b) exactly
        assert abs(np.dot(phi[field], g[field]) - 2 * O) <= 1e-12 * abs(O)
        # central differences at sites that are not mirror images of each other
        eps = 1e-5
        for site in (0, 7, 50, 101, 197):
            p_ = [f.copy() for f in phi]; m_ = [f.copy() for f in phi]
            p_[field][site] += eps; m_[field][site] -= eps
            kw = dict(kind=orc.OBS_SPECTRUM_BIN, field=field, bin=b)
            fd = (orc.observable(m, p_, pi, **kw) - orc.observable(m, m_, pi, **kw)) / (2 * eps)
            assert abs(fd - g[field][site]) <= 1e-7 * np.max(np.abs(g[field]))


def test_spectrum_bin_plane_wave_gradient(orc):
    # f = A cos(2 pi n.x / N) with |n| in shell b: the shell holds +n and -n,
    # each with |f~|^2 = (A N^3 / 2)^2, so Delta = 2 c_b (A N^3/2)^2 and the
    # gradient is 2 c_b N^3 f = (4 Delta / (A^2 N^3)) f.
    N, A = 8, 0.7
    m = model(orc, N)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    f = A * np.cos(2 * np.pi * (1 * x + 2 * y + 0 * z) / N).reshape(-1)
    phi = [f, np.zeros(N ** 3)]
    pi = [np.zeros(N ** 3), np.zeros(N ** 3)]
    O, g, gp, dq = orc.observable(m, phi, pi, with_grad=True, kind=orc.OBS_SPECTRUM_BIN, field=0, bin=2)
    kb = 2 * 2 * np.pi / (N * m.dx)
    cb = kb ** 3 / (2 * np.pi ** 2) * (m.dx / N) ** 3 / (4 * np.pi * 4)
    assert abs(O - 2 * cb * (A * N ** 3 / 2) ** 2) <= 1e-12 * O
    assert np.max(np.abs(g[0] - 2 * cb * N ** 3 * f)) <= 1e-12 * np.max(np.abs(g[0]))
    # a neighbouring shell sees nothing
    O1 = orc.observable(m, phi, pi, kind=orc.OBS_SPECTRUM_BIN, field=0, bin=1)
    assert abs(O1) <= 1e-20


@pytest.mark.parametrize("nsteps,field,b", [(1, 0, 1), (7, 1, 2), (30, 0, 2)])
def test_spectrum_bin_reverse_sweep_vs_finite_differences(orc, nsteps, field, b):
    N = 5
    m = model(orc, N, dt=0.02)
    phi, pi = state(N, 9)
    kw = dict(kind=orc.OBS_SPECTRUM_BIN, field=field, bin=b)
    O, g, gp, dq = orc.adjoint_vv2(m, phi, pi, nsteps, **kw)

    def O_of(phi_, pi_, q_):
        st = orc.ScalarState(model(orc, N, dt=0.02, q=q_), phi_, pi_)
        st.run(nsteps)
        return orc.observable(model(orc, N, dt=0.02, q=q_), st.phi, st.pi, **kw)

    assert abs(O - O_of(phi, pi, m.q)) <= 1e-14 * abs(O)
    rng = np.random.default_rng(17)
    for _ in range(3):
        v = [rng.standard_normal(N ** 3) for _ in range(4)]
        vq = rng.standard_normal()
        nrm = np.sqrt(sum(np.dot(a, a) for a in v) + vq * vq)
        v = [a / nrm for a in v]
        vq /= nrm
        eps = 1e-5
        fp = O_of([phi[0] + eps * v[0], phi[1] + eps * v[1]], [pi[0] + eps * v[2], pi[1] + eps * v[3]], m.q + eps * vq)
        fm = O_of([phi[0] - eps * v[0], phi[1] - eps * v[1]], [pi[0] - eps * v[2], pi[1] - eps * v[3]], m.q - eps * vq)
        fd = (fp - fm) / (2 * eps)
        ad = np.dot(g[0], v[0]) + np.dot(g[1], v[1]) + np.dot(gp[0], v[2]) + np.dot(gp[1], v[3]) + dq * vq
        scale = np.sqrt(sum(np.dot(a, a) for a in g + gp) + dq * dq)
        assert abs(fd - ad) <= 1e-6 * scale


def test_spectrum_bin_rejects_bad_selection(orc):
    N = 4
    m = model(orc, N)
    phi, pi = state(N, 2)
    for field, b in ((2, 1), (-1, 1), (0, 0)):
        with pytest.raises(RuntimeError):
            orc.observable(m, phi, pi, kind=orc.OBS_SPECTRUM_BIN, field=field, bin=b)


# Fixed background a(t) (power law, reading R3): kicks at a of the kick time,
# drifts at a of the drift midpoint.

def fixed_model(orc, N=5, dt=0.02, q=30.0, alpha=1.0):
    return orc.ScalarModel(N=N, dx=0.4, dt=dt, nfields=2, potential=orc.PHI4_CHI2, lam=1.0, q=q, alpha=alpha,
                           expansion=orc.FIXED, w_eos=1 / 3, H0=2.0, t0=0.0, a0=1.0, integrator=orc.VV2)


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_fixed_background_dot_product_and_tangent(orc, alpha):
    N, t = 4, 0.3
    m = fixed_model(orc, N, alpha=alpha)
    assert orc.fixed_background(m, t)[0] > 1.3   # the background really moves
    phi, pi = state(N, 4)
    rng = np.random.default_rng(5)
    v = [rng.standard_normal(N ** 3) for _ in range(4)]
    w = [rng.standard_normal(N ** 3) for _ in range(4)]
    dq = 0.4
    ph, pp = [f.copy() for f in phi], [f.copy() for f in pi]
    dph, dpp = [v[0].copy(), v[1].copy()], [v[2].copy(), v[3].copy()]
    orc.vv2_tangent(m, ph, pp, dph, dpp, dq, t=t)
    lhs = sum(np.dot(a, b) for a, b in zip(dph + dpp, w))
    lph, lpp = [w[0].copy(), w[1].copy()], [w[2].copy(), w[3].copy()]
    gq = orc.vv2_adjoint_step(m, phi, pi, lph, lpp, t=t)
    rhs = sum(np.dot(a, b) for a, b in zip(lph + lpp, v)) + dq * gq
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # tangent against central differences of the nonlinear step from time t
    eps = 1e-6

    def step(sign):
        mm = fixed_model(orc, N, q=m.q + sign * eps * dq, alpha=alpha)
        st = orc.ScalarState(mm, [phi[0] + sign * eps * v[0], phi[1] + sign * eps * v[1]],
                             [pi[0] + sign * eps * v[2], pi[1] + sign * eps * v[3]], t=t)
        st.run(1)
        return st.phi + st.pi

    fp, fm = step(1), step(-1)
    for a, b, c in zip(fp, fm, dph + dpp):
        assert np.max(np.abs((a - b) / (2 * eps) - c)) < 1e-6 * max(1, np.max(np.abs(c)))
    # the nonlinear step of the tangent routine is the integrator's own step
    st = orc.ScalarState(m, phi, pi, t=t).run(1)
    for a, b in zip(ph + pp, st.phi + st.pi):
        assert np.array_equal(a, b)


def test_observable_seed_at_scale_factor(orc):
    N, a = 4, 1.6
    m = fixed_model(orc, N)
    phi, pi = state(N, 6)
    O, g, gp, dq = orc.observable(m, phi, pi, with_grad=True, a=a)
    # the value is the chi share of the energies the integrator reports where
    # the background has this scale factor (radiation, H0 = 2: a = 1 + 2t)
    E = orc.ScalarState(m, phi, pi, t=0.3).energy()
    assert abs(E["a"] - a) <= 1e-14
    assert abs(O - (E["EK"][1] + E["EG"][1]) / E["rho"]) <= 1e-14 * O
    eps = 1e-6
    for s in range(2):
        for site in (0, 21, 63):
            for arr, grad in ((phi, g), (pi, gp)):
                p_ = [f.copy() for f in arr]; m_ = [f.copy() for f in arr]
                p_[s][site] += eps; m_[s][site] -= eps
                if arr is phi:
                    fd = (orc.observable(m, p_, pi, a=a) - orc.observable(m, m_, pi, a=a)) / (2 * eps)
                else:
                    fd = (orc.observable(m, phi, p_, a=a) - orc.observable(m, phi, m_, a=a)) / (2 * eps)
                assert abs(fd - grad[s][site]) < 1e-8 * max(1e-3, abs(fd))
    assert O != orc.observable(m, phi, pi, a=1.0)


@pytest.mark.parametrize("kind,alpha", [("chi", 1.0), ("chi", 0.5), ("bin", 1.0)])
def test_fixed_background_reverse_sweep_vs_finite_differences(orc, kind, alpha):
    N, nsteps, t0 = 5, 20, 0.25
    m = fixed_model(orc, N, alpha=alpha)
    phi, pi = state(N, 12)
    kw = dict(kind=orc.OBS_SPECTRUM_BIN, field=1, bin=2) if kind == "bin" else {}
    O, g, gp, dq = orc.adjoint_vv2(m, phi, pi, nsteps, t=t0, **kw)
    aT = orc.fixed_background(m, t0 + nsteps * m.dt)[0]

    def O_of(phi_, pi_, q_):
        mm = fixed_model(orc, N, q=q_, alpha=alpha)
        st = orc.ScalarState(mm, phi_, pi_, t=t0).run(nsteps)
        return orc.observable(mm, st.phi, st.pi, a=aT, **kw)

    assert abs(O - O_of(phi, pi, m.q)) <= 1e-13 * abs(O)
    rng = np.random.default_rng(19)
    for _ in range(3):
        v = [rng.standard_normal(N ** 3) for _ in range(4)]
        vq = rng.standard_normal()
        nrm = np.sqrt(sum(np.dot(a, a) for a in v) + vq * vq)
        v = [a / nrm for a in v]
        vq /= nrm
        eps = 1e-5
        fp = O_of([phi[0] + eps * v[0], phi[1] + eps * v[1]], [pi[0] + eps * v[2], pi[1] + eps * v[3]], m.q + eps * vq)
        fm = O_of([phi[0] - eps * v[0], phi[1] - eps * v[1]], [pi[0] - eps * v[2], pi[1] - eps * v[3]], m.q - eps * vq)
        fd = (fp - fm) / (2 * eps)
        ad = np.dot(g[0], v[0]) + np.dot(g[1], v[1]) + np.dot(gp[0], v[2]) + np.dot(gp[1], v[3]) + dq * vq
        scale = np.sqrt(sum(np.dot(a, a) for a in g + gp) + dq * dq)
        assert abs(fd - ad) <= 1e-6 * scale


def test_energy_fraction_of_phi(orc):
    """Field 0's energy fraction: with chi's it adds to 1 - E_V/rho; its seed
    and reverse sweep against central differences."""
    N = 5
    m = model(orc, N, dt=0.02)
    phi, pi = state(N, 14)
    Ophi, g, gp, dq = orc.observable(m, phi, pi, with_grad=True, field=0)
    Ochi = orc.observable(m, phi, pi, field=1)
    E = orc.ScalarState(m, phi, pi).energy()
    assert abs(Ophi + Ochi - (1 - sum(E["EV"]) / E["rho"])) <= 1e-14
    eps = 1e-6
    for s in range(2):
        for site in (3, 77):
            p_ = [f.copy() for f in phi]; m_ = [f.copy() for f in phi]
            p_[s][site] += eps; m_[s][site] -= eps
            fd = (orc.observable(m, p_, pi, field=0) - orc.observable(m, m_, pi, field=0)) / (2 * eps)
            # O is near 1/2 here: the differences carry ~1e-10 of rounding
            assert abs(fd - g[s][site]) < 1e-7 * max(1e-3, abs(fd))
    nsteps = 7
    O, g, gp, dq = orc.adjoint_vv2(m, phi, pi, nsteps, field=0)

    def O_of(phi_, q_):
        mm = model(orc, N, dt=0.02, q=q_)
        st = orc.ScalarState(mm, phi_, pi).run(nsteps)
        return orc.observable(mm, st.phi, st.pi, field=0)

    assert abs(O - O_of(phi, m.q)) <= 1e-14
    rng = np.random.default_rng(29)
    v = [rng.standard_normal(N ** 3) for _ in range(2)]
    vq = 0.3
    eps = 1e-5
    fd = (O_of([phi[0] + eps * v[0], phi[1] + eps * v[1]], m.q + eps * vq)
          - O_of([phi[0] - eps * v[0], phi[1] - eps * v[1]], m.q - eps * vq)) / (2 * eps)
    ad = np.dot(g[0], v[0]) + np.dot(g[1], v[1]) + dq * vq
    assert abs(fd - ad) <= 1e-6 * abs(ad)
