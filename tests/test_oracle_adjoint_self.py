"""Pins of the oracle's adjoint of velocity-Verlet with the self-consistent
expansion (reading R1): the gradient with respect to the initial fields,
momenta, coupling q, scale factor a0 and its derivative b0 (taken as an
independent input) against central differences of the oracle's own integrator
along random directions of all seven inputs, for both observables and two
values of alpha."""
import numpy as np
import pytest


def model(orc, N=5, dt=0.02, q=30.0, alpha=1.0):
    return orc.ScalarModel(N=N, dx=0.4, dt=dt, nfields=2, potential=orc.PHI4_CHI2, lam=1.0, q=q, alpha=alpha,
                           kappa2=4.0, expansion=orc.SELF, integrator=orc.VV2)


def state(N, seed):
    rng = np.random.default_rng(seed)
    V = N ** 3
    phi = [1.0 + 0.1 * rng.standard_normal(V), 0.05 * rng.standard_normal(V)]
    pi = [0.1 * rng.standard_normal(V), 0.05 * rng.standard_normal(V)]
    return phi, pi


CASES = [(1, 1.0, "fraction", 1, 0), (10, 0.5, "fraction", 0, 0), (12, 1.0, "bin", 1, 2), (6, 0.5, "bin", 0, 1)]


@pytest.mark.parametrize("nsteps,alpha,obs,field,b", CASES)
def test_self_consistent_reverse_sweep_vs_finite_differences(orc, nsteps, alpha, obs, field, b):
    N = 5
    m = model(orc, N, alpha=alpha)
    phi, pi = state(N, 31)
    a0 = 1.0
    b0 = orc.hubble_b0(m, phi, pi, a0)
    kind = orc.OBS_SPECTRUM_BIN if obs == "bin" else orc.OBS_ENERGY_FRACTION
    kw = dict(kind=kind, field=field, bin=b)
    O, g, gp, dq, da0, db0 = orc.adjoint_vv2_self(m, phi, pi, a0, b0, nsteps, **kw)

    def O_of(phi_, pi_, q_, a_, b_):
        mm = model(orc, N, q=q_, alpha=alpha)
        st = orc.ScalarState(mm, phi_, pi_, a=a_, b=b_).run(nsteps)
        return orc.observable(mm, st.phi, st.pi, a=st.a, **kw)

    O_ref = O_of(phi, pi, m.q, a0, b0)
    assert abs(O - O_ref) <= 1e-14 * abs(O)
    # the background really moves over the run
    st = orc.ScalarState(m, phi, pi, a=a0, b=b0).run(nsteps)
    assert st.a > 1.0 + 0.5 * nsteps * m.dt * b0
    rng = np.random.default_rng(41)
    scale = np.sqrt(sum(np.dot(x, x) for x in g + gp) + dq * dq + da0 * da0 + db0 * db0)
    for _ in range(3):
        v = [rng.standard_normal(N ** 3) for _ in range(4)]
        w = rng.standard_normal(3)
        nrm = np.sqrt(sum(np.dot(x, x) for x in v) + np.dot(w, w))
        v = [x / nrm for x in v]
        w = w / nrm
        eps = 1e-5

        def at(sg):
            return O_of([phi[0] + sg * eps * v[0], phi[1] + sg * eps * v[1]],
                        [pi[0] + sg * eps * v[2], pi[1] + sg * eps * v[3]],
                        m.q + sg * eps * w[0], a0 + sg * eps * w[1], b0 + sg * eps * w[2])

        fd = (at(1) - at(-1)) / (2 * eps)
        ad = (np.dot(g[0], v[0]) + np.dot(g[1], v[1]) + np.dot(gp[0], v[2]) + np.dot(gp[1], v[3])
              + dq * w[0] + da0 * w[1] + db0 * w[2])
        assert abs(fd - ad) <= 1e-6 * scale, (fd, ad, scale)


def test_self_consistent_scalar_sensitivities(orc):
    """The a0 and b0 sensitivities alone (the directions the field tests mix
    in), each against its own central difference."""
    N, nsteps = 4, 8
    m = model(orc, N)
    phi, pi = state(N, 33)
    a0, b0 = 1.1, 0.4
    O, g, gp, dq, da0, db0 = orc.adjoint_vv2_self(m, phi, pi, a0, b0, nsteps, field=1)

    def O_of(a_, b_):
        st = orc.ScalarState(m, phi, pi, a=a_, b=b_).run(nsteps)
        return orc.observable(m, st.phi, st.pi, a=st.a, field=1)

    eps = 1e-6
    fa = (O_of(a0 + eps, b0) - O_of(a0 - eps, b0)) / (2 * eps)
    fb = (O_of(a0, b0 + eps) - O_of(a0, b0 - eps)) / (2 * eps)
    assert abs(fa - da0) <= 1e-6 * abs(da0)
    assert abs(fb - db0) <= 1e-6 * abs(db0)
