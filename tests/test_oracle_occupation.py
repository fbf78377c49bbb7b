"""Pins of the oracle's lattice occupation number (eq. OccuppationNum).

A single Fourier mode n with |n| = b an integer (so k = b k_IR exactly) holds
E/omega quanta, E being the continuum energy of that wave in the box of side L.
The shell normalisation of eq. discretePS divides by 4 pi b^2, so
4 pi b^2 n_b = E / omega, for a travelling wave (E = L^3 A^2 omega^2 / 2) and
a standing wave (E = L^3 A^2 omega^2 / 4), with omega^2 = k^2 + a^2 <V''>
from the homogeneous background.  In an expanding background, momenta that
make phi' + (a'/a) phi vanish leave only the field term.

The alpha-time exponent is a choice of clock, not of physics: one physical
state (phi, its cosmic-time rate phi_t, a and H = a_t/a) written in alpha-time
has pi = a^{3-alpha} phi' = a^3 phi_t (phi' = a^alpha phi_t) and
a' = a^{alpha+1} H, and its occupation number must come out the same for every
alpha.  That fixes how the momentum term is weighted by a at alpha != 1."""
import numpy as np
import pytest


def grid(N):
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def model(orc, N, dx, lam=0.0, q=0.0, nfields=1, alpha=1.0):
    pot = orc.PHI4_CHI2 if nfields == 2 else orc.PHI4
    return orc.ScalarModel(N=N, dx=dx, dt=0.01, nfields=nfields, potential=pot, lam=lam, q=q, alpha=alpha,
                           expansion=orc.NONE, integrator=orc.VV2)


N, DX, A = 12, 0.5, 0.03
MODE = (0, 2, 0)   # |n| = 2
B = 2


def wave(N, mode):
    x, y, z = grid(N)
    return 2 * np.pi * (mode[0] * x + mode[1] * y + mode[2] * z) / N


def quanta(n, b):
    return 4 * np.pi * b * b * n[b]


def test_travelling_wave_massless(orc):
    m = model(orc, N, DX)
    L = N * DX
    k = B * 2 * np.pi / L
    th = wave(N, MODE)
    for phase in (0.0, 0.7, 2.1):   # the count does not depend on where the wave is in its cycle
        phi = [A * np.cos(th - phase)]
        pi = [A * k * np.sin(th - phase)]
        n, c = orc.occupation(m, 1.0, 0.0, phi, pi, 0)
        assert abs(quanta(n, B) - L ** 3 * A * A * k / 2) <= 1e-12 * L ** 3 * A * A * k
        others = np.delete(n, B)
        assert np.max(np.abs(others)) <= 1e-12 * n[B]
        _, _, cs = orc.spectrum(phi[0], DX)
        assert np.array_equal(c, cs)


def test_standing_wave_and_fstar_scaling(orc):
    m = model(orc, N, DX)
    L = N * DX
    k = B * 2 * np.pi / L
    phi = [A * np.cos(wave(N, MODE))]
    pi = [np.zeros(N ** 3)]
    n, _ = orc.occupation(m, 1.0, 0.0, phi, pi, 0)
    assert abs(quanta(n, B) - L ** 3 * A * A * k / 4) <= 1e-12 * L ** 3 * A * A * k
    n2, _ = orc.occupation(m, 1.0, 0.0, phi, pi, 0, fstar2=3.5)
    assert np.allclose(n2, 3.5 * n, rtol=1e-14, atol=0)


def test_mass_from_the_background(orc):
    # phi4: omega^2 = k^2 + 3 lambda <phi^2>, <phi^2> = phi0^2 + A^2/2
    lam, phi0 = 2.0, 0.8
    m = model(orc, N, DX, lam=lam)
    L = N * DX
    k = B * 2 * np.pi / L
    om = np.sqrt(k * k + 3 * lam * (phi0 ** 2 + A * A / 2))
    th = wave(N, MODE)
    n, _ = orc.occupation(m, 1.0, 0.0, [phi0 + A * np.cos(th)], [A * om * np.sin(th)], 0)
    assert abs(quanta(n, B) - L ** 3 * A * A * om / 2) <= 1e-12 * L ** 3 * A * A * om


@pytest.mark.parametrize("field", [0, 1])
def test_two_field_masses(orc, field):
    # phi^4 + q/2 phi^2 chi^2: omega_phi^2 = k^2 + 3 lam <phi^2> + q <chi^2>,
    # omega_chi^2 = k^2 + q <phi^2>; the other field is homogeneous
    lam, q, phi0, chi0 = 1.5, 40.0, 0.6, 0.05
    m = model(orc, N, DX, lam=lam, q=q, nfields=2)
    L = N * DX
    k = B * 2 * np.pi / L
    th = wave(N, MODE)
    V = N ** 3
    if field == 0:
        om = np.sqrt(k * k + 3 * lam * (phi0 ** 2 + A * A / 2) + q * chi0 ** 2)
        phi = [phi0 + A * np.cos(th), np.full(V, chi0)]
    else:
        om = np.sqrt(k * k + q * phi0 ** 2)
        phi = [np.full(V, phi0), chi0 + A * np.cos(th)]
    pi = [np.zeros(V), np.zeros(V)]
    pi[field] = A * om * np.sin(th)
    n, _ = orc.occupation(m, 1.0, 0.0, phi, pi, field)
    assert abs(quanta(n, B) - L ** 3 * A * A * om / 2) <= 1e-12 * L ** 3 * A * A * om


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_expanding_background_comoving_momentum(orc, alpha):
    # phi' = a^{alpha-3} pi; momenta with phi' = -(a'/a) phi cancel the second
    # term, leaving a^2 L^3 omega A^2 / 4 for a standing wave (omega = k, massless)
    a, bdot = 1.7, 0.3
    m = model(orc, N, DX, alpha=alpha)
    L = N * DX
    k = B * 2 * np.pi / L
    phi = [A * np.cos(wave(N, MODE))]
    pi = [-a ** (3 - alpha) * (bdot / a) * phi[0]]
    n, _ = orc.occupation(m, a, bdot, phi, pi, 0)
    assert abs(quanta(n, B) - a * a * L ** 3 * k * A * A / 4) <= 1e-12 * a * a * L ** 3 * k * A * A
    # with pi = 0 the second term is (a'/a)^2 |phi~|^2 / omega at alpha = 1
    if alpha == 1.0:
        n0, _ = orc.occupation(m, a, bdot, phi, [np.zeros(N ** 3)], 0)
        want = a * a * L ** 3 * A * A / 4 * (k + (bdot / a) ** 2 / k)
        assert abs(quanta(n0, B) - want) <= 1e-12 * want


@pytest.mark.parametrize("alpha", [0.5, 0.0, 1.5])
def test_same_state_any_alpha(orc, alpha):
    # a random field with a random rate, a != 1 and H != 0, so phi_t + H phi
    # is far from zero in every shell; the state is fixed in cosmic time
    rng = np.random.default_rng(11)
    a, H = 1.7, 0.45
    V = N ** 3
    phi = [0.3 + 0.05 * rng.standard_normal(V), 0.02 * rng.standard_normal(V)]
    phi_t = [0.07 * rng.standard_normal(V), 0.03 * rng.standard_normal(V)]
    pi = [a ** 3 * phi_t[0], a ** 3 * phi_t[1]]
    for field in (0, 1):
        ref, cref = orc.occupation(model(orc, N, DX, lam=1.3, q=20.0, nfields=2, alpha=1.0),
                                   a, a ** 2 * H, phi, pi, field)
        got, cgot = orc.occupation(model(orc, N, DX, lam=1.3, q=20.0, nfields=2, alpha=alpha),
                                   a, a ** (alpha + 1) * H, phi, pi, field)
        assert np.array_equal(cref, cgot)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale
        # the momentum term is a sizeable part of n in every filled shell, so a
        # wrong power of a in its weight cannot hide below the tolerance
        zero_rate = [np.zeros(V), np.zeros(V)]
        fld, _ = orc.occupation(model(orc, N, DX, lam=1.3, q=20.0, nfields=2, alpha=alpha),
                                a, 0.0, phi, zero_rate, field)
        filled = cref[1:] > 0
        assert np.all(np.abs(got[1:] - fld[1:])[filled] > 1e-3 * np.abs(got[1:])[filled])


def test_rejects_bad_arguments(orc):
    m = model(orc, 4, DX)
    f = [np.zeros(64)]
    with pytest.raises(RuntimeError):
        orc.occupation(m, 1.0, 0.0, f, f, 1)
    with pytest.raises(RuntimeError):
        orc.occupation(m, 0.0, 0.0, f, f, 0)
