"""Seeded synthetic initial conditions shared by the HIP path and the oracle.

This module draws random numbers and builds input arrays; it holds none of the
lattice-step arithmetic (no stencil, kick, drift, reduction or scale-factor
update) and imports nothing else from the package.

Scalar fluctuations follow the recipe of sec. 4.5.1 (eqs. fpr_influct,
fpr_influct2 and QuantumFlucts2): in Fourier space each mode is a sum of a
left- and a right-moving wave with Rayleigh amplitudes and uniform phases,

    dphi(n~)  = (r1 e^{i th1} + r2 e^{i th2}) / sqrt(2)
    dphi'(n~) = i w_k (r1 e^{i th1} - r2 e^{i th2}) / sqrt(2) / a^{1-alpha} - H dphi(n~)

with E[r^2] = (N/dx)^3 * amp / w_k, w_k = sqrt(k^2 + a^2 m^2), k = k_IR |n~|.
The amplitude constant ``amp`` stands for (omega_*/f_*)^2 / (2 a^2) of
eq. QuantumFlucts2.  The array is made Hermitian by the pairing
(d(n~) + conj(d(-n~)))/sqrt(2), which keeps E|d|^2 and makes self-conjugate
modes real; the zero mode is removed; the inverse DFT carries the 1/N^3 of
eq. FTdiscrete (numpy's convention, forward sign e^{-i}).
Draw order per field: theta1, theta2, r1, r2, each over the full N^3 array,
from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import numpy as np


def mode_numbers(N: int) -> np.ndarray:
    """|n~| on the (z, y, x) Fourier grid, components in (-N/2, N/2]."""
    f = np.fft.fftfreq(N, d=1.0 / N)            # integers in [-N/2, N/2)
    nz, ny, nx = np.meshgrid(f, f, f, indexing="ij")
    return np.sqrt(nx * nx + ny * ny + nz * nz)


def _hermitian(d: np.ndarray) -> np.ndarray:
    N = d.shape[0]
    neg = (-np.arange(N)) % N
    return (d + np.conj(d[np.ix_(neg, neg, neg)])) / np.sqrt(2.0)


def gaussian_fluctuations(N: int, dx: float, amp: float, mass2: float, H: float, seed: int,
                          a: float = 1.0, alpha: float = 1.0):
    """Real-space (dphi, dphi') of shape (N, N, N), float64, zero mean."""
    rng = np.random.default_rng(seed)
    kIR = 2.0 * np.pi / (N * dx)
    k = kIR * mode_numbers(N)
    w = np.sqrt(k * k + a * a * mass2)
    shape = (N, N, N)
    th1 = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    th2 = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    with np.errstate(divide="ignore"):
        sigma2 = np.where(w > 0, (N / dx) ** 3 * amp / np.where(w > 0, w, 1.0), 0.0)
    scale = np.sqrt(sigma2 / 2.0)                 # Rayleigh scale: E[r^2] = 2 scale^2
    r1 = rng.rayleigh(1.0, size=shape) * scale
    r2 = rng.rayleigh(1.0, size=shape) * scale
    e1 = r1 * np.exp(1j * th1)
    e2 = r2 * np.exp(1j * th2)
    d = (e1 + e2) / np.sqrt(2.0)
    dp = (1j * w / np.sqrt(2.0)) * (e1 - e2) / a ** (1.0 - alpha) - H * d
    d = _hermitian(d)
    dp = _hermitian(dp)
    d[0, 0, 0] = 0.0
    dp[0, 0, 0] = 0.0
    xd = np.fft.ifftn(d)
    xp = np.fft.ifftn(dp)
    return xd.real.copy(), xp.real.copy(), float(np.abs(xd.imag).max()), float(np.abs(xp.imag).max())


def expected_variance(N: int, dx: float, amp: float, mass2: float, a: float = 1.0) -> float:
    """Ensemble mean of the volume average <dphi^2> = L^-3 sum_{n~ != 0} amp / w_k (eq. discretePSII)."""
    kIR = 2.0 * np.pi / (N * dx)
    k = kIR * mode_numbers(N)
    w = np.sqrt(k * k + a * a * mass2)
    m = np.ones_like(w, dtype=bool)
    m[0, 0, 0] = False
    return float(np.sum(amp / w[m]) / (N * dx) ** 3)


def scalar_fields(N: int, dx: float, fields, H: float, a0: float = 1.0, alpha: float = 1.0):
    """fields: iterable of (phi0, amp, mass2, seed).  Returns lists phi, pi of (N,N,N) float64:
    phi = phi0 + dphi, pi = a0^{3-alpha} dphi' (the homogeneous velocity is zero)."""
    phis, pis = [], []
    for (phi0, amp, mass2, seed) in fields:
        d, dp, _, _ = gaussian_fluctuations(N, dx, amp, mass2, H, seed, a0, alpha)
        phis.append(phi0 + d)
        pis.append(a0 ** (3.0 - alpha) * dp)
    return phis, pis


def random_phase_u1(N: int, amplitude: float, seed: int):
    """Complex scalar of modulus ``amplitude`` with a white-noise phase per site, written
    in the real components of eq. ChargedScalars: phi0 = sqrt2 |phi| cos(th), phi1 = sqrt2 |phi| sin(th).
    Momenta, links and electric fields start at zero."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, 2.0 * np.pi, size=(N, N, N))
    r = np.sqrt(2.0) * amplitude
    phi = [r * np.cos(th), r * np.sin(th)]
    z = lambda: np.zeros((N, N, N))
    return phi, [z(), z()], [z(), z(), z()], [z(), z(), z()]


def batch_sizes(n_real: int = 256, seed: int = 2024, choices=(24, 32, 48, 64)) -> list:
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.choice(np.array(choices), size=n_real)]


def random_directions(n: int, N: int, seed: int):
    """n unit vectors in the space of (dphi field of N^3 values, dq)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        v = rng.standard_normal(N ** 3 + 1)
        v /= np.linalg.norm(v)
        out.append((v[:-1].reshape(N, N, N), float(v[-1])))
    return out


def random_direction_su2(N: int, amplitude: float, seed: int):
    """SU(2) doublet of modulus ``amplitude`` with a white-noise direction on the
    3-sphere per site, in the real components of eq. ChargedScalars:
    phi_c = sqrt2 |Phi| r_c with r a uniform unit 4-vector (normalised Gaussian).
    Momenta and electric fields start at zero, links at the identity, so the
    Gauss constraint holds exactly.  Layout: phi[4], pi[4], U[12] (link i,
    quaternion component k at 4 i + k, U = u0 I - i u.sigma), E[9] (3 i + a)."""
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((4, N, N, N))
    r /= np.sqrt((r * r).sum(axis=0))
    phi = [np.sqrt(2.0) * amplitude * r[c] for c in range(4)]
    z = lambda: np.zeros((N, N, N))
    U = []
    for _ in range(3):
        U += [np.ones((N, N, N)), z(), z(), z()]
    return phi, [z() for _ in range(4)], U, [z() for _ in range(9)]


def random_su2_state(N: int, seed: int, phi_amp: float = 0.3, pi_amp: float = 0.2, link_angle: float = 0.6,
                     e_amp: float = 0.3):
    """Generic seeded SU(2) state (no constraint imposed): Gaussian doublet and
    momenta, links exp(-i (theta/2) n.sigma) with theta uniform in [0, link_angle)
    and n a uniform unit axis, Gaussian electric fields."""
    rng = np.random.default_rng(seed)
    shape = (N, N, N)
    phi = [phi_amp * rng.standard_normal(shape) for _ in range(4)]
    pi = [pi_amp * rng.standard_normal(shape) for _ in range(4)]
    U = []
    for _ in range(3):
        th = rng.uniform(0.0, link_angle, size=shape)
        ax = rng.standard_normal((3,) + shape)
        ax /= np.sqrt((ax * ax).sum(axis=0))
        U += [np.cos(0.5 * th)] + [np.sin(0.5 * th) * ax[a] for a in range(3)]
    E = [e_amp * rng.standard_normal(shape) for _ in range(9)]
    return phi, pi, U, E


def _half_space_hermitian(d: np.ndarray) -> np.ndarray:
    """Hermitian array from the draws of one half of Fourier space: mode k keeps
    its draw where its flat index is below that of -k, takes conj(d(-k)) where
    it is above, and its real part where k = -k."""
    N = d.shape[0]
    neg = (-np.arange(N)) % N
    flat = np.arange(N ** 3).reshape(N, N, N)
    nflat = flat[np.ix_(neg, neg, neg)]
    dn = d[np.ix_(neg, neg, neg)]
    return np.where(flat < nflat, d, np.where(flat > nflat, np.conj(dn), d.real + 0j))


def charged_fluctuations(N: int, dx: float, ncomp: int, norm: float, amp: float, mass2: float, seed: int):
    """Charged scalar (ncomp = 2, eq. ChargedScalars' complex field) or doublet
    (ncomp = 4) with homogeneous components phi_n = norm/sqrt2 (so |Phi| = norm
    when ncomp = 4) plus fluctuations of eqs. fpr_influct3 and fpr_influct4 at
    a = 1, no expansion, with the constraints InConstr:1 and InConstr:2 that
    remove the homogeneous charge:
        dphi_n(k)  = r_n (e^{i th_n1} + e^{i th_n2}) / sqrt2,
        dphi'_n(k) = i w_k r_n (e^{i th_n1} - e^{i th_n2}) / sqrt2,
        th_n2 = th_02 + th_n1 - th_01,
    E[r_n^2] = (N/dx)^3 amp / w_k, w_k^2 = k^2 + mass2.  Each mode's momenta are
    then a real multiple of its fields, the same for every component, so the
    charge density has no homogeneous part; the half-space Hermitian
    construction keeps that (a pairwise average of k and -k would not).
    Draw order: th_01, th_02, then r_n for every n, then th_n1 for n >= 1,
    each over the full N^3 array, from numpy.random.default_rng(seed).
    Returns (phi, pi): lists of ncomp real (N, N, N) arrays."""
    rng = np.random.default_rng(seed)
    shape = (N, N, N)
    kIR = 2.0 * np.pi / (N * dx)
    k = kIR * mode_numbers(N)
    w = np.sqrt(k * k + mass2)
    th01 = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    th02 = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    with np.errstate(divide="ignore"):
        sigma2 = np.where(w > 0, (N / dx) ** 3 * amp / np.where(w > 0, w, 1.0), 0.0)
    scale = np.sqrt(sigma2 / 2.0)
    r = [rng.rayleigh(1.0, size=shape) * scale for _ in range(ncomp)]
    th1 = [th01] + [rng.uniform(0.0, 2.0 * np.pi, size=shape) for _ in range(1, ncomp)]
    phi, pi = [], []
    for n in range(ncomp):
        th2 = th02 + th1[n] - th01
        e1, e2 = r[n] * np.exp(1j * th1[n]), r[n] * np.exp(1j * th2)
        d = (e1 + e2) / np.sqrt(2.0)
        dp = (1j * w / np.sqrt(2.0)) * (e1 - e2)
        d[0, 0, 0] = 0.0
        dp[0, 0, 0] = 0.0
        d, dp = _half_space_hermitian(d), _half_space_hermitian(dp)
        phi.append(norm / np.sqrt(2.0) + np.fft.ifftn(d).real)
        pi.append(np.fft.ifftn(dp).real)
    return phi, pi
