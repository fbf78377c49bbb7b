"""Pins of the seeded initial-condition generator (T14): Hermitian symmetry,
the sum rule of eq. discretePSII for the spectrum of eq. QuantumFlucts2, and
the left/right-mover structure of eq. fpr_influct2."""
import numpy as np
import pytest

from paper_2102_01031_amd import inputs, workloads


def test_real_output_and_zero_mean():
    d, dp, im1, im2 = inputs.gaussian_fluctuations(16, 0.5, 1e-4, 3.0, 0.14, 1)
    assert im1 <= 1e-15 * np.abs(d).max() and im2 <= 1e-15 * np.abs(dp).max()
    assert abs(d.mean()) < 1e-17 and abs(dp.mean()) < 1e-16


def test_expected_variance_value():
    # config of the single-field workload: 32^3, dx = 0.5, P = 1e-4 / sqrt(k^2 + 3)
    v = inputs.expected_variance(32, 0.5, 1e-4, 3.0)
    assert abs(v - 1.386e-4) / 1.386e-4 < 2e-3
    # direct brute-force sum over the reciprocal lattice
    N, dx = 6, 0.7
    kIR = 2 * np.pi / (N * dx)
    s = 0.0
    for a in range(-N // 2 + 1, N // 2 + 1):
        for b in range(-N // 2 + 1, N // 2 + 1):
            for c in range(-N // 2 + 1, N // 2 + 1):
                if a == b == c == 0:
                    continue
                s += 1e-3 / np.sqrt(kIR ** 2 * (a * a + b * b + c * c) + 2.0)
    assert abs(inputs.expected_variance(N, dx, 1e-3, 2.0) - s / (N * dx) ** 3) < 1e-15


@pytest.mark.parametrize("N,dx,m2", [(32, 0.5, 3.0), (24, 0.3, 100.0)])
def test_sum_rule_statistics(N, dx, m2):
    vals = []
    for seed in range(12):
        d, _, _, _ = inputs.gaussian_fluctuations(N, dx, 1e-4, m2, 0.0, 100 + seed)
        vals.append(np.mean(d * d))
    vals = np.array(vals)
    expect = inputs.expected_variance(N, dx, 1e-4, m2)
    sem = vals.std(ddof=1) / np.sqrt(len(vals))
    assert abs(vals.mean() - expect) < 4 * sem + 1e-3 * expect


def test_mode_power_matches_spectrum():
    # E|d(n~)|^2 = (N/dx)^3 amp / w_k  (eq. QuantumFlucts2), checked on shells
    N, dx, amp, m2 = 16, 0.5, 1e-4, 3.0
    acc = np.zeros((N, N, N))
    R = 40
    for seed in range(R):
        d, _, _, _ = inputs.gaussian_fluctuations(N, dx, amp, m2, 0.0, seed)
        acc += np.abs(np.fft.fftn(d)) ** 2
    acc /= R
    k = 2 * np.pi / (N * dx) * inputs.mode_numbers(N)
    sig2 = (N / dx) ** 3 * amp / np.sqrt(k * k + m2)
    ratio = acc / sig2
    ratio[0, 0, 0] = 1.0
    assert abs(ratio.mean() - 1) < 0.02
    assert abs(np.median(ratio) - 1) < 0.1


def test_momentum_is_left_right_movers():
    # with H = 0: E|d'|^2 = w_k^2 E|d|^2 per mode (standing waves of both movers)
    N, dx, amp, m2 = 16, 0.5, 1e-4, 3.0
    P, Pp = np.zeros((N, N, N)), np.zeros((N, N, N))
    for seed in range(40):
        d, dp, _, _ = inputs.gaussian_fluctuations(N, dx, amp, m2, 0.0, seed)
        P += np.abs(np.fft.fftn(d)) ** 2
        Pp += np.abs(np.fft.fftn(dp)) ** 2
    k = 2 * np.pi / (N * dx) * inputs.mode_numbers(N)
    w2 = k * k + m2
    r = (Pp / np.where(P > 0, P, 1)) / w2
    r[0, 0, 0] = 1
    assert abs(np.mean(r) - 1) < 0.05
    # the Hubble term subtracts H d exactly
    d, dp0, _, _ = inputs.gaussian_fluctuations(N, dx, amp, m2, 0.0, 5)
    _, dp1, _, _ = inputs.gaussian_fluctuations(N, dx, amp, m2, 0.3, 5)
    assert np.max(np.abs(dp1 - (dp0 - 0.3 * d))) < 1e-15


def test_workload_fields_and_batch_sizes():
    phi, pi = workloads.LPHI4_32.initial_fields()
    assert phi[0].shape == (32, 32, 32) and abs(phi[0].mean() - 1.0) < 1e-12
    sizes = workloads.BATCH.sizes()
    assert len(sizes) == 256 and set(sizes) <= {24, 32, 48, 64}
    tot = sum(n ** 3 for n in sizes)
    assert 2.0e7 < tot < 3.4e7
    ph, pu, A, pa = workloads.ABELIAN_HIGGS_128.initial_fields(N=8)
    mod = np.sqrt((ph[0] ** 2 + ph[1] ** 2) / 2)
    assert np.max(np.abs(mod - 0.1)) < 1e-15
