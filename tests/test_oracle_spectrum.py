"""Pins of the oracle's power spectrum (eq. discretePS): the exact sum rule of
eq. discretePSII, a single plane wave, mode counts, and the raw DFT powers
against numpy's FFT (an independent transform)."""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("N,dx", [(8, 0.5), (9, 0.3), (12, 1.0)])
def test_sum_rule(N, dx):
    """sum_{b>=1} (k_IR / k_b) Delta(b) = <f^2> - <f>^2 (eq. discretePSII)."""
    rng = np.random.default_rng(N)
    f = 2.0 + rng.standard_normal(N ** 3)
    s, d, c = oracle.spectrum(f, dx)
    kir = 2 * math.pi / (N * dx)
    lhs = sum(kir / (b * kir) * d[b] for b in range(1, len(d)))
    rhs = np.mean(f * f) - np.mean(f) ** 2
    assert abs(lhs - rhs) <= 1e-13 * rhs
    assert abs(s[0] - f.sum() ** 2) <= 1e-13 * f.sum() ** 2      # zero mode: |sum f|^2
    assert c.sum() == N ** 3 and c[0] == 1


def test_plane_wave_single_bin():
    """cos(2 pi n.x / N) with n = (1, 2, 0): the two modes +-n carry (N^3/2)^2
    each and fall in bin floor(sqrt(5)) = 2; every other bin is empty."""
    N, dx = 10, 0.5
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    f = np.cos(2 * np.pi * (1 * x + 2 * y + 0 * z) / N).reshape(-1)
    s, d, c = oracle.spectrum(f, dx)
    assert abs(s[2] - 2 * (N ** 3 / 2) ** 2) <= 1e-12 * s[2]
    others = np.delete(s, 2)
    assert np.max(others) <= 1e-20 * s[2]


def test_mode_counts():
    """Bin 1 holds the modes with |n|^2 in {1, 2, 3}: 6 + 12 + 8 = 26."""
    s, d, c = oracle.spectrum(np.zeros(16 ** 3), 1.0)
    assert c[0] == 1 and c[1] == 26
    assert c.sum() == 16 ** 3


@pytest.mark.parametrize("N", [6, 7, 16])
def test_against_numpy_fft(N):
    """Per-bin sums of |f~|^2 equal those of numpy's FFT binned with numpy."""
    rng = np.random.default_rng(3)
    f = rng.standard_normal(N ** 3)
    s, d, c = oracle.spectrum(f, 0.7)
    F = np.fft.fftn(f.reshape(N, N, N))          # axes (z, y, x)
    k = np.fft.fftfreq(N) * N                    # 0, 1, ..., -1
    k = np.where(k > N / 2, k - N, k)
    k = np.where(k == -N / 2, N / 2, k)          # n in (-N/2, N/2]
    nz, ny, nx = np.meshgrid(k, k, k, indexing="ij")
    m = (nx ** 2 + ny ** 2 + nz ** 2).astype(np.int64)
    b = np.floor(np.sqrt(m)).astype(np.int64)
    b = np.where((b + 1) ** 2 <= m, b + 1, b)
    ref = np.bincount(b.reshape(-1), weights=(np.abs(F) ** 2).reshape(-1), minlength=len(s))
    assert np.max(np.abs(ref[:len(s)] - s)) <= 1e-11 * np.max(ref)
    assert np.array_equal(np.bincount(b.reshape(-1), minlength=len(s))[:len(s)], c)
