"""GPU power spectra (eq. discretePS, lattice_spectrum) against the oracle's
own-DFT spectrum on the same evolved states, and the sum rule of eq.
discretePSII on the GPU output."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import gpu_scalar, say, scalar_kwargs
from paper_2102_01031_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check_spectrum(sp, f, dx):
    """Bins in max-norm relative to the largest bin (transform rounding scales
    with the largest modes, here the zero mode), the mode counts exactly, and
    the sum rule on the GPU output."""
    s, d, c = oracle.spectrum(f, dx, nbins=len(sp["sum"]))
    assert np.array_equal(sp["count"], c)
    rel = np.max(np.abs(sp["sum"] - s)) / s.max()
    assert rel <= 1e-12, rel
    N = round(len(f) ** (1 / 3))
    kir = 2 * math.pi / (N * dx)
    lhs = sum(kir / (b * kir) * sp["delta"][b] for b in range(1, len(sp["delta"])))
    rhs = np.mean(f * f) - np.mean(f) ** 2
    assert abs(lhs - rhs) <= 1e-10 * rhs, (lhs, rhs)
    return rel


@pytest.mark.parametrize("N,precision", [(16, "f64"), (24, "f64"), (64, "f64"), (27, "f64"), (32, "f32")])
def test_spectrum_matches_oracle(N, precision):
    """Both fields, phi and pi, after three VV4 steps; float32 fields are widened
    to float64 exactly, so the oracle gets the same values."""
    wl = workloads.PREHEAT_128
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N)
    lat, tp, tq = gpu_scalar(kw, phi, pi, [3], precision=precision)
    for field in (0, 1):
        for arr, t in (("phi", tp), ("pi", tq)):
            sp = lat.spectrum(field, arr)
            f = t[field].double().cpu().numpy()       # the stored array, as the GPU holds it
            rel = check_spectrum(sp, f, kw["dx"])
            say(f"[spectrum] N={N} {precision} field {field} {arr}: max rel diff {rel:.2e}")
    lat.close()


