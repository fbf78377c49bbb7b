"""Host-side argument checks of the autograd wrapper: they raise before any
context is created, so they run without a GPU."""
import pytest
import torch

from paper_2102_01031_amd.autograd import chi_energy_fraction, spectrum_bin


def test_autograd_argument_checks():
    x = torch.zeros(8, dtype=torch.float64, requires_grad=True)
    kw = dict(N=2, dx=0.3, dt=0.005, nsteps=1)
    # self-consistent expansion needs a' at the start (it is an input of the map)
    with pytest.raises(ValueError):
        chi_energy_fraction(x, x, x, x, 1.0, expansion="self", **kw)
    with pytest.raises(ValueError):
        chi_energy_fraction(x, x, x, x, 1.0, expansion="self", b0=float("nan"), **kw)
    # a fixed background's a0 is a constant of the background
    with pytest.raises(ValueError):
        chi_energy_fraction(x, x, x, x, 1.0, expansion="fixed",
                            a0=torch.tensor(1.0, dtype=torch.float64, requires_grad=True), **kw)
    with pytest.raises(ValueError):
        chi_energy_fraction(x, x, x, x, 1.0, expansion="de Sitter", **kw)
    with pytest.raises(ValueError):
        spectrum_bin(x, x, x, x, 1.0, field=0, bin=1, expansion="", **kw)
