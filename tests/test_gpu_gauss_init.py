"""GPU parity of lattice_gauss_init (Gauss-consistent initial gauge momenta,
sec. 5.5.1) against the oracle's solve on the same seeded charged fluctuations,
the Gauss residual after the init and along the evolution, and its errors."""
import numpy as np
import pytest

import oracle
from gpu_util import rel_maxdiff, say, to_dev
from paper_2102_01031_amd import inputs, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _su2_state(N, seed, norm=0.5):
    wl = workloads.SU2_HIGGS_128
    phi, pi = inputs.charged_fluctuations(N, wl.dx, 4, norm, 2e-2, 0.5, seed)
    z = np.zeros((N, N, N))
    U = []
    for _ in range(3):
        U += [np.ones((N, N, N)), z, z, z]
    return wl, (phi, pi, U, [z] * 9)


def _su2_lattice(wl, N, fields):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    t = [to_dev(f, torch.float64) for f in fields]
    lat = Lattice(doublet=t[0], pi_doublet=t[1], U=t[2], E=t[3], N=N, dx=wl.dx, dt=wl.dt, integrator="lf",
                  expansion="none", potential="su2_higgs", lam=wl.lam, v=wl.v, g=wl.g)
    return lat, t


@pytest.mark.parametrize("N,seed", [(10, 1), (16, 2), (27, 3)])
def test_su2_gauss_init_matches_oracle(N, seed):
    wl, fields = _su2_state(N, seed)
    say(f"[gauss] SU(2) init N={N}")
    lat, t = _su2_lattice(wl, N, fields)
    e0 = lat.energy()
    assert e0["gauss_max"] > 1e-3
    mean = lat.gauss_init()
    st = oracle.SU2State(oracle.SU2Model(N=N, dx=wl.dx, dt=wl.dt, lam=wl.lam, v=wl.v, g=wl.g), *fields)
    omean = st.gauss_init()
    assert np.abs(mean).max() < 1e-14 and np.abs(omean).max() < 1e-14
    worst = max(rel_maxdiff(g.cpu().numpy(), o) for g, o in zip(t[3], st.E))
    say(f"[gauss]   E rel err {worst:.2e}")
    assert worst <= 1e-12
    e = lat.energy()
    scale = max(e["gauss_div_max"], e["gauss_charge_max"])
    assert e["gauss_max"] <= 1e-13 * scale
    lat.step(200)
    e = lat.energy()
    scale = max(e["gauss_div_max"], e["gauss_charge_max"])
    say(f"[gauss]   after 200 steps max|G| / scale = {e['gauss_max'] / scale:.2e}, EG_B {e['EG_B']:.3e}")
    assert e["gauss_max"] <= 1e-12 * scale
    lat.close()


@pytest.mark.parametrize("N,seed", [(12, 4), (20, 5)])
def test_u1_gauss_init_matches_oracle(N, seed):
    import torch
    from paper_2102_01031_amd.lattice import Lattice
    wl = workloads.ABELIAN_HIGGS_128
    phi, pi = inputs.charged_fluctuations(N, wl.dx, 2, 0.5, 2e-2, 0.5, seed)
    rng = np.random.default_rng(seed)
    A = [0.3 * rng.standard_normal((N, N, N)) for _ in range(3)]
    piA = [np.zeros((N, N, N))] * 3
    t = [to_dev(f, torch.float64) for f in (phi, pi, A, piA)]
    say(f"[gauss] U(1) init N={N}")
    lat = Lattice(t[0], t[1], A=t[2], piA=t[3], N=N, dx=wl.dx, dt=wl.dt, integrator="lf", expansion="none",
                  potential="abelian_higgs", lam=wl.lam, v=wl.v, e=wl.e, kappa_g=wl.kappa_g)
    mean = lat.gauss_init()
    st = oracle.U1State(oracle.U1Model(N=N, dx=wl.dx, dt=wl.dt, lam=wl.lam, v=wl.v, e=wl.e, kappa_g=wl.kappa_g),
                        phi, pi, A, piA)
    omean = st.gauss_init()
    assert abs(mean[0]) < 1e-14 and abs(omean[0]) < 1e-14
    worst = max(rel_maxdiff(g.cpu().numpy(), o) for g, o in zip(t[3], st.piA))
    assert worst <= 1e-12
    e = lat.energy()
    assert e["gauss_max"] <= 1e-13 * max(e["gauss_div_max"], e["gauss_charge_max"])
    lat.close()


def test_su2_gauss_init_full_size():
    """128^3: the lattice Gauss law holds after the init (a property at any size)."""
    import time

    import torch
    N = 128
    wl, fields = _su2_state(N, 6)
    lat, t = _su2_lattice(wl, N, fields)
    lat.gauss_init()
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    mean = lat.gauss_init()
    ms = 1e3 * (time.perf_counter() - c0)
    e = lat.energy()
    scale = max(e["gauss_div_max"], e["gauss_charge_max"])
    say(f"[gauss] 128^3 init {ms:.2f} ms, mean charge {np.abs(mean).max():.1e}, max|G| / scale {e['gauss_max'] / scale:.1e}")
    assert e["gauss_max"] <= 1e-12 * scale
    lat.close()


def test_gauss_init_errors():
    import torch
    from paper_2102_01031_amd.lattice import Lattice, LatticeError
    N = 8
    wl, fields = _su2_state(N, 7)
    fields[2][1] = fields[2][1].copy()
    fields[2][1][0, 0, 3] = 1e-3            # one link off the identity
    lat, t = _su2_lattice(wl, N, fields)
    with pytest.raises(LatticeError, match="ESTATE"):
        lat.gauss_init()
    assert max(float(e.abs().max()) for e in t[3]) == 0.0   # nothing written
    lat.close()
    w0 = workloads.LPHI4_32
    phi, pi = w0.initial_fields(N=N)
    l0 = Lattice(to_dev(phi, torch.float64), to_dev(pi, torch.float64), N=N, dx=w0.dx, dt=w0.dt)
    with pytest.raises(LatticeError, match="EINVAL"):
        l0.gauss_init()
    l0.close()
