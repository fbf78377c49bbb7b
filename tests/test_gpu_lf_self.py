"""GPU parity of the leapfrog with self-consistent expansion (reading A3 of the
oracle: staggered b, E_K of a full kick the mean of the kinetic energies before
and after it) against the oracle, float64 at 1e-12: the tiled kernel (N = 20,
32, one and two fields), the whole-row kernel (N = 64, 128), the energies and
b at integer time measured on a staggered state, the mutating sync, calls of
several lengths (graph capture and replay), a backward run back to the start,
and a staggered start with b0 given; float32 fields within a stated bound."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_energy, compare_state, gpu_scalar, oracle_model, rel_maxdiff, say, scalar_kwargs, to_dev
from paper_2102_01031_amd import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def kw_of(wl, N, **over):
    kw = scalar_kwargs(wl, N=N, integrator="lf", expansion="self", kappa2=4.0)
    kw.update(over)
    return kw


@pytest.mark.parametrize("wl_name,N,calls", [("PREHEAT_128", 20, [9]), ("PREHEAT_128", 32, [10, 10, 3]),
                                             ("LPHI4_32", 32, [12, 12]), ("PREHEAT_128", 64, [5, 11]),
                                             ("PREHEAT_128", 128, [8, 8])])
def test_lf_self_matches_oracle(wl_name, N, calls):
    wl = getattr(workloads, wl_name)
    phi, pi = wl.initial_fields(N=N)
    kw = kw_of(wl, N)
    say(f"[lf-self] {wl_name} N={N} calls={calls}")
    lat, tp, tq = gpu_scalar(kw, phi, pi, [])
    st = oracle.ScalarState(oracle_model(kw), phi, pi)
    e0g, e0o = lat.energy(), st.energy()
    compare_energy(e0g, e0o, TOL, "start")
    for n in calls:
        lat.step(n)
        st.run(n)
        err = compare_state(tp, tq, st, TOL, f"after {n}")
        eg, eo = lat.energy(), st.energy()
        compare_energy(eg, eo, TOL, f"after {n}")
        assert abs(eg["hubble_res"] - eo["hubble_res"]) <= 1e-11
        say(f"[lf-self]   +{n} steps: state {err:.2e}, a={eg['a']:.12f} b={eg['b']:.12e} "
            f"r_H={eg['hubble_res']:.3e} (oracle {eo['hubble_res']:.3e})")
    assert eg["a"] > 1.0 + 1e-4
    lat.sync()
    st.sync()
    compare_state(tp, tq, st, TOL, "synced")
    compare_energy(lat.energy(), st.energy(), TOL, "synced")
    lat.close()


def test_lf_self_sync_cadence_and_reversal():
    """GPU: run(7), sync, run(13) equals the oracle's run(20) (the trajectory
    does not depend on the sync), and a backward run returns to the start."""
    wl = workloads.PREHEAT_128
    N = 24
    phi, pi = wl.initial_fields(N=N)
    kw = kw_of(wl, N)
    lat, tp, tq = gpu_scalar(kw, phi, pi, [7])
    lat.sync()
    lat.step(13)
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(20)
    compare_state(tp, tq, st, TOL, "cadence")
    compare_energy(lat.energy(), st.energy(), TOL, "cadence")
    lat.sync()
    lat.step(-20)
    lat.sync()
    e = lat.energy()
    st0 = oracle.ScalarState(oracle_model(kw), phi, pi)
    for s in range(2):
        assert rel_maxdiff(tp[s].cpu().numpy(), phi[s]) <= 1e-12
        assert rel_maxdiff(tq[s].cpu().numpy(), pi[s]) <= 1e-11
    assert abs(e["a"] - st0.a) <= 1e-14 and abs(e["b"] - st0.b) <= 1e-12 * abs(st0.b)
    lat.close()


def test_lf_self_staggered_start():
    """A resumed run: momenta half a step behind (lf_staggered = 1) with b0 at
    the half step, against the oracle's state with the same phase."""
    wl = workloads.PREHEAT_128
    N = 20
    phi, pi = wl.initial_fields(N=N)
    kw = kw_of(wl, N)
    # make a staggered state with the oracle, then hand it over
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(3)
    phi1 = [f.copy() for f in st.phi]
    pi1 = [f.copy() for f in st.pi]
    kw1 = dict(kw, lf_staggered=1, a0=st.a, b0=st.b, t0=st.t)
    lat, tp, tq = gpu_scalar(kw1, phi1, pi1, [6])
    st.run(6)
    compare_state(tp, tq, st, TOL, "staggered start")
    compare_energy(lat.energy(), st.energy(), TOL, "staggered start")
    lat.close()
    # b0 is required for a staggered start
    from paper_2102_01031_amd.lattice import LatticeError
    with pytest.raises(LatticeError):
        gpu_scalar(dict(kw, lf_staggered=1), phi1, pi1, [])


def test_lf_self_float32_error_is_stated():
    """float32 fields with float64 reductions and scale factor: 40 steps at
    N = 64 against the float64 oracle, relative errors printed and bounded."""
    wl = workloads.PREHEAT_128
    N = 64
    phi, pi = wl.initial_fields(N=N)
    kw = kw_of(wl, N)
    lat, tp, tq = gpu_scalar(kw, phi, pi, [40], precision="f32")
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(40)
    eg, eo = lat.energy(), st.energy()
    ephi = max(rel_maxdiff(tp[s].cpu().numpy(), st.phi[s]) for s in range(2))
    epi = max(rel_maxdiff(tq[s].cpu().numpy(), st.pi[s]) for s in range(2))
    erho = abs(eg["rho"] - eo["rho"]) / abs(eo["rho"])
    ea = abs(eg["a"] - eo["a"]) / eo["a"]
    say(f"[lf-self] float32 N={N} 40 steps: phi {ephi:.2e} pi {epi:.2e} rho {erho:.2e} a {ea:.2e}")
    assert ephi < 1e-5 and epi < 1e-4 and erho < 1e-6 and ea < 1e-9
    lat.close()
