"""The energy pass in its own launch geometry at N = 256 (one plane ahead in
float64, two in float32, 32-plane z chunks): against the float64 oracle on
the workload's initial state, and against the stage passes' geometry
(LATTICE_ENERGY_GEOM=0) on a staggered leapfrog state, where the pass also
applies the sync half kick on the fly."""
import pytest

import oracle
from gpu_util import compare_energy, gpu_scalar, oracle_model, say, scalar_kwargs, tile_env
from paper_2102_01031_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_energy_geometry_256(precision, tol):
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields()
    kw = scalar_kwargs(wl, integrator="lf", expansion="fixed")
    say(f"[energy-geometry] 256^3 {precision}")
    lat, tp, tq = gpu_scalar(kw, phi, pi, [], precision=precision)
    e0 = lat.energy()
    st = oracle.ScalarState(oracle_model(kw), phi, pi, t=kw.get("t0", 0.0))
    compare_energy(e0, st.energy(), tol, "initial state vs oracle")
    lat.step(3)
    e1 = lat.energy()
    lat.close()
    with tile_env("0", "LATTICE_ENERGY_GEOM"):
        ref, rp, rq = gpu_scalar(kw, phi, pi, [3], precision=precision)
        e2 = ref.energy()
        ref.close()
    # the same site terms, summed over other blocks: rounding of the sums only
    compare_energy(e1, e2, 1e-12, "staggered state vs the stage geometry")
    say(f"[energy-geometry]   rho {e1['rho']:.15e} / {e2['rho']:.15e}")


@pytest.mark.parametrize("N,precision,nf", [(256, "f64", 2), (256, "f32", 2), (64, "f64", 2), (24, "f64", 1),
                                            (20, "f32", 2)])
def test_energy_deferred_sums_bitwise(N, precision, nf):
    """lattice_energy sums the pass's block partials in a one-block kernel after
    the pass (the pass's block size, so the same order) instead of in its last
    block: the energies equal, bit for bit, those of the ticketed pass
    (LATTICE_ENERGY_DEFER=0), on the whole-row kernel (N = 256 in the energy
    pass's own geometry, 64) and on tiles (24, 20), on a staggered leapfrog
    state."""
    import numpy as np
    wl = workloads.PREHEAT_256
    if N == 256:
        phi, pi = wl.initial_fields()
    else:
        rng = np.random.default_rng(5 + N)
        phi = [0.3 * rng.standard_normal((N, N, N)) for _ in range(nf)]
        pi = [0.2 * rng.standard_normal((N, N, N)) for _ in range(nf)]
    kw = scalar_kwargs(wl, integrator="lf", expansion="fixed")
    if N != 256:
        kw = dict(kw, N=N)
        if nf == 1:
            kw = dict(kw, potential="phi4")
    es = []
    for spec in (None, "0"):
        with tile_env(spec, "LATTICE_ENERGY_DEFER"):
            say(f"[energy-defer] N={N} {precision} nf={nf} LATTICE_ENERGY_DEFER={spec}")
            lat, tp, tq = gpu_scalar(kw, phi, pi, [3], precision=precision)
            es.append(lat.energy())
            lat.close()
    for k in ("EK", "EG", "EV"):
        assert list(es[0][k]) == list(es[1][k]), (k, es[0][k], es[1][k])
    assert es[0]["rho"] == es[1]["rho"]
