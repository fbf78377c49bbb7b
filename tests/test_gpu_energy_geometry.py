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
