"""Several leapfrog steps per launch for small lattices (stage_slab.hpp):
against the float64 oracle at 1e-12 and against the one-step-per-pass path,
for several steps per launch, planes and rows per block (ragged last slab and
band, step counts that are not a multiple of the steps per launch, the
fall-back when the window does not fit), one and two fields,
no and fixed expansion, float32 (within the float32 budget of the one-step
path), graph replays and direct launches, staggered energies and syncs."""
import pytest

import oracle
from gpu_util import compare_energy, compare_state, gpu_scalar, oracle_model, rel_maxdiff, say, scalar_kwargs, \
    tile_env
from paper_2102_01031_amd import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_both(kw, phi, pi, calls, slab, S, precision="f64"):
    """The slab path (S steps per launch expected) and the one-step path."""
    with tile_env(slab, "LATTICE_SLAB"):
        lat, tp, tq = gpu_scalar(kw, phi, pi, calls, precision=precision)
        n = lat.stats()["launches"]["kick_drift"]
        assert n == sum(-(-c // S) for c in calls), f"slab={slab}: {n} launches for {calls}, S={S} expected"
        e = lat.energy()
        lat.close()
    with tile_env("0", "LATTICE_SLAB"):
        ref, rp, rq = gpu_scalar(kw, phi, pi, calls, precision=precision)
        assert ref.stats()["launches"]["kick_drift"] == sum(calls)
        er = ref.energy()
        ref.close()
    return (tp, tq, e), (rp, rq, er)


@pytest.mark.parametrize("wl_name,N,expansion,slab,S,calls", [
    ("LPHI4_32", 32, "fixed", None, 4, [1000]),       # the full run, default launch shape
    ("LPHI4_32", 32, "fixed", "2,1", 2, [7, 20]),
    ("LPHI4_32", 13, "none", "3,2,3", 3, [11]),       # ragged last slab and band (13 = 6*2 + 1 = 4*3 + 1)
    ("LPHI4_32", 24, "fixed", "4,2,5", 4, [9, 6]),    # 24 = 4*5 + 4
    ("LPHI4_32", 16, "fixed", "2,1,1", 2, [5]),       # one own row per block
    ("LPHI4_32", 11, "fixed", "5,2,8", 4, [13]),      # 2 + 2*5 > 11: falls back to 4 steps, 3 rows
    ("PREHEAT_128", 16, "fixed", "3,1", 3, [10]),     # two fields
    ("PREHEAT_128", 16, "none", "5,1", 5, [12, 1]),   # 6 rows per band: 16 = 6 + 6 + 4
    ("PREHEAT_128", 20, "none", "2,2,16", 2, [5, 3]),
])
def test_slab_matches_oracle_and_single_step_path(wl_name, N, expansion, slab, S, calls):
    wl = getattr(workloads, wl_name)
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N, integrator="lf", expansion=expansion)
    say(f"[slab] {wl_name} N={N} {expansion} slab={slab} calls={calls}")
    (tp, tq, e), (rp, rq, er) = run_both(kw, phi, pi, calls, slab, S)
    st = oracle.ScalarState(oracle_model(kw), phi, pi, t=kw.get("t0", 0.0))
    for n in calls:
        st.run(n)
    err = compare_state(tp, tq, st, TOL, "slab")
    compare_energy(e, st.energy(), TOL, "slab")
    worst = 0.0
    for a, b in zip(tp + tq, rp + rq):
        worst = max(worst, rel_maxdiff(a.cpu().numpy(), b.cpu().numpy()))
    say(f"[slab]   vs oracle {err:.2e}, vs one step per pass {worst:.2e}")
    assert worst <= TOL


@pytest.mark.parametrize("N,slab,S", [(32, None, 4), (16, "3,2", 3)])
def test_slab_float32(N, slab, S):
    """float32 fields: the slab path and the one-step path agree to float32
    rounding, and both stay within the float32 budget against the oracle."""
    wl = workloads.LPHI4_32
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N, integrator="lf", expansion="fixed")
    (tp, tq, e), (rp, rq, er) = run_both(kw, phi, pi, [200], slab, S, precision="f32")
    st = oracle.ScalarState(oracle_model(kw), phi, pi, t=kw.get("t0", 0.0)).run(200)
    for a, b, o in zip(tp + tq, rp + rq, st.phi + st.pi):
        d = rel_maxdiff(a.cpu().double().numpy(), b.cpu().double().numpy())
        eo = rel_maxdiff(a.cpu().double().numpy(), o)
        say(f"[slab-f32] N={N}: vs one step {d:.2e}, vs oracle {eo:.2e}")
        assert d <= 1e-5 and eo <= 1e-4
    assert abs(e["rho"] - er["rho"]) <= 1e-5 * abs(er["rho"])


def test_slab_staggered_sync_and_energy():
    """A staggered leapfrog state: steps through the slab path, the on-the-fly
    synchronised energy, then an explicit sync, against the oracle."""
    wl = workloads.LPHI4_32
    N = 16
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N, integrator="lf", expansion="fixed")
    with tile_env("3,2", "LATTICE_SLAB"):
        lat, tp, tq = gpu_scalar(kw, phi, pi, [8])
        st = oracle.ScalarState(oracle_model(kw), phi, pi, t=kw.get("t0", 0.0)).run(8)
        compare_energy(lat.energy(), st.energy(), TOL, "staggered")
        lat.sync()
        st.sync()
        compare_state(tp, tq, st, TOL, "synced")
        lat.step(4)
        st.run(4)
        compare_state(tp, tq, st, TOL, "after sync")
        lat.close()


def test_slab_graph_replays_match_direct_launches(monkeypatch):
    """Calls of 40 steps (10 launches, captured once and replayed) give bitwise
    the arrays of the same calls launched directly (LATTICE_NO_GRAPH)."""
    import torch
    wl = workloads.LPHI4_32
    phi, pi = wl.initial_fields(N=32)
    kw = scalar_kwargs(wl, N=32, integrator="lf", expansion="fixed")
    with tile_env(None, "LATTICE_SLAB"):
        la, pa, qa = gpu_scalar(kw, phi, pi, [])
        lb, pb, qb = gpu_scalar(kw, phi, pi, [])
    for rep in range(3):
        monkeypatch.delenv("LATTICE_NO_GRAPH", raising=False)
        la.step(40)
        torch.cuda.synchronize()
        monkeypatch.setenv("LATTICE_NO_GRAPH", "1")
        lb.step(40)
        torch.cuda.synchronize()
        for x, y in zip(pa + qa, pb + qb):
            assert torch.equal(x, y), f"call {rep} differs"
    monkeypatch.delenv("LATTICE_NO_GRAPH", raising=False)
    assert la.stats()["launches"]["kick_drift"] == 30
    la.close()
    lb.close()
