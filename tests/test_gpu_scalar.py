"""GPU parity of the scalar-sector HIP path against the FP64 oracle on the same
seeded inputs (float64: 1e-12 relative, max-norm per array and per energy).

Sizes span several tiles and ragged tails (forced tile shapes), the workloads'
full sizes in the launch configuration the benchmark times, tiny lattices,
reversibility, determinism and the leapfrog sync semantics."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import (compare_energy, compare_state, gpu_scalar, oracle_model, rel_maxdiff, say,
                      scalar_kwargs, tile_env, to_dev)
from paper_2102_01031_amd import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_01031_amd import lattice
    lattice.lib()


def check_run(kw, phi, pi, steps, tol=TOL, tile=None, what=""):
    say(f"[parity] {what} N={kw['N']} {kw['integrator']} {kw['expansion']} steps={steps} tile={tile}")
    with tile_env(tile):
        lat, tp, tq = gpu_scalar(kw, phi, pi, [steps])
        eg = lat.energy()
    st = oracle.ScalarState(oracle_model(kw), phi, pi, t=kw.get("t0", 0.0)).run(steps)
    err = compare_state(tp, tq, st, tol, what)
    compare_energy(eg, st.energy(), tol, what)
    lat.close()
    return err


def test_lphi4_32_full_run():
    """Single field, fixed radiation background, 1000 leapfrog steps (the full run)."""
    wl = workloads.LPHI4_32
    phi, pi = wl.initial_fields()
    check_run(scalar_kwargs(wl), phi, pi, wl.steps, what="lphi4-32")


@pytest.mark.parametrize("tile", [None, "64,4,5", "32,8,7", "16,16,3", "8,8,11", "64,8,36", "32,8,1"])
def test_preheat_ragged_tiles(tile):
    wl = workloads.PREHEAT_128
    N = 36
    phi, pi = wl.initial_fields(N=N)
    check_run(scalar_kwargs(wl, N=N), phi, pi, 6, tile=tile, what="preheat-36")


@pytest.mark.parametrize("N,tile", [(64, "rows,8,5"), (64, "rows,4,64"), (128, "rows,8,9"), (128, "rows,4,23"),
                                    (64, None), (128, None), (64, "rows,4,1")])
def test_preheat_whole_row_kernel(N, tile):
    """The whole-row kernel (N = 64, 128) with ragged and one-plane z chunks."""
    wl = workloads.PREHEAT_128
    phi, pi = wl.initial_fields(N=N)
    check_run(scalar_kwargs(wl, N=N), phi, pi, 3, tile=tile, what=f"rows-{N}")
    kw = scalar_kwargs(wl, N=N, integrator="lf", expansion="fixed")
    check_run(kw, phi, pi, 4, tile=tile, what=f"rows-lf-{N}")


@pytest.mark.parametrize("integ,expn", [("vv2", "self"), ("vv2", "none"), ("vv2", "fixed"), ("vv4", "fixed"),
                                        ("vv4", "none"), ("lf", "none"), ("lf", "fixed")])
def test_integrator_expansion_matrix(integ, expn):
    wl = workloads.PREHEAT_128
    N = 20
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N, integrator=integ, expansion=expn)
    check_run(kw, phi, pi, 9, what=f"{integ}-{expn}")


@pytest.mark.parametrize("integ,expn,N,steps", [("vv6", "self", 24, 4), ("vv8", "fixed", 20, 2),
                                                ("vv10", "self", 16, 1), ("vv6", "none", 64, 2),
                                                ("vv8", "self", 64, 1)])
def test_higher_order_vv(integ, expn, N, steps):
    """VV6 / VV8 / VV10 (7, 15, 45 kick points per step: Yoshida's solutions
    A and D and the triple jump of D) on the tiled and on the whole-row kernel,
    against the oracle."""
    wl = workloads.PREHEAT_128
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N, integrator=integ, expansion=expn)
    check_run(kw, phi, pi, steps, what=f"{integ}-{expn}-{N}")


def test_preheat_128_full_size():
    wl = workloads.PREHEAT_128
    phi, pi = wl.initial_fields()
    check_run(scalar_kwargs(wl), phi, pi, wl.steps, what="preheat-128")


def test_preheat_256_bench_config():
    """The benchmark workload (256^3, two fields, VV4, self-consistent) in the
    benchmark's launch configuration: five steps (15 stencil passes, in calls of
    two and three steps) against
    the oracle at 1e-12, fields and energies after each call."""
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields()
    kw = scalar_kwargs(wl)
    say("[parity] preheat-256 5 VV4 steps")
    lat, tp, tq = gpu_scalar(kw, phi, pi, [])
    st = oracle.ScalarState(oracle_model(kw), phi, pi)
    for n in (2, 3):
        lat.step(n)
        st.run(n)
        err = compare_state(tp, tq, st, TOL, f"preheat-256 +{n}")
        compare_energy(lat.energy(), st.energy(), TOL, f"preheat-256 +{n}")
        say(f"[parity]   +{n} steps: max rel diff {err:.2e}")
    lat.close()


def test_preheat_256_f32_five_steps_error_is_stated():
    """The same five steps with float32 fields (float64 reductions, a, b, t):
    the error against the float64 oracle is printed and bounded."""
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields()
    kw = scalar_kwargs(wl)
    lat, tp, tq = gpu_scalar(kw, phi, pi, [5], precision="f32")
    eg = lat.energy()
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(5)
    eo = st.energy()
    ephi = max(rel_maxdiff(tp[s].cpu().numpy(), st.phi[s]) for s in range(2))
    epi = max(rel_maxdiff(tq[s].cpu().numpy(), st.pi[s]) for s in range(2))
    erho = abs(eg["rho"] - eo["rho"]) / eo["rho"]
    ea = abs(eg["a"] - eo["a"]) / eo["a"]
    say(f"[fp32] 256^3 5 VV4 steps: phi {ephi:.2e} pi {epi:.2e} rho {erho:.2e} a {ea:.2e}")
    assert ephi < 5e-6 and epi < 5e-4 and erho < 1e-5 and ea < 1e-7
    lat.close()


@pytest.mark.parametrize("tile,pf", [("rows,4,3", "2"), ("rows,4,1", "2"), ("rows,4,5", "3"), ("rows,4,2", "3"),
                                     ("rows,4,64", "3"), ("rows,4,6", "1")])
def test_preheat_256_prefetch_depth_ragged(tile, pf):
    """256^3 float64 on the whole-row kernel with loads PF planes ahead (PF + 1
    rotating register sets, z loop unrolled by PF + 1): z chunks that leave
    every remainder after the unrolled groups, or hold one or two planes."""
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields()
    with tile_env(pf, "LATTICE_ROWS_PF"):
        check_run(scalar_kwargs(wl), phi, pi, 1, tile=tile, what=f"preheat-256-{tile}-pf{pf}")


@pytest.mark.parametrize("tile,pf", [("rows,4,7", "4"), ("rows,4,64", "4"), ("rows,4,6", "3"), ("rows,4,9", "2"),
                                     ("rows,8,5", "2")])
def test_preheat_256_f32_prefetch_depth(tile, pf):
    """float32 fields with 16-byte accesses at each prefetch depth, ragged z
    chunks: the stated float32 bound against the float64 oracle, and the fields
    bitwise equal to one site per lane and access at one plane ahead (leapfrog
    on a fixed background, where no block sum feeds a coefficient)."""
    import torch
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields()
    kw = scalar_kwargs(wl)
    say(f"[parity] f32 256 tile={tile} pf={pf}")
    with tile_env(pf, "LATTICE_ROWS_PF"), tile_env(tile):
        lat, tp, tq = gpu_scalar(kw, phi, pi, [1], precision="f32")
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(1)
    for s in range(2):
        assert rel_maxdiff(tp[s].cpu().numpy(), st.phi[s]) < 2e-6
        assert rel_maxdiff(tq[s].cpu().numpy(), st.pi[s]) < 2e-4
    lat.close()
    kl = scalar_kwargs(wl, integrator="lf", expansion="fixed")
    out = []
    for env in ((pf, "4", tile), ("1", "1", None)):
        with tile_env(env[0], "LATTICE_ROWS_PF"), tile_env(env[1], "LATTICE_ROWS_VW"), tile_env(env[2]):
            lat, tp, tq = gpu_scalar(kl, phi, pi, [2], precision="f32")
        out.append([t.cpu() for t in (*tp, *tq)])
        lat.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("N,vw,tile,prec", [(128, "1", None, "f64"), (128, "2", "rows,8,9", "f64"),
                                             (128, "2", "rows,4,23", "f64"), (256, "1", None, "f64"),
                                             (256, "2", "rows,4,3", "f64"), (256, "2", "rows,8,7", "f64"),
                                             (256, "4", None, "f32"), (256, "4", "rows,4,5", "f32"),
                                             (256, "1", None, "f32")])
def test_row_access_width(N, vw, tile, prec):
    """Whole-row kernel with one site per lane and access (LATTICE_ROWS_VW=1)
    and with 16-byte accesses (two float64 or four float32 sites per lane, the
    default where the row allows them), ragged z chunks, against the oracle:
    1e-12 in float64; float32 fields against the float64 oracle at the
    precision mode's stated bound."""
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N)
    with tile_env(vw, "LATTICE_ROWS_VW"):
        if prec == "f64":
            check_run(kw, phi, pi, 1, tile=tile, what=f"rows-vw{vw}-{N}")
            return
        say(f"[parity] f32 rows-vw{vw}-{N} tile={tile}")
        with tile_env(tile):
            lat, tp, tq = gpu_scalar(kw, phi, pi, [1], precision="f32")
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(1)
    for s in range(2):
        assert rel_maxdiff(tp[s].cpu().numpy(), st.phi[s]) < 2e-6
        assert rel_maxdiff(tq[s].cpu().numpy(), st.pi[s]) < 2e-4
    lat.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_row_access_width_bitwise(prec):
    """Each site's arithmetic is the same expression in either access width, so
    without self-consistent expansion (whose coefficients depend on the order of
    the block sums) the fields after leapfrog steps are bitwise equal."""
    import torch
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields()
    kw = scalar_kwargs(wl, integrator="lf", expansion="fixed")
    out = []
    for vw in ("1", "2" if prec == "f64" else "4"):
        say(f"[bitwise] 256 {prec} LATTICE_ROWS_VW={vw}")
        with tile_env(vw, "LATTICE_ROWS_VW"):
            lat, tp, tq = gpu_scalar(kw, phi, pi, [3], precision=prec)
        out.append([t.cpu() for t in (*tp, *tq)])
        lat.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("N,tile", [(256, None), (256, "rows,4,32"), (256, "rows,4,7"), (128, "rows,8,5"),
                                    (64, "rows,4,3")])
def test_row_block_order(N, tile):
    """Whole-row kernel with the y tile as the fastest block index
    (LATTICE_ROWS_YFAST=1: each XCD's blocks form a slab of whole z planes), on
    ragged z chunks: VV4 with self-consistent expansion against the oracle, and
    leapfrog on a fixed background bitwise equal to the default block order."""
    import torch
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields(N=N)
    with tile_env("1", "LATTICE_ROWS_YFAST"):
        check_run(scalar_kwargs(wl, N=N), phi, pi, 1, tile=tile, what=f"rows-yfast-{N}")
    kw = scalar_kwargs(wl, N=N, integrator="lf", expansion="fixed")
    out = []
    for yf in ("0", "1"):
        with tile_env("1" if yf == "1" else "0", "LATTICE_ROWS_YFAST"), tile_env(tile):
            lat, tp, tq = gpu_scalar(kw, phi, pi, [3])
        out.append([t.cpu() for t in (*tp, *tq)])
        lat.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_tiny_lattices(N):
    wl = workloads.PREHEAT_128
    phi, pi = wl.initial_fields(N=N)
    for integ, expn in (("vv4", "self"), ("lf", "fixed")):
        check_run(scalar_kwargs(wl, N=N, integrator=integ, expansion=expn), phi, pi, 5, what=f"tiny-{N}")


def test_single_field_vv_self():
    wl = workloads.LPHI4_32
    phi, pi = wl.initial_fields(N=24)
    kw = scalar_kwargs(wl, N=24, integrator="vv4", expansion="self")
    check_run(kw, phi, pi, 10, what="lphi4-vv4-self")


def test_reversibility_on_gpu():
    import torch
    wl = workloads.PREHEAT_128
    N = 32
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N)
    lat, tp, tq = gpu_scalar(kw, phi, pi, [15, -15])
    e = lat.energy()
    for s in range(2):
        assert rel_maxdiff(tp[s].cpu().numpy(), phi[s]) < 1e-12
        assert rel_maxdiff(tq[s].cpu().numpy(), pi[s]) < 1e-11
    st0 = oracle.ScalarState(oracle_model(kw), phi, pi)
    assert abs(e["a"] - 1.0) < 1e-14 and abs(e["b"] - st0.b) < 1e-14 * st0.b and abs(e["t"]) < 1e-15
    lat.close()


def test_determinism_bitwise():
    wl = workloads.PREHEAT_128
    N = 48
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N)
    outs = []
    for _ in range(2):
        lat, tp, tq = gpu_scalar(kw, phi, pi, [7])
        e = lat.energy()
        outs.append(([t.cpu().numpy().copy() for t in tp + tq], e["a"], e["b"], e["rho"]))
        lat.close()
    for x, y in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(x, y)
    assert outs[0][1:] == outs[1][1:]


def test_step_chunking_is_invariant():
    """n steps in one call or in several calls give the same trajectory."""
    wl = workloads.PREHEAT_128
    N = 24
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N)
    la, ta, qa = gpu_scalar(kw, phi, pi, [12])
    lb, tb, qb = gpu_scalar(kw, phi, pi, [5, 4, 3])
    for x, y in zip(ta + qa, tb + qb):
        assert rel_maxdiff(x.cpu().numpy(), y.cpu().numpy()) < 1e-14
    assert abs(la.energy()["a"] - lb.energy()["a"]) < 1e-15
    la.close()
    lb.close()


def test_lf_sync_semantics():
    """Energy of a staggered leapfrog state uses synchronised momenta without
    writing them; lattice_sync writes them (sec. 6.1 sync)."""
    from paper_2102_01031_amd.lattice import LatticeError, LAT_ESTATE
    wl = workloads.LPHI4_32
    N = 24
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N)
    lat, tp, tq = gpu_scalar(kw, phi, pi, [11])
    before = [t.cpu().numpy().copy() for t in tq]
    eg = lat.energy()
    after = [t.cpu().numpy() for t in tq]
    assert all(np.array_equal(x, y) for x, y in zip(before, after))
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(11)
    compare_energy(eg, st.energy(), TOL, "lf-stag")
    with pytest.raises(LatticeError) as ei:
        lat.step(-1)
    assert ei.value.code == LAT_ESTATE
    lat.sync()
    st.sync()
    compare_state(tp, tq, st, TOL, "lf-synced")
    lat.step(-11).sync()
    st.run(-11).sync()
    compare_state(tp, tq, st, TOL, "lf-back")
    assert rel_maxdiff(tp[0].cpu().numpy(), phi[0]) < 1e-13
    lat.close()


def test_fp32_mode_error_is_stated():
    """float32 fields, float64 reductions and scale factor, against the float64
    oracle: the measured error is printed and must stay within a float32 budget."""
    wl = workloads.PREHEAT_128
    N = 64
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N)
    steps = 20
    lat, tp, tq = gpu_scalar(kw, phi, pi, [steps], precision="f32")
    eg = lat.energy()
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(steps)
    eo = st.energy()
    ephi = max(rel_maxdiff(tp[s].cpu().numpy(), st.phi[s]) for s in range(2))
    epi = max(rel_maxdiff(tq[s].cpu().numpy(), st.pi[s]) for s in range(2))
    erho = abs(eg["rho"] - eo["rho"]) / eo["rho"]
    ea = abs(eg["a"] - eo["a"]) / eo["a"]
    say(f"[fp32] N={N} steps={steps}: phi {ephi:.2e} pi {epi:.2e} rho {erho:.2e} a {ea:.2e}")
    assert ephi < 2e-6 and epi < 2e-4 and erho < 1e-5 and ea < 1e-7
    lat.close()


def test_graph_replays_match_eager_alternating(monkeypatch):
    """The same with the whole-row kernel alternating its z march direction pass
    by pass (LATTICE_ROWS_ALT=1; odd passes of a call march down)."""
    monkeypatch.setenv("LATTICE_ROWS_ALT", "1")
    test_graph_replays_match_eager("vv4", "self", 64, monkeypatch)
    test_graph_replays_match_eager("lf", "fixed", 64, monkeypatch)


@pytest.mark.parametrize("N,tile,prec", [(256, None, "f64"), (256, "rows,4,7", "f64"), (256, "rows,4,1", "f64"),
                                         (256, None, "f32"), (256, "rows,4,5", "f32"), (128, "rows,8,9", "f64"),
                                         (64, "rows,4,3", "f64")])
def test_row_march_direction(N, tile, prec):
    """Whole-row kernel with the z march direction alternating pass by pass and
    ordinary stores (LATTICE_ROWS_ALT=1, the default at N = 256; downward
    marches start at the top of each z chunk and take z + 1 from the plane
    behind them), on ragged and
    one-plane z chunks: two VV4 steps (six passes, both directions) with
    self-consistent expansion against the oracle, and leapfrog fields bitwise
    equal to upward marches with non-temporal stores."""
    import torch
    wl = workloads.PREHEAT_256
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N)
    with tile_env("1", "LATTICE_ROWS_ALT"):
        if prec == "f64":
            check_run(kw, phi, pi, 2, tile=tile, what=f"rows-alt-{N}")
        else:
            say(f"[parity] f32 rows-alt-{N} tile={tile}")
            with tile_env(tile):
                lat, tp, tq = gpu_scalar(kw, phi, pi, [2], precision="f32")
            st = oracle.ScalarState(oracle_model(kw), phi, pi).run(2)
            for s in range(2):
                assert rel_maxdiff(tp[s].cpu().numpy(), st.phi[s]) < 2e-6
                assert rel_maxdiff(tq[s].cpu().numpy(), st.pi[s]) < 2e-4
            lat.close()
    kl = scalar_kwargs(wl, N=N, integrator="lf", expansion="fixed")
    out = []
    for alt in ("1", "0"):
        with tile_env(alt, "LATTICE_ROWS_ALT"), tile_env(tile):
            lat, tp, tq = gpu_scalar(kl, phi, pi, [3], precision=prec)
        out.append([t.cpu() for t in (*tp, *tq)])
        lat.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("integ,expn,N", [("vv4", "self", 48), ("lf", "fixed", 32), ("vv2", "none", 64)])
def test_graph_replays_match_eager(integ, expn, N, monkeypatch):
    """Calls of eight or more passes are captured once into a HIP graph per step
    count and replayed on later calls.  Alternate two step counts (9: captured;
    4: captured for VV4 only), with eager work and synchronisations in between,
    and check every call bitwise against a run that launches eagerly
    (LATTICE_NO_GRAPH); then the whole run against the oracle."""
    import torch
    wl = workloads.PREHEAT_128
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N, integrator=integ, expansion=expn)
    lg, tg, qg = gpu_scalar(kw, phi, pi, [])
    monkeypatch.setenv("LATTICE_NO_GRAPH", "1")
    le, te, qe = gpu_scalar(kw, phi, pi, [])
    total = 0
    for rep in range(3):
        for n in (9, 4):
            monkeypatch.delenv("LATTICE_NO_GRAPH", raising=False)
            lg.step(n)
            torch.cuda.synchronize()
            eg = lg.energy()
            monkeypatch.setenv("LATTICE_NO_GRAPH", "1")
            le.step(n)
            torch.cuda.synchronize()
            ee = le.energy()
            total += n
            for x, y in zip(tg + qg, te + qe):
                assert torch.equal(x, y), f"call {rep}/{n} differs"
            assert eg["rho"] == ee["rho"] and eg["a"] == ee["a"] and eg["b"] == ee["b"]
            _ = (tg[0] * 1.0).sum().item()          # eager torch work between replays
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(total)
    compare_state(tg, qg, st, TOL, "graph")
    lg.close()
    le.close()


@pytest.mark.parametrize("integ,expn,steps,chunks", [("vv4", "self", 700, [234, 233, 233]),
                                                     ("lf", "fixed", 2100, [700, 700, 700])])
def test_long_call_runs_as_bounded_chunks(integ, expn, steps, chunks):
    """A call longer than 1024 stencil passes runs as consecutive calls of
    equal length (+-1 step), so its coefficient tables and graphs stay
    bounded: bitwise equal to those shorter calls, and within 1e-11 of the
    oracle's uninterrupted run (at most a few ulps per step of rounding growth)."""
    import torch
    wl = workloads.PREHEAT_128
    N = 16
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N, integrator=integ, expansion=expn)
    say(f"[chunks] {integ} {expn} {steps} steps as {chunks}")
    lat1, tp1, tq1 = gpu_scalar(kw, phi, pi, [steps])
    lat2, tp2, tq2 = gpu_scalar(kw, phi, pi, chunks)
    for s in range(2):
        assert torch.equal(tp1[s], tp2[s]) and torch.equal(tq1[s], tq2[s])
    e1, e2 = lat1.energy(), lat2.energy()
    assert e1["a"] == e2["a"] and e1["b"] == e2["b"] and e1["rho"] == e2["rho"] and e1["step"] == e2["step"] == steps
    st = oracle.ScalarState(oracle_model(kw), phi, pi).run(steps)
    compare_state(tp1, tq1, st, 1e-11, "long call")
    compare_energy(e1, st.energy(), 1e-11, "long call")
    lat1.close()
    lat2.close()


@pytest.mark.parametrize("N,integ", [(20, "vv2"), (64, "vv4")])
def test_energy_after_self_consistent_step_uses_the_last_pass_sums(N, integ):
    """After a velocity-Verlet call with self-consistent expansion the energies
    come from the sums the call's last pass reduced: no energy pass runs, the
    result matches the oracle at 1e-12 and repeats exactly."""
    wl = workloads.PREHEAT_128
    phi, pi = wl.initial_fields(N=N)
    kw = scalar_kwargs(wl, N=N, integrator=integ, expansion="self")
    lat, tp, tq = gpu_scalar(kw, phi, pi, [4])
    lat.stats(reset=True)
    lat.profile(True)
    e1 = lat.energy()
    e2 = lat.energy()
    st_ = lat.stats(reset=True)
    lat.profile(False)
    assert st_["launches"].get("energy", 0) == 0
    assert e1 == e2
    ref = oracle.ScalarState(oracle_model(kw), phi, pi).run(4)
    compare_state(tp, tq, ref, TOL, "reuse")
    compare_energy(e1, ref.energy(), TOL, "reuse")
    lat.close()
