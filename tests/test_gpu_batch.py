"""GPU checks of the batched ensemble path: independent single-field lattices
of uneven sizes, batched launches replayed from a captured graph (one launch
over all realizations per step, or segment after segment), autotuned modes.  FP64 batches match the oracle per realization to 1e-12; the
full float32 ensemble (256 realizations of 24^3..64^3, 2000 steps) is checked
on sampled realizations against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import rel_maxdiff, say, tile_env, to_dev
from paper_2102_01031_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def batch_kwargs(wl):
    b = wl.base
    return dict(dx=b.dx, dt=b.dt, integrator="lf", expansion="fixed", potential="phi4", lam=b.lam,
                alpha=b.alpha, w_eos=b.w_eos, H0=b.H0, a0=b.a0, t_ref=0.0, t0=0.0)


def oracle_run(wl, phi, pi, N, steps):
    b = wl.base
    m = oracle.ScalarModel(N=N, dx=b.dx, dt=b.dt, nfields=1, potential=oracle.PHI4, expansion=oracle.FIXED,
                           integrator=oracle.LF, lam=b.lam, alpha=b.alpha, w_eos=b.w_eos, H0=b.H0, t0=0.0,
                           a0=b.a0)
    return oracle.ScalarState(m, phi, pi).run(steps)


def make_batch(wl, sizes, dtype, precision, autotune=True):
    from paper_2102_01031_amd.lattice import LatticeBatch
    fields = [wl.initial_fields(r, N) for r, N in enumerate(sizes)]
    phis = [to_dev(f[0], dtype)[0] for f in fields]
    pis = [to_dev(f[1], dtype)[0] for f in fields]
    lb = LatticeBatch(phis, pis, sizes, autotune=autotune, precision=precision, **batch_kwargs(wl))
    return lb, fields, phis, pis


def test_batch_fp64_parity_uneven_sizes():
    import torch
    wl = workloads.BATCH
    sizes = [24, 32, 48, 64, 24, 40, 17, 32, 64, 5]
    lb, fields, phis, pis = make_batch(wl, sizes, torch.float64, "f64")
    for N in sorted(set(sizes)):
        say(f"[batch] N={N} tile={lb.tile(N)}")
    lb.step(17).step(13)
    torch.cuda.synchronize()
    for r, N in enumerate(sizes):
        st = oracle_run(wl, fields[r][0], fields[r][1], N, 30)
        assert rel_maxdiff(phis[r].cpu().numpy(), st.phi[0]) <= 1e-12, (r, N)
        assert rel_maxdiff(pis[r].cpu().numpy(), st.pi[0]) <= 1e-12, (r, N)
        e, eo = lb.energy(r), st.energy()
        assert abs(e["rho"] - eo["rho"]) <= 1e-12 * eo["rho"] and abs(e["a"] - eo["a"]) <= 1e-14
    lb.close()


@pytest.mark.parametrize("spec", ["site", "16,5"])
def test_batch_forced_shapes_fp64(spec):
    """Every realization in one mode: one thread per site ('site': 256 consecutive
    sites per block, the last block of each lattice partly empty for N = 5, 17,
    24, 40) or 16-wide tiles with a z chunk of 5 (ragged chunks), against the
    oracle per realization."""
    import torch
    wl = workloads.BATCH
    sizes = [24, 5, 17, 64, 40, 32, 17]
    with tile_env(spec, "LATTICE_BATCH_TILE"):
        lb, fields, phis, pis = make_batch(wl, sizes, torch.float64, "f64", autotune=False)
    for N in sorted(set(sizes)):
        t = lb.tile(N)
        say(f"[batch] forced {spec}: N={N} tile={t}")
        assert (t == (0, 0, 0)) if spec == "site" else (t[0] == 16 and t[2] == 5)
    lb.step(11).step(6)
    torch.cuda.synchronize()
    for r, N in enumerate(sizes):
        st = oracle_run(wl, fields[r][0], fields[r][1], N, 17)
        assert rel_maxdiff(phis[r].cpu().numpy(), st.phi[0]) <= 1e-12, (spec, r, N)
        assert rel_maxdiff(pis[r].cpu().numpy(), st.pi[0]) <= 1e-12, (spec, r, N)
    lb.close()


def test_batch_segments_bitwise_and_oracle():
    """lattice_step runs the realizations segment by segment (all steps of one
    segment, then the next).  Tiny segments (a 1 MB budget: most realizations
    alone) must give bitwise the arrays of one launch over all realizations
    per step, and both match the oracle."""
    import torch
    wl = workloads.BATCH
    sizes = [24, 64, 17, 48, 32, 5, 64, 40]
    with tile_env("0", "LATTICE_BATCH_SEG_MB"):
        la, fa, pa, qa = make_batch(wl, sizes, torch.float64, "f64", autotune=False)
    with tile_env("1", "LATTICE_BATCH_SEG_MB"):
        lb, fb, pb, qb = make_batch(wl, sizes, torch.float64, "f64", autotune=False)
    for n in (9, 4, 9):
        la.step(n)
        lb.step(n)
    torch.cuda.synchronize()
    for x, y in zip(pa + qa, pb + qb):
        assert torch.equal(x, y)
    for r, N in enumerate(sizes):
        st = oracle_run(wl, fa[r][0], fa[r][1], N, 22)
        assert rel_maxdiff(pb[r].cpu().numpy(), st.phi[0]) <= 1e-12, (r, N)
        assert rel_maxdiff(qb[r].cpu().numpy(), st.pi[0]) <= 1e-12, (r, N)
    la.close()
    lb.close()


def test_batch_graph_replay_matches_direct_steps():
    """Replays of one captured graph (same step count, several calls) equal a
    batch that captured a different chunking."""
    import torch
    wl = workloads.BATCH
    sizes = [24, 48, 32, 64]
    la, fa, pa, qa = make_batch(wl, sizes, torch.float64, "f64", autotune=False)
    lb, fb, pb, qb = make_batch(wl, sizes, torch.float64, "f64", autotune=False)
    for _ in range(4):
        la.step(6)
        torch.cuda.synchronize()
    lb.step(24)
    torch.cuda.synchronize()
    for x, y in zip(pa + qa, pb + qb):
        assert rel_maxdiff(x.cpu().numpy(), y.cpu().numpy()) <= 1e-14
    la.close()
    lb.close()


def test_batch_full_ensemble_fp32():
    import time
    import torch
    wl = workloads.BATCH
    sizes = wl.sizes()
    lb, fields, phis, pis = make_batch(wl, sizes, torch.float32, "f32")
    for N in sorted(set(sizes)):
        say(f"[batch] autotuned tile for {N}^3: {lb.tile(N)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.step(wl.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sites = sum(N ** 3 for N in sizes)
    say(f"[batch] {len(sizes)} realizations, {sites} sites, {wl.steps} steps in {wall * 1e3:.1f} ms: "
        f"{sites * wl.steps / wall:.3e} site-updates/s")
    # sampled realizations against the float64 oracle after the full run
    picked = {}
    for r, N in enumerate(sizes):
        picked.setdefault(N, r)
    for N, r in sorted(picked.items()):
        if N > 32:
            continue            # the oracle takes minutes for 2000 steps at 48^3 and 64^3
        st = oracle_run(wl, fields[r][0], fields[r][1], N, wl.steps)
        ephi = rel_maxdiff(phis[r].cpu().numpy(), st.phi[0])
        e = lb.energy(r)
        erho = abs(e["rho"] - st.energy()["rho"]) / st.energy()["rho"]
        say(f"[batch] realization {r} (N={N}) after {wl.steps} steps: phi rel {ephi:.2e}, rho rel {erho:.2e}")
        assert ephi < 1e-4 and erho < 1e-5
    lb.close()


def test_batch_fp32_short_vs_oracle_all_sizes():
    import torch
    wl = workloads.BATCH
    sizes = [24, 32, 48, 64]
    lb, fields, phis, pis = make_batch(wl, sizes, torch.float32, "f32")
    lb.step(100)
    torch.cuda.synchronize()
    for r, N in enumerate(sizes):
        st = oracle_run(wl, fields[r][0], fields[r][1], N, 100)
        ephi = rel_maxdiff(phis[r].cpu().numpy(), st.phi[0])
        epi = rel_maxdiff(pis[r].cpu().numpy(), st.pi[0])
        say(f"[batch] fp32 N={N} 100 steps: phi {ephi:.2e} pi {epi:.2e}")
        assert ephi < 2e-6 and epi < 2e-4
    lb.close()


def test_batch_graph_replays_match_eager(monkeypatch):
    import torch
    wl = workloads.BATCH
    sizes = [24, 32, 48, 64, 17]
    la, fa, pa, qa = make_batch(wl, sizes, torch.float32, "f32", autotune=False)
    monkeypatch.setenv("LATTICE_NO_GRAPH", "1")
    lb, fb, pb, qb = make_batch(wl, sizes, torch.float32, "f32", autotune=False)
    for rep in range(4):
        monkeypatch.delenv("LATTICE_NO_GRAPH", raising=False)
        la.step(9)
        torch.cuda.synchronize()
        monkeypatch.setenv("LATTICE_NO_GRAPH", "1")
        lb.step(9)
        torch.cuda.synchronize()
        for x, y in zip(pa + qa, pb + qb):
            assert torch.equal(x, y), f"replay {rep} differs"
        _ = (pa[0] * 2.0).sum().item()
    la.close()
    lb.close()
