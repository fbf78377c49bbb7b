"""Benchmark: site-updates/s per integrator stage on the two-field preheating
lattice (256^3, lambda phi^4 + q/2 phi^2 chi^2 with q = 100, 4th-order Yoshida
velocity-Verlet = 3 stages per step, self-consistent expansion, float64).

Prints one JSON line.  value = N^3 * 3 * steps / wall time of the timed steps
(inputs resident in HBM).  roofline: algorithmic bytes of one stencil pass
(read phi, pi of both fields, write them: 64 B/site) over the pass's mean
duration from HIP events on the context stream.  cpu_baseline: the FP64 oracle
on the host, a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "site-updates/s per integrator stage, % HBM peak; adjoint/forward time ratio"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def stored_traffic(kind: str, per_launch_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_stage_preheat256.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    from paper_2102_01031_amd.pmc_summary import kernel_hash
    if d.get("kernel_hash") != kernel_hash():
        return None
    k = d.get("kernels", {}).get(kind)
    if not k:
        return None
    return k["hbm_bytes_per_launch"]


def device_warmup(Lattice, tp, tq, stream, kw, log, min_ms=30.0):
    """Step a scratch context on copies of the fields for at least min_ms of
    wall time; returns what was run (reported in the JSON line)."""
    import torch
    cp = [t.clone() for t in tp]
    cq = [t.clone() for t in tq]
    scratch = Lattice(cp, cq, stream=stream, **kw)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    steps = 0
    while 1e3 * (time.perf_counter() - c0) < min_ms:
        scratch.step(5)
        torch.cuda.synchronize()
        steps += 5
    ms = 1e3 * (time.perf_counter() - c0)
    scratch.close()
    del cp, cq
    log(f"[bench] device warm-up: {steps} steps on a scratch copy, {ms:.1f} ms")
    return {"what": "steps of a scratch context on copies of the fields, before the W warmup steps",
            "steps": steps, "ms": ms}


def measured_ceiling(log):
    """Streaming ceiling of the stage kernel's access pattern (4 float64 arrays
    of 256^3 in, 4 out) from the probe csrc/ceiling, run as a child process
    before this process touches the GPU; None if the probe is not built or
    fails."""
    exe = os.path.join(ROOT, "paper_2102_01031_amd", "csrc", "ceiling")
    if not os.path.exists(exe):
        return None
    try:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    except (OSError, subprocess.TimeoutExpired):
        return None
    if r.returncode != 0:
        log(f"[bench] ceiling probe failed: {r.stderr.strip()[:200]}")
        return None
    out = {}
    for line in r.stdout.splitlines():
        try:
            d = json.loads(line)
        except ValueError:
            continue
        out[d["pattern"]] = d["GBs"]
    return out or None


def run_extras(args, log, only=None):
    """The other workloads' headline numbers: the adjoint/forward time ratio
    (two fields, 64^3, 2000 VV2 steps), the U(1) and SU(2) stages (128^3 leapfrog), the
    batched ensemble rate (256 lattices
    of 24^3..64^3, float32, 2000 LF steps, one captured graph) and the
    single-field 32^3 leapfrog run (1000 steps)."""
    import torch

    from paper_2102_01031_amd import workloads
    from paper_2102_01031_amd.lattice import Lattice, LatticeBatch

    dev = torch.device("cuda:0")
    res = {}
    if only in (None, "adjoint"):
        # adjoint / forward
        wl = workloads.ADJ_64
        phi, pi = wl.initial_fields()
        tp = [torch.tensor(f.reshape(-1), device=dev) for f in phi]
        tq = [torch.tensor(f.reshape(-1), device=dev) for f in pi]
        lat = Lattice(tp, tq, N=wl.N, dx=wl.dx, dt=wl.dt, integrator="vv2", expansion="none", potential="phi4_chi2",
                      lam=wl.lam, q=wl.q)
        lat.grad(50)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        lat.step(wl.steps)
        torch.cuda.synchronize()
        fwd = time.perf_counter() - c0
        lat.step(-wl.steps)
        torch.cuda.synchronize()
        # sweep times from a call without per-launch instrumentation
        c0 = time.perf_counter()
        r = lat.grad(wl.steps)
        gwall = time.perf_counter() - c0
        # per-pass kernel times from a second, instrumented call
        lat.stats(reset=True)
        lat.profile(True)
        lat.grad(wl.steps)
        st = lat.stats(reset=True)
        lat.profile(False)
        fus = 1e3 * st["kernel_ms"]["kick_drift"] / max(st["launches"]["kick_drift"], 1)
        aus = 1e3 * st["kernel_ms"]["adjoint"] / max(st["launches"]["adjoint"], 1)
        res["adjoint"] = {"workload": wl.name, "steps": wl.steps, "observable": "(E_K^chi + E_G^chi)/rho",
                          "value": r["value"], "dO_dq": r["dO_dq"],
                          "forward_ms": r["forward_ms"], "reverse_ms": r["reverse_ms"],
                          "ratio_reverse_over_forward": r["reverse_ms"] / r["forward_ms"],
                          "forward_plain_ms": 1e3 * fwd, "grad_call_ms": 1e3 * gwall,
                          "kernel_ratio_adjoint_over_forward_pass": aus / fus,
                          "forward_pass_us": fus, "adjoint_pass_us": aus}
        lat.close()
        log(f"[bench] adjoint: reverse/forward {r['reverse_ms'] / r['forward_ms']:.2f}, per pass {aus / fus:.2f}")
        # the same workload with the self-consistent expansion (kappa^2 = 0.25):
        # the forward sweep as one call per checkpoint segment, the reverse as
        # one fused pass per time point (a short call first builds the graphs)
        tp = [torch.tensor(f.reshape(-1), device=dev) for f in phi]
        tq = [torch.tensor(f.reshape(-1), device=dev) for f in pi]
        ls = Lattice(tp, tq, N=wl.N, dx=wl.dx, dt=wl.dt, integrator="vv2", expansion="self", potential="phi4_chi2",
                     lam=wl.lam, q=wl.q, kappa2=0.25)
        ls.grad(50)
        rs = ls.grad(wl.steps)
        res["adjoint_self"] = {"workload": wl.name + " self-consistent expansion", "steps": wl.steps,
                               "value": rs["value"], "dO_dq": rs["dO_dq"], "dO_da0": rs["dO_da0"],
                               "dO_db0": rs["dO_db0"], "forward_ms": rs["forward_ms"], "reverse_ms": rs["reverse_ms"],
                               "ratio_reverse_over_forward": rs["reverse_ms"] / rs["forward_ms"]}
        ls.close()
        log(f"[bench] adjoint, self-consistent: forward {rs['forward_ms']:.1f} ms, reverse {rs['reverse_ms']:.1f} ms")
    if only in (None, "u1"):
        # U(1) gauge + complex scalar, 128^3, leapfrog: ten N^3 float64 arrays, each
        # read once and written once per step (160 B per site)
        uw = workloads.ABELIAN_HIGGS_128
        uf = uw.initial_fields()
        ut = [[torch.tensor(a.reshape(-1), device=dev) for a in f] for f in uf]
        lu = Lattice(ut[0], ut[1], A=ut[2], piA=ut[3], N=uw.N, dx=uw.dx, dt=uw.dt, integrator="lf", expansion="none",
                     potential="abelian_higgs", lam=uw.lam, v=uw.v, e=uw.e, kappa_g=uw.kappa_g)
        lu.step(uw.steps)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        lu.step(uw.steps)
        torch.cuda.synchronize()
        uwall = time.perf_counter() - c0
        lu.stats(reset=True)
        lu.profile(True)
        lu.step(uw.steps)
        st = lu.stats(reset=True)
        lu.profile(False)
        uus = 1e3 * st["kernel_ms"]["gauge"] / max(st["launches"]["gauge"], 1)
        ue = lu.energy()
        res["u1"] = {"workload": uw.name, "steps": uw.steps, "us_per_step": 1e6 * uwall / uw.steps,
                     "value": uw.N ** 3 * uw.steps / uwall, "unit": "site-updates/s",
                     "mean_launch_us": uus, "achieved_GBs_alg": uw.N ** 3 * 160 / (uus * 1e-6) / 1e9,
                     "gauss_max_over_terms": ue["gauss_max"] / max(ue["gauss_div_max"], ue["gauss_charge_max"], 1e-300)}
        lu.close()
        log(f"[bench] U(1): {res['u1']['us_per_step']:.1f} us per step, stage {uus:.1f} us, "
            f"{res['u1']['achieved_GBs_alg']:.0f} GB/s algorithmic")
    if only in (None, "su2"):
        # SU(2) doublet + SU(2) links, 128^3, leapfrog: 29 N^3 float64 arrays (doublet 4,
        # momenta 4, links 12, electric 9), each read once and written once per step
        # (464 B per site)
        sw = workloads.SU2_HIGGS_128
        sf = sw.initial_fields()
        stt = [[torch.tensor(a.reshape(-1), device=dev) for a in f] for f in sf]
        ls2 = Lattice(doublet=stt[0], pi_doublet=stt[1], U=stt[2], E=stt[3], N=sw.N, dx=sw.dx, dt=sw.dt,
                      integrator="lf", expansion="none", potential="su2_higgs", lam=sw.lam, v=sw.v, g=sw.g)
        # Gauss-consistent initial gauge momenta on the device (three float64 Poisson
        # solves at 128^3) on the initial state, whose links are at the identity; the
        # workload starts charge-free, so E stays zero
        ls2.gauss_init()
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        ls2.gauss_init()
        gauss_ms = 1e3 * (time.perf_counter() - c0)
        ls2.step(sw.steps)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        ls2.step(sw.steps)
        torch.cuda.synchronize()
        swall = time.perf_counter() - c0
        ls2.stats(reset=True)
        ls2.profile(True)
        ls2.step(sw.steps)
        st = ls2.stats(reset=True)
        ls2.profile(False)
        sus = 1e3 * st["kernel_ms"]["gauge"] / max(st["launches"]["gauge"], 1)
        se = ls2.energy()
        res["su2"] = {"workload": sw.name, "steps": sw.steps, "us_per_step": 1e6 * swall / sw.steps,
                      "gauss_init_ms": gauss_ms,
                      "value": sw.N ** 3 * sw.steps / swall, "unit": "site-updates/s",
                      "mean_launch_us": sus, "achieved_GBs_alg": sw.N ** 3 * 464 / (sus * 1e-6) / 1e9,
                      "gauss_max_over_terms": se["gauss_max"] / max(se["gauss_div_max"], se["gauss_charge_max"],
                                                                    1e-300)}
        ls2.close()
        log(f"[bench] SU(2): {res['su2']['us_per_step']:.1f} us per step, stage {sus:.1f} us, "
            f"{res['su2']['achieved_GBs_alg']:.0f} GB/s algorithmic")
    if only in (None, "batch"):
        # batched ensemble
        bw = workloads.BATCH
        sizes = bw.sizes()
        phis, pis = [], []
        for rr, N in enumerate(sizes):
            f = bw.initial_fields(rr, N)
            phis.append(torch.tensor(f[0][0].reshape(-1), device=dev, dtype=torch.float32))
            pis.append(torch.tensor(f[1][0].reshape(-1), device=dev, dtype=torch.float32))
        b = bw.base
        lb = LatticeBatch(phis, pis, sizes, autotune=True, precision="f32", dx=b.dx, dt=b.dt, integrator="lf",
                          expansion="fixed", potential="phi4", lam=b.lam, alpha=b.alpha, w_eos=b.w_eos, H0=b.H0,
                          a0=b.a0)
        lb.step(bw.steps)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        lb.step(bw.steps)
        torch.cuda.synchronize()
        bwall = time.perf_counter() - c0
        sites = sum(N ** 3 for N in sizes)
        res["batch"] = {"workload": bw.name, "realizations": len(sizes), "sites": sites, "steps": bw.steps,
                        "value": sites * bw.steps / bwall, "unit": "site-updates/s", "ms": 1e3 * bwall,
                        "tiles": {str(N): list(lb.tile(N)) for N in sorted(set(sizes))},
                        "achieved_GBs_alg": sites * 16 * bw.steps / bwall / 1e9}
        lb.close()
        log(f"[bench] batch: {res['batch']['value']:.3e} site-updates/s")
    if only in (None, "lphi4_32"):
        # single field, 32^3, 1000 LF steps
        w0 = workloads.LPHI4_32
        phi, pi = w0.initial_fields()
        tp = [torch.tensor(phi[0].reshape(-1), device=dev)]
        tq = [torch.tensor(pi[0].reshape(-1), device=dev)]
        l0 = Lattice(tp, tq, N=w0.N, dx=w0.dx, dt=w0.dt, integrator="lf", expansion="fixed", potential="phi4",
                     lam=w0.lam, alpha=w0.alpha, w_eos=w0.w_eos, H0=w0.H0, a0=w0.a0)
        # the first call of a step count captures its graph; later calls replay it
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        l0.step(w0.steps)
        torch.cuda.synchronize()
        w_first = time.perf_counter() - c0
        c0 = time.perf_counter()
        l0.step(w0.steps)
        torch.cuda.synchronize()
        w = time.perf_counter() - c0
        res["lphi4_32"] = {"workload": w0.name, "steps": w0.steps, "us_per_step": 1e6 * w / w0.steps,
                           "us_per_step_first_call": 1e6 * w_first / w0.steps,
                           "value": w0.N ** 3 * w0.steps / w, "unit": "site-updates/s"}
        l0.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--main-only", action="store_true", help="only the 256^3 workload (for profiling)")
    ap.add_argument("--only", choices=["adjoint", "u1", "su2", "batch", "lphi4_32"],
                    help="only this other workload; prints its JSON object (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the lattice step "
              "runs on a single GPU; a multi-GPU run would split the lattice into z slabs with one-plane "
              "halos, which is not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.only:
        print(json.dumps(run_extras(args, log, only=args.only)))
        return
    ceilings = None if args.main_only else measured_ceiling(log)
    if ceilings:
        log(f"[bench] streaming ceilings (GB/s): {ceilings}")

    import numpy as np
    import torch

    from paper_2102_01031_amd import workloads
    from paper_2102_01031_amd.lattice import Lattice

    wl = workloads.PREHEAT_256
    N = wl.N
    log(f"[bench] generating seeded initial conditions for {wl.name}")
    phi, pi = wl.initial_fields()
    dt = torch.float32 if args.precision == "f32" else torch.float64
    dev = torch.device("cuda:0")
    tp = [torch.tensor(f.reshape(-1), device=dev, dtype=dt) for f in phi]
    tq = [torch.tensor(f.reshape(-1), device=dev, dtype=dt) for f in pi]
    kw = dict(N=N, dx=wl.dx, dt=wl.dt, integrator=wl.integrator, expansion=wl.expansion, potential=wl.potential,
              lam=wl.lam, q=wl.q, alpha=wl.alpha, kappa2=wl.kappa2, a0=wl.a0, precision=args.precision)
    stream = torch.cuda.current_stream()
    # device warm-up: the stage kernel reaches its steady per-pass time only
    # after about 10 ms of sustained stepping (measured on one GPU: 200 us per
    # pass in a first 20-step call after 5 steps, 191.9 us after 20, 206.9 us
    # after 0.2 s idle), so a scratch context on copies of the fields steps
    # for at least 30 ms first.  It touches neither the timed lattice nor its
    # state; the W warmup steps and the K timed steps below are unchanged.
    dw = device_warmup(Lattice, tp, tq, stream, kw, log)
    lat = Lattice(tp, tq, stream=stream, **kw)
    log(f"[bench] warmup {args.warmup} steps")
    lat.step(args.warmup)
    torch.cuda.synchronize()

    # timed region: K steps, no instrumentation
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = 3 * args.steps
    value = N ** 3 * stages / wall
    ms_per_step = 1e3 * wall / args.steps

    # roofline: mean duration of the dominant kernel from HIP events on the context stream
    lat.stats(reset=True)
    lat.profile(True)
    lat.step(args.steps)
    st = lat.stats(reset=True)
    lat.profile(False)
    kind = "drift_kick_red"
    n_launch = st["launches"][kind]
    avg_ms = st["kernel_ms"][kind] / max(n_launch, 1)
    esize = 4 if args.precision == "f32" else 8
    alg_bytes = N ** 3 * 2 * 4 * esize          # 2 fields x (read phi, pi + write phi, pi)
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = stored_traffic(kind + "_" + args.precision, alg_bytes)
    e = lat.energy()
    log(f"[bench] {n_launch} '{kind}' launches, mean {avg_ms * 1e3:.1f} us, {achieved:.0f} GB/s; "
        f"a={e['a']:.6f} hubble_res={e['hubble_res']:.2e}")
    # measurement pass (energies and Hubble residual; read-only over phi, pi).
    # After a step the context reports the sums its last pass reduced, so the
    # pass is timed on a second context over the same arrays.
    lm = Lattice(tp, tq, stream=stream, **kw)
    lm.stats(reset=True)
    lm.profile(True)
    for _ in range(5):
        lm.energy()
    se = lm.stats(reset=True)
    lm.profile(False)
    lm.close()
    e_us = 1e3 * se["kernel_ms"]["energy"] / max(se["launches"]["energy"], 1)
    energy_pass = {"mean_launch_us": e_us, "alg_bytes_per_launch": N ** 3 * 2 * 2 * esize,
                   "achieved_GBs_alg": N ** 3 * 2 * 2 * esize / (e_us * 1e-6) / 1e9}
    # power spectrum of one field (transform and binning on the device, result on the host)
    lat.spectrum(0, "phi")            # plan and buffers on the first call
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    sp = lat.spectrum(0, "phi")
    spectrum = {"ms": 1e3 * (time.perf_counter() - c0), "bins": len(sp["sum"]), "field": "phi",
                "includes": "copy to the transform buffer, float64 real-to-complex FFT, binning, host copy"}
    # occupation number of chi (two transforms, binning, <phi^2> reduction, host copy)
    lat.occupation(1)                 # second half-spectrum buffer on the first call
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    lat.occupation(1)
    spectrum["occupation_ms"] = 1e3 * (time.perf_counter() - c0)

    # float32-fields mode on the same workload
    f32 = None
    if args.precision == "f64" and not args.main_only:
        tp32 = [t.to(torch.float32) for t in tp]
        tq32 = [t.to(torch.float32) for t in tq]
        kw32 = dict(kw, precision="f32")
        l32 = Lattice(tp32, tq32, stream=stream, **kw32)
        l32.step(args.warmup)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        l32.step(args.steps)
        torch.cuda.synchronize()
        w32 = time.perf_counter() - c0
        l32.stats(reset=True)
        l32.profile(True)
        l32.step(args.steps)
        s32 = l32.stats(reset=True)
        us32 = 1e3 * s32["kernel_ms"][kind] / max(s32["launches"][kind], 1)
        f32 = {"value": N ** 3 * stages / w32, "unit": "site-updates/s", "mean_launch_us": us32,
               "achieved_GBs": N ** 3 * 2 * 4 * 4 / (us32 * 1e-6) / 1e9, "tile": list(s32["tile"]),
               "z_chunk": s32["z_chunk"]}
        l32.close()
        del tp32, tq32
        log(f"[bench] float32 fields: {f32['value']:.3e} site-updates/s, {us32:.1f} us per pass")

    extras = {} if args.main_only else run_extras(args, log)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        m = oracle.ScalarModel(N=N, dx=wl.dx, dt=wl.dt, nfields=2, potential=oracle.PHI4_CHI2,
                               expansion=oracle.SELF, integrator=oracle.VV4, lam=wl.lam, q=wl.q,
                               alpha=wl.alpha, kappa2=wl.kappa2, a0=wl.a0)
        # the oracle on one core, then on the host's cores (OpenMP over z planes
        # in its per-site loops; its volume sums stay serial)
        threads_all = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        before = oracle.set_threads(0)
        timing = {}
        for nt in (1, threads_all):
            used = oracle.set_threads(nt)
            log(f"[bench] oracle on the host, {used} thread(s): {args.cpu_steps} VV4 steps at {N}^3")
            ost = oracle.ScalarState(m, phi, pi)
            c0 = time.perf_counter()
            ost.run(args.cpu_steps)
            timing[nt] = (time.perf_counter() - c0, used)
        oracle.set_threads(before)
        cwall, used = timing[threads_all]
        w1, _ = timing[1]
        sample = (f"{args.cpu_steps} VV4 steps ({3 * args.cpu_steps} stages) of the same {N}^3 two-field "
                  f"self-consistent workload, plain C oracle")
        cpu = {"value": N ** 3 * 3 * args.cpu_steps / cwall, "unit": "site-updates/s", "cores": used,
               "kind": "oracle", "sample": f"{sample}, {used} threads, {cwall:.1f} s",
               "one_core": {"value": N ** 3 * 3 * args.cpu_steps / w1, "cores": 1,
                            "sample": f"{sample}, 1 thread, {w1:.1f} s"},
               "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count()}}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "device_warmup": dw,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": wl.name, "N": N, "fields": 2, "integrator": "VV4", "stages_per_step": 3,
                   "expansion": "self-consistent", "precision": args.precision,
                   "tile": list(st["tile"]), "z_chunk": st["z_chunk"], "blocks": st["blocks"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"scalar_stage {kind}", "alg_bytes_per_launch": alg_bytes,
                     "mean_launch_us": avg_ms * 1e3,
                     "measured_ceiling_GBs": (ceilings.get("streams4_256")
                                              if ceilings and args.precision == "f64" else None),
                     "frac_of_measured_ceiling": (achieved / ceilings["streams4_256"]
                                                  if ceilings and "streams4_256" in ceilings and args.precision == "f64"
                                                  else None)},
        "hbm_frac_of_peak": achieved / HBM_PEAK_GBS,
        "cpu_baseline": cpu,
        "energy_pass": energy_pass,
        "spectrum": spectrum,
        "precision_f32": f32,
    }
    out.update(extras)
    lat.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
