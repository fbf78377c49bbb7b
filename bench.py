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
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "site-updates/s per integrator stage, % HBM peak; adjoint/forward time ratio"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("stage_scalar.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2102_01031_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kind: str, per_launch_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_stage_preheat256.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != kernel_hash():
        return None
    k = d.get("kernels", {}).get(kind)
    if not k:
        return None
    return k["hbm_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the lattice step "
              "is single-GPU; see the sharding design in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

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

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        m = oracle.ScalarModel(N=N, dx=wl.dx, dt=wl.dt, nfields=2, potential=oracle.PHI4_CHI2,
                               expansion=oracle.SELF, integrator=oracle.VV4, lam=wl.lam, q=wl.q,
                               alpha=wl.alpha, kappa2=wl.kappa2, a0=wl.a0)
        log(f"[bench] oracle on the host: {args.cpu_steps} VV4 steps at {N}^3")
        ost = oracle.ScalarState(m, phi, pi)
        c0 = time.perf_counter()
        ost.run(args.cpu_steps)
        cwall = time.perf_counter() - c0
        cpu = {"value": N ** 3 * 3 * args.cpu_steps / cwall, "unit": "site-updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{args.cpu_steps} VV4 steps ({3 * args.cpu_steps} stages) of the same {N}^3 "
                         f"two-field self-consistent workload, single-threaded plain C oracle, {cwall:.1f} s"}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
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
                     "mean_launch_us": avg_ms * 1e3},
        "hbm_frac_of_peak": achieved / HBM_PEAK_GBS,
        "cpu_baseline": cpu,
    }
    lat.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
