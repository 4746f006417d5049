#!/usr/bin/env python3
"""Benchmark of the Wilson-Dirac CG hot path on one MI355X.

Default workload (one step = one whole solve on data resident in HBM):
16^3x32 lattice, links U = exp(0.3 i H), Gaussian complex128 source,
kappa = 0.1365, even-odd preconditioned, plain FP64 CG on D_hat^dag D_hat to
a true residual of 1e-10.  A step sets the gauge field (conversion into the
stencil's store), imports the source, runs the CG and exports x.

Printed: one JSON line with the D_W throughput of the step (GFLOP/s at 1320
flop per stencil output site), the stencil's roofline position (algorithmic
bytes / measured launch time vs 8 TB/s), time-to-solution, the same solve
with FP32 and FP16 inner iterations (FP64 reliable updates), and the CPU
oracle timed on a bounded sample.

Other workloads: --workload cfg1|cfg3|cfg4|cfg5 (see the design doc for each).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D_W GB/s & GFLOP/s vs HBM roofline; CG time-to-1e-10; solves/sec at p99"
HBM_PEAK_GBS = 8000.0
FLOP_PER_SITE = 1320
BC = (1, 1, 1, -1)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dw_flops(stats, half_sites, eo=True):
    """Useful D_W flops of a solve: 1320 per stencil output site."""
    hops_per_iter = 4 if eo else 4  # EO: 4 half-lattice hops; FULL: 2 full-lattice = 4 half
    n = stats["iters"] + stats["reliable_updates"]
    return FLOP_PER_SITE * half_sites * hops_per_iter * n


def make_workload(name):
    import qcdgen
    if name == "cfg2":
        L, width, kappa = (16, 16, 16, 32), 0.3, 0.1365
        seed = qcdgen.CONFIG_SEED_BASE + 1
    elif name == "cfg3":
        L, width, kappa = (24, 24, 24, 48), 0.4, 0.137
        seed = qcdgen.CONFIG_SEED_BASE + 2
    else:
        raise ValueError(name)
    U = qcdgen.links_exp(L, width, qcdgen.rng(seed))
    b = qcdgen.gaussian_spinor(L, qcdgen.rng(seed + 100))
    return L, width, kappa, U, b


def time_solves(lat, Ud, bd, kappa, params, steps, warmup, set_gauge=None):
    import torch
    for _ in range(warmup):
        lat.solve(bd, kappa, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        if set_gauge:
            for prec, recon in set_gauge:
                lat.set_gauge(Ud, prec, recon)
        x, st = lat.solve(bd, kappa, params)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return x, st[0], dt


def instrumented(lat, bd, kappa, params):
    """One solve with hipEvents around every stencil launch."""
    from paper_2409_03030_amd import wdirac as W
    p = W.SolveParams.from_buffer_copy(params)
    p.timing = 1
    x, st = lat.solve(bd, kappa, p)
    s = st[0]
    gbs = s["hop_bytes"] / (s["hop_ms"] * 1e-3) / 1e9
    return {
        "hop_ms_total": s["hop_ms"],
        "hop_launches": s["hop_launches"],
        "hop_ms_avg": s["hop_ms"] / max(1, s["hop_launches"]),
        "bytes_per_launch": s["hop_bytes"] / max(1, s["hop_launches"]),
        "achieved_gbs": gbs,
        "gflops": FLOP_PER_SITE * s["hop_site_updates"] / (s["hop_ms"] * 1e-3) / 1e9,
        "solve_seconds": s["seconds"],
    }


def cpu_baseline(U, b, kappa, L, budget_s):
    """The oracle's A_hat = D_hat^dag D_hat applied repeatedly on the host."""
    import numpy as np
    import oracle as O
    e = O.even_mask(L)
    v = b * e
    n = 0
    t0 = time.perf_counter()
    while True:
        v = O.apply_Ahat(U, v, kappa, BC)
        v = v / np.linalg.norm(v)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    half = (L[0] * L[1] * L[2] * L[3]) // 2
    flops = n * 4 * FLOP_PER_SITE * half
    return {
        "value": flops / dt / 1e9,
        "unit": "GFLOP/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n} applications of the oracle's D_hat^dag D_hat (4 even-odd hops each) on the "
                  f"{'x'.join(map(str, L))} workload in {dt:.1f} s, numpy FP64 single-threaded",
        "seconds_per_DdagD": dt / n,
    }


def bench_default(args):
    import numpy as np
    import torch
    from paper_2409_03030_amd import wdirac as W

    log("generating 16^3x32 workload ...")
    L, width, kappa, U, b = make_workload("cfg2")
    V = L[0] * L[1] * L[2] * L[3]
    half = V // 2
    dev = "cuda:0"
    Ud = torch.from_numpy(U).to(dev)
    bd = torch.from_numpy(b).to(dev)
    lat = W.Lattice(L, BC)
    lat.set_gauge(Ud, "f64", 18)
    lat.set_gauge(Ud, "f32", 12)
    lat.set_gauge(Ud, "f16", 12)
    for prec in ("f64", "f32", "f16"):
        sb, sw, sp = lat.autotune(prec, 1)
        log(f"autotune {prec}: sites/block {sb}, xcd swizzle {sw}, hop split {sp}")
    torch.cuda.synchronize()

    plain = W.default_params()  # EO, FP64 inner, tol 1e-10
    log("timing plain FP64 CG ...")
    x, st, dt = time_solves(lat, Ud, bd, kappa, plain, args.steps, args.warmup, set_gauge=[("f64", 18)])
    if st["status"] != 0 or st["true_resid"] > 1e-10:
        raise SystemExit(f"plain CG failed: {st}")
    flops = dw_flops(st, half)
    roof = instrumented(lat, bd, kappa, plain)
    log(f"plain FP64: {st['iters']} iters, {dt * 1e3:.2f} ms, stencil {roof['achieved_gbs']:.0f} GB/s")

    mixed = {}
    for inner in ("f32", "f16"):
        p = W.default_params(inner=inner, delta=1e-2)
        xm, sm, dtm = time_solves(lat, Ud, bd, kappa, p, max(3, args.steps), 1)
        if sm["status"] != 0:
            raise SystemExit(f"{inner} CG failed: {sm}")
        rm = instrumented(lat, bd, kappa, p)
        err = (torch.linalg.vector_norm(xm - x) / torch.linalg.vector_norm(x)).item()
        mixed[inner] = {
            "time_to_solution_ms": dtm * 1e3,
            "iters": sm["iters"],
            "reliable_updates": sm["reliable_updates"],
            "true_resid": sm["true_resid"],
            "rel_diff_vs_plain_fp64_x": err,
            "stencil_gbs": rm["achieved_gbs"],
            "stencil_ms_avg": rm["hop_ms_avg"],
            "speedup_vs_plain_fp64": dt / dtm,
        }
        log(f"{inner} inner: {sm['iters']} iters, {dtm * 1e3:.2f} ms, stencil {rm['achieved_gbs']:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle for ~{args.cpu_seconds:.0f} s ...")
        cpu = cpu_baseline(U, b, kappa, L, args.cpu_seconds)
        cpu["oracle_time_to_solution_est_s"] = cpu["seconds_per_DdagD"] * (st["iters"] + st["reliable_updates"])

    out = {
        "metric": METRIC,
        "value": flops / dt / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "16^3x32 Wilson-Dirac, U=exp(0.3iH), kappa=0.1365, even-odd, plain FP64 CG to true residual 1e-10",
            "lattice": list(L),
            "kappa": kappa,
            "link_width": width,
            "boundary": "antiperiodic t",
            "precond": "even-odd",
            "inner": "f64",
            "links": "f64 recon-18",
        },
        "time_to_solution_ms": dt * 1e3,
        "solves_per_s": 1.0 / dt,
        "iters": st["iters"],
        "reliable_updates": st["reliable_updates"],
        "true_resid": st["true_resid"],
        "roofline": {
            "bound": "hbm",
            "achieved": roof["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": roof["achieved_gbs"] / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "hop_kernel<F64,18,*> (all stencil launches of one solve)",
            "avg_launch_ms": roof["hop_ms_avg"],
            "bytes_per_launch": roof["bytes_per_launch"],
            "stencil_gflops": roof["gflops"],
        },
        "mixed_precision": mixed,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "cfg2":
        bench_default(args)
    else:
        import bench_workloads  # noqa: F401  (other configurations)
        bench_workloads.run(args)


if __name__ == "__main__":
    main()
