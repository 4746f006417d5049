#!/usr/bin/env python3
"""Benchmark of the Wilson-Dirac CG hot path on one MI355X.

Default workload (one step = one whole solve on data resident in HBM):
24^3x48 lattice, links U = exp(0.4 i H), Gaussian complex128 source,
kappa = 0.137, even-odd preconditioned, plain FP64 CG on D_hat^dag D_hat to
a true residual of 1e-10.  A step sets the gauge field (conversion into the
stencil's store), imports the source, runs the CG and exports x.  The FP64
link field (255-382 MB) and the CG vectors exceed the 256 MB Infinity Cache,
so the stencil streams from HBM.

Printed: one JSON line with the D_W throughput of the step (GFLOP/s at 1320
flop per stencil output site), the dominant stencil's roofline position
(algorithmic bytes / measured launch time vs 8 TB/s), time-to-solution, the
same solve with FP32 and FP16 inner iterations (recon-12 links, FP64 reliable
updates), each solution's FP64 true residual recomputed by the CPU oracle,
the cache-resident 16^3x32 solve beside it, and the oracle timed on the
host's cores.

Other workloads: --workload cfg2|cfg1|cfg4|cfg5|stencil|pion|force|staggered|oracle.
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


# Sources that determine the stencil kernels' code; counter-derived traffic is
# only reported while they are unchanged since the counters were taken.
KERNEL_SOURCES = ["paper_2409_03030_amd/csrc/hop.hip", "paper_2409_03030_amd/csrc/wd_device.h",
                  "paper_2409_03030_amd/csrc/wd_kcommon.h", "paper_2409_03030_amd/csrc/wd_launch.h",
                  "paper_2409_03030_amd/csrc/wd_fastdiv.h"]
TRAFFIC_DB = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def lookup_traffic(kernel, lattice):
    """Counter-derived HBM bytes per launch of `kernel`, or None if not measured
    for the current kernel sources."""
    try:
        db = json.load(open(TRAFFIC_DB))
    except (OSError, ValueError):
        return None
    e = db.get(f"{kernel}|{lattice}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def summarize_pmc(fetch_csv, write_csv, kernel, lattice, out=TRAFFIC_DB):
    """Fold two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch)
    into bytes per launch of `kernel`, scaled by what the same counters read for
    the 1 GiB device copy in the same runs."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals, copy = [], []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            if r["Kernel_Name"].startswith(kernel):
                vals.append(v)
            elif "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 131072:
                copy.append(v)
        return vals, copy

    fv, fc = per_kernel(fetch_csv, "FETCH_SIZE")
    wv, wc = per_kernel(write_csv, "WRITE_SIZE")
    gib = float(1 << 30)
    f_scale = gib / statistics.median(fc)
    w_scale = gib / statistics.median(wc)
    fetch = statistics.median(fv) * f_scale
    write = statistics.median(wv) * w_scale
    db = {}
    if os.path.exists(out):
        db = json.load(open(out))
    db[f"{kernel}|{lattice}"] = {
        "source_hash": kernel_source_hash(), "bytes_per_launch": fetch + write,
        "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
        "dispatches": [len(fv), len(wv)], "copy_scale": {"FETCH_SIZE": f_scale, "WRITE_SIZE": w_scale},
        "fetch_csv": fetch_csv, "write_csv": write_csv,
    }
    with open(out, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    return db[f"{kernel}|{lattice}"]


def calibration_copy():
    """A 1 GiB device-to-device copy: the known-size reference for the HBM counters."""
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / dt / 1e9


def read_bandwidth(nbytes=1 << 30):
    """The library's plain streaming-read kernel over nbytes: the attainable
    read rate on the same box (1 GiB: from HBM; 128 MiB: partly from the
    Infinity Cache, like the 16^3x32 working set)."""
    import torch
    from paper_2409_03030_amd import wdirac as W
    ms = W.time_read(nbytes, n=20 if nbytes <= (256 << 20) else 5)
    torch.cuda.empty_cache()
    return float(nbytes) / (ms * 1e-3) / 1e9


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


HOP_MODES = ("plain H", "aux - c H with |.|^2", "CG residual r -= alpha (aux - c g5 H) with |r|^2",
             "FP64 true residual b - (aux - c g5 H) with |.|^2")


def instrumented(lat, bd, kappa, params):
    """One solve with hipEvents around every stencil launch.  `dominant_mode`
    is the stencil variant with the largest summed launch time in the solve."""
    from paper_2409_03030_amd import wdirac as W
    p = W.SolveParams.from_buffer_copy(params)
    p.timing = 1
    x, st = lat.solve(bd, kappa, p)
    s = st[0]
    gbs = s["hop_bytes"] / (s["hop_ms"] * 1e-3) / 1e9
    modes = []
    for m in range(4):
        n, ms, nb = s["hop_mode_launches"][m], s["hop_mode_ms"][m], s["hop_mode_bytes"][m]
        modes.append({"mode": m, "what": HOP_MODES[m], "launches": n, "ms_total": ms,
                      "avg_launch_ms": ms / max(1, n), "bytes_per_launch": nb / max(1, n),
                      "achieved_gbs": nb / (ms * 1e-3) / 1e9 if ms > 0 else 0.0})
    dom = max(range(4), key=lambda m: s["hop_mode_ms"][m])
    return {
        "modes": modes,
        "dominant_mode": dom,
        "hop_ms_total": s["hop_ms"],
        "hop_launches": s["hop_launches"],
        "skipped_launches": s["hop_skipped"],
        "hop_ms_avg": s["hop_ms"] / max(1, s["hop_launches"]),
        "bytes_per_launch": s["hop_bytes"] / max(1, s["hop_launches"]),
        "achieved_gbs": gbs,
        "gflops": FLOP_PER_SITE * s["hop_site_updates"] / (s["hop_ms"] * 1e-3) / 1e9,
        "solve_seconds": s["seconds"],
    }


def inner_delta(inner):
    """Reliable-update threshold of the solves with inner precision `inner`: the
    FP64 true residual is recomputed once the iterated residual has dropped by
    this factor since the last update.  (24^3x48, kappa 0.137, thresholds
    1e-1 .. 1e-3: FP32 inner fastest at 3e-3, 15.6 against 16.4 ms at 1e-2,
    74 iterations either way; FP16 inner 12.2 ms at 1e-2, 11.9 ms at 3e-3 with
    78 iterations and 17.2 ms at 1e-3 with 117, so FP16 keeps 1e-2, which
    leaves a margin for harder systems.)"""
    return {"f64": 0.0, "f32": 3e-3, "f16": 1e-2}[inner]


def hop_bytes_per_site(prec, recon, mode):
    """Algorithmic bytes per output site of one stencil launch at one rhs: 8
    links, the input spinor once, and the epilogue's vectors once each."""
    link = {"f64": 16, "f32": 8, "f16": 4}[prec] * (9 if recon == 18 else 6)
    sp = {"f64": 192, "f32": 96, "f16": 52}[prec]
    acc = {"f64": 192, "f32": 96, "f16": 96}[prec]
    epi = (sp, 2 * sp, sp + 2 * acc, sp + 2 * 192)[mode]  # out | aux, out | aux, r in and out | aux, b, rh
    return 8 * link + sp + epi


def host_cpu():
    """The host's CPU model, sockets, physical cores and the CPUs this process may use."""
    info = {"model": None, "sockets": None, "physical_cores": None, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {l.split(":", 1)[0].strip(): l.split(":", 1)[1].strip() for l in txt.splitlines() if ":" in l}
        info["model"] = kv.get("Model name")
        if kv.get("Socket(s)", "").isdigit():
            info["sockets"] = int(kv["Socket(s)"])
        if info["sockets"] and kv.get("Core(s) per socket", "").isdigit():
            info["physical_cores"] = info["sockets"] * int(kv["Core(s) per socket"])
    except (OSError, ValueError):
        pass
    if info["physical_cores"] is None:
        cores = set()
        phys = None
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and not info["model"]:
                info["model"] = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                cores.add((phys, v))
        info["physical_cores"] = len(cores) or None
    return info


def oracle_threads(host):
    """Threads for the all-cores oracle timing: the physical cores this process
    may run on (at most 16, the host share of one GPU on the measurement box)."""
    n = min(host["usable_cpus"], host["physical_cores"] or host["usable_cpus"])
    return max(1, min(16, n))


def cpu_baseline(U, b, kappa, L, threads):
    """The oracle's A_hat = D_hat^dag D_hat on the host: one application on one
    thread, then `threads` applications at once on as many threads (numpy
    releases the interpreter lock in its array operations; each thread runs
    the unchanged oracle on its own vector), the throughput of all cores."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle as O
    e = O.even_mask(L)
    v = b * e
    half = (L[0] * L[1] * L[2] * L[3]) // 2
    flop = 4 * FLOP_PER_SITE * half
    t0 = time.perf_counter()
    O.apply_Ahat(U, v, kappa, BC)
    t1 = time.perf_counter() - t0
    vs = [v * (1.0 + 0.01 * k) for k in range(threads)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda w: O.apply_Ahat(U, w, kappa, BC), vs))
    tn = time.perf_counter() - t0
    host = host_cpu()
    lat = "x".join(map(str, L))
    return {
        "value": threads * flop / tn / 1e9,
        "unit": "GFLOP/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{threads} concurrent applications of the oracle's D_hat^dag D_hat (4 even-odd hops each, "
                  f"numpy FP64) on the {lat} workload, one per thread, in {tn:.1f} s; and one application on "
                  f"one thread in {t1:.1f} s",
        "single_thread_gflops": flop / t1 / 1e9,
        "seconds_per_DdagD_1_thread": t1,
        "seconds_per_DdagD_all_threads": tn / threads,
        "host": host,
    }


def oracle_residuals(U, L, kappa, cases):
    """err_vs_oracle of each solve: the oracle's FP64 true residual
    ||b - A_hat x|| / ||b|| of the returned x (threads, one case each)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle as O
    with ThreadPoolExecutor(len(cases)) as ex:
        return list(ex.map(lambda xb: float(O.residual_DdagD(U, xb[0], xb[1], kappa, BC, True)), cases))


# The link-load rule of the stencil launcher: links take the non-temporal hint
# (kernel hop_kernel_nt) when the item's link field exceeds 192 MB, or when an
# FP64 launch moves more than 768 MB.
def stencil_kernel_name(prec, recon, mode, split, L):
    half = L[0] * L[1] * L[2] * L[3] // 2
    link = {"f64": 16, "f32": 8, "f16": 4}[prec] * (9 if recon == 18 else 6)
    field = 2 * half * 4 * link
    nt = field > 192e6 or (prec == "f64" and half * hop_bytes_per_site(prec, recon, mode) > 768e6)
    p = {"f64": 0, "f32": 1, "f16": 2}[prec]
    return f"void wd::hop_kernel{'_nt' if nt else ''}<{p}, {recon}, {mode}, {split}>"


WORKLOAD_TEXT = {
    "cfg3": "24^3x48 Wilson-Dirac, U=exp(0.4iH), kappa=0.137, even-odd, plain FP64 CG to true residual 1e-10 "
            "(HBM-resident: the FP64 link field and the CG vectors exceed the 256 MB Infinity Cache)",
    "cfg2": "16^3x32 Wilson-Dirac, U=exp(0.3iH), kappa=0.1365, even-odd, plain FP64 CG to true residual 1e-10 "
            "(cache-resident: the working set fits in the 256 MB Infinity Cache)",
}


def solve_workload(args, name, W, torch, tuned):
    """Plain FP64 CG of one workload as the timed step, then the FP32- and
    FP16-inner solves and the stencil figures.  Returns (result dict, U, b, x)."""
    L, width, kappa, U, b = make_workload(name)
    half = L[0] * L[1] * L[2] * L[3] // 2
    dev = "cuda:0"
    Ud = torch.from_numpy(U).to(dev)
    bd = torch.from_numpy(b).to(dev)
    lat = W.Lattice(L, BC)
    # plain FP64 CG with recon-18 and recon-12 FP64 links (both exact FP64
    # arithmetic; recon-12 rebuilds the third row, error ~1e-16); the one with
    # the faster stencil is the headline
    links = {}
    for recon in (18, 12):
        lat.set_gauge(Ud, "f64", recon)
        if not tuned:
            sb, sw, sp = lat.autotune("f64", 1)
            log(f"{name} autotune f64-{recon}: sites/block {sb}, xcd swizzle {sw}, hop split {sp}")
        links[recon] = lat.time_hop("f64", 1, n=50)
    recon64 = min(links, key=links.get)
    lat.set_gauge(Ud, "f64", recon64)
    lat.set_gauge(Ud, "f32", 12)
    lat.set_gauge(Ud, "f16", 12)
    for prec in ("f32", "f16"):
        if not tuned:
            sb, sw, sp = lat.autotune(prec, 1)
            log(f"{name} autotune {prec}: sites/block {sb}, xcd swizzle {sw}, hop split {sp}")
    split64 = next(int(l.split()[9]) for l in W.tune_export().splitlines()
                   if l.split()[:7] == [str(v) for v in (*L, 0, recon64, 1)])
    torch.cuda.synchronize()

    plain = W.default_params()  # EO, FP64 inner, tol 1e-10
    log(f"{name}: timing plain FP64 CG (f64 links recon-{recon64}) ...")
    x, st, dt = time_solves(lat, Ud, bd, kappa, plain, args.steps, args.warmup, set_gauge=[("f64", recon64)])
    if st["status"] != 0 or st["true_resid"] > 1e-10:
        raise SystemExit(f"plain CG failed: {st}")
    roof = instrumented(lat, bd, kappa, plain)
    log(f"{name} plain FP64: {st['iters']} iters, {dt * 1e3:.2f} ms, stencil {roof['achieved_gbs']:.0f} GB/s")
    xs = {"f64": x}
    mixed = {}
    for inner in ("f32", "f16"):
        p = W.default_params(inner=inner, delta=inner_delta(inner))
        xm, sm, dtm = time_solves(lat, Ud, bd, kappa, p, max(3, args.steps), 1)
        if sm["status"] != 0:
            raise SystemExit(f"{inner} CG failed: {sm}")
        rm = instrumented(lat, bd, kappa, p)
        xs[inner] = xm
        mixed[inner] = {
            "time_to_solution_ms": dtm * 1e3,
            "iters": sm["iters"],
            "reliable_updates": sm["reliable_updates"],
            "true_resid": sm["true_resid"],
            "rel_diff_vs_plain_fp64_x": (torch.linalg.vector_norm(xm - x) / torch.linalg.vector_norm(x)).item(),
            "stencil_gbs": rm["achieved_gbs"],
            "stencil_ms_avg": rm["hop_ms_avg"],
            "stencil_note": "all stencil launches of the event-timed solve (inner precision and the FP64 "
                            "reliable updates): algorithmic bytes over summed durations; the inner link field "
                            "and vectors (at 24^3x48 FP32-12 links 127 MB, FP16-12 64 MB) partly stay in the "
                            "Infinity Cache, so this is not an HBM figure",
            "dw_gflops": dw_flops(sm, half) / dtm / 1e9,
            "speedup_vs_plain_fp64": dt / dtm,
        }
        log(f"{name} {inner} inner: {sm['iters']} iters, {dtm * 1e3:.2f} ms, stencil {rm['achieved_gbs']:.0f} GB/s")

    # The roofline kernel: the stencil variant with the largest share of the
    # plain FP64 solve, timed back to back in the launch shape of the CG; the
    # fused CG-residual stencil beside it.
    dom = roof["dominant_mode"]
    if dom > 2:
        raise SystemExit(f"unexpected dominant stencil mode {dom}")
    lname = "x".join(map(str, L))
    kernel_name = stencil_kernel_name("f64", recon64, dom, split64, L)
    dom_ms = lat.time_hop("f64", 1, n=200, mode=dom)
    dom_bytes = half * hop_bytes_per_site("f64", recon64, dom)
    cgr_name = stencil_kernel_name("f64", recon64, 2, split64, L)
    cgr_ms = lat.time_hop("f64", 1, n=200, mode=2)
    cgr_bytes = half * hop_bytes_per_site("f64", recon64, 2)
    # the four stencil launches of one CG iteration (D_hat^dag D_hat with the
    # fused epilogues), in order, back to back
    seq_ms = lat.time_hop("f64", 1, n=50, mode=4)
    seq_bytes = half * (2 * hop_bytes_per_site("f64", recon64, 0) + hop_bytes_per_site("f64", recon64, 1)
                        + hop_bytes_per_site("f64", recon64, 2))
    roofline = {
        "bound": "hbm",
        "achieved": dom_bytes / (dom_ms * 1e-3) / 1e9,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": dom_bytes / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "traffic": lookup_traffic(kernel_name, lname),
        "kernel": kernel_name,
        "what": HOP_MODES[dom],
        "avg_launch_ms": dom_ms,
        "bytes_per_launch": dom_bytes,
        "bytes_per_site": dom_bytes / half,
        "output_sites_per_launch": half,
        "in_solve": {"by_mode": roof["modes"],
                     "skipped_launches": roof["skipped_launches"],
                     "note": "hipEvents around each launch of one plain FP64 solve (event-to-event, so "
                             "each launch also carries its dispatch latency); launches whose slots all "
                             "skipped their work (flagged by the kernels) are left out"},
        "cg_residual_stencil": {
            "kernel": cgr_name, "avg_launch_ms": cgr_ms, "bytes_per_launch": cgr_bytes,
            "achieved": cgr_bytes / (cgr_ms * 1e-3) / 1e9,
            "frac": cgr_bytes / (cgr_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "traffic": lookup_traffic(cgr_name, lname)},
        "cg_iteration_stencils": {
            "what": "the 4 stencil launches of one CG iteration on D_hat^dag D_hat in order (plain H, aux - cH "
                    "with |.|^2, plain H, CG residual update with |r|^2), repeated 50 times back to back "
                    "(reductions' stage 1 included; stage 2 and the vector update not)",
            "avg_ms": seq_ms, "bytes": seq_bytes,
            "achieved": seq_bytes / (seq_ms * 1e-3) / 1e9,
            "frac": seq_bytes / (seq_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "all_stencil_launches": {"achieved_gbs": roof["achieved_gbs"], "avg_launch_ms": roof["hop_ms_avg"],
                                 "launches": roof["hop_launches"], "gflops": roof["gflops"]},
    }
    res = {
        "workload": WORKLOAD_TEXT[name], "lattice": list(L), "kappa": kappa, "link_width": width,
        "links": f"f64 recon-{recon64}", "time_to_solution_ms": dt * 1e3, "solves_per_s": 1.0 / dt,
        "iters": st["iters"], "reliable_updates": st["reliable_updates"], "true_resid": st["true_resid"],
        "dw_gflops": dw_flops(st, half) / dt / 1e9, "roofline": roofline, "mixed_precision": mixed,
    }
    xs = {k: v.cpu().numpy() for k, v in xs.items()}
    lat.close()
    del Ud, bd
    torch.cuda.empty_cache()
    return res, U, b, xs


def bench_default(args):
    import torch
    from paper_2409_03030_amd import wdirac as W

    tuned = args.tune_file is not None
    if tuned:
        W.tune_import(open(args.tune_file).read())
    name = args.workload
    log(f"generating the {name} workload ...")
    res, U, b, xs = solve_workload(args, name, W, torch, tuned)
    if args.save_tune:
        open(args.save_tune, "w").write(W.tune_export())
    copy_gbs = calibration_copy()
    read_gbs = read_bandwidth()
    read128_gbs = read_bandwidth(128 << 20)
    res["roofline"]["attainable_read_gbs"] = {"1GiB": read_gbs, "128MiB": read128_gbs,
                                             "note": "plain streaming-read kernel on the same box"}
    other = None
    if name == "cfg3" and not args.no_cfg2:
        log("the cache-resident 16^3x32 workload beside it ...")
        other, _, _, _ = solve_workload(args, "cfg2", W, torch, tuned)
    L = tuple(res["lattice"])
    kappa = res["kappa"]
    cpu = None
    if not args.no_cpu_baseline:
        host = host_cpu()
        nt = oracle_threads(host)
        log(f"oracle residuals of the returned solutions and the oracle timing ({nt} threads) ...")
        errs = oracle_residuals(U, L, kappa, [(xs[k], b) for k in ("f64", "f32", "f16")])
        res["err_vs_oracle"] = errs[0]
        res["mixed_precision"]["f32"]["err_vs_oracle"] = errs[1]
        res["mixed_precision"]["f16"]["err_vs_oracle"] = errs[2]
        cpu = cpu_baseline(U, b, kappa, L, nt)
        cpu["oracle_time_to_solution_est_s"] = cpu["seconds_per_DdagD_1_thread"] * (res["iters"] +
                                                                                     res["reliable_updates"])
        cpu["oracle_time_to_solution_note"] = ("estimate: CG iterations of the GPU solve x the oracle's time per "
                                               "D_hat^dag D_hat on one thread (vector updates not counted)")
    out = {
        "metric": METRIC,
        "value": res["dw_gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["time_to_solution_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": res["workload"],
            "lattice": list(L),
            "kappa": kappa,
            "link_width": res["link_width"],
            "boundary": "antiperiodic t",
            "precond": "even-odd",
            "inner": "f64",
            "links": res["links"],
        },
        "time_to_solution_ms": res["time_to_solution_ms"],
        "solves_per_s": res["solves_per_s"],
        "iters": res["iters"],
        "reliable_updates": res["reliable_updates"],
        "true_resid": res["true_resid"],
        "err_vs_oracle": res.get("err_vs_oracle"),
        "roofline": res["roofline"],
        "copy_1GiB_gbs": copy_gbs,
        "read_1GiB_gbs": read_gbs,
        "read_128MiB_gbs": read128_gbs,
        "mixed_precision": res["mixed_precision"],
        "cache_resident_16x16x16x32": other,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# other workloads
# ---------------------------------------------------------------------------
def _common_out(args, metric_value, unit, ms_per_step, dtype, config, extra):
    out = {
        "metric": METRIC,
        "value": metric_value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
    }
    out.update(extra)
    return out


def bench_cfg1(args):
    """4^4 Haar links, kappa 0.12, unpreconditioned: D once + plain FP64 CG."""
    import torch
    import qcdgen
    from paper_2409_03030_amd import wdirac as W
    L, kappa = (4, 4, 4, 4), 0.12
    U = qcdgen.links_haar(L, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 0))
    b = qcdgen.gaussian_spinor(L, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 100))
    Ud, bd = torch.from_numpy(U).cuda(), torch.from_numpy(b).cuda()
    lat = W.Lattice(L, BC)
    lat.set_gauge(Ud, "f64", 18)
    p = W.default_params(precond=W.FULL)
    y = lat.apply_D(bd, kappa, precond=W.FULL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(100):
        lat.apply_D(bd, kappa, precond=W.FULL, out=y)
    torch.cuda.synchronize()
    d_ms = (time.perf_counter() - t0) / 100 * 1e3
    x, st, dt = time_solves(lat, Ud, bd, kappa, p, args.steps, args.warmup)
    V = 256
    return _common_out(args, dw_flops(st, V // 2, eo=False) / dt / 1e9, "GFLOP/s", dt * 1e3, "f64",
                       {"workload": "4^4 Haar SU(3), kappa=0.12, unpreconditioned, plain FP64 CG to 1e-10",
                        "lattice": list(L), "kappa": kappa},
                       {"time_to_solution_ms": dt * 1e3, "iters": st["iters"], "true_resid": st["true_resid"],
                        "apply_D_ms": d_ms, "note": "latency-bound (128 sites per parity); not a roofline point"})


def bench_cfg4(args):
    """16^3x32, 12 point sources per kappa in one batched solve (FP32 inner, FP64 outer).
    --rhs-group G solves the 12 sources as 12/G slots of G right-hand sides in
    the same launches (0: the library's default)."""
    import torch
    import qcdgen
    from paper_2409_03030_amd import wdirac as W
    L, width, kappa0, U, b = make_workload("cfg2")
    half = L[0] * L[1] * L[2] * L[3] // 2
    Ud = torch.from_numpy(U).cuda()
    B = torch.from_numpy(qcdgen.point_sources(L)).cuda()
    lat = W.Lattice(L, BC)
    G = args.rhs_group if args.rhs_group > 0 else 4
    for prec, recon in (("f64", 18), ("f32", args.inner_recon)):
        lat.set_gauge(Ud, prec, recon)
        if args.tune_file:
            continue
        for nrhs in sorted({1, G}):
            sb, sw, sp = lat.autotune(prec, nrhs)
            log(f"autotune {prec} nrhs {nrhs}: sites/block {sb}, swizzle {sw}, split {sp}")
    p = W.default_params(inner="f32", delta=inner_delta("f32"), rhs_group=args.rhs_group)
    p1 = W.default_params(inner="f32", delta=inner_delta("f32"))
    res = {}
    tot_batched = tot_single = 0.0
    flops = 0.0
    for kappa in (0.130, 0.134, 0.1365):
        lat.solve(B, [kappa] * 12, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            X, st = lat.solve(B, [kappa] * 12, p)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / args.steps
        t0 = time.perf_counter()
        for r in range(12):
            lat.solve(B[r].contiguous(), kappa, p1)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        its = [s["iters"] for s in st]
        flops += sum(dw_flops(s, half) for s in st)
        tot_batched += tb
        tot_single += ts
        res[str(kappa)] = {"batched_12rhs_ms": tb * 1e3, "sequential_12_single_ms": ts * 1e3,
                           "speedup_batched": ts / tb, "iters_min": min(its), "iters_max": max(its),
                           "all_converged": all(s["status"] == 0 for s in st),
                           "max_true_resid": max(s["true_resid"] for s in st)}
        log(f"kappa {kappa}: 12 rhs batched {tb * 1e3:.1f} ms vs sequential {ts * 1e3:.1f} ms, iters {min(its)}..{max(its)}")
    # stress run: the 36 sources of the three kappas in one solve (kappa is per rhs)
    B36 = torch.cat([B, B, B], 0).contiguous()
    k36 = [0.130] * 12 + [0.134] * 12 + [0.1365] * 12
    lat.solve(B36, k36, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        X36, st36 = lat.solve(B36, k36, p)
    torch.cuda.synchronize()
    t36 = (time.perf_counter() - t0) / args.steps
    stress = {"ms": t36 * 1e3, "three_12rhs_batches_ms": tot_batched * 1e3,
              "all_converged": all(s["status"] == 0 for s in st36),
              "max_true_resid": max(s["true_resid"] for s in st36),
              "iters_by_kappa": {str(k): [s["iters"] for s, kk in zip(st36, k36) if kk == k][:1][0]
                                 for k in (0.130, 0.134, 0.1365)}}
    log(f"36 rhs, mixed kappa, one solve: {t36 * 1e3:.1f} ms vs three 12-rhs solves {tot_batched * 1e3:.1f} ms")
    # The 12-rhs stencil against the roofline: the plain hop H_oe over all 12
    # sources (one launch of 12/G slots), event-timed inside one solve, against
    # the algorithmic bytes of 12 sources sharing one read of the links:
    # 8 FP32-12 links (384 B; 576 B at recon 18) per site plus
    # 12 x (96 B in + 96 B out), i.e. 224 B (240 B) per site and source.
    pt = W.SolveParams.from_buffer_copy(p)
    pt.timing = 1
    X, st = lat.solve(B, [0.1365] * 12, pt)
    s0 = st[0]
    m0 = s0["hop_inner_mode_launches"][0]
    ms0 = s0["hop_inner_mode_ms"][0] / max(1, m0)
    ideal = half * (8 * (48 if args.inner_recon == 12 else 72) + 12 * 192)
    roof = {"bound": "hbm", "what": "FP32 plain hop H_oe over the 12 sources, event-timed in the solve (each "
                                     "launch also carries its dispatch latency; launches whose slots all skipped "
                                     "their work left out, launches that skipped some converged sources counted "
                                     "with every source's bytes)",
            "avg_launch_ms": ms0, "bytes_per_launch_12rhs_links_once": ideal, "bytes_per_site_rhs": ideal / half / 12,
            "achieved": ideal / (ms0 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ideal / (ms0 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "library_bytes_per_launch": s0["hop_inner_mode_bytes"][0] / max(1, m0),
            "note": f"{12 // G} slot(s) of {G} sources: the library's own count reads the links once per slot",
            "all_stencil_launches_gbs": s0["hop_bytes"] / (s0["hop_ms"] * 1e-3) / 1e9,
            "links": f"f32 recon-{args.inner_recon}",
            "cache_resident": "the 16^3x32 FP32 link field (25 MB) fits in the 256 MB Infinity Cache, the 12 "
                              "sources' inner-loop vectors (378 MB) partly"}
    return _common_out(args, flops / tot_batched / 1e9, "GFLOP/s", tot_batched / 3 * 1e3, "f32",
                       {"workload": "16^3x32, 12 spin-colour point sources per kappa in one batched CG launch, "
                                    "kappa in {0.130, 0.134, 0.1365}, complex64 inner / complex128 outer",
                        "lattice": list(L), "nrhs": 12, "rhs_group": G},
                       {"per_kappa": res, "speedup_batched_vs_sequential": tot_single / tot_batched,
                        "mixed_kappa_36rhs": stress, "stencil_12rhs": roof})


def bench_pion(args):
    """16^3x32 (the cfg2 field), kappa 0.1365: the 12 point-source propagators by
    the even-odd D x = b solve and the zero-momentum pion correlator."""
    import numpy as np
    import torch
    from paper_2409_03030_amd import wdirac as W
    L, width, kappa, U, _ = make_workload("cfg2")
    half = L[0] * L[1] * L[2] * L[3] // 2
    Ud = torch.from_numpy(U).cuda()
    lat = W.Lattice(L, BC)
    for prec in ("f64", "f32", "f16"):
        lat.set_gauge(Ud, prec, 12)
        if args.tune_file:
            continue
        for nrhs in (1, 4):
            lat.autotune(prec, nrhs)
    res = {}
    for inner in ("f32", "f16", "f64"):
        p = W.default_params(inner=inner, delta=inner_delta(inner))
        for _ in range(max(1, args.warmup)):
            S, st = lat.propagator(kappa, params=p)
            lat.pion_correlator(S)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            S, st = lat.propagator(kappa, params=p)
            torch.cuda.synchronize()
        tprop = (time.perf_counter() - t0) / args.steps
        t0 = time.perf_counter()
        n_c = 20
        for _ in range(n_c):
            C = lat.pion_correlator(S)
        tcorr = (time.perf_counter() - t0) / n_c
        res[inner] = {"propagators_ms": tprop * 1e3, "correlator_ms": tcorr * 1e3,
                      "time_to_correlator_ms": (tprop + tcorr) * 1e3,
                      "iters": [s["iters"] for s in st], "all_converged": all(s["status"] == 0 for s in st),
                      "dw_gflops": sum(dw_flops(s, half) for s in st) / tprop / 1e9,
                      "correlator": [float(v) for v in C]}
        log(f"pion, {inner} inner: 12 propagators {tprop * 1e3:.1f} ms, correlator {tcorr * 1e3:.2f} ms, "
            f"iters {min(res[inner]['iters'])}..{max(res[inner]['iters'])}")
    best = min(res, key=lambda k: res[k]["time_to_correlator_ms"])
    C = np.array(res[best]["correlator"])
    meff = [float(np.log(C[t] / C[t + 1])) for t in range(len(C) // 2)]
    return _common_out(args, res[best]["dw_gflops"], "GFLOP/s", res[best]["time_to_correlator_ms"], best,
                       {"workload": "16^3x32, U=exp(0.3iH), kappa=0.1365: 12 point-source propagators by the "
                                    "even-odd D x = b solve (one batched solve), then the zero-momentum pion "
                                    "correlator", "lattice": list(L), "nrhs": 12, "best_inner": best},
                       {"by_inner": res, "effective_mass_log_ratio": meff})


def bench_force(args):
    """16^3x32 (the cfg2 field), kappa 0.1365: pseudofermion heatbath eta = D^dag xi,
    then the action and the force U dS_f/dU (two D x = b solves and the force kernel)."""
    import numpy as np
    import torch
    import qcdgen
    from paper_2409_03030_amd import wdirac as W
    L, width, kappa, U, _ = make_workload("cfg2")
    half = L[0] * L[1] * L[2] * L[3] // 2
    Ud = torch.from_numpy(U).cuda()
    lat = W.Lattice(L, BC)
    for prec in ("f64", "f32", "f16"):
        lat.set_gauge(Ud, prec, 12)
        lat.autotune(prec, 1)
    xi = torch.from_numpy(qcdgen.gaussian_spinor(L, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 5))).cuda()
    eta = lat.pseudofermion(xi, kappa)
    xx = float(torch.vdot(xi.flatten(), xi.flatten()).real)
    res = {}
    for inner in ("f32", "f16", "f64"):
        p = W.default_params(inner=inner, delta=inner_delta(inner))
        for _ in range(max(1, args.warmup)):
            lat.fermion_force(eta, kappa, params=p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            F, S, st = lat.fermion_force(eta, kappa, params=p)
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t0) / args.steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, Sa, _ = lat.fermion_force(eta, kappa, params=p, force=False)
        torch.cuda.synchronize()
        ta = (time.perf_counter() - t0) / args.steps
        res[inner] = {"force_and_action_ms": tf * 1e3, "action_only_ms": ta * 1e3,
                      "iters": [st[0]["iters"], st[1]["iters"]],
                      "action_rel_to_xi2": S / xx - 1.0,
                      "dw_gflops": (dw_flops(st[0], half) + dw_flops(st[1], half)) / tf / 1e9,
                      "force_norm": float(torch.linalg.vector_norm(F).item())}
        log(f"force, {inner} inner: {tf * 1e3:.1f} ms (action alone {ta * 1e3:.1f} ms), "
            f"S/xi^2 - 1 = {S / xx - 1.0:.2e}, iters {st[0]['iters']}+{st[1]['iters']}")
    best = min(res, key=lambda k: res[k]["force_and_action_ms"])
    return _common_out(args, res[best]["dw_gflops"], "GFLOP/s", res[best]["force_and_action_ms"], best,
                       {"workload": "16^3x32, U=exp(0.3iH), kappa=0.1365: pseudofermion action "
                                    "eta^dag (D^dag D)^-1 eta and force U dS/dU for eta = D^dag xi "
                                    "(two even-odd D x = b solves and the force kernel)",
                        "lattice": list(L), "best_inner": best},
                       {"by_inner": res})


def bench_staggered(args):
    """16^3x32 (the cfg2 field), staggered operator with mass 0.1: D x = b by the
    even-odd CG on M_e = m^2 - H_eo H_oe, plain FP64 and FP32 inner iterations."""
    import numpy as np
    import torch
    import qcdgen
    from paper_2409_03030_amd import wdirac as W
    L, width, _, U, _ = make_workload("cfg2")
    mass = 0.1
    half = L[0] * L[1] * L[2] * L[3] // 2
    Ud = torch.from_numpy(U).cuda()
    lat = W.Lattice(L, BC)
    for prec in ("f64", "f32"):
        lat.set_gauge(Ud, prec, 12)
        if args.stag_shape:
            sb, sw, sp = (int(v) for v in args.stag_shape.split(","))
            lat.stag_set_shape(prec, 1, sb, sw, sp)
            log(f"staggered shape {prec} (given): sites/block {sb}, xcd swizzle {sw}, split {sp}")
        else:
            sb, sw, sp = lat.stag_autotune(prec, 1)
            log(f"staggered autotune {prec}: sites/block {sb}, xcd swizzle {sw}, split {sp}")
    g = qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 6)
    shape = qcdgen.site_shape(L) + (3,)
    b = torch.from_numpy(g.standard_normal(shape) + 1j * g.standard_normal(shape)).cuda()
    res = {}
    for inner in ("f64", "f32"):
        p = W.default_params(inner=inner, delta=inner_delta(inner))
        for _ in range(max(1, args.warmup)):
            lat.stag_solve(b, mass, params=p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x, st = lat.stag_solve(b, mass, params=p)
        torch.cuda.synchronize()
        tt = (time.perf_counter() - t0) / args.steps
        pt = W.SolveParams.from_buffer_copy(p)
        pt.timing = 1
        _, sti = lat.stag_solve(b, mass, params=pt)
        s0 = sti[0]
        n = st[0]["iters"] + st[0]["reliable_updates"]
        res[inner] = {"time_to_solution_ms": tt * 1e3, "iters": st[0]["iters"],
                      "reliable_updates": st[0]["reliable_updates"], "true_resid": st[0]["true_resid"],
                      "dw_gflops": 570.0 * half * 2 * n / tt / 1e9,
                      "stencil_gbs": s0["hop_bytes"] / (s0["hop_ms"] * 1e-3) / 1e9,
                      "stencil_ms_avg": s0["hop_ms"] / max(1, s0["hop_launches"])}
        log(f"staggered, {inner} inner: {st[0]['iters']} iters, {tt * 1e3:.2f} ms, "
            f"stencil {res[inner]['stencil_gbs']:.0f} GB/s")
    best = min(res, key=lambda k: res[k]["time_to_solution_ms"])
    # Goldstone pion: the 3 colour point-source propagators (one 3-field solve)
    # and the correlator, with the faster inner precision.
    sb, sw, sp = lat.stag_autotune(best, 3)
    log(f"staggered autotune {best}, 3 fields: sites/block {sb}, xcd swizzle {sw}, split {sp}")
    p = W.default_params(inner=best, delta=inner_delta(best))
    for _ in range(max(1, args.warmup)):
        G, st = lat.stag_propagator(mass, params=p)
        lat.stag_pion_correlator(G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G, st = lat.stag_propagator(mass, params=p)
    torch.cuda.synchronize()
    tprop = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(20):
        C = lat.stag_pion_correlator(G)
    tcorr = (time.perf_counter() - t0) / 20
    pion = {"inner": best, "propagators_ms": tprop * 1e3, "correlator_ms": tcorr * 1e3,
            "iters": [s["iters"] for s in st], "all_converged": all(s["status"] == 0 for s in st),
            "correlator": [float(v) for v in C]}
    log(f"staggered pion, {best} inner: 3 propagators {tprop * 1e3:.2f} ms, correlator {tcorr * 1e3:.3f} ms")
    return _common_out(args, res[best]["dw_gflops"], "GFLOP/s", res[best]["time_to_solution_ms"], best,
                       {"workload": "16^3x32, U=exp(0.3iH), staggered mass 0.1, even-odd CG on m^2 - H_eo H_oe "
                                    "to true residual 1e-10, then x_o", "lattice": list(L), "mass": mass,
                        "best_inner": best},
                       {"by_inner": res, "flop_per_site": 570, "pion": pion})


def bench_cfg5(args):
    """Served stream: Poisson arrivals at 50/s over four lattice sizes, continuous
    batching.  The requests arriving in the first warmup_s seconds are served
    but not counted; latency percentiles and throughput come from the next
    `requests` arrivals.  The offered load rho = lambda E[S] takes E[S] from
    each request's solve alone (its field's alone time at three kappa,
    interpolated in kappa)."""
    import threading
    import numpy as np
    import torch
    import qcdgen
    from paper_2409_03030_amd import wdirac as W
    sizes = [(8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32), (24, 24, 24, 48)]
    g = qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 4)
    fields = []   # resident gauge fields: (lattice, width)
    log("generating resident gauge fields ...")
    for L in sizes:
        for k in range(2 if L != (24, 24, 24, 48) else 1):
            w = float(g.uniform(0.2, 0.5))
            U = torch.from_numpy(qcdgen.links_exp(L, w, g)).cuda()
            lat = W.Lattice(L, BC)
            for prec, recon in (("f64", 18), ("f32", 12), ("f16", 12)):
                lat.set_gauge(U, prec, recon)
            del U
            fields.append((lat, w))
    rate = args.rate
    n_warm = int(round(args.warmup_s * rate))
    n_req = args.requests
    n_tot = n_warm + n_req
    arrivals = np.cumsum(g.exponential(1.0 / rate, n_tot))
    pick_f = [int(g.integers(0, len(fields))) for _ in range(n_tot)]
    pick_k = [float(g.uniform(0.12, 0.136)) for _ in range(n_tot)]
    sources = {}
    for fi in pick_f:
        lat = fields[fi][0]
        if lat.L not in sources:
            sources[lat.L] = [torch.from_numpy(qcdgen.gaussian_spinor(lat.L, g)).cuda() for _ in range(4)]
    torch.cuda.synchronize()
    kgrid = (0.12, 0.128, 0.136)

    def service_times(params):
        """Alone solve time of each field at the kappa grid (median of 3)."""
        t = []
        for lat, _ in fields:
            b = sources[lat.L][0]
            row = []
            for k in kgrid:
                lat.solve(b, k, params)
                ts = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    lat.solve(b, k, params)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                row.append(float(np.median(ts)))
            t.append(row)
        return t

    def run(params, label):
        talone = service_times(params)
        es = float(np.mean([np.interp(pick_k[i], kgrid, talone[pick_f[i]]) for i in range(n_warm, n_tot)]))
        free, total = torch.cuda.mem_get_info()
        pool = int(min(24 << 30, free * 0.5))
        srv = W.Server(pool, max_slots=16, params=params)
        done = {}
        tickets = []
        t_start = time.perf_counter()

        def submit_all():
            for i in range(n_tot):
                lat = fields[pick_f[i]][0]
                while time.perf_counter() - t_start < arrivals[i]:
                    time.sleep(0.0002)
                b = sources[lat.L][i % 4]
                t = srv.submit(lat, b, pick_k[i])
                tickets.append((t, i))
        th = threading.Thread(target=submit_all)
        th.start()
        pending = {}
        k = 0
        while len(done) < n_tot:
            while k < len(tickets):
                t, i = tickets[k]
                pending[t] = i
                k += 1
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    i = pending.pop(t)
                    done[i] = (time.perf_counter() - t_start, r[1][0])
            time.sleep(0.0005)
        th.join()
        srv.close()
        meas = range(n_warm, n_tot)
        lat_ms = np.array([(done[i][0] - arrivals[i]) * 1e3 for i in meas])
        t_first = arrivals[n_warm]
        t_last = max(done[i][0] for i in meas)
        ok = all(done[i][1]["status"] == 0 for i in range(n_tot))
        resid = max(done[i][1]["true_resid"] for i in range(n_tot))
        by_size = {}
        for i in meas:
            key = "x".join(map(str, fields[pick_f[i]][0].L))
            by_size.setdefault(key, []).append((done[i][0] - arrivals[i]) * 1e3)
        out = {"requests_measured": n_req, "warmup_requests": n_warm, "warmup_s": args.warmup_s,
               "offered_rate_per_s": rate, "mean_alone_service_ms": es * 1e3, "offered_load_rho": rate * es,
               "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
               "mean_ms": float(lat_ms.mean()), "max_ms": float(lat_ms.max()),
               "solves_per_s": n_req / (t_last - t_first), "all_converged": ok, "max_true_resid": resid,
               "alone_ms_by_field": {"x".join(map(str, fields[f][0].L)) + f"#{f}": [v * 1e3 for v in talone[f]]
                                     for f in range(len(fields))},
               "p50_p99_ms_by_size": {kk: [float(np.percentile(v, 50)), float(np.percentile(v, 99))]
                                      for kk, v in sorted(by_size.items())}}
        log(f"{label}: rho {out['offered_load_rho']:.2f}, p50 {out['p50_ms']:.1f} ms, p99 {out['p99_ms']:.1f} ms, "
            f"{out['solves_per_s']:.1f} solves/s")
        return out

    which = set(args.served.split(","))
    runs = {}
    if "f16" in which:
        runs["served_fp16_inner"] = run(W.default_params(inner="f16", delta=inner_delta("f16")), "served, FP16 inner")
    if "f32" in which:
        runs["served_fp32_inner"] = run(W.default_params(inner="f32", delta=inner_delta("f32")), "served, FP32 inner")
    if "f64" in which:
        runs["served_plain_fp64"] = run(W.default_params(), "served, plain FP64")
    if not runs:
        raise SystemExit("--served names none of f16, f32, f64")
    bk = min(runs, key=lambda k: runs[k]["p99_ms"])
    best = runs[bk]
    dt = {"served_fp16_inner": "f16", "served_fp32_inner": "f32", "served_plain_fp64": "f64"}[bk]
    return _common_out(args, best["solves_per_s"], "solves/s", best["mean_ms"], dt,
                       {"workload": f"served stream: Poisson arrivals at {rate}/s, lattices uniform over "
                                    "{8^4, 12^3x24, 16^3x32, 24^3x48}, kappa U[0.12,0.136], link width U[0.2,0.5], "
                                    "Gaussian sources, each to 1e-10, admission by HBM footprint; "
                                    f"{n_req} requests measured after a {args.warmup_s:g} s warm-up",
                        "requests": n_req},
                       dict(runs, p99_ms=best["p99_ms"], p50_ms=best["p50_ms"]))


def bench_stencil(args):
    """The stencil alone: n launches of the inner-iteration hop on a lattice, plus
    a device copy of known size (the calibration reference for HBM counters)."""
    import torch
    import qcdgen
    from paper_2409_03030_amd import wdirac as W
    L = tuple(int(v) for v in args.lattice.split(","))
    U = torch.from_numpy(qcdgen.links_exp(L, 0.4, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 2))).cuda()
    lat = W.Lattice(L, BC)
    half = L[0] * L[1] * L[2] * L[3] // 2
    res = {}
    for prec, recon in (("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12), ("f16", 18), ("f16", 12)):
        lat.set_gauge(U, prec, recon)
        sb, sw, sp = lat.autotune(prec, 1)
        ms = lat.time_hop(prec, 1, n=args.steps * 20)
        link = {"f64": 16, "f32": 8, "f16": 4}[prec] * (9 if recon == 18 else 6)
        sp_b = {"f64": 192, "f32": 96, "f16": 52}[prec]
        nbytes = half * (8 * link + 2 * sp_b)
        res[f"{prec}-{recon}"] = {"ms": ms, "bytes_per_launch": nbytes, "gbs": nbytes / (ms * 1e-3) / 1e9,
                                  "gflops": FLOP_PER_SITE * half / (ms * 1e-3) / 1e9,
                                  "shape": {"sites_per_block": sb, "swizzle": sw, "split": sp}}
        log(f"stencil {prec}-{recon}: {ms * 1e3:.1f} us, {res[f'{prec}-{recon}']['gbs']:.0f} GB/s")
    # calibration copy: 1 GiB read + 1 GiB written
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    cp = (time.perf_counter() - t0) / 5
    res["copy_1GiB"] = {"ms": cp * 1e3, "gbs_read_plus_write": 2 * (1 << 30) / cp / 1e9}
    del a, b
    torch.cuda.empty_cache()
    res["read_1GiB_gbs"] = read_bandwidth()
    best = res["f64-18"]
    return _common_out(args, best["gbs"], "GB/s", best["ms"], "f64",
                       {"workload": f"stencil only: one even-odd hop (V/2 output sites) on {'x'.join(map(str, L))}"},
                       {"stencil": res})


def bench_oracle(args):
    """The CPU oracle on every workload lattice, on this host's cores: one
    D_hat^dag D_hat (D^dag D on the full 4^4 lattice) on one thread, the
    throughput of one application per thread on all physical cores, and
    oracle CG solves to 1e-10 where they take seconds (4^4 unpreconditioned,
    8^4 even-odd); the longer solves are estimated as iterations x time per
    application (iterations from the GPU solves of the same workloads)."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle as O
    import qcdgen
    host = host_cpu()
    nt = oracle_threads(host)
    cases = [("cfg1 4^4 Haar, unpreconditioned", (4, 4, 4, 4), "haar", 0.12, False, qcdgen.CONFIG_SEED_BASE),
             ("cfg5 8^4", (8, 8, 8, 8), 0.35, 0.128, True, 7),
             ("cfg5 12^3x24", (12, 12, 12, 24), 0.35, 0.128, True, 8),
             ("cfg2/cfg4 16^3x32", (16, 16, 16, 32), 0.3, 0.1365, True, qcdgen.CONFIG_SEED_BASE + 1),
             ("cfg3 24^3x48", (24, 24, 24, 48), 0.4, 0.137, True, qcdgen.CONFIG_SEED_BASE + 2)]
    res = {}
    for label, L, w, kappa, eo, seed in cases:
        g = qcdgen.rng(seed)
        U = qcdgen.links_haar(L, g) if w == "haar" else qcdgen.links_exp(L, w, g)
        b = qcdgen.gaussian_spinor(L, g)
        V = L[0] * L[1] * L[2] * L[3]
        if eo:
            v = b * O.even_mask(L)
            op = lambda x: O.apply_Ahat(U, x, kappa, BC)
            flop = 4 * FLOP_PER_SITE * (V // 2)
        else:
            v = b
            op = lambda x: O.apply_DdagD(U, x, kappa, BC)
            flop = 2 * FLOP_PER_SITE * V
        ts = []
        t_all = time.perf_counter()
        while len(ts) < 5 and (not ts or time.perf_counter() - t_all < 20.0):
            t0 = time.perf_counter()
            op(v)
            ts.append(time.perf_counter() - t0)
        t1 = float(np.median(ts))
        vs = [v * (1.0 + 0.01 * k) for k in range(nt)]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(op, vs))
        tn = time.perf_counter() - t0
        r = {"lattice": list(L), "kappa": kappa, "operator": "D_hat^dag D_hat (even-odd)" if eo else "D^dag D (full)",
             "seconds_1_thread": t1, "gflops_1_thread": flop / t1 / 1e9,
             "threads": nt, "gflops_all_threads": nt * flop / tn / 1e9}
        if V <= 4096:
            t0 = time.perf_counter()
            x, info = O.solve_DdagD(U, b, kappa, BC, eo=eo)
            r["cg_to_1e-10_seconds"] = time.perf_counter() - t0
            r["cg_iterations"] = info["iters"]
            r["cg_true_residual"] = float(O.residual_DdagD(U, x, b, kappa, BC, eo))
        res[label] = r
        log(f"oracle {label}: {t1:.3f} s per application on 1 thread ({r['gflops_1_thread']:.3f} GFLOP/s), "
            f"{r['gflops_all_threads']:.2f} GFLOP/s on {nt} threads"
            + (f", CG {r['cg_iterations']} iterations in {r['cg_to_1e-10_seconds']:.1f} s" if "cg_iterations" in r else ""))
    # time-to-solution estimates from the GPU solves' iteration counts (74 at
    # 24^3x48, 151 at 16^3x32 plain FP64; one application per iteration)
    est = {"cfg3 24^3x48": 74 + 1, "cfg2/cfg4 16^3x32": 151 + 1}
    for k, it in est.items():
        res[k]["cg_to_1e-10_estimate_s_1_thread"] = it * res[k]["seconds_1_thread"]
    top = res["cfg3 24^3x48"]
    return _common_out(args, top["gflops_all_threads"], "GFLOP/s", top["seconds_1_thread"] * 1e3, "f64",
                       {"workload": "the CPU oracle (numpy FP64) on every workload lattice, on the host's cores"},
                       {"host": host, "by_lattice": res,
                        "note": "CPU only; the 50 solves/s served stream is far beyond the oracle (a 24^3x48 "
                                "solve alone takes minutes on one thread)"})


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cfg2", action="store_true", help="default workload: skip the 16^3x32 figures")
    ap.add_argument("--requests", type=int, default=2000, help="cfg5: served requests measured after the warm-up")
    ap.add_argument("--warmup-s", type=float, default=10.0, help="cfg5: seconds of arrivals served but not measured")
    ap.add_argument("--rate", type=float, default=50.0, help="cfg5: Poisson arrival rate per second")
    ap.add_argument("--served", default="f16,f32,f64", help="cfg5: inner precisions served, comma separated")
    ap.add_argument("--lattice", default="24,24,24,48", help="stencil: lattice extents x,y,z,t")
    ap.add_argument("--rhs-group", type=int, default=0, help="cfg4: sources per slot (0: library default)")
    ap.add_argument("--inner-recon", type=int, default=12, choices=(12, 18), help="cfg4: FP32 link recon")
    ap.add_argument("--save-tune", default=None, help="write the tuning table to this file")
    ap.add_argument("--tune-file", default=None, help="load this tuning table instead of autotuning")
    ap.add_argument("--stag-shape", default=None,
                    help="staggered: sites/block,swizzle,split for one field instead of autotuning (e.g. 128,1,2)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "KERNEL", "LATTICE"),
                    help="fold two rocprofv3 --pmc runs into profiles/traffic.json and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(*args.summarize_pmc), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    if args.workload in ("cfg2", "cfg3"):
        bench_default(args)
        return
    if args.tune_file:
        from paper_2409_03030_amd import wdirac as W
        W.tune_import(open(args.tune_file).read())
    fn = {"cfg1": bench_cfg1, "cfg4": bench_cfg4, "oracle": bench_oracle, "cfg5": bench_cfg5,
          "stencil": bench_stencil, "pion": bench_pion, "force": bench_force,
          "staggered": bench_staggered}.get(args.workload)
    if fn is None:
        raise SystemExit(f"unknown workload {args.workload}")
    out = fn(args)
    if args.save_tune:
        from paper_2409_03030_amd import wdirac as W
        open(args.save_tune, "w").write(W.tune_export())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
