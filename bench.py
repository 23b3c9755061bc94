"""Benchmark: solves/s of the PWL current-based VIE on one MI355X.

Workload (default): 64 x 64 x 64 voxels at 3 mm, 298 MHz, a seeded 6-class
ellipsoid tissue phantom (eps' ~ U[5, 80], sigma ~ U[0.05, 2] S/m), x-polarised
plane wave along z; left-preconditioned GMRES(50) to 1e-6 relative residual,
complex64 Krylov solves inside FP64 iterative refinement.  One step = one full
solve from x = 0 (operator products, Gram-Schmidt, refinement residuals) with
the operator, contrast and right-hand side already resident in HBM; operator
assembly is timed separately as set-up.

Printed as one JSON line: the metric, the plain FP64 solve rate for
comparison, the operator-product bandwidth, the roofline of the kernel that
takes the most device time (HIP events on the library stream over the timed
region, algorithmic bytes per launch), and the oracle's rate on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak as published (packed FMA: 256 CUs x 4 SIMDs x 16 lanes x
# 2 lanes per packed op x 2 flop x 2.4 GHz); without packed FP32 instructions,
# which this library does not emit, the FMA issue rate halves it
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_UNPACKED_PEAK_TFLOPS = 78.6
PROFILE_EVERY = 8


def block_flops(M, nrhs, nc=12):
    """Algorithmic flops of one x-pass launch: forward and inverse FFT along x
    of the nc components (5 n log2 n each) and the nc x nc complex block
    product (nc^2 complex multiply-adds of 8 flops) at every frequency:
    1152 flops for the PWL basis (nc = 12), 72 for the PWC basis (nc = 3)."""
    import math
    Mx, My, Mz = M
    pts = Mx * My * Mz
    return nrhs * (2 * 5 * nc * pts * math.log2(Mx) + 8 * nc * nc * pts)

# sources whose change invalidates counter measurements of the kernels
KERNEL_SOURCES = ["paper_1902_02196_amd/csrc/passes.hip", "paper_1902_02196_amd/csrc/strided.hip",
                  "paper_1902_02196_amd/csrc/fft.hpp", "paper_1902_02196_amd/csrc/fft_ct.hpp",
                  "paper_1902_02196_amd/csrc/passes.hpp", "paper_1902_02196_amd/csrc/common.hpp",
                  "paper_1902_02196_amd/csrc/krylov.hip", "paper_1902_02196_amd/csrc/apply.cpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_class, workload):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary (profiles/counters_<workload>.md, line 'traffic-json:'),
    or None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "counters_%s.md" % workload)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("source_hash") != kernel_source_hash():
                return None
            k = d.get("kernels", {}).get(kernel_class)
            if not k:
                return None
            return k["fetch_kib"] * d["fetch_scale"] * 1024 + k["write_kib"] * d["write_scale"] * 1024
    return None

WORKLOADS = {
    "phantom64": dict(N=(64, 64, 64), h=0.003, f=298e6, seed=190202196 + 1),
    # the same body with the PWC basis the paper compares against (3 unknowns
    # per voxel)
    "phantom64_pwc": dict(N=(64, 64, 64), h=0.003, f=298e6, seed=190202196 + 1, basis=3),
    # the same body with a per-class permeability, J-M formulation (24
    # unknowns per voxel)
    "phantom64_jm": dict(N=(64, 64, 64), h=0.003, f=298e6, seed=190202196 + 1, basis=24),
    "sphere16": dict(N=(16, 16, 16), h=0.005, f=298e6, seed=None),
    # head-sized box, 16 Hertzian dipoles on a 15 cm cylinder, one batched solve
    "batched16": dict(N=(96, 128, 128), h=0.002, f=298e6, seed=190202196 + 3, nrhs=16, cyl=0.15,
                      fp64_rhs=4),
    # whole-body box, 10-class layered phantom, 8 dipoles on a ring, solved
    # in groups of right-hand sides that fit HBM
    "body8": dict(N=(128, 256, 384), h=0.005, f=128e6, seed=190202196 + 5, nrhs=8, ring=(0.47, 0.47), group=2,
                  fp64_rhs=1, layered=True),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# host threads the oracle may use: a GPU machine gives each GPU a share of 16
# cores, whatever the machine's core count
CPU_SHARE = 16


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N, h, f, iters, restarts, seconds_budget=20.0, nc=12):
    """The oracle's FP64 GMRES (its own Arnoldi with modified Gram-Schmidt and
    its FFT operator product, numpy / scipy.fft) on this host's cores, timed
    on a bounded sample: one GMRES cycle of m steps, m chosen so the sample
    takes about seconds_budget; the solve time is the per-step time times
    the FP64 GPU solve's Arnoldi steps plus one residual product per restart
    cycle.  The oracle's block assembly is not included (random blocks and
    contrast of the right shapes: values do not change the time)."""
    from oracle import jm, matvec, pwc, solve
    import vie_inputs as vi
    cores = min(CPU_SHARE, os.cpu_count() or 1)
    Nx, Ny, Nz = N
    nb = 3 if nc == 3 else 12
    M = (2 * Nx, 2 * Ny, 2 * Nz)
    t0 = time.perf_counter()
    T = vi.complex_normal(5, (nb, nb, 2 * Nx - 1, 2 * Ny - 1, 2 * Nz - 1))
    Ch = matvec.circulant_spectrum(T, M, workers=cores) if nb == 12 else pwc.spectrum(T, M, workers=cores)
    del T
    if nc == 24:   # the J-M product also needs the curl operator's spectrum
        T = vi.complex_normal(8, (12, 12, 2 * Nx - 1, 2 * Ny - 1, 2 * Nz - 1))
        CK = matvec.circulant_spectrum(T, M, workers=cores)
        del T
    t_setup = time.perf_counter() - t0
    fft_N = matvec.fft_N if nb == 12 else pwc.fft_N
    tau = 0.1 * vi.complex_normal(7, tuple(N))
    D = (h, h, h)
    if nc == 24:
        fftw = lambda C_, u: matvec.fft_N(C_, u, workers=cores)
        op = lambda v: jm.apply_prec(Ch, CK, v, tau, tau, D, f, Nx_fn=fftw, Kx_fn=fftw)
    elif nc == 12:
        op = lambda v: matvec.apply_prec(None, v, tau, D, Nx_fn=lambda _t, u: fft_N(Ch, u, workers=cores))
    else:
        op = lambda v: pwc.apply_prec(None, v, tau, D, Nx_fn=lambda _t, u: fft_N(Ch, u, workers=cores))
    b = vi.complex_normal(6, (nc,) + tuple(N))
    t0 = time.perf_counter()
    op(b)
    t_mv = time.perf_counter() - t0
    m = int(max(4, min(50, seconds_budget / (2.5 * t_mv))))
    t0 = time.perf_counter()
    solve.gmres(op, b, restart=m, tol=1e-300, max_outer=1)   # one cycle: residual, m steps, residual
    t_cycle = time.perf_counter() - t0
    t_step = max(t_cycle - 2 * t_mv, 0.0) / m
    t_solve = t_step * iters + t_mv * (restarts + 1)
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpu_count": os.cpu_count(),
            "sample": "one oracle FP64 GMRES cycle of %d Arnoldi steps (modified Gram-Schmidt, FFT product with "
                      "scipy.fft on %d workers, %d unknowns per voxel) on the %dx%dx%d grid: %.2f s per step, "
                      "%.2f s per product; scaled to the FP64 GPU solve's %d steps and %d restart cycles; "
                      "spectrum set-up %.1f s excluded" % (m, cores, nc, Nx, Ny, Nz, t_step, t_mv, iters,
                                                          restarts, t_setup)}


SERVING = dict(edges=(32, 48, 64, 96, 128), h=0.003, freqs=(128e6, 298e6), rate=20.0, max_rhs=8,
               seed=190202196 + 4)


def serving_stream(n_req, seed):
    """Seeded finite Poisson stream: arrival offsets (s) and per-request
    (edge, frequency, dipole count, phantom seed, dipole seed)."""
    import vie_inputs as vi
    g = vi.rng(seed)
    gaps = g.exponential(1.0 / SERVING["rate"], size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n_req):
        edge = int(g.choice(SERVING["edges"]))
        f = float(g.choice(SERVING["freqs"]))
        nrhs = int(g.integers(1, SERVING["max_rhs"] + 1))
        reqs.append((edge, f, nrhs, seed + 1000 + i, seed + 2000 + i))
    return t, reqs


def serving_main(args):
    """Continuous-batching server fed by a seeded Poisson stream: latency
    percentiles (completion - arrival) and sustained solve rate."""
    import threading
    import torch
    import paper_1902_02196_amd as vie
    import vie_inputs as vi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    h = SERVING["h"]
    t_arr, reqs = serving_stream(args.requests, SERVING["seed"])
    inputs = []
    for edge, f, nrhs, pseed, dseed in reqs:
        N = (edge, edge, edge)
        e, s = vi.ellipsoid_phantom(N, (h, h, h), pseed)
        pos, mom = vi.dipoles_on_cylinder(dseed, nrhs, 0.75 * edge * h, edge * h)
        inputs.append((N, f, np.ascontiguousarray(e.transpose(2, 1, 0)),
                       np.ascontiguousarray(s.transpose(2, 1, 0)), pos, mom))
    log("serving stream: %s" % [(r[0], int(r[1] / 1e6), r[2]) for r in reqs])
    srv = vie.Server(0, hbm_budget=int(args.hbm_budget_gb * 2 ** 30), max_slots=args.slots)

    def submit(i):
        N, f, e, s, pos, mom = inputs[i]
        return srv.submit(N, (h, h, h), f, e, s, pos, mom, mode=vie.SOLVE_FP32_IR, tol=1e-6,
                          restart=args.restart)

    # warm-up request (kernel loading, first allocations), left out of the stats
    wid = submit(0)
    srv.wait()
    ids = []
    t0 = time.perf_counter()
    for i in range(len(inputs)):
        delay = t_arr[i] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        ids.append(submit(i))
        log("submitted %d at %.3f s" % (i, time.perf_counter() - t0))
    # progress while the queue drains (a long stream otherwise prints
    # nothing until the end)
    reported = 0
    while True:
        done = sum(1 for i in ids if srv.poll(i)["done"])
        if done == len(ids):
            break
        if done != reported:
            log("completed %d of %d at %.1f s" % (done, len(ids), time.perf_counter() - t0))
            reported = done
        time.sleep(0.25)
    srv.wait()
    wall = time.perf_counter() - t0
    st = srv.stats(first_id=wid + 1)
    infos = [srv.poll(i) for i in ids]
    bad = [(i, d["status"], d["message"]) for i, d in zip(ids, infos) if d["status"] != 0]
    assert not bad, bad
    nrhs_total = sum(r[2] for r in reqs)
    srv.close()
    out = {
        "metric": "serving: solves/s at 1e-6 relative residual with p50/p99 latency (continuous batching)",
        "value": round(len(ids) / st["makespan_s"], 4),
        "unit": "requests/s",
        "n_gpus": 1,
        "steps": len(ids),
        "warmup": 1,
        "ms_per_step": round(1e3 * st["makespan_s"] / len(ids), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "refinement": "FP64 residuals, updates, inner products and Givens",
        "data": "synthetic",
        "config": {"workload": "serving: %d requests, Poisson arrivals at %.0f req/s, edge in %s voxels at %.0f mm, "
                               "1-%d dipoles, %s MHz, 6-class ellipsoid phantoms, GMRES(%d) to 1e-6, "
                               "%d slots, %.0f GiB budget"
                               % (len(ids), SERVING["rate"], list(SERVING["edges"]), h * 1e3, SERVING["max_rhs"],
                                  [int(v / 1e6) for v in SERVING["freqs"]], args.restart, args.slots,
                                  args.hbm_budget_gb)},
        "p50_s": round(st["p50_s"], 4),
        "p99_s": round(st["p99_s"], 4),
        "mean_s": round(st["mean_s"], 4),
        "rhs_solves_per_s": round(nrhs_total / st["makespan_s"], 4),
        "offered_req_per_s": SERVING["rate"],
        "makespan_s": round(st["makespan_s"], 3),
        "wall_s": round(wall, 3),
        "peak_running": st["peak_running"],
        "peak_bytes": st["peak_bytes"],
        "iterations": [d["iterations"] for d in infos],
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="phantom64", choices=sorted(WORKLOADS) + ["serving"])
    ap.add_argument("--requests", type=int, default=12, help="serving: requests in the stream")
    ap.add_argument("--slots", type=int, default=4, help="serving: concurrent solves")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0, help="serving: admission budget")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--reorth", type=int, default=0, help="second Gram-Schmidt pass (1) or not (0)")
    ap.add_argument("--s-step", type=int, default=0,
                    help="Arnoldi steps per pass over the basis: 1 or 2 (0: the library's choice)")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--tuning", default="",
                    help="complex64 x-pass variant,sib_blocks,tile_z,tile_y installed instead of autotuning")
    ap.add_argument("--graph", type=int, default=-1,
                    help="replay the Arnoldi steps from HIP graphs (1), not (0), or when the vectors are small (-1)")
    ap.add_argument("--sync-steps", type=int, default=0,
                    help="Arnoldi steps per host check of the convergence flag (0: automatic)")
    ap.add_argument("--profile-every", type=int, default=PROFILE_EVERY,
                    help="time one launch in this many of each kernel class by its own events inside the timed "
                         "solves (0: none there; the classes are then timed in one more solve after the timed "
                         "region); graph replay implies 0, since a replayed launch carries no events")
    ap.add_argument("--tucker", type=float, default=0.0,
                    help="Tucker-compress the operator tensors to this relative tolerance and solve on the "
                         "operator rebuilt from the compressed form (0: off)")
    ap.add_argument("--products", type=int, default=0,
                    help="counter runs: after set-up and autotuning, time this many complex64 operator products "
                         "of one batch, run the 256 MiB calibration copy, print one JSON line and stop (no solves)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving":
        return serving_main(args)

    import torch
    import paper_1902_02196_amd as vie
    import vie_inputs as vi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    W = WORKLOADS[args.workload]
    N, h, f = W["N"], W["h"], W["f"]
    D = (h, h, h)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    ctx = vie.Context(0, stream)
    ctx.set_grid(N, D, f)
    nc = W.get("basis", 12)
    if nc != 12:
        ctx.set_basis(nc)
    torch.cuda.synchronize()
    t_grid = time.perf_counter() - t0
    tucker = None
    if args.tucker > 0:
        t0 = time.perf_counter()
        info = ctx.tucker_compress(args.tucker)
        t_c = time.perf_counter() - t0
        t0 = time.perf_counter()
        ctx.tucker_expand()
        torch.cuda.synchronize()
        t_e = time.perf_counter() - t0
        tucker = {"tol": args.tucker, "max_rank": [int(v) for v in info["ranks"].max(axis=0)],
                  "mean_rank": [round(float(v), 2) for v in info["ranks"].mean(axis=0)],
                  "max_rel_error": info["max_rel_error"], "bytes_dense": info["bytes_dense"],
                  "bytes_compressed": info["bytes_compressed"],
                  "compressed_fraction": round(info["bytes_compressed"] / info["bytes_dense"], 5),
                  "compress_s": round(t_c, 3), "expand_s": round(t_e, 3)}
        log("tucker: %s" % tucker)
    t0 = time.perf_counter()
    if args.tuning:
        # a fixed complex64 launch shape instead of the timed search (runs
        # whose counters are compared need the same kernels)
        v = [int(t) for t in args.tuning.split(",")]
        choice = dict(variant=v[0], sib_blocks=v[1], tile_z=v[2], tile_y=v[3])
        ctx.set_tuning(choice, vie.C64, W.get("group", W.get("nrhs", 1)))
        tune64 = (choice, None)
    else:
        tune64 = ctx.autotune(vie.C64, W.get("group", W.get("nrhs", 1)))
    tune128 = ctx.autotune(vie.C128, 1)
    t_tune = time.perf_counter() - t0
    log("autotune %.2f s: c64 %s, c128 %s" % (t_tune, tune64, tune128))
    mu = None
    if W["seed"] is None:
        e, s = vi.sphere(N, D, 0.03, 50.0, 0.7)
    elif W.get("layered"):
        e, s = vi.layered_phantom(N, D, W["seed"])
    elif nc == 24:
        e, s, mre, mim = vi.magnetic_phantom(N, D, W["seed"])
        mu = (mre, mim)
    else:
        e, s = vi.ellipsoid_phantom(N, D, W["seed"])
    ctx.set_contrast(np.ascontiguousarray(e.transpose(2, 1, 0)), np.ascontiguousarray(s.transpose(2, 1, 0)))
    if mu is not None:
        ctx.set_magnetic_contrast(np.ascontiguousarray(mu[0].transpose(2, 1, 0)),
                                  np.ascontiguousarray(mu[1].transpose(2, 1, 0)))
    nrhs = W.get("nrhs", 1)
    et = torch.empty(ctx.vec_shape(nrhs), dtype=torch.complex128, device=dev)
    if nrhs == 1:
        ctx.incident_planewave(et)
        excitation = "x-polarised plane wave"
    elif "ring" in W:
        pos, mom = vi.dipole_ring(nrhs, W["ring"][0] * N[0] * h, W["ring"][1] * N[1] * h)
        ctx.incident_dipoles(et, pos, mom)
        excitation = ("%d z-directed Hertzian dipoles on a %.0f x %.0f cm ring, solved in groups of %d"
                      % (nrhs, 200 * W["ring"][0] * N[0] * h, 200 * W["ring"][1] * N[1] * h, W["group"]))
    else:
        pos, mom = vi.dipoles_on_cylinder(W["seed"] + 1, nrhs, W["cyl"], N[2] * h)
        ctx.incident_dipoles(et, pos, mom)
        excitation = "%d z-directed Hertzian dipoles on a %.0f cm cylinder, one batched solve" % (nrhs, W["cyl"] * 100)
    group = W.get("group", nrhs)

    if args.products > 0:
        # the operator product alone at the batch the solves use, each pass
        # timed by the events its launch stamps, then the calibration copy
        xv = torch.randn(ctx.vec_shape(group), dtype=torch.complex64, device=dev)
        yv = torch.empty_like(xv)
        ctx.apply(xv, yv, op=vie.OP_PREC)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.products):
            ctx.apply(xv, yv, op=vie.OP_PREC)
        torch.cuda.synchronize()
        t_mv = (time.perf_counter() - t0) / args.products
        mvprof = {k: v for k, v in ctx.profile_read().items() if v[1] > 0 and v[0] > 0}
        ctx.profile(False)
        cbuf = torch.empty(16 * 1024 * 1024, dtype=torch.complex128, device=dev)
        cdst = torch.empty_like(cbuf)
        ctx.copy(cbuf, cdst)
        torch.cuda.synchronize()
        passes = {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1], "MB_per_launch": round(v[2] / v[1] / 1e6, 2),
                      "GBps_algorithmic": round(v[2] / (v[0] * 1e-3) / 1e9, 1)} for k, v in mvprof.items()}
        dev_ms = sum(v[0] for v in mvprof.values()) / args.products
        by = sum(v[2] for v in mvprof.values()) / args.products
        print(json.dumps({"workload": args.workload, "products": args.products, "nrhs": group, "fft_size": ctx.fft_size,
                          "tucker": tucker,
                          "autotune_c64": tune64, "product_ms": round(t_mv * 1e3, 4),
                          "product_device_ms": round(dev_ms, 4), "product_MB_algorithmic": round(by / 1e6, 1),
                          "product_GBps_algorithmic": round(by / (dev_ms * 1e-3) / 1e9, 1), "passes": passes,
                          "source_hash": kernel_source_hash()}), flush=True)
        return

    def solve_all(opts):
        """Solve every right-hand side, `group` at a time; returns the status
        and per-right-hand-side statistics."""
        code, stl = vie.VIE_OK, []
        for g0 in range(0, nrhs, group):
            if group == nrhs:
                c_, s_ = ctx.solve(et, x, opts)
            else:
                xg = torch.empty_like(et[g0:g0 + group])
                c_, s_ = ctx.solve(et[g0:g0 + group].contiguous(), xg, opts)
                x[g0:g0 + group].copy_(xg)
                del xg
                log("  right-hand sides %d-%d: %s" % (g0, g0 + group - 1, max(s_, key=lambda d: d["iterations"])))
            code = code if code != vie.VIE_OK else c_
            stl += s_
        return code, stl
    x = torch.empty_like(et)
    log("setup: grid+operator %.2f s" % t_grid)

    opts_ir = vie.default_opts(mode=vie.SOLVE_FP32_IR, tol=1e-6, restart=args.restart, inner_tol=1e-5,
                               reorth=args.reorth, graph=args.graph, sync_steps=args.sync_steps,
                               s_step=args.s_step)
    opts_64 = vie.default_opts(mode=vie.SOLVE_FP64, tol=1e-6, restart=args.restart, reorth=args.reorth,
                               graph=args.graph, sync_steps=args.sync_steps, s_step=args.s_step)
    for i in range(args.warmup):
        code, st = solve_all(opts_ir)
        log("warmup %d: %s" % (i, st[0]))

    every = 0 if args.graph > 0 else args.profile_every
    # timed region: K full solves; one launch in `every` of each kernel
    # class is bracketed by HIP events (average launch durations)
    torch.cuda.synchronize()
    if every:
        ctx.profile(True, every=every)
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        code, st = solve_all(opts_ir)
        stats.append(max(st, key=lambda d: d["iterations"]))
        log("step %d: %s" % (i, stats[-1]))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    if every:
        prof = ctx.profile_read()
        ctx.profile(False)
    else:
        # the kernel classes timed in one more solve, launched one by one
        ctx.profile(True, every=PROFILE_EVERY)
        solve_all(vie.default_opts(mode=vie.SOLVE_FP32_IR, tol=1e-6, restart=args.restart, inner_tol=1e-5,
                                   reorth=args.reorth, graph=0, sync_steps=args.sync_steps,
                                   s_step=args.s_step))
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
    assert code == vie.VIE_OK, "IR solve did not converge: %s" % stats[-1]
    n64 = min(nrhs, W.get("fp64_rhs", nrhs))
    x_ir = x[:n64].clone()

    # FP64 path for comparison, timed like the refinement path: one untimed
    # warm-up solve (it also grows the Krylov basis to complex128), then the
    # same number of timed solves with the same launch profiling; on the
    # first right-hand sides only when all of them would not fit in HBM
    et64 = et[:n64].contiguous()
    x64 = torch.empty_like(et64)
    code64, st64 = ctx.solve(et64, x64, opts_64)
    log("fp64 warmup: %s" % st64[0])
    torch.cuda.synchronize()
    if every:
        ctx.profile(True, every=every)
    t0 = time.perf_counter()
    for i in range(args.steps):
        code64, st64 = ctx.solve(et64, x64, opts_64)
    torch.cuda.synchronize()
    t_64 = (time.perf_counter() - t0) / args.steps
    ctx.profile(False)
    log("fp64: %s" % st64[0])
    assert code64 == vie.VIE_OK, "FP64 solve did not converge: %s" % st64[0]
    xi = x_ir[:n64].contiguous()
    e_ir = torch.empty_like(xi)
    e_64 = torch.empty_like(x64)
    ctx.fields(xi, e_ir)
    ctx.fields(x64, e_64)
    P_ir = ctx.absorbed_power(xi)
    P_64 = ctx.absorbed_power(x64)
    # field difference in the Gram-weighted norm (the L2 norm of the field
    # over the body: weight 1 for the pulse coefficients, 1/12 for the linear)
    gw = torch.tensor([1.0, 1 / 12, 1 / 12, 1 / 12] * (nc // 4) if nc in (12, 24) else [1.0] * nc,
                      dtype=torch.float64, device=dev).view(nc, 1, 1, 1)
    field_err = max(float(torch.sqrt((gw * (e_ir[r] - e_64[r]).abs() ** 2).sum() / (gw * e_64[r].abs() ** 2).sum()))
                    for r in range(n64))
    p_err = float(np.max(np.abs(P_ir - P_64) / np.abs(P_64)))
    del e_ir, e_64, xi, et64

    # operator product alone (complex64, preconditioned), for GB/s
    xv = torch.randn(ctx.vec_shape(group), dtype=torch.complex64, device=dev)
    yv = torch.empty_like(xv)
    for _ in range(3):
        ctx.apply(xv, yv, op=vie.OP_PREC)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nmv = 20
    for _ in range(nmv):
        ctx.apply(xv, yv, op=vie.OP_PREC)
    torch.cuda.synchronize()
    t_mv = (time.perf_counter() - t0) / nmv
    mvprof = ctx.profile_read()
    ctx.profile(False)
    mv_bytes = sum(v[2] for k, v in mvprof.items() if not k.startswith("gs_")) / nmv
    mv_dev_ms = sum(v[0] for k, v in mvprof.items() if not k.startswith("gs_")) / nmv

    # a plain copy of 256 MiB through the library's copy kernel: the known-size
    # reference that memory counters of profiled runs are scaled by
    cbuf = torch.empty(16 * 1024 * 1024, dtype=torch.complex128, device=dev)
    cdst = torch.empty_like(cbuf)
    ctx.copy(cbuf, cdst)
    torch.cuda.synchronize()

    # roofline of the kernel class with the most device time in the timed
    # solves: algorithmic bytes per launch (inputs read once, outputs written
    # once, the operator octant once per launch) over the average launch
    # duration from the events each sampled launch stamps.  The roof that
    # binds is the one with the longer time at the published peaks: for the
    # x pass (block) its bytes at 8 TB/s take longer than its flops at the
    # 157.3 TFLOP/s FP32 vector peak, so it is priced against HBM like the
    # other classes; its FP32 fractions (published peak, and the 78.6
    # TFLOP/s that FP32 without packed instructions can issue) ride along.
    dom = max(prof, key=lambda k: prof[k][0])
    ms, nl, by = prof[dom]
    avg_s = ms / nl * 1e-3
    tr = measured_traffic(dom, args.workload)
    hbm_achieved = (by / nl) / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(hbm_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_achieved / HBM_PEAK_GBS, 4), "traffic": tr, "kernel": dom,
                "launches_timed": nl, "avg_launch_us": round(avg_s * 1e6, 2), "bytes_per_launch": by / nl,
                "timed_in": "the timed solves" if every else "one more solve after the timed region"}
    if dom == "block":
        # a J-M x-pass launch is an N or a K pass over the 2 nrhs
        # 12-component halves
        fl = block_flops(ctx.fft_size, 2 * group, 12) if nc == 24 else block_flops(ctx.fft_size, group, nc)
        achieved = fl / avg_s / 1e12
        t_hbm, t_alu = (by / nl) / (HBM_PEAK_GBS * 1e9), fl / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
        if t_alu > t_hbm:   # flops bind at the published peaks
            roofline.update(bound="alu", achieved=round(achieved, 2), peak=FP32_VECTOR_PEAK_TFLOPS,
                            unit="TFLOP/s", frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4))
        roofline.update(flops_per_launch=fl, fp32_TFLOPs=round(achieved, 2),
                        fp32_frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                        fp32_frac_unpacked=round(achieved / FP32_UNPACKED_PEAK_TFLOPS, 4),
                        hbm_GBps=round(hbm_achieved, 1), hbm_frac=round(hbm_achieved / HBM_PEAK_GBS, 4),
                        roof_time_us={"hbm": round(t_hbm * 1e6, 2), "fp32": round(t_alu * 1e6, 2),
                                      "fp32_unpacked": round(fl / (FP32_UNPACKED_PEAK_TFLOPS * 1e12) * 1e6, 2)})
    kernels = {k: {"ms": round(v[0], 3), "launches": v[1],
                   "GB/s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None} for k, v in prof.items()}

    sps = args.steps * nrhs / t_total
    out = {
        "metric": "solves/s at 1e-6 relative residual (FP32 + FP64 refinement)",
        "value": round(sps, 4),
        "unit": "solves/s" if nrhs == 1 else "right-hand-side solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "refinement": "FP64 residuals, updates, inner products and Givens",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%dx%d voxels at %.0f mm, %.0f MHz, %s, %s, "
                               "GMRES(%d) to 1e-6, complex64 + FP64 refinement, %s basis"
                               % (args.workload, N[0], N[1], N[2], h * 1e3, f / 1e6,
                                  ("10-class layered phantom" if W.get("layered") else "6-class ellipsoid phantom")
                                  if W["seed"] else "eps 50 sigma 0.7 sphere r=3 cm",
                                  excitation, args.restart,
                                  {12: "PWL (12 unknowns per voxel)", 3: "PWC (3 unknowns per voxel)",
                                   24: "PWL J-M formulation with a per-class permeability (24 unknowns per "
                                       "voxel)"}[nc]),
                   "nrhs": nrhs},
        "fp64_solves_per_s": round(n64 / t_64, 4),
        "fp64_rhs": n64,
        "fp64_steps": args.steps,
        "ir_vs_fp64_speedup": round(sps * t_64 / n64, 3),
        "field_rel_err_ir_vs_fp64": field_err,
        "p_abs_ir_vs_fp64": p_err,
        "iterations_ir": stats[-1]["iterations"],
        "iterations_fp64": max(d["iterations"] for d in st64),
        "matvec_c64_ms": round(t_mv * 1e3, 4),
        "matvec_c64_device_ms": round(mv_dev_ms, 4),
        "matvec_c64_GBps_algorithmic": round(mv_bytes / (mv_dev_ms * 1e-3) / 1e9, 1),
        "setup_s": round(t_grid, 3),
        "autotune": {"c64": tune64[0], "c128": tune128[0], "seconds": round(t_tune, 2)},
        "solver": {"graph": args.graph, "sync_steps": args.sync_steps, "s_step": args.s_step,
                   "profile_every": every},
        "tucker": tucker,
        "kernel_source_hash": kernel_source_hash(),
        "kernels": kernels,
        "roofline": roofline,
    }
    if not args.no_cpu and nrhs == 1:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(N, h, f, st64[0]["iterations"], st64[0]["restarts"], nc=nc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
