"""Benchmark: cell-updates/s of the full extended-Boussinesq time step (FP32)
on one MI355X, on the 4096 x 4096 continental-shelf workload (64 JONSWAP
components at the west side, 64-cell sponge east, walls north/south,
fractal bathymetry noise; predictor + 2 correctors per step).

Prints one JSON line.  `value` = cells * steps / wall seconds of the timed
steps (inputs resident in HBM).  `roofline` reports the dominant kernel:
algorithmic bytes per launch (the kernel's compulsory reads and writes, see
ALG_BYTES) divided by its average duration, timed with HIP events recorded on
the library's launch stream over a second pass of the same steps.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload (after its two Euler start-up steps, a few full steps).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TUNING_CACHE = os.path.join(ROOT, "paper_1611_05984_amd", "tuning_cache.txt")

# Compulsory FP32 words per cell of each kernel class (reads + writes), for
# the default configuration (linear F* extrapolation, two correctors):
#   predictor: reads eta, P, Q, corner depth, history n-1 (E, F, G, F*, G*),
#              history n-2 (E, F, G); writes history n (5), corrector bases (3),
#              eta, dU*, dV*                                 -> 12 + 11 = 23
#   corrector: reads eta, P, Q, depth, bases (3); writes eta, dU*, dV* -> 7 + 3 = 10
#   reduce:    reads dU*, dV*, depth; writes, per 16-cell row segment and
#              16-cell column segment, two reduced equations (4 words each;
#              PCR and lane Thomas) or two right-hand sides (factored solve)
#                                                           -> 3 + 1 or 0.25
#   reduced solve: PCR reads the equations, writes the solutions: 1 + 0.25;
#              lane Thomas also writes and rereads its sweep values: 1 + 0.5 +
#              0.5 + 0.25; the factored solves (one- or two-ended) read the
#              right-hand sides and three factors, write the solutions:
#              0.25 + 0.75 + 0.25
#   expand:    reads dU*, dV* (2), P^n, Q^n, eta, depth, end values;
#              writes P, Q                                  -> 6.25 + 2
def alg_words(solver):
    reduce_w = 3.25 if solver in (2, 3) else 4.0
    solve_w = {0: 1.25, 1: 2.25, 2: 1.25, 3: 1.25}[solver]
    return {"k_stencil[predictor]": 23.0, "k_stencil[corrector]": 10.0,
            "k_reduce": reduce_w, "reduced_solve": solve_w, "k_expand": 8.25}


# kernel function -> its launch classes
FUNCS = {"k_stencil": ("k_stencil[predictor]", "k_stencil[corrector]"), "k_reduce": ("k_reduce",),
         "reduced_solve": ("reduced_solve",), "k_expand": ("k_expand",)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096, help="grid side (cells)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--retune", action="store_true",
                    help="measure the launch shapes instead of reading the tuning cache")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-plain ensemble measurement")
    ap.add_argument("--ens-steps", type=int, default=30, help="timed steps of the ensemble runs")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="wall seconds of the session-serving run (0: skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-no-recover", action="store_true",
                    help="retire failed sessions instead of rolling them back into NLSW")
    ap.add_argument("--no-k-variants", action="store_true",
                    help="skip the K = 0 and K = 1 corrector-count rates")
    return ap.parse_args()


def cpu_baseline(w, steps):
    import numpy as np
    import oracle
    z = w.z.astype(np.float32).astype(np.float64)
    D = oracle.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z)
    for s, side in enumerate(w.sides):
        if side.kind != 0:
            D.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta,
                           side.phase or None)
    D.advance(2)                      # Euler start-up steps (one pass each), untimed
    t = time.perf_counter()
    D.advance(steps)
    dt = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.nx * w.ny * steps / dt, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%s, %d full steps (predictor + 2 correctors) after the 2 Euler "
                      "start-up steps, FP64, %.1f s" % (w.name, steps, dt)}


def _make(ws, w, **params):
    d = ws.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, w.z, device="cuda:0", **params)
    for s, side in enumerate(w.sides):
        if side.kind != 0:
            d.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta,
                           side.phase or None)
    for (H, th, x0, y0) in w.solitary:
        d.add_solitary(H, th, x0, y0)
    return d


def _timed(torch, fn, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def batched_vs_plain(args, torch, ws, wl):
    """Ensemble of 256 uneven domains: batched stepping (one launch per phase
    for all domains, one graph replay per step) against per-domain stepping
    with the single-domain kernels on one stream, eager and graph-captured."""
    ens = wl.config4()
    cells = sum(w.cells for w in ens)
    doms = [_make(ws, w) for w in ens]
    B = ws.Batch(len(doms))
    for d in doms:
        B.attach(d)
    B.advance(4)                       # Euler start-up, untimed
    tuning = B.tune()                  # batch autotuner
    B.advance(2)                       # graph capture with the chosen shapes, untimed
    B.sync()
    n = args.ens_steps
    t_b = _timed(torch, lambda k: (B.advance(k), B.sync()), n)
    B.close()                          # domains usable alone again
    for d in doms:                     # same launch shapes for the per-domain runs
        d.set_tuning(*tuning)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for d in doms:
            d.advance(1, stream=st)
    t_p = _timed(torch, lambda k: [d.advance(k_, stream=st) for k_ in [1] * k for d in doms], n)
    # per-domain launches captured as a graph: three steps (the period of the
    # history ring and buffer rotation for two correctors), replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        for _ in range(3):
            for d in doms:
                d.advance(1, stream=st)
    reps = max(1, n // 3)
    t_g = _timed(torch, lambda k: [g.replay() for _ in range(k)], reps)
    health = [d.query()[2] for d in doms]
    del g
    return {"workload": "ensemble256_U256-1024_flat-or-beach_solitary", "domains": len(doms),
            "cells": cells, "steps": n,
            "batched": cells * n / t_b, "plain_eager": cells * n / t_p,
            "plain_graph": cells * 3 * reps / t_g,
            "batched_over_plain_graph": (cells * n / t_b) / (cells * 3 * reps / t_g),
            "batched_over_plain_eager": (cells * n / t_b) / (cells * n / t_p),
            "unit": "cell-updates/s", "healthy": all(h == 0 for h in health),
            "batch_tuning": {"stencil_rows": tuning[0], "corrector_rows": tuning[3] or tuning[0],
                             "pcr_threads": tuning[1],
                             "solver": ("pcr", "thomas", "lu", "lu2")[tuning[2]]}}


def serving(args):
    """Session serving: the Poisson trace (4 sessions/s, grids 512^2..2048^2,
    an edit every 50 steps) served with continuous batching for a bounded
    wall-time window; failed sessions are rolled back to their last edit
    pause and continued in NLSW unless --serve-no-recover."""
    from paper_1611_05984_amd import serving as sv
    from paper_1611_05984_amd import workloads as wl
    srv = sv.Server(budget_bytes=int(args.serve_budget_gb * 2**30), max_sessions=256, tick_steps=10,
                    recover=not args.serve_no_recover)
    rep = srv.run(wl.config5_trace(), wall_limit=args.serve_seconds,
                  log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    rep["workload"] = "sessions_poisson4ps_512-2048_edits50"
    return rep


def k_variants(args, torch, ws, wl):
    """Rates of the big-domain workload with K = 0 and K = 1 correctors, and
    in the NLSW model (K = 2; no dispersion, so no tridiagonal solves)."""
    w = wl.config3(n=args.n)
    out = {}
    for key, params in (("K0", dict(n_corr=0)), ("K1", dict(n_corr=1)), ("nlsw_K2", dict(model=ws.NLSW))):
        d = _make(ws, w, **params)
        d.advance(5)
        n = max(10, args.steps // 4)
        t = _timed(torch, lambda k: d.advance(k), n)
        out[key] = w.nx * w.ny * n / t
        d.close()
        del d
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: measures one GPU only; --gpus %d is not supported "
              "(the multi-GPU decomposition is design-only)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1611_05984_amd import wavestep as ws
    from paper_1611_05984_amd import workloads as wl

    torch.cuda.set_device(0)
    copy_gbs = None
    if args.copy_calib:
        # 256 MiB device-to-device copy: calibrates the HBM byte counters of a
        # profiled run and gives the practical copy bandwidth of this GPU
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        copy_gbs = 5 * 2 * src.numel() * 4 / (ev0.elapsed_time(ev1) / 1e3) / 1e9
        del src, dst
    w = wl.config3(n=args.n)
    D = ws.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, w.z, device="cuda:0")
    for s, side in enumerate(w.sides):
        if side.kind != 0:
            D.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta,
                           side.phase or None)
    print("bench: %s ready, warmup %d steps" % (w.name, args.warmup), file=sys.stderr, flush=True)
    D.advance(args.warmup)
    # autotuner: launch shapes for this grid, read from its cache when this
    # shape was measured before (the cache file ships with the package)
    tuning = D.tune(cache_path=None if args.retune else TUNING_CACHE)
    print("bench: tuned %s" % (tuning,), file=sys.stderr, flush=True)
    D.advance(2)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    D.advance(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step, tsim, health = D.query()
    if health:
        print("bench: non-finite state", file=sys.stderr)
        sys.exit(1)
    cells = w.nx * w.ny
    value = cells * args.steps / wall
    print("bench: timed %d steps in %.3f s" % (args.steps, wall), file=sys.stderr, flush=True)

    # per-kernel durations from HIP events on the launch stream (second pass)
    D.profile(True)
    D.advance(args.steps)
    prof = D.profile_collect()
    D.profile(False)
    tot = sum(ms for ms, n in prof.values())
    ALG_WORDS = alg_words(tuning[2])
    fsum = {f: (sum(prof[c][0] for c in cs), sum(prof[c][1] for c in cs),
                sum(ALG_WORDS[c] * prof[c][1] for c in cs)) for f, cs in FUNCS.items()}
    dom_func = max(fsum, key=lambda f: fsum[f][0])
    # kernel symbol as the profiler names it (template instance of the tuned shape)
    dom_name = {"k_stencil": "k_stencil_p<%d>,k_stencil_c<%d>" % (tuning[0], tuning[3] or tuning[0]),
                "reduced_solve": ("k_pcr", "k_thomas", "k_luw_solve", "k_lu2_solve")[tuning[2]]}.get(dom_func, dom_func)
    dom_ms, dom_n, dom_words = fsum[dom_func]
    avg_s = dom_ms / dom_n / 1e3
    alg_bytes = dom_words / dom_n * 4.0 * cells
    achieved = alg_bytes / avg_s / 1e9
    step_words = (ALG_WORDS["k_stencil[predictor]"] + 2 * ALG_WORDS["k_stencil[corrector]"] +
                  3 * (ALG_WORDS["k_reduce"] + ALG_WORDS["reduced_solve"] + ALG_WORDS["k_expand"]))
    kernels = {k: {"ms_avg": (ms / n if n else 0.0), "launches": n,
                   "share": (ms / tot if tot else 0.0),
                   "alg_GBs": (ALG_WORDS[k] * 4 * cells / (ms / n / 1e3) / 1e9 if n else 0.0)}
               for k, (ms, n) in prof.items()}
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        tr = json.load(open(tpath))
        if tr.get("kernel") == dom_name and tr.get("source_hash") == _source_hash():
            traffic = tr.get("bytes_per_launch")

    out = {
        "metric": "cell-updates/s per full step (FP32)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded shelf bathymetry + fractal noise, JONSWAP maker)",
        "config": {"workload": w.name + "_jonswap64_sponge64", "nx": w.nx, "ny": w.ny,
                   "dx_m": w.dx, "dt_s": w.dt, "n_corr": 2, "fstar_extrap": 1,
                   "tuning": {"stencil_rows": tuning[0], "corrector_rows": tuning[3] or tuning[0],
                              "pcr_threads": tuning[1],
                              "solver": ("pcr", "thomas", "lu", "lu2")[tuning[2]]},
                   "boundaries": "W waves(64 comps) / E sponge(64) / N,S walls"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": dom_name, "kernel_ms_avg": dom_ms / dom_n,
                     "alg_bytes_per_launch": alg_bytes},
        "copy_GBs": copy_gbs,
        "step_hbm": {"alg_bytes_per_cell_step": step_words * 4,
                     "alg_GBs": value * step_words * 4 / 1e9,
                     "frac_of_peak": value * step_words * 4 / 1e9 / HBM_PEAK_GBS},
        "kernels": kernels,
        "sim": {"step": step, "t_s": tsim},
    }
    D.close()
    del D
    torch.cuda.empty_cache()
    if not args.no_k_variants:
        print("bench: K = 0, 1 rates", file=sys.stderr, flush=True)
        out["k_variants"] = k_variants(args, torch, ws, wl)
    if not args.no_batched:
        print("bench: ensemble batched vs plain", file=sys.stderr, flush=True)
        out["ensemble"] = batched_vs_plain(args, torch, ws, wl)
    if args.serve_seconds > 0:
        print("bench: session serving, %.0f s" % args.serve_seconds, file=sys.stderr, flush=True)
        out["serving"] = serving(args)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


def _source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("ws_device.hpp", "ws_kernels.hpp", "ws_batch.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1611_05984_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
