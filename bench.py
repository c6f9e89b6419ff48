"""Benchmark: cell-updates/s of the full extended-Boussinesq time step (FP32)
on one MI355X, on the 4096 x 4096 continental-shelf workload (64 JONSWAP
components at the west side, 64-cell sponge east, walls north/south,
fractal bathymetry noise; predictor + 2 correctors per step).

Prints one JSON line.  `value` = cells * steps / wall seconds of the timed
steps (inputs resident in HBM), the median over `--windows` timed windows of
`--steps` steps each.  `roofline` reports the kernel with the largest share
of the step time: its algorithmic bytes per launch (the kernel's compulsory
reads and writes, see alg_words) divided by its average duration, timed with
HIP events recorded on the library's launch stream over a further window;
beside it, the whole step on the fused-ideal byte count (88 B per cell for
the predictor pass and 84 B per corrector pass: 256 B at K = 2) and on this
design's own count.  `copy_GBs` is the rate of a hand-written streaming
kernel with the corrector stencil's access shape (7 fields read, 3 written,
one wave per 64-column strip), measured in every run.  `cpu_baseline` times
the FP64 CPU oracle on a bounded sample of the same workload on all host
threads (`--cpu-table` adds 1-thread and all-thread rates of the three
single-domain workloads).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SOLVERS = ("pcr", "thomas", "lu", "lu2", "pcr_wave")
# fused-ideal compulsory bytes per cell of one pass: predictor 22 words, corrector 21
FUSED_PRED_B, FUSED_CORR_B = 88.0, 84.0
# non-packed FP32 VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-instructions/s);
# the library is compiled without packed FP32 instructions
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9
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
    solve_w = {0: 1.25, 1: 2.25, 2: 1.25, 3: 1.25, 4: 1.25}[solver]
    return {"k_stencil[predictor]": 23.0, "k_stencil[corrector]": 10.0,
            "k_reduce": reduce_w, "reduced_solve": solve_w, "k_expand": 8.25}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--windows", type=int, default=5, help="timed windows of --steps steps (median)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096, help="grid side (cells)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--cpu-table", action="store_true",
                    help="also time the oracle on 1 and all threads on the 128x64 basin (500 steps), "
                         "the 1024x512 beach (200) and the 4096^2 shelf (3)")
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


def cpu_model():
    """Host CPU model name and the logical CPUs this process may use."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def _oracle_rate(w, steps, threads):
    """Cell-updates/s of the oracle on workload w: `steps` full steps after
    its two Euler start-up steps (untimed), on `threads` OpenMP threads."""
    import numpy as np
    import oracle
    used = oracle.set_threads(threads)
    z = w.z.astype(np.float32).astype(np.float64)
    D = oracle.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z)
    for s, side in enumerate(w.sides):
        if side.kind != 0:
            D.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta,
                           side.phase or None)
    for (H, th, x0, y0) in w.solitary:
        D.add_solitary(H, th, x0, y0)
    D.advance(2)
    t = time.perf_counter()
    D.advance(steps)
    dt = time.perf_counter() - t
    return w.nx * w.ny * steps / dt, dt, used


def cpu_baseline(w, steps):
    import oracle
    all_threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    rate, dt, used = _oracle_rate(w, steps, all_threads)
    model, ncpu = cpu_model()
    return {"value": rate, "unit": "cell-updates/s", "cores": used, "kind": "oracle",
            "cpu_model": model, "cpus_available": ncpu,
            "sample": "%s, %d full steps (predictor + 2 correctors) after the 2 Euler "
                      "start-up steps, FP64, %d threads, %.1f s" % (w.name, steps, used, dt)}


def cpu_table(wl):
    """The oracle on 1 thread and on all threads: 128x64 basin 500 steps,
    1024x512 beach 200 steps, 4096^2 shelf 3 steps (after the start-up)."""
    all_threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    rows = []
    for w, steps in ((wl.config1(), 500), (wl.config2(steps=200), 200), (wl.config3(), 3)):
        for th in (1, all_threads):
            rate, dt, used = _oracle_rate(w, steps, th)
            rows.append({"workload": w.name, "steps": steps, "threads": used,
                         "cell_updates_per_s": rate, "s_per_step": dt / steps})
            print("bench: oracle %s %d steps, %d threads: %.3g cell-updates/s"
                  % (w.name, steps, used, rate), file=sys.stderr, flush=True)
    return rows


def stream_ceilings(torch, n):
    """HBM rates (GB/s, bytes moved / event time) of the hand-written
    streaming kernels: a 16-byte-lane copy of one n x n field, and the
    corrector (7 read + 3 written words a cell) and predictor (12 + 11)
    shapes of the stencil at 8 rows per wave, each with one dword stream per
    word and with the words packed into fewer, wider streams."""
    import ctypes as C
    from paper_1611_05984_amd import build as bld
    if not os.path.exists(bld.PROBE_LIB):
        raise RuntimeError("libwsprobe.so is not built; run paper_1611_05984_amd/build.py")
    L = C.CDLL(bld.PROBE_LIB)
    L.wsp_stream.restype = C.c_int
    L.wsp_stream.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                             C.c_void_p, C.POINTER(C.c_float)]
    pitch = (n + 63) // 64 * 64
    out = {}
    st = torch.cuda.current_stream()
    # (kind, words read, words written, room in fields for the input and output buffers)
    for kind, nr, nw, rin, rout, key in ((0, 1, 1, 1, 1, "copy16_GBs"), (1, 7, 3, 7, 3, "stencil_7r3w_GBs"),
                                         (2, 12, 11, 12, 11, "stencil_12r11w_GBs"),
                                         (3, 12, 11, 12, 11, "stencil_12r11w_packed_GBs"),
                                         (4, 7, 3, 12, 11, "stencil_7r3w_packed_GBs")):
        a = torch.ones(rin * n * pitch, dtype=torch.float32, device="cuda")
        b = torch.empty(rout * n * pitch, dtype=torch.float32, device="cuda")
        ms = C.c_float(0.0)
        rc = L.wsp_stream(kind, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), pitch, n, 8, 20,
                          C.c_void_p(st.cuda_stream), C.byref(ms))
        if rc != 0:
            raise RuntimeError("wsp_stream kind %d failed (%d)" % (kind, rc))
        out[key] = (nr + nw) * n * pitch * 4 / (ms.value / 1e3) / 1e9
        del a, b
    torch.cuda.empty_cache()
    out["shape"] = "%dx%d floats per field" % (n, pitch)
    return out


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
                             "solver": SOLVERS[tuning[2]]}}


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
    in the NLSW model (K = 2; no dispersion, so no tridiagonal solves), each
    with its own launch shapes from the autotuner (read from its cache when
    that shape was measured before).  The AB3 predictor alone (K = 0) is
    unstable on this dispersive workload (the state turns non-finite after
    60-70 steps, in the FP64 oracle too), so it is timed over three windows of
    10 steps right after the start-up, while the state is finite; every rate
    is reported with the health word at the end of its windows (a rate of a
    non-finite state is reported as null)."""
    w = wl.config3(n=args.n)
    out = {}
    for key, params, n in (("K0", dict(n_corr=0), 10), ("K1", dict(n_corr=1), max(10, args.steps // 2)),
                           ("nlsw_K2", dict(model=ws.NLSW), max(10, args.steps // 2))):
        d = _make(ws, w, **params)
        d.advance(5)
        tun = d.tune(cache_path=None if args.retune else TUNING_CACHE)
        d.advance(3)
        rates = [w.nx * w.ny * n / _timed(torch, lambda k: d.advance(k), n) for _ in range(3)]
        step, _, health = d.query()
        out[key] = sorted(rates)[1] if health == 0 else None
        out[key + "_tuning"] = list(tun)
        out[key + "_healthy_at_step"] = [step, health == 0]
        print("bench: %s tuned %s: %s cell-updates/s (health %d at step %d)"
              % (key, tun, out[key], health, step), file=sys.stderr, flush=True)
        d.close()
        del d
        torch.cuda.empty_cache()
    return out


# kernel class (as the library's event profiler reports it) -> the symbol the
# profiler's kernel trace shows for the tuned launch shape
def kernel_symbol(cls, tuning):
    rows, _, solver, crows = tuning
    return {"k_stencil[predictor]": "k_stencil_p<%d>" % rows,
            "k_stencil[corrector]": "k_stencil_c<%d>" % (crows or rows),
            "reduced_solve": ("k_pcr", "k_thomas", "k_luw_solve", "k_lu2_solve", "k_pcrw")[solver]}.get(cls, cls)


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
    ceil = stream_ceilings(torch, args.n)
    print("bench: streaming ceilings %s" % json.dumps(ceil), file=sys.stderr, flush=True)
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

    cells = w.nx * w.ny
    walls = []
    for _ in range(max(1, args.windows)):
        t0 = time.perf_counter()
        D.advance(args.steps)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    step, tsim, health = D.query()
    if health:
        print("bench: non-finite state", file=sys.stderr)
        sys.exit(1)
    wall = sorted(walls)[len(walls) // 2]
    value = cells * args.steps / wall
    print("bench: %d windows of %d steps: %s s" % (len(walls), args.steps, ["%.4f" % x for x in walls]),
          file=sys.stderr, flush=True)

    # per-kernel durations from HIP events on the launch stream (another window)
    D.profile(True)
    D.advance(args.steps)
    prof = D.profile_collect()
    D.profile(False)
    tot = sum(ms for ms, n in prof.values())
    ALG_WORDS = alg_words(tuning[2])
    kernels = {k: {"symbol": kernel_symbol(k, tuning), "ms_avg": (ms / n if n else 0.0), "launches": n,
                   "share": (ms / tot if tot else 0.0), "alg_bytes_per_cell": ALG_WORDS[k] * 4,
                   "alg_GBs": (ALG_WORDS[k] * 4 * cells / (ms / n / 1e3) / 1e9 if n else 0.0)}
               for k, (ms, n) in prof.items()}
    # the dominant kernel: the largest share of the step's kernel time
    dom = max((k for k in kernels if kernels[k]["launches"]), key=lambda k: kernels[k]["share"])
    dom_name = kernels[dom]["symbol"]
    avg_s = kernels[dom]["ms_avg"] / 1e3
    alg_bytes = ALG_WORDS[dom] * 4.0 * cells
    achieved = alg_bytes / avg_s / 1e9
    kernel_ms_step = tot / args.steps
    step_words = (ALG_WORDS["k_stencil[predictor]"] + 2 * ALG_WORDS["k_stencil[corrector]"] +
                  3 * (ALG_WORDS["k_reduce"] + ALG_WORDS["reduced_solve"] + ALG_WORDS["k_expand"]))
    fused_b = FUSED_PRED_B + 2 * FUSED_CORR_B
    # counter figures of the dominant kernel from the committed profile, used
    # only while the kernel sources are those the counters were taken on
    traffic, valu = None, None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        tr = json.load(open(tpath))
        if tr.get("kernel") == dom_name and tr.get("source_hash") == _source_hash():
            traffic = tr.get("bytes_per_launch")
            if tr.get("valu_lane_instr_per_launch"):
                li = tr["valu_lane_instr_per_launch"]
                valu = {"lane_instr_per_cell": li / cells,
                        "issue_frac": li / (kernels[dom]["ms_avg"] / 1e3) / VALU_ISSUE_PEAK,
                        "peak_lane_instr_per_s": VALU_ISSUE_PEAK}

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
                              "solver": SOLVERS[tuning[2]]},
                   "boundaries": "W waves(64 comps) / E sponge(64) / N,S walls"},
        "windows_s": walls,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": dom_name, "kernel_ms_avg": kernels[dom]["ms_avg"], "valu": valu,
                     "alg_bytes_per_launch": alg_bytes, "alg_bytes_per_cell": ALG_WORDS[dom] * 4,
                     "step": {"alg_bytes_per_cell_fused_ideal": fused_b,
                              "achieved_GBs": value * fused_b / 1e9,
                              "frac": value * fused_b / 1e9 / HBM_PEAK_GBS,
                              "alg_bytes_per_cell_this_design": step_words * 4,
                              "achieved_GBs_this_design": value * step_words * 4 / 1e9,
                              "frac_this_design": value * step_words * 4 / 1e9 / HBM_PEAK_GBS,
                              "kernel_ms_per_step": kernel_ms_step}},
        "copy_GBs": ceil["stencil_7r3w_GBs"],
        "copy_ceilings": ceil,
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
        if args.cpu_table:
            out["cpu_baseline"]["table"] = cpu_table(wl)
    print(json.dumps(out), flush=True)


def _source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("ws_device.hpp", "ws_kernels.hpp", "ws_batch.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1611_05984_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
