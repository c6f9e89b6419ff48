"""Summarize rocprofv3 result databases of a wavestep run.

Usage:
  python -m paper_1611_05984_amd.profile_summary --trace KT.db [--fetch F.db --write W.db]
         [--cells N] [--out summary.txt] [--traffic-json traffic.json --command "..."]

--trace: database of `rocprofv3 --kernel-trace --stats`; prints per-kernel calls,
average and total duration.
--fetch/--write: databases of `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
runs of the same command.  The byte counters are calibrated against the
streaming probe's copy kernel in the same run (bench.py measures it in every
run: k_copy4 reads and writes --copy-bytes bytes, one 4096 x 4096 float field
by default): scale = known bytes / counter bytes of that dispatch, per
counter.  Per kernel class the calibrated bytes per dispatch are reported
(words per cell when --cells is given).
"""
import argparse
import hashlib
import json
import os
import sqlite3
from collections import defaultdict

COPY_BYTES = 4096 * 4096 * 4  # the probe copy of bench.py: one 4096 x 4096 float field each way


def _q(db, sql, args=()):
    con = sqlite3.connect(db)
    try:
        return con.execute(sql, args).fetchall()
    finally:
        con.close()


def trace_table(db):
    """(name, calls, total us, average us, percent) per kernel; the database's
    top_kernels view reports durations in microseconds."""
    rows = _q(db, "select name, total_calls, total_duration, average, percentage from top_kernels")
    return [(n, int(c), float(t), float(a), float(p)) for n, c, t, a, p in rows]


def counter_values(db, counter):
    rows = _q(db, "select kernel_name, value from counters_collection where counter_name=? "
                  "order by dispatch_id", (counter,))
    out = defaultdict(list)
    for name, v in rows:
        out[name].append(float(v) * 1024.0)  # KiB -> bytes
    return out


def calib(values, copy_bytes):
    """Scale of a byte counter: known bytes of the probe copy / its counter
    bytes (the median over its dispatches)."""
    copies = sorted(v for k, vs in values.items() if "k_copy4" in k for v in vs)
    if not copies:
        return None
    mid = copies[len(copies) // 2]
    return copy_bytes / mid if mid > 0 else None


def short(name):
    """Kernel name without return type, namespace and parameter list."""
    n = name[5:] if name.startswith("void ") else name
    return n.replace("(anonymous namespace)::", "").split("(")[0].replace("ws::", "")


def source_hash(root):
    h = hashlib.sha256()
    for f in ("ws_device.hpp", "ws_kernels.hpp", "ws_batch.hpp"):
        h.update(open(os.path.join(root, "paper_1611_05984_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


VALU_PEAK = 256 * 4 * 16 * 2.4e9  # lane-instructions/s: CUs x SIMDs x lanes x clock (non-packed FP32)


def sq_table(sq_db, trace_db, cells):
    """Per kernel: VALU instructions per dispatch, lane-instructions per cell
    and VALU issue utilisation over the kernel's average traced duration."""
    per = defaultdict(lambda: defaultdict(list))
    for name, counter, v in _q(sq_db, "select kernel_name, counter_name, value from counters_collection"):
        per[short(name)][counter].append(float(v))
    avg_us = {short(n): a for n, _, _, a, _ in trace_table(trace_db)}
    lines = ["VALU rate against one wave64 instruction per 4 cycles per SIMD: 256 CU x 4 SIMD x 16 lanes "
             "x 2.4 GHz = %.1fe12 lane-instructions/s" % (VALU_PEAK / 1e12),
             "(a rate above 100% means gfx950 issues some VALU instructions faster than that model, so "
             "it is a reference, not a ceiling)",
             "%-20s %13s %15s %11s %10s" % ("kernel", "VALU/disp", "lane-instr/cell", "avg_us", "VALU rate")]
    for k in sorted(per):
        if k not in avg_us or "SQ_INSTS_VALU" not in per[k]:
            continue
        vals = per[k]["SQ_INSTS_VALU"]
        valu = sum(vals) / len(vals)
        lane = valu * 64
        util = lane / (avg_us[k] * 1e-6) / VALU_PEAK
        lines.append("%-20s %13.4g %15.1f %11.1f %9.0f%%" % (k, valu, lane / cells if cells else 0, avg_us[k],
                                                             100 * util))
    return lines


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--cells", type=int, default=0)
    ap.add_argument("--copy-bytes", type=int, default=COPY_BYTES,
                    help="bytes the probe copy kernel reads (and writes) per dispatch")
    ap.add_argument("--out")
    ap.add_argument("--traffic-json")
    ap.add_argument("--command", default="")
    ap.add_argument("--kernel", default="k_stencil_p<8>,k_stencil_c<8>",
                    help="kernel, or comma-separated kernels taken as one group (as the trace names "
                         "them, without namespace), whose traffic goes to --traffic-json")
    ap.add_argument("--sq", help="database of a rocprofv3 --pmc SQ_INSTS_VALU ... run (VALU table)")
    ap.add_argument("--skip", type=int, default=2,
                    help="leading dispatches per kernel left out of the averages (Euler start-up)")
    a = ap.parse_args()
    lines = []
    if a.command:
        lines.append("command: " + a.command)
    lines.append("%-32s %7s %12s %12s %7s" % ("kernel", "calls", "avg_us", "total_us", "pct"))
    for n, c, t, avg, p in trace_table(a.trace):
        lines.append("%-32s %7d %12.1f %12.1f %6.1f%%" % (short(n)[:32], c, avg, t, p))
    traffic = {}
    if a.fetch and a.write:
        fv, wv = counter_values(a.fetch, "FETCH_SIZE"), counter_values(a.write, "WRITE_SIZE")
        fs, wsc = calib(fv, a.copy_bytes), calib(wv, a.copy_bytes)
        lines.append("")
        lines.append("HBM bytes per dispatch (FETCH_SIZE x %.3f, WRITE_SIZE x %.3f; factors from the "
                     "probe copy kernel, %d bytes each way)" % (fs or 0, wsc or 0, a.copy_bytes))
        for name in sorted(fv):
            head = name.replace("(anonymous namespace)::", "").split("(")[0]
            if "ws::" not in head and "k_stream" not in head and "k_copy4" not in head:
                continue
            rd = [v * fs for v in fv[name]][a.skip:]
            wr = [v * wsc for v in wv.get(name, [])][a.skip:]
            n = min(len(rd), len(wr))
            per = [(rd[i], wr[i]) for i in range(n)]
            avg_r, avg_w = sum(x for x, _ in per) / n, sum(y for _, y in per) / n
            txt = "%-24s dispatches %3d  read %9.3e B  write %9.3e B" % (short(name), n, avg_r, avg_w)
            if a.cells:
                txt += "  (%.2f + %.2f words/cell)" % (avg_r / a.cells / 4, avg_w / a.cells / 4)
            lines.append(txt)
            traffic[short(name)] = {"read": avg_r, "write": avg_w, "dispatches": n,
                                    "per_dispatch": per}
    if a.sq:
        lines.append("")
        lines.extend(sq_table(a.sq, a.trace, a.cells))
    text = "\n".join(lines)
    print(text)
    if a.out:
        open(a.out, "w").write(text + "\n")
    names = a.kernel.split(",")
    if a.traffic_json and all(n in traffic for n in names):
        # one kernel, or a group of kernels: the average over all dispatches
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        n = sum(traffic[k]["dispatches"] for k in names)
        rd = sum(traffic[k]["read"] * traffic[k]["dispatches"] for k in names) / n
        wr = sum(traffic[k]["write"] * traffic[k]["dispatches"] for k in names) / n
        out = {"kernel": a.kernel, "bytes_per_launch": rd + wr, "read": rd, "write": wr,
               "dispatches": n, "source_hash": source_hash(root), "command": a.command}
        if a.sq:
            valu = sq_valu(a.sq)
            if all(k in valu for k in names):
                out["valu_lane_instr_per_launch"] = sum(valu[k] for k in names) / len(names)
        json.dump(out, open(a.traffic_json, "w"), indent=1)


def sq_valu(sq_db):
    """Average VALU lane-instructions per dispatch of each kernel."""
    per = defaultdict(list)
    for name, counter, v in _q(sq_db, "select kernel_name, counter_name, value from counters_collection"):
        if counter == "SQ_INSTS_VALU":
            per[short(name)].append(float(v) * 64)
    return {k: sum(v) / len(v) for k, v in per.items()}


if __name__ == "__main__":
    main()
