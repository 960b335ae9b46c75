#!/usr/bin/env python3
"""Throughput benchmark of the Proportional Similarity hot path on one GPU.

A step is one pass of the whole path over the resident synthetic input:
per-vector sums, the min-product numerators and the FP64 metric epilogue
(2-way), plus the pair-numerator prepass for 3-way.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME]

Workloads (seeded, synthetic; shapes of the paper's problems):
  gwas_20000x16384   2-way, 20000 fields x 16384 vectors, FP32, 70% zeros,
                     nonzeros Exponential(mean 2)            (default)
  uniform_1024x256   2-way, FP32 U[0,1)
  levels_8192x32768  2-way, uint8 levels {0..3}
  binary_8192x32768  2-way, uint8 {0, 1} (the Sorensen case; --path bits)
  sparse_4096x1024   3-way, FP32 U[0,1) with 50% zeros
  levels_4096x1024   3-way, uint8 levels {0..3} (--path mfma | mfma_fp4 | valu)
  batched_64_uneven  64 independent 2-way problems in one captured launch

Comparisons are counted as the paper counts them: one per field and unique
tuple (n_f C(n_v,2) for 2-way, n_f C(n_v,3) for 3-way).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz.  FP32 vector 157.3 TFLOP/s = 128 FP32 lanes per
# clock per CU (an FMA, a min or an add is one lane-op); measured: v_min_f32 and
# v_add_f32 issue at that rate, while v_pk_min_f16, v_dot2c_f32_f16, v_sad_u8
# and the v_and_b32 + v_bcnt_u32_b32 pair of the bits path issue at 64 lanes
# per clock per CU.
FP32_LANE_OPS_TOPS = 256 * 128 * 2.4e9 / 1e12   # 78.64
HALF_RATE_OPS_TOPS = 256 * 64 * 2.4e9 / 1e12    # 39.32
INT8_MFMA_PEAK_TOPS = 5000.0                    # dense int8 matrix-core ops / s (2 per MAC)
FP4_MFMA_PEAK_TOPS = 10100.0                    # dense fp4 matrix-core ops / s
HBM_PEAK_GBS = 8000.0


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gwas_20000x16384")
    ap.add_argument("--storage", default="auto", choices=["auto", "f32", "f16", "f64"])
    ap.add_argument("--acc", default="auto", choices=["auto", "plain", "blocked"])
    ap.add_argument("--path", default="auto",
                    choices=["auto", "valu", "mfma", "mfma_fp4", "bits"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-3way", action="store_true",
                    help="default workload: skip the 3-way measurement of the same line")
    ap.add_argument("--shard-of", type=int, default=0, metavar="N",
                    help="2-way workloads: time one GPU's share when the pairs are spread "
                         "over N GPUs by tiles (shard 0 of N, ps2_compute_shard); the whole "
                         "call is timed beside it")
    ap.add_argument("--per-problem", action="store_true",
                    help="batched workload: one launch per problem instead of the plan")
    ap.add_argument("--campaign", type=int, default=0, metavar="STAGES",
                    help="3-way workloads: run as a staged campaign of STAGES stages, one "
                         "byte per metric copied to host memory (Section 6.5 output)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device (a plain copy kernel of known "
                         "size, to scale HBM byte counters of a profiler run)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "KERNEL"),
                    help="no benchmark: summarise two rocprofv3 --pmc runs (FETCH_SIZE, "
                         "WRITE_SIZE) of this script for --workload/--storage/--path into "
                         "the traffic file read by later runs")
    ap.add_argument("--counter-summary", nargs=2, metavar=("PMC_DIR", "KERNEL"),
                    help="no benchmark: per-dispatch means of every counter of one "
                         "rocprofv3 --pmc run for KERNEL, with busy fractions")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "BENCH_LOG"),
                    help="no benchmark: the kernel table of one rocprofv3 --kernel-trace "
                         "--stats run of this script (csv) with the bench line it printed")
    ap.add_argument("--pmc-command", action="append", default=[],
                    help="command line recorded in the --pmc-summary output")
    return ap.parse_args(argv)


class Timer:
    """HIP events on torch's current stream (the stream libps launches on)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def mark(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def add(self, a, b):
        self.pairs.append((a, b))

    def mean_ms(self):
        self.torch.cuda.synchronize()
        v = [a.elapsed_time(b) for a, b in self.pairs]
        return sum(v) / len(v) if v else float("nan")


def _oracle_rate(run, seconds, m0=256, cap=1 << 24):
    """Grow the sample until one run takes 0.2 s, then size it to `seconds`.
    run(m) -> (seconds taken, tuples done)."""
    m = m0
    t, m = run(m)
    while t < 0.2 and m < cap:
        t, m = run(m * 4)
    return run(max(m0, int(m * seconds / max(t, 1e-9))))


def cpu_baseline(V, n_f, seconds, way, seed=123):
    """The oracle timed on the host: c2 (way 2) or c3 (way 3) of random
    tuples of the full input, once on all threads and once on one thread
    (each about `seconds`)."""
    import numpy as np

    import oracle
    g = np.random.default_rng(seed)
    n_v = V.shape[0]
    s = oracle.sums(V)

    def run(m):
        if way == 2:
            a = g.integers(0, n_v, size=m)
            b = (a + 1 + g.integers(0, n_v - 1, size=m)) % n_v
            t0 = time.perf_counter()
            oracle.c2_pairs(V, a, b, s=s)
            return time.perf_counter() - t0, m
        t = np.sort(g.integers(0, n_v, size=(3 * m, 3)), axis=1)
        t = t[(t[:, 0] < t[:, 1]) & (t[:, 1] < t[:, 2])][:m]
        t0 = time.perf_counter()
        oracle.c3_triples(V, t[:, 0], t[:, 1], t[:, 2], s=s)
        return time.perf_counter() - t0, len(t)

    threads = oracle.num_threads()
    t, m = _oracle_rate(run, seconds)
    oracle.set_threads(1)
    try:
        t1, m1 = _oracle_rate(run, seconds)
    finally:
        oracle.set_threads(threads)
    what = "pairs" if way == 2 else "triples"
    extra = "" if way == 2 else ", pair terms included"
    return {"value": m * n_f / t, "unit": "comparisons/s", "cores": threads, "kind": "oracle",
            "value_1thread": m1 * n_f / t1,
            "sample": f"{m} random {what} of the full input on {threads} threads ({t:.1f} s) "
                      f"and {m1} on 1 thread ({t1:.1f} s), {n_f} fields each (oracle c{way} of "
                      f"listed {what}{extra})"}


# Source files that decide what each kernel does and how it is launched; their
# digest stamps a recorded HBM-traffic figure, which is reported only while
# the sources are unchanged.
CSRC = os.path.join(ROOT, "paper_1705_08210_amd", "csrc")
_VALU_SOURCES = ["ps_internal.h", "mgemm_core.h", "mgemm_kernels.h", "mg_common.hip",
                 "mg_f32.hip", "mg_f16.hip", "mg_u8.hip", "policy.hip"]
_MFMA_SOURCES = ["ps_internal.h", "mfma.hip", "policy.hip"]
KERNEL_SOURCES = {
    "ps_mg2_kernel": _VALU_SOURCES,
    "ps_mg3f_kernel": _VALU_SOURCES,
    "ps_mgb_kernel": _VALU_SOURCES,
    "ps_mfma2_lv_kernel": _MFMA_SOURCES,
    "ps_mfma2_lvd_kernel": _MFMA_SOURCES,
    "ps_mfma2_kernel": _MFMA_SOURCES,
    "ps_mfma2_dma_kernel": _MFMA_SOURCES,
    "ps_mfma3_lv_kernel": _MFMA_SOURCES,
    "ps_mfma3_lvs_kernel": _MFMA_SOURCES,
    "ps_mfma3_lvsd_kernel": _MFMA_SOURCES,
    "ps_mfma3_kernel": _MFMA_SOURCES,
}
PROFILES = os.path.join(ROOT, "profiles")
GIB = 1 << 30


def source_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def traffic_file(kernel, key):
    return os.path.join(PROFILES, f"traffic_{kernel}_{key}.txt")


def recorded_traffic(kernel, key):
    """HBM bytes per call (all dispatches of the kernel in one library call)
    from a committed counter summary, or None when there is none, it predates
    this format, or the kernel's sources changed since it was taken."""
    path = traffic_file(kernel, key)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("sources_sha256") != source_digest(kernel) or \
            "traffic_bytes_per_call" not in fields:
        return None
    return int(fields["traffic_bytes_per_call"])


def roofline(bound, ops_per_cmp, cmp, kernel_ms, peak, traffic=None):
    """achieved = algorithmic ops of one launch / its mean duration."""
    achieved = ops_per_cmp * cmp / (kernel_ms * 1e-3) / 1e12
    return {"bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 2),
            "unit": "TOP/s", "frac": round(achieved / peak, 4), "traffic": traffic}


def _counters(d):
    """Per-dispatch KiB of one rocprofv3 --pmc csv output directory."""
    import csv
    import glob
    out = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = (r["Dispatch_Id"], r["Kernel_Name"], int(r["Grid_Size"]))
                out[k] = out.get(k, 0.0) + float(r["Counter_Value"])
    return out


def pmc_summary(fetch_dir, write_dir, kernel, key, commands):
    """Text summary of a FETCH_SIZE run and a WRITE_SIZE run of this script
    with --copy-calibration: each counter is scaled by what it reads for the
    1 GiB device-to-device copy (one copy kernel dispatch of known size)."""
    fetch, write = _counters(fetch_dir), _counters(write_dir)

    def calib(cnt):
        # the calibration copy is the copy dispatch with the most bytes
        cands = [(v, k) for k, v in cnt.items() if "copyBuffer" in k[1]]
        v, k = max(cands)
        return GIB / (v * 1024.0), v, k

    ff, fv, fk = calib(fetch)
    wf, wv, wk = calib(write)

    def mean(cnt):
        # per call: the mean over the dispatches of each instance of the
        # kernel (the 3-way slices launch two tile sizes per call), summed
        inst = {}
        for k, x in cnt.items():
            if k[1].startswith(f"void ps::{kernel}<") or k[1].startswith(f"ps::{kernel}("):
                inst.setdefault(k[1], []).append(x)
        return (sum(sum(v) / len(v) for v in inst.values()),
                f"{len(inst)} kernel instance(s), mean of {min(len(v) for v in inst.values())}"
                " dispatches each")

    fm, fn = mean(fetch)
    wm, wn = mean(write)
    traffic = fm * 1024.0 * ff + wm * 1024.0 * wf
    lines = [f"kernel: {kernel}", f"workload: {key}"]
    lines += [f"command: {c}" for c in commands]
    lines += [
        f"calibration fetch: copy dispatch {fk[0]} reads 1 GiB, FETCH_SIZE {fv:.1f} KiB "
        f"-> factor {ff:.4f}",
        f"calibration write: copy dispatch {wk[0]} writes 1 GiB, WRITE_SIZE {wv:.1f} KiB "
        f"-> factor {wf:.4f}",
        f"FETCH_SIZE per call: {fm:.1f} KiB ({fn}) -> {fm * 1024 * ff / 1e9:.3f} GB",
        f"WRITE_SIZE per call: {wm:.1f} KiB ({wn}) -> {wm * 1024 * wf / 1e9:.3f} GB",
        f"traffic_bytes_per_call: {int(round(traffic))}",
        f"sources_sha256: {source_digest(kernel)}",
    ]
    return "\n".join(lines) + "\n"


def counter_summary(d, kernel, commands):
    """Per-call sums of the counters of one rocprofv3 --pmc run and what
    they give.  GRBM_GUI_ACTIVE counts GPU cycles on each of the 8 XCDs, so
    cycles = GRBM_GUI_ACTIVE / 8 and the clock = cycles / dispatch duration.
    MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x cycles); VALU issue
    = SQ_INSTS_VALU / (256 CUs x cycles), wave instructions per CU per cycle
    (FP32 min/add issue up to 2, packed FP16 and v_sad_u8 up to 1)."""
    import csv
    import glob
    per, dur, name = {}, {}, {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                n = r["Kernel_Name"]
                if not (n.startswith(f"void ps::{kernel}<") or n.startswith(f"ps::{kernel}(")):
                    continue
                key = (r["Dispatch_Id"], r["Counter_Name"])
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
                dur[r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                name[r["Dispatch_Id"]] = n
    # per call: means over the dispatches of each kernel instance, summed over
    # the instances (the 3-way slices launch two tile sizes per call)
    inst = {}
    for (disp, c), v in per.items():
        inst.setdefault((name[disp], c), []).append(v)
    m = {}
    for (n, c), v in inst.items():
        m[c] = m.get(c, 0.0) + sum(v) / len(v)
    idur = {}
    for disp, ns_ in dur.items():
        idur.setdefault(name[disp], []).append(ns_)
    lines = [f"kernel: {kernel}"] + [f"command: {c}" for c in commands]
    lines += [f"{c} per call: {m[c]:.6g}" for c in sorted(m)]
    if dur:
        ns = sum(sum(v) / len(v) for v in idur.values())
        lines.append(f"duration per call: {ns / 1e6:.3f} ms ({len(idur)} kernel instance(s), "
                     f"mean of {min(len(v) for v in idur.values())} dispatches each)")
    if "GRBM_GUI_ACTIVE" in m:
        cyc = m["GRBM_GUI_ACTIVE"] / 8.0
        if dur:
            lines.append(f"GPU clock: {cyc / ns:.3f} GHz (GRBM_GUI_ACTIVE / 8 / duration)")
        if m.get("SQ_VALU_MFMA_BUSY_CYCLES"):
            lines.append(f"MFMA busy: {m['SQ_VALU_MFMA_BUSY_CYCLES'] / (1024 * cyc):.3f} "
                         "of SIMD cycles")
        if "SQ_INSTS_VALU" in m:
            lines.append(f"VALU issue: {m['SQ_INSTS_VALU'] / (256 * cyc):.3f} wave instructions "
                         "per CU per cycle")
    if "SQ_WAIT_INST_LDS" in m and "SQ_WAVE_CYCLES" in m:
        lines.append(f"LDS instruction wait: {m['SQ_WAIT_INST_LDS'] / m['SQ_WAVE_CYCLES']:.3f}"
                     " of wave cycles")
    return "\n".join(lines) + "\n"


def trace_summary(d, log, commands):
    """The kernel statistics of a rocprofv3 --kernel-trace --stats csv run
    and the bench line of the same run (with the clock it measured)."""
    import csv
    import glob
    lines = [f"command: {c}" for c in commands]
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        lines += ["", f"rocprofv3 kernel stats ({os.path.basename(f)}):",
                  f"{'kernel':<72}{'calls':>7}{'avg_us':>13}{'min_us':>13}{'max_us':>13}{'pct':>7}"]
        with open(f) as fh:
            for r in csv.DictReader(fh):
                lines.append(f"{r['Name'][:71]:<72}{int(r['Calls']):>7}"
                             f"{float(r['AverageNs']) / 1e3:>13.1f}"
                             f"{float(r['MinNs']) / 1e3:>13.1f}{float(r['MaxNs']) / 1e3:>13.1f}"
                             f"{float(r['Percentage']):>7.2f}")
    bench = None
    with open(log) as fh:
        for line in fh:
            if line.startswith("{"):
                bench = json.loads(line)
    if bench is not None:
        def brief(b):
            return (f"value={b['value']:.4g} {b['unit']} ms_per_step={b['ms_per_step']:.3f} "
                    f"config={json.dumps(b['config'])} roofline={json.dumps(b['roofline'])}")
        lines += ["", "bench line (same run): " + brief(bench)]
        if "three_way" in bench:
            lines.append("  three_way: " + brief(bench["three_way"]))
        lines.append(f"GPU clock (bench clock probe, same run): {bench.get('gpu_clock_ghz')} GHz")
    return "\n".join(lines) + "\n"


def traffic_key(args, wl):
    """Workload and operand type of a run: names its traffic file."""
    if wl in ("levels_8192x32768", "binary_8192x32768", "levels_4096x1024"):
        return wl + {"mfma_fp4": "_fp4", "bits": "_bits"}.get(args.path, "_u8")
    return wl + {"f16": "_f16", "f64": "_f64"}.get(args.storage, "_f32")


def resolved_path(args, V, way):
    """The path the library runs for this input and --path (AUTO resolved by
    the library's own policy and tuning table)."""
    import numpy as np
    from paper_1705_08210_amd import ps
    levels = int(V.max()) if V.dtype == np.uint8 else 0
    code = ps.path_choice(V.dtype, way, V.shape[1], V.shape[0], path=args.path, levels=levels,
                          tile=args.tile)
    return {v: k for k, v in ps.PATH.items()}[code]


def _parity_pairs(Vh, c2_dev, n_v, m, seed, dev_to_host):
    """Sampled pairs of a 2-way output against the oracle."""
    import numpy as np

    import oracle
    g = np.random.default_rng(seed)
    I = g.integers(0, n_v, m)
    J = (I + 1 + g.integers(0, n_v - 1, m)) % n_v
    I, J = np.minimum(I, J), np.maximum(I, J)
    got = dev_to_host(c2_dev)[J * (J - 1) // 2 + I]
    return got, oracle.c2_pairs(Vh, I, J)


def _parity_triples(Vh, c3_dev, n_v, m, seed, dev_to_host):
    import numpy as np

    import oracle
    g = np.random.default_rng(seed)
    t = np.sort(g.integers(0, n_v, size=(3 * m, 3)), axis=1)
    t = t[(t[:, 0] < t[:, 1]) & (t[:, 1] < t[:, 2])][:m]
    i, j, k = t[:, 0], t[:, 1], t[:, 2]
    off = (n_v - 1) * (j * (j - 1) // 2) - ((j - 1) * j * (2 * j - 1)) // 6
    got = dev_to_host(c3_dev)[off + (k - j - 1) * j + i]
    return got, oracle.c3_triples(Vh, i, j, k)


def _errors(got, ref):
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    nz = ref > 0
    rel = np.abs(got[nz] - ref[nz]) / ref[nz]
    return {"tuples": int(len(ref)), "max_rel_err": float(rel.max()) if rel.size else 0.0,
            "max_abs_err": float(np.abs(got - ref).max()) if len(ref) else 0.0,
            "zero_mismatches": int(np.count_nonzero(got[~nz] != 0))}


def measure(args, wl, K, W, with_cpu=True):
    """Times K steps of one workload after W warm-ups; returns the bench
    line's fields (metric, value, roofline, parity sample, oracle rates)."""
    import numpy as np
    import torch

    import workloads
    from paper_1705_08210_amd import ps

    dev = torch.device("cuda:0")
    timer = Timer(torch)
    extra = {}
    f16_source = None          # FP16 storage: the FP32 input it was rounded from

    def to_host(t):
        torch.cuda.synchronize()
        return t.cpu().numpy()

    if wl in ("gwas_20000x16384", "uniform_1024x256", "levels_8192x32768",
              "binary_8192x32768"):
        V = workloads.WORKLOADS[wl](0)
        if args.storage == "f16" and V.dtype == np.float32:
            f16_source, V = V, workloads.to_f16(V)
        elif args.storage == "f64" and V.dtype == np.float32:
            V = V.astype(np.float64)
        n_v, n_f = V.shape
        Vd = torch.from_numpy(V).to(dev)
        s = torch.empty(n_v, dtype=torch.float64, device=dev)
        m = n_v * (n_v - 1) // 2
        c2 = torch.empty(m, dtype=torch.float32, device=dev)
        levels = int(V.max()) if V.dtype == np.uint8 else 0

        N = args.shard_of

        def step(rec):
            ps.vector_sums(Vd, out=s, want_bad=False)
            a = timer.mark() if rec else None
            if N > 1:
                ps.ps2_shard(Vd, 0, N, s=s, c2=c2, acc=args.acc, path=args.path,
                             levels=levels, tile=args.tile)
            else:
                ps.ps2(Vd, s=s, c2=c2, acc=args.acc, path=args.path, levels=levels,
                       tile=args.tile)
            if rec:
                timer.add(a, timer.mark())

        cmp = n_f * m
        if N > 1:   # the shard's pairs: those it writes into a NaN-filled output
            c2.fill_(float("nan"))
            ps.ps2_shard(Vd, 0, N, c2=c2, acc=args.acc, path=args.path, levels=levels,
                         tile=args.tile)
            shard_pairs = int((~torch.isnan(c2)).sum())
            cmp = n_f * shard_pairs
            # the whole call on the same box, for comparison (not the timed work)
            for _ in range(2):
                ps.ps2(Vd, s=s, c2=c2, acc=args.acc, path=args.path, levels=levels,
                       tile=args.tile)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(3):
                ps.ps2(Vd, s=s, c2=c2, acc=args.acc, path=args.path, levels=levels,
                       tile=args.tile)
            torch.cuda.synchronize()
            full_ms = (time.perf_counter() - t1) / 3 * 1e3
            c2.fill_(float("nan"))
            extra["shard"] = {"shard": 0, "of": N, "pairs": shard_pairs, "pairs_total": m,
                              "tiles": "upper-triangle tiles t with t mod N == 0",
                              "whole_call_ms": round(full_ms, 3),
                              "whole_call_cmp_per_s": n_f * m / (full_ms * 1e-3)}
        path = resolved_path(args, V, 2)
        if path == "bits":   # v_and + v_bcnt per 32 comparisons
            dtype, bound, ops_per_cmp, peak = "b1", "alu", 2.0 / 32, HALF_RATE_OPS_TOPS
            kernel = "ps_mg2_kernel"
        elif path == "mfma_fp4":   # e2m1 planes, FP32 sums
            dtype, bound, ops_per_cmp, peak = "fp4", "mfma", 2.0 * levels, FP4_MFMA_PEAK_TOPS
            kernel = "ps_mfma2_dma_kernel"
        elif path == "mfma":   # thermometer levels: `levels` int8 MACs (2 ops) per comparison
            dtype, bound, ops_per_cmp, peak = "u8", "mfma", 2.0 * levels, INT8_MFMA_PEAK_TOPS
            kernel = ("ps_mfma2_kernel" if args.tile == 2 else
                      "ps_mfma2_lvd_kernel" if n_f % 64 == 0 else "ps_mfma2_lv_kernel")
        elif V.dtype == np.uint8:   # v_sad_u8: 4 comparisons per op
            dtype, bound, ops_per_cmp, peak = "u8", "alu", 0.25, HALF_RATE_OPS_TOPS
            kernel = "ps_mg2_kernel"
        elif V.dtype == np.float64:  # v_min_f64 + v_add_f64 at the FP64 rate
            dtype, bound, ops_per_cmp, peak = "f64", "alu", 2.0, HALF_RATE_OPS_TOPS
            kernel = "ps_mg2_kernel"
        elif V.dtype == np.float16:  # pk_min + dot2 per 2 comparisons
            dtype, bound, ops_per_cmp, peak = "f16", "alu", 1.0, HALF_RATE_OPS_TOPS
            kernel = "ps_mg2_kernel"
        else:                        # min + add per comparison
            dtype, bound, ops_per_cmp, peak = "f32", "alu", 2.0, FP32_LANE_OPS_TOPS
            kernel = "ps_mg2_kernel"
        config = {"workload": wl, "way": 2, "n_f": n_f, "n_v": n_v, "path": path}
        if N > 1:
            config["shard"] = f"0 of {N}"
        cpu = (lambda: cpu_baseline(V, n_f, args.cpu_seconds, 2))

        def parity():
            if N > 1:   # pairs of the shard only
                import oracle
                h = to_host(c2)
                idx = np.flatnonzero(~np.isnan(h))
                idx = np.random.default_rng(7).choice(idx, 2048)
                J = ((1 + np.sqrt(1 + 8 * idx.astype(np.float64))) // 2).astype(np.int64)
                J -= (J * (J - 1) // 2 > idx)
                J += ((J + 1) * J // 2 <= idx)
                I = idx - J * (J - 1) // 2
                return _errors(h[idx], oracle.c2_pairs(V, I, J))
            got, ref = _parity_pairs(V, c2, n_v, 2048, 7, to_host)
            out = _errors(got, ref)
            if f16_source is not None:   # the user-visible error: against the FP32 input
                got, ref = _parity_pairs(f16_source, c2, n_v, 2048, 7, to_host)
                out["vs_fp32_source"] = _errors(got, ref)
            return out
    elif wl in ("sparse_4096x1024", "levels_4096x1024"):
        V = workloads.WORKLOADS[wl](0)
        if args.storage == "f16" and V.dtype == np.float32:
            f16_source, V = V, workloads.to_f16(V)
        elif args.storage == "f64" and V.dtype == np.float32:
            V = V.astype(np.float64)
        n_v, n_f = V.shape
        Vd = torch.from_numpy(V).to(dev)
        levels = int(V.max()) if V.dtype == np.uint8 else 0
        s = torch.empty(n_v, dtype=torch.float64, device=dev)
        n2 = torch.empty(n_v * (n_v - 1) // 2, dtype=ps.n2_dtype(Vd.dtype), device=dev)
        c3 = torch.empty(math.comb(n_v, 3), dtype=torch.float32, device=dev)

        def step(rec):
            ps.vector_sums(Vd, out=s, want_bad=False)
            ps.ps2(Vd, s=s, want_c2=False, want_n2=True, n2=n2, acc=args.acc,
                   tile=args.tile, path=args.path, levels=levels)
            a = timer.mark() if rec else None
            ps.ps3(Vd, s=s, n2=n2, c3=c3, acc=args.acc, tile=args.tile, path=args.path,
                   levels=levels)
            if rec:
                timer.add(a, timer.mark())

        def parity():
            got, ref = _parity_triples(V, c3, n_v, 2048, 7, to_host)
            out = _errors(got, ref)
            if f16_source is not None:
                got, ref = _parity_triples(f16_source, c3, n_v, 2048, 7, to_host)
                out["vs_fp32_source"] = _errors(got, ref)
            return out

        if args.campaign > 0:   # staged: every stage's bytes end in host memory
            from paper_1705_08210_amd import campaign
            host_out = np.empty(math.comb(n_v, 3), dtype=np.uint8)

            def sink(st):
                host_out[st.first:st.first + st.size] = st.u8.numpy()

            def step(rec):   # noqa: F811 -- the campaign replaces the plain step
                a = timer.mark() if rec else None
                campaign.run3(Vd, args.campaign, sink, reduce="u8", acc=args.acc,
                              tile=args.tile, path=args.path, levels=levels)
                if rec:
                    timer.add(a, timer.mark())
            extra["campaign"] = {"stages": args.campaign, "output": "u8 to host",
                                 "timed": "whole campaign (sums, pair numerators, stages, "
                                          "quantize, device-to-host copies, host sink)"}
            parity = None

        cmp = n_f * math.comb(n_v, 3)
        path = resolved_path(args, V, 3)
        if path == "mfma_fp4":   # e2m1 planes: `levels` MACs per comparison
            dtype, bound, ops_per_cmp, peak = "fp4", "mfma", 2.0 * levels, FP4_MFMA_PEAK_TOPS
            kernel = "ps_mfma3_kernel"
        elif path == "mfma":
            dtype, bound, ops_per_cmp, peak = "u8", "mfma", 2.0 * levels, INT8_MFMA_PEAK_TOPS
            # opts.tile 2: per-slab tiles; else the split tiling (pairs x vectors)
            kernel = ("ps_mfma3_lv_kernel" if args.tile == 2 else
                      "ps_mfma3_lvsd_kernel" if levels == 3 and n_f % 64 == 0 else
                      "ps_mfma3_lvs_kernel")
        elif V.dtype == np.uint8:
            dtype, bound, ops_per_cmp, peak = "u8", "alu", 0.25, HALF_RATE_OPS_TOPS
            kernel = "ps_mg3f_kernel"
        else:
            dtype = {np.dtype(np.float16): "f16", np.dtype(np.float64): "f64"}.get(V.dtype, "f32")
            bound = "alu"
            ops_per_cmp, peak = {"f16": (1.0, HALF_RATE_OPS_TOPS),
                                 "f64": (2.0, HALF_RATE_OPS_TOPS)}.get(dtype,
                                                                    (2.0, FP32_LANE_OPS_TOPS))
            kernel = "ps_mg3f_kernel"
        config = {"workload": wl, "way": 3, "n_f": n_f, "n_v": n_v, "path": path}
        cpu = (lambda: cpu_baseline(V, n_f, args.cpu_seconds, 3))
    elif wl == "batched_64_uneven":
        Vs_np = workloads.batched_64_uneven(0)
        Vs = [torch.from_numpy(x).to(dev) for x in Vs_np]
        cmp = sum(x.shape[1] * x.shape[0] * (x.shape[0] - 1) // 2 for x in Vs_np)
        outs = ps._batch_outputs(Vs)
        if args.per_problem:
            def step(rec):
                a = timer.mark() if rec else None
                for V_, (c, _, _) in zip(Vs, outs):
                    ps.ps2(V_, c2=c, acc=args.acc, tile=args.tile)
                if rec:
                    timer.add(a, timer.mark())
        else:
            plan = ps.BatchedPlan(Vs, outs=outs, acc=args.acc, tile=args.tile)

            def step(rec):
                a = timer.mark() if rec else None
                plan.run()
                if rec:
                    timer.add(a, timer.mark())
        dtype, bound, ops_per_cmp, peak = "f32", "alu", 2.0, FP32_LANE_OPS_TOPS
        kernel = "ps_mgb_kernel" if not args.per_problem else "ps_mg2_kernel"
        config = {"workload": wl, "way": 2, "problems": len(Vs),
                  "mode": "per-problem launches" if args.per_problem else "one graph"}
        big = max(range(len(Vs_np)), key=lambda t: Vs_np[t].size)
        cpu = (lambda: cpu_baseline(Vs_np[big], Vs_np[big].shape[1], args.cpu_seconds, 2))

        def parity():   # 64 pairs of every problem
            got, ref = [], []
            for p, (Vh, (c, _, _)) in enumerate(zip(Vs_np, outs)):
                g_, r_ = _parity_pairs(Vh, c, Vh.shape[0], 64, 100 + p, to_host)
                got.append(g_)
                ref.append(r_)
            return _errors(np.concatenate(got), np.concatenate(ref))
    else:
        raise ValueError(f"unknown workload {wl}")

    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        extra["copy_calibration_bytes"] = 1 << 30
        del src, dst

    for _ in range(W):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = timer.mean_ms()
    if args.campaign > 0:
        from paper_1705_08210_amd import campaign
        campaign.release()

    if parity is not None:   # sampled parity against the oracle (not timed)
        extra["parity_sample"] = parity()
    line = {
        "value": cmp * K / wall, "unit": "comparisons/s", "ms_per_step": wall / K * 1e3,
        "dtype": dtype, "config": config,
        "roofline": dict(roofline(bound, ops_per_cmp, cmp, kernel_ms, peak,
                                  None if args.shard_of > 1 else
                                  recorded_traffic(kernel, traffic_key(args, wl))),
                         kernel=kernel, kernel_ms=round(kernel_ms, 4)),
    }
    if with_cpu:
        line["cpu_baseline"] = cpu()
    line.update(extra)
    if wl == "batched_64_uneven" and not args.per_problem:
        plan.close()
    return line


def main(argv=None):
    args = parse(argv)
    if args.counter_summary:
        sys.stdout.write(counter_summary(args.counter_summary[0], args.counter_summary[1],
                                         args.pmc_command))
        return 0
    if args.trace_summary:
        sys.stdout.write(trace_summary(args.trace_summary[0], args.trace_summary[1],
                                       args.pmc_command))
        return 0
    if args.pmc_summary:
        fetch_dir, write_dir, kernel = args.pmc_summary
        sys.stdout.write(pmc_summary(fetch_dir, write_dir, kernel,
                                     traffic_key(args, args.workload), args.pmc_command))
        return 0
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        return 2

    import torch

    from paper_1705_08210_amd import ps

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if args.workload not in WORKLOADS:
        print(f"unknown workload {args.workload}", file=sys.stderr)
        return 2
    K, W = args.steps, args.warmup
    head = measure(args, args.workload, K, W, with_cpu=not args.no_cpu_baseline)
    line = {
        "metric": "elementwise comparisons/sec, 2-way & 3-way PS, 1 MI355X; % of VALU/MFMA peak",
        "value": head.pop("value"), "unit": head.pop("unit"), "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": head.pop("ms_per_step"), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head.pop("dtype"),
        "data": "synthetic (seeded numpy PCG64)", "config": head.pop("config"),
    }
    line.update(head)
    if args.workload == "gwas_20000x16384" and not args.no_3way and args.storage == "auto" \
            and args.campaign == 0:
        # the metric's 3-way half: the 3-way FP32 workload, same steps
        tw = measure(args, "sparse_4096x1024", K, W, with_cpu=not args.no_cpu_baseline)
        tw["steps"], tw["warmup"] = K, W
        line["three_way"] = tw
    line["gpu_clock_ghz"] = round(ps.clock_probe(), 3)
    print(json.dumps(line), flush=True)
    return 0


WORKLOADS = ("gwas_20000x16384", "uniform_1024x256", "levels_8192x32768", "binary_8192x32768",
             "sparse_4096x1024", "levels_4096x1024", "batched_64_uneven")


if __name__ == "__main__":
    sys.exit(main())
