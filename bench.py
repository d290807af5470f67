"""Benchmark: FP32 eval_vgh orbital-evals/s on the paper-scale table.

Workload: periodic 48^3 grid (51^3 padded), N = 2048 splines, FP32
coefficients uniform in (-1, 1), 512 positions uniform in the unit cell per
batch.  One step is one eval_vgh launch on each of 16 pre-generated batches,
so that repeated steps do not re-read the same rows from the Infinity Cache;
an event after every step gives the mean and the median step time.  Inputs
and outputs stay resident in HBM.

Printed: one JSON line with value = VGH orbital-evals/s (positions * N /
time), the HBM roofline of the kernel (algorithmic bytes 64*4 + 10*4 per
eval) against the 8 TB/s peak and the measured 86/14 streaming ceiling, the
FP64 oracle timed on the host cores as cpu_baseline with the error of every
output component of the FP32/FP16/BF16 tables against it, and extras: V and
VGL, a hexagonal cell, plain against spline-blocked tables, FP16/BF16
against FP32 at 512 and 4096 positions, the four-table batched workload,
the fused ratios, the latency mode, the interpolating fit and the 96^3 x
4096 tables.

Modes for profiling: --profile (headline kernel only, few steps; with
--npos/--dtype/--tile, --batched or --large for the other workloads),
--copy-probe (a plain device copy of known size, to scale HBM counters),
--stream-probe GIB (the 86/14 ceiling probe alone); --sweep prints the
throughput-vs-N and tile-width study instead of the benchmark line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "VGH orbital-evals/s + achieved HBM GB/s; FP16-table vs FP32 at stated err"
HBM_PEAK_GBS = 8000.0
GRID = (48, 48, 48)
NSPL = 2048
NPOS = 512
NBATCH = 16
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_eval_vgh_f32_48cubed_N2048_512pos.txt")
# sources of the FP32 evaluation kernel (the one the counter profile covers)
KERNEL_SRCS = [os.path.join(ROOT, "paper_1611_02665_amd", "csrc", f)
               for f in ("eval_device.hpp", "eval_f32.hip", "internal.hpp")]
# Tile wisdom for gfx950, written by the autotuner (python bench.py --retune)
WISDOM_FILE = os.path.join(ROOT, "paper_1611_02665_amd", "wisdom_gfx950.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters(tile):
    """The committed counter summary's values, if it was taken on the current
    kernel source with the same tile (else None)."""
    if not os.path.exists(PMC_FILE):
        return None
    vals = {}
    for line in open(PMC_FILE):
        if line.startswith("#") or "=" not in line:
            continue
        k, v = line.split("=", 1)
        vals[k.strip()] = v.strip()
    if vals.get("kernel_sha256_16") != kernel_hash():
        return None
    if vals.get("tile") != ",".join(str(x) for x in tile.as_tuple()):
        return None
    return vals


def read_traffic(per_launch_alg_bytes, tile):
    """HBM bytes per launch from the committed counter summary (or None)."""
    vals = read_counters(tile)
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def read_l2_hit_rate(tile):
    """L2 hits / (hits + misses) of the headline launch from the same summary."""
    vals = read_counters(tile)
    try:
        hits = float(vals["l2_hits_per_dispatch"])
        return hits / (hits + float(vals["l2_misses_per_dispatch"]))
    except (KeyError, ValueError, TypeError, ZeroDivisionError):
        return None


def wisdom_holds(torch, kind, npos):
    """Whether the wisdom file has an entry for the headline table shape on
    this device's architecture (keys: single|arch|dtype|kind|N|grid|p<pow2>)."""
    if not os.path.exists(WISDOM_FILE):
        return False
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    bucket = 1
    while bucket < npos:
        bucket <<= 1
    key = f"single|{arch}|f32|{kind}|N{NSPL}|{GRID[0]}x{GRID[1]}x{GRID[2]}|p{bucket}"
    with open(WISDOM_FILE) as f:  # key vw wx wy grid order split [time_us]
        return any(len(line.split()) >= 8 and line.split()[0] == key for line in f)


def timed(torch, fn, steps, warmup):
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(steps):
        fn(i)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps  # ms per call


def timed_steps(torch, fn, nb, steps, warmup):
    """Timed region of exactly `steps` steps, each one launch per batch of the
    nb batches (fn(i) launches batch i % nb), with an event after every
    step.  Returns (mean ms per step over the region, per-step ms list)."""
    for i in range(warmup * nb):
        fn(i)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for s in range(steps):
        for b in range(nb):
            fn(s * nb + b)
        ev[s + 1].record()
    torch.cuda.synchronize()
    per = [ev[s].elapsed_time(ev[s + 1]) for s in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / steps, per


def memory_ceiling(torch, B, footprints_gib=(1, 16)):
    """Best bandwidth of the streaming probe (spline_stream_probe: 6 reads of
    16 bytes per 16-byte write, the evaluation's 86/14 read/write mix) over
    its launch variants, at each footprint (reads plus writes): reads from
    six planes, from one 6 KiB span per wavefront in order, or from spans
    drawn at random (the statistics of rows gathered for random positions,
    Infinity Cache hits included)."""
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for gib in footprints_gib:
        units = (gib << 30) // 112 // 64 * 64
        src = torch.ones(6 * units * 4, dtype=torch.int32, device="cuda")
        dst = torch.empty(units * 4, dtype=torch.int32, device="cuda")
        modes = {"planes": 0, "chunked": B.BSPL_PROBE_CHUNKED, "random": B.BSPL_PROBE_RANDOM}
        row = {}
        for mname, mflag in modes.items():
            best = None
            for nt in (0, B.BSPL_PROBE_NT_STORES):
                for u in (1, 2, 4):
                    for grid in (0, 2048, 8192):
                        # a new salt per call: random spans differ between calls
                        ms = timed(torch, lambda i: B.spline_stream_probe(
                            src, dst, units, u, grid, mflag | nt, 1000 + i, stream),
                            20 if gib == 1 else 5, 2)
                        gbs = 112 * units / (ms * 1e-3) / 1e9
                        if best is None or gbs > best[0]:
                            best = (gbs, u, grid, nt)
            row[mname] = {"gbs": best[0], "per_lane": best[1], "grid": best[2],
                          "nt_stores": bool(best[3])}
        torch.cuda.synchronize()
        if int(dst[0].item()) != 6:
            raise RuntimeError("stream probe wrote a wrong sum")
        top = max(row, key=lambda k: row[k]["gbs"])
        row["best_mode"] = top
        row["gbs"] = row[top]["gbs"]
        out[f"mix_86_14_{gib}GiB"] = row
        del src, dst
        torch.cuda.empty_cache()
    return out


def copy_probe(torch, nbytes=1 << 30, reps=20):
    """Plain device-to-device copy of known size (calibration of the HBM
    traffic counters: the bytes it reads and writes are known)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ms = timed(torch, lambda i: dst.copy_(src), reps, 3)
    return 2.0 * nbytes / (ms * 1e-3) / 1e9, ms


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=125,
                    help="timed steps; a step is one launch on each of the 16 batches")
    ap.add_argument("--warmup", type=int, default=3, help="untimed steps before them")
    ap.add_argument("--profile", action="store_true", help="headline kernel only")
    ap.add_argument("--blocked", action="store_true",
                    help="profiling: a spline-blocked table instead of the plain one")
    ap.add_argument("--copy-probe", action="store_true", help="only a 1 GiB device copy")
    ap.add_argument("--stream-probe", type=float, default=None, metavar="GIB",
                    help="only the 86/14 streaming probe over a footprint of GIB GiB "
                         "(six planes, 2 units per lane), 5 warm-up and 20 timed calls")
    ap.add_argument("--tile", default=None,
                    help="profiling: fixed tile vw,wx,wy,grid,order instead of the wisdom")
    ap.add_argument("--retune", action="store_true",
                    help="autotune the headline tile and append it to the wisdom file")
    ap.add_argument("--npos", type=int, default=NPOS,
                    help="profiling: positions per batch (the benchmark itself uses 512)")
    ap.add_argument("--sweep", action="store_true",
                    help="throughput vs N (128..4096 at 48^3) and vs tile size at N=2048, "
                         "one JSON line each, instead of the benchmark line")
    ap.add_argument("--dtype", default="f32", choices=("f32", "f16", "bf16"),
                    help="profiling: table dtype of the --profile run")
    ap.add_argument("--batched", action="store_true",
                    help="profiling: the four-table plan (autotuned, or --tile), 20 replays")
    ap.add_argument("--large", action="store_true",
                    help="profiling: eval_vgh on the 96^3 x N=4096 table (--dtype), 8192 "
                         "positions per batch, 2 batches, autotuned or --tile, 20 launches")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args(argv)
    if args.blocked and not args.profile:
        ap.error("--blocked is for --profile runs")

    if (args.npos != NPOS or args.dtype != "f32" or args.batched or args.large) \
            and not args.profile:
        ap.error("--npos, --dtype, --batched and --large are for --profile runs only")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the evaluation "
              "shards by replicating the table and splitting positions, with no "
              "communication, so the per-GPU figure is the whole story.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_1611_02665_amd import accounting as A
    from paper_1611_02665_amd import binding as B

    torch.cuda.set_device(0)
    if args.sweep:
        return sweep_mode(torch, B, A, synth)
    if args.copy_probe:
        gbs, ms = copy_probe(torch)
        print(json.dumps({"copy_probe_bytes": 1 << 30, "copy_ms": ms, "copy_gbs": gbs}))
        return 0
    if args.stream_probe is not None:
        units = int(args.stream_probe * (1 << 30)) // 112 // 64 * 64
        src = torch.ones(6 * units * 4, dtype=torch.int32, device="cuda")
        dst = torch.empty(units * 4, dtype=torch.int32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        ms = timed(torch, lambda i: B.spline_stream_probe(src, dst, units, 2, 0,
                                                          B.BSPL_PROBE_NT_STORES, 0, stream),
                   20, 5)
        print(json.dumps({"stream_probe_bytes": 112 * units, "ms": ms,
                          "gbs": 112 * units / (ms * 1e-3) / 1e9}))
        return 0
    if args.batched:
        return batched_profile(torch, B, A, synth, args)
    if args.large:
        return large_profile(torch, B, A, synth, args)

    t0 = time.time()
    coef = synth.coef_table(*GRID, NSPL, stream=synth.table_stream(0))
    log(f"[bench] coefficients generated in {time.time() - t0:.1f}s")
    t32 = B.spline_table_create(*GRID, NSPL, coef, args.dtype,
                                flags=B.BSPL_LAYOUT_BLOCKED if args.blocked else 0)
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    npos = args.npos
    nbatch = NBATCH if npos <= NPOS else 4
    batches = [torch.from_numpy(synth.positions(npos, stream=synth.position_stream(0), batch=b))
               .to(dev) for b in range(nbatch)]
    ldo = NSPL
    v = torch.empty(npos, ldo, device=dev)
    g = torch.empty(npos, 3, ldo, device=dev)
    h = torch.empty(npos, 6, ldo, device=dev)
    l = torch.empty(npos, ldo, device=dev)
    pp = [b.data_ptr() for b in batches]
    vp, gp, hp, lp = v.data_ptr(), g.data_ptr(), h.data_ptr(), l.data_ptr()
    if args.tile:
        tile, tile_source = B.bspl_tile(*[int(x) for x in args.tile.split(",")]), "fixed"
    elif args.retune:
        tile, tile_source = B.spline_autotune(t32, "vgh", npos, WISDOM_FILE), "autotune"
    else:
        # the tile the autotuner chose for this shape on this architecture,
        # else a live sweep (recorded in the in-process wisdom)
        tile_source = ("wisdom" if args.dtype == "f32" and wisdom_holds(torch, "vgh", npos)
                       else "autotune")
        if tile_source == "wisdom":
            B.spline_wisdom_load(WISDOM_FILE)
            tile = B.spline_tile_select(t32, "vgh", npos)
        else:
            tile = B.spline_autotune(t32, "vgh", npos)
    log(f"[bench] table ready, tile {tile} ({tile_source})")
    tref = B.ctypes.byref(tile)

    def vgh_step(i):
        B._check(B.lib.spline_eval(t32, B.BSPL_VGH, npos, pp[i % nbatch], vp, gp, hp, ldo, tref,
                                   stream), "spline_eval")

    steps = 2 if args.profile else args.steps
    warmup = 1 if args.profile else args.warmup
    ms_step, per_step = timed_steps(torch, vgh_step, nbatch, steps, warmup)
    ms = ms_step / nbatch  # mean launch duration over the timed region
    evals = npos * NSPL
    value = evals / (ms * 1e-3)
    alg_bytes = A.batch_bytes("vgh", args.dtype, npos, NSPL)
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    log(f"[bench] VGH {ms * 1e3:.2f} us/launch, {value:.4g} evals/s, {achieved:.0f} GB/s")
    if args.profile:
        B.spline_table_destroy(t32)
        return 0
    per_step.sort()
    med_step = per_step[len(per_step) // 2] if len(per_step) % 2 else \
        0.5 * (per_step[len(per_step) // 2 - 1] + per_step[len(per_step) // 2])

    traffic = read_traffic(alg_bytes, tile)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "orbital-evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_step,
        "median_ms_per_step": med_step,
        "us_per_launch": ms * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "eval_vgh, 48^3 periodic grid (51^3 padded) x N=2048 FP32 table "
                        "(1.09 GB), 512 uniform positions per batch; one step = one launch "
                        "on each of 16 pre-generated batches (8192 positions)",
            "launches_per_step": nbatch,
            "grid": list(GRID), "n_splines": NSPL, "npos": NPOS, "kernel": "eval_vgh",
            "table_dtype": "f32", "tile": list(tile.as_tuple()), "tile_source": tile_source,
        },
        "hbm_gbs": achieved,
        # the paper prints no absolute evals/s; its measured VGH read bandwidth
        # bounds its rate (other hardware, single precision)
        "paper_context": {
            "hardware": "Xeon Phi 7250P (KNL, 68 cores, MCDRAM)",
            "vgh_read_gbs": 238, "n_splines": 256,
            "implied_vgh_evals_per_s_max": 238e9 / (64 * 4),
            "note": "SoA VGH kernel, AoS-to-SoA subsection of the results"},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "l2_hit_rate": read_l2_hit_rate(tile),
            "alg_bytes_per_launch": alg_bytes,
            "bytes_per_eval": A.bytes_per_eval("vgh", "f32"),
        },
    }

    # context: the fraction of a batch's row reads that are unique (no
    # reuse credited in the algorithmic bytes), lambda = 64 npos / points
    lam = 64.0 * NPOS / float((GRID[0] + 3) * (GRID[1] + 3) * (GRID[2] + 3))
    line["config"]["unique_row_fraction"] = (1.0 - math.exp(-lam)) / lam
    line["gpu_clocks"] = gpu_clocks()
    extra = {}
    keep = {}
    # the extras time single launches: warm-up launches and repetitions
    warmup = max(10, warmup * nbatch)
    steps = max(200, steps * nbatch // 4)
    if not args.no_extras:
        # V and VGL on the same table and batches
        tile_v = B.spline_autotune(t32, "v", NPOS)
        ms_v = timed(torch, lambda i: B.spline_eval(t32, "v", NPOS, pp[i % nbatch], v, None, None,
                                                    ldo, tile=tile_v, stream=stream),
                     max(100, steps // 2), warmup)
        extra["v"] = {"evals_per_s": evals / (ms_v * 1e-3), "us_per_launch": ms_v * 1e3,
                      "hbm_gbs": A.batch_bytes("v", "f32", NPOS, NSPL) / (ms_v * 1e-3) / 1e9,
                      "tile": list(tile_v.as_tuple())}
        def vgl_step(i):
            B.spline_eval_vgl(t32, NPOS, pp[i % nbatch], vp, gp, lp, ldo, stream)
        tile_l = B.spline_autotune(t32, "vgl", NPOS)
        ms_l = timed(torch, vgl_step, max(100, steps // 2), warmup)
        extra["vgl"] = {"evals_per_s": evals / (ms_l * 1e-3), "us_per_launch": ms_l * 1e3,
                        "hbm_gbs": A.batch_bytes("vgl", "f32", NPOS, NSPL) / (ms_l * 1e-3) / 1e9,
                        "tile": list(tile_l.as_tuple())}
        # the same coefficients on a hexagonal cell (a general lattice: grid
        # coordinates u = M r, derivatives carried to Cartesian ones)
        # (positions uniform in the cell: r = s A with the same s batches)
        hexcell = [[1.0, 0.0, 0.0], [-0.5, 0.75 ** 0.5, 0.0], [0.0, 0.0, 1.6]]
        thex = B.spline_table_create_lattice(*GRID, NSPL, coef, hexcell)
        cell_t = torch.tensor(hexcell, dtype=torch.float64, device=dev).t().contiguous()
        hex_batches = [(cell_t @ b).contiguous() for b in batches]
        hpp = [b.data_ptr() for b in hex_batches]
        extra["lattice_hex"] = {}
        for kind, ob in (("vgh", hp), ("vgl", lp)):
            ht = B.spline_autotune(thex, kind, NPOS)
            href = B.ctypes.byref(ht)
            ms_h = timed(torch, lambda i: B._check(B.lib.spline_eval(
                thex, B.KINDS[kind], NPOS, hpp[i % nbatch], vp, gp, ob, ldo, href, stream),
                "spline_eval"), max(100, steps // 2), warmup)
            extra["lattice_hex"][kind] = {
                "evals_per_s": evals / (ms_h * 1e-3), "us_per_launch": ms_h * 1e3,
                "hbm_gbs": A.batch_bytes(kind, "f32", NPOS, NSPL) / (ms_h * 1e-3) / 1e9,
                "tile": list(ht.as_tuple())}
        B.spline_table_destroy(thex)
        extra["layout"] = layout_extra(torch, B, synth, coef, t32, steps, warmup)
        log("[bench] layout extra done")
        # the FP16 table on the headline's own 512-position batches
        # (the two dtypes timed interleaved: 25 reps of 16 launches, medians)
        t16 = B.spline_table_create(*GRID, NSPL, coef, "f16")
        tile16 = B.spline_autotune(t16, "vgh", NPOS)
        pair = interleaved(torch, [
            lambda i: B.spline_eval(t32, "vgh", NPOS, pp[i % nbatch], v, g, h, ldo, tile=tile,
                                    stream=stream),
            lambda i: B.spline_eval(t16, "vgh", NPOS, pp[i % nbatch], v, g, h, ldo, tile=tile16,
                                    stream=stream)], nbatch, reps=25)
        ms32i, ms16 = median(pair[0]), median(pair[1])
        B.spline_table_destroy(t16)
        extra["f16_headline_batches"] = {
            "evals_per_s": evals / (ms16 * 1e-3), "us_per_launch": ms16 * 1e3,
            "hbm_gbs": A.batch_bytes("vgh", "f16", NPOS, NSPL) / (ms16 * 1e-3) / 1e9,
            "tile": list(tile16.as_tuple()), "f32_us_per_launch_interleaved": ms32i * 1e3,
            "speedup_vs_f32_headline": ms32i / ms16}
        # interpolating coefficients from grid values (table set-up, once per
        # orbital set): one HBM read and one write per element and axis
        vals = torch.from_numpy(coef).to(dev)
        fitted = torch.empty_like(vals)
        ms_f = timed(torch, lambda i: B.spline_fit_interpolating(*GRID, NSPL, vals, fitted,
                                                                 stream=stream), 10, 2)
        fit_bytes = 3 * 8 * vals.numel()
        extra["fit_interpolating"] = {"ms": ms_f, "alg_bytes": fit_bytes,
                                      "hbm_gbs": fit_bytes / (ms_f * 1e-3) / 1e9}
        del vals, fitted
        # fused determinant ratios on the same workload: 64*4 table bytes +
        # 4 bytes of inverse-matrix row per eval, no N-wide output rows
        ainv = torch.randn(NPOS, NSPL, device=dev)
        rout = torch.empty(NPOS, 10, dtype=torch.float64, device=dev)
        for kind, nc in (("vgh", 10), ("vgl", 5)):
            best = None
            for rt in [(vw, wx, 1, 0, 0) for vw in (1, 2, 4) for wx in (2, 4, 8)]:
                ms_r = timed(torch, lambda i: B.spline_eval_ratio(
                    t32, kind, NPOS, pp[i % nbatch], ainv, NSPL, rout, tile=rt, stream=stream),
                    50, 5)
                if best is None or ms_r < best[1]:
                    best = (rt, ms_r)
            rt = best[0]
            ms_r = timed(torch, lambda i: B.spline_eval_ratio(t32, kind, NPOS, pp[i % nbatch],
                                                              ainv, NSPL, rout, tile=rt,
                                                              stream=stream),
                         max(100, steps // 2), warmup)
            rb = NPOS * NSPL * (64 * 4 + 4) + NPOS * (24 + 8 * nc)
            extra[f"ratio_{kind}"] = {"evals_per_s": evals / (ms_r * 1e-3),
                                      "us_per_launch": ms_r * 1e3, "tile": list(rt),
                                      "alg_bytes_per_launch": rb,
                                      "hbm_gbs": rb / (ms_r * 1e-3) / 1e9}
        # the practical memory ceiling with the kernel's read/write mix
        ceil = memory_ceiling(torch, B)
        extra["memory_ceiling"] = ceil
        line["roofline"]["measured_ceiling_gbs"] = ceil["mix_86_14_1GiB"]["gbs"]
        line["roofline"]["frac_of_measured_ceiling"] = achieved / ceil["mix_86_14_1GiB"]["gbs"]
        log("[bench] memory ceiling probe done")
        extra["precision"] = precision_extra(torch, np, B, A, synth, coef, t32, steps, warmup)
        log("[bench] precision extra done")
        extra["batched"] = batched_extra(torch, B, A, synth, steps, warmup, keep)
        log("[bench] batched extra done")
        extra["latency"] = latency_extra(torch, B, synth, t32)
        log("[bench] latency extra done")
        extra["large"] = large_extra(torch, B, A, synth, warmup)
        log("[bench] large-table extra done")
        line["extra"] = extra

    samples = None if args.no_cpu else gpu_samples(torch, np, B, synth, coef, t32)
    B.spline_table_destroy(t32)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(np, synth, coef)
        line["cpu_baseline"]["error_vs_oracle"] = oracle_errors(
            np, coef, samples, sample_positions(np, synth))
        log("[bench] oracle errors done")
        line["cpu_baseline"]["per_config"] = cpu_oracle_configs(np, synth, coef,
                                                               keep.get("cfg4_coefs"))
    print(json.dumps(line), flush=True)
    return 0


def precision_extra(torch, np, B, A, synth, coef, t32, steps, warmup):
    """FP16 and BF16 tables vs FP32 on the same 4096-position batches.

    Each dtype runs at its own autotuned tile (and, as context, its best
    input-order tile and the batch-plan forms).  The three dtypes of one
    form are timed back to back (interleaved(): 15 repetitions of 4
    launches each, rotating which goes first, medians), so that clock and
    cache drift between separate timing loops cannot decide the ratios.
    The deviation from the FP32-table outputs on 64 positions is context;
    the errors against the FP64 oracle are in cpu_baseline.error_vs_oracle."""
    npos = 4096
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    nb = 4
    batches = [torch.from_numpy(synth.positions(npos, stream=synth.position_stream(0),
                                                batch=100 + b)).to(dev) for b in range(nb)]
    v = torch.empty(npos, NSPL, device=dev)
    g = torch.empty(npos, 3, NSPL, device=dev)
    h = torch.empty(npos, 6, NSPL, device=dev)
    dts = ("f32", "f16", "bf16")
    tabs = {dt: (t32 if dt == "f32" else B.spline_table_create(*GRID, NSPL, coef, dt))
            for dt in dts}
    tiles = {dt: B.spline_autotune(tabs[dt], "vgh", npos) for dt in dts}
    in_tiles = {dt: best_input_order(torch, B, tabs[dt], dt, npos, batches, nb, v, g, h, stream)
                for dt in dts}

    def eval_fn(dt, tile):
        t = tabs[dt]
        return lambda i: B.spline_eval(t, "vgh", npos, batches[i % nb], v, g, h, NSPL,
                                       tile=tile, stream=stream)

    ms = dict(zip(dts, map(median, interleaved(torch, [eval_fn(d, tiles[d]) for d in dts],
                                               4, reps=15))))
    ms_in = dict(zip(dts, map(median, interleaved(
        torch, [eval_fn(d, in_tiles[d]) for d in dts], 4, reps=15))))
    # the batched form: the same work as one launch replayed from a HIP graph,
    # with the plan's own autotuned tile, and with the best input-order tile
    plans, plans_in = {}, {}
    for dt in dts:
        plans[dt] = [B.spline_batch_plan_create([tabs[dt]], [npos], "vgh", [b], [v], [g], [h],
                                                [NSPL], stream=stream) for b in batches]
        plans_in[dt] = [B.spline_batch_plan_create([tabs[dt]], [npos], "vgh", [b], [v], [g], [h],
                                                   [NSPL], tile=tuple(in_tiles[dt][:3]) + (0, 0, 1),
                                                   stream=stream) for b in batches]

    def plan_fn(pl):
        return lambda i: B.spline_batch_execute(pl[i % len(pl)], stream)

    ms_b = dict(zip(dts, map(median, interleaved(torch, [plan_fn(plans[d]) for d in dts],
                                                 4, reps=15))))
    ms_bi = dict(zip(dts, map(median, interleaved(torch, [plan_fn(plans_in[d]) for d in dts],
                                                  4, reps=15))))
    ptiles = {dt: B.spline_batch_plan_tile(plans[dt][0]) for dt in dts}
    for dt in dts:
        for pl in plans[dt] + plans_in[dt]:
            B.spline_batch_plan_destroy(pl)
    # deviation on 64 positions from the FP32-table outputs (context)
    sample = synth.positions(64, stream=synth.position_stream(0), batch=100)
    sample_d = torch.from_numpy(sample).to(dev)  # [3][64]: npos is also the row stride
    out, ref = {}, None
    for dt in dts:
        B.spline_eval_vgh(tabs[dt], 64, sample_d.data_ptr(), v.data_ptr(), g.data_ptr(),
                          h.data_ptr(), NSPL, stream)
        torch.cuda.synchronize()
        got = {"v": v[:64].cpu().numpy().astype(np.float64),
               "g": g[:64].cpu().numpy().astype(np.float64),
               "h": h[:64].cpu().numpy().astype(np.float64)}
        if ref is None:
            ref = got
        errs = {}
        for name in ("v", "g", "h"):
            a, r = got[name], ref[name]
            if r.ndim == 2:
                errs[name] = float(np.abs(a - r).max() / np.abs(r).max())
            else:
                for c in range(r.shape[1]):
                    key = name + ("xyz"[c] if name == "g" else
                                  ["xx", "xy", "xz", "yy", "yz", "zz"][c])
                    errs[key] = float(np.abs(a[:, c] - r[:, c]).max() / np.abs(r[:, c]).max())
        out[dt] = {"evals_per_s": npos * NSPL / (ms[dt] * 1e-3), "us_per_launch": ms[dt] * 1e3,
                   "hbm_gbs": A.batch_bytes("vgh", dt, npos, NSPL) / (ms[dt] * 1e-3) / 1e9,
                   "tile": list(tiles[dt].as_tuple()),
                   "input_order_evals_per_s": npos * NSPL / (ms_in[dt] * 1e-3),
                   "input_order_us_per_launch": ms_in[dt] * 1e3,
                   "input_order_tile": list(in_tiles[dt]),
                   "batched_evals_per_s": npos * NSPL / (ms_b[dt] * 1e-3),
                   "batched_us_per_launch": ms_b[dt] * 1e3,
                   "batched_tile": list(ptiles[dt].as_tuple()),
                   "batched_input_order_evals_per_s": npos * NSPL / (ms_bi[dt] * 1e-3),
                   "max_norm_err_vs_f32_table": max(errs.values()),
                   "err_vs_f32_table_per_component": errs}
    for dt in ("f16", "bf16"):
        B.spline_table_destroy(tabs[dt])
        for key in ("evals_per_s", "input_order_evals_per_s", "batched_evals_per_s",
                    "batched_input_order_evals_per_s"):
            name = key.replace("evals_per_s", "speedup_vs_f32")
            out[dt][name] = out[dt][key] / out["f32"][key]
    out["npos"] = npos
    out["workload"] = ("eval_vgh on the same 48^3 x N=2048 coefficients stored as FP32, FP16 "
                       "and BF16 (per-spline FP32 scales), 4096 uniform positions per batch, "
                       "4 batches cycled; the dtypes of each form timed interleaved (15 reps "
                       "of 4 launches, medians); deviation on 64 positions from the "
                       "FP32-table outputs, normalised per component by max|reference|")
    return out


def best_input_order(torch, B, t, dt, npos, batches, nb, v, g, h, stream):
    """Fastest input-order (order = 0) tile from a small sweep."""
    vws = (1, 2, 4) if dt == "f32" else (2, 4, 8)
    best = None
    for vw in vws:
        for wx, wy in ((4, 1), (2, 1), (2, 2), (1, 4)):
            tile = (vw, wx, wy, 0, 0)
            ms = timed(torch, lambda i: B.spline_eval(t, "vgh", npos, batches[i % nb], v, g, h,
                                                      NSPL, tile=tile, stream=stream), 20, 3)
            if best is None or ms < best[1]:
                best = (tile, ms)
    return best[0]


CFG4 = [((32, 32, 32), 256, 97), ((40, 40, 40), 512, 512), ((48, 48, 48), 1152, 1500),
        ((64, 64, 64), 2048, 3000)]


def large_profile(torch, B, A, synth, args):
    """eval_vgh on the 96^3 x N=4096 table alone (for counter and trace runs):
    --dtype, autotuned or --tile, 5 warm-up and 20 timed launches alternating
    two 8192-position batches."""
    grid, n, npos = (96, 96, 96), 4096, 8192
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    src = synth.coef_table_torch(torch, *grid, n, device=dev, stream=synth.table_stream(0))
    t = B.spline_table_create(*grid, n, src, args.dtype, flags=B.BSPL_COEFS_DEVICE)
    del src
    torch.cuda.empty_cache()
    pos = [torch.from_numpy(synth.positions(npos, stream=synth.position_stream(0), batch=b))
           .to(dev) for b in range(2)]
    v = torch.empty(npos, n, device=dev)
    g = torch.empty(npos, 3, n, device=dev)
    h = torch.empty(npos, 6, n, device=dev)
    tile = (B.bspl_tile(*[int(x) for x in args.tile.split(",")]) if args.tile
            else B.spline_autotune(t, "vgh", npos))
    ms = timed(torch, lambda i: B.spline_eval(t, "vgh", npos, pos[i % 2], v, g, h, n, tile=tile,
                                              stream=stream), 20, 5)
    alg = A.batch_bytes("vgh", args.dtype, npos, n)
    log(f"[bench] large {args.dtype} tile {tile}: {ms * 1e3:.1f} us/launch, "
        f"{alg / (ms * 1e-3) / 1e9:.0f} GB/s")
    B.spline_table_destroy(t)
    return 0


def batched_profile(torch, B, A, synth, args):
    """The four-table plan alone (for counter and trace runs): autotuned or
    --tile, 5 warm-up and 20 timed replays of one position set."""
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    tabs = [B.spline_table_create(*grid, n, synth.coef_table(*grid, n, stream=synth.table_stream(i)),
                                  args.dtype) for i, (grid, n, _) in enumerate(CFG4)]
    npos = [c[2] for c in CFG4]
    pos = [torch.from_numpy(synth.positions(m, stream=synth.position_stream(i))).to(dev)
           for i, m in enumerate(npos)]
    outs = [(torch.empty(m, n, device=dev), torch.empty(m, 3, n, device=dev),
             torch.empty(m, 6, n, device=dev)) for (_, n, m) in CFG4]
    tile = B.bspl_tile(*[int(x) for x in args.tile.split(",")]) if args.tile else None
    plan = B.spline_batch_plan_create(tabs, npos, "vgh", pos, [o[0] for o in outs],
                                      [o[1] for o in outs], [o[2] for o in outs],
                                      [n for (_, n, _) in CFG4], tile=tile, stream=stream)
    ms = timed(torch, lambda i: B.spline_batch_execute(plan, stream), 20, 5)
    alg = sum(A.batch_bytes("vgh", args.dtype, m, n) for (_, n, m) in CFG4)
    log(f"[bench] batched {args.dtype} plan tile {B.spline_batch_plan_tile(plan)}: "
        f"{ms * 1e3:.1f} us/replay, {alg / (ms * 1e-3) / 1e9:.0f} GB/s")
    B.spline_batch_plan_destroy(plan)
    for t in tabs:
        B.spline_table_destroy(t)
    return 0


def batched_extra(torch, B, A, synth, steps, warmup, keep=None):
    """Four tables of uneven shape and batch size in one launch replayed from
    a HIP graph, FP32 and FP16 tables, each plan at its autotuned tile; the
    two dtypes timed back to back (15 repetitions of 4 replays, rotating
    which goes first, medians), as graph replays and as direct launches.
    The host coefficients are left in keep["cfg4_coefs"] for the CPU leg."""
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    coefs = [synth.coef_table(*grid, n, stream=synth.table_stream(i))
             for i, (grid, n, _) in enumerate(CFG4)]
    if keep is not None:
        keep["cfg4_coefs"] = coefs
    npos = [c[2] for c in CFG4]
    nb = 2
    pos = [[torch.from_numpy(synth.positions(m, stream=synth.position_stream(i), batch=b))
            .to(dev) for i, m in enumerate(npos)] for b in range(nb)]
    outs = [(torch.empty(m, n, device=dev), torch.empty(m, 3, n, device=dev),
             torch.empty(m, 6, n, device=dev)) for (_, n, m) in CFG4]
    evals = sum(n * m for (_, n, m) in CFG4)
    res = {"evals_per_replay": evals,
           "workload": "eval_vgh, tables 32^3xN=256, 40^3xN=512, 48^3xN=1152, 64^3xN=2048 "
                       "with 97/512/1500/3000 uniform positions, one launch per "
                       "replay, 2 position sets alternated; FP32 and FP16 timed "
                       "interleaved (15 reps of 4 replays, medians)"}
    dts = ("f32", "f16")
    tabs, plans = {}, {}
    for dt in dts:
        tabs[dt] = [B.spline_table_create(*grid, n, c, dt)
                    for (grid, n, _), c in zip(CFG4, coefs)]
        plans[dt] = [B.spline_batch_plan_create(tabs[dt], npos, "vgh", pos[b],
                                                [o[0] for o in outs], [o[1] for o in outs],
                                                [o[2] for o in outs], [n for (_, n, _) in CFG4],
                                                stream=stream) for b in range(nb)]
    ms = dict(zip(dts, map(median, interleaved(
        torch, [lambda i, d=d: B.spline_batch_execute(plans[d][i % nb], stream) for d in dts],
        4, reps=15))))
    # the same plans issued as plain kernel launches (no graph)
    ms_d = dict(zip(dts, map(median, interleaved(
        torch, [lambda i, d=d: B.spline_batch_launch(plans[d][i % nb], stream) for d in dts],
        4, reps=15))))
    for dt in dts:
        alg = sum(A.batch_bytes("vgh", dt, m, n) for (_, n, m) in CFG4)
        res[dt] = {"evals_per_s": evals / (ms[dt] * 1e-3), "us_per_replay": ms[dt] * 1e3,
                   "hbm_gbs": alg / (ms[dt] * 1e-3) / 1e9,
                   "direct_launch_evals_per_s": evals / (ms_d[dt] * 1e-3),
                   "us_per_direct_launch": ms_d[dt] * 1e3,
                   "tile": list(B.spline_batch_plan_tile(plans[dt][0]).as_tuple())}
        for pl in plans[dt]:
            B.spline_batch_plan_destroy(pl)
        for t in tabs[dt]:
            B.spline_table_destroy(t)
    res["f16_speedup_vs_f32"] = res["f16"]["evals_per_s"] / res["f32"]["evals_per_s"]
    res["f16_speedup_vs_f32_direct_launch"] = (res["f16"]["direct_launch_evals_per_s"] /
                                               res["f32"]["direct_launch_evals_per_s"])
    return res


def gpu_clocks():
    """Current and available shader/memory clocks from rocm-smi (a child
    process), or None where it cannot report them."""
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True,
                           text=True, timeout=30)
        data = json.loads(r.stdout)
    except (OSError, ValueError, subprocess.SubprocessError):
        return None
    card = data.get("card0") if isinstance(data, dict) else None
    if not isinstance(card, dict):
        return None
    return {k: v for k, v in card.items() if "clock" in k.lower() or "clk" in k.lower()}


def interleaved(torch, fns, k, reps=25):
    """Per-launch ms of each of the callables fns[l](i), timed back to back:
    rep r runs k launches of every layout in turn, rotating which goes first.
    Returns the per-rep times, one list per callable."""
    n = len(fns)
    for f in fns:
        for i in range(3):
            f(i)
    torch.cuda.synchronize()
    times = [[] for _ in range(n)]
    for r in range(reps):
        order = [(r + j) % n for j in range(n)]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        ev[0].record()
        for j, l in enumerate(order):
            for i in range(k):
                fns[l](r * k + i)
            ev[j + 1].record()
        torch.cuda.synchronize()
        for j, l in enumerate(order):
            times[l].append(ev[j].elapsed_time(ev[j + 1]) / k)
    return times


def median(xs):
    xs = sorted(xs)
    m = len(xs) // 2
    return xs[m] if len(xs) % 2 else 0.5 * (xs[m - 1] + xs[m])


def layout_extra(torch, B, synth, coef, t32, steps, warmup):
    """Plain against spline-blocked tables (the paper's AoSoA sub-tables), each
    at its own autotuned tile, timed back to back on the same batches (25
    reps, alternating which layout goes first): FP32 VGH on the headline's
    512-position batches and FP16 VGH on 4096 positions, with the layout that
    spline_layout_select picks."""
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    res = {"workload": "eval_vgh on the 48^3 x N=2048 coefficients; blocks of 256 (FP32) or "
                       "512 (FP16) splines, [N/B][51][51][51][B]; uniform positions, "
                       "batches cycled; 25 interleaved reps, medians",
           "rule": "the selector keeps plain unless blocked is faster by more than "
                   "max(3 %, 2 x 1.4826 x MAD of the per-rep time ratio)"}
    for dt, npos, nb in (("f32", NPOS, NBATCH), ("f16", 4096, 4)):
        batches = [torch.from_numpy(synth.positions(npos, stream=synth.position_stream(0),
                                                    batch=b)).to(dev) for b in range(nb)]
        v = torch.empty(npos, NSPL, device=dev)
        g = torch.empty(npos, 3, NSPL, device=dev)
        h = torch.empty(npos, 6, NSPL, device=dev)
        row = {}
        tabs, fns = [], []
        for name, flags in (("plain", 0), ("blocked", B.BSPL_LAYOUT_BLOCKED)):
            t = t32 if (dt == "f32" and flags == 0) else B.spline_table_create(
                *GRID, NSPL, coef, dt, flags=flags)
            tile = B.spline_autotune(t, "vgh", npos)
            row[f"{name}_tile"] = list(tile.as_tuple())
            tabs.append(t)
            fns.append(lambda i, t=t, tile=tile: B.spline_eval(
                t, "vgh", npos, batches[i % nb], v, g, h, NSPL, tile=tile, stream=stream))
        k = 16 if npos <= NPOS else 4
        times = interleaved(torch, fns, k)
        ratios = [b / p for p, b in zip(times[0], times[1])]
        r_med = median(ratios)
        noise = 1.4826 * median([abs(x - r_med) for x in ratios])
        for l, name in enumerate(("plain", "blocked")):
            ms = median(times[l])
            row[f"{name}_us_per_launch"] = ms * 1e3
            row[f"{name}_evals_per_s"] = npos * NSPL / (ms * 1e-3)
        for t in tabs:
            if t != t32:
                B.spline_table_destroy(t)
        row["blocked_over_plain_time"] = r_med
        row["ratio_noise"] = noise
        row["faster"] = "blocked" if r_med < 1.0 else "plain"
        row["difference_within_margin"] = abs(1.0 - r_med) <= max(0.03, 2.0 * noise)
        sel = B.spline_layout_select(*GRID, NSPL, dt, "vgh", npos)
        row["selected"] = "blocked" if sel == B.BSPL_LAYOUT_BLOCKED else "plain"
        res[f"{dt}_vgh_{npos}pos"] = row
        del v, g, h, batches
    return res


def latency_extra(torch, B, synth, t32, k=64, reps=20):
    """Latency mode: one eval_vgh of a few positions per launch, k launches
    on distinct position sets captured in a HIP graph and replayed; time per
    evaluation with unsplit units and with 4 wavefronts per unit."""
    dev = torch.device("cuda")
    out = {}
    for npos in (1, 4, 16):
        pos = [torch.from_numpy(synth.positions(npos, stream=synth.position_stream(0),
                                                batch=500 + b)).to(dev) for b in range(k)]
        v = torch.empty(npos, NSPL, device=dev)
        g = torch.empty(npos, 3, NSPL, device=dev)
        h = torch.empty(npos, 6, NSPL, device=dev)
        row = {}
        for name, tile in (("unsplit", (1, 1, 1, 0, 0, 1)), ("split4", (1, 1, 1, 0, 0, 4))):
            gs = torch.cuda.Stream()
            gs.wait_stream(torch.cuda.current_stream())
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.stream(gs):
                B.spline_eval(t32, "vgh", npos, pos[0], v, g, h, NSPL, tile=tile,
                              stream=gs.cuda_stream)
                torch.cuda.synchronize()
                with torch.cuda.graph(graph, stream=gs):
                    for i in range(k):
                        B.spline_eval(t32, "vgh", npos, pos[i], v, g, h, NSPL, tile=tile,
                                      stream=gs.cuda_stream)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                graph.replay()
            b.record()
            torch.cuda.synchronize()
            row[f"{name}_us_per_eval"] = a.elapsed_time(b) / (reps * k) * 1e3
            del graph
        out[f"npos{npos}"] = row
    return out


def large_extra(torch, B, A, synth, warmup):
    """96^3 (99^3 padded) x N=4096 tables beyond the Infinity Cache: FP32
    (15.9 GB) and FP16 (7.9 GB), 8192 positions per batch, VGH and VGL."""
    grid, n, npos = (96, 96, 96), 4096, 8192
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    src = synth.coef_table_torch(torch, *grid, n, device=dev, stream=synth.table_stream(0))
    tabs = {dt: B.spline_table_create(*grid, n, src, dt, flags=B.BSPL_COEFS_DEVICE)
            for dt in ("f32", "f16")}
    # the interpolating fit at this size, in place on the coefficient array
    # (three axis passes, 24 bytes per element: one read and one write each)
    ms_fit = timed(torch, lambda i: B.spline_fit_interpolating(*grid, n, src, src, stream=stream),
                   3, 1)
    fit_bytes = 3 * 8 * src.numel()
    del src
    torch.cuda.empty_cache()
    nb = 2
    pos = [torch.from_numpy(synth.positions(npos, stream=synth.position_stream(0), batch=b))
           .to(dev) for b in range(nb)]
    v = torch.empty(npos, n, device=dev)
    g = torch.empty(npos, 3, n, device=dev)
    lh = torch.empty(npos, 6, n, device=dev)
    res = {"workload": "96^3 (99^3 padded) x N=4096 table, FP32 15.9 GB / FP16 7.9 GB, "
                       "8192 uniform positions per batch, 2 batches alternated; FP32 and "
                       "FP16 of one kind timed interleaved (10 reps of 6 launches, medians)",
           "fit_interpolating": {"ms": ms_fit, "alg_bytes": fit_bytes,
                                 "hbm_gbs": fit_bytes / (ms_fit * 1e-3) / 1e9,
                                 "frac_of_peak": fit_bytes / (ms_fit * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    for kind in ("vgh", "vgl"):
        tiles = {dt: B.spline_autotune(t, kind, npos) for dt, t in tabs.items()}
        dts = list(tabs)
        times = interleaved(torch, [lambda i, d=d: B.spline_eval(
            tabs[d], kind, npos, pos[i % nb], v, g, lh, n, tile=tiles[d], stream=stream)
            for d in dts], 6, reps=10)
        for dt, ts in zip(dts, times):
            ms = median(ts)
            res[f"{dt}_{kind}"] = {
                "evals_per_s": npos * n / (ms * 1e-3), "ms_per_launch": ms,
                "hbm_gbs": A.batch_bytes(kind, dt, npos, n) / (ms * 1e-3) / 1e9,
                "tile": list(tiles[dt].as_tuple())}
    for kind in ("vgh", "vgl"):
        res[f"f16_speedup_{kind}"] = (res[f"f16_{kind}"]["evals_per_s"]
                                      / res[f"f32_{kind}"]["evals_per_s"])
    for t in tabs.values():
        B.spline_table_destroy(t)
    return res


def sweep_mode(torch, B, A, synth):
    """The paper's throughput-vs-N and tile-size studies on this GPU:
    T = npos * N / t for N = 128 ... 4096 at 48^3 (512 positions), each with
    its autotuned tile, then T against the spline tile width at N = 2048."""
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    npos = NPOS
    batches = [torch.from_numpy(synth.positions(npos, stream=synth.position_stream(0), batch=b))
               .to(dev) for b in range(NBATCH)]
    for n in (128, 256, 512, 1024, 2048, 4096):
        coef = synth.coef_table(*GRID, n, stream=synth.table_stream(0))
        t = B.spline_table_create(*GRID, n, coef, "f32")
        del coef
        v = torch.empty(npos, n, device=dev)
        g = torch.empty(npos, 3, n, device=dev)
        h = torch.empty(npos, 6, n, device=dev)
        for kind in ("vgh", "vgl", "v"):
            tile = B.spline_autotune(t, kind, npos)
            ms = timed(torch, lambda i: B.spline_eval(t, kind, npos, batches[i % NBATCH], v, g, h,
                                                      n, stream=stream), 200, 20)
            print(json.dumps({"sweep": "n_splines", "grid": list(GRID), "n_splines": n,
                              "npos": npos, "kernel": "eval_" + kind, "us_per_launch": ms * 1e3,
                              "evals_per_s": npos * n / (ms * 1e-3),
                              "hbm_gbs": A.batch_bytes(kind, "f32", npos, n) / (ms * 1e-3) / 1e9,
                              "frac_of_peak": A.batch_bytes(kind, "f32", npos, n)
                              / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "tile": list(tile.as_tuple())}), flush=True)
            if n == 2048 and kind == "vgh":
                # tile-width study: splines per workgroup 64*vw*wx, one position row
                for vw in (1, 2, 4):
                    for wx in (1, 2, 4, 8):
                        tl = (vw, wx, 1, 0, 0)
                        ms = timed(torch, lambda i: B.spline_eval(t, kind, npos,
                                                                  batches[i % NBATCH], v, g, h,
                                                                  n, tile=tl, stream=stream),
                                   200, 20)
                        print(json.dumps({"sweep": "tile", "n_splines": n, "npos": npos,
                                          "kernel": "eval_vgh", "tile": list(tl),
                                          "splines_per_wavefront": 64 * vw,
                                          "splines_per_workgroup": 64 * vw * wx,
                                          "us_per_launch": ms * 1e3,
                                          "evals_per_s": npos * n / (ms * 1e-3)}), flush=True)
        # many walker batches per launch: the 16 batches of 512 positions
        # as one batch plan (16 entries of the same table), issued as
        # direct launches and as a graph replay
        outs = [(torch.empty(npos, n, device=dev), torch.empty(npos, 3, n, device=dev),
                 torch.empty(npos, 6, n, device=dev)) for _ in range(NBATCH)]
        plan = B.spline_batch_plan_create([t] * NBATCH, [npos] * NBATCH, "vgh", batches,
                                          [o[0] for o in outs], [o[1] for o in outs],
                                          [o[2] for o in outs], [n] * NBATCH,
                                          stream=stream)
        ms_d = timed(torch, lambda i: B.spline_batch_launch(plan, stream), 100, 10)
        ms_g = timed(torch, lambda i: B.spline_batch_execute(plan, stream), 100, 10)
        alg = NBATCH * A.batch_bytes("vgh", "f32", npos, n)
        print(json.dumps({"sweep": "n_splines_batched", "grid": list(GRID), "n_splines": n,
                          "npos": npos, "walker_batches_per_launch": NBATCH,
                          "kernel": "eval_vgh", "us_per_launch": ms_d * 1e3,
                          "evals_per_s": NBATCH * npos * n / (ms_d * 1e-3),
                          "hbm_gbs": alg / (ms_d * 1e-3) / 1e9,
                          "frac_of_peak": alg / (ms_d * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "us_per_graph_replay": ms_g * 1e3,
                          "graph_evals_per_s": NBATCH * npos * n / (ms_g * 1e-3),
                          "tile": list(B.spline_batch_plan_tile(plan).as_tuple())}),
              flush=True)
        B.spline_batch_plan_destroy(plan)
        del outs
        B.spline_table_destroy(t)
        # the same table stored as FP16 (per-spline scales), VGH
        coef = synth.coef_table(*GRID, n, stream=synth.table_stream(0))
        t16 = B.spline_table_create(*GRID, n, coef, "f16")
        del coef
        tile = B.spline_autotune(t16, "vgh", npos)
        ms = timed(torch, lambda i: B.spline_eval(t16, "vgh", npos, batches[i % NBATCH], v, g, h,
                                                  n, stream=stream), 200, 20)
        print(json.dumps({"sweep": "n_splines", "grid": list(GRID), "n_splines": n,
                          "npos": npos, "kernel": "eval_vgh", "table_dtype": "f16",
                          "us_per_launch": ms * 1e3, "evals_per_s": npos * n / (ms * 1e-3),
                          "hbm_gbs": A.batch_bytes("vgh", "f16", npos, n) / (ms * 1e-3) / 1e9,
                          "frac_of_peak": A.batch_bytes("vgh", "f16", npos, n)
                          / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "tile": list(tile.as_tuple())}), flush=True)
        B.spline_table_destroy(t16)
        del v, g, h
        torch.cuda.empty_cache()
    return 0


def cpu_baseline(np, synth, coef, budget_cpu_s=12.0, max_batches=64):
    """The FP64 oracle on the host cores, on 512-position batches of the same
    workload until about budget_cpu_s CPU-seconds have been spent."""
    import oracle
    nth = oracle.num_threads()
    done, wall = 0, 0.0
    b = 0
    while b < max_batches and wall * nth < budget_cpu_s:
        pos = synth.positions(NPOS, stream=synth.position_stream(0), batch=b)
        t = time.perf_counter()
        oracle.evaluate("vgh", coef, pos)
        wall += time.perf_counter() - t
        done += NPOS
        b += 1
    # one core on one batch, for scale
    oracle.set_num_threads(1)
    pos = synth.positions(NPOS, stream=synth.position_stream(0), batch=0)
    t = time.perf_counter()
    oracle.evaluate("vgh", coef, pos)
    one = NPOS * NSPL / (time.perf_counter() - t)
    oracle.set_num_threads(nth)
    cpu = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": done * NSPL / wall, "unit": "orbital-evals/s", "cores": nth,
            "kind": "oracle",
            "sample": f"eval_vgh FP64 oracle (C, OpenMP over positions), {b} batches x "
                      f"{NPOS} positions x N={NSPL} of the same 48^3 table, {wall:.2f} s wall",
            "cpu_model": cpu, "nproc": os.cpu_count(), "single_core_value": one}


ACC_PER_BATCH = 16  # positions sampled from each timed batch for the error report
ERR_BOUND = {"f32": 1e-5, "f16": 2e-3, "bf16": 5e-3}
COMP_NAMES = {"vgh": ["v", "gx", "gy", "gz", "hxx", "hxy", "hxz", "hyy", "hyz", "hzz"],
              "vgl": ["v", "gx", "gy", "gz", "l"]}


def sample_positions(np, synth):
    """The first ACC_PER_BATCH positions of each of the 16 timed batches."""
    return np.ascontiguousarray(np.concatenate(
        [synth.positions(NPOS, stream=synth.position_stream(0), batch=b)[:, :ACC_PER_BATCH]
         for b in range(NBATCH)], axis=1))


def gpu_samples(torch, np, B, synth, coef, t32):
    """GPU outputs of VGH and VGL at the sampled positions for the FP32, FP16
    and BF16 tables (each with its tuned or default tile), as host arrays."""
    dev = torch.device("cuda")
    pos = sample_positions(np, synth)
    m = pos.shape[1]
    p = torch.from_numpy(pos).to(dev)
    v = torch.empty(m, NSPL, device=dev)
    g = torch.empty(m, 3, NSPL, device=dev)
    lh = torch.empty(m, 6, NSPL, device=dev)
    out = {}
    for dt in ("f32", "f16", "bf16"):
        t = t32 if dt == "f32" else B.spline_table_create(*GRID, NSPL, coef, dt)
        for kind in ("vgh", "vgl"):
            B.spline_eval(t, kind, m, p, v, g, lh, NSPL)
            torch.cuda.synchronize()
            comps = [v.cpu().numpy()] + [g[:, c].cpu().numpy() for c in range(3)]
            if kind == "vgh":
                comps += [lh[:, c].cpu().numpy() for c in range(6)]
            else:
                comps.append(lh.view(-1)[:m * NSPL].cpu().numpy().reshape(m, NSPL))
            out[(dt, kind)] = [c.astype(np.float64) for c in comps]
        if dt != "f32":
            B.spline_table_destroy(t)
    return out


def dequantized(np, coef, dt):
    """The values an FP16/BF16 table stores, restated on the host from the
    storage rule: per-spline scale s_n = 2^ceil(log2 max|c_n|) (1 for an
    all-zero spline) and the code c/s_n rounded to nearest-even."""
    m = np.abs(coef.reshape(-1, coef.shape[-1])).max(axis=0).astype(np.float64)
    sc = np.ones_like(m)
    sc[m > 0] = 2.0 ** np.ceil(np.log2(m[m > 0]))
    x = (coef / sc.astype(np.float32)).astype(np.float32)
    if dt == "f16":
        q = x.astype(np.float16).astype(np.float32)
    else:
        b = x.view(np.uint32).astype(np.uint64)
        q = (((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32)
    return q * sc.astype(np.float32)


def oracle_errors(np, coef, samples, pos):
    """Error of every output component of the GPU samples against the FP64
    oracle: max |gpu - oracle| / max |oracle| per component, with the oracle
    on the original coefficients and, for FP16/BF16, also on the values the
    table stores (which isolates the kernel from the storage rounding)."""
    import oracle

    def errs(kind, got, ref):
        keys = ["v", ("g", 0), ("g", 1), ("g", 2)]
        keys += [("h", c) for c in range(6)] if kind == "vgh" else ["l"]
        out = {}
        for name, k, a in zip(COMP_NAMES[kind], keys, got):
            r = ref[k] if isinstance(k, str) else ref[k[0]][:, k[1]]
            out[name] = float(np.abs(a - r).max() / np.abs(r).max())
        return out

    res = {"reference": "FP64 oracle (C)", "positions": int(pos.shape[1]),
           "sample": f"the first {ACC_PER_BATCH} positions of each of the {NBATCH} timed "
                     f"512-position batches, all {NSPL} splines",
           "normalisation": "per component: max |gpu - oracle| / max |oracle|",
           "bound": dict(ERR_BOUND)}
    refs = {kind: oracle.evaluate(kind, coef, pos) for kind in ("vgh", "vgl")}
    for dt in ("f32", "f16", "bf16"):
        row = {}
        deq = dequantized(np, coef, dt) if dt != "f32" else None
        for kind in ("vgh", "vgl"):
            row[kind] = errs(kind, samples[(dt, kind)], refs[kind])
            if deq is not None:
                row[kind + "_vs_stored_values"] = errs(kind, samples[(dt, kind)],
                                                       oracle.evaluate(kind, deq, pos))
        row["max"] = max(max(row[k].values()) for k in ("vgh", "vgl"))
        row["within_bound"] = row["max"] <= ERR_BOUND[dt]
        res[dt] = row
        del deq
    return res


def cpu_oracle_configs(np, synth, coef48, cfg4_coefs):
    """The oracle's VGH rate on the other workloads, for scale: the 16^3 x 64
    parity table and the 4096-position batch in full, 256 positions of each
    four-table table (when the batched extra ran), and 256 positions of the
    96^3 x 4096 table on 64 of its splines (the whole table is 16 GB)."""
    import oracle

    def rate(tab, pos):
        t = time.perf_counter()
        oracle.evaluate("vgh", tab, pos)
        return pos.shape[1] * tab.shape[-1], time.perf_counter() - t

    out = {"unit": "orbital-evals/s", "cores": oracle.num_threads()}
    c1 = synth.coef_table(16, 16, 16, 64, stream=synth.table_stream(0))
    e, w = rate(c1, synth.positions(1024, stream=synth.position_stream(0)))
    out["16^3xN64, 1024 positions (full)"] = e / w
    e, w = rate(coef48, synth.positions(4096, stream=synth.position_stream(0), batch=100))
    out["48^3xN2048, 4096 positions (full; the FP16/BF16 batch, same oracle cost)"] = e / w
    if cfg4_coefs is not None:
        ev, wall = 0, 0.0
        for i, c in enumerate(cfg4_coefs):
            e, w = rate(c, synth.positions(256, stream=synth.position_stream(i)))
            ev, wall = ev + e, wall + w
        out["four tables, 256 positions each"] = ev / wall
    cols = np.arange(0, 4096, 64)
    c5 = synth.coef_table(96, 96, 96, 4096, stream=synth.table_stream(0), splines=cols)
    e, w = rate(c5, synth.positions(256, stream=synth.position_stream(0)))
    out["96^3xN4096, 256 positions on 64 of the splines"] = e / w
    return out


if __name__ == "__main__":
    sys.exit(main())
