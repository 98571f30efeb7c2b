"""Benchmark of the guiding hot path on one MI355X.

Workload (frame scale): a closed room with 64 random boxes and three area
lights voxelized to an SVO of depth 10 (~7.9M leaves); one step =
svo_accumulate of 2,000,000 FP32 RGB exitance splats (splat + bottom-up
average) followed by guide_sample over the 1920x1080 primary-hit queue
(2,073,600 vertices) with a 16 x 16 direction field. All inputs are seeded
synthetic stand-ins for the paper's scenes and are resident in device memory
before timing starts.

Prints one JSON line: guided samples per second of the whole step, the
roofline of the dominant kernel (the guide kernel) and the CPU oracle's rate
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
SIMDS = 256 * 4           # 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9          # peak engine clock (cancels in the VALU fraction)

# VALU issue ceiling of the guide kernel: its own mix of instruction forms,
# each at its issue cost per wave64 instruction per SIMD. The issue probe
# (libwfpg_probe.so, one CU, four waves per SIMD, run live and reported
# beside the ceiling) splits the forms into two rates whatever their
# encoding: 32-bit adds and subtracts, logic ops, right shifts, moves and
# v_bitop3_b32 issue every 2 cycles (32 lanes per clock, the rate behind the
# 157.3 TFLOP/s FP32 vector figure; the probe reads 2.5-3), and selects on
# lane masks, compares, left shifts, min/max, 24-bit products, bit-field ops
# and 64-bit forms every 4 cycles (the probe reads 4.5-5). The mix is counted
# in the compiler listing (hipcc -S of guide.hip) of the eight unrolled steps
# of the pool loop of k_guide<16, SAMPLE, no blur, 3-byte records> (1,305 VALU
# instructions) and describes the sources below only.
PROBE_FORMS = ["add_e32", "xor_e32", "cndmask_e64", "cmp_e64", "cmp64_e64", "mad_u64", "lshl_add_u64",
               "bitop3", "lshl_e64"]
GUIDE_STEP_MIX = {
    "sources_sha256": "c6379962211547571b1be6b9d62057aaa8ddce3e8209bdac25d3bb9e11a2c879",
    # class: (instructions in the listing, issue cycles, probe forms of the class)
    "classes": {
        "32-bit add / sub / logic / right shift / move / bitop3": (1049, 2, ["add_e32", "xor_e32", "bitop3"]),
        "other 32-bit (selects, compares, left shifts, min/max, 24-bit products)":
            (160, 4, ["cndmask_e64", "cmp_e64", "lshl_e64"]),
        "v_mad_u64_u32 / v_mad_i64_i32": (88, 4, ["mad_u64"]),
        "64-bit adds and compares": (8, 4, ["lshl_add_u64", "cmp64_e64"]),
    },
}

# HBM bytes per launch of k_guide<16, SAMPLE> on this workload, from two
# rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) each scaled by what the same
# counter reads for a 1 GiB streaming kernel; the record is
# profiles/k_guide_sample_room_d10_n16_counters.md. It describes the kernel
# sources it was taken on and the default tile, and is reported only for them.
MEASURED_TRAFFIC = {
    "sources_sha256": "c6379962211547571b1be6b9d62057aaa8ddce3e8209bdac25d3bb9e11a2c879",
    "N": 16,
    "tile": {"waves_per_block": 12, "blocks_per_cu": 2},
    "bytes_per_launch": 1570617035,
    "valu_wave_instrs_per_launch": 12664715492,
}
KERNEL_SOURCES = ["guide.hip", "march_core.h", "wfpg_internal.h", "product_core.h", "antialias_core.h"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_06997_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(N, tile):
    """The counter-derived figures (HBM bytes, VALU instructions per launch) if
    they still describe the kernel that runs, else None."""
    m = MEASURED_TRAFFIC
    if kernel_sources_sha256() != m["sources_sha256"] or N != m["N"] or tile != m["tile"]:
        return None
    return m


def valu_issue_cycles(waves_per_simd=4, iters=20000):
    """Cycles (at CLOCK_HZ) per wave64 instruction per SIMD of each probe form:
    one workgroup, waves_per_simd waves on each SIMD of one CU, twelve
    independent chains of that form per wave."""
    import ctypes
    path = os.path.join(ROOT, "paper_2405_06997_amd", "libwfpg_probe.so")
    if not os.path.exists(path):
        return None   # the probe is built with the library; its figures are context only
    lib = ctypes.CDLL(path)
    lib.wfpg_probe_valu_issue.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)]
    assert lib.wfpg_probe_valu_forms() == len(PROBE_FORMS)
    out = {}
    for op, name in enumerate(PROBE_FORMS):
        ms, n = ctypes.c_float(), ctypes.c_double()
        err = lib.wfpg_probe_valu_issue(op, waves_per_simd, iters, ctypes.byref(ms), ctypes.byref(n))
        if err != 0:
            raise RuntimeError("VALU issue probe failed (hipError %d)" % err)
        out[name] = ms.value * 1e-3 * CLOCK_HZ / n.value
    return out


def valu_roofline(instrs_per_launch, launch_ms):
    """The guide kernel's VALU issue rate against the ceiling of its own mix of
    instruction forms (None when the mix no longer describes the sources)."""
    if instrs_per_launch is None or kernel_sources_sha256() != GUIDE_STEP_MIX["sources_sha256"]:
        return None
    classes = list(GUIDE_STEP_MIX["classes"].values())
    total = sum(n for n, _, _ in classes)
    mix_cycles = sum(n * c for n, c, _ in classes) / total
    cyc = valu_issue_cycles()
    probe_mix = None if cyc is None else \
        sum(n * sum(cyc[f] for f in forms) / len(forms) for n, _, forms in classes) / total
    peak = SIMDS * CLOCK_HZ / mix_cycles
    achieved = instrs_per_launch / (launch_ms * 1e-3)
    return {"bound": "valu issue", "achieved": achieved, "peak": peak, "unit": "wave64 VALU instructions/s",
            "frac": achieved / peak, "mix_cycles_per_instr": mix_cycles,
            "kernel_cycles_per_instr": SIMDS * CLOCK_HZ / achieved,
            "probe_cycles_per_instr": cyc, "probe_mix_cycles_per_instr": probe_mix}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--autotune", action="store_true",
                    help="sweep the guide kernel's launch shape first (its launches then show up in a "
                         "kernel trace of this command); default: the library's default tile")
    ap.add_argument("--no-autotune", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device copy of this size before timing (counter calibration)")
    ap.add_argument("--sections", default="tiny,stress,binned,product,extract,learned,batching,precision",
                    help="comma-separated extra sections after the headline march step "
                         "(binned, product, extract, learned, batching, precision; empty for none)")
    ap.add_argument("--only-march", action="store_true", help="same as --sections ''")
    ap.add_argument("--train-pairs", type=int, default=50_000_000,
                    help="(vertex, march pdf) pairs the learned model is trained on")
    ap.add_argument("--budget-ns", type=float, default=30.0,
                    help="guiding time budget per vertex for the autotuner's choice of N")
    ap.add_argument("--train-frames", type=int, default=4,
                    help="jittered camera frames that supply the training vertices")
    return ap.parse_args()


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; the path would shard by queue "
                                   "ranges over replicated SVOs, with one all-reduce of the splat "
                                   "accumulators per frame, but runs on several GPUs are not "
                                   "supported", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2405_06997_amd as w
    import synth

    dev = torch.device("cuda:0")
    log("building the frame-scale room SVO and inputs")
    room = synth.room()
    svo = w.svo_build(room, 10)
    splats = synth.room_splats(room, 2_000_000, 13)
    sp = [torch.from_numpy(a).to(dev) for a in splats]
    cam, cnrm, _ = synth.camera_queue(room)
    pos = torch.from_numpy(cam).to(dev)
    n = pos.shape[1]
    opts = w.make_opts(N=args.N)
    NN = args.N * args.N
    d_out = torch.empty((3, n), device=dev)
    p_out = torch.empty((n,), device=dev)

    # launch shape: autotuned on an evenly strided quarter-million-vertex subset
    if args.autotune and not args.no_autotune:
        sub = pos[:, :: max(1, n // 262144)].contiguous()
        w.autotune(svo, sub, args.N, reps=3)
    tile = w.get_tile(svo, args.N)

    # algorithmic work of the march (untimed): node tests at levels >= 5 and hits
    cnt = w.march_counts(svo, pos, opts).to(torch.int64).sum(0).cpu().numpy()
    visits, hits = int(cnt[0]), int(cnt[1])
    e_bytes = 8  # FP32 exitance pair
    alg_bytes = n * (12 + 16) + 8 * visits + hits * (e_bytes + 12)

    if args.copy_calib_mib > 0:   # plain streaming kernel of known traffic, for HBM counter scaling
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)   # reads and writes copy_calib_mib MiB each
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream()
    log(f"timing {args.steps} steps of accumulate + guide_sample")
    for _ in range(args.warmup):
        w.svo_accumulate(svo, *sp)
        w.guide_sample(svo, pos, opts, seed=1, bounce=0, dir_out=d_out, pdf_out=p_out)
    torch.cuda.synchronize()
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    t0 = time.perf_counter()
    for s in range(K):
        ev[s][0].record(stream)
        w.svo_accumulate(svo, *sp)
        ev[s][1].record(stream)
        w.guide_sample(svo, pos, opts, seed=1 + s, bounce=0, dir_out=d_out, pdf_out=p_out)
        ev[s][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    acc_ms = [ev[s][0].elapsed_time(ev[s][1]) for s in range(K)]
    gs_ms = [ev[s][1].elapsed_time(ev[s][2]) for s in range(K)]
    step_ms = ev[0][0].elapsed_time(ev[K - 1][2]) / K
    st = svo.stats()
    assert st["errors"] == 0
    assert torch.isfinite(p_out).all() and (p_out > 0).all()

    gs_avg = float(np.mean(gs_ms))
    achieved = alg_bytes / (gs_avg * 1e-3) / 1e9
    copy_gbs = copy_bandwidth(dev)
    acc_avg = float(np.mean(acc_ms))
    # svo_accumulate: per splat 36 B in + 8 (D - 4) B of occupancy lookups + 12 B
    # normal + 16 B of atomics (112 B at depth 10); the bottom-up average reads
    # the leaf accumulators and writes every node's exitance (~214 MB here)
    acc_alg = 2_000_000 * (36 + 8 * (10 - 4) + 12 + 16) + acc_prop_bytes(st_levels(svo))
    counters = measured_counters(args.N, tile)
    traffic = None if counters is None else counters["bytes_per_launch"]
    out = {
        "metric": "guided samples/sec (PDF build+sample) on 1 MI355X; MLP vs SVO march at KL<=0.05",
        "value": n / (step_ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded procedural room; stands in for the paper's scenes)",
        "config": {
            "workload": "room D=10 (%d leaves), 1920x1080 camera queue (%d vertices), N=%d, "
                        "svo_accumulate of 2M splats then guide_sample" % (st["leaves"], n, args.N),
            "svo_depth": 10, "bins": NN, "queue": n, "splats": 2_000_000, "exitance": "fp32",
            "tile": tile,
        },
        "breakdown_ms": {"svo_accumulate": float(np.mean(acc_ms)), "guide_sample": gs_avg,
                         "guide_sample_median": float(np.median(gs_ms)), "wall_per_step": wall / K * 1e3},
        "guide_samples_per_s": n / (gs_avg * 1e-3),
        "accumulate_roofline": {"bound": "hbm", "kernels": "k_splat + k_prop_leaf + k_prop_inner",
                                "alg_bytes_per_call": acc_alg, "achieved": acc_alg / (acc_avg * 1e-3) / 1e9,
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": acc_alg / (acc_avg * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "roofline": {
            "bound": "hbm", "kernel": "k_guide<16, SAMPLE>",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes,
            "traffic_gbs": None if traffic is None else traffic / (gs_avg * 1e-3) / 1e9,
            "node_tests_per_bin": visits / (n * NN), "hit_fraction": hits / (n * NN),
            "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
            # the march is bound by VALU issue: its rate beside the logical HBM fraction
            "valu": valu_roofline(None if counters is None else counters["valu_wave_instrs_per_launch"], gs_avg),
        },
    }
    orc = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"], orc, ref = cpu_baseline(room, splats, cam, args.N, args.cpu_sample, n, seed=K)
        out["parity"] = parity(d_out, p_out, ref, args.N)
    sections = set() if args.only_march else {x for x in args.sections.split(",") if x}
    unknown = sections - {"tiny", "stress", "binned", "product", "extract", "learned", "batching", "precision"}
    if unknown:
        raise SystemExit(f"unknown sections: {sorted(unknown)}")
    if "tiny" in sections:
        log("tiny-box section")
        out["tiny"] = tiny_section(w, args)
    if "stress" in sections:
        log("stress-queue section")
        out["stress"] = stress_section(w, svo, room, args)
    if "binned" in sections:
        log("binned section")
        out["binned"] = binned_section(w, svo, pos, n, args, gs_avg)
    if "product" in sections:
        log("product section")
        out["product"] = product_section(w, svo, pos, cnrm, n, args, gs_avg)
    if "extract" in sections:
        log("extract section")
        out["extract"] = extract_section(w, room, args)
    if "learned" in sections:
        log("learned section")
        out["learned"] = learned_section(w, svo, room, pos, cnrm, n, args, gs_avg, acc_ms, sp)
    if "batching" in sections:
        log("batching section")
        out["batching"] = batching_section(w, svo, room, cam, cnrm, args)
    if "precision" in sections:
        log("precision section")
        out["precision"] = precision_section(w, room, sp, pos, cam, args, orc, tile)
    print(json.dumps(out))


def copy_bandwidth(dev):
    """HBM bandwidth of a plain streaming kernel measured in the same run:
    torch's copy of 1 GiB (1 GiB read and 1 GiB written), HIP events."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms = _timed(lambda: dst.copy_(src), 10, 3)
    del src, dst
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def st_levels(svo):
    return svo.level_sizes()


def acc_prop_bytes(level_sizes):
    """Bottom-up averaging: every leaf's two (sum, count) pairs read (16 B) and
    its FP32 exitance pair written (8 B); every inner node reads its children's
    pairs, its own normal and theirs (about 8 + 16 B per child) and writes its
    pair (8 B)."""
    leaves = level_sizes[-1]
    inner = sum(level_sizes[:-1])
    return leaves * (16 + 8) + sum(level_sizes[1:]) * (8 + 16) + inner * 8


def tiny_section(w, args):
    """The tiny Cornell box (depth 6, one exitance splat per leaf side, 4096
    area-uniform vertices, N = 8): one step (accumulate + guide_sample) timed
    on the GPU, and the oracle running the same step on all 4096 vertices on
    the host cores, with the GPU's samples checked against it."""
    import math

    import numpy as np
    import torch

    import oracle
    import synth
    dev = torch.device("cuda:0")
    box = synth.cornell_box()
    D, N = 6, 8
    o = oracle.SVO(box, D)
    xyz, em = o.leaf_info()
    sp = synth.leaf_splats(xyz, o.normals(D), em, D, seed=2)
    g = w.svo_build(box, D)
    dsp = [torch.from_numpy(a).to(dev) for a in sp]
    pos_h, _, _ = synth.area_points(box, 4096, 3)
    pos = torch.from_numpy(pos_h).to(dev)
    opts = w.make_opts(N=N)
    d = torch.empty((3, 4096), device=dev)
    p = torch.empty((4096,), device=dev)

    def step():
        w.svo_accumulate(g, *dsp)
        w.guide_sample(g, pos, opts, seed=9, bounce=0, dir_out=d, pdf_out=p)
    ms = _timed(step, args.steps, args.warmup)
    t = time.perf_counter()
    o.accumulate(*sp)
    o.propagate()
    ref = o.guide_sample(pos_h, N, seed=9, bounce=0)
    t_orc = time.perf_counter() - t
    dd = d.cpu().numpy().astype(np.float64)
    pp = p.cpu().numpy().astype(np.float64)
    uv = oracle.oct_encode_many(dd)
    gb = np.minimum((uv * N).astype(np.int64), N - 1)
    same = (gb[0] == ref["bin"][:, 0]) & (gb[1] == ref["bin"][:, 1])
    band = (ref["margin"] < (4 * math.log2(N) + 3) * 2.0 ** -24).any(1)
    rel = np.abs(pp[same] - ref["pdf"][same]) / ref["pdf"][same]
    return {"workload": "Cornell box D=6 (%d leaves), 4096 area-uniform vertices, N=8, one splat per leaf side"
                        % o.level_size(D),
            "ms_per_step": ms, "samples_per_s": 4096 / (ms * 1e-3),
            "oracle": {"seconds": t_orc, "samples_per_s": 4096 / t_orc, "cores": oracle.num_threads(),
                       "sample": "all 4096 vertices, accumulate + propagate + guide_sample"},
            "parity": {"same_bin": float(same.mean()), "differing_outside_scan_band": int((~same & ~band).sum()),
                       "pdf_max_rel_err": float(rel.max())}}


def stress_section(w, svo, room, args):
    """The frame-scale room with the stress queue: 2,073,600 area-uniform
    surface points in random order (no camera coherence), N = 16."""
    import numpy as np
    import torch

    import synth
    dev = torch.device("cuda:0")
    rnd, _, _ = synth.area_points(room, 2_073_600, 14)
    pos = torch.from_numpy(rnd).to(dev)
    n = pos.shape[1]
    opts = w.make_opts(N=16)
    cnt = w.march_counts(svo, pos, opts).to(torch.int64).sum(0).cpu().numpy()
    alg = n * (12 + 16) + 8 * int(cnt[0]) + int(cnt[1]) * (8 + 12)
    d = torch.empty((3, n), device=dev)
    p = torch.empty((n,), device=dev)
    ms = _timed(lambda: w.guide_sample(svo, pos, opts, seed=2, bounce=1, dir_out=d, pdf_out=p), args.steps,
                args.warmup)
    assert torch.isfinite(p).all() and (p > 0).all()
    return {"workload": "room D=10, 2073600 area-uniform vertices in random order, N=16",
            "guide_sample_ms": ms, "samples_per_s": n / (ms * 1e-3),
            "roofline": {"bound": "hbm", "alg_bytes_per_launch": alg, "achieved": alg / (ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "node_tests_per_bin": int(cnt[0]) / (n * 256), "hit_fraction": int(cnt[1]) / (n * 256)}}


def _timed(fn, K, warmup):
    """Mean milliseconds of fn() over K calls, HIP events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for k in range(K):
        ev[k][0].record(stream)
        fn()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / K


def binned_section(w, svo, pos, n, args, march_ms):
    """Positional binning (Alg. 2, c_ray = 512, l_min = 5 as in the paper's
    runs) and one field per bin at a random member (Alg. 3), every member
    sampling its bin's field: the paper's own amortization, on the headline
    queue."""
    import numpy as np
    import torch
    out = {}
    for N in (16, 32, 64, 128):
        log(f"binned N={N}")
        o = w.bin_opts(N=N, c_ray=512, l_min=5)
        d_out = torch.empty((3, n), device=pos.device)
        p_out = torch.empty((n,), device=pos.device)
        ms = _timed(lambda: w.guide_sample_binned(svo, pos, o, seed=5, bounce=0, dir_out=d_out, pdf_out=p_out),
                    args.steps, args.warmup)
        _, _, b = w.guide_sample_binned(svo, pos, o, seed=5, bounce=0, dir_out=d_out, pdf_out=p_out, bins=True)
        bins = b.cpu().numpy()
        nb = int(len(np.unique(bins[bins >= 0])))
        assert torch.isfinite(p_out).all() and (p_out > 0).all()
        out[str(N)] = {"guide_sample_binned_ms": ms, "samples_per_s": n / (ms * 1e-3), "bins": nb,
                       "rays_per_bin": n / max(nb, 1), "field_cone_traces": nb * N * N}
    out["c_ray"], out["l_min"] = 512, 5
    out["speedup_vs_per_vertex_march_N16"] = march_ms / out["16"]["guide_sample_binned_ms"]
    return out


def product_section(w, svo, pos, cnrm, n, args, march_ms):
    """Product path guiding (Sec. 3.6) with the Lambertian table of each
    vertex's camera-facing normal: per vertex (own field, N = 16) and over
    the positional bins (c_ray = 512, l_min = 5), one wave per member."""
    import torch
    nrm = torch.from_numpy(cnrm).to(pos.device)
    d_out = torch.empty((3, n), device=pos.device)
    p_out = torch.empty((n,), device=pos.device)
    out = {}
    log("product per vertex N=16")
    opts = w.make_opts(N=16)
    ms = _timed(lambda: w.guide_sample_product(svo, pos, opts, 5, 0, nrm=nrm, dir_out=d_out, pdf_out=p_out),
                args.steps, args.warmup)
    assert torch.isfinite(p_out).all() and (p_out > 0).all()
    out["per_vertex_16"] = {"guide_sample_product_ms": ms, "samples_per_s": n / (ms * 1e-3),
                            "cost_vs_plain": ms / march_ms}
    for N in (16, 32, 64, 128):
        log(f"product binned N={N}")
        o = w.bin_opts(N=N, c_ray=512, l_min=5)
        ms = _timed(lambda: w.guide_sample_binned_product(svo, pos, o, 5, 0, nrm=nrm, dir_out=d_out,
                                                          pdf_out=p_out), args.steps, args.warmup)
        assert torch.isfinite(p_out).all() and (p_out > 0).all()
        out[f"binned_{N}"] = {"guide_sample_binned_product_ms": ms, "samples_per_s": n / (ms * 1e-3)}
    return out


def extract_section(w, room, args):
    """Exitance extraction (Eq. 5) from the path memory of a frame-sized
    wavefront: 2,073,600 paths of up to 8 vertices, 70 % reaching an emitter,
    splatted and propagated into a fresh room SVO (depth 10)."""
    import numpy as np
    import torch

    import synth
    dev = torch.device("cuda:0")
    P, d = 2073600, 8
    log("extract: generating path memory")
    pos, T, eye, hit, Le = synth.path_wavefront(room, P, d, seed=31)
    splats = int(hit[hit >= 1].sum())
    args_d = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (pos, T, eye, hit, Le)]
    del pos, T
    g = w.svo_build(room, 10)
    ms = _timed(lambda: w.svo_accumulate_paths(g, *args_d), args.steps, args.warmup)
    # algorithmic bytes: per path-depth thread, hit (4 B); per splat, p_k, T_k,
    # T_n, p_{k-1}, Le (5 x 12 B) plus the leaf word, rank and normal reads and
    # the 8 B of atomics, taken as 60 + 8 + 4 + 16 + 8 B
    alg = P * d * 4 + splats * (60 + 8 + 4 + 16 + 8)
    return {"paths": P, "depths": d, "splats": splats, "svo_accumulate_paths_ms": ms,
            "splats_per_s": splats / (ms * 1e-3), "paths_per_s": P / (ms * 1e-3),
            "alg_bytes": alg, "alg_gbs": alg / (ms * 1e-3) / 1e9, "includes": "splat + bottom-up propagation"}


def learned_section(w, svo, room, pos, cnrm, n, args, march_ms, acc_ms, svo_splats_for_learned):
    """Hash-grid MLP trained on march pdfs of jittered frames of the same
    camera (as a progressive renderer sees them), then guide_sample in mode 1
    (network sample + march probes every 256th vertex + KL judge with the
    march as fallback) on the headline queue."""
    import numpy as np
    import torch

    import synth
    dev = pos.device
    t0 = time.perf_counter()
    frames = [synth.camera_queue(room, jitter_seed=100 + f)[:2] for f in range(args.train_frames)]
    tp = np.concatenate([f[0] for f in frames], 1)
    tn = np.concatenate([f[1] for f in frames], 1)
    perm = np.random.default_rng(7).permutation(tp.shape[1])
    tp = torch.from_numpy(np.ascontiguousarray(tp[:, perm])).to(dev)
    tn = torch.from_numpy(np.ascontiguousarray(tn[:, perm])).to(dev)
    gen_s = time.perf_counter() - t0
    batch = 65536
    steps = max(1, args.train_pairs // batch)
    nrm = torch.from_numpy(cnrm).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    log(f"training {steps} steps of {batch}")
    loss = w.guide_train(svo, tp, tn, steps=steps, batch=batch)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    opts1 = w.make_opts(N=16, mode=1, kl_bound=0.05, probe_stride=256)
    d_out = torch.empty((3, n), device=dev)
    p_out = torch.empty((n,), device=dev)
    fb0 = w.learned_stats(svo)["fallbacks"]
    K = args.steps
    ms = _timed(lambda: w.guide_sample(svo, pos, opts1, seed=3, bounce=0, nrm=nrm, dir_out=d_out,
                                       pdf_out=p_out), K, args.warmup)
    st = w.learned_stats(svo)
    fallbacks = st["fallbacks"] - fb0
    assert torch.isfinite(p_out).all() and (p_out > 0).all()
    fwd_ms = _timed(lambda: w.nn_forward(svo, pos, nrm), 3, 1)
    # the learned path's own cost: network samples + probe march + judge, no fallback
    opts_nf = w.make_opts(N=16, mode=1, kl_bound=3.0e38, probe_stride=256)
    nf_ms = _timed(lambda: w.guide_sample(svo, pos, opts_nf, seed=3, bounce=0, nrm=nrm, dir_out=d_out,
                                          pdf_out=p_out), K, args.warmup)
    # per-vertex KL(march || network) on an evenly strided sample
    sub = slice(0, n, max(1, n // 65536))
    sp_, sn_ = pos[:, sub].contiguous(), nrm[:, sub].contiguous()
    t = w.guide_pdf(svo, sp_, w.make_opts(N=16)).double()
    t = t / t.sum(1, keepdim=True)
    q = w.nn_forward(svo, sp_, sn_).double()
    kl = torch.where(t > 0, t * (t.log() - q.log()), torch.zeros_like(t)).sum(1).cpu().numpy()
    # how much the march pdf itself moves within a pixel: centre vs the jittered
    # training point of the same pixel (every pixel hits, so indices correspond)
    jp = torch.from_numpy(np.ascontiguousarray(frames[0][0][:, sub])).to(dev)
    tj = w.guide_pdf(svo, jp, w.make_opts(N=16)).double()
    tj = tj / tj.sum(1, keepdim=True)
    klj = torch.where(t > 0, t * (t.log() - tj.log()), torch.zeros_like(t)).sum(1).cpu().numpy()
    flops = 2 * (35 * 64 + 3 * 64 * 64 + 64 * 256)   # algorithmic MACs x 2 per vertex
    # smoother target fields (Sec. 4): the blurred field with a larger initial
    # value eps; a fresh model per field, trained and judged on that field
    log("learned: blurred targets")
    smooth = []
    for eps in (0.01, 0.1, 0.3, 1.0):
        g2 = w.svo_build(room, 10)
        w.svo_accumulate(g2, *svo_splats_for_learned)
        w.guide_train(g2, tp, tn, steps=steps, batch=batch, target_eps=eps, target_blur=1)
        o0 = w.make_opts(N=16, eps=eps, blur=True)
        t2 = w.guide_pdf(g2, sp_, o0).double()
        t2 = t2 / t2.sum(1, keepdim=True)
        q2 = w.nn_forward(g2, sp_, sn_).double()
        k2 = torch.where(t2 > 0, t2 * (t2.log() - q2.log()), torch.zeros_like(t2)).sum(1).cpu().numpy()
        o1 = w.make_opts(N=16, eps=eps, blur=True, mode=1, kl_bound=0.05, probe_stride=256)
        fb = w.learned_stats(g2)["fallbacks"]
        m1 = _timed(lambda: w.guide_sample(g2, pos, o1, seed=3, bounce=0, nrm=nrm, dir_out=d_out, pdf_out=p_out),
                    K, args.warmup)
        fb = w.learned_stats(g2)["fallbacks"] - fb
        m0 = _timed(lambda: w.guide_sample(g2, pos, o0, seed=3, bounce=0, dir_out=d_out, pdf_out=p_out),
                    K, args.warmup)
        smooth.append({"eps": eps, "blur": True, "kl_mean": float(k2.mean()), "kl_median": float(np.median(k2)),
                       "frac_vertices_kl_le_0.05": float((k2 <= 0.05).mean()),
                       "judge_probe_kl": w.learned_stats(g2)["last_probe_kl"], "fallbacks": fb,
                       "calls": K + args.warmup, "mode1_ms": m1, "march_ms": m0, "speedup_vs_march": m0 / m1})
        del g2
    del tp, tn
    return {
        "what": "hash-grid (16 x 2^19 x 2) + MLP 35-64-64-64-64-256, BF16 MFMA, trained on the GPU "
                "on march pdfs; mode-1 guide_sample with KL judge (bound 0.05 nats, probe every "
                "256th vertex) and march fallback",
        "train": {"pairs": steps * batch, "steps": steps, "batch": batch, "frames": args.train_frames,
                  "seconds": train_s, "final_loss": loss, "data_gen_seconds": gen_s},
        "guide_sample_ms": ms,
        "samples_per_s": n / (ms * 1e-3),
        "step_samples_per_s": n / ((ms + float(np.mean(acc_ms))) * 1e-3),
        "speedup_vs_march": march_ms / ms,
        "fallbacks": fallbacks, "calls": K + args.warmup,
        "judge_probe_kl": st["last_probe_kl"],
        "kl_per_vertex": {"mean": float(kl.mean()), "median": float(np.median(kl)),
                          "p90": float(np.quantile(kl, 0.9)), "vertices": int(kl.size)},
        "march_kl_within_pixel": {"mean": float(klj.mean()), "median": float(np.median(klj)),
                                  "what": "KL(march pdf at the pixel centre || march pdf at a "
                                          "jittered point of the same pixel), same vertices"},
        "nn_forward_ms": fwd_ms,
        "blurred_targets": smooth,
        "no_fallback_guide_sample_ms": nf_ms,
        "no_fallback_speedup_vs_march": march_ms / nf_ms,
        "mfma_flops_per_vertex": flops,
        "inference_roofline": inference_roofline(n, flops, fwd_ms),
    }


def inference_roofline(n, flops, fwd_ms):
    """The network forward (nn_forward: the 256 probabilities of every vertex
    written out) against the dense BF16 matrix-core peak and against a
    library GEMM measured in the same run (8192^3 BF16 torch.matmul), and its
    bytes (24 in; 16 levels x 8 corners x 2 BF16 features gathered, 512; 1024
    out) against HBM."""
    import torch
    dev = torch.device("cuda:0")
    a = torch.randn(8192, 8192, device=dev).to(torch.bfloat16).contiguous()
    b = torch.randn(8192, 8192, device=dev).to(torch.bfloat16).contiguous()
    gms = _timed(lambda: torch.matmul(a, b), 5, 2)
    del a, b
    gemm = 2.0 * 8192 ** 3 / (gms * 1e-3) / 1e12
    achieved = flops * n / (fwd_ms * 1e-3) / 1e12
    nbytes = n * (24 + 512 + 1024)
    return {"bound": "mfma", "kernel": "k_nn_infer (nn_forward)", "achieved": achieved, "peak": 2500.0,
            "unit": "TFLOP/s", "frac": achieved / 2500.0, "gemm_tflops": gemm, "frac_of_gemm": achieved / gemm,
            "bytes": {"bound": "hbm", "per_vertex": 24 + 512 + 1024, "achieved_gbs": nbytes / (fwd_ms * 1e-3) / 1e9,
                      "peak": HBM_PEAK_GBS, "frac": nbytes / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def batching_section(w, svo, room, cam, cnrm, args):
    """Eight-bounce wavefront (queue sizes decaying by U[0.5, 0.8] per bounce)
    replayed as one captured graph of persistent guide kernels. The autotuner
    picks N in {8, 16, 32} and the tile: the finest N whose time per vertex
    on the whole queue fits the budget, for the camera bounce and for the
    first secondary bounce (later bounces share its vertex distribution)."""
    import torch

    import synth
    dev = torch.device("cuda:0")
    queues, sizes = synth.bounce_queues(room, cam, cnrm, 8, 15)
    qpos = [torch.from_numpy(q[0]).to(dev) for q in queues]
    picks = []
    for b in (0, 1):
        log(f"choosing N for bounce {b} ({sizes[b]} vertices)")
        picks.append(w.autotune_n(svo, qpos[b], args.budget_ns, reps=3))
    Ns = [picks[0]["N"]] + [picks[1]["N"]] * (len(sizes) - 1)
    n_dev = torch.tensor(sizes, dtype=torch.int64, device=dev)
    G = w.BounceGraph(svo, qpos, n_dev, Ns, seed=7)
    K = args.steps
    g_ms = _timed(G.launch, K, args.warmup)

    def eager():
        for b, q in enumerate(qpos):
            w.guide_sample(svo, q, w.make_opts(N=Ns[b]), seed=7, bounce=b,
                           dir_out=G.dirs[b], pdf_out=G.pdfs[b])
    e_ms = _timed(eager, K, args.warmup)
    fixed = {}
    for N in (8, 16, 32):
        Gn = w.BounceGraph(svo, qpos, n_dev, [N] * len(sizes), seed=7)
        ms = _timed(Gn.launch, max(3, K // 4), 1)
        fixed[str(N)] = {"graph_ms": ms, "samples_per_s": sum(sizes) / (ms * 1e-3)}
        del Gn
    # the paper's decaying resolution: N halved per bounce (down to 8)
    log("depth-halving N")
    halving = [max(8, 32 >> b) for b in range(len(sizes))]
    Gh = w.BounceGraph(svo, qpos, n_dev, halving, seed=7)
    h_ms = _timed(Gh.launch, max(3, K // 4), 1)
    del Gh
    bhalving = [max(8, 128 >> b) for b in range(len(sizes))]

    def binned_halving():
        for b, q in enumerate(qpos):
            w.guide_sample_binned(svo, q, w.bin_opts(N=bhalving[b], c_ray=512, l_min=5), 7, b,
                                  dir_out=G.dirs[b], pdf_out=G.pdfs[b])
    bh_ms = _timed(binned_halving, max(3, K // 4), 1)
    # the same binned frame captured once in a HIP graph (the binned calls never
    # wait for the device) and replayed
    log("binned depth-halving as a graph")
    binned_halving()   # scratch grown to these sizes before capture
    torch.cuda.synchronize()
    bg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(bg):
        binned_halving()
    bg_ms = _timed(bg.replay, max(3, K // 4), 1)
    del bg
    depth_halving = {"per_vertex": {"N_per_bounce": halving, "graph_ms": h_ms,
                                    "samples_per_s": sum(sizes) / (h_ms * 1e-3)},
                     "binned": {"N_per_bounce": bhalving, "c_ray": 512, "l_min": 5, "eager_ms": bh_ms,
                                "graph_ms": bg_ms, "samples_per_s": sum(sizes) / (bg_ms * 1e-3),
                                "graph_speedup_vs_eager": bh_ms / bg_ms}}
    return {"bounces": len(sizes), "queue_sizes": sizes, "vertices": sum(sizes),
            "depth_halving": depth_halving,
            "budget_ns_per_vertex": args.budget_ns, "N_per_bounce": Ns,
            "tuned": [{"bounce": b, "N": p["N"], "tile": p["tile"],
                       "queue_ms_per_N": {str(k): v for k, v in p["ms_per_N"].items()}}
                      for b, p in zip((0, 1), picks)],
            "graph_ms": g_ms, "samples_per_s": sum(sizes) / (g_ms * 1e-3),
            "eager_ms": e_ms, "graph_speedup_vs_eager": e_ms / g_ms,
            "fixed_N": fixed}


def precision_section(w, room, sp, pos, cam, args, orc, tile):
    """Exitance and field bins stored in FP16 / BF16 (CDF and pdf in FP32):
    guide_sample rate on the headline queue, per-bin pdf error against the
    FP64 oracle on a strided sample of vertices, and a chi-square test of
    2^20 samples drawn at 64 vertices against the FP64 oracle pdf."""
    import numpy as np
    import torch
    dev = pos.device
    n = pos.shape[1]
    out = {}
    opts = w.make_opts(N=args.N)
    NN = args.N * args.N
    for name, fmt in (("fp16", w.WFPG_FP16), ("bf16", w.WFPG_BF16), ("fp32", w.WFPG_FP32)):
        log(f"precision {name}")
        g = w.svo_build(room, 10, fmt)
        w.svo_accumulate(g, *sp)
        d_out = torch.empty((3, n), device=dev)
        p_out = torch.empty((n,), device=dev)
        w.set_tile(g, args.N, **tile)     # the launch shape tuned for the FP32 SVO
        ms = _timed(lambda: w.guide_sample(g, pos, opts, seed=1, bounce=0, dir_out=d_out, pdf_out=p_out),
                    args.steps, args.warmup)
        r = {"guide_sample_ms": ms, "samples_per_s": n / (ms * 1e-3)}
        if orc is not None:
            S = 2048
            sub = np.ascontiguousarray(cam[:, :: n // S][:, :S])
            _, truth = orc.guide_pdf(sub, args.N, truth=True)
            gp = w.guide_pdf(g, torch.from_numpy(sub).to(dev), opts).cpu().numpy().astype(np.float64)
            rel = np.abs(gp - truth) / truth
            tv = 0.5 * np.abs(gp - truth).sum(1) * (4 * np.pi / NN)
            r["pdf_rel_err_vs_fp64"] = {"max": float(rel.max()), "mean": float(rel.mean()),
                                        "p99": float(np.quantile(rel, 0.99)), "vertices": S}
            r["tv_distance_vs_fp64"] = {"max": float(tv.max()), "mean": float(tv.mean())}
            r["chi_square"] = chi_square(w, g, orc, cam, args.N, dev)
        out[name] = r
        del g
    return out


def chi_square(w, g, orc, cam, N, dev, V=64, per=16384):
    """Samples of guide_sample at V vertices (per each) binned against the
    FP64 oracle pdf of those vertices; bins with expected count < 5 pooled per
    vertex."""
    import numpy as np
    import torch
    from scipy.stats import chi2
    n = cam.shape[1]
    base = np.ascontiguousarray(cam[:, :: n // V][:, :V])
    _, truth = orc.guide_pdf(base, N, truth=True)
    prob = truth * (4 * np.pi / (N * N))
    prob /= prob.sum(1, keepdims=True)
    rep = torch.from_numpy(np.repeat(base, per, axis=1)).to(dev)
    d, _ = w.guide_sample(g, rep, w.make_opts(N=N), seed=77, bounce=1)
    import oracle
    uv = oracle.oct_encode_many(d.cpu().numpy().astype(np.float64))
    b = np.minimum((uv * N).astype(np.int64), N - 1)
    bins = (b[1] * N + b[0]).reshape(V, per)
    stat, dof = 0.0, 0
    for v in range(V):
        cnt = np.bincount(bins[v], minlength=N * N).astype(np.float64)
        e = prob[v] * per
        big = e >= 5
        stat += float((((cnt - e) ** 2) / e)[big].sum())
        k = int(big.sum())
        if (~big).any() and e[~big].sum() > 0:
            stat += float((cnt[~big].sum() - e[~big].sum()) ** 2 / e[~big].sum())
            k += 1
        dof += k - 1
    return {"samples": V * per, "vertices": V, "stat": stat, "dof": dof, "p_value": float(chi2.sf(stat, dof))}


def cpu_baseline(room, splats, cam, N, S, n, seed):
    """The oracle, as it stands, on the host cores: accumulate + propagate of
    all 2M splats timed in full, guide_sample on an evenly strided sample of S
    queue vertices (with their queue indices as RNG counters and the seed of
    the last timed step, so its samples are that step's), extrapolated to the
    whole queue; then the same on one thread for a smaller sample."""
    import numpy as np

    import oracle
    o = oracle.SVO(room, 10)
    t = time.perf_counter()
    o.accumulate(*splats)
    o.propagate()
    t_acc = time.perf_counter() - t
    stride = max(1, n // S)
    idx = np.arange(0, n, stride)[:S]
    sub = np.ascontiguousarray(cam[:, idx])
    S = sub.shape[1]
    t = time.perf_counter()
    ref = o.guide_sample(sub, N, seed=seed, bounce=0, counter=idx)
    t_gs = time.perf_counter() - t
    ref["index"] = idx
    ref["max_splats"] = int(max(1, o.leaf_accum()[2].max()))
    step = t_acc + t_gs / S * n
    cores = oracle.num_threads()
    S1 = max(1, S // 32)
    oracle.set_num_threads(1)
    t = time.perf_counter()
    o.guide_sample(np.ascontiguousarray(sub[:, :S1]), N, seed=seed, bounce=0, counter=idx[:S1])
    t1 = time.perf_counter() - t
    oracle.set_num_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    base = {"value": n / step, "unit": "samples/s", "cores": cores, "kind": "oracle", "cpu_model": model,
            "sample": f"accumulate+propagate of all 2M splats ({t_acc:.2f} s) + guide_sample on "
                      f"every {stride}th camera-queue vertex ({S} of {n}, {t_gs:.2f} s), extrapolated "
                      f"to one full step",
            "single_thread_guide_samples_per_s": S1 / t1}
    return base, o, ref


def parity(d_out, p_out, ref, N):
    """The last timed step's samples against the oracle's on the CPU-baseline
    sample: sampled bins equal outside the FP32 scan band, pdf and direction
    errors on the equal ones. Bars: pdf 1e-5 relative; direction chord 2e-6;
    the scan band (4 log2 N + 3 + 2 (C - 1)) 2^-24 of the total, C the most
    splats any leaf side received (the FP32 atomic order then moves a stored
    value by at most (C - 1) 2^-24; two Hillis-Steele scans of depth log2 N
    sit between the field and a CDF boundary)."""
    import math

    import numpy as np

    import oracle
    idx = ref["index"]
    d = d_out[:, idx].cpu().numpy().astype(np.float64)
    p = p_out[idx].cpu().numpy().astype(np.float64)
    uv = oracle.oct_encode_many(d)
    gb = np.minimum((uv * N).astype(np.int64), N - 1)
    same = (gb[0] == ref["bin"][:, 0]) & (gb[1] == ref["bin"][:, 1])
    C = ref["max_splats"]
    band_rel = (4 * math.log2(N) + 3 + 2 * (C - 1)) * 2.0 ** -24
    band = (ref["margin"] < band_rel).any(1)
    rel = np.abs(p[same] - ref["pdf"][same]) / ref["pdf"][same]
    chord = np.linalg.norm(d[:, same] - ref["dir"][:, same], axis=0)
    return {"vertices": int(len(idx)), "same_bin": float(same.mean()),
            "scan_band": band_rel, "differing_outside_scan_band": int((~same & ~band).sum()),
            "pdf_max_rel_err": float(rel.max()), "dir_max_chord": float(chord.max()),
            "ok": bool((~same & ~band).sum() == 0 and rel.max() <= 1e-5 and chord.max() < 2e-6)}


if __name__ == "__main__":
    main()
