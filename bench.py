#!/usr/bin/env python3
"""Benchmark of the BYSDF hot path on one MI355X.

One step = one pass of the path over the per-block workload: 2^24 queries in
65,536 parameter blocks of 256 (one 3-ply yarn geometry; beta and albedo
drawn per block), inputs resident in HBM:
    bysdf_eval_sample     per query: value, lobes and pdf at (wi, wo), and one
                          importance-sampled direction with its weight and pdf
                          (state at the hit and forward nodes shared)
    bysdf_furnace_blocks  per-block white-furnace mean/variance (256 draws)
value = queries per second (2^24 queries per step / step time).  The same
work through the separate entry points (bysdf_eval, bysdf_sample_pdf, and
bysdf_eval again at the sampled directions) is timed after the steps and
reported under "unfused".

Prints ONE JSON line.  `roofline` is for the kernel with the largest time
per step, priced with the algorithmic operation count of the kernels'
formulation (bysdf_count_ops) against the VALU issue peak; `cpu_baseline`
is the FP64 oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s; an FMA
# counts 2 flops.  FP64 FMA and unpacked FP32 FMA issue at this rate (packed
# FP32, which doubles FP32 to 157.3 TFLOP/s, is not used by these kernels).
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # 78.64
PEAK_HBM_GBS = 8000.0


# sources the BYSDF kernels are built from: counters taken on another
# version of these no longer describe the kernels
_KERNEL_SOURCES = ("bysdf_lib.hip", "bysdf_math.hpp", "bysdf_model.hpp", "bysdf_dual.hpp",
                   "bysdf_opcount.hpp")


def _src_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2401_12724_amd", "csrc")
    for f in _KERNEL_SOURCES:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


# bench stage -> kernel name prefix in rocprofv3 output
_STAGE_KERNEL = {"eval_sample": "k_eval_sample<", "furnace": "k_furnace_w<"}


def _kname(full):
    full = full.replace("(anonymous namespace)::", "")
    return full.split("(")[0].replace("void ", "").strip()


def _summarize(prof_dir, bench_json, workload_tag):
    """Turn the rocprofv3 CSV output of the profiling passes under prof_dir
    (stats/, inst/, flops/, fetch/, write/) into short text summaries under
    profiles/ and profiles/traffic.json (HBM bytes per launch of each stage's
    kernel, FETCH_SIZE and WRITE_SIZE scaled by what the same counters read
    for the 1 GiB device copy of --copy-calibration)."""
    import csv
    import collections

    def counters(pas):
        f = os.path.join(prof_dir, pas, "run_counter_collection.csv")
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        meta = {}
        for r in csv.DictReader(open(f)):
            k = _kname(r["Kernel_Name"])
            per[k][r["Counter_Name"]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"]),
                                              int(r["Grid_Size"])))
            meta[k] = {c: r[c] for c in ("VGPR_Count", "Accum_VGPR_Count", "SGPR_Count",
                                         "Scratch_Size", "LDS_Block_Size", "Workgroup_Size")}
        return per, meta

    stats = {}
    for r in csv.DictReader(open(os.path.join(prof_dir, "stats", "run_kernel_stats.csv"))):
        stats[_kname(r["Name"])] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                                    float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                                    float(r["Percentage"]))
    bj = json.loads(open(bench_json).read().strip().splitlines()[-1])
    cmd = open(os.path.join(prof_dir, "commands.txt")).read().strip()
    N = bj["config"]["queries"]
    lines = ["# rocprofv3 kernel trace: %s" % workload_tag, "",
             "Commands (repo root on the GPU host):", "", cmd, "",
             "Average kernel durations from the trace against the HIP-event times that "
             "bench.py measured in the same run (ms per launch):", "",
             "| kernel | calls | trace avg us | min us | max us | % of GPU time |",
             "|---|---|---|---|---|---|"]
    for k, (c, a, mn, mx, pc) in sorted(stats.items(), key=lambda kv: -kv[1][4]):
        lines.append("| `%s` | %d | %.1f | %.1f | %.1f | %.2f |" % (k, c, a, mn, mx, pc))
    # per-dispatch durations of the step's launches: in dispatch order the
    # bench issues eval_sample, furnace, step after step, before any other work
    trace = sorted(csv.DictReader(open(os.path.join(prof_dir, "stats", "run_kernel_trace.csv"))),
                   key=lambda r: int(r["Dispatch_Id"]))
    stages = list(bj["kernels_ms"])
    seq = [r for r in trace if _kname(r["Kernel_Name"]) != "k_fiber_table"]
    per_stage = collections.defaultdict(list)
    for i, r in enumerate(seq):
        st = stages[i % len(stages)]
        if not _kname(r["Kernel_Name"]).startswith(_STAGE_KERNEL[st]):
            break
        per_stage[st].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    lines += ["", "| bench stage | kernel | HIP events ms (timed steps) | trace avg ms "
              "(warm-up + timed launches) |", "|---|---|---|---|"]
    for st, ms in bj["kernels_ms"].items():
        d = per_stage.get(st, [])
        lines.append("| %s | `%s` | %.3f | %s (%d launches) |" % (
            st, _STAGE_KERNEL[st].rstrip("<"), ms, ("%.3f" % (sum(d) / len(d))) if d else "n/a",
            len(d)))
    lines += ["", "bench.py line of the traced run: value %.4g queries/s, %.3f ms/step"
              % (bj["value"], bj["ms_per_step"])]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    tag = workload_tag.replace(" ", "_")
    open(os.path.join(ROOT, "profiles", "bysdf_%s_kernel_trace.md" % tag), "w").write(
        "\n".join(lines) + "\n")

    inst, meta = counters("inst")
    flops, _ = counters("flops")
    fetch, _ = counters("fetch")
    write, _ = counters("write")
    copy = [k for k in fetch if "copyBuffer" in k or "copy" in k.lower()]
    fmax = max(v for k in copy for (_, v, _) in fetch[k]["FETCH_SIZE"])
    wmax = max(v for k in copy for (_, v, _) in write[k]["WRITE_SIZE"])
    gib_kib = 1 << 20
    f_scale, w_scale = gib_kib / fmax, gib_kib / wmax
    lines = ["# rocprofv3 counters: %s" % workload_tag, "",
             "Commands (repo root on the GPU host; one counter pass per run):", "", cmd, "",
             "Calibration: the 1 GiB device-to-device copy reads FETCH_SIZE %.0f KiB and "
             "WRITE_SIZE %.0f KiB per dispatch, so the counters are scaled by %.4f (fetch) "
             "and %.4f (write) to bytes moved." % (fmax, wmax, f_scale, w_scale), "",
             "Per dispatch (mean over the dispatches of the kernel); queries = %d per "
             "launch; VALU issue = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x GRBM_GUI_ACTIVE/8 "
             "XCDs):" % N, "",
             "| kernel | VGPR | AGPR | scratch B/lane | LDS B | VALU lane-instr./query | "
             "SALU instr./query (x64) | VALU issue | FETCH GB | WRITE GB |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    traffic = {}
    mean = lambda xs: sum(xs) / len(xs)
    main_kernels = ("k_eval_sample<", "k_furnace_w<", "k_eval<", "k_sample<")
    for k in inst:
        if "copy" in k.lower() or k not in fetch or not k.startswith(main_kernels):
            continue
        g = mean([gs for (_, _, gs) in inst[k]["SQ_INSTS_VALU"]])
        valu = mean([v for (_, v, _) in inst[k]["SQ_INSTS_VALU"]])
        salu = mean([v for (_, v, _) in inst[k]["SQ_INSTS_SALU"]])
        gui = mean([v for (_, v, _) in inst[k]["GRBM_GUI_ACTIVE"]])
        nq = N if g < N else g
        fb = mean([v for (_, v, _) in fetch[k]["FETCH_SIZE"]]) * 1024 * f_scale
        wb = mean([v for (_, v, _) in write[k]["WRITE_SIZE"]]) * 1024 * w_scale
        m = meta[k]
        lines.append("| `%s` | %s | %s | %s | %s | %.0f | %.1f | %.2f | %.3f | %.3f |" % (
            k, m["VGPR_Count"], m["Accum_VGPR_Count"], m["Scratch_Size"], m["LDS_Block_Size"],
            valu * 64 / nq, salu * 64 / nq, valu * 4 / (1024 * gui / 8), fb / 1e9, wb / 1e9))
        # a stage's kernel is the variant the step launches most (the extras
        # launch other instantiations a few times)
        nd = len(inst[k]["SQ_INSTS_VALU"])
        for st, pre in _STAGE_KERNEL.items():
            if k.startswith(pre) and nd > traffic.get(st, {}).get("dispatches", 0):
                traffic[st] = {"fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb,
                               "kernel": k, "dispatches": nd}
    lines += ["", "FLOP-class counters per query (counter total / queries):", "",
              "| kernel | " + " | ".join(c.replace("SQ_INSTS_VALU_", "") for c in
                                        sorted(next(iter(flops.values())))) + " |",
              "|---|" + "---|" * len(next(iter(flops.values())))]
    for k, cs in flops.items():
        if "copy" in k.lower() or not k.startswith(main_kernels):
            continue
        lines.append("| `%s` | " % k + " | ".join(
            "%.1f" % (mean([v for (_, v, _) in cs[c]]) / N) for c in sorted(cs)) + " |")
    # executed floating-point work from the FLOPS counters (per wavefront
    # instruction, an FMA counting 2; x 64 lanes), priced at the kernel's
    # HIP-event time in the traced bench run
    kms = dict(bj.get("unfused", {}).get("kernels_ms", {}))
    kms.update(bj["kernels_ms"])
    stage_of = {"k_eval_sample<": "eval_sample", "k_furnace<": "furnace", "k_eval<": "eval",
                "k_sample<": "sample"}
    lines += ["", "Executed FLOPs from the counters, (FLOPS_FP64 + FLOPS_FP64_TRANS + FLOPS_FP32 + "
              "FLOPS_FP32_TRANS) x 64 lanes per query (per draw for the furnace), at the kernel's "
              "HIP-event time in this run, against the 78.6 TFLOP/s FP64 / unpacked FP32 vector "
              "peak (and the 157.3 TFLOP/s packed FP32 figure):", "",
              "| kernel | executed FLOP/query | ms | executed TFLOP/s | of 78.6 | of 157.3 |",
              "|---|---|---|---|---|---|"]
    for k, cs in flops.items():
        st = next((v for pre, v in stage_of.items() if k.startswith(pre)), None)
        if st is None or st not in kms:
            continue
        fq = 64 * sum(mean([v for (_, v, _) in cs[c]]) for c in cs if "FLOPS" in c) / N
        rate = fq * N / (kms[st] * 1e-3) / 1e12
        lines.append("| `%s` | %.0f | %.3f | %.1f | %.1f %% | %.1f %% |" % (
            k, fq, kms[st], rate, 100 * rate / PEAK_VALU_TFLOPS, 100 * rate / 157.3))
    open(os.path.join(ROOT, "profiles", "bysdf_%s_counters.md" % tag), "w").write(
        "\n".join(lines) + "\n")
    if os.path.isdir(os.path.join(prof_dir, "l2")):
        _summarize_all(prof_dir, stats, counters, f_scale, w_scale, cmd)
    json.dump({"src_hash": _src_hash(), "workload": workload_tag,
               "unit": "bytes per launch",
               "calibration": {"fetch_scale": f_scale, "write_scale": w_scale,
                               "copy_bytes": 1 << 30},
               "kernels": traffic},
              open(os.path.join(ROOT, "profiles", "traffic.json"), "w"), indent=1)
    print("\n".join(lines))


def _summarize_all(prof_dir, stats, counters, f_scale, w_scale, cmd):
    """Every kernel of the profiled bench run (main step and extras): per
    launch, the executed floating-point work from the FLOPS counters and
    the HBM bytes from FETCH_SIZE and WRITE_SIZE, priced at the kernel's
    trace-average duration against the 78.6 TFLOP/s vector peak and 8 TB/s;
    VALU issue; L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS))."""
    inst, meta = counters("inst")
    flops, _ = counters("flops")
    fetch, _ = counters("fetch")
    write, _ = counters("write")
    l2, _ = counters("l2")
    # optional pass: VALU lane utilisation and the share of wave time spent
    # waiting (SQ_THREAD_CYCLES_VALU, SQ_ACTIVE_INST_VALU, SQ_WAIT_ANY,
    # SQ_WAVE_CYCLES)
    util = counters("util")[0] if os.path.isdir(os.path.join(prof_dir, "util")) else {}
    mean = lambda xs: sum(xs) / len(xs) if xs else float("nan")
    lines = ["# rocprofv3: every kernel of the bench run", "",
             "Commands (repo root on the GPU host; one counter pass per run):", "", cmd, "",
             "Per launch (mean over the launches of the kernel in the counter passes), priced at "
             "the kernel-trace average duration.  Executed TFLOP/s = (FLOPS_FP64 + FLOPS_FP64_TRANS "
             "+ FLOPS_FP32 + FLOPS_FP32_TRANS) x 64 lanes / duration, against 78.6 TFLOP/s; HBM = "
             "FETCH_SIZE + WRITE_SIZE (scaled by the 1 GiB copy: %.4f, %.4f) / duration, against "
             "8 TB/s; VALU issue = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 "
             "XCDs); L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS); lane util. = SQ_THREAD_CYCLES_VALU / "
             "(64 x SQ_ACTIVE_INST_VALU), the share of the 64 lanes active in the VALU cycles "
             "issued; waiting = SQ_WAIT_ANY / SQ_WAVE_CYCLES, the share of resident-wave time spent "
             "at a wait." % (f_scale, w_scale), "",
             "| kernel | launches | avg us | VGPR | scratch B/lane | VALU issue | executed TFLOP/s "
             "| of 78.6 | HBM GB/launch | HBM GB/s | of 8 TB/s | L2 hit | lane util. | waiting |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    rows = []
    for k, (calls, avg_us, _, _, _) in stats.items():
        if k not in inst or "copy" in k.lower() or "fill" in k.lower():
            continue
        t = avg_us * 1e-6
        fl = 64 * sum(mean([v for (_, v, _) in flops[k][c]]) for c in flops.get(k, {}) if "FLOPS" in c)
        fb = mean([v for (_, v, _) in fetch[k]["FETCH_SIZE"]]) * 1024 * f_scale if k in fetch else 0.0
        wb = mean([v for (_, v, _) in write[k]["WRITE_SIZE"]]) * 1024 * w_scale if k in write else 0.0
        gui = mean([v for (_, v, _) in inst[k]["GRBM_GUI_ACTIVE"]])
        valu = mean([v for (_, v, _) in inst[k]["SQ_INSTS_VALU"]])
        hit = mean([v for (_, v, _) in l2[k]["TCC_HIT_sum"]]) if k in l2 else float("nan")
        miss = mean([v for (_, v, _) in l2[k]["TCC_MISS_sum"]]) if k in l2 else float("nan")
        tf = fl / t / 1e12 if t > 0 else 0.0
        gbs = (fb + wb) / t / 1e9 if t > 0 else 0.0
        m = meta[k]
        lane = wait = float("nan")
        if k in util:
            u = {c: mean([v for (_, v, _) in util[k][c]]) for c in util[k]}
            if u.get("SQ_ACTIVE_INST_VALU", 0) > 0:
                lane = u["SQ_THREAD_CYCLES_VALU"] / (64 * u["SQ_ACTIVE_INST_VALU"])
            if u.get("SQ_WAVE_CYCLES", 0) > 0:
                wait = u["SQ_WAIT_ANY"] / u["SQ_WAVE_CYCLES"]
        rows.append((calls * avg_us, "| `%s` | %d | %.1f | %s | %s | %.2f | %.2f | %.1f %% | %.3f | %.0f | "
                     "%.1f %% | %.2f | %.2f | %.2f |" % (k, calls, avg_us, m["VGPR_Count"], m["Scratch_Size"],
                                                      valu * 4 / (1024 * gui / 8) if gui else 0.0, tf,
                                                      100 * tf / PEAK_VALU_TFLOPS, (fb + wb) / 1e9, gbs,
                                                      100 * gbs / PEAK_HBM_GBS, hit / (hit + miss)
                                                      if hit + miss > 0 else float("nan"), lane, wait)))
    lines += [r for _, r in sorted(rows, key=lambda x: -x[0])]
    open(os.path.join(ROOT, "profiles", "all_kernels_bench_counters.md"), "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _op_counts(bysdf, T, P, q, mode, n=4096):
    L = bysdf.lib()
    L.bysdf_count_ops.argtypes = ([C.POINTER(bysdf.TypeParams), C.c_void_p, C.c_int64]
                                  + [C.c_void_p] * 6 + [C.c_int32, C.c_void_p])
    arr = bysdf.params_array(P[:1])
    tab = np.ascontiguousarray(bysdf.bysdf_types_table(T, 0))
    f = lambda a: np.ascontiguousarray(a, np.float32).ctypes.data_as(C.c_void_p)
    c = np.zeros(10)
    rc = L.bysdf_count_ops(arr, tab.ctypes.data_as(C.c_void_p), n, f(q["h"][:n]), f(q["u"][:n]),
                           f(q["v"][:n]), f(q["wi"][:, :n]), f(q["wo"][:, :n]),
                           f(q["xi"][:, :n]), mode, c.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise RuntimeError("bysdf_count_ops failed")
    return c


def _host_cores():
    """Cores this process may run on (its affinity set) and the host's count."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, aff), os.cpu_count()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        return None


def _cpu_baseline(P, q, target_s):
    """FP64 oracle on the first blocks of the workload, same stages (eval at
    wo, one sampled direction with its pdf, furnace per block), on every core
    the process may use."""
    import oracle
    cores, host_cpus = _host_cores()

    def run(nb):
        n = nb * 256
        sub = {k: (v[..., :n] if v is not None else None) for k, v in q.items()}
        sub["type"] = sub["type"].copy()
        ts = oracle.TypeSet(P[:nb])
        t0 = time.perf_counter()
        oracle.eval(ts, sub, nthreads=cores)
        oracle.sample(ts, sub, nthreads=cores)
        oracle.furnace(ts, sub, 256, nthreads=cores)
        return time.perf_counter() - t0

    # grow the sample until it takes about target_s (a small first run is
    # dominated by fixed costs, so one extrapolation undershoots)
    nb = 16
    dt = run(nb)
    for _ in range(4):
        if dt >= 0.5 * target_s or nb >= len(P):
            break
        nb = int(min(len(P), max(nb + 1, nb * target_s / max(dt, 1e-3))))
        dt = run(nb)
    n = nb * 256
    return {"value": n / dt, "unit": "queries/s", "cores": cores, "host_cpus": host_cpus,
            "kind": "oracle", "cpu": _cpu_model(),
            "sample": "first %d blocks (%d queries) of the per-block workload, same "
                      "stages (eval, sample with pdf, furnace), %.1f s" % (nb, n, dt)}


def _cpu_configs(torch, bysdf, W):
    """The oracle on the other workloads, on every core the process may use:
    the single-type 2^16-query evaluation and the 4,096-type batch in full,
    the fitting workload (forward at the hidden and the starting parameters,
    and the 17-evaluation central-difference gradient of the loss), and the
    two 64 x 64 crops of the weave view at 64 spp.  The fitting record also
    carries what needs the oracle's targets and differences: the GPU
    adjoint's gradient error against them and an Adam fit's parameter
    recovery."""
    import oracle
    cores, _ = _host_cores()
    out = {}
    # single type, 2^16 queries
    P0, q0 = W.single_type(65536, 0)
    t0 = time.perf_counter()
    oracle.eval(P0, q0, nthreads=cores)
    dt = time.perf_counter() - t0
    out["single_type_2e16"] = {"queries": 65536, "s": dt, "value": 65536 / dt, "unit": "queries/s",
                               "stage": "eval"}
    # 4,096 types, ~2^26 queries, in chunks of 4 M queries
    P3, q3, off3 = W.heterogeneous(4096, 3)
    ts3 = oracle.TypeSet(P3)
    n3 = len(q3["h"])
    t0 = time.perf_counter()
    for a in range(0, n3, 1 << 22):
        b = min(n3, a + (1 << 22))
        oracle.eval(ts3, {k: (v[..., a:b] if v is not None else None) for k, v in q3.items()},
                    nthreads=cores)
    dt = time.perf_counter() - t0
    out["hetero_4096_types"] = {"queries": n3, "s": dt, "value": n3 / dt, "unit": "queries/s",
                                "stage": "eval (in full)"}
    del q3, ts3
    out["fitting_64x65536"] = _fit_c4(torch, bysdf, W, oracle, cores)
    out["weave_crops_64spp"] = _weave_crops_oracle(W, oracle, cores)
    return out


def _fit_c4(torch, bysdf, W, oracle, cores, steps=500):
    """Fitting workload (64 types x 65,536 queries): the oracle's forward and
    its 17-evaluation central-difference gradient of the loss at the
    starting parameters; the GPU adjoint's per-type gradient against those
    differences; and an Adam fit (lr 1e-2, 500 steps, every parameter free,
    projected into the valid ranges) from the range midpoints towards the
    oracle's targets at the hidden parameters."""
    from paper_2401_12724_amd.autograd import bysdf_fit_step
    hidden, start, q = W.fitting(64, 65536, 4)
    n = len(q["h"])
    ts_h, ts_s = oracle.TypeSet(hidden), oracle.TypeSet(start)
    t0 = time.perf_counter()
    target = oracle.eval(ts_h, q, nthreads=cores)[0][:, :3]
    fwd_s = time.perf_counter() - t0
    E0 = oracle.eval(ts_s, q, nthreads=cores)[0][:, :3]
    gE = (2.0 * (E0 - target)).astype(np.float32)
    t0 = time.perf_counter()
    _, pa = oracle.grad_fd(ts_s, q, gE, 1e-7, nthreads=cores)
    fd_s = time.perf_counter() - t0
    # a difference quotient counts where a second step size agrees with it:
    # a texel centre of the piecewise-linear fiber table inside the step, or
    # a non-contracting ply fixed point, makes it meaningless elsewhere
    _, pb = oracle.grad_fd(ts_s, q, gE, 3e-8, nthreads=cores)
    ok = np.abs(pa - pb) <= 1e-4 * np.maximum(np.abs(pa), 1e-7) + 1e-9
    # the GPU adjoint of the same loss at the same parameters, per query
    T = bysdf.bysdf_types_create(start)
    qd = bysdf.to_device(q)
    off = torch.from_numpy(np.arange(65, dtype=np.int64) * 65536).cuda()
    _, pq = bysdf.bysdf_eval_backward(T, qd, off, torch.from_numpy(gE).cuda(), per_query=True)
    pq = pq.cpu().numpy().astype(np.float64)
    tid = q["type"]
    g_fd = np.zeros((64, 8))
    g_gpu = np.zeros((64, 8))
    np.add.at(g_fd, tid, np.where(ok, pa, 0.0))
    np.add.at(g_gpu, tid, np.where(ok, pq, 0.0))
    rel = np.abs(g_gpu - g_fd) / np.maximum(np.abs(g_fd), 1e-30)
    names = W.THETA_NAMES
    grad_err = {nm: {"median": float(np.median(rel[:, k])), "p90": float(np.percentile(rel[:, k], 90)),
                     "max": float(rel[:, k].max()), "queries_counted": float(ok[:, k].mean())}
                for k, nm in enumerate(names)}
    # Adam fits against the oracle's targets: every parameter free, and with
    # the twists known (held at their hidden values, as the paper's fitting
    # takes the geometry as given)
    tgt = torch.from_numpy(target.astype(np.float32)).cuda()
    th_true = np.stack([W.theta_of(p) for p in hidden])
    th_mid = np.stack([W.theta_of(p) for p in start])
    groups = {"albedo": [0, 1, 2], "beta": [3], "ply_twist": [4], "fiber_twist": [5],
              "densities": [6, 7]}
    fits = {}
    fit_s = 0.0
    for label, known in (("all_free", ()), ("twists_known", (4, 5))):
        th0 = th_mid.copy()
        free = np.ones(8, np.float32)
        for k in known:
            th0[:, k] = th_true[:, k]
            free[k] = 0.0
        theta = torch.tensor(th0, dtype=torch.float32, device="cuda", requires_grad=True)
        mask = torch.from_numpy(free).cuda()
        theta.register_hook(lambda g, m=mask: g * m)
        opt = torch.optim.Adam([theta], lr=1e-2, betas=(0.9, 0.999))
        losses = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            losses.append(bysdf_fit_step(theta, T, qd, off, tgt, opt))
        torch.cuda.synchronize()
        fit_s = time.perf_counter() - t0
        err0 = np.abs(th0 - th_true)
        err1 = np.abs(theta.detach().cpu().numpy() - th_true)
        fits[label] = {"loss_start": float(losses[0]), "loss_end": float(losses[-1]),
                       "mean_abs_param_error": {
                           g: {"start": float(err0[:, ix].mean()), "fitted": float(err1[:, ix].mean())}
                           for g, ix in groups.items() if not set(ix) & set(known)}}
    return {"queries": n, "types": 64, "cores": cores,
            "oracle_forward_s": fwd_s, "oracle_forward_queries_per_s": n / fwd_s,
            "oracle_fd_gradient_s": fd_s, "oracle_fd_queries_per_s": n / fd_s,
            "fd_evaluations_per_query": 17,
            "gpu_grad_rel_error_vs_fd": grad_err,
            "grad_note": "per type and parameter, the GPU adjoint of the loss sum_q sum_c "
                         "(E - E*)^2 at the starting parameters against the oracle's central "
                         "differences of the same sum, over the queries whose differences at "
                         "relative steps 1e-7 and 3e-8 agree to 1e-4 (queries_counted)",
            "fit": dict(steps=steps, lr=1e-2, ms_per_step=fit_s / steps * 1e3, **fits)}


def _weave_crops_oracle(W, oracle, cores):
    """The oracle's path tracer on the two 64 x 64 validation crops of the
    weave view at 64 spp (centre; far edge with the far field); the
    full-frame time is extrapolated from the crops' path rate."""
    ctrl, off, ty, ph = W.weave()
    S = oracle.Scene(ctrl, off)
    cam = W.weave_camera()
    rows = {}
    total_paths, total_s = 0, 0.0
    for name, (cx, cy), lod in (("centre", (928, 508), 1.0), ("far_edge", (928, 384), 4.0)):
        rs = dict(eye=cam["eye"], look_at=cam["look_at"], up=cam["up"], vfov=cam["vfov"],
                  width=cam["width"], height=cam["height"], crop_x=cx, crop_y=cy, crop_w=64,
                  crop_h=64, light_corner=(-5.0, -5.0, 30.0), light_u=(0.0, 10.0, 0.0),
                  light_v=(10.0, 0.0, 0.0), light_radiance=(5.0, 5.0, 5.0),
                  env_radiance=(0.2, 0.2, 0.2), spp=64, max_depth=8, lod_px=lod, n_h=4, seed=2,
                  ray_eps=1e-4, spp_batch=0)
        t0 = time.perf_counter()
        oracle.render(S, [W.default_params()], ty, ph, rs, nthreads=cores)
        dt = time.perf_counter() - t0
        paths = 64 * 64 * 64
        rows[name] = {"paths": paths, "s": dt, "paths_per_s": paths / dt}
        total_paths += paths
        total_s += dt
    rate = total_paths / total_s
    rows["full_frame_extrapolated_s"] = cam["width"] * cam["height"] * 64 / rate
    rows["note"] = ("full_frame_extrapolated_s: 1920 x 1080 x 64 paths at the crops' mean "
                    "path rate (extrapolated, not run)")
    return rows


def _timed(torch, fn, reps):
    stream = torch.cuda.current_stream()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return float(np.median(ms))


def _hetero(torch, bysdf, W, single_type_eval_qps):
    """4,096 types with lognormal counts (~2^26 queries) in one persistent
    launch: autotuned schedule, captured in a graph, replayed."""
    from paper_2401_12724_amd import autotune
    P, q, off = W.heterogeneous(4096, 3)
    n = len(q["h"])
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    del q
    offd = torch.from_numpy(off).cuda()
    out = bysdf.alloc_eval_out(n)
    cands = [dict(chunk=c, grid=g, use_lds=l, block=b, min_waves=w) for c in (1, 4, 16)
             for g in (1024, 4096) for l in (1, 0) for b in (128, 256) for w in (1, 2)]
    tune = autotune.autotune_batched(T, offd, qd, off, out=out, candidates=cands, reps=2)
    ws = bysdf.alloc_workspace(bysdf.bysdf_batched_workspace_size(T.n_types))
    sc = tune["schedule"]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bysdf.bysdf_eval_batched(T, offd, qd, out, sc, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bysdf.bysdf_eval_batched(T, offd, qd, out, sc, ws)
    ms = _timed(torch, g.replay, 5)
    qps = n / (ms * 1e-3)
    return {"queries": n, "types": 4096, "ms": ms, "queries_per_s": qps,
            "schedule": sc, "single_type_eval_queries_per_s": single_type_eval_qps,
            "vs_single_type": qps / single_type_eval_qps, "launch": "hipGraph replay",
            "candidates": len(cands)}


def _fwd_bwd(torch, bysdf, W):
    """64 types x 65,536 queries grouped by type: plain forward (bysdf_eval)
    against forward + adjoint (bysdf_eval + bysdf_eval_backward)."""
    hidden, start, q = W.fitting(64, 65536, 4)
    n = len(q["h"])
    off = torch.from_numpy(np.arange(65, dtype=np.int64) * 65536).cuda()
    T = bysdf.bysdf_types_create(hidden)
    qd = bysdf.to_device(q)
    out = bysdf.alloc_eval_out(n)
    gE = torch.randn((n, 3), dtype=torch.float32, device="cuda")
    gt = torch.empty((64, 8), dtype=torch.float32, device="cuda")
    ws = torch.empty(bysdf.bysdf_backward_workspace_size(n, 64) + 256, dtype=torch.uint8,
                     device="cuda")
    fwd = lambda: bysdf.bysdf_eval(T, qd, out)
    both = lambda: (bysdf.bysdf_eval(T, qd, out),
                    bysdf.bysdf_eval_backward(T, qd, off, gE, gt, workspace=ws))
    fwd()
    both()
    torch.cuda.synchronize()
    f_ms = _timed(torch, fwd, 5)
    b_ms = _timed(torch, both, 3)
    return {"queries": n, "types": 64, "fwd_ms": f_ms, "fwd_bwd_ms": b_ms,
            "fwd_queries_per_s": n / (f_ms * 1e-3), "fwd_bwd_queries_per_s": n / (b_ms * 1e-3),
            "fwd_bwd_over_fwd_time": b_ms / f_ms}


def _migration(torch, bysdf, W, P, qd, q, base_ms):
    """The per-block workload with fiber migration on every type (4 tables,
    period 3 yarn radii, blend 0.25, spread 0.4): the fused eval + sample."""
    Pm = [dict(p, mig_tables=4, mig_period=3.0, mig_blend=0.25, mig_spread=0.4, mig_seed=11)
          for p in P]
    T = bysdf.bysdf_types_create(Pm)
    n = int(qd["h"].numel())
    out = (bysdf.alloc_eval_out(n), bysdf.alloc_sample_out(n))
    f = lambda: bysdf.bysdf_eval_sample(T, qd, out)
    f()
    torch.cuda.synchronize()
    ms = _timed(torch, f, 5)
    ops = _op_counts(bysdf, T, Pm, q, 2).sum()
    return {"queries": n, "tables_per_type": 4, "eval_sample_ms": ms,
            "queries_per_s": n / (ms * 1e-3), "vs_without": base_ms / ms,
            "ops_per_query": ops,
            "valu_frac": ops * n / (ms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS}


def _k_sweep(torch, bysdf, P, q, qd, Ks=(1, 4, 8)):
    """The per-block workload with K forward nodes per query: the
    evaluation alone and the fused eval + sample, against the VALU peak and
    against HBM (92 and 156 algorithmic bytes per query).  At small K the
    evaluation does the least arithmetic per byte."""
    n = int(qd["h"].numel())
    res = {}
    for K in Ks:
        PK = [dict(p, K=K) for p in P]
        T = bysdf.bysdf_types_create(PK)
        ev = bysdf.alloc_eval_out(n)
        out = (ev, bysdf.alloc_sample_out(n))
        row = {}
        for name, mode, nbytes, f in (("eval", 0, 92, lambda: bysdf.bysdf_eval(T, qd, ev)),
                                      ("eval_sample", 2, 156, lambda: bysdf.bysdf_eval_sample(T, qd, out))):
            f()
            torch.cuda.synchronize()
            ms = _timed(torch, f, 5)
            ops = _op_counts(bysdf, T, PK, q, mode).sum()
            gbs = nbytes * n / (ms * 1e-3) / 1e9
            row[name] = {"ms": ms, "queries_per_s": n / (ms * 1e-3), "ops_per_query": ops,
                         "valu_frac": ops * n / (ms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS,
                         "gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
        res["K%d" % K] = row
        del T, ev, out
    return res


def _multiscale(torch, bysdf, W, P, q, qd, near_ms, n_max=4):
    """The per-block workload with a pixel footprint per query (widths
    log-uniform in [2^-6, 2] yarn half-widths, so from a point to the whole
    yarn): the multi-scale evaluation and sampler with up to n_max strata."""
    qf = W.footprints(dict(q), 1)
    qm = dict(qd)
    qm.update(bysdf.to_device({k: qf[k] for k in ("h1", "h2", "zeta", "xi_s")}))
    n = int(qd["h"].numel())
    w = qf["h2"].astype(np.float64) - qf["h1"]
    strata = np.clip(np.ceil(n_max * w / 2), 1, n_max)
    T = bysdf.bysdf_types_create(P)
    eo, so = bysdf.alloc_eval_out(n), bysdf.alloc_sample_out(n)
    fe = lambda: bysdf.bysdf_eval_multi(T, qm, n_max, eo)
    fs = lambda: bysdf.bysdf_sample_multi(T, qm, n_max, so)
    fe()
    fs()
    torch.cuda.synchronize()
    e_ms, s_ms = _timed(torch, fe, 5), _timed(torch, fs, 5)
    return {"queries": n, "n_max": n_max, "strata_per_query": float(strata.mean()),
            "eval_multi_ms": e_ms, "sample_multi_ms": s_ms,
            "eval_queries_per_s": n / (e_ms * 1e-3), "sample_queries_per_s": n / (s_ms * 1e-3),
            "eval_time_vs_near": e_ms / near_ms["eval"],
            "sample_time_vs_near": s_ms / near_ms["sample"],
            # each stratum is one near-field evaluation with the aggregated
            # geometry: their rate against the near-field kernel's
            "eval_strata_per_s": n * float(strata.mean()) / (e_ms * 1e-3),
            "eval_strata_rate_vs_near": (n * float(strata.mean()) / e_ms) / (n / near_ms["eval"]),
            "note": "strata_per_query near-field states per query enter the aggregated "
                    "geometry and as many again the lobes; the sampler adds its draw"}


def _fit(torch, bysdf, W, steps=100):
    """Image-space fitting (r, k^B, sigma_t by Adam on rendered gradients)
    on a 48 x 48 crop of a 12 x 12 weave at 16 spp per step: time per step
    (type record, image, image + gradient) and the parameters reached."""
    from paper_2401_12724_amd import fit_image
    ctrl, off, ty, ph = W.weave(12, 12, 0.15, 0.05, 4)
    S = bysdf.yarn_scene_create(ctrl, off, ty, ph)
    cam = W.camera((0.0, -1.4, 0.8), (0.0, 0.0, 0.0), width=96, height=72)
    rs = dict(eye=cam["eye"], look_at=cam["look_at"], up=cam["up"], vfov=cam["vfov"], width=96,
              height=72, crop_x=24, crop_y=12, crop_w=48, crop_h=48, light_corner=(-5.0, -5.0, 30.0),
              light_u=(0.0, 10.0, 0.0), light_v=(10.0, 0.0, 0.0), light_radiance=(5.0, 5.0, 5.0),
              env_radiance=(0.2, 0.2, 0.2), spp=16, max_depth=4, lod_px=1.0, n_h=4, seed=7,
              ray_eps=1e-4, spp_batch=0)
    hidden = W.default_params(r=0.35, sigma_t=1.2, albedo=(0.75, 0.45, 0.25))
    target = bysdf.shade_wavefront(S, bysdf.bysdf_types_create([hidden]), dict(rs, spp=1024, seed=99))
    th0 = fit_image.theta_of(W.default_params(r=0.6, sigma_t=0.4, albedo=(0.5, 0.5, 0.5)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th, hist = fit_image.fit(S, [hidden], 0, target, rs, th0, steps=steps, lr=0.08)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"steps": steps, "ms_per_step": dt / steps * 1e3, "theta": [float(x) for x in th],
            "truth": [float(x) for x in fit_image.theta_of(hidden)],
            "params": "r, k^B (RGB), sigma_t"}


def _cross_section(torch, bysdf, W, P, qd):
    """The implicit ply hit alone (Sec. 3.4) on the per-block workload, with
    the elliptical cross-section (5 fixed-point updates per ply) and the
    circular one (none)."""
    n = int(qd["h"].numel())
    out = {"queries": n}
    for name, it in (("circular", 0), ("elliptical", 5)):
        T = bysdf.bysdf_types_create([dict(p, n_iter=it) for p in P])
        f = lambda: bysdf.bysdf_ply_geometry(T, qd)
        f()
        torch.cuda.synchronize()
        ms = _timed(torch, f, 5)
        out[name] = {"n_iter": it, "ms": ms, "queries_per_s": n / (ms * 1e-3)}
    return out


def _weave_render(torch, bysdf, W, spp=4, spp_full=64):
    """The plain weave (256 + 256 B-spline yarns, 524,288 spans) seen by the
    grazing 1920 x 1080 camera: primary-ray intersection of every pixel
    centre, the full frame at spp_full samples per pixel (depth <= 8,
    next-event estimation with MIS, 1-pixel LOD), and at spp samples per
    pixel the same frame plain, in multi-scale mode and with the image
    gradient."""
    ctrl, off, ty, ph = W.weave()
    t0 = time.perf_counter()
    S = bysdf.yarn_scene_create(ctrl, off, ty, ph)
    build_s = time.perf_counter() - t0
    info = bysdf.yarn_scene_info(S)
    cam = W.weave_camera()
    py, px = np.meshgrid(np.arange(cam["height"]), np.arange(cam["width"]), indexing="ij")
    o, d = W.pinhole_rays(cam, px.ravel(), py.ravel())
    n = len(o)
    od = torch.from_numpy(np.ascontiguousarray(o.T)).cuda()
    dd = torch.from_numpy(np.ascontiguousarray(d.T)).cuda()
    tm = torch.full((n,), 1e3, dtype=torch.float32, device="cuda")
    hits = bysdf.alloc_hits(n)
    isect = lambda: bysdf.yarn_tube_intersect(S, od, dd, tm, 1e-4, hits)
    isect()
    torch.cuda.synchronize()
    ims = _timed(torch, isect, 5)
    hit_frac = float((hits["flags"] & 1).eq(0).float().mean())
    T = bysdf.bysdf_types_create([W.default_params()])
    rs = dict(eye=cam["eye"], look_at=cam["look_at"], up=cam["up"], vfov=cam["vfov"],
              width=cam["width"], height=cam["height"], crop_x=0, crop_y=0,
              crop_w=cam["width"], crop_h=cam["height"], light_corner=(-5.0, -5.0, 30.0),
              light_u=(0.0, 10.0, 0.0), light_v=(10.0, 0.0, 0.0), light_radiance=(5.0, 5.0, 5.0),
              env_radiance=(0.2, 0.2, 0.2), spp=spp, max_depth=8, lod_px=1.0, n_h=4, seed=2,
              ray_eps=1e-4, spp_batch=1)
    ws = bysdf.alloc_workspace(bysdf.shade_wavefront_workspace_size(rs))
    fb = torch.empty((cam["height"], cam["width"], 3), dtype=torch.float32, device="cuda")
    # the full frame at its configured sample count
    rf = dict(rs, spp=spp_full)
    _, fcounts = bysdf.shade_wavefront(S, T, rf, fb, ws, counts=True)
    fms = _timed(torch, lambda: bysdf.shade_wavefront(S, T, rf, fb, ws), 1)
    full_mean = float(fb.mean())
    _, counts = bysdf.shade_wavefront(S, T, rs, fb, ws, counts=True)
    rms = _timed(torch, lambda: bysdf.shade_wavefront(S, T, rs, fb, ws), 3)
    rays = counts[0] + counts[1]
    # the same frame in multi-scale mode: camera hits over their pixel
    # footprint (up to 8 strata), later bounces near field
    rm = dict(rs, multiscale=1, n_h=8)
    fbm = torch.empty_like(fb)
    _, mcounts = bysdf.shade_wavefront(S, T, rm, fbm, ws, counts=True)
    mms = _timed(torch, lambda: bysdf.shade_wavefront(S, T, rm, fbm, ws), 3)
    # the same frame with the image gradient in (r, k^B, sigma_t)
    wsg = bysdf.alloc_workspace(bysdf.shade_wavefront_grad_workspace_size(rs))
    fbg = torch.empty_like(fb)
    grd = torch.empty((cam["height"], cam["width"], 3, 3), dtype=torch.float32, device="cuda")
    bysdf.shade_wavefront_grad(S, T, rs, 0, fbg, grd, wsg)
    gms = _timed(torch, lambda: bysdf.shade_wavefront_grad(S, T, rs, 0, fbg, grd, wsg), 3)
    return {"scene": {"yarns": info["n_yarns"], "spans": info["n_spans"],
                      "bvh_nodes": info["n_nodes"], "bvh_depth": info["depth"],
                      "device_bytes": info["bytes"], "build_s": build_s},
            "intersect": {"rays": n, "ms": ims, "rays_per_s": n / (ims * 1e-3),
                          "hit_fraction": hit_frac},
            "render": {"width": cam["width"], "height": cam["height"], "spp": spp_full, "ms": fms,
                       "extension_rays": fcounts[0], "shadow_rays": fcounts[1],
                       "rays_per_s": (fcounts[0] + fcounts[1]) / (fms * 1e-3),
                       "paths_per_s": cam["width"] * cam["height"] * spp_full / (fms * 1e-3),
                       "mean_radiance": full_mean},
            "render_4spp": {"width": cam["width"], "height": cam["height"], "spp": spp, "ms": rms,
                       "extension_rays": counts[0], "shadow_rays": counts[1],
                       "rays_per_s": rays / (rms * 1e-3),
                       "paths_per_s": cam["width"] * cam["height"] * spp / (rms * 1e-3),
                       "mean_radiance": float(fb.mean())},
            "render_grad": {"spp": spp, "ms": gms, "over_render_time": gms / rms,
                            "mean_radiance": float(fbg.mean()),
                            "note": "image and its gradient in r, k^B (RGB), sigma_t"},
            "render_multiscale": {"spp": spp, "n_max": 8, "ms": mms,
                                  "extension_rays": mcounts[0], "shadow_rays": mcounts[1],
                                  "paths_per_s": cam["width"] * cam["height"] * spp / (mms * 1e-3),
                                  "mean_radiance": float(fbm.mean())}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--blocks", type=int, default=65536, help="parameter blocks of 256 queries")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-configs", action="store_true",
                    help="time the oracle on the bench workload only")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for PMC byte scaling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the heterogeneous-batch and adjoint measurements")
    ap.add_argument("--summarize", metavar="PROF_DIR",
                    help="no run: summarize rocprofv3 passes under PROF_DIR into profiles/")
    args = ap.parse_args()
    if args.summarize:
        _summarize(args.summarize, os.path.join(args.summarize, "bench.json"),
                   "perblock 2e24")
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the path runs on a single GPU "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2401_12724_amd import build as hip_build
    if not os.path.exists(hip_build.LIB):
        hip_build.build()
    from paper_2401_12724_amd import bysdf, workloads as W

    torch.cuda.set_device(0)
    P, q = W.per_block(args.blocks, 256, seed=1)
    N = len(q["h"])
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    ev = bysdf.alloc_eval_out(N)
    sv = bysdf.alloc_sample_out(N)
    fm = torch.empty((N // 256, 3), dtype=torch.float32, device="cuda")
    fv = torch.empty_like(fm)
    torch.cuda.synchronize()

    names = ("eval_sample", "furnace")
    stream = torch.cuda.current_stream()

    def step(events=None):
        calls = (lambda: bysdf.bysdf_eval_sample(T, qd, (ev, sv)),
                 lambda: bysdf.bysdf_furnace_blocks(T, qd, 256, fm, fv))
        for k, c in enumerate(calls):
            if events is not None:
                events[k][0].record(stream)
            c()
            if events is not None:
                events[k][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in names] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ktime = {nm: float(np.mean([evs[s][k][0].elapsed_time(evs[s][k][1])
                                for s in range(args.steps)])) for k, nm in enumerate(names)}
    ms_per_step = 1e3 * elapsed / args.steps
    value = N * args.steps / elapsed

    # the same work through the separate entry points, for comparison
    ev2 = bysdf.alloc_eval_out(N)
    sv2 = bysdf.alloc_sample_out(N)
    q2 = dict(qd)
    q2["wo"] = sv2[0][0:3]  # sampled directions, rows of the sample output
    sep = {"eval": lambda: bysdf.bysdf_eval(T, qd, ev2),
           "sample": lambda: bysdf.bysdf_sample_pdf(T, qd, sv2),
           "eval_at_sample": lambda: bysdf.bysdf_eval(T, q2, ev2)}
    for f in sep.values():
        f()
    unfused = {k: _timed(torch, f, max(3, args.steps)) for k, f in sep.items()}
    del ev2, sv2, q2

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # algorithmic operations per query (kernels' own formulation)
    ops_eval = _op_counts(bysdf, T, P, q, 0)
    ops_samp = _op_counts(bysdf, T, P, q, 1)
    ops_both = _op_counts(bysdf, T, P, q, 2)
    per_query = {"eval_sample": ops_both.sum(), "furnace": ops_samp.sum()}
    dom = max(ktime, key=ktime.get)
    achieved = per_query[dom] * N / (ktime[dom] * 1e-3) / 1e12
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        tj = json.load(open(tpath))
        if tj.get("src_hash") == _src_hash() and dom in tj.get("kernels", {}):
            traffic = tj["kernels"][dom]["bytes"]
    # algorithmic bytes per query of each kernel (SoA records, 4 B fields)
    # eval_sample: type, h, u, v, wi, wo, xi in (52 B); eval out 12 floats +
    # flags, sample out 10 floats + lobe + node + flags (104 B)
    bytes_q = {"eval_sample": 52 + 104, "furnace": 4 * 8 + 24.0 / 256}
    out = {
        "metric": "BYSDF queries/s (eval+sample, fp32), % VALU peak; fwd+bwd vs plain fwd",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry + f32 lobes",
        "data": "synthetic",
        "config": {"workload": "per-block: %d queries in %d blocks of 256, 3-ply yarn "
                               "(64 fibers/ply, twist 28/15 deg, r_p 0.45, eta 1.55), beta "
                               "U[0.05,0.3] and albedo U[0.3,0.95]^3 per block; step = eval "
                               "at (wi, wo) and one sampled wo with its weight and pdf (one "
                               "kernel), furnace per block" % (N, N // 256),
                   "queries": N, "blocks": N // 256, "K": 4, "n_iter": 5},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_VALU_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, "
                                     "scaled by a 1 GiB copy)",
                     "algorithmic_bytes": bytes_q[dom] * N,
                     "ops_per_query": per_query[dom]},
        "kernels_ms": ktime,
        "kernel_gbs": {k: bytes_q[k] * N / (ktime[k] * 1e-3) / 1e9 for k in names},
        "ops_per_query": {"eval_sample": {"fp64": ops_both[:5].tolist(),
                                          "fp32": ops_both[5:].tolist()},
                          "eval": {"fp64": ops_eval[:5].tolist(), "fp32": ops_eval[5:].tolist()},
                          "sample": {"fp64": ops_samp[:5].tolist(), "fp32": ops_samp[5:].tolist()},
                          "order": "add mul div sqrt transcendental"},
        "unfused": {"kernels_ms": unfused,
                    "step_ms": unfused["eval"] + unfused["sample"] + unfused["eval_at_sample"]
                    + ktime["furnace"],
                    "eval_queries_per_s": N / (unfused["eval"] * 1e-3),
                    "sample_queries_per_s": N / (unfused["sample"] * 1e-3),
                    "note": "bysdf_eval, bysdf_sample_pdf and bysdf_eval at the sampled "
                            "directions as separate launches, plus the furnace"},
        "src_hash": _src_hash(),
    }
    if not args.no_extras:
        eval_qps = N / (unfused["eval"] * 1e-3)
        del ev, sv
        extras = (("migration", lambda: _migration(torch, bysdf, W, P, qd, q, ktime["eval_sample"])),
                  ("k_sweep", lambda: _k_sweep(torch, bysdf, P, q, qd)),
                  ("multiscale", lambda: _multiscale(torch, bysdf, W, P, q, qd, unfused)),
                  ("cross_section", lambda: _cross_section(torch, bysdf, W, P, qd)),
                  ("hetero", lambda: _hetero(torch, bysdf, W, eval_qps)),
                  ("fwd_bwd", lambda: _fwd_bwd(torch, bysdf, W)),
                  ("weave", lambda: _weave_render(torch, bysdf, W)),
                  ("fit", lambda: _fit(torch, bysdf, W)))
        for name, fn in extras:
            out[name] = fn()
            print("bench.py: %s done" % name, file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(P, q, args.cpu_seconds)
        if not args.no_cpu_configs:
            out["cpu_baseline"]["configs"] = _cpu_configs(torch, bysdf, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
