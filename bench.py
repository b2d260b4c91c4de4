#!/usr/bin/env python3
"""Benchmark of the per-cycle layer cascade on one MI355X.

Metric: instance-cycles/s (instances x clock cycles simulated per second),
for the batched form (many stimulus instances of one design) and the plain
form (one instance), plus the achieved fraction of the HBM / LDS roofline of
the simulation kernel and the CPU oracle's rate on a bounded sample.

A step is one rteaal_step of `cycles_per_step` cycles over the whole batch;
inputs (design, state, seeds) are resident on the device before timing.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

Workloads: large-5m (default; 5M operations, 4,096 instances), single-200k,
plain-2k, multi-64 (64 uneven designs in one rteaal_step_many), serving
(continuous batching of a Poisson job stream), levelize-5m (the device
levelizer on the shuffled large-5m graph), waveform (value-change capture),
muxchain-2m (the same mux-heavy design as drawn and after mux-chain fusion),
block-probe (the common kernel's gather rate by block size).
"""
import argparse
import hashlib
import json
import math
import re
import os
import sys
import time

import numpy as np

# More hardware queues than HIP's default of 4, so that the streams
# rteaal_step_many uses (a chain of captured cycles, RESIDENT configurations
# beside it) each get their own queue rather than waiting behind another's
# long launch.  Set before the HIP runtime starts; an explicit setting wins.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import rtlgen  # noqa: E402

METRIC = "instance-cycles/s (batched vs plain) + % HBM/LDS roofline, bit-exact"
HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E
LDS_PEAK_GBS = 256 * 128 * 2.4        # 256 CUs x 128 B/clk x 2.4 GHz = 78,643 GB/s

# Workloads: design recipe, batched instance count, default cycles per step
# and default number of timed steps (a bounded sample of the workload's run:
# the rate is steady from the first cycles on).
WORKLOADS = {
    "large-5m": dict(cfg=rtlgen.CFG3, seed=3, instances=4096, cycles=10_000, cycles_per_step=5,
                     steps=10, profile_cycles=10, plain_cycles=200),
    "single-200k": dict(cfg=rtlgen.CFG1, seed=1, instances=1024, cycles=100_000,
                        cycles_per_step=100, steps=10, profile_cycles=50, plain_cycles=2000),
    "plain-2k": dict(cfg=rtlgen.CFG0, seed=0, instances=1, cycles=10_000, cycles_per_step=10_000,
                     steps=1, profile_cycles=1024, plain_cycles=10_000),
}


# The paper's own results, as context (its text prints no simulation rate:
# speeds appear only in figures).
PAPER_CONTEXT = ("paper: single-threaded generated C++ kernels on four CPUs (Core i9-13900K, "
                 "Xeon Gold 5512U, Ryzen 7 4800HS, Graviton 4), Chipyard designs; the best kernel "
                 "beats Verilator on every machine and ESSENT on SmallBOOM-8c (Ryzen); no GPU, "
                 "batched or instance-cycles/s figures")


def wb(w):
    """Bytes one value of width w takes in the canonical word model (1-bit values bit-sliced)."""
    w = np.asarray(w, dtype=np.int64)
    return np.where(w == 1, 0.125, np.where(w <= 32, 4.0, np.where(w <= 64, 8.0, 8.0 * ((w + 63) // 64))))


def eb(w):
    """Bytes one value of width w takes in the library's storage encoding:
    1-bit values bit-sliced, 2-8 and 9-16 bits in 1 and 2 bytes, then as wb."""
    w = np.asarray(w, dtype=np.int64)
    return np.where(w <= 8, np.where(w == 1, 0.125, 1.0), np.where(w <= 16, 2.0, wb(w)))


def algorithmic_bytes(d, bytes_of=wb):
    """Algorithmic bytes of one cycle, split by the kernel that moves them.

    X: per instance-cycle state bytes (operand gathers + result stores,
    register commit, input writes); G: per-cycle bytes of the packed graph
    tensor (coordinates at the layer's bit width, a 9-bit type code, 8-bit
    immediates).  "light" covers the operations whose values are all at most
    64 bits wide (the common SWEEP kernel), "heavy" the wider ones and the
    sources (the SWEEP kernel of heavy operations).  bytes_of gives a value's
    bytes: wb for the canonical word model, eb for the storage encoding."""
    W = d.slot_width.astype(np.int64)
    ar = d.op_arity()
    n = d.n_ops
    src_b = bytes_of(W[d.op_src])
    src_w = W[d.op_src]
    ptr = d.op_src_ptr.astype(np.int64)
    op_x = bytes_of(W[d.op_dst]).astype(np.float64)
    op_wmax = W[d.op_dst].copy()
    has = ar > 0
    if src_b.size:
        idx = ptr[:-1][has]
        op_x[has] += np.add.reduceat(src_b, idx)
        op_wmax[has] = np.maximum(op_wmax[has], np.maximum.reduceat(src_w, idx))
    # wide values, and the types the encoder always runs in the wide form
    # (the FIRRTL primitives DIV .. SEXT and fused mux chains)
    op_heavy = (op_wmax > 64) | ((d.op_type >= rtlgen.DIV) & (d.op_type <= rtlgen.MUXC))
    op_g = np.zeros(n, dtype=np.float64)
    for i in range(d.n_layers):
        a, b = int(d.layer_ptr[i]), int(d.layer_ptr[i + 1])
        if a == b:
            continue
        sl = slice(int(d.op_src_ptr[a]), int(d.op_src_ptr[b]))
        cb = max(int(d.op_dst[a:b].max()), int(d.op_src[sl].max())).bit_length()
        imm = np.isin(d.op_type[a:b], (rtlgen.SHL, rtlgen.SHR, rtlgen.EXTRACT))
        op_g[a:b] = ((1 + ar[a:b]) * cb + 9 + 8 * imm) / 8.0
    reg_x = bytes_of(W[d.reg_next]) + bytes_of(W[d.reg_slot])
    reg_heavy = W[d.reg_slot] > 64
    x_in = float(bytes_of(W[d.input_slot]).sum())
    out = {
        "x_light": float(op_x[~op_heavy].sum() + reg_x[~reg_heavy].sum()),
        "x_heavy": float(op_x[op_heavy].sum() + reg_x[reg_heavy].sum() + x_in),
        "g_light": float(op_g[~op_heavy].sum()),
        "g_heavy": float(op_g[op_heavy].sum()),
    }
    out["x"] = out["x_light"] + out["x_heavy"]
    out["g"] = out["g_light"] + out["g_heavy"]
    return out


def kernel_sources_sha256():
    """Hash of the device code (kernels and the record encoding they read),
    comments and whitespace removed, so that only code changes alter it."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2601_18140_amd", "csrc")
    for f in ("internal.h", "kernels.hip", "ops_device.h"):   # device code and its encoding
        with open(os.path.join(d, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(f.encode())
        h.update("".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(role, workload, opts):
    """HBM bytes per launch of kernel `role` from the committed rocprofv3
    counter record (FETCH_SIZE and WRITE_SIZE runs, scaled by the copy
    calibration), or None when no record matches this workload and launch
    shape or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not opts or not os.path.exists(path):
        return None
    key = (f"{role}|{workload}|sweep/opw{opts['ops_per_wave']}/u{opts['unroll']}"
           f"/tg{opts['tiles_per_wave']}/as{opts.get('arity_split', 0)}"
           f"/tpp{opts.get('tiles_per_pass', 0)}" + ("/pb1" if opts.get("pass_branches") else ""))
    with open(path) as fh:
        rec = json.load(fh).get(key)
    if rec is None or rec["source_sha256"] != kernel_sources_sha256():
        return None
    return float(rec["bytes_per_launch"])


def timed_runs(torch, stream, run, repeats):
    """Milliseconds of `repeats` timed regions, each bracketed by a device
    synchronisation and HIP events on the library's stream."""
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        ev0.record(stream)
        run()
        ev1.record(stream)
        ev1.synchronize()
        torch.cuda.synchronize()
        out.append(ev0.elapsed_time(ev1))
    return out


def start_oracle(d, seeds, cycles, threads=None):
    """The oracle (registers and register digest) on a background thread:
    its C code releases the interpreter lock, so the GPU work goes on."""
    import threading
    import oracle
    res = {}

    def go():
        t0 = time.perf_counter()
        dg = {}
        res["regs"], _, _ = oracle.run(d, seeds, cycles, n_threads=threads or len(seeds), digests=dg)
        res["digest"] = dg["final"]
        res["seconds"] = time.perf_counter() - t0

    th = threading.Thread(target=go, daemon=True)
    th.start()
    return th, res


def host_threads():
    """Host threads the oracle may use: the machine's CPU share for one GPU (16)
    or fewer when fewer CPUs are visible."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(d, seeds, cycles, full_instances, full_cycles):
    """The oracle timed on the host cores on a bounded sample (instance-
    parallel: one instance per thread), with the per-core rate and the
    full workload's oracle time extrapolated from it."""
    import oracle
    threads = min(host_threads(), len(seeds))
    t0 = time.perf_counter()
    oracle.run(d, seeds, cycles, n_threads=threads)
    dt = time.perf_counter() - t0
    rate = len(seeds) * cycles / dt
    return {"value": rate, "unit": "instance-cycles/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(seeds)} instances x {cycles} cycles of the same design, "
                      f"{dt:.1f} s wall on {threads} host threads",
            "per_core": rate / threads, "host_cpus_visible": os.cpu_count(),
            "extrapolated_full_workload": {
                "instances": full_instances, "cycles": full_cycles,
                "seconds": round(full_instances * full_cycles / rate, 1),
                "label": f"extrapolation: the sample's rate on {threads} cores (instance-parallel, "
                         "so it holds for any batch of at least that many instances)"}}


def whole_cycle(AB, ABE, n_inst, ms_per_cycle, counter_bytes_per_cycle):
    """Graded fraction of one cycle: the method's compulsory bytes of a
    cycle (n_inst * X + G) over 8 TB/s, divided by the measured time per
    cycle; word model, storage encoding and (when counter records exist)
    the measured HBM bytes."""
    t = ms_per_cycle / 1e3
    word = AB["x"] * n_inst + AB["g"]
    enc = ABE["x"] * n_inst + ABE["g"]
    out = {"ms_per_cycle": round(ms_per_cycle, 4),
           "word_model_bytes": round(word, 1), "word_model_GBps": round(word / t / 1e9, 2),
           "word_model_frac": round(word / t / 1e9 / HBM_PEAK_GBS, 4),
           "encoded_bytes": round(enc, 1), "encoded_GBps": round(enc / t / 1e9, 2),
           "encoded_frac": round(enc / t / 1e9 / HBM_PEAK_GBS, 4),
           "counter_bytes": None, "counter_GBps": None, "counter_frac": None}
    if counter_bytes_per_cycle:
        out["counter_bytes"] = round(counter_bytes_per_cycle, 1)
        out["counter_GBps"] = round(counter_bytes_per_cycle / t / 1e9, 2)
        out["counter_frac"] = round(counter_bytes_per_cycle / t / 1e9 / HBM_PEAK_GBS, 4)
    return out


def bench_single(args, R, torch):
    """One design: the batched form (autotuned), its kernels' roofline, the
    plain single-instance form, and the CPU oracle; parity on the timed batch
    itself (two instances read back after every timed cycle has run, against
    the oracle run to the same cycle count, registers and digest)."""
    wl = WORKLOADS[args.workload]
    n_inst = args.instances or wl["instances"]
    cps = args.cycles_per_step or wl["cycles_per_step"]
    steps = args.steps if args.steps is not None else wl["steps"]
    repeats = max(1, args.repeats)
    mapping = {"auto": R.RTEAAL_MAP_AUTO, "resident": R.RTEAAL_MAP_RESIDENT,
               "sweep": R.RTEAAL_MAP_SWEEP, "layered": R.RTEAAL_MAP_LAYERED,
               "partitioned": R.RTEAAL_MAP_PARTITIONED}[args.mapping]

    t0 = time.perf_counter()
    d = rtlgen.generate(wl["cfg"], wl["seed"])
    seeds = rtlgen.instance_seeds(n_inst)
    print(f"[bench] design {d.summary()} generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    AB = algorithmic_bytes(d)
    ABE = algorithmic_bytes(d, eb)
    X, G = AB["x"], AB["g"]
    prof_cycles = args.profile_cycles or wl["profile_cycles"]
    total_cycles = (args.warmup + repeats * steps) * cps + prof_cycles
    check = sorted({0, n_inst - 1})
    oracle_thread = None
    if not args.no_parity:
        oracle_thread, oracle_res = start_oracle(d, seeds[check], total_cycles)
        print(f"[bench] oracle started: instances {check} x {total_cycles} cycles "
              f"(the timed batch's total)", file=sys.stderr, flush=True)

    ctx = R.rteaal_create(0)
    stream = ctx.stream
    did = R.rteaal_load_design(ctx, d)
    manual = (args.mapping != "auto" or args.block or args.ops_per_wave or args.unroll
              or args.tiles_per_wave or args.arity_split or args.tiles_per_pass or args.partitions
              or args.pass_branches)
    if not manual and not args.no_autotune:
        t0 = time.perf_counter()
        tuned, trate = R.rteaal_autotune(ctx, did, n_inst)
        print(f"[bench] autotune batched ({time.perf_counter() - t0:.1f}s): {tuned} "
              f"-> {trate:.4g} instance-cycles/s", file=sys.stderr, flush=True)
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping, block_threads=args.block,
                                ops_per_wave=args.ops_per_wave, unroll=args.unroll,
                                tiles_per_wave=args.tiles_per_wave, arity_split=args.arity_split,
                                tiles_per_pass=args.tiles_per_pass, partitions=args.partitions,
                                pass_branches=args.pass_branches)
    used_map, _ = R.rteaal_batch_info(ctx, bid)
    bopts = R.rteaal_batch_options(ctx, bid)
    for _ in range(args.warmup):
        R.rteaal_step(ctx, bid, cps)
    R.rteaal_sync(ctx)
    print(f"[bench] warmup done ({args.warmup} x {cps} cycles)", file=sys.stderr, flush=True)

    def run():
        for _ in range(steps):
            R.rteaal_step(ctx, bid, cps)

    runs = timed_runs(torch, stream, run, repeats)
    ms = float(np.median(runs))
    value = n_inst * cps * steps / (ms / 1e3)
    print(f"[bench] batched: {repeats} x ({steps} x {cps} cycles) x {n_inst} inst, median "
          f"{ms:.1f} ms -> {value:.4g} instance-cycles/s (runs {[round(r, 1) for r in runs]})",
          file=sys.stderr, flush=True)

    # Kernel timing with HIP events around each simulation-kernel launch.
    R.rteaal_kernel_timing(ctx, bid, True)
    R.rteaal_step(ctx, bid, prof_cycles)
    (launches, kms), (h_launches, h_kms) = R.rteaal_kernel_timing(ctx, bid, False)
    avg_ms = kms / max(launches, 1)
    # Parity: the timed batch itself, after all of its cycles.
    got_regs = R.unpack_limbs(np.concatenate([R.rteaal_read_state(ctx, bid, first=k, n=1)
                                              for k in check]), d.slot_width[d.reg_slot])
    got_dg = np.concatenate([R.rteaal_read_digest(ctx, bid, first=k, n=1) for k in check])
    assert R.rteaal_batch_info(ctx, bid)[1] == total_cycles
    lds = used_map == R.RTEAAL_MAP_RESIDENT and R.rteaal_batch_footprint(
        ctx, did, n_inst, mapping=R.RTEAAL_MAP_RESIDENT) // max(n_inst, 1) <= 160 * 1024
    if used_map == R.RTEAAL_MAP_SWEEP:
        # The common kernel moves the light operations' bytes; the heavy
        # kernel's are reported beside it.
        bound, peak = "hbm", HBM_PEAK_GBS
        per_launch = (AB["x_light"] * n_inst + AB["g_light"]) * prof_cycles / max(launches, 1)
    elif not lds:
        bound, peak = "hbm", HBM_PEAK_GBS
        per_launch = (X * n_inst + G) * prof_cycles / max(launches, 1)
    else:
        bound, peak = "lds", LDS_PEAK_GBS
        per_launch = X * n_inst * prof_cycles / max(launches, 1)
    achieved = per_launch / (avg_ms / 1e3) / 1e9
    traffic = (measured_traffic("k_sweep", args.workload, bopts)
               if used_map == R.RTEAAL_MAP_SWEEP else None)
    roofline = {"bound": bound, "achieved": round(achieved, 2), "peak": round(peak, 1),
                "unit": "GB/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": {R.RTEAAL_MAP_SWEEP: "k_sweep", R.RTEAAL_MAP_LAYERED: "k_layer"}.get(used_map, "k_resident"),
                "launches": launches, "avg_launch_ms": round(avg_ms, 5),
                "bytes_per_launch": round(per_launch, 1),
                "bytes_model": "word model: 1/8 B for a 1-bit value, 4 B up to 32 bits, 8 B per "
                               "64-bit limb; graph once per cycle",
                "algorithmic_bytes_per_instance_cycle": round(X, 1),
                "graph_bytes_per_cycle": round(G, 1)}
    counter_cycle = None
    if used_map == R.RTEAAL_MAP_SWEEP:
        # What the storage encoding moves for the same work (1- and 2-byte
        # classes for values of at most 16 bits): below the canonical word
        # model, so `achieved` can exceed what the HBM moves.
        enc = (ABE["x_light"] * n_inst + ABE["g_light"]) * prof_cycles / max(launches, 1)
        roofline["encoded_bytes_per_launch"] = round(enc, 1)
        roofline["encoded_GBps"] = round(enc / (avg_ms / 1e3) / 1e9, 2)
        roofline["encoded_frac"] = round(enc / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        if traffic:
            roofline["traffic_over_encoded"] = round(traffic / enc, 3)
    if traffic:
        roofline["traffic_over_algorithmic"] = round(traffic / per_launch, 3)
        roofline["traffic_GBps"] = round(traffic / (avg_ms / 1e3) / 1e9, 2)
        roofline["counter_frac"] = round(traffic / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    if h_launches:
        h_avg = h_kms / h_launches
        h_bytes = (AB["x_heavy"] * n_inst + AB["g_heavy"]) * prof_cycles / h_launches
        h_enc = (ABE["x_heavy"] * n_inst + ABE["g_heavy"]) * prof_cycles / h_launches
        h_traffic = measured_traffic("k_sweep_heavy", args.workload, bopts)
        roofline["heavy_kernel"] = {
            "kernel": "k_sweep_heavy", "launches": h_launches, "avg_launch_ms": round(h_avg, 5),
            "bytes_per_launch": round(h_bytes, 1), "encoded_bytes_per_launch": round(h_enc, 1),
            "achieved": round(h_bytes / (h_avg / 1e3) / 1e9, 2),
            "encoded_GBps": round(h_enc / (h_avg / 1e3) / 1e9, 2), "traffic": h_traffic,
            "counter_frac": (round(h_traffic / (h_avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                             if h_traffic else None),
            "share_of_kernel_time": round(h_kms / (h_kms + kms), 4)}
        if traffic and h_traffic:
            counter_cycle = (traffic * launches + h_traffic * h_launches) / prof_cycles
    roofline["whole_cycle"] = whole_cycle(AB, ABE, n_inst, ms / (steps * cps), counter_cycle)
    R.rteaal_free_batch(ctx, bid)

    plain = None
    if not args.no_plain:
        pc = args.plain_cycles or wl["plain_cycles"]
        plain_opts = {"mapping": R.RTEAAL_MAP_RESIDENT}
        if not args.no_autotune:
            plain_opts, prate = R.rteaal_autotune(ctx, did, 1)
            print(f"[bench] autotune plain: {plain_opts} -> {prate:.4g}", file=sys.stderr, flush=True)
        pb = R.rteaal_create_batch(ctx, did, seeds[:1], **plain_opts)
        R.rteaal_step(ctx, pb, min(pc, 200))
        R.rteaal_sync(ctx)
        pruns = timed_runs(torch, stream, lambda: R.rteaal_step(ctx, pb, pc), repeats)
        pms = float(np.median(pruns))
        # Roofline of the plain form's simulation kernel, timed as above.
        p_map, _ = R.rteaal_batch_info(ctx, pb)
        pbo = R.rteaal_batch_options(ctx, pb)
        ppc = min(pc, 50)
        R.rteaal_kernel_timing(ctx, pb, True)
        R.rteaal_step(ctx, pb, ppc)
        (pl, pkms), (phl, phkms) = R.rteaal_kernel_timing(ctx, pb, False)
        R.rteaal_free_batch(ctx, pb)
        # RESIDENT and PARTITIONED keep the state in LDS when it fits
        p_lds = (p_map in (R.RTEAAL_MAP_RESIDENT, R.RTEAAL_MAP_PARTITIONED)
                 and pbo["lds_state"] == 0)
        p_launches, p_ms = pl + phl, pkms + phkms
        p_bytes = (X + (0 if p_lds else G)) * ppc / max(p_launches, 1)
        p_avg = p_ms / max(p_launches, 1)
        p_peak = LDS_PEAK_GBS if p_lds else HBM_PEAK_GBS
        p_ach = p_bytes / (p_avg / 1e3) / 1e9 if p_avg > 0 else 0.0
        plain = {"value": pc / (pms / 1e3), "unit": "instance-cycles/s", "instances": 1,
                 "cycles": pc, "repeats": repeats, "opts": pbo,
                 "roofline": {"bound": "lds" if p_lds else "hbm",
                              "kernel": {R.RTEAAL_MAP_SWEEP: "k_sweep", R.RTEAAL_MAP_LAYERED: "k_layer",
                                         R.RTEAAL_MAP_PARTITIONED: "k_partitioned"}.get(
                                  p_map, "k_resident"),
                              "achieved": round(p_ach, 2), "peak": round(p_peak, 1), "unit": "GB/s",
                              "frac": round(p_ach / p_peak, 4), "launches": p_launches,
                              "avg_launch_ms": round(p_avg, 5), "bytes_per_launch": round(p_bytes, 1),
                              "note": "one instance: latency-bound (dependent gathers per layer)"}}
        print(f"[bench] plain: {pc} cycles, median {pms:.1f} ms -> {plain['value']:.4g}",
              file=sys.stderr, flush=True)
    R.rteaal_unload_design(ctx, did)
    R.rteaal_destroy(ctx)

    parity = None
    if oracle_thread is not None:
        print("[bench] waiting for the parity oracle", file=sys.stderr, flush=True)
        oracle_thread.join()
        regs_ok = bool(np.array_equal(got_regs, oracle_res["regs"]))
        dg_ok = bool(np.array_equal(got_dg, oracle_res["digest"]))
        parity = {"instances": check, "cycles": total_cycles, "registers_equal": regs_ok,
                  "digest_equal": dg_ok, "oracle_seconds": round(oracle_res["seconds"], 1),
                  "what": "the timed batch itself after its warm-up, timed, profiled cycles: "
                          "registers and the per-cycle register digest vs the oracle"}
        print(f"[bench] parity on the timed batch: {parity}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        per_ic = max(d.n_ops, 1) * 45e-9                 # rough oracle cost per instance-cycle
        k = min(host_threads(), len(seeds))
        cyc = max(1, int(min(2000, 12.0 * host_threads() / (k * per_ic))))
        cpu = cpu_baseline(d, seeds[:k], cyc, n_inst, wl["cycles"])
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)

    return {
        "metric": METRIC, "value": round(value, 2), "unit": "instance-cycles/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(ms / steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "ops": d.n_ops, "layers": d.n_layers,
                   "registers": d.n_regs, "inputs": d.n_inputs, "instances": n_inst,
                   "cycles_per_step": cps,
                   "timed": f"median of {repeats} timed runs of {steps} steps x {cps} cycles "
                            f"({[round(r, 1) for r in runs]} ms): a sample of the workload's "
                            f"{wl['cycles']} cycles (the rate is steady from the first cycles on)",
                   "mapping": {R.RTEAAL_MAP_SWEEP: "sweep", R.RTEAAL_MAP_LAYERED: "layered"}.get(
                       used_map, "resident"),
                   "opts": bopts,
                   "design_fingerprint": d.fingerprint()},
        "plain": plain,
        "batched_over_plain": round(value / plain["value"], 2) if plain else None,
        "paper_context": PAPER_CONTEXT,
        "parity_sample_ok": (parity["registers_equal"] and parity["digest_equal"]) if parity else None,
        "parity": parity,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def start_oracle_jobs(jobs, threads):
    """Oracle runs (design, seeds, cycles) side by side on `threads` host
    threads, one thread per run, largest first; each run's registers,
    digest and wall time."""
    import threading
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    res = [None] * len(jobs)

    def one(k):
        d, seeds, cyc = jobs[k]
        t0 = time.perf_counter()
        dg = {}
        regs, _, _ = oracle.run(d, seeds, cyc, n_threads=1, digests=dg)
        res[k] = (regs, dg["final"], time.perf_counter() - t0)

    order = sorted(range(len(jobs)), key=lambda k: -jobs[k][0].n_ops * len(jobs[k][1]) * jobs[k][2])

    def go():
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, order))

    th = threading.Thread(target=go, daemon=True)
    th.start()
    return th, res


def bench_multi(args, R, torch):
    """64 designs of uneven size, each with its own instance count, advanced
    together by rteaal_step_many.  Parity: the first instance of every
    design of the timed batches, after all of their cycles, registers and
    digest against the oracle; those oracle runs (one per design, side by
    side on the host threads) also give the CPU baseline."""
    t0 = time.perf_counter()
    plan = rtlgen.multidesign_batch(seed=2, n_designs=args.designs)
    designs = [rtlgen.generate(cfg, seed) for cfg, seed, _ in plan]
    n_inst = [n for _, _, n in plan]
    seeds_of = [rtlgen.instance_seeds(n, design_index=k) for k, n in enumerate(n_inst)]
    print(f"[bench] {len(designs)} designs ({sum(d.n_ops for d in designs)} ops, "
          f"{sum(n_inst)} instances) generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    cps = args.cycles_per_step or 100
    steps = args.steps if args.steps is not None else 5
    repeats = max(1, args.repeats)
    total_cycles = (args.warmup + repeats * steps) * cps
    threads = host_threads()
    oracle_thread = None
    if not args.no_parity:
        oracle_thread, ores = start_oracle_jobs(
            [(d, seeds_of[k][:1], total_cycles) for k, d in enumerate(designs)], threads)
    ctx = R.rteaal_create(0)
    dids = [R.rteaal_load_design(ctx, d) for d in designs]
    t0 = time.perf_counter()
    tuned_rate = None
    if not args.no_autotune:
        # The set's launch policy is tuned jointly, on the step time of all
        # designs together (each design alone would pick shapes that do not
        # share the device well).
        _, tuned_rate = R.rteaal_autotune_many(ctx, dids, n_inst)
    bids = [R.rteaal_create_batch(ctx, did, seeds_of[k]) for k, did in enumerate(dids)]
    print(f"[bench] batches created (joint autotune {time.perf_counter() - t0:.1f}s, "
          f"{tuned_rate})", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        R.rteaal_step_many(ctx, bids, [cps] * len(bids))
    R.rteaal_sync(ctx)

    def run():
        for _ in range(steps):
            R.rteaal_step_many(ctx, bids, [cps] * len(bids))

    runs = timed_runs(torch, ctx.stream, run, repeats)
    ms = float(np.median(runs))
    value = sum(n_inst) * cps * steps / (ms / 1e3)
    print(f"[bench] multi: median {ms:.1f} ms of {runs} -> {value:.4g} instance-cycles/s",
          file=sys.stderr, flush=True)
    got = [(R.unpack_limbs(R.rteaal_read_state(ctx, b, 0, 1), d.slot_width[d.reg_slot]),
            R.rteaal_read_digest(ctx, b, 0, 1)) for b, d in zip(bids, designs)]
    maps = [R.rteaal_batch_info(ctx, b)[0] for b in bids]
    opts = [R.rteaal_batch_options(ctx, b) for b in bids]
    for b in bids:
        R.rteaal_free_batch(ctx, b)
    R.rteaal_destroy(ctx)

    word = sum(n * algorithmic_bytes(d)["x"] + algorithmic_bytes(d)["g"] for d, n in zip(designs, n_inst))
    enc = sum(n * algorithmic_bytes(d, eb)["x"] + algorithmic_bytes(d, eb)["g"]
              for d, n in zip(designs, n_inst))
    t_cycle = ms / 1e3 / (steps * cps)
    roofline = {"bound": "hbm", "kernel": "every kernel of rteaal_step_many (whole step)",
                "achieved": round(word / t_cycle / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(word / t_cycle / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_cycle": round(word, 1),
                "bytes_model": "sum over designs of (instances x X + G), word model",
                "encoded_bytes_per_cycle": round(enc, 1),
                "encoded_GBps": round(enc / t_cycle / 1e9, 2),
                "encoded_frac": round(enc / t_cycle / 1e9 / HBM_PEAK_GBS, 4)}
    parity, cpu, ok = None, None, None
    if oracle_thread is not None:
        oracle_thread.join()
        bad = [k for k in range(len(designs))
               if not (np.array_equal(got[k][0], ores[k][0]) and np.array_equal(got[k][1], ores[k][1]))]
        ok = not bad
        parity = {"instances": "the first of every design", "cycles": total_cycles,
                  "mismatching_designs": bad,
                  "what": "the timed batches after all their cycles: registers and digest"}
        if not args.no_cpu_baseline:
            # Per instance-cycle oracle time of each design (its run had one
            # thread, beside the others), weighted by the design's instances.
            per_ic = [ores[k][2] / total_cycles for k in range(len(designs))]
            rate_core = sum(n_inst) / sum(n * t for n, t in zip(n_inst, per_ic))
            cpu = {"value": rate_core * threads, "unit": "instance-cycles/s", "cores": threads,
                   "kind": "oracle", "per_core": rate_core, "host_cpus_visible": os.cpu_count(),
                   "sample": f"the first instance of each of the {len(designs)} designs x "
                             f"{total_cycles} cycles (the parity runs), one thread each, "
                             f"{threads} at a time; rate weighted by each design's instances",
                   "extrapolated_full_workload": {
                       "cycles": 20_000,
                       "seconds": round(sum(n_inst) * 20_000 / (rate_core * threads), 1),
                       "label": f"extrapolation: per-core rate x {threads} cores"}}
    return {
        "metric": METRIC, "value": round(value, 2), "unit": "instance-cycles/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(ms / steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "multi-64", "designs": len(designs),
                   "ops": sum(d.n_ops for d in designs), "instances": sum(n_inst),
                   "cycles_per_step": cps,
                   "timed": f"median of {repeats} timed runs of {steps} steps x {cps} cycles "
                            f"({[round(r, 1) for r in runs]} ms) of the workload's 20,000",
                   "resident_batches": maps.count(R.RTEAAL_MAP_RESIDENT),
                   "sweep_batches": maps.count(R.RTEAAL_MAP_SWEEP),
                   "layered_batches": maps.count(R.RTEAAL_MAP_LAYERED)},
        "parity_sample_ok": ok, "parity": parity, "roofline": roofline, "cpu_baseline": cpu,
        "shapes": opts if args.verbose_shapes else None,
    }


def shuffled_graph(d, seed):
    """(n_slots, op_src_ptr, op_src, op_dst) of design d with its operations
    in a random order: the order a netlist may arrive in."""
    rng = np.random.default_rng(seed)
    o = rng.permutation(d.op_type.size)
    ptr = d.op_src_ptr.astype(np.int64)
    lens = (ptr[1:] - ptr[:-1])[o]
    new_ptr = np.zeros(o.size + 1, np.int64)
    np.cumsum(lens, out=new_ptr[1:])
    take = np.repeat(ptr[:-1][o] - new_ptr[:-1], lens) + np.arange(int(new_ptr[-1]))
    return (int(d.slot_width.size), new_ptr.astype(np.uint32), np.ascontiguousarray(d.op_src[take]),
            np.ascontiguousarray(d.op_dst[o]))


def levelization_ok(g, layer, order, lptr):
    """Validity and tightness of a layering (they characterize the layering
    by longest chains), plus the order and layer ranges."""
    n_slots, ptr, src, dst = g
    L = layer.astype(np.int64)
    prod = np.full(n_slots, -1, np.int64)
    prod[dst.astype(np.int64)] = np.arange(L.size)
    p = prod[src.astype(np.int64)]
    owner = np.repeat(np.arange(L.size), np.diff(ptr.astype(np.int64)))
    fed = p >= 0
    best = np.full(L.size, -1, np.int64)
    np.maximum.at(best, owner[fed], L[p[fed]])
    return bool((L[owner[fed]] > L[p[fed]]).all() and np.array_equal(L, best + 1)
                and (np.diff(L[order.astype(np.int64)]) >= 0).all()
                and np.array_equal(np.diff(lptr.astype(np.int64)),
                                   np.bincount(L, minlength=lptr.size - 1)))


def bench_levelize(args, R, torch):
    """rteaal_levelize on the large-5m graph with its operations shuffled; the
    oracle levelizer timed beside it on a bounded sample of the same recipe."""
    wl = WORKLOADS["large-5m"]
    t0 = time.perf_counter()
    d = rtlgen.generate(wl["cfg"], wl["seed"])
    g = shuffled_graph(d, 5)
    n, e = int(g[3].size), int(g[2].size)
    print(f"[bench] large-5m graph shuffled: {n} ops, {e} operand entries "
          f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
    ctx = R.rteaal_create(0)
    for _ in range(args.warmup):
        R.rteaal_levelize(ctx, *g)
    steps = args.steps if args.steps is not None else 5
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        layer, order, lptr = R.rteaal_levelize(ctx, *g)
        times.append(time.perf_counter() - t0)
    ms = float(np.median(times)) * 1e3
    ok = levelization_ok(g, layer, order, lptr)
    n_layers = int(lptr.size - 1)
    print(f"[bench] levelize: {ms:.1f} ms per call (median of {steps}), {n_layers} layers, "
          f"properties {'ok' if ok else 'FAILED'}", file=sys.stderr, flush=True)
    R.rteaal_destroy(ctx)
    # Compulsory bytes of one call: the graph read once, the three results written once.
    algo = 4.0 * ((n + 1) + e + n) + 4.0 * (2 * n + n_layers + 1)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sample = rtlgen.generate(rtlgen.generator.scaled(wl["cfg"], 0.5, "levelize-sample"), wl["seed"])
        gs = shuffled_graph(sample, 5)
        t0 = time.perf_counter()
        oracle.levelize(*gs)
        dt = time.perf_counter() - t0
        cpu = {"value": round(gs[3].size / dt, 1), "unit": "operations/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{gs[3].size} operations of the large-5m recipe (half scale), shuffled, "
                         f"{dt:.1f} s on one host thread"}
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)
    return {
        "metric": "operations levelized/s", "value": round(n / (ms / 1e3), 1),
        "unit": "operations/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "levelize-5m", "ops": n, "operand_entries": e, "layers": n_layers,
                   "timed": "whole rteaal_levelize call: uploads, kernels, read-back"},
        "parity_sample_ok": ok,
        "roofline": {"bound": "hbm", "achieved": round(algo / (ms / 1e3) / 1e9, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(algo / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "rteaal_levelize (all kernels of the call)",
                     "bytes_per_launch": round(algo, 1),
                     "note": "bound by the frontier steps' latency (one launch per layer, a "
                             "read-back per 8 layers) and the uploads; not by HBM bandwidth"},
        "cpu_baseline": cpu,
    }


def bench_blocks(args, R, torch):
    """Gather rate by block size, measured with the common kernel itself:
    four designs of 200,000 two-operand XORs (20 layers) whose every value
    has one width (8, 16, 32 or 64 bits), run batched with one 64-instance
    tile per wavefront, so that every gather and store instruction touches
    one block of 64 x (element bytes) = 64, 128, 256 or 512 bytes.  Per cycle
    an operation moves 3 blocks per tile (two gathers, one store)."""
    n_inst = args.instances or 4096
    tiles = (n_inst + 63) // 64
    cps = args.cycles_per_step or 20
    steps = args.steps if args.steps is not None else 5
    rows, ok = [], True
    for w, e in ((8, 1), (16, 2), (32, 4), (64, 8)):
        cfg = rtlgen.GenConfig(200_000, 20, 256, 16, ((w, w, 1.0),), f"blocks-{w}",
                               op_mix=((rtlgen.XOR, 2, 1.0),))
        d = rtlgen.generate(cfg, 5)
        seeds = rtlgen.instance_seeds(n_inst)
        ctx = R.rteaal_create(0)
        did = R.rteaal_load_design(ctx, d)
        bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP, ops_per_wave=8,
                                    unroll=1, tiles_per_wave=1)
        for _ in range(args.warmup):
            R.rteaal_step(ctx, bid, cps)

        def run():
            for _ in range(steps):
                R.rteaal_step(ctx, bid, cps)

        runs = timed_runs(torch, ctx.stream, run, max(1, args.repeats))
        t_cycle = float(np.median(runs)) / 1e3 / (steps * cps)
        cycles = (args.warmup + max(1, args.repeats) * steps) * cps
        got = R.unpack_limbs(R.rteaal_read_state(ctx, bid, 0, 1), d.slot_width[d.reg_slot])
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_destroy(ctx)
        import oracle
        ref, _, _ = oracle.run(d, seeds[:1], cycles)
        ok = ok and bool(np.array_equal(got, ref))
        blocks = 3.0 * d.n_ops * tiles
        rows.append({"bits": w, "block_bytes": 64 * e, "ms_per_cycle": round(t_cycle * 1e3, 4),
                     "G_blocks_per_s": round(blocks / t_cycle / 1e9, 2),
                     "useful_GBps": round(blocks * 64 * e / t_cycle / 1e9, 1)})
        print(f"[bench] blocks {64 * e} B: {rows[-1]}", file=sys.stderr, flush=True)
    return {
        "metric": "gather blocks/s by block size", "value": rows[0]["G_blocks_per_s"],
        "unit": "G blocks/s (64-byte blocks)", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": rows[0]["ms_per_cycle"] * cps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "block-probe", "instances": n_inst, "ops": 200_000, "layers": 20,
                   "shape": "SWEEP, 8 operations per wavefront, U = 1, one tile per wavefront",
                   "timed": "whole cycles (common kernel, sources, register commit, digest)"},
        "parity_sample_ok": ok, "rows": rows, "roofline": None, "cpu_baseline": None,
    }


def bench_waveform(args, R, torch):
    """Value-change capture on single-200k (every slot kept, 1,024 instances):
    the rate with 8,192 watched signals (the 4,096 registers and 4,096 operation
    outputs) against the same batch unwatched, the change log drained after
    every step of 5 cycles (random logic changes about a third of its values
    every cycle, so a step logs ~15M transitions)."""
    wl = WORKLOADS["single-200k"]
    d = rtlgen.generate(wl["cfg"], wl["seed"])
    n_inst = args.instances or wl["instances"]
    seeds = rtlgen.instance_seeds(n_inst)
    ctx = R.rteaal_create(0)
    did = R.rteaal_load_design(ctx, d, keep_all_slots=True)
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP, ops_per_wave=2,
                                unroll=2, tiles_per_wave=4)
    rng = np.random.default_rng(7)
    ops = np.sort(rng.choice(d.op_dst.astype(np.int64), 4096, replace=False))
    slots = np.concatenate([d.reg_slot.astype(np.int64), ops]).astype(np.uint32)
    cps = args.cycles_per_step or 5
    steps = args.steps if args.steps is not None else 20
    stream = ctx.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(watch):
        ms, recs, dropped = 0.0, 0, 0
        for k in range(args.warmup + steps):
            ev0.record(stream)
            R.rteaal_step(ctx, bid, cps)
            ev1.record(stream)
            ev1.synchronize()
            if k >= args.warmup:
                ms += ev0.elapsed_time(ev1)
            if watch:
                r, dr = R.rteaal_read_changes(ctx, bid)
                if k >= args.warmup:
                    recs += r.size
                    dropped += dr
        return ms, recs, dropped

    ms0, _, _ = timed(False)
    R.rteaal_watch(ctx, bid, slots, capacity=1 << 25)
    ms1, recs, dropped = timed(True)
    # parity sample: the last step's registers against the oracle
    total_cycles = (args.warmup + steps) * cps * 2
    got = R.unpack_limbs(R.rteaal_read_state(ctx, bid, 0, 2), d.slot_width[d.reg_slot])
    import oracle
    ref, _, _ = oracle.run(d, seeds[:2], total_cycles)
    ok = bool(np.array_equal(got, ref))
    R.rteaal_free_batch(ctx, bid)
    R.rteaal_unload_design(ctx, did)
    R.rteaal_destroy(ctx)
    cyc = steps * cps
    v0 = n_inst * cyc / (ms0 / 1e3)
    v1 = n_inst * cyc / (ms1 / 1e3)
    # Capture bytes per cycle: every watched value read and compared with its
    # 8-byte copy, and per transition the copy rewritten and a 48-byte record.
    w = d.slot_width[slots.astype(np.int64)].astype(np.int64)
    per_cycle = n_inst * float(eb(w).sum() + 8.0 * ((w + 63) // 64).sum()) + (recs + dropped) / cyc * 8 \
        + recs / cyc * 48
    extra_s = max(ms1 - ms0, 1e-9) / 1e3 / cyc
    print(f"[bench] waveform: unwatched {v0:.4g}, watched {v1:.4g} instance-cycles/s; "
          f"{(recs + dropped) / cyc:.0f} transitions per cycle, {dropped} dropped", file=sys.stderr,
          flush=True)
    return {
        "metric": METRIC, "value": round(v1, 2), "unit": "instance-cycles/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(ms1 / steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "waveform", "design": "single-200k (every slot kept)",
                   "instances": n_inst, "watched_signals": int(slots.size),
                   "cycles_per_step": cps},
        "unwatched_value": round(v0, 2), "capture_overhead": round(ms1 / ms0 - 1.0, 4),
        "transitions_per_cycle": round((recs + dropped) / cyc, 1), "dropped": dropped,
        "parity_sample_ok": ok,
        "roofline": {"bound": "hbm", "kernel": "k_capture (from the added time per cycle)",
                     "achieved": round(per_cycle / extra_s / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(per_cycle / extra_s / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": round(per_cycle, 1)},
        "cpu_baseline": None,
    }


def bench_muxchain(args, R, torch):
    """Mux-chain fusion on muxchain-2m (2,000,000 operations, 35 % MUX with
    80 % of them in priority chains, 4,096 instances): the batched rate of the
    design as drawn against the same design after rteaal_fuse_mux_chains and
    rteaal_levelize, each in its autotuned shape, with the fused batch's
    parity sample taken against the oracle run of the unfused design."""
    import oracle
    cfg = rtlgen.CFG_MUXCHAIN
    n_inst = args.instances or 4096
    cps = args.cycles_per_step or 20
    steps = args.steps if args.steps is not None else 10
    t0 = time.perf_counter()
    d = rtlgen.generate(cfg, 6)
    print(f"[bench] design {d.summary()} generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    seeds = rtlgen.instance_seeds(n_inst)
    ctx = R.rteaal_create(0)
    stream = ctx.stream
    t0 = time.perf_counter()
    f, cnt = R.rteaal_fuse_mux_chains(d)
    t_fuse = time.perf_counter() - t0
    t0 = time.perf_counter()
    lv = R.levelized_design(ctx, f)
    t_lev = time.perf_counter() - t0
    print(f"[bench] fused in {t_fuse:.2f}s: {cnt}; levelized in {t_lev:.2f}s: "
          f"{d.n_layers} -> {lv.n_layers} layers", file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for label, des in (("unfused", d), ("fused", lv)):
        did = R.rteaal_load_design(ctx, des)
        opts = {}
        if args.mapping != "auto":      # one given shape for both designs
            opts = {"mapping": {"resident": R.RTEAAL_MAP_RESIDENT, "sweep": R.RTEAAL_MAP_SWEEP,
                                "layered": R.RTEAAL_MAP_LAYERED}[args.mapping],
                    "block_threads": args.block, "ops_per_wave": args.ops_per_wave,
                    "unroll": args.unroll, "tiles_per_wave": args.tiles_per_wave}
        elif not args.no_autotune:
            opts, trate = R.rteaal_autotune(ctx, did, n_inst)
            print(f"[bench] autotune {label}: {opts} -> {trate:.4g}", file=sys.stderr, flush=True)
        bid = R.rteaal_create_batch(ctx, did, seeds, **opts)
        bopts = R.rteaal_batch_options(ctx, bid)
        # the fused batch is checked against the oracle of the design as drawn
        pick = [0, n_inst // 2, n_inst - 1]
        R.rteaal_step(ctx, bid, 3)
        got = np.concatenate([R.rteaal_read_state(ctx, bid, first=k, n=1) for k in pick])
        ref, _, _ = oracle.run(d, seeds[pick], 3, n_threads=3)
        ok = bool(np.array_equal(R.unpack_limbs(got, d.slot_width[d.reg_slot]), ref))
        print(f"[bench] {label} parity sample vs oracle of the unfused design: {ok}",
              file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            R.rteaal_step(ctx, bid, cps)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            R.rteaal_step(ctx, bid, cps)
        ev1.record(stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1)
        rate = n_inst * cps * steps / (ms / 1e3)
        pc = min(cps, 50)
        R.rteaal_kernel_timing(ctx, bid, True)
        R.rteaal_step(ctx, bid, pc)
        (lau, kms), (hl, hkms) = R.rteaal_kernel_timing(ctx, bid, False)
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)
        AB = algorithmic_bytes(des)
        per_cycle = AB["x"] * n_inst + AB["g"]
        res[label] = {"value": rate, "ms": ms, "ok": ok, "opts": bopts, "layers": des.n_layers,
                      "ops": des.n_ops, "x": AB["x"], "g": AB["g"],
                      "kernel_ms_per_cycle": (kms + hkms) / pc, "heavy_share": hkms / max(kms + hkms, 1e-9),
                      "light": (lau, kms, AB["x_light"] * n_inst + AB["g_light"]),
                      "heavy": (hl, hkms, AB["x_heavy"] * n_inst + AB["g_heavy"]),
                      "pc": pc, "per_cycle": per_cycle}
        print(f"[bench] {label}: {steps} x {cps} cycles x {n_inst} inst in {ms:.1f} ms -> "
              f"{rate:.4g} instance-cycles/s; {AB['x'] / 1e6:.2f} MB per instance-cycle",
              file=sys.stderr, flush=True)
    R.rteaal_destroy(ctx)
    fz, un = res["fused"], res["unfused"]

    def kern(name, rec, pc):
        n, kms, b = rec
        if not n:
            return None
        avg = kms / n
        per = b * pc / n
        return {"kernel": name, "launches": n, "avg_launch_ms": round(avg, 5),
                "bytes_per_launch": round(per, 1), "achieved": round(per / (avg / 1e3) / 1e9, 2)}

    light = kern("k_sweep", fz["light"], fz["pc"])
    heavy = kern("k_sweep_heavy", fz["heavy"], fz["pc"])
    dom = heavy if fz["heavy_share"] > 0.5 else light
    roof = dict(dom, bound="hbm", peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(dom["achieved"] / HBM_PEAK_GBS, 4), traffic=None,
                other_kernel=light if dom is heavy else heavy,
                algorithmic_bytes_per_instance_cycle=round(fz["x"], 1))
    return {
        "metric": METRIC, "value": round(fz["value"], 2), "unit": "instance-cycles/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(fz["ms"] / steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "muxchain-2m", "ops": d.n_ops, "layers": d.n_layers,
                   "registers": d.n_regs, "inputs": d.n_inputs, "instances": n_inst,
                   "cycles_per_step": cps, "fused_opts": fz["opts"], "unfused_opts": un["opts"],
                   "design_fingerprint": d.fingerprint()},
        "fusion": dict(cnt, seconds=round(t_fuse, 3), levelize_seconds=round(t_lev, 3),
                       layers_before=d.n_layers, layers_after=lv.n_layers,
                       bytes_per_instance_cycle_before=round(un["x"], 1),
                       bytes_per_instance_cycle_after=round(fz["x"], 1)),
        "unfused_value": round(un["value"], 2),
        "fused_over_unfused": round(fz["value"] / un["value"], 3),
        "kernel_ms_per_cycle": {"unfused": round(un["kernel_ms_per_cycle"], 4),
                                "fused": round(fz["kernel_ms_per_cycle"], 4)},
        "parity_sample_ok": fz["ok"] and un["ok"],
        "roofline": roof,
        "cpu_baseline": None,
    }


def bench_serving(args, R, torch):
    """Poisson stream of jobs over a pool of designs with continuous batching.
    Checks: finished jobs rerun alone equal their results in the mix; the
    first instance of finished jobs small enough for the oracle equals it."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_2601_18140_amd import serving
    import oracle
    t0 = time.perf_counter()
    pool_cfg = rtlgen.serving_pool(seed=4, n_designs=args.designs,
                                   ops_hi=args.serving_ops_hi)
    pool = [rtlgen.generate(cfg, seed) for cfg, seed in pool_cfg]
    print(f"[bench] pool of {len(pool)} designs generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    log = lambda m: print(f"[serve] {m}", file=sys.stderr, flush=True)  # noqa: E731
    quiet = lambda m: None if m.startswith(("admit", "done")) else log(m)  # noqa: E731
    ctx = R.rteaal_create(0)
    budget = int(args.serving_budget_gb * (1 << 30))
    rate = args.serving_rate
    calib = None
    if args.serving_calibrate:
        # Saturated throughput: a set of jobs (its own seed) all arriving at
        # once; the timed stream then arrives at --serving-load of that rate.
        cspec = rtlgen.serving_jobs(seed=40, n_jobs=args.serving_calibrate, pool_size=len(pool),
                                    inst_hi=args.serving_inst_hi, cyc_hi=args.serving_cycles_hi)
        cjobs = [serving.Job(job_id=(1 << 20) + k, design=d, n_inst=n, n_cycles=c)
                 for k, (d, n, c) in enumerate(cspec)]
        csrv = serving.Server(ctx, pool, budget_bytes=budget, log=quiet)
        cstats = csrv.run(cjobs, np.zeros(len(cjobs)))
        csrv.close()
        sat = cstats["jobs"] / cstats["wall_s"]
        rate = args.serving_load * sat
        calib = {"jobs": cstats["jobs"], "wall_s": round(cstats["wall_s"], 2),
                 "saturated_jobs_per_s": round(sat, 4), "load": args.serving_load,
                 "rate_per_s": round(rate, 4),
                 "instance_cycles_per_s": round(cstats["instance_cycles_per_s"], 1)}
        print(f"[bench] serving calibration: {calib}", file=sys.stderr, flush=True)
    n_jobs = args.serving_jobs
    spec = rtlgen.serving_jobs(seed=4, n_jobs=n_jobs, pool_size=len(pool),
                               inst_hi=args.serving_inst_hi, cyc_hi=args.serving_cycles_hi)
    jobs = [serving.Job(job_id=k, design=d, n_inst=n, n_cycles=c) for k, (d, n, c) in enumerate(spec)]
    arrivals = serving.poisson_arrivals(rate, n_jobs, seed=4)
    srv = serving.Server(ctx, pool, budget_bytes=budget, log=quiet)
    stats = srv.run(jobs, arrivals, duration=args.serving_seconds)
    srv.close()
    stats["gpu_busy_s"] = round(srv.gpu_busy_s, 2)
    # Each checked job, re-run alone: identical registers.
    same = True
    check = [j for j in srv.finished][: args.serving_verify]
    for j in check:
        d = pool[j.design]
        did = R.rteaal_load_design(ctx, d)
        b = R.rteaal_create_batch(ctx, did, j.seeds)
        R.rteaal_step(ctx, b, j.n_cycles)
        alone = R.rteaal_read_state(ctx, b)
        R.rteaal_free_batch(ctx, b)
        R.rteaal_unload_design(ctx, did)
        same = same and bool(np.array_equal(alone, j.regs))
    R.rteaal_destroy(ctx)
    # The oracle on the first instance of finished jobs it can afford (at
    # most 2e9 operation evaluations each), side by side.
    small = [j for j in srv.finished if pool[j.design].n_ops * j.n_cycles <= 2e9][:16]

    def ref(j):
        d = pool[j.design]
        r, _, _ = oracle.run(d, j.seeds[:1], j.n_cycles, n_threads=1)
        return np.array_equal(R.unpack_limbs(j.regs[:1], d.slot_width[d.reg_slot]), r)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(host_threads()) as ex:
        oracle_ok = all(ex.map(ref, small))
    t_or = time.perf_counter() - t0
    # Bytes the finished jobs' cycles needed (word model), over the window.
    ab = {}
    word = 0.0
    for j in srv.finished:
        if j.design not in ab:
            ab[j.design] = algorithmic_bytes(pool[j.design])
        word += j.n_cycles * (j.n_inst * ab[j.design]["x"] + ab[j.design]["g"])
    wall = stats["wall_s"]
    roofline = {"bound": "hbm", "kernel": "every kernel of the serving loop's steps (whole window)",
                "achieved": round(word / wall / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(word / wall / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes": round(word, 1),
                "note": "over the whole window, idle time between arrivals included; per second "
                        "of steps (gpu_busy_s): " + f"{word / max(srv.gpu_busy_s, 1e-9) / 1e9:.1f} GB/s"}
    cpu = None
    if not args.no_cpu_baseline:
        # Oracle time per instance-cycle of each pool design (one instance,
        # 300 cycles, one thread each, side by side), weighted by the
        # finished jobs' instance-cycles.
        used = sorted({j.design for j in srv.finished})

        def per_ic(k):
            t1 = time.perf_counter()
            oracle.run(pool[k], np.array([1], np.uint64), 300, n_threads=1)
            return (time.perf_counter() - t1) / 300
        t0 = time.perf_counter()
        with ThreadPoolExecutor(host_threads()) as ex:
            t_ic = dict(zip(used, ex.map(per_ic, used)))
        w = sum(j.n_inst * j.n_cycles for j in srv.finished)
        t_all = sum(j.n_inst * j.n_cycles * t_ic[j.design] for j in srv.finished)
        rate_core = w / t_all if t_all else 0.0
        cpu = {"value": rate_core * host_threads(), "unit": "instance-cycles/s",
               "cores": host_threads(), "kind": "oracle", "per_core": rate_core,
               "host_cpus_visible": os.cpu_count(),
               "sample": f"one instance x 300 cycles of each of the {len(used)} designs the "
                         f"finished jobs used, one thread each, {host_threads()} at a time "
                         f"({time.perf_counter() - t0:.1f} s); rate weighted by the jobs' "
                         "instance-cycles",
               "extrapolated_full_workload": {
                   "seconds": round(w / (rate_core * host_threads()), 1) if rate_core else None,
                   "label": f"extrapolation: the finished jobs' instance-cycles at the per-core "
                            f"rate x {host_threads()} cores"}}
    return {
        "metric": METRIC, "value": round(stats["instance_cycles_per_s"], 2),
        "unit": "instance-cycles/s", "n_gpus": 1, "steps": stats["jobs"], "warmup": 0,
        "ms_per_step": round(1e3 * stats["wall_s"] / max(stats["jobs"], 1), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "serving", "designs": len(pool), "jobs_offered": n_jobs,
                   "arrival_rate_per_s": round(rate, 4), "admission_seconds": args.serving_seconds,
                   "budget_gb": args.serving_budget_gb, "calibration": calib},
        "serving": stats, "alone_equals_mix": same, "verified_jobs": len(check),
        "parity_sample_ok": same and oracle_ok,
        "parity": {"alone_equals_mix_jobs": len(check), "oracle_jobs": len(small),
                   "oracle_equal": oracle_ok, "oracle_seconds": round(t_or, 1)},
        "roofline": roofline, "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large-5m",
                    choices=sorted(WORKLOADS) + ["multi-64", "serving", "levelize-5m", "waveform",
                                                 "muxchain-2m", "block-probe"])
    ap.add_argument("--designs", type=int, default=None)
    ap.add_argument("--serving-jobs", type=int, default=2000)
    ap.add_argument("--serving-rate", type=float, default=4.0, help="job arrivals per second")
    ap.add_argument("--serving-seconds", type=float, default=600.0,
                    help="admission window (the workload's 10 minutes)")
    ap.add_argument("--serving-budget-gb", type=float, default=200.0)
    ap.add_argument("--serving-ops-hi", type=int, default=1_000_000)
    ap.add_argument("--serving-inst-hi", type=int, default=512)
    ap.add_argument("--serving-cycles-hi", type=int, default=50_000)
    ap.add_argument("--serving-verify", type=int, default=8)
    ap.add_argument("--serving-calibrate", type=int, default=0, metavar="JOBS",
                    help="first measure the saturated job rate on JOBS jobs arriving at once, "
                         "then offer the timed stream at --serving-load times it")
    ap.add_argument("--serving-load", type=float, default=0.7,
                    help="offered load as a fraction of the calibrated saturated job rate")
    ap.add_argument("--cycles-per-step", type=int, default=None)
    ap.add_argument("--instances", type=int, default=None)
    ap.add_argument("--mapping", default="auto",
                    choices=["auto", "resident", "sweep", "layered", "partitioned"])
    ap.add_argument("--partitions", type=int, default=0, help="PARTITIONED: register partitions")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--ops-per-wave", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--tiles-per-wave", type=int, default=0)
    ap.add_argument("--arity-split", type=int, default=0, help="SWEEP: 0 auto, 1 never, 2 always")
    ap.add_argument("--tiles-per-pass", type=int, default=0, help="SWEEP: 0 all tiles per pass")
    ap.add_argument("--pass-branches", type=int, default=0,
                    help="SWEEP: 1 = tile passes as parallel graph branches")
    ap.add_argument("--plain-cycles", type=int, default=None)
    ap.add_argument("--profile-cycles", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the oracle check of the timed batch")
    ap.add_argument("--verbose-shapes", action="store_true",
                    help="multi-64: list every batch's launch shape in the JSON line")
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed runs of --steps steps each; the median is reported")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default shapes instead of autotuned ones")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (counter scale)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": n, "copies": 3}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: every workload here is a single-GPU "
              "configuration (instances shard across GPUs with no exchange); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_18140_amd import rteaal as R

    if args.workload == "multi-64":
        args.designs = args.designs or 64
        result = bench_multi(args, R, torch)
    elif args.workload == "serving":
        args.designs = args.designs or 32
        result = bench_serving(args, R, torch)
    elif args.workload == "levelize-5m":
        result = bench_levelize(args, R, torch)
    elif args.workload == "waveform":
        result = bench_waveform(args, R, torch)
    elif args.workload == "muxchain-2m":
        result = bench_muxchain(args, R, torch)
    elif args.workload == "block-probe":
        result = bench_blocks(args, R, torch)
    else:
        result = bench_single(args, R, torch)
    print(json.dumps(result), flush=True)
    if result.get("parity_sample_ok") is False:
        print("[bench] PARITY MISMATCH against the oracle (see the parity field)", file=sys.stderr,
              flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
