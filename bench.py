#!/usr/bin/env python3
"""Benchmark of the per-cycle layer cascade on one MI355X.

Metric: instance-cycles/s (instances x clock cycles simulated per second),
for the batched form (many stimulus instances of one design) and the plain
form (one instance), plus the achieved fraction of the HBM / LDS roofline of
the simulation kernel and the CPU oracle's rate on a bounded sample.

A step is one rteaal_step of `cycles_per_step` cycles over the whole batch;
inputs (design, state, seeds) are resident on the device before timing.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import rtlgen  # noqa: E402

METRIC = "instance-cycles/s (batched vs plain) + % HBM/LDS roofline, bit-exact"
HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E
LDS_PEAK_GBS = 256 * 128 * 2.4        # 256 CUs x 128 B/clk x 2.4 GHz = 78,643 GB/s

# Workloads: design recipe, batched instance count, default cycles per step.
WORKLOADS = {
    "single-200k": dict(cfg=rtlgen.CFG1, seed=1, instances=1024, cycles_per_step=10_000,
                        total_cycles=100_000),
    "plain-2k": dict(cfg=rtlgen.CFG0, seed=0, instances=1, cycles_per_step=10_000,
                     total_cycles=10_000),
    "large-5m": dict(cfg=rtlgen.CFG3, seed=3, instances=4096, cycles_per_step=20,
                     total_cycles=10_000),
}


def wb(w):
    """Bytes one value of width w takes in the canonical word model (1-bit values bit-sliced)."""
    w = np.asarray(w, dtype=np.int64)
    return np.where(w == 1, 0.125, np.where(w <= 32, 4.0, np.where(w <= 64, 8.0, 8.0 * ((w + 63) // 64))))


def algorithmic_bytes(d):
    """Per instance-cycle state bytes X (operand gathers + result stores, register
    commit, input writes) and per-cycle graph bytes G of the packed graph tensor."""
    W = d.slot_width.astype(np.int64)
    x_ops = wb(W[d.op_src]).sum() + wb(W[d.op_dst]).sum()
    x_regs = wb(W[d.reg_next]).sum() + wb(W[d.reg_slot]).sum()
    x_in = wb(W[d.input_slot]).sum()
    g_bits = 0
    ar = d.op_arity()
    for i in range(d.n_layers):
        a, b = int(d.layer_ptr[i]), int(d.layer_ptr[i + 1])
        if a == b:
            continue
        sl = slice(int(d.op_src_ptr[a]), int(d.op_src_ptr[b]))
        cb = max(int(d.op_dst[a:b].max()), int(d.op_src[sl].max())).bit_length()
        imm = np.count_nonzero(np.isin(d.op_type[a:b], (rtlgen.SHL, rtlgen.SHR, rtlgen.EXTRACT)))
        g_bits += int((1 + ar[a:b]).sum()) * cb + 9 * (b - a) + 8 * imm
    return float(x_ops + x_regs + x_in), g_bits / 8.0


def cpu_baseline(d, seeds, cycles):
    import oracle
    threads = min(16, os.cpu_count() or 1, len(seeds))
    t0 = time.perf_counter()
    oracle.run(d, seeds, cycles, n_threads=threads)
    dt = time.perf_counter() - t0
    return {"value": len(seeds) * cycles / dt, "unit": "instance-cycles/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(seeds)} instances x {cycles} cycles of the same design, "
                      f"{dt:.1f} s wall on {threads} host threads"}


def parity_sample(R, ctx, did, d, seeds, mapping, cycles=3):
    """Fresh batch, a few cycles, two instances against the oracle."""
    import oracle
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping)
    R.rteaal_step(ctx, bid, cycles)
    pick = [0, len(seeds) - 1]
    got = R.unpack_limbs(R.rteaal_read_state(ctx, bid), d.slot_width[d.reg_slot])[pick]
    R.rteaal_free_batch(ctx, bid)
    ref, _, _ = oracle.run(d, np.asarray(seeds)[pick], cycles)
    return bool(np.array_equal(got, ref))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single-200k", choices=sorted(WORKLOADS))
    ap.add_argument("--cycles-per-step", type=int, default=None)
    ap.add_argument("--instances", type=int, default=None)
    ap.add_argument("--mapping", default="auto", choices=["auto", "resident", "sweep"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--ops-per-wave", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--plain-cycles", type=int, default=None)
    ap.add_argument("--profile-cycles", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    wl = WORKLOADS[args.workload]
    n_inst = args.instances or wl["instances"]
    cps = args.cycles_per_step or wl["cycles_per_step"]
    steps = args.steps if args.steps is not None else max(1, wl["total_cycles"] // cps)
    mapping = {"auto": R.RTEAAL_MAP_AUTO, "resident": R.RTEAAL_MAP_RESIDENT,
               "sweep": R.RTEAAL_MAP_SWEEP}[args.mapping]

    t0 = time.perf_counter()
    d = rtlgen.generate(wl["cfg"], wl["seed"])
    seeds = rtlgen.instance_seeds(n_inst)
    print(f"[bench] design {d.summary()} generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    X, G = algorithmic_bytes(d)

    ctx = R.rteaal_create(0)
    stream = ctx.stream
    did = R.rteaal_load_design(ctx, d)

    ok = parity_sample(R, ctx, did, d, seeds, mapping)
    print(f"[bench] parity sample vs oracle: {ok}", file=sys.stderr, flush=True)

    manual = args.mapping != "auto" or args.block or args.ops_per_wave or args.unroll
    tuned = None
    if not manual and not args.no_autotune:
        t0 = time.perf_counter()
        tuned, trate = R.rteaal_autotune(ctx, did, n_inst)
        print(f"[bench] autotune batched ({time.perf_counter() - t0:.1f}s): {tuned} "
              f"-> {trate:.4g} instance-cycles/s", file=sys.stderr, flush=True)
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping, block_threads=args.block,
                                ops_per_wave=args.ops_per_wave, unroll=args.unroll)
    used_map, _ = R.rteaal_batch_info(ctx, bid)
    for _ in range(args.warmup):
        R.rteaal_step(ctx, bid, cps)
    R.rteaal_sync(ctx)
    print(f"[bench] warmup done ({args.warmup} x {cps} cycles)", file=sys.stderr, flush=True)

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        R.rteaal_step(ctx, bid, cps)
    ev1.record(stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    value = n_inst * cps * steps / (ms / 1e3)
    print(f"[bench] batched: {steps} x {cps} cycles x {n_inst} inst in {ms:.1f} ms "
          f"-> {value:.4g} instance-cycles/s", file=sys.stderr, flush=True)

    # Kernel timing with HIP events around each simulation-kernel launch.
    prof_cycles = args.profile_cycles or (min(cps, 1024) if used_map == R.RTEAAL_MAP_RESIDENT else min(cps, 50))
    R.rteaal_kernel_timing(ctx, bid, True)
    R.rteaal_step(ctx, bid, prof_cycles)
    launches, kms = R.rteaal_kernel_timing(ctx, bid, False)
    avg_ms = kms / max(launches, 1)
    state_bytes = X * n_inst * prof_cycles
    lds = used_map == R.RTEAAL_MAP_RESIDENT and R.rteaal_batch_footprint(
        ctx, did, n_inst, mapping=R.RTEAAL_MAP_RESIDENT) // max(n_inst, 1) <= 160 * 1024
    if used_map == R.RTEAAL_MAP_SWEEP or not lds:
        bound, peak = "hbm", HBM_PEAK_GBS
        per_launch = (state_bytes + G * prof_cycles) / max(launches, 1)
    else:
        bound, peak = "lds", LDS_PEAK_GBS
        per_launch = state_bytes / max(launches, 1)
    achieved = per_launch / (avg_ms / 1e3) / 1e9
    roofline = {"bound": bound, "achieved": round(achieved, 2), "peak": round(peak, 1),
                "unit": "GB/s", "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": "k_sweep" if used_map == R.RTEAAL_MAP_SWEEP else "k_resident",
                "launches": launches, "avg_launch_ms": round(avg_ms, 5),
                "algorithmic_bytes_per_instance_cycle": round(X, 1),
                "graph_bytes_per_cycle": round(G, 1)}
    R.rteaal_free_batch(ctx, bid)

    plain = None
    if not args.no_plain:
        pc = args.plain_cycles or min(cps, 2000)
        plain_opts = {"mapping": R.RTEAAL_MAP_RESIDENT}
        if not args.no_autotune:
            plain_opts, prate = R.rteaal_autotune(ctx, did, 1)
            print(f"[bench] autotune plain: {plain_opts} -> {prate:.4g}", file=sys.stderr, flush=True)
        pb = R.rteaal_create_batch(ctx, did, seeds[:1], **plain_opts)
        R.rteaal_step(ctx, pb, min(pc, 200))
        R.rteaal_sync(ctx)
        ev0.record(stream)
        R.rteaal_step(ctx, pb, pc)
        ev1.record(stream)
        ev1.synchronize()
        pms = ev0.elapsed_time(ev1)
        R.rteaal_free_batch(ctx, pb)
        plain = {"value": pc / (pms / 1e3), "unit": "instance-cycles/s", "instances": 1,
                 "cycles": pc, "opts": plain_opts}
        print(f"[bench] plain: {pc} cycles in {pms:.1f} ms -> {plain['value']:.4g}",
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        per_ic = max(d.n_ops, 1) * 45e-9                 # rough oracle cost per instance-cycle
        k = min(16, len(seeds))
        cyc = max(1, int(min(2000, 12.0 * min(16, os.cpu_count() or 1) / (k * per_ic))))
        cpu = cpu_baseline(d, seeds[:k], cyc)
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)

    R.rteaal_unload_design(ctx, did)
    R.rteaal_destroy(ctx)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "instance-cycles/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(ms / steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "ops": d.n_ops, "layers": d.n_layers,
                   "registers": d.n_regs, "inputs": d.n_inputs, "instances": n_inst,
                   "cycles_per_step": cps,
                   "mapping": "sweep" if used_map == R.RTEAAL_MAP_SWEEP else "resident",
                   "opts": tuned,
                   "design_fingerprint": d.fingerprint()},
        "plain": plain,
        "batched_over_plain": round(value / plain["value"], 2) if plain else None,
        "parity_sample_ok": ok,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
