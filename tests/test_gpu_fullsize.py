"""Parity at the full workload sizes (GPU), on sampled instances.

The oracle cannot afford every instance of the large batches, so each
comparison picks fixed instances (first, last, and a seeded draw) and runs
the full-size batch on the GPU in the launch shapes the bench measures.
Registers and the per-cycle register digest (which folds the register
vector of every cycle) are compared.  Integer arithmetic: tolerance 0.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from tests.gpu_util import assert_same, gpu_ctx

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    R.rteaal_destroy(c)


def read_regs(ctx, bid, d, inst):
    rows = [R.rteaal_read_state(ctx, bid, first=int(k), n=1) for k in inst]
    return R.unpack_limbs(np.concatenate(rows), d.slot_width[d.reg_slot])


def read_digest(ctx, bid, inst):
    return np.concatenate([R.rteaal_read_digest(ctx, bid, first=int(k), n=1) for k in inst])


def oracle_with_digest(d, seeds, cycles, threads=16):
    dg = {}
    regs, _, _ = oracle.run(d, seeds, cycles, n_threads=threads, digests=dg)
    return regs, dg["final"]


def oracle_jobs(jobs, workers=8):
    """oracle_with_digest over (design, seeds, cycles, threads) jobs, run
    side by side (the oracle's C code releases the interpreter lock)."""
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda j: oracle_with_digest(*j), jobs))


def test_large_5m_batched_sampled(ctx):
    """5,000,000 ops, 120 layers, 4,096 instances: 32 sampled instances
    ({0, 4095} plus 30 drawn with seed 11) after 3 cycles, in the two shapes
    the bench's autotuner picks between (8 and 2 operations per wavefront
    with 8 tiles, 4 and 8 with 16), an older shape with 2 operations per lane, and the default
    shape; then the plain single-instance form, LAYERED (as the bench
    measures it) and the default."""
    w = rtlgen.WORKLOADS["large-5m"]
    d = rtlgen.generate(w["cfg"], w["seed"])
    n = w["instances"]
    seeds = rtlgen.instance_seeds(n)
    rng = np.random.default_rng(11)
    pick = sorted({0, n - 1} | set(rng.choice(np.arange(1, n - 1), 30, replace=False).tolist()))
    cyc = 3
    ref, ref_dg = oracle_with_digest(d, seeds[pick], cyc)
    did = R.rteaal_load_design(ctx, d)
    try:
        for shape in ({"ops_per_wave": 8, "unroll": 1, "tiles_per_wave": 8},
                      {"ops_per_wave": 2, "unroll": 1, "tiles_per_wave": 8},
                      {"ops_per_wave": 4, "unroll": 1, "tiles_per_wave": 16},
                      {"ops_per_wave": 8, "unroll": 1, "tiles_per_wave": 16},
                      {"ops_per_wave": 2, "unroll": 2, "tiles_per_wave": 4}, {}):
            note(f"large-5m batched {n} x {cyc} cycles, shape {shape}")
            bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP, **shape)
            try:
                R.rteaal_step(ctx, bid, 1)
                R.rteaal_step(ctx, bid, cyc - 1)
                got = read_regs(ctx, bid, d, pick)
                got_dg = read_digest(ctx, bid, pick)
            finally:
                R.rteaal_free_batch(ctx, bid)
            assert_same(got, ref, f"large-5m sample, shape {shape}")
            assert_same(got_dg, ref_dg, f"large-5m sample digest, shape {shape}")
        for opts in ({"mapping": R.RTEAAL_MAP_LAYERED, "block_threads": 64, "unroll": 1}, {}):
            note(f"large-5m plain 1 instance x 3 cycles, {opts}")
            bid = R.rteaal_create_batch(ctx, did, seeds[:1], **opts)
            try:
                R.rteaal_step(ctx, bid, cyc)
                got = read_regs(ctx, bid, d, [0])
                got_dg = read_digest(ctx, bid, [0])
            finally:
                R.rteaal_free_batch(ctx, bid)
            assert_same(got, ref[:1], f"large-5m plain {opts}")
            assert_same(got_dg, ref_dg[:1], f"large-5m plain digest {opts}")
    finally:
        R.rteaal_unload_design(ctx, did)


def test_large_5m_benched_shape_200_cycles(ctx):
    """large-5m in the shape the bench's autotuner picks (8 operations per
    wavefront, 16 tiles, unroll 1): 16 sampled instances ({0, 4095} plus 14
    drawn with seed 11) after 200 cycles, registers and digest, so every
    cycle's register vector of those instances is compared."""
    w = rtlgen.WORKLOADS["large-5m"]
    d = rtlgen.generate(w["cfg"], w["seed"])
    n = w["instances"]
    seeds = rtlgen.instance_seeds(n)
    rng = np.random.default_rng(11)
    pick = sorted({0, n - 1} | set(rng.choice(np.arange(1, n - 1), 14, replace=False).tolist()))
    cyc = 200
    with ThreadPoolExecutor(1) as ex:
        fut = ex.submit(oracle_with_digest, d, seeds[pick], cyc)
        did = R.rteaal_load_design(ctx, d)
        try:
            note(f"large-5m batched {n} x {cyc} cycles, benched shape")
            bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP,
                                        ops_per_wave=8, unroll=1, tiles_per_wave=16)
            try:
                for k in (20, 80, 100):
                    R.rteaal_step(ctx, bid, k)
                got = read_regs(ctx, bid, d, pick)
                got_dg = read_digest(ctx, bid, pick)
            finally:
                R.rteaal_free_batch(ctx, bid)
        finally:
            R.rteaal_unload_design(ctx, did)
        note("large-5m: waiting for the oracle")
        ref, ref_dg = fut.result()
    assert_same(got, ref, "large-5m 200 cycles")
    assert_same(got_dg, ref_dg, "large-5m 200 cycles digest")


def test_single_200k_2000_cycles(ctx):
    """single-200k, 1,024 instances in the bench's batched shape (SWEEP, 2
    operations per wavefront, unroll 1, 8 tiles) for 2,000 cycles: 64
    sampled instances ({0, 1, 2, 511, 512, 1022, 1023} plus 57 drawn with
    seed 7); then the plain form (LAYERED, one instance) for the same
    cycles."""
    w = rtlgen.WORKLOADS["single-200k"]
    d = rtlgen.generate(w["cfg"], w["seed"])
    n = w["instances"]
    seeds = rtlgen.instance_seeds(n)
    fixed = {0, 1, 2, 511, 512, 1022, 1023}
    rng = np.random.default_rng(7)
    rest = sorted(set(range(n)) - fixed)
    pick = sorted(fixed | set(rng.choice(rest, 57, replace=False).tolist()))
    cyc = 2000
    with ThreadPoolExecutor(1) as ex:
        fut = ex.submit(oracle_with_digest, d, seeds[pick], cyc)
        did = R.rteaal_load_design(ctx, d)
        try:
            note(f"single-200k batched {n} x {cyc} cycles")
            bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP,
                                        ops_per_wave=2, unroll=1, tiles_per_wave=8)
            try:
                R.rteaal_step(ctx, bid, 700)
                R.rteaal_step(ctx, bid, 1300)
                got = read_regs(ctx, bid, d, pick)
                got_dg = read_digest(ctx, bid, pick)
            finally:
                R.rteaal_free_batch(ctx, bid)
            note(f"single-200k plain 1 x {cyc} cycles")
            bid = R.rteaal_create_batch(ctx, did, seeds[:1], mapping=R.RTEAAL_MAP_LAYERED,
                                        block_threads=64, unroll=1)
            try:
                R.rteaal_step(ctx, bid, cyc)
                got_p = read_regs(ctx, bid, d, [0])
                got_pdg = read_digest(ctx, bid, [0])
            finally:
                R.rteaal_free_batch(ctx, bid)
        finally:
            R.rteaal_unload_design(ctx, did)
        note("single-200k: waiting for the oracle")
        ref, ref_dg = fut.result()
    assert_same(got, ref, "single-200k 2000 cycles")
    assert_same(got_dg, ref_dg, "single-200k 2000 cycles digest")
    assert_same(got_p, ref[:1], "single-200k plain")
    assert_same(got_pdg, ref_dg[:1], "single-200k plain digest")


def test_muxchain_2m_fused_sampled(ctx):
    """muxchain-2m (2,000,000 ops, 4,096 instances) fused and levelized as the
    bench runs it: 16 sampled instances after 100 cycles, registers and
    digest, against the oracle of the design as drawn."""
    d = rtlgen.generate(rtlgen.CFG_MUXCHAIN, 6)
    f, cnt = R.rteaal_fuse_mux_chains(d)
    lv = R.levelized_design(ctx, f)
    n = 4096
    seeds = rtlgen.instance_seeds(n)
    rng = np.random.default_rng(12)
    pick = sorted({0, n - 1} | set(rng.choice(np.arange(1, n - 1), 14, replace=False).tolist()))
    cyc = 100
    ref, ref_dg = oracle_with_digest(d, seeds[pick], cyc)
    did = R.rteaal_load_design(ctx, lv)
    try:
        for shape in ({"ops_per_wave": 2, "unroll": 1, "tiles_per_wave": 8}, {}):
            note(f"muxchain-2m fused ({cnt['n_fused']} MUXC) {n} x {cyc} cycles, shape {shape}")
            bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP, **shape)
            try:
                R.rteaal_step(ctx, bid, 30)
                R.rteaal_step(ctx, bid, cyc - 30)
                got = read_regs(ctx, bid, lv, pick)
                got_dg = read_digest(ctx, bid, pick)
            finally:
                R.rteaal_free_batch(ctx, bid)
            assert_same(got, ref, f"muxchain-2m sample, shape {shape}")
            assert_same(got_dg, ref_dg, f"muxchain-2m sample digest, shape {shape}")
    finally:
        R.rteaal_unload_design(ctx, did)


def test_multidesign_64_sampled(ctx):
    """The uneven multi-design batch: 64 designs of 5,000-500,000 ops with 10%
    of widths at 65-128 bits, 1-256 instances each, advanced together by
    rteaal_step_many (three steps, 200 cycles); first and last instance of
    every design, registers and digest."""
    plan = rtlgen.multidesign_batch()
    designs, dids, bids, seeds_of = [], [], [], []
    try:
        for k, (cfg, dseed, n) in enumerate(plan):
            d = rtlgen.generate(cfg, dseed)
            designs.append(d)
            dids.append(R.rteaal_load_design(ctx, d))
            seeds_of.append(rtlgen.instance_seeds(n, design_index=k))
            bids.append(R.rteaal_create_batch(ctx, dids[-1], seeds_of[-1]))
        cyc = 200
        picks = [sorted({0, len(s) - 1}) for s in seeds_of]
        note(f"multi-design: {len(plan)} designs, {sum(p[2] for p in plan)} instances, {cyc} cycles")
        with ThreadPoolExecutor(1) as ex:
            fut = ex.submit(oracle_jobs, [(d, seeds_of[k][picks[k]], cyc, len(picks[k]))
                                          for k, d in enumerate(designs)])
            R.rteaal_step_many(ctx, bids, [2] * len(bids))
            R.rteaal_step_many(ctx, bids, [3] * len(bids))
            R.rteaal_step_many(ctx, bids, [cyc - 5] * len(bids))
            got = [(read_regs(ctx, bids[k], d, picks[k]), read_digest(ctx, bids[k], picks[k]))
                   for k, d in enumerate(designs)]
            note("multi-design: waiting for the oracle")
            refs = fut.result()
        for k, d in enumerate(designs):
            n = len(seeds_of[k])
            assert_same(got[k][0], refs[k][0], f"design {k} ({d.n_ops} ops, {n} instances)")
            assert_same(got[k][1], refs[k][1], f"design {k} digest")
            assert R.rteaal_batch_info(ctx, bids[k])[1] == cyc
    finally:
        for b in bids:
            R.rteaal_free_batch(ctx, b)
        for x in dids:
            R.rteaal_unload_design(ctx, x)
