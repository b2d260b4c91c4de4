"""Parity at the full workload sizes (GPU), on sampled instances.

The oracle cannot afford every instance of the large batches, so each
comparison picks fixed instances (first, last, and a seeded draw) and runs
the full-size batch on the GPU in the launch shapes the bench measures.
Integer arithmetic: tolerance 0.
"""
import sys

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
    ref, _, _ = oracle.run(d, seeds[pick], cyc, n_threads=16)
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
            finally:
                R.rteaal_free_batch(ctx, bid)
            assert_same(got, ref, f"large-5m sample, shape {shape}")
        for opts in ({"mapping": R.RTEAAL_MAP_LAYERED, "block_threads": 64, "unroll": 1}, {}):
            note(f"large-5m plain 1 instance x 3 cycles, {opts}")
            bid = R.rteaal_create_batch(ctx, did, seeds[:1], **opts)
            try:
                R.rteaal_step(ctx, bid, cyc)
                got = read_regs(ctx, bid, d, [0])
            finally:
                R.rteaal_free_batch(ctx, bid)
            assert_same(got, ref[:1], f"large-5m plain {opts}")
    finally:
        R.rteaal_unload_design(ctx, did)


def test_muxchain_2m_fused_sampled(ctx):
    """muxchain-2m (2,000,000 ops, 4,096 instances) fused and levelized as the
    bench runs it: 16 sampled instances after 3 cycles, against the oracle of
    the design as drawn."""
    d = rtlgen.generate(rtlgen.CFG_MUXCHAIN, 6)
    f, cnt = R.rteaal_fuse_mux_chains(d)
    lv = R.levelized_design(ctx, f)
    n = 4096
    seeds = rtlgen.instance_seeds(n)
    rng = np.random.default_rng(12)
    pick = sorted({0, n - 1} | set(rng.choice(np.arange(1, n - 1), 14, replace=False).tolist()))
    ref, _, _ = oracle.run(d, seeds[pick], 3, n_threads=16)
    did = R.rteaal_load_design(ctx, lv)
    try:
        for shape in ({"ops_per_wave": 2, "unroll": 1, "tiles_per_wave": 8}, {}):
            note(f"muxchain-2m fused ({cnt['n_fused']} MUXC) {n} x 3 cycles, shape {shape}")
            bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP, **shape)
            try:
                R.rteaal_step(ctx, bid, 3)
                got = read_regs(ctx, bid, lv, pick)
            finally:
                R.rteaal_free_batch(ctx, bid)
            assert_same(got, ref, f"muxchain-2m sample, shape {shape}")
    finally:
        R.rteaal_unload_design(ctx, did)


def test_multidesign_64_sampled(ctx):
    """The uneven multi-design batch: 64 designs of 5,000-500,000 ops with 10%
    of widths at 65-128 bits, 1-256 instances each, advanced together by
    rteaal_step_many (two steps); first and last instance of every design."""
    plan = rtlgen.multidesign_batch()
    designs, dids, bids, seeds_of = [], [], [], []
    try:
        for k, (cfg, dseed, n) in enumerate(plan):
            d = rtlgen.generate(cfg, dseed)
            designs.append(d)
            dids.append(R.rteaal_load_design(ctx, d))
            seeds_of.append(rtlgen.instance_seeds(n, design_index=k))
            bids.append(R.rteaal_create_batch(ctx, dids[-1], seeds_of[-1]))
        note(f"multi-design: {len(plan)} designs, {sum(p[2] for p in plan)} instances")
        R.rteaal_step_many(ctx, bids, [2] * len(bids))
        R.rteaal_step_many(ctx, bids, [3] * len(bids))
        for k, d in enumerate(designs):
            n = len(seeds_of[k])
            pick = sorted({0, n - 1})
            got = read_regs(ctx, bids[k], d, pick)
            ref, _, _ = oracle.run(d, seeds_of[k][pick], 5, n_threads=len(pick))
            assert_same(got, ref, f"design {k} ({d.n_ops} ops, {n} instances)")
            assert R.rteaal_batch_info(ctx, bids[k])[1] == 5
    finally:
        for b in bids:
            R.rteaal_free_batch(ctx, b)
        for x in dids:
            R.rteaal_unload_design(ctx, x)
