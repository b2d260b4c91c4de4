"""Per-cycle register digest of the HIP path against the oracle (GPU).

The digest folds the whole register vector after every cycle into one word
per instance (the definition is in include/rteaal.h and oracle/oracle.h,
written separately on each side), so equal digests after n cycles compare
the register state after each of the n cycles, not just the last one.
Integer arithmetic: tolerance 0.
"""
import sys

import numpy as np
import pytest

import oracle
import rtlgen
from rtlgen import circuits as cir
from paper_2601_18140_amd import rteaal as R
from tests.gpu_util import assert_same, gpu_ctx

pytestmark = pytest.mark.gpu

MAPS = [R.RTEAAL_MAP_RESIDENT, R.RTEAAL_MAP_SWEEP, R.RTEAAL_MAP_LAYERED]
MAP_IDS = ["resident", "sweep", "layered"]

SMALL = rtlgen.GenConfig(900, 9, 48, 12, rtlgen.generator.WIDTHS_LARGE, "dg-wide")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    R.rteaal_destroy(c)


def oracle_digest(d, seeds, cycles, trace=False, **kw):
    dg = {}
    regs, _, _ = oracle.run(d, seeds, cycles, digests=dg, digest_trace=trace, **kw)
    return regs, dg


def gpu_regs(ctx, bid, d):
    return R.unpack_limbs(R.rteaal_read_state(ctx, bid), d.slot_width[d.reg_slot])


@pytest.mark.parametrize("mapping", MAPS, ids=MAP_IDS)
def test_digest_after_every_cycle(ctx, mapping):
    """One cycle per step, the digest read after each: every value of the
    oracle's digest trace, for 70 instances (two SWEEP tiles, one ragged)."""
    d = rtlgen.generate(SMALL, 11)
    seeds = np.arange(70, dtype=np.uint64) * 13 + 1
    cyc = 12
    _, ref = oracle_digest(d, seeds, cyc, trace=True)
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping)
    try:
        assert (R.rteaal_read_digest(ctx, bid) == 0).all(), "digest starts at 0"
        for c in range(cyc):
            R.rteaal_step(ctx, bid, 1)
            got = R.rteaal_read_digest(ctx, bid)
            assert_same(got, ref["trace"][:, c], f"digest after cycle {c + 1}")
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


@pytest.mark.parametrize("mapping", MAPS, ids=MAP_IDS)
def test_digest_long_run_and_chunks(ctx, mapping):
    """plain-2k's recipe over 2,100 cycles in uneven steps (RESIDENT runs
    1,024 cycles per launch, so the digest crosses launch boundaries)."""
    d = rtlgen.generate(rtlgen.CFG0, 0)
    seeds = np.array([0, 5, 9], np.uint64)
    regs_ref, ref = oracle_digest(d, seeds, 2100)
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping)
    try:
        for k in (1, 1023, 1025, 51):
            R.rteaal_step(ctx, bid, k)
        assert_same(gpu_regs(ctx, bid, d), regs_ref, "registers")
        assert_same(R.rteaal_read_digest(ctx, bid), ref["final"], "digest")
        assert_same(R.rteaal_read_digest(ctx, bid, first=1, n=2), ref["final"][1:], "digest range")
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


def test_digest_sweep_shapes_and_passes(ctx):
    """SWEEP tile groups, operations per wavefront and tile passes: 300
    instances (5 tiles, the last ragged)."""
    d = rtlgen.generate(SMALL, 12)
    seeds = np.arange(300, dtype=np.uint64) + 1000
    _, ref = oracle_digest(d, seeds, 9)
    did = R.rteaal_load_design(ctx, d)
    try:
        for shape in ({"tiles_per_wave": 1, "ops_per_wave": 3}, {"tiles_per_wave": 2, "unroll": 4},
                      {"tiles_per_wave": 4, "unroll": 1, "tiles_per_pass": 4},
                      {"tiles_per_wave": 8, "unroll": 1}, {"tiles_per_wave": 16, "unroll": 1}):
            note(f"digest, SWEEP shape {shape}")
            bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP, **shape)
            try:
                R.rteaal_step(ctx, bid, 4)
                R.rteaal_step(ctx, bid, 5)
                assert_same(R.rteaal_read_digest(ctx, bid), ref["final"], f"shape {shape}")
            finally:
                R.rteaal_free_batch(ctx, bid)
    finally:
        R.rteaal_unload_design(ctx, did)


@pytest.mark.parametrize("mapping", MAPS, ids=MAP_IDS)
def test_digest_no_registers_and_wide_registers(ctx, mapping):
    """A design with no registers (the digest is s applied once per cycle to
    0, independent of everything else) and 130-bit counters (three limbs
    per register fold)."""
    d = rtlgen.generate(rtlgen.GenConfig(300, 5, 0, 6, rtlgen.generator.WIDTHS_STD, "no-regs"), 1)
    assert d.n_regs == 0
    exp = 0
    for _ in range(7):
        exp = oracle.splitmix64(exp)
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, [3, 4], mapping=mapping)
    try:
        R.rteaal_step(ctx, bid, 7)
        assert (R.rteaal_read_digest(ctx, bid) == np.uint64(exp)).all()
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)
    d = cir.counter(130, 3**70)
    _, ref = oracle_digest(d, [0, 1], 40)
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, [0, 1], mapping=mapping)
    try:
        R.rteaal_step(ctx, bid, 40)
        assert_same(R.rteaal_read_digest(ctx, bid), ref["final"], "130-bit counter")
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


@pytest.mark.parametrize("mapping", MAPS, ids=MAP_IDS)
def test_digest_checkpoint_and_host_poke(ctx, mapping):
    """A checkpoint (registers, digest, cycle) restored into a fresh batch
    continues the same chain; a host write of registers between cycles is
    matched by the oracle continuing from the written registers."""
    d = rtlgen.generate(SMALL, 13)
    seeds = np.arange(6, dtype=np.uint64) + 40
    regs_all, ref_all = oracle_digest(d, seeds, 20)
    widths = d.slot_width[d.reg_slot]
    did = R.rteaal_load_design(ctx, d)
    try:
        a = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping)
        R.rteaal_step(ctx, a, 8)
        regs8 = R.rteaal_read_state(ctx, a)
        dig8 = R.rteaal_read_digest(ctx, a)
        b = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping)
        R.rteaal_write_state(ctx, b, 0, regs8, 8)
        R.rteaal_write_digest(ctx, b, 0, dig8)
        R.rteaal_step(ctx, b, 12)
        assert_same(R.rteaal_read_digest(ctx, b), ref_all["final"], "restored chain")
        assert_same(R.unpack_limbs(R.rteaal_read_state(ctx, b), widths), regs_all, "restored regs")
        # host poke: instance 2's registers replaced after cycle 8, on batch a
        poke = R.unpack_limbs(regs8, widths)
        rng = np.random.default_rng(5)
        for j in range(d.n_regs):
            w = int(widths[j])
            v = int(rng.integers(0, 2**63)) | (int(rng.integers(0, 2**63)) << 63)
            v %= 1 << w
            poke[2, j] = [(v >> (64 * k)) & (2**64 - 1) for k in range(4)]
        R.rteaal_write_state(ctx, a, 2, R.pack_limbs(poke[2:3], widths), 8)
        R.rteaal_step(ctx, a, 12)
        r2, ref2 = oracle_digest(d, seeds[2:3], 12, start_cycle=8, init_regs=poke[2:3],
                                 init_digest=dig8[2:3])
        assert_same(R.rteaal_read_digest(ctx, a, 2, 1), ref2["final"], "poked instance digest")
        assert_same(R.unpack_limbs(R.rteaal_read_state(ctx, a, 2, 1), widths), r2, "poked regs")
        assert_same(R.rteaal_read_digest(ctx, a, 3, 3), ref_all["final"][3:], "untouched instances")
        R.rteaal_free_batch(ctx, a)
        R.rteaal_free_batch(ctx, b)
    finally:
        R.rteaal_unload_design(ctx, did)


def test_digest_step_many_watched_and_profiled(ctx):
    """step_many over RESIDENT, SWEEP and LAYERED batches; a watched batch
    (capture after every cycle); a batch with kernel timing on (launches
    issued one by one instead of through the cycle graph)."""
    d = rtlgen.generate(SMALL, 14)
    seeds = np.arange(90, dtype=np.uint64) * 3 + 7
    _, ref = oracle_digest(d, seeds, 10)
    did = R.rteaal_load_design(ctx, d)
    try:
        bs = [R.rteaal_create_batch(ctx, did, seeds, mapping=m) for m in MAPS]
        R.rteaal_step_many(ctx, bs, [4, 4, 4])
        R.rteaal_step_many(ctx, bs, [6, 6, 6])
        for b, name in zip(bs, MAP_IDS):
            assert_same(R.rteaal_read_digest(ctx, b), ref["final"], f"step_many {name}")
            R.rteaal_free_batch(ctx, b)
        for m, name in zip(MAPS, MAP_IDS):
            b = R.rteaal_create_batch(ctx, did, seeds, mapping=m)
            R.rteaal_watch(ctx, b, d.reg_slot[:5])
            R.rteaal_step(ctx, b, 3)
            R.rteaal_kernel_timing(ctx, b, True)
            R.rteaal_step(ctx, b, 4)
            R.rteaal_kernel_timing(ctx, b, False)
            R.rteaal_watch(ctx, b, [])
            R.rteaal_step(ctx, b, 3)
            assert_same(R.rteaal_read_digest(ctx, b), ref["final"], f"watched/profiled {name}")
            R.rteaal_free_batch(ctx, b)
    finally:
        R.rteaal_unload_design(ctx, did)


def test_read_digest_rejects_bad_ranges(ctx):
    d = cir.counter(8)
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, [1, 2])
    try:
        with pytest.raises(R.RteaalError):
            R.rteaal_read_state(ctx, bid, first=1, n=2, what=R.RTEAAL_READ_DIGEST)
        with pytest.raises(R.RteaalError):
            R.rteaal_write_digest(ctx, bid, 2, [1])
        with pytest.raises(R.RteaalError):
            R.rteaal_read_state(ctx, bid, what=R.RTEAAL_READ_DIGEST | R.RTEAAL_READ_REGS)
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)
