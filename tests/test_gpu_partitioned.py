"""PARTITIONED batches: the replicated register partitioning of App. C
(Cascade 2 with a partition rank), one workgroup per (instance, partition),
registers exchanged once per cycle across a grid-wide barrier (GPU).

Registers and the per-cycle register digest must equal the oracle for one
and several instances, partition counts from one to one per register, the
state in LDS or in HBM, across launch chunks (1,024 cycles), with host
stimulus words, after a restore that writes only the owners' copies (the
next launch's first exchange must carry it to every partition), and inside
rteaal_step_many beside every other mapping.  A request for more
workgroups than the device holds at once fails on the host before any
launch.  Integer arithmetic: tolerance 0.
"""
import numpy as np
import pytest

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from tests.gpu_util import assert_same, gpu_ctx

pytestmark = pytest.mark.gpu

PART = dict(mapping=R.RTEAAL_MAP_PARTITIONED)


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    R.rteaal_destroy(c)


def regs_of(ctx, bid, d):
    return R.unpack_limbs(R.rteaal_read_state(ctx, bid), d.slot_width[d.reg_slot])


def expect(ctx, bid, d, seeds, cycles, what, **kw):
    dg = {}
    ref, _, _ = oracle.run(d, seeds, cycles, digests=dg, **kw)
    assert_same(regs_of(ctx, bid, d), ref, what)
    assert_same(R.rteaal_read_digest(ctx, bid), dg["final"], what + " digest")


@pytest.mark.parametrize("n_inst,parts,lds_state", [
    (1, 0, 0),      # default count (one per register here), state in LDS
    (1, 7, 0),
    (1, 7, 1),      # state in HBM
    (3, 16, 0),
    (2, 1, 0),      # one partition: the whole program, no exchange partner
])
def test_partitioned_matches_oracle(ctx, n_inst, parts, lds_state):
    d = rtlgen.generate(rtlgen.GenConfig(3000, 20, 100, 16, rtlgen.generator.WIDTHS_LARGE,
                                         "part"), 50 + n_inst)
    seeds = np.arange(n_inst, dtype=np.uint64) * 5 + 3
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, seeds, partitions=parts, lds_state=lds_state, **PART)
    try:
        o = R.rteaal_batch_options(ctx, bid)
        assert o["mapping"] == R.RTEAAL_MAP_PARTITIONED
        assert o["partitions"] == (parts or min(256 // n_inst, d.reg_slot.shape[0]))
        assert o["lds_state"] == lds_state
        for k in (1, 30, 9):
            R.rteaal_step(ctx, bid, k)
        expect(ctx, bid, d, seeds, 40, f"{n_inst} instances, {parts} partitions, lds_state {lds_state}")
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


def test_partitioned_long_run_chunks(ctx):
    d = rtlgen.generate(rtlgen.CFG0, 0)
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, [0, 7], partitions=32, **PART)
    try:
        R.rteaal_step(ctx, bid, 1500)
        R.rteaal_step(ctx, bid, 700)
        expect(ctx, bid, d, [0, 7], 2200, "plain-2k 2,200 cycles")
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


def test_partitioned_host_words(ctx):
    d = rtlgen.generate(rtlgen.GenConfig(900, 12, 40, 7, rtlgen.generator.WIDTHS_STD, "pw"), 8)
    n_words = int(((d.slot_width[d.input_slot].astype(np.int64) + 63) // 64).sum())
    seeds = np.array([2, 9, 4], np.uint64)
    rng = np.random.default_rng(5)
    w = rng.integers(0, 2**63, (6, 3, n_words), dtype=np.uint64) * np.uint64(2)
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, seeds, partitions=8, **PART)
    try:
        R.rteaal_step(ctx, bid, 6, words=w)
        expect(ctx, bid, d, seeds, 6, "host words", stim_words=w)
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


def test_partitioned_restore_reaches_every_partition(ctx):
    """Registers written by rteaal_write_state go to their owners' copies;
    the first exchange of the next launch must hand them to every partition
    whose cones read them."""
    d = rtlgen.generate(rtlgen.GenConfig(2000, 16, 80, 12, rtlgen.generator.WIDTHS_LARGE, "pr"), 4)
    seeds = np.array([11, 12], np.uint64)
    did = R.rteaal_load_design(ctx, d)
    a = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_RESIDENT)
    b = R.rteaal_create_batch(ctx, did, seeds, partitions=20, **PART)
    try:
        R.rteaal_step(ctx, a, 10)
        saved = R.rteaal_read_state(ctx, a)
        dig = R.rteaal_read_digest(ctx, a)
        R.rteaal_step(ctx, b, 3)             # something else in every copy first
        R.rteaal_write_state(ctx, b, 0, saved, 10)
        R.rteaal_write_digest(ctx, b, 0, dig)
        assert_same(regs_of(ctx, b, d), regs_of(ctx, a, d), "restored registers")
        R.rteaal_step(ctx, a, 15)
        R.rteaal_step(ctx, b, 15)
        assert_same(regs_of(ctx, b, d), regs_of(ctx, a, d), "15 cycles after the restore")
        assert_same(R.rteaal_read_digest(ctx, b), R.rteaal_read_digest(ctx, a), "digest")
        expect(ctx, b, d, seeds, 25, "restored PARTITIONED batch vs the oracle")
    finally:
        for x in (a, b):
            R.rteaal_free_batch(ctx, x)
        R.rteaal_unload_design(ctx, did)


def test_partitioned_in_step_many(ctx):
    d = rtlgen.generate(rtlgen.GenConfig(800, 8, 40, 8, rtlgen.generator.WIDTHS_STD, "pm"), 3)
    did = R.rteaal_load_design(ctx, d)
    s2 = np.array([4, 5], np.uint64)
    s100 = np.arange(100, dtype=np.uint64)
    bs = [R.rteaal_create_batch(ctx, did, s2, partitions=10, **PART),
          R.rteaal_create_batch(ctx, did, s2, partitions=3, lds_state=1, **PART),
          R.rteaal_create_batch(ctx, did, s2, mapping=R.RTEAAL_MAP_LAYERED, persistent=1),
          R.rteaal_create_batch(ctx, did, s2, mapping=R.RTEAAL_MAP_RESIDENT),
          R.rteaal_create_batch(ctx, did, s100, mapping=R.RTEAAL_MAP_SWEEP),
          R.rteaal_create_batch(ctx, did, s100, mapping=R.RTEAAL_MAP_SWEEP, tiles_per_wave=2)]
    seeds = [s2, s2, s2, s2, s100, s100]
    try:
        R.rteaal_step_many(ctx, bs, [5, 7, 5, 3, 6, 2])
        R.rteaal_step_many(ctx, bs, [2, 0, 2, 4, 1, 5])
        for b, s, c in zip(bs, seeds, [7, 7, 7, 7, 7, 7]):
            expect(ctx, b, d, s, c, f"batch {b} in step_many")
    finally:
        for b in bs:
            R.rteaal_free_batch(ctx, b)
        R.rteaal_unload_design(ctx, did)


def test_partitioned_refusals(ctx):
    d = rtlgen.generate(rtlgen.GenConfig(500, 6, 30, 4, rtlgen.generator.WIDTHS_STD, "pf"), 1)
    did = R.rteaal_load_design(ctx, d)
    try:
        with pytest.raises(R.RteaalError) as e:       # more partitions than registers
            R.rteaal_create_batch(ctx, did, [1], partitions=31, **PART)
        assert e.value.status == 1
        with pytest.raises(R.RteaalError) as e:       # more workgroups than fit at once
            R.rteaal_create_batch(ctx, did, np.arange(4000, dtype=np.uint64), partitions=30,
                                  **PART)
        assert e.value.status == 1 and "resident" in str(e.value)
        bid = R.rteaal_create_batch(ctx, did, [1], partitions=30, **PART)
        try:
            with pytest.raises(R.RteaalError) as e:
                R.rteaal_watch(ctx, bid, d.reg_slot[:2])
            assert e.value.status == 7
            R.rteaal_step(ctx, bid, 4)
            expect(ctx, bid, d, [1], 4, "after the refusals")
        finally:
            R.rteaal_free_batch(ctx, bid)
    finally:
        R.rteaal_unload_design(ctx, did)


def test_partition_plan_stats(ctx):
    """Host-side size of the partitioned form: every cone of one partition is
    the union of all cones (the operations that reach a register), each
    partition count replicates at least that much, and the exchange is empty
    for one partition."""
    d = rtlgen.generate(rtlgen.GenConfig(3000, 20, 100, 16, rtlgen.generator.WIDTHS_LARGE,
                                         "part"), 51)
    did = R.rteaal_load_design(ctx, d)
    try:
        one = R.rteaal_partition_plan_stats(ctx, did, 1)
        assert one["exchange"] == 0 and one["cone_ops"] <= one["design_ops"]
        assert one["max_part_ops"] == one["padded_ops"] >= one["cone_ops"]
        for p in (2, 7, 100):
            st = R.rteaal_partition_plan_stats(ctx, did, p)
            assert st["design_ops"] == one["design_ops"]
            assert one["cone_ops"] <= st["cone_ops"] <= p * one["cone_ops"]
            assert st["cone_ops"] <= st["padded_ops"] and st["max_part_ops"] <= st["padded_ops"]
            assert st["exchange"] > 0
        with pytest.raises(R.RteaalError):
            R.rteaal_partition_plan_stats(ctx, did, 101)
    finally:
        R.rteaal_unload_design(ctx, did)
