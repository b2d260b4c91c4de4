"""Persistent LAYERED batches: every cycle of a step in one cooperative launch
with a grid-wide barrier per layer (GPU).

Registers and the per-cycle register digest must equal the oracle across
launch chunks (1,024 cycles), for one and several instances, watched (one
cycle per launch, change log equal to the per-layer form's) and inside
rteaal_step_many.  A barrier wait past its spin limit is reported as a
device error at the next synchronisation (forced from the host with a
limit of one spin; every wait is bounded, so every block still ends).
Integer arithmetic: tolerance 0.
"""
import os

import numpy as np
import pytest

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from tests.gpu_util import assert_same, gpu_ctx

pytestmark = pytest.mark.gpu

PERSIST = dict(mapping=R.RTEAAL_MAP_LAYERED, persistent=1)


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    R.rteaal_destroy(c)


def expect(ctx, bid, d, seeds, cycles, what):
    dg = {}
    ref, _, _ = oracle.run(d, seeds, cycles, digests=dg)
    got = R.unpack_limbs(R.rteaal_read_state(ctx, bid), d.slot_width[d.reg_slot])
    assert_same(got, ref, what)
    assert_same(R.rteaal_read_digest(ctx, bid), dg["final"], what + " digest")


@pytest.mark.parametrize("unroll", [1, 2])
@pytest.mark.parametrize("n_inst", [1, 3, 16])
def test_persistent_matches_oracle(ctx, unroll, n_inst):
    d = rtlgen.generate(rtlgen.GenConfig(3000, 20, 100, 16, rtlgen.generator.WIDTHS_LARGE,
                                         "persist"), 40 + n_inst)
    seeds = np.arange(n_inst, dtype=np.uint64) * 5 + 1
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, seeds, unroll=unroll, **PERSIST)
    try:
        assert R.rteaal_batch_options(ctx, bid)["persistent"] == 1
        for k in (1, 30, 9):
            R.rteaal_step(ctx, bid, k)
        expect(ctx, bid, d, seeds, 40, f"{n_inst} instances, unroll {unroll}")
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


def test_persistent_long_run_chunks(ctx):
    d = rtlgen.generate(rtlgen.CFG0, 0)
    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, [0, 7], **PERSIST)
    try:
        R.rteaal_step(ctx, bid, 1500)
        R.rteaal_step(ctx, bid, 700)
        expect(ctx, bid, d, [0, 7], 2200, "plain-2k 2,200 cycles")
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


def test_persistent_watched_and_in_step_many(ctx):
    d = rtlgen.generate(rtlgen.GenConfig(800, 8, 40, 8, rtlgen.generator.WIDTHS_STD, "pw"), 3)
    did = R.rteaal_load_design(ctx, d)
    seeds = np.array([4, 5], np.uint64)
    a = R.rteaal_create_batch(ctx, did, seeds, **PERSIST)
    b = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_LAYERED)
    c = R.rteaal_create_batch(ctx, did, np.arange(100, dtype=np.uint64), mapping=R.RTEAAL_MAP_SWEEP)
    try:
        for x in (a, b):
            R.rteaal_watch(ctx, x, d.reg_slot[:10])
        R.rteaal_step(ctx, a, 6)
        R.rteaal_step(ctx, b, 6)
        la, _ = R.rteaal_read_changes(ctx, a)
        lb, _ = R.rteaal_read_changes(ctx, b)
        key = lambda r: (int(r["cycle"]), int(r["instance"]), int(r["signal"]))  # noqa: E731
        assert sorted(map(key, la)) == sorted(map(key, lb)) and len(la) > 0
        R.rteaal_watch(ctx, a, [])
        R.rteaal_step_many(ctx, [a, c], [5, 5])
        expect(ctx, a, d, seeds, 11, "persistent batch after a watched step and step_many")
        expect(ctx, c, d, np.arange(100, dtype=np.uint64), 5, "SWEEP batch beside it")
    finally:
        for x in (a, b, c):
            R.rteaal_free_batch(ctx, x)
        R.rteaal_unload_design(ctx, did)


def test_barrier_spin_limit_is_reported():
    """A spin limit of one makes (almost) every barrier wait run out: the
    launch still completes and the next synchronisation reports it."""
    old = os.environ.get("RTEAAL_GRID_SPIN_LIMIT")
    os.environ["RTEAAL_GRID_SPIN_LIMIT"] = "1"
    try:
        c = R.rteaal_create(0)
    finally:
        if old is None:
            del os.environ["RTEAAL_GRID_SPIN_LIMIT"]
        else:
            os.environ["RTEAAL_GRID_SPIN_LIMIT"] = old
    try:
        d = rtlgen.generate(rtlgen.GenConfig(20_000, 40, 300, 16, rtlgen.generator.WIDTHS_STD,
                                             "spin"), 1)
        did = R.rteaal_load_design(c, d)
        bid = R.rteaal_create_batch(c, did, [1], **PERSIST)
        R.rteaal_step(c, bid, 20)
        with pytest.raises(R.RteaalError) as e:
            R.rteaal_sync(c)
        assert e.value.status == 5 and "grid barrier" in str(e.value)
    finally:
        R.rteaal_destroy(c)
