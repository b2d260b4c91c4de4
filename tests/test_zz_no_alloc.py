"""rteaal_read_state_noalloc against rteaal_read_state (GPU).

The no-allocation variant stages the read-out through a fixed device array
instead of a buffer allocated per call.  Through the C interface it must
return exactly what rteaal_read_state returns, on two calls in a row (the
second smaller, so stale contents of the shared array would show), for
registers, digests and every slot, on SWEEP and RESIDENT batches, without
asking the allocator for memory; read-outs larger than the array are
refused.
"""
import numpy as np
import pytest

import rtlgen
from paper_2601_18140_amd import rteaal as R

pytestmark = pytest.mark.gpu


def test_noalloc_read_equals_read_state():
    ctx = R.rteaal_create(0)
    try:
        d = rtlgen.generate(rtlgen.GenConfig(1500, 10, 300, 12, rtlgen.generator.WIDTHS_LARGE,
                                             "noalloc"), 21)
        did = R.rteaal_load_design(ctx, d, keep_all_slots=True)
        for mapping, n_inst in ((R.RTEAAL_MAP_SWEEP, 200), (R.RTEAAL_MAP_RESIDENT, 9)):
            seeds = np.arange(n_inst, dtype=np.uint64) * 31 + 2
            bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping)
            R.rteaal_step(ctx, bid, 17)
            R.rteaal_sync(ctx)
            for what in (R.RTEAAL_READ_REGS, R.RTEAAL_READ_ALL_SLOTS, R.RTEAAL_READ_DIGEST):
                # two calls in a row, the second over fewer instances
                for first, n in ((0, n_inst), (n_inst // 3, max(1, n_inst // 4))):
                    exp = R.rteaal_read_state(ctx, bid, first, n, what)
                    before = ctx.device_allocations()
                    got = R.rteaal_read_state_noalloc(ctx, bid, first, n, what)
                    assert ctx.device_allocations() == before, "the no-allocation read allocated"
                    assert got.shape == exp.shape
                    assert np.array_equal(got, exp), (mapping, what, first, n)
            R.rteaal_free_batch(ctx, bid)
        # A read-out larger than the staging array is refused.
        big = rtlgen.generate(rtlgen.GenConfig(20_000, 8, 4000, 16, rtlgen.generator.WIDTHS_STD,
                                               "noalloc-big"), 22)
        bd = R.rteaal_load_design(ctx, big, keep_all_slots=True)
        n_inst = 64
        bb = R.rteaal_create_batch(ctx, bd, np.arange(n_inst, dtype=np.uint64),
                                   mapping=R.RTEAAL_MAP_SWEEP)
        R.rteaal_step(ctx, bb, 2)
        words = int(((big.slot_width.astype(np.int64) + 63) // 64).sum())
        assert words * n_inst > R.RTEAAL_NOALLOC_MAX_WORDS
        with pytest.raises(R.RteaalError) as e:
            R.rteaal_read_state_noalloc(ctx, bb, 0, n_inst, R.RTEAAL_READ_ALL_SLOTS)
        assert e.value.status == 1
        fit = R.RTEAAL_NOALLOC_MAX_WORDS // words
        assert np.array_equal(R.rteaal_read_state_noalloc(ctx, bb, 0, fit, R.RTEAAL_READ_ALL_SLOTS),
                              R.rteaal_read_state(ctx, bb, 0, fit, R.RTEAAL_READ_ALL_SLOTS))
        R.rteaal_free_batch(ctx, bb)
        R.rteaal_unload_design(ctx, bd)
        R.rteaal_unload_design(ctx, did)
    finally:
        R.rteaal_destroy(ctx)
