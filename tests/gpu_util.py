"""Helpers shared by the GPU tests: run a design through the C interface."""
import numpy as np

from paper_2601_18140_amd import rteaal as R


def gpu_ctx():
    return R.rteaal_create(0)


def run_gpu(ctx, design, seeds, steps, mapping=R.RTEAAL_MAP_AUTO, words=None, slots=False,
            **opts):
    """Simulate; `steps` is a cycle count or a list of step sizes.  Returns
    (regs[n, n_regs, 4], slots[n, n_slots, 4] or None, batch mapping).

    With slots=True the design is loaded with every slot keeping its own
    storage (so all slots can be read), and the same run is repeated on the
    default live-range layout, whose registers must be identical."""
    if slots:
        regs, sl, used = _run(ctx, design, seeds, steps, mapping, words, True, **opts)
        regs2, _, used2 = _run(ctx, design, seeds, steps, mapping, words, False, **opts)
        assert_same(regs2, regs, "live-range layout vs all-slot layout")
        assert used2 == used
        return regs, sl, used
    return _run(ctx, design, seeds, steps, mapping, words, False, **opts)


def _run(ctx, design, seeds, steps, mapping, words, slots, **opts):
    did = R.rteaal_load_design(ctx, design, keep_all_slots=slots)
    try:
        bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping, **opts)
        try:
            steps = [steps] if np.isscalar(steps) else list(steps)
            done = 0
            for k in steps:
                w = None if words is None else words[done:done + k]
                R.rteaal_step(ctx, bid, k, words=w)
                done += k
            R.rteaal_sync(ctx)
            regs = R.unpack_limbs(R.rteaal_read_state(ctx, bid), design.slot_width[design.reg_slot])
            sl = None
            if slots:
                sl = R.unpack_limbs(R.rteaal_read_state(ctx, bid, what=R.RTEAAL_READ_ALL_SLOTS),
                                    design.slot_width)
            mapping_used, cycle = R.rteaal_batch_info(ctx, bid)
            assert cycle == done
            return regs, sl, mapping_used
        finally:
            R.rteaal_free_batch(ctx, bid)
    finally:
        R.rteaal_unload_design(ctx, did)


def driven_slots(design):
    """Slots that have a driver (undriven slots read back as zero)."""
    m = np.zeros(design.n_slots, bool)
    for a in (design.const_slot, design.input_slot, design.reg_slot, design.op_dst):
        m[np.asarray(a, dtype=np.int64)] = True
    return m


def assert_same(got, exp, what=""):
    if not np.array_equal(got, exp):
        bad = np.argwhere(got != exp)
        i = tuple(bad[0])
        raise AssertionError(f"{what}: {len(bad)} mismatching limbs, first at {i}: "
                             f"got {got[i]} expected {exp[i]}")
