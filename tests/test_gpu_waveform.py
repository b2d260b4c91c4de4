"""Waveform capture and per-cycle host–DUT interaction, against the oracle.

The oracle gives every slot's value after each cycle (one-cycle runs from
the previous registers); a transition is a watched value that differs from
its value one cycle earlier (before the first cycle: the reset state, all
zero).  The device's change log must hold exactly these records (compared as
sorted sets, bit-exact).  The host–DUT loop reads registers after every
cycle and derives the next cycle's input words and register pokes from them;
the oracle runs the same loop.
"""
import sys

import numpy as np
import pytest

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from tests.gpu_util import assert_same, gpu_ctx

pytestmark = pytest.mark.gpu

MAPS = [R.RTEAAL_MAP_RESIDENT, R.RTEAAL_MAP_SWEEP, R.RTEAAL_MAP_LAYERED]
MAP_IDS = ["resident", "sweep", "layered"]


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    R.rteaal_destroy(c)


@pytest.fixture(scope="module")
def design():
    return rtlgen.generate(rtlgen.GenConfig(3_000, 10, 48, 8, rtlgen.generator.WIDTHS_LARGE, "w3k"), 31)


def pick_slots(d):
    """Registers, inputs and operation outputs of every width class."""
    w = d.slot_width.astype(np.int64)
    ops = d.op_dst.astype(np.int64)
    out = list(d.reg_slot[:6]) + list(d.input_slot[:3])
    for lo, hi in ((1, 1), (2, 8), (9, 16), (17, 32), (33, 64), (65, 256)):
        out += [int(s) for s in ops[(w[ops] >= lo) & (w[ops] <= hi)][:4]]
    return np.array(out, np.uint32)


def oracle_changes(d, seeds, n_cycles, slots):
    prev = np.zeros((len(seeds), len(slots), 4), np.uint64)
    regs, out = None, set()
    for c in range(n_cycles):
        regs, sl, _ = oracle.run(d, seeds, 1, start_cycle=c, init_regs=regs, want_slots=True)
        cur = sl[:, slots.astype(np.int64), :]
        for j, k in zip(*np.nonzero((cur != prev).any(axis=2))):
            out.add((c + 1, int(j), int(k), tuple(int(x) for x in cur[j, k])))
        prev = cur
    return out


def as_set(recs):
    return {(int(r["cycle"]), int(r["instance"]), int(r["signal"]), tuple(int(x) for x in r["value"]))
            for r in recs}


@pytest.mark.parametrize("mapping", MAPS, ids=MAP_IDS)
def test_changes_match_oracle(ctx, design, mapping):
    d = design
    slots = pick_slots(d)
    seeds = rtlgen.instance_seeds(70)
    did = R.rteaal_load_design(ctx, d, keep_all_slots=True)
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping)
    try:
        R.rteaal_watch(ctx, bid, slots, capacity=1 << 20)
        got = set()
        for k in (5, 1, 10, 14):                     # drained between steps
            R.rteaal_step(ctx, bid, k)
            recs, dropped = R.rteaal_read_changes(ctx, bid)
            assert dropped == 0
            got |= as_set(recs)
        note(f"waveform mapping={mapping}: {len(got)} transitions of {slots.size} signals")
        ref = oracle_changes(d, seeds, 30, slots)
        assert len(ref) > 1000
        assert got == ref
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


def test_compact_design_registers_and_overflow(ctx, design):
    d = design
    seeds = rtlgen.instance_seeds(40)
    did = R.rteaal_load_design(ctx, d)                # live-range layout
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=R.RTEAAL_MAP_SWEEP)
    try:
        with pytest.raises(R.RteaalError) as e:
            R.rteaal_watch(ctx, bid, [int(d.op_dst[5])])
        assert e.value.status == 7
        with pytest.raises(R.RteaalError) as e:
            R.rteaal_watch(ctx, bid, [d.slot_width.size])
        assert e.value.status == 1
        regs = np.asarray(d.reg_slot, np.uint32)
        R.rteaal_watch(ctx, bid, regs, capacity=1 << 16)
        R.rteaal_step(ctx, bid, 12)
        recs, dropped = R.rteaal_read_changes(ctx, bid)
        ref = oracle_changes(d, seeds, 12, regs)
        assert dropped == 0 and as_set(recs) == ref
        # a small log keeps some records and counts the rest
        R.rteaal_watch(ctx, bid, regs, capacity=100)
        R.rteaal_step(ctx, bid, 8)
        recs, dropped = R.rteaal_read_changes(ctx, bid)
        full = {r for r in oracle_changes(d, seeds, 20, regs) if r[0] > 12}
        assert len(recs) == 100 and dropped == len(full) - 100
        assert as_set(recs) <= full
        R.rteaal_watch(ctx, bid, [])                 # stop; reading is then an error
        with pytest.raises(R.RteaalError):
            R.rteaal_read_changes(ctx, bid)
        R.rteaal_step(ctx, bid, 2)
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)


def test_step_many_with_a_watched_resident_batch(ctx, design):
    d = design
    s1, s2 = rtlgen.instance_seeds(9, design_index=1), rtlgen.instance_seeds(100, design_index=2)
    did = R.rteaal_load_design(ctx, d, keep_all_slots=True)
    b1 = R.rteaal_create_batch(ctx, did, s1, mapping=R.RTEAAL_MAP_RESIDENT)
    b2 = R.rteaal_create_batch(ctx, did, s2, mapping=R.RTEAAL_MAP_RESIDENT)
    try:
        slots = pick_slots(d)
        R.rteaal_watch(ctx, b1, slots)
        R.rteaal_step_many(ctx, [b1, b2], [7, 9])
        R.rteaal_sync(ctx)
        recs, _ = R.rteaal_read_changes(ctx, b1)
        assert as_set(recs) == oracle_changes(d, s1, 7, slots)
        wr = d.slot_width[d.reg_slot]
        assert_same(R.unpack_limbs(R.rteaal_read_state(ctx, b2), wr), oracle.run(d, s2, 9)[0], "b2")
        assert_same(R.unpack_limbs(R.rteaal_read_state(ctx, b1), wr), oracle.run(d, s1, 7)[0], "b1")
    finally:
        R.rteaal_free_batch(ctx, b1)
        R.rteaal_free_batch(ctx, b2)
        R.rteaal_unload_design(ctx, did)


@pytest.mark.parametrize("mapping", MAPS, ids=MAP_IDS)
def test_host_dut_loop(ctx, design, mapping):
    """Each cycle the host reads the registers, writes the next input words
    from them and, every third cycle, pokes register 0 (a host-side responder
    in the style of a debug-module interface)."""
    d = design
    n_inst, n_cycles = 65, 24
    seeds = rtlgen.instance_seeds(n_inst)
    wr = d.slot_width[d.reg_slot]
    W = int(((d.slot_width[d.input_slot].astype(np.int64) + 63) // 64).sum())

    def respond(regs, c):
        acc = regs[:, :, 0].sum(axis=1, dtype=np.uint64)
        words = np.empty((n_inst, W), np.uint64)
        for k in range(W):
            words[:, k] = acc * np.uint64(2 * k + 3) + np.uint64(c)
        return words[None]

    did = R.rteaal_load_design(ctx, d)
    bid = R.rteaal_create_batch(ctx, did, seeds, mapping=mapping)
    try:
        g_regs = np.zeros((n_inst, d.reg_slot.size, 4), np.uint64)
        o_regs = None
        for c in range(n_cycles):
            words = respond(g_regs, c)
            R.rteaal_step(ctx, bid, 1, words=words)
            g_regs = R.unpack_limbs(R.rteaal_read_state(ctx, bid), wr)
            o_regs, _, _ = oracle.run(d, seeds, 1, start_cycle=c, stim_words=words, init_regs=o_regs)
            assert_same(g_regs, o_regs, f"cycle {c}")
            if c % 3 == 2:                               # host pokes register 0
                poke = g_regs.copy()
                poke[:, 0, 0] = np.uint64(0x5A5A) + np.uint64(c)
                mask = (1 << int(wr[0])) - 1 if wr[0] < 64 else (1 << 64) - 1
                poke[:, 0, 0] &= np.uint64(mask)
                R.rteaal_write_state(ctx, bid, 0, R.pack_limbs(poke, wr), c + 1)
                g_regs = poke
                o_regs = poke.copy()
        note(f"host-DUT loop mapping={mapping}: {n_cycles} cycles")
    finally:
        R.rteaal_free_batch(ctx, bid)
        R.rteaal_unload_design(ctx, did)
