"""Pins for the oracle's per-instance register digest (no GPU).

The digest is this library's reading of what "state" is compared: after
every cycle's register commit, h = sum over registers j and limbs l of
s(s(4 j + l) ^ limb) mod 2^64 and D = s(D ^ h), s being SplitMix64's output
function (pinned to its published test vector in test_oracle_pins.py).  The
register values it is folded over come here from sources other than the
oracle: closed forms (a counter, a swap, a design without registers) and the
independent Python interpreter; a digest taken before the commit, a dropped
limb or register, or a wrong key fails one of them.
"""
import numpy as np
import pytest

import rtlgen
from rtlgen import circuits as cir
from tests.intref import digest_step, simulate, splitmix64

M64 = (1 << 64) - 1


@pytest.mark.parametrize("w,step", [(1, 1), (7, 3), (64, 2**64 - 1), (65, 2**64 + 5),
                                    (200, 3**100), (256, 2**255 + 1)])
def test_digest_counter_closed_form(oracle_lib, w, step):
    """r <- r + step: after cycle t (0-based) r = (t + 1) step mod 2^w."""
    d = cir.counter(w, step % (1 << w))
    n = 40
    dg = {}
    oracle_lib.run(d, [0], n, digests=dg, digest_trace=True)
    D, want = 0, []
    for t in range(n):
        D = digest_step(D, [((t + 1) * step) % (1 << w)], [w])
        want.append(D)
    assert [int(x) for x in dg["trace"][0]] == want
    assert int(dg["final"][0]) == want[-1]


def test_digest_without_registers(oracle_lib):
    """No registers: h = 0 every cycle, so D after n cycles is s applied n times to 0."""
    b = cir.Builder("no-regs")
    x = b.input(5)
    b.op(cir.NOT, [x], 5)
    d = b.build()
    dg = {}
    oracle_lib.run(d, [3], 25, digests=dg, digest_trace=True)
    D = 0
    for t in range(25):
        D = splitmix64(D)
        assert int(dg["trace"][0, t]) == D


def test_digest_sees_the_committed_values(oracle_lib):
    """A two-register swap from a known state: (a, b) -> (b, a) each cycle,
    so the digest of cycle t folds the values after the swap, keyed by
    register index (a digest of the values before the commit, or one that
    ignored the key, would be the other order's)."""
    b = cir.Builder("swap")
    ra, rb = b.reg(70), b.reg(70)
    b.connect(ra, rb)
    b.connect(rb, ra)
    d = b.build()
    a0, b0 = (1 << 69) + 12345, 987654321
    init = np.zeros((1, 2, 4), np.uint64)
    for j, v in enumerate((a0, b0)):
        for l in range(2):
            init[0, j, l] = (v >> (64 * l)) & M64
    dg = {}
    oracle_lib.run(d, [0], 6, init_regs=init, digests=dg, digest_trace=True)
    D, cur = 0, (a0, b0)
    for t in range(6):
        cur = (cur[1], cur[0])
        D = digest_step(D, list(cur), [70, 70])
        assert int(dg["trace"][0, t]) == D
    # the key separates the two orders
    assert digest_step(0, [a0, b0], [70, 70]) != digest_step(0, [b0, a0], [70, 70])


CASES = [
    rtlgen.GenConfig(120, 5, 10, 6, rtlgen.generator.WIDTHS_STD, "tiny-std"),
    rtlgen.GenConfig(150, 7, 12, 5, rtlgen.generator.WIDTHS_LARGE, "tiny-wide"),
    rtlgen.GenConfig(160, 6, 10, 6, rtlgen.generator.WIDTHS_LARGE, "tiny-all-types",
                     rtlgen.OP_MIX_FULL),
]


@pytest.mark.parametrize("cfg", CASES, ids=[c.name for c in CASES])
def test_digest_against_python_interpreter(oracle_lib, cfg):
    """Per-cycle digests of generated designs (registers up to 256 bits)
    equal the Python fold over the independent interpreter's registers."""
    d = rtlgen.generate(cfg, 1)
    seeds = [11, 12]
    dg = {}
    oracle_lib.run(d, seeds, 10, start_cycle=3, digests=dg, digest_trace=True)
    widths = [int(d.slot_width[s]) for s in d.reg_slot]
    for i, s in enumerate(seeds):
        want = []
        state = {"D": 0}

        def on_cycle(t, V):
            state["D"] = digest_step(state["D"], [V[int(r)] for r in d.reg_slot], widths)
            want.append(state["D"])

        simulate(d, s, 10, start_cycle=3, on_cycle=on_cycle)
        assert [int(x) for x in dg["trace"][i]] == want


def test_digest_continues_across_runs(oracle_lib):
    """A run split in two (registers and digest carried over) gives the
    whole run's digest: the chain depends only on the register sequence."""
    d = rtlgen.generate(CASES[1], 4)
    seeds = [5, 6, 7]
    whole = {}
    regs_all, _, _ = oracle_lib.run(d, seeds, 17, digests=whole)
    first = {}
    regs_a, _, _ = oracle_lib.run(d, seeds, 9, digests=first)
    second = {}
    regs_b, _, _ = oracle_lib.run(d, seeds, 8, start_cycle=9, init_regs=regs_a,
                                  init_digest=first["final"], digests=second)
    assert np.array_equal(regs_b, regs_all)
    assert np.array_equal(second["final"], whole["final"])
    assert not np.array_equal(first["final"], whole["final"])
