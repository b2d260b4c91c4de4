"""Pins for the CPU oracle (no GPU).

The oracle is trusted only through these checks, none of which re-uses its
code: exhaustive truth tables against the integer definitions of the
operation types, hand-derived examples, circuits with closed-form behaviour
(ripple-carry adder, counter, maximal LFSR, the prefix-sum iterative rank,
a shift-register chain, the paper's single-multiply example), a published
test vector of the stimulus generator, and invariants of the method.
"""
import itertools
import os
import random

import numpy as np
import pytest

import rtlgen
from rtlgen import circuits as cir
from rtlgen.design import (ADD, AND, ANDR, CONCAT, DIV, DSHL, DSHR, EQ, EXTRACT, LT, MUL, MUX, NOT,
                           OR, ORR, REM, SEXT, SHL, SHR, SUB, XOR, XORR, limbs_to_int)
from tests.intref import textbook

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NAME2OP = {n: i for i, n in enumerate(rtlgen.OP_NAMES)}


ARITIES = [(AND, 2), (AND, 3), (OR, 2), (OR, 3), (XOR, 2), (XOR, 3), (NOT, 1), (ADD, 2),
           (SUB, 2), (MUL, 2), (MUX, 3), (EQ, 2), (LT, 2), (SHL, 1), (SHR, 1), (EXTRACT, 1),
           (CONCAT, 2), (ORR, 1), (DIV, 2), (REM, 2), (DSHL, 2), (DSHR, 2), (ANDR, 1), (XORR, 1),
           (SEXT, 1)]


@pytest.mark.parametrize("typ,arity", ARITIES, ids=[f"{rtlgen.OP_NAMES[t]}{a}" for t, a in ARITIES])
def test_truth_tables_small_widths(oracle_lib, typ, arity):
    """Every operand value at operand widths 1..4 (1..3 for 3 operands), dst widths 1..4."""
    maxw = 4 if arity < 3 else 3
    n = 0
    for ws in itertools.product(range(1, maxw + 1), repeat=arity):
        imms = range(0, ws[0] + 2) if typ in (SHL, SHR, EXTRACT) else (0,)
        for wd in range(1, 5):
            for imm in imms:
                for vals in itertools.product(*[range(1 << w) for w in ws]):
                    got = oracle_lib.eval_op(typ, vals, ws, wd, imm)
                    assert got == textbook(typ, vals, ws, wd, imm), (typ, vals, ws, wd, imm)
                    n += 1
    assert n > 0


@pytest.mark.parametrize("typ,arity", ARITIES, ids=[f"{rtlgen.OP_NAMES[t]}{a}" for t, a in ARITIES])
def test_wide_operands_random(oracle_lib, typ, arity):
    """Operands and results of 1..256 bits, including limb boundaries."""
    rng = random.Random(1000 + typ * 7 + arity)
    edge = [1, 2, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256]
    for _ in range(400):
        ws = [rng.choice(edge + [rng.randint(1, 256)]) for _ in range(arity)]
        wd = rng.choice(edge + [rng.randint(1, 256)])
        vals = []
        for w in ws:
            kind = rng.random()
            if kind < 0.15:
                vals.append((1 << w) - 1)
            elif kind < 0.25:
                vals.append(0)
            else:
                vals.append(rng.getrandbits(w))
        imm = rng.randint(0, 255) if typ in (SHL, SHR, EXTRACT) else 0
        if typ == MUX and rng.random() < 0.5:
            vals[0] = 0
        got = oracle_lib.eval_op(typ, vals, ws, wd, imm)
        assert got == textbook(typ, vals, ws, wd, imm), (typ, vals, ws, wd, imm)


def test_added_types_edges(oracle_lib):
    """Dynamic shifts by small amounts of wide values, divisors of 255-256
    bits (the long division's top bit), sign extension across limb
    boundaries, and ANDR of all-ones values."""
    rng = random.Random(77)
    edge = [1, 2, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256]
    for _ in range(300):
        w0, wd = rng.choice(edge), rng.choice(edge)
        a = rng.getrandbits(w0)
        k = rng.randint(0, 300)
        for typ in (DSHL, DSHR):
            assert oracle_lib.eval_op(typ, (a, k), (w0, 9), wd, 0) == textbook(typ, (a, k), (w0, 9), wd, 0)
        for typ in (SEXT, ANDR):
            for x in (a, (1 << w0) - 1, 1 << (w0 - 1), (1 << (w0 - 1)) - 1):
                assert oracle_lib.eval_op(typ, (x,), (w0,), wd, 0) == textbook(typ, (x,), (w0,), wd, 0)
    for _ in range(300):
        b = (1 << 255) | rng.getrandbits(255) if rng.random() < 0.5 else (1 << 256) - 1 - rng.getrandbits(8)
        a = (1 << 256) - 1 - rng.getrandbits(rng.choice([8, 64, 200, 256]))
        for typ in (DIV, REM):
            assert oracle_lib.eval_op(typ, (a, b), (256, 256), 256, 0) == textbook(typ, (a, b), (256, 256), 256, 0)


def test_hand_examples(oracle_lib):
    n = 0
    with open(os.path.join(GOLDEN, "hand_examples.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, wd, ops, imm, exp = line.split()
            ws, vals = zip(*[(int(p.split(":")[0]), int(p.split(":")[1])) for p in ops.split(",")])
            assert oracle_lib.eval_op(NAME2OP[name], vals, ws, int(wd), int(imm)) == int(exp), line
            n += 1
    assert n >= 15


def test_splitmix64_published_vector(oracle_lib):
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        exp = [int(x) for x in f if x.strip() and not x.startswith("#")]
    state = 1234567
    for k, e in enumerate(exp):
        assert oracle_lib.splitmix64((state + k * 0x9E3779B97F4A7C15) % (1 << 64)) == e


def test_stimulus_composition_and_masking(oracle_lib):
    sm = oracle_lib.splitmix64
    for seed, cyc, k, limb in [(0, 0, 0, 0), (5, 17, 3, 1), (2**63, 2**40, 255, 3)]:
        assert oracle_lib.stim(seed, cyc, k, limb) == sm(sm(sm(seed) ^ cyc) ^ ((k << 8) | limb))
    b = cir.Builder("pi")
    ins = [b.input(w) for w in (1, 7, 64, 65, 200)]
    r = b.reg(1)
    b.connect(r, ins[0])
    d = b.build()
    _, slots, _ = oracle_lib.run(d, [9], 3, want_slots=True, start_cycle=40)
    for k, s in enumerate(ins):
        w = int(d.slot_width[s])
        full = sum(oracle_lib.stim(9, 42, k, l) << (64 * l) for l in range((w + 63) // 64))
        assert limbs_to_int(slots[0, s]) == full % (1 << w)


def _words(vals_per_cycle, widths):
    """Buffer-mode stimulus [n_cycles][1][sum limbs] from Python ints."""
    rows = []
    for vals in vals_per_cycle:
        row = []
        for v, w in zip(vals, widths):
            row += [(v >> (64 * l)) & ((1 << 64) - 1) for l in range((w + 63) // 64)]
        rows.append([row])
    return np.array(rows, dtype=np.uint64)


@pytest.mark.parametrize("w", [1, 2, 3, 4, 5, 6])
def test_ripple_carry_adder_exhaustive(oracle_lib, w):
    d = cir.ripple_carry_adder(w)
    pairs = list(itertools.product(range(1 << w), repeat=2))
    _, _, tr = oracle_lib.run(d, [0], len(pairs), stim_words=_words(pairs, [w, w]), trace_reg=0)
    assert [int(x) for x in tr[0]] == [a + b for a, b in pairs]


@pytest.mark.parametrize("w", [31, 64, 65, 128, 200, 255])
def test_ripple_carry_adder_wide(oracle_lib, w):
    rng = random.Random(w)
    d = cir.ripple_carry_adder(w)
    pairs = [(rng.getrandbits(w), rng.getrandbits(w)) for _ in range(6)] + [((1 << w) - 1, 1)]
    words = np.concatenate([_words([p], [w, w]) for p in pairs], axis=1)
    regs, _, _ = oracle_lib.run(d, np.zeros(len(pairs)), 1, stim_words=words)
    for i, (a, b) in enumerate(pairs):
        assert limbs_to_int(regs[i, 0]) == a + b


@pytest.mark.parametrize("w,step", [(1, 1), (3, 1), (8, 1), (64, 1), (65, 2**64 - 1),
                                    (130, 3**70), (256, 2**255 + 12345)])
def test_counter_closed_form(oracle_lib, w, step):
    d = cir.counter(w, step % (1 << w))
    regs, _, _ = oracle_lib.run(d, [0], 777)
    assert limbs_to_int(regs[0, 0]) == (777 * step) % (1 << w)


@pytest.mark.parametrize("n", list(range(3, 21)))
def test_xnor_lfsr_maximal_period(oracle_lib, n):
    d = cir.xnor_lfsr(n)
    P = (1 << n) - 1
    _, _, tr = oracle_lib.run(d, [0], P + 3, trace_reg=0)
    states = tr[0]
    zeros = np.nonzero(states == 0)[0]
    assert zeros.size and int(zeros[0]) + 1 == P          # first return to reset state
    assert len(np.unique(states[:P])) == P                 # every state visited once
    assert not np.any(states == P)                         # never the all-ones lock-up state


def test_prefix_sum_iterative_rank(oracle_lib):
    rng = random.Random(3)
    n, w = 16, 12
    rows = [[rng.getrandbits(w) for _ in range(n)] for _ in range(50)]
    d = cir.prefix_sum_chain(n, w)
    _, _, tr = oracle_lib.run(d, [0], len(rows), stim_words=_words(rows, [w] * n), trace_reg=0)
    assert [int(x) for x in tr[0]] == [sum(r) % (1 << w) for r in rows]


@pytest.mark.parametrize("reverse", [False, True])
def test_register_commit_is_simultaneous(oracle_lib, reverse):
    depth, w, cycles = 4, 8, 10
    xs = [[random.Random(c).getrandbits(w)] for c in range(cycles)]
    d = cir.shift_chain(depth, w, reverse=reverse)
    regs, _, _ = oracle_lib.run(d, [0], cycles, stim_words=_words(xs, [w]))
    order = list(range(depth))[::-1] if reverse else list(range(depth))
    for j, k in enumerate(order):
        assert limbs_to_int(regs[0, j]) == xs[cycles - 1 - k][0]


def test_paper_single_multiply_example(oracle_lib):
    regs, _, _ = oracle_lib.run(cir.paper_multiply_example(), [0], 1)
    assert limbs_to_int(regs[0, 0]) == 4


# ---------------------------------------------------------------------------
# Invariants on generated designs.
# ---------------------------------------------------------------------------
SMALL = rtlgen.GenConfig(600, 8, 40, 12, rtlgen.generator.WIDTHS_LARGE, "small-wide")


@pytest.fixture(scope="module")
def small_design():
    return rtlgen.generate(SMALL, 11)


def test_every_slot_within_width(oracle_lib, small_design):
    d = small_design
    _, slots, _ = oracle_lib.run(d, [1, 2, 3], 25, want_slots=True)
    for s in range(d.n_slots):
        w = int(d.slot_width[s])
        for i in range(3):
            assert limbs_to_int(slots[i, s]) < (1 << w)


def test_reset_state_is_zero(oracle_lib, small_design):
    regs, _, _ = oracle_lib.run(small_design, [1, 2], 0)
    assert not regs.any()


def test_permuting_ops_within_layers(oracle_lib, small_design):
    a, _, _ = oracle_lib.run(small_design, [4, 5], 30)
    b, _, _ = oracle_lib.run(small_design.permuted_within_layers(99), [4, 5], 30)
    assert np.array_equal(a, b)


def test_step_splitting(oracle_lib, small_design):
    full, _, _ = oracle_lib.run(small_design, [7, 8], 40)
    half, _, _ = oracle_lib.run(small_design, [7, 8], 17)
    rest, _, _ = oracle_lib.run(small_design, [7, 8], 23, start_cycle=17, init_regs=half)
    assert np.array_equal(full, rest)


def test_instances_are_independent(oracle_lib, small_design):
    both, _, _ = oracle_lib.run(small_design, [3, 1000, 77], 20)
    for i, s in enumerate([3, 1000, 77]):
        one, _, _ = oracle_lib.run(small_design, [s], 20)
        assert np.array_equal(both[i], one[0])


def test_state_depends_on_seed_and_evolves(oracle_lib, small_design):
    a, _, _ = oracle_lib.run(small_design, [1, 2], 20)
    assert not np.array_equal(a[0], a[1])
    assert a.any()
