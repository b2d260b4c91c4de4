"""Pins for the fused mux-chain type MUXC and the oracle's mux-chain fusion.

MUXC (o0, o1, ..., o2k) is pinned against the integer definition (first
nonzero selector's value, else the last operand) and against MUX for one
pair.  The fusion pass is pinned by exact results on hand-built chains (the
pieces and operand lists the chain reading fixes, and the links each rule
must refuse) and by equivalence: the fused design, run by the oracle, gives
the unfused design's values in every register and every slot it still
writes, on generated designs full of chains, including links that break
each rule.  A naive interpreter cross-checks the oracle on a fused design.
"""
import random

import numpy as np
import pytest

import oracle
import rtlgen
from rtlgen import circuits as cir
from rtlgen.design import AND, MUX, MUXC
from tests.intref import simulate, textbook


def test_muxc_matches_definition_and_mux():
    rng = random.Random(11)
    for _ in range(400):
        k = rng.choice([1, 2, 3, 5, 16, 32])
        wd = rng.choice([1, 3, 8, 33, 64, 65, 200, 256])
        ws, vals = [], []
        for _ in range(k):
            w = rng.choice([1, 2, 64, 100])
            ws.append(w)
            vals.append(rng.getrandbits(w) if rng.random() < 0.3 else 0)
            w = rng.choice([1, 8, 64, 256])
            ws.append(w)
            vals.append(rng.getrandbits(w))
        w = rng.choice([1, 64, 256])
        ws.append(w)
        vals.append(rng.getrandbits(w))
        got = oracle.eval_op(MUXC, vals, ws, wd)
        assert got == textbook(MUXC, vals, ws, wd, 0)
        if k == 1:
            assert got == oracle.eval_op(MUX, vals, ws, wd)
    # every selector pattern of three pairs: the first nonzero one wins
    for pat in range(8):
        sel = [(pat >> i) & 1 for i in range(3)]
        vals = [sel[0], 10, sel[1], 20, sel[2], 30, 40]
        exp = next((v for s, v in zip(sel, (10, 20, 30)) if s), 40)
        assert oracle.eval_op(MUXC, vals, [1, 8, 1, 8, 1, 8, 8], 8) == exp


def test_muxc_arity_bounds():
    for ar in (2, 4, 67):
        with pytest.raises(ValueError):
            oracle.eval_op(MUXC, [1] * ar, [8] * ar, 8)
    assert oracle.eval_op(MUXC, [0] * 64 + [7], [1] * 64 + [8], 8) == 7


def chain(variant="plain"):
    """m1 = s1 ? a : m2, m2 = s2 ? b : m3, m3 = s3 ? c : m4, m4 = s4 ? d : e."""
    b = cir.Builder(variant)
    s = [b.input(1) for _ in range(4)]
    a, bb, c, dd, e = (b.input(8) for _ in range(5))
    m4 = b.op(MUX, [s[3], dd, e], 8)
    m3 = b.op(MUX, [s[2], c, m4], 4 if variant == "narrow" else 8)
    m2 = b.op(MUX, [s[1], bb, m3], 8)
    m1 = b.op(MUX, [s[0], a, m2], 8)
    r = b.reg(8)
    b.connect(r, m1)
    if variant == "fanout":
        r2 = b.reg(8)
        b.connect(r2, b.op(AND, [m3, a], 8))
    if variant == "latched":
        r2 = b.reg(8)
        b.connect(r2, m3)
    return b.build(), (s, a, bb, c, dd, e), (m1, m2, m3, m4)


def fused_ops(f):
    out = {}
    for o in range(f.n_ops):
        srcs = [int(x) for x in f.op_src[f.op_src_ptr[o]:f.op_src_ptr[o + 1]]]
        out[int(f.op_dst[o])] = (int(f.op_type[o]), srcs)
    return out


def same_values(d, f, n_seeds=64, cycles=3):
    seeds = rtlgen.instance_seeds(n_seeds)
    r0, s0, _ = oracle.run(d, seeds, cycles, want_slots=True)
    r1, s1, _ = oracle.run(f, seeds, cycles, want_slots=True)
    alive = f.op_dst.astype(np.int64)
    return np.array_equal(r0, r1) and np.array_equal(s0[:, alive], s1[:, alive])


@pytest.mark.parametrize("max_pairs", [32, 4, 3, 2, 1])
def test_hand_chain_pieces(max_pairs):
    d, (s, a, b, c, dd, e), (m1, m2, m3, m4) = chain()
    f, n_fused, n_abs = oracle.fuse_mux_chains(d, max_pairs)
    ops = fused_ops(f)
    full = [s[0], a, s[1], b, s[2], c, s[3], dd, e]
    exp = {
        32: {m1: (MUXC, full)},
        4: {m1: (MUXC, full)},
        3: {m1: (MUXC, [s[0], a, s[1], b, s[2], c, m4]), m4: (MUX, [s[3], dd, e])},
        2: {m1: (MUXC, [s[0], a, s[1], b, m3]), m3: (MUXC, [s[2], c, s[3], dd, e])},
        1: {m1: (MUX, [s[0], a, m2]), m2: (MUX, [s[1], b, m3]), m3: (MUX, [s[2], c, m4]),
            m4: (MUX, [s[3], dd, e])},
    }[max_pairs]
    assert ops == exp
    assert n_abs == 4 - len(exp) and n_fused == sum(t == MUXC for t, _ in exp.values())
    assert f.n_layers == d.n_layers and int(f.layer_ptr[-1]) == f.n_ops
    assert same_values(d, f)


@pytest.mark.parametrize("variant", ["fanout", "latched", "narrow"])
def test_rules_refuse_the_link_into_m3(variant):
    d, (s, a, b, c, dd, e), (m1, m2, m3, m4) = chain(variant)
    f, _, _ = oracle.fuse_mux_chains(d)
    ops = fused_ops(f)
    assert ops[m1] == (MUXC, [s[0], a, s[1], b, m3])
    assert ops[m3] == (MUXC, [s[2], c, s[3], dd, e])
    assert m2 not in ops and m4 not in ops
    assert same_values(d, f)


def test_narrow_link_would_change_values():
    """Fusing through the 4-bit m3 anyway (the width rule broken by hand)
    changes the register: the equivalence check sees such a mistake."""
    d, (s, a, b, c, dd, e), (m1, m2, m3, m4) = chain("narrow")
    bad = cir.Builder("bad")
    ins = [bad.input(int(d.slot_width[x])) for x in d.input_slot]
    m = bad.op(MUXC, [ins[0], ins[4], ins[1], ins[5], ins[2], ins[6], ins[3], ins[7], ins[8]], 8)
    r = bad.reg(8)
    bad.connect(r, m)
    wrong = bad.build()
    seeds = rtlgen.instance_seeds(64)
    r0, _, _ = oracle.run(d, seeds, 2)
    r1, _, _ = oracle.run(wrong, seeds, 2)
    assert not np.array_equal(r0, r1)


@pytest.mark.parametrize("seed,max_pairs", [(1, 32), (2, 3), (3, 32)])
def test_generated_chains_keep_values(seed, max_pairs):
    cfg = rtlgen.GenConfig(30_000, 24, 600, 16, rtlgen.generator.WIDTHS_LARGE, "chains",
                           mux_chain=0.85)
    d = rtlgen.generate(cfg, seed)
    f, n_fused, n_abs = oracle.fuse_mux_chains(d, max_pairs)
    assert n_fused > 300 and n_abs > 2 * n_fused * (0.5 if max_pairs == 3 else 1)
    ar = np.diff(f.op_src_ptr)[f.op_type == MUXC]
    assert (ar % 2 == 1).all() and ar.min() >= 5 and ar.max() <= 2 * max_pairs + 1
    assert f.n_ops == d.n_ops - n_abs
    # the rules had work to do: some links were refused
    link = oracle.mux_links(d)
    producer = np.full(d.n_slots, -1, np.int64)
    producer[d.op_dst.astype(np.int64)] = np.arange(d.n_ops)
    ext = np.nonzero(d.op_type == MUX)[0]
    p = producer[d.op_src[d.op_src_ptr[ext] + 2].astype(np.int64)]
    default_is_mux = (p >= 0) & (d.op_type[np.maximum(p, 0)] == MUX)
    assert (default_is_mux & (link[ext] < 0)).sum() > 20
    assert same_values(d, f, n_seeds=16, cycles=3)


def test_interpreter_agrees_on_a_fused_design():
    cfg = rtlgen.GenConfig(400, 8, 24, 4, rtlgen.generator.WIDTHS_LARGE, "tiny-chains", mux_chain=0.9)
    d = rtlgen.generate(cfg, 7)
    f, n_fused, _ = oracle.fuse_mux_chains(d)
    assert n_fused >= 3
    _, slots, _ = oracle.run(f, [5], 4, want_slots=True)
    ref = simulate(f, 5, 4)
    got = [rtlgen.limbs_to_int(slots[0, k]) for k in range(f.n_slots)]
    assert got == ref


def priority_encoder(n=16, as_chain=False):
    """out = index of the lowest set bit among n 1-bit inputs, else 31; as one
    MUXC, or as the nested MUX chain that fusion turns into it."""
    b = cir.Builder("prio")
    bits = [b.input(1) for _ in range(n)]
    idx = [b.const(5, i) for i in range(n)]
    none = b.const(5, 31)
    if as_chain:
        out = none
        for i in reversed(range(n)):
            out = b.op(MUX, [bits[i], idx[i], out], 5)
    else:
        srcs = []
        for i in range(n):
            srcs += [bits[i], idx[i]]
        out = b.op(MUXC, srcs + [none], 5)
    r = b.reg(5)
    b.connect(r, out)
    return b.build(), bits


def test_priority_encoder_closed_form():
    """The register after one cycle is the lowest set input bit's index (31
    when none is set), from the stimulus words themselves."""
    seeds = np.arange(200, dtype=np.uint64)
    for as_chain in (False, True):
        d, bits = priority_encoder(as_chain=as_chain)
        if as_chain:
            f, n_fused, n_abs = oracle.fuse_mux_chains(d)
            assert n_fused == 1 and n_abs == 15
            m, _ = priority_encoder()
            assert [int(x) for x in f.op_src] == [int(x) for x in m.op_src]
        regs, _, _ = oracle.run(d, seeds, 1)
        for j, sd in enumerate(seeds):
            on = [k for k in range(16) if oracle.stim(int(sd), 0, k, 0) & 1]
            assert int(regs[j, 0, 0]) == (on[0] if on else 31)


def test_fused_then_levelized_keeps_values():
    """Fusion, then the oracle levelizer's layering of the fused graph: no
    more layers than before (a fused operation reads only what its absorbed
    MUXes read), every operation after its producers, and the same register
    values as the design as drawn."""
    cfg = rtlgen.GenConfig(6_000, 20, 200, 8, rtlgen.generator.WIDTHS_LARGE, "fl", mux_chain=0.9)
    d = rtlgen.generate(cfg, 9)
    f, n_fused, _ = oracle.fuse_mux_chains(d)
    assert n_fused > 50
    layer = oracle.levelize(f.n_slots, f.op_src_ptr, f.op_src, f.op_dst)
    order, lptr = oracle.layer_order(layer)
    assert len(lptr) - 1 <= d.n_layers
    o = np.asarray(order, np.int64)
    ptr = f.op_src_ptr.astype(np.int64)
    lens = np.diff(ptr)[o]
    new_ptr = np.concatenate([[0], np.cumsum(lens)])
    src = np.concatenate([f.op_src[ptr[k]:ptr[k + 1]] for k in o])
    lv = rtlgen.Design(name="fl-lv", slot_width=f.slot_width, const_slot=f.const_slot,
                       const_limbs=f.const_limbs, input_slot=f.input_slot, reg_slot=f.reg_slot,
                       reg_next=f.reg_next, layer_ptr=lptr, op_type=f.op_type[o],
                       op_dst=f.op_dst[o], op_src_ptr=new_ptr, op_src=src, op_imm=f.op_imm[o])
    seeds = rtlgen.instance_seeds(12)
    r0, _, _ = oracle.run(d, seeds, 4)
    r1, _, _ = oracle.run(lv, seeds, 4)
    assert np.array_equal(r0, r1)
