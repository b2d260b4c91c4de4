"""Hand-built circuits whose behaviour has a closed form.

`Builder` places each operation in the earliest layer after all of its
operands (levelization by longest path), so circuits can be written in any
order.  The circuits below are structure only; what they compute is stated
in each docstring and checked by the tests against plain integer formulas.
"""
from __future__ import annotations

import numpy as np

from .design import (ADD, AND, CONCAT, EXTRACT, MUL, NOT, OR, XOR, Design, int_to_limbs)


class Builder:
    def __init__(self, name="circuit"):
        self.name = name
        self.width = []       # per slot
        self.level = []       # -1 for sources (inputs, registers, constants)
        self.inputs, self.regs, self.reg_next = [], [], []
        self.consts, self.const_vals = [], []
        self.ops = []         # (type, dst, srcs, imm)

    def _slot(self, w, level):
        assert 1 <= w <= 256
        self.width.append(int(w))
        self.level.append(level)
        return len(self.width) - 1

    def input(self, w):
        s = self._slot(w, -1)
        self.inputs.append(s)
        return s

    def reg(self, w):
        s = self._slot(w, -1)
        self.regs.append(s)
        self.reg_next.append(None)
        return s

    def const(self, w, value):
        s = self._slot(w, -1)
        self.consts.append(s)
        self.const_vals.append(int(value) % (1 << w))
        return s

    def connect(self, reg, nxt):
        self.reg_next[self.regs.index(reg)] = nxt

    def op(self, typ, srcs, w, imm=0):
        lvl = 1 + max(self.level[s] for s in srcs)
        d = self._slot(w, lvl)
        self.ops.append((typ, d, list(srcs), int(imm)))
        return d

    def build(self) -> Design:
        assert all(n is not None for n in self.reg_next), "unconnected register"
        ops = sorted(self.ops, key=lambda o: self.level[o[1]])
        n_layers = max((self.level[o[1]] for o in ops), default=-1) + 1
        layer_ptr = np.zeros(n_layers + 1, np.int64)
        for o in ops:
            layer_ptr[self.level[o[1]] + 1] += 1
        layer_ptr = np.cumsum(layer_ptr)
        src_ptr = np.zeros(len(ops) + 1, np.int64)
        src_ptr[1:] = np.cumsum([len(o[2]) for o in ops])
        return Design(
            name=self.name, slot_width=np.array(self.width),
            const_slot=np.array(self.consts, np.int64),
            const_limbs=np.array([int_to_limbs(v) for v in self.const_vals], np.uint64).reshape(-1, 4),
            input_slot=np.array(self.inputs, np.int64), reg_slot=np.array(self.regs, np.int64),
            reg_next=np.array(self.reg_next, np.int64), layer_ptr=layer_ptr,
            op_type=np.array([o[0] for o in ops], np.int64),
            op_dst=np.array([o[1] for o in ops], np.int64), op_src_ptr=src_ptr,
            op_src=np.array([s for o in ops for s in o[2]], np.int64),
            op_imm=np.array([o[3] for o in ops], np.int64),
        )


def ripple_carry_adder(w: int) -> Design:
    """Inputs a, b (w bits); register `sum` (w+1 bits) latches a + b.

    Built only from 1-bit AND/OR/XOR full adders over EXTRACTed bits,
    reassembled with CONCAT, so after any cycle the register equals the
    integer sum of that cycle's inputs.
    """
    b = Builder(f"rca{w}")
    a_in, b_in = b.input(w), b.input(w)
    out = b.reg(w + 1)
    carry = None
    acc = None
    for k in range(w):
        ak = b.op(EXTRACT, [a_in], 1, imm=k)
        bk = b.op(EXTRACT, [b_in], 1, imm=k)
        if carry is None:
            s = b.op(XOR, [ak, bk], 1)
            carry = b.op(AND, [ak, bk], 1)
        else:
            s = b.op(XOR, [ak, bk, carry], 1)
            g = b.op(AND, [ak, bk], 1)
            p = b.op(XOR, [ak, bk], 1)
            carry = b.op(OR, [g, b.op(AND, [p, carry], 1)], 1)
        acc = s if acc is None else b.op(CONCAT, [s, acc], k + 1)
    b.connect(out, b.op(CONCAT, [carry, acc], w + 1))
    return b.build()


def counter(w: int, step: int = 1) -> Design:
    """Register r (w bits) with r <- r + step; after n cycles r = n*step mod 2^w."""
    b = Builder(f"counter{w}")
    r = b.reg(w)
    one = b.const(w, step)
    b.connect(r, b.op(ADD, [r, one], w))
    return b.build()


# Feedback taps (1-based bit positions) of maximal-length shift registers.
LFSR_TAPS = {
    3: (3, 2), 4: (4, 3), 5: (5, 3), 6: (6, 5), 7: (7, 6), 8: (8, 6, 5, 4), 9: (9, 5),
    10: (10, 7), 11: (11, 9), 12: (12, 6, 4, 1), 13: (13, 4, 3, 1), 14: (14, 5, 3, 1),
    15: (15, 14), 16: (16, 15, 13, 4), 17: (17, 14), 18: (18, 11), 19: (19, 6, 2, 1),
    20: (20, 17),
}


def xnor_lfsr(n: int) -> Design:
    """n-bit Fibonacci shift register with XNOR feedback, reset state 0.

    new r = ((r mod 2^(n-1)) << 1) | XNOR(taps); maximal taps give period 2^n - 1.
    """
    taps = LFSR_TAPS[n]
    b = Builder(f"lfsr{n}")
    r = b.reg(n)
    bits = [b.op(EXTRACT, [r], 1, imm=t - 1) for t in taps]
    x = bits[0]
    rest = bits[1:]
    while rest:
        grp, rest = rest[:2], rest[2:]
        x = b.op(XOR, [x] + grp, 1)
    fb = b.op(NOT, [x], 1)
    low = b.op(EXTRACT, [r], n - 1, imm=0)
    b.connect(r, b.op(CONCAT, [low, fb], n))
    return b.build()


def prefix_sum_chain(n_terms: int, w: int) -> Design:
    """Iterative-rank example: S_{i+1} = S_i + A_i with S_0 = 0.

    Inputs A_0..A_{n-1}; register `s` latches S_n = sum(A) mod 2^w.
    """
    b = Builder(f"prefix{n_terms}x{w}")
    A = [b.input(w) for _ in range(n_terms)]
    s = b.const(w, 0)
    for a in A:
        s = b.op(ADD, [s, a], w)
    out = b.reg(w)
    b.connect(out, s)
    return b.build()


def shift_chain(depth: int, w: int, reverse: bool = False) -> Design:
    """Input x feeds r_0 <- x, r_k <- r_{k-1}: r_k after cycle c equals x from cycle c-k.

    `reverse` lists the registers last-to-first, so a commit that is not
    simultaneous would fail in one of the two orders.
    """
    b = Builder(f"shift{depth}x{w}")
    x = b.input(w)
    regs = [b.reg(w) for _ in range(depth)]
    order = list(range(depth))[::-1] if reverse else list(range(depth))
    for k in order:
        b.connect(regs[k], x if k == 0 else regs[k - 1])
    if reverse:
        b.regs = [regs[k] for k in order]
        b.reg_next = [x if k == 0 else regs[k - 1] for k in order]
    return b.build()


def paper_multiply_example() -> Design:
    """Single multiply over register inputs 1, 2 and 4 (section "Evaluating a
    Single Operation"): operands are the first and third inputs, product 4."""
    b = Builder("paper-mul")
    li = [b.const(8, 1), b.const(8, 2), b.const(8, 4)]
    out = b.reg(8)
    b.connect(out, b.op(MUL, [li[0], li[2]], 8))
    return b.build()


def single_op(typ, src_widths, dst_w, imm=0) -> Design:
    """One operation over fresh primary inputs; register `out` latches it."""
    b = Builder("single")
    ins = [b.input(w) for w in src_widths]
    out = b.reg(dst_w)
    b.connect(out, b.op(typ, ins, dst_w, imm))
    return b.build()


__all__ = ["Builder", "ripple_carry_adder", "counter", "xnor_lfsr", "prefix_sum_chain",
           "shift_chain", "paper_multiply_example", "single_op", "LFSR_TAPS", "NOT", "OR", "AND"]
