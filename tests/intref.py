"""Integer definitions used by the tests (unbounded Python ints).

`textbook` is the plain definition of each operation type; `simulate`
is an independent, deliberately naive interpreter of a whole design built
on it (used only to cross-check the C oracle on tiny designs).
"""
from rtlgen.design import (ADD, AND, ANDR, CONCAT, DIV, DSHL, DSHR, EQ, EXTRACT, LT, MUL, MUX, MUXC,
                           NOT, OR, ORR, REM, SEXT, SHL, SHR, SUB, XOR, XORR)

M64 = (1 << 64) - 1


def textbook(typ, vals, widths, wd, imm):
    """Integer definition of each operation type (unbounded ints, then mod 2^wd)."""
    a = vals[0]
    if typ == AND:
        r = a
        for v in vals[1:]:
            r &= v
    elif typ == OR:
        r = a
        for v in vals[1:]:
            r |= v
    elif typ == XOR:
        r = a
        for v in vals[1:]:
            r ^= v
    elif typ == NOT:
        r = (1 << wd) - 1 - (a % (1 << wd))
    elif typ == ADD:
        r = a + vals[1]
    elif typ == SUB:
        r = a - vals[1]
    elif typ == MUL:
        r = a * vals[1]
    elif typ == MUX:
        r = vals[1] if a != 0 else vals[2]
    elif typ == MUXC:                 # first pair with a nonzero selector, else the last operand
        r = vals[-1]
        for k in range(len(vals) // 2 - 1, -1, -1):
            if vals[2 * k]:
                r = vals[2 * k + 1]
    elif typ == EQ:
        r = int(a == vals[1])
    elif typ == LT:
        r = int(a < vals[1])
    elif typ == SHL:
        r = a * (2 ** imm)
    elif typ in (SHR, EXTRACT):
        r = a // (2 ** imm)
    elif typ == CONCAT:
        r = a * (2 ** widths[1]) + vals[1]
    elif typ == ORR:
        r = int(a != 0)
    elif typ == DIV:                  # division by zero reads as quotient 0
        r = a // vals[1] if vals[1] else 0
    elif typ == REM:                  # ... and remainder a
        r = a % vals[1] if vals[1] else a
    elif typ == DSHL:
        r = a * 2 ** min(vals[1], 1024)
    elif typ == DSHR:
        r = a // 2 ** min(vals[1], 1024)
    elif typ == ANDR:
        r = int(a == 2 ** widths[0] - 1)
    elif typ == XORR:
        r = bin(a).count("1") % 2
    elif typ == SEXT:                 # a as a widths[0]-bit two's-complement integer
        r = a - 2 ** widths[0] if a >= 2 ** (widths[0] - 1) else a
    else:
        raise ValueError(typ)
    return r % (1 << wd)


def splitmix64(x):
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def stim_value(seed, cycle, k, w):
    v = 0
    for limb in range((w + 63) // 64):
        v |= splitmix64(splitmix64(splitmix64(seed) ^ cycle) ^ ((k << 8) | limb)) << (64 * limb)
    return v % (1 << w)


def digest_step(prev, reg_values, reg_widths):
    """One cycle of the per-instance register digest, on Python ints: the sum
    over registers j and their 64-bit limbs l of s(s(4 j + l) ^ limb), mod
    2^64, then s(prev ^ sum); s is the SplitMix64 output function above."""
    h = 0
    for j, (v, w) in enumerate(zip(reg_values, reg_widths)):
        for l in range((int(w) + 63) // 64):
            h += splitmix64(splitmix64(4 * j + l) ^ ((int(v) >> (64 * l)) & M64))
    return splitmix64(prev ^ (h & M64))


def simulate(d, seed, n_cycles, start_cycle=0, on_cycle=None):
    """All slot values (Python ints) of one instance after n_cycles.
    on_cycle(t, values), if given, sees the slot values after each cycle's
    register commit."""
    W = [int(x) for x in d.slot_width]
    V = [0] * d.n_slots
    for c, s in enumerate(d.const_slot):
        V[int(s)] = sum(int(x) << (64 * l) for l, x in enumerate(d.const_limbs[c])) % (1 << W[int(s)])
    ops = []
    for j in range(d.n_ops):
        srcs = [int(x) for x in d.op_src[d.op_src_ptr[j]:d.op_src_ptr[j + 1]]]
        ops.append((int(d.op_type[j]), int(d.op_dst[j]), srcs, int(d.op_imm[j])))
    for t in range(n_cycles):
        for k, s in enumerate(d.input_slot):
            V[int(s)] = stim_value(seed, start_cycle + t, k, W[int(s)])
        for i in range(d.n_layers):
            out = []
            for typ, dst, srcs, imm in ops[int(d.layer_ptr[i]):int(d.layer_ptr[i + 1])]:
                out.append((dst, textbook(typ, [V[s] for s in srcs], [W[s] for s in srcs], W[dst], imm)))
            for dst, v in out:
                V[dst] = v
        nxt = [V[int(s)] for s in d.reg_next]
        for j, s in enumerate(d.reg_slot):
            V[int(s)] = nxt[j] % (1 << W[int(s)])
        if on_cycle is not None:
            on_cycle(t, V)
    return V
