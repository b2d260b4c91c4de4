"""Seeded synthetic levelized dataflow graphs with the shapes of the workloads.

The paper evaluates on Chipyard designs that are not available here, so
random levelized DAGs stand in for them.  The recipe (op mix, width mix,
fan-in, operand distance distribution, register/input counts) is fixed per
workload below; every draw comes from numpy's PCG64 seeded explicitly, so a
(workload, seed) pair always yields the same design.

Only graph *structure* is produced here: no value is ever computed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .design import (ADD, AND, ANDR, CONCAT, DIV, DSHL, DSHR, EQ, EXTRACT, LT, MUL, MUX, NOT, OR,
                     ORR, REM, SEXT, SHL, SHR, SUB, XOR, XORR, Design)

# (type, arity, probability): and/or/xor/not 30 %, add/sub 15 %, mux 15 %,
# eq/lt 10 %, shift-by-const 10 %, extract/concat 10 %, mul 5 %, reduce-or 5 %.
OP_MIX = (
    (AND, 2, 0.0375), (AND, 3, 0.0375), (OR, 2, 0.0375), (OR, 3, 0.0375),
    (XOR, 2, 0.0375), (XOR, 3, 0.0375), (NOT, 1, 0.075),
    (ADD, 2, 0.075), (SUB, 2, 0.075), (MUX, 3, 0.15),
    (EQ, 2, 0.05), (LT, 2, 0.05), (SHL, 1, 0.05), (SHR, 1, 0.05),
    (EXTRACT, 1, 0.05), (CONCAT, 2, 0.05), (MUL, 2, 0.05), (ORR, 1, 0.05),
)
# Every type, the FIRRTL primitives without an expansion in the others
# included: for test designs (the workloads keep OP_MIX).
OP_MIX_FULL = OP_MIX + (
    (DIV, 2, 0.03), (REM, 2, 0.03), (DSHL, 2, 0.03), (DSHR, 2, 0.03),
    (ANDR, 1, 0.03), (XORR, 1, 0.03), (SEXT, 1, 0.04),
)
ONE_BIT_TYPES = (EQ, LT, ORR, ANDR, XORR)

# Width buckets: (lo, hi inclusive, probability).
WIDTHS_STD = ((1, 1, 0.40), (2, 8, 0.25), (9, 32, 0.25), (33, 64, 0.10))
WIDTHS_MULTIDESIGN = ((1, 1, 0.36), (2, 8, 0.225), (9, 32, 0.225), (33, 64, 0.09), (65, 128, 0.10))
WIDTHS_LARGE = ((1, 1, 0.35), (2, 8, 0.25), (9, 32, 0.25), (33, 64, 0.10), (65, 256, 0.05))


@dataclasses.dataclass(frozen=True)
class GenConfig:
    n_ops: int
    n_layers: int
    n_regs: int
    n_inputs: int
    widths: tuple = WIDTHS_STD
    name: str = "design"
    op_mix: tuple = OP_MIX
    # Probability that a MUX of layer i >= 1 takes as its default operand
    # (o = 2) a MUX of layer i - 1 that nothing else reads: priority chains
    # (when / elsewhen / otherwise).  0 leaves the design as drawn.
    mux_chain: float = 0.0


def _bucket_draw(rng, buckets, n):
    p = np.array([b[2] for b in buckets], dtype=np.float64)
    p = p / p.sum()
    which = rng.choice(len(buckets), size=n, p=p)
    lo = np.array([b[0] for b in buckets], dtype=np.int64)[which]
    hi = np.array([b[1] for b in buckets], dtype=np.int64)[which]
    return lo + (rng.random(n) * (hi - lo + 1)).astype(np.int64)


def _conditional_buckets(buckets, mix=OP_MIX):
    """Width mix for ops not forced to 1 bit, so the overall mix matches `buckets`."""
    forced = sum(p for t, _, p in mix if t in ONE_BIT_TYPES) / sum(p for _, _, p in mix)
    out = []
    for lo, hi, p in buckets:
        q = p - (forced if (lo, hi) == (1, 1) else 0.0)
        out.append((lo, hi, max(q, 0.0) / (1.0 - forced)))
    return tuple(out)


def generate(cfg: GenConfig, seed: int) -> Design:
    rng = np.random.Generator(np.random.PCG64(seed))
    n_ops, L = int(cfg.n_ops), int(cfg.n_layers)
    n_in, n_reg = int(cfg.n_inputs), int(cfg.n_regs)
    if L < 1 or n_ops < L:
        raise ValueError("need at least one op per layer")
    if n_in + n_reg == 0:
        raise ValueError("need at least one register or input")

    # Layer sizes: equal split, the first n_ops mod L layers get one more.
    sizes = np.full(L, n_ops // L, dtype=np.int64)
    sizes[: n_ops % L] += 1
    layer_ptr = np.zeros(L + 1, dtype=np.int64)
    np.cumsum(sizes, out=layer_ptr[1:])

    # Types and arities.
    mix = cfg.op_mix
    mix_p = np.array([m[2] for m in mix])
    mix_p /= mix_p.sum()
    pick = rng.choice(len(mix), size=n_ops, p=mix_p)
    op_type = np.array([m[0] for m in mix], dtype=np.int64)[pick]
    arity = np.array([m[1] for m in mix], dtype=np.int64)[pick]

    # Slot layout: [inputs][registers][one destination per op, in layer order].
    base_in, base_reg, base_op = 0, n_in, n_in + n_reg
    n_slots = base_op + n_ops
    width = np.zeros(n_slots, dtype=np.int64)
    width[: base_op] = _bucket_draw(rng, cfg.widths, base_op)
    w_ops = _bucket_draw(rng, _conditional_buckets(cfg.widths, mix), n_ops)
    w_ops[np.isin(op_type, ONE_BIT_TYPES)] = 1
    width[base_op:] = w_ops

    src_ptr = np.zeros(n_ops + 1, dtype=np.int64)
    np.cumsum(arity, out=src_ptr[1:])
    op_src = np.zeros(int(src_ptr[-1]), dtype=np.int64)
    op_imm = np.zeros(n_ops, dtype=np.int64)

    def draw_sources(layer, k):
        """k operand slots for ops in `layer` (geometric bias toward layer-1)."""
        u = rng.random(k)
        out = np.empty(k, dtype=np.int64)
        if layer == 0:
            p_reg, p_in = (2.0 / 3.0, 1.0 / 3.0)
        else:
            p_reg, p_in = 0.10, 0.05
        if n_reg == 0:
            p_reg, p_in = 0.0, (1.0 if layer == 0 else p_in + p_reg)
        if n_in == 0:
            p_reg, p_in = (1.0 if layer == 0 else p_reg + p_in), 0.0
        is_reg = u < p_reg
        is_in = (u >= p_reg) & (u < p_reg + p_in)
        is_op = ~(is_reg | is_in)
        out[is_reg] = base_reg + rng.integers(0, max(n_reg, 1), int(is_reg.sum()))
        out[is_in] = base_in + rng.integers(0, max(n_in, 1), int(is_in.sum()))
        m = int(is_op.sum())
        if m:
            d = rng.geometric(0.5, m)
            bad = d > layer
            while bad.any():
                d[bad] = rng.geometric(0.5, int(bad.sum()))
                bad = d > layer
            src_layer = layer - d
            off = (rng.random(m) * sizes[src_layer]).astype(np.int64)
            out[is_op] = base_op + layer_ptr[src_layer] + off
        return out

    for i in range(L):
        a, b = int(layer_ptr[i]), int(layer_ptr[i + 1])
        s0, s1 = int(src_ptr[a]), int(src_ptr[b])
        op_src[s0:s1] = draw_sources(i, s1 - s0)
        # Mux selectors prefer a 1-bit candidate (up to 8 draws).
        mux = np.nonzero(op_type[a:b] == MUX)[0] + a
        if mux.size:
            cand = np.stack([draw_sources(i, mux.size) for _ in range(8)])
            ok = width[cand] == 1
            first = np.where(ok.any(axis=0), ok.argmax(axis=0), 7)
            op_src[src_ptr[mux]] = cand[first, np.arange(mux.size)]
        # Immediates from the width of the (single) operand.
        t = op_type[a:b]
        for typ, off in ((SHL, 1), (SHR, 1), (EXTRACT, 0)):
            j = np.nonzero(t == typ)[0] + a
            if j.size:
                ws = width[op_src[src_ptr[j]]]
                op_imm[j] = (rng.random(j.size) * (ws + off)).astype(np.int64)

    # Register next-state drivers: uniform op in the last ceil(L/4) layers.
    tail = layer_ptr[L - int(math.ceil(L / 4))]
    reg_slot = base_reg + np.arange(n_reg, dtype=np.int64)
    reg_next = base_op + tail + (rng.random(n_reg) * (n_ops - tail)).astype(np.int64)
    if cfg.mux_chain > 0:
        _chain_muxes(rng, cfg.mux_chain, op_type, layer_ptr, src_ptr, op_src, reg_next, width, base_op)

    return Design(
        name=cfg.name, slot_width=width, const_slot=np.zeros(0, np.uint32),
        const_limbs=np.zeros((0, 4), np.uint64), input_slot=base_in + np.arange(n_in),
        reg_slot=reg_slot, reg_next=reg_next, layer_ptr=layer_ptr, op_type=op_type,
        op_dst=base_op + np.arange(n_ops), op_src_ptr=src_ptr, op_src=op_src, op_imm=op_imm,
        meta={"generator": dataclasses.asdict(cfg), "seed": int(seed)},
    )


def _chain_muxes(rng, p, op_type, layer_ptr, src_ptr, op_src, reg_next, width, base_op):
    """Links MUXes into priority chains, in place.

    From the last layer down, each MUX of layer i takes, with probability p,
    a MUX of layer i - 1 (each taken once) as its default operand; the inner
    MUX's width is raised to the outer's (skipped for 10 % of the links).
    Other reads of an inner MUX, and registers latching one, then move to a
    random untaken operation of the same layer (kept for 4 % of them).  The skipped and kept cases are links that a fusion pass
    must leave alone.
    """
    L = layer_ptr.size - 1
    n = op_type.size
    taken_by = np.full(n, -1, np.int64)
    for i in range(L - 1, 0, -1):
        outer = np.nonzero(op_type[layer_ptr[i]:layer_ptr[i + 1]] == MUX)[0] + layer_ptr[i]
        inner = np.nonzero(op_type[layer_ptr[i - 1]:layer_ptr[i]] == MUX)[0] + layer_ptr[i - 1]
        outer = outer[rng.random(outer.size) < p]
        k = min(outer.size, inner.size)
        if k == 0:
            continue
        outer = outer[:k]
        inner = rng.permutation(inner)[:k]
        op_src[src_ptr[outer] + 2] = base_op + inner
        taken_by[inner] = outer
        widen = rng.random(k) >= 0.10
        wi, wo = width[base_op + inner], width[base_op + outer]
        width[base_op + inner[widen]] = np.maximum(wi[widen], wo[widen])
    layer_of = np.repeat(np.arange(L), np.diff(layer_ptr))
    free = [np.nonzero(taken_by[layer_ptr[i]:layer_ptr[i + 1]] < 0)[0] + layer_ptr[i] for i in range(L)]

    def move(slots):
        ops = slots - base_op
        out = slots.copy()
        for i in np.unique(layer_of[ops]):
            sel = layer_of[ops] == i
            if free[i].size == 0:
                continue
            out[sel] = base_op + free[i][(rng.random(int(sel.sum())) * free[i].size).astype(np.int64)]
        return out

    entry_op = np.repeat(np.arange(n), np.diff(src_ptr))
    rd = op_src - base_op
    is_op = rd >= 0
    hit = np.zeros(op_src.size, bool)
    hit[is_op] = taken_by[rd[is_op]] >= 0
    own = hit & (taken_by[np.where(is_op, rd, 0)] == entry_op) & (np.arange(op_src.size) == src_ptr[entry_op] + 2)
    redo = hit & ~own & (rng.random(op_src.size) >= 0.04)
    op_src[redo] = move(op_src[redo])
    rn = reg_next - base_op
    redo = (taken_by[rn] >= 0) & (rng.random(rn.size) >= 0.04)
    reg_next[redo] = move(reg_next[redo])


# ---------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------
CFG0 = GenConfig(2_000, 16, 64, 16, WIDTHS_STD, "plain-2k")
CFG1 = GenConfig(200_000, 48, 4_096, 64, WIDTHS_STD, "single-200k")
CFG3 = GenConfig(5_000_000, 120, 64_000, 256, WIDTHS_LARGE, "large-5m")
# Mux-heavy logic with priority chains (35 % MUX, 80 % of them chained):
# the input of the mux-chain fusion measurement.
OP_MIX_MUX = tuple((t, a, 0.35 if t == MUX else p) for t, a, p in OP_MIX)
CFG_MUXCHAIN = GenConfig(2_000_000, 100, 32_000, 256, WIDTHS_STD, "muxchain-2m", OP_MIX_MUX,
                         mux_chain=0.8)

WORKLOADS = {
    "plain-2k": dict(cfg=CFG0, seed=0, instances=1, cycles=10_000),
    "single-200k": dict(cfg=CFG1, seed=1, instances=1024, cycles=100_000),
    "large-5m": dict(cfg=CFG3, seed=3, instances=4096, cycles=10_000),
}


def _log_uniform_int(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n)).round().astype(np.int64).clip(lo, hi)


def multidesign_batch(seed: int = 2, n_designs: int = 64, ops_lo: int = 5_000, ops_hi: int = 500_000,
                      inst_lo: int = 1, inst_hi: int = 256, widths=WIDTHS_MULTIDESIGN):
    """Uneven multi-design batch: (GenConfig, design seed, instance count) per design."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops = _log_uniform_int(rng, ops_lo, ops_hi, n_designs)
    layers = rng.integers(16, 81, n_designs)
    inst = _log_uniform_int(rng, inst_lo, inst_hi, n_designs)
    out = []
    for d in range(n_designs):
        n = int(ops[d])
        cfg = GenConfig(n, int(min(layers[d], n)), max(64, round(0.02 * n)), 64, widths, f"multi-{d}")
        out.append((cfg, 200 + d, int(inst[d])))
    return out


def serving_pool(seed: int = 4, n_designs: int = 32, ops_lo: int = 10_000, ops_hi: int = 1_000_000):
    """Design pool for the serving workload: (GenConfig, design seed) per design."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops = _log_uniform_int(rng, ops_lo, ops_hi, n_designs)
    layers = rng.integers(16, 121, n_designs)
    return [(GenConfig(int(ops[d]), int(layers[d]), max(64, round(0.02 * int(ops[d]))), 64,
                       WIDTHS_STD, f"pool-{d}"), 400 + d) for d in range(n_designs)]


def serving_jobs(seed: int, n_jobs: int, pool_size: int = 32, inst_hi: int = 512,
                 cyc_lo: int = 1_000, cyc_hi: int = 50_000):
    """Job list: (design index, instances, cycles) with log-uniform sizes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.integers(0, pool_size, n_jobs)
    inst = _log_uniform_int(rng, 1, inst_hi, n_jobs)
    cyc = _log_uniform_int(rng, cyc_lo, cyc_hi, n_jobs)
    return [(int(d[j]), int(inst[j]), int(cyc[j])) for j in range(n_jobs)]


def instance_seeds(n: int, design_index: int | None = None) -> np.ndarray:
    """Stimulus seeds: 0..n-1, or (design << 16) | j inside a multi-design batch."""
    j = np.arange(n, dtype=np.uint64)
    if design_index is None:
        return j
    return (np.uint64(design_index) << np.uint64(16)) | j


def scaled(cfg: GenConfig, factor: float, name: str | None = None) -> GenConfig:
    """Same recipe at a fraction of the op/register/input counts (for tests)."""
    n = max(int(cfg.n_ops * factor), cfg.n_layers)
    return dataclasses.replace(cfg, n_ops=n, n_regs=max(1, int(cfg.n_regs * factor)),
                               n_inputs=max(1, int(cfg.n_inputs * factor)),
                               name=name or f"{cfg.name}-x{factor:g}")
