"""Mux-chain fusion of a levelized design: the oracle's version.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
leg use this module; the GPU library has its own pass and shares nothing
with this one.

Paper: among the compiler's dataflow-graph optimizations (section "Design
Overview" of the proof-of-concept simulator) is operator fusion by mux-chain
extraction, and the N rank has a custom mux-chain operation type; App. B
("Implemented Optimizations", operator fusion) gives the reason: a chain of
muxes evaluated as one larger operation needs fewer memory accesses.

The paper names the optimization without defining a chain.  Reading used
here: MUX m (o0 ? o1 : o2) links to MUX m' when m's default operand o2 is
the slot m' writes and
  * that slot has exactly one reader in the whole design (this operand),
  * no register latches it, and
  * its width is at least the width of m's destination,
so removing m' and evaluating its pairs inside m changes no value that
remains observable (a value passes through the masks of every MUX between it
and the head, and under the width condition the head's mask is the
narrowest).  Links form disjoint paths; each path, from its head (a MUX that
no other MUX links to) inward, becomes MUXC operations of at most
`max_pairs` pairs: (s1, v1, s2, v2, ..., sk, vk, d), the first pair with a
nonzero selector giving the value, else d.  When a path is longer than
`max_pairs`, the MUX after the last absorbed one stays and heads the rest.
Fused operations keep the head's place (its layer and position); the
absorbed MUXes are removed and the slots they wrote are no longer driven.
A path of one MUX stays a MUX.
"""
from __future__ import annotations

import numpy as np

from rtlgen.design import MUX, MUXC, Design

MAX_PAIRS = 32


def mux_links(d: Design) -> np.ndarray:
    """link[o] = the MUX absorbed through o's default operand, or -1."""
    n = d.n_ops
    readers = np.zeros(d.n_slots, np.int64)
    np.add.at(readers, d.op_src.astype(np.int64), 1)
    latched = np.zeros(d.n_slots, bool)
    latched[d.reg_next.astype(np.int64)] = True
    producer = np.full(d.n_slots, -1, np.int64)
    producer[d.op_dst.astype(np.int64)] = np.arange(n)
    link = np.full(n, -1, np.int64)
    for o in range(n):
        if d.op_type[o] != MUX:
            continue
        e = int(d.op_src[int(d.op_src_ptr[o]) + 2])
        p = int(producer[e])
        if p < 0 or d.op_type[p] != MUX:
            continue
        if readers[e] != 1 or latched[e]:
            continue
        if int(d.slot_width[e]) < int(d.slot_width[int(d.op_dst[o])]):
            continue
        link[o] = p
    return link


def fuse_mux_chains(d: Design, max_pairs: int = MAX_PAIRS):
    """Returns (fused design, number of MUXC operations, number of MUXes absorbed)."""
    if not 1 <= max_pairs <= MAX_PAIRS:
        raise ValueError("max_pairs must be 1..32")
    n = d.n_ops
    link = mux_links(d)
    is_target = np.zeros(n, bool)
    is_target[link[link >= 0]] = True
    fused = {}                                   # head op -> operand slots
    absorbed = np.zeros(n, bool)
    for o in range(n):
        if d.op_type[o] != MUX or is_target[o] or link[o] < 0:
            continue
        head = o
        while head >= 0:                         # one MUXC per piece of the path
            srcs, m = [], head
            while True:
                s = [int(x) for x in d.op_src[int(d.op_src_ptr[m]):int(d.op_src_ptr[m]) + 3]]
                srcs += s[:2]
                if link[m] < 0 or len(srcs) // 2 == max_pairs:
                    srcs.append(s[2])
                    break
                m = int(link[m])
                absorbed[m] = True
            if len(srcs) > 3:
                fused[head] = srcs
            head = int(link[m])                  # the MUX the default reads, if linked
    types, dsts, ptr, srcs_out, imms, lay = [], [], [0], [], [], [0]
    for i in range(d.n_layers):
        for o in range(int(d.layer_ptr[i]), int(d.layer_ptr[i + 1])):
            if absorbed[o]:
                continue
            if o in fused:
                types.append(MUXC)
                srcs_out += fused[o]
                imms.append(0)
            else:
                types.append(int(d.op_type[o]))
                srcs_out += [int(x) for x in d.op_src[int(d.op_src_ptr[o]):int(d.op_src_ptr[o + 1])]]
                imms.append(int(d.op_imm[o]))
            dsts.append(int(d.op_dst[o]))
            ptr.append(len(srcs_out))
        lay.append(len(types))
    out = Design(
        name=d.name + "+fused", slot_width=d.slot_width, const_slot=d.const_slot,
        const_limbs=d.const_limbs, input_slot=d.input_slot, reg_slot=d.reg_slot,
        reg_next=d.reg_next, layer_ptr=np.array(lay), op_type=np.array(types, np.int64),
        op_dst=np.array(dsts, np.int64), op_src_ptr=np.array(ptr),
        op_src=np.array(srcs_out, np.int64), op_imm=np.array(imms, np.int64),
        meta=dict(d.meta, fused_from=d.name),
    )
    return out, len(fused), int(absorbed.sum())
