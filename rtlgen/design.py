"""Container for a levelized RTL dataflow graph as plain arrays.

This module only holds structure (which slot feeds which operation); it
contains none of the simulation arithmetic.  Both the CPU oracle and the
GPU library consume the same arrays.

Vocabulary follows the paper's Cascade 1 (section "RTL Simulation as a
Cascade of Einsums"):

* a *slot* is one coordinate of the signal-state vector LI (rank R / S once
  identity operations are elided, section "Identity Operator Elision");
* every operation has one type (rank N), an ordered operand list (rank O,
  each point holding one R coordinate) and one destination S coordinate;
* operations are grouped into layers (iterative rank I); an operation may
  only read slots produced by strictly earlier layers, registers, primary
  inputs or constants.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

# Operation-type coordinates (rank N).  The numeric values are part of the
# C interface of both the library and the oracle.
(AND, OR, XOR, NOT, ADD, SUB, MUL, MUX, EQ, LT, SHL, SHR, EXTRACT, CONCAT, ORR,
 DIV, REM, DSHL, DSHR, ANDR, XORR, SEXT, MUXC) = range(23)
OP_COUNT = 23
OP_NAMES = ["and", "or", "xor", "not", "add", "sub", "mul", "mux", "eq", "lt",
            "shl", "shr", "extract", "concat", "orr",
            "div", "rem", "dshl", "dshr", "andr", "xorr", "sext", "muxc"]

# MUXC is a fused mux chain: (selector, value) pairs, then a default.
MUXC_MAX_PAIRS = 32

# Allowed occupancies of the O fiber for each type.
OP_ARITIES = {
    AND: (2, 3), OR: (2, 3), XOR: (2, 3), NOT: (1,), ADD: (2,), SUB: (2,),
    MUL: (2,), MUX: (3,), EQ: (2,), LT: (2,), SHL: (1,), SHR: (1,),
    EXTRACT: (1,), CONCAT: (2,), ORR: (1,),
    DIV: (2,), REM: (2,), DSHL: (2,), DSHR: (2,), ANDR: (1,), XORR: (1,), SEXT: (1,),
    MUXC: tuple(range(3, 2 * MUXC_MAX_PAIRS + 2, 2)),
}

MAX_WIDTH = 256
LIMBS = 4  # 64-bit limbs needed for MAX_WIDTH


@dataclasses.dataclass
class Design:
    """One synchronous single-clock design, already levelized.

    Arrays (all numpy, C-contiguous):
      slot_width   uint16[n_slots]        declared bit width, 1..256
      const_slot   uint32[n_consts]       slots holding a literal
      const_limbs  uint64[n_consts, 4]    little-endian literal limbs
      input_slot   uint32[n_inputs]       primary-input slots
      reg_slot     uint32[n_regs]         register (Q) slots
      reg_next     uint32[n_regs]         slot whose value the register latches
      layer_ptr    uint32[n_layers + 1]   op ranges per layer
      op_type      uint8[n_ops]           N coordinate
      op_dst       uint32[n_ops]          S coordinate
      op_src_ptr   uint32[n_ops + 1]      O-fiber ranges into op_src
      op_src       uint32[nnz]            R coordinates in O order
      op_imm       uint16[n_ops]          shift amount / extract low bit; else 0
    """

    name: str
    slot_width: np.ndarray
    const_slot: np.ndarray
    const_limbs: np.ndarray
    input_slot: np.ndarray
    reg_slot: np.ndarray
    reg_next: np.ndarray
    layer_ptr: np.ndarray
    op_type: np.ndarray
    op_dst: np.ndarray
    op_src_ptr: np.ndarray
    op_src: np.ndarray
    op_imm: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)

    def __post_init__(self):
        conv = {
            "slot_width": np.uint16, "const_slot": np.uint32, "const_limbs": np.uint64,
            "input_slot": np.uint32, "reg_slot": np.uint32, "reg_next": np.uint32,
            "layer_ptr": np.uint32, "op_type": np.uint8, "op_dst": np.uint32,
            "op_src_ptr": np.uint32, "op_src": np.uint32, "op_imm": np.uint16,
        }
        for k, t in conv.items():
            setattr(self, k, np.ascontiguousarray(getattr(self, k), dtype=t))
        self.const_limbs = self.const_limbs.reshape(-1, LIMBS)

    # ---- sizes -------------------------------------------------------------
    @property
    def n_slots(self) -> int:
        return int(self.slot_width.shape[0])

    @property
    def n_ops(self) -> int:
        return int(self.op_type.shape[0])

    @property
    def n_layers(self) -> int:
        return int(self.layer_ptr.shape[0]) - 1

    @property
    def n_regs(self) -> int:
        return int(self.reg_slot.shape[0])

    @property
    def n_inputs(self) -> int:
        return int(self.input_slot.shape[0])

    @property
    def n_consts(self) -> int:
        return int(self.const_slot.shape[0])

    def op_arity(self) -> np.ndarray:
        return np.diff(self.op_src_ptr).astype(np.int64)

    def limbs_of(self, slots) -> np.ndarray:
        w = self.slot_width[np.asarray(slots, dtype=np.int64)].astype(np.int64)
        return (w + 63) // 64

    def fingerprint(self) -> str:
        h = hashlib.sha256()
        for k in ("slot_width", "const_slot", "const_limbs", "input_slot", "reg_slot",
                  "reg_next", "layer_ptr", "op_type", "op_dst", "op_src_ptr", "op_src", "op_imm"):
            h.update(getattr(self, k).tobytes())
        return h.hexdigest()[:16]

    def permuted_within_layers(self, seed: int) -> "Design":
        """Same design with the operations of every layer listed in another order."""
        rng = np.random.Generator(np.random.PCG64(seed))
        order = []
        for i in range(self.n_layers):
            a, b = int(self.layer_ptr[i]), int(self.layer_ptr[i + 1])
            order.append(a + rng.permutation(b - a))
        order = np.concatenate(order) if order else np.zeros(0, np.int64)
        ar = self.op_arity()[order]
        src_ptr = np.zeros(self.n_ops + 1, np.int64)
        np.cumsum(ar, out=src_ptr[1:])
        src = np.concatenate([self.op_src[self.op_src_ptr[j]:self.op_src_ptr[j + 1]] for j in order]) \
            if self.n_ops else np.zeros(0, np.uint32)
        return Design(self.name + f"-perm{seed}", self.slot_width, self.const_slot, self.const_limbs,
                      self.input_slot, self.reg_slot, self.reg_next, self.layer_ptr,
                      self.op_type[order], self.op_dst[order], src_ptr, src, self.op_imm[order],
                      dict(self.meta))

    def summary(self) -> dict:
        w = self.slot_width[self.op_dst].astype(np.int64) if self.n_ops else np.zeros(0, np.int64)
        return {
            "name": self.name, "ops": self.n_ops, "layers": self.n_layers, "regs": self.n_regs,
            "inputs": self.n_inputs, "consts": self.n_consts, "slots": self.n_slots,
            "operands": int(self.op_src.shape[0]),
            "dst_w1": float(np.mean(w == 1)) if w.size else 0.0,
            "dst_wide": float(np.mean(w > 64)) if w.size else 0.0,
            "fingerprint": self.fingerprint(),
        }


def int_to_limbs(v: int) -> list:
    return [(v >> (64 * k)) & ((1 << 64) - 1) for k in range(LIMBS)]


def limbs_to_int(limbs) -> int:
    return sum(int(x) << (64 * k) for k, x in enumerate(limbs))
