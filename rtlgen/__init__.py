"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

Holds graph structure and seeds only; no simulation arithmetic lives here.
"""
from .design import (ADD, AND, ANDR, CONCAT, DIV, DSHL, DSHR, EQ, EXTRACT, LT, MUL, MUX, MUXC,
                     MUXC_MAX_PAIRS, NOT, OP_ARITIES, OP_COUNT, OP_NAMES, OR, ORR, REM, SEXT, SHL, SHR, SUB, XOR, XORR,
                     Design, int_to_limbs, limbs_to_int)
from .generator import (CFG0, CFG1, CFG3, CFG_MUXCHAIN, OP_MIX, OP_MIX_FULL, WORKLOADS, GenConfig, generate,
                        instance_seeds, multidesign_batch, scaled, serving_jobs, serving_pool)

__all__ = [
    "ADD", "AND", "CONCAT", "EQ", "EXTRACT", "LT", "MUL", "MUX", "NOT", "OP_ARITIES", "OP_COUNT",
    "OP_NAMES", "OR", "ORR", "SHL", "SHR", "SUB", "XOR", "Design", "int_to_limbs", "limbs_to_int",
    "DIV", "REM", "DSHL", "DSHR", "ANDR", "XORR", "SEXT", "MUXC", "MUXC_MAX_PAIRS",
    "CFG0", "CFG1", "CFG3", "CFG_MUXCHAIN", "OP_MIX", "OP_MIX_FULL", "WORKLOADS", "GenConfig", "generate",
    "instance_seeds",
    "multidesign_batch", "scaled", "serving_jobs", "serving_pool",
]
