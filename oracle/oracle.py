"""ctypes front end of the C oracle (test infrastructure only).

`run` takes a design (any object with the array attributes of
`rtlgen.Design`), instance seeds and a cycle count, and returns the final
register values as an array [n_inst, n_regs, 4] of uint64 limbs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def lib_path() -> str:
    return LIB


def build(extra_flags=()) -> str:
    """Compile liboracle.so with gcc (plain -O2, generic x86-64)."""
    tmp = LIB + f".tmp{os.getpid()}"   # one per process: test workers may build at once
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
           *extra_flags, SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Design(C.Structure):
    _fields_ = [
        ("n_slots", C.c_uint32), ("slot_width", C.c_void_p),
        ("n_consts", C.c_uint32), ("const_slot", C.c_void_p), ("const_limbs", C.c_void_p),
        ("n_inputs", C.c_uint32), ("input_slot", C.c_void_p),
        ("n_regs", C.c_uint32), ("reg_slot", C.c_void_p), ("reg_next", C.c_void_p),
        ("n_layers", C.c_uint32), ("layer_ptr", C.c_void_p),
        ("n_ops", C.c_uint32), ("op_type", C.c_void_p), ("op_dst", C.c_void_p),
        ("op_src_ptr", C.c_void_p), ("op_src", C.c_void_p), ("op_imm", C.c_void_p),
    ]


class _Args(C.Structure):
    _fields_ = [
        ("n_inst", C.c_uint32), ("seeds", C.c_void_p),
        ("start_cycle", C.c_uint64), ("n_cycles", C.c_uint64),
        ("stim_mode", C.c_int32), ("stim_words", C.c_void_p),
        ("init_regs", C.c_void_p), ("out_regs", C.c_void_p), ("out_slots", C.c_void_p),
        ("trace_reg", C.c_int32), ("trace", C.c_void_p), ("n_threads", C.c_int32),
        ("init_digest", C.c_void_p), ("out_digest", C.c_void_p), ("digest_trace", C.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _lib.oracle_run.argtypes = [C.POINTER(_Design), C.POINTER(_Args)]
        _lib.oracle_run.restype = C.c_int
        _lib.oracle_eval_op.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                        C.c_int, C.c_void_p]
        _lib.oracle_eval_op.restype = C.c_int
        _lib.oracle_stim.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]
        _lib.oracle_stim.restype = C.c_uint64
        _lib.oracle_splitmix64.argtypes = [C.c_uint64]
        _lib.oracle_splitmix64.restype = C.c_uint64
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def run(design, seeds, n_cycles, *, start_cycle=0, stim_words=None, init_regs=None,
        want_slots=False, trace_reg=-1, n_threads=None, init_digest=None, digests=None,
        digest_trace=False):
    """Simulate `len(seeds)` instances for `n_cycles` cycles.

    Returns (regs[n_inst, n_regs, 4], slots or None, trace or None).  With
    `digests` (a dict), digests["final"] receives the register digest of
    every instance after the last cycle ([n_inst] uint64) and, with
    digest_trace, digests["trace"] the digest after every cycle
    ([n_inst, n_cycles]); init_digest ([n_inst]) continues a digest chain.
    """
    lib = _load()
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a

    d = _Design()
    d.n_slots = design.slot_width.shape[0]
    d.slot_width = _ptr(arr(design.slot_width, np.uint16))
    d.n_consts = design.const_slot.shape[0]
    d.const_slot = _ptr(arr(design.const_slot, np.uint32))
    d.const_limbs = _ptr(arr(design.const_limbs, np.uint64))
    d.n_inputs = design.input_slot.shape[0]
    d.input_slot = _ptr(arr(design.input_slot, np.uint32))
    d.n_regs = design.reg_slot.shape[0]
    d.reg_slot = _ptr(arr(design.reg_slot, np.uint32))
    d.reg_next = _ptr(arr(design.reg_next, np.uint32))
    d.n_layers = design.layer_ptr.shape[0] - 1
    d.layer_ptr = _ptr(arr(design.layer_ptr, np.uint32))
    d.n_ops = design.op_type.shape[0]
    d.op_type = _ptr(arr(design.op_type, np.uint8))
    d.op_dst = _ptr(arr(design.op_dst, np.uint32))
    d.op_src_ptr = _ptr(arr(design.op_src_ptr, np.uint32))
    d.op_src = _ptr(arr(design.op_src, np.uint32))
    d.op_imm = _ptr(arr(design.op_imm, np.uint16))

    seeds = arr(seeds, np.uint64)
    n_inst = seeds.shape[0]
    n_regs = int(d.n_regs)
    out_regs = np.zeros((n_inst, n_regs, 4), np.uint64)
    out_slots = np.zeros((n_inst, int(d.n_slots), 4), np.uint64) if want_slots else None
    trace = np.zeros((n_inst, int(n_cycles)), np.uint64) if trace_reg >= 0 else None

    a = _Args()
    a.n_inst = n_inst
    a.seeds = _ptr(seeds)
    a.start_cycle = int(start_cycle)
    a.n_cycles = int(n_cycles)
    if stim_words is not None:
        a.stim_mode = 1
        a.stim_words = _ptr(arr(stim_words, np.uint64))
    else:
        a.stim_mode = 0
    a.init_regs = _ptr(arr(init_regs, np.uint64)) if init_regs is not None else None
    a.out_regs = _ptr(out_regs)
    a.out_slots = _ptr(out_slots) if out_slots is not None else None
    a.trace_reg = int(trace_reg)
    a.trace = _ptr(trace) if trace is not None else None
    a.n_threads = int(n_threads or min(os.cpu_count() or 1, max(n_inst, 1)))
    a.init_digest = _ptr(arr(init_digest, np.uint64)) if init_digest is not None else None
    out_digest = dtrace = None
    if digests is not None:
        out_digest = np.zeros(n_inst, np.uint64)
        a.out_digest = _ptr(out_digest)
        if digest_trace:
            dtrace = np.zeros((n_inst, int(n_cycles)), np.uint64)
            a.digest_trace = _ptr(dtrace)
    rc = lib.oracle_run(C.byref(d), C.byref(a))
    if rc != 0:
        raise ValueError(f"oracle_run failed with code {rc}")
    if digests is not None:
        digests["final"] = out_digest
        if digest_trace:
            digests["trace"] = dtrace
    return out_regs, out_slots, trace


def eval_op(typ, operands, src_widths, dst_w, imm=0) -> int:
    """One operation on Python-int operands; returns a Python int."""
    lib = _load()
    ar = len(operands)
    ops = np.zeros((max(ar, 1), 4), np.uint64)
    for o, v in enumerate(operands):
        for k in range(4):
            ops[o, k] = (int(v) >> (64 * k)) & ((1 << 64) - 1)
    sw = np.zeros(max(ar, 3), np.uint16)
    sw[:ar] = src_widths
    out = np.zeros(4, np.uint64)
    rc = lib.oracle_eval_op(int(typ), ar, ops.ctypes.data, sw.ctypes.data, int(dst_w), int(imm),
                            out.ctypes.data)
    if rc != 0:
        raise ValueError("bad operation")
    return sum(int(out[k]) << (64 * k) for k in range(4))


def stim(seed, cycle, k, limb) -> int:
    return int(_load().oracle_stim(int(seed), int(cycle), int(k), int(limb)))


def splitmix64(x) -> int:
    return int(_load().oracle_splitmix64(int(x)))
