"""Python binding of librteaal.so: the C entry points under the same names.

Only argument marshalling happens here; every simulation step runs in the
HIP kernels of the library.  Device memory for designs and batches comes
from PyTorch's caching allocator through the allocator callback, and the
work is enqueued on a torch stream.  If the shared library is missing the
import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librteaal.so")

__all__ = [
    "RTEAAL_OK", "RTEAAL_MAP_AUTO", "RTEAAL_MAP_RESIDENT", "RTEAAL_MAP_SWEEP", "RTEAAL_MAP_LAYERED",
    "RTEAAL_MAP_PARTITIONED",
    "RTEAAL_READ_REGS", "RTEAAL_READ_DIGEST", "RTEAAL_READ_ALL_SLOTS", "RteaalError", "Context", "library",
    "exported_symbols", "rteaal_create", "rteaal_destroy", "rteaal_last_error",
    "rteaal_validate_design", "rteaal_load_design", "rteaal_unload_design", "rteaal_design_format",
    "RTEAAL_LOAD_KEEP_ALL_SLOTS",
    "rteaal_batch_footprint", "rteaal_batch_resources", "rteaal_create_batch", "rteaal_free_batch",
    "rteaal_partition_plan_stats",
    "rteaal_batch_info",
    "rteaal_batch_options",
    "rteaal_step", "rteaal_step_many", "rteaal_sync", "rteaal_read_state", "rteaal_write_state",
    "rteaal_write_digest", "rteaal_read_digest", "rteaal_read_state_noalloc",
    "RTEAAL_NOALLOC_MAX_WORDS",
    "rteaal_kernel_timing", "rteaal_autotune", "rteaal_autotune_many", "opts_dict", "unpack_limbs", "pack_limbs", "rteaal_layer_format", "rteaal_rank_format",
    "rteaal_dag_desc", "rteaal_levelize", "levelized_design",
    "CHANGE_DTYPE", "rteaal_watch", "rteaal_read_changes",
]

RTEAAL_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "BAD_DESIGN", 3: "FORMAT", 4: "NO_MEMORY",
                5: "DEVICE", 6: "BUSY", 7: "UNSUPPORTED"}
RTEAAL_MAP_AUTO, RTEAAL_MAP_RESIDENT, RTEAAL_MAP_SWEEP, RTEAAL_MAP_LAYERED = 0, 1, 2, 3
RTEAAL_MAP_PARTITIONED = 4
RTEAAL_READ_REGS, RTEAAL_READ_DIGEST, RTEAAL_READ_ALL_SLOTS = 1, 2, 4
RTEAAL_MUXC, RTEAAL_MUXC_MAX_PAIRS = 22, 32
RTEAAL_NOALLOC_MAX_WORDS = 1 << 20


class RteaalError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class rteaal_rank_format(C.Structure):
    _fields_ = [("compressed", C.c_uint8), ("cbits", C.c_uint8), ("pbits", C.c_uint8)]


class rteaal_layer_format(C.Structure):
    _fields_ = [("oim", rteaal_rank_format * 5), ("li", rteaal_rank_format),
                ("lo", rteaal_rank_format)]


class rteaal_design_desc(C.Structure):
    _fields_ = [
        ("n_slots", C.c_uint32), ("slot_width", C.c_void_p),
        ("n_consts", C.c_uint32), ("const_slot", C.c_void_p), ("const_limbs", C.c_void_p),
        ("n_inputs", C.c_uint32), ("input_slot", C.c_void_p),
        ("n_regs", C.c_uint32), ("reg_slot", C.c_void_p), ("reg_next", C.c_void_p),
        ("n_layers", C.c_uint32), ("layer_op_ptr", C.c_void_p),
        ("n_ops", C.c_uint32), ("op_type", C.c_void_p), ("op_dst", C.c_void_p),
        ("op_src_ptr", C.c_void_p), ("op_src", C.c_void_p), ("op_imm", C.c_void_p),
        ("layer_fmt", C.c_void_p),
    ]


class rteaal_fuse_result(C.Structure):
    _fields_ = [("n_ops", C.c_uint32), ("n_operands", C.c_uint32), ("n_fused", C.c_uint32),
                ("n_absorbed", C.c_uint32)]


class rteaal_dag_desc(C.Structure):
    _fields_ = [("n_slots", C.c_uint32), ("n_ops", C.c_uint32), ("op_src_ptr", C.c_void_p),
                ("op_src", C.c_void_p), ("op_dst", C.c_void_p)]


class rteaal_batch_opts(C.Structure):
    _fields_ = [("mapping", C.c_uint32), ("block_threads", C.c_uint32),
                ("ops_per_wave", C.c_uint32), ("lds_state", C.c_uint32),
                ("lds_ops", C.c_uint32), ("unroll", C.c_uint32),
                ("tiles_per_wave", C.c_uint32), ("arity_split", C.c_uint32),
                ("tiles_per_pass", C.c_uint32), ("persistent", C.c_uint32),
                ("partitions", C.c_uint32), ("pass_branches", C.c_uint32)]


class rteaal_partition_stats(C.Structure):
    _fields_ = [("design_ops", C.c_uint64), ("cone_ops", C.c_uint64), ("padded_ops", C.c_uint64),
                ("max_part_ops", C.c_uint64), ("exchange", C.c_uint64)]


class rteaal_stimulus(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("words_on_device", C.c_uint32), ("words", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class rteaal_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


_lib = None


def library():
    """The loaded librteaal.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2601_18140_amd/build.py")
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes the library bind to that runtime, so one HIP
    # runtime serves the process and torch's streams and memory are valid here.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, u32, u64, st = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    sig = {
        "rteaal_create": ([C.c_int, vp, C.POINTER(rteaal_allocator), C.POINTER(vp)], st),
        "rteaal_destroy": ([vp], None),
        "rteaal_last_error": ([vp], C.c_char_p),
        "rteaal_validate_design": ([C.POINTER(rteaal_design_desc), C.c_char_p, C.c_size_t], st),
        "rteaal_load_design": ([vp, C.POINTER(rteaal_design_desc), C.POINTER(u32)], st),
        "rteaal_load_design_ex": ([vp, C.POINTER(rteaal_design_desc), u32, C.POINTER(u32)], st),
        "rteaal_unload_design": ([vp, u32], st),
        "rteaal_design_format": ([vp, u32, u32, C.POINTER(rteaal_layer_format)], st),
        "rteaal_batch_footprint": ([vp, u32, u32, C.POINTER(rteaal_batch_opts), C.POINTER(u64)], st),
        "rteaal_batch_resources": ([vp, u32, u32, C.POINTER(rteaal_batch_opts), C.POINTER(u64),
                                    C.POINTER(u64)], st),
        "rteaal_partition_plan_stats": ([vp, u32, u32, C.POINTER(rteaal_partition_stats)], st),
        "rteaal_create_batch": ([vp, u32, u32, vp, C.POINTER(rteaal_batch_opts), C.POINTER(u32)], st),
        "rteaal_free_batch": ([vp, u32], st),
        "rteaal_batch_info": ([vp, u32, C.POINTER(u32), C.POINTER(u64)], st),
        "rteaal_batch_options": ([vp, u32, C.POINTER(rteaal_batch_opts)], st),
        "rteaal_step": ([vp, u32, u64, C.POINTER(rteaal_stimulus)], st),
        "rteaal_step_many": ([vp, u32, vp, vp, vp], st),
        "rteaal_sync": ([vp], st),
        "rteaal_read_state": ([vp, u32, u32, u32, u32, vp, C.c_size_t, C.POINTER(C.c_size_t)], st),
        "rteaal_write_state": ([vp, u32, u32, u32, vp, u64], st),
        "rteaal_write_digest": ([vp, u32, u32, u32, vp], st),
        "rteaal_read_state_noalloc": ([vp, u32, u32, u32, u32, vp, C.c_size_t, C.POINTER(C.c_size_t)], st),
        "rteaal_kernel_timing": ([vp, u32, C.c_int, C.POINTER(u64), C.POINTER(C.c_double)], st),
        "rteaal_autotune": ([vp, u32, u32, u32, C.POINTER(rteaal_batch_opts), C.POINTER(C.c_double)], st),
        "rteaal_autotune_many": ([vp, u32, vp, vp, u32, vp, C.POINTER(C.c_double)], st),
        "rteaal_levelize": ([vp, C.POINTER(rteaal_dag_desc), vp, vp, vp, C.POINTER(u32)], st),
        "rteaal_watch": ([vp, u32, vp, u32, u64], st),
        "rteaal_read_changes": ([vp, u32, vp, u64, C.POINTER(u64), C.POINTER(u64)], st),
        "rteaal_fuse_mux_chains": ([C.POINTER(rteaal_design_desc), u32, vp, vp, vp, vp, vp, vp,
                                    C.POINTER(rteaal_fuse_result)], st),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def exported_symbols():
    return ["rteaal_create", "rteaal_destroy", "rteaal_last_error", "rteaal_validate_design",
            "rteaal_load_design", "rteaal_load_design_ex", "rteaal_unload_design",
            "rteaal_design_format",
            "rteaal_batch_footprint", "rteaal_batch_resources", "rteaal_partition_plan_stats",
            "rteaal_create_batch", "rteaal_free_batch",
            "rteaal_batch_info", "rteaal_batch_options", "rteaal_step", "rteaal_step_many", "rteaal_sync",
            "rteaal_read_state", "rteaal_read_state_noalloc", "rteaal_write_state",
            "rteaal_write_digest",
            "rteaal_kernel_timing", "rteaal_autotune", "rteaal_autotune_many",
            "rteaal_levelize", "rteaal_watch", "rteaal_read_changes", "rteaal_fuse_mux_chains"]


def _check(ctx, status):
    if status != RTEAAL_OK:
        msg = library().rteaal_last_error(ctx)
        raise RteaalError(status, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# Handles.
# ---------------------------------------------------------------------------
class Context:
    """An rteaal_ctx plus what the binding needs to size host buffers."""

    def device_allocations(self):
        """Device allocations the library has requested through the torch
        allocator callback so far (None with the hipMalloc allocator)."""
        for k in self._keep:
            if isinstance(k, tuple) and len(k) == 4:
                return k[3][0]
        return None

    def __init__(self, handle, stream, allocator, keep):
        self.handle = handle
        self.stream = stream
        self._allocator = allocator
        self._keep = keep
        self.designs = {}   # id -> (reg widths, slot widths, inputs words)
        self.batches = {}   # id -> (design id, n_instances)

    @property
    def _as_parameter_(self):
        return self.handle


def _torch_allocator(device, stream):
    """Allocator callbacks over torch's caching allocator, blocks tied to `stream`
    (the library's stream; it synchronises before it frees anything)."""
    import torch
    live = {}
    calls = [0]   # allocations requested so far

    def _alloc(nbytes, _user):
        calls[0] += 1
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except RuntimeError:
            return None
        live[p] = nbytes
        return p

    def _free(ptr, _nbytes, _user):
        if ptr in live:
            del live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

    a = rteaal_allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    return a, (_alloc, _free, live, calls)


def rteaal_create(device=0, stream=None, allocator="torch"):
    """New context.  stream: a torch.cuda.Stream, a raw hipStream_t int, or None
    (a fresh torch stream at default priority).  allocator: "torch" or None (hipMalloc)."""
    lib = library()
    keep = []
    s_handle = None
    s_obj = None
    if allocator == "torch" or stream is None or hasattr(stream, "cuda_stream"):
        import torch
        if stream is None:
            s_obj = torch.cuda.Stream(device=device)
            stream = s_obj
        if hasattr(stream, "cuda_stream"):
            s_obj = stream
            s_handle = stream.cuda_stream
    if s_handle is None and stream is not None:
        s_handle = int(stream)
    alloc_struct = None
    if allocator == "torch":
        import torch
        alloc_struct, fns = _torch_allocator(device, s_obj)
        keep.append(fns)
    out = C.c_void_p()
    st = lib.rteaal_create(int(device), C.c_void_p(s_handle) if s_handle else None,
                           C.byref(alloc_struct) if alloc_struct is not None else None, C.byref(out))
    _check(None, st)
    return Context(out.value, s_obj if s_obj is not None else s_handle, alloc_struct, keep)


def rteaal_destroy(ctx):
    if ctx is not None and ctx.handle:
        library().rteaal_destroy(ctx.handle)
        ctx.handle = None


def rteaal_last_error(ctx=None):
    msg = library().rteaal_last_error(ctx.handle if ctx is not None else None)
    return msg.decode() if msg else ""


def _desc(design, layer_fmt=None):
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a.ctypes.data if a.size else None

    d = rteaal_design_desc()
    d.n_slots = int(design.slot_width.shape[0])
    d.slot_width = arr(design.slot_width, np.uint16)
    d.n_consts = int(design.const_slot.shape[0])
    d.const_slot = arr(design.const_slot, np.uint32)
    d.const_limbs = arr(np.asarray(design.const_limbs).reshape(-1), np.uint64)
    d.n_inputs = int(design.input_slot.shape[0])
    d.input_slot = arr(design.input_slot, np.uint32)
    d.n_regs = int(design.reg_slot.shape[0])
    d.reg_slot = arr(design.reg_slot, np.uint32)
    d.reg_next = arr(design.reg_next, np.uint32)
    d.n_layers = int(design.layer_ptr.shape[0]) - 1
    d.layer_op_ptr = arr(design.layer_ptr, np.uint32)
    d.n_ops = int(design.op_type.shape[0])
    d.op_type = arr(design.op_type, np.uint8)
    d.op_dst = arr(design.op_dst, np.uint32)
    d.op_src_ptr = arr(design.op_src_ptr, np.uint32)
    d.op_src = arr(design.op_src, np.uint32)
    d.op_imm = arr(design.op_imm, np.uint16)
    if layer_fmt is not None:
        fmts = (rteaal_layer_format * len(layer_fmt))(*layer_fmt)
        keep.append(fmts)
        d.layer_fmt = C.addressof(fmts)
    else:
        d.layer_fmt = None
    return d, keep


def rteaal_validate_design(design, layer_fmt=None):
    """(status, message) from the host-only validator."""
    d, keep = _desc(design, layer_fmt)
    buf = C.create_string_buffer(512)
    st = library().rteaal_validate_design(C.byref(d), buf, 512)
    return st, buf.value.decode()


def rteaal_levelize(ctx, n_slots, op_src_ptr, op_src, op_dst):
    """Layers of a dataflow graph in any operation order, computed on the
    device: (op_layer, order, layer_ptr) as uint32 arrays, layer_ptr holding
    n_layers + 1 entries (see rteaal_levelize in rteaal.h)."""
    ptr = np.ascontiguousarray(op_src_ptr, dtype=np.uint32)
    src = np.ascontiguousarray(op_src, dtype=np.uint32)
    dst = np.ascontiguousarray(op_dst, dtype=np.uint32)
    n = int(dst.shape[0])
    if ptr.shape[0] != n + 1:
        raise ValueError("op_src_ptr needs n_ops + 1 entries")
    g = rteaal_dag_desc(int(n_slots), n, ptr.ctypes.data, src.ctypes.data if src.size else None,
                        dst.ctypes.data if n else None)
    layer = np.zeros(n, np.uint32)
    order = np.zeros(n, np.uint32)
    lptr = np.zeros(n + 1, np.uint32)
    nl = C.c_uint32()
    _check(ctx.handle, library().rteaal_levelize(
        ctx.handle, C.byref(g), layer.ctypes.data if n else None,
        order.ctypes.data if n else None, lptr.ctypes.data, C.byref(nl)))
    return layer, order, lptr[: nl.value + 1].copy()


def levelized_design(ctx, design):
    """A copy of `design` (any object with the array attributes of a design
    description) whose operations are reordered into the layers that
    rteaal_levelize assigns; its own layer_ptr and operation order are
    ignored.  Only the reordering of the operation arrays happens here."""
    import copy
    ptr = np.asarray(design.op_src_ptr, dtype=np.int64)
    _, order, lptr = rteaal_levelize(ctx, design.slot_width.shape[0], design.op_src_ptr,
                                     design.op_src, design.op_dst)
    o = order.astype(np.int64)
    lens = (ptr[1:] - ptr[:-1])[o]
    new_ptr = np.zeros(o.shape[0] + 1, np.int64)
    np.cumsum(lens, out=new_ptr[1:])
    # Operand entries of the reordered operations, each run copied whole.
    starts = np.repeat(ptr[:-1][o] - new_ptr[:-1], lens)
    take = starts + np.arange(int(new_ptr[-1]), dtype=np.int64)
    out = copy.copy(design)
    out.op_type = np.asarray(design.op_type)[o]
    out.op_dst = np.asarray(design.op_dst)[o]
    out.op_imm = np.asarray(design.op_imm)[o]
    out.op_src = np.asarray(design.op_src)[take]
    out.op_src_ptr = new_ptr.astype(np.uint32)
    out.layer_ptr = lptr.astype(np.uint32)
    return out


def rteaal_fuse_mux_chains(design, max_pairs=RTEAAL_MUXC_MAX_PAIRS):
    """Mux-chain fusion on the host (rteaal_fuse_mux_chains in rteaal.h):
    (copy of `design` with the fused operation arrays, counts as a dict)."""
    import copy
    d, keep = _desc(design)
    n, ne, nl = d.n_ops, int(np.asarray(design.op_src_ptr)[-1]), d.n_layers
    lptr = np.zeros(nl + 1, np.uint32)
    typ = np.zeros(max(n, 1), np.uint8)
    dst = np.zeros(max(n, 1), np.uint32)
    sptr = np.zeros(n + 1, np.uint32)
    src = np.zeros(max(ne, 1), np.uint32)
    imm = np.zeros(max(n, 1), np.uint16)
    res = rteaal_fuse_result()
    st = library().rteaal_fuse_mux_chains(C.byref(d), int(max_pairs), lptr.ctypes.data,
                                          typ.ctypes.data, dst.ctypes.data, sptr.ctypes.data,
                                          src.ctypes.data, imm.ctypes.data, C.byref(res))
    _check(None, st)
    k = res.n_ops
    out = copy.copy(design)
    out.layer_ptr = lptr
    out.op_type = typ[:k].copy()
    out.op_dst = dst[:k].copy()
    out.op_src_ptr = sptr[:k + 1].copy()
    out.op_src = src[:res.n_operands].copy()
    out.op_imm = imm[:k].copy()
    return out, {"n_ops": k, "n_operands": res.n_operands, "n_fused": res.n_fused,
                 "n_absorbed": res.n_absorbed}


# Layout of rteaal_change (48 bytes).
CHANGE_DTYPE = np.dtype([("cycle", np.uint64), ("instance", np.uint32), ("signal", np.uint32),
                         ("value", np.uint64, (4,))])


def rteaal_watch(ctx, batch_id, slots, capacity=1 << 20):
    """Watch `slots` of every instance of the batch (empty: stop watching)."""
    sl = np.ascontiguousarray(slots, dtype=np.uint32)
    _check(ctx.handle, library().rteaal_watch(ctx.handle, int(batch_id),
                                              sl.ctypes.data if sl.size else None, int(sl.size),
                                              int(capacity)))


def rteaal_read_changes(ctx, batch_id):
    """Drain the change log: (records as a CHANGE_DTYPE array, dropped count)."""
    lib = library()
    n, dropped = C.c_uint64(), C.c_uint64()
    _check(ctx.handle, lib.rteaal_read_changes(ctx.handle, int(batch_id), None, 0, C.byref(n),
                                               C.byref(dropped)))
    out = np.zeros(max(n.value, 1), CHANGE_DTYPE)
    _check(ctx.handle, lib.rteaal_read_changes(ctx.handle, int(batch_id), out.ctypes.data,
                                               out.size, C.byref(n), C.byref(dropped)))
    return out[: n.value].copy(), int(dropped.value)


RTEAAL_LOAD_KEEP_ALL_SLOTS = 1


def rteaal_load_design(ctx, design, layer_fmt=None, keep_all_slots=False):
    """keep_all_slots: every slot keeps its own storage (rteaal_load_design_ex
    with RTEAAL_LOAD_KEEP_ALL_SLOTS), so RTEAAL_READ_ALL_SLOTS works."""
    d, keep = _desc(design, layer_fmt)
    out = C.c_uint32()
    if keep_all_slots:
        _check(ctx.handle, library().rteaal_load_design_ex(ctx.handle, C.byref(d),
                                                           RTEAAL_LOAD_KEEP_ALL_SLOTS, C.byref(out)))
    else:
        _check(ctx.handle, library().rteaal_load_design(ctx.handle, C.byref(d), C.byref(out)))
    w = np.asarray(design.slot_width, dtype=np.int64)
    regw = w[np.asarray(design.reg_slot, dtype=np.int64)] if design.reg_slot.size else np.zeros(0, np.int64)
    inw = w[np.asarray(design.input_slot, dtype=np.int64)] if design.input_slot.size else np.zeros(0, np.int64)
    ctx.designs[out.value] = (regw, w, int(((inw + 63) // 64).sum()))
    return out.value


def rteaal_unload_design(ctx, design_id):
    _check(ctx.handle, library().rteaal_unload_design(ctx.handle, int(design_id)))
    ctx.designs.pop(design_id, None)


def rteaal_design_format(ctx, design_id, layer):
    f = rteaal_layer_format()
    _check(ctx.handle, library().rteaal_design_format(ctx.handle, int(design_id), int(layer), C.byref(f)))
    return f


def _opts(mapping, block_threads=0, ops_per_wave=0, lds_state=0, lds_ops=0, unroll=0,
          tiles_per_wave=0, arity_split=0, tiles_per_pass=0, persistent=0, partitions=0,
          pass_branches=0):
    return rteaal_batch_opts(int(mapping), int(block_threads), int(ops_per_wave), int(lds_state),
                             int(lds_ops), int(unroll), int(tiles_per_wave), int(arity_split),
                             int(tiles_per_pass), int(persistent), int(partitions),
                             int(pass_branches))


def rteaal_batch_footprint(ctx, design_id, n_instances, mapping=RTEAAL_MAP_AUTO, **opts):
    o = _opts(mapping, **opts)
    out = C.c_uint64()
    _check(ctx.handle, library().rteaal_batch_footprint(ctx.handle, int(design_id), int(n_instances),
                                                        C.byref(o), C.byref(out)))
    return out.value


def rteaal_batch_resources(ctx, design_id, n_instances, mapping=RTEAAL_MAP_AUTO, **opts):
    """(device bytes, LDS bytes held for a whole step) of a batch."""
    o = _opts(mapping, **opts)
    hbm, lds = C.c_uint64(), C.c_uint64()
    _check(ctx.handle, library().rteaal_batch_resources(ctx.handle, int(design_id), int(n_instances),
                                                        C.byref(o), C.byref(hbm), C.byref(lds)))
    return hbm.value, lds.value


def rteaal_partition_plan_stats(ctx, design_id, partitions):
    """The partitioned form's size for `partitions` register partitions (host
    only): dict of design_ops, cone_ops, padded_ops, max_part_ops, exchange."""
    o = rteaal_partition_stats()
    _check(ctx.handle, library().rteaal_partition_plan_stats(ctx.handle, int(design_id),
                                                             int(partitions), C.byref(o)))
    return {k: int(getattr(o, k)) for k, _ in o._fields_}


def rteaal_create_batch(ctx, design_id, seeds, mapping=RTEAAL_MAP_AUTO, **opts):
    """opts: block_threads, ops_per_wave, lds_state, lds_ops, unroll, tiles_per_wave,
    arity_split, tiles_per_pass, persistent, partitions, pass_branches (see
    rteaal_batch_opts)."""
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    o = _opts(mapping, **opts)
    out = C.c_uint32()
    _check(ctx.handle, library().rteaal_create_batch(ctx.handle, int(design_id), int(seeds.shape[0]),
                                                     seeds.ctypes.data, C.byref(o), C.byref(out)))
    ctx.batches[out.value] = (int(design_id), int(seeds.shape[0]))
    return out.value


def rteaal_free_batch(ctx, batch_id):
    _check(ctx.handle, library().rteaal_free_batch(ctx.handle, int(batch_id)))
    ctx.batches.pop(batch_id, None)


def rteaal_batch_info(ctx, batch_id):
    m, c = C.c_uint32(), C.c_uint64()
    _check(ctx.handle, library().rteaal_batch_info(ctx.handle, int(batch_id), C.byref(m), C.byref(c)))
    return m.value, c.value


def rteaal_batch_options(ctx, batch_id):
    """The launch shape the batch resolved to, as a dict."""
    o = rteaal_batch_opts()
    _check(ctx.handle, library().rteaal_batch_options(ctx.handle, int(batch_id), C.byref(o)))
    return opts_dict(o)


def rteaal_step(ctx, batch_id, n_cycles, words=None, words_on_device=False):
    """Enqueue n_cycles.  words: None (generator stimulus), a uint64 numpy array
    [n_cycles][n_inst][W] (host), or a device pointer (int) with words_on_device."""
    if words is None:
        stim = None
    elif words_on_device:
        stim = rteaal_stimulus(1, 1, int(words))
    else:
        words = np.ascontiguousarray(words, dtype=np.uint64)
        stim = rteaal_stimulus(1, 0, words.ctypes.data)
    _check(ctx.handle, library().rteaal_step(ctx.handle, int(batch_id), int(n_cycles),
                                             C.byref(stim) if stim is not None else None))


def _stimulus(words, words_on_device=False):
    """(rteaal_stimulus, buffer to keep alive) for rteaal_step's words argument."""
    if words is None:
        return rteaal_stimulus(0, 0, None), None
    if words_on_device:
        return rteaal_stimulus(1, 1, int(words)), None
    w = np.ascontiguousarray(words, dtype=np.uint64)
    return rteaal_stimulus(1, 0, w.ctypes.data if w.size else None), w


def rteaal_step_many(ctx, batch_ids, n_cycles, words=None, words_on_device=False):
    """words: None (generator stimulus everywhere) or one entry per batch, each
    None or that batch's words as in rteaal_step."""
    ids = np.ascontiguousarray(batch_ids, dtype=np.uint32)
    cyc = np.ascontiguousarray(n_cycles, dtype=np.uint64)
    stims, keep = None, []
    if words is not None:
        if len(words) != ids.shape[0]:
            raise ValueError("words needs one entry per batch")
        arr = (rteaal_stimulus * max(len(words), 1))()
        for k, w in enumerate(words):
            arr[k], buf = _stimulus(w, words_on_device)
            keep.append(buf)
        stims = arr
    _check(ctx.handle, library().rteaal_step_many(ctx.handle, int(ids.shape[0]), ids.ctypes.data,
                                                  cyc.ctypes.data, stims))


def rteaal_sync(ctx):
    _check(ctx.handle, library().rteaal_sync(ctx.handle))


def rteaal_read_state(ctx, batch_id, first=0, n=None, what=RTEAAL_READ_REGS):
    """uint64 array [n][words per instance]: packed limbs (REGS, ALL_SLOTS) or
    the one-word register digest (DIGEST)."""
    design_id, n_inst = ctx.batches[batch_id]
    regw, slotw, _ = ctx.designs[design_id]
    n = n_inst - first if n is None else n
    if what == RTEAAL_READ_DIGEST:
        wpi = 1
    else:
        widths = regw if what == RTEAAL_READ_REGS else slotw
        wpi = int(((widths + 63) // 64).sum())
    out = np.zeros((n, wpi), dtype=np.uint64)
    written = C.c_size_t()
    _check(ctx.handle, library().rteaal_read_state(ctx.handle, int(batch_id), int(first), int(n),
                                                   int(what), out.ctypes.data if out.size else None,
                                                   out.size, C.byref(written)))
    return out


def rteaal_read_state_noalloc(ctx, batch_id, first=0, n=None, what=RTEAAL_READ_REGS):
    """rteaal_read_state through the library's fixed staging array: no device
    allocation (read-outs above RTEAAL_NOALLOC_MAX_WORDS words are refused)."""
    design_id, n_inst = ctx.batches[batch_id]
    regw, slotw, _ = ctx.designs[design_id]
    n = n_inst - first if n is None else n
    if what == RTEAAL_READ_DIGEST:
        wpi = 1
    else:
        widths = regw if what == RTEAAL_READ_REGS else slotw
        wpi = int(((widths + 63) // 64).sum())
    out = np.zeros((n, wpi), dtype=np.uint64)
    written = C.c_size_t()
    _check(ctx.handle, library().rteaal_read_state_noalloc(
        ctx.handle, int(batch_id), int(first), int(n), int(what),
        out.ctypes.data if out.size else None, out.size, C.byref(written)))
    return out


def rteaal_read_digest(ctx, batch_id, first=0, n=None):
    """Register digest of instances [first, first + n): uint64 array [n]."""
    return rteaal_read_state(ctx, batch_id, first, n, RTEAAL_READ_DIGEST).reshape(-1)


def rteaal_write_digest(ctx, batch_id, first, digest):
    dg = np.ascontiguousarray(digest, dtype=np.uint64).reshape(-1)
    _check(ctx.handle, library().rteaal_write_digest(ctx.handle, int(batch_id), int(first),
                                                     int(dg.size), dg.ctypes.data if dg.size else None))


def rteaal_write_state(ctx, batch_id, first, regs, cycle):
    regs = np.ascontiguousarray(regs, dtype=np.uint64)
    n = regs.shape[0]
    _check(ctx.handle, library().rteaal_write_state(ctx.handle, int(batch_id), int(first), int(n),
                                                    regs.ctypes.data if regs.size else None,
                                                    int(cycle)))


def opts_dict(o):
    return {"mapping": o.mapping, "block_threads": o.block_threads, "ops_per_wave": o.ops_per_wave,
            "lds_state": o.lds_state, "lds_ops": o.lds_ops, "unroll": o.unroll,
            "tiles_per_wave": o.tiles_per_wave, "arity_split": o.arity_split,
            "tiles_per_pass": o.tiles_per_pass, "persistent": o.persistent,
            "partitions": o.partitions, "pass_branches": o.pass_branches}


def rteaal_autotune(ctx, design_id, n_instances, trial_cycles=0):
    """(best options as a dict, instance-cycles/s); later AUTO batches use them."""
    o, r = rteaal_batch_opts(), C.c_double()
    _check(ctx.handle, library().rteaal_autotune(ctx.handle, int(design_id), int(n_instances),
                                                 int(trial_cycles), C.byref(o), C.byref(r)))
    return opts_dict(o), r.value


def rteaal_autotune_many(ctx, design_ids, n_instances, trial_cycles=0):
    """(options per batch as dicts, instance-cycles/s of the set); later AUTO
    batches of these (design, instance count) pairs use them."""
    ids = np.ascontiguousarray(design_ids, dtype=np.uint32)
    ni = np.ascontiguousarray(n_instances, dtype=np.uint32)
    out = (rteaal_batch_opts * max(ids.size, 1))()
    r = C.c_double()
    _check(ctx.handle, library().rteaal_autotune_many(ctx.handle, int(ids.size), ids.ctypes.data,
                                                      ni.ctypes.data, int(trial_cycles), out,
                                                      C.byref(r)))
    return [opts_dict(out[k]) for k in range(ids.size)], r.value


def rteaal_kernel_timing(ctx, batch_id, enable):
    """((main launches, main ms), (heavy launches, heavy ms)) recorded since the
    previous call; then sets recording."""
    n, ms = (C.c_uint64 * 2)(), (C.c_double * 2)()
    _check(ctx.handle, library().rteaal_kernel_timing(ctx.handle, int(batch_id), int(bool(enable)),
                                                      n, ms))
    return (n[0], ms[0]), (n[1], ms[1])


# ---------------------------------------------------------------------------
# Layout helpers (host-side reshaping only).
# ---------------------------------------------------------------------------
def unpack_limbs(packed, widths):
    """[n][sum ceil(w/64)] packed limbs -> [n][len(widths)][4] zero-padded limbs."""
    widths = np.asarray(widths, dtype=np.int64)
    nl = (widths + 63) // 64
    off = np.concatenate([[0], np.cumsum(nl)[:-1]]) if nl.size else np.zeros(0, np.int64)
    out = np.zeros((packed.shape[0], widths.shape[0], 4), dtype=np.uint64)
    for l in range(4):
        sel = nl > l
        if sel.any():
            out[:, sel, l] = packed[:, off[sel] + l]
    return out


def pack_limbs(values, widths):
    """[n][len(widths)][4] -> [n][sum ceil(w/64)] packed limbs."""
    widths = np.asarray(widths, dtype=np.int64)
    nl = (widths + 63) // 64
    off = np.concatenate([[0], np.cumsum(nl)[:-1]]) if nl.size else np.zeros(0, np.int64)
    out = np.zeros((values.shape[0], int(nl.sum())), dtype=np.uint64)
    for l in range(4):
        sel = nl > l
        if sel.any():
            out[:, off[sel] + l] = values[:, sel, l]
    return out
