"""The C interface on the host (no GPU): exports, validation and error paths."""
import copy
import re
import os

import numpy as np
import pytest

import rtlgen
from rtlgen import circuits as cir
from paper_2601_18140_amd import rteaal as R

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "rteaal.h")


def test_library_exports_every_declared_function():
    lib = R.library()
    decl = set(re.findall(r"\b(rteaal_[a-z_]+)\s*\(", open(HEADER).read()))
    assert decl == set(R.exported_symbols())
    for name in decl:
        assert hasattr(lib, name), name


def _clone(d):
    return copy.deepcopy(d)


@pytest.fixture(scope="module")
def good():
    return rtlgen.generate(rtlgen.GenConfig(300, 6, 20, 8, rtlgen.generator.WIDTHS_LARGE, "v"), 5)


def expect(design, status, fragment=""):
    st, msg = R.rteaal_validate_design(design)
    assert st == status, (st, msg)
    assert fragment in msg, msg


def test_generated_and_closed_form_designs_validate(good):
    expect(good, 0)
    for d in (cir.ripple_carry_adder(5), cir.counter(70), cir.xnor_lfsr(9),
              cir.shift_chain(3, 4, True), cir.paper_multiply_example()):
        expect(d, 0)
    expect(rtlgen.generate(rtlgen.CFG0, 0), 0)


def test_width_out_of_range(good):
    d = _clone(good)
    d.slot_width[3] = 0
    expect(d, 2, "width")
    d.slot_width[3] = 257
    expect(d, 2, "width")


def test_two_drivers(good):
    d = _clone(good)
    d.op_dst[5] = d.op_dst[6]
    expect(d, 2, "more than one driver")


def test_not_levelized(good):
    d = _clone(good)
    j = int(d.layer_ptr[2])                      # first op of layer 2
    d.op_src[d.op_src_ptr[j]] = d.op_dst[j + 1]  # reads an output of its own layer
    expect(d, 2, "not levelized")
    d = _clone(good)
    j = int(d.layer_ptr[1])
    d.op_src[d.op_src_ptr[j]] = d.op_dst[int(d.layer_ptr[4])]  # a later layer
    expect(d, 2, "not levelized")


def test_undriven_operand(good):
    d = _clone(good)
    d.slot_width = np.concatenate([d.slot_width, [7]]).astype(np.uint16)
    j = int(d.layer_ptr[3])
    d.op_src[d.op_src_ptr[j]] = d.n_slots - 1
    expect(d, 2, "no driver")


def test_wrong_arity(good):
    d = _clone(good)
    j = int(np.nonzero(d.op_type == rtlgen.NOT)[0][0])
    d.op_type[j] = rtlgen.SUB
    expect(d, 2, "cannot take")


def test_immediate_out_of_range(good):
    d = _clone(good)
    j = int(np.nonzero(d.op_type == rtlgen.SHL)[0][0])
    d.op_imm[j] = 300
    expect(d, 2, "immediate")
    d = _clone(good)
    j = int(np.nonzero(d.op_type == rtlgen.ADD)[0][0])
    d.op_imm[j] = 1
    expect(d, 2, "immediate")


def test_register_out_of_range(good):
    d = _clone(good)
    d.reg_next[0] = d.n_slots + 10
    expect(d, 2, "out of range")


def test_layer_pointer_errors(good):
    d = _clone(good)
    d.layer_ptr[-1] = d.layer_ptr[-1] - 1
    expect(d, 2, "layer_op_ptr")


def _formats(d):
    out = []
    for i in range(d.n_layers):
        f = R.rteaal_layer_format()
        a, b = int(d.layer_ptr[i]), int(d.layer_ptr[i + 1])
        maxs = int(d.op_dst[a:b].max())
        maxr = int(d.op_src[d.op_src_ptr[a]:d.op_src_ptr[b]].max())
        cnt = np.bincount(d.op_type[a:b], minlength=15).max()
        f.oim[1].pbits = int(cnt).bit_length()
        f.oim[2].compressed, f.oim[2].cbits = 1, max(1, maxs.bit_length())
        f.oim[4].compressed, f.oim[4].cbits = 1, max(1, maxr.bit_length())
        out.append(f)
    return out


def test_caller_formats_checked(good):
    fm = _formats(good)
    st, msg = R.rteaal_validate_design(good, fm)
    assert st == 0, msg
    fm[2].oim[4].cbits -= 1                      # R coordinates no longer fit
    st, msg = R.rteaal_validate_design(good, fm)
    assert st == 3 and "rank 4" in msg
    fm = _formats(good)
    fm[1].oim[1].pbits -= 1                      # N payloads no longer fit
    st, msg = R.rteaal_validate_design(good, fm)
    assert st == 3 and "payloads" in msg


def test_null_descriptor():
    lib = R.library()
    buf = R.C.create_string_buffer(128)
    assert lib.rteaal_validate_design(None, buf, 128) == 1


def test_no_device_is_a_clean_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    out = R.C.c_void_p()
    st = R.library().rteaal_create(0, None, None, R.C.byref(out))
    assert st == 1 and not out.value
    assert "device" in R.rteaal_last_error(None)


def test_limb_packing_roundtrip():
    rng = np.random.default_rng(0)
    widths = np.array([1, 64, 65, 200, 256, 7])
    vals = rng.integers(0, 2**63, size=(3, 6, 4), dtype=np.uint64)
    nl = (widths + 63) // 64
    for k in range(6):
        vals[:, k, nl[k]:] = 0
    assert np.array_equal(R.unpack_limbs(R.pack_limbs(vals, widths), widths), vals)


@pytest.mark.parametrize("seed,max_pairs", [(1, 32), (2, 3), (3, 2), (4, 1)])
def test_fuse_mux_chains_matches_the_oracle_pass(seed, max_pairs):
    """The library's fusion (host code, no device) gives exactly the
    operation arrays of the oracle's pass; the result validates."""
    import oracle
    cfg = rtlgen.GenConfig(20_000, 20, 400, 16, rtlgen.generator.WIDTHS_LARGE, "chains", mux_chain=0.85)
    d = rtlgen.generate(cfg, seed)
    ref, n_fused, n_abs = oracle.fuse_mux_chains(d, max_pairs)
    got, cnt = R.rteaal_fuse_mux_chains(d, max_pairs)
    assert cnt == {"n_ops": ref.n_ops, "n_operands": int(ref.op_src_ptr[-1]), "n_fused": n_fused,
                   "n_absorbed": n_abs}
    for k in ("layer_ptr", "op_type", "op_dst", "op_src_ptr", "op_src", "op_imm"):
        assert np.array_equal(np.asarray(getattr(got, k), np.int64), np.asarray(getattr(ref, k), np.int64)), k
    assert R.rteaal_validate_design(got)[0] == 0
    # fusing again finds nothing more (MUXC is never absorbed or extended)
    again, cnt2 = R.rteaal_fuse_mux_chains(got, max_pairs)
    assert cnt2["n_fused"] == 0 and cnt2["n_absorbed"] == 0 and again.n_ops == got.n_ops


def test_fuse_mux_chains_errors_and_muxc_arity(good):
    for mp in (0, 33):
        with pytest.raises(R.RteaalError) as e:
            R.rteaal_fuse_mux_chains(good, mp)
        assert e.value.status == 1
    bad = _clone(good)
    bad.slot_width[0] = 0
    with pytest.raises(R.RteaalError) as e:
        R.rteaal_fuse_mux_chains(bad, 32)
    assert e.value.status == 2
    # MUXC takes an odd number 3..65 of operands
    b = cir.Builder("m")
    ins = [b.input(8) for _ in range(67)]
    ok = b.op(rtlgen.MUXC, ins[:65], 8)
    r = b.reg(8)
    b.connect(r, ok)
    assert R.rteaal_validate_design(b.build())[0] == 0
    for n in (2, 4, 67):
        b2 = cir.Builder("m")
        ins = [b2.input(8) for _ in range(n)]
        r = b2.reg(8)
        b2.connect(r, b2.op(rtlgen.MUXC, ins, 8))
        assert R.rteaal_validate_design(b2.build())[0] == 2


def test_fuse_mux_chains_edge_designs():
    """No operations; MUXes whose default is a register or an input (no link);
    a chain whose head is latched by a register (the head stays, fused)."""
    b = cir.Builder("empty")
    r = b.reg(4)
    b.connect(r, b.input(4))
    d = b.build()
    f, cnt = R.rteaal_fuse_mux_chains(d)
    assert cnt == {"n_ops": 0, "n_operands": 0, "n_fused": 0, "n_absorbed": 0}
    assert list(f.layer_ptr) == list(d.layer_ptr)
    b = cir.Builder("sources")
    s, x, y = b.input(1), b.input(8), b.reg(8)
    m1 = b.op(rtlgen.MUX, [s, x, y], 8)
    m2 = b.op(rtlgen.MUX, [s, x, b.input(8)], 8)
    b.connect(y, b.op(rtlgen.XOR, [m1, m2], 8))
    f, cnt = R.rteaal_fuse_mux_chains(b.build())
    assert cnt["n_fused"] == 0 and cnt["n_absorbed"] == 0
    b = cir.Builder("latched-head")
    s1, s2, a, c, e = b.input(1), b.input(1), b.input(8), b.input(8), b.input(8)
    inner = b.op(rtlgen.MUX, [s2, c, e], 8)
    head = b.op(rtlgen.MUX, [s1, a, inner], 8)
    r = b.reg(8)
    b.connect(r, head)
    f, cnt = R.rteaal_fuse_mux_chains(b.build())
    assert cnt == {"n_ops": 1, "n_operands": 5, "n_fused": 1, "n_absorbed": 1}
    assert int(f.op_type[0]) == rtlgen.MUXC and int(f.op_dst[0]) == head
    assert [int(v) for v in f.op_src] == [s1, a, s2, c, e]


def test_header_is_plain_c(tmp_path):
    """include/rteaal.h is a C header: it compiles as C99 with -pedantic and
    declares every exported entry point."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "rteaal.h"\n'
                   "int main(void) {\n"
                   "  rteaal_fuse_result r; rteaal_batch_opts o; rteaal_change c;\n"
                   "  rteaal_status (*fuse)(const rteaal_design_desc*, uint32_t, uint32_t*, uint8_t*,\n"
                   "                        uint32_t*, uint32_t*, uint32_t*, uint16_t*,\n"
                   "                        rteaal_fuse_result*) = rteaal_fuse_mux_chains;\n"
                   "  rteaal_status (*many)(rteaal_ctx*, uint32_t, const rteaal_batch_id*,\n"
                   "                        const uint64_t*, const rteaal_stimulus*) = rteaal_step_many;\n"
                   "  rteaal_status (*wdig)(rteaal_ctx*, rteaal_batch_id, uint32_t, uint32_t,\n"
                   "                        const uint64_t*) = rteaal_write_digest;\n"
                   "  (void)r; (void)o; (void)c; (void)fuse; (void)many; (void)wdig;\n"
                   "  return RTEAAL_MUXC == 22 && RTEAAL_MUXC_MAX_PAIRS == 32 &&\n"
                   "         RTEAAL_READ_REGS == 1 && RTEAAL_READ_DIGEST == 2 &&\n"
                   "         RTEAAL_READ_ALL_SLOTS == 4 ? 0 : 1;\n"
                   "}\n")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-fsyntax-only",
                        "-I", os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
