"""Parity of the device levelizer (rteaal_levelize) with the oracle levelizer.

Layers are integers: every comparison is exact.  Graphs: generated designs
with their operations shuffled (the order a netlist may come in), deep
chains, wide single layers, heavy fan-out, repeated operands, and the error
cases.  A levelized design must also simulate exactly as the original.  At
the full 5M-operation size, where the Python oracle is too slow, the result
is checked against the two properties that characterize the oracle's
layering (validity and tightness, pinned in test_oracle_levelize.py).
"""
import copy
import sys

import numpy as np
import pytest

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from tests.gpu_util import assert_same, gpu_ctx, run_gpu

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    R.rteaal_destroy(c)


def shuffled(d, seed):
    """The design with its operations in a random order (layer_ptr dropped)."""
    rng = np.random.default_rng(seed)
    o = rng.permutation(d.op_type.size)
    ptr = d.op_src_ptr.astype(np.int64)
    lens = (ptr[1:] - ptr[:-1])[o]
    new_ptr = np.zeros(o.size + 1, np.int64)
    np.cumsum(lens, out=new_ptr[1:])
    take = np.repeat(ptr[:-1][o] - new_ptr[:-1], lens) + np.arange(int(new_ptr[-1]))
    return dict(n_slots=d.slot_width.size, op_src_ptr=new_ptr.astype(np.uint32),
                op_src=d.op_src[take], op_dst=d.op_dst[o], perm=o)


def check_against_oracle(ctx, n_slots, ptr, src, dst):
    layer, order, lptr = R.rteaal_levelize(ctx, n_slots, ptr, src, dst)
    ref = oracle.levelize(n_slots, ptr, src, dst)
    ref_order, ref_ptr = oracle.layer_order(ref)
    assert np.array_equal(layer.astype(np.int64), ref)
    assert np.array_equal(order.astype(np.int64), ref_order)
    assert np.array_equal(lptr.astype(np.int64), ref_ptr)
    return layer


def csr(ops):
    ptr, src, dst = [0], [], []
    for d, s in ops:
        dst.append(d)
        src.extend(s)
        ptr.append(len(src))
    return np.array(ptr, np.uint32), np.array(src, np.uint32), np.array(dst, np.uint32)


@pytest.mark.parametrize("cfg,seed", [(rtlgen.CFG0, 0),
                                      (rtlgen.GenConfig(30_001, 37, 300, 17,
                                                        rtlgen.generator.WIDTHS_LARGE, "l30k"), 9)],
                         ids=["plain-2k", "30k-ragged"])
def test_shuffled_generated_designs(ctx, cfg, seed):
    d = rtlgen.generate(cfg, seed)
    g = shuffled(d, seed + 1)
    note(f"levelize {cfg.name}: {d.op_type.size} ops")
    layer = check_against_oracle(ctx, g["n_slots"], g["op_src_ptr"], g["op_src"], g["op_dst"])
    assert layer.max() + 1 <= d.layer_ptr.size - 1


def test_special_graphs(ctx):
    rng = np.random.default_rng(4)
    k = 3000   # deep chain, shuffled: one operation per layer
    perm = rng.permutation(k)
    ops = [(perm_j + 1, [perm_j]) for perm_j in perm]
    check_against_oracle(ctx, k + 1, *csr(ops))
    # wide: 100k operations reading only sources (one layer, ragged grid)
    n = 100_003
    ops = [(16 + j, [j % 16, (j * 7) % 16]) for j in range(n)]
    check_against_oracle(ctx, 16 + n, *csr(ops))
    # fan-out: 50k consumers of one operation, repeated operands, unary and ternary
    ops = [(1, [0])] + [(2 + j, [1, 1, 0][: 1 + j % 3]) for j in range(50_000)]
    check_against_oracle(ctx, 2 + 50_000, *csr(ops))
    # a single operation; then no operation at all
    check_against_oracle(ctx, 2, *csr([(1, [0])]))
    layer, order, lptr = R.rteaal_levelize(ctx, 5, np.zeros(1, np.uint32), np.zeros(0, np.uint32),
                                           np.zeros(0, np.uint32))
    assert layer.size == 0 and order.size == 0 and list(lptr) == [0]


def test_errors(ctx):
    # two writers of slot 3 (and of 4): the smaller slot is named
    with pytest.raises(R.RteaalError, match="slot 3") as e:
        R.rteaal_levelize(ctx, 6, *csr([(4, [0]), (3, [0]), (3, [1]), (4, [2])]))
    assert e.value.status == 2
    # cycle 2 -> 3 -> 4 -> 2 with operation 3 behind it; operation 0 is fine
    ops = [(1, [0]), (2, [4, 1]), (3, [2]), (4, [3]), (5, [4])]
    with pytest.raises(R.RteaalError, match="operation 1 lies on or behind a cycle") as e:
        R.rteaal_levelize(ctx, 6, *csr(ops))
    assert e.value.status == 2
    with pytest.raises(R.RteaalError, match="cycle") as e:
        R.rteaal_levelize(ctx, 3, *csr([(2, [0, 2])]))            # reads its own output
    # arguments the kernels would index with
    with pytest.raises(R.RteaalError) as e:
        R.rteaal_levelize(ctx, 3, *csr([(2, [0, 7])]))
    assert e.value.status == 1
    with pytest.raises(R.RteaalError) as e:
        R.rteaal_levelize(ctx, 3, *csr([(5, [0])]))
    assert e.value.status == 1
    with pytest.raises(R.RteaalError) as e:
        R.rteaal_levelize(ctx, 3, np.array([0, 2, 1], np.uint32), np.array([0, 1], np.uint32),
                          np.array([1, 2], np.uint32))
    assert e.value.status == 1
    # the context stays usable
    check_against_oracle(ctx, 2, *csr([(1, [0])]))


@pytest.mark.parametrize("mapping", [R.RTEAAL_MAP_RESIDENT, R.RTEAAL_MAP_SWEEP],
                         ids=["resident", "sweep"])
def test_levelized_design_simulates_like_the_original(ctx, mapping):
    d = rtlgen.generate(rtlgen.GenConfig(4_000, 12, 64, 8, rtlgen.generator.WIDTHS_LARGE, "l4k"), 21)
    g = shuffled(d, 22)
    s = copy.copy(d)
    o = g["perm"]
    s.op_type, s.op_dst, s.op_imm = d.op_type[o], d.op_dst[o], d.op_imm[o]
    s.op_src_ptr, s.op_src = g["op_src_ptr"], g["op_src"]
    s.layer_ptr = np.array([0, o.size], np.uint32)         # one layer: not levelized
    assert R.rteaal_validate_design(s)[0] == 2
    lv = R.levelized_design(ctx, s)
    assert R.rteaal_validate_design(lv)[0] == 0
    seeds = rtlgen.instance_seeds(70)
    note(f"simulate levelized l4k, mapping {mapping}")
    got, _, _ = run_gpu(ctx, lv, seeds, 40, mapping=mapping)
    ref, _, _ = oracle.run(d, seeds, 40)
    assert_same(got, ref, "levelized design vs original (oracle)")


def test_full_size_properties(ctx):
    cfg = rtlgen.WORKLOADS["large-5m"]
    d = rtlgen.generate(cfg["cfg"], cfg["seed"])
    g = shuffled(d, 5)
    note(f"levelize large-5m shuffled: {d.op_type.size} ops")
    layer, order, lptr = R.rteaal_levelize(ctx, g["n_slots"], g["op_src_ptr"], g["op_src"],
                                           g["op_dst"])
    L = layer.astype(np.int64)
    ptr = g["op_src_ptr"].astype(np.int64)
    prod = np.full(g["n_slots"], -1, np.int64)
    prod[g["op_dst"].astype(np.int64)] = np.arange(L.size)
    p = prod[g["op_src"].astype(np.int64)]
    owner = np.repeat(np.arange(L.size), np.diff(ptr))
    fed = p >= 0
    assert (L[owner[fed]] > L[p[fed]]).all()                          # validity
    best = np.full(L.size, -1, np.int64)
    np.maximum.at(best, owner[fed], L[p[fed]])
    assert np.array_equal(L, best + 1)                                # tightness
    n_layers = lptr.size - 1
    assert n_layers == L.max() + 1 <= d.layer_ptr.size - 1
    assert np.array_equal(np.sort(order), np.arange(L.size))
    assert (np.diff(L[order.astype(np.int64)]) >= 0).all()
    assert np.array_equal(np.diff(lptr.astype(np.int64)), np.bincount(L, minlength=n_layers))
