"""Pins of the oracle levelizer against facts that do not come from it.

* Closed forms: a chain of k operations has layers 0..k-1 in chain order; a
  reduction tree over 2^d sources has its level-j operations in layer j - 1.
* Brute force on tiny graphs: the longest chain of operations ending at each
  operation, by enumerating every chain (no memoization), and the presence
  of a cycle by transitive closure.
* Characterization at any size: a layering in which every operation sits
  strictly above all its producers (validity) and directly above at least
  one of them unless it reads only sources (tightness) is exactly the
  longest-chain layering (induction on the layer), so the two properties pin
  the result on generated designs too.
"""
import itertools

import numpy as np
import pytest

import oracle
import rtlgen
from oracle.levelize import NotLevelizable


def _graph(n_slots, ops):
    """ops: list of (dst, [src...]) -> CSR arrays."""
    ptr = [0]
    src = []
    dst = []
    for d, s in ops:
        dst.append(d)
        src.extend(s)
        ptr.append(len(src))
    return n_slots, np.array(ptr, np.uint32), np.array(src, np.uint32), np.array(dst, np.uint32)


def _shuffled(n_slots, ops, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(ops))
    return [ops[i] for i in perm], perm


def test_chain_closed_form():
    k = 40
    # slot 0 is a source; operation j writes slot j + 1 from slot j.
    ops = [(j + 1, [j]) for j in range(k)]
    sh, perm = _shuffled(k + 1, ops, 3)
    layer = oracle.levelize(*_graph(k + 1, sh))
    assert list(layer) == [int(p) for p in perm]        # operation j of the chain -> layer j


def test_reduction_tree_closed_form():
    d = 6
    n_src = 1 << d
    ops, level = [], []
    cur = list(range(n_src))
    nxt_slot = n_src
    for lv in range(1, d + 1):
        nxt = []
        for a, b in zip(cur[0::2], cur[1::2]):
            ops.append((nxt_slot, [a, b]))
            level.append(lv)
            nxt.append(nxt_slot)
            nxt_slot += 1
        cur = nxt
    sh, perm = _shuffled(nxt_slot, ops, 5)
    layer = oracle.levelize(*_graph(nxt_slot, sh))
    assert list(layer) == [level[p] - 1 for p in perm]
    assert layer.max() == d - 1


def _random_dag(rng, n_ops, n_src, max_ar=3):
    """Operation j may read sources and outputs of operations < j (a hidden
    topological order); the list is returned shuffled."""
    ops = []
    for j in range(n_ops):
        ar = int(rng.integers(1, max_ar + 1))
        s = [int(rng.integers(0, n_src + j)) for _ in range(ar)]   # slot n_src + i = output of op i
        ops.append((n_src + j, s))
    perm = rng.permutation(n_ops)
    return [ops[i] for i in perm]


def _brute_longest(n_src, ops):
    """Longest chain of operations ending at each operation, by enumerating
    every chain through the producers (exponential: tiny graphs only)."""
    prod = {d: i for i, (d, _) in enumerate(ops)}

    def longest(i):
        best = 0
        for s in ops[i][1]:
            if s in prod:
                best = max(best, 1 + longest(prod[s]))
        return best
    return [longest(i) for i in range(len(ops))]


def test_brute_force_longest_chains():
    rng = np.random.default_rng(11)
    for trial in range(300):
        n_src = int(rng.integers(1, 4))
        n_ops = int(rng.integers(1, 11))
        ops = _random_dag(rng, n_ops, n_src)
        layer = oracle.levelize(*_graph(n_src + n_ops, ops))
        assert list(layer) == _brute_longest(n_src, ops), trial


def _has_cycle(n_src, ops):
    """Transitive closure of 'operation a feeds operation b'."""
    n = len(ops)
    prod = {d: i for i, (d, _) in enumerate(ops)}
    reach = np.zeros((n, n), bool)
    for b, (_, s) in enumerate(ops):
        for x in s:
            if x in prod:
                reach[prod[x], b] = True
    for k, i, j in itertools.product(range(n), repeat=3):
        if reach[i, k] and reach[k, j]:
            reach[i, j] = True
    return bool(reach.diagonal().any())


def test_cycles_detected_exactly():
    rng = np.random.default_rng(12)
    seen = {True: 0, False: 0}
    for trial in range(300):
        n_src = 2
        n_ops = int(rng.integers(1, 7))
        ops = []
        for j in range(n_ops):     # operands anywhere, own output included: cycles happen
            ar = int(rng.integers(1, 3))
            ops.append((n_src + j, [int(rng.integers(0, n_src + n_ops)) for _ in range(ar)]))
        cyc = _has_cycle(n_src, ops)
        seen[cyc] += 1
        if cyc:
            with pytest.raises(NotLevelizable):
                oracle.levelize(*_graph(n_src + n_ops, ops))
        else:
            layer = oracle.levelize(*_graph(n_src + n_ops, ops))
            assert list(layer) == _brute_longest(n_src, ops)
    assert seen[True] > 20 and seen[False] > 20


def test_two_writers_rejected():
    with pytest.raises(NotLevelizable, match="slot 3"):
        oracle.levelize(*_graph(5, [(3, [0]), (4, [3]), (3, [1])]))


def test_self_loop_is_a_cycle():
    with pytest.raises(NotLevelizable):
        oracle.levelize(*_graph(3, [(2, [0, 2])]))


def _check_characterization(n_slots, ptr, src, dst, layer):
    prod = np.full(n_slots, -1, np.int64)
    prod[dst.astype(np.int64)] = np.arange(dst.size)
    for o in range(dst.size):
        ps = [int(prod[s]) for s in src[ptr[o]:ptr[o + 1]] if prod[s] >= 0]
        assert all(layer[o] > layer[p] for p in ps)                          # validity
        assert (layer[o] == 0) if not ps else (max(layer[p] for p in ps) == layer[o] - 1)  # tightness


def test_generated_designs_characterization():
    for cfg, seed in ((rtlgen.CFG0, 0), (rtlgen.GenConfig(20_000, 30, 200, 16,
                                                           rtlgen.generator.WIDTHS_LARGE, "g"), 7)):
        d = rtlgen.generate(cfg, seed)
        layer = oracle.levelize(d.slot_width.size, d.op_src_ptr, d.op_src, d.op_dst)
        _check_characterization(d.slot_width.size, d.op_src_ptr, d.op_src, d.op_dst, layer)
        # The generator's layers are a valid slicing, so the fewest layers is at most its count.
        assert layer.max() + 1 <= d.layer_ptr.size - 1
        gen_layer = np.repeat(np.arange(d.layer_ptr.size - 1), np.diff(d.layer_ptr.astype(np.int64)))
        assert (layer <= gen_layer).all()


def test_layer_order():
    layer = np.array([2, 0, 1, 0, 2, 1, 0])
    order, ptr = oracle.layer_order(layer)
    assert list(order) == [1, 3, 6, 2, 5, 0, 4]
    assert list(ptr) == [0, 3, 5, 7]
    order, ptr = oracle.layer_order(np.zeros(0, np.int64))
    assert order.size == 0 and list(ptr) == [0]
