"""Oracle levelizer (test infrastructure only).

Levelization as the paper states it (section "Evaluating Arbitrary Dataflow
Graphs"): slice the dataflow graph into layers so that every operation
depends only on outputs of layers above it.  Of all such slicings this
oracle gives the one with the fewest layers, where an operation's layer is
the length of the longest chain of operations ending at it:

    layer(o) = 0                                  if every operand of o is a source,
    layer(o) = 1 + max{ layer(p) : p produces an operand of o }   otherwise,

a source being a slot that no operation writes (primary input, register or
constant).  The definition is followed literally: a depth-first walk from
each operation to its producers, memoizing finished operations.  A graph
with a slot written twice, or with a cycle, has no levelization and raises.

Plain Python loops: meant for graphs of up to a few hundred thousand
operations.
"""
from __future__ import annotations

import numpy as np


class NotLevelizable(ValueError):
    """The graph has a slot with two writers or a combinational cycle."""


def producers(n_slots, op_dst):
    """producer[slot] = the operation writing it, or -1 for a source."""
    prod = [-1] * int(n_slots)
    for o, d in enumerate(op_dst):
        d = int(d)
        if prod[d] != -1:
            raise NotLevelizable(f"slot {d} is written by operations {prod[d]} and {o}")
        prod[d] = o
    return prod


def levelize(n_slots, op_src_ptr, op_src, op_dst):
    """Layer of every operation (int64 array) by the definition above."""
    n = len(op_dst)
    ptr = [int(x) for x in op_src_ptr]
    src = [int(x) for x in op_src]
    prod = producers(n_slots, op_dst)
    feeds = [[prod[src[k]] for k in range(ptr[o], ptr[o + 1]) if prod[src[k]] != -1]
             for o in range(n)]
    UNSEEN, OPEN = -2, -1           # states before a layer is known
    layer = [UNSEEN] * n
    for root in range(n):
        if layer[root] != UNSEEN:
            continue
        stack = [(root, 0)]
        layer[root] = OPEN
        while stack:
            o, i = stack[-1]
            if i < len(feeds[o]):
                stack[-1] = (o, i + 1)
                p = feeds[o][i]
                if layer[p] == OPEN:
                    raise NotLevelizable(f"operation {p} lies on a cycle")
                if layer[p] == UNSEEN:
                    layer[p] = OPEN
                    stack.append((p, 0))
            else:
                stack.pop()
                layer[o] = 1 + max((layer[p] for p in feeds[o]), default=-1)
    return np.asarray(layer, dtype=np.int64)


def layer_order(layer):
    """Operations sorted by (layer, index) and the layer ranges in it."""
    layer = np.asarray(layer, dtype=np.int64)
    n_layers = int(layer.max()) + 1 if layer.size else 0
    order = sorted(range(layer.size), key=lambda o: (int(layer[o]), o))
    counts = np.bincount(layer, minlength=n_layers) if layer.size else np.zeros(0, np.int64)
    ptr = np.zeros(n_layers + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return np.asarray(order, dtype=np.int64), ptr
