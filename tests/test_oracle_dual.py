"""The C oracle against an independent pure-Python interpreter (no GPU).

Supplements the pins in test_oracle_pins.py: both sides start from the
same integer definitions, but the whole-design plumbing (stimulus, operand
gather, layer write-back, register commit, limbs) is written twice.
"""
import numpy as np
import pytest

import rtlgen
from rtlgen.design import limbs_to_int
from tests.intref import simulate

CASES = [
    rtlgen.GenConfig(120, 5, 10, 6, rtlgen.generator.WIDTHS_STD, "tiny-std"),
    rtlgen.GenConfig(150, 7, 12, 5, rtlgen.generator.WIDTHS_LARGE, "tiny-wide"),
    rtlgen.GenConfig(90, 3, 4, 3, rtlgen.generator.WIDTHS_MULTIDESIGN, "tiny-multi"),
    rtlgen.GenConfig(160, 6, 10, 6, rtlgen.generator.WIDTHS_LARGE, "tiny-all-types",
                     rtlgen.OP_MIX_FULL),
]


@pytest.mark.parametrize("cfg", CASES, ids=[c.name for c in CASES])
@pytest.mark.parametrize("seed", [0, 1])
def test_dual_interpreter(oracle_lib, cfg, seed):
    d = rtlgen.generate(cfg, seed)
    seeds = [seed * 100 + 1, seed * 100 + 2]
    _, slots, _ = oracle_lib.run(d, seeds, 12, want_slots=True, start_cycle=5)
    for i, s in enumerate(seeds):
        ref = simulate(d, s, 12, start_cycle=5)
        got = [limbs_to_int(slots[i, k]) for k in range(d.n_slots)]
        assert got == ref
