"""Autotuners and their cache on disk (GPU).

rteaal_autotune_many picks one launch policy for a set of designs stepped
together; AUTO batches created afterwards take the chosen options, and the
set stepped with them still equals the oracle.  With RTEAAL_TUNE_CACHE set,
a tuning is written once and read back by a later context instead of being
timed again.  Tolerance 0.
"""
import os

import numpy as np
import pytest

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from tests.gpu_util import assert_same

pytestmark = pytest.mark.gpu

CFGS = [(rtlgen.GenConfig(2000, 10, 60, 8, rtlgen.generator.WIDTHS_MULTIDESIGN, "at-a"), 200),
        (rtlgen.GenConfig(6000, 20, 100, 16, rtlgen.generator.WIDTHS_STD, "at-b"), 3),
        (rtlgen.GenConfig(1000, 5, 20, 8, rtlgen.generator.WIDTHS_LARGE, "at-c"), 20)]


def test_joint_autotune_and_parity():
    ctx = R.rteaal_create(0)
    try:
        ds = [rtlgen.generate(c, 70 + k) for k, (c, _) in enumerate(CFGS)]
        ns = [n for _, n in CFGS]
        ids = [R.rteaal_load_design(ctx, d) for d in ds]
        opts, rate = R.rteaal_autotune_many(ctx, ids, ns, trial_cycles=3)
        assert rate > 0 and len(opts) == 3
        seeds = [np.arange(n, dtype=np.uint64) + 9 * k for k, n in enumerate(ns)]
        bids = [R.rteaal_create_batch(ctx, i, s) for i, s in zip(ids, seeds)]
        for b, o in zip(bids, opts):
            got = R.rteaal_batch_options(ctx, b)
            assert got["mapping"] == o["mapping"], (got, o)
        R.rteaal_step_many(ctx, bids, [7, 7, 7])
        for b, d, s in zip(bids, ds, seeds):
            dg = {}
            ref, _, _ = oracle.run(d, s, 7, digests=dg)
            assert_same(R.unpack_limbs(R.rteaal_read_state(ctx, b), d.slot_width[d.reg_slot]), ref,
                        d.name)
            assert_same(R.rteaal_read_digest(ctx, b), dg["final"], d.name + " digest")
        with pytest.raises(R.RteaalError):
            R.rteaal_autotune_many(ctx, [ids[0], ids[0]], [5, 5])
    finally:
        R.rteaal_destroy(ctx)


def test_tune_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.txt")
    old = os.environ.get("RTEAAL_TUNE_CACHE")
    os.environ["RTEAAL_TUNE_CACHE"] = path
    try:
        d = rtlgen.generate(CFGS[2][0], 72)
        results = []
        for _ in range(2):
            ctx = R.rteaal_create(0)
            try:
                did = R.rteaal_load_design(ctx, d)
                single = R.rteaal_autotune(ctx, did, 100, trial_cycles=2)
                joint = R.rteaal_autotune_many(ctx, [did], [100], trial_cycles=2)
                results.append((single, joint))
            finally:
                R.rteaal_destroy(ctx)
            with open(path) as f:
                lines = f.read().splitlines()
            assert len(lines) == 2, lines          # written by the first context only
        assert results[0][0][0] == results[1][0][0] and results[0][1][0] == results[1][1][0]
        assert abs(results[0][0][1] / results[1][0][1] - 1) < 1e-5
        assert lines[0].startswith("single|") and lines[1].startswith("joint|")
    finally:
        if old is None:
            del os.environ["RTEAAL_TUNE_CACHE"]
        else:
            os.environ["RTEAAL_TUNE_CACHE"] = old
