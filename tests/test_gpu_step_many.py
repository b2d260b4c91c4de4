"""rteaal_step_many with per-batch stimulus (GPU).

Each batch of one multi-batch step takes its own primary-input source:
the generator, host words or device words.  Registers and digests must
equal the oracle run with the same inputs, for batches of every mapping
stepped together; invalid stimulus is refused before anything runs.
Integer arithmetic: tolerance 0.
"""
import numpy as np
import pytest
import torch

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from tests.gpu_util import assert_same, gpu_ctx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    R.rteaal_destroy(c)


def input_words(d):
    return int(((d.slot_width[d.input_slot].astype(np.int64) + 63) // 64).sum())


def test_step_many_words_per_batch(ctx):
    cfgs = [rtlgen.GenConfig(600, 8, 30, 10, rtlgen.generator.WIDTHS_LARGE, "sm-a"),
            rtlgen.GenConfig(900, 12, 40, 7, rtlgen.generator.WIDTHS_STD, "sm-b")]
    designs = [rtlgen.generate(c, 30 + k) for k, c in enumerate(cfgs)]
    dids = [R.rteaal_load_design(ctx, d) for d in designs]
    rng = np.random.default_rng(3)
    plan = []   # (design index, mapping, n_inst, stimulus kind)
    for k in range(2):
        for m in (R.RTEAAL_MAP_RESIDENT, R.RTEAAL_MAP_SWEEP, R.RTEAAL_MAP_LAYERED):
            plan.append((k, m, int(rng.integers(1, 100)), "host"))
    plan += [(0, R.RTEAAL_MAP_SWEEP, 70, "generator"), (1, R.RTEAAL_MAP_RESIDENT, 3, "device")]
    bids, seeds = [], []
    try:
        for k, m, n, _ in plan:
            s = np.arange(n, dtype=np.uint64) * 17 + 5 + k
            seeds.append(s)
            bids.append(R.rteaal_create_batch(ctx, dids[k], s, mapping=m))
        regs = [None] * len(plan)
        dig = [None] * len(plan)
        done = 0
        for step_cycles in (3, 5):
            host_words, args, keep = [], [], []
            for (k, m, n, kind), s in zip(plan, seeds):
                w = rng.integers(0, 2**63, (step_cycles, n, input_words(designs[k])),
                                 dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, dtype=np.uint64)
                if kind == "generator":
                    host_words.append(None)
                    args.append(None)
                elif kind == "device":
                    t = torch.from_numpy(w.view(np.int64).copy()).cuda()
                    torch.cuda.synchronize()
                    keep.append(t)
                    host_words.append(w)
                    args.append(t.data_ptr())
                else:
                    host_words.append(w)
                    args.append(w)
            # words_on_device applies to a whole call: device words go in a call of their own
            host_idx = [i for i, p in enumerate(plan) if p[3] != "device"]
            dev_idx = [i for i, p in enumerate(plan) if p[3] == "device"]
            R.rteaal_step_many(ctx, [bids[i] for i in host_idx], [step_cycles] * len(host_idx),
                               words=[args[i] for i in host_idx])
            R.rteaal_step_many(ctx, [bids[i] for i in dev_idx], [step_cycles] * len(dev_idx),
                               words=[args[i] for i in dev_idx], words_on_device=True)
            R.rteaal_sync(ctx)
            for i, ((k, m, n, kind), s) in enumerate(zip(plan, seeds)):
                dg = {}
                r, _, _ = oracle.run(designs[k], s, step_cycles, start_cycle=done,
                                     stim_words=host_words[i], init_regs=regs[i],
                                     init_digest=dig[i], digests=dg)
                regs[i], dig[i] = r, dg["final"]
            done += step_cycles
        for i, ((k, m, n, kind), b) in enumerate(zip(plan, bids)):
            d = designs[k]
            got = R.unpack_limbs(R.rteaal_read_state(ctx, b), d.slot_width[d.reg_slot])
            assert_same(got, regs[i], f"batch {i} ({kind}, mapping {m}, {n} instances)")
            assert_same(R.rteaal_read_digest(ctx, b), dig[i], f"batch {i} digest")
            assert R.rteaal_batch_info(ctx, b)[1] == 8
    finally:
        for b in bids:
            R.rteaal_free_batch(ctx, b)
        for x in dids:
            R.rteaal_unload_design(ctx, x)


def test_step_many_rejects_bad_stimulus_before_running(ctx):
    d = rtlgen.generate(rtlgen.GenConfig(300, 5, 10, 4, rtlgen.generator.WIDTHS_STD, "sm-bad"), 2)
    did = R.rteaal_load_design(ctx, d)
    a = R.rteaal_create_batch(ctx, did, [1, 2], mapping=R.RTEAAL_MAP_SWEEP)
    b = R.rteaal_create_batch(ctx, did, [3], mapping=R.RTEAAL_MAP_RESIDENT)
    try:
        lib = R.library()
        import ctypes as C
        ids = np.array([a, b], np.uint32)
        cyc = np.array([4, 4], np.uint64)
        stims = (R.rteaal_stimulus * 2)()
        stims[0] = R.rteaal_stimulus(0, 0, None)
        stims[1] = R.rteaal_stimulus(7, 0, None)          # unknown mode
        assert lib.rteaal_step_many(ctx.handle, 2, ids.ctypes.data, cyc.ctypes.data, stims) == 1
        stims[1] = R.rteaal_stimulus(1, 0, None)          # words mode without words
        assert lib.rteaal_step_many(ctx.handle, 2, ids.ctypes.data, cyc.ctypes.data, stims) == 1
        assert lib.rteaal_step_many(ctx.handle, 2, np.array([a, a], np.uint32).ctypes.data,
                                    cyc.ctypes.data, None) == 1      # batch listed twice
        assert R.rteaal_batch_info(ctx, a)[1] == 0 and R.rteaal_batch_info(ctx, b)[1] == 0
        assert (R.rteaal_read_digest(ctx, a) == 0).all()
        del C
    finally:
        R.rteaal_free_batch(ctx, a)
        R.rteaal_free_batch(ctx, b)
        R.rteaal_unload_design(ctx, did)
