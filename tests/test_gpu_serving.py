"""Continuous-batching serving loop (GPU).

Jobs of several designs arrive while others run; a small memory budget
forces queueing.  Each job's result must equal the oracle and the job run
alone (integer arithmetic: tolerance 0), and the budget must hold at every
tick.
"""
import numpy as np
import pytest

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from paper_2601_18140_amd import serving
from tests.gpu_util import assert_same, gpu_ctx, run_gpu

pytestmark = pytest.mark.gpu


class BudgetWatch(serving.Server):
    peak = 0

    def tick(self):
        n = super().tick()
        self.peak = max(self.peak, self.used)
        assert self.used <= self.budget
        return n


def test_serving_matches_alone_and_oracle():
    ctx = gpu_ctx()
    try:
        pool = [rtlgen.generate(rtlgen.GenConfig(n, l, 24, 8, w, f"pool{i}"), 500 + i)
                for i, (n, l, w) in enumerate([(800, 6, rtlgen.generator.WIDTHS_STD),
                                               (3000, 14, rtlgen.generator.WIDTHS_LARGE),
                                               (1500, 9, rtlgen.generator.WIDTHS_MULTIDESIGN),
                                               (400, 4, rtlgen.generator.WIDTHS_STD)])]
        rng = np.random.default_rng(3)
        jobs = [serving.Job(job_id=k, design=int(rng.integers(0, 4)),
                            n_inst=int(rng.choice([1, 2, 5, 33, 64, 90])),
                            n_cycles=int(rng.integers(20, 300))) for k in range(14)]
        # Budget: room for the designs plus about three typical batches.
        srv = BudgetWatch(ctx, pool, budget_bytes=6 << 20, chunk_cycles=37)
        arrivals = serving.poisson_arrivals(200.0, len(jobs), seed=9)
        stats = srv.run(jobs, arrivals)
        assert stats["jobs"] == len(jobs)
        assert stats["latency_p50_s"] is not None and stats["latency_p99_s"] >= stats["latency_p50_s"]
        assert srv.peak <= srv.budget
        assert max(j.admitted - j.arrival for j in jobs) > 0   # some job had to wait
        srv.close()
        for j in jobs:
            d = pool[j.design]
            got = R.unpack_limbs(j.regs, d.slot_width[d.reg_slot])
            alone, _, _ = run_gpu(ctx, d, j.seeds, j.n_cycles)
            assert_same(got, alone, f"job {j.job_id} alone")
            pick = [0, j.n_inst - 1]
            ref, _, _ = oracle.run(d, j.seeds[pick], j.n_cycles)
            assert_same(got[pick], ref, f"job {j.job_id} oracle")
    finally:
        R.rteaal_destroy(ctx)
