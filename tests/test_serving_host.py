"""Host logic of the continuous-batching loop, on the CPU.

The loop drives the library only through the binding's calls, so here a
stand-in binding advances every batch with the oracle (resuming from the
batch's registers and cycle).  This checks, without a GPU: admission by
device memory and by LDS within their budgets (jobs wait when either is
full), per-tick chunks,
retirement, that every job's registers equal one uninterrupted oracle run,
and the latency summary.
"""
import numpy as np
import pytest

import oracle
import rtlgen
from paper_2601_18140_amd import rteaal as R
from paper_2601_18140_amd import serving


class FakeBinding:
    """The binding calls serving.Server makes, simulated with the oracle."""

    def __init__(self, pool, design_bytes=None):
        self.pool = pool
        self.design_bytes = design_bytes   # what the server charges per loaded design
        self.designs = {}   # id -> design
        self.batches = {}   # id -> dict(design, seeds, regs, cycle)
        self.next = 1
        self.live_bytes = 0
        self.peak_bytes = 0
        self.live_lds = 0
        self.peak_lds = 0
        self.steps = []

    # footprint model: a fixed cost per instance and cycle-independent; LDS
    # held by the batches of design 2 only
    def rteaal_batch_footprint(self, ctx, did, n_inst, **_):
        return 1000 * n_inst

    def rteaal_batch_resources(self, ctx, did, n_inst, **_):
        lds = 100 * n_inst if self.designs[did] is self.pool[2] else 0
        return self.rteaal_batch_footprint(ctx, did, n_inst), lds

    def rteaal_load_design(self, ctx, d, **_):
        did = self.next
        self.next += 1
        self.designs[did] = d
        return did

    def rteaal_unload_design(self, ctx, did):
        assert not any(b["design"] == did for b in self.batches.values())
        del self.designs[did]

    def rteaal_create_batch(self, ctx, did, seeds, **_):
        bid = self.next
        self.next += 1
        d = self.designs[did]
        self.batches[bid] = {"design": did, "seeds": np.asarray(seeds, np.uint64),
                             "regs": None, "cycle": 0}
        self.live_bytes += self.rteaal_batch_footprint(ctx, did, len(seeds))
        self.live_lds += self.rteaal_batch_resources(ctx, did, len(seeds))[1]
        self.peak_lds = max(self.peak_lds, self.live_lds)
        charged = self.live_bytes + (self.design_bytes or 0) * len(self.designs)
        self.peak_bytes = max(self.peak_bytes, charged)
        return bid

    def rteaal_free_batch(self, ctx, bid):
        b = self.batches.pop(bid)
        self.live_bytes -= self.rteaal_batch_footprint(ctx, b["design"], len(b["seeds"]))
        self.live_lds -= self.rteaal_batch_resources(ctx, b["design"], len(b["seeds"]))[1]

    def rteaal_step_many(self, ctx, bids, n_cycles):
        assert len(set(bids)) == len(bids)
        self.steps.append(list(zip(bids, n_cycles)))
        for bid, c in zip(bids, n_cycles):
            b = self.batches[bid]
            d = self.designs[b["design"]]
            regs, _, _ = oracle.run(d, b["seeds"], int(c), start_cycle=b["cycle"],
                                    init_regs=b["regs"])
            b["regs"], b["cycle"] = regs, b["cycle"] + int(c)

    def rteaal_sync(self, ctx):
        pass

    def rteaal_read_state(self, ctx, bid, **_):
        b = self.batches[bid]
        d = self.designs[b["design"]]
        return R.pack_limbs(b["regs"], d.slot_width[d.reg_slot])


@pytest.fixture
def fake(monkeypatch):
    pool = [rtlgen.generate(rtlgen.GenConfig(n, l, 12, 6, rtlgen.generator.WIDTHS_LARGE, f"p{i}"),
                            60 + i)
            for i, (n, l) in enumerate([(150, 4), (300, 6), (90, 3)])]
    fb = FakeBinding(pool)
    monkeypatch.setattr(serving, "R", fb)
    return pool, fb


def test_jobs_match_uninterrupted_oracle_runs(fake):
    pool, fb = fake
    rng = np.random.default_rng(5)
    jobs = [serving.Job(job_id=k, design=int(rng.integers(0, 3)), n_inst=int(rng.integers(1, 6)),
                        n_cycles=int(rng.integers(5, 60))) for k in range(12)]
    # Room for about 8 instances at a time: later jobs must wait.
    budget = 8000 + 3 * 10 ** 6
    srv = serving.Server(None, pool, budget_bytes=budget, chunk_cycles=7, preload=False)
    srv._design_bytes = lambda k: 10 ** 6
    fb.design_bytes = 10 ** 6
    stats = srv.run(jobs, np.zeros(len(jobs)))
    srv.close()
    assert stats["jobs"] == len(jobs)
    assert fb.peak_bytes <= budget
    assert max(j.admitted - j.arrival for j in jobs) > 0            # someone waited
    assert all(c <= 7 for step in fb.steps for _, c in step)        # chunks of the tick
    assert not fb.batches and not fb.designs                        # everything freed
    for j in jobs:
        d = pool[j.design]
        ref, _, _ = oracle.run(d, j.seeds, j.n_cycles)
        got = R.unpack_limbs(j.regs, d.slot_width[d.reg_slot])
        assert np.array_equal(got, ref), j.job_id
        assert j.finished >= j.admitted >= j.arrival
    assert stats["latency_p99_s"] >= stats["latency_p50_s"] > 0
    assert stats["instance_cycles"] == sum(j.n_inst * j.n_cycles for j in jobs)


def test_lds_admission(fake):
    """Jobs of design 2 hold LDS (100 bytes per instance here): with an LDS
    budget of 500 bytes, at most 5 of its instances run at once, while jobs
    of the other designs are admitted beside them."""
    pool, fb = fake
    jobs = [serving.Job(job_id=k, design=2 if k % 2 == 0 else 1, n_inst=3, n_cycles=9)
            for k in range(8)]
    srv = serving.Server(None, pool, budget_bytes=10 ** 9, chunk_cycles=4, lds_budget_bytes=500)
    assert len(fb.designs) == 3                  # the pool is loaded before any job arrives
    stats = srv.run(jobs, np.zeros(len(jobs)))
    srv.close()
    assert stats["jobs"] == 8
    assert 0 < fb.peak_lds <= 500
    for j in jobs:
        d = pool[j.design]
        ref, _, _ = oracle.run(d, j.seeds, j.n_cycles)
        assert np.array_equal(R.unpack_limbs(j.regs, d.slot_width[d.reg_slot]), ref), j.job_id
    # an LDS demand above the whole budget still runs, alone
    srv = serving.Server(None, pool, budget_bytes=10 ** 9, chunk_cycles=4, lds_budget_bytes=200)
    stats = srv.run([serving.Job(job_id=20, design=2, n_inst=4, n_cycles=5)], np.zeros(1))
    srv.close()
    assert stats["jobs"] == 1


def test_admission_window_and_oversized_job(fake):
    pool, fb = fake
    jobs = [serving.Job(job_id=k, design=0, n_inst=1, n_cycles=3) for k in range(4)]
    srv = serving.Server(None, pool, budget_bytes=10 ** 7, chunk_cycles=2)
    # Two jobs arrive in the window, two after it: only the first two run,
    # and the loop returns as soon as they are done.
    stats = srv.run(jobs, np.array([0.0, 0.0, 50.0, 60.0]), duration=0.5)
    srv.close()
    assert stats["jobs"] == 2 and stats["wall_s"] < 30
    big = serving.Server(None, pool, budget_bytes=500)
    with pytest.raises(RuntimeError):
        big.run([serving.Job(job_id=9, design=1, n_inst=2, n_cycles=1)], np.zeros(1))
