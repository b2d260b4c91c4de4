// Call sequences through the C interface for the host-only runtime build
// (host.cpp linked with hip_mock.cpp, under ASan and UBSan; test
// infrastructure only): batches of every mapping, multi-batch steps with
// uneven cycle counts, batches freed while their set's captured cycle is
// cached, more batch sets than the cache holds, watched and timed batches,
// stimulus words, read-out and restore, PARTITIONED batches, and both
// autotuners.  No result is
// computed (kernels do nothing); every call must succeed and the sanitizers
// and the mock's pointer checks must stay silent.
//
// Usage: host_scenarios design_file...   (the input format of oracle_main.c)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/rteaal.h"

namespace {

struct Design {
  std::vector<uint16_t> slot_width;
  std::vector<uint32_t> const_slot, input_slot, reg_slot, reg_next, layer_ptr, op_dst, op_src_ptr,
      op_src;
  std::vector<uint64_t> const_limbs;
  std::vector<uint8_t> op_type;
  std::vector<uint16_t> op_imm;
  rteaal_design_desc desc{};
};

template <class T>
void take(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  if (n && std::fread(v.data(), sizeof(T), n, f) != n) {
    std::fprintf(stderr, "short input\n");
    std::exit(2);
  }
}

Design load(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) std::exit(2);
  uint32_t h[10];
  uint64_t h64[2];
  if (std::fread(h, 4, 10, f) != 10 || std::fread(h64, 8, 2, f) != 2 || h[0] != 0x524f5452u)
    std::exit(2);
  Design d;
  take(f, d.slot_width, h[1]);
  take(f, d.const_slot, h[2]);
  take(f, d.const_limbs, 4 * (size_t)h[2]);
  take(f, d.input_slot, h[3]);
  take(f, d.reg_slot, h[4]);
  take(f, d.reg_next, h[4]);
  take(f, d.layer_ptr, h[5] + 1);
  take(f, d.op_type, h[6]);
  take(f, d.op_dst, h[6]);
  take(f, d.op_src_ptr, h[6] + 1);
  take(f, d.op_src, h[7]);
  take(f, d.op_imm, h[6]);
  std::fclose(f);
  rteaal_design_desc& x = d.desc;
  x.n_slots = h[1];
  x.slot_width = d.slot_width.data();
  x.n_consts = h[2];
  x.const_slot = d.const_slot.data();
  x.const_limbs = d.const_limbs.data();
  x.n_inputs = h[3];
  x.input_slot = d.input_slot.data();
  x.n_regs = h[4];
  x.reg_slot = d.reg_slot.data();
  x.reg_next = d.reg_next.data();
  x.n_layers = h[5];
  x.layer_op_ptr = d.layer_ptr.data();
  x.n_ops = h[6];
  x.op_type = d.op_type.data();
  x.op_dst = d.op_dst.data();
  x.op_src_ptr = d.op_src_ptr.data();
  x.op_src = d.op_src.data();
  x.op_imm = d.op_imm.data();
  x.layer_fmt = nullptr;
  return d;
}

rteaal_ctx* g_ctx = nullptr;

void ok(rteaal_status st, const char* what) {
  if (st != RTEAAL_OK) {
    std::fprintf(stderr, "%s failed: %d %s\n", what, (int)st, rteaal_last_error(g_ctx));
    std::exit(3);
  }
}

rteaal_batch_id batch(rteaal_design_id d, uint32_t n, rteaal_batch_opts o) {
  std::vector<uint64_t> seeds(n);
  for (uint32_t i = 0; i < n; ++i) seeds[i] = i * 7 + 1;
  rteaal_batch_id b = 0;
  ok(rteaal_create_batch(g_ctx, d, n, seeds.data(), &o, &b), "create_batch");
  return b;
}

rteaal_batch_opts sweep(uint32_t tg) {
  rteaal_batch_opts o{};
  o.mapping = RTEAAL_MAP_SWEEP;
  o.tiles_per_wave = tg;
  o.unroll = 1;
  return o;
}

void many(const std::vector<rteaal_batch_id>& bs, const std::vector<uint64_t>& cyc,
          const rteaal_stimulus* st = nullptr) {
  ok(rteaal_step_many(g_ctx, (uint32_t)bs.size(), bs.data(), cyc.data(), st), "step_many");
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 4) {
    std::fprintf(stderr, "usage: %s design design design...\n", argv[0]);
    return 2;
  }
  std::vector<Design> ds;
  for (int i = 1; i < argc; ++i) ds.push_back(load(argv[i]));
  ok(rteaal_create(0, nullptr, nullptr, &g_ctx), "create");
  std::vector<rteaal_design_id> ids;
  for (auto& d : ds) {
    rteaal_design_id id = 0;
    ok(rteaal_load_design(g_ctx, &d.desc, &id), "load_design");
    ids.push_back(id);
  }
  const size_t D = ids.size();

  // 1. The cache of captured multi-batch cycles: a batch of a cached set is
  //    freed, then more distinct sets than the cache holds.
  {
    std::vector<rteaal_batch_id> bs;
    for (uint32_t k = 0; k < 8; ++k) bs.push_back(batch(ids[k % D], 130, sweep(1 + k % 2)));
    many(bs, std::vector<uint64_t>(8, 2));
    ok(rteaal_free_batch(g_ctx, bs[3]), "free_batch");
    std::vector<rteaal_batch_id> rest;
    for (uint32_t k = 0; k < 8; ++k)
      if (k != 3) rest.push_back(bs[k]);
    many(rest, std::vector<uint64_t>(7, 3));
    for (size_t i = 0; i < rest.size(); ++i)
      for (size_t j = i + 1; j < rest.size(); ++j) many({rest[i], rest[j]}, {1, 2});
    // many cycle counts in one call: a captured cycle per phase
    std::vector<uint64_t> cyc;
    for (size_t i = 0; i < rest.size(); ++i) cyc.push_back(1 + i);
    many(rest, cyc);
    for (rteaal_batch_id b : rest) ok(rteaal_free_batch(g_ctx, b), "free_batch");
  }
  // 2. Every mapping in one call, uneven and zero cycle counts, repeated.
  {
    std::vector<rteaal_batch_id> bs;
    rteaal_batch_opts lay{}, per{}, res{};
    lay.mapping = RTEAAL_MAP_LAYERED;
    per.mapping = RTEAAL_MAP_LAYERED;
    per.persistent = 1;
    res.mapping = RTEAAL_MAP_RESIDENT;
    const uint32_t tgs[] = {1, 2, 4, 8, 16};
    for (uint32_t k = 0; k < 5; ++k) bs.push_back(batch(ids[k % D], 100 + 150 * k, sweep(tgs[k])));
    bs.push_back(batch(ids[0], 3, lay));
    bs.push_back(batch(ids[1 % D], 2, per));
    bs.push_back(batch(ids[2 % D], 40, res));
    for (uint64_t r = 0; r < 3; ++r) {
      std::vector<uint64_t> cyc;
      for (size_t k = 0; k < bs.size(); ++k) cyc.push_back((k * 3 + r) % 5);
      many(bs, cyc);
    }
    // stimulus words for every batch
    std::vector<std::vector<uint64_t>> words(bs.size());
    std::vector<rteaal_stimulus> st(bs.size());
    std::vector<uint64_t> cyc(bs.size(), 2);
    for (size_t k = 0; k < bs.size(); ++k) {
      uint32_t map = 0;
      uint64_t c = 0;
      ok(rteaal_batch_info(g_ctx, bs[k], &map, &c), "batch_info");
      const Design& d = ds[k == 5 ? 0 : k == 6 ? 1 % D : k == 7 ? 2 % D : k % D];
      size_t w = 0;
      for (uint32_t s : d.input_slot) w += (d.slot_width[s] + 63) / 64;
      const uint32_t n = k < 5 ? 100 + 150 * (uint32_t)k : k == 5 ? 3 : k == 6 ? 2 : 40;
      words[k].assign(2 * n * w + 1, 0x1234u);
      st[k].mode = 1;
      st[k].words_on_device = 0;
      st[k].words = words[k].data();
    }
    many(bs, cyc, st.data());
    // watched, timed and tile-pass batches beside the others
    ok(rteaal_watch(g_ctx, bs[0], ds[0].reg_slot.data(), 3, 1000), "watch");
    ok(rteaal_kernel_timing(g_ctx, bs[1], 1, nullptr, nullptr), "kernel_timing");
    many(bs, std::vector<uint64_t>(bs.size(), 2));
    ok(rteaal_kernel_timing(g_ctx, bs[1], 0, nullptr, nullptr), "kernel_timing");
    ok(rteaal_watch(g_ctx, bs[0], nullptr, 0, 0), "unwatch");
    // read-out (allocating and not), restore
    for (size_t k = 0; k < bs.size(); ++k) {
      std::vector<uint64_t> out(1 << 16);
      size_t wr = 0;
      ok(rteaal_read_state(g_ctx, bs[k], 0, 1, RTEAAL_READ_REGS, out.data(), out.size(), &wr),
         "read_state");
      ok(rteaal_read_state_noalloc(g_ctx, bs[k], 0, 1, RTEAAL_READ_REGS, out.data(), out.size(), &wr),
         "read_state_noalloc");
      ok(rteaal_read_state(g_ctx, bs[k], 0, 1, RTEAAL_READ_DIGEST, out.data(), out.size(), &wr),
         "read digest");
      ok(rteaal_write_state(g_ctx, bs[k], 0, 1, out.data(), 5), "write_state");
      ok(rteaal_write_digest(g_ctx, bs[k], 0, 1, out.data()), "write_digest");
    }
    ok(rteaal_sync(g_ctx), "sync");
    for (rteaal_batch_id b : bs) ok(rteaal_free_batch(g_ctx, b), "free_batch");
  }
  // 3. PARTITIONED batches: alone, beside others in one call, read-out and
  //    restore through the owners' copies; watching is refused.
  {
    rteaal_batch_opts po{};
    po.mapping = RTEAAL_MAP_PARTITIONED;
    std::vector<rteaal_batch_id> bs;
    for (uint32_t k = 0; k < 3; ++k) {
      po.partitions = ds[k % D].reg_slot.size() >= 2 ? 2u + k : 1u;
      bs.push_back(batch(ids[k % D], 1 + k, po));
    }
    bs.push_back(batch(ids[0], 70, sweep(1)));
    for (size_t k = 0; k < 3; ++k) ok(rteaal_step(g_ctx, bs[k], 1500, nullptr), "step");
    many(bs, {3, 0, 2000, 4});
    for (size_t k = 0; k < 3; ++k) {
      rteaal_batch_opts got{};
      ok(rteaal_batch_options(g_ctx, bs[k], &got), "batch_options");
      if (got.mapping != RTEAAL_MAP_PARTITIONED || got.partitions == 0) {
        std::fprintf(stderr, "batch_options: mapping %u partitions %u\n", got.mapping, got.partitions);
        return 3;
      }
      std::vector<uint64_t> out(1 << 16);
      size_t wr = 0;
      ok(rteaal_read_state(g_ctx, bs[k], 0, 1, RTEAAL_READ_REGS, out.data(), out.size(), &wr),
         "read_state");
      ok(rteaal_write_state(g_ctx, bs[k], 0, 1, out.data(), 9), "write_state");
      ok(rteaal_read_state(g_ctx, bs[k], 0, 1, RTEAAL_READ_DIGEST, out.data(), out.size(), &wr),
         "read digest");
      if (rteaal_watch(g_ctx, bs[k], ds[k % D].reg_slot.data(), 1, 10) != RTEAAL_E_UNSUPPORTED ||
          rteaal_read_state(g_ctx, bs[k], 0, 1, RTEAAL_READ_ALL_SLOTS, out.data(), out.size(),
                            &wr) != RTEAAL_E_UNSUPPORTED) {
        std::fprintf(stderr, "PARTITIONED watch / all-slot read-out not refused\n");
        return 3;
      }
    }
    ok(rteaal_sync(g_ctx), "sync");
    for (rteaal_batch_id b : bs) ok(rteaal_free_batch(g_ctx, b), "free_batch");
    for (size_t k = 0; k < D; ++k) {
      const uint32_t nr = (uint32_t)ds[k].reg_slot.size();
      for (uint32_t p : {1u, 2u, nr}) {
        if (p == 0 || p > nr || p > 1024) continue;
        rteaal_partition_stats st{};
        ok(rteaal_partition_plan_stats(g_ctx, ids[k], p, &st), "partition_plan_stats");
        if (st.cone_ops > st.padded_ops || st.max_part_ops > st.padded_ops ||
            (p == 1 && (st.exchange != 0 || st.cone_ops > st.design_ops))) {
          std::fprintf(stderr, "partition stats out of range\n");
          return 3;
        }
      }
    }
  }
  // 4. Autotuners.
  {
    rteaal_batch_opts best{};
    double rate = 0;
    ok(rteaal_autotune(g_ctx, ids[0], 70, 2, &best, &rate), "autotune");
    std::vector<uint32_t> ns;
    for (size_t k = 0; k < D; ++k) ns.push_back(k == 0 ? 200 : (uint32_t)(3 + 10 * k));
    std::vector<rteaal_batch_opts> bo(D);
    ok(rteaal_autotune_many(g_ctx, (uint32_t)D, ids.data(), ns.data(), 2, bo.data(), &rate),
       "autotune_many");
  }
  for (rteaal_design_id id : ids) ok(rteaal_unload_design(g_ctx, id), "unload");
  rteaal_destroy(g_ctx);
  // 5. Captured cycles split into several chains (a context created with
  //    RTEAAL_MULTI_CHAINS set), uneven cycle counts, RESIDENT beside them.
  for (const char* chains : {"2", "3"}) {
    setenv("RTEAAL_MULTI_CHAINS", chains, 1);
    ok(rteaal_create(0, nullptr, nullptr, &g_ctx), "create");
    unsetenv("RTEAAL_MULTI_CHAINS");
    ids.clear();
    for (auto& d : ds) {
      rteaal_design_id id = 0;
      ok(rteaal_load_design(g_ctx, &d.desc, &id), "load_design");
      ids.push_back(id);
    }
    std::vector<rteaal_batch_id> bs;
    for (uint32_t k = 0; k < 9; ++k) bs.push_back(batch(ids[k % D], 70 + 10 * k, sweep(1 + k % 2)));
    rteaal_batch_opts res{};
    res.mapping = RTEAAL_MAP_RESIDENT;
    bs.push_back(batch(ids[0], 5, res));
    many(bs, std::vector<uint64_t>(bs.size(), 3));
    std::vector<uint64_t> cyc;
    for (size_t k = 0; k < bs.size(); ++k) cyc.push_back(k % 4);
    many(bs, cyc);
    ok(rteaal_free_batch(g_ctx, bs[2]), "free_batch");
    bs.erase(bs.begin() + 2);
    many(bs, std::vector<uint64_t>(bs.size(), 2));
    ok(rteaal_sync(g_ctx), "sync");
    for (rteaal_batch_id b : bs) ok(rteaal_free_batch(g_ctx, b), "free_batch");
    for (rteaal_design_id id : ids) ok(rteaal_unload_design(g_ctx, id), "unload");
    rteaal_destroy(g_ctx);
  }
  std::printf("scenarios ok\n");
  return 0;
}
