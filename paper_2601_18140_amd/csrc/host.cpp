// Host runtime behind include/rteaal.h: design validation and encoding,
// device memory, batches, stepping, state read-out and restore.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rteaal.h"
#include "internal.h"
#include "levelize.h"

using namespace rteaal;

// Staging buffer of rteaal_read_state_noalloc: a fixed device array, so that
// the call allocates nothing.  Each device holds its own copy; host code
// uses only the device address found by hipGetSymbolAddress (the array's
// name is not a device address in host code).
static __device__ __align__(256) uint64_t scratch[size_t(1) << 20];

namespace {

thread_local std::string g_err;  // failures with no context

constexpr size_t kNoAllocWords = size_t(1) << 20;  // 8 MiB
static_assert(kNoAllocWords == RTEAAL_NOALLOC_MAX_WORDS &&
                  sizeof(scratch) == kNoAllocWords * sizeof(uint64_t), "scratch size");
std::mutex g_scratch_mu;
std::map<int, uint64_t*> g_scratch;  // device -> address of its scratch

// The scratch's device address on `device` (the current device), found once
// per device; null if the lookup fails.
uint64_t* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  if (it != g_scratch.end()) return it->second;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  g_scratch[device] = (uint64_t*)p;
  return (uint64_t*)p;
}

struct DesignHost;
struct Batch;

struct Mem {
  void* p = nullptr;
  size_t bytes = 0;
};

// One captured cycle of a set of SWEEP and LAYERED batches stepped together
// (rteaal_step_many): per layer slot a few launches over segment tables, then
// the digest, fold and cycle advance of every batch.  `table` holds the
// segment tables the launches read; ids are the batches, sorted.
struct MultiGraph {
  std::vector<uint32_t> ids;
  hipGraphExec_t exec = nullptr;
  Mem table;
  uint64_t last_use = 0;
  uint32_t launches = 0;
};

}  // namespace

struct rteaal_ctx {
  int device = 0;
  uint32_t spin_limit = 1u << 22;  // grid barrier waits of persistent launches
  // Captured multi-batch cycles: the pieces of one layer index run as one
  // mixed launch while they total at most this many wavefronts (0: never).
  uint32_t mixed_max_waves = 1u << 20;
  uint64_t* scratch = nullptr;  // this device's staging array (rteaal_read_state_noalloc)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  rteaal_allocator alloc{};
  bool has_alloc = false;
  bool poisoned = false;
  std::string err;
  uint32_t next_id = 1;
  std::map<uint32_t, std::unique_ptr<DesignHost>> designs;
  std::map<uint32_t, std::unique_ptr<Batch>> batches;
  size_t max_lds = 0;
  // rteaal_step_many: auxiliary streams (default priority) for SWEEP batches,
  // fork/join events, and a grow-only device scratch for job tables.
  // Auxiliary streams of rteaal_step_many: 0..3 for captured multi-batch
  // cycles (one chain each) and batches stepped alone, 4..7 for RESIDENT
  // configurations beyond the first.
  static constexpr int kAux = 8;
  hipStream_t aux[kAux] = {};
  hipEvent_t fork = nullptr, join[kAux] = {};
  // Captured multi-batch cycles per call: SWEEP and LAYERED batches split by
  // layer count into this many independent chains (environment
  // RTEAAL_MULTI_CHAINS, 1..4).
  uint32_t multi_chains = 1;
  // Streams and events that only serve graph capture: the launches of one
  // layer fork onto them, so the captured graph runs them concurrently.
  hipStream_t cap[3] = {nullptr, nullptr, nullptr};
  hipEvent_t cap_fork = nullptr, cap_join[3] = {nullptr, nullptr, nullptr};
  Mem multi;
  // Captured cycles of batch sets stepped together, least recently used
  // first to go (at most kMaxMultiGraphs).
  std::vector<std::unique_ptr<MultiGraph>> mgraphs;
  uint64_t mg_clock = 0;
  // Autotuned batch options, keyed by (design, instance count).
  std::map<std::pair<uint32_t, uint32_t>, rteaal_batch_opts> tuned;
};

namespace {

rteaal_status fail(rteaal_ctx* ctx, rteaal_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  else g_err = buf;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      (ctx)->poisoned = true;                                                                  \
      return fail((ctx), RTEAAL_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    }                                                                                          \
  } while (0)

void* dev_alloc(rteaal_ctx* ctx, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  if (ctx->has_alloc) return ctx->alloc.alloc(bytes, ctx->alloc.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(rteaal_ctx* ctx, Mem& m) {
  if (!m.p) return;
  size_t bytes = (std::max<size_t>(m.bytes, 256) + 255) & ~size_t(255);
  if (ctx->has_alloc) ctx->alloc.free(m.p, bytes, ctx->alloc.user);
  else (void)hipFree(m.p);
  m.p = nullptr;
  m.bytes = 0;
}

// Allocates every request or none.
bool alloc_all(rteaal_ctx* ctx, std::vector<std::pair<Mem*, size_t>> reqs) {
  for (size_t i = 0; i < reqs.size(); ++i) {
    Mem* m = reqs[i].first;
    m->p = dev_alloc(ctx, reqs[i].second);
    m->bytes = reqs[i].second;
    if (!m->p) {
      m->bytes = 0;
      for (size_t k = 0; k < i; ++k) dev_free(ctx, *reqs[k].first);
      return false;
    }
  }
  return true;
}

uint32_t bits_for(uint64_t v) {  // bits needed to represent 0..v
  uint32_t b = 1;
  while (b < 64 && (v >> b)) ++b;
  return b;
}

uint32_t expected_arity_ok(uint32_t t, uint32_t a) {
  switch (t) {
    case RTEAAL_AND: case RTEAAL_OR: case RTEAAL_XOR: return a == 2 || a == 3;
    case RTEAAL_MUX: return a == 3;
    case RTEAAL_MUXC: return a >= 3 && a <= 2u * RTEAAL_MUXC_MAX_PAIRS + 1u && a % 2 == 1;
    case RTEAAL_ADD: case RTEAAL_SUB: case RTEAAL_MUL: case RTEAAL_EQ: case RTEAAL_LT:
    case RTEAAL_CONCAT: case RTEAAL_DIV: case RTEAAL_REM: case RTEAAL_DSHL: case RTEAAL_DSHR:
      return a == 2;
    case RTEAAL_NOT: case RTEAAL_SHL: case RTEAAL_SHR: case RTEAAL_EXTRACT: case RTEAAL_ORR:
    case RTEAAL_ANDR: case RTEAAL_XORR: case RTEAAL_SEXT:
      return a == 1;
    default: return 0;
  }
}

// ---------------------------------------------------------------------------
// Validation (host only).
// ---------------------------------------------------------------------------
enum DrvKind : uint8_t { DRV_NONE = 0, DRV_CONST, DRV_INPUT, DRV_REG, DRV_OP };

struct Drivers {
  std::vector<uint8_t> kind;
  std::vector<uint32_t> layer;  // for DRV_OP
  std::vector<uint32_t> which;  // const / input / reg / op index
};

rteaal_status validate(const rteaal_design_desc* d, Drivers* drv, std::string* why,
                       std::vector<rteaal_layer_format>* fmt_out) {
  auto bad = [&](rteaal_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    *why = buf;
    return st;
  };
  if (!d) return bad(RTEAAL_E_INVALID_ARG, "null design descriptor");
  if (d->n_slots == 0 || !d->slot_width) return bad(RTEAAL_E_INVALID_ARG, "no slots");
  if (d->n_consts && (!d->const_slot || !d->const_limbs))
    return bad(RTEAAL_E_INVALID_ARG, "null constant arrays");
  if (d->n_inputs && !d->input_slot) return bad(RTEAAL_E_INVALID_ARG, "null input array");
  if (d->n_regs && (!d->reg_slot || !d->reg_next))
    return bad(RTEAAL_E_INVALID_ARG, "null register arrays");
  if (!d->layer_op_ptr) return bad(RTEAAL_E_INVALID_ARG, "null layer_op_ptr");
  if (d->n_ops && (!d->op_type || !d->op_dst || !d->op_src_ptr || !d->op_src || !d->op_imm))
    return bad(RTEAAL_E_INVALID_ARG, "null operation arrays");
  if (!d->n_ops && !d->op_src_ptr) return bad(RTEAAL_E_INVALID_ARG, "null op_src_ptr");
  if (d->n_slots > (1u << 30)) return bad(RTEAAL_E_BAD_DESIGN, "too many slots");

  for (uint32_t s = 0; s < d->n_slots; ++s)
    if (d->slot_width[s] < 1 || d->slot_width[s] > 256)
      return bad(RTEAAL_E_BAD_DESIGN, "slot %u has width %u (must be 1..256)", s,
                 (unsigned)d->slot_width[s]);

  drv->kind.assign(d->n_slots, DRV_NONE);
  drv->layer.assign(d->n_slots, 0);
  drv->which.assign(d->n_slots, 0);
  auto claim = [&](uint32_t s, uint8_t k, uint32_t w, uint32_t layer) -> bool {
    if (drv->kind[s] != DRV_NONE) return false;
    drv->kind[s] = k;
    drv->which[s] = w;
    drv->layer[s] = layer;
    return true;
  };
  for (uint32_t c = 0; c < d->n_consts; ++c) {
    if (d->const_slot[c] >= d->n_slots) return bad(RTEAAL_E_BAD_DESIGN, "constant %u: slot out of range", c);
    if (!claim(d->const_slot[c], DRV_CONST, c, 0))
      return bad(RTEAAL_E_BAD_DESIGN, "slot %u has more than one driver", d->const_slot[c]);
  }
  for (uint32_t k = 0; k < d->n_inputs; ++k) {
    if (d->input_slot[k] >= d->n_slots) return bad(RTEAAL_E_BAD_DESIGN, "input %u: slot out of range", k);
    if (!claim(d->input_slot[k], DRV_INPUT, k, 0))
      return bad(RTEAAL_E_BAD_DESIGN, "slot %u has more than one driver", d->input_slot[k]);
  }
  for (uint32_t j = 0; j < d->n_regs; ++j) {
    if (d->reg_slot[j] >= d->n_slots || d->reg_next[j] >= d->n_slots)
      return bad(RTEAAL_E_BAD_DESIGN, "register %u: slot out of range", j);
    if (!claim(d->reg_slot[j], DRV_REG, j, 0))
      return bad(RTEAAL_E_BAD_DESIGN, "slot %u has more than one driver", d->reg_slot[j]);
  }
  if (d->layer_op_ptr[0] != 0 || d->layer_op_ptr[d->n_layers] != d->n_ops)
    return bad(RTEAAL_E_BAD_DESIGN, "layer_op_ptr must start at 0 and end at n_ops");
  for (uint32_t i = 0; i < d->n_layers; ++i)
    if (d->layer_op_ptr[i + 1] < d->layer_op_ptr[i])
      return bad(RTEAAL_E_BAD_DESIGN, "layer_op_ptr decreases at layer %u", i);
  if (d->op_src_ptr[0] != 0) return bad(RTEAAL_E_BAD_DESIGN, "op_src_ptr[0] must be 0");
  for (uint32_t i = 0; i < d->n_layers; ++i)
    for (uint32_t o = d->layer_op_ptr[i]; o < d->layer_op_ptr[i + 1]; ++o) {
      if (d->op_type[o] >= RTEAAL_OP_COUNT) return bad(RTEAAL_E_BAD_DESIGN, "op %u: unknown type %u", o, d->op_type[o]);
      if (d->op_src_ptr[o + 1] < d->op_src_ptr[o]) return bad(RTEAAL_E_BAD_DESIGN, "op_src_ptr decreases at op %u", o);
      const uint32_t ar = d->op_src_ptr[o + 1] - d->op_src_ptr[o];
      if (!expected_arity_ok(d->op_type[o], ar))
        return bad(RTEAAL_E_BAD_DESIGN, "op %u: type %u cannot take %u operands", o, d->op_type[o], ar);
      if (d->op_dst[o] >= d->n_slots) return bad(RTEAAL_E_BAD_DESIGN, "op %u: destination out of range", o);
      const uint32_t t = d->op_type[o], imm = d->op_imm[o];
      if ((t == RTEAAL_SHL || t == RTEAAL_SHR || t == RTEAAL_EXTRACT) ? imm > 255 : imm != 0)
        return bad(RTEAAL_E_BAD_DESIGN, "op %u: immediate %u out of range", o, imm);
      if (!claim(d->op_dst[o], DRV_OP, o, i))
        return bad(RTEAAL_E_BAD_DESIGN, "slot %u has more than one driver", d->op_dst[o]);
    }
  // Levelization: every operand is a source or was produced by an earlier layer.
  for (uint32_t i = 0; i < d->n_layers; ++i)
    for (uint32_t o = d->layer_op_ptr[i]; o < d->layer_op_ptr[i + 1]; ++o)
      for (uint32_t q = d->op_src_ptr[o]; q < d->op_src_ptr[o + 1]; ++q) {
        const uint32_t r = d->op_src[q];
        if (r >= d->n_slots) return bad(RTEAAL_E_BAD_DESIGN, "op %u: operand slot out of range", o);
        const uint8_t k = drv->kind[r];
        if (k == DRV_NONE) return bad(RTEAAL_E_BAD_DESIGN, "op %u reads slot %u, which has no driver", o, r);
        if (k == DRV_OP && drv->layer[r] >= i)
          return bad(RTEAAL_E_BAD_DESIGN,
                     "op %u in layer %u reads slot %u produced in layer %u (not levelized)", o, i,
                     r, drv->layer[r]);
      }
  for (uint32_t j = 0; j < d->n_regs; ++j)
    if (drv->kind[d->reg_next[j]] == DRV_NONE)
      return bad(RTEAAL_E_BAD_DESIGN, "register %u latches slot %u, which has no driver", j, d->reg_next[j]);

  // Per-layer formats, derived from the maximum coordinate / payload values.
  std::vector<rteaal_layer_format> fmt(d->n_layers);
  for (uint32_t i = 0; i < d->n_layers; ++i) {
    uint32_t maxs = 0, maxr = 0, maxcount = 0, max_fiber = 0;
    uint32_t count[RTEAAL_OP_COUNT] = {0};
    for (uint32_t o = d->layer_op_ptr[i]; o < d->layer_op_ptr[i + 1]; ++o) {
      maxs = std::max(maxs, d->op_dst[o]);
      count[d->op_type[o]]++;
      if (d->op_type[o] == RTEAAL_MUXC)
        max_fiber = std::max(max_fiber, d->op_src_ptr[o + 1] - d->op_src_ptr[o]);
      for (uint32_t q = d->op_src_ptr[o]; q < d->op_src_ptr[o + 1]; ++q) maxr = std::max(maxr, d->op_src[q]);
    }
    for (uint32_t t = 0; t < RTEAAL_OP_COUNT; ++t) maxcount = std::max(maxcount, count[t]);
    rteaal_layer_format f{};
    f.oim[0] = {0, 0, 0};                                   // I: uncompressed, payloads eliminated
    f.oim[1] = {0, 0, (uint8_t)bits_for(maxcount)};        // N: uncompressed, ops per type
    f.oim[2] = {1, (uint8_t)bits_for(maxs), 0};            // S: compressed, coordinates only
    f.oim[3] = {0, 0, 0};                                   // O: uncompressed, implied by N
    if (max_fiber)                                          // ... except for mux chains
      f.oim[3] = {1, (uint8_t)bits_for(max_fiber - 1), 0};
    f.oim[4] = {1, (uint8_t)bits_for(maxr), 0};            // R: compressed, mask payload dropped
    f.li = {0, 0, 0};
    f.lo = {0, 0, 0};
    if (d->layer_fmt) {
      const rteaal_layer_format& u = d->layer_fmt[i];
      const uint8_t need_c[5] = {0, 0, f.oim[2].cbits, 0, f.oim[4].cbits};
      const uint8_t need_p[5] = {0, f.oim[1].pbits, 0, 0, 0};
      for (int r = 0; r < 5; ++r) {
        if (need_c[r] && u.oim[r].cbits < need_c[r])
          return bad(RTEAAL_E_FORMAT, "layer %u rank %d: coordinates need %u bits, format gives %u",
                     i, r, need_c[r], u.oim[r].cbits);
        if (need_p[r] && u.oim[r].pbits < need_p[r])
          return bad(RTEAAL_E_FORMAT, "layer %u rank %d: payloads need %u bits, format gives %u",
                     i, r, need_p[r], u.oim[r].pbits);
      }
      f = u;
    }
    fmt[i] = f;
  }
  if (fmt_out) fmt_out->swap(fmt);
  return RTEAAL_OK;
}

// ---------------------------------------------------------------------------
// Encoded design.
// ---------------------------------------------------------------------------
struct DesignHost {
  uint32_t id = 0;
  uint32_t n_slots = 0, n_regs = 0, n_inputs = 0, n_design_layers = 0;
  uint32_t n_idx[NCLS] = {0};
  uint64_t n_rows = 0;      // 64-bit rows of one instance's state
  bool compact = false;     // storage reused by live range (no all-slot read-out)
  std::vector<char> kept;   // per slot: its storage holds only it, all cycle long
  std::vector<DevOp> ops;
  std::vector<DevLayer> layers;
  std::vector<std::array<OpRanges, 3>> light;  // per layer, per arity 1..3
  std::vector<uint64_t> const_limbs;
  std::vector<SlotRef> reg_refs, slot_refs;
  uint32_t reg_words = 0, slot_words = 0, words_per_inst = 0;
  uint32_t max_layer_ops = 0;
  std::vector<rteaal_layer_format> fmt;
  uint64_t n_user_ops = 0;
  Mem d_ops, d_layers, d_consts, d_reg_refs, d_slot_refs;
  uint32_t n_batches = 0;
  uint64_t fingerprint = 0;  // of the encoded program, for the tuner's cache
  // Slot-level form of the encoded program (for partitioning): per encoded
  // operation its destination slot and its source slots (mux-chain pairs
  // included); slots >= n_slots are the staging temporaries.
  std::vector<uint32_t> enc_dst, enc_src_ptr, enc_src, reg_slot;
  uint32_t n_enc_slots = 0;
};

// FNV-1a over bytes (Fowler, Noll, Vo), continuing from h.
uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

struct EncOp {
  uint32_t opc, arity, dst_slot;  // dst_slot: user slot or n_slots + temp index
  uint32_t src_slot[3];           // MUXC: s1, v1 and the default
  uint32_t imm, aux0, aux1;       // MUXC: first extra slot in `extra`, extra pairs
  uint32_t dcls, kind, width;
  bool narrow_chain;              // MUXC whose values all fit 64 bits
};

// compact: storage is assigned by live range (an element or 1-bit row is
// reused once every value in it has had its last reader); otherwise every
// slot keeps its own storage for the whole cycle.
void encode(const rteaal_design_desc* d, const Drivers& drv, bool compact, DesignHost* h) {
  const uint32_t NS = d->n_slots;
  std::vector<uint16_t> width(d->slot_width, d->slot_width + NS);
  // Registers whose next-state slot is itself a register are staged first,
  // so the commit of all registers is simultaneous.
  std::vector<uint32_t> temp_of_reg(d->n_regs, UINT32_MAX);
  uint32_t n_temps = 0;
  for (uint32_t j = 0; j < d->n_regs; ++j)
    if (drv.kind[d->reg_next[j]] == DRV_REG) {
      temp_of_reg[j] = NS + n_temps++;
      width.push_back(width[d->reg_next[j]]);
    }
  auto cls_of = [&](uint32_t slot) { return cls_of_width(width[slot]); };
  // Operand slots of the (selector, value) pairs after the first of every
  // fused mux chain, in O order; the record holds s1, v1 and the default.
  std::vector<uint32_t> extra;
  auto mk = [&](uint32_t opc, uint32_t arity, uint32_t dst, const uint32_t* src, uint32_t imm,
                uint32_t aux0, uint32_t aux1) {
    uint32_t rec[3];
    bool narrow_chain = false;
    if (opc == OP_MUXC) {
      narrow_chain = width[dst] <= 64;
      for (uint32_t q = 0; q < arity; ++q) narrow_chain = narrow_chain && width[src[q]] <= 64;
      rec[0] = src[0];
      rec[1] = src[1];
      rec[2] = src[arity - 1];
      aux0 = (uint32_t)extra.size();
      aux1 = (arity - 3) / 2;
      extra.insert(extra.end(), src + 2, src + arity - 1);
      src = rec;
      arity = 3;
    }
    EncOp e{};
    e.narrow_chain = narrow_chain;
    e.opc = opc;
    e.arity = arity;
    e.dst_slot = dst;
    for (uint32_t o = 0; o < 3; ++o) e.src_slot[o] = o < arity ? src[o] : 0;
    e.imm = imm;
    e.aux0 = aux0;
    e.aux1 = aux1;
    e.width = width[dst];
    e.dcls = cls_of(dst);
    bool all_b = e.dcls == CB, any_wide = e.dcls >= CL2, all_32 = e.dcls <= CW;
    for (uint32_t o = 0; o < arity; ++o) {
      all_b = all_b && cls_of(src[o]) == CB;
      any_wide = any_wide || cls_of(src[o]) >= CL2;
      all_32 = all_32 && cls_of(src[o]) <= CW;
    }
    if (opc >= OP_STIM) all_b = all_32 = false;
    // The FIRRTL primitives DIV .. SEXT and fused mux chains always run in
    // the wide form, which keeps them out of the common kernel.
    if (opc >= OP_DIV && opc <= OP_MUXC) any_wide = true;
    e.kind = any_wide ? K_WIDE : all_b ? K_BIT : all_32 ? K_U32 : K_U64;
    return e;
  };

  std::vector<std::vector<EncOp>> L;
  {  // sources: constants and primary inputs
    std::vector<EncOp> src;
    for (uint32_t c = 0; c < d->n_consts; ++c) src.push_back(mk(OP_CONST, 0, d->const_slot[c], nullptr, 0, c, 0));
    uint32_t woff = 0;
    for (uint32_t k = 0; k < d->n_inputs; ++k) {
      src.push_back(mk(OP_STIM, 0, d->input_slot[k], nullptr, 0, k, woff));
      woff += (width[d->input_slot[k]] + 63) / 64;
    }
    h->words_per_inst = woff;
    if (!src.empty()) L.push_back(std::move(src));
  }
  for (uint32_t i = 0; i < d->n_layers; ++i) {
    std::vector<EncOp> lay;
    for (uint32_t o = d->layer_op_ptr[i]; o < d->layer_op_ptr[i + 1]; ++o) {
      const uint32_t t = d->op_type[o];
      const uint32_t* s = d->op_src + d->op_src_ptr[o];
      const uint32_t ar = d->op_src_ptr[o + 1] - d->op_src_ptr[o];
      uint32_t imm = d->op_imm[o];
      if (t == RTEAAL_CONCAT) imm = width[s[1]];
      if (t == RTEAAL_ANDR || t == RTEAAL_SEXT) imm = width[s[0]];
      lay.push_back(mk(t, ar, d->op_dst[o], s, imm, 0, 0));
    }
    L.push_back(std::move(lay));  // empty design layers still separate their neighbours
  }
  if (n_temps) {
    std::vector<EncOp> hold;
    for (uint32_t j = 0; j < d->n_regs; ++j)
      if (temp_of_reg[j] != UINT32_MAX) hold.push_back(mk(OP_COPY, 1, temp_of_reg[j], &d->reg_next[j], 0, 0, 0));
    L.push_back(std::move(hold));
  }
  if (d->n_regs) {
    std::vector<EncOp> commit;
    for (uint32_t j = 0; j < d->n_regs; ++j) {
      const uint32_t src = temp_of_reg[j] != UINT32_MAX ? temp_of_reg[j] : d->reg_next[j];
      commit.push_back(mk(OP_COPY, 1, d->reg_slot[j], &src, 0, 0, 0));
    }
    L.push_back(std::move(commit));
  }

  // Group each layer by (1-bit destination first, kind, type, class): the
  // N-rank swizzle, which also makes 1-bit destinations a prefix.  Heavy
  // operations (a value wider than 64 bits, a wide-form type, or a source) go
  // last among the 1-bit destinations and first among the others, so they
  // are contiguous, with the fused mux chains at their middle (last among
  // the 1-bit heavy ones, first among the others); the common operations are
  // ordered by arity, 3-2-1 before the heavy range and 1-2-3 after it, so
  // every arity is one range on each side.
  auto heavy = [](const EncOp& e) { return e.kind == K_WIDE || e.opc >= OP_STIM; };
  auto rank = [&](const EncOp& e) {
    const bool hv = heavy(e);
    const bool chain = e.opc == OP_MUXC;
    if (e.dcls == CB) return hv ? (chain ? 4u : 3u) : 3u - e.arity;
    return hv ? (chain ? 0u : 1u) : 1u + e.arity;
  };
  for (auto& lay : L)
    std::stable_sort(lay.begin(), lay.end(), [&](const EncOp& a, const EncOp& b) {
      const uint32_t ka = a.dcls != CB, kb = b.dcls != CB;
      if (ka != kb) return ka < kb;
      const uint32_t ra = rank(a), rb = rank(b);
      if (ra != rb) return ra < rb;
      if (a.kind != b.kind) return a.kind < b.kind;
      if (a.opc != b.opc) return a.opc < b.opc;
      return a.dcls < b.dcls;
    });

  // Storage indices.  A 1-bit destination gets bit (i mod 64) of the row
  // given to its group of 64 consecutive 1-bit destinations in the layer
  // (one wavefront's ballot fills exactly that row); every other slot gets
  // an element index in its class.  Lifetimes are layer positions: a value
  // lives from the layer that writes it to the last layer that reads it.
  // Registers (written by the commit layer, read in the next cycle) and,
  // without compaction, every slot keep their storage; the rest returns to
  // its class's free list after its last reader's layer, so no layer writes
  // over a value that the same layer still reads.
  const uint32_t NW = (uint32_t)width.size();
  const uint32_t NL = (uint32_t)L.size();
  std::vector<uint32_t> scls(NW, CNONE), sidx(NW, 0);
  std::vector<uint32_t> last(NW, 0);
  std::vector<char> keep(NW, compact ? 0 : 1);
  for (uint32_t j = 0; j < d->n_regs; ++j) keep[d->reg_slot[j]] = 1;
  for (uint32_t k = 0; k < NL; ++k)
    for (const EncOp& e : L[k]) {
      last[e.dst_slot] = std::max(last[e.dst_slot], k);
      for (uint32_t q = 0; q < e.arity; ++q) last[e.src_slot[q]] = std::max(last[e.src_slot[q]], k);
      if (e.opc == OP_MUXC)
        for (uint32_t q = 0; q < 2 * e.aux1; ++q) last[extra[e.aux0 + q]] = std::max(last[extra[e.aux0 + q]], k);
    }
  uint32_t cnt[NCLS] = {0};                        // elements (CB: rows) ever used per class
  std::vector<uint32_t> free_el[NCLS];             // LIFO: recently freed storage is warm
  std::vector<std::vector<std::pair<uint32_t, uint32_t>>> release(NL + 1);
  auto take = [&](uint32_t c) {
    if (free_el[c].empty()) return cnt[c]++;
    const uint32_t i = free_el[c].back();
    free_el[c].pop_back();
    return i;
  };
  // Places the destinations of layer k: with only_kept, just the kept ones
  // (and the 1-bit rows holding one) on fresh storage; otherwise the rest,
  // on recycled storage where possible.  Kept values live across the cycle
  // boundary (a register is read by the layers before the commit that
  // writes it), so their storage must never have held anything else.
  auto place = [&](uint32_t k, bool only_kept) {
    const auto& lay = L[k];
    uint32_t nb = 0;
    while (nb < lay.size() && lay[nb].dcls == CB) ++nb;
    for (uint32_t g0 = 0; g0 < nb; g0 += 64) {
      const uint32_t g1 = std::min(nb, g0 + 64);
      if (scls[lay[g0].dst_slot] != CNONE) continue;  // placed by the kept pass
      uint32_t end = k;
      bool kept = false;
      for (uint32_t i = g0; i < g1; ++i) {
        end = std::max(end, last[lay[i].dst_slot]);
        kept = kept || keep[lay[i].dst_slot];
      }
      if (only_kept && !kept) continue;
      const uint32_t row = kept ? cnt[CB]++ : take(CB);
      for (uint32_t i = g0; i < g1; ++i) {
        scls[lay[i].dst_slot] = CB;
        sidx[lay[i].dst_slot] = row * 64u + (i - g0);
      }
      if (!kept) release[end + 1].push_back({CB, row});
    }
    for (uint32_t i = nb; i < lay.size(); ++i) {
      const uint32_t sl = lay[i].dst_slot, c = lay[i].dcls;
      if (scls[sl] != CNONE || (only_kept && !keep[sl])) continue;
      const uint32_t idx = keep[sl] ? cnt[c]++ : take(c);
      scls[sl] = c;
      sidx[sl] = idx;
      if (!keep[sl]) release[last[sl] + 1].push_back({c, idx});
    }
  };
  for (uint32_t k = 0; k < NL; ++k) place(k, true);
  h->layers.clear();
  h->light.clear();
  uint32_t pos = 0;
  for (uint32_t k = 0; k < NL; ++k) {
    auto& lay = L[k];
    for (const auto& r : release[k]) free_el[r.first].push_back(r.second);
    place(k, false);
    DevLayer dl{};
    dl.begin = pos;
    dl.end = pos + (uint32_t)lay.size();
    uint32_t nb = 0;
    while (nb < lay.size() && lay[nb].dcls == CB) ++nb;
    if (nb) dl.b_base = sidx[lay[0].dst_slot];
    dl.n_bdst = nb;
    uint32_t first_heavy = dl.end, n_heavy = 0;
    for (uint32_t i = 0; i < lay.size(); ++i)
      if (heavy(lay[i])) {
        first_heavy = std::min(first_heavy, dl.begin + i);
        ++n_heavy;
      }
    dl.hbeg = n_heavy ? first_heavy : dl.begin;
    dl.hend = dl.hbeg + n_heavy;
    dl.hm0 = dl.hm1 = dl.hbeg;
    {
      bool seen = false;
      for (uint32_t i = 0; i < lay.size(); ++i)
        if (lay[i].opc == OP_MUXC) {
          if (!seen) dl.hm0 = dl.begin + i, seen = true;
          dl.hm1 = dl.begin + i + 1;
        }
    }
    h->layers.push_back(dl);
    std::array<OpRanges, 3> ar{};
    for (uint32_t a = 1; a <= 3; ++a) {
      OpRanges& r = ar[a - 1];
      r.b0 = r.e0 = dl.hbeg;
      r.b1 = r.e1 = dl.hend;
      bool s0 = false, s1 = false;
      for (uint32_t i = 0; i < lay.size(); ++i) {
        const EncOp& e = lay[i];
        if (heavy(e) || e.arity != a) continue;
        const uint32_t k = dl.begin + i;
        if (k < dl.hbeg) {
          if (!s0) r.b0 = k, s0 = true;
          r.e0 = k + 1;
        } else {
          if (!s1) r.b1 = k, s1 = true;
          r.e1 = k + 1;
        }
      }
    }
    h->light.push_back(ar);
    h->max_layer_ops = std::max<uint32_t>(h->max_layer_ops, (uint32_t)lay.size());
    pos = dl.end;
  }
  for (int c = 0; c < NCLS; ++c) h->n_idx[c] = cnt[c];
  h->compact = compact;
  h->kept.assign(keep.begin(), keep.begin() + NS);

  // Rows of one instance: the 1-bit rows (at least one, since absent
  // operands read field 0), then the wide rows.  The wide values are laid out
  // by byte offset Y in regions of C8, C16, CW elements (1, 2, 4 bytes, eight,
  // four, two to a row), then CD, CL2, CL3, CL4 (8 bytes per limb), each
  // class starting on a 16-byte boundary; Y becomes the field
  // 64*(first wide row + Y/8) + 8*(Y%8), the last term being the value's bit
  // offset in its row.  A 1-bit slot's field is its bit index.
  const uint64_t b_rows = std::max<uint64_t>(cnt[CB], 1);
  uint64_t base[NCLS] = {0};
  uint64_t wb = 0;
  for (uint32_t c = C8; c < NCLS; ++c) {
    base[c] = wb;
    wb = (wb + (uint64_t)cnt[c] * cls_bytes(c) + 15) & ~uint64_t(15);
  }
  h->n_rows = b_rows + wb / 8;
  for (uint32_t k = 0; k < NW; ++k)
    if (scls[k] != CB && scls[k] != CNONE) {
      const uint64_t y = base[scls[k]] + (uint64_t)sidx[k] * cls_bytes(scls[k]);
      sidx[k] = (uint32_t)((b_rows + y / 8) * 64 + (y % 8) * 8);
    }

  // The word table: the literals' limbs (four words each, at least one
  // literal's worth), then one word per extra mux-chain operand, its field
  // in bits 0..31 and its class in bits 32..34.
  h->const_limbs.assign(d->const_limbs, d->const_limbs + 4ull * d->n_consts);
  if (h->const_limbs.empty()) h->const_limbs.assign(4, 0);
  h->ops.clear();
  h->ops.reserve(pos);
  h->enc_dst.clear();
  h->enc_src.clear();
  h->enc_src_ptr.assign(1, 0);
  for (auto& lay : L)
    for (auto& e : lay) {
      h->enc_dst.push_back(e.dst_slot);
      for (uint32_t q = 0; q < e.arity; ++q) h->enc_src.push_back(e.src_slot[q]);
      if (e.opc == OP_MUXC)
        for (uint32_t q = 0; q < 2 * e.aux1; ++q) h->enc_src.push_back(extra[e.aux0 + q]);
      h->enc_src_ptr.push_back((uint32_t)h->enc_src.size());
      DevOp o{};
      uint32_t code = (e.opc & 63u) | (e.kind << 6) | (e.arity << 8) | (e.dcls << 10);
      for (uint32_t q = 0; q < e.arity; ++q) {
        code |= scls[e.src_slot[q]] << (13 + 3 * q);
        o.src[q] = sidx[e.src_slot[q]];
      }
      o.code = code;
      o.wimm = (e.width & 511u) | ((e.imm & 511u) << 9);
      o.dst = sidx[e.dst_slot];
      o.aux0 = e.aux0;
      o.aux1 = e.aux1;
      if (e.opc == OP_MUXC) {
        o.aux0 = (uint32_t)h->const_limbs.size();
        for (uint32_t q = 0; q < 2 * e.aux1; ++q) {
          const uint32_t sl = extra[e.aux0 + q];
          h->const_limbs.push_back((uint64_t)sidx[sl] | ((uint64_t)scls[sl] << 32));
        }
        if (e.narrow_chain) o.code |= 1u << 22;
      }
      h->ops.push_back(o);
    }

  h->reg_refs.clear();
  uint32_t off = 0;
  for (uint32_t j = 0; j < d->n_regs; ++j) {
    const uint32_t s = d->reg_slot[j];
    h->reg_refs.push_back(SlotRef{scls[s], sidx[s], off, width[s]});
    off += (width[s] + 63) / 64;
  }
  h->reg_words = off;
  h->slot_refs.clear();
  off = 0;
  for (uint32_t s = 0; s < NS; ++s) {
    h->slot_refs.push_back(SlotRef{scls[s], sidx[s], off, width[s]});
    off += (width[s] + 63) / 64;
  }
  h->slot_words = off;
  h->n_slots = NS;
  h->n_regs = d->n_regs;
  h->n_inputs = d->n_inputs;
  h->n_design_layers = d->n_layers;
  h->n_user_ops = d->n_ops;
  h->reg_slot.assign(d->reg_slot, d->reg_slot + d->n_regs);
  h->n_enc_slots = NW;
  uint64_t fp = fnv1a(h->ops.data(), h->ops.size() * sizeof(DevOp));
  fp = fnv1a(h->layers.data(), h->layers.size() * sizeof(DevLayer), fp);
  fp = fnv1a(h->const_limbs.data(), h->const_limbs.size() * 8, fp);
  fp = fnv1a(h->reg_refs.data(), h->reg_refs.size() * sizeof(SlotRef), fp);
  h->fingerprint = fnv1a(&h->n_rows, sizeof h->n_rows, fp);
}

// ---------------------------------------------------------------------------
// Batches.
// ---------------------------------------------------------------------------
struct Batch {
  uint32_t id = 0, design = 0, n_inst = 0, mapping = 0, block = 0, opw = 0, unroll = 0, tg = 1;
  uint32_t arity_split = 0;
  uint32_t tpp = 0;  // SWEEP tiles per pass, 0 = all
  bool pbranch = false;  // SWEEP: tile passes as parallel graph branches
  bool lds = false, lds_ops = false;
  bool persistent = false;  // LAYERED: one cooperative launch per chunk of cycles
  Mem gsync;                // its grid barrier state
  std::vector<uint64_t> seeds_host;  // sources of the initial copies (enqueued at creation)
  DevCtl ctl_host{};
  // PARTITIONED: partitions, bytes of one state copy, the sub-programs and
  // their job table, the exchange rows, the digest sums, and the register
  // refs of the owners' copies (for read-out and restore).
  uint32_t parts = 0;
  uint64_t copy_pitch = 0;
  Mem part_mem, xch, pacc, preg_refs;
  uint64_t part_jobs_off = 0;
  std::vector<char> part_host;  // source of part_mem's copy (enqueued at creation)
  std::vector<SlotRef> preg_host;
  uint64_t cycle = 0;
  StateLayout L{};
  // dig: the running register digest of every instance slot (n_slot words),
  // then the per-cycle sums the digest kernels add into (n_slot words).
  Mem state, seeds, ctl, dig;
  uint64_t n_slot = 0;             // instance slots: allocated tiles x 64 (SWEEP) or n_inst
  hipGraphExec_t graph = nullptr;  // one cycle of SWEEP launches
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
  std::vector<uint8_t> ev_kind;  // per used pair: 0 main kernel, 1 heavy SWEEP kernel
  // Value-change capture (rteaal_watch): watched signals, their values after
  // the last cycle (shadow), the change log and its count.
  uint32_t n_watch = 0, watch_words = 0;
  uint64_t log_cap = 0;
  Mem watch_refs, shadow, log, log_count;
};

void free_parts(rteaal_ctx* ctx, Batch& b) {
  dev_free(ctx, b.part_mem);
  dev_free(ctx, b.xch);
  dev_free(ctx, b.pacc);
  dev_free(ctx, b.preg_refs);
}

void free_watch(rteaal_ctx* ctx, Batch& b) {
  dev_free(ctx, b.watch_refs);
  dev_free(ctx, b.shadow);
  dev_free(ctx, b.log);
  dev_free(ctx, b.log_count);
  b.n_watch = b.watch_words = 0;
  b.log_cap = 0;
}

// Appends the capture of the batch's watched signals after a cycle.
hipError_t capture(const Batch& b, hipStream_t s) {
  if (!b.n_watch) return hipSuccess;
  return launch_capture(b.mapping == RTEAAL_MAP_SWEEP, b.L, (const char*)b.state.p,
                        (const SlotRef*)b.watch_refs.p, b.n_watch, (uint64_t*)b.shadow.p,
                        b.n_inst, false, (const DevCtl*)b.ctl.p, (ChangeRec*)b.log.p, b.log_cap,
                        (unsigned long long*)b.log_count.p, s);
}

void release_events(Batch& b) {
  for (auto& e : b.ev_used) b.ev_free.push_back(e);
  b.ev_used.clear();
  b.ev_kind.clear();
}

void destroy_events(Batch& b) {
  release_events(b);
  for (auto& e : b.ev_free) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  b.ev_free.clear();
}

// Records a start event, runs `launch`, records an end event.
template <class F>
hipError_t timed(Batch& b, hipStream_t s, uint8_t kind, F&& launch) {
  if (!b.profile) return launch();
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (!b.ev_free.empty()) {
    ev = b.ev_free.back();
    b.ev_free.pop_back();
  } else {
    hipError_t e = hipEventCreate(&ev.first);
    if (e == hipSuccess) e = hipEventCreate(&ev.second);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipEventRecord(ev.first, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(ev.second, s);
  b.ev_used.push_back(ev);
  b.ev_kind.push_back(kind);
  return e;
}

// Layout of a batch's state; false if SWEEP rows would not fit 32-bit sizes.
bool make_layout(const DesignHost& h, uint32_t mapping, uint32_t n_inst, uint32_t tg,
                 StateLayout* out, uint64_t* bytes) {
  StateLayout L{};
  L.n_rows = (uint32_t)h.n_rows;
  if (mapping == RTEAAL_MAP_SWEEP) {
    tg = (tg == 2 || tg == 4 || tg == 8 || tg == 16) ? tg : 1u;
    L.lg = tg == 16 ? 4u : tg == 8 ? 3u : tg == 4 ? 2u : tg == 2 ? 1u : 0u;
    L.n_tiles = (n_inst + 63) / 64;
    L.n_tiles_alloc = (L.n_tiles + tg - 1) / tg * tg;
    if ((uint64_t)L.n_tiles_alloc * 512 >= (1ull << 32)) return false;
    L.row_bytes = L.n_tiles_alloc * 512u;
    L.pitch = 0;
    *bytes = h.n_rows * L.row_bytes;
  } else if (mapping == RTEAAL_MAP_PARTITIONED) {
    // tg is the number of partitions: every instance holds one copy of its
    // state per partition, copy p of instance i at (i P + p) copy_pitch.
    L.pitch = ((h.n_rows * 8 + 15) & ~uint64_t(15)) * std::max(tg, 1u);
    *bytes = L.pitch * n_inst;
  } else {
    L.pitch = (h.n_rows * 8 + 15) & ~uint64_t(15);
    *bytes = L.pitch * n_inst;
  }
  *out = L;
  return true;
}

uint32_t sweep_tg(const rteaal_batch_opts* o) { return o && o->tiles_per_wave ? o->tiles_per_wave : 1u; }

// Partitions of a PARTITIONED batch: the option, else as many as fit the
// device with every instance (one workgroup each), at most one per register.
uint32_t part_count(const DesignHost& h, uint32_t n_inst, const rteaal_batch_opts* o) {
  if (o && o->partitions) return o->partitions;
  const uint32_t p = std::max<uint32_t>(1, 256 / std::max<uint32_t>(n_inst, 1));
  return std::max<uint32_t>(1, std::min<uint32_t>(p, std::max<uint32_t>(h.n_regs, 1)));
}

// The layout parameter of make_layout: the tile group (SWEEP) or the
// partition count (PARTITIONED).
uint32_t layout_param(const DesignHost& h, uint32_t mapping, uint32_t n_inst,
                      const rteaal_batch_opts* o) {
  return mapping == RTEAAL_MAP_PARTITIONED ? part_count(h, n_inst, o) : sweep_tg(o);
}

// The partitioned form of a design for P register partitions (registers
// split into P contiguous blocks): for every partition, its sub-program
// (the design's layers restricted to the operations in the fan-in cones of
// its registers: cones closed backwards from the register commits, every
// 1-bit destination group of 64 whole, since one ballot stores its row),
// the registers it owns and the registers of other partitions its cones
// read.
struct PartPlan {
  std::vector<DevOp> ops;
  std::vector<DevLayer> layers;           // [P][n_layers]
  std::vector<uint32_t> lists;            // per partition: own, then need
  std::vector<uint32_t> op_begin, own_begin, own_n, need_begin, need_n;
  uint64_t cone_ops = 0;                  // operations in all cones (without padding)
  uint64_t padded_ops = 0, max_part_ops = 0, exchange = 0;
};

// materialize: false only counts (cone_ops, padded_ops, max_part_ops,
// exchange), without building the sub-programs.
void plan_partitions(const DesignHost& h, uint32_t P, PartPlan* out, bool materialize) {
  const uint32_t W = (P + 63) / 64;
  const size_t NW = h.n_enc_slots, NL = h.layers.size(), NO = h.ops.size();
  std::vector<uint64_t> need((size_t)NW * W, 0), mask(NO * W, 0);
  std::vector<uint32_t> reg_of(NW, UINT32_MAX);
  for (uint32_t j = 0; j < h.n_regs; ++j) reg_of[h.reg_slot[j]] = j;
  auto owner = [&](uint32_t j) { return (uint32_t)((uint64_t)j * P / std::max(h.n_regs, 1u)); };
  for (size_t k = NL; k-- > 0;) {
    const DevLayer& ly = h.layers[k];
    const bool commit = h.n_regs && k + 1 == NL;   // the commit layer is the last one
    for (uint32_t pos = ly.begin; pos < ly.end; ++pos) {
      uint64_t* m = &mask[(size_t)pos * W];
      const uint32_t d = h.enc_dst[pos];
      if (commit) {
        const uint32_t p = owner(reg_of[d]);
        m[p / 64] |= 1ull << (p % 64);
      } else {
        for (uint32_t w = 0; w < W; ++w) m[w] = need[(size_t)d * W + w];
      }
      for (uint32_t q = h.enc_src_ptr[pos]; q < h.enc_src_ptr[pos + 1]; ++q)
        for (uint32_t w = 0; w < W; ++w) need[(size_t)h.enc_src[q] * W + w] |= m[w];
    }
  }
  PartPlan& pl = *out;
  for (uint32_t p = 0; p < P; ++p) {
    const uint32_t pw = p / 64;
    const uint64_t pb = 1ull << (p % 64);
    auto in = [&](uint32_t pos) { return (mask[(size_t)pos * W + pw] & pb) != 0; };
    const uint64_t before = pl.padded_ops;
    if (materialize) pl.op_begin.push_back((uint32_t)pl.ops.size());
    for (size_t k = 0; k < NL; ++k) {
      const DevLayer& ly = h.layers[k];
      DevLayer sl{};
      sl.begin = (uint32_t)(pl.padded_ops - before);
      for (uint32_t g0 = 0; g0 < ly.n_bdst; g0 += 64) {
        const uint32_t g1 = std::min(ly.n_bdst, g0 + 64);
        bool any = false;
        for (uint32_t i = g0; i < g1; ++i) {
          const bool x = in(ly.begin + i);
          any = any || x;
          pl.cone_ops += x;
        }
        if (!any) continue;
        pl.padded_ops += g1 - g0;
        if (materialize)
          pl.ops.insert(pl.ops.end(), h.ops.begin() + ly.begin + g0, h.ops.begin() + ly.begin + g1);
      }
      for (uint32_t pos = ly.begin + ly.n_bdst; pos < ly.end; ++pos)
        if (in(pos)) {
          ++pl.cone_ops;
          ++pl.padded_ops;
          if (materialize) pl.ops.push_back(h.ops[pos]);
        }
      sl.end = (uint32_t)(pl.padded_ops - before);
      if (materialize) pl.layers.push_back(sl);
    }
    pl.max_part_ops = std::max<uint64_t>(pl.max_part_ops, pl.padded_ops - before);
    if (materialize) {
      pl.own_begin.push_back((uint32_t)pl.lists.size());
      for (uint32_t j = 0; j < h.n_regs; ++j)
        if (owner(j) == p) pl.lists.push_back(j);
      pl.own_n.push_back((uint32_t)pl.lists.size() - pl.own_begin.back());
      pl.need_begin.push_back((uint32_t)pl.lists.size());
    }
    for (uint32_t j = 0; j < h.n_regs; ++j)
      if (owner(j) != p && (need[(size_t)h.reg_slot[j] * W + pw] & pb)) {
        pl.exchange += (h.reg_refs[j].width + 63) / 64;
        if (materialize) pl.lists.push_back(j);
      }
    if (materialize) pl.need_n.push_back((uint32_t)pl.lists.size() - pl.need_begin.back());
  }
}

// Largest partitioned program a batch may hold (operation records, 32 bytes
// each): 2^27 operations, 4 GiB.
constexpr uint64_t kMaxPartOps = 1ull << 27;

// PARTITIONED set-up on the host: the partition count, the plan, the block
// size, LDS use and the co-residency check, and the host image of the
// sub-program table (device pointers are filled in by finish_part_table once
// the table is allocated).
rteaal_status plan_batch_partitions(rteaal_ctx* ctx, const DesignHost& h, uint32_t n_inst,
                                    const rteaal_batch_opts* o, Batch* b, PartPlan* plan) {
  const uint32_t P = part_count(h, n_inst, o);
  if (P < 1 || P > 1024)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "PARTITIONED partitions must be 1 .. 1024");
  if (P > std::max<uint32_t>(h.n_regs, 1))
    return fail(ctx, RTEAAL_E_INVALID_ARG, "%u partitions for %u registers", P, h.n_regs);
  const uint64_t copy_pitch = (h.n_rows * 8 + 15) & ~uint64_t(15);
  if (copy_pitch * P * 8 >= (1ull << 32))
    return fail(ctx, RTEAAL_E_INVALID_ARG, "PARTITIONED: %u copies of the state exceed 512 MB", P);
  try {
    PartPlan count;
    plan_partitions(h, P, &count, false);
    if (count.padded_ops > kMaxPartOps)
      return fail(ctx, RTEAAL_E_INVALID_ARG,
                  "PARTITIONED: %u partitions replicate the design into %llu operations (at most "
                  "%llu); use fewer partitions",
                  P, (unsigned long long)count.padded_ops, (unsigned long long)kMaxPartOps);
    plan_partitions(h, P, plan, true);
  } catch (const std::bad_alloc&) {
    return fail(ctx, RTEAAL_E_NO_MEMORY, "PARTITIONED: host memory for the partition plan");
  }
  uint32_t m = 0;
  for (const DevLayer& l : plan->layers) m = std::max(m, l.end - l.begin);
  uint32_t blk = o && o->block_threads ? o->block_threads : 0;
  if (blk && (blk % 64 || blk > 1024))
    return fail(ctx, RTEAAL_E_INVALID_ARG, "block_threads must be a multiple of 64 up to 1024");
  if (!blk) {
    blk = std::min<uint32_t>(1024, std::max<uint32_t>(64, ((m + 63) / 64) * 64));
    if (blk > 256 && m < 2048) blk = 256;
  }
  const bool lds = !(o && o->lds_state == 1) && copy_pitch <= ctx->max_lds;
  const uint32_t cap = partitioned_capacity(blk, lds, lds ? (size_t)copy_pitch : 0);
  if ((uint64_t)n_inst * P > cap)
    return fail(ctx, RTEAAL_E_INVALID_ARG,
                "PARTITIONED: %u instances x %u partitions = %llu workgroups, but at most %u can "
                "be resident at once (block %u, state %s)",
                n_inst, P, (unsigned long long)n_inst * P, cap, blk, lds ? "in LDS" : "in HBM");
  b->parts = P;
  b->copy_pitch = copy_pitch;
  b->block = blk;
  b->lds = lds;
  b->unroll = 1;
  // Image: ops | layers | lists | jobs, each part 16-byte aligned.
  auto al = [](uint64_t x) { return (x + 15) & ~uint64_t(15); };
  const uint64_t o_lay = al(plan->ops.size() * sizeof(DevOp));
  const uint64_t o_lst = o_lay + al(plan->layers.size() * sizeof(DevLayer));
  const uint64_t o_job = o_lst + al(plan->lists.size() * 4);
  b->part_jobs_off = o_job;
  b->part_host.assign(o_job + P * sizeof(PartJob), 0);
  if (!plan->ops.empty()) memcpy(b->part_host.data(), plan->ops.data(), plan->ops.size() * sizeof(DevOp));
  if (!plan->layers.empty())
    memcpy(b->part_host.data() + o_lay, plan->layers.data(), plan->layers.size() * sizeof(DevLayer));
  if (!plan->lists.empty())
    memcpy(b->part_host.data() + o_lst, plan->lists.data(), plan->lists.size() * 4);
  // Register refs of the owners' copies.
  b->preg_host = h.reg_refs;
  for (uint32_t j = 0; j < h.n_regs; ++j) {
    const uint64_t owner = (uint64_t)j * P / std::max(h.n_regs, 1u);
    b->preg_host[j].pos += (uint32_t)(owner * copy_pitch * 8);
  }
  return RTEAAL_OK;
}

// The job table of a PARTITIONED batch, now that part_mem is allocated.
void finish_part_table(Batch& b, const PartPlan& plan) {
  char* base = (char*)b.part_mem.p;
  auto al = [](uint64_t x) { return (x + 15) & ~uint64_t(15); };
  const uint64_t o_lay = al(plan.ops.size() * sizeof(DevOp));
  const uint64_t o_lst = o_lay + al(plan.layers.size() * sizeof(DevLayer));
  const uint32_t NL = b.parts ? (uint32_t)(plan.layers.size() / b.parts) : 0;
  for (uint32_t p = 0; p < b.parts; ++p) {
    PartJob J{};
    J.ops = (const DevOp*)(base + (uint64_t)plan.op_begin[p] * sizeof(DevOp));
    J.layers = (const DevLayer*)(base + o_lay + (uint64_t)p * NL * sizeof(DevLayer));
    J.own = (const uint32_t*)(base + o_lst + (uint64_t)plan.own_begin[p] * 4);
    J.need = (const uint32_t*)(base + o_lst + (uint64_t)plan.need_begin[p] * 4);
    J.n_layers = NL;
    J.n_own = plan.own_n[p];
    J.n_need = plan.need_n[p];
    memcpy(b.part_host.data() + b.part_jobs_off + (uint64_t)p * sizeof(PartJob), &J, sizeof J);
  }
}

uint32_t choose_mapping(const DesignHost& h, uint32_t n_inst, const rteaal_batch_opts* o) {
  if (o && o->mapping == RTEAAL_MAP_PARTITIONED) return RTEAAL_MAP_PARTITIONED;
  if (o && o->mapping == RTEAAL_MAP_RESIDENT) return RTEAAL_MAP_RESIDENT;
  if (o && o->mapping == RTEAAL_MAP_SWEEP) return RTEAAL_MAP_SWEEP;
  if (o && o->mapping == RTEAAL_MAP_LAYERED) return RTEAAL_MAP_LAYERED;
  (void)h;
  return n_inst < 32 ? RTEAAL_MAP_RESIDENT : RTEAAL_MAP_SWEEP;
}

// AUTO options with a tuned entry for (design, n_inst) resolve to that entry.
const rteaal_batch_opts* resolve_opts(rteaal_ctx* ctx, uint32_t design, uint32_t n_inst,
                                      const rteaal_batch_opts* o) {
  if (o && o->mapping != RTEAAL_MAP_AUTO) return o;
  auto it = ctx->tuned.find({design, n_inst});
  return it == ctx->tuned.end() ? o : &it->second;
}

DesignHost* find_design(rteaal_ctx* ctx, rteaal_design_id id) {
  auto it = ctx->designs.find(id);
  return it == ctx->designs.end() ? nullptr : it->second.get();
}

Batch* find_batch(rteaal_ctx* ctx, rteaal_batch_id id) {
  auto it = ctx->batches.find(id);
  return it == ctx->batches.end() ? nullptr : it->second.get();
}

Program program_of(const DesignHost& h) {
  Program p{};
  p.ops = (const DevOp*)h.d_ops.p;
  p.layers = (const DevLayer*)h.d_layers.p;
  p.const_limbs = (const uint64_t*)h.d_consts.p;
  p.n_layers = (uint32_t)h.layers.size();
  p.words_per_inst = h.words_per_inst;
  return p;
}

constexpr uint64_t kResidentChunk = 1024;  // cycles per RESIDENT launch

ResJob res_job(const DesignHost& h, const Batch& b, uint64_t n_cycles) {
  ResJob J{};
  J.ops = (const DevOp*)h.d_ops.p;
  J.layers = (const DevLayer*)h.d_layers.p;
  J.const_limbs = (const uint64_t*)h.d_consts.p;
  J.n_layers = (uint32_t)h.layers.size();
  J.words_per_inst = h.words_per_inst;
  J.n_ops_total = (uint32_t)h.ops.size();
  J.n_inst_total = b.n_inst;
  J.L = b.L;
  J.state = (char*)b.state.p;
  J.seeds = (const uint64_t*)b.seeds.p;
  J.ctl = (const DevCtl*)b.ctl.p;
  J.n_cycles = n_cycles;
  J.regs = (const SlotRef*)h.d_reg_refs.p;
  J.digest = (uint64_t*)b.dig.p;
  J.n_regs = h.n_regs;
  return J;
}

// After the stream has drained: a persistent batch whose grid barrier wait
// ran out (its error flag set) leaves its state undefined, so the context
// becomes unusable.
rteaal_status check_grid(rteaal_ctx* ctx, const Batch& b) {
  if ((!b.persistent && b.mapping != RTEAAL_MAP_PARTITIONED) || !b.gsync.p) return RTEAAL_OK;
  GridSync g{};
  HIP_TRY(ctx, hipMemcpy(&g, b.gsync.p, sizeof g, hipMemcpyDeviceToHost));
  if (g.error) {
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "batch %u: a grid barrier wait exceeded its limit of %u spins",
                b.id, ctx->spin_limit);
  }
  return RTEAAL_OK;
}

// The register digest of every instance after a cycle (SWEEP and LAYERED;
// RESIDENT folds it inside its kernel).
hipError_t digest(const DesignHost& h, const Batch& b, hipStream_t s) {
  uint64_t* d = (uint64_t*)b.dig.p;
  return launch_digest(b.mapping == RTEAAL_MAP_SWEEP, b.L, (const char*)b.state.p,
                       (const SlotRef*)h.d_reg_refs.p, h.n_regs, b.n_inst, d, d + b.n_slot, s);
}

// Launches of one layer's common operations: one per operand count when the
// layer is large enough for the extra launches to pay, else one for all.
template <class F>
hipError_t for_light_launches(const DesignHost& h, const Batch& b, uint32_t li, TilePass tp,
                              F&& launch) {
  const DevLayer& ly = h.layers[li];
  const uint64_t n_light = (ly.end - ly.begin) - (ly.hend - ly.hbeg);
  if (n_light == 0) return hipSuccess;
  const bool split = b.arity_split == 2 ||
                     (b.arity_split == 0 && n_light * tp.count >= (1ull << 20));
  if (!split) return launch(OpRanges{ly.begin, ly.hbeg, ly.hend, ly.end}, 3u);
  for (uint32_t a = 1; a <= 3; ++a) {
    const OpRanges& r = h.light[li][a - 1];
    if (r.e0 == r.b0 && r.e1 == r.b1) continue;
    const hipError_t e = launch(r, a);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The tile passes of one SWEEP cycle.
std::vector<TilePass> tile_passes(const Batch& b) {
  const uint32_t n = b.L.n_tiles_alloc, step = b.tpp ? b.tpp : n;
  std::vector<TilePass> out;
  for (uint32_t t = 0; t < n; t += step) out.push_back(TilePass{t, std::min(step, n - t)});
  return out;
}

// Captured multi-batch cycles kept per context.  A full cache is not
// evicted: sets beyond it are stepped batch by batch, and a captured cycle
// goes when one of its batches is freed.
constexpr size_t kMaxMultiGraphs = 16;

void drop_multi_graph(rteaal_ctx* ctx, size_t k) {
  MultiGraph& g = *ctx->mgraphs[k];
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  dev_free(ctx, g.table);
  ctx->mgraphs.erase(ctx->mgraphs.begin() + (long)k);
}

// Forgets every captured multi-batch cycle that involves batch id (before
// its memory is freed).  The caller has waited for the stream.
void drop_multi_graphs_of(rteaal_ctx* ctx, uint32_t id) {
  for (size_t k = ctx->mgraphs.size(); k-- > 0;) {
    const auto& ids = ctx->mgraphs[k]->ids;
    if (std::binary_search(ids.begin(), ids.end(), id)) drop_multi_graph(ctx, k);
  }
}

// Captures one cycle of the batches `bs` (SWEEP or LAYERED, not watched, no
// tile passes, not timed) as a single graph.  Every batch's layers are
// spread over S = (most layers of any batch) slots, layer i of a batch with
// L layers at slot floor(i S / L), so that each slot holds a similar share
// of the work; the launches of one slot (common operations per tile group,
// heavy operations, fused mux chains, LAYERED layers) each cover every batch
// with a layer there, read only earlier slots' results and write disjoint
// slots, so they run as parallel branches.
rteaal_status build_multi_graph(rteaal_ctx* ctx, const std::vector<Batch*>& bs,
                                std::unique_ptr<MultiGraph>* out) {
  struct Launch {
    uint32_t kind, tg;
    bool narrow;  // heavy pieces of designs with no value wider than 128 bits
    std::vector<MultiSeg> segs;
    std::vector<uint32_t> wave0;
    size_t off = 0;  // byte offset of the table in the device buffer
  };
  uint32_t S = 0;
  for (Batch* b : bs) S = std::max<uint32_t>(S, (uint32_t)find_design(ctx, b->design)->layers.size());
  std::vector<std::vector<Launch>> slots(S);
  auto add = [&](uint32_t t, uint32_t kind, uint32_t tg, bool narrow, const MultiSeg& seg,
                 uint64_t waves) {
    if (!waves) return true;
    auto& v = slots[t];
    Launch* l = nullptr;
    for (auto& x : v)
      if (x.kind == kind && x.tg == tg && x.narrow == narrow) l = &x;
    if (!l) {
      v.push_back(Launch{kind, tg, narrow, {}, {0u}, 0});
      l = &v.back();
    }
    const uint64_t end = (uint64_t)l->wave0.back() + waves;
    if (end >= (1ull << 31)) return false;
    l->segs.push_back(seg);
    l->wave0.push_back((uint32_t)end);
    return true;
  };
  std::vector<DigestSeg> dsegs;
  std::vector<uint32_t> dwave0{0u};
  uint32_t max_inst = 0;
  for (Batch* b : bs) {
    const DesignHost& h = *find_design(ctx, b->design);
    const uint32_t Lb = (uint32_t)h.layers.size();
    MultiSeg base{};
    base.ops = (const DevOp*)h.d_ops.p;
    base.layers = (const DevLayer*)h.d_layers.p;
    base.const_limbs = (const uint64_t*)h.d_consts.p;
    base.state = (char*)b->state.p;
    base.seeds = (const uint64_t*)b->seeds.p;
    base.ctl = (const DevCtl*)b->ctl.p;
    base.L = b->L;
    base.n_inst = b->n_inst;
    base.words_per_inst = h.words_per_inst;
    base.opw = b->opw ? b->opw : 16u;
    base.unroll = b->unroll ? b->unroll : 1u;
    const bool sweep = b->mapping == RTEAAL_MAP_SWEEP;
    const uint32_t T = b->L.n_tiles_alloc;
    for (uint32_t li = 0; li < Lb; ++li) {
      const uint32_t t = (uint32_t)((uint64_t)li * S / Lb);
      const DevLayer& ly = h.layers[li];
      MultiSeg g = base;
      g.layer = li;
      bool ok = true;
      if (sweep) {
        const uint32_t opw = g.opw;
        const uint32_t n1 = ly.hbeg - ly.begin, n2 = ly.end - ly.hend;
        g.r = OpRanges{ly.begin, ly.hbeg, ly.hend, ly.end};
        g.split = (n1 + opw - 1) / opw;
        g.n_groups = T / b->tg;
        ok = ok && add(t, 0, b->tg, false, g, (uint64_t)(g.split + (n2 + opw - 1) / opw) * g.n_groups);
        // Heavy pieces take one tile per wavefront when the batch's tile
        // group is at most 2, so that a layer index stays within the lean
        // mixed variants.  A design with no value wider than 128 bits runs
        // them in the two-limb form only (narrow: fewer instructions and
        // registers).  Two tiles per wavefront in that form measured slower
        // on multi-64 (1.40e6 against 1.60e6): it needs the larger lean set.
        const bool narrow = h.n_idx[CL3] == 0 && h.n_idx[CL4] == 0;
        const uint32_t th = b->tg <= 2 ? 1u : 2u;
        const uint32_t h1 = ly.hm0 - ly.hbeg, h2 = ly.hend - ly.hm1;
        g.r = OpRanges{ly.hbeg, ly.hm0, ly.hm1, ly.hend};  // the heavy range (see MultiSeg)
        g.n_groups = T / th;
        ok = ok && add(t, 1, th, narrow, g,
                       (uint64_t)((h1 + opw - 1) / opw + (h2 + opw - 1) / opw) * g.n_groups);
        const uint32_t tm = b->tg >= 4 ? 4u : b->tg;
        g.n_groups = T / tm;
        ok = ok && add(t, 2, tm, false, g, (uint64_t)(ly.hm1 - ly.hm0) * g.n_groups);
      } else {
        const uint32_t n = ly.end - ly.begin;
        g.n_groups = (n + 63u) / 64u;
        ok = ok && add(t, 3, 1, false, g, (uint64_t)g.n_groups * b->n_inst);
      }
      if (!ok) return fail(ctx, RTEAAL_E_UNSUPPORTED, "too many wavefronts for one multi-batch launch");
    }
    DigestSeg d{};
    d.L = b->L;
    d.state = (const char*)b->state.p;
    d.regs = (const SlotRef*)h.d_reg_refs.p;
    d.digest = (uint64_t*)b->dig.p;
    d.acc = (uint64_t*)b->dig.p + b->n_slot;
    d.ctl = (DevCtl*)b->ctl.p;
    d.n_regs = h.n_regs;
    d.n_inst = b->n_inst;
    d.sweep = sweep ? 1u : 0u;
    digest_shape(sweep, h.n_regs, b->n_inst, &d.n_units, &d.per);
    const uint64_t dw = h.n_regs ? (uint64_t)d.n_units * ((h.n_regs + d.per - 1) / d.per) : 0;
    if ((uint64_t)dwave0.back() + dw >= (1ull << 31))
      return fail(ctx, RTEAAL_E_UNSUPPORTED, "too many wavefronts for one multi-batch digest");
    dsegs.push_back(d);
    dwave0.push_back(dwave0.back() + (uint32_t)dw);
    max_inst = std::max(max_inst, b->n_inst);
  }
  // Small layer indices: their launches become one mixed launch (each
  // segment carrying its kind and tile group), which the cycle runs without
  // forking.
  for (auto& v : slots) {
    if (v.size() < 2) continue;
    uint64_t waves = 0;
    bool ok = true, lean = true, small = true;
    for (const Launch& l : v) {
      waves += l.wave0.back();
      ok = ok && multi_mixable(l.kind, l.tg);
      lean = lean && multi_lean(l.kind, l.tg, l.narrow);
      // the smallest set: no LAYERED pieces, heavy pieces on one tile, at
      // most 2 operations in flight
      small = small && l.kind != 3 && (l.kind != 1 || l.tg == 1);
      for (const MultiSeg& x : l.segs) small = small && (l.kind != 0 || x.unroll <= 2);
    }
    if (!ok || waves > ctx->mixed_max_waves) continue;
    Launch m{lean ? (small ? 6u : 5u) : 4u, 0u, false, {}, {0u}, 0};
    for (const Launch& l : v) {
      for (size_t k = 0; k < l.segs.size(); ++k) {
        MultiSeg x = l.segs[k];
        x.variant = multi_variant(l.kind, l.tg, x.unroll, lean, l.narrow);
        m.segs.push_back(x);
        m.wave0.push_back(m.wave0.back() + (l.wave0[k + 1] - l.wave0[k]));
      }
    }
    v.clear();
    v.push_back(std::move(m));
  }
  // One device buffer: every launch's segments and prefix, then the digest's.
  size_t bytes = 0;
  auto place = [&](size_t n) {
    const size_t o = bytes;
    bytes = (bytes + n + 255) & ~size_t(255);
    return o;
  };
  // Per launch: the segments, then the prefix wave0 and the segment of
  // every wavefront after it.
  for (auto& v : slots)
    for (auto& l : v) {
      l.off = place(l.segs.size() * sizeof(MultiSeg));
      place((l.wave0.size() + l.wave0.back()) * 4);
    }
  const size_t doff = place(dsegs.size() * sizeof(DigestSeg));
  const size_t dwoff = place(dwave0.size() * 4);
  std::vector<char> host(bytes, 0);
  for (auto& v : slots)
    for (auto& l : v) {
      memcpy(host.data() + l.off, l.segs.data(), l.segs.size() * sizeof(MultiSeg));
      const size_t woff = (l.off + l.segs.size() * sizeof(MultiSeg) + 255) & ~size_t(255);
      memcpy(host.data() + woff, l.wave0.data(), l.wave0.size() * 4);
      uint32_t* seg_of = (uint32_t*)(host.data() + woff) + l.wave0.size();
      for (uint32_t k = 0; k + 1 < l.wave0.size(); ++k)
        for (uint32_t w = l.wave0[k]; w < l.wave0[k + 1]; ++w) seg_of[w] = k;
    }
  memcpy(host.data() + doff, dsegs.data(), dsegs.size() * sizeof(DigestSeg));
  memcpy(host.data() + dwoff, dwave0.data(), dwave0.size() * 4);
  auto g = std::make_unique<MultiGraph>();
  for (Batch* b : bs) g->ids.push_back(b->id);
  std::sort(g->ids.begin(), g->ids.end());
  if (!alloc_all(ctx, {{&g->table, bytes}}))
    return fail(ctx, RTEAAL_E_NO_MEMORY, "multi-batch table allocation failed");
  char* dev = (char*)g->table.p;
  hipError_t e = hipMemcpyAsync(dev, host.data(), bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    if (!ctx->cap[k]) e = hipStreamCreateWithFlags(&ctx->cap[k], hipStreamNonBlocking);
    if (e == hipSuccess && !ctx->cap_join[k])
      e = hipEventCreateWithFlags(&ctx->cap_join[k], hipEventDisableTiming);
  }
  if (e == hipSuccess && !ctx->cap_fork) e = hipEventCreateWithFlags(&ctx->cap_fork, hipEventDisableTiming);
  if (e != hipSuccess) {
    dev_free(ctx, g->table);
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "multi-batch set-up: %s", hipGetErrorString(e));
  }
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
  for (auto& v : slots) {
    if (e != hipSuccess) break;
    const size_t n_fork = std::min<size_t>(v.size(), 4) - (v.empty() ? 0 : 1);
    if (n_fork) {
      e = hipEventRecord(ctx->cap_fork, ctx->stream);
      for (size_t k = 0; k < n_fork && e == hipSuccess; ++k)
        e = hipStreamWaitEvent(ctx->cap[k], ctx->cap_fork, 0);
    }
    for (size_t k = 0; k < v.size() && e == hipSuccess; ++k) {
      const Launch& l = v[k];
      const size_t woff = (l.off + l.segs.size() * sizeof(MultiSeg) + 255) & ~size_t(255);
      hipStream_t s2 = k == 0 || k > n_fork ? ctx->stream : ctx->cap[k - 1];
      e = launch_multi(l.kind, l.tg, (const MultiSeg*)(dev + l.off), (const uint32_t*)(dev + woff),
                       (uint32_t)l.segs.size(), l.wave0.back(), s2);
      ++g->launches;
    }
    for (size_t k = 0; k < n_fork && e == hipSuccess; ++k) {
      e = hipEventRecord(ctx->cap_join[k], ctx->cap[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(ctx->stream, ctx->cap_join[k], 0);
    }
  }
  if (e == hipSuccess)
    e = launch_digest_multi((const DigestSeg*)(dev + doff), (const uint32_t*)(dev + dwoff),
                            (uint32_t)dsegs.size(), dwave0.back(), max_inst, ctx->stream);
  hipError_t e2 = hipStreamEndCapture(ctx->stream, &graph);
  if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    g->exec = nullptr;
    dev_free(ctx, g->table);
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "multi-batch graph capture failed: %s",
                hipGetErrorString(e != hipSuccess ? e : e2));
  }
  *out = std::move(g);
  return RTEAAL_OK;
}

// The cached captured cycle of batch set bs, or null.
MultiGraph* cached_multi_graph(rteaal_ctx* ctx, const std::vector<Batch*>& bs) {
  std::vector<uint32_t> ids;
  for (Batch* b : bs) ids.push_back(b->id);
  std::sort(ids.begin(), ids.end());
  for (auto& g : ctx->mgraphs)
    if (g->ids == ids) return g.get();
  return nullptr;
}

// The captured cycle of batch set bs, built on first use.  The caller has
// checked that the cache has room (a captured cycle is dropped only when one
// of its batches is freed, or with the context).
rteaal_status multi_graph(rteaal_ctx* ctx, const std::vector<Batch*>& bs, MultiGraph** out) {
  if (MultiGraph* g = cached_multi_graph(ctx, bs)) {
    g->last_use = ++ctx->mg_clock;
    *out = g;
    return RTEAAL_OK;
  }
  if (ctx->mgraphs.size() >= kMaxMultiGraphs)
    return fail(ctx, RTEAAL_E_UNSUPPORTED, "multi-batch graph cache full");
  std::unique_ptr<MultiGraph> g;
  const rteaal_status st = build_multi_graph(ctx, bs, &g);
  if (st != RTEAAL_OK) return st;
  g->last_use = ++ctx->mg_clock;
  *out = g.get();
  ctx->mgraphs.push_back(std::move(g));
  return RTEAAL_OK;
}

// LAYERED: one launch per (non-empty) layer for all instances, then the
// cycle advance and the capture; the cycle is captured once as a HIP graph.
rteaal_status enqueue_layered(rteaal_ctx* ctx, DesignHost& h, Batch& b, uint64_t n_cycles) {
  const ResJob J = res_job(h, b, 1);
  DevCtl* ctl = (DevCtl*)b.ctl.p;
  if (b.persistent) {
    // A watched batch runs one cycle per launch, so each cycle is captured.
    const uint64_t chunk = b.n_watch ? 1 : kResidentChunk;
    for (uint64_t done = 0; done < n_cycles;) {
      const uint64_t n = std::min(chunk, n_cycles - done);
      HIP_TRY(ctx, timed(b, ctx->stream, 0, [&] {
                return launch_layer_persistent(res_job(h, b, n), b.n_inst, b.unroll,
                                               (GridSync*)b.gsync.p, (uint64_t*)b.dig.p + b.n_slot,
                                               ctx->spin_limit, 0, ctx->stream);
              }));
      HIP_TRY(ctx, launch_advance(ctl, n, ctx->stream));
      HIP_TRY(ctx, capture(b, ctx->stream));
      done += n;
    }
    return RTEAAL_OK;
  }
  auto cycle = [&](hipStream_t s, bool timed_launches) -> hipError_t {
    hipError_t e = hipSuccess;
    for (uint32_t li = 0; li < h.layers.size() && e == hipSuccess; ++li) {
      const uint32_t n = h.layers[li].end - h.layers[li].begin;
      if (!n) continue;
      auto go = [&] { return launch_layer(J, li, n, b.n_inst, b.block, b.unroll, s); };
      e = timed_launches ? timed(b, s, 0, go) : go();
    }
    if (e == hipSuccess) e = digest(h, b, s);
    if (e == hipSuccess) e = launch_advance(ctl, 1, s);
    if (e == hipSuccess) e = capture(b, s);
    return e;
  };
  if (b.profile) {
    for (uint64_t c = 0; c < n_cycles; ++c) HIP_TRY(ctx, cycle(ctx->stream, true));
    return RTEAAL_OK;
  }
  if (!b.graph) {
    hipGraph_t g = nullptr;
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = cycle(ctx->stream, false);
    hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
    if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess || e2 != hipSuccess) {
      b.graph = nullptr;
      ctx->poisoned = true;
      return fail(ctx, RTEAAL_E_DEVICE, "graph capture failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
  }
  for (uint64_t c = 0; c < n_cycles; ++c) HIP_TRY(ctx, hipGraphLaunch(b.graph, ctx->stream));
  return RTEAAL_OK;
}

PartRun part_run(rteaal_ctx* ctx, const DesignHost& h, const Batch& b, uint64_t n_cycles) {
  PartRun R{};
  R.parts = (const PartJob*)((const char*)b.part_mem.p + b.part_jobs_off);
  R.const_limbs = (const uint64_t*)h.d_consts.p;
  R.regs = (const SlotRef*)h.d_reg_refs.p;
  R.state = (char*)b.state.p;
  R.seeds = (const uint64_t*)b.seeds.p;
  R.ctl = (const DevCtl*)b.ctl.p;
  R.xch = (uint64_t*)b.xch.p;
  R.acc = (unsigned long long*)b.pacc.p;
  R.digest = (uint64_t*)b.dig.p;
  R.gs = (GridSync*)b.gsync.p;
  R.pitch = b.copy_pitch;
  R.n_cycles = n_cycles;
  R.n_parts = b.parts;
  R.n_inst = b.n_inst;
  R.reg_words = h.reg_words;
  R.words_per_inst = h.words_per_inst;
  R.spin_limit = ctx->spin_limit;
  return R;
}

rteaal_status enqueue_cycles(rteaal_ctx* ctx, DesignHost& h, Batch& b, uint64_t n_cycles) {
  const Program p = program_of(h);
  DevCtl* ctl = (DevCtl*)b.ctl.p;
  if (b.mapping == RTEAAL_MAP_PARTITIONED) {
    for (uint64_t done = 0; done < n_cycles;) {
      const uint64_t n = std::min(kResidentChunk, n_cycles - done);
      HIP_TRY(ctx, timed(b, ctx->stream, 0, [&] {
                return launch_partitioned(part_run(ctx, h, b, n), b.block, b.lds, ctx->stream);
              }));
      HIP_TRY(ctx, launch_advance(ctl, n, ctx->stream));
      done += n;
    }
    return RTEAAL_OK;
  }
  if (b.mapping == RTEAAL_MAP_RESIDENT) {
    // A watched batch runs one cycle per launch, so each cycle is captured.
    const uint64_t chunk = b.n_watch ? 1 : kResidentChunk;
    for (uint64_t done = 0; done < n_cycles;) {
      const uint64_t n = std::min(chunk, n_cycles - done);
      HIP_TRY(ctx, timed(b, ctx->stream, 0, [&] {
                const ResJob J = res_job(h, b, n);
                return launch_resident(J, b.n_inst, 0, b.block, b.lds, b.lds_ops, b.unroll,
                                       ctx->stream);
              }));
      HIP_TRY(ctx, launch_advance(ctl, n, ctx->stream));
      HIP_TRY(ctx, capture(b, ctx->stream));
      done += n;
    }
    return RTEAAL_OK;
  }
  if (b.mapping == RTEAAL_MAP_LAYERED) return enqueue_layered(ctx, h, b, n_cycles);
  // SWEEP: per layer the common kernel and the heavy one, the cycle captured
  // once as a HIP graph.
  char* st = (char*)b.state.p;
  const uint64_t* seeds = (const uint64_t*)b.seeds.p;
  const std::vector<TilePass> passes = tile_passes(b);
  if (b.profile) {
    for (uint64_t c = 0; c < n_cycles; ++c) {
      for (const TilePass& tp : passes)
        for (uint32_t li = 0; li < h.layers.size(); ++li) {
          const DevLayer& ly = h.layers[li];
          HIP_TRY(ctx, for_light_launches(h, b, li, tp, [&](const OpRanges& r, uint32_t a) {
                    return timed(b, ctx->stream, 0, [&] {
                      return launch_sweep_light(p, b.L, st, r, a, b.opw, b.unroll, b.tg, tp,
                                                ctx->stream);
                    });
                  }));
          if (ly.hend > ly.hbeg)
            HIP_TRY(ctx, timed(b, ctx->stream, 1, [&] {
                      return launch_sweep_heavy(p, b.L, st, seeds, ctl, b.n_inst, li, ly, b.opw,
                                                b.tg, tp, ctx->stream);
                    }));
        }
      HIP_TRY(ctx, digest(h, b, ctx->stream));
      HIP_TRY(ctx, launch_advance(ctl, 1, ctx->stream));
      HIP_TRY(ctx, capture(b, ctx->stream));
    }
    return RTEAAL_OK;
  }
  if (!b.graph) {
    for (int k = 0; k < 3; ++k) {
      if (!ctx->cap[k]) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap[k], hipStreamNonBlocking));
      if (!ctx->cap_join[k])
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->cap_join[k], hipEventDisableTiming));
    }
    if (!ctx->cap_fork) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->cap_fork, hipEventDisableTiming));
    hipGraph_t g = nullptr;
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    // The launches of one layer (its common operations, per operand count or
    // together, and its heavy ones) write disjoint slots and read only earlier
    // layers: they become parallel branches of the graph, joined before the
    // next layer.
    struct Piece {
      OpRanges r;
      uint32_t n_src;  // 0: the heavy launch
    };
    std::vector<Piece> pieces;
    // Parallel passes: every tile pass is a graph branch of its own (its
    // layers in order on one stream), joined before the digest.
    const bool branches = b.pbranch && passes.size() > 1;
    if (branches) {
      e = hipEventRecord(ctx->cap_fork, ctx->stream);
      for (size_t k = 0; k + 1 < passes.size() && e == hipSuccess; ++k)
        e = hipStreamWaitEvent(ctx->cap[k], ctx->cap_fork, 0);
    }
    for (size_t pi = 0; pi < passes.size(); ++pi) {
      const TilePass& tp = passes[pi];
      hipStream_t ps = branches && pi > 0 ? ctx->cap[pi - 1] : ctx->stream;
      for (uint32_t li = 0; li < h.layers.size() && e == hipSuccess; ++li) {
        const DevLayer& ly = h.layers[li];
        pieces.clear();
        e = for_light_launches(h, b, li, tp, [&](const OpRanges& r, uint32_t a) {
          pieces.push_back(Piece{r, a});
          return hipSuccess;
        });
        if (ly.hend > ly.hbeg) pieces.push_back(Piece{OpRanges{}, 0u});
        auto run = [&](const Piece& pc, hipStream_t s2) {
          return pc.n_src ? launch_sweep_light(p, b.L, st, pc.r, pc.n_src, b.opw, b.unroll, b.tg,
                                               tp, s2)
                          : launch_sweep_heavy(p, b.L, st, seeds, ctl, b.n_inst, li, ly, b.opw,
                                               b.tg, tp, s2);
        };
        // Only large layers fork: for small ones the branches' scheduling costs
        // more than the overlap returns, and batches stepped together already
        // overlap on their own streams.
        // (Parallel passes use the branch streams, so their layers do not fork.)
        const bool large = (uint64_t)(ly.end - ly.begin) * tp.count >= (1ull << 20);
        const size_t n_fork =
            large && !branches ? std::min<size_t>(pieces.size(), 4) - (pieces.empty() ? 0 : 1) : 0;
        if (e == hipSuccess && n_fork) {
          e = hipEventRecord(ctx->cap_fork, ps);
          for (size_t k = 0; k < n_fork && e == hipSuccess; ++k)
            e = hipStreamWaitEvent(ctx->cap[k], ctx->cap_fork, 0);
        }
        for (size_t k = 0; k < pieces.size() && e == hipSuccess; ++k)
          e = run(pieces[k], k == 0 || k > n_fork ? ps : ctx->cap[k - 1]);
        // (pieces beyond the forked ones, if any, run on the capturing stream)
        for (size_t k = 0; k < n_fork && e == hipSuccess; ++k) {
          e = hipEventRecord(ctx->cap_join[k], ctx->cap[k]);
          if (e == hipSuccess) e = hipStreamWaitEvent(ps, ctx->cap_join[k], 0);
        }
      }
    }
    if (branches)
      for (size_t k = 0; k + 1 < passes.size() && e == hipSuccess; ++k) {
        e = hipEventRecord(ctx->cap_join[k], ctx->cap[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(ctx->stream, ctx->cap_join[k], 0);
      }
    if (e == hipSuccess) e = digest(h, b, ctx->stream);
    if (e == hipSuccess) e = launch_advance(ctl, 1, ctx->stream);
    if (e == hipSuccess) e = capture(b, ctx->stream);
    hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      ctx->poisoned = true;
      return fail(ctx, RTEAAL_E_DEVICE, "graph capture failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b.graph = nullptr;
      ctx->poisoned = true;
      return fail(ctx, RTEAAL_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
  }
  for (uint64_t c = 0; c < n_cycles; ++c) HIP_TRY(ctx, hipGraphLaunch(b.graph, ctx->stream));
  return RTEAAL_OK;
}

}  // namespace

// ===========================================================================
// C interface.
// ===========================================================================
extern "C" {

rteaal_status rteaal_create(int device, void* stream, const rteaal_allocator* alloc,
                            rteaal_ctx** out) {
  if (!out) return fail(nullptr, RTEAAL_E_INVALID_ARG, "out is null");
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(nullptr, RTEAAL_E_INVALID_ARG, "allocator needs both alloc and free");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || device < 0 || device >= n)
    return fail(nullptr, RTEAAL_E_INVALID_ARG, "no HIP device %d (%d visible)", device, n);
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, RTEAAL_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  auto ctx = std::make_unique<rteaal_ctx>();
  ctx->device = device;
  if (alloc) {
    ctx->alloc = *alloc;
    ctx->has_alloc = true;
  }
  if (stream) {
    ctx->stream = (hipStream_t)stream;
  } else {
    e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(nullptr, RTEAAL_E_DEVICE, "stream: %s", hipGetErrorString(e));
    ctx->own_stream = true;
  }
  if (const char* sl = std::getenv("RTEAAL_GRID_SPIN_LIMIT"))
    ctx->spin_limit = (uint32_t)std::max(1L, std::min(std::atol(sl), (long)UINT32_MAX));
  if (const char* mc = std::getenv("RTEAAL_MULTI_CHAINS"))
    ctx->multi_chains = (uint32_t)std::max(1L, std::min(std::atol(mc), 4L));
  if (const char* mw = std::getenv("RTEAAL_MIXED_MAX_WAVES"))
    ctx->mixed_max_waves = (uint32_t)std::max(0L, std::min(std::atol(mw), (long)UINT32_MAX));
  ctx->scratch = scratch_on(device);
  if (!ctx->scratch) {
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    return fail(nullptr, RTEAAL_E_DEVICE, "hipGetSymbolAddress of the staging array failed");
  }
  // The auxiliary streams of rteaal_step_many, created now and in this
  // order (the first chain's, then the RESIDENT configurations', then the
  // rest), so that the runtime hands them hardware queues in that order:
  // with enough queues (GPU_MAX_HW_QUEUES) a chain of captured cycles does
  // not share a queue with a long RESIDENT launch.
  for (int a : {0, 4, 5, 6, 1, 2, 3, 7}) {
    e = hipStreamCreateWithFlags(&ctx->aux[a], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join[a], hipEventDisableTiming);
    if (e != hipSuccess) {
      for (int k = 0; k < rteaal_ctx::kAux; ++k) {
        if (ctx->aux[k]) (void)hipStreamDestroy(ctx->aux[k]);
        if (ctx->join[k]) (void)hipEventDestroy(ctx->join[k]);
      }
      if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
      return fail(nullptr, RTEAAL_E_DEVICE, "auxiliary stream: %s", hipGetErrorString(e));
    }
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess)
    ctx->max_lds = std::min<size_t>(prop.maxSharedMemoryPerMultiProcessor, resident_max_lds());
  if (ctx->max_lds == 0) ctx->max_lds = 64 * 1024;
  *out = ctx.release();
  return RTEAAL_OK;
}

void rteaal_destroy(rteaal_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->batches) {
    Batch& b = *kv.second;
    if (b.graph) (void)hipGraphExecDestroy(b.graph);
    destroy_events(b);
    free_watch(ctx, b);
    dev_free(ctx, b.state);
    dev_free(ctx, b.seeds);
    dev_free(ctx, b.ctl);
    dev_free(ctx, b.dig);
    dev_free(ctx, b.gsync);
    free_parts(ctx, b);
  }
  for (auto& kv : ctx->designs) {
    DesignHost& h = *kv.second;
    dev_free(ctx, h.d_ops);
    dev_free(ctx, h.d_layers);
    dev_free(ctx, h.d_consts);
    dev_free(ctx, h.d_reg_refs);
    dev_free(ctx, h.d_slot_refs);
  }
  dev_free(ctx, ctx->multi);
  while (!ctx->mgraphs.empty()) drop_multi_graph(ctx, ctx->mgraphs.size() - 1);
  for (int k = 0; k < rteaal_ctx::kAux; ++k) {
    if (ctx->aux[k]) (void)hipStreamDestroy(ctx->aux[k]);
    if (ctx->join[k]) (void)hipEventDestroy(ctx->join[k]);
  }
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  for (int k = 0; k < 3; ++k) {
    if (ctx->cap[k]) (void)hipStreamDestroy(ctx->cap[k]);
    if (ctx->cap_join[k]) (void)hipEventDestroy(ctx->cap_join[k]);
  }
  if (ctx->cap_fork) (void)hipEventDestroy(ctx->cap_fork);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* rteaal_last_error(const rteaal_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_err.c_str();
}

rteaal_status rteaal_validate_design(const rteaal_design_desc* desc, char* err, size_t err_len) {
  Drivers drv;
  std::string why;
  rteaal_status st = validate(desc, &drv, &why, nullptr);
  if (err && err_len) {
    snprintf(err, err_len, "%s", st == RTEAAL_OK ? "" : why.c_str());
  }
  if (st != RTEAAL_OK) g_err = why;
  return st;
}

rteaal_status rteaal_fuse_mux_chains(const rteaal_design_desc* d, uint32_t max_pairs,
                                     uint32_t* layer_op_ptr, uint8_t* op_type, uint32_t* op_dst,
                                     uint32_t* op_src_ptr, uint32_t* op_src, uint16_t* op_imm,
                                     rteaal_fuse_result* result) {
  if (!d || !layer_op_ptr || !op_src_ptr || !result ||
      (d->n_ops && (!op_type || !op_dst || !op_imm || !op_src))) {
    g_err = "null argument";
    return RTEAAL_E_INVALID_ARG;
  }
  if (max_pairs < 1 || max_pairs > RTEAAL_MUXC_MAX_PAIRS) {
    g_err = "max_pairs must be 1.." + std::to_string(RTEAAL_MUXC_MAX_PAIRS);
    return RTEAAL_E_INVALID_ARG;
  }
  Drivers drv;
  std::string why;
  const rteaal_status st = validate(d, &drv, &why, nullptr);
  if (st != RTEAAL_OK) {
    g_err = why;
    return st;
  }
  const uint32_t n = d->n_ops;
  // Readers per slot (operand entries) and latched slots.
  std::vector<uint32_t> readers(d->n_slots, 0);
  for (uint32_t q = 0; q < d->op_src_ptr[n]; ++q) ++readers[d->op_src[q]];
  std::vector<char> latched(d->n_slots, 0);
  for (uint32_t j = 0; j < d->n_regs; ++j) latched[d->reg_next[j]] = 1;
  // inner[o]: the MUX whose result o's default operand is, when o may absorb it.
  constexpr uint32_t kNone = UINT32_MAX;
  std::vector<uint32_t> inner(n, kNone);
  std::vector<char> is_inner(n, 0);
  for (uint32_t o = 0; o < n; ++o) {
    if (d->op_type[o] != RTEAAL_MUX) continue;
    const uint32_t x = d->op_src[d->op_src_ptr[o] + 2];
    if (drv.kind[x] != DRV_OP) continue;
    const uint32_t p = drv.which[x];
    if (d->op_type[p] != RTEAAL_MUX || readers[x] != 1 || latched[x] ||
        d->slot_width[x] < d->slot_width[d->op_dst[o]])
      continue;
    inner[o] = p;
    is_inner[p] = 1;
  }
  // Walk every path from its outermost MUX; cut it into pieces of at most
  // max_pairs pairs.  A fused head's operands are lists[at[o], at[o] + len[o]).
  std::vector<uint32_t> at(n, kNone), len(n, 0), lists;
  std::vector<char> absorbed(n, 0);
  uint32_t n_fused = 0, n_absorbed = 0;
  for (uint32_t o = 0; o < n; ++o) {
    if (d->op_type[o] != RTEAAL_MUX || is_inner[o] || inner[o] == kNone) continue;
    for (uint32_t head = o; head != kNone;) {
      const uint32_t start = (uint32_t)lists.size();
      uint32_t m = head, pairs = 0;
      for (;;) {
        const uint32_t* sm = d->op_src + d->op_src_ptr[m];
        lists.push_back(sm[0]);
        lists.push_back(sm[1]);
        ++pairs;
        if (inner[m] == kNone || pairs == max_pairs) {
          lists.push_back(sm[2]);
          break;
        }
        m = inner[m];
        absorbed[m] = 1;
        ++n_absorbed;
      }
      if (pairs > 1) {
        at[head] = start;
        len[head] = (uint32_t)lists.size() - start;
        ++n_fused;
      } else {
        lists.resize(start);
      }
      head = inner[m];
    }
  }
  // The fused design: the operations in their order, absorbed ones dropped.
  uint32_t k = 0;
  op_src_ptr[0] = 0;
  for (uint32_t i = 0; i < d->n_layers; ++i) {
    layer_op_ptr[i] = k;
    for (uint32_t o = d->layer_op_ptr[i]; o < d->layer_op_ptr[i + 1]; ++o) {
      if (absorbed[o]) continue;
      const bool f = at[o] != kNone;
      const uint32_t* src = f ? lists.data() + at[o] : d->op_src + d->op_src_ptr[o];
      const uint32_t ar = f ? len[o] : d->op_src_ptr[o + 1] - d->op_src_ptr[o];
      op_type[k] = f ? (uint8_t)RTEAAL_MUXC : d->op_type[o];
      op_dst[k] = d->op_dst[o];
      op_imm[k] = f ? 0 : d->op_imm[o];
      std::copy(src, src + ar, op_src + op_src_ptr[k]);
      op_src_ptr[k + 1] = op_src_ptr[k] + ar;
      ++k;
    }
  }
  layer_op_ptr[d->n_layers] = k;
  result->n_ops = k;
  result->n_operands = op_src_ptr[k];
  result->n_fused = n_fused;
  result->n_absorbed = n_absorbed;
  return RTEAAL_OK;
}

rteaal_status rteaal_levelize(rteaal_ctx* ctx, const rteaal_dag_desc* g, uint32_t* op_layer,
                              uint32_t* order, uint32_t* layer_ptr, uint32_t* n_layers) {
  if (!ctx || !g || !layer_ptr || !n_layers) return fail(ctx, RTEAAL_E_INVALID_ARG, "null argument");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  const uint32_t n = g->n_ops;
  if (n >= (1u << 31)) return fail(ctx, RTEAAL_E_INVALID_ARG, "n_ops %u is too large", n);
  if (n == 0) {
    layer_ptr[0] = 0;
    *n_layers = 0;
    return RTEAAL_OK;
  }
  if (!op_layer || !order || !g->op_src_ptr || !g->op_dst)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "null argument");
  // The remaining range checks run on the device before any kernel indexes
  // with the graph.
  if (g->op_src_ptr[0] != 0) return fail(ctx, RTEAAL_E_INVALID_ARG, "op_src_ptr[0] is not 0");
  const uint32_t ne = g->op_src_ptr[n];
  if (ne && !g->op_src) return fail(ctx, RTEAAL_E_INVALID_ARG, "null op_src");

  size_t temp = 0;
  HIP_TRY(ctx, levelize_temp_bytes(n, &temp));
  const size_t w = 4, n1 = (size_t)n + 1;
  Mem m_ptr, m_src, m_dst, m_prod, m_indeg, m_outdeg, m_optr, m_cur, m_oidx, m_f0, m_f1, m_layer,
      m_keys, m_vals, m_order, m_lptr, m_sizes, m_scal, m_temp;
  std::vector<std::pair<Mem*, size_t>> req = {
      {&m_ptr, n1 * w}, {&m_src, std::max<size_t>(ne, 1) * w}, {&m_dst, n * w},
      {&m_prod, (size_t)g->n_slots * w}, {&m_indeg, n * w}, {&m_outdeg, n1 * w},
      {&m_optr, n1 * w}, {&m_cur, n * w}, {&m_oidx, std::max<size_t>(ne, 1) * w},
      {&m_f0, n * w}, {&m_f1, n * w}, {&m_layer, n * w}, {&m_keys, n * w}, {&m_vals, n * w},
      {&m_order, n * w}, {&m_lptr, n1 * w}, {&m_sizes, (n + 16ull) * w}, {&m_scal, 8 * w},
      {&m_temp, temp}};
  if (!alloc_all(ctx, req))
    return fail(ctx, RTEAAL_E_NO_MEMORY, "device scratch for levelizing %u operations", n);
  auto release = [&] {
    for (auto& r : req) dev_free(ctx, *r.first);
  };
  LvBuffers B{};
  B.src_ptr = (const uint32_t*)m_ptr.p;
  B.src = (const uint32_t*)m_src.p;
  B.dst = (const uint32_t*)m_dst.p;
  B.producer = (uint32_t*)m_prod.p;
  B.indeg = (uint32_t*)m_indeg.p;
  B.outdeg = (uint32_t*)m_outdeg.p;
  B.out_ptr = (uint32_t*)m_optr.p;
  B.cursor = (uint32_t*)m_cur.p;
  B.out_idx = (uint32_t*)m_oidx.p;
  B.front[0] = (uint32_t*)m_f0.p;
  B.front[1] = (uint32_t*)m_f1.p;
  B.layer = (uint32_t*)m_layer.p;
  B.keys_out = (uint32_t*)m_keys.p;
  B.vals_in = (uint32_t*)m_vals.p;
  B.order = (uint32_t*)m_order.p;
  B.layer_ptr = (uint32_t*)m_lptr.p;
  B.sizes = (uint32_t*)m_sizes.p;
  B.scalars = (uint32_t*)m_scal.p;
  B.temp = m_temp.p;
  B.temp_bytes = temp;
  LvResult res{};
  hipError_t e = hipMemcpyAsync(m_ptr.p, g->op_src_ptr, n1 * w, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && ne)
    e = hipMemcpyAsync(m_src.p, g->op_src, (size_t)ne * w, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m_dst.p, g->op_dst, n * w, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = levelize_run(B, g->n_slots, n, ne, ctx->stream, &res);
  const bool in_range = res.bad[0] == kLvNone && res.bad[1] == kLvNone && res.bad[2] == kLvNone;
  if (e == hipSuccess && in_range && res.dup_slot == kLvNone)
    e = hipMemcpyAsync(op_layer, B.layer, n * w, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess && in_range && res.dup_slot == kLvNone && res.processed == n) {
    e = hipMemcpyAsync(order, B.order, n * w, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(layer_ptr, B.layer_ptr, ((size_t)res.n_layers + 1) * w,
                         hipMemcpyDeviceToHost, ctx->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  release();
  if (e != hipSuccess) {
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "levelization failed: %s", hipGetErrorString(e));
  }
  if (res.bad[0] != kLvNone)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "op_src_ptr decreases at operation %u", res.bad[0]);
  if (res.bad[1] != kLvNone)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "operand entry %u reads slot %u of %u", res.bad[1],
                g->op_src[res.bad[1]], g->n_slots);
  if (res.bad[2] != kLvNone)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "operation %u writes slot %u of %u", res.bad[2],
                g->op_dst[res.bad[2]], g->n_slots);
  if (res.dup_slot != kLvNone)
    return fail(ctx, RTEAAL_E_BAD_DESIGN, "slot %u is written by more than one operation",
                res.dup_slot);
  if (res.processed < n) {
    uint32_t o = 0;
    while (o < n && op_layer[o] != kLvNone) ++o;
    return fail(ctx, RTEAAL_E_BAD_DESIGN,
                "combinational cycle: operation %u lies on or behind a cycle (%u of %u operations "
                "levelized)", o, res.processed, n);
  }
  *n_layers = res.n_layers;
  return RTEAAL_OK;
}

rteaal_status rteaal_load_design(rteaal_ctx* ctx, const rteaal_design_desc* desc,
                                 rteaal_design_id* out) {
  return rteaal_load_design_ex(ctx, desc, 0, out);
}

rteaal_status rteaal_load_design_ex(rteaal_ctx* ctx, const rteaal_design_desc* desc,
                                    uint32_t flags, rteaal_design_id* out) {
  if (!ctx || !out) return fail(ctx, RTEAAL_E_INVALID_ARG, "null argument");
  if (flags & ~uint32_t(RTEAAL_LOAD_KEEP_ALL_SLOTS))
    return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown load flags %#x", flags);
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  Drivers drv;
  std::string why;
  auto h = std::make_unique<DesignHost>();
  rteaal_status st = validate(desc, &drv, &why, &h->fmt);
  if (st != RTEAAL_OK) return fail(ctx, st, "%s", why.c_str());
  encode(desc, drv, !(flags & RTEAAL_LOAD_KEEP_ALL_SLOTS), h.get());
  if (h->n_rows >= (1ull << 26))
    return fail(ctx, RTEAAL_E_UNSUPPORTED, "one instance's state (%llu bytes) exceeds 512 MiB",
                (unsigned long long)(h->n_rows * 8));
  const size_t ops_b = h->ops.size() * sizeof(DevOp), lay_b = h->layers.size() * sizeof(DevLayer);
  const size_t con_b = h->const_limbs.size() * 8, reg_b = std::max<size_t>(h->reg_refs.size(), 1) * sizeof(SlotRef);
  if (!alloc_all(ctx, {{&h->d_ops, ops_b}, {&h->d_layers, lay_b}, {&h->d_consts, con_b},
                       {&h->d_reg_refs, reg_b}}))
    return fail(ctx, RTEAAL_E_NO_MEMORY, "device allocation for the design failed");
  HIP_TRY(ctx, hipMemcpyAsync(h->d_ops.p, h->ops.data(), ops_b, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(h->d_layers.p, h->layers.data(), lay_b, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(h->d_consts.p, h->const_limbs.data(), con_b, hipMemcpyHostToDevice, ctx->stream));
  if (!h->reg_refs.empty())
    HIP_TRY(ctx, hipMemcpyAsync(h->d_reg_refs.p, h->reg_refs.data(), h->reg_refs.size() * sizeof(SlotRef),
                                hipMemcpyHostToDevice, ctx->stream));
  if (!h->compact && !h->slot_refs.empty()) {  // all-slot read-out needs the slot table
    if (!alloc_all(ctx, {{&h->d_slot_refs, h->slot_refs.size() * sizeof(SlotRef)}})) {
      (void)hipStreamSynchronize(ctx->stream);
      dev_free(ctx, h->d_ops);
      dev_free(ctx, h->d_layers);
      dev_free(ctx, h->d_consts);
      dev_free(ctx, h->d_reg_refs);
      return fail(ctx, RTEAAL_E_NO_MEMORY, "device allocation for the design failed");
    }
    HIP_TRY(ctx, hipMemcpyAsync(h->d_slot_refs.p, h->slot_refs.data(),
                                h->slot_refs.size() * sizeof(SlotRef), hipMemcpyHostToDevice,
                                ctx->stream));
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // host vectors stay alive; uploads done
  h->id = ctx->next_id++;
  *out = h->id;
  ctx->designs[h->id] = std::move(h);
  return RTEAAL_OK;
}

rteaal_status rteaal_unload_design(rteaal_ctx* ctx, rteaal_design_id id) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  DesignHost* h = find_design(ctx, id);
  if (!h) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown design %u", id);
  if (h->n_batches) return fail(ctx, RTEAAL_E_BUSY, "design %u still has %u batches", id, h->n_batches);
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, h->d_ops);
  dev_free(ctx, h->d_layers);
  dev_free(ctx, h->d_consts);
  dev_free(ctx, h->d_reg_refs);
  dev_free(ctx, h->d_slot_refs);
  ctx->designs.erase(id);
  return RTEAAL_OK;
}

rteaal_status rteaal_design_format(rteaal_ctx* ctx, rteaal_design_id id, uint32_t layer,
                                   rteaal_layer_format* out) {
  if (!ctx || !out) return fail(ctx, RTEAAL_E_INVALID_ARG, "null argument");
  DesignHost* h = find_design(ctx, id);
  if (!h) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown design %u", id);
  if (layer >= h->fmt.size()) return fail(ctx, RTEAAL_E_INVALID_ARG, "layer %u out of range", layer);
  *out = h->fmt[layer];
  return RTEAAL_OK;
}

rteaal_status rteaal_batch_footprint(rteaal_ctx* ctx, rteaal_design_id id, uint32_t n_inst,
                                     const rteaal_batch_opts* opts, uint64_t* bytes) {
  if (!ctx || !bytes || n_inst == 0) return fail(ctx, RTEAAL_E_INVALID_ARG, "bad argument");
  DesignHost* h = find_design(ctx, id);
  if (!h) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown design %u", id);
  if (opts && opts->mapping > RTEAAL_MAP_PARTITIONED)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown mapping %u", opts->mapping);
  opts = resolve_opts(ctx, id, n_inst, opts);
  const uint32_t m = choose_mapping(*h, n_inst, opts);
  uint64_t sb = 0;
  StateLayout L;
  if (!make_layout(*h, m, n_inst, layout_param(*h, m, n_inst, opts), &L, &sb))
    return fail(ctx, RTEAAL_E_INVALID_ARG, "too many instances for one SWEEP batch");
  const uint64_t pad = m == RTEAAL_MAP_SWEEP ? (uint64_t)L.n_tiles_alloc * 64 : n_inst;
  *bytes = sb + pad * 24 + 256 + 512;
  if (m == RTEAAL_MAP_PARTITIONED) {
    // exchange rows, digest sums, register refs, and the sub-programs (at
    // most the design's program per partition)
    const uint64_t P = part_count(*h, n_inst, opts);
    *bytes += 16ull * n_inst * std::max<uint32_t>(h->reg_words, 1) + 24ull * n_inst +
              16ull * h->n_regs + P * (h->ops.size() * sizeof(DevOp) + h->layers.size() * sizeof(DevLayer) +
                                       4ull * h->n_regs + sizeof(PartJob));
  }
  return RTEAAL_OK;
}

rteaal_status rteaal_batch_resources(rteaal_ctx* ctx, rteaal_design_id id, uint32_t n_inst,
                                     const rteaal_batch_opts* opts, uint64_t* hbm_bytes,
                                     uint64_t* lds_bytes) {
  if (!ctx || !hbm_bytes || !lds_bytes || n_inst == 0)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "bad argument");
  const rteaal_status st = rteaal_batch_footprint(ctx, id, n_inst, opts, hbm_bytes);
  if (st != RTEAAL_OK) return st;
  DesignHost* h = find_design(ctx, id);
  opts = resolve_opts(ctx, id, n_inst, opts);
  *lds_bytes = 0;
  const uint32_t m = choose_mapping(*h, n_inst, opts);
  if (m == RTEAAL_MAP_PARTITIONED) {
    const uint64_t copy = (h->n_rows * 8 + 15) & ~uint64_t(15);
    if (!(opts && opts->lds_state == 1) && copy <= ctx->max_lds)
      *lds_bytes = copy * part_count(*h, n_inst, opts) * n_inst;
    return RTEAAL_OK;
  }
  if (m != RTEAAL_MAP_RESIDENT) return RTEAAL_OK;
  StateLayout L;
  uint64_t sb = 0;
  make_layout(*h, RTEAAL_MAP_RESIDENT, n_inst, 1, &L, &sb);
  // The same choices rteaal_create_batch makes.
  const uint32_t n_ops = (uint32_t)h->ops.size(), n_lay = (uint32_t)h->layers.size();
  const bool lds = !(opts && opts->lds_state == 1) &&
                   resident_lds_bytes(L, n_ops, n_lay, true, false) <= ctx->max_lds;
  const bool lds_ops = !(opts && opts->lds_ops == 1) &&
                       resident_lds_bytes(L, n_ops, n_lay, lds, true) <= ctx->max_lds;
  *lds_bytes = (uint64_t)resident_lds_bytes(L, n_ops, n_lay, lds, lds_ops) * n_inst;
  return RTEAAL_OK;
}

rteaal_status rteaal_partition_plan_stats(rteaal_ctx* ctx, rteaal_design_id id, uint32_t partitions,
                                          rteaal_partition_stats* out) {
  if (!ctx || !out) return fail(ctx, RTEAAL_E_INVALID_ARG, "null argument");
  DesignHost* h = find_design(ctx, id);
  if (!h) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown design %u", id);
  if (partitions == 0 || partitions > 1024 || partitions > std::max<uint32_t>(h->n_regs, 1))
    return fail(ctx, RTEAAL_E_INVALID_ARG, "%u partitions for %u registers", partitions, h->n_regs);
  PartPlan pl;
  try {
    plan_partitions(*h, partitions, &pl, false);
  } catch (const std::bad_alloc&) {
    return fail(ctx, RTEAAL_E_NO_MEMORY, "host memory for the partition plan");
  }
  out->design_ops = h->ops.size();
  out->cone_ops = pl.cone_ops;
  out->padded_ops = pl.padded_ops;
  out->max_part_ops = pl.max_part_ops;
  out->exchange = pl.exchange;
  return RTEAAL_OK;
}

rteaal_status rteaal_create_batch(rteaal_ctx* ctx, rteaal_design_id id, uint32_t n_inst,
                                  const uint64_t* seeds, const rteaal_batch_opts* opts,
                                  rteaal_batch_id* out) {
  if (!ctx || !out || !seeds || n_inst == 0) return fail(ctx, RTEAAL_E_INVALID_ARG, "bad argument");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  DesignHost* h = find_design(ctx, id);
  if (!h) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown design %u", id);
  if (opts && opts->mapping > RTEAAL_MAP_PARTITIONED)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown mapping %u", opts->mapping);
  opts = resolve_opts(ctx, id, n_inst, opts);
  auto b = std::make_unique<Batch>();
  b->design = id;
  b->n_inst = n_inst;
  b->mapping = choose_mapping(*h, n_inst, opts);
  uint64_t sb = 0;
  PartPlan plan;
  if (b->mapping == RTEAAL_MAP_PARTITIONED) {
    const rteaal_status st = plan_batch_partitions(ctx, *h, n_inst, opts, b.get(), &plan);
    if (st != RTEAAL_OK) return st;
  }
  if (!make_layout(*h, b->mapping, n_inst, layout_param(*h, b->mapping, n_inst, opts), &b->L, &sb))
    return fail(ctx, RTEAAL_E_INVALID_ARG, "too many instances for one SWEEP batch");
  if (b->mapping == RTEAAL_MAP_PARTITIONED) {
    // (block, LDS and co-residency are settled by plan_batch_partitions)
  } else if (b->mapping == RTEAAL_MAP_RESIDENT) {
    uint32_t blk = opts && opts->block_threads ? opts->block_threads : 0;
    if (blk && (blk % 64 || blk > 1024))
      return fail(ctx, RTEAAL_E_INVALID_ARG, "block_threads must be a multiple of 64 up to 1024");
    if (!blk) {
      const uint32_t m = ((h->max_layer_ops + 63) / 64) * 64;
      blk = std::min<uint32_t>(1024, std::max<uint32_t>(64, m));
      if (blk > 256 && h->max_layer_ops < 2048) blk = 256;
    }
    b->block = blk;
    const uint32_t n_ops = (uint32_t)h->ops.size(), n_lay = (uint32_t)h->layers.size();
    b->lds = !(opts && opts->lds_state == 1) &&
             resident_lds_bytes(b->L, n_ops, n_lay, true, false) <= ctx->max_lds;
    b->lds_ops = !(opts && opts->lds_ops == 1) &&
                 resident_lds_bytes(b->L, n_ops, n_lay, b->lds, true) <= ctx->max_lds;
    const uint32_t u = opts && opts->unroll ? opts->unroll : (b->lds ? 1u : 4u);
    if (u != 1 && u != 2 && u != 4)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "RESIDENT unroll must be 1, 2 or 4");
    b->unroll = u;
  } else if (b->mapping == RTEAAL_MAP_LAYERED) {
    if (n_inst > 65535)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "LAYERED batches hold at most 65535 instances");
    const uint32_t u = opts && opts->unroll ? opts->unroll : 1u;
    if (u != 1 && u != 2 && u != 4)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "LAYERED unroll must be 1, 2 or 4");
    b->unroll = u;
    const uint32_t blk = opts && opts->block_threads ? opts->block_threads : 64u;
    if (blk % 64 || blk > 256)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "LAYERED block_threads must be 64, 128, 192 or 256");
    b->block = blk;
    if (opts && opts->persistent > 1)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "LAYERED persistent must be 0 or 1");
    b->persistent = opts && opts->persistent == 1;
    if (b->persistent && u == 4)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "persistent LAYERED unroll must be 1 or 2");
  } else {
    b->opw = opts && opts->ops_per_wave ? opts->ops_per_wave : 16;
    const uint32_t u = opts && opts->unroll ? opts->unroll : 2u;
    if (u != 1 && u != 2 && u != 4)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "SWEEP unroll must be 1, 2 or 4");
    b->unroll = u;
    const uint32_t tg = opts && opts->tiles_per_wave ? opts->tiles_per_wave : 1u;
    if (tg != 1 && tg != 2 && tg != 4 && tg != 8 && tg != 16)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "SWEEP tiles_per_wave must be 1, 2, 4, 8 or 16");
    if (tg * u > 8 && !(tg == 16 && u == 1))
      return fail(ctx, RTEAAL_E_INVALID_ARG,
                  "SWEEP unroll x tiles_per_wave must be at most 8 (16 tiles: unroll 1)");
    b->tg = tg;
    const uint32_t as = opts ? opts->arity_split : 0u;
    if (as > 2) return fail(ctx, RTEAAL_E_INVALID_ARG, "SWEEP arity_split must be 0, 1 or 2");
    b->arity_split = as;
    const uint32_t tpp = opts ? opts->tiles_per_pass : 0u;
    if (tpp % tg != 0)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "SWEEP tiles_per_pass must be a multiple of tiles_per_wave");
    b->tpp = tpp >= b->L.n_tiles_alloc ? 0u : tpp;
    const uint32_t pb = opts ? opts->pass_branches : 0u;
    if (pb > 1) return fail(ctx, RTEAAL_E_INVALID_ARG, "SWEEP pass_branches must be 0 or 1");
    if (pb && b->tpp && (b->L.n_tiles_alloc + b->tpp - 1) / b->tpp > 4)
      return fail(ctx, RTEAAL_E_INVALID_ARG,
                  "SWEEP pass_branches: at most 4 tile passes (tiles_per_pass %u of %u tiles)", b->tpp,
                  b->L.n_tiles_alloc);
    b->pbranch = pb == 1 && b->tpp != 0;
  }
  const uint64_t n_seed = b->mapping == RTEAAL_MAP_SWEEP ? (uint64_t)b->L.n_tiles_alloc * 64 : n_inst;
  b->n_slot = n_seed;
  const bool part = b->mapping == RTEAAL_MAP_PARTITIONED;
  const bool coop = b->persistent || part;
  if (!alloc_all(ctx, {{&b->state, sb}, {&b->seeds, n_seed * 8}, {&b->ctl, sizeof(DevCtl)},
                       {&b->dig, n_seed * 16}, {&b->gsync, coop ? sizeof(GridSync) : 0},
                       {&b->part_mem, part ? b->part_host.size() : 0},
                       {&b->xch, part ? 16ull * n_inst * std::max<uint32_t>(h->reg_words, 1) : 0},
                       {&b->pacc, part ? 24ull * n_inst : 0},
                       {&b->preg_refs, part ? std::max<size_t>(b->preg_host.size(), 1) * sizeof(SlotRef) : 0}}))
    return fail(ctx, RTEAAL_E_NO_MEMORY, "device allocation of %llu bytes for the batch failed",
                (unsigned long long)sb);
  if (part) finish_part_table(*b, plan);
  // The initial contents are copied from host buffers the batch keeps, so
  // the call only enqueues (a serving loop admits jobs while a step runs).
  b->seeds_host.assign(n_seed, 0);
  std::copy(seeds, seeds + n_inst, b->seeds_host.begin());
  b->ctl_host = DevCtl{};
  hipError_t e = hipMemsetAsync(b->state.p, 0, sb ? sb : 256, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(b->dig.p, 0, n_seed * 16, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->seeds.p, b->seeds_host.data(), n_seed * 8, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->ctl.p, &b->ctl_host, sizeof(DevCtl), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && part)
    e = hipMemcpyAsync(b->part_mem.p, b->part_host.data(), b->part_host.size(), hipMemcpyHostToDevice,
                       ctx->stream);
  if (e == hipSuccess && part && !b->preg_host.empty())
    e = hipMemcpyAsync(b->preg_refs.p, b->preg_host.data(), b->preg_host.size() * sizeof(SlotRef),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) {
    dev_free(ctx, b->state);
    dev_free(ctx, b->seeds);
    dev_free(ctx, b->ctl);
    dev_free(ctx, b->dig);
    dev_free(ctx, b->gsync);
    free_parts(ctx, *b);
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "batch initialisation failed: %s", hipGetErrorString(e));
  }
  b->id = ctx->next_id++;
  *out = b->id;
  h->n_batches++;
  ctx->batches[b->id] = std::move(b);
  return RTEAAL_OK;
}

rteaal_status rteaal_free_batch(rteaal_ctx* ctx, rteaal_batch_id id) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  (void)hipStreamSynchronize(ctx->stream);
  drop_multi_graphs_of(ctx, id);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  destroy_events(*b);
  free_watch(ctx, *b);
  dev_free(ctx, b->state);
  dev_free(ctx, b->seeds);
  dev_free(ctx, b->ctl);
  dev_free(ctx, b->dig);
  dev_free(ctx, b->gsync);
  free_parts(ctx, *b);
  DesignHost* h = find_design(ctx, b->design);
  if (h) h->n_batches--;
  ctx->batches.erase(id);
  return RTEAAL_OK;
}

rteaal_status rteaal_batch_info(rteaal_ctx* ctx, rteaal_batch_id id, uint32_t* mapping,
                                uint64_t* cycle) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  if (mapping) *mapping = b->mapping;
  if (cycle) *cycle = b->cycle;
  return RTEAAL_OK;
}

rteaal_status rteaal_batch_options(rteaal_ctx* ctx, rteaal_batch_id id, rteaal_batch_opts* out) {
  if (!ctx || !out) return fail(ctx, RTEAAL_E_INVALID_ARG, "null argument");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  rteaal_batch_opts o{};
  o.mapping = b->mapping;
  o.unroll = b->unroll;
  if (b->mapping == RTEAAL_MAP_RESIDENT) {
    o.block_threads = b->block;
    o.lds_state = b->lds ? 0u : 1u;
    o.lds_ops = b->lds_ops ? 0u : 1u;
  } else if (b->mapping == RTEAAL_MAP_LAYERED) {
    o.block_threads = b->block;
    o.persistent = b->persistent ? 1u : 0u;
  } else if (b->mapping == RTEAAL_MAP_PARTITIONED) {
    o.unroll = 0;
    o.block_threads = b->block;
    o.lds_state = b->lds ? 0u : 1u;
    o.partitions = b->parts;
  } else if (b->mapping == RTEAAL_MAP_SWEEP) {
    o.ops_per_wave = b->opw;
    o.tiles_per_wave = b->tg;
    o.arity_split = b->arity_split;
    o.tiles_per_pass = b->tpp;
    o.pass_branches = b->pbranch ? 1u : 0u;
  }
  *out = o;
  return RTEAAL_OK;
}

}  // extern "C"

namespace {

// Checks a step's stimulus for batch b over n_cycles.
rteaal_status check_stimulus(rteaal_ctx* ctx, const DesignHost& h, const rteaal_stimulus* stim,
                             uint64_t n_cycles) {
  if (stim && stim->mode > 1) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown stimulus mode %u", stim->mode);
  if (stim && stim->mode == 1 && !stim->words && h.words_per_inst && n_cycles)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "stimulus words are null");
  return RTEAAL_OK;
}

// Device address of a step's words stimulus (null for the generator): the
// caller's device buffer, or host words copied into *tmp on the context's
// stream (the caller frees *tmp once the step has completed).
rteaal_status stimulus_words(rteaal_ctx* ctx, const DesignHost& h, const Batch& b,
                             const rteaal_stimulus* stim, uint64_t n_cycles, Mem* tmp,
                             const uint64_t** words) {
  *words = nullptr;
  if (!stim || stim->mode != 1 || !h.words_per_inst || !n_cycles) return RTEAAL_OK;
  if (stim->words_on_device) {
    *words = stim->words;
    return RTEAAL_OK;
  }
  const size_t wb = (size_t)n_cycles * b.n_inst * h.words_per_inst * 8;
  if (!alloc_all(ctx, {{tmp, wb}})) return fail(ctx, RTEAAL_E_NO_MEMORY, "stimulus buffer allocation failed");
  hipError_t e = hipMemcpyAsync(tmp->p, stim->words, wb, hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) {
    dev_free(ctx, *tmp);
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "stimulus upload: %s", hipGetErrorString(e));
  }
  *words = (const uint64_t*)tmp->p;
  return RTEAAL_OK;
}

}  // namespace

extern "C" {

rteaal_status rteaal_step(rteaal_ctx* ctx, rteaal_batch_id id, uint64_t n_cycles,
                          const rteaal_stimulus* stim) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  DesignHost& h = *find_design(ctx, b->design);
  rteaal_status st0 = check_stimulus(ctx, h, stim, n_cycles);
  if (st0 != RTEAAL_OK) return st0;
  if (n_cycles == 0) return RTEAAL_OK;
  DevCtl* ctl = (DevCtl*)b->ctl.p;
  Mem tmp;
  const uint64_t* words = nullptr;
  st0 = stimulus_words(ctx, h, *b, stim, n_cycles, &tmp, &words);
  if (st0 != RTEAAL_OK) return st0;
  HIP_TRY(ctx, launch_set_words(ctl, words, ctx->stream));
  rteaal_status st = enqueue_cycles(ctx, h, *b, n_cycles);
  if (tmp.p) {
    (void)hipStreamSynchronize(ctx->stream);  // the host buffer copy must outlive the step
    dev_free(ctx, tmp);
  }
  if (st != RTEAAL_OK) return st;
  b->cycle += n_cycles;
  return RTEAAL_OK;
}

rteaal_status rteaal_step_many(rteaal_ctx* ctx, uint32_t n, const rteaal_batch_id* ids,
                               const uint64_t* n_cycles, const rteaal_stimulus* stims) {
  if (!ctx || (n && (!ids || !n_cycles))) return fail(ctx, RTEAAL_E_INVALID_ARG, "bad argument");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  std::vector<Batch*> bs(n);
  for (uint32_t k = 0; k < n; ++k) {
    bs[k] = find_batch(ctx, ids[k]);
    if (!bs[k]) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", ids[k]);
    for (uint32_t q = 0; q < k; ++q)
      if (ids[q] == ids[k]) return fail(ctx, RTEAAL_E_INVALID_ARG, "batch %u listed twice", ids[k]);
    const rteaal_status st = check_stimulus(ctx, *find_design(ctx, bs[k]->design),
                                            stims ? &stims[k] : nullptr, n_cycles[k]);
    if (st != RTEAAL_OK) return st;
  }
  // Host words are copied to device buffers that live until the step has
  // completed; auxiliary streams forked below are joined back into the
  // context stream on every exit path, so that nothing the step enqueued
  // outlives a later wait on the context stream.
  std::vector<Mem> tmps(n);
  uint32_t forked = 0;  // bit a: auxiliary stream a has forked in this call
  struct Finish {
    rteaal_ctx* ctx;
    std::vector<Mem>& tmps;
    uint32_t& forked;
    ~Finish() {
      for (int a = 0; a < rteaal_ctx::kAux; ++a) {
        if (!(forked >> a & 1u)) continue;
        if (hipEventRecord(ctx->join[a], ctx->aux[a]) != hipSuccess ||
            hipStreamWaitEvent(ctx->stream, ctx->join[a], 0) != hipSuccess)
          (void)hipStreamSynchronize(ctx->aux[a]);
      }
      bool any = false;
      for (Mem& m : tmps) any = any || m.p;
      if (any) {
        (void)hipStreamSynchronize(ctx->stream);
        for (Mem& m : tmps) dev_free(ctx, m);
      }
    }
  } finish{ctx, tmps, forked};
  for (uint32_t k = 0; k < n; ++k) {
    const uint64_t* words = nullptr;
    const rteaal_status st = stimulus_words(ctx, *find_design(ctx, bs[k]->design), *bs[k],
                                            stims ? &stims[k] : nullptr, n_cycles[k], &tmps[k], &words);
    if (st != RTEAAL_OK) return st;
    HIP_TRY(ctx, launch_set_words((DevCtl*)bs[k]->ctl.p, words, ctx->stream));
  }

  // SWEEP and LAYERED batches.  Those that are not watched, timed or run in
  // tile passes advance together through captured multi-batch cycles (one
  // graph per set of batches that still have cycles to go, so batches with
  // fewer cycles drop out in order), in one or more chains; the rest each
  // replay their own cycle graph.  All of them run on auxiliary streams
  // forked from the context stream, beside the RESIDENT launches (below).
  // Cooperative batches (persistent LAYERED, PARTITIONED) run at the end,
  // alone.
  std::vector<uint32_t> multi, single, coop;
  for (uint32_t k = 0; k < n; ++k) {
    const Batch& b = *bs[k];
    if (b.mapping == RTEAAL_MAP_RESIDENT || n_cycles[k] == 0) continue;
    if (b.persistent || b.mapping == RTEAAL_MAP_PARTITIONED) coop.push_back(k);
    else if (!b.n_watch && !b.profile && b.tpp == 0) multi.push_back(k);
    else single.push_back(k);
  }
  // Chains: the batches sorted by layer count and cut into contiguous groups
  // of about equal work (operations x instances), each stepped through its
  // own captured cycles on its own stream, so a group of shallow designs
  // does not wait at the layer indices of the deepest.
  std::vector<std::vector<uint32_t>> chain_ks;
  {
    const uint32_t C = std::min<uint32_t>(ctx->multi_chains, (uint32_t)(multi.size() / 2));
    if (C <= 1) {
      if (!multi.empty()) chain_ks.push_back(multi);
    } else {
      auto layers_of = [&](uint32_t k) { return find_design(ctx, bs[k]->design)->layers.size(); };
      auto work_of = [&](uint32_t k) {
        return (double)find_design(ctx, bs[k]->design)->ops.size() * bs[k]->n_inst;
      };
      std::vector<uint32_t> ord = multi;
      std::stable_sort(ord.begin(), ord.end(),
                       [&](uint32_t x, uint32_t y) { return layers_of(x) < layers_of(y); });
      double total = 0;
      for (uint32_t k : ord) total += work_of(k);
      double acc = 0;
      chain_ks.emplace_back();
      for (uint32_t k : ord) {
        if (acc >= total * chain_ks.size() / C && chain_ks.size() < C && chain_ks.back().size() >= 2)
          chain_ks.emplace_back();
        chain_ks.back().push_back(k);
        acc += work_of(k);
      }
      if (chain_ks.size() > 1 && chain_ks.back().size() < 2) {  // a lone last batch joins the one before
        const uint32_t k = chain_ks.back()[0];
        chain_ks.pop_back();
        chain_ks.back().push_back(k);
      }
    }
  }
  for (size_t c = 0; c < chain_ks.size();) {
    if (chain_ks[c].size() == 1) {
      single.push_back(chain_ks[c][0]);
      chain_ks.erase(chain_ks.begin() + c);
    } else {
      ++c;
    }
  }
  // Per chain: the replays (graph, cycles) of its phases and a batch left
  // alone for the last cycles (tail), after the replays.
  struct ChainPlan {
    std::vector<std::pair<MultiGraph*, uint64_t>> replays;
    int tail = -1;
    uint64_t tail_cycles = 0;
  };
  std::vector<ChainPlan> chains(chain_ks.size());
  {
    // The cache must hold every set of this call's phases; otherwise the
    // batches are stepped one by one (captured cycles are not evicted).
    auto phases = [&](const std::vector<uint32_t>& ks) {
      std::vector<uint64_t> counts;
      for (uint32_t k : ks) counts.push_back(n_cycles[k]);
      std::sort(counts.begin(), counts.end());
      counts.erase(std::unique(counts.begin(), counts.end()), counts.end());
      return counts;
    };
    size_t need = 0;
    for (const auto& ks : chain_ks)
      for (uint64_t c : phases(ks)) {
        std::vector<Batch*> set;
        for (uint32_t k : ks)
          if (n_cycles[k] >= c) set.push_back(bs[k]);
        if (set.size() >= 2 && !cached_multi_graph(ctx, set)) ++need;
      }
    if (ctx->mgraphs.size() + need > kMaxMultiGraphs) {
      for (const auto& ks : chain_ks) single.insert(single.end(), ks.begin(), ks.end());
      chain_ks.clear();
      chains.clear();
    }
    for (size_t ci = 0; ci < chain_ks.size(); ++ci) {
      const auto& ks = chain_ks[ci];
      ChainPlan& cp = chains[ci];
      uint64_t prev = 0;
      for (uint64_t c : phases(ks)) {
        std::vector<Batch*> set;
        int last = -1;
        for (uint32_t k : ks)
          if (n_cycles[k] >= c) {
            set.push_back(bs[k]);
            last = (int)k;
          }
        if (set.size() == 1) {
          cp.tail = last;
          cp.tail_cycles = n_cycles[last] - prev;
          break;
        }
        MultiGraph* g = nullptr;
        const rteaal_status st = multi_graph(ctx, set, &g);
        if (st != RTEAAL_OK) return st;
        cp.replays.push_back({g, c - prev});
        prev = c;
      }
    }
  }
  // Forks auxiliary stream a from the context stream's current position.
  auto fork_aux = [&](uint32_t a) -> rteaal_status {
    if (!ctx->aux[a]) {
      HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->aux[a], hipStreamNonBlocking));
      HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->join[a], hipEventDisableTiming));
    }
    if (!ctx->fork) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    if (!(forked >> a & 1u)) {
      HIP_TRY(ctx, hipEventRecord(ctx->fork, ctx->stream));
      HIP_TRY(ctx, hipStreamWaitEvent(ctx->aux[a], ctx->fork, 0));
      forked |= 1u << a;
    }
    return RTEAAL_OK;
  };
  // Streams: chain c on auxiliary stream c; batches stepped alone on the
  // streams after the chains (up to 3); RESIDENT configuration g >= 1 on
  // stream 4 + (g - 1) mod 4.
  const uint32_t n_chain_streams = (uint32_t)chains.size();
  auto single_stream = [&](size_t j) {
    const uint32_t first = std::min<uint32_t>(n_chain_streams, 3);
    return first + (uint32_t)(j % (4 - first));
  };
  // Runs batch k alone for c cycles on auxiliary stream a.
  auto run_alone = [&](uint32_t k, uint64_t c, uint32_t a) -> rteaal_status {
    Batch& b = *bs[k];
    hipStream_t keep = ctx->stream;
    ctx->stream = ctx->aux[a];
    const rteaal_status st = enqueue_cycles(ctx, *find_design(ctx, b.design), b, c);
    ctx->stream = keep;
    return st;
  };
  // RESIDENT batches: one persistent launch per kernel configuration, every
  // workgroup running one instance of one batch for that batch's cycles.
  // Watched RESIDENT batches run one cycle per launch (captured after each)
  // on the context stream instead.
  // A launch gives every workgroup the largest LDS of its jobs, so jobs are
  // also grouped by how many of their workgroups fit a compute unit's LDS
  // (1, 2, 4 or 8): small designs then share compute units instead of each
  // holding one as large designs do.
  struct Key {
    bool lds, ops;
    uint32_t unroll, block, per_cu;
    bool operator<(const Key& o) const {
      return std::tie(lds, ops, unroll, block, per_cu) <
             std::tie(o.lds, o.ops, o.unroll, o.block, o.per_cu);
    }
  };
  std::map<Key, std::vector<uint32_t>> group_map;
  std::vector<uint32_t> watched_res;
  for (uint32_t k = 0; k < n; ++k) {
    Batch& b = *bs[k];
    if (b.mapping != RTEAAL_MAP_RESIDENT || !n_cycles[k]) continue;
    if (b.n_watch) {
      watched_res.push_back(k);
      continue;
    }
    const DesignHost& h = *find_design(ctx, b.design);
    const size_t lb = resident_lds_bytes(b.L, (uint32_t)h.ops.size(), (uint32_t)h.layers.size(),
                                         b.lds, b.lds_ops);
    uint32_t per_cu = lb ? (uint32_t)std::min<size_t>(8, (160u * 1024u) / (lb + 256)) : 8u;
    per_cu = per_cu >= 8 ? 8 : per_cu >= 4 ? 4 : per_cu >= 2 ? 2 : 1;
    group_map[Key{b.lds, b.lds_ops, b.unroll, b.block, per_cu}].push_back(k);
  }
  std::vector<std::pair<Key, std::vector<uint32_t>>> groups(group_map.begin(), group_map.end());
  // Group g runs on the context stream (g = 0) or on auxiliary stream
  // 1 + (g - 1) mod 3, so that configurations run side by side.
  auto group_aux = [&](size_t g) { return (uint32_t)(4 + (g - 1) % 4); };
  auto group_stream = [&](size_t g) { return g == 0 ? ctx->stream : ctx->aux[group_aux(g)]; };

  // Every auxiliary stream this call uses forks here, before anything else
  // is enqueued, so that the captured cycles, the single batches and the
  // RESIDENT launches overlap.  The RESIDENT launches are enqueued first:
  // submitting many cycle replays can block the host until the device has
  // run most of them.
  {
    uint32_t want = 0;
    for (uint32_t c = 0; c < n_chain_streams; ++c) want |= 1u << c;
    for (size_t j = 0; j < single.size(); ++j) want |= 1u << single_stream(j);
    for (size_t g = 1; g < groups.size(); ++g) want |= 1u << group_aux(g);
    for (uint32_t a = 0; a < (uint32_t)rteaal_ctx::kAux; ++a)
      if (want >> a & 1u) {
        const rteaal_status st = fork_aux(a);
        if (st != RTEAAL_OK) return st;
      }
  }
  // Job tables: one region of the context's table buffer per group (its
  // first chunk is its largest), so that groups on different streams never
  // share one.  The buffer is reused only by later calls, which are ordered
  // after this one's launches (the call ends by joining its streams).
  std::vector<size_t> goff(groups.size() + 1, 0);
  for (size_t g = 0; g < groups.size(); ++g) {
    size_t need = groups[g].second.size() * sizeof(ResJob);
    for (uint32_t k : groups[g].second) need += (size_t)bs[k]->n_inst * sizeof(uint2);
    goff[g + 1] = goff[g] + ((need + 255) & ~size_t(255));
  }
  if (ctx->multi.bytes < goff.back()) {
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    dev_free(ctx, ctx->multi);
    if (!alloc_all(ctx, {{&ctx->multi, std::max<size_t>(goff.back(), 1u << 16) * 2}}))
      return fail(ctx, RTEAAL_E_NO_MEMORY, "job table allocation failed");
  }
  for (uint32_t k : watched_res) {
    Batch& b = *bs[k];
    rteaal_status st = enqueue_cycles(ctx, *find_design(ctx, b.design), b, n_cycles[k]);
    if (st != RTEAAL_OK) return st;
    b.cycle += n_cycles[k];
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    auto& g = groups[gi];
    hipStream_t gs = group_stream(gi);
    char* table = (char*)ctx->multi.p + goff[gi];
    std::vector<uint64_t> left(g.second.size());
    for (size_t q = 0; q < g.second.size(); ++q) left[q] = n_cycles[g.second[q]];
    for (;;) {
      std::vector<ResJob> jobs;
      std::vector<uint2> map;
      std::vector<std::pair<DevCtl*, uint64_t>> adv;
      size_t lds = 0;
      for (size_t q = 0; q < g.second.size(); ++q) {
        if (!left[q]) continue;
        Batch& b = *bs[g.second[q]];
        DesignHost& h = *find_design(ctx, b.design);
        const uint64_t c = std::min(kResidentChunk, left[q]);
        left[q] -= c;
        const uint32_t j = (uint32_t)jobs.size();
        jobs.push_back(res_job(h, b, c));
        for (uint32_t i = 0; i < b.n_inst; ++i) map.push_back(make_uint2(j, i));
        adv.push_back({(DevCtl*)b.ctl.p, c});
        lds = std::max(lds, resident_lds_bytes(b.L, (uint32_t)h.ops.size(), (uint32_t)h.layers.size(),
                                               b.lds, b.lds_ops));
      }
      if (jobs.empty()) break;
      const size_t need = jobs.size() * sizeof(ResJob) + map.size() * sizeof(uint2);
      std::vector<char> blob(need);
      memcpy(blob.data(), jobs.data(), jobs.size() * sizeof(ResJob));
      memcpy(blob.data() + jobs.size() * sizeof(ResJob), map.data(), map.size() * sizeof(uint2));
      // Staged from pageable memory; the group's next chunk reuses the
      // region after this launch on the same stream.
      HIP_TRY(ctx, hipMemcpyAsync(table, blob.data(), need, hipMemcpyHostToDevice, gs));
      const ResJob* dj = (const ResJob*)table;
      const uint2* dm = (const uint2*)(table + jobs.size() * sizeof(ResJob));
      HIP_TRY(ctx, launch_resident_multi(dj, dm, (uint32_t)map.size(), g.first.block, g.first.lds,
                                         g.first.ops, g.first.unroll, lds, gs));
      for (auto& a : adv) HIP_TRY(ctx, launch_advance(a.first, a.second, gs));
    }
    for (uint32_t k : g.second) bs[k]->cycle += n_cycles[k];
  }
  // The chains' replays, interleaved one cycle at a time across chains, so
  // that a host blocked by a full queue still feeds every chain.
  {
    std::vector<size_t> ri(chains.size(), 0);
    std::vector<uint64_t> done(chains.size(), 0);
    for (bool more = true; more;) {
      more = false;
      for (size_t c = 0; c < chains.size(); ++c) {
        ChainPlan& cp = chains[c];
        if (ri[c] >= cp.replays.size()) continue;
        HIP_TRY(ctx, hipGraphLaunch(cp.replays[ri[c]].first->exec, ctx->aux[c]));
        if (++done[c] == cp.replays[ri[c]].second) {
          ++ri[c];
          done[c] = 0;
        }
        more = more || ri[c] < cp.replays.size();
      }
    }
    for (size_t c = 0; c < chains.size(); ++c) {
      if (chains[c].tail >= 0) {
        const rteaal_status st = run_alone((uint32_t)chains[c].tail, chains[c].tail_cycles, (uint32_t)c);
        if (st != RTEAAL_OK) return st;
      }
      for (uint32_t k : chain_ks[c]) bs[k]->cycle += n_cycles[k];
    }
  }
  for (size_t j = 0; j < single.size(); ++j) {
    const uint32_t k = single[j];
    const rteaal_status st = run_alone(k, n_cycles[k], single_stream(j));
    if (st != RTEAAL_OK) return st;
    bs[k]->cycle += n_cycles[k];
  }
  // Cooperative batches last, on the context stream once everything above
  // (the auxiliary streams included) has finished: their workgroups spin at
  // grid barriers until all are resident, so they must not wait for
  // long-running workgroups of other launches to leave the device.
  if (!coop.empty()) {
    for (int a = 0; a < rteaal_ctx::kAux; ++a) {
      if (!(forked >> a & 1u)) continue;
      HIP_TRY(ctx, hipEventRecord(ctx->join[a], ctx->aux[a]));
      HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, ctx->join[a], 0));
    }
    forked = 0;
    for (uint32_t k : coop) {
      const rteaal_status st = enqueue_cycles(ctx, *find_design(ctx, bs[k]->design), *bs[k], n_cycles[k]);
      if (st != RTEAAL_OK) return st;
      bs[k]->cycle += n_cycles[k];
    }
  }
  return RTEAAL_OK;  // `finish` joins the auxiliary streams
}

rteaal_status rteaal_sync(rteaal_ctx* ctx) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& kv : ctx->batches) {
    const rteaal_status st = check_grid(ctx, *kv.second);
    if (st != RTEAAL_OK) return st;
  }
  return RTEAAL_OK;
}

}  // extern "C"

namespace {

// rteaal_read_state; stage: null (a buffer is allocated for the call) or a
// device buffer of stage_words words (rteaal_read_state_noalloc).
rteaal_status read_state(rteaal_ctx* ctx, rteaal_batch_id id, uint32_t first, uint32_t n,
                         uint32_t what, uint64_t* out, size_t out_words, size_t* written,
                         uint64_t* stage, size_t stage_words) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  if ((uint64_t)first + n > b->n_inst) return fail(ctx, RTEAAL_E_INVALID_ARG, "instance range out of bounds");
  if (what != RTEAAL_READ_REGS && what != RTEAAL_READ_ALL_SLOTS && what != RTEAAL_READ_DIGEST)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown read kind %u", what);
  DesignHost& h = *find_design(ctx, b->design);
  if (what == RTEAAL_READ_DIGEST) {
    if (written) *written = n;
    if (n == 0) return RTEAAL_OK;
    if (!out || out_words < n)
      return fail(ctx, RTEAAL_E_INVALID_ARG, "output holds %zu words, %u needed", out_words, n);
    hipError_t e = hipMemcpyAsync(out, (const uint64_t*)b->dig.p + first, (size_t)n * 8,
                                  hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      ctx->poisoned = true;
      return fail(ctx, RTEAAL_E_DEVICE, "read_state: %s", hipGetErrorString(e));
    }
    return check_grid(ctx, *b);
  }
  const bool slots = what == RTEAAL_READ_ALL_SLOTS;
  if (slots && b->mapping == RTEAAL_MAP_PARTITIONED)
    return fail(ctx, RTEAAL_E_UNSUPPORTED, "all-slot read-out of a PARTITIONED batch");
  if (slots && h.compact)
    return fail(ctx, RTEAAL_E_UNSUPPORTED,
                "all-slot read-out needs a design loaded with RTEAAL_LOAD_KEEP_ALL_SLOTS");
  const uint32_t wpi = slots ? h.slot_words : h.reg_words;
  const uint32_t n_refs = slots ? h.n_slots : h.n_regs;
  const size_t need = (size_t)wpi * n;
  if (written) *written = need;
  if (need == 0) return RTEAAL_OK;
  if (!out || out_words < need)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "output holds %zu words, %zu needed", out_words, need);
  if (stage && need > stage_words)
    return fail(ctx, RTEAAL_E_INVALID_ARG,
                "the read-out needs %zu words, more than the %zu of the no-allocation staging "
                "array; read fewer instances per call", need, stage_words);
  Mem tmp;
  if (!stage) {
    if (!alloc_all(ctx, {{&tmp, need * 8}}))
      return fail(ctx, RTEAAL_E_NO_MEMORY, "read-out buffer allocation failed");
    stage = (uint64_t*)tmp.p;
  }
  const SlotRef* refs = (const SlotRef*)(slots ? h.d_slot_refs.p
                                         : b->mapping == RTEAAL_MAP_PARTITIONED ? b->preg_refs.p
                                                                                : h.d_reg_refs.p);
  hipError_t e = launch_pack(b->mapping == RTEAAL_MAP_SWEEP, b->L, (const char*)b->state.p, refs,
                             n_refs, wpi, first, n, stage, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, stage, need * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dev_free(ctx, tmp);
  if (e != hipSuccess) {
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "read_state: %s", hipGetErrorString(e));
  }
  return check_grid(ctx, *b);
}

}  // namespace

extern "C" {

rteaal_status rteaal_read_state(rteaal_ctx* ctx, rteaal_batch_id id, uint32_t first, uint32_t n,
                                uint32_t what, uint64_t* out, size_t out_words, size_t* written) {
  return read_state(ctx, id, first, n, what, out, out_words, written, nullptr, 0);
}

rteaal_status rteaal_read_state_noalloc(rteaal_ctx* ctx, rteaal_batch_id id, uint32_t first,
                                        uint32_t n, uint32_t what, uint64_t* out,
                                        size_t out_words, size_t* written) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  return read_state(ctx, id, first, n, what, out, out_words, written, ctx->scratch, kNoAllocWords);
}

rteaal_status rteaal_write_state(rteaal_ctx* ctx, rteaal_batch_id id, uint32_t first, uint32_t n,
                                 const uint64_t* regs, uint64_t cycle) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  if ((uint64_t)first + n > b->n_inst) return fail(ctx, RTEAAL_E_INVALID_ARG, "instance range out of bounds");
  DesignHost& h = *find_design(ctx, b->design);
  const size_t need = (size_t)h.reg_words * n;
  if (need && !regs) return fail(ctx, RTEAAL_E_INVALID_ARG, "regs is null");
  Mem tmp;
  if (need && !alloc_all(ctx, {{&tmp, need * 8}})) return fail(ctx, RTEAAL_E_NO_MEMORY, "restore buffer allocation failed");
  hipError_t e = hipSuccess;
  if (need) {
    e = hipMemcpyAsync(tmp.p, regs, need * 8, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
      e = launch_unpack(b->mapping == RTEAAL_MAP_SWEEP, b->L, (char*)b->state.p,
                        (const SlotRef*)(b->mapping == RTEAAL_MAP_PARTITIONED ? b->preg_refs.p
                                                                              : h.d_reg_refs.p),
                        h.n_regs, h.reg_words, first, n,
                        (const uint64_t*)tmp.p, ctx->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(&((DevCtl*)b->ctl.p)->cycle, &cycle, 8, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dev_free(ctx, tmp);
  if (e != hipSuccess) {
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "write_state: %s", hipGetErrorString(e));
  }
  b->cycle = cycle;
  return RTEAAL_OK;
}

rteaal_status rteaal_write_digest(rteaal_ctx* ctx, rteaal_batch_id id, uint32_t first, uint32_t n,
                                  const uint64_t* digest) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  if ((uint64_t)first + n > b->n_inst) return fail(ctx, RTEAAL_E_INVALID_ARG, "instance range out of bounds");
  if (n && !digest) return fail(ctx, RTEAAL_E_INVALID_ARG, "digest is null");
  if (n == 0) return RTEAAL_OK;
  hipError_t e = hipMemcpyAsync((uint64_t*)b->dig.p + first, digest, (size_t)n * 8,
                                hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    ctx->poisoned = true;
    return fail(ctx, RTEAAL_E_DEVICE, "write_digest: %s", hipGetErrorString(e));
  }
  return RTEAAL_OK;
}

static_assert(sizeof(rteaal_change) == sizeof(ChangeRec), "rteaal_change layout");

rteaal_status rteaal_watch(rteaal_ctx* ctx, rteaal_batch_id id, const uint32_t* slots, uint32_t n,
                           uint64_t capacity) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  if (n && !slots) return fail(ctx, RTEAAL_E_INVALID_ARG, "null slots");
  if (n && b->mapping == RTEAAL_MAP_PARTITIONED)
    return fail(ctx, RTEAAL_E_UNSUPPORTED, "PARTITIONED batches cannot be watched");
  DesignHost& h = *find_design(ctx, b->design);
  std::vector<SlotRef> refs(n);
  uint32_t words = 0;
  for (uint32_t k = 0; k < n; ++k) {
    const uint32_t sl = slots[k];
    if (sl >= h.n_slots) return fail(ctx, RTEAAL_E_INVALID_ARG, "slot %u of %u", sl, h.n_slots);
    if (!h.kept[sl])
      return fail(ctx, RTEAAL_E_UNSUPPORTED,
                  "slot %u is not a register: watching it needs a design loaded with "
                  "RTEAAL_LOAD_KEEP_ALL_SLOTS", sl);
    refs[k] = h.slot_refs[sl];
    refs[k].out_off = words;
    words += (refs[k].width + 63) / 64;
  }
  if (capacity > (uint64_t(1) << 40) / sizeof(ChangeRec))
    return fail(ctx, RTEAAL_E_INVALID_ARG, "log capacity %llu is too large",
                (unsigned long long)capacity);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  // The captured cycle graph holds the old buffers: rebuild it.
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  free_watch(ctx, *b);
  if (n == 0) return RTEAAL_OK;
  if (!alloc_all(ctx, {{&b->watch_refs, n * sizeof(SlotRef)},
                       {&b->shadow, (size_t)b->n_inst * words * 8},
                       {&b->log, std::max<uint64_t>(capacity, 1) * sizeof(ChangeRec)},
                       {&b->log_count, 8}}))
    return fail(ctx, RTEAAL_E_NO_MEMORY, "change log of %llu records",
                (unsigned long long)capacity);
  b->n_watch = n;
  b->watch_words = words;
  b->log_cap = capacity;
  HIP_TRY(ctx, hipMemcpyAsync(b->watch_refs.p, refs.data(), n * sizeof(SlotRef),
                              hipMemcpyHostToDevice, ctx->stream));
  // The values at the call are the reference for the first cycle.
  HIP_TRY(ctx, launch_capture(b->mapping == RTEAAL_MAP_SWEEP, b->L, (const char*)b->state.p,
                              (const SlotRef*)b->watch_refs.p, n, (uint64_t*)b->shadow.p,
                              b->n_inst, true, (const DevCtl*)b->ctl.p, (ChangeRec*)b->log.p,
                              b->log_cap, (unsigned long long*)b->log_count.p, ctx->stream));
  HIP_TRY(ctx, launch_fill_u64((uint64_t*)b->log_count.p, 0, 1, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // refs staged from host memory
  return RTEAAL_OK;
}

rteaal_status rteaal_read_changes(rteaal_ctx* ctx, rteaal_batch_id id, rteaal_change* out,
                                  uint64_t max, uint64_t* n_out, uint64_t* n_dropped) {
  if (!ctx || !n_out || !n_dropped) return fail(ctx, RTEAAL_E_INVALID_ARG, "null argument");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  if (!b->n_watch) return fail(ctx, RTEAAL_E_INVALID_ARG, "batch %u is not watched", id);
  uint64_t total = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&total, b->log_count.p, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const uint64_t stored = std::min(total, b->log_cap);
  *n_out = stored;
  *n_dropped = total - stored;
  if (!out || max == 0) return RTEAAL_OK;
  if (max < stored)
    return fail(ctx, RTEAAL_E_INVALID_ARG, "the change log holds %llu records, room for %llu",
                (unsigned long long)stored, (unsigned long long)max);
  if (stored)
    HIP_TRY(ctx, hipMemcpyAsync(out, b->log.p, stored * sizeof(ChangeRec), hipMemcpyDeviceToHost,
                                ctx->stream));
  HIP_TRY(ctx, launch_fill_u64((uint64_t*)b->log_count.p, 0, 1, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return RTEAAL_OK;
}

}  // extern "C"

namespace {

// Tuner cache on disk (environment RTEAAL_TUNE_CACHE = file path): one line
// per tuning, "key rate n o[0] .. o[n-1]", each o ten numbers in the order of
// rteaal_batch_opts; the last line with a key wins.  The key names the
// device (architecture and compute units), the designs (fingerprints of
// their encoded programs) and the instance counts.
const char* tune_cache_path() {
  const char* p = std::getenv("RTEAAL_TUNE_CACHE");
  return p && *p ? p : nullptr;
}

std::string device_tag(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s/%dcu", prop.gcnArchName, prop.multiProcessorCount);
  std::string t = buf;
  for (char& c : t)
    if (c == ' ' || c == ':') c = '_';
  return t;
}

constexpr int kOptFields = 12;  // (entries name their field count in the key: "o12")

void opts_to(const rteaal_batch_opts& o, uint32_t* v) {
  const uint32_t a[kOptFields] = {o.mapping, o.block_threads, o.ops_per_wave, o.lds_state, o.lds_ops,
                                  o.unroll, o.tiles_per_wave, o.arity_split, o.tiles_per_pass,
                                  o.persistent, o.partitions, o.pass_branches};
  std::copy(a, a + kOptFields, v);
}

rteaal_batch_opts opts_from(const uint32_t* v) {
  rteaal_batch_opts o{};
  o.mapping = v[0];
  o.block_threads = v[1];
  o.ops_per_wave = v[2];
  o.lds_state = v[3];
  o.lds_ops = v[4];
  o.unroll = v[5];
  o.tiles_per_wave = v[6];
  o.arity_split = v[7];
  o.tiles_per_pass = v[8];
  o.persistent = v[9];
  o.partitions = v[10];
  o.pass_branches = v[11];
  return o;
}

bool cache_get(const std::string& key, std::vector<rteaal_batch_opts>* out, double* rate) {
  const char* path = tune_cache_path();
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  std::vector<char> line(1 << 20);
  while (std::fgets(line.data(), (int)line.size(), f)) {
    const char* q = line.data();
    const size_t kl = key.size();
    if (std::strncmp(q, key.c_str(), kl) != 0 || q[kl] != ' ') continue;
    q += kl;
    char* e = nullptr;
    const double r = std::strtod(q, &e);
    if (e == q) continue;
    q = e;
    const unsigned long n = std::strtoul(q, &e, 10);
    if (e == q || n == 0 || n > (1u << 16)) continue;
    q = e;
    std::vector<rteaal_batch_opts> v;
    bool ok = true;
    for (unsigned long k = 0; k < n && ok; ++k) {
      uint32_t a[kOptFields];
      for (int i = 0; i < kOptFields && ok; ++i) {
        a[i] = (uint32_t)std::strtoul(q, &e, 10);
        ok = e != q;
        q = e;
      }
      if (ok) v.push_back(opts_from(a));
    }
    if (!ok) continue;
    *out = v;
    *rate = r;
    found = true;
  }
  std::fclose(f);
  return found;
}

void cache_put(const std::string& key, const std::vector<rteaal_batch_opts>& v, double rate) {
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %.6g %zu", key.c_str(), rate, v.size());
  for (const auto& o : v) {
    uint32_t a[kOptFields];
    opts_to(o, a);
    for (int i = 0; i < kOptFields; ++i) std::fprintf(f, " %u", a[i]);
  }
  std::fprintf(f, "\n");
  std::fclose(f);
}

std::string single_key(rteaal_ctx* ctx, const DesignHost& h, uint32_t n_inst, uint64_t cycles) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "|%016llx|%u|%llu", (unsigned long long)h.fingerprint, n_inst,
                (unsigned long long)cycles);
  return "single|o12|" + device_tag(ctx->device) + buf;
}

}  // namespace

extern "C" {

rteaal_status rteaal_autotune(rteaal_ctx* ctx, rteaal_design_id id, uint32_t n_inst,
                              uint32_t trial_cycles, rteaal_batch_opts* best, double* rate) {
  if (!ctx || n_inst == 0) return fail(ctx, RTEAAL_E_INVALID_ARG, "bad argument");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  DesignHost* h = find_design(ctx, id);
  if (!h) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown design %u", id);
  // Trial length: about 2e9 op-evaluations per candidate, 1..64 cycles.
  uint64_t cyc = trial_cycles;
  if (!cyc) {
    const double per_cycle = (double)h->ops.size() * n_inst;
    cyc = (uint64_t)std::max(1.0, std::min(64.0, 2e9 / std::max(per_cycle, 1.0)));
  }
  const std::string key = single_key(ctx, *h, n_inst, cyc);
  {
    std::vector<rteaal_batch_opts> v;
    double r = 0;
    if (cache_get(key, &v, &r) && v.size() == 1) {
      ctx->tuned[{id, n_inst}] = v[0];
      if (best) *best = v[0];
      if (rate) *rate = r;
      return RTEAAL_OK;
    }
  }
  std::vector<rteaal_batch_opts> cand;
  const uint32_t m64 = ((h->max_layer_ops + 63) / 64) * 64;
  for (uint32_t blk : {128u, 256u, 512u, 1024u}) {
    if (blk > 2 * std::max<uint32_t>(m64, 128u)) continue;
    for (uint32_t u : {1u, 2u, 4u})
      cand.push_back(rteaal_batch_opts{RTEAAL_MAP_RESIDENT, blk, 0, 0, 0, u, 0});
  }
  if (n_inst <= 16) {
    for (uint32_t blk : {64u, 128u, 256u})
      for (uint32_t u : {1u, 2u})
        cand.push_back(rteaal_batch_opts{RTEAAL_MAP_LAYERED, blk, 0, 0, 0, u, 0});
    for (uint32_t u : {1u, 2u}) {
      rteaal_batch_opts o{RTEAAL_MAP_LAYERED, 0, 0, 0, 0, u, 0};
      o.persistent = 1;
      cand.push_back(o);
    }
  }
  // PARTITIONED: the default count and a few others that fit the device
  // (candidates that do not fit are skipped).
  if (n_inst <= 4 && h->n_regs >= 2)
    for (uint32_t pc : {0u, 64u, 128u, 512u / n_inst, 1024u / n_inst}) {
      if (pc > h->n_regs) continue;
      rteaal_batch_opts o{};
      o.mapping = RTEAAL_MAP_PARTITIONED;
      o.partitions = pc;
      cand.push_back(o);
    }
  const uint32_t n_tiles = (n_inst + 63) / 64;
  for (uint32_t tg : {1u, 2u, 4u, 8u, 16u}) {
    if (tg > 1 && tg > n_tiles) continue;
    for (uint32_t opw : {2u, 4u, 8u, 16u, 32u})
      for (uint32_t u : {1u, 2u, 4u})
        if (u * tg <= 8 || (tg == 16 && u == 1))
          cand.push_back(rteaal_batch_opts{RTEAAL_MAP_SWEEP, 0, opw, 0, 0, u, tg});
  }
  // Tile passes as parallel graph branches (2 or 4 passes), for a few of
  // the shapes that do well one pass at a time.
  if (n_tiles >= 4) {
    for (uint32_t np : {2u, 4u})
      for (uint32_t tg : {2u, 4u})
        for (uint32_t u : {1u, 2u}) {
          if (n_tiles % (np * tg) != 0) continue;
          rteaal_batch_opts o{RTEAAL_MAP_SWEEP, 0, 2, 0, 0, u, tg};
          o.tiles_per_pass = n_tiles / np;
          o.pass_branches = 1;
          cand.push_back(o);
        }
    for (uint32_t tg : {16u})          // two passes of the widest tile groups
      for (uint32_t opw : {2u, 8u}) {
        if (n_tiles % (2 * tg) != 0) continue;
        rteaal_batch_opts o{RTEAAL_MAP_SWEEP, 0, opw, 0, 0, 1, tg};
        o.tiles_per_pass = n_tiles / 2;
        o.pass_branches = 1;
        cand.push_back(o);
      }
  }
  std::vector<uint64_t> seeds(n_inst);
  for (uint32_t i = 0; i < n_inst; ++i) seeds[i] = i;
  const char* log_env = std::getenv("RTEAAL_AUTOTUNE_LOG");
  const bool log = log_env && *log_env && *log_env != '0';
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  double best_rate = -1.0;
  rteaal_batch_opts best_o{};
  rteaal_status st = RTEAAL_OK;
  std::string keep_err;
  for (const auto& o : cand) {
    rteaal_batch_id b = 0;
    st = rteaal_create_batch(ctx, id, n_inst, seeds.data(), &o, &b);
    if (st == RTEAAL_E_NO_MEMORY ||
        (st == RTEAAL_E_INVALID_ARG && o.mapping == RTEAAL_MAP_PARTITIONED)) {
      st = RTEAAL_OK;  // does not fit the device
      continue;
    }
    if (st != RTEAAL_OK) break;
    st = rteaal_step(ctx, b, 1, nullptr);  // warm-up (and graph capture)
    hipError_t e = hipSuccess;
    if (st == RTEAAL_OK) e = hipEventRecord(e0, ctx->stream);
    if (st == RTEAAL_OK && e == hipSuccess) st = rteaal_step(ctx, b, cyc, nullptr);
    if (st == RTEAAL_OK && e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (st == RTEAAL_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (st == RTEAAL_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    rteaal_free_batch(ctx, b);
    if (e != hipSuccess) {
      ctx->poisoned = true;
      st = fail(ctx, RTEAAL_E_DEVICE, "autotune timing: %s", hipGetErrorString(e));
    }
    if (st != RTEAAL_OK) break;
    const double r = (double)n_inst * (double)cyc / (std::max(ms, 1e-3f) * 1e-3);
    if (log)
      std::fprintf(stderr, "rteaal_autotune: mapping %u block %u ops/wave %u unroll %u tiles %u "
                   "persistent %u partitions %u passes of %u tiles%s -> %.4g\n", o.mapping,
                   o.block_threads, o.ops_per_wave, o.unroll, o.tiles_per_wave, o.persistent,
                   o.partitions, o.tiles_per_pass, o.pass_branches ? " in parallel" : "", r);
    if (r > best_rate) {
      best_rate = r;
      best_o = o;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != RTEAAL_OK) return st;
  if (best_rate < 0) return fail(ctx, RTEAAL_E_NO_MEMORY, "no candidate fits in device memory");
  ctx->tuned[{id, n_inst}] = best_o;
  cache_put(key, {best_o}, best_rate);
  if (best) *best = best_o;
  if (rate) *rate = best_rate;
  return RTEAAL_OK;
}

rteaal_status rteaal_autotune_many(rteaal_ctx* ctx, uint32_t n, const rteaal_design_id* ids,
                                   const uint32_t* n_inst, uint32_t trial_cycles,
                                   rteaal_batch_opts* best, double* rate) {
  if (!ctx || n == 0 || !ids || !n_inst) return fail(ctx, RTEAAL_E_INVALID_ARG, "bad argument");
  if (ctx->poisoned) return fail(ctx, RTEAAL_E_DEVICE, "context unusable after a device error");
  std::vector<DesignHost*> hs(n);
  uint64_t total = 0;
  for (uint32_t k = 0; k < n; ++k) {
    hs[k] = find_design(ctx, ids[k]);
    if (!hs[k]) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown design %u", ids[k]);
    if (n_inst[k] == 0) return fail(ctx, RTEAAL_E_INVALID_ARG, "instance count 0");
    for (uint32_t q = 0; q < k; ++q)
      if (ids[q] == ids[k] && n_inst[q] == n_inst[k])
        return fail(ctx, RTEAAL_E_INVALID_ARG, "design %u with %u instances listed twice", ids[k], n_inst[k]);
    total += (uint64_t)hs[k]->ops.size() * n_inst[k];
  }
  // Trial length: about 4e9 op-evaluations per policy, 2..32 cycles.
  const uint64_t cyc = trial_cycles ? trial_cycles
                                    : (uint64_t)std::max(2.0, std::min(32.0, 4e9 / std::max<double>((double)total, 1.0)));
  std::string key = "joint|o12s18|" + device_tag(ctx->device);
  {
    uint64_t fp = 1469598103934665603ull;
    for (uint32_t k = 0; k < n; ++k) {
      fp = fnv1a(&hs[k]->fingerprint, 8, fp);
      fp = fnv1a(&n_inst[k], 4, fp);
    }
    char buf[64];
    std::snprintf(buf, sizeof buf, "|%016llx|%u|%llu", (unsigned long long)fp, n,
                  (unsigned long long)cyc);
    key += buf;
  }
  std::vector<rteaal_batch_opts> chosen;
  double chosen_rate = 0;
  if (!cache_get(key, &chosen, &chosen_rate) || chosen.size() != n) {
    // Policies for the whole set: batches of at least `sweep_min` instances
    // run SWEEP (records shared by a wavefront's instances, tile groups up
    // to tg_cap tiles), smaller ones RESIDENT, or LAYERED when their design
    // is large (a layer over the whole device rather than one compute unit).
    // SWEEP batches take ops_per_wave operations per wavefront: fewer give
    // a captured cycle's small launches more, shorter wavefronts.  RESIDENT
    // batches take at most res_block threads per workgroup (0: the
    // design's default): smaller workgroups put more instances on a compute
    // unit, whose layer barriers then stall less of it.
    // Designs of at least sweep_ops operations run SWEEP whatever their
    // instance count: a RESIDENT instance of a large design keeps one
    // compute unit busy for the whole step.  With lds_only, RESIDENT is
    // kept only for designs whose state and program records both fit a
    // workgroup's LDS (the records then are read from HBM once per launch,
    // not once per instance and cycle); the others run SWEEP.
    // unroll: SWEEP batches' operations in flight per wavefront.
    struct Policy {
      uint32_t sweep_min, tg_cap, layered_ops, opw, res_block, sweep_ops, lds_only, unroll;
    };
    constexpr uint32_t kNever = UINT32_MAX;
    const Policy pol[] = {
        {16, 4, kNever, 8, 0, kNever, 0, 1},     {48, 4, 100000, 8, 0, kNever, 0, 1},
        {48, 2, kNever, 8, 0, kNever, 0, 1},     {48, 2, kNever, 2, 0, kNever, 0, 1},
        {48, 2, kNever, 4, 0, kNever, 0, 1},     {96, 2, kNever, 2, 0, kNever, 0, 1},
        {kNever, 1, kNever, 8, 0, kNever, 0, 1}, {48, 2, kNever, 4, 256, kNever, 0, 1},
        {48, 2, 100000, 4, 256, kNever, 0, 1},   {48, 2, kNever, 4, 256, kNever, 1, 1},
        {48, 2, kNever, 4, 0, kNever, 0, 2},     {48, 2, kNever, 8, 0, kNever, 0, 2},
        {48, 2, kNever, 8, 0, kNever, 0, 4},     {48, 2, kNever, 16, 0, kNever, 0, 4},
        {32, 2, kNever, 8, 0, kNever, 0, 2},     {96, 2, kNever, 8, 0, kNever, 0, 2},
        {48, 2, kNever, 8, 256, kNever, 0, 2},   {48, 2, kNever, 8, 0, kNever, 1, 2}};
    auto opts_of = [&](const Policy& p, uint32_t k) {
      rteaal_batch_opts o{};
      const uint32_t ni = n_inst[k];
      bool res_fits = true;
      if (p.lds_only) {
        StateLayout L;
        uint64_t sb = 0;
        make_layout(*hs[k], RTEAAL_MAP_RESIDENT, ni, 1, &L, &sb);
        res_fits = resident_lds_bytes(L, (uint32_t)hs[k]->ops.size(), (uint32_t)hs[k]->layers.size(),
                                      true, true) <= ctx->max_lds;
      }
      if (ni >= p.sweep_min || hs[k]->ops.size() >= p.sweep_ops || !res_fits) {
        const uint32_t tiles = (ni + 63) / 64;
        uint32_t tg = 1;
        while (tg * 2 <= std::min(tiles, p.tg_cap)) tg *= 2;
        o.mapping = RTEAAL_MAP_SWEEP;
        o.ops_per_wave = p.opw;
        o.unroll = p.unroll;
        o.tiles_per_wave = tg;
      } else if (hs[k]->ops.size() >= p.layered_ops && ni <= 65535) {
        o.mapping = RTEAAL_MAP_LAYERED;
        o.block_threads = 64;
        o.unroll = 1;
      } else {
        o.mapping = RTEAAL_MAP_RESIDENT;
        const uint32_t m = ((hs[k]->max_layer_ops + 63) / 64) * 64;
        if (p.res_block && m > p.res_block) o.block_threads = p.res_block;
      }
      return o;
    };
    const char* log_env = std::getenv("RTEAAL_AUTOTUNE_LOG");
    const bool log = log_env && *log_env && *log_env != '0';
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    double best_rate = -1;
    rteaal_status st = RTEAAL_OK;
    for (const Policy& p : pol) {
      std::vector<rteaal_batch_opts> os(n);
      std::vector<rteaal_batch_id> bs;
      bool fits = true;
      for (uint32_t k = 0; k < n && st == RTEAAL_OK; ++k) {
        os[k] = opts_of(p, k);
        std::vector<uint64_t> seeds(n_inst[k]);
        for (uint32_t i = 0; i < n_inst[k]; ++i) seeds[i] = i;
        rteaal_batch_id b = 0;
        st = rteaal_create_batch(ctx, ids[k], n_inst[k], seeds.data(), &os[k], &b);
        if (st == RTEAAL_E_NO_MEMORY) {
          st = RTEAAL_OK;
          fits = false;
          break;
        }
        if (st == RTEAAL_OK) bs.push_back(b);
      }
      double r = -1;
      if (st == RTEAAL_OK && fits) {
        std::vector<uint64_t> one(bs.size(), 1), many(bs.size(), cyc);
        st = rteaal_step_many(ctx, (uint32_t)bs.size(), bs.data(), one.data(), nullptr);  // warm-up, capture
        hipError_t e = hipSuccess;
        if (st == RTEAAL_OK) e = hipEventRecord(e0, ctx->stream);
        if (st == RTEAAL_OK && e == hipSuccess)
          st = rteaal_step_many(ctx, (uint32_t)bs.size(), bs.data(), many.data(), nullptr);
        if (st == RTEAAL_OK && e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (st == RTEAAL_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (st == RTEAAL_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          ctx->poisoned = true;
          st = fail(ctx, RTEAAL_E_DEVICE, "autotune timing: %s", hipGetErrorString(e));
        }
        uint64_t inst = 0;
        for (uint32_t k = 0; k < n; ++k) inst += n_inst[k];
        r = (double)inst * (double)cyc / (std::max(ms, 1e-3f) * 1e-3);
      }
      for (rteaal_batch_id b : bs) rteaal_free_batch(ctx, b);
      if (st != RTEAAL_OK) break;
      if (log)
        std::fprintf(stderr, "rteaal_autotune_many: sweep from %u instances or %u ops%s, tile "
                     "groups up to %u, %u ops per wavefront, unroll %u, LAYERED from %u ops, "
                     "RESIDENT blocks up to %u -> %.4g\n", p.sweep_min, p.sweep_ops,
                     p.lds_only ? " or records beyond LDS" : "", p.tg_cap, p.opw, p.unroll,
                     p.layered_ops, p.res_block, r);
      if (r > best_rate) {
        best_rate = r;
        chosen = os;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RTEAAL_OK) return st;
    if (best_rate < 0) return fail(ctx, RTEAAL_E_NO_MEMORY, "no policy fits in device memory");
    chosen_rate = best_rate;
    cache_put(key, chosen, chosen_rate);
  }
  for (uint32_t k = 0; k < n; ++k) {
    ctx->tuned[{ids[k], n_inst[k]}] = chosen[k];
    if (best) best[k] = chosen[k];
  }
  if (rate) *rate = chosen_rate;
  return RTEAAL_OK;
}

rteaal_status rteaal_kernel_timing(rteaal_ctx* ctx, rteaal_batch_id id, int enable,
                                   uint64_t* launches, double* total_ms) {
  if (!ctx) return fail(ctx, RTEAAL_E_INVALID_ARG, "null context");
  Batch* b = find_batch(ctx, id);
  if (!b) return fail(ctx, RTEAAL_E_INVALID_ARG, "unknown batch %u", id);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double total[2] = {0.0, 0.0};
  uint64_t count[2] = {0, 0};
  for (size_t i = 0; i < b->ev_used.size(); ++i) {
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, b->ev_used[i].first, b->ev_used[i].second));
    total[b->ev_kind[i]] += ms;
    ++count[b->ev_kind[i]];
  }
  for (int k = 0; k < 2; ++k) {
    if (launches) launches[k] = count[k];
    if (total_ms) total_ms[k] = total[k];
  }
  release_events(*b);
  b->profile = enable != 0;
  return RTEAAL_OK;
}

}  // extern "C"
