// HIP kernels for gfx950: evaluation of the per-cycle layer cascade.
//
// Two mappings of the same encoded program (internal.h):
//
//  * k_resident — one workgroup per instance, one lane per operation.  All
//    cycles of a step run inside one launch; layers are separated by a
//    workgroup barrier (the iterative rank I of Cascade 1).  The instance's
//    signal vector LI, and optionally the whole program, live in LDS when
//    they fit, else LI stays in HBM/L2.
//
//  * k_sweep / k_sweep_heavy — one lane per instance (64 instances per
//    wavefront, a wavefront covering one to eight such tiles), launched per
//    layer: k_sweep for the operations of at most 64 bits (per operand count
//    in large layers), k_sweep_heavy for the wider ones and the sources.  An
//    operation record is read once per wavefront with scalar loads (shared
//    by its instances), each operand gather is one coalesced row of 64
//    instance values per tile, and 1-bit signals are bit-sliced so that one
//    64-bit word holds the signal for a tile's 64 instances.
//
// Within a layer every operation reads only slots written by earlier layers
// (levelization), so the operations of a layer may run in any order, several
// of them may be in flight at once, and each layer output LO is stored
// straight into its LI slot (identity elision).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "ops_device.h"

namespace rteaal {

// Value of a STIM or CONST operation for one instance.
__device__ __forceinline__ V4 source_value(const uint64_t* const_limbs, const DevOp& op,
                                           uint64_t seed, uint64_t cycle, const uint64_t* words,
                                           uint64_t words_row, uint32_t w) {
  V4 v = v4_from(0);
  const uint32_t nl = (w + 63u) >> 6;
  if (op_opc(op.code) == OP_CONST) {
#pragma unroll
    for (uint32_t l = 0; l < 4; ++l)
      if (l < nl) v.l[l] = const_limbs[(uint64_t)op.aux0 * 4u + l];
  } else if (words) {
#pragma unroll
    for (uint32_t l = 0; l < 4; ++l)
      if (l < nl) v.l[l] = words[words_row + op.aux1 + l];
  } else {
#pragma unroll
    for (uint32_t l = 0; l < 4; ++l)
      if (l < nl) v.l[l] = stim_word(seed, cycle, op.aux0, l);
  }
  return v4_mask(v, w);
}

// ---------------------------------------------------------------------------
// RESIDENT: per-instance state block at `s` (LDS or global).
// ---------------------------------------------------------------------------

// Operand fetch without branches: one aligned 8-byte load per operand, the
// row named by the slot field, shifted down by the field's shift; only the
// final cut depends on the class.  Absent operands (arity < 3) carry field 0
// of class CB and read a valid word that is never used.
__device__ __forceinline__ uint64_t res_fetch(const char* s, uint32_t cls, uint32_t f) {
  const uint64_t v = *(const uint64_t*)(s + (uint64_t)(f >> 6) * 8u) >> (f & 63u);
  return cls == CB ? v & 1ull : cls == CW ? v & 0xffffffffull : v;
}

__device__ __forceinline__ V4 res_ldv(const char* s, uint32_t cls, uint32_t f) {
  const char* q = s + (uint64_t)(f >> 6) * 8u;
  if (cls == CB) return v4_from((*(const uint64_t*)q >> (f & 63u)) & 1ull);
  if (cls == CW) return v4_from(*(const uint32_t*)(q + ((f & 63u) >> 3)));
  const uint32_t k = cls_limbs(cls);
  V4 r = v4_from(*(const uint64_t*)q);
  if (k > 1) r.l[1] = *(const uint64_t*)(q + 8);
  if (k > 2) r.l[2] = *(const uint64_t*)(q + 16);
  if (k > 3) r.l[3] = *(const uint64_t*)(q + 24);
  return r;
}

__device__ __forceinline__ void res_st64(char* s, uint32_t cls, uint32_t f, uint64_t v) {
  char* q = s + (uint64_t)(f >> 6) * 8u;
  if (cls == CW) *(uint32_t*)(q + ((f & 63u) >> 3)) = (uint32_t)v;
  else *(uint64_t*)q = v;
}

__device__ __forceinline__ void res_stv(char* s, uint32_t cls, uint32_t f, const V4& v) {
  char* q = s + (uint64_t)(f >> 6) * 8u;
  if (cls == CW) {
    *(uint32_t*)(q + ((f & 63u) >> 3)) = (uint32_t)v.l[0];
    return;
  }
  const uint32_t k = cls_limbs(cls);
  *(uint64_t*)q = v.l[0];
  if (k > 1) *(uint64_t*)(q + 8) = v.l[1];
  if (k > 2) *(uint64_t*)(q + 16) = v.l[2];
  if (k > 3) *(uint64_t*)(q + 24) = v.l[3];
}

// One RESIDENT instance for n_cycles.
// LDS_STATE: the instance's signal vector is copied into LDS for the launch.
// LDS_OPS:   the whole program (operation and layer records) is copied into
//            LDS as well, so no global load remains in the cycle loop.
// U:         positions per thread handled together (records, then operands,
//            then evaluation), so U gathers are in flight per lane.
template <bool LDS_STATE, bool LDS_OPS, int U>
__device__ __forceinline__ void resident_run(const ResJob& J, uint32_t inst, uint4* lds_dyn) {
  const StateLayout& L = J.L;
  char* g = J.state + (uint64_t)inst * L.pitch;
  char* s = LDS_STATE ? (char*)lds_dyn : g;
  const uint64_t state_lds = LDS_STATE ? L.pitch : 0;
  const DevOp* ops = J.ops;
  const DevLayer* layers = J.layers;
  const uint32_t n_layers = J.n_layers;
  if (LDS_OPS) {
    uint4* o4 = (uint4*)((char*)lds_dyn + state_lds);
    const uint4* go = (const uint4*)J.ops;
    for (uint32_t i = threadIdx.x; i < J.n_ops_total * 2u; i += blockDim.x) o4[i] = go[i];
    uint4* l4 = o4 + J.n_ops_total * 2u;
    const uint4* gl = (const uint4*)J.layers;
    for (uint32_t i = threadIdx.x; i < n_layers * 2u; i += blockDim.x) l4[i] = gl[i];
    ops = (const DevOp*)o4;
    layers = (const DevLayer*)l4;
  }
  if (LDS_STATE)
    for (uint64_t i = threadIdx.x; i < L.pitch / 16u; i += blockDim.x)
      lds_dyn[i] = ((const uint4*)g)[i];
  if (LDS_STATE || LDS_OPS) __syncthreads();

  const uint64_t seed = J.seeds[inst];
  const uint64_t c0 = J.ctl->cycle, wc0 = J.ctl->step_cycle0;
  const uint64_t* words = J.ctl->words;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t bd = blockDim.x;

  for (uint64_t t = 0; t < J.n_cycles; ++t) {
    const uint64_t cycle = c0 + t;
    const uint64_t words_row =
        ((cycle - wc0) * (uint64_t)J.n_inst_total + inst) * (uint64_t)J.words_per_inst;
    for (uint32_t li = 0; li < n_layers; ++li) {
      const DevLayer ly = layers[li];
      const uint32_t n = ly.end - ly.begin;
      const uint32_t n64 = (n + 63u) & ~63u;
      for (uint32_t q0 = threadIdx.x; q0 < n64; q0 += U * bd) {
        DevOp op[U];
#pragma unroll
        for (int u = 0; u < U; ++u) op[u] = ops[ly.begin + min(q0 + u * bd, n - 1u)];
        uint64_t va[U], vb[U], vc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t q = q0 + u * bd, code = op[u].code, ar = op_arity(code);
          (void)q;
          (void)ar;
          va[u] = res_fetch(s, op_scls(code, 0), op[u].src[0]);
          vb[u] = res_fetch(s, op_scls(code, 1), op[u].src[1]);
          vc[u] = res_fetch(s, op_scls(code, 2), op[u].src[2]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t q = q0 + u * bd;
          if (q < n64) {  // the same for every lane of a wavefront
            uint64_t bit = 0;
            bool bdst = false;
            if (q < n) {
              const DevOp& o = op[u];
              const uint32_t code = o.code, opc = op_opc(code), ar = op_arity(code);
              const uint32_t dc = op_dcls(code), w = op_width(o.wimm), imm = op_imm(o.wimm);
              if (opc >= OP_STIM) {
                const V4 x = source_value(J.const_limbs, o, seed, cycle, words, words_row, w);
                if (dc == CB) {
                  bdst = true;
                  bit = x.l[0] & 1ull;
                } else {
                  res_stv(s, dc, o.dst, x);
                }
              } else if (op_kind(code) == K_U32 || op_kind(code) == K_BIT) {
                const uint32_t r = eval_u32(opc, ar, (uint32_t)va[u], (uint32_t)vb[u],
                                            (uint32_t)vc[u], imm, w);
                if (dc == CB) {
                  bdst = true;
                  bit = r & 1u;
                } else {
                  res_st64(s, dc, o.dst, r);
                }
              } else if (op_kind(code) != K_WIDE) {
                const uint64_t r = eval_u64(opc, ar, va[u], vb[u], vc[u], imm, w);
                if (dc == CB) {
                  bdst = true;
                  bit = r & 1ull;
                } else {
                  res_st64(s, dc, o.dst, r);
                }
              } else {
                const V4 a = res_ldv(s, op_scls(code, 0), o.src[0]);
                const V4 b = ar > 1 ? res_ldv(s, op_scls(code, 1), o.src[1]) : v4_from(0);
                const V4 c = ar > 2 ? res_ldv(s, op_scls(code, 2), o.src[2]) : v4_from(0);
                const V4 r = eval_wide(opc, ar, a, b, c, imm, w);
                if (dc == CB) {
                  bdst = true;
                  bit = r.l[0] & 1ull;
                } else {
                  res_stv(s, dc, o.dst, r);
                }
              }
            }
            // 1-bit outputs: the wavefront's 64 consecutive operations own one
            // row, named by the first one's destination field (1-bit
            // destinations lead the layer, so lane 0 holds one when any does).
            const uint64_t m = __ballot(bit != 0ull);
            const uint64_t any = __ballot(bdst);
            if (any != 0ull && lane == 0) *(uint64_t*)(s + (uint64_t)(op[u].dst >> 6) * 8u) = m;
          }
        }
      }
      __syncthreads();
    }
  }
  if (LDS_STATE) {
    for (uint64_t i = threadIdx.x; i < L.pitch / 16u; i += blockDim.x)
      ((uint4*)g)[i] = lds_dyn[i];
  }
}

// One batch: workgroup b runs instance inst_base + b.
template <bool LDS_STATE, bool LDS_OPS, int U>
__global__ void __launch_bounds__(1024) k_resident(ResJob J, uint32_t inst_base) {
  extern __shared__ uint4 lds_dyn[];
  resident_run<LDS_STATE, LDS_OPS, U>(J, inst_base + blockIdx.x, lds_dyn);
}

// Many batches (of possibly different designs and cycle counts) in one
// persistent launch: workgroup b runs instance map[b].y of job map[b].x.
template <bool LDS_STATE, bool LDS_OPS, int U>
__global__ void __launch_bounds__(1024)
k_resident_multi(const ResJob* __restrict__ jobs, const uint2* __restrict__ map) {
  extern __shared__ uint4 lds_dyn[];
  const uint2 m = map[blockIdx.x];
  const ResJob J = jobs[m.x];
  resident_run<LDS_STATE, LDS_OPS, U>(J, m.y, lds_dyn);
}

// ---------------------------------------------------------------------------
// SWEEP: lane = instance.  A wavefront owns TG consecutive tiles.
//  * 1-bit slots are slot-major: the TG words of slot i for the wavefront's
//    tiles are contiguous, so one scalar load brings them all in, and the
//    results of a 1-bit destination leave as one TG-lane store.
//  * Wide rows are tile-interleaved: the row address is found once per
//    operation (scalar arithmetic on the record's field) and the wavefront's
//    tiles sit at fixed 512-byte steps from it, so per tile only the load or
//    store immediate changes.
// ---------------------------------------------------------------------------
struct SweepView {
  char* base;          // state + 512 * (first tile): wide rows
  char* bits;          // state + 8 * (first tile): 1-bit words
  uint32_t row_bytes;  // bytes of one wide row over all allocated tiles
  uint32_t nta;        // allocated tiles (words per 1-bit slot)
  uint32_t lane;

  __device__ __forceinline__ SweepView(char* state, const StateLayout& L, uint32_t tile0,
                                       uint32_t ln)
      : base(state + (uint64_t)tile0 * 512u), bits(state + (uint64_t)tile0 * 8u),
        row_bytes(L.row_bytes), nta(L.n_tiles_alloc), lane(ln) {}

  // Start of the 64 lane values of wide slot f in the wavefront's first tile.
  __device__ __forceinline__ char* row(uint32_t f) const {
    return base + (uint64_t)(f >> 6) * row_bytes + ((f & 63u) << 3);
  }
  // Word of 1-bit slot i for the wavefront's first tile (the next TG-1 tiles
  // follow it).
  __device__ __forceinline__ uint64_t word_off(uint32_t i) const { return (uint64_t)i * nta * 8u; }
  // Operand gather without branches: one 8-byte load per tile from
  // base + this lane's offset + g * step.
  //   CB: base = the slot's word for the first tile, step 8, offset 0 (one
  //       word for the whole wavefront; the TG words are contiguous);
  //   CW: base = the row, step 512, offset = the aligned word holding this
  //       lane's value (lanes 2k and 2k+1 share it, so a row is read once);
  //   others: base = the row, step 512, offset = the lane's own value.
  __device__ __forceinline__ const char* gather_base(uint32_t cls, uint32_t f) const {
    return cls == CB ? bits + word_off(f) : (const char*)row(f);
  }
  __device__ __forceinline__ uint32_t ld_off(uint32_t cls) const {
    const uint32_t w = cls == CW ? 1u : 0u;
    const uint32_t mask = (cls == CB ? 0u : ~0u) & ~(w * 7u);
    return (lane << (3u - w)) & mask;
  }
  // The operand's value in this lane from its loaded word (CB: the
  // wavefront's bit-sliced word).
  __device__ __forceinline__ uint32_t lane_val32(uint32_t cls, uint64_t raw) const {
    const uint32_t lo = (uint32_t)raw, hi = (uint32_t)(raw >> 32);
    return cls == CB ? (uint32_t)((raw >> lane) & 1ull) : (lane & 1u) ? hi : lo;
  }
  __device__ __forceinline__ uint64_t lane_val(uint32_t cls, uint64_t raw) const {
    return cls == CB ? (raw >> lane) & 1ull
         : cls == CW ? (raw >> ((lane & 1u) * 32u)) & 0xffffffffull : raw;
  }
  // 1-bit results of the TG tiles (wave-uniform words): lane g stores tile g's
  // word, one contiguous store for the wavefront.  The word is picked with
  // masks rather than a select chain, which the compiler would turn into an
  // indexed (scratch) array.
  template <int TG>
  __device__ __forceinline__ void st_bits(uint32_t i, const uint64_t* m) const {
    uint64_t mine = 0;
#pragma unroll
    for (int g = 0; g < TG; ++g) mine |= m[g] & (0ull - (uint64_t)(lane == (uint32_t)g));
    if (lane < (uint32_t)TG) *(uint64_t*)(bits + word_off(i) + lane * 8u) = mine;
  }
  __device__ __forceinline__ void st32(char* r, uint32_t g, uint32_t x) const {
    *(uint32_t*)(r + g * 512u + lane * 4u) = x;
  }
  __device__ __forceinline__ void st64(uint32_t cls, char* r, uint32_t g, uint64_t x) const {
    if (cls == CW) st32(r, g, (uint32_t)x);
    else *(uint64_t*)(r + g * 512u + lane * 8u) = x;
  }
  __device__ __forceinline__ V4 ldv(uint32_t cls, uint32_t f, uint32_t g) const {
    if (cls == CB) return v4_from((*(const uint64_t*)(bits + word_off(f) + g * 8u) >> lane) & 1ull);
    const char* q = row(f) + g * 512u;
    if (cls == CW) return v4_from(*(const uint32_t*)(q + lane * 4u));
    q += lane * 8u;
    const uint32_t k = cls_limbs(cls);
    V4 x = v4_from(*(const uint64_t*)q);
    if (k > 1) x.l[1] = *(const uint64_t*)(q + row_bytes);
    if (k > 2) x.l[2] = *(const uint64_t*)(q + 2ull * row_bytes);
    if (k > 3) x.l[3] = *(const uint64_t*)(q + 3ull * row_bytes);
    return x;
  }
  __device__ __forceinline__ void stv(uint32_t cls, uint32_t f, uint32_t g, const V4& x) const {
    char* r = row(f);
    if (cls == CW) {
      st32(r, g, (uint32_t)x.l[0]);
      return;
    }
    char* q = r + g * 512u + lane * 8u;
    const uint32_t k = cls_limbs(cls);
    *(uint64_t*)q = x.l[0];
    if (k > 1) *(uint64_t*)(q + row_bytes) = x.l[1];
    if (k > 2) *(uint64_t*)(q + 2ull * row_bytes) = x.l[2];
    if (k > 3) *(uint64_t*)(q + 3ull * row_bytes) = x.l[3];
  }
};

// Common operations of one layer (every value at most 64 bits, no source)
// with NS operands, NS = 1, 2 or 3: the ranges [r.b0, r.e0) and [r.b1, r.e1);
// the first `split` chunks cover the first.  A kernel per operand count keeps
// absent operands from costing loads and registers.
// A wavefront handles a chunk of operations for TG tiles (64 instances each).
// Operations are processed U at a time: first the U records (scalar loads,
// decoded once for all TG tiles), then every operand for every tile (NS*U*TG
// gathers in flight per wavefront), then the evaluations and stores.  Tiles
// past the last instance (allocation padding up to a multiple of TG) are
// evaluated like the others and never read back.
template <int U, int TG, int NS>
__global__ void __launch_bounds__(256)
k_sweep(const DevOp* __restrict__ ops, StateLayout L, char* __restrict__ state, OpRanges r,
        uint32_t opw, uint32_t split, uint32_t tile_base, uint32_t n_groups) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const uint32_t grp = wave % n_groups, chunk = wave / n_groups;
  const bool first = chunk < split;
  const uint32_t o0 = first ? r.b0 + chunk * opw : r.b1 + (chunk - split) * opw;
  const uint32_t oe = first ? r.e0 : r.e1;
  if (o0 >= oe) return;
  const uint32_t o1 = min(o0 + opw, oe);
  const uint32_t tile0 = tile_base + grp * TG;
  const SweepView v(state, L, tile0, lane);

  for (uint32_t o = o0; o < o1; o += U) {
    DevOp op[U];
#pragma unroll
    for (int u = 0; u < U; ++u) op[u] = ops[min(o + (uint32_t)u, o1 - 1u)];
    uint64_t raw[U][3][TG];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t code = op[u].code;
#pragma unroll
      for (int k = NS; k < 3; ++k)
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[u][k][g] = 0;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const uint32_t cls = op_scls(code, k);
        const char* p = v.gather_base(cls, op[u].src[k]) + v.ld_off(cls);
        const uint32_t step = cls == CB ? 8u : 512u;
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[u][k][g] = *(const uint64_t*)(p + g * step);
      }
    }
    // Every gathered word counts as used on every path (unary operators,
    // absent operands ignore some of them), so that no load is still in
    // flight when the next group's loads reuse its registers: otherwise the
    // top of the loop would also wait for this group's stores.
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int g = 0; g < TG; ++g) asm volatile("" ::"v"(raw[u][k][g]));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (o + u < o1) {
        const DevOp& q = op[u];
        const uint32_t code = q.code, opc = op_opc(code), ar = op_arity(code), kind = op_kind(code);
        const uint32_t dc = op_dcls(code), w = op_width(q.wimm), imm = op_imm(q.wimm);
        const uint32_t c0 = op_scls(code, 0), c1 = op_scls(code, 1), c2 = op_scls(code, 2);
        if (kind == K_BIT) {
          uint64_t m[TG];
#pragma unroll
          for (int g = 0; g < TG; ++g)
            m[g] = eval_bits(opc, ar, raw[u][0][g], raw[u][1][g], raw[u][2][g], imm);
          v.st_bits<TG>(q.dst, m);
        } else if (kind == K_U32) {
          uint32_t a[TG], b[TG], c[TG], r[TG];
#pragma unroll
          for (int g = 0; g < TG; ++g) {
            a[g] = v.lane_val32(c0, raw[u][0][g]);
            b[g] = v.lane_val32(c1, raw[u][1][g]);
            c[g] = v.lane_val32(c2, raw[u][2][g]);
          }
          eval_u32_n<TG>(opc, ar, a, b, c, imm, w, r);
          if (dc == CB) {
            uint64_t m[TG];
#pragma unroll
            for (int g = 0; g < TG; ++g) m[g] = __ballot((r[g] & 1u) != 0u);
            v.st_bits<TG>(q.dst, m);
          } else {
            char* rd = v.row(q.dst);
#pragma unroll
            for (int g = 0; g < TG; ++g) v.st32(rd, g, r[g]);
          }
        } else {  // K_U64
          uint64_t r[TG];
#pragma unroll
          for (int g = 0; g < TG; ++g) {
            const uint64_t a = v.lane_val(c0, raw[u][0][g]);
            const uint64_t b = v.lane_val(c1, raw[u][1][g]);
            const uint64_t c = v.lane_val(c2, raw[u][2][g]);
            r[g] = eval_u64(opc, ar, a, b, c, imm, w);
          }
          if (dc == CB) {
            uint64_t m[TG];
#pragma unroll
            for (int g = 0; g < TG; ++g) m[g] = __ballot((r[g] & 1ull) != 0ull);
            v.st_bits<TG>(q.dst, m);
          } else {
            char* rd = v.row(q.dst);
#pragma unroll
            for (int g = 0; g < TG; ++g) v.st64(dc, rd, g, r[g]);
          }
        }
      }
    }
  }
}

// Heavy operations of one layer, [hbeg, hend): values wider than 64 bits
// (limb arithmetic on up to four 64-bit limbs) and the sources (stimulus
// words and literals).  One operation at a time per wavefront, for TG tiles.
template <int TG>
__global__ void __launch_bounds__(256)
k_sweep_heavy(const DevOp* __restrict__ ops, const DevLayer* __restrict__ layers,
              const uint64_t* __restrict__ const_limbs, uint32_t words_per_inst, StateLayout L,
              char* __restrict__ state, const uint64_t* __restrict__ seeds,
              const DevCtl* __restrict__ ctl, uint32_t n_inst, uint32_t layer, uint32_t opw,
              uint32_t tile_base, uint32_t n_groups) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const uint32_t grp = wave % n_groups, chunk = wave / n_groups;
  const DevLayer ly = layers[layer];
  const uint32_t o0 = ly.hbeg + chunk * opw;
  if (o0 >= ly.hend) return;
  const uint32_t o1 = min(o0 + opw, ly.hend);
  const uint32_t tile0 = tile_base + grp * TG;
  const SweepView v(state, L, tile0, lane);

  for (uint32_t o = o0; o < o1; ++o) {
    const DevOp q = ops[o];
    const uint32_t code = q.code, opc = op_opc(code), ar = op_arity(code);
    const uint32_t dc = op_dcls(code), w = op_width(q.wimm), imm = op_imm(q.wimm);
    uint64_t m[TG];
#pragma unroll
    for (int g = 0; g < TG; ++g) {
      V4 r;
      if (opc >= OP_STIM) {
        const uint32_t inst = (tile0 + g) * 64u + lane;
        const uint64_t cycle = ctl->cycle;
        const uint64_t words_row =
            ((cycle - ctl->step_cycle0) * (uint64_t)n_inst + inst) * (uint64_t)words_per_inst;
        r = v4_from(0);
        if (inst < n_inst)
          r = source_value(const_limbs, q, seeds[inst], cycle, ctl->words, words_row, w);
      } else {
        const V4 a = v.ldv(op_scls(code, 0), q.src[0], g);
        const V4 b = ar > 1 ? v.ldv(op_scls(code, 1), q.src[1], g) : v4_from(0);
        const V4 c = ar > 2 ? v.ldv(op_scls(code, 2), q.src[2], g) : v4_from(0);
        r = eval_wide(opc, ar, a, b, c, imm, w);
      }
      if (dc == CB) m[g] = __ballot((r.l[0] & 1ull) != 0ull);
      else v.stv(dc, q.dst, g, r);
    }
    if (dc == CB) v.st_bits<TG>(q.dst, m);
  }
}

// ---------------------------------------------------------------------------
// Control, read-out and restore.
// ---------------------------------------------------------------------------
__global__ void k_advance(DevCtl* ctl, uint64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->cycle += n;
}

__global__ void k_set_words(DevCtl* ctl, const uint64_t* words) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->words = words;
    ctl->step_cycle0 = ctl->cycle;
  }
}

// Address of limb `limb` of the stored value with slot field f of instance
// `inst` (for CB: the word holding its bit, with the bit position in *bitpos).
__device__ __forceinline__ char* elem_addr(bool sweep, const StateLayout& L, char* state,
                                           uint32_t cls, uint32_t f, uint32_t limb,
                                           uint32_t inst, uint32_t* bitpos) {
  const uint64_t row = (f >> 6) + limb;
  if (sweep) {
    const uint32_t t = inst >> 6, ln = inst & 63u;
    if (cls == CB) {
      *bitpos = ln;
      return state + ((uint64_t)f * L.n_tiles_alloc + t) * 8u;
    }
    return state + row * L.row_bytes + (uint64_t)t * 512u + ((f & 63u) << 3) +
           ln * (cls == CW ? 4u : 8u);
  }
  char* r = state + (uint64_t)inst * L.pitch + row * 8u;
  if (cls == CB) {
    *bitpos = f & 63u;
    return r;
  }
  return r + ((f & 63u) >> 3);
}

__global__ void k_pack(bool sweep, StateLayout L, const char* state, const SlotRef* refs,
                       uint32_t n_refs, uint32_t wpi, uint32_t first, uint32_t n, uint64_t* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint64_t)n_refs * n) return;
  const uint32_t r = (uint32_t)(i % n_refs), k = (uint32_t)(i / n_refs);
  const SlotRef ref = refs[r];
  const uint32_t inst = first + k;
  const uint32_t nl = (ref.width + 63u) >> 6;
  uint64_t* o = out + (uint64_t)k * wpi + ref.out_off;
  for (uint32_t l = 0; l < nl; ++l) {
    uint64_t x = 0;
    if (ref.cls != CNONE) {
      uint32_t bp = 0;
      const char* e = elem_addr(sweep, L, (char*)state, ref.cls, ref.pos, l, inst, &bp);
      if (ref.cls == CB) x = (*(const uint64_t*)e >> bp) & 1ull;
      else if (ref.cls == CW) x = *(const uint32_t*)e;
      else x = *(const uint64_t*)e;
    }
    o[l] = x;
  }
}

__global__ void k_unpack(bool sweep, StateLayout L, char* state, const SlotRef* refs,
                         uint32_t n_refs, uint32_t wpi, uint32_t first, uint32_t n,
                         const uint64_t* in) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint64_t)n_refs * n) return;
  const uint32_t r = (uint32_t)(i % n_refs), k = (uint32_t)(i / n_refs);
  const SlotRef ref = refs[r];
  if (ref.cls == CNONE) return;
  const uint32_t inst = first + k;
  const uint64_t* src = in + (uint64_t)k * wpi + ref.out_off;
  V4 v = v4_from(0);
  const uint32_t nl = (ref.width + 63u) >> 6;
#pragma unroll
  for (uint32_t l = 0; l < 4; ++l)
    if (l < nl) v.l[l] = src[l];
  v = v4_mask(v, ref.width);
  uint32_t bp = 0;
  if (ref.cls == CB) {
    unsigned long long* e =
        (unsigned long long*)elem_addr(sweep, L, state, CB, ref.pos, 0, inst, &bp);
    if (v.l[0] & 1ull) atomicOr(e, 1ull << bp);
    else atomicAnd(e, ~(1ull << bp));
  } else if (ref.cls == CW) {
    *(uint32_t*)elem_addr(sweep, L, state, CW, ref.pos, 0, inst, &bp) = (uint32_t)v.l[0];
  } else {
    const uint32_t k2 = cls_limbs(ref.cls);
#pragma unroll
    for (uint32_t l = 0; l < 4; ++l)
      if (l < k2) *(uint64_t*)elem_addr(sweep, L, state, ref.cls, ref.pos, l, inst, &bp) = v.l[l];
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
size_t resident_max_lds() { return 160u * 1024u; }

namespace {
template <class K>
hipError_t allow_lds(K kernel, size_t lds) {
  if (lds <= 64u * 1024u) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)resident_max_lds());
}

template <bool S, bool O, int U>
hipError_t launch_res_t(const ResJob& J, uint32_t n_inst, uint32_t inst_base, uint32_t block,
                        size_t lds, hipStream_t s) {
  hipError_t e = allow_lds(k_resident<S, O, U>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_resident<S, O, U>), dim3(n_inst), dim3(block), lds, s, J, inst_base);
  return hipGetLastError();
}

template <bool S, bool O, int U>
hipError_t launch_resm_t(const ResJob* jobs, const uint2* map, uint32_t n_blocks, uint32_t block,
                         size_t lds, hipStream_t s) {
  hipError_t e = allow_lds(k_resident_multi<S, O, U>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_resident_multi<S, O, U>), dim3(n_blocks), dim3(block), lds, s, jobs, map);
  return hipGetLastError();
}

// Dispatch on the run-time configuration to the kernel instantiation.
template <template <bool, bool, int> class F, class... A>
hipError_t dispatch_res(bool S, bool O, uint32_t U, A&&... a) {
  if (S && O) {
    if (U == 1) return F<true, true, 1>::go(a...);
    if (U == 2) return F<true, true, 2>::go(a...);
    return F<true, true, 4>::go(a...);
  }
  if (S) {
    if (U == 1) return F<true, false, 1>::go(a...);
    if (U == 2) return F<true, false, 2>::go(a...);
    return F<true, false, 4>::go(a...);
  }
  if (O) {
    if (U == 1) return F<false, true, 1>::go(a...);
    if (U == 2) return F<false, true, 2>::go(a...);
    return F<false, true, 4>::go(a...);
  }
  if (U == 1) return F<false, false, 1>::go(a...);
  if (U == 2) return F<false, false, 2>::go(a...);
  return F<false, false, 4>::go(a...);
}

template <bool S, bool O, int U>
struct ResOne {
  static hipError_t go(const ResJob& J, uint32_t n_inst, uint32_t inst_base, uint32_t block,
                       size_t lds, hipStream_t s) {
    return launch_res_t<S, O, U>(J, n_inst, inst_base, block, lds, s);
  }
};

template <bool S, bool O, int U>
struct ResMany {
  static hipError_t go(const ResJob* jobs, const uint2* map, uint32_t n_blocks, uint32_t block,
                       size_t lds, hipStream_t s) {
    return launch_resm_t<S, O, U>(jobs, map, n_blocks, block, lds, s);
  }
};
}  // namespace

size_t resident_lds_bytes(const StateLayout& L, uint32_t n_ops_total, uint32_t n_layers,
                          bool lds_state, bool lds_ops) {
  size_t b = lds_state ? L.pitch : 0;
  if (lds_ops) b += (size_t)n_ops_total * sizeof(DevOp) + (size_t)n_layers * sizeof(DevLayer);
  return b;
}

hipError_t launch_resident(const ResJob& J, uint32_t n_inst, uint32_t inst_base, uint32_t block,
                           bool lds_state, bool lds_ops, uint32_t unroll, hipStream_t s) {
  if (n_inst == 0 || J.n_cycles == 0) return hipSuccess;
  const size_t lds = resident_lds_bytes(J.L, J.n_ops_total, J.n_layers, lds_state, lds_ops);
  return dispatch_res<ResOne>(lds_state, lds_ops, unroll, J, n_inst, inst_base, block, lds, s);
}

hipError_t launch_resident_multi(const ResJob* jobs, const uint2* map, uint32_t n_blocks,
                                 uint32_t block, bool lds_state, bool lds_ops, uint32_t unroll,
                                 size_t lds, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  return dispatch_res<ResMany>(lds_state, lds_ops, unroll, jobs, map, n_blocks, block, lds, s);
}

// A tile pass must lie inside the allocated tiles and be whole tile groups.
static bool pass_ok(const StateLayout& L, TilePass tp, uint32_t tg) {
  return tp.count > 0 && tp.count % tg == 0 && tp.base % tg == 0 &&
         (uint64_t)tp.base + tp.count <= L.n_tiles_alloc;
}

hipError_t launch_sweep_light(const Program& p, const StateLayout& L, char* state,
                              const OpRanges& r, uint32_t n_src, uint32_t ops_per_wave,
                              uint32_t unroll, uint32_t tiles_per_wave, TilePass tp,
                              hipStream_t s) {
  const uint32_t n1 = r.e0 - r.b0, n2 = r.e1 - r.b1;
  if (n1 + n2 == 0) return hipSuccess;
  const uint32_t tg = tiles_per_wave == 8 ? 8u : tiles_per_wave == 4 ? 4u
                    : tiles_per_wave == 2 ? 2u : 1u;
  if (ops_per_wave == 0 || n_src < 1 || n_src > 3 || !pass_ok(L, tp, tg))
    return hipErrorInvalidValue;
  const uint32_t split = (n1 + ops_per_wave - 1) / ops_per_wave;
  const uint64_t chunks = split + (n2 + ops_per_wave - 1) / ops_per_wave;
  const uint32_t n_groups = tp.count / tg;
  const uint64_t waves = chunks * n_groups;
  const dim3 grid((uint32_t)((waves + 3) / 4)), blk(256);
#define RTEAAL_SWEEP(UU, GG, NN)                                                          \
  hipLaunchKernelGGL((k_sweep<UU, GG, NN>), grid, blk, 0, s, p.ops, L, state, r, ops_per_wave, \
                     split, tp.base, n_groups)
#define RTEAAL_SWEEP_N(UU, GG)          \
  if (n_src == 1) RTEAAL_SWEEP(UU, GG, 1); \
  else if (n_src == 2) RTEAAL_SWEEP(UU, GG, 2); \
  else RTEAAL_SWEEP(UU, GG, 3);
  // unroll x tiles_per_wave is at most 8: larger products run out of
  // registers and spill to scratch.
  switch (tg * 8 + unroll) {
    case 8 + 1: RTEAAL_SWEEP_N(1, 1) break;
    case 8 + 4: RTEAAL_SWEEP_N(4, 1) break;
    case 16 + 1: RTEAAL_SWEEP_N(1, 2) break;
    case 16 + 2: RTEAAL_SWEEP_N(2, 2) break;
    case 16 + 4: RTEAAL_SWEEP_N(4, 2) break;
    case 32 + 1: RTEAAL_SWEEP_N(1, 4) break;
    case 32 + 2: RTEAAL_SWEEP_N(2, 4) break;
    case 64 + 1: RTEAAL_SWEEP_N(1, 8) break;
    default: RTEAAL_SWEEP_N(2, 1) break;
  }
#undef RTEAAL_SWEEP_N
#undef RTEAAL_SWEEP
  return hipGetLastError();
}

hipError_t launch_sweep_heavy(const Program& p, const StateLayout& L, char* state,
                              const uint64_t* seeds, const DevCtl* ctl, uint32_t n_inst,
                              uint32_t layer, const DevLayer& ly, uint32_t ops_per_wave,
                              uint32_t tiles_per_wave, TilePass tp, hipStream_t s) {
  const uint32_t n = ly.hend - ly.hbeg;
  if (n == 0) return hipSuccess;
  const uint32_t tg = tiles_per_wave >= 4 ? 4u : tiles_per_wave == 2 ? 2u : 1u;
  if (ops_per_wave == 0 || !pass_ok(L, tp, tg)) return hipErrorInvalidValue;
  const uint64_t chunks = (n + ops_per_wave - 1) / ops_per_wave;
  const uint32_t n_groups = tp.count / tg;
  const uint64_t waves = chunks * n_groups;
  const dim3 grid((uint32_t)((waves + 3) / 4)), blk(256);
#define RTEAAL_HEAVY(GG)                                                                     \
  hipLaunchKernelGGL((k_sweep_heavy<GG>), grid, blk, 0, s, p.ops, p.layers, p.const_limbs,   \
                     p.words_per_inst, L, state, seeds, ctl, n_inst, layer, ops_per_wave,    \
                     tp.base, n_groups)
  if (tg == 4) RTEAAL_HEAVY(4);
  else if (tg == 2) RTEAAL_HEAVY(2);
  else RTEAAL_HEAVY(1);
#undef RTEAAL_HEAVY
  return hipGetLastError();
}

hipError_t launch_advance(DevCtl* ctl, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctl, n);
  return hipGetLastError();
}

hipError_t launch_set_words(DevCtl* ctl, const uint64_t* words, hipStream_t s) {
  hipLaunchKernelGGL(k_set_words, dim3(1), dim3(64), 0, s, ctl, words);
  return hipGetLastError();
}

hipError_t launch_pack(bool sweep, const StateLayout& L, const char* state, const SlotRef* refs,
                       uint32_t n_refs, uint32_t wpi, uint32_t first, uint32_t n, uint64_t* out,
                       hipStream_t s) {
  const uint64_t total = (uint64_t)n_refs * n;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, sweep, L,
                     state, refs, n_refs, wpi, first, n, out);
  return hipGetLastError();
}

hipError_t launch_unpack(bool sweep, const StateLayout& L, char* state, const SlotRef* refs,
                         uint32_t n_refs, uint32_t wpi, uint32_t first, uint32_t n,
                         const uint64_t* in, hipStream_t s) {
  const uint64_t total = (uint64_t)n_refs * n;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, sweep, L,
                     state, refs, n_refs, wpi, first, n, in);
  return hipGetLastError();
}

}  // namespace rteaal
