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

#include <algorithm>

#include "internal.h"
#include "ops_device.h"

namespace rteaal {

// Value of a STIM or CONST operation for one instance (w <= 64 NL).
template <int NL = 4>
__device__ __forceinline__ VN<NL> source_value(const uint64_t* const_limbs, const DevOp& op,
                                               uint64_t seed, uint64_t cycle, const uint64_t* words,
                                               uint64_t words_row, uint32_t w) {
  VN<NL> v = v4_from<NL>(0);
  const uint32_t nl = (w + 63u) >> 6;
  if (op_opc(op.code) == OP_CONST) {
#pragma unroll
    for (uint32_t l = 0; l < (uint32_t)NL; ++l)
      if (l < nl) v.l[l] = const_limbs[(uint64_t)op.aux0 * 4u + l];
  } else if (words) {
#pragma unroll
    for (uint32_t l = 0; l < (uint32_t)NL; ++l)
      if (l < nl) v.l[l] = words[words_row + op.aux1 + l];
  } else {
#pragma unroll
    for (uint32_t l = 0; l < (uint32_t)NL; ++l)
      if (l < nl) v.l[l] = stim_word(seed, cycle, op.aux0, l);
  }
  return v4_mask(v, w);
}

// ---------------------------------------------------------------------------
// RESIDENT: per-instance state block at `s` (LDS or global).
// ---------------------------------------------------------------------------

// Low-bit mask of a value of class c (all 64 bits for CD and for limbs):
// ~0 shifted right by 64 - element bits, taken from a byte table
// (63, 56, 48, 32 for CB, C8, C16, CW; 0 for the rest).
__device__ __forceinline__ uint64_t cls_mask64(uint32_t c) {
  return ~0ull >> ((0x2030383Full >> (c << 3)) & 63u);
}

// Operand fetch without branches: one aligned 8-byte load per operand, the
// row named by the slot field, shifted down by the field's shift; only the
// final cut depends on the class.  Absent operands (arity < 3) carry field 0
// of class CB and read a valid word that is never used.
__device__ __forceinline__ uint64_t res_fetch(const char* s, uint32_t cls, uint32_t f) {
  const uint64_t v = *(const uint64_t*)(s + (uint64_t)(f >> 6) * 8u) >> (f & 63u);
  return v & cls_mask64(cls);
}

// A value of class cls (at most NL limbs) at slot field f.
template <int NL = 4>
__device__ __forceinline__ VN<NL> res_ldv(const char* s, uint32_t cls, uint32_t f) {
  if (cls <= CW) return v4_from<NL>(res_fetch(s, cls, f));
  const char* q = s + (uint64_t)(f >> 6) * 8u;
  const uint32_t k = cls_limbs(cls);
  VN<NL> r = v4_from<NL>(*(const uint64_t*)q);
#pragma unroll
  for (int l = 1; l < NL; ++l)
    if ((uint32_t)l < k) r.l[l] = *(const uint64_t*)(q + 8 * l);
  return r;
}

// Store of a value of class C8..CD at its byte offset in the row (values of
// these classes never straddle a row).
__device__ __forceinline__ void res_st64(char* s, uint32_t cls, uint32_t f, uint64_t v) {
  char* q = s + (uint64_t)(f >> 6) * 8u + ((f & 63u) >> 3);
  if (cls == C8) *(uint8_t*)q = (uint8_t)v;
  else if (cls == C16) *(uint16_t*)q = (uint16_t)v;
  else if (cls == CW) *(uint32_t*)q = (uint32_t)v;
  else *(uint64_t*)q = v;
}

template <int NL>
__device__ __forceinline__ void res_stv(char* s, uint32_t cls, uint32_t f, const VN<NL>& v) {
  if (cls <= CD) {
    res_st64(s, cls, f, v.l[0]);
    return;
  }
  char* q = s + (uint64_t)(f >> 6) * 8u;
  const uint32_t k = cls_limbs(cls);
  *(uint64_t*)q = v.l[0];
#pragma unroll
  for (int l = 1; l < NL; ++l)
    if ((uint32_t)l < k) *(uint64_t*)(q + 8 * l) = v.l[l];
}

// One RESIDENT instance for n_cycles.
// LDS_STATE: the instance's signal vector is copied into LDS for the launch.
// LDS_OPS:   the whole program (operation and layer records) is copied into
//            LDS as well, so no global load remains in the cycle loop.
// U:         positions per thread handled together (records, then operands,
//            then evaluation), so U gathers are in flight per lane.
// The operations at positions q0 + u * stride (u < U) of layer ly for one
// instance whose state rows are at s: U records, then their operands, then
// evaluation and stores.  A position past the layer holds no operation; the
// positions of a wavefront are 64 consecutive ones, so 1-bit results leave
// as one ballot word per wavefront.
template <int U>
__device__ __forceinline__ void resident_ops(const uint64_t* const_limbs, char* s, const DevOp* ops,
                                             const DevLayer& ly, uint32_t q0, uint32_t stride,
                                             uint32_t n, uint32_t n64, uint64_t seed,
                                             uint64_t cycle, const uint64_t* words,
                                             uint64_t words_row, uint32_t lane) {
  DevOp op[U];
#pragma unroll
  for (int u = 0; u < U; ++u) op[u] = ops[ly.begin + min(q0 + u * stride, n - 1u)];
  uint64_t va[U], vb[U], vc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t q = q0 + u * stride, code = op[u].code, ar = op_arity(code);
    (void)q;
    (void)ar;
    va[u] = res_fetch(s, op_scls(code, 0), op[u].src[0]);
    vb[u] = res_fetch(s, op_scls(code, 1), op[u].src[1]);
    vc[u] = res_fetch(s, op_scls(code, 2), op[u].src[2]);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t q = q0 + u * stride;
    if (q < n64) {  // the same for every lane of a wavefront
      uint64_t bit = 0;
      bool bdst = false;
      if (q < n) {
        const DevOp& o = op[u];
        const uint32_t code = o.code, opc = op_opc(code), ar = op_arity(code);
        const uint32_t dc = op_dcls(code), w = op_width(o.wimm), imm = op_imm(o.wimm);
        if (opc >= OP_STIM) {
          const V4 x = source_value(const_limbs, o, seed, cycle, words, words_row, w);
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
          V4 c = ar > 2 ? res_ldv(s, op_scls(code, 2), o.src[2]) : v4_from(0);
          if (opc == OP_MUXC)  // further pairs, innermost first, onto the default
            for (uint32_t i = o.aux1; i-- > 0;) {
              const uint64_t es = const_limbs[o.aux0 + 2u * i];
              const uint64_t ev = const_limbs[o.aux0 + 2u * i + 1u];
              const V4 sv = res_ldv(s, (uint32_t)(es >> 32), (uint32_t)es);
              const V4 vv = res_ldv(s, (uint32_t)(ev >> 32), (uint32_t)ev);
              if (v4_nonzero(sv)) c = vv;
            }
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

// Sum of a 64-bit value over the 64 lanes of a wavefront.
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// Digest terms of register j (stored value ref r) of a RESIDENT state block
// s: the sum over its limbs l of s(s(4 j + l) ^ limb), s = SplitMix64's
// output function.
__device__ __forceinline__ uint64_t res_reg_terms(const char* s, const SlotRef& r, uint32_t j) {
  if (r.cls <= CD) return splitmix64(splitmix64((uint64_t)j << 2) ^ res_fetch(s, r.cls, r.pos));
  const uint64_t* q = (const uint64_t*)(s + (uint64_t)(r.pos >> 6) * 8u);
  const uint32_t nl = (r.width + 63u) >> 6;
  uint64_t h = 0;
  for (uint32_t l = 0; l < nl; ++l) h += splitmix64(splitmix64(((uint64_t)j << 2) | l) ^ q[l]);
  return h;
}

template <bool LDS_STATE, bool LDS_OPS, int U>
__device__ __forceinline__ void resident_run(const ResJob& J, uint32_t inst, uint4* lds_dyn) {
  __shared__ unsigned long long s_dig;  // the workgroup's digest sum of one cycle
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
  if (threadIdx.x == 0) s_dig = 0ull;
  __syncthreads();

  const uint64_t seed = J.seeds[inst];
  const uint64_t c0 = J.ctl->cycle, wc0 = J.ctl->step_cycle0;
  const uint64_t* words = J.ctl->words;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t bd = blockDim.x;
  uint64_t dig = threadIdx.x == 0 ? J.digest[inst] : 0ull;

  for (uint64_t t = 0; t < J.n_cycles; ++t) {
    const uint64_t cycle = c0 + t;
    const uint64_t words_row =
        ((cycle - wc0) * (uint64_t)J.n_inst_total + inst) * (uint64_t)J.words_per_inst;
    for (uint32_t li = 0; li < n_layers; ++li) {
      const DevLayer ly = layers[li];
      const uint32_t n = ly.end - ly.begin;
      const uint32_t n64 = (n + 63u) & ~63u;
      for (uint32_t q0 = threadIdx.x; q0 < n64; q0 += U * bd)
        resident_ops<U>(J.const_limbs, s, ops, ly, q0, bd, n, n64, seed, cycle, words, words_row,
                        lane);
      __syncthreads();
    }
    // Register digest of this cycle (the commit layer has run).  Thread 0
    // clears the sum before the next cycle's first layer barrier, and every
    // other thread adds to it only after that barrier.
    if (J.n_regs) {
      uint64_t h = 0;
      for (uint32_t j = threadIdx.x; j < J.n_regs; j += bd) h += res_reg_terms(s, J.regs[j], j);
      h = wave_sum64(h);
      if (lane == 0) atomicAdd(&s_dig, (unsigned long long)h);
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      dig = splitmix64(dig ^ s_dig);
      s_dig = 0ull;
    }
  }
  if (threadIdx.x == 0) J.digest[inst] = dig;
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

// LAYERED: layer li of every instance, one launch over the whole device.
// Block (x, y) of B threads takes positions [B U x, B U (x + 1)) of the layer
// for instance y; the state stays in HBM (RESIDENT layout), and the launch
// boundary separates the layers.
template <int U>
__global__ void __launch_bounds__(256) k_layer(ResJob J, uint32_t li) {
  const uint32_t inst = blockIdx.y, bd = blockDim.x;
  const DevLayer ly = J.layers[li];
  const uint32_t n = ly.end - ly.begin, n64 = (n + 63u) & ~63u;
  const uint32_t q0 = blockIdx.x * (bd * U) + threadIdx.x;
  const uint64_t cycle = J.ctl->cycle;
  const uint64_t words_row =
      ((cycle - J.ctl->step_cycle0) * (uint64_t)J.n_inst_total + inst) * (uint64_t)J.words_per_inst;
  resident_ops<U>(J.const_limbs, J.state + (uint64_t)inst * J.L.pitch, J.ops, ly, q0, bd, n, n64,
                  J.seeds[inst], cycle, J.ctl->words, words_row, threadIdx.x & 63u);
}

// ---------------------------------------------------------------------------
// LAYERED, persistent: one cooperative launch runs every cycle of a step.
// ---------------------------------------------------------------------------

// Barrier of all blocks of a cooperative launch (all of them resident).  The
// block whose arrival completes round r opens it; the others wait with a
// bounded spin.  A wait past spin_limit sets the error flag and goes on, so
// every block still ends (the host then reports a device error).  Each
// arrival is a release at device scope and the opening one also acquires
// before it releases the open count; a waiter spins on plain device-scope
// loads and acquires once it sees the barrier open, so every store before
// the barrier is visible to every block after it without a cache
// invalidation per spin.
__device__ __forceinline__ void grid_barrier(GridSync* gs, uint32_t& round, uint32_t spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t want = round + 1u;
    const uint32_t arrived =
        __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == want * gridDim.x) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&gs->opened, want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&gs->opened, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
        if (++spins > spin_limit) {
          __hip_atomic_store(&gs->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  round += 1u;
  __syncthreads();
}

template <int U>
__global__ void __launch_bounds__(256)
k_layer_persistent(ResJob J, uint32_t n_inst, GridSync* gs, unsigned long long* acc,
                   uint32_t spin_limit) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wpb = blockDim.x >> 6;
  const uint32_t n_waves = gridDim.x * wpb;
  const uint32_t wave = blockIdx.x * wpb + (threadIdx.x >> 6);
  const uint64_t c0 = J.ctl->cycle, wc0 = J.ctl->step_cycle0;
  const uint64_t* words = J.ctl->words;
  uint32_t round = 0;
  for (uint64_t t = 0; t < J.n_cycles; ++t) {
    const uint64_t cycle = c0 + t;
    for (uint32_t li = 0; li < J.n_layers; ++li) {
      const DevLayer ly = J.layers[li];
      const uint32_t n = ly.end - ly.begin, n64 = (n + 63u) & ~63u;
      // Units of 64 U positions of one instance: positions q0 + 64 u.
      const uint32_t per = (n64 + 64u * U - 1u) / (64u * U);
      const uint64_t units = (uint64_t)per * n_inst;
      for (uint64_t c = wave; c < units; c += n_waves) {
        const uint32_t inst = (uint32_t)(c / per), q0 = (uint32_t)(c % per) * 64u * U + lane;
        const uint64_t words_row =
            ((cycle - wc0) * (uint64_t)J.n_inst_total + inst) * (uint64_t)J.words_per_inst;
        resident_ops<U>(J.const_limbs, J.state + (uint64_t)inst * J.L.pitch, J.ops, ly, q0, 64u,
                        n, n64, J.seeds[inst], cycle, words, words_row, lane);
      }
      grid_barrier(gs, round, spin_limit);
    }
    // Register digest: 64 registers of one instance per wavefront, then the
    // fold (the sums are cleared before the next cycle's first barrier).
    const uint32_t rc = (J.n_regs + 63u) / 64u;
    for (uint64_t c = wave; c < (uint64_t)rc * n_inst; c += n_waves) {
      const uint32_t inst = (uint32_t)(c / rc), j = (uint32_t)(c % rc) * 64u + lane;
      uint64_t h = j < J.n_regs ? res_reg_terms(J.state + (uint64_t)inst * J.L.pitch, J.regs[j], j) : 0ull;
      h = wave_sum64(h);
      if (lane == 0) atomicAdd(&acc[inst], (unsigned long long)h);
    }
    grid_barrier(gs, round, spin_limit);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_inst; i += gridDim.x * blockDim.x) {
      J.digest[i] = splitmix64(J.digest[i] ^ acc[i]);
      acc[i] = 0ull;
    }
  }
}

// ---------------------------------------------------------------------------
// PARTITIONED: workgroup (instance, partition) runs its partition's
// sub-program on its copy of the instance state; once per cycle the
// partitions publish their registers, meet at a grid barrier and load the
// registers of other partitions their cones read.
// ---------------------------------------------------------------------------

// Register value (ref r) of a RESIDENT state block s to x[0 .. limbs).
__device__ __forceinline__ void reg_publish(const char* s, const SlotRef& r, uint64_t* x) {
  if (r.cls <= CD) {
    x[0] = res_fetch(s, r.cls, r.pos);
    return;
  }
  const uint64_t* q = (const uint64_t*)(s + (uint64_t)(r.pos >> 6) * 8u);
  const uint32_t nl = (r.width + 63u) >> 6;
  for (uint32_t l = 0; l < nl; ++l) x[l] = q[l];
}

// x[0 .. limbs) into register r of state block s; a 1-bit register is one
// bit of a word that other threads may update at the same time.
__device__ __forceinline__ void reg_load(char* s, const SlotRef& r, const uint64_t* x) {
  if (r.cls == CB) {
    unsigned long long* w = (unsigned long long*)(s + (uint64_t)(r.pos >> 6) * 8u);
    const unsigned long long bit = 1ull << (r.pos & 63u);
    if (x[0] & 1ull) atomicOr(w, bit);
    else atomicAnd(w, ~bit);
  } else if (r.cls <= CD) {
    res_st64(s, r.cls, r.pos, x[0]);
  } else {
    uint64_t* q = (uint64_t*)(s + (uint64_t)(r.pos >> 6) * 8u);
    const uint32_t nl = (r.width + 63u) >> 6;
    for (uint32_t l = 0; l < nl; ++l) q[l] = x[l];
  }
}

template <bool LDS_STATE>
__global__ void __launch_bounds__(1024) k_partitioned(PartRun R) {
  extern __shared__ uint4 lds_dyn[];
  const uint32_t P = R.n_parts;
  const uint32_t inst = blockIdx.x / P, part = blockIdx.x % P;
  const PartJob J = R.parts[part];
  char* g = R.state + ((uint64_t)inst * P + part) * R.pitch;
  char* s = LDS_STATE ? (char*)lds_dyn : g;
  if (LDS_STATE)
    for (uint64_t i = threadIdx.x; i < R.pitch / 16u; i += blockDim.x) lds_dyn[i] = ((const uint4*)g)[i];
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, bd = blockDim.x;
  const uint64_t seed = R.seeds[inst];
  const uint64_t c0 = R.ctl->cycle, wc0 = R.ctl->step_cycle0;
  const uint64_t* words = R.ctl->words;
  const bool lead = part == 0 && threadIdx.x == 0;
  uint64_t dig = lead ? R.digest[inst] : 0ull;
  uint32_t round = 0;
  // Exchange e uses buffer e & 1: e = 0 opens the launch (registers written
  // by the host since the last launch reach every partition), e = t + 1
  // follows cycle t.  A partition writes buffer e + 1 only after barrier e,
  // which every partition passes after it has read buffer e - 1.
  auto xrow = [&](uint32_t e) {
    return R.xch + ((uint64_t)(e & 1u) * R.n_inst + inst) * (uint64_t)R.reg_words;
  };
  auto publish = [&](uint64_t* x) {
    for (uint32_t i = threadIdx.x; i < J.n_own; i += bd) {
      const SlotRef r = R.regs[J.own[i]];
      reg_publish(s, r, x + r.out_off);
    }
  };
  auto load = [&](const uint64_t* x) {
    for (uint32_t i = threadIdx.x; i < J.n_need; i += bd) {
      const SlotRef r = R.regs[J.need[i]];
      reg_load(s, r, x + r.out_off);
    }
    __syncthreads();
  };
  publish(xrow(0));
  grid_barrier(R.gs, round, R.spin_limit);
  load(xrow(0));
  for (uint64_t t = 0; t < R.n_cycles; ++t) {
    const uint64_t cycle = c0 + t;
    const uint64_t words_row =
        ((cycle - wc0) * (uint64_t)R.n_inst + inst) * (uint64_t)R.words_per_inst;
    for (uint32_t li = 0; li < J.n_layers; ++li) {
      const DevLayer ly = J.layers[li];
      const uint32_t n = ly.end - ly.begin, n64 = (n + 63u) & ~63u;
      for (uint32_t q0 = threadIdx.x; q0 < n64; q0 += bd)
        resident_ops<1>(R.const_limbs, s, J.ops, ly, q0, bd, n, n64, seed, cycle, words,
                        words_row, lane);
      __syncthreads();
    }
    // Own registers out, with their digest terms.
    uint64_t* x = xrow((uint32_t)t + 1u);
    uint64_t h = 0;
    for (uint32_t i = threadIdx.x; i < J.n_own; i += bd) {
      const uint32_t j = J.own[i];
      const SlotRef r = R.regs[j];
      reg_publish(s, r, x + r.out_off);
      h += res_reg_terms(s, r, j);
    }
    h = wave_sum64(h);
    if (lane == 0 && h) atomicAdd(&R.acc[(t % 3u) * R.n_inst + inst], (unsigned long long)h);
    grid_barrier(R.gs, round, R.spin_limit);
    if (lead) {
      dig = splitmix64(dig ^ R.acc[(t % 3u) * R.n_inst + inst]);
      R.acc[((t + 2u) % 3u) * R.n_inst + inst] = 0ull;
    }
    load(x);
  }
  if (lead) R.digest[inst] = dig;
  if (LDS_STATE) {
    for (uint64_t i = threadIdx.x; i < R.pitch / 16u; i += blockDim.x) ((uint4*)g)[i] = lds_dyn[i];
  }
}

// ---------------------------------------------------------------------------
// SWEEP: lane = instance.  A wavefront owns TG consecutive tiles of one tile
// group of the layout (TG divides the group).  A value's blocks for the
// tiles of a group are contiguous (StateLayout), so each operand of an
// operation is one contiguous block of 64 TG e bytes for the wavefront, e
// being the element size (1/8 for 1-bit values): every class is gathered
// with one load per tile at base + this lane's offset + g * (64 e), with no
// branch on the class.  The value's address is found once per operation by
// scalar arithmetic on the record's field.
// ---------------------------------------------------------------------------
struct SweepView {
  char* base;          // state + 512 * (first tile of the wavefront's tile group)
  uint32_t row_bytes;  // bytes of one row over all allocated tiles
  uint32_t lg3;        // 3 + log2(tile group): (f % 64) << lg3 = 8 G (f % 64)
  uint32_t tt0;        // the wavefront's first tile within its group
  uint32_t lane;

  __device__ __forceinline__ SweepView(char* state, const StateLayout& L, uint32_t tile0,
                                       uint32_t ln)
      : row_bytes(L.row_bytes), lg3(3u + L.lg), tt0(tile0 & ((1u << L.lg) - 1u)), lane(ln) {
    base = state + (uint64_t)(tile0 - tt0) * 512u;
  }

  // Block of value f for tile tt0 + g, elements of 8 >> w3 bytes (w3 = 6:
  // the 64-bit word of a 1-bit value).
  __device__ __forceinline__ char* at(uint32_t f, uint32_t w3, uint32_t g) const {
    return base + (uint64_t)(f >> 6) * row_bytes + ((f & 63u) << lg3) + (tt0 + g) * (512u >> w3);
  }

  // This lane's element in a 32-bit gather: byte offset of the aligned 4-byte
  // word holding it and its bit offset there (classes CB..CW).
  __device__ __forceinline__ uint32_t off32(uint32_t w3) const {
    return ((lane << (6u - w3)) >> 5) << 2;
  }
  __device__ __forceinline__ uint32_t sh32(uint32_t w3) const { return (lane << (6u - w3)) & 31u; }
  // The same for a 64-bit gather (classes CB..CD).
  __device__ __forceinline__ uint32_t off64(uint32_t w3) const {
    return ((lane << (6u - w3)) >> 6) << 3;
  }
  __device__ __forceinline__ uint32_t sh64(uint32_t w3) const { return (lane << (6u - w3)) & 63u; }

  // The TG tiles' 64-bit words of 1-bit value f are 8 TG contiguous bytes:
  // one load for the wavefront, lane i taking dword i mod 2 TG, instead of
  // one load per tile (1-bit gathers are the smallest blocks, and the common
  // kernel is bound by its load count more than by bytes).  bits_word32 and
  // bits_word64 then hand out tile g's word (the dword of it each lane's
  // per-tile 4-byte load would have read, or the whole word).
  template <int TG>
  __device__ __forceinline__ uint32_t bits_load(uint32_t f) const {
    return *(const uint32_t*)(at(f, 6u, 0u) + 4u * (lane & (2u * TG - 1u)));
  }
  __device__ __forceinline__ uint32_t bits_word32(uint32_t x, int g) const {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)x, 2 * g);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)x, 2 * g + 1);
    return lane & 32u ? hi : lo;
  }
  __device__ __forceinline__ uint64_t bits_word64(uint32_t x, int g) const {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)x, 2 * g);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)x, 2 * g + 1);
    return ((uint64_t)hi << 32) | lo;
  }

  // 1-bit results of the TG tiles (wave-uniform words): lane g stores tile g's
  // word, one contiguous store for the wavefront.  The word is picked with
  // masks rather than a select chain, which the compiler would turn into an
  // indexed (scratch) array.
  template <int TG>
  __device__ __forceinline__ void st_bits(uint32_t f, const uint64_t* m) const {
    uint64_t mine = 0;
#pragma unroll
    for (int g = 0; g < TG; ++g) mine |= m[g] & (0ull - (uint64_t)(lane == (uint32_t)g));
    if (lane < (uint32_t)TG) *(uint64_t*)(at(f, 6u, 0u) + lane * 8u) = mine;
  }
  // The TG tiles' values of destination f, elements of type E (the class is
  // chosen once, so each tile's store differs only by its immediate offset).
  template <class E, int TG, class T>
  __device__ __forceinline__ void st_tiles(uint32_t f, const T* x) const {
    constexpr uint32_t step = 64u * sizeof(E);
    char* q = base + (uint64_t)(f >> 6) * row_bytes + ((f & 63u) << lg3) + tt0 * step +
              lane * (uint32_t)sizeof(E);
#pragma unroll
    for (int g = 0; g < TG; ++g) *(E*)(q + g * step) = (E)x[g];
  }
  // Destination of class C8..CD (C8..CW when W64 is false).
  template <int TG, bool W64, class T>
  __device__ __forceinline__ void st_dst(uint32_t cls, uint32_t f, const T* x) const {
    if (cls == C8) st_tiles<uint8_t, TG>(f, x);
    else if (cls == C16) st_tiles<uint16_t, TG>(f, x);
    else if (!W64 || cls == CW) st_tiles<uint32_t, TG>(f, x);
    else st_tiles<uint64_t, TG>(f, x);
  }
};

// Every gathered word counts as used on every path (unary operators, absent
// operands ignore some of them), so that no load is still in flight when the
// next group's loads reuse its registers: otherwise the top of the loop
// would also wait for this group's stores.
template <class T, int N>
__device__ __forceinline__ void keep_loaded(const T (&x)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" ::"v"(x[i]));
}

// B1: 1-bit operands take one load for the tile group (SweepView::bits_load).
// The kernel sets it for one operation per lane and at least 4 tiles: with
// more operations per lane, the class branch around each operand's loads
// splits them into more waits than the saved loads return.

// U operations whose classes all fit 32 bits: one 4-byte load per operand
// and tile, the lane's element cut out with a shift and a mask.
template <int U, int TG, int NS, bool B1>
__device__ __forceinline__ void sweep_u32(const SweepView& v, const DevOp* op, uint32_t n_valid) {
  uint32_t raw[U * NS * TG];
  uint32_t sh[U * NS], m[U * NS];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t cls = op_scls(op[u].code, k), w3 = cls_w3(cls);
      sh[u * NS + k] = v.sh32(w3);
      m[u * NS + k] = 0xffffffffu >> ((0x0010181Fu >> (8u * cls)) & 31u);
      if (B1 && cls == CB) {
        raw[(u * NS + k) * TG] = v.bits_load<TG>(op[u].src[k]);
      } else {
        const char* p = v.at(op[u].src[k], w3, 0u) + v.off32(w3);
        const uint32_t step = 512u >> w3;
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[(u * NS + k) * TG + g] = *(const uint32_t*)(p + g * step);
      }
    }
  keep_loaded(raw);
  if constexpr (B1) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (op_scls(op[u].code, k) == CB) {
          const uint32_t x = raw[(u * NS + k) * TG];
#pragma unroll
          for (int g = 0; g < TG; ++g) raw[(u * NS + k) * TG + g] = v.bits_word32(x, g);
        }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if ((uint32_t)u < n_valid) {
      const DevOp& q = op[u];
      const uint32_t code = q.code, opc = op_opc(code), ar = op_arity(code);
      const uint32_t dc = op_dcls(code), w = op_width(q.wimm), imm = op_imm(q.wimm);
      uint32_t a[TG], b[TG], c[TG], r[TG];
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        a[g] = (raw[(u * NS) * TG + g] >> sh[u * NS]) & m[u * NS];
        b[g] = c[g] = 0u;
        if constexpr (NS > 1) b[g] = (raw[(u * NS + 1) * TG + g] >> sh[u * NS + 1]) & m[u * NS + 1];
        if constexpr (NS > 2) c[g] = (raw[(u * NS + 2) * TG + g] >> sh[u * NS + 2]) & m[u * NS + 2];
      }
      eval_u32_n<TG>(opc, ar, a, b, c, imm, w, r);
      if (dc == CB) {
        uint64_t bits[TG];
#pragma unroll
        for (int g = 0; g < TG; ++g) bits[g] = __ballot((r[g] & 1u) != 0u);
        v.st_bits<TG>(q.dst, bits);
      } else {
        v.st_dst<TG, false>(dc, q.dst, r);
      }
    }
  }
}

// U operations with a value of 33..64 bits: one 8-byte load per operand and
// tile.
template <int U, int TG, int NS, bool B1>
__device__ __forceinline__ void sweep_u64(const SweepView& v, const DevOp* op, uint32_t n_valid) {
  uint64_t raw[U * NS * TG];
  uint32_t sh[U * NS];
  uint64_t m[U * NS];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t cls = op_scls(op[u].code, k), w3 = cls_w3(cls);
      sh[u * NS + k] = v.sh64(w3);
      m[u * NS + k] = cls_mask64(cls);
      if (B1 && cls == CB) {
        raw[(u * NS + k) * TG] = v.bits_load<TG>(op[u].src[k]);
      } else {
        const char* p = v.at(op[u].src[k], w3, 0u) + v.off64(w3);
        const uint32_t step = 512u >> w3;
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[(u * NS + k) * TG + g] = *(const uint64_t*)(p + g * step);
      }
    }
  keep_loaded(raw);
  if constexpr (B1) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (op_scls(op[u].code, k) == CB) {
          const uint32_t x = (uint32_t)raw[(u * NS + k) * TG];
#pragma unroll
          for (int g = 0; g < TG; ++g) raw[(u * NS + k) * TG + g] = v.bits_word64(x, g);
        }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if ((uint32_t)u < n_valid) {
      const DevOp& q = op[u];
      const uint32_t code = q.code, opc = op_opc(code), ar = op_arity(code);
      const uint32_t dc = op_dcls(code), w = op_width(q.wimm), imm = op_imm(q.wimm);
      uint64_t r[TG];
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        const uint64_t a = (raw[(u * NS) * TG + g] >> sh[u * NS]) & m[u * NS];
        uint64_t b = 0, c = 0;
        if constexpr (NS > 1) b = (raw[(u * NS + 1) * TG + g] >> sh[u * NS + 1]) & m[u * NS + 1];
        if constexpr (NS > 2) c = (raw[(u * NS + 2) * TG + g] >> sh[u * NS + 2]) & m[u * NS + 2];
        r[g] = eval_u64(opc, ar, a, b, c, imm, w);
      }
      if (dc == CB) {
        uint64_t bits[TG];
#pragma unroll
        for (int g = 0; g < TG; ++g) bits[g] = __ballot((r[g] & 1ull) != 0ull);
        v.st_bits<TG>(q.dst, bits);
      } else {
        v.st_dst<TG, true>(dc, q.dst, r);
      }
    }
  }
}

// U operations on 1-bit values only: the tiles' bit-sliced words, the same
// for every lane, evaluated word-wide.
template <int U, int TG, int NS, bool B1>
__device__ __forceinline__ void sweep_bit(const SweepView& v, const DevOp* op, uint32_t n_valid) {
  uint64_t raw[U * 3 * TG];
#pragma unroll
  for (int i = NS * TG; i < 3 * TG; ++i)
#pragma unroll
    for (int u = 0; u < U; ++u) raw[u * 3 * TG + i] = 0;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if constexpr (B1) {
        raw[(u * 3 + k) * TG] = v.bits_load<TG>(op[u].src[k]);
      } else {
        const char* p = v.at(op[u].src[k], 6u, 0u);
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[(u * 3 + k) * TG + g] = *(const uint64_t*)(p + g * 8u);
      }
    }
  keep_loaded(raw);
  if constexpr (B1) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const uint32_t x = (uint32_t)raw[(u * 3 + k) * TG];
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[(u * 3 + k) * TG + g] = v.bits_word64(x, g);
      }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if ((uint32_t)u < n_valid) {
      const DevOp& q = op[u];
      const uint32_t code = q.code, opc = op_opc(code), ar = op_arity(code);
      uint64_t bits[TG];
#pragma unroll
      for (int g = 0; g < TG; ++g)
        bits[g] = eval_bits(opc, ar, raw[(u * 3) * TG + g], raw[(u * 3 + 1) * TG + g],
                            raw[(u * 3 + 2) * TG + g], op_imm(q.wimm));
      v.st_bits<TG>(q.dst, bits);
    }
  }
}

template <int U, int TG, int NS, bool B1>
__device__ __forceinline__ void sweep_group(const SweepView& v, const DevOp* op, uint32_t n_valid,
                                            uint32_t kind) {
  if (kind == K_U32) sweep_u32<U, TG, NS, B1>(v, op, n_valid);
  else if (kind == K_U64) sweep_u64<U, TG, NS, B1>(v, op, n_valid);
  else sweep_bit<U, TG, NS, B1>(v, op, n_valid);
}

// The common operations (at most 64 bits, no source) of the ranges r with NS
// operand gathers each (NS >= the arity of every operation in r; absent
// operands read field 0 of class CB, a valid word).  Wave w runs the
// operation chunk w / n_groups (opw operations) on tile group w % n_groups.
// Operations of a chunk run U at a time when the U share their evaluation
// kind (ranges are sorted by kind, so mixed groups are rare), else one by one.
template <int U, int TG, int NS>
__device__ __forceinline__ void sweep_wave(const DevOp* __restrict__ ops, const StateLayout& L,
                                           char* __restrict__ state, const OpRanges& r,
                                           uint32_t opw, uint32_t split, uint32_t tile_base,
                                           uint32_t n_groups, uint32_t wave, uint32_t lane) {
  constexpr bool B1 = U == 1 && TG >= 4;
  const uint32_t grp = wave % n_groups, chunk = wave / n_groups;
  const bool first = chunk < split;
  const uint32_t o0 = first ? r.b0 + chunk * opw : r.b1 + (chunk - split) * opw;
  const uint32_t oe = first ? r.e0 : r.e1;
  if (o0 >= oe) return;
  const uint32_t o1 = min(o0 + opw, oe);
  const SweepView v(state, L, tile_base + grp * TG, lane);

  for (uint32_t o = o0; o < o1; o += U) {
    DevOp op[U];
#pragma unroll
    for (int u = 0; u < U; ++u) op[u] = ops[min(o + (uint32_t)u, o1 - 1u)];
    const uint32_t n_valid = min((uint32_t)U, o1 - o);
    const uint32_t k0 = op_kind(op[0].code);
    bool same = true;
#pragma unroll
    for (int u = 1; u < U; ++u) same = same && ((uint32_t)u >= n_valid || op_kind(op[u].code) == k0);
    if (same) {
      sweep_group<U, TG, NS, B1>(v, op, n_valid, k0);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if ((uint32_t)u < n_valid) sweep_group<1, TG, NS, B1>(v, &op[u], 1u, op_kind(op[u].code));
    }
  }
}

template <int U, int TG, int NS>
__global__ void __launch_bounds__(256)
k_sweep(const DevOp* __restrict__ ops, StateLayout L, char* __restrict__ state, OpRanges r,
        uint32_t opw, uint32_t split, uint32_t tile_base, uint32_t n_groups) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  sweep_wave<U, TG, NS>(ops, L, state, r, opw, split, tile_base, n_groups, wave,
                        threadIdx.x & 63u);
}

// One operand (slot field f of class cls) for the TG tiles of the heavy
// kernel: limb 0 from an 8-byte load holding the lane's element, further
// limbs only for values wider than 64 bits.
template <int TG>
__device__ __forceinline__ void heavy_operand(const SweepView& v, uint32_t f, uint32_t cls,
                                              V4 (&x)[TG]) {
  const uint32_t w3 = cls_w3(cls), step = 512u >> w3, sh = v.sh64(w3), kl = cls_limbs(cls);
  const uint64_t m = cls_mask64(cls);
  const char* p = v.at(f, w3, 0u) + v.off64(w3);
#pragma unroll
  for (int g = 0; g < TG; ++g) {
    x[g].l[0] = (*(const uint64_t*)(p + g * step) >> sh) & m;
#pragma unroll
    for (int l = 1; l < 4; ++l)
      x[g].l[l] = (uint32_t)l < kl ? *(const uint64_t*)(p + (uint64_t)l * v.row_bytes + g * 512u) : 0ull;
  }
}

// A fused mux chain for the TG tiles (values up to 4 limbs): the record's
// default in e, then the further pairs from the word table, innermost first
// (a nonzero selector replaces the running default with its value), then
// the record's first pair.
template <int TG>
__device__ __forceinline__ void heavy_muxc(const SweepView& v, const DevOp& q,
                                           const uint64_t* __restrict__ words, V4 (&r)[TG]) {
  V4 e[TG];
  heavy_operand<TG>(v, q.src[2], op_scls(q.code, 2), e);
  for (uint32_t i = q.aux1; i-- > 0;) {
    const uint64_t es = words[q.aux0 + 2u * i], ev = words[q.aux0 + 2u * i + 1u];
    V4 sv[TG], vv[TG];
    heavy_operand<TG>(v, (uint32_t)es, (uint32_t)(es >> 32), sv);
    heavy_operand<TG>(v, (uint32_t)ev, (uint32_t)(ev >> 32), vv);
#pragma unroll
    for (int g = 0; g < TG; ++g)
      if (v4_nonzero(sv[g])) e[g] = vv[g];
  }
  V4 s1[TG], v1[TG];
  heavy_operand<TG>(v, q.src[0], op_scls(q.code, 0), s1);
  heavy_operand<TG>(v, q.src[1], op_scls(q.code, 1), v1);
  const uint32_t w = op_width(q.wimm);
#pragma unroll
  for (int g = 0; g < TG; ++g) r[g] = eval_wide(OP_MUXC, 3u, s1[g], v1[g], e[g], 0u, w);
}

// A fused mux chain whose values all fit 64 bits: the raw 8-byte words of C
// pairs (2 C TG gathers) are in flight before the first select, so a chain
// of k pairs waits for memory about k / C times rather than k times.  Pairs
// are folded innermost first onto the default, as in heavy_muxc.
template <int TG>
__device__ __forceinline__ void heavy_muxc64(const SweepView& v, const DevOp& q,
                                             const uint64_t* __restrict__ words, V4 (&r)[TG]) {
  constexpr int C = TG >= 4 ? 4 : 8;  // 2 C TG gathers per batch
  const uint32_t np = q.aux1;
  // The record's operands (s1, v1, default) are cut only once the first
  // batch of further pairs is in flight too.
  uint64_t rec[3][TG];
  uint32_t rsh[3];
  uint64_t rm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint32_t cls = op_scls(q.code, k), w3 = cls_w3(cls), step = 512u >> w3;
    const char* p = v.at(q.src[k], w3, 0u) + v.off64(w3);
    rsh[k] = v.sh64(w3);
    rm[k] = cls_mask64(cls);
#pragma unroll
    for (int g = 0; g < TG; ++g) rec[k][g] = *(const uint64_t*)(p + g * step);
  }
  uint64_t e[TG];
  bool cut = false;
  for (int c0 = ((int)np - 1) / C * C; np && c0 >= 0; c0 -= C) {
    uint64_t raw[2 * C][TG];
    uint32_t sh[2 * C];
    uint64_t m[2 * C];
    const uint32_t nw = 2u * min((uint32_t)C, np - (uint32_t)c0);  // operands in this batch
#pragma unroll
    for (int j = 0; j < 2 * C; ++j) {
      // Only the innermost batch can be partial; its missing pairs load
      // nothing, and the fold below skips them.
      sh[j] = 0u;
      m[j] = 0ull;
      if ((uint32_t)j < nw) {
        const uint64_t wd = words[q.aux0 + 2u * (uint32_t)c0 + (uint32_t)j];
        const uint32_t cls = (uint32_t)(wd >> 32), w3 = cls_w3(cls), step = 512u >> w3;
        const char* p = v.at((uint32_t)wd, w3, 0u) + v.off64(w3);
        sh[j] = v.sh64(w3);
        m[j] = cls_mask64(cls);
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[j][g] = *(const uint64_t*)(p + g * step);
      } else {
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[j][g] = 0ull;
      }
    }
    if (!cut) {
#pragma unroll
      for (int g = 0; g < TG; ++g) e[g] = (rec[2][g] >> rsh[2]) & rm[2];
      cut = true;
    }
#pragma unroll
    for (int j = C - 1; j >= 0; --j)
      if ((uint32_t)(c0 + j) < np) {
#pragma unroll
        for (int g = 0; g < TG; ++g)
          if ((raw[2 * j][g] >> sh[2 * j]) & m[2 * j]) e[g] = (raw[2 * j + 1][g] >> sh[2 * j + 1]) & m[2 * j + 1];
      }
  }
  if (!cut) {
#pragma unroll
    for (int g = 0; g < TG; ++g) e[g] = (rec[2][g] >> rsh[2]) & rm[2];
  }
  const uint32_t w = op_width(q.wimm);
  const uint64_t mw = w >= 64 ? ~0ull : (1ull << w) - 1ull;
#pragma unroll
  for (int g = 0; g < TG; ++g) {
    const uint64_t s1 = (rec[0][g] >> rsh[0]) & rm[0], v1 = (rec[1][g] >> rsh[1]) & rm[1];
    r[g] = v4_from(0);
    r[g].l[0] = (s1 ? v1 : e[g]) & mw;
  }
}

// The fused mux chains of one layer, [hm0, hm1): each wavefront takes
// ops_per_wave of them over TG tiles of its tile group.
template <int TG>
__device__ __forceinline__ void muxc_wave(const DevOp* __restrict__ ops, const DevLayer& ly,
                                          const uint64_t* __restrict__ words, const StateLayout& L,
                                          char* __restrict__ state, uint32_t opw,
                                          uint32_t tile_base, uint32_t n_groups, uint32_t wave,
                                          uint32_t lane) {
  const uint32_t grp = wave % n_groups, chunk = wave / n_groups;
  const uint32_t o0 = ly.hm0 + chunk * opw;
  if (o0 >= ly.hm1) return;
  const uint32_t o1 = min(o0 + opw, ly.hm1);
  const SweepView v(state, L, tile_base + grp * TG, lane);
  DevOp next = ops[o0];
  for (uint32_t o = o0; o < o1; ++o) {
    const DevOp q = next;
    if (o + 1 < o1) next = ops[o + 1];  // the next record on its way meanwhile
    V4 r[TG];
    if (op_narrow_chain(q.code)) heavy_muxc64<TG>(v, q, words, r);
    else heavy_muxc<TG>(v, q, words, r);
    const uint32_t dc = op_dcls(q.code);
    uint64_t x[TG];
    if (dc == CB) {
#pragma unroll
      for (int g = 0; g < TG; ++g) x[g] = __ballot((r[g].l[0] & 1ull) != 0ull);
      v.st_bits<TG>(q.dst, x);
    } else if (dc <= CD) {
#pragma unroll
      for (int g = 0; g < TG; ++g) x[g] = r[g].l[0];
      v.st_dst<TG, true>(dc, q.dst, x);
    } else {
      const uint32_t kd = cls_limbs(dc);
      char* d0 = v.at(q.dst, 0u, 0u) + lane * 8u;
#pragma unroll
      for (int l = 0; l < 4; ++l)
        if ((uint32_t)l < kd) {
#pragma unroll
          for (int g = 0; g < TG; ++g)
            *(uint64_t*)(d0 + (uint64_t)l * v.row_bytes + g * 512u) = r[g].l[l];
        }
    }
  }
}

template <int TG>
__global__ void __launch_bounds__(256)
k_sweep_muxc(const DevOp* __restrict__ ops, const DevLayer* __restrict__ layers,
             const uint64_t* __restrict__ words, StateLayout L, char* __restrict__ state,
             uint32_t layer, uint32_t opw, uint32_t tile_base, uint32_t n_groups) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  muxc_wave<TG>(ops, layers[layer], words, L, state, opw, tile_base, n_groups, wave,
                threadIdx.x & 63u);
}

// Operands and value of heavy operation q (not a source) for the TG tiles, on
// NL limbs: limb 0 of every operand from an 8-byte load holding the lane's
// element, cut out as in the common kernel; the further limbs of wide
// operands under a uniform branch.  All loads are in flight before the first
// is used.
template <int NL, int TG>
__device__ __forceinline__ void heavy_eval(const SweepView& v, const DevOp& q, VN<NL> (&r)[TG]) {
  const uint32_t code = q.code, opc = op_opc(code), ar = op_arity(code);
  const uint32_t w = op_width(q.wimm), imm = op_imm(q.wimm);
  uint64_t raw[3 * NL * TG];
  uint32_t sh[3];
  uint64_t m[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint32_t cls = op_scls(code, k), w3 = cls_w3(cls), kl = cls_limbs(cls);
    const char* p = v.at(q.src[k], w3, 0u) + v.off64(w3);
    const uint32_t step = 512u >> w3;
    sh[k] = v.sh64(w3);
    m[k] = cls_mask64(cls);
#pragma unroll
    for (int g = 0; g < TG; ++g) raw[(k * NL) * TG + g] = *(const uint64_t*)(p + g * step);
    // Limbs 1.. exist only for values wider than 64 bits (then the lane
    // offset is 8 lane and the step 512).
#pragma unroll
    for (int l = 1; l < NL; ++l) {
      if ((uint32_t)l < kl) {
#pragma unroll
        for (int g = 0; g < TG; ++g)
          raw[(k * NL + l) * TG + g] = *(const uint64_t*)(p + (uint64_t)l * v.row_bytes + g * 512u);
      } else {
#pragma unroll
        for (int g = 0; g < TG; ++g) raw[(k * NL + l) * TG + g] = 0ull;
      }
    }
  }
  keep_loaded(raw);
#pragma unroll
  for (int g = 0; g < TG; ++g) {
    VN<NL> x[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      x[k].l[0] = (raw[(k * NL) * TG + g] >> sh[k]) & m[k];
#pragma unroll
      for (int l = 1; l < NL; ++l) x[k].l[l] = raw[(k * NL + l) * TG + g];
    }
    r[g] = eval_wide(opc, ar, x[0], x[1], x[2], imm, w);
  }
}

// Stores the TG tiles' results r of an operation with destination class dc
// at slot field dst (dc has at most NL limbs).
template <int NL, int TG>
__device__ __forceinline__ void heavy_store(const SweepView& v, uint32_t dc, uint32_t dst,
                                            const VN<NL> (&r)[TG]) {
  if (dc == CB) {
    uint64_t bits[TG];
#pragma unroll
    for (int g = 0; g < TG; ++g) bits[g] = __ballot((r[g].l[0] & 1ull) != 0ull);
    v.st_bits<TG>(dst, bits);
  } else if (dc <= CD) {
    uint64_t x[TG];
#pragma unroll
    for (int g = 0; g < TG; ++g) x[g] = r[g].l[0];
    v.st_dst<TG, true>(dc, dst, x);
  } else {
    const uint32_t kd = cls_limbs(dc);
    char* d0 = v.at(dst, 0u, 0u) + v.lane * 8u;
#pragma unroll
    for (int l = 0; l < NL; ++l)
      if ((uint32_t)l < kd) {
#pragma unroll
        for (int g = 0; g < TG; ++g)
          *(uint64_t*)(d0 + (uint64_t)l * v.row_bytes + g * 512u) = r[g].l[l];
      }
  }
}

// The heavy operations of one layer (a value wider than 64 bits, a type run
// in the wide form, or a source) other than the fused mux chains.  An
// operation whose destination and operands all fit 128 bits runs on two
// limbs, a wider one on four; NARROW: the design holds no value wider than
// 128 bits, so only the two-limb form is compiled (fewer registers).
template <int TG, bool NARROW = false>
__device__ __forceinline__ void heavy_wave(const DevOp* __restrict__ ops, const DevLayer& ly,
                                           const uint64_t* __restrict__ const_limbs,
                                           uint32_t words_per_inst, const StateLayout& L,
                                           char* __restrict__ state,
                                           const uint64_t* __restrict__ seeds,
                                           const DevCtl* __restrict__ ctl, uint32_t n_inst,
                                           uint32_t opw, uint32_t tile_base, uint32_t n_groups,
                                           uint32_t wave, uint32_t lane) {
  const uint32_t grp = wave % n_groups, chunk = wave / n_groups;
  // [hbeg, hm0) then [hm1, hend): the fused mux chains between them have a
  // kernel of their own.
  const uint32_t split = (ly.hm0 - ly.hbeg + opw - 1) / opw;
  const uint32_t o0 = chunk < split ? ly.hbeg + chunk * opw : ly.hm1 + (chunk - split) * opw;
  const uint32_t oe = chunk < split ? ly.hm0 : ly.hend;
  if (o0 >= oe) return;
  const uint32_t o1 = min(o0 + opw, oe);
  const uint32_t tile0 = tile_base + grp * TG;
  const SweepView v(state, L, tile0, lane);

  for (uint32_t o = o0; o < o1; ++o) {
    const DevOp q = ops[o];
    const uint32_t code = q.code, opc = op_opc(code), dc = op_dcls(code);
    if (opc >= OP_STIM) {
      constexpr int SL = NARROW ? 2 : 4;
      const uint32_t w = op_width(q.wimm);
      const uint64_t cycle = ctl->cycle;
      VN<SL> r[TG];
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        const uint32_t inst = (tile0 + g) * 64u + lane;
        const uint64_t words_row =
            ((cycle - ctl->step_cycle0) * (uint64_t)n_inst + inst) * (uint64_t)words_per_inst;
        r[g] = v4_from<SL>(0);
        if (inst < n_inst)
          r[g] = source_value<SL>(const_limbs, q, seeds[inst], cycle, ctl->words, words_row, w);
      }
      heavy_store<SL, TG>(v, dc, q.dst, r);
    } else if (NARROW || (dc <= CL2 && op_scls(code, 0) <= CL2 && op_scls(code, 1) <= CL2 &&
                          op_scls(code, 2) <= CL2)) {
      VN<2> r[TG];
      heavy_eval<2, TG>(v, q, r);
      heavy_store<2, TG>(v, dc, q.dst, r);
    } else if constexpr (!NARROW) {
      V4 r[TG];
      heavy_eval<4, TG>(v, q, r);
      heavy_store<4, TG>(v, dc, q.dst, r);
    }
  }
}

template <int TG>
__global__ void __launch_bounds__(256)
k_sweep_heavy(const DevOp* __restrict__ ops, const DevLayer* __restrict__ layers,
              const uint64_t* __restrict__ const_limbs, uint32_t words_per_inst, StateLayout L,
              char* __restrict__ state, const uint64_t* __restrict__ seeds,
              const DevCtl* __restrict__ ctl, uint32_t n_inst, uint32_t layer, uint32_t opw,
              uint32_t tile_base, uint32_t n_groups) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  heavy_wave<TG>(ops, layers[layer], const_limbs, words_per_inst, L, state, seeds, ctl, n_inst,
                 opw, tile_base, n_groups, wave, threadIdx.x & 63u);
}

// ---------------------------------------------------------------------------
// Several batches in one launch (rteaal_step_many): a table of segments, each
// a piece of one batch's layer (its operation ranges, launch shape and
// state), the launch's wavefronts split among them by the prefix wave0.
// The segment launches also carry, after wave0's n_seg + 1 entries, the
// segment of every wavefront, so a wavefront finds its segment with one
// scalar load (the digest launch searches wave0 instead) and runs the same
// body as the per-batch kernels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t find_seg(const uint32_t* __restrict__ wave0, uint32_t n_seg,
                                             uint32_t wave) {
  uint32_t lo = 0, hi = n_seg;  // wave0[lo] <= wave < wave0[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (wave0[mid] <= wave) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int TG>
__global__ void __launch_bounds__(256)
k_sweep_multi(const MultiSeg* __restrict__ segs, const uint32_t* __restrict__ wave0,
              uint32_t n_seg) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (wave >= wave0[n_seg]) return;
  const uint32_t k = wave0[n_seg + 1u + wave];
  const MultiSeg& g = segs[k];
  sweep_wave<1, TG, 3>(g.ops, g.L, g.state, g.r, g.opw, g.split, 0u, g.n_groups, wave - wave0[k],
                       threadIdx.x & 63u);
}

// Heavy and mux-chain segments carry their layer's heavy range in r
// (hbeg, hm0, hm1, hend), so a wavefront needs no load of the layer record.
__device__ __forceinline__ DevLayer seg_heavy_range(const MultiSeg& g) {
  DevLayer ly{};
  ly.hbeg = g.r.b0;
  ly.hm0 = g.r.e0;
  ly.hm1 = g.r.b1;
  ly.hend = g.r.e1;
  return ly;
}

template <int TG>
__global__ void __launch_bounds__(256)
k_sweep_heavy_multi(const MultiSeg* __restrict__ segs, const uint32_t* __restrict__ wave0,
                    uint32_t n_seg) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (wave >= wave0[n_seg]) return;
  const uint32_t k = wave0[n_seg + 1u + wave];
  const MultiSeg& g = segs[k];
  heavy_wave<TG>(g.ops, seg_heavy_range(g), g.const_limbs, g.words_per_inst, g.L, g.state, g.seeds,
                 g.ctl, g.n_inst, g.opw, 0u, g.n_groups, wave - wave0[k], threadIdx.x & 63u);
}

template <int TG>
__global__ void __launch_bounds__(256)
k_sweep_muxc_multi(const MultiSeg* __restrict__ segs, const uint32_t* __restrict__ wave0,
                   uint32_t n_seg) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (wave >= wave0[n_seg]) return;
  const uint32_t k = wave0[n_seg + 1u + wave];
  const MultiSeg& g = segs[k];
  muxc_wave<TG>(g.ops, seg_heavy_range(g), g.const_limbs, g.L, g.state, 1u, 0u, g.n_groups,
                wave - wave0[k], threadIdx.x & 63u);
}

// LAYERED segments: wavefront (block of 64 threads) w of segment g runs
// positions [64 (w % n_groups), +64) of layer g.layer for instance
// w / n_groups.
__device__ __forceinline__ void layer_wave(const MultiSeg& g, uint32_t local, uint32_t lane) {
  const uint32_t inst = local / g.n_groups, q0 = (local % g.n_groups) * 64u + lane;
  const DevLayer ly = g.layers[g.layer];
  const uint32_t n = ly.end - ly.begin, n64 = (n + 63u) & ~63u;
  const uint64_t cycle = g.ctl->cycle;
  const uint64_t words_row =
      ((cycle - g.ctl->step_cycle0) * (uint64_t)g.n_inst + inst) * (uint64_t)g.words_per_inst;
  resident_ops<1>(g.const_limbs, g.state + (uint64_t)inst * g.L.pitch, g.ops, ly, q0, 64u, n, n64,
                  g.seeds[inst], cycle, g.ctl->words, words_row, lane);
}

__global__ void __launch_bounds__(64)
k_layer_multi(const MultiSeg* __restrict__ segs, const uint32_t* __restrict__ wave0,
              uint32_t n_seg) {
  const uint32_t wave = blockIdx.x;
  if (wave >= wave0[n_seg]) return;
  const uint32_t k = wave0[n_seg + 1u + wave];
  layer_wave(segs[k], wave - wave0[k], threadIdx.x);
}

// Mixed launch: every segment names its own kind and tile group (variant);
// the branch on it is uniform over the wavefront.  SET 0 holds every
// variant; 1 (lean) only those of small register footprint (common
// operations with 1 or 2 tiles, 4 in flight on one, heavy operations with
// 1, or 2 in the two-limb form only, LAYERED), so that its wavefronts still
// find room beside long-running
// RESIDENT workgroups on a compute unit; 2 the lean set without LAYERED and
// 4 in flight, smaller still.
template <int SET>
__device__ __forceinline__ void mixed_body(const MultiSeg* __restrict__ segs,
                                           const uint32_t* __restrict__ wave0, uint32_t n_seg) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (wave >= wave0[n_seg]) return;
  const uint32_t k = wave0[n_seg + 1u + wave];
  const MultiSeg& g = segs[k];
  const uint32_t local = wave - wave0[k], lane = threadIdx.x & 63u;
  const uint32_t v = __builtin_amdgcn_readfirstlane(g.variant);
#define RTEAAL_MIX_SWEEP(U, TG) \
  sweep_wave<U, TG, 3>(g.ops, g.L, g.state, g.r, g.opw, g.split, 0u, g.n_groups, local, lane)
  if (v == 0) {
    RTEAAL_MIX_SWEEP(1, 1);
  } else if (v == 1) {
    RTEAAL_MIX_SWEEP(1, 2);
  } else if (v == 64) {
    RTEAAL_MIX_SWEEP(2, 1);
  } else if (v == 65) {
    RTEAAL_MIX_SWEEP(2, 2);
  } else if (v == 8) {
    heavy_wave<1>(g.ops, seg_heavy_range(g), g.const_limbs, g.words_per_inst, g.L, g.state, g.seeds,
                  g.ctl, g.n_inst, g.opw, 0u, g.n_groups, local, lane);
  } else if (v == 264) {
    heavy_wave<1, true>(g.ops, seg_heavy_range(g), g.const_limbs, g.words_per_inst, g.L, g.state,
                        g.seeds, g.ctl, g.n_inst, g.opw, 0u, g.n_groups, local, lane);
  } else if (SET <= 1 && v == 265) {
    heavy_wave<2, true>(g.ops, seg_heavy_range(g), g.const_limbs, g.words_per_inst, g.L, g.state,
                        g.seeds, g.ctl, g.n_inst, g.opw, 0u, g.n_groups, local, lane);
  } else if (SET <= 1 && v == 128) {
    RTEAAL_MIX_SWEEP(4, 1);
  } else if (SET <= 1 && v == 24) {
    layer_wave(g, local, lane);
  } else if (SET == 0) {
    switch (v) {
      case 2: RTEAAL_MIX_SWEEP(1, 4); break;
      case 66: RTEAAL_MIX_SWEEP(2, 4); break;
      case 129: RTEAAL_MIX_SWEEP(4, 2); break;
      case 9:
        heavy_wave<2>(g.ops, seg_heavy_range(g), g.const_limbs, g.words_per_inst, g.L, g.state, g.seeds,
                      g.ctl, g.n_inst, g.opw, 0u, g.n_groups, local, lane);
        break;
      case 16: muxc_wave<1>(g.ops, seg_heavy_range(g), g.const_limbs, g.L, g.state, 1u, 0u, g.n_groups, local, lane); break;
      case 17: muxc_wave<2>(g.ops, seg_heavy_range(g), g.const_limbs, g.L, g.state, 1u, 0u, g.n_groups, local, lane); break;
      case 18: muxc_wave<4>(g.ops, seg_heavy_range(g), g.const_limbs, g.L, g.state, 1u, 0u, g.n_groups, local, lane); break;
      default: break;
    }
  }
#undef RTEAAL_MIX_SWEEP
}

// The smallest set keeps six wavefronts per SIMD (at most 80 VGPRs).
template <int SET>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SET == 2 ? 6 : 1)))
k_mixed_multi(const MultiSeg* __restrict__ segs, const uint32_t* __restrict__ wave0,
              uint32_t n_seg) {
  mixed_body<SET>(segs, wave0, n_seg);
}

bool multi_lean(uint32_t kind, uint32_t tg, bool narrow) {
  return (kind == 0 && tg <= 2) || (kind == 1 && (tg == 1 || (narrow && tg == 2))) || kind == 3;
}

uint32_t multi_variant(uint32_t kind, uint32_t tg, uint32_t unroll, bool lean, bool narrow) {
  const uint32_t lg = tg >= 4 ? 2u : tg >= 2 ? 1u : 0u;
  uint32_t lu = 0;
  if (kind == 0) {  // common operations may keep their batch's unroll depth
    if (unroll == 2 && tg <= 4) lu = 1;
    if (unroll == 4 && tg <= 2) lu = 2;
    if (lean && lu == 1 && tg > 2) lu = 0;
    if (lean && lu == 2 && tg > 1) lu = 1;  // the lean kernel runs 4 in flight on one tile only
  }
  return kind * 8u + lg + 64u * lu + (kind == 1 && narrow ? 256u : 0u);
}

bool multi_mixable(uint32_t kind, uint32_t tg) {
  switch (kind) {
    case 0: return tg == 1 || tg == 2 || tg == 4;
    case 1: return tg == 1 || tg == 2;
    case 2: return tg == 1 || tg == 2 || tg == 4;
    case 3: return true;
    default: return false;
  }
}

// Digest of several batches: segment g's wavefronts run k_digest's body for
// batch g (g.layer: 1 for the SWEEP layout; g.opw: registers per chunk;
// g.n_groups: units).
__device__ __forceinline__ void digest_wave(bool sweep, const StateLayout& L,
                                            const char* __restrict__ state,
                                            const SlotRef* __restrict__ regs, uint32_t n_regs,
                                            uint32_t n_inst, uint32_t n_units, uint32_t per,
                                            unsigned long long* __restrict__ acc, uint32_t wave,
                                            uint32_t lane);

__global__ void __launch_bounds__(256)
k_digest_multi(const DigestSeg* __restrict__ segs, const uint32_t* __restrict__ wave0,
               uint32_t n_seg) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (wave >= wave0[n_seg]) return;
  const uint32_t k = find_seg(wave0, n_seg, wave);
  const DigestSeg& g = segs[k];
  digest_wave(g.sweep != 0u, g.L, g.state, g.regs, g.n_regs, g.n_inst, g.n_units, g.per,
              (unsigned long long*)g.acc, wave - wave0[k], threadIdx.x & 63u);
}

// Digest fold and cycle advance of several batches: block row y serves
// batch y.
__global__ void k_fold_advance_multi(const DigestSeg* __restrict__ segs) {
  const DigestSeg& g = segs[blockIdx.y];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.n_inst) {
    g.digest[i] = splitmix64(g.digest[i] ^ g.acc[i]);
    g.acc[i] = 0ull;
  }
  if (i == 0) g.ctl->cycle += 1;
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
    const uint32_t t = inst >> 6, ln = inst & 63u, tt = t & ((1u << L.lg) - 1u);
    const uint32_t w3 = cls_w3(cls);
    char* r = state + row * L.row_bytes + (uint64_t)(t - tt) * 512u + ((f & 63u) << (3u + L.lg)) +
              tt * (512u >> w3);
    if (cls == CB) {
      *bitpos = ln;
      return r;
    }
    return r + (ln << 3 >> w3);
  }
  char* r = state + (uint64_t)inst * L.pitch + row * 8u;
  if (cls == CB) {
    *bitpos = f & 63u;
    return r;
  }
  return r + ((f & 63u) >> 3);
}

// Value of limb `limb` of the stored value of ref for instance inst (0 for a
// slot without storage).
__device__ __forceinline__ uint64_t load_limb(bool sweep, const StateLayout& L, const char* state,
                                              const SlotRef& ref, uint32_t limb, uint32_t inst) {
  if (ref.cls == CNONE) return 0;
  uint32_t bp = 0;
  const char* e = elem_addr(sweep, L, (char*)state, ref.cls, ref.pos, limb, inst, &bp);
  if (ref.cls == CB) return (*(const uint64_t*)e >> bp) & 1ull;
  if (ref.cls == C8) return *(const uint8_t*)e;
  if (ref.cls == C16) return *(const uint16_t*)e;
  if (ref.cls == CW) return *(const uint32_t*)e;
  return *(const uint64_t*)e;
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
    x = load_limb(sweep, L, state, ref, l, inst);
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
  } else if (ref.cls <= CW) {
    char* e = elem_addr(sweep, L, state, ref.cls, ref.pos, 0, inst, &bp);
    if (ref.cls == C8) *(uint8_t*)e = (uint8_t)v.l[0];
    else if (ref.cls == C16) *(uint16_t*)e = (uint16_t)v.l[0];
    else *(uint32_t*)e = (uint32_t)v.l[0];
  } else {
    const uint32_t k2 = cls_limbs(ref.cls);
#pragma unroll
    for (uint32_t l = 0; l < 4; ++l)
      if (l < k2) *(uint64_t*)elem_addr(sweep, L, state, ref.cls, ref.pos, l, inst, &bp) = v.l[l];
  }
}

// Waveform capture.  Items are (watched signal, instance) pairs, consecutive
// items on consecutive instances of one signal (adjacent in the SWEEP
// layout); a value that differs from its copy after the previous cycle is a
// transition.  shadow is signal-major: limb k of the copies at
// shadow[k * n_inst ...].  With init, only the copies are written.
// A block of 256 threads takes 256 * CAP_ITEMS consecutive items, each thread
// CAP_ITEMS of them 256 apart.  The block's transitions get consecutive log
// positions from a block-wide scan and one atomic on the shared count (its
// atomics serialize across the device, so they are kept few); the records
// are then written from the updated copies.
constexpr uint32_t CAP_ITEMS = 8;

__global__ void __launch_bounds__(256)
k_capture(bool sweep, StateLayout L, const char* __restrict__ state, const SlotRef* __restrict__ refs,
          uint32_t n_refs, uint64_t* shadow, uint32_t n_inst, bool init,
          const DevCtl* __restrict__ ctl, ChangeRec* log, uint64_t cap, unsigned long long* count) {
  __shared__ uint32_t s_wave[4];
  __shared__ unsigned long long s_base;
  const uint64_t total = (uint64_t)n_refs * n_inst;
  const uint64_t b0 = (uint64_t)blockIdx.x * (256u * CAP_ITEMS);
  uint32_t mask = 0;
#pragma unroll
  for (uint32_t k = 0; k < CAP_ITEMS; ++k) {
    const uint64_t i = b0 + k * 256u + threadIdx.x;
    if (i < total) {
      const uint32_t inst = (uint32_t)(i % n_inst), r = (uint32_t)(i / n_inst);
      const SlotRef ref = refs[r];
      const uint32_t nl = (ref.width + 63u) >> 6;
      bool ch = false;
#pragma unroll
      for (uint32_t l = 0; l < 4; ++l)
        if (l < nl) {
          uint64_t* sh = shadow + (uint64_t)(ref.out_off + l) * n_inst + inst;
          const uint64_t x = load_limb(sweep, L, state, ref, l, inst);
          if (init || x != *sh) {
            ch = true;
            *sh = x;
          }
        }
      if (ch) mask |= 1u << k;
    }
  }
  if (init) return;  // the same for every thread of the launch
  // Exclusive scan of the per-thread transition counts over the block.
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t c = (uint32_t)__popc(mask);
  uint32_t x = c;
#pragma unroll
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63u) s_wave[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (uint32_t w = 0; w < 4; ++w) {
      const uint32_t v = s_wave[w];
      s_wave[w] = t;
      t += v;
    }
    s_base = t ? atomicAdd(count, (unsigned long long)t) : 0ull;
  }
  __syncthreads();
  uint64_t pos = s_base + s_wave[wave] + (x - c);
  const uint64_t cyc = ctl->cycle;
#pragma unroll
  for (uint32_t k = 0; k < CAP_ITEMS; ++k)
    if ((mask >> k) & 1u) {
      const uint64_t i = b0 + k * 256u + threadIdx.x;
      const uint32_t inst = (uint32_t)(i % n_inst), r = (uint32_t)(i / n_inst);
      if (pos < cap) {
        const SlotRef ref = refs[r];
        const uint32_t nl = (ref.width + 63u) >> 6;
        ChangeRec& rec = log[pos];
        rec.cycle = cyc;
        rec.instance = inst;
        rec.signal = r;
#pragma unroll
        for (uint32_t l = 0; l < 4; ++l)
          rec.value[l] = l < nl ? shadow[(uint64_t)(ref.out_off + l) * n_inst + inst] : 0ull;
      }
      ++pos;
    }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Register digest, first part: the terms of registers [per c, per (c + 1))
// added into acc[inst].  SWEEP: wavefront w takes tile w % n_units and
// chunk c = w / n_units, lane = instance, every lane walking the chunk's
// registers (a register's 64 values of a tile are one contiguous block).
// RESIDENT layout: wavefront w takes instance w % n_units and chunk
// c = w / n_units, the lanes spread over the chunk's registers, summed
// across the wavefront.  The sum is order-independent, so the atomics give
// the same result in any order.
__device__ __forceinline__ void digest_wave(bool sweep, const StateLayout& L,
                                            const char* __restrict__ state,
                                            const SlotRef* __restrict__ regs, uint32_t n_regs,
                                            uint32_t n_inst, uint32_t n_units, uint32_t per,
                                            unsigned long long* __restrict__ acc, uint32_t wave,
                                            uint32_t lane) {
  const uint32_t unit = wave % n_units, chunk = wave / n_units;
  const uint32_t j0 = chunk * per;
  if (j0 >= n_regs) return;
  const uint32_t j1 = min(j0 + per, n_regs);
  uint64_t h = 0;
  if (sweep) {
    // Limb 0 of K registers in flight at once, each one branch-free 8-byte
    // load of the word holding this lane's element (as the SWEEP kernels
    // gather), cut to the class; further limbs of wide registers after.
    constexpr int K = 8;
    const uint32_t inst = unit * 64u + lane;  // below the allocated tiles' instances
    const SweepView v((char*)state, L, unit, lane);
    for (uint32_t j = j0; j < j1; j += K) {
      uint64_t raw[K], m[K];
      uint32_t sh[K], f[K], kl[K];
#pragma unroll
      for (int u = 0; u < K; ++u) {
        const SlotRef r = regs[min(j + (uint32_t)u, j1 - 1u)];
        const uint32_t w3 = cls_w3(r.cls);
        f[u] = r.pos;
        kl[u] = cls_limbs(r.cls);
        sh[u] = v.sh64(w3);
        m[u] = cls_mask64(r.cls);
        raw[u] = *(const uint64_t*)(v.at(r.pos, w3, 0u) + v.off64(w3));
      }
#pragma unroll
      for (int u = 0; u < K; ++u) {
        if (j + (uint32_t)u < j1) {
          const uint64_t jj = (uint64_t)(j + (uint32_t)u) << 2;
          h += splitmix64(splitmix64(jj) ^ ((raw[u] >> sh[u]) & m[u]));
          for (uint32_t l = 1; l < kl[u]; ++l) {
            const uint64_t x =
                *(const uint64_t*)(v.at(f[u], 0u, 0u) + lane * 8u + (uint64_t)l * v.row_bytes);
            h += splitmix64(splitmix64(jj | l) ^ x);
          }
        }
      }
    }
    if (inst < n_inst) atomicAdd(&acc[inst], (unsigned long long)h);
  } else {
    const char* s = state + (uint64_t)unit * L.pitch;
    for (uint32_t j = j0 + lane; j < j1; j += 64u) h += res_reg_terms(s, regs[j], j);
    h = wave_sum64(h);
    if (lane == 0) atomicAdd(&acc[unit], (unsigned long long)h);
  }
}

__global__ void __launch_bounds__(256)
k_digest(bool sweep, StateLayout L, const char* __restrict__ state,
         const SlotRef* __restrict__ regs, uint32_t n_regs, uint32_t n_inst, uint32_t n_units,
         uint32_t per, unsigned long long* __restrict__ acc) {
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  digest_wave(sweep, L, state, regs, n_regs, n_inst, n_units, per, acc, wave, threadIdx.x & 63u);
}

// Register digest, second part: D = s(D ^ acc), then acc = 0.
__global__ void k_digest_fold(uint64_t* __restrict__ digest, uint64_t* __restrict__ acc,
                              uint32_t n_inst) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  digest[i] = splitmix64(digest[i] ^ acc[i]);
  acc[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// Dynamic LDS a RESIDENT workgroup may use: the 160 KB of a CU less a
// reserve for the kernel's static shared variables (the digest sum), since
// static and dynamic LDS together must fit.
size_t resident_max_lds() { return 160u * 1024u - 256u; }

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

// A tile pass must lie inside the allocated tiles and be whole tile groups
// of the wavefront, each inside one tile group of the layout.
static bool pass_ok(const StateLayout& L, TilePass tp, uint32_t tg) {
  return tp.count > 0 && tp.count % tg == 0 && tp.base % tg == 0 &&
         (uint64_t)tp.base + tp.count <= L.n_tiles_alloc && ((1u << L.lg) % tg) == 0;
}

hipError_t launch_sweep_light(const Program& p, const StateLayout& L, char* state,
                              const OpRanges& r, uint32_t n_src, uint32_t ops_per_wave,
                              uint32_t unroll, uint32_t tiles_per_wave, TilePass tp,
                              hipStream_t s) {
  const uint32_t n1 = r.e0 - r.b0, n2 = r.e1 - r.b1;
  if (n1 + n2 == 0) return hipSuccess;
  const uint32_t tg = tiles_per_wave == 16 ? 16u : tiles_per_wave == 8 ? 8u
                    : tiles_per_wave == 4 ? 4u : tiles_per_wave == 2 ? 2u : 1u;
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
    case 128 + 1: RTEAAL_SWEEP_N(1, 16) break;
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
  if (ly.hend == ly.hbeg) return hipSuccess;
  if (ops_per_wave == 0 || ly.hm0 < ly.hbeg || ly.hm1 < ly.hm0 || ly.hend < ly.hm1)
    return hipErrorInvalidValue;
  const uint32_t n_chain = ly.hm1 - ly.hm0;
  if (n_chain) {
    // Fused mux chains: up to 4 tiles and one chain per wavefront.  Measured
    // on a chain-heavy design (2M operations, 4,096 instances), per layer:
    // 4 tiles 45.1 us, 8 tiles 53.7 (fewer pairs per batch), 2 tiles 50.0;
    // 2 chains per wavefront 46.7, 4 chains 49.9.
    const uint32_t tg = tiles_per_wave >= 4 ? 4u : tiles_per_wave == 2 ? 2u : 1u;
    const uint32_t opwm = 1u;
    if (!pass_ok(L, tp, tg)) return hipErrorInvalidValue;
    const uint64_t waves = (uint64_t)((n_chain + opwm - 1) / opwm) * (tp.count / tg);
    const dim3 grid((uint32_t)((waves + 3) / 4)), blk(256);
#define RTEAAL_MUXC_K(GG)                                                                   \
  hipLaunchKernelGGL((k_sweep_muxc<GG>), grid, blk, 0, s, p.ops, p.layers, p.const_limbs,   \
                     L, state, layer, opwm, tp.base, tp.count / tg)
    if (tg == 4) RTEAAL_MUXC_K(4);
    else if (tg == 2) RTEAAL_MUXC_K(2);
    else RTEAAL_MUXC_K(1);
#undef RTEAAL_MUXC_K
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const uint32_t n1 = ly.hm0 - ly.hbeg, n2 = ly.hend - ly.hm1;
  if (n1 + n2 == 0) return hipSuccess;
  const uint32_t tg = tiles_per_wave >= 2 ? 2u : 1u;
  if (!pass_ok(L, tp, tg)) return hipErrorInvalidValue;
  const uint64_t chunks = (n1 + ops_per_wave - 1) / ops_per_wave + (n2 + ops_per_wave - 1) / ops_per_wave;
  const uint32_t n_groups = tp.count / tg;
  const uint64_t waves = chunks * n_groups;
  const dim3 grid((uint32_t)((waves + 3) / 4)), blk(256);
#define RTEAAL_HEAVY(GG)                                                                     \
  hipLaunchKernelGGL((k_sweep_heavy<GG>), grid, blk, 0, s, p.ops, p.layers, p.const_limbs,   \
                     p.words_per_inst, L, state, seeds, ctl, n_inst, layer, ops_per_wave,    \
                     tp.base, n_groups)
  if (tg == 2) RTEAAL_HEAVY(2);
  else RTEAAL_HEAVY(1);
#undef RTEAAL_HEAVY
  return hipGetLastError();
}

hipError_t launch_layer(const ResJob& J, uint32_t li, uint32_t n_layer_ops, uint32_t n_inst,
                        uint32_t block, uint32_t unroll, hipStream_t s) {
  if (n_layer_ops == 0 || n_inst == 0 || n_inst > 65535 || block == 0 || block > 256 ||
      block % 64)
    return hipErrorInvalidValue;
  const uint32_t n64 = (n_layer_ops + 63u) & ~63u;
  const uint32_t u = unroll == 4 ? 4u : unroll == 2 ? 2u : 1u, per = block * u;
  const dim3 grid((n64 + per - 1) / per, n_inst), blk(block);
  if (u == 4) hipLaunchKernelGGL(k_layer<4>, grid, blk, 0, s, J, li);
  else if (u == 2) hipLaunchKernelGGL(k_layer<2>, grid, blk, 0, s, J, li);
  else hipLaunchKernelGGL(k_layer<1>, grid, blk, 0, s, J, li);
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

hipError_t launch_capture(bool sweep, const StateLayout& L, const char* state, const SlotRef* refs,
                          uint32_t n_refs, uint64_t* shadow, uint32_t n_inst, bool init,
                          const DevCtl* ctl, ChangeRec* log, uint64_t cap,
                          unsigned long long* count, hipStream_t s) {
  const uint64_t total = (uint64_t)n_refs * n_inst;
  if (total == 0) return hipSuccess;
  const uint64_t per_block = 256ull * CAP_ITEMS;
  hipLaunchKernelGGL(k_capture, dim3((uint32_t)((total + per_block - 1) / per_block)), dim3(256), 0,
                     s, sweep, L, state, refs, n_refs, shadow, n_inst, init, ctl, log, cap, count);
  return hipGetLastError();
}

void digest_shape(bool sweep, uint32_t n_regs, uint32_t n_inst, uint32_t* n_units, uint32_t* per) {
  // About 16,384 wavefronts (64 per compute unit) to keep many loads in
  // flight, with few atomics: in the SWEEP layout every lane of a wavefront
  // adds its instance's sum with one atomic, so a wavefront takes at least
  // 32 registers (small batches would otherwise spend one atomic per term).
  *n_units = sweep ? (n_inst + 63u) / 64u : n_inst;
  const uint64_t want = std::max<uint64_t>(1, (16384u + *n_units - 1) / *n_units);
  uint64_t p = ((uint64_t)std::max<uint32_t>(n_regs, 1u) + want - 1) / want;
  if (sweep) p = std::max<uint64_t>(p, 32u);
  else p = (p + 63u) & ~uint64_t(63);
  *per = (uint32_t)p;
}

hipError_t launch_digest(bool sweep, const StateLayout& L, const char* state, const SlotRef* regs,
                         uint32_t n_regs, uint32_t n_inst, uint64_t* digest, uint64_t* acc,
                         hipStream_t s) {
  if (n_inst == 0) return hipSuccess;
  if (n_regs) {
    uint32_t n_units = 0, per = 0;
    digest_shape(sweep, n_regs, n_inst, &n_units, &per);
    if (sweep && n_units > L.n_tiles) return hipErrorInvalidValue;
    const uint64_t chunks = ((uint64_t)n_regs + per - 1) / per;
    const uint64_t waves = chunks * n_units;
    if ((waves + 3) / 4 >= (1ull << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_digest, dim3((uint32_t)((waves + 3) / 4)), dim3(256), 0, s, sweep, L,
                       state, regs, n_regs, n_inst, n_units, per, (unsigned long long*)acc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_digest_fold, dim3((n_inst + 255u) / 256u), dim3(256), 0, s, digest, acc,
                     n_inst);
  return hipGetLastError();
}

hipError_t launch_layer_persistent(const ResJob& J, uint32_t n_inst, uint32_t unroll,
                                   GridSync* gs, uint64_t* acc, uint32_t spin_limit,
                                   uint32_t blocks, hipStream_t s) {
  if (n_inst == 0 || J.n_cycles == 0) return hipSuccess;
  const uint32_t u = unroll == 2 ? 2u : 1u;
  const void* fn = u == 2 ? (const void*)k_layer_persistent<2> : (const void*)k_layer_persistent<1>;
  if (blocks == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0);
    if (e != hipSuccess) return e;
    blocks = (uint32_t)(cus * std::min(per_cu, 2));
    if (blocks == 0) return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (uint64_t*)gs, 0ull,
                     (uint64_t)(sizeof(GridSync) / 8));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ResJob j = J;
  GridSync* g = gs;
  unsigned long long* a = (unsigned long long*)acc;
  uint32_t ni = n_inst, sl = spin_limit;
  void* args[] = {&j, &ni, &g, &a, &sl};
  return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(256), args, 0, s);
}

uint32_t partitioned_capacity(uint32_t block, bool lds_state, size_t lds) {
  const void* fn = lds_state ? (const void*)k_partitioned<true> : (const void*)k_partitioned<false>;
  int dev = 0, cus = 0, per_cu = 0;
  if (lds > 64u * 1024u &&
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)resident_max_lds()) !=
          hipSuccess)
    return 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)block, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return (uint32_t)(cus * per_cu);
}

hipError_t launch_partitioned(const PartRun& R, uint32_t block, bool lds_state, hipStream_t s) {
  if (R.n_cycles == 0 || R.n_inst == 0 || R.n_parts == 0) return hipSuccess;
  const size_t lds = lds_state ? (size_t)R.pitch : 0;
  const uint64_t blocks = (uint64_t)R.n_inst * R.n_parts;
  if (blocks > partitioned_capacity(block, lds_state, lds)) return hipErrorCooperativeLaunchTooLarge;
  hipLaunchKernelGGL(k_fill_u64, dim3((3u * R.n_inst + 255u) / 256u), dim3(256), 0, s,
                     (uint64_t*)R.acc, 0ull, (uint64_t)3 * R.n_inst);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (uint64_t*)R.gs, 0ull,
                     (uint64_t)(sizeof(GridSync) / 8));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  PartRun r = R;
  void* args[] = {&r};
  const void* fn = lds_state ? (const void*)k_partitioned<true> : (const void*)k_partitioned<false>;
  return hipLaunchCooperativeKernel(fn, dim3((uint32_t)blocks), dim3(block), args, lds, s);
}

hipError_t launch_multi(uint32_t kind, uint32_t tg, const MultiSeg* segs, const uint32_t* wave0,
                        uint32_t n_seg, uint64_t n_waves, hipStream_t s) {
  if (n_seg == 0 || n_waves == 0) return hipSuccess;
  if (n_waves >= (1ull << 32)) return hipErrorInvalidValue;
  if (kind >= 4 && kind <= 6) {
    const dim3 grid((uint32_t)((n_waves + 3) / 4)), blk(256);
    if (kind == 6) hipLaunchKernelGGL(k_mixed_multi<2>, grid, blk, 0, s, segs, wave0, n_seg);
    else if (kind == 5) hipLaunchKernelGGL(k_mixed_multi<1>, grid, blk, 0, s, segs, wave0, n_seg);
    else hipLaunchKernelGGL(k_mixed_multi<0>, grid, blk, 0, s, segs, wave0, n_seg);
    return hipGetLastError();
  }
  if (kind == 3) {
    hipLaunchKernelGGL(k_layer_multi, dim3((uint32_t)n_waves), dim3(64), 0, s, segs, wave0, n_seg);
    return hipGetLastError();
  }
  const dim3 grid((uint32_t)((n_waves + 3) / 4)), blk(256);
  if (kind == 0) {
    switch (tg) {
      case 1: hipLaunchKernelGGL(k_sweep_multi<1>, grid, blk, 0, s, segs, wave0, n_seg); break;
      case 2: hipLaunchKernelGGL(k_sweep_multi<2>, grid, blk, 0, s, segs, wave0, n_seg); break;
      case 4: hipLaunchKernelGGL(k_sweep_multi<4>, grid, blk, 0, s, segs, wave0, n_seg); break;
      case 8: hipLaunchKernelGGL(k_sweep_multi<8>, grid, blk, 0, s, segs, wave0, n_seg); break;
      case 16: hipLaunchKernelGGL(k_sweep_multi<16>, grid, blk, 0, s, segs, wave0, n_seg); break;
      default: return hipErrorInvalidValue;
    }
  } else if (kind == 1) {
    if (tg == 2) hipLaunchKernelGGL(k_sweep_heavy_multi<2>, grid, blk, 0, s, segs, wave0, n_seg);
    else if (tg == 1) hipLaunchKernelGGL(k_sweep_heavy_multi<1>, grid, blk, 0, s, segs, wave0, n_seg);
    else return hipErrorInvalidValue;
  } else if (kind == 2) {
    if (tg == 4) hipLaunchKernelGGL(k_sweep_muxc_multi<4>, grid, blk, 0, s, segs, wave0, n_seg);
    else if (tg == 2) hipLaunchKernelGGL(k_sweep_muxc_multi<2>, grid, blk, 0, s, segs, wave0, n_seg);
    else if (tg == 1) hipLaunchKernelGGL(k_sweep_muxc_multi<1>, grid, blk, 0, s, segs, wave0, n_seg);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_digest_multi(const DigestSeg* segs, const uint32_t* wave0, uint32_t n_seg,
                               uint64_t n_waves, uint32_t max_inst, hipStream_t s) {
  if (n_seg == 0) return hipSuccess;
  if (n_waves >= (1ull << 32) || n_seg > 65535) return hipErrorInvalidValue;
  if (n_waves) {
    hipLaunchKernelGGL(k_digest_multi, dim3((uint32_t)((n_waves + 3) / 4)), dim3(256), 0, s, segs,
                       wave0, n_seg);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_fold_advance_multi, dim3((std::max(max_inst, 1u) + 255u) / 256u, n_seg),
                     dim3(256), 0, s, segs);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace rteaal
