// HIP kernels for gfx950: evaluation of the per-cycle layer cascade.
//
// Two mappings of the same encoded program (internal.h):
//
//  * k_resident — one workgroup per instance, one lane per operation.  All
//    cycles of a step run inside one launch; layers are separated by a
//    workgroup barrier (the iterative rank I of Cascade 1).  The instance's
//    signal vector LI lives in LDS when it fits, else in HBM/L2.
//
//  * k_sweep — one lane per instance (64 instances per wavefront), one
//    launch per layer.  An operation record is read once per wavefront
//    (wave-uniform, shared by 64 instances) and each operand gather is one
//    coalesced row of 64 instance values; 1-bit signals are bit-sliced so
//    that a whole row is one 64-bit word.
//
// Within a layer, every operation reads only slots written by earlier
// layers (levelization), so operations of one layer may run in any order
// and the store of each layer output LO goes straight to its LI slot
// (identity elision).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "ops_device.h"

namespace rteaal {

// ---------------------------------------------------------------------------
// RESIDENT: per-instance state at `s` (LDS or global).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t res_ld64(const char* s, const StateLayout& L, uint32_t cls,
                                             uint32_t idx) {
  if (cls == CB) {
    const uint64_t w = *(const uint64_t*)(s + L.off[CB] + (uint64_t)(idx >> 6) * 8u);
    return (w >> (idx & 63u)) & 1ull;
  }
  if (cls == CW) return *(const uint32_t*)(s + L.off[CW] + (uint64_t)idx * 4u);
  return *(const uint64_t*)(s + L.off[CD] + (uint64_t)idx * 8u);
}

__device__ __forceinline__ V4 res_ldv(const char* s, const StateLayout& L, uint32_t cls,
                                      uint32_t idx) {
  if (cls <= CD) return v4_from(res_ld64(s, L, cls, idx));
  const uint32_t k = cls_limbs(cls);
  const uint64_t* q = (const uint64_t*)(s + L.off[cls]) + (uint64_t)idx * k;
  V4 r = v4_from(q[0]);
  r.l[1] = q[1];
  if (k > 2) r.l[2] = q[2];
  if (k > 3) r.l[3] = q[3];
  return r;
}

__device__ __forceinline__ void res_st64(char* s, const StateLayout& L, uint32_t cls, uint32_t idx,
                                         uint64_t v) {
  if (cls == CW) *(uint32_t*)(s + L.off[CW] + (uint64_t)idx * 4u) = (uint32_t)v;
  else *(uint64_t*)(s + L.off[CD] + (uint64_t)idx * 8u) = v;
}

__device__ __forceinline__ void res_stv(char* s, const StateLayout& L, uint32_t cls, uint32_t idx,
                                        const V4& v) {
  if (cls <= CD) {
    res_st64(s, L, cls, idx, v.l[0]);
    return;
  }
  const uint32_t k = cls_limbs(cls);
  uint64_t* q = (uint64_t*)(s + L.off[cls]) + (uint64_t)idx * k;
  q[0] = v.l[0];
  q[1] = v.l[1];
  if (k > 2) q[2] = v.l[2];
  if (k > 3) q[3] = v.l[3];
}

// Value of a STIM or CONST operation for one instance.
__device__ __forceinline__ V4 source_value(const Program& p, const DevOp& op, uint64_t seed,
                                           uint64_t cycle, const uint64_t* words,
                                           uint64_t words_row, uint32_t w) {
  V4 v = v4_from(0);
  const uint32_t nl = (w + 63u) >> 6;
  if (op_opc(op.code) == OP_CONST) {
    for (uint32_t l = 0; l < nl; ++l) v.l[l] = p.const_limbs[(uint64_t)op.aux0 * 4u + l];
  } else if (words) {
    for (uint32_t l = 0; l < nl; ++l) v.l[l] = words[words_row + op.aux1 + l];
  } else {
    for (uint32_t l = 0; l < nl; ++l) v.l[l] = stim_word(seed, cycle, op.aux0, l);
  }
  return v4_mask(v, w);
}

template <bool LDS>
__global__ void __launch_bounds__(1024)
k_resident(Program p, StateLayout L, char* __restrict__ state, const uint64_t* __restrict__ seeds,
           const DevCtl* __restrict__ ctl, uint32_t n_inst_total, uint32_t inst_base,
           uint64_t n_cycles) {
  extern __shared__ uint4 lds_state[];
  const uint32_t inst = inst_base + blockIdx.x;
  char* g = state + (uint64_t)inst * L.pitch;
  char* s = LDS ? (char*)lds_state : g;
  if (LDS) {
    for (uint64_t i = threadIdx.x; i < L.pitch / 16u; i += blockDim.x)
      lds_state[i] = ((const uint4*)g)[i];
    __syncthreads();
  }
  const uint64_t seed = seeds[inst];
  const uint64_t c0 = ctl->cycle, wc0 = ctl->step_cycle0;
  const uint64_t* words = ctl->words;
  const uint32_t lane = threadIdx.x & 63u;

  for (uint64_t t = 0; t < n_cycles; ++t) {
    const uint64_t cycle = c0 + t;
    const uint64_t words_row =
        ((cycle - wc0) * (uint64_t)n_inst_total + inst) * (uint64_t)p.words_per_inst;
    for (uint32_t li = 0; li < p.n_layers; ++li) {
      const DevLayer ly = p.layers[li];
      const uint32_t n = ly.end - ly.begin;
      const uint32_t n64 = (n + 63u) & ~63u;
      for (uint32_t q = threadIdx.x; q < n64; q += blockDim.x) {
        uint64_t bit = 0;
        bool bdst = false;
        if (q < n) {
          const DevOp op = p.ops[ly.begin + q];
          const uint32_t code = op.code, opc = op_opc(code), ar = op_arity(code);
          const uint32_t dc = op_dcls(code), w = op_width(op.wimm), imm = op_imm(op.wimm);
          if (opc >= OP_STIM) {
            const V4 v = source_value(p, op, seed, cycle, words, words_row, w);
            if (dc == CB) {
              bdst = true;
              bit = v.l[0] & 1ull;
            } else {
              res_stv(s, L, dc, op.dst, v);
            }
          } else if (op_kind(code) != K_WIDE) {
            const uint64_t a = res_ld64(s, L, op_scls(code, 0), op.src[0]);
            const uint64_t b = ar > 1 ? res_ld64(s, L, op_scls(code, 1), op.src[1]) : 0ull;
            const uint64_t c = ar > 2 ? res_ld64(s, L, op_scls(code, 2), op.src[2]) : 0ull;
            const uint64_t r = eval_u64(opc, ar, a, b, c, imm, w);
            if (dc == CB) {
              bdst = true;
              bit = r & 1ull;
            } else {
              res_st64(s, L, dc, op.dst, r);
            }
          } else {
            const V4 a = res_ldv(s, L, op_scls(code, 0), op.src[0]);
            const V4 b = ar > 1 ? res_ldv(s, L, op_scls(code, 1), op.src[1]) : v4_from(0);
            const V4 c = ar > 2 ? res_ldv(s, L, op_scls(code, 2), op.src[2]) : v4_from(0);
            const V4 r = eval_wide(opc, ar, a, b, c, imm, w);
            if (dc == CB) {
              bdst = true;
              bit = r.l[0] & 1ull;
            } else {
              res_stv(s, L, dc, op.dst, r);
            }
          }
        }
        // 1-bit outputs: the wavefront's 64 consecutive operations own one word.
        const uint64_t m = __ballot(bit != 0ull);
        const uint64_t any = __ballot(bdst);
        if (any != 0ull && lane == 0)
          *(uint64_t*)(s + L.off[CB] + (uint64_t)((ly.b_base + q) >> 6) * 8u) = m;
      }
      __syncthreads();
    }
  }
  if (LDS) {
    for (uint64_t i = threadIdx.x; i < L.pitch / 16u; i += blockDim.x)
      ((uint4*)g)[i] = lds_state[i];
  }
}

// ---------------------------------------------------------------------------
// SWEEP: slot-major state, lane = instance.
// ---------------------------------------------------------------------------
struct SweepView {
  char* base;
  StateLayout L;
  uint32_t tile, lane, j;

  __device__ __forceinline__ uint64_t ld_word(uint32_t idx) const {  // CB row of this tile
    return ((const uint64_t*)(base + L.off[CB]))[(uint64_t)idx * L.n_tiles + tile];
  }
  __device__ __forceinline__ uint64_t ld64(uint32_t cls, uint32_t idx) const {
    if (cls == CB) return (ld_word(idx) >> lane) & 1ull;
    if (cls == CW) return ((const uint32_t*)(base + L.off[CW]))[(uint64_t)idx * L.n_pad + j];
    return ((const uint64_t*)(base + L.off[CD]))[(uint64_t)idx * L.n_pad + j];
  }
  __device__ __forceinline__ V4 ldv(uint32_t cls, uint32_t idx) const {
    if (cls <= CD) return v4_from(ld64(cls, idx));
    const uint32_t k = cls_limbs(cls);
    const uint64_t* q = (const uint64_t*)(base + L.off[cls]) + (uint64_t)idx * k * L.n_pad + j;
    V4 r = v4_from(q[0]);
    r.l[1] = q[L.n_pad];
    if (k > 2) r.l[2] = q[2ull * L.n_pad];
    if (k > 3) r.l[3] = q[3ull * L.n_pad];
    return r;
  }
  __device__ __forceinline__ void st_word(uint32_t idx, uint64_t w) const {
    ((uint64_t*)(base + L.off[CB]))[(uint64_t)idx * L.n_tiles + tile] = w;
  }
  __device__ __forceinline__ void st64(uint32_t cls, uint32_t idx, uint64_t v) const {
    if (cls == CW) ((uint32_t*)(base + L.off[CW]))[(uint64_t)idx * L.n_pad + j] = (uint32_t)v;
    else ((uint64_t*)(base + L.off[CD]))[(uint64_t)idx * L.n_pad + j] = v;
  }
  __device__ __forceinline__ void stv(uint32_t cls, uint32_t idx, const V4& v) const {
    if (cls <= CD) {
      st64(cls, idx, v.l[0]);
      return;
    }
    const uint32_t k = cls_limbs(cls);
    uint64_t* q = (uint64_t*)(base + L.off[cls]) + (uint64_t)idx * k * L.n_pad + j;
    q[0] = v.l[0];
    q[L.n_pad] = v.l[1];
    if (k > 2) q[2ull * L.n_pad] = v.l[2];
    if (k > 3) q[3ull * L.n_pad] = v.l[3];
  }
};

__global__ void __launch_bounds__(256)
k_sweep(Program p, StateLayout L, char* __restrict__ state, const uint64_t* __restrict__ seeds,
        const DevCtl* __restrict__ ctl, uint32_t n_inst, uint32_t layer, uint32_t opw) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const uint32_t tile = wave % L.n_tiles, chunk = wave / L.n_tiles;
  const DevLayer ly = p.layers[layer];
  const uint32_t o0 = ly.begin + chunk * opw;
  if (o0 >= ly.end) return;
  const uint32_t o1 = min(o0 + opw, ly.end);
  SweepView v{state, L, tile, lane, tile * 64u + lane};
  const bool live = v.j < n_inst;
  const uint64_t seed = seeds[v.j];
  const uint64_t cycle = ctl->cycle;
  const uint64_t* words = ctl->words;
  const uint64_t words_row =
      ((cycle - ctl->step_cycle0) * (uint64_t)n_inst + v.j) * (uint64_t)p.words_per_inst;

  for (uint32_t o = o0; o < o1; ++o) {
    const DevOp op = p.ops[o];
    const uint32_t code = op.code, opc = op_opc(code), ar = op_arity(code), kind = op_kind(code);
    const uint32_t dc = op_dcls(code), w = op_width(op.wimm), imm = op_imm(op.wimm);
    if (opc >= OP_STIM) {
      V4 x = v4_from(0);
      if (live) x = source_value(p, op, seed, cycle, words, words_row, w);
      if (dc == CB) {
        const uint64_t m = __ballot((x.l[0] & 1ull) != 0ull);
        if (lane == 0) v.st_word(op.dst, m);
      } else {
        v.stv(dc, op.dst, x);
      }
    } else if (kind == K_BIT) {
      const uint64_t a = v.ld_word(op.src[0]);
      const uint64_t b = ar > 1 ? v.ld_word(op.src[1]) : 0ull;
      const uint64_t c = ar > 2 ? v.ld_word(op.src[2]) : 0ull;
      const uint64_t r = eval_bits(opc, ar, a, b, c, imm);
      if (lane == 0) v.st_word(op.dst, r);
    } else if (kind == K_U64) {
      const uint64_t a = v.ld64(op_scls(code, 0), op.src[0]);
      const uint64_t b = ar > 1 ? v.ld64(op_scls(code, 1), op.src[1]) : 0ull;
      const uint64_t c = ar > 2 ? v.ld64(op_scls(code, 2), op.src[2]) : 0ull;
      const uint64_t r = eval_u64(opc, ar, a, b, c, imm, w);
      if (dc == CB) {
        const uint64_t m = __ballot((r & 1ull) != 0ull);
        if (lane == 0) v.st_word(op.dst, m);
      } else {
        v.st64(dc, op.dst, r);
      }
    } else {
      const V4 a = v.ldv(op_scls(code, 0), op.src[0]);
      const V4 b = ar > 1 ? v.ldv(op_scls(code, 1), op.src[1]) : v4_from(0);
      const V4 c = ar > 2 ? v.ldv(op_scls(code, 2), op.src[2]) : v4_from(0);
      const V4 r = eval_wide(opc, ar, a, b, c, imm, w);
      if (dc == CB) {
        const uint64_t m = __ballot((r.l[0] & 1ull) != 0ull);
        if (lane == 0) v.st_word(op.dst, m);
      } else {
        v.stv(dc, op.dst, r);
      }
    }
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

__device__ __forceinline__ uint64_t* elem_ptr(bool sweep, const StateLayout& L, char* state,
                                              uint32_t cls, uint32_t idx, uint32_t limb,
                                              uint32_t inst, uint32_t* bitpos) {
  if (sweep) {
    if (cls == CB) {
      *bitpos = inst & 63u;
      return (uint64_t*)(state + L.off[CB]) + (uint64_t)idx * L.n_tiles + (inst >> 6);
    }
    if (cls == CW) return nullptr;  // 32-bit element, handled by the caller
    const uint32_t k = cls_limbs(cls);
    return (uint64_t*)(state + L.off[cls]) + ((uint64_t)idx * k + limb) * L.n_pad + inst;
  }
  char* s = state + (uint64_t)inst * L.pitch;
  if (cls == CB) {
    *bitpos = idx & 63u;
    return (uint64_t*)(s + L.off[CB]) + (idx >> 6);
  }
  if (cls == CW) return nullptr;
  const uint32_t k = cls_limbs(cls);
  return (uint64_t*)(s + L.off[cls]) + (uint64_t)idx * k + limb;
}

__device__ __forceinline__ uint32_t* elem32_ptr(bool sweep, const StateLayout& L, char* state,
                                                uint32_t idx, uint32_t inst) {
  if (sweep) return (uint32_t*)(state + L.off[CW]) + (uint64_t)idx * L.n_pad + inst;
  return (uint32_t*)(state + (uint64_t)inst * L.pitch + L.off[CW]) + idx;
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
    if (ref.cls == CNONE) {
      x = 0;
    } else if (ref.cls == CW) {
      x = *elem32_ptr(sweep, L, (char*)state, ref.idx, inst);
    } else {
      uint32_t bp = 0;
      const uint64_t* e = elem_ptr(sweep, L, (char*)state, ref.cls, ref.idx, l, inst, &bp);
      x = ref.cls == CB ? ((*e >> bp) & 1ull) : *e;
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
  for (uint32_t l = 0; l < nl; ++l) v.l[l] = src[l];
  v = v4_mask(v, ref.width);
  if (ref.cls == CW) {
    *elem32_ptr(sweep, L, state, ref.idx, inst) = (uint32_t)v.l[0];
  } else if (ref.cls == CB) {
    uint32_t bp = 0;
    unsigned long long* e =
        (unsigned long long*)elem_ptr(sweep, L, state, CB, ref.idx, 0, inst, &bp);
    if (v.l[0] & 1ull) atomicOr(e, 1ull << bp);
    else atomicAnd(e, ~(1ull << bp));
  } else {
    for (uint32_t l = 0; l < cls_limbs(ref.cls); ++l) {
      uint32_t bp = 0;
      *elem_ptr(sweep, L, state, ref.cls, ref.idx, l, inst, &bp) = v.l[l];
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
size_t resident_max_lds() { return 160u * 1024u; }

hipError_t launch_resident(const Program& p, const StateLayout& L, char* state,
                           const uint64_t* seeds, DevCtl* ctl, uint32_t n_inst,
                           uint32_t n_inst_total, uint32_t inst_base, uint64_t n_cycles,
                           uint32_t block, bool lds, hipStream_t s) {
  if (n_inst == 0 || n_cycles == 0) return hipSuccess;
  if (lds) {
    static bool attr_set = false;
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute((const void*)k_resident<true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)resident_max_lds());
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    hipLaunchKernelGGL(k_resident<true>, dim3(n_inst), dim3(block), (size_t)L.pitch, s, p, L,
                       state, seeds, (const DevCtl*)ctl, n_inst_total, inst_base, n_cycles);
  } else {
    hipLaunchKernelGGL(k_resident<false>, dim3(n_inst), dim3(block), 0, s, p, L, state, seeds,
                       (const DevCtl*)ctl, n_inst_total, inst_base, n_cycles);
  }
  return hipGetLastError();
}

hipError_t launch_sweep_layer(const Program& p, const StateLayout& L, char* state,
                              const uint64_t* seeds, DevCtl* ctl, uint32_t n_inst,
                              uint32_t layer, uint32_t layer_ops, uint32_t ops_per_wave,
                              hipStream_t s) {
  if (layer_ops == 0) return hipSuccess;
  const uint64_t chunks = (layer_ops + ops_per_wave - 1) / ops_per_wave;
  const uint64_t waves = chunks * L.n_tiles;
  const uint32_t blocks = (uint32_t)((waves + 3) / 4);
  hipLaunchKernelGGL(k_sweep, dim3(blocks), dim3(256), 0, s, p, L, state, seeds,
                     (const DevCtl*)ctl, n_inst, layer, ops_per_wave);
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
