// Internal device encoding of a design and the launch interfaces of the
// kernels.  Shared by the host runtime (host.cpp) and the kernels
// (kernels.hip); not part of the public C interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rteaal {

// Width classes of a slot.  A value of class CB is one bit; CW fits 32 bits;
// CD fits 64 bits; CL2/CL3/CL4 take 2/3/4 64-bit limbs.
enum Cls : uint32_t { CB = 0, CW = 1, CD = 2, CL2 = 3, CL3 = 4, CL4 = 5, NCLS = 6, CNONE = 7 };

__host__ __device__ inline uint32_t cls_limbs(uint32_t c) { return c <= CD ? 1u : c - 1u; }
__host__ __device__ inline uint32_t cls_of_width(uint32_t w) {
  return w == 1 ? CB : w <= 32 ? CW : w <= 64 ? CD : w <= 128 ? CL2 : w <= 192 ? CL3 : CL4;
}
// Bytes one value of class c takes in an instance's wide region (c != CB).
__host__ __device__ inline uint32_t cls_bytes(uint32_t c) { return c == CW ? 4u : 8u * cls_limbs(c); }

// Operation codes: the public rank-N coordinates 0..14 plus three
// bookkeeping operations the encoder adds around the design's layers:
// COPY (register commit and its staging), STIM (primary input from the
// stimulus) and CONST (literal).
enum Opc : uint32_t {
  OP_AND = 0, OP_OR, OP_XOR, OP_NOT, OP_ADD, OP_SUB, OP_MUL, OP_MUX, OP_EQ, OP_LT, OP_SHL,
  OP_SHR, OP_EXTRACT, OP_CONCAT, OP_ORR, OP_COPY = 15, OP_STIM = 16, OP_CONST = 17
};

// Evaluation kind: every class is CB (1-bit logic on whole words of
// bit-sliced instances), every class fits 32 bits, every class fits 64 bits,
// or some class is wider.
enum Kind : uint32_t { K_BIT = 0, K_U64 = 1, K_WIDE = 2, K_U32 = 3 };

// One operation, 32 bytes.
//   code: opc[0:5] kind[6:7] arity[8:9] dst class[10:12] src classes [13:15][16:18][19:21]
//   wimm: dst width[0:8] (1..256), imm[9:17] (shift, low bit, width of o1 for CONCAT)
//   dst, src[3]: bit index of a 1-bit slot, else its byte offset Y (see StateLayout)
//   aux0: STIM input number / CONST literal index;  aux1: STIM limb offset in a words row
struct DevOp {
  uint32_t code, wimm, dst, src[3], aux0, aux1;
};
static_assert(sizeof(DevOp) == 32, "DevOp layout");

__host__ __device__ inline uint32_t op_opc(uint32_t c) { return c & 63u; }
__host__ __device__ inline uint32_t op_kind(uint32_t c) { return (c >> 6) & 3u; }
__host__ __device__ inline uint32_t op_arity(uint32_t c) { return (c >> 8) & 3u; }
__host__ __device__ inline uint32_t op_dcls(uint32_t c) { return (c >> 10) & 7u; }
__host__ __device__ inline uint32_t op_scls(uint32_t c, int o) { return (c >> (13 + 3 * o)) & 7u; }
__host__ __device__ inline uint32_t op_width(uint32_t w) { return w & 511u; }
__host__ __device__ inline uint32_t op_imm(uint32_t w) { return (w >> 9) & 511u; }

// One encoded layer: operations [begin, end).  Operations whose destination
// is 1-bit come first, and the i-th of them writes bit index b_base + i
// (b_base a multiple of 64), so one wavefront of consecutive operations
// fills exactly one 64-bit word.
struct DevLayer {
  uint32_t begin, end, b_base, n_bdst;
};

// Per-batch control block in device memory.
struct DevCtl {
  uint64_t cycle;         // cycle number of the next cycle to run
  uint64_t step_cycle0;   // cycle at which the words buffer of the current step starts
  const uint64_t* words;  // buffer stimulus of the current step, or null
  uint64_t pad;
};

// Byte layout of one batch's signal state.
//
// Every 1-bit slot has a bit index i; every other slot has a byte offset Y
// inside one instance's "wide region" (CW elements take 4 bytes, CD 8, CLk
// 8k with the limbs contiguous).  Operation records carry i or Y, so one
// record format serves both mappings:
//   RESIDENT, instance j at j*pitch:
//     1-bit slot i: bit i of the 64-bit words at b_off;
//     other slot:   its bytes at nb_off + Y (limb l at + 8l).
//   SWEEP, tile t = j / 64, lane = j % 64:
//     1-bit slot i: bit `lane` of the word at b_off + ((i << b_shift) + t*8),
//       b_shift = 3 + log2(tile count rounded up to a power of two) (the words
//       of one slot are adjacent across tiles);
//     other slot:   tile t's block starts at nb_off + t*tile_bytes; the 4- or
//       8-byte element at resident offset Y (limb l: Y + 8l) becomes a row of
//       64 lanes at (Y + 8l)*64, lane at +4*lane (CW) or +8*lane (others).
//   zero_off: zero bytes (16 per instance block for RESIDENT, 256 for SWEEP)
//   read in place of an absent operand or high half.
struct StateLayout {
  uint64_t b_off, nb_off, zero_off, pitch, tile_bytes;
  uint32_t n_tiles, n_pad, b_shift, pad;
};

struct Program {
  const DevOp* ops;
  const DevLayer* layers;
  const uint64_t* const_limbs;  // [n_consts][4]
  uint32_t n_layers;
  uint32_t words_per_inst;      // stimulus limbs per instance and cycle
};

// Reference to a stored value for state read-out and restore: class, bit
// index (1-bit) or wide-region byte offset Y (others), offset in the packed
// output row, declared width.
struct SlotRef {
  uint32_t cls, pos, out_off, width;
};

// Everything a RESIDENT workgroup needs to run its instance of one batch.
struct ResJob {
  const DevOp* ops;
  const DevLayer* layers;
  const uint64_t* const_limbs;
  uint32_t n_layers, words_per_inst, n_ops_total, n_inst_total;
  StateLayout L;
  char* state;
  const uint64_t* seeds;
  const DevCtl* ctl;
  uint64_t n_cycles;
};

// ---- kernel launchers (kernels.hip) ---------------------------------------
hipError_t launch_resident(const ResJob& J, uint32_t n_inst, uint32_t inst_base, uint32_t block,
                           bool lds_state, bool lds_ops, uint32_t unroll, hipStream_t s);
hipError_t launch_resident_multi(const ResJob* jobs, const uint2* map, uint32_t n_blocks,
                                 uint32_t block, bool lds_state, bool lds_ops, uint32_t unroll,
                                 size_t lds, hipStream_t s);
size_t resident_lds_bytes(const StateLayout& L, uint32_t n_ops_total, uint32_t n_layers,
                          bool lds_state, bool lds_ops);
hipError_t launch_sweep_layer(const Program& p, const StateLayout& L, char* state,
                              const uint64_t* seeds, DevCtl* ctl, uint32_t n_inst,
                              uint32_t layer, uint32_t layer_ops, uint32_t ops_per_wave,
                              uint32_t unroll, uint32_t tiles_per_wave, hipStream_t s);
hipError_t launch_advance(DevCtl* ctl, uint64_t n, hipStream_t s);
hipError_t launch_set_words(DevCtl* ctl, const uint64_t* words, hipStream_t s);
hipError_t launch_pack(bool sweep, const StateLayout& L, const char* state, const SlotRef* refs,
                       uint32_t n_refs, uint32_t words_per_inst, uint32_t first, uint32_t n,
                       uint64_t* out, hipStream_t s);
hipError_t launch_unpack(bool sweep, const StateLayout& L, char* state, const SlotRef* refs,
                         uint32_t n_refs, uint32_t words_per_inst, uint32_t first, uint32_t n,
                         const uint64_t* in, hipStream_t s);
size_t resident_max_lds();

}  // namespace rteaal
