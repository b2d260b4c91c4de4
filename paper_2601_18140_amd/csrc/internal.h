// Internal device encoding of a design and the launch interfaces of the
// kernels.  Shared by the host runtime (host.cpp) and the kernels
// (kernels.hip); not part of the public C interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rteaal {

// Width classes of a slot.  A value of class CB is one bit; C8, C16 and CW
// fit 8, 16 and 32 bits and are stored in 1, 2 and 4 bytes; CD fits 64 bits;
// CL2/CL3/CL4 take 2/3/4 64-bit limbs.  CNONE (host only) marks a slot
// without storage.
enum Cls : uint32_t {
  CB = 0, C8 = 1, C16 = 2, CW = 3, CD = 4, CL2 = 5, CL3 = 6, CL4 = 7, NCLS = 8, CNONE = 15
};

__host__ __device__ inline uint32_t cls_limbs(uint32_t c) { return c <= CD ? 1u : c - 3u; }
__host__ __device__ inline uint32_t cls_of_width(uint32_t w) {
  return w == 1 ? CB : w <= 8 ? C8 : w <= 16 ? C16 : w <= 32 ? CW : w <= 64 ? CD
       : w <= 128 ? CL2 : w <= 192 ? CL3 : CL4;
}
// log2(64 / element bits) of class c (c < NCLS): 6 for CB, 3 for C8, 2 for
// C16, 1 for CW, 0 for CD and the limbs of wider values.  64 >> cls_w3(c)
// elements share one 64-bit word.
__host__ __device__ inline uint32_t cls_w3(uint32_t c) { return (0x1236u >> (4u * c)) & 15u; }
// Bytes one value of class c takes in an instance's wide region (c != CB).
__host__ __device__ inline uint32_t cls_bytes(uint32_t c) {
  return c <= CW ? (8u >> cls_w3(c)) : 8u * cls_limbs(c);
}

// Operation codes: the public rank-N coordinates 0..21 plus three
// bookkeeping operations the encoder adds around the design's layers:
// COPY (register commit and its staging), STIM (primary input from the
// stimulus) and CONST (literal).
enum Opc : uint32_t {
  OP_AND = 0, OP_OR, OP_XOR, OP_NOT, OP_ADD, OP_SUB, OP_MUL, OP_MUX, OP_EQ, OP_LT, OP_SHL,
  OP_SHR, OP_EXTRACT, OP_CONCAT, OP_ORR, OP_DIV, OP_REM, OP_DSHL, OP_DSHR, OP_ANDR, OP_XORR,
  OP_SEXT, OP_MUXC, OP_COPY = 60, OP_STIM = 61, OP_CONST = 62
};

// Evaluation kind: every class is CB (1-bit logic on whole words of
// bit-sliced instances), every class fits 32 bits, every class fits 64 bits,
// or some class is wider.
enum Kind : uint32_t { K_BIT = 0, K_U64 = 1, K_WIDE = 2, K_U32 = 3 };

// One operation, 32 bytes.
//   code: opc[0:5] kind[6:7] arity[8:9] dst class[10:12] src classes [13:15][16:18][19:21]
//         narrow chain[22]
//   wimm: dst width[0:8] (1..256), imm[9:17] (shift, low bit, width of o1 for CONCAT,
//         width of o0 for ANDR and SEXT)
//   dst, src[3]: slot fields 64*row + shift (see StateLayout)
//   aux0: STIM input number / CONST literal index;  aux1: STIM limb offset in a words row
//   MUXC: src = (s1, v1, default); aux0: index in the word table of the
//         further pairs' operands (selector, value, selector, ...; one word
//         each: field in bits 0..31, class in bits 32..34); aux1: their
//         number of pairs
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
// MUXC whose destination and operands all fit 64 bits (bit 22 of code).
__host__ __device__ inline bool op_narrow_chain(uint32_t c) { return (c >> 22) & 1u; }

// One encoded layer: operations [begin, end).  Operations whose destination
// is 1-bit come first, and each group of 64 of them (i = 64g .. 64g+63)
// writes bits 0..63 of one row of its own, so one wavefront of consecutive
// operations fills exactly one 64-bit word (b_base: the first group's row
// times 64).  The "heavy" operations (a value wider than 64 bits, a type
// always run in the wide form, or a source: STIM, CONST) form the contiguous
// range [hbeg, hend) (the last 1-bit destinations and the first others), so
// the SWEEP mapping runs them in a kernel of their own and keeps the common
// kernel small.  Inside it, the fused mux chains (MUXC) form the sub-range
// [hm0, hm1) (the last 1-bit destinations of the heavy range and the first
// others), run by a third kernel; [hbeg, hm0) and [hm1, hend) hold the other
// heavy operations.
struct DevLayer {
  uint32_t begin, end, b_base, n_bdst, hbeg, hend, hm0, hm1;
};
static_assert(sizeof(DevLayer) == 32, "DevLayer layout");

__host__ __device__ inline bool op_heavy(uint32_t code) {
  return op_kind(code) == K_WIDE || op_opc(code) >= OP_STIM;
}

// The common (non-heavy) operations of one layer with a given arity: two
// ranges of operation indices, [b0, e0) among the 1-bit destinations and
// [b1, e1) among the others (each layer orders its common operations by
// arity, mirrored around the heavy range, so every arity is two ranges).
struct OpRanges {
  uint32_t b0, e0, b1, e1;
};

// SWEEP: the tiles [base, base + count) one launch covers.  A cycle may run
// as several passes over disjoint tile ranges (instances are independent), so
// that a pass's recent layer outputs stay in the device's last-level cache.
struct TilePass {
  uint32_t base, count;
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
// An instance's stored values occupy 64-bit rows: the first rows each hold
// 64 1-bit slots (bit k of row r is 1-bit slot 64r + k), the remaining rows
// ("wide rows") each hold eight 8-bit, four 16-bit or two 32-bit values, one
// 64-bit value, or one limb of a wider value (limb l of a value in row r is
// in row r + l).  A slot is named by one 32-bit field f = 64*row + shift,
// where shift is the bit offset of the value in its row (the bit index for a
// 1-bit slot, a multiple of the element size otherwise).  Operation records
// carry these fields, so one record format serves both mappings:
//   RESIDENT, instance j at j*pitch: row r at 8r; the value is the row's
//     word shifted down by `shift` (then cut to the class).
//   SWEEP, tile t = j / 64, lane = j % 64, tiles in groups of G = 2^lg
//     (T = allocated tiles, a multiple of G; row_bytes = 512 T): row r takes
//     512 bytes per tile, grouped by tile group, so group q's part of row r
//     starts at r row_bytes + 512 G q.  Inside it, the value at shift s
//     occupies 8 G s bytes on: the G tiles' element blocks in tile order,
//     64 elements of e bytes each (a 1-bit value: one 64-bit word per tile,
//     bit `lane` = the instance's value).  For the element size e (1/8 for
//     1-bit values), the byte address of slot f for tile t = G q + u is
//       (f / 64) row_bytes + 512 G q + 8 G (f % 64) + 64 e u + e lane,
//     so the G tiles of one value are contiguous: a wavefront covering a
//     tile group reads one block of 64 G e bytes per operand.
struct StateLayout {
  uint64_t pitch;          // RESIDENT: bytes per instance (multiple of 16)
  uint32_t row_bytes;      // SWEEP: bytes of one row over all allocated tiles
  uint32_t n_rows;         // 64-bit rows per instance
  uint32_t n_tiles;        // SWEEP: tiles that hold instances
  uint32_t n_tiles_alloc;  // SWEEP: allocated tiles, a multiple of the tile group
  uint32_t lg;             // SWEEP: log2 of the tile group of the layout
  uint32_t pad;
};

struct Program {
  const DevOp* ops;
  const DevLayer* layers;
  const uint64_t* const_limbs;  // word table: [n_consts][4] literal limbs, then mux-chain operands
  uint32_t n_layers;
  uint32_t words_per_inst;      // stimulus limbs per instance and cycle
};

// Reference to a stored value for state read-out and restore: class, slot
// field (see StateLayout), offset in the packed output row, declared width.
struct SlotRef {
  uint32_t cls, pos, out_off, width;
};

// Everything a RESIDENT workgroup needs to run its instance of one batch.
// regs / n_regs: the registers' stored values (slot refs, in register
// order) that the per-cycle digest folds; digest: one running digest per
// instance.
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
  const SlotRef* regs;
  uint64_t* digest;
  uint32_t n_regs, pad;
};

// One segment of a launch over several batches (rteaal_step_many): a piece
// of one batch's layer.  SWEEP common operations: the ranges r in chunks of
// opw operations (split: chunks in [b0, e0)) times n_groups tile groups;
// SWEEP heavy operations and fused mux chains: those of layer `layer` in the
// same way, r then holding the layer's (hbeg, hm0, hm1, hend); LAYERED: layer `layer`, n_groups wavefronts of 64 positions per
// instance.  variant (mixed launches only, multi_variant): kind x 8 +
// log2(tile group) + 64 x log2(unroll depth of common operations) + 256 for
// the heavy pieces of a design with no value wider than 128 bits, the kinds
// as in launch_multi.  unroll: the batch's unroll depth (mixed launches run
// common operations with it; the other multi-batch launches with 1).
struct MultiSeg {
  const DevOp* ops;
  const DevLayer* layers;
  const uint64_t* const_limbs;
  char* state;
  const uint64_t* seeds;
  const DevCtl* ctl;
  StateLayout L;
  OpRanges r;
  uint32_t layer, n_inst, words_per_inst, opw, split, n_groups, variant, unroll;
};
static_assert(sizeof(MultiSeg) == 128, "MultiSeg layout");

// One batch of a multi-batch register digest (k_digest's arguments) and its
// cycle counter, which the fold advances.
struct DigestSeg {
  StateLayout L;
  const char* state;
  const SlotRef* regs;
  uint64_t* digest;
  uint64_t* acc;
  DevCtl* ctl;
  uint32_t n_regs, n_inst, n_units, per, sweep, pad;
};
static_assert(sizeof(DigestSeg) == 96, "DigestSeg layout");

// State of the grid-wide barrier of a persistent launch (device memory,
// zero before each launch): arrivals so far (every block adds one per
// barrier, never reset during the launch), the number of barriers opened,
// and an error flag, set when a block's wait exceeds the spin limit.
struct GridSync {
  uint32_t count, opened, error, pad;
};

// PARTITIONED (the RepCut cascade of App. C): the registers are split into
// P partitions; partition p evaluates, on a private copy of the instance's
// state, the operations of the fan-in cones of the registers it owns (its
// sub-program: the design's layers restricted to those operations), commits
// its own registers, and once per cycle the partitions exchange register
// values through device memory (Cascade 2's register update map RUM).
struct PartJob {
  const DevOp* ops;        // the partition's operations, layer after layer
  const DevLayer* layers;  // [n_layers]: ranges into ops (begin, end; the rest 0)
  const uint32_t* own;     // registers (indices into the design's) it commits
  const uint32_t* need;    // registers of other partitions its cone reads
  uint32_t n_layers, n_own, n_need, pad;
};

struct PartRun {
  const PartJob* parts;        // [n_parts]
  const uint64_t* const_limbs;
  const SlotRef* regs;         // the design's register refs (fields within one copy)
  char* state;                 // copy of (instance i, partition p) at (i n_parts + p) pitch
  const uint64_t* seeds;
  const DevCtl* ctl;
  uint64_t* xch;               // [2][n_inst][reg_words]: published register values
  unsigned long long* acc;     // [3][n_inst]: digest sums, by cycle mod 3 (zero at launch)
  uint64_t* digest;            // [n_inst]
  GridSync* gs;
  uint64_t pitch;              // bytes of one copy
  uint64_t n_cycles;
  uint32_t n_parts, n_inst, reg_words, words_per_inst, spin_limit, pad;
};

// ---- kernel launchers (kernels.hip) ---------------------------------------
hipError_t launch_resident(const ResJob& J, uint32_t n_inst, uint32_t inst_base, uint32_t block,
                           bool lds_state, bool lds_ops, uint32_t unroll, hipStream_t s);
hipError_t launch_resident_multi(const ResJob* jobs, const uint2* map, uint32_t n_blocks,
                                 uint32_t block, bool lds_state, bool lds_ops, uint32_t unroll,
                                 size_t lds, hipStream_t s);
size_t resident_lds_bytes(const StateLayout& L, uint32_t n_ops_total, uint32_t n_layers,
                          bool lds_state, bool lds_ops);
// SWEEP, one layer: the common operations of arity n_src (launch_sweep_light,
// ranges r) and the heavy ones (launch_sweep_heavy, ly: the host copy of the
// layer record); either returns without launching when its ranges are empty.
hipError_t launch_sweep_light(const Program& p, const StateLayout& L, char* state,
                              const OpRanges& r, uint32_t n_src, uint32_t ops_per_wave,
                              uint32_t unroll, uint32_t tiles_per_wave, TilePass tp,
                              hipStream_t s);
hipError_t launch_sweep_heavy(const Program& p, const StateLayout& L, char* state,
                              const uint64_t* seeds, const DevCtl* ctl, uint32_t n_inst,
                              uint32_t layer, const DevLayer& ly, uint32_t ops_per_wave,
                              uint32_t tiles_per_wave, TilePass tp, hipStream_t s);
// LAYERED: layer li (n_layer_ops >= 1 operations) of n_inst instances,
// blocks of `block` threads (64, 128, 192 or 256).
hipError_t launch_layer(const ResJob& J, uint32_t li, uint32_t n_layer_ops, uint32_t n_inst,
                        uint32_t block, uint32_t unroll, hipStream_t s);
hipError_t launch_advance(DevCtl* ctl, uint64_t n, hipStream_t s);
// LAYERED, persistent: all J.n_cycles cycles of n_inst instances in one
// cooperative launch, every layer spread over the whole grid and followed by
// a grid-wide barrier; the register digest after every cycle (acc: one
// zeroed word per instance).  gs is zeroed by this call first.  blocks = 0:
// as many blocks of 256 threads as are resident at once (at most two per
// compute unit); spin_limit bounds every barrier wait.
hipError_t launch_layer_persistent(const ResJob& J, uint32_t n_inst, uint32_t unroll,
                                   GridSync* gs, uint64_t* acc, uint32_t spin_limit,
                                   uint32_t blocks, hipStream_t s);
// PARTITIONED: R.n_cycles cycles of R.n_inst instances in one cooperative
// launch of n_inst x n_parts workgroups of `block` threads (R.acc and R.gs
// are cleared by this call first).  lds_state: each copy in LDS.  Fails
// (hipErrorCooperativeLaunchTooLarge or similar) when the workgroups cannot
// all be resident at once.
hipError_t launch_partitioned(const PartRun& R, uint32_t block, bool lds_state, hipStream_t s);
// Workgroups of `block` threads with `lds` bytes of LDS each that the device
// holds at once (0 on error).
uint32_t partitioned_capacity(uint32_t block, bool lds_state, size_t lds);

// Launches over several batches: segs[0 .. n_seg) and wave0[0 .. n_seg] in
// device memory, wave0 the prefix of the segments' wavefronts (n_waves =
// wave0[n_seg]), followed by the segment of every wavefront
// (wave0[n_seg + 1 + w], w < n_waves).  kind 0: SWEEP common operations (tile group tg: 1, 2, 4,
// 8 or 16), 1: SWEEP heavy (tg 1 or 2), 2: fused mux chains (tg 1, 2 or 4),
// 3: LAYERED (tg ignored), 4: mixed, each segment of its own kind and tile
// group (its variant; common operations with tile groups up to 4), so that
// the small pieces of one layer index need one launch instead of one per
// kind and tile group; 5: the same for the variants of small register
// footprint only (multi_lean); 6: the lean variants without LAYERED pieces
// and with at most 2 common operations in flight, smaller still.  narrow:
// heavy pieces of a design with no value wider than 128 bits, which run in
// the two-limb form only (lean with tile groups up to 2; variant + 256).
bool multi_mixable(uint32_t kind, uint32_t tg);
bool multi_lean(uint32_t kind, uint32_t tg, bool narrow = false);
uint32_t multi_variant(uint32_t kind, uint32_t tg, uint32_t unroll, bool lean, bool narrow = false);
hipError_t launch_multi(uint32_t kind, uint32_t tg, const MultiSeg* segs, const uint32_t* wave0,
                        uint32_t n_seg, uint64_t n_waves, hipStream_t s);
// Register digest of several batches, then their folds and cycle advance
// (every batch: D = s(D ^ acc), acc = 0, cycle + 1); max_inst: the largest
// n_inst among them.
hipError_t launch_digest_multi(const DigestSeg* segs, const uint32_t* wave0, uint32_t n_seg,
                               uint64_t n_waves, uint32_t max_inst, hipStream_t s);
// The digest's chunking of one batch: units (tiles or instances) and
// registers per wavefront; wavefronts = units x ceil(n_regs / per).
void digest_shape(bool sweep, uint32_t n_regs, uint32_t n_inst, uint32_t* n_units, uint32_t* per);
hipError_t launch_set_words(DevCtl* ctl, const uint64_t* words, hipStream_t s);
hipError_t launch_pack(bool sweep, const StateLayout& L, const char* state, const SlotRef* refs,
                       uint32_t n_refs, uint32_t words_per_inst, uint32_t first, uint32_t n,
                       uint64_t* out, hipStream_t s);
hipError_t launch_unpack(bool sweep, const StateLayout& L, char* state, const SlotRef* refs,
                         uint32_t n_refs, uint32_t words_per_inst, uint32_t first, uint32_t n,
                         const uint64_t* in, hipStream_t s);
size_t resident_max_lds();

// One record of a batch's change log (the layout of the public rteaal_change).
struct ChangeRec {
  uint64_t cycle;
  uint32_t instance, signal;
  uint64_t value[4];
};
static_assert(sizeof(ChangeRec) == 48, "ChangeRec layout");

// Value-change capture after a cycle: for every instance and watched signal
// (refs, out_off = the signal's first limb row in shadow), compare the stored
// value with shadow (signal-major: limb row k holds the n_inst copies at
// shadow[k * n_inst ...]), update shadow and append a ChangeRec when it
// differs.  *count counts every change; records at positions >= cap are not
// stored.  The record's cycle is ctl->cycle.  With init, shadow is filled
// from the state and nothing is recorded.
hipError_t launch_capture(bool sweep, const StateLayout& L, const char* state, const SlotRef* refs,
                          uint32_t n_refs, uint64_t* shadow, uint32_t n_inst, bool init,
                          const DevCtl* ctl, ChangeRec* log, uint64_t cap,
                          unsigned long long* count, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);

// Register digest after a cycle's commit, for the SWEEP and RESIDENT
// layouts (RESIDENT batches fold it inside k_resident instead).  With
// s = SplitMix64's output function and v[j][l] limb l of register j:
//   h = sum over j, l of s(s(4 j + l) ^ v[j][l])   (mod 2^64)
//   D = s(D ^ h).
// launch_digest adds the terms of every register into acc[inst] (zero on
// entry) and then folds acc into digest[inst] and clears acc again, for
// instances [0, n_inst).
hipError_t launch_digest(bool sweep, const StateLayout& L, const char* state, const SlotRef* regs,
                         uint32_t n_regs, uint32_t n_inst, uint64_t* digest, uint64_t* acc,
                         hipStream_t s);

}  // namespace rteaal
