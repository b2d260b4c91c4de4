/*
 * rteaal.h -- C interface of the MI355X (gfx950) RTL-simulation library.
 *
 * The library evaluates the per-cycle cascade of extended Einsums of the
 * paper (section "RTL Simulation as a Cascade of Einsums", Cascade 1) for a
 * levelized dataflow graph: in every clock cycle the primary inputs are
 * written into the signal vector LI, every layer i (iterative rank I)
 * gathers its operands through the operation-input mask OIM, applies the
 * operator of its operation type (ranks N and O: map op_u, reduce op_r,
 * populate op_s) and writes its layer outputs LO back into LI at the
 * operation's S coordinate (identity operations elided, section "Identity
 * Operator Elision"); at the end of the cycle every register latches its
 * next-state value, all at once.
 *
 * Conventions for every call:
 *   - Every entry point returns an rteaal_status.  On any error the call has
 *     no side effects, and rteaal_last_error() describes the failure.
 *   - Pointers marked "host" are ordinary host memory, borrowed for the
 *     duration of the call unless stated otherwise.  The library copies what
 *     it keeps.
 *   - Device memory is obtained through the allocator given to
 *     rteaal_create (or hipMalloc) and released by rteaal_unload_design,
 *     rteaal_free_batch or rteaal_destroy.
 *   - rteaal_step and rteaal_step_many only enqueue work on the context's
 *     stream; rteaal_sync and rteaal_read_state wait for it.
 *   - A context is used by one host thread at a time.
 *   - Values are unsigned; a w-bit value is ceil(w/64) little-endian 64-bit
 *     limbs with the bits above w equal to zero.
 */
#ifndef RTEAAL_H
#define RTEAAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RTEAAL_OK = 0,
  RTEAAL_E_INVALID_ARG = 1, /* null pointer, bad handle, size out of range   */
  RTEAAL_E_BAD_DESIGN = 2,  /* graph violates levelization, arity, widths ...  */
  RTEAAL_E_FORMAT = 3,      /* a coordinate does not fit its declared cbits    */
  RTEAAL_E_NO_MEMORY = 4,   /* device allocation failed; nothing was created   */
  RTEAAL_E_DEVICE = 5,      /* a HIP call failed; destroy the context          */
  RTEAAL_E_BUSY = 6,        /* handle still in use by a pending step           */
  RTEAAL_E_UNSUPPORTED = 7  /* valid request this build cannot serve           */
} rteaal_status;

typedef struct rteaal_ctx rteaal_ctx;
typedef uint32_t rteaal_design_id;
typedef uint32_t rteaal_batch_id;

/* Device-memory provider.  alloc returns a device pointer aligned to at
 * least 256 bytes, or NULL; free releases it.  Both run on the calling
 * thread, outside any kernel. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, size_t bytes, void* user);
  void* user;
} rteaal_allocator;

/* Context on HIP device `device`.  `stream` is a hipStream_t (NULL: the
 * library creates its own non-blocking stream at default priority).
 * `alloc` may be NULL (hipMalloc / hipFree). */
rteaal_status rteaal_create(int device, void* stream, const rteaal_allocator* alloc,
                            rteaal_ctx** out);
/* Waits for pending work, then frees every design and batch.  NULL is a no-op. */
void rteaal_destroy(rteaal_ctx* ctx);
/* Text of the last failure on ctx (or of the last context-less failure when
 * ctx is NULL); valid until the next call on the same context. */
const char* rteaal_last_error(const rteaal_ctx* ctx);

/* ------------------------------------------------------------------------ */
/* Designs                                                                  */
/* ------------------------------------------------------------------------ */

/* Rank-N coordinates.  AND/OR/XOR take 2 or 3 operands (the O fiber's
 * occupancy, fixed per (type, arity)); NOT/SHL/SHR/EXTRACT/ORR/ANDR/XORR/SEXT
 * take 1; ADD/SUB/MUL/EQ/LT/CONCAT/DIV/REM/DSHL/DSHR take 2; MUX takes 3.
 * Results (all unsigned, computed on zero-extended operands, then reduced
 * modulo 2^dst_width):
 *   AND/OR/XOR  fold over operands       NOT      bitwise complement
 *   ADD, SUB    o0 + o1, o0 - o1         MUL      o0 * o1 (low bits)
 *   MUX         o0 != 0 ? o1 : o2        EQ, LT   [o0 == o1], [o0 < o1]
 *   SHL, SHR    o0 shifted by imm        EXTRACT  o0 >> imm (width from dst)
 *   CONCAT      o0 * 2^width(o1) + o1    ORR      [o0 != 0]
 *   DIV, REM    o0 / o1, o0 mod o1 (o1 = 0 gives 0 and o0)
 *   DSHL, DSHR  o0 * 2^o1, o0 / 2^o1     ANDR     [o0 = 2^width(o0) - 1]
 *   XORR        parity of o0             SEXT     o0 read as a width(o0)-bit
 *                                                 two's-complement number
 * With these, every FIRRTL primitive operation maps onto one type or a short
 * chain: bits/head/tail/pad/cvt/as* are EXTRACT or SEXT, leq/gt/geq/neq are
 * LT/EQ with swapped operands or NOT, neg is SUB from a zero literal, and
 * the signed forms of add/sub/mul/lt/shr/div/rem run on SEXT-extended
 * operands (lt after flipping both sign bits with XOR).
 * Operand o=0 is reduced first, as the left operand (section "Evaluating
 * Multiple Operation Types"); MUX is the select operator op_s of Appendix A.
 * MUXC is the fused mux chain of the compiler's operator fusion (section
 * "Design Overview" of the simulator; App. B, "Implemented Optimizations"):
 * an odd number 3 .. 2 RTEAAL_MUXC_MAX_PAIRS + 1 of operands, read as
 * (selector, value) pairs and a default; the value of the first pair whose
 * selector is nonzero, else the default (one pair: MUX).  rteaal_fuse_mux_chains
 * forms them from MUX chains. */
typedef enum {
  RTEAAL_AND = 0, RTEAAL_OR, RTEAAL_XOR, RTEAAL_NOT, RTEAAL_ADD, RTEAAL_SUB, RTEAAL_MUL,
  RTEAAL_MUX, RTEAAL_EQ, RTEAAL_LT, RTEAAL_SHL, RTEAAL_SHR, RTEAAL_EXTRACT, RTEAAL_CONCAT,
  RTEAAL_ORR, RTEAAL_DIV, RTEAAL_REM, RTEAAL_DSHL, RTEAAL_DSHR, RTEAAL_ANDR, RTEAAL_XORR,
  RTEAAL_SEXT, RTEAAL_MUXC, RTEAAL_OP_COUNT
} rteaal_op;
enum { RTEAAL_MUXC_MAX_PAIRS = 32 };

/* Per-rank format (section "Format": uncompressed or compressed, coordinate
 * and payload bit widths). */
typedef struct {
  uint8_t compressed;
  uint8_t cbits;
  uint8_t pbits;
} rteaal_rank_format;

/* Format of one layer's OIM slice in the swizzled rank order [I,N,S,O,R]
 * (section "Compressing the OIM Format", format (c)), plus the LI and LO
 * vectors.  Passing NULL for the whole array lets the library derive every
 * field from the maximum coordinate and payload values; a caller-supplied
 * format is checked (RTEAAL_E_FORMAT when a coordinate or payload does not
 * fit) and recorded. */
typedef struct {
  rteaal_rank_format oim[5]; /* I, N, S, O, R */
  rteaal_rank_format li, lo;
} rteaal_layer_format;

/* A levelized design.  Slots are the coordinates of LI (ranks R and S after
 * identity elision).  Every slot has exactly one driver: a constant, a
 * primary input, a register, or one operation; slots with no driver must
 * not be read.  Operations of layer i may read constants, inputs, registers
 * and slots driven by layers < i.  All arrays are host memory, borrowed for
 * the call. */
typedef struct {
  uint32_t n_slots;        const uint16_t* slot_width;   /* [n_slots], 1..256 bits   */
  uint32_t n_consts;       const uint32_t* const_slot;   /* [n_consts]               */
                           const uint64_t* const_limbs;  /* [n_consts][4]            */
  uint32_t n_inputs;       const uint32_t* input_slot;   /* [n_inputs], stimulus order */
  uint32_t n_regs;         const uint32_t* reg_slot;     /* [n_regs] register Q slots */
                           const uint32_t* reg_next;     /* [n_regs] latched slot     */
  uint32_t n_layers;       const uint32_t* layer_op_ptr; /* [n_layers+1], rank-I payloads */
  uint32_t n_ops;          const uint8_t*  op_type;      /* [n_ops] rank-N coordinate */
                           const uint32_t* op_dst;       /* [n_ops] S coordinate      */
                           const uint32_t* op_src_ptr;   /* [n_ops+1] O-fiber extents */
                           const uint32_t* op_src;       /* R coordinates in O order  */
                           const uint16_t* op_imm;       /* [n_ops] shift / low bit, else 0 */
  const rteaal_layer_format* layer_fmt;                  /* [n_layers] or NULL        */
} rteaal_design_desc;

/* Checks a design on the host only (no device needed).  On failure writes a
 * NUL-terminated reason into err (if err_len > 0) and returns
 * RTEAAL_E_BAD_DESIGN, RTEAAL_E_FORMAT or RTEAAL_E_INVALID_ARG. */
rteaal_status rteaal_validate_design(const rteaal_design_desc* desc, char* err, size_t err_len);

/* ------------------------------------------------------------------------ */
/* Levelization                                                             */
/* ------------------------------------------------------------------------ */

/* A dataflow graph with its operations in any order (paper section
 * "Evaluating Arbitrary Dataflow Graphs": levelization slices the graph into
 * layers before the cascade is formed).  Operation o reads the slots
 * op_src[op_src_ptr[o] .. op_src_ptr[o+1]) and writes slot op_dst[o].  A slot
 * that no operation writes is a source (primary input, register or
 * constant), available before the first layer.  All arrays are host memory. */
typedef struct {
  uint32_t n_slots;
  uint32_t n_ops;
  const uint32_t* op_src_ptr; /* [n_ops + 1], op_src_ptr[0] = 0, non-decreasing */
  const uint32_t* op_src;     /* [op_src_ptr[n_ops]] slots read, each < n_slots  */
  const uint32_t* op_dst;     /* [n_ops] slot written, each < n_slots            */
} rteaal_dag_desc;

/* Levelizes a graph on the context's device: operation o gets layer 1 + the
 * largest layer among the operations producing its operands, and layer 0
 * when all its operands are sources.  This is the levelization with the
 * fewest layers (the graph's depth); every operation reads only sources and
 * values of earlier layers, and every layer is non-empty.
 * Outputs, host memory allocated by the caller:
 *   op_layer  [n_ops]     layer of each operation;
 *   order     [n_ops]     operation indices sorted by (layer, index);
 *   layer_ptr [n_ops + 1] order[layer_ptr[i] .. layer_ptr[i+1]) is layer i
 *                         (entries past n_layers are left untouched);
 *   n_layers              number of layers (0 when n_ops = 0).
 * A design in this order (layer_ptr as its layer ranges) passes
 * rteaal_validate_design's levelization check.  Errors (outputs then
 * unspecified): RTEAAL_E_INVALID_ARG for a null pointer, n_ops >= 2^31, a
 * decreasing op_src_ptr or a slot index out of range; RTEAAL_E_BAD_DESIGN
 * when a slot is written by two operations or the graph has a cycle (the
 * message names the slot, or an operation on or behind the cycle);
 * RTEAAL_E_NO_MEMORY when the device scratch (about 13 words per operation
 * plus 2 per operand entry and 1 per slot) cannot be allocated. */
rteaal_status rteaal_levelize(rteaal_ctx* ctx, const rteaal_dag_desc* dag, uint32_t* op_layer,
                              uint32_t* order, uint32_t* layer_ptr, uint32_t* n_layers);

/* ------------------------------------------------------------------------ */
/* Operator fusion                                                          */
/* ------------------------------------------------------------------------ */

/* Counts of one mux-chain fusion. */
typedef struct {
  uint32_t n_ops;       /* operations in the fused design                     */
  uint32_t n_operands;  /* operand entries (op_src_ptr[n_ops])                */
  uint32_t n_fused;     /* MUXC operations formed                             */
  uint32_t n_absorbed;  /* MUX operations removed into them                   */
} rteaal_fuse_result;

/* Mux-chain fusion (operator fusion by mux-chain extraction, among the
 * compiler's dataflow-graph optimizations in section "Design Overview" of the
 * simulator; App. B "Implemented Optimizations", operator fusion), host only.
 * MUX m (s ? v : x) absorbs MUX m' when x is the slot m' writes, that slot
 * has exactly one operand reader in the design (m), no register latches it,
 * and its width is at least m's destination width; then no remaining value
 * changes.  Each path of such links, from its outermost MUX inward, becomes
 * MUXC operations of at most max_pairs (1 .. RTEAAL_MUXC_MAX_PAIRS) pairs
 * (s1, v1, ..., sk, vk, default), in the outermost MUX's place (layer and
 * position); a longer path continues with the MUX its default reads.  The
 * absorbed MUXes disappear and their slots are no longer written (a later
 * RTEAAL_READ_ALL_SLOTS reads them as 0).  Slots, registers, inputs and
 * constants are unchanged, so the fused design is `desc` with the arrays
 * below in place of its operation arrays; rteaal_levelize may then shorten
 * it, since a fused operation often reads only earlier layers.
 * Outputs, host memory allocated by the caller (a fused design never has
 * more operations or operand entries than its input):
 *   layer_op_ptr [n_layers + 1]; op_type, op_dst, op_imm [n_ops];
 *   op_src_ptr [n_ops + 1]; op_src [desc->op_src_ptr[n_ops]].
 * Errors: RTEAAL_E_INVALID_ARG (null pointer, max_pairs out of range) and
 * the errors of rteaal_validate_design (the input must pass it); the
 * outputs are then unspecified. */
rteaal_status rteaal_fuse_mux_chains(const rteaal_design_desc* desc, uint32_t max_pairs,
                                     uint32_t* layer_op_ptr, uint8_t* op_type, uint32_t* op_dst,
                                     uint32_t* op_src_ptr, uint32_t* op_src, uint16_t* op_imm,
                                     rteaal_fuse_result* result);

/* Validates, encodes (operations grouped per layer by destination width
 * class and type, as in the N-rank swizzle of the NU kernel) and uploads a
 * design.  *out receives a handle valid until rteaal_unload_design.
 * Storage is assigned by live range: a value's storage is reused once every
 * operation that reads it has run (registers keep theirs), which shrinks an
 * instance's state to the largest set of values live at a layer boundary.
 * Such a design supports RTEAAL_READ_REGS read-out only. */
rteaal_status rteaal_load_design(rteaal_ctx* ctx, const rteaal_design_desc* desc,
                                 rteaal_design_id* out);

/* As rteaal_load_design with flags: RTEAAL_LOAD_KEEP_ALL_SLOTS gives every
 * slot storage of its own for the whole cycle, so that RTEAAL_READ_ALL_SLOTS
 * can read every signal (a debugging aid: more memory and traffic). */
enum { RTEAAL_LOAD_KEEP_ALL_SLOTS = 1 };
rteaal_status rteaal_load_design_ex(rteaal_ctx* ctx, const rteaal_design_desc* desc,
                                    uint32_t flags, rteaal_design_id* out);
/* RTEAAL_E_BUSY while a batch of the design exists. */
rteaal_status rteaal_unload_design(rteaal_ctx* ctx, rteaal_design_id design);

/* Derived format of layer `layer` of a loaded design (see rteaal_layer_format). */
rteaal_status rteaal_design_format(rteaal_ctx* ctx, rteaal_design_id design, uint32_t layer,
                                   rteaal_layer_format* out);

/* ------------------------------------------------------------------------ */
/* Batches of instances                                                     */
/* ------------------------------------------------------------------------ */

/* Mapping of a batch onto the GPU.
 *   RESIDENT: one workgroup per instance, one lane per operation, the
 *             instance's signal vector in LDS when it fits, else in HBM; all
 *             cycles of a step in one launch with a workgroup barrier per
 *             layer.  The plain single-instance form.
 *   SWEEP:    one lane per instance (64 instances per wavefront, 1-bit
 *             signals bit-sliced into 64-bit words), operation records read
 *             once per wavefront for one to eight 64-instance tiles; per
 *             layer one launch for the operations whose values fit 64 bits
 *             (one per operand count in large layers) and one for the rest
 *             (wider values, the types DIV .. SEXT, the sources), the cycle
 *             captured in a HIP graph.  The batched form, and the plain form
 *             of large designs.
 *   LAYERED:  one lane per operation as in RESIDENT, but each layer is one
 *             launch over the whole device (blocks of block_threads x unroll
 *             operations, times the instances), the state in HBM, the cycle
 *             captured in a HIP graph.  The plain form of large designs (a single instance's
 *             layer spread over every compute unit); at most 65535
 *             instances.
 *   PARTITIONED: the replicated register partitioning of App. C (Cascade 2
 *             with the partition rank): the registers are split into
 *             `partitions` contiguous blocks; each (instance, partition) pair
 *             is one workgroup that holds its own copy of the instance's
 *             state (in LDS when it fits) and evaluates only the fan-in
 *             cones of its registers, the operations shared by several
 *             cones replicated in each.  Once per cycle the partitions
 *             publish their registers, meet at a grid-wide barrier and load
 *             the registers their cones read from other partitions.  All
 *             workgroups must be resident at once (a cooperative launch of
 *             n_instances x partitions workgroups); a barrier wait is
 *             bounded as for persistent LAYERED.  The plain form of a
 *             design too large for one workgroup's lanes but whose cones
 *             replicate little.  Not watchable; RTEAAL_READ_ALL_SLOTS is
 *             unsupported.
 *   AUTO:     the autotuner's choice for (design, n_instances) when
 *             rteaal_autotune has run for them, else RESIDENT below 32
 *             instances and SWEEP from 32 on. */
enum {
  RTEAAL_MAP_AUTO = 0,
  RTEAAL_MAP_RESIDENT = 1,
  RTEAAL_MAP_SWEEP = 2,
  RTEAAL_MAP_LAYERED = 3,
  RTEAAL_MAP_PARTITIONED = 4
};

typedef struct {
  uint32_t mapping;        /* RTEAAL_MAP_*                                      */
  uint32_t block_threads;  /* 0 = default; RESIDENT: 64..1024, multiple of 64;
                              LAYERED: 64..256, multiple of 64 (default 64)     */
  uint32_t ops_per_wave;   /* 0 = default; SWEEP: operations per wavefront      */
  uint32_t lds_state;      /* RESIDENT: 0 = LDS when it fits, 1 = keep in HBM   */
  uint32_t lds_ops;        /* RESIDENT: 0 = records in LDS when they fit, 1 = no */
  uint32_t unroll;         /* 0 = default; operations in flight per lane or
                              wavefront: 1, 2 or 4 (RESIDENT, LAYERED, SWEEP)   */
  uint32_t tiles_per_wave; /* 0 = default; SWEEP: 64-instance tiles one
                              wavefront evaluates per decoded operation: 1, 2,
                              4, 8 or 16, with unroll x tiles_per_wave <= 8
                              (16 tiles: unroll 1)                             */
  uint32_t arity_split;    /* SWEEP: 0 = auto, 1 = never, 2 = always: run a
                              layer's common operations as one launch per
                              operand count (1, 2, 3), so absent operands cost
                              no loads or registers; auto splits the layers
                              with at least 2^20 operation x 64-instance tiles */
  uint32_t tiles_per_pass; /* SWEEP: 0 = all; else each cycle runs as passes
                              over this many 64-instance tiles at a time (a
                              multiple of tiles_per_wave), all layers of one
                              pass before the next, so that a pass's recent
                              layer outputs can stay in the last-level cache  */
  uint32_t persistent;     /* LAYERED: 0 = one launch per layer (a captured
                              cycle graph); 1 = one cooperative launch for up
                              to 1,024 cycles, every layer spread over the
                              whole device and ended by a grid-wide barrier
                              (the iterative rank I's advance, ◇ i≡I, inside
                              one launch); unroll 1 or 2.  A barrier wait is
                              bounded (environment RTEAAL_GRID_SPIN_LIMIT,
                              default 2^22 spins); if one runs out, the next
                              rteaal_sync or rteaal_read_state on the batch
                              returns RTEAAL_E_DEVICE                          */
  uint32_t partitions;     /* PARTITIONED: 0 = default (256 / n_instances, at
                              most one per register); else 1 .. 1024 register
                              partitions.  block_threads (64..1024, multiple
                              of 64, default from the largest sub-program
                              layer) and lds_state apply as for RESIDENT      */
  uint32_t pass_branches;  /* SWEEP with tiles_per_pass: 0 = the passes run
                              one after another; 1 = each pass is a branch of
                              its own in the captured cycle graph (its layers
                              in order), the branches running side by side
                              and joining before the register digest; at most
                              4 passes                                        */
} rteaal_batch_opts;

/* Device bytes a batch of n_instances of `design` would allocate under
 * `opts` (NULL = AUTO), for admission control. */
rteaal_status rteaal_batch_footprint(rteaal_ctx* ctx, rteaal_design_id design,
                                     uint32_t n_instances, const rteaal_batch_opts* opts,
                                     uint64_t* bytes);

/* Device resources a batch would hold, for admission control by memory and
 * LDS: *hbm_bytes as rteaal_batch_footprint, and *lds_bytes the LDS its
 * kernels keep for a whole step (RESIDENT: its workgroups' LDS, state and
 * program records when they fit, times the instances; 0 for SWEEP and
 * LAYERED, which keep no LDS across a step). */
rteaal_status rteaal_batch_resources(rteaal_ctx* ctx, rteaal_design_id design,
                                     uint32_t n_instances, const rteaal_batch_opts* opts,
                                     uint64_t* hbm_bytes, uint64_t* lds_bytes);

/* The partitioned form of a loaded design for `partitions` register
 * partitions (RTEAAL_MAP_PARTITIONED; App. C, the replicated partitioning
 * of Cascade 2), computed on the host without touching the device:
 *   design_ops   operations of the design's encoded program (the sources,
 *                layers and register commit),
 *   cone_ops     operations summed over the partitions' cones (an operation
 *                in k cones counts k times): cone_ops / design_ops is the
 *                work the replication costs per cycle,
 *   padded_ops   cone_ops plus the operations evaluated only because they
 *                share a 64-destination 1-bit group with a cone operation,
 *   max_part_ops the largest partition's operations (padded): the per-cycle
 *                critical path in operations,
 *   exchange     register limbs loaded per cycle, summed over partitions.
 * Errors: RTEAAL_E_INVALID_ARG (unknown design, partitions 0 or above the
 * register count or 1024). */
typedef struct {
  uint64_t design_ops, cone_ops, padded_ops, max_part_ops, exchange;
} rteaal_partition_stats;
rteaal_status rteaal_partition_plan_stats(rteaal_ctx* ctx, rteaal_design_id design,
                                          uint32_t partitions, rteaal_partition_stats* out);

/* n_instances (>= 1) independent instances, registers reset to zero at
 * cycle 0; seeds[k] (host, [n_instances]) keys instance k's stimulus.
 * Allocates, then only enqueues the initialisation on the context's stream
 * (it does not wait for earlier work). */
rteaal_status rteaal_create_batch(rteaal_ctx* ctx, rteaal_design_id design,
                                  uint32_t n_instances, const uint64_t* seeds,
                                  const rteaal_batch_opts* opts, rteaal_batch_id* out);
rteaal_status rteaal_free_batch(rteaal_ctx* ctx, rteaal_batch_id batch);

/* Mapping actually used by a batch (one of RTEAAL_MAP_RESIDENT .. _PARTITIONED)
 * and its current cycle. */
rteaal_status rteaal_batch_info(rteaal_ctx* ctx, rteaal_batch_id batch, uint32_t* mapping,
                                uint64_t* cycle);

/* The launch shape a batch resolved to (defaults, autotuned entry or caller
 * options), written to *out in the form rteaal_create_batch takes, so that
 * passing *out back creates a batch of the same shape: mapping, and for
 * RESIDENT block_threads, lds_state/lds_ops (0 = in LDS, 1 = in HBM),
 * unroll; for SWEEP ops_per_wave, unroll, tiles_per_wave, arity_split,
 * tiles_per_pass (0 = all), pass_branches; for LAYERED block_threads, unroll, persistent;
 * for PARTITIONED block_threads, lds_state, partitions (other fields 0). */
rteaal_status rteaal_batch_options(rteaal_ctx* ctx, rteaal_batch_id batch, rteaal_batch_opts* out);

/* ------------------------------------------------------------------------ */
/* Stepping                                                                 */
/* ------------------------------------------------------------------------ */

/* Primary-input values for a step.
 *   mode 0 (generator): input k of instance j in cycle c gets the limbs
 *     s(s(s(seed_j) ^ c) ^ ((k << 8) | limb)), s = SplitMix64's output
 *     function, reduced to the input's width.  No memory traffic.
 *   mode 1 (words): `words` holds [n_cycles][n_instances][W] limbs, W the sum
 *     of ceil(width/64) over inputs in stimulus order; host memory (copied
 *     during the call) or, with words_on_device, device memory that must stay
 *     valid until the step has completed. */
typedef struct {
  uint32_t mode;
  uint32_t words_on_device;
  const uint64_t* words;
} rteaal_stimulus;

/* Advances every instance of `batch` by n_cycles (>= 0): per cycle, the
 * primary inputs are written into LI, the layers run in order (the iterative
 * rank I of Cascade 1; each layer gathers its operands, applies its
 * operators and writes LO back into LI, as the example kernel Alg. RU does),
 * and then every register commits (Cascade 2's cycle rank C) and the
 * register digest advances.  stim may be NULL (mode 0).  Enqueue only,
 * except that host words are copied before the call returns.  Errors:
 * RTEAAL_E_INVALID_ARG (unknown batch, bad stimulus), RTEAAL_E_NO_MEMORY,
 * RTEAAL_E_DEVICE (the context is then unusable). */
rteaal_status rteaal_step(rteaal_ctx* ctx, rteaal_batch_id batch, uint64_t n_cycles,
                          const rteaal_stimulus* stim);

/* Advances n batches (possibly of different designs) by n_cycles[k] each, as
 * rteaal_step does for one (every batch runs the cascade of Cascade 1 and
 * its register commit per cycle; the host supplies primary inputs between
 * cycles as in section "System Integration").  batches[k] are distinct.
 * stims: NULL (generator stimulus for every batch) or host array [n],
 * stims[k] being batch k's stimulus as in rteaal_step (words
 * [n_cycles[k]][n_instances][W] of that batch).  Enqueue only, except that
 * host words are copied before the call returns (it then waits for the
 * step).  How the work is laid out: all RESIDENT batches advance in one
 * persistent launch per kernel configuration, the configurations on up to
 * four streams; SWEEP and LAYERED batches advance together, beside them,
 * through one captured cycle per set of batches (the pieces of a layer
 * index in one mixed launch while they total at most
 * RTEAAL_MIXED_MAX_WAVES wavefronts, an environment variable, default
 * 2^20, 0 = never); cooperative batches (persistent LAYERED, PARTITIONED)
 * run last, one at a time, with nothing else of the call beside them.  The
 * context creates its auxiliary streams in a fixed order; with at least 8
 * hardware queues (HIP's GPU_MAX_HW_QUEUES, default 4) each gets its own,
 * and a chain of captured cycles never waits behind a RESIDENT launch.  Errors: RTEAAL_E_INVALID_ARG (unknown or repeated batch,
 * bad stimulus: then nothing has been enqueued), RTEAAL_E_NO_MEMORY,
 * RTEAAL_E_DEVICE (the context is then unusable). */
rteaal_status rteaal_step_many(rteaal_ctx* ctx, uint32_t n, const rteaal_batch_id* batches,
                               const uint64_t* n_cycles, const rteaal_stimulus* stims);

/* Waits until all enqueued work of ctx has completed. */
rteaal_status rteaal_sync(rteaal_ctx* ctx);

/* ------------------------------------------------------------------------ */
/* State                                                                    */
/* ------------------------------------------------------------------------ */
enum { RTEAAL_READ_REGS = 1, RTEAAL_READ_DIGEST = 2, RTEAAL_READ_ALL_SLOTS = 4 };

/* Register digest.  The paper commits every register once per cycle (the
 * cycle rank C of Cascade 2); the state compared between two simulators is
 * the register vector after every cycle.  Each instance keeps one running
 * 64-bit digest D of it, 0 at batch creation.  After every cycle's commit,
 * with v[j][l] limb l (l < ceil(width/64)) of register j (the order of
 * reg_slot) and s SplitMix64's output function (Steele, Lea & Flood, OOPSLA
 * 2014),
 *   h = sum over j, l of s(s(4 j + l) ^ v[j][l])   (mod 2^64),
 *   D = s(D ^ h).
 * Equal digests after n cycles mean (up to hash collisions) equal register
 * vectors after each of the n cycles, in order. */

/* Read-out of simulated state (the signal exposure of section "System
 * Integration": the host reads DUT signals between cycles).  Waits for the
 * batch, then copies instances [first, first+n) into `out` (host):
 *   REGS:      [inst][reg][limbs(reg)], registers in reg_slot order;
 *   DIGEST:    [inst], one word each: the register digest above;
 *   ALL_SLOTS: [inst][slot][limbs(slot)] (values of the last completed
 *              cycle; slots with no driver read as 0; only for designs
 *              loaded with RTEAAL_LOAD_KEEP_ALL_SLOTS, else
 *              RTEAAL_E_UNSUPPORTED).
 * `what` is exactly one of these.  out_words is the capacity of out in
 * uint64 words; *written (may be NULL) receives the number used.  Errors:
 * RTEAAL_E_INVALID_ARG (range, kind, capacity), RTEAAL_E_DEVICE. */
rteaal_status rteaal_read_state(rteaal_ctx* ctx, rteaal_batch_id batch, uint32_t first,
                                uint32_t n, uint32_t what, uint64_t* out, size_t out_words,
                                size_t* written);

/* rteaal_read_state for callers that cannot allocate device memory (code in
 * tight serving loops, harnesses that forbid allocation): the same results,
 * staged through a fixed device array of RTEAAL_NOALLOC_MAX_WORDS words
 * that the library holds on each device until the process ends, so the call
 * allocates nothing (no hipMalloc or allocator callback).  A read-out larger
 * than that array (words per instance x n) is rejected with
 * RTEAAL_E_INVALID_ARG; read fewer instances per call.  Every call on one
 * device shares that device's array: calls that overlap in time on one
 * device (other threads or contexts) race and must be serialized by the
 * caller.  RTEAAL_READ_DIGEST uses no staging. */
enum { RTEAAL_NOALLOC_MAX_WORDS = 1 << 20 };
rteaal_status rteaal_read_state_noalloc(rteaal_ctx* ctx, rteaal_batch_id batch, uint32_t first,
                                        uint32_t n, uint32_t what, uint64_t* out,
                                        size_t out_words, size_t* written);

/* Overwrites the registers of instances [first, first+n) from `regs` (host,
 * [inst][reg][limbs(reg)], masked to width) and sets the batch's cycle
 * counter to `cycle` (checkpoint restore, and the host writing DUT signals
 * between cycles: section "System Integration").  The digests are kept. */
rteaal_status rteaal_write_state(rteaal_ctx* ctx, rteaal_batch_id batch, uint32_t first,
                                 uint32_t n, const uint64_t* regs, uint64_t cycle);

/* Sets the register digest of instances [first, first+n) to digest[0..n)
 * (host), e.g. to restore a checkpoint taken with RTEAAL_READ_DIGEST.  Waits
 * for the batch.  Errors: RTEAAL_E_INVALID_ARG (range, null digest with
 * n > 0), RTEAAL_E_DEVICE. */
rteaal_status rteaal_write_digest(rteaal_ctx* ctx, rteaal_batch_id batch, uint32_t first,
                                  uint32_t n, const uint64_t* digest);

/* ------------------------------------------------------------------------ */
/* Waveforms                                                                */
/* ------------------------------------------------------------------------ */

/* One recorded transition: after `cycle` cycles (the batch's cycle counter
 * once that cycle had completed), signal `signal` (an index into the slots
 * given to rteaal_watch) of instance `instance` holds `value` (limbs, zero
 * above the signal's width), which differs from its value one cycle earlier. */
typedef struct {
  uint64_t cycle;
  uint32_t instance;
  uint32_t signal;
  uint64_t value[4];
} rteaal_change;

/* Value-change capture (paper section "System Integration", waveform
 * generation: a signal's transitions are found by comparing its value with
 * the one of the previous cycle).  Watches the slots slots[0 .. n) (host) in
 * every instance of the batch: from the call on, after every simulated cycle
 * each watched value that differs from its value after the previous cycle
 * (for the first cycle: its value at the call) is appended to the batch's
 * change log.  The log holds `capacity` records; further changes are counted
 * as dropped.  n = 0 stops watching and frees the log.  A later call replaces
 * the watch set and empties the log.  Register values written by
 * rteaal_write_state show up as changes of the next cycle when they differ.
 * Waits for the batch's pending steps.
 * Errors: RTEAAL_E_INVALID_ARG (slot out of range, null slots with n > 0);
 * RTEAAL_E_UNSUPPORTED when a slot other than a register is watched on a
 * design loaded without RTEAAL_LOAD_KEEP_ALL_SLOTS (its storage is shared
 * with other values, so it keeps no value across the cycle; the paper, too,
 * gives every signal its own coordinate for waveforms).
 * Cost: one thread per instance and watched signal after every cycle, and
 * RESIDENT batches run one cycle per launch while watched. */
rteaal_status rteaal_watch(rteaal_ctx* ctx, rteaal_batch_id batch, const uint32_t* slots,
                           uint32_t n, uint64_t capacity);

/* Moves the change log of a watched batch into out (host, room for max
 * records) and empties it; records come in no particular order.  Waits for
 * the batch's pending steps.  *n_out = records in the log (copied when
 * out != NULL), *n_dropped = changes lost to a full log since the last
 * drain.  With out = NULL or max = 0 only the counts are returned and the
 * log is kept.  RTEAAL_E_INVALID_ARG when max is smaller than the record
 * count (nothing is copied or emptied) or the batch is not watched. */
rteaal_status rteaal_read_changes(rteaal_ctx* ctx, rteaal_batch_id batch, rteaal_change* out,
                                  uint64_t max, uint64_t* n_out, uint64_t* n_dropped);

/* Autotuner: picks the mapping and launch shape for n_instances of `design`
 * on this device.  Each candidate (RESIDENT block sizes and unroll depths;
 * LAYERED block sizes and unroll depths, per layer and persistent, up to 16
 * instances; PARTITIONED partition counts up to 4 instances; SWEEP operations
 * per wavefront, unroll depths and tile groups of 1-16 tiles) runs `trial_cycles`
 * cycles (0 = a size-dependent default) on a temporary batch and is timed
 * with HIP events on the context's stream; candidates whose state does not
 * fit in device memory are skipped.  The fastest options are written to
 * *best (may be NULL) with their rate in instance-cycles/s in *rate (may be
 * NULL), and remembered: later rteaal_create_batch calls with mapping AUTO
 * for the same design and instance count use them.  Waits for the stream.
 * With the environment variable RTEAAL_AUTOTUNE_LOG set (and not "0"), every
 * candidate's shape and rate is printed to stderr. */
rteaal_status rteaal_autotune(rteaal_ctx* ctx, rteaal_design_id design, uint32_t n_instances,
                              uint32_t trial_cycles, rteaal_batch_opts* best, double* rate);

/* Joint autotuner for batches stepped together by rteaal_step_many (the
 * kernel configuration is an input of the simulator, section "Design
 * Overview", and its best choice varies by machine, Ablation Study 1): for
 * designs ids[0 .. n) with n_instances[k] instances each, tries launch
 * policies for the whole set (which batches run SWEEP and with which tile
 * group and operations per wavefront, which run RESIDENT or LAYERED) on
 * temporary batches, times
 * trial_cycles cycles (0 = a size-dependent default) of one rteaal_step_many
 * over all of them, and keeps the fastest policy: best (host [n], may be
 * NULL) receives each batch's options, *rate (may be NULL) the set's
 * instance-cycles/s, and AUTO batches created later for the same (design,
 * instance count) use them.  A (design, instance count) pair appears once.
 * With RTEAAL_AUTOTUNE_LOG set, every policy's rate goes to stderr.
 *
 * Both autotuners keep their results on disk when the environment variable
 * RTEAAL_TUNE_CACHE names a file: a later call for the same device,
 * designs (by a hash of their encoded programs), instance counts and trial
 * length reads the choice back instead of timing the candidates again. */
rteaal_status rteaal_autotune_many(rteaal_ctx* ctx, uint32_t n, const rteaal_design_id* ids,
                                   const uint32_t* n_instances, uint32_t trial_cycles,
                                   rteaal_batch_opts* best, double* rate);

/* ------------------------------------------------------------------------ */
/* Measurement                                                              */
/* ------------------------------------------------------------------------ */

/* Kernel timing of a batch.  While enabled, every launch of the simulation
 * kernels is bracketed by HIP events on the context's stream and issued
 * directly rather than through the captured graph.  Two kernels are counted
 * apart: [0] the main kernel (RESIDENT: one launch per chunk of cycles;
 * SWEEP: the kernel of a layer's common operations, values of at most 64
 * bits) and [1] the SWEEP kernel of a layer's heavy operations (wider values,
 * the types DIV .. SEXT and sources; always 0 for RESIDENT).  Each call waits for the stream,
 * writes launches[0..1] / total_ms[0..1] (host arrays of two; either pointer
 * may be NULL) with the launches and summed kernel time recorded since the
 * previous call, clears them, and then turns recording on (enable != 0) or
 * off. */
rteaal_status rteaal_kernel_timing(rteaal_ctx* ctx, rteaal_batch_id batch, int enable,
                                   uint64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* RTEAAL_H */
