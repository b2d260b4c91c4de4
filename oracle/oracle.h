/*
 * Plain CPU oracle for RTL simulation as a cascade of extended Einsums.
 *
 * TEST INFRASTRUCTURE ONLY.  The GPU library never links, includes or calls
 * this code; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no source with the GPU path.
 *
 * What it computes (paper, section "RTL Simulation as a Cascade of Einsums",
 * Cascade 1, and the example kernel Alg. RU): per instance and per clock
 * cycle, the primary inputs are written into the signal vector LI, every
 * layer i of the levelized dataflow graph gathers its operands through the
 * operation-input mask (OI = LI . OIM), applies the map / reduce / populate
 * operators op_u[n], op_r[n], op_s[n] of its operation type n, and the layer
 * outputs LO are written back into LI; at the end of the cycle all registers
 * latch their next-state slots simultaneously.  Values are unsigned, at most
 * 256 bits, held as four little-endian 64-bit limbs.
 */
#ifndef RTEAAL_ORACLE_H
#define RTEAAL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_LIMBS 4

/* Rank-N coordinates (operation types). */
enum {
  ORC_AND = 0, ORC_OR, ORC_XOR, ORC_NOT, ORC_ADD, ORC_SUB, ORC_MUL, ORC_MUX,
  ORC_EQ, ORC_LT, ORC_SHL, ORC_SHR, ORC_EXTRACT, ORC_CONCAT, ORC_ORR,
  ORC_DIV, ORC_REM, ORC_DSHL, ORC_DSHR, ORC_ANDR, ORC_XORR, ORC_SEXT, ORC_MUXC, ORC_NTYPES
};

/* Longest O fiber of one operation: a mux chain of 32 (selector, value)
 * pairs and its default. */
#define ORACLE_MAX_ARITY 65

typedef struct {
  uint32_t n_slots;   const uint16_t* slot_width;
  uint32_t n_consts;  const uint32_t* const_slot; const uint64_t* const_limbs; /* [n_consts][4] */
  uint32_t n_inputs;  const uint32_t* input_slot;
  uint32_t n_regs;    const uint32_t* reg_slot;   const uint32_t* reg_next;
  uint32_t n_layers;  const uint32_t* layer_ptr;  /* [n_layers + 1] */
  uint32_t n_ops;     const uint8_t*  op_type;    const uint32_t* op_dst;
                      const uint32_t* op_src_ptr; /* [n_ops + 1] */
                      const uint32_t* op_src;     const uint16_t* op_imm;
} oracle_design;

typedef struct {
  uint32_t n_inst;            const uint64_t* seeds;        /* [n_inst] */
  uint64_t start_cycle;       uint64_t n_cycles;
  int32_t  stim_mode;         /* 0: counter-based generator; 1: stim_words */
  const uint64_t* stim_words; /* [n_cycles][n_inst][sum of input limbs] */
  const uint64_t* init_regs;  /* NULL (reset to 0) or [n_inst][n_regs][4] */
  uint64_t* out_regs;         /* [n_inst][n_regs][4] */
  uint64_t* out_slots;        /* NULL or [n_inst][n_slots][4] */
  int32_t  trace_reg;         /* -1, or a register index traced below */
  uint64_t* trace;            /* [n_inst][n_cycles]: limb 0 of that register after each cycle */
  int32_t  n_threads;
  const uint64_t* init_digest;  /* NULL (0) or [n_inst]: digest before the first cycle */
  uint64_t* out_digest;         /* NULL or [n_inst]: digest after the last cycle */
  uint64_t* digest_trace;       /* NULL or [n_inst][n_cycles]: digest after each cycle */
} oracle_run_args;

/* Per-instance register digest (a reading of what "state" is compared: the
 * paper commits the registers once per cycle, Cascade 2's cycle rank C).
 * It starts at 0; after every cycle's register commit, with v[j][l] limb l
 * of register j (l < ceil(width/64)) and s the SplitMix64 output function,
 *   h = sum over j, l of s(s(4 j + l) ^ v[j][l])   (mod 2^64)
 *   D = s(D ^ h).
 * The sum makes h independent of the order registers are visited in; the
 * outer s makes D depend on every cycle's register vector, in order. */

/* Returns 0, or a negative code if an index is out of range. */
int oracle_run(const oracle_design* d, const oracle_run_args* a);

/* One operation on explicit operands ([arity][4] limbs, already within their
 * widths); writes the 4-limb result masked to dst_w.  Returns 0 or -1. */
int oracle_eval_op(int type, int arity, const uint64_t* operands, const uint16_t* src_w,
                   int dst_w, int imm, uint64_t* out);

/* Stimulus word: SplitMix64 output function applied three times,
 * s(s(s(seed) ^ cycle) ^ ((input << 8) | limb)). */
uint64_t oracle_stim(uint64_t seed, uint64_t cycle, uint32_t input, uint32_t limb);

/* The SplitMix64 output function for generator state x (first output). */
uint64_t oracle_splitmix64(uint64_t x);

#ifdef __cplusplus
}
#endif
#endif
