/*
 * Stand-alone driver of the CPU oracle for sanitizer runs (test
 * infrastructure only): reads a design and a run description from a binary
 * file, runs oracle_run, and writes the final registers and register
 * digests.  The sanitizer test builds it together with oracle/oracle.c
 * under AddressSanitizer and UndefinedBehaviorSanitizer, so that every
 * memory access and integer operation of the oracle is checked on real
 * designs.
 *
 * Input (little-endian):
 *   u32 magic 0x524f5452, n_slots, n_consts, n_inputs, n_regs, n_layers,
 *       n_ops, n_operands, n_inst, n_threads; u64 start_cycle, n_cycles;
 *   u16 slot_width[n_slots]; u32 const_slot[n_consts];
 *   u64 const_limbs[4 n_consts]; u32 input_slot[n_inputs];
 *   u32 reg_slot[n_regs]; u32 reg_next[n_regs]; u32 layer_ptr[n_layers + 1];
 *   u8 op_type[n_ops]; u32 op_dst[n_ops]; u32 op_src_ptr[n_ops + 1];
 *   u32 op_src[n_operands]; u16 op_imm[n_ops]; u64 seeds[n_inst].
 * Output: u64 regs[n_inst][n_regs][4], then u64 digest[n_inst].
 * Exit status: 0, 2 for a malformed input, 3 when oracle_run fails.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/oracle.h"

static FILE* in;

static void* take(size_t n, size_t size) {
  void* p = calloc(n ? n : 1, size);
  if (!p || fread(p, size, n, in) != n) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  in = fopen(argv[1], "rb");
  if (!in) return 2;
  uint32_t* h = take(10, 4);
  uint64_t* h64 = take(2, 8);
  if (h[0] != 0x524f5452u) return 2;
  oracle_design d;
  d.n_slots = h[1];
  d.n_consts = h[2];
  d.n_inputs = h[3];
  d.n_regs = h[4];
  d.n_layers = h[5];
  d.n_ops = h[6];
  const uint32_t n_operands = h[7], n_inst = h[8];
  d.slot_width = take(d.n_slots, 2);
  d.const_slot = take(d.n_consts, 4);
  d.const_limbs = take(4 * (size_t)d.n_consts, 8);
  d.input_slot = take(d.n_inputs, 4);
  d.reg_slot = take(d.n_regs, 4);
  d.reg_next = take(d.n_regs, 4);
  d.layer_ptr = take(d.n_layers + 1, 4);
  d.op_type = take(d.n_ops, 1);
  d.op_dst = take(d.n_ops, 4);
  d.op_src_ptr = take(d.n_ops + 1, 4);
  d.op_src = take(n_operands, 4);
  d.op_imm = take(d.n_ops, 2);
  oracle_run_args a = {0};
  a.n_inst = n_inst;
  a.seeds = take(n_inst, 8);
  a.start_cycle = h64[0];
  a.n_cycles = h64[1];
  a.stim_mode = 0;
  a.trace_reg = -1;
  a.n_threads = (int32_t)h[9];
  uint64_t* regs = calloc((size_t)n_inst * d.n_regs * 4 + 1, 8);
  uint64_t* dig = calloc((size_t)n_inst + 1, 8);
  a.out_regs = regs;
  a.out_digest = dig;
  fclose(in);
  if (oracle_run(&d, &a) != 0) return 3;
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  fwrite(regs, 8, (size_t)n_inst * d.n_regs * 4, out);
  fwrite(dig, 8, n_inst, out);
  fclose(out);
  free(regs);
  free(dig);
  free((void*)a.seeds);
  free((void*)d.slot_width);
  free((void*)d.const_slot);
  free((void*)d.const_limbs);
  free((void*)d.input_slot);
  free((void*)d.reg_slot);
  free((void*)d.reg_next);
  free((void*)d.layer_ptr);
  free((void*)d.op_type);
  free((void*)d.op_dst);
  free((void*)d.op_src_ptr);
  free((void*)d.op_src);
  free((void*)d.op_imm);
  free(h);
  free(h64);
  return 0;
}
