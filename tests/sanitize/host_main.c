/*
 * Stand-alone driver of the library's host-only entry points for sanitizer
 * runs (test infrastructure only): reads a design in the input format of
 * oracle_main.c (the run fields are ignored), calls rteaal_validate_design
 * and rteaal_fuse_mux_chains, and writes what they return.  The sanitizer
 * test builds the library's host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer and links it with this driver; neither call
 * touches a GPU.
 *
 * Usage: host_main input output max_pairs
 * Output (little-endian): i32 validate status; then, when it is 0,
 *   i32 fuse status, u32 n_ops, n_operands, n_fused, n_absorbed,
 *   u32 layer_op_ptr[n_layers + 1], u8 op_type[n_ops], u32 op_dst[n_ops],
 *   u32 op_src_ptr[n_ops + 1], u32 op_src[n_operands], u16 op_imm[n_ops].
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../include/rteaal.h"

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
  if (argc != 4) {
    fprintf(stderr, "usage: %s input output max_pairs\n", argv[0]);
    return 2;
  }
  in = fopen(argv[1], "rb");
  if (!in) return 2;
  uint32_t* h = take(10, 4);
  uint64_t* h64 = take(2, 8);
  if (h[0] != 0x524f5452u) return 2;
  rteaal_design_desc d = {0};
  d.n_slots = h[1];
  d.n_consts = h[2];
  d.n_inputs = h[3];
  d.n_regs = h[4];
  d.n_layers = h[5];
  d.n_ops = h[6];
  const uint32_t n_operands = h[7];
  d.slot_width = take(d.n_slots, 2);
  d.const_slot = take(d.n_consts, 4);
  d.const_limbs = take(4 * (size_t)d.n_consts, 8);
  d.input_slot = take(d.n_inputs, 4);
  d.reg_slot = take(d.n_regs, 4);
  d.reg_next = take(d.n_regs, 4);
  d.layer_op_ptr = take(d.n_layers + 1, 4);
  d.op_type = take(d.n_ops, 1);
  d.op_dst = take(d.n_ops, 4);
  d.op_src_ptr = take(d.n_ops + 1, 4);
  d.op_src = take(n_operands, 4);
  d.op_imm = take(d.n_ops, 2);
  d.layer_fmt = NULL;
  fclose(in);
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  char err[256];
  const int32_t vs = (int32_t)rteaal_validate_design(&d, err, sizeof err);
  fwrite(&vs, 4, 1, out);
  if (vs == 0) {
    uint32_t* lptr = calloc(d.n_layers + 1, 4);
    uint8_t* typ = calloc(d.n_ops + 1, 1);
    uint32_t* dst = calloc(d.n_ops + 1, 4);
    uint32_t* sptr = calloc(d.n_ops + 1, 4);
    uint32_t* src = calloc(n_operands + 1, 4);
    uint16_t* imm = calloc(d.n_ops + 1, 2);
    rteaal_fuse_result r = {0};
    const int32_t fs = (int32_t)rteaal_fuse_mux_chains(&d, (uint32_t)atoi(argv[3]), lptr, typ, dst,
                                                       sptr, src, imm, &r);
    fwrite(&fs, 4, 1, out);
    fwrite(&r, 4, 4, out);
    fwrite(lptr, 4, d.n_layers + 1, out);
    fwrite(typ, 1, r.n_ops, out);
    fwrite(dst, 4, r.n_ops, out);
    fwrite(sptr, 4, r.n_ops + 1, out);
    fwrite(src, 4, r.n_operands, out);
    fwrite(imm, 2, r.n_ops, out);
    free(lptr);
    free(typ);
    free(dst);
    free(sptr);
    free(src);
    free(imm);
  }
  fclose(out);
  free((void*)d.slot_width);
  free((void*)d.const_slot);
  free((void*)d.const_limbs);
  free((void*)d.input_slot);
  free((void*)d.reg_slot);
  free((void*)d.reg_next);
  free((void*)d.layer_op_ptr);
  free((void*)d.op_type);
  free((void*)d.op_dst);
  free((void*)d.op_src_ptr);
  free((void*)d.op_src);
  free((void*)d.op_imm);
  free(h);
  free(h64);
  return 0;
}
