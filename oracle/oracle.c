/*
 * Plain CPU oracle for RTL simulation as a cascade of extended Einsums.
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).
 *
 * Written for clarity, not speed: every value is a fixed 256-bit number
 * (four 64-bit limbs), every operation is evaluated one at a time through a
 * switch, and each layer is evaluated in two passes exactly as the paper's
 * example kernel (Alg. RU) does: first all layer outputs LO[s] are computed
 * from LI, then LO is written back into LI.
 */
#include "oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t l[ORACLE_LIMBS]; } val;

/* ------------------------------------------------------------------------ */
/* 256-bit helpers.  Every result is exact modulo 2^256; since destination   */
/* widths are at most 256 bits, masking afterwards gives the value modulo    */
/* 2^w of the unbounded-integer result.                                      */
/* ------------------------------------------------------------------------ */
static val v_zero(void) { val r; memset(&r, 0, sizeof r); return r; }

static int v_is_zero(const val* a) {
  for (int i = 0; i < ORACLE_LIMBS; i++) if (a->l[i]) return 0;
  return 1;
}

static val v_mask(val a, int w) {
  for (int i = 0; i < ORACLE_LIMBS; i++) {
    int lo = 64 * i;
    if (w <= lo) a.l[i] = 0;
    else if (w < lo + 64) a.l[i] &= (((uint64_t)1) << (w - lo)) - 1;
  }
  return a;
}

static val v_add(val a, val b) {
  val r; unsigned __int128 c = 0;
  for (int i = 0; i < ORACLE_LIMBS; i++) {
    c += (unsigned __int128)a.l[i] + b.l[i];
    r.l[i] = (uint64_t)c;
    c >>= 64;
  }
  return r;
}

static val v_not(val a) {
  for (int i = 0; i < ORACLE_LIMBS; i++) a.l[i] = ~a.l[i];
  return a;
}

static val v_sub(val a, val b) {          /* a - b = a + (~b + 1) mod 2^256 */
  val one = v_zero(); one.l[0] = 1;
  return v_add(a, v_add(v_not(b), one));
}

static val v_mul(val a, val b) {          /* schoolbook, low 256 bits */
  val r = v_zero();
  for (int i = 0; i < ORACLE_LIMBS; i++) {
    unsigned __int128 carry = 0;
    for (int j = 0; i + j < ORACLE_LIMBS; j++) {
      unsigned __int128 t = (unsigned __int128)a.l[i] * b.l[j] + r.l[i + j] + carry;
      r.l[i + j] = (uint64_t)t;
      carry = t >> 64;
    }
  }
  return r;
}

static val v_shl(val a, int k) {
  val r = v_zero();
  if (k >= 64 * ORACLE_LIMBS) return r;
  int q = k / 64, s = k % 64;
  for (int i = ORACLE_LIMBS - 1; i >= q; i--) {
    uint64_t x = a.l[i - q] << s;
    if (s && i - q - 1 >= 0) x |= a.l[i - q - 1] >> (64 - s);
    r.l[i] = x;
  }
  return r;
}

static val v_shr(val a, int k) {
  val r = v_zero();
  if (k >= 64 * ORACLE_LIMBS) return r;
  int q = k / 64, s = k % 64;
  for (int i = 0; i + q < ORACLE_LIMBS; i++) {
    uint64_t x = a.l[i + q] >> s;
    if (s && i + q + 1 < ORACLE_LIMBS) x |= a.l[i + q + 1] << (64 - s);
    r.l[i] = x;
  }
  return r;
}

static int v_cmp(const val* a, const val* b) {
  for (int i = ORACLE_LIMBS - 1; i >= 0; i--) {
    if (a->l[i] < b->l[i]) return -1;
    if (a->l[i] > b->l[i]) return 1;
  }
  return 0;
}

static val v_bool(int x) { val r = v_zero(); r.l[0] = x ? 1 : 0; return r; }

/* Quotient and remainder by restoring long division, one bit at a time from
 * the top (schoolbook binary division).  The partial remainder stays below b
 * but doubling it can need bit 256: `top` keeps that bit.  b = 0 is handled
 * by the caller. */
static void v_divmod(val a, val b, val* q, val* r) {
  *q = v_zero();
  *r = v_zero();
  for (int i = 64 * ORACLE_LIMBS - 1; i >= 0; i--) {
    const int top = (int)(r->l[ORACLE_LIMBS - 1] >> 63);
    *r = v_shl(*r, 1);
    r->l[0] |= (a.l[i / 64] >> (i % 64)) & 1;
    if (top || v_cmp(r, &b) >= 0) {
      *r = v_sub(*r, b);
      q->l[i / 64] |= (uint64_t)1 << (i % 64);
    }
  }
}

/* A shift amount held in a value: its number, or 2^32 when it exceeds every
 * useful shift (every bit shifted out). */
static int v_shift_amount(const val* b) {
  for (int i = 1; i < ORACLE_LIMBS; i++) if (b->l[i]) return 1 << 30;
  return b->l[0] >= (1u << 30) ? 1 << 30 : (int)b->l[0];
}

/* ------------------------------------------------------------------------ */
/* The per-type operators of Cascade 1.                                     */
/*   reducible types: map is pass-through, op_r folds operands in O order   */
/*                    (o = 0 first; the first map temporary is copied, and  */
/*                    the reduce's left operand is the running temporary);  */
/*   unary types:     op_u maps the single operand;                         */
/*   select types:    op_s looks at the whole O fiber (mux).                */
/* ------------------------------------------------------------------------ */
static int is_unary(int n) {
  return n == ORC_NOT || n == ORC_SHL || n == ORC_SHR || n == ORC_EXTRACT || n == ORC_ORR ||
         n == ORC_ANDR || n == ORC_XORR || n == ORC_SEXT;
}
static int is_select(int n) { return n == ORC_MUX || n == ORC_MUXC; }

/* x_w: declared width of the operand. */
static val op_u(int n, val x, int imm, int x_w) {
  switch (n) {
    case ORC_NOT:     return v_not(x);
    case ORC_SHL:     return v_shl(x, imm);
    case ORC_SHR:     return v_shr(x, imm);
    case ORC_EXTRACT: return v_shr(x, imm);      /* low bit index; width from dst */
    case ORC_ORR:     return v_bool(!v_is_zero(&x));
    case ORC_ANDR: {                             /* every one of the x_w bits set */
      val ones = v_mask(v_not(v_zero()), x_w);
      return v_bool(v_cmp(&x, &ones) == 0);
    }
    case ORC_XORR: {                             /* parity of the bits */
      int p = 0;
      for (int i = 0; i < 64 * ORACLE_LIMBS; i++) p ^= (int)((x.l[i / 64] >> (i % 64)) & 1);
      return v_bool(p);
    }
    case ORC_SEXT:                               /* x as an x_w-bit two's-complement number */
      if ((x.l[(x_w - 1) / 64] >> ((x_w - 1) % 64)) & 1) {
        val high = v_shl(v_not(v_zero()), x_w);  /* every bit from x_w up */
        for (int i = 0; i < ORACLE_LIMBS; i++) x.l[i] |= high.l[i];
      }
      return x;
    default:          return x;                  /* pass-through map */
  }
}

/* prev: current reduce temporary (left); cur: new map temporary (right);
 * cur_w: declared width of the operand that produced cur. */
static val op_r(int n, val prev, val cur, int cur_w) {
  val r;
  switch (n) {
    case ORC_AND: for (int i = 0; i < ORACLE_LIMBS; i++) r.l[i] = prev.l[i] & cur.l[i]; return r;
    case ORC_OR:  for (int i = 0; i < ORACLE_LIMBS; i++) r.l[i] = prev.l[i] | cur.l[i]; return r;
    case ORC_XOR: for (int i = 0; i < ORACLE_LIMBS; i++) r.l[i] = prev.l[i] ^ cur.l[i]; return r;
    case ORC_ADD: return v_add(prev, cur);
    case ORC_SUB: return v_sub(prev, cur);
    case ORC_MUL: return v_mul(prev, cur);
    case ORC_EQ:  return v_bool(v_cmp(&prev, &cur) == 0);
    case ORC_LT:  return v_bool(v_cmp(&prev, &cur) < 0);
    case ORC_CONCAT: {                            /* left operand is the high part */
      val hi = v_shl(prev, cur_w);
      for (int i = 0; i < ORACLE_LIMBS; i++) hi.l[i] |= cur.l[i];
      return hi;
    }
    case ORC_DIV: case ORC_REM: {                 /* by zero: quotient 0, remainder prev */
      if (v_is_zero(&cur)) return n == ORC_DIV ? v_zero() : prev;
      val q, r;
      v_divmod(prev, cur, &q, &r);
      return n == ORC_DIV ? q : r;
    }
    case ORC_DSHL: return v_shl(prev, v_shift_amount(&cur));
    case ORC_DSHR: return v_shr(prev, v_shift_amount(&cur));
    default: return cur;                          /* non-reducible: copy */
  }
}

/* Select over the whole O fiber.  The fiber is (selector, value) pairs at
 * o = 2i, 2i + 1, then a default at o = arity - 1: the first pair whose
 * selector is nonzero gives its value, and the default is taken when none
 * is.  MUX is the one-pair case; MUXC, the fused mux chain of the
 * compiler's operator fusion (section "Design Overview" of the simulator,
 * and App. B "Implemented Optimizations"), has up to 32 pairs. */
static val op_s(int n, const val* sel, int arity) {
  (void)n;
  for (int o = 0; o + 1 < arity; o += 2)
    if (!v_is_zero(&sel[o])) return sel[o + 1];
  return sel[arity - 1];
}

static int arity_ok(int n, int a) {
  switch (n) {
    case ORC_AND: case ORC_OR: case ORC_XOR: return a == 2 || a == 3;
    case ORC_MUX: return a == 3;
    case ORC_MUXC: return a >= 3 && a <= ORACLE_MAX_ARITY && a % 2 == 1;
    case ORC_ADD: case ORC_SUB: case ORC_MUL: case ORC_EQ: case ORC_LT: case ORC_CONCAT:
    case ORC_DIV: case ORC_REM: case ORC_DSHL: case ORC_DSHR:
      return a == 2;
    case ORC_NOT: case ORC_SHL: case ORC_SHR: case ORC_EXTRACT: case ORC_ORR:
    case ORC_ANDR: case ORC_XORR: case ORC_SEXT: return a == 1;
    default: return 0;
  }
}

/* LO for one operation from its selected inputs OI (in O order). */
static val eval_one(int n, int arity, const val* oi, const uint16_t* oi_w, int imm) {
  if (is_select(n)) return op_s(n, oi, arity);
  if (is_unary(n)) return op_u(n, oi[0], imm, oi_w[0]);
  val acc = oi[0];                                /* first map temporary copied */
  for (int o = 1; o < arity; o++) acc = op_r(n, acc, oi[o], oi_w[o]);
  return acc;
}

int oracle_eval_op(int type, int arity, const uint64_t* operands, const uint16_t* src_w,
                   int dst_w, int imm, uint64_t* out) {
  if (type < 0 || type >= ORC_NTYPES || !arity_ok(type, arity)) return -1;
  if (dst_w < 1 || dst_w > 256) return -1;
  val oi[ORACLE_MAX_ARITY];
  for (int o = 0; o < arity; o++) memcpy(oi[o].l, operands + 4 * o, sizeof(val));
  val r = v_mask(eval_one(type, arity, oi, src_w, imm), dst_w);
  memcpy(out, r.l, sizeof(val));
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Stimulus: SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).  */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t x) { return splitmix64(x); }

uint64_t oracle_stim(uint64_t seed, uint64_t cycle, uint32_t input, uint32_t limb) {
  return splitmix64(splitmix64(splitmix64(seed) ^ cycle) ^ (((uint64_t)input << 8) | limb));
}

/* ------------------------------------------------------------------------ */
/* One instance, all cycles.                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
  const oracle_design* d;
  const oracle_run_args* a;
  uint32_t first, step;
  uint32_t max_layer_ops;
  uint32_t input_words;
} job;

static int limbs_of(int w) { return (w + 63) / 64; }

static void run_instance(const job* jb, uint32_t inst, val* LI, val* LO, val* nxt) {
  const oracle_design* d = jb->d;
  const oracle_run_args* a = jb->a;
  for (uint32_t s = 0; s < d->n_slots; s++) LI[s] = v_zero();
  for (uint32_t c = 0; c < d->n_consts; c++) {
    val v; memcpy(v.l, d->const_limbs + 4 * (size_t)c, sizeof v);
    LI[d->const_slot[c]] = v_mask(v, d->slot_width[d->const_slot[c]]);
  }
  if (a->init_regs)
    for (uint32_t j = 0; j < d->n_regs; j++) {
      val v; memcpy(v.l, a->init_regs + ((size_t)inst * d->n_regs + j) * 4, sizeof v);
      LI[d->reg_slot[j]] = v_mask(v, d->slot_width[d->reg_slot[j]]);
    }

  uint64_t digest = a->init_digest ? a->init_digest[inst] : 0;
  for (uint64_t t = 0; t < a->n_cycles; t++) {
    uint64_t cycle = a->start_cycle + t;
    /* Host/testbench writes the primary inputs into LI for this cycle. */
    size_t woff = 0;
    for (uint32_t k = 0; k < d->n_inputs; k++) {
      uint32_t s = d->input_slot[k];
      int w = d->slot_width[s], nl = limbs_of(w);
      val v = v_zero();
      for (int l = 0; l < nl; l++) {
        if (a->stim_mode == 0)
          v.l[l] = oracle_stim(a->seeds[inst], cycle, k, (uint32_t)l);
        else
          v.l[l] = a->stim_words[(t * a->n_inst + inst) * jb->input_words + woff + l];
      }
      woff += nl;
      LI[s] = v_mask(v, w);
    }
    /* Rank I: layers in order. */
    for (uint32_t i = 0; i < d->n_layers; i++) {
      uint32_t s0 = d->layer_ptr[i], s1 = d->layer_ptr[i + 1];
      /* OI = LI . OIM, then LO via op_u / op_r / op_s. */
      for (uint32_t s = s0; s < s1; s++) {
        int n = d->op_type[s];
        uint32_t p0 = d->op_src_ptr[s];
        int arity = (int)(d->op_src_ptr[s + 1] - p0);
        val oi[ORACLE_MAX_ARITY]; uint16_t oi_w[ORACLE_MAX_ARITY];
        for (int o = 0; o < arity; o++) {
          uint32_t r = d->op_src[p0 + o];
          oi[o] = LI[r];
          oi_w[o] = d->slot_width[r];
        }
        LO[s - s0] = eval_one(n, arity, oi, oi_w, d->op_imm[s]);
      }
      /* Write LO back into LI at each op's S coordinate, masked to its width. */
      for (uint32_t s = s0; s < s1; s++) {
        uint32_t dst = d->op_dst[s];
        LI[dst] = v_mask(LO[s - s0], d->slot_width[dst]);
      }
    }
    /* End of cycle: every register latches its next-state slot at once. */
    for (uint32_t j = 0; j < d->n_regs; j++) nxt[j] = LI[d->reg_next[j]];
    for (uint32_t j = 0; j < d->n_regs; j++)
      LI[d->reg_slot[j]] = v_mask(nxt[j], d->slot_width[d->reg_slot[j]]);
    if (a->trace && a->trace_reg >= 0)
      a->trace[(size_t)inst * a->n_cycles + t] = LI[d->reg_slot[a->trace_reg]].l[0];
    /* Register digest of this cycle, after the commit (see oracle.h). */
    uint64_t h = 0;
    for (uint32_t j = 0; j < d->n_regs; j++) {
      const val* r = &LI[d->reg_slot[j]];
      int nl = limbs_of(d->slot_width[d->reg_slot[j]]);
      for (int l = 0; l < nl; l++)
        h += splitmix64(splitmix64(((uint64_t)j << 2) | (uint64_t)l) ^ r->l[l]);
    }
    digest = splitmix64(digest ^ h);
    if (a->digest_trace) a->digest_trace[(size_t)inst * a->n_cycles + t] = digest;
  }
  if (a->out_digest) a->out_digest[inst] = digest;

  for (uint32_t j = 0; j < d->n_regs; j++)
    memcpy(a->out_regs + ((size_t)inst * d->n_regs + j) * 4, LI[d->reg_slot[j]].l, sizeof(val));
  if (a->out_slots)
    memcpy(a->out_slots + (size_t)inst * d->n_slots * 4, LI, sizeof(val) * d->n_slots);
}

static void* worker(void* p) {
  const job* jb = (const job*)p;
  val* LI = (val*)malloc(sizeof(val) * (jb->d->n_slots ? jb->d->n_slots : 1));
  val* LO = (val*)malloc(sizeof(val) * (jb->max_layer_ops ? jb->max_layer_ops : 1));
  val* nx = (val*)malloc(sizeof(val) * (jb->d->n_regs ? jb->d->n_regs : 1));
  if (LI && LO && nx)
    for (uint32_t inst = jb->first; inst < jb->a->n_inst; inst += jb->step)
      run_instance(jb, inst, LI, LO, nx);
  free(LI); free(LO); free(nx);
  return NULL;
}

static int check_design(const oracle_design* d) {
  for (uint32_t s = 0; s < d->n_slots; s++)
    if (d->slot_width[s] < 1 || d->slot_width[s] > 256) return -2;
  for (uint32_t c = 0; c < d->n_consts; c++) if (d->const_slot[c] >= d->n_slots) return -3;
  for (uint32_t k = 0; k < d->n_inputs; k++) if (d->input_slot[k] >= d->n_slots) return -3;
  for (uint32_t j = 0; j < d->n_regs; j++)
    if (d->reg_slot[j] >= d->n_slots || d->reg_next[j] >= d->n_slots) return -3;
  if (d->layer_ptr[0] != 0 || d->layer_ptr[d->n_layers] != d->n_ops) return -4;
  for (uint32_t i = 0; i < d->n_layers; i++) if (d->layer_ptr[i + 1] < d->layer_ptr[i]) return -4;
  if (d->op_src_ptr[0] != 0) return -5;
  for (uint32_t s = 0; s < d->n_ops; s++) {
    if (d->op_type[s] >= ORC_NTYPES || d->op_dst[s] >= d->n_slots) return -5;
    uint32_t a = d->op_src_ptr[s + 1] - d->op_src_ptr[s];
    if (d->op_src_ptr[s + 1] < d->op_src_ptr[s] || !arity_ok(d->op_type[s], (int)a)) return -5;
    for (uint32_t o = d->op_src_ptr[s]; o < d->op_src_ptr[s + 1]; o++)
      if (d->op_src[o] >= d->n_slots) return -5;
  }
  return 0;
}

int oracle_run(const oracle_design* d, const oracle_run_args* a) {
  int rc = check_design(d);
  if (rc) return rc;
  if ((!a->out_regs && d->n_regs) || (a->n_inst && !a->seeds && a->stim_mode == 0)) return -1;
  if (a->stim_mode == 1 && !a->stim_words && d->n_inputs) return -1;
  if (a->trace_reg >= (int32_t)d->n_regs) return -1;
  uint32_t mx = 0, words = 0;
  for (uint32_t i = 0; i < d->n_layers; i++) {
    uint32_t n = d->layer_ptr[i + 1] - d->layer_ptr[i];
    if (n > mx) mx = n;
  }
  for (uint32_t k = 0; k < d->n_inputs; k++) words += (uint32_t)limbs_of(d->slot_width[d->input_slot[k]]);
  int nt = a->n_threads > 0 ? a->n_threads : 1;
  if ((uint32_t)nt > a->n_inst) nt = a->n_inst ? (int)a->n_inst : 1;
  job* jobs = (job*)calloc((size_t)nt, sizeof(job));
  pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -6; }
  for (int t = 0; t < nt; t++) {
    jobs[t].d = d; jobs[t].a = a; jobs[t].first = (uint32_t)t; jobs[t].step = (uint32_t)nt;
    jobs[t].max_layer_ops = mx; jobs[t].input_words = words;
  }
  for (int t = 1; t < nt; t++) pthread_create(&th[t], NULL, worker, &jobs[t]);
  worker(&jobs[0]);
  for (int t = 1; t < nt; t++) pthread_join(th[t], NULL);
  free(jobs); free(th);
  return 0;
}
