// Per-type operators (op_u / op_r / op_s of the paper's Cascade 1) on the
// device, in three forms:
//   eval_u64  : every operand and the result fit 64 bits (one lane = one value);
//   eval_bits : every operand and the result are 1 bit and each 64-bit word
//               holds that signal for 64 instances (bit-sliced);
//   eval_wide : up to 64 NL bits in NL 64-bit limbs, NL = 2 or 4 (also every
//               operation of the types DIV .. SEXT, whatever its widths).
// All results are reduced modulo 2^width of the destination.
#pragma once
#include "internal.h"

namespace rteaal {

__device__ __forceinline__ uint64_t mask64(uint32_t w) {
  return w >= 64 ? ~0ull : ((1ull << w) - 1ull);
}

// Operand order follows the O rank: a = o0 (left / high / selector), b = o1, c = o2.
__device__ __forceinline__ uint64_t eval_u64(uint32_t opc, uint32_t arity, uint64_t a, uint64_t b,
                                             uint64_t c, uint32_t imm, uint32_t w) {
  uint64_t r;
  switch (opc) {
    case OP_AND: r = a & b & (arity == 3 ? c : ~0ull); break;
    case OP_OR: r = a | b | (arity == 3 ? c : 0ull); break;
    case OP_XOR: r = a ^ b ^ (arity == 3 ? c : 0ull); break;
    case OP_NOT: r = ~a; break;
    case OP_ADD: r = a + b; break;
    case OP_SUB: r = a - b; break;
    case OP_MUL: r = a * b; break;
    case OP_MUX: r = a ? b : c; break;
    case OP_EQ: r = a == b; break;
    case OP_LT: r = a < b; break;
    case OP_SHL: r = imm >= 64 ? 0ull : a << imm; break;
    case OP_SHR:
    case OP_EXTRACT: r = imm >= 64 ? 0ull : a >> imm; break;
    case OP_CONCAT: r = (imm >= 64 ? 0ull : a << imm) | b; break;
    case OP_ORR: r = a != 0; break;
    default: r = a; break;  // COPY
  }
  return r & mask64(w);
}

// Every operand and the result fit 32 bits (so 32-bit arithmetic modulo 2^32,
// then the mask, equals the unbounded result modulo 2^w).
__device__ __forceinline__ uint32_t eval_u32(uint32_t opc, uint32_t arity, uint32_t a, uint32_t b,
                                             uint32_t c, uint32_t imm, uint32_t w) {
  uint32_t r;
  switch (opc) {
    case OP_AND: r = a & b & (arity == 3 ? c : ~0u); break;
    case OP_OR: r = a | b | (arity == 3 ? c : 0u); break;
    case OP_XOR: r = a ^ b ^ (arity == 3 ? c : 0u); break;
    case OP_NOT: r = ~a; break;
    case OP_ADD: r = a + b; break;
    case OP_SUB: r = a - b; break;
    case OP_MUL: r = a * b; break;
    case OP_MUX: r = a ? b : c; break;
    case OP_EQ: r = a == b; break;
    case OP_LT: r = a < b; break;
    case OP_SHL: r = imm >= 32 ? 0u : a << imm; break;
    case OP_SHR:
    case OP_EXTRACT: r = imm >= 32 ? 0u : a >> imm; break;
    case OP_CONCAT: r = (imm >= 32 ? 0u : a << imm) | b; break;
    case OP_ORR: r = a != 0; break;
    default: r = a; break;  // COPY
  }
  return r & (w >= 32 ? ~0u : ((1u << w) - 1u));
}

// The same operator applied to N independent value sets (one per tile of a
// wavefront), with the type dispatch done once.
template <int N>
__device__ __forceinline__ void eval_u32_n(uint32_t opc, uint32_t arity, const uint32_t* a,
                                           const uint32_t* b, const uint32_t* c, uint32_t imm,
                                           uint32_t w, uint32_t* r) {
  const bool a3 = arity == 3;
  switch (opc) {
    case OP_AND:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] & b[g] & (a3 ? c[g] : ~0u);
      break;
    case OP_OR:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] | b[g] | (a3 ? c[g] : 0u);
      break;
    case OP_XOR:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] ^ b[g] ^ (a3 ? c[g] : 0u);
      break;
    case OP_NOT:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = ~a[g];
      break;
    case OP_ADD:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] + b[g];
      break;
    case OP_SUB:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] - b[g];
      break;
    case OP_MUL:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] * b[g];
      break;
    case OP_MUX:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] ? b[g] : c[g];
      break;
    case OP_EQ:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] == b[g];
      break;
    case OP_LT:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] < b[g];
      break;
    case OP_SHL:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = imm >= 32 ? 0u : a[g] << imm;
      break;
    case OP_SHR:
    case OP_EXTRACT:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = imm >= 32 ? 0u : a[g] >> imm;
      break;
    case OP_CONCAT:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = (imm >= 32 ? 0u : a[g] << imm) | b[g];
      break;
    case OP_ORR:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g] != 0;
      break;
    default:
#pragma unroll
      for (int g = 0; g < N; ++g) r[g] = a[g];
      break;
  }
  const uint32_t m = w >= 32 ? ~0u : ((1u << w) - 1u);
#pragma unroll
  for (int g = 0; g < N; ++g) r[g] &= m;
}

// 1-bit destination, 1-bit operands, 64 instances per word.  Each identity
// is the 1-bit case of the integer definition: a+b and a-b are a^b modulo 2,
// a*b is a&b, [a==b] is ~(a^b), [a<b] is ~a&b, a shift by k>0 leaves bit 0
// empty, CONCAT keeps the low operand, ORR of one bit is the bit.
__device__ __forceinline__ uint64_t eval_bits(uint32_t opc, uint32_t arity, uint64_t a, uint64_t b,
                                              uint64_t c, uint32_t imm) {
  switch (opc) {
    case OP_AND: return a & b & (arity == 3 ? c : ~0ull);
    case OP_OR: return a | b | (arity == 3 ? c : 0ull);
    case OP_XOR: return a ^ b ^ (arity == 3 ? c : 0ull);
    case OP_NOT: return ~a;
    case OP_ADD:
    case OP_SUB: return a ^ b;
    case OP_MUL: return a & b;
    case OP_MUX: return (a & b) | (~a & c);
    case OP_EQ: return ~(a ^ b);
    case OP_LT: return ~a & b;
    case OP_SHL:
    case OP_SHR:
    case OP_EXTRACT: return imm == 0 ? a : 0ull;
    case OP_CONCAT: return b;
    default: return a;  // ORR, COPY
  }
}

// A value of up to 64 NL bits in NL 64-bit limbs, least significant first.
// Every operation below is exact modulo 2^(64 NL), so a value and its
// operands that all fit 128 bits give the same result with NL = 2 as with
// NL = 4 (the result is cut to its width w <= 64 NL either way).
template <int NL>
struct VN {
  uint64_t l[NL];
};
using V4 = VN<4>;

template <int NL = 4>
__device__ __forceinline__ VN<NL> v4_from(uint64_t x) {
  VN<NL> r;
  r.l[0] = x;
#pragma unroll
  for (int i = 1; i < NL; i++) r.l[i] = 0ull;
  return r;
}

template <int NL>
__device__ __forceinline__ VN<NL> v4_ones() {
  VN<NL> r;
#pragma unroll
  for (int i = 0; i < NL; i++) r.l[i] = ~0ull;
  return r;
}

template <int NL>
__device__ __forceinline__ bool v4_nonzero(const VN<NL>& a) {
  uint64_t x = 0;
#pragma unroll
  for (int i = 0; i < NL; i++) x |= a.l[i];
  return x != 0ull;
}

template <int NL>
__device__ __forceinline__ VN<NL> v4_add(const VN<NL>& a, const VN<NL>& b) {
  VN<NL> r;
  uint64_t carry = 0;
#pragma unroll
  for (int i = 0; i < NL; i++) {
    uint64_t t = a.l[i] + b.l[i];
    uint64_t c1 = t < a.l[i];
    uint64_t s = t + carry;
    uint64_t c2 = s < t;
    r.l[i] = s;
    carry = c1 | c2;
  }
  return r;
}

template <int NL>
__device__ __forceinline__ VN<NL> v4_sub(const VN<NL>& a, const VN<NL>& b) {
  VN<NL> r;
  uint64_t borrow = 0;
#pragma unroll
  for (int i = 0; i < NL; i++) {
    uint64_t t = a.l[i] - b.l[i];
    uint64_t b1 = a.l[i] < b.l[i];
    uint64_t s = t - borrow;
    uint64_t b2 = t < borrow;
    r.l[i] = s;
    borrow = b1 | b2;
  }
  return r;
}

template <int NL>
__device__ __forceinline__ VN<NL> v4_mul(const VN<NL>& a, const VN<NL>& b) {
  VN<NL> r = v4_from<NL>(0);
#pragma unroll
  for (int i = 0; i < NL; i++) {
    uint64_t carry = 0;
#pragma unroll
    for (int j = 0; i + j < NL; j++) {
      uint64_t lo = a.l[i] * b.l[j];
      uint64_t hi = __umul64hi(a.l[i], b.l[j]);
      uint64_t t = r.l[i + j] + lo;
      uint64_t c1 = t < lo;
      uint64_t t2 = t + carry;
      uint64_t c2 = t2 < t;
      r.l[i + j] = t2;
      carry = hi + c1 + c2;  // a_i*b_j + r + carry < 2^128, so this cannot wrap
    }
  }
  return r;
}

// Limb k of a (0 outside 0..NL-1), as a select chain so that no local array
// is indexed with a run-time value.
template <int NL>
__device__ __forceinline__ uint64_t v4_limb(const VN<NL>& a, int k) {
  uint64_t x = 0ull;
#pragma unroll
  for (int i = 0; i < NL; i++) x = k == i ? a.l[i] : x;
  return x;
}

template <int NL>
__device__ __forceinline__ VN<NL> v4_shl(const VN<NL>& a, uint32_t k) {
  VN<NL> r = v4_from<NL>(0);
  if (k >= 64u * NL) return r;
  const int q = (int)(k >> 6);
  const uint32_t s = k & 63u;
#pragma unroll
  for (int i = 0; i < NL; i++) {
    const uint64_t hi = v4_limb(a, i - q), lo = v4_limb(a, i - q - 1);
    r.l[i] = s ? (hi << s) | (lo >> (64u - s)) : hi;
  }
  return r;
}

template <int NL>
__device__ __forceinline__ VN<NL> v4_shr(const VN<NL>& a, uint32_t k) {
  VN<NL> r = v4_from<NL>(0);
  if (k >= 64u * NL) return r;
  const int q = (int)(k >> 6);
  const uint32_t s = k & 63u;
#pragma unroll
  for (int i = 0; i < NL; i++) {
    const uint64_t lo = v4_limb(a, i + q), hi = v4_limb(a, i + q + 1);
    r.l[i] = s ? (lo >> s) | (hi << (64u - s)) : lo;
  }
  return r;
}

template <int NL>
__device__ __forceinline__ bool v4_lt(const VN<NL>& a, const VN<NL>& b) {
#pragma unroll
  for (int i = NL - 1; i > 0; i--)
    if (a.l[i] != b.l[i]) return a.l[i] < b.l[i];
  return a.l[0] < b.l[0];
}

template <int NL>
__device__ __forceinline__ VN<NL> v4_mask(VN<NL> a, uint32_t w) {
#pragma unroll
  for (int i = 0; i < NL; i++) {
    const uint32_t lo = 64u * i;
    if (w <= lo) a.l[i] = 0;
    else if (w < lo + 64) a.l[i] &= (1ull << (w - lo)) - 1ull;
  }
  return a;
}

// Quotient (want_q) or remainder of a / b, b != 0, by restoring long
// division over a's significant bits.  The partial remainder stays below b,
// but doubling it can need bit 64 NL, which `top` keeps.
template <int NL>
__device__ __forceinline__ VN<NL> v4_divmod(const VN<NL>& a, const VN<NL>& b, bool want_q) {
  int n = 0;  // significant bits of a
#pragma unroll
  for (int k = NL - 1; k >= 0; --k)
    if (n == 0 && a.l[k]) n = 64 * k + 64 - __clzll((long long)a.l[k]);
  VN<NL> q = v4_from<NL>(0), r = v4_from<NL>(0);
  for (int i = n - 1; i >= 0; --i) {
    const uint64_t top = r.l[NL - 1] >> 63;
    r = v4_shl(r, 1u);
    r.l[0] |= (v4_limb(a, i >> 6) >> (i & 63)) & 1ull;
    if (top || !v4_lt(r, b)) {
      r = v4_sub(r, b);
#pragma unroll
      for (int k = 0; k < NL; ++k) q.l[k] |= (k == (i >> 6)) ? 1ull << (i & 63) : 0ull;
    }
  }
  return want_q ? q : r;
}

// A shift amount held in a value, capped at 64 NL (everything shifted out).
template <int NL>
__device__ __forceinline__ uint32_t v4_amount(const VN<NL>& b) {
  uint64_t hi = 0;
#pragma unroll
  for (int i = 1; i < NL; i++) hi |= b.l[i];
  return hi || b.l[0] >= 64ull * NL ? 64u * NL : (uint32_t)b.l[0];
}

template <int NL>
__device__ __forceinline__ VN<NL> eval_wide(uint32_t opc, uint32_t arity, const VN<NL>& a,
                                            const VN<NL>& b, const VN<NL>& c, uint32_t imm,
                                            uint32_t w) {
  VN<NL> r;
  switch (opc) {
    case OP_AND:
#pragma unroll
      for (int i = 0; i < NL; i++) r.l[i] = a.l[i] & b.l[i] & (arity == 3 ? c.l[i] : ~0ull);
      break;
    case OP_OR:
#pragma unroll
      for (int i = 0; i < NL; i++) r.l[i] = a.l[i] | b.l[i] | (arity == 3 ? c.l[i] : 0ull);
      break;
    case OP_XOR:
#pragma unroll
      for (int i = 0; i < NL; i++) r.l[i] = a.l[i] ^ b.l[i] ^ (arity == 3 ? c.l[i] : 0ull);
      break;
    case OP_NOT:
#pragma unroll
      for (int i = 0; i < NL; i++) r.l[i] = ~a.l[i];
      break;
    case OP_ADD: r = v4_add(a, b); break;
    case OP_SUB: r = v4_sub(a, b); break;
    case OP_MUL: r = v4_mul(a, b); break;
    case OP_MUX:
    case OP_MUXC: r = v4_nonzero(a) ? b : c; break;  // MUXC: c holds the folded further pairs
    case OP_EQ: {
      bool eq = true;
#pragma unroll
      for (int i = 0; i < NL; i++) eq = eq & (a.l[i] == b.l[i]);
      r = v4_from<NL>(eq);
      break;
    }
    case OP_LT: r = v4_from<NL>(v4_lt(a, b)); break;
    case OP_SHL: r = v4_shl(a, imm); break;
    case OP_SHR:
    case OP_EXTRACT: r = v4_shr(a, imm); break;
    case OP_CONCAT: {
      r = v4_shl(a, imm);
#pragma unroll
      for (int i = 0; i < NL; i++) r.l[i] |= b.l[i];
      break;
    }
    case OP_ORR: r = v4_from<NL>(v4_nonzero(a)); break;
    // The FIRRTL primitives with no expansion in the types above; the
    // encoder runs them in this form whatever their widths.
    case OP_DIV:  // division by zero reads as quotient 0 ...
      r = v4_nonzero(b) ? v4_divmod(a, b, true) : v4_from<NL>(0);
      break;
    case OP_REM:  // ... and remainder a
      r = v4_nonzero(b) ? v4_divmod(a, b, false) : a;
      break;
    case OP_DSHL: r = v4_shl(a, v4_amount(b)); break;
    case OP_DSHR: r = v4_shr(a, v4_amount(b)); break;
    case OP_ANDR: {  // imm = width of o0: are all its bits set?
      const VN<NL> ones = v4_mask(v4_ones<NL>(), imm);
      bool all = true;
#pragma unroll
      for (int i = 0; i < NL; i++) all = all & (a.l[i] == ones.l[i]);
      r = v4_from<NL>(all);
      break;
    }
    case OP_XORR: {
      uint64_t x = 0;
#pragma unroll
      for (int i = 0; i < NL; i++) x ^= a.l[i];
      r = v4_from<NL>((uint64_t)__popcll(x) & 1ull);
      break;
    }
    case OP_SEXT: {  // imm = width of o0, read as two's complement
      r = a;
      const uint32_t sb = imm - 1u;
      if ((v4_limb(a, (int)(sb >> 6)) >> (sb & 63u)) & 1ull) {
        const VN<NL> high = v4_shl(v4_ones<NL>(), imm);
#pragma unroll
        for (int i = 0; i < NL; i++) r.l[i] |= high.l[i];
      }
      break;
    }
    default: r = a; break;  // COPY
  }
  return v4_mask(r, w);
}

// Stimulus: SplitMix64's output function (Steele, Lea & Flood, OOPSLA 2014)
// applied to seed, cycle and (input, limb) in turn.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t stim_word(uint64_t seed, uint64_t cycle, uint32_t input,
                                              uint32_t limb) {
  return splitmix64(splitmix64(splitmix64(seed) ^ cycle) ^ (((uint64_t)input << 8) | limb));
}

}  // namespace rteaal
