// Device modular arithmetic for word-size primes q < 2^62 (limbs of 36 and 54
// bits, the special prime and the plaintext modulus).  Everything is exact
// integer arithmetic on the VALU: gfx950 has no 64x64 multiplier, so 64-bit
// products are built by the compiler from v_mad_u64_u32 / v_mul_hi_u32, which
// issue at close to full rate on this chip.
//
// Reduction strategy (lazy reduction, paper §7.1 "NTT ... with lazy modular
// reduction" and the accumulation of many plaintext products before one
// reduction):
//  * products with a constant (twiddles, n^-1, P^-1) use Shoup's method:
//    w' = floor(w * 2^64 / q) precomputed on the host, result in [0, 2q);
//  * sums of products of two variables are accumulated in 128 bits and
//    reduced once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wally {

struct u128w {
  uint64_t lo, hi;
};

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// a * w mod q in [0, 2q) for any a < 2^64, w < q, wp = floor(w 2^64 / q).
__device__ __forceinline__ uint64_t shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  const uint64_t qh = mulhi64(a, wp);
  return a * w - qh * q;
}

// a * w mod q in [0, 4q) for any a < 2^64, w < q, wp = floor(w 2^64 / q).
// Shoup's quotient floor(a wp / 2^64) without the low x low partial product
// and without the carry between the two middle ones:
//   a wp = a1 p1 2^64 + (a0 p1 + a1 p0) 2^32 + a0 p0 (p1, p0 the words of wp),
//   and the dropped parts add
//   less than 3 to the quotient, so qh is exact or up to 2 below it.
//
// The remainder a w - qh q is formed mod 2^64 as a w + qh (2^64 - q): with
// nq = 2^64 - q the two low x low products chain through one 64-bit addend
// and the four cross products only touch the high word, so no 64-bit
// subtraction is needed (8 instead of 10 VALU operations).
__device__ __forceinline__ uint64_t shoup4(uint64_t a, uint64_t w, uint64_t wp, uint64_t nq) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t p0 = (uint32_t)wp, p1 = (uint32_t)(wp >> 32);
  uint64_t mid = (uint64_t)__umulhi(a0, p1) + __umulhi(a1, p0);
  // Empty asm operands keep the compiler from re-associating these sums into
  // forms that need zero-extended register pairs (one extra move each).
  asm("" : "+v"(mid));
  const uint64_t qh = (uint64_t)a1 * p1 + mid;
  const uint32_t h0 = (uint32_t)qh, h1 = (uint32_t)(qh >> 32);
  const uint32_t w0 = (uint32_t)w, w1 = (uint32_t)(w >> 32);
  const uint32_t n0 = (uint32_t)nq, n1 = (uint32_t)(nq >> 32);
  const uint64_t lo = (uint64_t)a0 * w0 + (uint64_t)h0 * n0;  // wraps mod 2^64
  uint32_t lo_hi = (uint32_t)(lo >> 32);
  asm("" : "+v"(lo_hi));
  const uint32_t hi = lo_hi + a0 * w1 + a1 * w0 + h0 * n1 + h1 * n0;
  return ((uint64_t)hi << 32) | (uint32_t)lo;
}

// x - m when x >= m, else x, for x < 2^63 + m.  The sign of x - m picks the
// result through a bit select: no compare, so no VCC write and none of the
// wait states a VCC read right after it needs (empty asm operands keep the
// compiler from turning it back into compare and select).
__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) {
  uint64_t nm = 0 - m;
  asm("" : "+s"(nm));
  const uint64_t w = x + nm;
  uint32_t keep = (uint32_t)((int32_t)(uint32_t)(w >> 32) >> 31);  // all ones when x < m
  asm("" : "+v"(keep));
  const uint32_t lo = (keep & (uint32_t)x) | (~keep & (uint32_t)w);
  const uint32_t hi = (keep & (uint32_t)(x >> 32)) | (~keep & (uint32_t)(w >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// x in [0, 4q) -> [0, q)
__device__ __forceinline__ uint64_t reduce4(uint64_t x, uint64_t q, uint64_t q2) {
  x = x >= q2 ? x - q2 : x;
  return x >= q ? x - q : x;
}

// any x < 2^64 -> [0, q), given onep = floor(2^64 / q) (Shoup with w = 1)
__device__ __forceinline__ uint64_t reduce_lazy(uint64_t x, uint64_t q, uint64_t onep) {
  return csub(x - mulhi64(x, onep) * q, q);
}

__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return csub(a + b, q); }
__device__ __forceinline__ uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

// acc += a * b (128-bit)
__device__ __forceinline__ void mac128(u128w& acc, uint64_t a, uint64_t b) {
  const uint64_t lo = a * b;
  const uint64_t hi = mulhi64(a, b);
  const uint64_t s = acc.lo + lo;
  acc.hi += hi + (s < lo ? 1u : 0u);
  acc.lo = s;
}

// (hi * 2^64 + lo) mod q for any hi, lo < 2^64: result in [0, q).
__device__ __forceinline__ uint64_t reduce128(u128w x, uint64_t q, uint64_t r64, uint64_t r64p, uint64_t onep) {
  const uint64_t a = shoup(x.hi, r64, r64p, q);   // hi * 2^64 mod q, [0, 2q)
  const uint64_t b = x.lo - mulhi64(x.lo, onep) * q;  // lo mod q, [0, 2q)
  uint64_t s = a + b;                              // [0, 4q)
  s = s >= 2 * q ? s - 2 * q : s;
  return s >= q ? s - q : s;
}

}  // namespace wally
