// 64-bit-modulus arithmetic used by the 64-bit word paths (host and device).
//
// Remainders of 128-bit values by a 64-bit q use division by an invariant
// integer with a precomputed reciprocal (Moller and Granlund, "Improved
// division by invariant integers", IEEE TC 2011, the 2/1 division with a
// normalised divisor).  Only 64-bit operations appear, so the same code runs
// on the GPU and, for testing, on the host.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

struct U128 {
  uint64_t lo, hi;
};

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ __forceinline__ U128 mul64x64(uint64_t a, uint64_t b) {
  U128 r;
  r.lo = a * b;
  r.hi = mulhi64(a, b);
  return r;
}

__host__ __device__ __forceinline__ U128 add128(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1u : 0u);
  return r;
}

__host__ __device__ __forceinline__ int clz64(uint64_t x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __clzll((long long)x);
#else
  return __builtin_clzll(x);
#endif
}

// Per-modulus constants for 64-bit moduli.
struct ModQ64 {
  uint64_t q;
  uint64_t thr;     // digit representative threshold: x <= thr ? x : x - q
  uint64_t d;       // q << sh, top bit set
  uint64_t v;       // floor((2^128 - 1) / d) - 2^64
  uint32_t sh;      // normalisation shift, 0..63
  uint32_t pad;
  uint64_t r[16];   // 2^(8s) mod q for s < 15
  uint64_t foff;    // (2^56 * sum_j 2^(32j)) mod q over the ceil((2L-1)/4) class groups of a flush
};

// One 2/1 division step: (u1, u0) with u1 < d -> remainder mod d.
__host__ __device__ __forceinline__ uint64_t rem_2by1(uint64_t u1, uint64_t u0, uint64_t d, uint64_t v) {
  U128 qq = mul64x64(v, u1);
  qq = add128(qq, U128{u0, u1 + 1});
  uint64_t q1 = qq.hi;
  uint64_t r = u0 - q1 * d;
  if (r > qq.lo) r += d;
  if (r >= d) r -= d;
  return r;
}

// (hi * 2^64 + lo) mod q.
__host__ __device__ __forceinline__ uint64_t mod_u128(uint64_t hi, uint64_t lo, const ModQ64& m) {
  const uint32_t s = m.sh;
  uint64_t n2, n1, n0;
  if (s == 0) {
    n2 = 0; n1 = hi; n0 = lo;
  } else {
    n2 = hi >> (64 - s);
    n1 = (hi << s) | (lo >> (64 - s));
    n0 = lo << s;
  }
  // n2 < 2^s <= d, so each step's high word is below d
  uint64_t r = rem_2by1(n2, n1, m.d, m.v);
  r = rem_2by1(r, n0, m.d, m.v);
  return r >> s;
}

__host__ __device__ __forceinline__ uint64_t mod_u64(uint64_t x, const ModQ64& m) {
  return mod_u128(0, x, m);
}

__host__ __device__ __forceinline__ uint64_t addmod64(uint64_t a, uint64_t b, uint64_t q) {
  // a, b < q
  uint64_t s = a + b;
  if (s < a || s >= q) s -= q;
  return s;
}

__host__ __device__ __forceinline__ uint64_t submod64(uint64_t a, uint64_t b, uint64_t q) {
  return a >= b ? a - b : a + (q - b);
}

}  // namespace pm
