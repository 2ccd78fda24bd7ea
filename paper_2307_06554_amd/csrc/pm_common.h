// Internal definitions of the GPU library (host and device).  Not installed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

// ---------------------------------------------------------------------------
// Balanced signed radix-2^8 limbs (paper Sec. 2.4, strategy (ii): a wide
// coefficient is held as several small units that the matrix engine takes
// natively).  With L limbs the digit window is
//     W_L = [-128 * S_L, 127 * S_L],  S_L = sum_{i<L} 256^i,
// which holds exactly 256^L consecutive integers, so every residue class mod
// q <= 256^L has a representative in it: x itself when x <= 127*S_L, else
// x - q.  Adding BIAS_L = 128*S_L maps the window onto [0, 256^L) and the
// bytes of (v + BIAS_L) XOR 0x80.. are the digits d_i in [-128, 127] with
// v = sum_i d_i 256^i.  No digit is ever negated (the negative wrap sign of
// Eq. (3) is carried by the digits of q - x instead), so -128 never overflows.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr uint64_t limb_sum(int L) {
  uint64_t s = 0;
  for (int i = 0; i < L; ++i) s |= (uint64_t)1 << (8 * i);
  return s;
}
__host__ __device__ constexpr uint64_t limb_bias(int L) { return 0x80ull * limb_sum(L); }
__host__ __device__ constexpr uint64_t limb_top(int L) { return 0x7Full * limb_sum(L); }

// Smallest limb count whose window covers q residues (q <= 256^L).
inline int limbs_for_q32(uint32_t q) {
  if (q <= 256u) return 1;
  if (q <= 65536u) return 2;
  if (q <= (1u << 24)) return 3;
  return 4;
}
inline int limbs_for_q64(uint64_t q) {
  int L = 1;
  while (L < 8 && q > ((uint64_t)1 << (8 * L))) ++L;
  return L;
}

// Per-modulus constants for the 32-bit-modulus paths.
struct ModQ32 {
  uint32_t q;
  uint32_t thr;     // digit representative threshold: x <= thr ? x : x - q
  uint64_t mu;      // floor(2^64 / q) for Barrett reduction (q >= 2)
  uint64_t lift;    // multiple of q in [2^62, 2^62 + q): makes |x| < 2^62 non-negative
  uint32_t r64;     // 2^64 mod q
  uint32_t m32;     // floor(2^32 / q), for reducing 32-bit words
};

inline ModQ32 make_mod32(uint32_t q, int L) {
  ModQ32 m{};
  m.q = q;
  uint64_t top = limb_top(L);
  m.thr = top >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)top;
  // floor(2^64 / q) = floor((2^64 - 1) / q) unless q divides 2^64 (q a power of two).
  uint64_t mu = UINT64_MAX / q;
  if ((q & (q - 1)) == 0) mu += 1;  // exact power of two: 2^64/q = (2^64-1)/q + 1
  if (q == 1) mu = UINT64_MAX;       // unreachable (q >= 2 is validated)
  m.mu = mu;
  uint64_t k = ((uint64_t)1 << 62) / q + 1;
  m.lift = k * q;
  unsigned __int128 t = ((unsigned __int128)1 << 64) % q;
  m.r64 = (uint32_t)t;
  uint64_t m32 = ((uint64_t)1 << 32) / q;
  m.m32 = m32 > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)m32;
  return m;
}

// High halves of products (device intrinsics; plain wide arithmetic on the host,
// where these helpers are tested).
__host__ __device__ __forceinline__ uint64_t mul_hi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}
__host__ __device__ __forceinline__ uint32_t mul_hi32(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umulhi(a, b);
#else
  return (uint32_t)(((uint64_t)a * b) >> 32);
#endif
}
__host__ __device__ __forceinline__ uint32_t min_u32(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Barrett: x mod q for any 64-bit x, q < 2^32.  With mu = floor(2^64/q) >=
// 2^64/q - 1 and x < 2^64, x*mu/2^64 > x/q - 1, so the quotient estimate is
// floor(x/q) or one less and r = x - estimate*q lies in [0, 2q).
__host__ __device__ __forceinline__ uint32_t reduce_u64(uint64_t x, const ModQ32& m) {
  const uint64_t qe = mul_hi64(x, m.mu);
  uint64_t r = x - qe * (uint64_t)m.q;
  if (r >= m.q) r -= m.q;
  return (uint32_t)r;
}
// The same for q < 2^31: then r < 2q < 2^32, so r is the low word of
// x - estimate*q and the tail is 32-bit arithmetic.
__host__ __device__ __forceinline__ uint32_t reduce_u64_q31(uint64_t x, uint64_t mu, uint32_t q) {
  const uint64_t qe = mul_hi64(x, mu);
  const uint32_t r = (uint32_t)x - (uint32_t)qe * q;
  return min_u32(r, r - q);
}
// x mod q for a 32-bit word.  With m32 = floor(2^32/q) >= 2^32/q - 1 and x < 2^32,
// x*m32/2^32 > x/q - 1, so the estimate floor(x*m32/2^32) is floor(x/q) or one
// less and r = x - estimate*q lies in [0, 2q) (and below 2^32: m32 = 1 when
// q > 2^31).  One conditional subtraction ends it; min(r, r - q) is that
// subtraction, r - q wrapping above r when r < q.
__host__ __device__ __forceinline__ uint32_t reduce_u32(uint32_t x, const ModQ32& m) {
  const uint32_t qe = mul_hi32(x, m.m32);
  const uint32_t r = x - qe * m.q;
  return min_u32(r, r - m.q);
}
// Signed |x| < 2^62 (x + lift is in (0, 2^63 + 2^32), added as unsigned words).
__host__ __device__ __forceinline__ uint32_t reduce_i64(int64_t x, const ModQ32& m) {
  return reduce_u64((uint64_t)x + m.lift, m);
}

// L digits of the residue x (already in [0, q)), packed little-endian in a word.
template <int L>
__host__ __device__ __forceinline__ uint32_t digits32(uint32_t x, uint32_t q, uint32_t thr) {
  constexpr uint32_t B = (uint32_t)limb_bias(L);
  uint32_t v = x <= thr ? x : x - q;  // wraps mod 2^32: the representative in W_L
  return (v + B) ^ B;
}
// Digits of -x mod q.
template <int L>
__host__ __device__ __forceinline__ uint32_t neg_digits32(uint32_t x, uint32_t q, uint32_t thr) {
  return digits32<L>(x == 0 ? 0u : q - x, q, thr);
}
// Both digit words of residues x in [0, q): of x and of a representative of -x.
// When q <= thr (the window's top: 0x7F7F7F7F for L = 4, so every 30-bit q)
// x and q - x are in the window as they are; q - 0 = q stands for 0.
// Four residues at a time, the window test taken once.
template <int L>
__host__ __device__ __forceinline__ void digits_pm32(const uint32_t (&x)[4], uint32_t q, uint32_t thr, uint32_t (&pos)[4],
                                            uint32_t (&neg)[4]) {
  constexpr uint32_t B = (uint32_t)limb_bias(L);
  if (q <= thr) {
    const uint32_t qb = q + B;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pos[k] = (x[k] + B) ^ B;
      neg[k] = (qb - x[k]) ^ B;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pos[k] = digits32<L>(x[k], q, thr);
      neg[k] = neg_digits32<L>(x[k], q, thr);
    }
  }
}

// ---------------------------------------------------------------------------
// Small moduli (the residue-number-system path, paper Sec. 2.4 and 2.6).
// ---------------------------------------------------------------------------
// The centred residue of v mod m as an int32 in [-128, 127], for |v| < 2^31 and
// 2 <= m <= 256.  Write v = 2^16 vh + vl (vl in [0, 2^16)); with R = 2^16 mod m,
// x = vh R + vl = v (mod m) and |x| < 2^23 + 2^16, so x is exact in fp32.  k =
// rint of the rounded fp32 quotient x (1/m) and r = x - k m by one fma are exact
// integers, r = v (mod m).  The quotient is off by less than 1.01 / m, so k is off
// by at most one and only when the exact centred residue lies within 1.01 of
// +-m/2: |r| <= m/2 + 1, an int8 for m <= 253; 255 needs r = 128 folded to -127;
// for 256 the residue is the low byte of v.
// The same for |x| < 2^23 + 2^16 (m < 256), the range vh R + vl takes.
__host__ __device__ __forceinline__ int32_t centred_mod_small(int32_t x, uint32_t m, float mf, float invm) {
  const float xf = (float)x;
  const float kf = rintf(xf * invm);
  int32_t r = (int32_t)fmaf(-kf, mf, xf);
  if (m > 253 && r > 127) r -= (int32_t)m;
  return r;
}
__host__ __device__ __forceinline__ int32_t residue_centred(int32_t v, uint32_t m, int32_t r16, float mf,
                                                            float invm) {
  if (m == 256) return (int32_t)(int8_t)(uint8_t)v;
  const int32_t vh = v >> 16, vl = v & 0xFFFF;
#if defined(__HIP_DEVICE_COMPILE__)
  const int32_t x = __mul24(vh, r16) + vl;  // both factors fit 24 bits: the full-rate multiply
#else
  const int32_t x = vh * r16 + vl;
#endif
  return centred_mod_small(x, m, mf, invm);
}

}  // namespace pm
