// Host check of the library's modular-arithmetic helpers against plain 128-bit
// integer arithmetic: the Barrett reductions and balanced digit splits of the
// 32-bit-modulus paths (pm_common.h), the centred small-modulus residues of the
// CRT path (pm_common.h) and the reciprocal 128/64 remainder and per-modulus
// constants of the 64-bit paths (pm_wide.h, pm_wide_host.h).  These
// helpers are __host__ __device__, so the code the kernels run is the code
// compiled here for the CPU.  Built by tests/test_host_arith.py (also under the
// address and undefined-behaviour sanitizers); prints "ok <cases>" or the first
// failure and exits non-zero.
#include <stdio.h>
#include <stdlib.h>

#include "pm_common.h"
#include "pm_wide_host.h"

using namespace pm;
typedef unsigned __int128 u128;

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static uint64_t next64() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static unsigned long long g_cases = 0;

#define CHECK(cond, ...)                                        \
  do {                                                          \
    ++g_cases;                                                  \
    if (!(cond)) {                                              \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);      \
      fprintf(stderr, __VA_ARGS__);                             \
      fprintf(stderr, "\n");                                    \
      exit(1);                                                  \
    }                                                           \
  } while (0)

// Signed value of L balanced digits packed little-endian in a word.
static int64_t digit_value(uint64_t w, int L) {
  int64_t v = 0, p = 1;
  for (int i = 0; i < L; ++i) {
    v += (int64_t)(int8_t)(uint8_t)(w >> (8 * i)) * p;
    p *= 256;
  }
  return v;
}

static int64_t mod_signed(int64_t v, uint64_t q) {
  int64_t r = v % (int64_t)q;
  return r < 0 ? r + (int64_t)q : r;
}

template <int L>
static void check_digits32(uint32_t q, uint32_t x) {
  const ModQ32 m = make_mod32(q, L);
  const int64_t top = (int64_t)limb_top(L), bottom = -(int64_t)limb_bias(L);
  const uint32_t d = digits32<L>(x, q, m.thr);
  const int64_t v = digit_value(d, L);
  CHECK(v >= bottom && v <= top && mod_signed(v, q) == (int64_t)x, "digits32<%d> q=%u x=%u -> %lld", L, q, x,
        (long long)v);
  if (L < 4) CHECK((d >> (8 * L)) == 0, "digits32<%d> q=%u x=%u: bytes above the limbs", L, q, x);
  const uint32_t nd = neg_digits32<L>(x, q, m.thr);
  const int64_t nv = digit_value(nd, L);
  CHECK(nv >= bottom && nv <= top && mod_signed(-nv, q) == (int64_t)x, "neg_digits32<%d> q=%u x=%u", L, q, x);
  // four at a time, with the window test taken once
  const uint32_t xs[4] = {x, (uint32_t)(next64() % q), 0u, q - 1};
  uint32_t pos[4], neg[4];
  digits_pm32<L>(xs, q, m.thr, pos, neg);
  for (int k = 0; k < 4; ++k) {
    const int64_t pv = digit_value(pos[k], L), ngv = digit_value(neg[k], L);
    CHECK(pv >= bottom && pv <= top && mod_signed(pv, q) == (int64_t)xs[k], "digits_pm32<%d> q=%u x=%u", L, q,
          xs[k]);
    CHECK(ngv >= bottom && ngv <= top && mod_signed(-ngv, q) == (int64_t)xs[k], "digits_pm32<%d> neg q=%u x=%u",
          L, q, xs[k]);
  }
}

static void check_mod32(uint32_t q) {
  const int L = limbs_for_q32(q);
  const ModQ32 m = make_mod32(q, L < 2 ? 2 : L);
  // 64-bit words: edges next to multiples of q and the top of the range, then random
  const uint64_t k = UINT64_MAX / q;
  const uint64_t edges[] = {0, 1, q - 1ull, q, 2ull * q - 1, 2ull * q, UINT64_MAX, UINT64_MAX - 1, k * q,
                            k * q - 1, (k - 1) * q, 1ull << 62, (1ull << 62) + q, 1ull << 63};
  for (uint64_t x : edges) {
    CHECK(reduce_u64(x, m) == x % q, "reduce_u64 q=%u x=%llu", q, (unsigned long long)x);
    if (q < 0x80000000u)
      CHECK(reduce_u64_q31(x, m.mu, q) == x % q, "reduce_u64_q31 q=%u x=%llu", q, (unsigned long long)x);
  }
  for (int i = 0; i < 20000; ++i) {
    const uint64_t x = next64() >> (next64() & 63);
    CHECK(reduce_u64(x, m) == x % q, "reduce_u64 q=%u x=%llu", q, (unsigned long long)x);
    if (q < 0x80000000u)
      CHECK(reduce_u64_q31(x, m.mu, q) == x % q, "reduce_u64_q31 q=%u x=%llu", q, (unsigned long long)x);
    const int64_t y = (int64_t)(next64() >> 2) * ((next64() & 1) ? 1 : -1);  // |y| < 2^62
    CHECK((int64_t)reduce_i64(y, m) == mod_signed(y, q), "reduce_i64 q=%u y=%lld", q, (long long)y);
  }
  // 32-bit words
  const uint32_t k32 = UINT32_MAX / q;
  const uint32_t e32[] = {0u, 1u, q - 1, q, UINT32_MAX, UINT32_MAX - 1, k32 * q, k32 * q - 1, 0x80000000u};
  for (uint32_t x : e32) CHECK(reduce_u32(x, m) == x % q, "reduce_u32 q=%u x=%u", q, x);
  for (int i = 0; i < 20000; ++i) {
    const uint32_t x = (uint32_t)next64();
    CHECK(reduce_u32(x, m) == x % q, "reduce_u32 q=%u x=%u", q, x);
  }
  // digit splits, for every limb count whose window covers q
  const uint32_t xe[] = {0u, 1u, q - 1, q / 2, (q + 1) / 2 < q ? (q + 1) / 2 : 0u, 0x80u % q, 0x8080u % q,
                         0x808080u % q, 0x80808080u % q, 0x7F7F7F7Fu % q, 0x7F7F7F80u % q};
  for (int i = 0; i < 4000 + (int)(sizeof(xe) / sizeof(xe[0])); ++i) {
    const uint32_t x = i < (int)(sizeof(xe) / sizeof(xe[0])) ? xe[i] : (uint32_t)(next64() % q);
    if (q <= 256u) check_digits32<1>(q, x);
    if (q <= 65536u) check_digits32<2>(q, x);
    if (q <= (1u << 24)) check_digits32<3>(q, x);
    check_digits32<4>(q, x);
  }
}

static void check_mod64(uint64_t q) {
  const int L = limbs_for_q64(q);
  const ModQ64 m = make_mod64(q, L);
  CHECK(m.d >> 63 == 1 && (m.d >> m.sh) == q, "normalisation q=%llu", (unsigned long long)q);
  u128 pw = 1 % q;
  for (int s = 0; s < 16; ++s) {
    CHECK(m.r[s] == (uint64_t)pw, "r[%d] q=%llu", s, (unsigned long long)q);
    pw = (pw * 256) % q;
  }
  const int groups = (2 * L - 1 + 3) / 4;
  u128 rs = 0;
  for (int j = 0; j < groups; ++j) rs = (rs + m.r[4 * j]) % q;
  CHECK(m.foff == (uint64_t)((((u128)1 << 56) % q) * rs % q), "foff q=%llu", (unsigned long long)q);
  const uint64_t edges[] = {0, 1, q - 1, q, UINT64_MAX, UINT64_MAX - 1, UINT64_MAX - q, 1ull << 63};
  for (uint64_t hi : edges)
    for (uint64_t lo : edges) {
      const u128 x = ((u128)hi << 64) | lo;
      CHECK(mod_u128(hi, lo, m) == (uint64_t)(x % q), "mod_u128 q=%llu hi=%llu lo=%llu", (unsigned long long)q,
            (unsigned long long)hi, (unsigned long long)lo);
    }
  for (int i = 0; i < 40000; ++i) {
    const uint64_t hi = next64() >> (next64() & 63), lo = next64();
    const u128 x = ((u128)hi << 64) | lo;
    CHECK(mod_u128(hi, lo, m) == (uint64_t)(x % q), "mod_u128 q=%llu hi=%llu lo=%llu", (unsigned long long)q,
          (unsigned long long)hi, (unsigned long long)lo);
    CHECK(mod_u64(lo, m) == lo % q, "mod_u64 q=%llu x=%llu", (unsigned long long)q, (unsigned long long)lo);
    const uint64_t a = next64() % q, b = next64() % q;
    CHECK(addmod64(a, b, q) == (uint64_t)(((u128)a + b) % q), "addmod64 q=%llu", (unsigned long long)q);
    CHECK(submod64(a, b, q) == (uint64_t)(((u128)a + q - b) % q), "submod64 q=%llu", (unsigned long long)q);
    const U128 p = mul64x64(a, b);
    CHECK((((u128)p.hi << 64) | p.lo) == (u128)a * b, "mul64x64");
    const U128 sum = add128(U128{lo, hi}, U128{b, a});
    CHECK((((u128)sum.hi << 64) | sum.lo) == ((((u128)hi << 64) | lo) + (((u128)a << 64) | b)), "add128");
  }
  // a + b wrapping past 2^64 in addmod64
  if (q > (1ull << 63))
    CHECK(addmod64(q - 1, q - 1, q) == (uint64_t)(((u128)(q - 1) * 2) % q), "addmod64 wrap q=%llu",
          (unsigned long long)q);
}

// residue_centred: r = v (mod m) and r in [-128, 127] for every 32-bit v.
static void check_residue8(uint32_t m) {
  const int32_t r16 = (int32_t)((1u << 16) % m);
  const float mf = (float)m, im = 1.0f / (float)m;
  auto one = [&](int32_t v) {
    const int32_t r = residue_centred(v, m, r16, mf, im);
    int64_t d = ((int64_t)v - r) % (int64_t)m;
    CHECK(d == 0 && r >= -128 && r <= 127, "residue_centred m=%u v=%d -> %d", m, v, r);
  };
  for (int32_t v = -(1 << 18); v <= (1 << 18); ++v) one(v);
  for (int32_t hi = -32768; hi < 32768; hi += 1) {  // around every multiple of 2^16
    one((int32_t)((uint32_t)hi << 16));
    one((int32_t)((uint32_t)hi << 16) + 0xFFFF);
    one((int32_t)((uint32_t)hi << 16) + (int32_t)(next64() & 0xFFFF));
  }
  const int32_t e[] = {INT32_MAX, INT32_MIN, INT32_MIN + 1, INT32_MAX - 1, (int32_t)0x7F7F7F7F, (int32_t)0x80808080};
  for (int32_t v : e) one(v);
  for (int i = 0; i < 200000; ++i) one((int32_t)next64());
  // the fp32 step itself, exhaustively over every |x| < 2^23 + 2^16
  if (m < 256) {
    const int32_t xmax = (1 << 23) + (1 << 16);
    for (int32_t x = -xmax + 1; x < xmax; ++x) {
      const int32_t r = centred_mod_small(x, m, mf, im);
      if (r < -128 || r > 127 || ((int64_t)x - r) % (int64_t)m != 0) {
        CHECK(false, "centred_mod_small m=%u x=%d -> %d", m, x, r);
      }
    }
    g_cases += 2u * (uint32_t)xmax - 1;
  }
}

int main(int argc, char** argv) {
  if (argc > 1) g_state ^= strtoull(argv[1], nullptr, 10);
  const uint32_t q32[] = {2u, 3u, 17u, 251u, 256u, 257u, 3329u, 12289u, 65536u, 65537u, 1u << 24, (1u << 24) + 1,
                          1068236801u, 998244353u, (1u << 31) - 1, 1u << 31, (1u << 31) + 6, 4294967291u,
                          4294967295u};
  for (uint32_t q : q32) check_mod32(q);
  for (int i = 0; i < 24; ++i) {
    uint32_t q = (uint32_t)(next64() >> (32 + (next64() % 31)));
    check_mod32(q < 2 ? 2 : q);
  }
  const uint64_t q64[] = {0xFFFFFFFF00000001ull, 0xFFFFFFFFFFFFFFC5ull, (1ull << 63) + 1, (1ull << 62) - 57,
                          (1ull << 40) - 87, (1ull << 32) + 15, 3329ull, 17ull, 2ull, 3ull, UINT64_MAX - 1};
  for (uint64_t q : q64) check_mod64(q);
  for (int i = 0; i < 24; ++i) {
    uint64_t q = next64() >> (next64() % 62);
    check_mod64(q < 2 ? 2 : q);
  }
  const uint32_t m8[] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 2, 3, 5, 7, 17, 127, 128, 254};
  for (uint32_t m : m8) check_residue8(m);
  printf("ok %llu\n", g_cases);
  return 0;
}
