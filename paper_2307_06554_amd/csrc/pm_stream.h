// K-streaming split-limb MFMA kernel: 64-bit moduli (up to 8 limbs) at every
// degree, and 32-bit moduli at degrees too large to hold both operands in LDS.
//
// Same recast as the resident kernel (C[z][u] = sum_(d,w) A[z][(d,w)] B[(d,w)][u],
// n = t*r, Eq. (3) Toeplitz tiles and the Sec. 2.5 block split), with t <= 64
// and one workgroup per 64 (z) x 64 (u) block of one product.  The K loop runs
// over d in chunks of dc values:
//   - A (reversed ext window of the chunk) is double-buffered in LDS;
//   - B rows v = u - d live in a ring of 128 rows indexed by v mod 128 (a chunk
//     uses dc + 63 rows and the next chunk's dc new rows never collide);
//   - the input words of chunk c+1 are loaded into registers before chunk c's
//     MFMAs and converted into LDS after them.
// Accumulator bound (K-split): a shift class holds at most L limb pairs of
// |product| <= 2^14, so its int32 sum is exact for K <= (2^31-1) / (L 2^14);
// the host sets flush_every so that every flush covers at most 2^17 / L - 1 K
// values (32767 for L = 4, 16383 for L = 8).  A flush folds sum_s T_s 2^(8s)
// into a running residue mod q with 128-bit arithmetic (Sec. 2.4 limbs
// recombined, then the modular reduction the paper leaves to Barrett /
// Montgomery, Sec. 2.6).  In grouped plans a block's chunks can be cut into
// runs on several workgroups (kparts), whose residues a second kernel adds.
#pragma once
#include "pm_common.h"
#include "pm_wide.h"
#include "pm_mfma32.h"

namespace pm {

constexpr int kMaxQS = 8;        // moduli per streaming launch
constexpr int kRing = 128;       // B rows held in LDS
constexpr int kStreamThreads = 256;

struct StreamParams {
  const void* a;
  const void* b;
  void* c;
  uint64_t nprod;
  uint32_t n, t, log2t, r;
  uint32_t spd, log2spd, rowlen, rs;  // K-steps per d, bytes per B row read, row stride
  uint32_t tz;            // 32-row z tiles in use (1 or 2)
  uint32_t ublocks;       // 64-column workgroup blocks per product
  uint32_t dc;            // d values per chunk
  uint32_t nchunks;       // r / dc
  uint32_t flush_every;   // chunks between int32 -> residue flushes
  uint32_t a_win;         // bytes per limb of one A window buffer
  uint32_t lds_b;         // LDS offset of the B ring
  uint32_t lds_res;       // L = 8: LDS offset of the running residues, [16][256] words
  uint32_t lc, nq_total, l0;  // product i -> global (i/lc)*nq_total + l0 + i%lc, modulus i%lc
  uint32_t lrep;              // > 1: product i is global i with modulus (i/lrep)%lc
  uint32_t b_shared;          // 1: one b per channel, b + (l0 + channel) * n, for every product
  uint32_t cyclic;            // 1: ring Z_q[x]/(x^n - 1): wrapped terms keep their sign
  // K split across workgroups (grouped plans): block (product, u-block) is cut into kparts
  // runs of nchunks / kparts chunks; run p stores its residues where c's would go in
  // part_ws + p * nprod * n, and a separate kernel adds the runs up mod q.
  uint32_t kparts;
  void* part_ws;              // [kparts][nprod][n] words
  ModQ64 mods[kMaxQS];
};

template <typename W>
__device__ __forceinline__ uint64_t word_reduce(W x, const ModQ64& m) {
  if (sizeof(W) == 4) {
    uint64_t v = (uint64_t)x;
    return v < m.q ? v : mod_u64(v, m);
  }
  const uint64_t v = (uint64_t)x;
  return v < m.q ? v : mod_u64(v, m);
}

// L digits of the residue x in [0, q), packed little-endian (digit i in byte i).
template <int L>
__device__ __forceinline__ uint64_t digits64(uint64_t x, const ModQ64& m) {
  constexpr uint64_t B = limb_bias(L);
  const uint64_t v = x <= m.thr ? x : x - m.q;  // wraps mod 2^64: the representative in W_L
  return (v + B) ^ B;
}
template <int L>
__device__ __forceinline__ uint64_t neg_digits64(uint64_t x, const ModQ64& m) {
  return digits64<L>(x == 0 ? 0ull : m.q - x, m);
}

// Byte i of four packed digit words -> plane i, one dword per plane: the byte
// transpose of the resident kernel on the low words (planes 0-3) and, past
// four limbs, on the high words (planes 4-7).
template <int L>
__device__ __forceinline__ void transpose_store64(uint8_t* base, uint32_t plane, uint32_t off, const uint64_t (&w)[4]) {
  const uint32_t lo[4] = {(uint32_t)w[0], (uint32_t)w[1], (uint32_t)w[2], (uint32_t)w[3]};
  transpose_store<(L < 4 ? L : 4)>(base, plane, off, lo);
  if constexpr (L > 4) {
    const uint32_t hi[4] = {(uint32_t)(w[0] >> 32), (uint32_t)(w[1] >> 32), (uint32_t)(w[2] >> 32),
                            (uint32_t)(w[3] >> 32)};
    transpose_store<L - 4>(base + 4 * plane, plane, off, hi);
  }
}

// Four consecutive words starting at element `idx` (idx a multiple of 4).
template <typename W>
struct Quad {
  W w[4];
};
template <typename W>
__device__ __forceinline__ Quad<W> load_quad(const W* p) {
  Quad<W> q;
  if (sizeof(W) == 4) {
    const uint4 x = *(const uint4*)p;
    q.w[0] = (W)x.x; q.w[1] = (W)x.y; q.w[2] = (W)x.z; q.w[3] = (W)x.w;
  } else {
    const uint4 x = *(const uint4*)p;
    const uint4 y = *(const uint4*)(p + 2);
    q.w[0] = (W)(((uint64_t)x.y << 32) | x.x);
    q.w[1] = (W)(((uint64_t)x.w << 32) | x.z);
    q.w[2] = (W)(((uint64_t)y.y << 32) | y.x);
    q.w[3] = (W)(((uint64_t)y.w << 32) | y.z);
  }
  return q;
}

// Staging items of one workgroup.  An item is four consecutive words.
//   A item m: ext[4m .. 4m+3] of the chunk window (a, -a wrapped, or zero).
//   B item:   words w = 4k .. 4k+3 of source row v of the ring (b or -b or zero).
struct StreamItem {
  int kind;   // 0 none/zero, 1 A, 2 B
  int e;      // A: group m; B: row v
  int k;      // B: word group in the row
};

struct ChunkItems {
  int a_groups;   // A groups of the window
  int a_m0;       // first group index (lowest ext index / 4)
  int b_rows;     // rows staged
  int b_v0;       // first row
  int row_groups; // word groups per row
  __device__ __forceinline__ int count() const { return a_groups + b_rows * row_groups; }
  __device__ __forceinline__ StreamItem item(int i) const {
    StreamItem it;
    if (i < a_groups) { it.kind = 1; it.e = a_m0 + i; it.k = 0; return it; }
    i -= a_groups;
    it.kind = 2;
    it.e = b_v0 + i / row_groups;
    it.k = i % row_groups;
    return it;
  }
};

__device__ __forceinline__ ChunkItems chunk_items(const StreamParams& P, int c, int U0, bool first) {
  ChunkItems ci;
  const int D0 = c * (int)P.dc;
  const int I1 = (D0 + (int)P.dc - 1) * (int)P.t + 32 * (int)P.tz - 1;  // highest ext index of the window
  ci.a_groups = (int)(P.a_win >> 2);
  ci.a_m0 = ((I1 + 1) >> 2) - ci.a_groups;
  ci.row_groups = (int)(P.rowlen >> 2);
  if (first) {
    // every row this chunk reads: v = u - d for the block's 64 u and the chunk's dc d
    ci.b_v0 = U0 - (c + 1) * (int)P.dc + 1;
    ci.b_rows = 63 + (int)P.dc;
  } else {
    ci.b_v0 = U0 - (c + 1) * (int)P.dc + 1;
    ci.b_rows = (int)P.dc;
  }
  return ci;
}

// Global source of an item (nullptr: the item is all zeros).
template <typename W>
__device__ __forceinline__ const W* item_ptr(const StreamParams& P, const StreamItem& it, uint64_t gp, uint64_t bgp,
                                             bool* neg) {
  const int n = (int)P.n, t = (int)P.t, r = (int)P.r;
  *neg = false;
  if (it.kind == 1) {
    const int i0 = 4 * it.e;
    if (n < 4) return nullptr;  // handled element-wise
    if (i0 >= 0 && i0 < n) return (const W*)P.a + gp * P.n + i0;
    if (i0 < 0 && i0 >= -n) { *neg = !P.cyclic; return (const W*)P.a + gp * P.n + (n + i0); }
    return nullptr;
  }
  if (it.kind == 2) {
    const int v = it.e, w = 4 * it.k;
    if (t < 4 || w >= t) return nullptr;
    if (v >= 0 && v < r) return (const W*)P.b + bgp * P.n + (size_t)v * t + w;
    if (v < 0 && v > -r) { *neg = !P.cyclic; return (const W*)P.b + bgp * P.n + (size_t)(v + r) * t + w; }
  }
  return nullptr;
}

// Convert one item (its four words already loaded, or element-wise for tiny n) and write it.
template <int L, typename W>
__device__ __forceinline__ void item_write(const StreamParams& P, const StreamItem& it, const Quad<W>& x, bool live,
                                           bool neg, uint64_t gp, uint64_t bgp, const ModQ64& m, uint8_t* abuf,
                                           uint8_t* ring, int I1) {
  uint64_t d[4] = {0, 0, 0, 0};
  const int n = (int)P.n, t = (int)P.t, r = (int)P.r;
  if (it.kind == 1) {
    const int i0 = 4 * it.e;
    if (n < 4) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int idx = i0 + k;
        if (idx >= 0 && idx < n) d[k] = digits64<L>(word_reduce<W>(((const W*)P.a)[gp * P.n + idx], m), m);
        else if (idx < 0 && idx > -n) {
          const uint64_t xr = word_reduce<W>(((const W*)P.a)[gp * P.n + n + idx], m);
          d[k] = P.cyclic ? digits64<L>(xr, m) : neg_digits64<L>(xr, m);
        }
      }
    } else if (live) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t xr = word_reduce<W>(x.w[k], m);
        d[k] = neg ? neg_digits64<L>(xr, m) : digits64<L>(xr, m);
      }
    }
    // reversed: position p = I1 - idx; byte j of dword (I1 - i0 - 3)/4 holds idx = i0 + 3 - j
    const uint64_t w4[4] = {d[3], d[2], d[1], d[0]};
    transpose_store64<L>(abuf, P.a_win, (uint32_t)(I1 - i0 - 3), w4);
  } else if (it.kind == 2) {
    const int v = it.e, w = 4 * it.k;
    if (t < 4) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int ww = w + k;
        if (ww >= t) continue;
        if (v >= 0 && v < r) d[k] = digits64<L>(word_reduce<W>(((const W*)P.b)[bgp * P.n + (size_t)v * t + ww], m), m);
        else if (v < 0 && v > -r) {
          const uint64_t xr = word_reduce<W>(((const W*)P.b)[bgp * P.n + (size_t)(v + r) * t + ww], m);
          d[k] = P.cyclic ? digits64<L>(xr, m) : neg_digits64<L>(xr, m);
        }
      }
    } else if (live) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t xr = word_reduce<W>(x.w[k], m);
        d[k] = neg ? neg_digits64<L>(xr, m) : digits64<L>(xr, m);
      }
    }
    const uint32_t slot = (uint32_t)(v & (kRing - 1));
    transpose_store64<L>(ring, kRing * P.rs, slot * P.rs + (uint32_t)w, d);
  }
}

// Running residues: res = (res + sum_s T_s 2^(8s)) mod q, then T_s = 0.  The
// classes are taken four at a time: Y_j = sum_{k<4} T_{4j+k} 2^(8k) is exact in
// int64 (|Y_j| < 2^31 (1 + 2^8 + 2^16 + 2^24) < 2^56), and with R_j = 2^(32j) mod q
// the sum sum_j (Y_j + 2^56) R_j is a non-negative integer below 4 * 2^57 * 2^64
// = 2^123.  One remainder of it, less foff = (2^56 sum_j R_j) mod q, is the
// flush's contribution (sum_s T_s 2^(8s) = sum_j Y_j 2^(32j)).
template <int L>
__device__ __forceinline__ uint64_t flush_value(const v16i (&acc)[2 * L - 1], int rr, const ModQ64& m) {
  constexpr int S = 2 * L - 1, G = (S + 3) / 4;
  U128 x{0, 0};
#pragma unroll
  for (int j = 0; j < G; ++j) {
    int64_t y = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (4 * j + k < S) y += (int64_t)acc[4 * j + k][rr] * ((int64_t)1 << (8 * k));
    const uint64_t yo = (uint64_t)y + ((uint64_t)1 << 56);  // in (0, 2^57)
    x = add128(x, j == 0 ? U128{yo, 0} : mul64x64(yo, m.r[4 * j]));
  }
  return submod64(mod_u128(x.hi, x.lo, m), m.foff, m.q);
}
// Running residues in registers (up to four limbs; eight limbs: stream8_block).
template <int L, typename W>
__device__ __forceinline__ void stream_flush(v16i (&acc)[2 * L - 1], W (&res)[16], const ModQ64& m) {
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const uint64_t v = flush_value<L>(acc, rr, m);
    res[rr] = (W)addmod64((uint64_t)res[rr], v, m.q);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int s = 0; s < 2 * L - 1; ++s) acc[s] = v16i{};
}

// One 64 (z) x 64 (u) block of one product, the whole K loop.  Block index
// wg = product * ublocks + u-block.
template <int L, typename W>
__device__ __forceinline__ void stream_block(const StreamParams& P, uint64_t item, uint8_t* smem) {
  static_assert(L <= 4, "eight limbs run stream8_block");
  const uint64_t wg = item / P.kparts;  // block (product, u-block)
  const uint32_t part = (uint32_t)(item - wg * P.kparts);
  const int cpp = (int)(P.nchunks / P.kparts);
  const int c0 = (int)part * cpp, c1 = c0 + cpp;
  const uint64_t prod = wg / P.ublocks;
  const int U0 = 64 * (int)(wg - prod * P.ublocks);
  const uint32_t li = P.lrep > 1 ? (uint32_t)((prod / P.lrep) % P.lc) : (uint32_t)(prod % P.lc);
  const uint64_t gp = P.lrep > 1 ? prod : (prod / P.lc) * P.nq_total + P.l0 + li;
  const uint64_t bgp = P.b_shared ? (uint64_t)(P.l0 + li) : gp;
  const ModQ64& m = P.mods[li];
  uint8_t* ring = smem + P.lds_b;
  const int wave = (int)(threadIdx.x >> 6);
  const int lane = (int)(threadIdx.x & 63);
  const int zt = wave & 1, ut = wave >> 1;
  const bool active = zt < (int)P.tz;
  const int z0 = 32 * zt, u0 = U0 + 32 * ut;
  const int zl = lane & 31, g = lane >> 5;
  const int t = (int)P.t, rs = (int)P.rs;

  // ---- first chunk: everything it needs, loaded synchronously
  {
    const ChunkItems ci = chunk_items(P, c0, U0, true);
    const int I1 = (c0 * (int)P.dc + (int)P.dc - 1) * t + 32 * (int)P.tz - 1;
    uint8_t* abuf0 = smem + (c0 & 1) * (L * P.a_win);
    for (int i = threadIdx.x; i < ci.count(); i += kStreamThreads) {
      const StreamItem it = ci.item(i);
      bool neg;
      const W* src = item_ptr<W>(P, it, gp, bgp, &neg);
      Quad<W> x{};
      if (src) x = load_quad<W>(src);
      item_write<L, W>(P, it, x, src != nullptr, neg, gp, bgp, m, abuf0, ring, I1);
    }
  }
  __syncthreads();

  v16i acc[2 * L - 1];
#pragma unroll
  for (int s = 0; s < 2 * L - 1; ++s) acc[s] = v16i{};
  W res[16];  // running residues of the lane's 16 outputs
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) res[rr] = 0;

  // per-lane A base: S = S_base + (dc - 1 - dl) t + w0 inside the chunk's window
  const int S_base = 32 * (int)P.tz - 1 - z0 - zl + 16 * g;
  constexpr int kItems = 3;  // items per thread carried over a chunk (dc <= 16, t <= 64)
  const int steps = (int)(P.dc << P.log2spd);

  for (int c = c0; c < c1; ++c) {
    // ---- issue the next chunk's loads
    const bool more = c + 1 < c1;
    ChunkItems cn{};
    Quad<W> pf[kItems];
    bool pl[kItems], pn[kItems];
    if (more) {
      cn = chunk_items(P, c + 1, U0, false);
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const int i = (int)threadIdx.x + k * kStreamThreads;
        pl[k] = false;
        pn[k] = false;
        if (i < cn.count()) {
          const StreamItem it = cn.item(i);
          const W* src = item_ptr<W>(P, it, gp, bgp, &pn[k]);
          if (src) { pf[k] = load_quad<W>(src); pl[k] = true; }
        }
      }
    }
    // ---- this chunk's MFMAs
    if (active) {
      // the lane's dword base and byte shift are fixed: a K-step moves the runs by a
      // multiple of four bytes (for t = 1 or 2, n = t and d is always 0)
      const uint8_t* abuf = smem + (c & 1) * (L * P.a_win) + 4 * (S_base >> 2);
      const uint32_t sh = (uint32_t)(S_base & 3);
      const int D0 = c * (int)P.dc;
      uint32_t araw[L][5];
      v4i af[L], b[L];
      auto S_of = [&](int st) {
        const int dl = st >> P.log2spd;
        return ((int)P.dc - 1 - dl) * t + ((st & ((int)P.spd - 1)) << 5);
      };
      auto B_of = [&](int st) {
        const int d = D0 + (st >> P.log2spd);
        return ((u0 + zl - d) & (kRing - 1)) * rs + ((st & ((int)P.spd - 1)) << 5) + 16 * g;
      };
      // af: step st aligned; araw: step st + 1's runs; the last steps re-read their own
      araw_load<L>(araw, abuf, P.a_win, S_of(0));
      a_align<L>(af, araw, sh);
      araw_load<L>(araw, abuf, P.a_win, S_of(steps > 1 ? 1 : 0));
      b_load<L>(b, ring, kRing * P.rs, B_of(0));
      for (int st = 0; st < steps; ++st) {
        const int sn = st + 1 < steps ? st + 1 : st;
        const int s2 = st + 2 < steps ? st + 2 : steps - 1;
        mfma_step_tail<L>(acc, af, araw, sh, abuf, P.a_win, S_of(s2), b, ring, kRing * P.rs, B_of(sn));
      }
      if (!more || (c + 1 - c0) % (int)P.flush_every == 0) stream_flush<L, W>(acc, res, m);
    }
    if (!more) break;
    // ---- convert and write the next chunk (its A buffer and ring rows are not read now)
    {
      uint8_t* abuf_n = smem + ((c + 1) & 1) * (L * P.a_win);
      const int I1n = ((c + 1) * (int)P.dc + (int)P.dc - 1) * t + 32 * (int)P.tz - 1;
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const int i = (int)threadIdx.x + k * kStreamThreads;
        if (i < cn.count()) item_write<L, W>(P, cn.item(i), pf[k], pl[k], pn[k], gp, bgp, m, abuf_n, ring, I1n);
      }
      for (int i = (int)threadIdx.x + kItems * kStreamThreads; i < cn.count(); i += kStreamThreads) {
        const StreamItem it = cn.item(i);
        bool neg;
        const W* src = item_ptr<W>(P, it, gp, bgp, &neg);
        Quad<W> x{};
        if (src) x = load_quad<W>(src);
        item_write<L, W>(P, it, x, src != nullptr, neg, gp, bgp, m, abuf_n, ring, I1n);
      }
    }
    __syncthreads();
  }
  if (!active) return;

  // ---- store the residues: lane holds z = z0 + 8 blk + 4 g + e, u = u0 + zl
  const int u = u0 + zl;
  if (u >= (int)P.r) return;
  W* C = (P.kparts > 1 ? (W*)P.part_ws + (uint64_t)part * P.nprod * P.n : (W*)P.c) + gp * P.n;
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const int z = z0 + 8 * (rr >> 2) + 4 * g + (rr & 3);
    if (z < t) C[(size_t)u * t + z] = res[rr];
  }
}

// ---------------------------------------------------------------------------
// Eight limbs (64-bit words): the 15 shift classes s = i + j split by parity over
// a pair of waves, so that a wave holds 8 (even s) or 7 (odd s) accumulator sets
// instead of 15 and two waves fit on a SIMD.  512 threads: wave w computes tile
// (zt, ut) = (w & 1, (w >> 1) & 1) of the 64 x 64 block for the classes of parity
// par = w >> 2, i.e. the limb pairs (i, j) with i + j = par (mod 2), 32 of the 64.
// Both waves of a pair read the same staged runs; each flushes its own classes'
// part sum_s T_s 2^(8s) into the pair's running residues in LDS, the two at
// different chunks (so the updates never overlap) and the last after a barrier.
// ---------------------------------------------------------------------------
constexpr int kStream8Threads = 512;

template <int PAR>
__device__ __forceinline__ uint64_t flush_value_par(const v16i (&acc)[8], int rr, const ModQ64& m) {
  U128 x{0, 0};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int64_t y = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int sc = 4 * j + k;
      if (sc < 15 && (sc & 1) == PAR) y += (int64_t)acc[sc >> 1][rr] * ((int64_t)1 << (8 * k));
    }
    const uint64_t yo = (uint64_t)y + ((uint64_t)1 << 56);  // in (0, 2^57), as in flush_value
    x = add128(x, j == 0 ? U128{yo, 0} : mul64x64(yo, m.r[4 * j]));
  }
  return submod64(mod_u128(x.hi, x.lo, m), m.foff, m.q);
}

template <int PAR, typename W>
__device__ __forceinline__ void stream_flush_par(v16i (&acc)[8], W* resl, const ModQ64& m) {
  const uint32_t tid = threadIdx.x & (kStreamThreads - 1);
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const uint64_t v = flush_value_par<PAR>(acc, rr, m);
    W& r = resl[rr * kStreamThreads + tid];
    r = (W)addmod64((uint64_t)r, v, m.q);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) acc[s] = v16i{};
}

__device__ __forceinline__ v4i align_run(const uint32_t (&x)[5], uint32_t sh) {
  v4i a;
  a[0] = (int)__builtin_amdgcn_alignbyte(x[1], x[0], sh);
  a[1] = (int)__builtin_amdgcn_alignbyte(x[2], x[1], sh);
  a[2] = (int)__builtin_amdgcn_alignbyte(x[3], x[2], sh);
  a[3] = (int)__builtin_amdgcn_alignbyte(x[4], x[3], sh);
  return a;
}
__device__ __forceinline__ void load_run(uint32_t (&x)[5], const uint8_t* plane, int S) {
  const uint32_t* p = (const uint32_t*)plane + (S >> 2);
#pragma unroll
  for (int k = 0; k < 5; ++k) x[k] = p[k];
}

// One K-step of the parity-PAR classes.  On entry a holds limb 0's aligned A run
// of this step, x[0] and x[1] the raw runs of limbs 1 and 2, b all eight B runs.
// A limbs are taken one at a time, their runs read two limbs ahead (limb k of
// the next step counted as limb 8 + k); the B runs of the next step are read
// once the last limb that uses them has issued (limb 6 for j = PAR mod 2, limb 7
// for the others).  On exit the registers hold the next step's entry state.
template <int PAR>
__device__ __forceinline__ void mfma_step_par(v16i (&acc)[8], v4i& a, uint32_t (&x)[2][5], v4i (&b)[8],
                                              const uint8_t* abuf, uint32_t a_win, int S, int S_next,
                                              const uint8_t* ring, uint32_t b_plane, int boff_next, uint32_t sh) {
  const uint32_t sh_next = sh;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int j = (PAR + i) & 1; j < 8; j += 2)
      acc[(i + j) >> 1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b[j], acc[(i + j) >> 1], 0, 0, 0);
    a = align_run(x[i & 1], i + 1 < 8 ? sh : sh_next);  // limb i + 1
    const int k = i + 3;                                 // the limb whose runs are read now
    load_run(x[i & 1], abuf + (k & 7) * a_win, k < 8 ? S : S_next);
    if (i == 6) {
#pragma unroll
      for (int j = PAR; j < 8; j += 2) b[j] = *(const v4i*)(ring + j * b_plane + boff_next);
    } else if (i == 7) {
#pragma unroll
      for (int j = 1 - PAR; j < 8; j += 2) b[j] = *(const v4i*)(ring + j * b_plane + boff_next);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The K loop of one chunk for this wave's parity.  A K-step moves the A runs by
// (dc - 1 - d) t + 32 c bytes, a multiple of four: for t = 1 or 2 (n = t, r = 1) d is
// always 0.  So each run keeps the byte shift S_base & 3 and the lane's dword base,
// and a step adds a uniform offset.
template <int PAR>
__device__ __forceinline__ void chunk_mfma_par(v16i (&acc)[8], const uint8_t* abuf, uint32_t a_win,
                                               const uint8_t* ring, uint32_t b_plane, int S_base, int dc, int t,
                                               int spd, uint32_t log2spd, int D0, int u0, int zl, int g, int rs,
                                               int steps) {
  abuf += 4 * (S_base >> 2);
  const uint32_t sh = (uint32_t)(S_base & 3);
  auto S_of = [&](int st) { return (dc - 1 - (st >> log2spd)) * t + ((st & (spd - 1)) << 5); };
  auto B_of = [&](int st) {
    const int d = D0 + (st >> log2spd);
    return ((u0 + zl - d) & (kRing - 1)) * rs + ((st & (spd - 1)) << 5) + 16 * g;
  };
  v4i b[8];
  const int B0 = B_of(0);
#pragma unroll
  for (int j = 0; j < 8; ++j) b[j] = *(const v4i*)(ring + j * b_plane + B0);
  uint32_t x[2][5];
  const int S0 = S_of(0);
  load_run(x[0], abuf, S0);
  v4i a = align_run(x[0], sh);
  load_run(x[0], abuf + a_win, S0);
  load_run(x[1], abuf + 2 * a_win, S0);
  for (int st = 0; st < steps; ++st) {
    const int sn = st + 1 < steps ? st + 1 : st;  // the last step re-reads its own runs
    mfma_step_par<PAR>(acc, a, x, b, abuf, a_win, S_of(st), S_of(sn), ring, b_plane, B_of(sn), sh);
  }
}

template <int PAR, typename W>
__device__ __forceinline__ void stream8_block(const StreamParams& P, uint64_t item, uint8_t* smem) {
  const uint64_t wg = item / P.kparts;  // block (product, u-block)
  const uint32_t part = (uint32_t)(item - wg * P.kparts);
  const int cpp = (int)(P.nchunks / P.kparts);
  const int c0 = (int)part * cpp, c1 = c0 + cpp;
  const uint64_t prod = wg / P.ublocks;
  const int U0 = 64 * (int)(wg - prod * P.ublocks);
  const uint32_t li = P.lrep > 1 ? (uint32_t)((prod / P.lrep) % P.lc) : (uint32_t)(prod % P.lc);
  const uint64_t gp = P.lrep > 1 ? prod : (prod / P.lc) * P.nq_total + P.l0 + li;
  const uint64_t bgp = P.b_shared ? (uint64_t)(P.l0 + li) : gp;
  const ModQ64& m = P.mods[li];
  uint8_t* ring = smem + P.lds_b;
  const uint32_t tid = threadIdx.x & (kStreamThreads - 1);  // position in the wave pair's tile
  const int wave = (int)(tid >> 6);
  const int lane = (int)(tid & 63);
  const int zt = wave & 1, ut = wave >> 1;
  const bool active = zt < (int)P.tz;
  const int z0 = 32 * zt, u0 = U0 + 32 * ut;
  const int zl = lane & 31, g = lane >> 5;
  const int t = (int)P.t, rs = (int)P.rs;
  const uint32_t b_plane = kRing * P.rs;

  // ---- first chunk, loaded synchronously by all 512 threads
  {
    const ChunkItems ci = chunk_items(P, c0, U0, true);
    const int I1 = (c0 * (int)P.dc + (int)P.dc - 1) * t + 32 * (int)P.tz - 1;
    uint8_t* abuf0 = smem + (c0 & 1) * (8 * P.a_win);
    for (int i = threadIdx.x; i < ci.count(); i += kStream8Threads) {
      const StreamItem it = ci.item(i);
      bool neg;
      const W* src = item_ptr<W>(P, it, gp, bgp, &neg);
      Quad<W> x{};
      if (src) x = load_quad<W>(src);
      item_write<8, W>(P, it, x, src != nullptr, neg, gp, bgp, m, abuf0, ring, I1);
    }
  }
  // running residues of the pair's outputs in LDS, zeroed by the even-class wave
  W* resl = (W*)(smem + P.lds_res);
  if (PAR == 0) {
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) resl[rr * kStreamThreads + tid] = 0;
  }
  __syncthreads();

  v16i acc[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) acc[s] = v16i{};
  const int S_base = 32 * (int)P.tz - 1 - z0 - zl + 16 * g;
  const int steps = (int)(P.dc << P.log2spd);
  const int fe = (int)P.flush_every;  // >= 15 for eight limbs
  for (int c = c0; c < c1; ++c) {
    const bool more = c + 1 < c1;
    if (active) {
      const uint8_t* abuf = smem + (c & 1) * (8 * P.a_win);
      chunk_mfma_par<PAR>(acc, abuf, P.a_win, ring, b_plane, S_base, (int)P.dc, t, (int)P.spd, P.log2spd,
                          c * (int)P.dc, u0, zl, g, rs, steps);
      // even classes flush every fe chunks, odd ones half a period later; the last
      // chunk's even flush is here, its odd flush after the loop
      const int done = c + 1 - c0;
      if (more ? (done + PAR * (fe / 2)) % fe == 0 : PAR == 0) stream_flush_par<PAR, W>(acc, resl, m);
    }
    if (!more) break;
    // The even-class waves, which the MFMA arbitration serves first, stage the next
    // chunk (its A buffer and ring rows are not read by this chunk) while the
    // odd-class waves are still in their K loop.
    if (PAR == 0) {
      const ChunkItems cn = chunk_items(P, c + 1, U0, false);
      uint8_t* abuf_n = smem + ((c + 1) & 1) * (8 * P.a_win);
      const int I1n = ((c + 1) * (int)P.dc + (int)P.dc - 1) * t + 32 * (int)P.tz - 1;
      constexpr int kPf = 3;  // loads in flight per thread (a chunk has at most 3 * 256 items for t <= 64)
      for (int base = 0; base < cn.count(); base += kPf * kStreamThreads) {
        Quad<W> pf[kPf];
        bool pl[kPf], pn[kPf];
#pragma unroll
        for (int k = 0; k < kPf; ++k) {
          const int i = base + (int)tid + k * kStreamThreads;
          pl[k] = false;
          pn[k] = false;
          if (i < cn.count()) {
            const W* src = item_ptr<W>(P, cn.item(i), gp, bgp, &pn[k]);
            if (src) { pf[k] = load_quad<W>(src); pl[k] = true; }
          }
        }
#pragma unroll
        for (int k = 0; k < kPf; ++k) {
          const int i = base + (int)tid + k * kStreamThreads;
          if (i < cn.count()) item_write<8, W>(P, cn.item(i), pf[k], pl[k], pn[k], gp, bgp, m, abuf_n, ring, I1n);
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();  // the even flush of the last chunk is in LDS
  if (PAR == 1 && active) stream_flush_par<1, W>(acc, resl, m);
  __syncthreads();  // both halves of every residue are in
  if (PAR == 1 || !active) return;

  // ---- store the residues: lane holds z = z0 + 8 blk + 4 g + e, u = u0 + zl
  const int u = u0 + zl;
  if (u >= (int)P.r) return;
  W* C = (P.kparts > 1 ? (W*)P.part_ws + (uint64_t)part * P.nprod * P.n : (W*)P.c) + gp * P.n;
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const int z = z0 + 8 * (rr >> 2) + 4 * g + (rr & 3);
    if (z < t) C[(size_t)u * t + z] = resl[rr * kStreamThreads + tid];
  }
}

template <typename W>
__global__ __launch_bounds__(kStream8Threads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void stream8_kernel(const StreamParams P) {
  extern __shared__ __align__(16) uint8_t smem[];
  if (threadIdx.x < kStreamThreads) stream8_block<0, W>(P, blockIdx.x, smem);
  else stream8_block<1, W>(P, blockIdx.x, smem);
}

template <int L, typename W, int WPE>
__global__ __launch_bounds__(kStreamThreads) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void stream_kernel(const StreamParams P) {
  extern __shared__ __align__(16) uint8_t smem[];
  stream_block<L, W>(P, blockIdx.x, smem);
}

}  // namespace pm
