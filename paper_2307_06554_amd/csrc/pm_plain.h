// Plain integer schoolbook kernel: the comparison baseline for the MFMA path.
// c_j = sum_i a_i * bx[j - i] with bx[k] = b_k (k >= 0) and bx[k] = q - b_{n+k}
// (k < 0), i.e. the negacyclic wrap folded into the second operand as in
// Eq. (3); every term is a non-negative 32x32->64-bit product of residues
// (v_mad_u64_u32, multiply and 64-bit accumulate in one instruction).
//
// Each thread computes kPlainR = 8 consecutive outputs j0 .. j0 + 7.  For input
// index i they need bx[j0 - i .. j0 - i + 7]: from i to i + 1 the window slides
// down by one value.  The loop takes 16 inputs per step: their a values (two
// broadcast LDS read pairs) and the 16 window values that slide in (two LDS
// read pairs) feed 128 multiply-adds, with every operand in a register.
//
// Sums are lazy.  A 64-bit sum s is folded to hi * R + lo (R = 2^32 mod q,
// hi and lo its words; same value mod q) by one multiply-add; after a fold
// s <= (2^32 - 1)(R + 1), and F = floor((2^64 - 1 - that) / (q - 1)^2) >= 1 more
// products fit before the next (F = 16 for a 30-bit q).  The sum is reduced
// mod q (Barrett) once, at the end.
#pragma once
#include "pm_common.h"

namespace pm {

struct PlainParams {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* c;
  uint64_t batch;
  uint32_t n;
  uint32_t blocks_per_prod;  // output chunks of kPlainOut per product
  uint32_t fold_bodies;      // 16-input steps between folds; 0: fold after every input (F < 16)
  uint32_t r32;              // 2^32 mod q
  ModQ32 m;
};

constexpr int kPlainThreads = 512;  // two halves of 256 threads
constexpr int kPlainR = 8;          // consecutive outputs per thread
constexpr int kPlainOut = 256 * kPlainR;  // outputs per workgroup
constexpr int kPlainKC = 2048;      // inputs staged in LDS per chunk (multiple of 32)
// sb holds bx from offset `off` in [16, 20); below it zero words for the window
// reads of the padded inputs (a chunk is padded to a multiple of 32 inputs).
constexpr int kPlainSB = kPlainKC + kPlainOut + 32;

__device__ __forceinline__ uint64_t plain_fold(uint64_t s, uint32_t r32) {
  return (uint64_t)(uint32_t)(s >> 32) * r32 + (uint32_t)s;
}

// Eight inputs (a values av[t]) against outputs e = 0..7: output e at input t
// takes the window value at e - t, w[e - t] (values at the eight inputs'
// first input) or, below 0, the value that slid in, nv[8 + e - t].
template <bool kFoldEach>
__device__ __forceinline__ void plain_unit(const uint32_t (&av)[8], const uint32_t (&w)[8], const uint32_t (&nv)[8],
                                           uint32_t r32, uint64_t (&s)[kPlainR]) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const uint64_t ai = av[t];
#pragma unroll
    for (int e = 0; e < kPlainR; ++e) {
      const int k = e - t;
      s[e] += ai * (uint64_t)(k >= 0 ? w[k] : nv[8 + k]);
    }
    if (kFoldEach) {
#pragma unroll
      for (int e = 0; e < kPlainR; ++e) s[e] = plain_fold(s[e], r32);
    }
  }
}

__device__ __forceinline__ void plain_load8(uint32_t (&v)[8], const uint32_t* p) {
  const uint4 x = *(const uint4*)p, y = *(const uint4*)(p + 4);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
}

// `count` (multiple of 16) inputs of a chunk: sa[ii] = a value of input ii
// (zero past the chunk's end); sb[base + e - ii] is the value of output e at
// input ii.  Sums are folded every `fold_bodies` steps of 16 inputs and at the end.
template <bool kFoldEach>
__device__ __forceinline__ void plain_chunk(const uint32_t* sa, const uint32_t* sb, int count, int base,
                                            uint32_t fold_bodies, uint32_t r32, uint64_t (&s)[kPlainR]) {
  uint32_t w[8];  // w[k] = sb[base + k]: values of the outputs k at the step's first input
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = sb[base + k];
  uint32_t pending = 0;  // steps since the last fold
  for (int ii0 = 0; ii0 < count; ii0 += 16, base -= 16) {
    uint32_t av0[8], av1[8], nv0[8], nv1[8];
    plain_load8(av0, sa + ii0);
    plain_load8(av1, sa + ii0 + 8);
    plain_load8(nv0, sb + base - 8);
    plain_load8(nv1, sb + base - 16);
    plain_unit<kFoldEach>(av0, w, nv0, r32, s);
    plain_unit<kFoldEach>(av1, nv0, nv1, r32, s);
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = nv1[k];
    if (!kFoldEach && ++pending == fold_bodies) {
#pragma unroll
      for (int e = 0; e < kPlainR; ++e) s[e] = plain_fold(s[e], r32);
      pending = 0;
    }
  }
  if (!kFoldEach) {
#pragma unroll
    for (int e = 0; e < kPlainR; ++e) s[e] = plain_fold(s[e], r32);
  }
}

// Two half-blocks of 256 threads share a staged chunk: half h takes its inputs
// [h kcp/2, (h + 1) kcp/2) for the same 2048 outputs (twice the waves per SIMD to
// hide LDS latency); the upper half's residues are added in through LDS.
__global__ __launch_bounds__(kPlainThreads) void plain_kernel(const PlainParams P) {
  __shared__ __align__(16) uint32_t sa[kPlainKC];
  __shared__ __align__(16) uint32_t sb[kPlainSB];
  const uint64_t prod = blockIdx.x / P.blocks_per_prod;
  const int jb = (int)(blockIdx.x % P.blocks_per_prod) * kPlainOut;
  const int n = (int)P.n;
  const uint32_t q = P.m.q;
  const uint32_t* A = P.a + prod * n;
  const uint32_t* B = P.b + prod * n;
  const int jcount = min(kPlainOut, n - jb);
  const int half = (int)wave_uniform(threadIdx.x >> 8);
  const int jl0 = (int)(threadIdx.x & 255) * kPlainR;  // this thread's first output, relative to jb
  uint64_t s[kPlainR];
#pragma unroll
  for (int e = 0; e < kPlainR; ++e) s[e] = 0;

  for (int i0 = 0; i0 < n; i0 += kPlainKC) {
    const int kc = min(kPlainKC, n - i0);
    const int kcp = (kc + 31) & ~31;
    // sb[off + x] = bx[jb - i0 - kc + 1 + x], x < kc + jcount - 1; off makes
    // the 8-value window reads 16-byte aligned.  Everything else is zero.
    const int off = 16 + ((9 - kc) & 3);
    for (int x = threadIdx.x; x < kcp; x += kPlainThreads) sa[x] = x < kc ? reduce_u32(A[i0 + x], P.m) : 0u;
    const int kbase = jb - i0 - kc + 1;
    const int nsb = kc + jcount - 1;
    for (int x = threadIdx.x; x < kPlainSB; x += kPlainThreads) {
      const int k = kbase + x - off;
      uint32_t v = 0;
      if (x >= off && x < off + nsb) {
        if (k >= 0) v = reduce_u32(B[k], P.m);
        else {
          const uint32_t bb = reduce_u32(B[n + k], P.m);
          v = bb == 0 ? 0 : q - bb;
        }
      }
      sb[x] = v;
    }
    __syncthreads();
    // every thread runs the loop (uniform control flow); outputs past jcount are
    // not stored.  Output e at input ii reads sb[off + jl0 + kc - 1 - ii + e].
    const int h0 = half * (kcp >> 1);
    const int base = off + jl0 + kc - 1 - h0;
    if (P.fold_bodies == 0) plain_chunk<true>(sa + h0, sb, kcp >> 1, base, 0, P.r32, s);
    else plain_chunk<false>(sa + h0, sb, kcp >> 1, base, P.fold_bodies, P.r32, s);
    __syncthreads();
  }
  uint32_t out[kPlainR];
#pragma unroll
  for (int e = 0; e < kPlainR; ++e) out[e] = reduce_u64(s[e], P.m);
  uint32_t* comb = sa;  // the upper half's residues, 2048 words
  if (half == 1) {
    *(uint4*)(comb + jl0) = make_uint4(out[0], out[1], out[2], out[3]);
    *(uint4*)(comb + jl0 + 4) = make_uint4(out[4], out[5], out[6], out[7]);
  }
  __syncthreads();
  if (half == 1 || jl0 >= jcount) return;
  uint32_t up[8];
  plain_load8(up, comb + jl0);
#pragma unroll
  for (int e = 0; e < kPlainR; ++e) {
    const uint32_t t = out[e] + up[e];  // both < q <= 2^32 - 1: compare in 64 bits
    out[e] = (uint64_t)out[e] + up[e] >= q ? t - q : t;
  }
  uint32_t* C = P.c + prod * n + jb + jl0;
  if (jl0 + kPlainR <= jcount) {
    *(uint4*)C = make_uint4(out[0], out[1], out[2], out[3]);
    *(uint4*)(C + 4) = make_uint4(out[4], out[5], out[6], out[7]);
  } else {
#pragma unroll
    for (int e = 0; e < kPlainR; ++e)
      if (jl0 + e < jcount) C[e] = out[e];
  }
}

}  // namespace pm
