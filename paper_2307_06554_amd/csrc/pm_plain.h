// Plain integer schoolbook kernel: the comparison baseline for the MFMA path.
// c_j = sum_i a_i * bx[j - i] with bx[k] = b_k (k >= 0) and bx[k] = q - b_{n+k}
// (k < 0), i.e. the negacyclic wrap folded into the second operand as in
// Eq. (3); every term is a non-negative 32x32->64-bit product summed into a
// 96-bit accumulator (64-bit low word plus carry count), reduced once.
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
  ModQ32 m;
};

constexpr int kPlainThreads = 256;
constexpr int kPlainR = 8;                        // outputs per thread (strided by 256)
constexpr int kPlainOut = kPlainThreads * kPlainR;  // outputs per workgroup
constexpr int kPlainKC = 2048;                    // K-chunk staged in LDS

// LDS: a[kPlainKC] + bx window [kPlainKC + kPlainOut - 1]
constexpr int kPlainLdsWords = kPlainKC + kPlainKC + kPlainOut;

__global__ __launch_bounds__(kPlainThreads) void plain_kernel(const PlainParams P) {
  __shared__ uint32_t sa[kPlainKC];
  __shared__ uint32_t sb[kPlainKC + kPlainOut];
  const uint64_t prod = blockIdx.x / P.blocks_per_prod;
  const int jb = (int)(blockIdx.x % P.blocks_per_prod) * kPlainOut;
  const int n = (int)P.n;
  const uint32_t q = P.m.q;
  const uint32_t* A = P.a + prod * n;
  const uint32_t* B = P.b + prod * n;
  uint64_t lo[kPlainR];
  uint32_t hi[kPlainR];
#pragma unroll
  for (int e = 0; e < kPlainR; ++e) { lo[e] = 0; hi[e] = 0; }
  const int jcount = min(kPlainOut, n - jb);

  for (int i0 = 0; i0 < n; i0 += kPlainKC) {
    const int kc = min(kPlainKC, n - i0);
    // sa[ii] = a[i0 + ii]; sb[x] = bx[jb - i0 - kc + 1 + x]
    for (int x = threadIdx.x; x < kc; x += kPlainThreads) sa[x] = reduce_u64(A[i0 + x], P.m);
    const int kbase = jb - i0 - kc + 1;
    const int nsb = kc + jcount - 1;
    for (int x = threadIdx.x; x < nsb; x += kPlainThreads) {
      int k = kbase + x;
      uint32_t v;
      if (k >= 0) v = reduce_u64(B[k], P.m);
      else {
        uint32_t bb = reduce_u64(B[n + k], P.m);
        v = bb == 0 ? 0 : q - bb;
      }
      sb[x] = v;
    }
    __syncthreads();
    // output j = jb + tid + 256 e uses sb[j - jb - ii + kc - 1]
    for (int ii = 0; ii < kc; ++ii) {
      const uint64_t ai = sa[ii];
#pragma unroll
      for (int e = 0; e < kPlainR; ++e) {
        const int jl = (int)threadIdx.x + kPlainThreads * e;
        if (jl < jcount) {
          uint64_t p = ai * (uint64_t)sb[jl - ii + kc - 1];
          uint64_t s = lo[e] + p;
          hi[e] += s < p;
          lo[e] = s;
        }
      }
    }
    __syncthreads();
  }
  uint32_t* C = P.c + prod * n;
#pragma unroll
  for (int e = 0; e < kPlainR; ++e) {
    const int jl = (int)threadIdx.x + kPlainThreads * e;
    if (jl < jcount) {
      uint32_t x = reduce_u64(lo[e], P.m);
      uint32_t y = reduce_u64((uint64_t)hi[e] * P.m.r64, P.m);
      uint32_t s = x + y;  // both < q < 2^32: use 64-bit compare to avoid wrap
      uint64_t s64 = (uint64_t)x + y;
      s = (uint32_t)(s64 >= q ? s64 - q : s64);
      C[jb + jl] = s;
    }
  }
}

}  // namespace pm
