// Karatsuba over even/odd halves on top of the MFMA product (paper Sec. 4:
// the schoolbook count can be cut with Karatsuba's 3-for-4 recursion).
//
// In Z_q[x]/(x^n+1) write a(x) = a_e(x^2) + x a_o(x^2); with z = x^2 the halves
// live in Z_q[z]/(z^(n/2)+1) (z^(n/2) = x^n = -1, still negacyclic) and
//   c_e = P0 + z P1,   c_o = P2 - P0 - P1,
//   P0 = a_e b_e, P1 = a_o b_o, P2 = (a_e + a_o)(b_e + b_o),
// so one product of degree bound n becomes three of n/2.  Depth k repeats the
// split: sub-product s = d_1 + 3 d_2 + 9 d_3 (d_l = 0 even, 1 odd, 2 sum at
// level l) multiplies sub_s(a) and sub_s(b), where
//   sub_s(x)[i] = sum over r in [0, 2^k) whose bit l-1 is allowed by d_l of x[2^k i + r]
// (bit 0 for d = 0, bit 1 for d = 1, either for d = 2).  The recombination needs,
// per column i of the sub-products, only column i and the last element of the
// previous block (z times a block shifts it by one; at i = 0 the negacyclic
// wrap brings -P[n'-1]), level by level.
#pragma once
#include <type_traits>
#include "pm_common.h"
#include "pm_wide.h"

namespace pm {

// W: 32-bit words with up to 16 moduli (RNS channels), or 64-bit words with one.
template <typename W, typename Mod, int NM>
struct KaraParamsT {
  const W* a;
  const W* b;
  W* c;
  W* sa;   // [nprod][3^k][n'] sub-operands of a
  W* sb;   // same for b
  const W* sc;  // [nprod][3^k][n'] sub-products
  uint64_t nprod;
  uint32_t n, np, depth, nsub;  // n' = n >> depth, nsub = 3^depth
  uint32_t L;                   // moduli: product p uses mods[p % L]
  Mod mods[NM];
};
typedef KaraParamsT<uint32_t, ModQ32, 16> KaraParams;
typedef KaraParamsT<uint64_t, ModQ64, 1> KaraParams64;

__device__ __forceinline__ uint32_t addq(uint32_t x, uint32_t y, uint32_t q) {
  const uint64_t s = (uint64_t)x + y;
  return (uint32_t)(s >= q ? s - q : s);
}
__device__ __forceinline__ uint32_t subq(uint32_t x, uint32_t y, uint32_t q) {
  return x >= y ? x - y : (uint32_t)((uint64_t)x + q - y);
}
__device__ __forceinline__ uint64_t addq(uint64_t x, uint64_t y, uint64_t q) { return addmod64(x, y, q); }
__device__ __forceinline__ uint64_t subq(uint64_t x, uint64_t y, uint64_t q) { return submod64(x, y, q); }
__device__ __forceinline__ uint32_t kara_reduce(uint32_t x, const ModQ32& m) { return reduce_u32(x, m); }
__device__ __forceinline__ uint64_t kara_reduce(uint64_t x, const ModQ64& m) { return x < m.q ? x : mod_u64(x, m); }

// One thread per (product, column i): reads x[2^k i .. 2^k i + 2^k) of a and b,
// writes column i of every sub-operand.
template <int K, typename KP>
__global__ __launch_bounds__(256) void kara_split_kernel(const KP P) {
  typedef typename std::remove_const<typename std::remove_pointer<decltype(P.a)>::type>::type W;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t p = gid / P.np;
  const uint32_t i = (uint32_t)(gid - p * P.np);
  if (p >= P.nprod) return;
  const auto& m = P.mods[p % P.L];
  constexpr int R = 1 << K;
  int nsub = 1;
  for (int l = 0; l < K; ++l) nsub *= 3;
#pragma unroll
  for (int op = 0; op < 2; ++op) {
    const W* X = (op == 0 ? P.a : P.b) + p * P.n + (uint64_t)R * i;
    W* S = (op == 0 ? P.sa : P.sb) + p * (uint64_t)nsub * P.np + i;
    W x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = kara_reduce(X[r], m);
    // level by level: v holds, for every choice prefix, the 2^(K-l) partial sums still split by the deeper bits
    W v[R * 27 / 8 + 1];  // enough for 3^K values at the end (K <= 3)
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = x[r];
    int cnt = 1, width = R;  // cnt prefixes, each with `width` values (indexed by the remaining bits)
#pragma unroll
    for (int l = 0; l < K; ++l) {
      // split on bit 0 of the remaining index: even part, odd part, their sum
      W nv[R * 27 / 8 + 1];
      const int hw = width / 2;
#pragma unroll
      for (int c0 = 0; c0 < cnt; ++c0)
#pragma unroll
        for (int h = 0; h < hw; ++h) {
          const W e = v[c0 * width + 2 * h], o = v[c0 * width + 2 * h + 1];
          // new prefix index d_l * cnt + c0 keeps s = d_1 + 3 d_2 + ... ordering
          nv[(0 * cnt + c0) * hw + h] = e;
          nv[(1 * cnt + c0) * hw + h] = o;
          nv[(2 * cnt + c0) * hw + h] = addq(e, o, (W)m.q);
        }
      cnt *= 3;
      width = hw;
#pragma unroll
      for (int k = 0; k < cnt * width; ++k) v[k] = nv[k];
    }
#pragma unroll
    for (int s = 0; s < nsub; ++s) S[(uint64_t)s * P.np] = v[s];
  }
}

// One thread per (product, column i): c[2^k i + r] for r < 2^k.
template <int K, typename KP>
__global__ __launch_bounds__(256) void kara_combine_kernel(const KP P) {
  typedef typename std::remove_const<typename std::remove_pointer<decltype(P.a)>::type>::type W;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t p = gid / P.np;
  const uint32_t i = (uint32_t)(gid - p * P.np);
  if (p >= P.nprod) return;
  const W q = (W)P.mods[p % P.L].q;
  constexpr int NS = K == 1 ? 3 : K == 2 ? 9 : 27;
  const W* S = P.sc + p * (uint64_t)NS * P.np;
  // blocks: cur[s][j] (block of size B per sub-product), prev[s] = last element of the previous block
  W cur[NS * 1];
  W prv[NS];
  const uint32_t ip = i ? i - 1 : P.np - 1;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    cur[s] = S[(uint64_t)s * P.np + i];
    const W pv = S[(uint64_t)s * P.np + ip];
    prv[s] = i ? pv : (pv ? q - pv : (W)0);  // z^(n') = -1 at the deepest level
  }
  // combine the deepest level first: children differ in the most significant choice digit
  W blk[1 << K][NS];  // blk[j][parent] values; starts with B = 1
  W pl[NS];
  int count = NS, B = 1;
#pragma unroll
  for (int s = 0; s < NS; ++s) { blk[0][s] = cur[s]; pl[s] = prv[s]; }
#pragma unroll
  for (int l = K; l >= 1; --l) {
    const int parents = count / 3;  // children of parent x: x + parents * d, d = 0, 1, 2
    W nb[1 << K][NS];
    W npl[NS];
#pragma unroll
    for (int x = 0; x < parents; ++x) {
      const int c0 = x, c1 = x + parents, c2 = x + 2 * parents;
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const W s1 = j ? blk[j - 1][c1] : pl[c1];  // (z * P1)[j]
        nb[2 * j][x] = addq(blk[j][c0], s1, q);
        nb[2 * j + 1][x] = subq(subq(blk[j][c2], blk[j][c0], q), blk[j][c1], q);
      }
      npl[x] = subq(subq(pl[c2], pl[c0], q), pl[c1], q);
    }
    count = parents;
    B *= 2;
#pragma unroll
    for (int j = 0; j < B; ++j)
#pragma unroll
      for (int x = 0; x < count; ++x) blk[j][x] = nb[j][x];
#pragma unroll
    for (int x = 0; x < count; ++x) pl[x] = npl[x];
  }
  W* C = P.c + p * P.n + ((uint64_t)i << K);
#pragma unroll
  for (int r = 0; r < (1 << K); ++r) C[r] = blk[r][0];
}

}  // namespace pm
