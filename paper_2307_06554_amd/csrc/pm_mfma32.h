// Split-limb int8 MFMA kernel for 32-bit moduli, whole operands resident in LDS.
//
// Mapping of the product onto a matrix product (paper Sec. 2.2, Eq. (3), and
// the block split of Sec. 2.5 / Fig. 1): write n = t*r, output index
// j = u*t + z (z in [0,t), u in [0,r)) and input index k = d*t + w.  With the
// extended sequence ext[i] = a_i (0 <= i < n), ext[i] = -a_{n+i} (-t < i < 0),
//
//   c[u*t + z] = sum_{d<r} sum_{w<t} ext[d*t + z - w] * s(u,d) * b[((u-d) mod r)*t + w],
//   s(u,d) = -1 if u < d (the block wrapped past x^n) else +1.
//
// That is C[z][u] = sum_{(d,w)} A[z][(d,w)] * B[(d,w)][u]: a GEMM with M = t,
// N = r, K = n per product.  A is r Toeplitz t x t tiles cut from a window of
// ext (never materialised: each lane reads a reversed 16-byte run of digits),
// B is b reshaped to t x r with a circular column shift whose wrapped columns
// take the digits of q - b.
//
// Each operand is split into L balanced int8 limbs; the L*L limb products go
// through v_mfma_i32_32x32x32_i8 and are summed per shift class s = i + j in
// int32 (2L-1 accumulator sets).  Bound: |digit product| <= 2^14 and at most L
// pairs share a class, so |T_s| <= L * n * 2^14 < 2^31 for L*n <= 2^16 - 1;
// the host only routes n <= 8192 here (L <= 4).  Recombination
// c = sum_s T_s 2^(8s) mod q runs as Horner steps with Barrett reduction.
#pragma once
#include "pm_common.h"

namespace pm {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kMaxQ = 16;  // moduli per launch (RNS channels are chunked above this)

struct Mfma32Params {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* c;
  uint64_t nprod;        // products handled by this launch
  uint32_t n, t, r;      // n = t * r
  uint32_t log2t, log2spd, spd;  // K-steps of 32 per d: spd = max(1, t/32)
  uint32_t rowlen;       // bytes of one B row that are read (= 32 * spd)
  uint32_t tz, tu, log2U;  // output tiles of 32x32 per product: tz * tu = 2^log2U
  uint32_t slots;        // products staged per workgroup
  uint32_t a_plane;      // bytes per limb plane of the reversed ext array
  uint32_t b_rows, b_rowstride, b_plane;  // B rows staged per product, their stride, plane size
  uint32_t slot_bytes;   // L * (a_plane + b_plane)
  uint32_t E;            // ext index held at reversed position 0
  // Product i of this launch is global product (i / lc) * nq_total + l0 + (i % lc)
  // and uses modulus mods[i % lc].
  uint32_t lc, nq_total, l0;
  ModQ32 mods[kMaxQ];
};

template <int L>
__device__ __forceinline__ void mfma32_stage(const Mfma32Params& P, uint8_t* slot, uint64_t gprod,
                                             const ModQ32& m, int v_lo) {
  const uint32_t* A = P.a + gprod * P.n;
  const uint32_t* B = P.b + gprod * P.n;
  const uint32_t q = m.q, thr = m.thr;
  const int n = (int)P.n;
  // Reversed ext planes: position p holds ext[E - p].
  const int a_dw = (int)(P.a_plane >> 2);
  for (int dw = threadIdx.x; dw < a_dw; dw += blockDim.x) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int idx = (int)P.E - (dw * 4 + k);
      uint32_t dg = 0;
      if (idx >= 0 && idx < n) dg = digits32<L>(reduce_u64(A[idx], m), q, thr);
      else if (idx < 0 && idx > -n) dg = neg_digits32<L>(reduce_u64(A[n + idx], m), q, thr);
      w[k] = dg;
    }
#pragma unroll
    for (int i = 0; i < L; ++i) {
      uint32_t v = ((w[0] >> (8 * i)) & 0xFF) | (((w[1] >> (8 * i)) & 0xFF) << 8) |
                   (((w[2] >> (8 * i)) & 0xFF) << 16) | (((w[3] >> (8 * i)) & 0xFF) << 24);
      *(uint32_t*)(slot + i * P.a_plane + dw * 4) = v;
    }
  }
  // B rows v in [v_lo, v_lo + b_rows): v in [0, r) -> b[v t + w]; v < 0 -> -b[(v+r) t + w];
  // v >= r or w >= t -> 0 (padding of a tile wider than the product).
  uint8_t* bbase = slot + L * P.a_plane;
  const int row_dw = (int)(P.rowlen >> 2);
  const int nb = (int)P.b_rows * row_dw;
  const int t = (int)P.t, r = (int)P.r;
  for (int e = threadIdx.x; e < nb; e += blockDim.x) {
    int row = e / row_dw, wd = e - row * row_dw;
    int v = v_lo + row;
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int ww = wd * 4 + k;
      uint32_t dg = 0;
      if (ww < t) {
        if (v >= 0 && v < r) dg = digits32<L>(reduce_u64(B[v * t + ww], m), q, thr);
        else if (v < 0 && v > -r) dg = neg_digits32<L>(reduce_u64(B[(v + r) * t + ww], m), q, thr);
      }
      w[k] = dg;
    }
#pragma unroll
    for (int i = 0; i < L; ++i) {
      uint32_t val = ((w[0] >> (8 * i)) & 0xFF) | (((w[1] >> (8 * i)) & 0xFF) << 8) |
                     (((w[2] >> (8 * i)) & 0xFF) << 16) | (((w[3] >> (8 * i)) & 0xFF) << 24);
      *(uint32_t*)(bbase + i * P.b_plane + row * P.b_rowstride + wd * 4) = val;
    }
  }
}

// One 32x32 output tile of one product: the whole K loop for all L*L limb pairs.
template <int L>
__device__ __forceinline__ void mfma32_tile(const Mfma32Params& P, const uint8_t* slot, int z0, int u0,
                                            int v_lo, v16i (&acc)[2 * L - 1]) {
  const int lane = threadIdx.x & 63;
  const int zl = lane & 31, g = lane >> 5;
  const uint8_t* aplane = slot;
  const uint8_t* bplane = slot + L * P.a_plane;
  // A: lane reads reversed positions S .. S+15 with S = E - (d t + z - w0 - 16 g).
  const int S0 = (int)P.E - (z0 + zl) + 16 * g;
  // B: lane reads row (u - d) - v_lo, bytes w0 + 16 g .. + 15.
  const int B0 = (u0 + zl - v_lo) * (int)P.b_rowstride + 16 * g;
  const int steps = (int)(P.r << P.log2spd);
#pragma unroll
  for (int s = 0; s < 2 * L - 1; ++s) acc[s] = v16i{};

  for (int st = 0; st < steps; ++st) {
    const int d = st >> P.log2spd;
    const int w0 = (st & (P.spd - 1)) << 5;
    const int S = S0 - (d << P.log2t) + w0;
    const int boff = B0 - d * (int)P.b_rowstride + w0;
    v4i af[L], bf[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint32_t* p = (const uint32_t*)(aplane + i * P.a_plane) + (S >> 2);
      uint32_t x0 = p[0], x1 = p[1], x2 = p[2], x3 = p[3], x4 = p[4];
      const uint32_t sh = (uint32_t)(S & 3);
      af[i][0] = (int)__builtin_amdgcn_alignbyte(x1, x0, sh);
      af[i][1] = (int)__builtin_amdgcn_alignbyte(x2, x1, sh);
      af[i][2] = (int)__builtin_amdgcn_alignbyte(x3, x2, sh);
      af[i][3] = (int)__builtin_amdgcn_alignbyte(x4, x3, sh);
      bf[i] = *(const v4i*)(bplane + i * P.b_plane + boff);
    }
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
      for (int j = 0; j < L; ++j)
        acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[i], bf[j], acc[i + j], 0, 0, 0);
  }
}

template <int L>
__device__ __forceinline__ void mfma32_epilogue(const Mfma32Params& P, uint64_t gprod, const ModQ32& m,
                                                int z0, int u0, const v16i (&acc)[2 * L - 1]) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 5;
  const int u = u0 + (lane & 31);
  if (u >= (int)P.r) return;
  uint32_t* C = P.c + gprod * P.n;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int zb = z0 + 8 * blk + 4 * g;
    uint32_t out[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int rr = blk * 4 + e;
      // Horner in radix 2^8 from the top shift class down.
      uint32_t v = reduce_i64((int64_t)acc[2 * L - 2][rr], m);
#pragma unroll
      for (int s = 2 * L - 3; s >= 0; --s) v = reduce_i64((int64_t)v * 256 + (int64_t)acc[s][rr], m);
      out[e] = v;
    }
    if (zb + 3 < (int)P.t) {
      *(uint4*)(C + (size_t)u * P.t + zb) = make_uint4(out[0], out[1], out[2], out[3]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (zb + e < (int)P.t) C[(size_t)u * P.t + zb + e] = out[e];
    }
  }
}

template <int L>
__global__ __launch_bounds__(256) void mfma32_resident_kernel(const Mfma32Params P) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t U = 1u << P.log2U;
  const uint64_t unit0 = (uint64_t)blockIdx.x * 4;
  const uint64_t first = unit0 >> P.log2U;  // first product of this workgroup
  const uint64_t total_units = P.nprod << P.log2U;
  // u-range covered by this workgroup inside each staged product.
  int ut_lo, ut_hi;
  if (U >= 4) {
    const uint32_t t0 = (uint32_t)(unit0 & (U - 1));
    ut_lo = (int)(t0 / P.tz);
    ut_hi = (int)((t0 + 3) / P.tz);
  } else {
    ut_lo = 0;
    ut_hi = (int)P.tu - 1;
  }
  const int v_lo = 32 * ut_lo - ((int)P.r - 1);

  for (uint32_t k = 0; k < P.slots; ++k) {
    const uint64_t prod = first + k;
    if (prod >= P.nprod) break;
    const uint32_t li = (uint32_t)(prod % P.lc);
    const uint64_t gprod = (prod / P.lc) * P.nq_total + P.l0 + li;
    mfma32_stage<L>(P, smem + k * P.slot_bytes, gprod, P.mods[li], v_lo);
  }
  __syncthreads();

  const uint64_t unit = unit0 + (threadIdx.x >> 6);
  if (unit >= total_units) return;
  const uint64_t prod = unit >> P.log2U;
  const uint32_t tile = (uint32_t)(unit & (U - 1));
  const int zt = (int)(tile % P.tz), ut = (int)(tile / P.tz);
  const uint32_t li = (uint32_t)(prod % P.lc);
  const uint64_t gprod = (prod / P.lc) * P.nq_total + P.l0 + li;
  const uint8_t* slot = smem + (uint32_t)(prod - first) * P.slot_bytes;
  v16i acc[2 * L - 1];
  mfma32_tile<L>(P, slot, 32 * zt, 32 * ut, v_lo, acc);
  mfma32_epilogue<L>(P, gprod, P.mods[li], 32 * zt, 32 * ut, acc);
}

}  // namespace pm
