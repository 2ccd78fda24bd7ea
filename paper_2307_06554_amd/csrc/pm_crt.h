// The paper's own coefficient method on int8 MFMA: a residue number system of
// small co-prime moduli (paper Sec. 2.4, RNS base rules of Sec. 2.6, the three
// steps of Algorithm 1).
//
// Each coefficient x of Z_q is lifted to its centred integer v in
// (-q/2, q/2]; the integer negacyclic sums X_j = sum +-v_i w_k then satisfy
// |X_j| <= n floor(q/2)^2 = B.  With co-prime moduli m_c <= 256 whose product
// M exceeds 2B (a little more, see below), X_j is fixed by its residues
// X_j mod m_c.  Residues are held centred, so each fits an int8; the wrapped
// (negated) terms of Eq. (3) take the byte-wise negation of a residue, which is
// again a valid residue (for m = 256 the byte -128 stands for 128).  Channel c
// is one int8 matrix product of residues with int32 sums (|T| <= n 2^14), run
// on the same Toeplitz tiles as the limb kernel, one MFMA per channel and
// K-step instead of L^2 limb pairs.
//
// Reconstruction (ConvertMatrix): s_c = (T_c mod m_c) (M/m_c)^-1 mod m_c gives
// X' = sum_c s_c M/m_c = X + kappa M with kappa = round(sum_c s_c / m_c), since
// |X| / M < 1/2.  The sum of fractions is taken in fp32; M > 2B (1 + 2^-16)
// keeps it at least 2^-17 away from a rounding boundary, far more than the
// fp32 error of at most 11 * 2^-23.  Then c_j = (sum_c s_c (M/m_c mod q) -
// kappa (M mod q)) mod q.
#pragma once
#include "pm_mfma32.h"

namespace pm {

constexpr int kMaxCh = 11;  // small moduli per product
constexpr int kMaxQC = 8;   // q-level moduli per launch

struct CrtConsts {
  uint32_t C;                  // small moduli in use
  uint32_t m[kMaxCh];          // co-prime, <= 256, largest first
  uint32_t magic[kMaxCh];      // floor(2^32 / m)
  uint32_t off[kMaxCh];        // 2^31 mod m
  uint32_t y[kMaxCh];          // (M / m)^-1 mod m
  uint32_t yp[kMaxCh];         // floor(y 2^32 / m): Shoup's companion of y
  uint32_t oy[kMaxCh];         // (2^31 y) mod m
  float invm[kMaxCh];          // 1 / m
  uint32_t w[kMaxQC][kMaxCh];  // (M / m) mod q
  uint32_t Mq[kMaxQC];         // M mod q
};

// w mod m for a 32-bit w: with magic = floor(2^32 / m) the quotient estimate is
// floor(w / m) or one less (as for the word reduction mod q), so one conditional
// subtraction ends it.
__device__ __forceinline__ uint32_t small_mod(uint32_t w, uint32_t m, uint32_t magic) {
  const uint32_t r = w - __umulhi(w, magic) * m;
  return min(r, r - m);
}
// v mod m in [0, m) for a signed v, |v| < 2^31.
__device__ __forceinline__ uint32_t signed_mod(int32_t v, uint32_t m, uint32_t magic, uint32_t off) {
  const uint32_t r = small_mod((uint32_t)v + 0x80000000u, m, magic);  // (v + 2^31) mod m
  return r >= off ? r - off : r + m - off;
}
// The centred residue of v mod m as an int8 byte.
__device__ __forceinline__ uint32_t centred_byte(int32_t v, uint32_t m, uint32_t magic, uint32_t off) {
  const uint32_t r = signed_mod(v, m, magic, off);
  return (r > (m - 1) / 2 ? r - m : r) & 0xFFu;
}
// Byte-wise negation mod 256 of four packed bytes.
__device__ __forceinline__ uint32_t neg_bytes(uint32_t x) {
  const uint32_t nx = ~x;
  return ((nx & 0x7F7F7F7Fu) + 0x01010101u) ^ (nx & 0x80808080u);
}
// Centred lift of a residue x in [0, q).
__device__ __forceinline__ int32_t centred_lift(uint32_t x, uint32_t q) {
  return x > (q >> 1) ? (int32_t)(x - q) : (int32_t)x;
}

// Residue planes of four consecutive words (v[k] already lifted): plane c gets
// the dword whose byte k is the residue of v[order[k]].
template <int C>
__device__ __forceinline__ void crt_store4(const CrtConsts& K, uint8_t* base, uint32_t plane, uint32_t off,
                                           const int32_t (&v)[4], bool store_neg, uint8_t* nbase, uint32_t noff) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const uint32_t m = K.m[c], mg = K.magic[c], of = K.off[c];
    const uint32_t d = centred_byte(v[0], m, mg, of) | (centred_byte(v[1], m, mg, of) << 8) |
                       (centred_byte(v[2], m, mg, of) << 16) | (centred_byte(v[3], m, mg, of) << 24);
    *(uint32_t*)(base + c * plane + off) = d;
    if (store_neg) *(uint32_t*)(nbase + c * plane + noff) = neg_bytes(d);
  }
}

// One staged item (n >= 4): a's word group j into the reversed ext planes (and
// its negated copy inside the window), or b's word group into rows vs (+) and
// vs - r (-).
template <int C>
__device__ __forceinline__ void crt_item_store(const Mfma32Params& P, const CrtConsts& K, const GroupInfo& gi,
                                               uint8_t* smem, uint32_t i, uint4 x) {
  const uint32_t lper = P.log2n - 1, quarter = P.n >> 2;
  const uint32_t s = i >> lper, j = i & ((1u << lper) - 1);
  const ModQ32& m = P.mods[slot_li(gi, s)];
  uint8_t* slot = smem + s * P.slot_bytes;
  if (j < quarter) {
    // reversed: byte k of dword (E+1)/4 - 1 - j holds ext[4j + 3 - k]
    const int32_t v[4] = {centred_lift(reduce_u32(x.w, m), m.q), centred_lift(reduce_u32(x.z, m), m.q),
                          centred_lift(reduce_u32(x.y, m), m.q), centred_lift(reduce_u32(x.x, m), m.q)};
    const uint32_t dw = ((P.E + 1) >> 2) - 1 - j;
    const uint32_t dwn = dw + quarter;
    crt_store4<C>(K, slot, P.a_plane, dw * 4, v, dwn < (P.a_plane >> 2), slot, dwn * 4);
  } else {
    const uint32_t e = j - quarter;
    const int vs = (int)(e >> (P.log2t - 2)), wd = (int)(e & ((P.t >> 2) - 1));
    const int32_t v[4] = {centred_lift(reduce_u32(x.x, m), m.q), centred_lift(reduce_u32(x.y, m), m.q),
                          centred_lift(reduce_u32(x.z, m), m.q), centred_lift(reduce_u32(x.w, m), m.q)};
    uint8_t* bbase = slot + C * P.a_plane;
    const int rp = vs - gi.v_lo, rn = vs - (int)P.r - gi.v_lo;
    const bool pos = rp >= 0 && rp < (int)P.b_rows, neg = rn >= 0 && rn < (int)P.b_rows;
    if (pos) crt_store4<C>(K, bbase, P.b_plane, rp * P.b_rowstride + wd * 4, v, neg, bbase,
                           neg ? rn * P.b_rowstride + wd * 4 : 0);
    else if (neg) {
      const int32_t nv[4] = {-v[0], -v[1], -v[2], -v[3]};
      crt_store4<C>(K, bbase, P.b_plane, rn * P.b_rowstride + wd * 4, nv, false, bbase, 0);
    }
  }
}

// n < 4: the planes of one product byte by byte.
template <int C>
__device__ __forceinline__ void crt_stage_small(const Mfma32Params& P, const CrtConsts& K, uint8_t* slot,
                                                uint64_t gprod, const ModQ32& m, int v_lo) {
  const uint32_t* A = P.a + gprod * P.n;
  const uint32_t* B = P.b + gprod * P.n;
  const int n = (int)P.n, t = (int)P.t, r = (int)P.r;
  for (int p = threadIdx.x; p < (int)P.a_plane; p += kThreads) {
    const int idx = (int)P.E - p;
    int32_t v = 0;
    if (idx >= 0 && idx < n) v = centred_lift(reduce_u32(A[idx], m), m.q);
    else if (idx < 0 && idx > -n) v = -centred_lift(reduce_u32(A[n + idx], m), m.q);
#pragma unroll
    for (int c = 0; c < C; ++c) slot[c * P.a_plane + p] = (uint8_t)centred_byte(v, K.m[c], K.magic[c], K.off[c]);
  }
  uint8_t* bbase = slot + C * P.a_plane;
  const int nb = (int)(P.b_rows * P.rowlen);
  for (int e = threadIdx.x; e < nb; e += kThreads) {
    const int row = e / (int)P.rowlen, ww = e - row * (int)P.rowlen;
    const int v_row = v_lo + row;
    int32_t v = 0;
    if (ww < t) {
      if (v_row >= 0 && v_row < r) v = centred_lift(reduce_u32(B[v_row * t + ww], m), m.q);
      else if (v_row < 0 && v_row > -r) v = -centred_lift(reduce_u32(B[(v_row + r) * t + ww], m), m.q);
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
      bbase[c * P.b_plane + row * P.b_rowstride + ww] = (uint8_t)centred_byte(v, K.m[c], K.magic[c], K.off[c]);
  }
}

// One K-step: channel by channel, its MFMA, its B refill, then its next A
// fragment aligned from runs read a step earlier and the runs after that read.
template <int C>
__device__ __forceinline__ void crt_step(v16i (&acc)[C], const v4i (&a)[C], v4i (&an)[C], uint32_t (&araw)[C][5],
                                         uint32_t sh_next, const uint8_t* aplane, uint32_t a_plane, int S_after,
                                         v4i (&b)[C], const uint8_t* bplane, uint32_t b_plane, int boff_next) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[c], b[c], acc[c], 0, 0, 0);
    b[c] = *(const v4i*)(bplane + c * b_plane + boff_next);
    an[c][0] = (int)__builtin_amdgcn_alignbyte(araw[c][1], araw[c][0], sh_next);
    an[c][1] = (int)__builtin_amdgcn_alignbyte(araw[c][2], araw[c][1], sh_next);
    an[c][2] = (int)__builtin_amdgcn_alignbyte(araw[c][3], araw[c][2], sh_next);
    an[c][3] = (int)__builtin_amdgcn_alignbyte(araw[c][4], araw[c][3], sh_next);
    const uint32_t* p = (const uint32_t*)(aplane + c * a_plane) + (S_after >> 2);
#pragma unroll
    for (int k = 0; k < 5; ++k) araw[c][k] = p[k];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One 32x32 output tile: all channels over the whole K loop.
template <int C>
__device__ __forceinline__ void crt_tile(const Mfma32Params& P, const uint8_t* aplane, const uint8_t* bplane, int z0,
                                         int u0, int v_lo, v16i (&acc)[C]) {
  const int lane = threadIdx.x & 63;
  const int zl = lane & 31, g = lane >> 5;
  const int S0 = (int)P.E - (z0 + zl) + 16 * g;
  const int B0 = (u0 + zl - v_lo) * (int)P.b_rowstride + 16 * g;
  const int steps = (int)(P.r << P.log2spd);
  const int rs = (int)P.b_rowstride;
  const uint32_t a_plane = P.a_plane, b_plane = P.b_plane;
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = v16i{};
  auto S_of = [&](int st) { return S0 - ((st >> P.log2spd) << P.log2t) + ((st & (P.spd - 1)) << 5); };
  auto B_of = [&](int st) { return B0 - (st >> P.log2spd) * rs + ((st & (P.spd - 1)) << 5); };
  auto clamp = [&](int st) { return st < steps ? st : steps - 1; };
  uint32_t araw[C][5];
  v4i a0[C], a1[C], b[C];
  const int S_first = S_of(0);
  araw_load<C>(araw, aplane, a_plane, S_first);
  b_load<C>(b, bplane, b_plane, B_of(0));
  a_align<C>(a0, araw, (uint32_t)(S_first & 3));
  araw_load<C>(araw, aplane, a_plane, S_of(clamp(1)));
  int st = 0;
  for (; st + 1 < steps; st += 2) {
    crt_step<C>(acc, a0, a1, araw, (uint32_t)(S_of(st + 1) & 3), aplane, a_plane, S_of(clamp(st + 2)), b, bplane,
                b_plane, B_of(st + 1));
    crt_step<C>(acc, a1, a0, araw, (uint32_t)(S_of(clamp(st + 2)) & 3), aplane, a_plane, S_of(clamp(st + 3)), b,
                bplane, b_plane, B_of(clamp(st + 2)));
  }
  if (st < steps)
    crt_step<C>(acc, a0, a1, araw, (uint32_t)(S_of(st) & 3), aplane, a_plane, S_of(st), b, bplane, b_plane,
                B_of(st));
}

// Reconstruction of the 16 outputs a lane holds, then the stores.  Per channel,
// s = (T mod m) y mod m is one Shoup product: for the 32-bit word T + 2^31 and
// y < m, (T + 2^31) y - floor((T + 2^31) yp / 2^32) m lies in [0, 2m), and the
// precomputed (2^31 y) mod m removes the offset.  The running sum
// lift + sum_c s w_c - kappa (M mod q) stays in (2^62 - 2^36, 2^62 + 2^44 + q).
template <int C>
__device__ __forceinline__ void crt_epilogue(const Mfma32Params& P, const CrtConsts& K, uint64_t gprod, uint32_t li,
                                             int z0, int u0, const v16i (&acc)[C]) {
  const ModQ32 m = P.mods[li];
  const int lane = threadIdx.x & 63;
  const int g = lane >> 5;
  const int u = u0 + (lane & 31);
  uint32_t mc[C], yv[C], yp[C], oy[C], wv[C];
  float im[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    mc[c] = K.m[c];
    yv[c] = K.y[c];
    yp[c] = K.yp[c];
    oy[c] = K.oy[c];
    wv[c] = K.w[li][c];
    im[c] = K.invm[c];
  }
  const uint32_t Mq = K.Mq[li];
  uint32_t out[16];
  auto reconstruct = [&](auto reduce) {
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      float f = 0.0f;
      uint64_t x = m.lift;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const uint32_t tu = (uint32_t)acc[c][rr] + 0x80000000u;
        uint32_t su = tu * yv[c] - __umulhi(tu, yp[c]) * mc[c];
        su = min(su, su - mc[c]);
        const uint32_t sc = su >= oy[c] ? su - oy[c] : su + mc[c] - oy[c];
        f += (float)sc * im[c];
        x += (uint64_t)sc * wv[c];
      }
      const uint32_t kappa = (uint32_t)floorf(f + 0.5f);
      x -= (uint64_t)kappa * Mq;
      out[rr] = reduce(x);
    }
  };
  if (m.q < 0x80000000u) reconstruct([&](uint64_t x) { return reduce_u64_q31(x, m.mu, m.q); });
  else reconstruct([&](uint64_t x) { return reduce_u64(x, m); });
  if (u >= (int)P.r) return;
  uint32_t* Cout = P.c + gprod * P.n;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int zb = z0 + 8 * blk + 4 * g;
    if (zb + 3 < (int)P.t) {
      *(uint4*)(Cout + (size_t)u * P.t + zb) =
          make_uint4(out[4 * blk], out[4 * blk + 1], out[4 * blk + 2], out[4 * blk + 3]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (zb + e < (int)P.t) Cout[(size_t)u * P.t + zb + e] = out[4 * blk + e];
    }
  }
}

// One group of four 32x32 tiles (as the limb kernel's groups), C residue planes per operand.
template <int C, bool SMALL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void crt_group_kernel(const Mfma32Params P, const CrtConsts K) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint64_t grp = blockIdx.x;
  const uint64_t total_units = P.nprod << P.log2U;
  const uint32_t U = 1u << P.log2U;
  const GroupInfo gi = group_info(P, grp);
  if constexpr (SMALL) {
    for (uint32_t s = 0; s < gi.nslots; ++s)
      crt_stage_small<C>(P, K, smem + s * P.slot_bytes, slot_gp(gi, s), P.mods[slot_li(gi, s)], gi.v_lo);
  } else {
    const uint32_t nitems = gi.nslots * (P.n >> 1);
    for (uint32_t base = 0; base < nitems; base += kPrefetch * kThreads) {
      uint4 pf[kPrefetch];
#pragma unroll
      for (int k = 0; k < kPrefetch; ++k) {
        const uint32_t i = base + threadIdx.x + k * kThreads;
        const uint4* src = i < nitems ? item_src(P, gi, i) : nullptr;
        pf[k] = src ? *src : make_uint4(0, 0, 0, 0);
      }
#pragma clang loop unroll(full)
      for (int k = 0; k < kPrefetch; ++k) {
        const uint32_t i = base + threadIdx.x + k * kThreads;
        if (i < nitems) crt_item_store<C>(P, K, gi, smem, i, pf[k]);
      }
    }
    stage_zero_fill<C>(P, gi, smem);
  }
  __syncthreads();
  const uint64_t unit = grp * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (unit >= total_units) return;
  const uint64_t prod = unit >> P.log2U;
  const uint32_t tile = (uint32_t)(unit & (U - 1));
  const int zt = (int)(tile % P.tz), ut = (int)(tile / P.tz);
  const uint8_t* slot = smem + (uint32_t)(prod - gi.first) * P.slot_bytes;
  v16i acc[C];
  crt_tile<C>(P, slot, slot + C * P.a_plane, 32 * zt, 32 * ut, gi.v_lo, acc);
  uint32_t li;
  const uint64_t gprod = global_product(P, prod, &li);
  crt_epilogue<C>(P, K, gprod, li, 32 * zt, 32 * ut, acc);
}

}  // namespace pm
