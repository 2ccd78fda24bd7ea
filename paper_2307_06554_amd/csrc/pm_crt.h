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
// |X| / M < 1/2.  The sum of fractions is taken in fp32: M > 2B (1 + 2^-16)
// keeps the true sum at least 2^-17 (about 7.6e-6) away from a rounding
// boundary, and with u = 2^-24 the fp32 value is within (2C + C(C+1)/2 + C + 1) u
// of it -- two roundings per term (1/m and the product), one per running sum
// (below k after k terms) and the final + 0.5 -- at most 100 u (about 6.0e-6) for
// C <= 11, so kappa is exact.  Then c_j = (sum_c s_c (M/m_c mod q) -
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
  float mf[kMaxCh];            // m
  int32_t r16[kMaxCh];         // 2^16 mod m
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

// One staging pass of the wave kernel: each thread loads up to kStageItems word
// groups (a's, into the reversed ext planes, or b's, into the B rows), lifts
// them to centred integers and notes where their residue dwords go (a dword and,
// where the window or the rows need it, its byte-wise negation); then the
// channels are taken one at a time, so that only one channel's constants are
// live while every item's four residues are formed and stored.
constexpr int kStageItems = 4;

// CP channels from c0 into planes 0..CP-1 of slots laid out for CL planes (CL >= CP).
template <int CP, int NT, int CL = CP>
__device__ __forceinline__ void crt_stage_pass(const Mfma32Params& P, const CrtConsts& K, const GroupInfo& gi,
                                               uint8_t* smem, uint32_t base, uint32_t nitems, int c0 = 0) {
  const uint32_t lper = P.log2n - 1, quarter = P.n >> 2;
  uint4 pf[kStageItems];
#pragma unroll
  for (int k = 0; k < kStageItems; ++k) {
    const uint32_t i = base + threadIdx.x + k * NT;
    const uint4* src = i < nitems ? item_src(P, gi, i) : nullptr;
    pf[k] = src ? *src : make_uint4(0, 0, 0, 0);
  }
  int32_t v[kStageItems][4];
  uint32_t dst1[kStageItems], dst2[kStageItems], pstride[kStageItems], flags[kStageItems];
#pragma unroll
  for (int k = 0; k < kStageItems; ++k) {
    const uint32_t i = base + threadIdx.x + k * NT;
    flags[k] = 0;
    dst1[k] = dst2[k] = 0;
    pstride[k] = 0;
    v[k][0] = v[k][1] = v[k][2] = v[k][3] = 0;
    if (i >= nitems) continue;
    const uint32_t s = i >> lper, j = i & ((1u << lper) - 1);
    const ModQ32& m = P.mods[slot_li(gi, s)];
    const uint4 x = pf[k];
    const uint32_t slot = s * P.slot_bytes;
    if (j < quarter) {
      // reversed: byte k of dword (E+1)/4 - 1 - j holds ext[4j + 3 - k]; the negated
      // copy n/4 dwords further where the window reaches it
      v[k][0] = centred_lift(reduce_u32(x.w, m), m.q);
      v[k][1] = centred_lift(reduce_u32(x.z, m), m.q);
      v[k][2] = centred_lift(reduce_u32(x.y, m), m.q);
      v[k][3] = centred_lift(reduce_u32(x.x, m), m.q);
      const uint32_t dw = ((P.E + 1) >> 2) - 1 - j, dwn = dw + quarter;
      dst1[k] = slot + dw * 4;
      dst2[k] = slot + dwn * 4;
      pstride[k] = P.a_plane;
      flags[k] = 1u | (dwn < (P.a_plane >> 2) ? 2u : 0u);
    } else {
      const uint32_t e = j - quarter;
      const int vs = (int)(e >> (P.log2t - 2)), wd = (int)(e & ((P.t >> 2) - 1));
      v[k][0] = centred_lift(reduce_u32(x.x, m), m.q);
      v[k][1] = centred_lift(reduce_u32(x.y, m), m.q);
      v[k][2] = centred_lift(reduce_u32(x.z, m), m.q);
      v[k][3] = centred_lift(reduce_u32(x.w, m), m.q);
      const uint32_t bbase = slot + CL * P.a_plane;
      const int rp = vs - gi.v_lo, rn = vs - (int)P.r - gi.v_lo;
      dst1[k] = bbase + (uint32_t)(rp * (int)P.b_rowstride + wd * 4);
      dst2[k] = bbase + (uint32_t)(rn * (int)P.b_rowstride + wd * 4);
      pstride[k] = P.b_plane;
      flags[k] = (rp >= 0 && rp < (int)P.b_rows ? 1u : 0u) | (rn >= 0 && rn < (int)P.b_rows ? 2u : 0u);
    }
  }
  auto store = [&](int c, int k, uint32_t d) {
    uint8_t* plane = smem + c * pstride[k];
    if (flags[k] & 1u) *(uint32_t*)(plane + dst1[k]) = d;
    if (flags[k] & 2u) *(uint32_t*)(plane + dst2[k]) = neg_bytes(d);
  };
#pragma unroll 1
  for (int c = 0; c < CP; ++c) {
    const uint32_t m = K.m[c0 + c];
    if (m == 256) {  // uniform: the centred residue is the low byte
#pragma unroll
      for (int k = 0; k < kStageItems; ++k) {
        if (!flags[k]) continue;
        const uint32_t lo01 = __builtin_amdgcn_perm((uint32_t)v[k][1], (uint32_t)v[k][0], 0x0c0c0400u);
        const uint32_t lo23 = __builtin_amdgcn_perm((uint32_t)v[k][3], (uint32_t)v[k][2], 0x0c0c0400u);
        store(c, k, __builtin_amdgcn_perm(lo23, lo01, 0x05040100u));
      }
      continue;
    }
    const int32_t r16 = K.r16[c0 + c];
    const float mf = K.mf[c0 + c], im = K.invm[c0 + c];
    // v = 2^16 vh + vl, x = vh (2^16 mod m) + vl, r = x - m rint(x / m) as in
    // residue_centred; |r| <= m/2 + 1 leaves r > 127 only for m = 254, 255 (folded to
    // r - m), so the fold needs no test of m
    auto res = [&](int32_t vv) {
      const int32_t x = __mul24(vv >> 16, r16) + (vv & 0xFFFF);
      const float xf = (float)x;
      const int32_t r = (int32_t)fmaf(-rintf(xf * im), mf, xf);
      return (uint32_t)(r > 127 ? r - (int32_t)m : r);
    };
#pragma unroll
    for (int k = 0; k < kStageItems; ++k) {
      if (!flags[k]) continue;
      const uint32_t r0 = res(v[k][0]), r1 = res(v[k][1]), r2 = res(v[k][2]), r3 = res(v[k][3]);
      store(c, k, __builtin_amdgcn_perm(__builtin_amdgcn_perm(r3, r2, 0x0c0c0400u),
                                        __builtin_amdgcn_perm(r1, r0, 0x0c0c0400u), 0x05040100u));
    }
  }
}

// n < 4: the planes of one product byte by byte (NT threads).
template <int C, int NT>
__device__ __forceinline__ void crt_stage_small(const Mfma32Params& P, const CrtConsts& K, uint8_t* slot,
                                                uint64_t gprod, const ModQ32& m, int v_lo) {
  const uint32_t* A = P.a + gprod * P.n;
  const uint32_t* B = P.b + gprod * P.n;
  const int n = (int)P.n, t = (int)P.t, r = (int)P.r;
  for (int p = threadIdx.x; p < (int)P.a_plane; p += NT) {
    const int idx = (int)P.E - p;
    int32_t v = 0;
    if (idx >= 0 && idx < n) v = centred_lift(reduce_u32(A[idx], m), m.q);
    else if (idx < 0 && idx > -n) v = -centred_lift(reduce_u32(A[n + idx], m), m.q);
#pragma unroll
    for (int c = 0; c < C; ++c) slot[c * P.a_plane + p] = (uint8_t)centred_byte(v, K.m[c], K.magic[c], K.off[c]);
  }
  uint8_t* bbase = slot + C * P.a_plane;
  const int nb = (int)(P.b_rows * P.rowlen);
  for (int e = threadIdx.x; e < nb; e += NT) {
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

// ---------------------------------------------------------------------------
// One residue channel per wave (the paper's independent instance per modulus,
// Sec. 2.4): a workgroup holds the residue planes of a group of four 32x32
// output tiles and runs 4 ceil(C/4) waves.  Wave w < 4 floor(C/4) computes all
// four tiles of channel w over the whole K range; the R = C mod 4 remaining
// channels are spread over the last four waves (R = 1: one channel cut into four
// K quarters; R = 2: two channels in K halves; R = 3: one channel per wave, the
// fourth wave idle), so that every SIMD carries the same matrix work.  Sharing a
// channel, the four tiles reuse fragments: where the group is one product in
// 2 x 2 tiles, each K-step reads two A and two B fragments for four MFMAs (18
// bytes of LDS per lane and MFMA against 36 when every MFMA reads its own pair).
// After the K loop the channels meet in LDS: the waves of a cut channel add their
// int32 partial sums, each channel's (T mod m) (M/m)^-1 mod m goes in as a byte
// per output, and all threads then rebuild the outputs by the CRT.
// ---------------------------------------------------------------------------
template <int C>
struct CrtWaves {
  static constexpr int kFull = 4 * (C / 4);            // waves with a whole channel
  static constexpr int kRest = C - kFull;               // channels left for the last four waves
  static constexpr int kWaves = kFull + (kRest ? 4 : 0);
  static constexpr int kThreadsW = 64 * kWaves;
  // channel, part and number of parts of wave w (channel -1: idle)
  __device__ static void role(int w, int& ch, int& part, int& parts) {
    if (w < kFull) { ch = w; part = 0; parts = 1; return; }
    const int x = w - kFull;
    if (kRest == 1) { ch = kFull; part = x; parts = 4; }
    else if (kRest == 2) { ch = kFull + x / 2; part = x % 2; parts = 2; }
    else { ch = x < 3 ? kFull + x : -1; part = 0; parts = 1; }
  }
};

// LDS of the combine step, laid over the (no longer read) residue planes:
// the s bytes, dword [c][unit][blk][lane] holding the four outputs z = 8 blk + 4 g
// + e (e = 0..3) of the lane's column; then, for cut channels, the int32 partial
// sums of parts 1.., [slot][unit][rr][lane].
constexpr uint32_t kCrtSBytes = 4 * 4 * 64 * 4;    // per channel: 4 units x 4 blk x 64 lanes dwords
constexpr uint32_t kCrtPartBytes = 4 * 16 * 64 * 4;  // per part: 4 units x 16 values x 64 lanes int32

template <int C>
__host__ __device__ constexpr uint32_t crt_combine_bytes() {
  return C * kCrtSBytes + (C % 4 == 1 ? 3 : C % 4 == 2 ? 2 : 0) * kCrtPartBytes;
}

// A unit (one 32x32 tile) of the group: its slot, tile offsets, validity.
struct CrtUnit {
  int slot, z0, u0;
  bool valid;
};

__device__ __forceinline__ CrtUnit crt_unit(const Mfma32Params& P, const GroupInfo& gi, uint64_t grp, int i) {
  const uint64_t total_units = P.nprod << P.log2U;
  const uint32_t U = 1u << P.log2U;
  const uint64_t unit = grp * 4 + (uint64_t)i;
  CrtUnit cu;
  cu.valid = unit < total_units;
  const uint64_t prod = unit >> P.log2U;
  const uint32_t tile = (uint32_t)(unit & (U - 1));
  cu.slot = cu.valid ? (int)(prod - gi.first) : 0;
  cu.z0 = 32 * (int)(tile % P.tz);
  cu.u0 = 32 * (int)(tile / P.tz);
  return cu;
}

// The K loop of one channel over K-steps [st_lo, st_hi) for the group's four
// units.  SHARE22: one product in 2 x 2 tiles (units 0..3 = (z,u) = (0,0),
// (1,0), (0,1), (1,1)): A fragments by z, B fragments by u.  The next step's
// fragments are read while the current step's MFMAs run.  T4: t >= 4, so every
// K-step moves an A run by a multiple of four bytes (d t, 32-byte chunks): its
// byte shift and dword base are then fixed for the whole loop.
template <bool SHARE22, bool T4 = true>
__device__ __forceinline__ void crt_channel_loop(const Mfma32Params& P, const uint8_t* smem, int ch, int C,
                                                 const CrtUnit (&un)[4], int v_lo, int st_lo, int st_hi,
                                                 v16i (&acc)[4]) {
  const int lane = threadIdx.x & 63;
  const int zl = lane & 31, g = lane >> 5;
  const int rs = (int)P.b_rowstride;
  constexpr int NA = SHARE22 ? 2 : 4;  // A fragments per K-step (units 0..NA-1)
  constexpr int NB = SHARE22 ? 2 : 4;  // B fragments per K-step (units 0, 2 when shared)
  const uint32_t* ap[NA];
  const uint8_t* bp[NB];
  int Sb[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const uint8_t* slot = smem + un[i].slot * P.slot_bytes;
    ap[i] = (const uint32_t*)(slot + ch * P.a_plane);
    Sb[i] = (int)P.E - (un[i].z0 + zl) + 16 * g;
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int u = SHARE22 ? 2 * j : j;
    const uint8_t* slot = smem + un[u].slot * P.slot_bytes;
    bp[j] = slot + C * P.a_plane + ch * P.b_plane + (un[u].u0 + zl - v_lo) * rs + 16 * g;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = v16i{};
  if (st_lo >= st_hi) return;
  auto soff = [&](int st) { return -((st >> P.log2spd) << P.log2t) + ((st & (P.spd - 1)) << 5); };
  auto boff = [&](int st) { return -(st >> P.log2spd) * rs + ((st & (P.spd - 1)) << 5); };
  const uint32_t* apb[NA];  // T4: dword base and byte shift of each A run
  uint32_t shb[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    apb[i] = ap[i] + (Sb[i] >> 2);  // Sb >= 0
    shb[i] = (uint32_t)(Sb[i] & 3);
  }
  uint32_t x[NA][5];
  v4i b[NB];
  auto load = [&](int st) {
    const int so = soff(st), bo = boff(st);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const uint32_t* p = T4 ? apb[i] + (so >> 2) : ap[i] + ((Sb[i] + so) >> 2);
#pragma unroll
      for (int k = 0; k < 5; ++k) x[i][k] = p[k];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) b[j] = *(const v4i*)(bp[j] + bo);
  };
  load(st_lo);
  for (int st = st_lo; st < st_hi; ++st) {
    v4i a[NA], bc[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const uint32_t sh = T4 ? shb[i] : (uint32_t)((Sb[i] + soff(st)) & 3);
      a[i][0] = (int)__builtin_amdgcn_alignbyte(x[i][1], x[i][0], sh);
      a[i][1] = (int)__builtin_amdgcn_alignbyte(x[i][2], x[i][1], sh);
      a[i][2] = (int)__builtin_amdgcn_alignbyte(x[i][3], x[i][2], sh);
      a[i][3] = (int)__builtin_amdgcn_alignbyte(x[i][4], x[i][3], sh);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) bc[j] = b[j];
    // the last step re-reads its own fragments (in bounds, unused)
    load(st + 1 < st_hi ? st + 1 : st);
    if constexpr (SHARE22) {
      acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0], bc[0], acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1], bc[0], acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0], bc[1], acc[2], 0, 0, 0);
      acc[3] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1], bc[1], acc[3], 0, 0, 0);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], bc[i], acc[i], 0, 0, 0);
    }
  }
}

// s = (T mod m) y mod m as one Shoup product: for the 32-bit word T + 2^31 and
// y < m, (T + 2^31) y - floor((T + 2^31) yp / 2^32) m lies in [0, 2m), and the
// precomputed (2^31 y) mod m removes the offset.
__device__ __forceinline__ uint32_t crt_s(int32_t T, uint32_t m, uint32_t y, uint32_t yp, uint32_t oy) {
  const uint32_t tu = (uint32_t)T + 0x80000000u;
  uint32_t su = tu * y - __umulhi(tu, yp) * m;
  su = min(su, su - m);
  return su >= oy ? su - oy : su + m - oy;
}

template <int C, bool SMALL, bool SHARE22>
__global__ __launch_bounds__(CrtWaves<C>::kThreadsW)
void crt_wave_kernel(const Mfma32Params P, const CrtConsts K) {
  constexpr int NT = CrtWaves<C>::kThreadsW;
  extern __shared__ __align__(16) uint8_t smem[];
  const uint64_t grp = blockIdx.x;
  const GroupInfo gi = group_info(P, grp);
  // ---- stage the residue planes of the group's products
  if constexpr (SMALL) {
    for (uint32_t s = 0; s < gi.nslots; ++s)
      crt_stage_small<C, NT>(P, K, smem + s * P.slot_bytes, slot_gp(gi, s), P.mods[slot_li(gi, s)], gi.v_lo);
  } else {
    const uint32_t nitems = gi.nslots * (P.n >> 1);
    for (uint32_t base = 0; base < nitems; base += kStageItems * NT) {
      crt_stage_pass<C, NT>(P, K, gi, smem, base, nitems);
    }
    stage_zero_fill<C, NT>(P, gi, smem);
  }
  __syncthreads();

  // ---- this wave's channel over its share of K
  const int wave = (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int ch, part, parts;
  CrtWaves<C>::role(wave, ch, part, parts);
  CrtUnit un[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) un[i] = crt_unit(P, gi, grp, i);
  v16i acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = v16i{};
  if (ch >= 0) {
    const int steps = (int)(P.r << P.log2spd);
    const int st_lo = part * steps / parts, st_hi = (part + 1) * steps / parts;
    crt_channel_loop<SHARE22, !SMALL>(P, smem, ch, C, un, gi.v_lo, st_lo, st_hi, acc);
  }
  __syncthreads();  // the residue planes are read for the last time

  // ---- cut channels: parts 1.. leave their partial sums, part 0 adds them
  uint32_t* sb = (uint32_t*)smem;                        // [C][4 units][4 blk][64 lanes]
  int32_t* parts_lds = (int32_t*)(smem + C * kCrtSBytes);  // [slot][4 units][16][64 lanes]
  if (ch >= 0 && part > 0) {
    const int slot = CrtWaves<C>::kRest == 1 ? part - 1 : (ch - CrtWaves<C>::kFull);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) parts_lds[((slot * 4 + i) * 16 + rr) * 64 + lane] = acc[i][rr];
  }
  __syncthreads();
  if (ch >= 0 && part == 0) {
    if (parts > 1) {
      for (int pp = 1; pp < parts; ++pp) {
        const int slot = CrtWaves<C>::kRest == 1 ? pp - 1 : (ch - CrtWaves<C>::kFull);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int rr = 0; rr < 16; ++rr) acc[i][rr] += parts_lds[((slot * 4 + i) * 16 + rr) * 64 + lane];
      }
    }
    const uint32_t m = K.m[ch], y = K.y[ch], yp = K.yp[ch], oy = K.oy[ch];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= crt_s(acc[i][4 * blk + e], m, y, yp, oy) << (8 * e);
        sb[((ch * 4 + i) * 4 + blk) * 64 + lane] = w;
      }
  }
  __syncthreads();

  // ---- reconstruction: thread -> (unit, blk, lane) word groups, four outputs each.
  // X' = sum_c s_c M/m_c = X + kappa M with kappa = round(sum_c s_c / m_c), since
  // |X| / M < 1/2; the fp32 sum is within about 100 2^-24 of the true fraction
  // (C <= 11), inside the 2^-17 margin the moduli leave, so kappa is exact.
  for (int idx = threadIdx.x; idx < 4 * 4 * 64; idx += NT) {
    const int i = idx >> 8, blk = (idx >> 6) & 3, ln = idx & 63;
    const CrtUnit ui = crt_unit(P, gi, grp, i);  // recomputed: a dynamic index into un[] would go to scratch
    if (!ui.valid) continue;
    const int u = ui.u0 + (ln & 31);
    const int zb = ui.z0 + 8 * blk + 4 * (ln >> 5);
    if (u >= (int)P.r || zb >= (int)P.t) continue;
    uint32_t li;
    const uint64_t gprod = global_product(P, gi.first + (uint64_t)ui.slot, &li);
    const ModQ32 mq = P.mods[li];
    uint32_t sw[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sw[c] = sb[((c * 4 + i) * 4 + blk) * 64 + ln];
    uint32_t out[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float f = 0.0f;
      uint64_t x = mq.lift;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const uint32_t sc = (sw[c] >> (8 * e)) & 0xFFu;
        f += (float)sc * K.invm[c];
        x += (uint64_t)sc * K.w[li][c];
      }
      const uint32_t kappa = (uint32_t)floorf(f + 0.5f);
      x -= (uint64_t)kappa * K.Mq[li];
      out[e] = mq.q < 0x80000000u ? reduce_u64_q31(x, mq.mu, mq.q) : reduce_u64(x, mq);
    }
    uint32_t* Cout = P.c + gprod * P.n + (size_t)u * P.t;
    if (zb + 3 < (int)P.t) {
      *(uint4*)(Cout + zb) = make_uint4(out[0], out[1], out[2], out[3]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (zb + e < (int)P.t) Cout[zb + e] = out[e];
    }
  }
}

// ---------------------------------------------------------------------------
// Two-phase form for one product in 2 x 2 tiles with C = 8 or 9 channels, whose
// C residue planes would hold a workgroup of their own per CU (9 x 14 KiB at
// n = 4096).  A workgroup of eight waves stages and multiplies channels
// [0, CA) (CA = ceil(C / 2)), then [CA, C), each phase in planes 0.. of the
// same LDS; its largest LDS use is 76 KiB, so two workgroups share a CU and one
// stages or reconstructs while the other multiplies.  Within a phase of CP
// channels: CP = 5 puts channels 0-3 on waves 0-3 and channel 4 on waves 4-7
// in K quarters; CP = 4 puts channel k on waves k and k + 4 in K halves (every
// SIMD gets the same matrix work).  A K part other than a channel's first hands
// over its partial sums as residues mod m (one byte per output: T mod m is all
// the reconstruction needs, and it is additive), which the first part adds in
// before forming s = (T mod m) (M/m)^-1 mod m.  The s bytes of phase 0 go just
// past phase 1's planes, those of phase 1 just below, so the reconstruction finds
// all C channels in one run of LDS.
// ---------------------------------------------------------------------------
template <int CP>
struct CrtPhaseWaves {
  static_assert(CP == 4 || CP == 5, "phases of four or five channels");
  static constexpr int kOtherParts = CP == 4 ? 4 : 3;  // parts that hand over residues
  __device__ static void role(int w, int& ch, int& part, int& parts) {
    if (CP == 4) { ch = w & 3; part = w >> 2; parts = 2; return; }
    if (w < 4) { ch = w; part = 0; parts = 1; return; }
    ch = 4; part = w - 4; parts = 4;
  }
  __device__ static int other_slot(int ch, int part) { return CP == 4 ? ch : part - 1; }
};

template <int C>
__host__ __device__ constexpr uint32_t crt_phase_lds(uint32_t plane_bytes) {
  constexpr uint32_t CA = (C + 1) / 2, CB = C - CA;
  const uint32_t p0 = CA * plane_bytes, p1 = CB * plane_bytes + CA * kCrtSBytes;
  return p0 > p1 ? p0 : p1;
}

// One phase: channels [c0, c0 + CP) staged, multiplied and turned into s bytes at sbase.
template <int CP>
__device__ __forceinline__ void crt_phase(const Mfma32Params& P, const CrtConsts& K, const GroupInfo& gi,
                                          const CrtUnit (&un)[4], uint8_t* smem, int c0, uint32_t sbase) {
  constexpr int NT = 8 * 64;
  const uint32_t nitems = gi.nslots * (P.n >> 1);
  for (uint32_t base = 0; base < nitems; base += kStageItems * NT)
    crt_stage_pass<CP, NT>(P, K, gi, smem, base, nitems, c0);
  stage_zero_fill<CP, NT>(P, gi, smem);
  __syncthreads();
  const int wave = (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int ch, part, parts;
  CrtPhaseWaves<CP>::role(wave, ch, part, parts);
  v16i acc[4];
  const int steps = (int)(P.r << P.log2spd);
  crt_channel_loop<true>(P, smem, ch, CP, un, gi.v_lo, part * steps / parts, (part + 1) * steps / parts, acc);
  __syncthreads();  // the planes are read for the last time
  const int gc = c0 + ch;
  const uint32_t m = K.m[gc];
  uint32_t* other = (uint32_t*)smem;  // [slot][4 units][4 blk][64 lanes], four residue bytes a dword
  if (part > 0) {
    const int sl = CrtPhaseWaves<CP>::other_slot(ch, part);
    const uint32_t magic = K.magic[gc], off = K.off[gc];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= signed_mod(acc[i][4 * blk + e], m, magic, off) << (8 * e);
        other[((sl * 4 + i) * 4 + blk) * 64 + lane] = w;
      }
  }
  __syncthreads();
  if (part == 0) {
    uint32_t* sb = (uint32_t*)(smem + sbase);
    const uint32_t y = K.y[gc], yp = K.yp[gc], oy = K.oy[gc];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        int32_t T[4] = {acc[i][4 * blk], acc[i][4 * blk + 1], acc[i][4 * blk + 2], acc[i][4 * blk + 3]};
        for (int pp = 1; pp < parts; ++pp) {
          const uint32_t w = other[((CrtPhaseWaves<CP>::other_slot(ch, pp) * 4 + i) * 4 + blk) * 64 + lane];
#pragma unroll
          for (int e = 0; e < 4; ++e) T[e] += (int32_t)((w >> (8 * e)) & 0xFFu);
        }
        uint32_t sw = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) sw |= crt_s(T[e], m, y, yp, oy) << (8 * e);
        sb[((ch * 4 + i) * 4 + blk) * 64 + lane] = sw;
      }
  }
  __syncthreads();  // the residue bytes are read before the next phase stages over them
}

template <int C>
__global__ __launch_bounds__(8 * 64) __attribute__((amdgpu_waves_per_eu(4, 4)))
void crt_phase_kernel(const Mfma32Params P, const CrtConsts K) {
  static_assert(C == 8 || C == 9, "two phases of four or five channels");
  constexpr int CA = (C + 1) / 2, CB = C - CA;
  constexpr int NT = 8 * 64;
  extern __shared__ __align__(16) uint8_t smem[];
  const uint64_t grp = blockIdx.x;
  const GroupInfo gi = group_info(P, grp);
  CrtUnit un[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) un[i] = crt_unit(P, gi, grp, i);
  const uint32_t plane_bytes = P.a_plane + P.b_plane;
  const uint32_t sb0 = CB * plane_bytes;                // s bytes of channels [0, CA)
  const uint32_t sb1 = sb0 - CB * kCrtSBytes;           // s bytes of channels [CA, C)
  crt_phase<CA>(P, K, gi, un, smem, 0, sb0);
  crt_phase<CB>(P, K, gi, un, smem, CA, sb1);

  // ---- reconstruction (as in crt_wave_kernel), channel c's s bytes at
  // sb0 + c * kCrtSBytes for c < CA, sb1 + (c - CA) * kCrtSBytes after
  for (int idx = threadIdx.x; idx < 4 * 4 * 64; idx += NT) {
    const int i = idx >> 8, blk = (idx >> 6) & 3, ln = idx & 63;
    const CrtUnit ui = crt_unit(P, gi, grp, i);
    if (!ui.valid) continue;
    const int u = ui.u0 + (ln & 31);
    const int zb = ui.z0 + 8 * blk + 4 * (ln >> 5);
    if (u >= (int)P.r || zb >= (int)P.t) continue;
    uint32_t li;
    const uint64_t gprod = global_product(P, gi.first + (uint64_t)ui.slot, &li);
    const ModQ32 mq = P.mods[li];
    uint32_t sw[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const uint32_t* sb = (const uint32_t*)(smem + (c < CA ? sb0 + c * kCrtSBytes : sb1 + (c - CA) * kCrtSBytes));
      sw[c] = sb[(i * 4 + blk) * 64 + ln];
    }
    uint32_t out[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float f = 0.0f;
      uint64_t x = mq.lift;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const uint32_t sc = (sw[c] >> (8 * e)) & 0xFFu;
        f += (float)sc * K.invm[c];
        x += (uint64_t)sc * K.w[li][c];
      }
      const uint32_t kappa = (uint32_t)floorf(f + 0.5f);
      x -= (uint64_t)kappa * K.Mq[li];
      out[e] = mq.q < 0x80000000u ? reduce_u64_q31(x, mq.mu, mq.q) : reduce_u64(x, mq);
    }
    uint32_t* Cout = P.c + gprod * P.n + (size_t)u * P.t;
    if (zb + 3 < (int)P.t) {
      *(uint4*)(Cout + zb) = make_uint4(out[0], out[1], out[2], out[3]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (zb + e < (int)P.t) Cout[zb + e] = out[e];
    }
  }
}

}  // namespace pm
