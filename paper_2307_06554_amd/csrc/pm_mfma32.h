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
// c = sum_s T_s 2^(8s) mod q is one signed 64-bit dot product of the T_s with the
// centred residues of 2^(8s) when the host has shown it stays below 2^62, else
// Horner steps; either way a Barrett reduction ends it.  In the cyclic ring
// x^n - 1 (the `cyclic` flag) the wrapped terms keep their sign.
#pragma once
#include "pm_common.h"

namespace pm {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kMaxQ = 16;  // moduli per launch (RNS channels are chunked above this)
constexpr int kThreads = 256;  // threads per workgroup (4 waves)

struct Mfma32Params {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* c;
  uint64_t nprod;        // products handled by this launch
  uint32_t n, t, r;      // n = t * r
  uint32_t log2n;
  uint32_t log2t, log2spd, spd;  // K-steps of 32 per d: spd = max(1, t/32)
  uint32_t rowlen;       // bytes of one B row that are read (= 32 * spd)
  uint32_t tz, tu, log2U;  // output tiles of 32x32 per product: tz * tu = 2^log2U
  uint32_t slots;        // products staged per workgroup
  uint32_t a_plane;      // bytes per limb plane of the reversed ext array
  uint32_t b_rows, b_rowstride, b_plane;  // B rows staged per product, their stride, plane size
  uint32_t slot_bytes;   // L * (a_plane + b_plane)
  uint32_t E;            // ext index held at reversed position 0
  // Product i of this launch is global product (i / lc) * nq_total + l0 + (i % lc)
  // and uses modulus mods[i % lc]; with lrep > 1 (dense sub-product batches)
  // product i is global product i and uses modulus mods[(i / lrep) % lc].
  uint32_t lc, nq_total, l0, lrep;
  uint32_t fast_epilogue;  // 1: sum_s T_s * rcent[s] is known to stay below 2^62 in magnitude
  uint32_t cyclic;         // 1: ring Z_q[x]/(x^n - 1): wrapped terms keep their sign
  uint32_t b_shared;       // 1: one b per modulus channel, b + (l0 + channel) * n, for every product
  // K split across workgroups (grouped plans, groups of one product only): group g is
  // cut into kparts runs of K-steps; run p stores its residues where c's would go in
  // part_ws + p * nprod * n, and a separate kernel adds the runs up mod q.
  uint32_t kparts;
  uint32_t* part_ws;       // [kparts][nprod][n]
  ModQ32 mods[kMaxQ];
  int32_t rcent[kMaxQ][8];  // 2^(8s) mod q as a centred residue, s < 2L-1
};

// Byte i of each of the four digit words, packed into one word (byte k from w[k]):
// a 4x4 byte transpose in two rounds of byte permutes (v_perm_b32 picks bytes of
// the pair {src0 : src1}, src1 holding bytes 0-3).
template <int L>
__device__ __forceinline__ void transpose_store(uint8_t* base, uint32_t plane, uint32_t off, const uint32_t (&w)[4]) {
  const uint32_t lo01 = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);  // w0.0 w1.0 w0.1 w1.1
  const uint32_t lo23 = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);  // w2.0 w3.0 w2.1 w3.1
  *(uint32_t*)(base + off) = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
  if constexpr (L > 1) *(uint32_t*)(base + plane + off) = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
  if constexpr (L > 2) {
    const uint32_t hi01 = __builtin_amdgcn_perm(w[1], w[0], 0x07030602u);  // w0.2 w1.2 w0.3 w1.3
    const uint32_t hi23 = __builtin_amdgcn_perm(w[3], w[2], 0x07030602u);
    *(uint32_t*)(base + 2 * plane + off) = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
    if constexpr (L > 3) *(uint32_t*)(base + 3 * plane + off) = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
  }
}

// Stage the digit planes of one product of degree bound n < 4 into an LDS slot,
// byte by byte (larger degrees are staged a word group at a time, below).
//   A: reversed ext planes, position p holds ext[E - p] (ext[i] = a_i for i >= 0,
//      -a_{n+i} for i < 0, zero outside (-n, n)).
//   B: rows v in [v_lo, v_lo + b_rows): row v < r holds b[v t + w] for v >= 0 and
//      -b[(v + r) t + w] for v < 0; rows v >= r and bytes w >= t are zero.
template <int L>
__device__ __forceinline__ void mfma32_stage(const Mfma32Params& P, uint8_t* slot, uint64_t gprod, uint64_t bprod,
                                             const ModQ32& m, int v_lo) {
  const uint32_t* A = P.a + gprod * P.n;
  const uint32_t* B = P.b + bprod * P.n;
  const uint32_t q = m.q, thr = m.thr;
  const int n = (int)P.n, t = (int)P.t, r = (int)P.r;
  const int a_dw = (int)(P.a_plane >> 2);
  uint8_t* bbase = slot + L * P.a_plane;
  const int row_dw = (int)(P.rowlen >> 2);
  for (int dw = threadIdx.x; dw < a_dw; dw += blockDim.x) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int idx = (int)P.E - (dw * 4 + k);
      uint32_t dg = 0;
      if (idx >= 0 && idx < n) dg = digits32<L>(reduce_u32(A[idx], m), q, thr);
      else if (idx < 0 && idx > -n) {
        const uint32_t xr = reduce_u32(A[n + idx], m);
        dg = P.cyclic ? digits32<L>(xr, q, thr) : neg_digits32<L>(xr, q, thr);
      }
      w[k] = dg;
    }
    transpose_store<L>(slot, P.a_plane, dw * 4, w);
  }
  const int nb = (int)P.b_rows * row_dw;
  for (int e = threadIdx.x; e < nb; e += blockDim.x) {
    const int row = e / row_dw, wd = e - row * row_dw;
    const int v = v_lo + row;
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ww = wd * 4 + k;
      uint32_t dg = 0;
      if (ww < t) {
        if (v >= 0 && v < r) dg = digits32<L>(reduce_u32(B[v * t + ww], m), q, thr);
        else if (v < 0 && v > -r) {
          const uint32_t xr = reduce_u32(B[(v + r) * t + ww], m);
          dg = P.cyclic ? digits32<L>(xr, q, thr) : neg_digits32<L>(xr, q, thr);
        }
      }
      w[k] = dg;
    }
    transpose_store<L>(bbase, P.b_plane, row * P.b_rowstride + wd * 4, w);
  }
}

// LDS reads of one K-step: five dwords around each limb's 16-byte A run
// (starting at byte S, any alignment) and each limb's 16-byte B run.
template <int L>
__device__ __forceinline__ void araw_load(uint32_t (&x)[L][5], const uint8_t* aplane, uint32_t a_plane, int S) {
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint32_t* p = (const uint32_t*)(aplane + i * a_plane) + (S >> 2);
#pragma unroll
    for (int k = 0; k < 5; ++k) x[i][k] = p[k];
  }
}
template <int L>
__device__ __forceinline__ void b_load(v4i (&b)[L], const uint8_t* bplane, uint32_t b_plane, int boff) {
#pragma unroll
  for (int j = 0; j < L; ++j) b[j] = *(const v4i*)(bplane + j * b_plane + boff);
}
template <int L>
__device__ __forceinline__ void a_align(v4i (&a)[L], const uint32_t (&x)[L][5], uint32_t sh) {
#pragma unroll
  for (int i = 0; i < L; ++i) {
    a[i][0] = (int)__builtin_amdgcn_alignbyte(x[i][1], x[i][0], sh);
    a[i][1] = (int)__builtin_amdgcn_alignbyte(x[i][2], x[i][1], sh);
    a[i][2] = (int)__builtin_amdgcn_alignbyte(x[i][3], x[i][2], sh);
    a[i][3] = (int)__builtin_amdgcn_alignbyte(x[i][4], x[i][3], sh);
  }
}
// The same K-step with the next step's A fragments aligned in place during the
// last column: right after the column's MFMA on limb i (the last to read a[i]),
// a[i] takes limb i of the next step (its runs read a step earlier) and the raw
// registers are re-read for the step after that, so no bubble separates the
// steps and no second A register set is needed.
template <int L>
__device__ __forceinline__ void mfma_step_tail(v16i (&acc)[2 * L - 1], v4i (&a)[L], uint32_t (&araw)[L][5],
                                               uint32_t sh_next, const uint8_t* aplane, uint32_t a_plane,
                                               int S_after, v4i (&b)[L], const uint8_t* bplane, uint32_t b_plane,
                                               int boff_next) {
#pragma unroll
  for (int j = 0; j < L - 1; ++j) {
#pragma unroll
    for (int i = 0; i < L; ++i)
      acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i + j], 0, 0, 0);
    b[j] = *(const v4i*)(bplane + j * b_plane + boff_next);
    __builtin_amdgcn_sched_barrier(0);
  }
  constexpr int j = L - 1;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i + j], 0, 0, 0);
    a[i][0] = (int)__builtin_amdgcn_alignbyte(araw[i][1], araw[i][0], sh_next);
    a[i][1] = (int)__builtin_amdgcn_alignbyte(araw[i][2], araw[i][1], sh_next);
    a[i][2] = (int)__builtin_amdgcn_alignbyte(araw[i][3], araw[i][2], sh_next);
    a[i][3] = (int)__builtin_amdgcn_alignbyte(araw[i][4], araw[i][3], sh_next);
    const uint32_t* p = (const uint32_t*)(aplane + i * a_plane) + (S_after >> 2);
#pragma unroll
    for (int k = 0; k < 5; ++k) araw[i][k] = p[k];
    __builtin_amdgcn_sched_barrier(0);
  }
  b[j] = *(const v4i*)(bplane + j * b_plane + boff_next);
  __builtin_amdgcn_sched_barrier(0);
}

// The same K-step with the A fragments double-buffered: with column j, limb j
// of the next step's runs (read one step earlier) is aligned into `an` and the
// limb's runs of the step after that are read, so the next step starts
// straight with MFMAs and at most a few LDS reads are in flight at a time.
template <int L>
__device__ __forceinline__ void mfma_step_pp(v16i (&acc)[2 * L - 1], const v4i (&a)[L], v4i (&an)[L],
                                             uint32_t (&araw)[L][5], uint32_t sh_next, const uint8_t* aplane,
                                             uint32_t a_plane, int S_after, v4i (&b)[L], const uint8_t* bplane,
                                             uint32_t b_plane, int boff_next) {
#pragma unroll
  for (int j = 0; j < L; ++j) {
#pragma unroll
    for (int i = 0; i < L; ++i)
      acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i + j], 0, 0, 0);
    b[j] = *(const v4i*)(bplane + j * b_plane + boff_next);
    // limb j of the next step's A: align the runs read a step earlier, then re-read
    // the freed raw registers (spread over the columns to keep few LDS reads in flight)
    an[j][0] = (int)__builtin_amdgcn_alignbyte(araw[j][1], araw[j][0], sh_next);
    an[j][1] = (int)__builtin_amdgcn_alignbyte(araw[j][2], araw[j][1], sh_next);
    an[j][2] = (int)__builtin_amdgcn_alignbyte(araw[j][3], araw[j][2], sh_next);
    an[j][3] = (int)__builtin_amdgcn_alignbyte(araw[j][4], araw[j][3], sh_next);
    const uint32_t* p = (const uint32_t*)(aplane + j * a_plane) + (S_after >> 2);
#pragma unroll
    for (int k = 0; k < 5; ++k) araw[j][k] = p[k];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One 32x32 output tile of one product: the K loop (K-steps [st_lo, st_hi), all
// of them by default) for all L*L limb pairs, two steps per iteration so that
// the two A fragment sets swap roles without register copies.  T4: t >= 4, so a
// K-step moves the A runs by a multiple of four bytes (d t, 32-byte chunks): the
// byte shift and the lane's dword base are then fixed for the whole loop and each
// step adds only a uniform offset (likewise the B rows' lane base).
template <int L, bool T4 = true>
__device__ __forceinline__ void mfma32_tile(const Mfma32Params& P, const uint8_t* aplane, const uint8_t* bplane,
                                            int z0, int u0, int v_lo, v16i (&acc)[2 * L - 1], int st_lo = 0,
                                            int st_hi = -1, int E = -1) {
  const int lane = threadIdx.x & 63;
  const int zl = lane & 31, g = lane >> 5;
  // A: lane reads reversed positions S .. S+15 with S = E - (d t + z - w0 - 16 g)
  // (E: the ext index at reversed position 0, P.E unless a K window says otherwise).
  const int S0 = (E < 0 ? (int)P.E : E) - (z0 + zl) + 16 * g;  // >= 0
  // B: lane reads row (u - d) - v_lo, bytes w0 + 16 g .. + 15.
  const int B0 = (u0 + zl - v_lo) * (int)P.b_rowstride + 16 * g;
  const int steps = st_hi < 0 ? (int)(P.r << P.log2spd) : st_hi;  // one past the last K-step
  const int rs = (int)P.b_rowstride;
  const uint32_t a_plane = P.a_plane, b_plane = P.b_plane;
#pragma unroll
  for (int s = 0; s < 2 * L - 1; ++s) acc[s] = v16i{};
  // with T4 the lane's parts go into the plane bases and S_of / B_of are uniform
  const uint8_t* ap = T4 ? aplane + 4 * (S0 >> 2) : aplane;
  const uint8_t* bp = T4 ? bplane + B0 : bplane;
  const int Sl = T4 ? 0 : S0, Bl = T4 ? 0 : B0;
  const uint32_t sh0 = (uint32_t)(S0 & 3);
  auto S_of = [&](int st) { return Sl - ((st >> P.log2spd) << P.log2t) + ((st & (P.spd - 1)) << 5); };
  auto B_of = [&](int st) { return Bl - (st >> P.log2spd) * rs + ((st & (P.spd - 1)) << 5); };
  auto sh_of = [&](int st) { return T4 ? sh0 : (uint32_t)(S_of(st) & 3); };

  // Steps past the end are clamped to the last one: their reads stay in bounds
  // and their results are never used.
  auto clamp = [&](int st) { return st < steps ? st : steps - 1; };
  uint32_t araw[L][5];
  v4i a0[L], a1[L], b[L];
  araw_load<L>(araw, ap, a_plane, S_of(st_lo));
  b_load<L>(b, bp, b_plane, B_of(st_lo));
  a_align<L>(a0, araw, sh_of(st_lo));
  araw_load<L>(araw, ap, a_plane, S_of(clamp(st_lo + 1)));
  int st = st_lo;
  for (; st + 1 < steps; st += 2) {
    mfma_step_pp<L>(acc, a0, a1, araw, sh_of(st + 1), ap, a_plane, S_of(clamp(st + 2)), b, bp, b_plane,
                    B_of(st + 1));
    mfma_step_pp<L>(acc, a1, a0, araw, sh_of(clamp(st + 2)), ap, a_plane, S_of(clamp(st + 3)), b, bp, b_plane,
                    B_of(clamp(st + 2)));
  }
  if (st < steps)
    mfma_step_pp<L>(acc, a0, a1, araw, sh_of(st), ap, a_plane, S_of(st), b, bp, b_plane, B_of(st));
}

// Recombination c = sum_s T_s 2^(8s) mod q of the 16 outputs a lane holds, then
// the stores.
template <int L>
__device__ __forceinline__ void mfma32_reduce(const Mfma32Params& P, const ModQ32& mp, const int32_t* rcp,
                                              const v16i (&acc)[2 * L - 1], uint32_t (&out)[16]) {
  // constants read once (the loops below would otherwise reload them per value)
  const ModQ32 m = mp;
  int32_t rc[2 * L - 1];
#pragma unroll
  for (int s = 0; s < 2 * L - 1; ++s) rc[s] = rcp[s];
  if (P.fast_epilogue) {
    // sum_s T_s * (2^(8s) mod q, centred) stays below 2^62 in magnitude (checked on
    // the host); adding lift makes it non-negative
    if (m.q < 0x80000000u) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        uint64_t x = m.lift;  // unsigned words: the sum may pass 2^63
#pragma unroll
        for (int s = 0; s < 2 * L - 1; ++s) x += (uint64_t)((int64_t)acc[s][rr] * (int64_t)rc[s]);
        out[rr] = reduce_u64_q31(x, m.mu, m.q);
      }
    } else {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        int64_t x = 0;
#pragma unroll
        for (int s = 0; s < 2 * L - 1; ++s) x += (int64_t)acc[s][rr] * (int64_t)rc[s];
        out[rr] = reduce_i64(x, m);
      }
    }
  } else {
    // Horner in radix 2^8 from the top shift class down.
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      uint32_t v = reduce_i64((int64_t)acc[2 * L - 2][rr], m);
#pragma unroll
      for (int s = 2 * L - 3; s >= 0; --s) v = reduce_i64((int64_t)v * 256 + (int64_t)acc[s][rr], m);
      out[rr] = v;
    }
  }
}
// The 16 residues of a lane to c: z = z0 + 8 blk + 4 g + e, u = u0 + (lane & 31).
__device__ __forceinline__ void mfma32_store(const Mfma32Params& P, uint64_t gprod, int z0, int u0,
                                             const uint32_t (&out)[16]) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 5;
  const int u = u0 + (lane & 31);
  if (u >= (int)P.r) return;
  uint32_t* C = P.c + gprod * P.n;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int zb = z0 + 8 * blk + 4 * g;
    if (zb + 3 < (int)P.t) {
      *(uint4*)(C + (size_t)u * P.t + zb) = make_uint4(out[4 * blk], out[4 * blk + 1], out[4 * blk + 2], out[4 * blk + 3]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (zb + e < (int)P.t) C[(size_t)u * P.t + zb + e] = out[4 * blk + e];
    }
  }
}
template <int L>
__device__ __forceinline__ void mfma32_epilogue(const Mfma32Params& P, uint64_t gprod, const ModQ32& m,
                                                const int32_t* rc, int z0, int u0, const v16i (&acc)[2 * L - 1]) {
  uint32_t out[16];
  mfma32_reduce<L>(P, m, rc, acc, out);
  mfma32_store(P, gprod, z0, u0, out);
}

// ---------------------------------------------------------------------------
// Workgroup = group of 4 output tiles (grp*4 .. grp*4+3 over (product, tile)).
// Staging items of one group (n >= 4): per staged product, n/4 A items (a word
// group a[4m..4m+3] -> reversed dword E/4 - m, and its negated copy n/4 dwords
// further) and n/4 B items (b[vs t + 4wd ..] -> row vs (+) and row vs - r (-)).
// ---------------------------------------------------------------------------
constexpr int kPrefetch = 8;  // uint4 loads in flight per thread during staging

struct GroupInfo {
  uint64_t first;     // first product of the group
  uint32_t nslots;    // products staged
  int v_lo;           // first staged B row
  uint64_t gp[4];     // global product index of each staged slot
  uint32_t li[4];     // modulus index of each staged slot
};

__device__ __forceinline__ uint64_t global_product(const Mfma32Params& P, uint64_t prod, uint32_t* li) {
  if ((prod >> 32) == 0) {  // 32-bit quotients (the usual case) are much cheaper
    const uint32_t p32 = (uint32_t)prod;
    if (P.lrep > 1) {
      *li = (p32 / P.lrep) % P.lc;
      return prod;
    }
    const uint32_t qt = p32 / P.lc;
    *li = p32 - qt * P.lc;
    return (uint64_t)qt * P.nq_total + P.l0 + *li;
  }
  if (P.lrep > 1) {
    *li = (uint32_t)((prod / P.lrep) % P.lc);
    return prod;
  }
  *li = (uint32_t)(prod % P.lc);
  return (prod / P.lc) * P.nq_total + P.l0 + *li;
}

// Product whose b a staged product uses: its own, or its channel's shared one.
__device__ __forceinline__ uint64_t b_product(const Mfma32Params& P, uint64_t gp, uint32_t li) {
  return P.b_shared ? (uint64_t)(P.l0 + li) : gp;
}

// Slot-indexed fields by selects (a dynamic index would put the arrays in scratch).
__device__ __forceinline__ uint64_t slot_gp(const GroupInfo& g, uint32_t s) {
  return s == 0 ? g.gp[0] : s == 1 ? g.gp[1] : s == 2 ? g.gp[2] : g.gp[3];
}
__device__ __forceinline__ uint32_t slot_li(const GroupInfo& g, uint32_t s) {
  return s == 0 ? g.li[0] : s == 1 ? g.li[1] : s == 2 ? g.li[2] : g.li[3];
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t wave_uniform(uint64_t x) {
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)) << 32) |
         __builtin_amdgcn_readfirstlane((uint32_t)x);
}
__device__ __forceinline__ uint64_t sel4(const uint64_t (&v)[4], uint32_t s) {
  return s == 0 ? v[0] : s == 1 ? v[1] : s == 2 ? v[2] : v[3];
}
__device__ __forceinline__ uint32_t sel4(const uint32_t (&v)[4], uint32_t s) {
  return s == 0 ? v[0] : s == 1 ? v[1] : s == 2 ? v[2] : v[3];
}

// The group's products and moduli; grp is the same in every lane, and so is the
// result (kept in scalar registers).
__device__ __forceinline__ GroupInfo group_info(const Mfma32Params& P, uint64_t grp) {
  GroupInfo gi;
  const uint32_t U = 1u << P.log2U;
  const uint64_t unit0 = grp * 4;
  gi.first = unit0 >> P.log2U;
  const uint64_t left = P.nprod - gi.first;
  gi.nslots = left < P.slots ? (uint32_t)left : P.slots;
  const int ut_lo = U >= 4 ? (int)((uint32_t)(unit0 & (U - 1)) / P.tz) : 0;
  gi.v_lo = 32 * ut_lo - ((int)P.r - 1);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    gi.gp[s] = 0;
    gi.li[s] = 0;
    if ((uint32_t)s < gi.nslots) gi.gp[s] = global_product(P, gi.first + s, &gi.li[s]);
    gi.gp[s] = wave_uniform(gi.gp[s]);
    gi.li[s] = wave_uniform(gi.li[s]);
  }
  return gi;
}

// Global address of item i of a group (n >= 4), or null past the end.
__device__ __forceinline__ const uint4* item_src(const Mfma32Params& P, const GroupInfo& gi, uint32_t i) {
  const uint32_t lper = P.log2n - 1, quarter = P.n >> 2;
  const uint32_t s = i >> lper, j = i & ((1u << lper) - 1);
  if (s >= gi.nslots) return nullptr;
  const uint64_t gp = slot_gp(gi, s);
  if (j < quarter) return (const uint4*)(P.a + gp * P.n) + j;
  return (const uint4*)(P.b + b_product(P, gp, slot_li(gi, s)) * P.n) + (j - quarter);
}

// Word group a[4j .. 4j+3] into the reversed ext planes at abase: dword
// (E+1)/4 - 1 - j, byte k holding ext[4j + 3 - k], and its negated copy n/4
// dwords further when that lands inside the window.
// kWin: the plane holds a K window (E below n - 1), so the positive copy may fall
// outside it too (dw "below zero" wraps to a large unsigned value and is skipped).
template <int L, bool kWin = false>
__device__ __forceinline__ void stage_a_item(const Mfma32Params& P, uint8_t* abase, uint32_t j, uint4 x,
                                             const ModQ32& m, uint32_t E) {
  const uint32_t q = m.q, thr = m.thr, quarter = P.n >> 2;
  const uint32_t xr[4] = {reduce_u32(x.w, m), reduce_u32(x.z, m), reduce_u32(x.y, m), reduce_u32(x.x, m)};
  uint32_t w[4], nw[4];
  digits_pm32<L>(xr, q, thr, w, nw);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (P.cyclic) nw[k] = w[k];
  const uint32_t dw = ((E + 1) >> 2) - 1 - j;
  if (!kWin || dw < (P.a_plane >> 2)) transpose_store<L>(abase, P.a_plane, dw * 4, w);
  const uint32_t dwn = dw + quarter;
  if (dwn < (P.a_plane >> 2)) transpose_store<L>(abase, P.a_plane, dwn * 4, nw);
}
template <int L>
__device__ __forceinline__ void stage_a_item(const Mfma32Params& P, uint8_t* abase, uint32_t j, uint4 x,
                                             const ModQ32& m) {
  stage_a_item<L, false>(P, abase, j, x, m, P.E);
}

// Word group e of b (row vs = e / (t/4), words 4wd..) into the staged B rows at
// bbase: row vs (+) and row vs - r (-), relative to v_lo, where they are staged.
template <int L>
__device__ __forceinline__ void stage_b_item(const Mfma32Params& P, uint8_t* bbase, int v_lo, uint32_t e, uint4 x,
                                             const ModQ32& m) {
  const uint32_t q = m.q, thr = m.thr;
  const uint32_t xr[4] = {reduce_u32(x.x, m), reduce_u32(x.y, m), reduce_u32(x.z, m), reduce_u32(x.w, m)};
  const int vs = (int)(e >> (P.log2t - 2)), wd = (int)(e & ((P.t >> 2) - 1));
  uint32_t w[4], nw[4];
  digits_pm32<L>(xr, q, thr, w, nw);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (P.cyclic) nw[k] = w[k];
  const int rp = vs - v_lo, rn = vs - (int)P.r - v_lo;
  if (rp >= 0 && rp < (int)P.b_rows) transpose_store<L>(bbase, P.b_plane, rp * P.b_rowstride + wd * 4, w);
  if (rn >= 0 && rn < (int)P.b_rows) transpose_store<L>(bbase, P.b_plane, rn * P.b_rowstride + wd * 4, nw);
}

template <int L>
__device__ __forceinline__ void item_store(const Mfma32Params& P, const GroupInfo& gi, uint8_t* smem, uint32_t i,
                                           uint4 x) {
  const uint32_t lper = P.log2n - 1, quarter = P.n >> 2;
  const uint32_t s = i >> lper, j = i & ((1u << lper) - 1);
  const ModQ32& m = P.mods[slot_li(gi, s)];
  uint8_t* slot = smem + s * P.slot_bytes;
  if (j < quarter) stage_a_item<L>(P, slot, j, x, m);
  else stage_b_item<L>(P, slot + L * P.a_plane, gi.v_lo, j - quarter, x, m);
}

// Parts of the staged B rows that no item writes but valid outputs read: bytes
// w in [t, rowlen) of rows v < r (only when t < 32).  Rows v >= r feed only
// discarded output columns; they are cleared too so LDS content is deterministic.
template <int L, int NT = kThreads>
__device__ __forceinline__ void zero_fill_b(const Mfma32Params& P, uint8_t* bbase, int v_lo) {
  const int row_dw = (int)(P.rowlen >> 2);
  const int tq = (int)(P.t >> 2);
  const int zr0 = max(0, (int)P.r - v_lo);  // first row with v >= r
  {
    if (tq < row_dw) {
      const int pad = row_dw - tq;
      const int cnt = zr0 < (int)P.b_rows ? zr0 * pad : (int)P.b_rows * pad;
      for (int e = threadIdx.x; e < cnt; e += NT) {
        const int row = e / pad, wd = tq + e % pad;
#pragma unroll
        for (int i = 0; i < L; ++i) *(uint32_t*)(bbase + i * P.b_plane + row * P.b_rowstride + wd * 4) = 0u;
      }
    }
    const int nz = ((int)P.b_rows - zr0) * row_dw;
    for (int e = threadIdx.x; e < nz; e += NT) {
      const int row = zr0 + e / row_dw, wd = e % row_dw;
#pragma unroll
      for (int i = 0; i < L; ++i) *(uint32_t*)(bbase + i * P.b_plane + row * P.b_rowstride + wd * 4) = 0u;
    }
  }
}
template <int L, int NT = kThreads>
__device__ __forceinline__ void stage_zero_fill(const Mfma32Params& P, const GroupInfo& gi, uint8_t* smem) {
  for (uint32_t s = 0; s < gi.nslots; ++s) zero_fill_b<L, NT>(P, smem + s * P.slot_bytes + L * P.a_plane, gi.v_lo);
}

// Staging for n >= 256.  The group's items, in order (slot, then a's n/4 word
// groups, then b's), fall into runs of 64 that each lie in one slot and one
// operand (n/4 >= 64), so wave w takes runs w, w + 4, ... and slot, operand and
// modulus are uniform over the wave; lane l handles item 64 run + l.  The slots'
// operand offsets and modulus constants sit in lanes 0..3 and are picked with
// v_readlane, so the per-run selection has no branches.  A pass covers the
// wave's next kPrefetch runs: its loads are issued first (runs_issue), then
// converted into LDS (runs_convert).
struct RunConsts {
  uint32_t lao, lao_hi, lbo, lbo_hi;  // lane s < 4: word offsets of slot s's a and b
  uint32_t lq, lthr, lm32;            // lane s < 4: slot s's modulus constants
};

__device__ __forceinline__ RunConsts run_consts(const Mfma32Params& P, const GroupInfo& gi) {
  RunConsts rc;
  uint64_t ao[4], bo[4];
  uint32_t mq[4], mthr[4], mm32[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    ao[s] = gi.gp[s] * P.n;
    bo[s] = b_product(P, gi.gp[s], gi.li[s]) * P.n;
    const ModQ32& m = P.mods[gi.li[s]];
    mq[s] = m.q;
    mthr[s] = m.thr;
    mm32[s] = m.m32;
  }
  const uint32_t ls = threadIdx.x & 3;
  const uint64_t a64 = sel4(ao, ls), b64 = sel4(bo, ls);
  rc.lao = (uint32_t)a64; rc.lao_hi = (uint32_t)(a64 >> 32);
  rc.lbo = (uint32_t)b64; rc.lbo_hi = (uint32_t)(b64 >> 32);
  rc.lq = sel4(mq, ls); rc.lthr = sel4(mthr, ls); rc.lm32 = sel4(mm32, ls);
  return rc;
}

__device__ __forceinline__ uint32_t pick_lane(uint32_t v, uint32_t s) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)s);
}

// Loads of the pass starting at run r0 (r0 = wave + 4 kPrefetch * pass).  Every
// load is issued (a run past the wave's last re-reads the last one), so that the
// conversion can start on the first run while the rest are in flight.
__device__ __forceinline__ void runs_issue(const Mfma32Params& P, const GroupInfo& gi, const RunConsts& rc,
                                           uint32_t r0, uint4 (&pf)[kPrefetch]) {
  const uint32_t log2rps = P.log2n - 7, a_runs = P.n >> 8;  // runs per slot (n/2) / 64, of them a's (n/4) / 64
  const uint32_t nruns = gi.nslots << log2rps, rmask = (1u << log2rps) - 1;
  const uint32_t lane = threadIdx.x & 63, wave = wave_uniform(threadIdx.x >> 6);
  if (wave >= nruns) return;
  const uint32_t last = wave + 4 * ((nruns - 1 - wave) >> 2);  // this wave's last run
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) {
    const uint32_t run = min(r0 + 4 * k, last);
    const uint32_t sl = run >> log2rps, cr = run & rmask;
    const uint32_t* src =
        cr < a_runs ? P.a + (((uint64_t)pick_lane(rc.lao_hi, sl) << 32) | pick_lane(rc.lao, sl)) + cr * 256u
                    : P.b + (((uint64_t)pick_lane(rc.lbo_hi, sl) << 32) | pick_lane(rc.lbo, sl)) + (cr - a_runs) * 256u;
    pf[k] = ((const uint4*)src)[lane];
  }
}

template <int L>
__device__ __forceinline__ void runs_convert(const Mfma32Params& P, const GroupInfo& gi, const RunConsts& rc,
                                             uint8_t* smem, uint32_t r0, const uint4 (&pf)[kPrefetch]) {
  const uint32_t log2rps = P.log2n - 7, a_runs = P.n >> 8;
  const uint32_t nruns = gi.nslots << log2rps, rmask = (1u << log2rps) - 1;
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) {
    const uint32_t run = r0 + 4 * k;
    if (run < nruns) {
      const uint32_t sl = run >> log2rps, cr = run & rmask;
      ModQ32 m{};
      m.q = pick_lane(rc.lq, sl);
      m.thr = pick_lane(rc.lthr, sl);
      m.m32 = pick_lane(rc.lm32, sl);
      uint8_t* slot = smem + sl * P.slot_bytes;
      if (cr < a_runs) stage_a_item<L>(P, slot, cr * 64 + lane, pf[k], m);
      else stage_b_item<L>(P, slot + L * P.a_plane, gi.v_lo, (cr - a_runs) * 64 + lane, pf[k], m);
    }
  }
}

template <int L>
__device__ __forceinline__ void stage_runs(const Mfma32Params& P, const GroupInfo& gi, uint8_t* smem) {
  const uint32_t nruns = gi.nslots << (P.log2n - 7);
  const uint32_t wave = wave_uniform(threadIdx.x >> 6);
  const RunConsts rc = run_consts(P, gi);
  for (uint32_t r0 = wave; r0 < nruns; r0 += 4 * kPrefetch) {
    uint4 pf[kPrefetch];
    runs_issue(P, gi, rc, r0, pf);
    runs_convert<L>(P, gi, rc, smem, r0, pf);
  }
}

// The compute half of a group (after its staging barrier): each wave runs its
// tile's K loop, then the recombination, reduction and stores.
template <int L, bool T4 = true>
__device__ __forceinline__ void resident_compute(const Mfma32Params& P, uint64_t grp, const GroupInfo& gi,
                                                 const uint8_t* smem) {
  const uint64_t total_units = P.nprod << P.log2U;
  const uint32_t U = 1u << P.log2U;
  const uint64_t unit = grp * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (unit >= total_units) return;
  const uint64_t prod = unit >> P.log2U;
  const uint32_t tile = (uint32_t)(unit & (U - 1));
  const int zt = (int)(tile % P.tz), ut = (int)(tile / P.tz);
  const uint32_t sl = (uint32_t)(prod - gi.first);
  const uint8_t* slot = smem + sl * P.slot_bytes;
  v16i acc[2 * L - 1];
  mfma32_tile<L, T4>(P, slot, slot + L * P.a_plane, 32 * zt, 32 * ut, gi.v_lo, acc);
  uint32_t li;
  const uint64_t gprod = global_product(P, prod, &li);
  mfma32_epilogue<L>(P, gprod, P.mods[li], P.rcent[li], 32 * zt, 32 * ut, acc);
}

// One group of four 32x32 tiles: stage the products it touches, then each wave
// runs its tile.  SMALL: n < 4, staged byte by byte.  Ends with every wave
// past its last LDS read only if the caller synchronises afterwards.
template <int L, bool SMALL>
__device__ __forceinline__ void resident_group(const Mfma32Params& P, uint64_t grp, uint8_t* smem) {
  const GroupInfo gi = group_info(P, grp);
  if constexpr (SMALL) {
    for (uint32_t s = 0; s < gi.nslots; ++s)
      mfma32_stage<L>(P, smem + s * P.slot_bytes, slot_gp(gi, s), b_product(P, slot_gp(gi, s), slot_li(gi, s)),
                      P.mods[slot_li(gi, s)], gi.v_lo);
  } else if (P.n >= 256) {
    stage_runs<L>(P, gi, smem);
    stage_zero_fill<L>(P, gi, smem);
  } else {
    // all loads of a pass are issued before any is converted
    const uint32_t nitems = gi.nslots * (P.n >> 1);
    for (uint32_t base = 0; base < nitems; base += kPrefetch * kThreads) {
      uint4 pf[kPrefetch];
#pragma unroll
      for (int k = 0; k < kPrefetch; ++k) {
        const uint32_t i = base + threadIdx.x + k * kThreads;
        const uint4* src = i < nitems ? item_src(P, gi, i) : nullptr;
        pf[k] = src ? *src : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < kPrefetch; ++k) {
        const uint32_t i = base + threadIdx.x + k * kThreads;
        if (i < nitems) item_store<L>(P, gi, smem, i, pf[k]);
      }
    }
    stage_zero_fill<L>(P, gi, smem);
  }
  __syncthreads();
  resident_compute<L, !SMALL>(P, grp, gi, smem);  // SMALL: n < 4, t = n
}

// The K window of one run of a K-split group (one product, t >= 32, so the group's
// tiles cover every z): K-steps [st_lo, st_hi) touch d in [d_lo, d_hi), hence
// ext[d_lo t - t + 1 .. d_hi t - 1], held with E = d_hi t - 1 at reversed position 0,
// and B rows v = u - d for the group's u, from v_lo = u_lo - d_hi + 1 on (the host
// sizes a_plane and b_rows for the widest run).  The staged items are the runs of 64
// word groups (a's, then b's; n >= 256) that hold a byte of the window: up to two
// ranges of a (positive and negated copies) and two of b (rows v and v - r).
struct KWindow {
  uint32_t E;
  int v_lo;
  uint32_t lo[4], cnt[4];  // item-run ranges within the product, in order, disjoint
};

// Range i (a constant after unrolling: no dynamic index, nothing in scratch) of the
// runs holding items [lo, hi) (+ base runs); the ranges come in order of lo, and each
// starts where the previous ones end, so that no run is staged twice.
__device__ __forceinline__ void kwin_range(KWindow& w, int i, int& end, int lo, int hi, int base) {
  int rlo = base + (lo >> 6), rhi = base + ((hi + 63) >> 6);
  if (lo >= hi) rlo = rhi = end;
  rlo = max(rlo, end);
  rhi = max(rhi, rlo);
  w.lo[i] = (uint32_t)rlo;
  w.cnt[i] = (uint32_t)(rhi - rlo);
  end = rhi;
}

__device__ __forceinline__ KWindow k_window(const Mfma32Params& P, const GroupInfo& gi, int st_lo, int st_hi) {
  const int t = (int)P.t, r = (int)P.r, q4 = (int)(P.n >> 2);
  const int d_lo = st_lo >> P.log2spd, d_hi = ((st_hi - 1) >> P.log2spd) + 1;
  KWindow w;
  w.E = (uint32_t)(d_hi * t - 1);
  w.v_lo = gi.v_lo + r - d_hi;  // group_info's v_lo is u_lo - (r - 1)
  int end = 0;
  const int e4 = (int)((w.E + 1) >> 2), A4 = (int)(P.a_plane >> 2);
  kwin_range(w, 0, end, max(0, e4 - A4), min(q4, e4), 0);            // positive copies: dword e4 - 1 - j
  kwin_range(w, 1, end, max(0, e4 + q4 - A4), min(q4, e4 + q4), 0);  // negated copies, n/4 dwords further
  const int rw = t >> 2, a_runs = (int)(P.n >> 8);                    // word groups per b row
  kwin_range(w, 2, end, max(0, w.v_lo) * rw, min(r, w.v_lo + (int)P.b_rows) * rw, a_runs);
  kwin_range(w, 3, end, max(0, w.v_lo + r) * rw, min(r, w.v_lo + r + (int)P.b_rows) * rw, a_runs);
  return w;
}

// A window of n <= 8192 spans at most 64 runs, one pass of kWinPrefetch loads per
// thread (a pass is a load latency exposed: 33 runs in two passes of eight took 1.5x
// the time of 32 runs in one).
constexpr int kWinPrefetch = 16;

template <int L>
__device__ __forceinline__ void stage_window(const Mfma32Params& P, const GroupInfo& gi, uint8_t* smem,
                                             const KWindow& w) {
  const uint32_t a_runs = P.n >> 8;
  const uint32_t lane = threadIdx.x & 63, wave = wave_uniform(threadIdx.x >> 6);
  const uint32_t total = w.cnt[0] + w.cnt[1] + w.cnt[2] + w.cnt[3];
  if (wave >= total) return;
  const uint32_t last = wave + 4 * ((total - 1 - wave) >> 2);  // this wave's last run
  const ModQ32& m = P.mods[gi.li[0]];
  const uint32_t* A = P.a + gi.gp[0] * P.n;
  const uint32_t* B = P.b + b_product(P, gi.gp[0], gi.li[0]) * P.n;
  auto run_of = [&](uint32_t v) {  // v-th staged run -> run within the product
    if (v < w.cnt[0]) return w.lo[0] + v;
    v -= w.cnt[0];
    if (v < w.cnt[1]) return w.lo[1] + v;
    v -= w.cnt[1];
    if (v < w.cnt[2]) return w.lo[2] + v;
    return w.lo[3] + (v - w.cnt[2]);
  };
  for (uint32_t v0 = wave; v0 < total; v0 += 4 * kWinPrefetch) {
    uint4 pf[kWinPrefetch];
#pragma unroll
    for (int k = 0; k < kWinPrefetch; ++k) {  // every load issued (past the last run: the last again)
      const uint32_t cr = run_of(min(v0 + 4 * k, last));
      const uint32_t* src = cr < a_runs ? A + cr * 256u : B + (cr - a_runs) * 256u;
      pf[k] = ((const uint4*)src)[lane];
    }
#pragma unroll
    for (int k = 0; k < kWinPrefetch; ++k) {
      if (v0 + 4 * k < total) {
        const uint32_t cr = run_of(v0 + 4 * k);
        if (cr < a_runs) stage_a_item<L, true>(P, smem, cr * 64 + lane, pf[k], m, w.E);
        else stage_b_item<L>(P, smem + L * P.a_plane, w.v_lo, (cr - a_runs) * 64 + lane, pf[k], m);
      }
    }
  }
}

// One run of a K-split group (one product, U >= 4: every wave has a tile, n >= 256):
// K-steps [part, part + 1) * steps / kparts of all four tiles, from the run's K
// window only; residues stored in the run's copy of c.
template <int L>
__device__ __forceinline__ void resident_group_split(const Mfma32Params& P, uint32_t item, uint8_t* smem) {
  const uint32_t grp = item / P.kparts, part = item - grp * P.kparts;
  const uint32_t U = 1u << P.log2U;
  const GroupInfo gi = group_info(P, grp);
  const int steps = (int)(P.r << P.log2spd);
  const int st_lo = (int)(part * (uint32_t)steps / P.kparts), st_hi = (int)((part + 1) * (uint32_t)steps / P.kparts);
  const KWindow win = k_window(P, gi, st_lo, st_hi);
  stage_window<L>(P, gi, smem, win);
  zero_fill_b<L>(P, smem + L * P.a_plane, win.v_lo);
  __syncthreads();
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t unit = (uint64_t)grp * 4 + wave;
  const uint64_t prod = unit >> P.log2U;
  const uint32_t tile = (uint32_t)(unit & (U - 1));
  const int zt = (int)(tile % P.tz), ut = (int)(tile / P.tz);
  v16i acc[2 * L - 1];
  mfma32_tile<L>(P, smem, smem + L * P.a_plane, 32 * zt, 32 * ut, win.v_lo, acc, st_lo, st_hi, (int)win.E);
  uint32_t li;
  const uint64_t gprod = global_product(P, prod, &li);
  uint32_t out[16];
  mfma32_reduce<L>(P, P.mods[li], P.rcent[li], acc, out);
  Mfma32Params Q = P;  // the run's copy of c
  Q.c = P.part_ws + (uint64_t)part * P.nprod * P.n;
  mfma32_store(Q, gprod, 32 * zt, 32 * ut, out);
}

// c = sum of the kparts runs' residues mod q, word by word, for every K-split job of
// a plan in one launch: segment k owns blocks [first_block, next first_block).
struct SplitSeg {
  const uint32_t* ws;  // [kparts][words]
  uint32_t* c;
  uint64_t words;      // a multiple of 4
  uint32_t kparts;
  uint32_t first_block;
  ModQ32 m;
};
__global__ __launch_bounds__(256) void split_sum_kernel(const SplitSeg* __restrict__ segs, uint32_t nseg) {
  uint32_t k = 0;
  while (k + 1 < nseg && segs[k + 1].first_block <= blockIdx.x) ++k;  // uniform: a few segments
  const SplitSeg& sg = segs[k];
  const uint64_t i = ((uint64_t)(blockIdx.x - sg.first_block) * 256 + threadIdx.x) * 4;
  if (i >= sg.words) return;
  uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (uint32_t p = 0; p < sg.kparts; ++p) {
    const uint4 x = *(const uint4*)(sg.ws + (uint64_t)p * sg.words + i);
    s0 += x.x; s1 += x.y; s2 += x.z; s3 += x.w;
  }
  *(uint4*)(sg.c + i) =
      make_uint4(reduce_u64(s0, sg.m), reduce_u64(s1, sg.m), reduce_u64(s2, sg.m), reduce_u64(s3, sg.m));
}

// One group of four 32x32 tiles per workgroup.
template <int L, bool SMALL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void mfma32_group_kernel(const Mfma32Params P) {
  extern __shared__ __align__(16) uint8_t smem[];
  resident_group<L, SMALL>(P, blockIdx.x, smem);
}

// ---------------------------------------------------------------------------
// One b shared by a whole batch (paper Sec. 4, fine-tuning (i): keep one operand
// fixed and reuse what was prepared for it).  A workgroup takes a chunk of
// consecutive groups of one modulus channel and one tile position; b's digit
// rows are staged once per chunk, each group then stages only a.  LDS layout:
// [L planes of B rows][slots x L planes of A].
// ---------------------------------------------------------------------------
struct SharedChunks {
  uint64_t batch;             // products per channel
  uint32_t npos;              // tile positions per product: max(1, U / 4)
  uint32_t groups_per_class;  // U >= 4: batch; else ceil(batch / slots)
  uint32_t chunk;             // groups per workgroup
  uint32_t chunks_per_class;  // ceil(groups_per_class / chunk)
};

template <int L>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void mfma32_shared_kernel(const Mfma32Params P, const SharedChunks C) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t cls = blockIdx.x / C.chunks_per_class;
  const uint32_t part = blockIdx.x - cls * C.chunks_per_class;
  const uint32_t l = cls / C.npos, pos = cls - l * C.npos;
  const uint32_t U = 1u << P.log2U;
  const int ut_lo = U >= 4 ? (int)((pos * 4) / P.tz) : 0;
  const int v_lo = 32 * ut_lo - ((int)P.r - 1);
  const ModQ32& m = P.mods[l];
  uint8_t* bbase = smem;
  uint8_t* abase = smem + L * P.b_plane;
  const uint32_t a_slot = L * P.a_plane;
  const uint32_t quarter = P.n >> 2;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // b's rows for this channel and tile position, once per chunk
  {
    const uint4* src = (const uint4*)(P.b + (uint64_t)(P.l0 + l) * P.n);
    for (uint32_t base = 0; base < quarter; base += kPrefetch * kThreads) {
      uint4 pf[kPrefetch];
#pragma unroll
      for (int k = 0; k < kPrefetch; ++k) {
        const uint32_t e = base + threadIdx.x + k * kThreads;
        pf[k] = e < quarter ? src[e] : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < kPrefetch; ++k) {
        const uint32_t e = base + threadIdx.x + k * kThreads;
        if (e < quarter) stage_b_item<L>(P, bbase, v_lo, e, pf[k], m);
      }
    }
    zero_fill_b<L>(P, bbase, v_lo);
  }

  const uint32_t g0 = part * C.chunk;
  const uint32_t g1 = min(g0 + C.chunk, C.groups_per_class);
  for (uint32_t g = g0; g < g1; ++g) {
    // batch indices of this group's products and how many exist
    const uint64_t i0 = U >= 4 ? (uint64_t)g : (uint64_t)g * P.slots;
    const uint32_t nsl = U >= 4 ? 1u : (uint32_t)min((uint64_t)P.slots, C.batch - i0);
    const uint32_t nitems = nsl * quarter;  // a's word groups
    for (uint32_t base = 0; base < nitems; base += kPrefetch * kThreads) {
      uint4 pf[kPrefetch];
#pragma unroll
      for (int k = 0; k < kPrefetch; ++k) {
        const uint32_t i = base + threadIdx.x + k * kThreads;
        pf[k] = make_uint4(0, 0, 0, 0);
        if (i < nitems) {
          const uint32_t sl = i >> (P.log2n - 2), j = i & (quarter - 1);
          uint32_t li;
          const uint64_t gp = global_product(P, (i0 + sl) * P.lc + l, &li);
          pf[k] = ((const uint4*)(P.a + gp * P.n))[j];
        }
      }
#pragma unroll
      for (int k = 0; k < kPrefetch; ++k) {
        const uint32_t i = base + threadIdx.x + k * kThreads;
        if (i < nitems) {
          const uint32_t sl = i >> (P.log2n - 2), j = i & (quarter - 1);
          stage_a_item<L>(P, abase + sl * a_slot, j, pf[k], m);
        }
      }
    }
    __syncthreads();
    // wave -> (slot, tile)
    const uint32_t sl = U >= 4 ? 0u : wave >> P.log2U;
    const uint32_t tile = U >= 4 ? pos * 4 + wave : (wave & (U - 1));
    if (sl < nsl) {
      const int zt = (int)(tile % P.tz), ut = (int)(tile / P.tz);
      v16i acc[2 * L - 1];
      mfma32_tile<L>(P, abase + sl * a_slot, bbase, 32 * zt, 32 * ut, v_lo, acc);
      uint32_t li;
      const uint64_t gp = global_product(P, (i0 + sl) * P.lc + l, &li);
      mfma32_epilogue<L>(P, gp, m, P.rcent[l], 32 * zt, 32 * ut, acc);
    }
    __syncthreads();  // a's planes are restaged for the next group
  }
}

}  // namespace pm
