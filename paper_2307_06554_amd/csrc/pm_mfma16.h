// Split-limb int8 MFMA kernel for small degrees (64 <= n <= 512) on 16x16 output
// tiles, v_mfma_i32_16x16x64_i8.
//
// The recast is the resident kernel's (Eq. (3) Toeplitz tiles, Sec. 2.5 block
// split; see pm_mfma32.h) with the Toeplitz side t = 16: n = 16 r, output
// index j = 16 u + z (z < 16), input index k = 16 d + w, and
//   C[z][u] = sum_(d,w) ext[16 d + z - w] s(u,d) b[((u - d) mod r) 16 + w].
// One 16x16 output tile covers z < 16 and 16 values of u, so a product is
// ceil(r / 16) tiles and, from n = 256 on, no MFMA lane computes an output that
// is thrown away (a 32x32 tile at n = 256 leaves three quarters of its columns
// empty).  A K-step of 64 spans four values of d: lane group g = lane / 16 takes
// d = 4 st + g, w = 0..15, i.e. the reversed 16-byte run of ext at
// S = E - (16 d + z) and the 16 bytes of B row u - d.
//
// A workgroup stages `slots` consecutive products (up to 16) and its four waves
// take the (product, tile) units in turn; the digit planes, the limb split, the
// shift classes and the epilogue are those of the resident kernel.  SHB (one b
// for every product of the launch, Sec. 4 fine-tuning (i)): b's digit rows are
// staged once per workgroup, ahead of the slots' A planes.
#pragma once
#include "pm_mfma32.h"

namespace pm {

typedef int v4i_acc __attribute__((ext_vector_type(4)));

constexpr int kSlots16 = 16;  // products staged per workgroup, at most

// Per-slot table in LDS: the slot's global product, its b product and modulus index.
struct Slot16 {
  uint32_t a_lo, a_hi;  // word offset of a (and c) of the product
  uint32_t b_lo, b_hi;  // word offset of b
  uint32_t li;          // modulus index
  uint32_t pad[3];
};

// One K-step of one tile: L A runs (five dwords, any byte offset) and L B rows.
template <int L>
__device__ __forceinline__ void mfma16_step(v4i_acc (&acc)[2 * L - 1], const uint8_t* aplane, uint32_t a_plane,
                                            int S, const uint8_t* bplane, uint32_t b_plane, int boff) {
  uint32_t x[L][5];
  v4i a[L], b[L];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint32_t* p = (const uint32_t*)(aplane + i * a_plane) + (S >> 2);
#pragma unroll
    for (int k = 0; k < 5; ++k) x[i][k] = p[k];
    b[i] = *(const v4i*)(bplane + i * b_plane + boff);
  }
  const uint32_t sh = (uint32_t)(S & 3);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    a[i][0] = (int)__builtin_amdgcn_alignbyte(x[i][1], x[i][0], sh);
    a[i][1] = (int)__builtin_amdgcn_alignbyte(x[i][2], x[i][1], sh);
    a[i][2] = (int)__builtin_amdgcn_alignbyte(x[i][3], x[i][2], sh);
    a[i][3] = (int)__builtin_amdgcn_alignbyte(x[i][4], x[i][3], sh);
  }
#pragma unroll
  for (int j = 0; j < L; ++j)
#pragma unroll
    for (int i = 0; i < L; ++i)
      acc[i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i + j], 0, 0, 0);
}

// Recombination c = sum_s T_s 2^(8s) mod q of the 4 outputs a lane holds (as the
// resident kernel's, four values instead of sixteen).
template <int L>
__device__ __forceinline__ void mfma16_reduce(const Mfma32Params& P, const ModQ32& m, const int32_t* rcp,
                                              const v4i_acc (&acc)[2 * L - 1], uint32_t (&out)[4]) {
  int32_t rc[2 * L - 1];
#pragma unroll
  for (int s = 0; s < 2 * L - 1; ++s) rc[s] = rcp[s];
  if (P.fast_epilogue) {
    if (m.q < 0x80000000u) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint64_t x = m.lift;
#pragma unroll
        for (int s = 0; s < 2 * L - 1; ++s) x += (uint64_t)((int64_t)acc[s][e] * (int64_t)rc[s]);
        out[e] = reduce_u64_q31(x, m.mu, m.q);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t x = 0;
#pragma unroll
        for (int s = 0; s < 2 * L - 1; ++s) x += (int64_t)acc[s][e] * (int64_t)rc[s];
        out[e] = reduce_i64(x, m);
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint32_t v = reduce_i64((int64_t)acc[2 * L - 2][e], m);
#pragma unroll
      for (int s = 2 * L - 3; s >= 0; --s) v = reduce_i64((int64_t)v * 256 + (int64_t)acc[s][e], m);
      out[e] = v;
    }
  }
}

// Stage the group's slots: word group j of a (j < n/4) and of b (n/4 <= j < n/2)
// of every slot, kPrefetch loads per thread in flight before any is converted.
// SHB: items [0, nslots n/4) are the slots' a word groups, the last n/4 b's
// (from slot 0's product), written once to the B planes at bshared; slot s's A
// planes at smem + s * L * a_plane.
template <int L, bool SHB = false>
__device__ __forceinline__ void stage16(const Mfma32Params& P, const Slot16* tab, uint32_t nslots, uint8_t* smem,
                                        int v_lo, uint8_t* bshared = nullptr) {
  const uint32_t half = P.n >> 1, quarter = P.n >> 2, log2half = P.log2n - 1, log2q = P.log2n - 2;
  const uint32_t nitems = SHB ? (nslots + 1) << log2q : nslots << log2half;
  for (uint32_t base = 0; base < nitems; base += kPrefetch * kThreads) {
    uint4 pf[kPrefetch];
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
      const uint32_t i = base + threadIdx.x + k * kThreads;
      pf[k] = make_uint4(0, 0, 0, 0);
      if (i < nitems) {
        if (SHB) {
          const uint32_t s = i >> log2q, j = i & (quarter - 1);
          const Slot16& sl = tab[s < nslots ? s : 0];
          pf[k] = s < nslots ? ((const uint4*)(P.a + (((uint64_t)sl.a_hi << 32) | sl.a_lo)))[j]
                             : ((const uint4*)(P.b + (((uint64_t)sl.b_hi << 32) | sl.b_lo)))[j];
        } else {
          const Slot16& sl = tab[i >> log2half];
          const uint32_t j = i & (half - 1);
          pf[k] = j < quarter ? ((const uint4*)(P.a + (((uint64_t)sl.a_hi << 32) | sl.a_lo)))[j]
                              : ((const uint4*)(P.b + (((uint64_t)sl.b_hi << 32) | sl.b_lo)))[j - quarter];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
      const uint32_t i = base + threadIdx.x + k * kThreads;
      if (i < nitems) {
        if (SHB) {
          const uint32_t s = i >> log2q, j = i & (quarter - 1);
          const ModQ32& m = P.mods[tab[s < nslots ? s : 0].li];
          if (s < nslots) stage_a_item<L>(P, smem + s * L * P.a_plane, j, pf[k], m);
          else stage_b_item<L>(P, bshared, v_lo, j, pf[k], m);
        } else {
          const uint32_t s = i >> log2half, j = i & (half - 1);
          const ModQ32& m = P.mods[tab[s].li];
          uint8_t* slot = smem + s * P.slot_bytes;
          if (j < quarter) stage_a_item<L>(P, slot, j, pf[k], m);
          else stage_b_item<L>(P, slot + L * P.a_plane, v_lo, j - quarter, pf[k], m);
        }
      }
    }
  }
  // rows v >= r of the last tile (n < 256 only) feed discarded columns: cleared so
  // that LDS content is deterministic
  const int row_dw = (int)(P.rowlen >> 2);
  const int zr0 = (int)P.r - v_lo;
  const int nz = ((int)P.b_rows - zr0) * row_dw;
  for (uint32_t s = 0; s < (SHB ? 1u : nslots); ++s) {
    uint8_t* bbase = SHB ? bshared : smem + s * P.slot_bytes + L * P.a_plane;
    for (int e = threadIdx.x; e < nz; e += kThreads) {
      const int row = zr0 + e / row_dw, wd = e % row_dw;
#pragma unroll
      for (int i = 0; i < L; ++i) *(uint32_t*)(bbase + i * P.b_plane + row * P.b_rowstride + wd * 4) = 0u;
    }
  }
}

// One group of P.slots consecutive products (the last group may hold fewer).
template <int L, bool SHB = false>
__device__ __forceinline__ void small_group(const Mfma32Params& P, uint64_t grp, uint8_t* smem, Slot16* tab,
                                            uint8_t* bshared = nullptr) {
  const uint64_t first = grp * P.slots;
  const uint64_t left = P.nprod - first;
  const uint32_t nslots = left < P.slots ? (uint32_t)left : P.slots;
  if (threadIdx.x < nslots) {
    uint32_t li;
    const uint64_t gp = global_product(P, first + threadIdx.x, &li);
    const uint64_t ao = gp * P.n, bo = b_product(P, gp, li) * P.n;
    tab[threadIdx.x] = Slot16{(uint32_t)ao, (uint32_t)(ao >> 32), (uint32_t)bo, (uint32_t)(bo >> 32), li, {0, 0, 0}};
  }
  __syncthreads();
  const int v_lo = -((int)P.r - 1);
  stage16<L, SHB>(P, tab, nslots, smem, v_lo, bshared);
  __syncthreads();

  const uint32_t lane = threadIdx.x & 63, wave = wave_uniform(threadIdx.x >> 6);
  const int zl = (int)(lane & 15), g = (int)(lane >> 4);
  const uint32_t U = 1u << P.log2U;
  const uint32_t units = nslots << P.log2U;
  const int steps = (int)(P.n >> 6);
  for (uint32_t unit = wave; unit < units; unit += 4) {
    const uint32_t s = unit >> P.log2U, tile = unit & (U - 1);
    const int u0 = 16 * (int)tile;
    const uint8_t* slot = smem + s * (SHB ? L * P.a_plane : P.slot_bytes);
    const uint8_t* bplane = SHB ? bshared : slot + L * P.a_plane;
    // lane (zl, g), K-step st: d = 4 st + g; A run at S = E - (16 d + zl), B row u0 + zl - d
    const int S0 = (int)P.E - 16 * g - zl;
    const int B0 = (u0 + zl - g - v_lo) * (int)P.b_rowstride;
    v4i_acc acc[2 * L - 1];
#pragma unroll
    for (int c = 0; c < 2 * L - 1; ++c) acc[c] = v4i_acc{0, 0, 0, 0};
    for (int st = 0; st < steps; ++st)
      mfma16_step<L>(acc, slot, P.a_plane, S0 - 64 * st, bplane, P.b_plane, B0 - 4 * st * (int)P.b_rowstride);
    const Slot16 sl = tab[s];
    uint32_t out[4];
    mfma16_reduce<L>(P, P.mods[sl.li], P.rcent[sl.li], acc, out);
    // lane holds z = 4 g + e of column u = u0 + zl: four consecutive words of c
    const int u = u0 + zl;
    if (u < (int)P.r) {
      uint32_t* C = P.c + (((uint64_t)sl.a_hi << 32) | sl.a_lo);
      *(uint4*)(C + (size_t)u * 16 + 4 * g) = make_uint4(out[0], out[1], out[2], out[3]);
    }
  }
}

// Dynamic LDS: the slots' digit planes, then the slot table.  SHB: the slots'
// A planes, the B planes of the shared b, then the slot table.
template <int L, bool SHB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void mfma16_group_kernel(const Mfma32Params P) {
  extern __shared__ __align__(16) uint8_t smem[];
  if constexpr (SHB) {
    uint8_t* bshared = smem + P.slots * L * P.a_plane;
    small_group<L, true>(P, blockIdx.x, smem, (Slot16*)(bshared + L * P.b_plane), bshared);
  } else {
    small_group<L>(P, blockIdx.x, smem, (Slot16*)(smem + P.slots * P.slot_bytes));
  }
}

}  // namespace pm
