// C-ABI of the GPU library: argument checks, launch geometry, dispatch, plans.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

#include "../../include/polymul.h"
#include "pm_common.h"
#include "pm_mfma32.h"
#include "pm_mfma16.h"
#include "pm_plain.h"
#include "pm_stream.h"
#include "pm_grouped.h"
#include "pm_karatsuba.h"
#include "pm_crt.h"
#include "pm_wide_host.h"

using namespace pm;

namespace {

// Dynamic LDS limit per workgroup: the 160 KiB of a CU less room for static LDS.
constexpr uint32_t kMaxLds = 160 * 1024 - 256;

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
int ilog2(uint64_t x) {
  int l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

// [p, p + bytes) intersects [q, q + bytes2)?
bool overlaps(const void* p, uint64_t bytes, const void* q, uint64_t bytes2) {
  uintptr_t a0 = (uintptr_t)p, a1 = a0 + bytes, b0 = (uintptr_t)q, b1 = b0 + bytes2;
  return a0 < b1 && b0 < a1;
}

// Common checks for [batch][n] word arrays; *bytes gets the size of one array.
polymul_status check_arrays(const void* a, const void* b, const void* c, uint64_t n, uint64_t batch,
                            uint64_t words_per_item, uint32_t elem, uint64_t* bytes) {
  if (!is_pow2(n) || n > 65536) return POLYMUL_EINVAL;
  if (batch == 0) { *bytes = 0; return POLYMUL_OK; }
  if (!a || !b || !c) return POLYMUL_EINVAL;
  // word groups are moved with 16-byte loads and stores
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) return POLYMUL_EINVAL;
  unsigned __int128 total = (unsigned __int128)batch * words_per_item * n * elem;
  if (total >> 62) return POLYMUL_EINVAL;
  *bytes = (uint64_t)total;
  if (overlaps(c, *bytes, a, *bytes) || overlaps(c, *bytes, b, *bytes)) return POLYMUL_EALIAS;
  return POLYMUL_OK;
}

// Checks for the shared-operand layout: a and c are [batch][channels][n], b is [channels][n].
polymul_status check_shared(const void* a, const void* b, const void* c, uint64_t n, uint64_t batch,
                            uint64_t channels, uint32_t elem) {
  if (!is_pow2(n) || n > 65536) return POLYMUL_EINVAL;
  if (batch == 0) return POLYMUL_OK;
  if (!a || !b || !c) return POLYMUL_EINVAL;
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) return POLYMUL_EINVAL;
  const unsigned __int128 big = (unsigned __int128)batch * channels * n * elem;
  if (big >> 62) return POLYMUL_EINVAL;
  const uint64_t bytes = (uint64_t)big, bbytes = channels * n * elem;
  if (overlaps(c, bytes, a, bytes) || overlaps(c, bytes, b, bbytes)) return POLYMUL_EALIAS;
  return POLYMUL_OK;
}

// POLYMUL_LOG=1 in the environment prints failing HIP calls to stderr.
bool log_enabled() {
  static const bool on = [] {
    const char* v = getenv("POLYMUL_LOG");
    return v && *v && *v != '0';
  }();
  return on;
}

polymul_status hip_fail(hipError_t e, const char* what) {
  if (log_enabled()) fprintf(stderr, "polymul: %s failed: %s\n", what, hipGetErrorString(e));
  return POLYMUL_EDEVICE;
}

polymul_status launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? POLYMUL_OK : hip_fail(e, "kernel launch");
}

// Compute units of the current device (cached per device).
uint32_t device_cus() {
  static std::mutex mu;
  static int cached_dev = -1;
  static uint32_t cached = 256;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return cached;
  std::lock_guard<std::mutex> g(mu);
  if (dev != cached_dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) {
      cached = (uint32_t)prop.multiProcessorCount;
      cached_dev = dev;
    }
  }
  return cached;
}

// ------------------------------------------------------------- tile table
// Toeplitz tile side t for the resident 32-bit path, per (log2 n, L); 0 = built-in choice.
// Written by polymul_tune_set (the autotuner), read at every launch.
std::atomic<uint32_t> g_tile[17][5];

uint32_t default_tile(uint32_t n) {
  if (n <= 32) return n;
  if (n <= 512) return 16;  // the 16x16-tile kernel
  if (n <= 1024) return 32;
  return 64;
}

uint32_t tile_for(uint32_t n, int L) {
  const uint32_t t = g_tile[ilog2(n)][L].load(std::memory_order_relaxed);
  return t ? t : default_tile(n);
}

// Karatsuba depth per (log2 n, log2 of the products in the call): 0 = direct route,
// 1..3 = levels; 0xFF = not tuned (the built-in choice).
std::atomic<uint32_t> g_kara_depth[17][41];
std::atomic<uint32_t> g_kara64_depth[17][41];
constexpr uint32_t kNotTuned = 0xFF;
struct KaraTableInit {
  KaraTableInit() {
    for (auto& row : g_kara_depth)
      for (auto& v : row) v.store(kNotTuned);
    for (auto& row : g_kara64_depth)
      for (auto& v : row) v.store(kNotTuned);
  }
} g_kara_table_init;

int ilog2_floor(uint64_t x) {
  int l = 0;
  while (l < 40 && (2ull << l) <= x) ++l;
  return l;
}

// Depth for a call of `products` products of degree bound n: the table's, else the
// built-in choice (two levels from n = 1024 on, one at 512 for 32-bit words; for
// 64-bit words three from n = 8192 on, else one), never below n / 2^depth = 4.
uint32_t kara_depth_for(uint64_t n, uint64_t products, bool wide) {
  uint32_t d = (wide ? g_kara64_depth : g_kara_depth)[ilog2(n)][ilog2_floor(products)].load(std::memory_order_relaxed);
  if (d == kNotTuned) d = wide ? (n >= 8192 ? 3 : 1) : (n >= 1024 ? 2 : n >= 512 ? 1 : 0);
  while (d > 0 && (n >> d) < 4) --d;
  return d;
}

// Grouped plans take the tuned side too (16: the 16x16-tile kernel).
uint32_t plan_tile(uint32_t n, int L) { return tile_for(n, L); }

// Products per item of a plan's 16x16-tile groups: up to 16, within half a CU's LDS.
uint32_t plan_small_slots(uint32_t slot_bytes) {
  uint32_t slots = kSlots16;
  while (slots > 1 && (uint64_t)slots * slot_bytes + kSlots16 * sizeof(Slot16) > kMaxLds / 2) slots /= 2;
  return slots;
}

// Valid tile sides for the resident path: n itself when n <= 32, else a power of two in [32, min(n, 128)].
// t = 16 for 64 <= n <= 512 selects the 16x16-tile kernel (v_mfma_i32_16x16x64_i8).
bool tile_ok(uint32_t n, uint32_t t) {
  if (t == 16 && n >= 64 && n <= 512) return true;
  if (n <= 32) return t == n;
  return is_pow2(t) && t >= 32 && t <= 128 && t <= n;
}

// ----------------------------------------------------------- MFMA, 32-bit q
struct Geometry32 {
  uint32_t t, r, spd, rowlen, tz, tu, U, slots, a_plane, b_rows, b_rowstride, b_plane, E;
};

// Degree split n = t * r (Sec. 2.5): t is the Toeplitz tile side.
Geometry32 geometry32(uint32_t n, uint32_t t) {
  Geometry32 g{};
  if (t == 16 && n >= 64) {
    // 16x16 tiles: z < 16, u in tiles of 16, K-steps of 64 (four d values);
    // reversed ext positions 0 .. n + 15 and the 5-dword over-read, B rows
    // v in [-(r - 1), 16 tu - 1] of 16 bytes
    g.t = 16;
    g.r = n / 16;
    g.spd = 1;
    g.rowlen = 16;
    g.tz = 1;
    g.tu = (g.r + 15) / 16;
    g.U = g.tu;
    g.slots = kSlots16;
    g.E = n - 1;
    g.a_plane = (g.E + 24 + 15) & ~15u;
    g.b_rows = 16 * g.tu + g.r - 1;
    g.b_rowstride = 16;
    g.b_plane = g.b_rows * 16;
    return g;
  }
  g.t = t;
  g.r = n / t;
  g.spd = g.t >= 32 ? g.t / 32 : 1;
  g.rowlen = 32 * g.spd;
  g.tz = (g.t + 31) / 32;
  g.tu = (g.r + 31) / 32;
  g.U = g.tz * g.tu;
  g.slots = g.U >= 4 ? 1 : 4 / g.U;
  g.E = (g.r - 1) * g.t + 32 * g.tz - 1;
  g.a_plane = (g.E + g.rowlen + 4 + 15) & ~15u;
  uint32_t utiles = g.U >= 4 ? (4 / g.tz ? 4 / g.tz : 1) : g.tu;
  g.b_rows = 32 * utiles + g.r - 1;
  g.b_rowstride = ((g.rowlen / 16) & 1) ? g.rowlen : g.rowlen + 16;
  g.b_plane = (g.b_rows * g.b_rowstride + 15) & ~15u;
  return g;
}

int limbs32(const uint32_t* qs, uint32_t lc) {
  int L = 2;
  for (uint32_t i = 0; i < lc; ++i) L = std::max(L, limbs_for_q32(qs[i]));
  return L;
}

// Resident-kernel parameters; *lds gets the dynamic LDS bytes per workgroup.
polymul_status fill_mfma32(Mfma32Params& P, const uint32_t* a, const uint32_t* b, uint32_t* c, uint32_t n,
                           const uint32_t* qs, uint32_t lc, uint32_t nq_total, uint32_t l0, uint64_t nprod, int L,
                           uint32_t t, uint32_t* lds, bool cyclic = false, uint32_t lrep = 1,
                           bool b_shared = false, int planes = 0) {
  if (!tile_ok(n, t)) return POLYMUL_EINVAL;
  const Geometry32 g = geometry32(n, t);
  P = Mfma32Params{};
  P.a = a; P.b = b; P.c = c;
  P.nprod = nprod;
  P.n = n; P.t = g.t; P.r = g.r;
  P.log2n = (uint32_t)ilog2(n);
  P.log2t = (uint32_t)ilog2(g.t);
  P.spd = g.spd; P.log2spd = (uint32_t)ilog2(g.spd);
  P.rowlen = g.rowlen;
  P.tz = g.tz; P.tu = g.tu; P.log2U = (uint32_t)ilog2(g.U);
  P.slots = g.slots;
  P.a_plane = g.a_plane; P.b_rows = g.b_rows; P.b_rowstride = g.b_rowstride; P.b_plane = g.b_plane;
  P.E = g.E;
  P.lc = lc; P.nq_total = nq_total; P.l0 = l0; P.lrep = lrep;
  // byte planes per operand: one per limb, or one per small modulus on the RNS-CRT path
  P.slot_bytes = (uint32_t)(planes ? planes : L) * (g.a_plane + g.b_plane);
  // Epilogue choice: the one-reduction form needs sum_s P_s * n * 2^14 * |rcent_s| < 2^62,
  // P_s = number of limb pairs (i, j) with i + j = s.
  bool fast = true;
  for (uint32_t i = 0; i < lc; ++i) {
    P.mods[i] = make_mod32(qs[i], L);
    unsigned __int128 bound = 0;
    uint64_t pw = 1 % qs[i];
    for (int s = 0; s < 2 * L - 1; ++s) {
      int64_t cc = (int64_t)pw;
      if (pw > qs[i] / 2) cc -= (int64_t)qs[i];
      P.rcent[i][s] = (int32_t)cc;
      const uint64_t pairs = (uint64_t)((s < L ? s : 2 * L - 2 - s) + 1);
      bound += (unsigned __int128)pairs * n * 16384u * (uint64_t)(cc < 0 ? -cc : cc);
      pw = (pw * 256) % qs[i];
    }
    if (bound >= ((unsigned __int128)1 << 62)) fast = false;
  }
  P.fast_epilogue = fast ? 1u : 0u;
  P.cyclic = cyclic ? 1u : 0u;
  P.b_shared = b_shared ? 1u : 0u;
  P.kparts = 1;
  *lds = P.slots * P.slot_bytes;
  return *lds <= kMaxLds ? POLYMUL_OK : POLYMUL_EUNSUPPORTED;
}

// Allow up to kMaxLds of dynamic LDS for kernel K (once per process).  Called
// outside stream capture: plans set their kernels' attributes before capturing.
template <const void* (*K)()>
polymul_status allow_lds() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] { err = hipFuncSetAttribute(K(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds); });
  return err == hipSuccess ? POLYMUL_OK : hip_fail(err, "hipFuncSetAttribute");
}
template <int L, bool SMALL> const void* k_group() { return (const void*)mfma32_group_kernel<L, SMALL>; }
template <int L, typename W, int WPE> const void* k_stream() { return (const void*)stream_kernel<L, W, WPE>; }
template <typename W> const void* k_stream8() { return (const void*)stream8_kernel<W>; }
const void* k_grouped() { return (const void*)grouped_kernel; }
template <int L> const void* k_shared() { return (const void*)mfma32_shared_kernel<L>; }
template <int L, bool SHB> const void* k_small() { return (const void*)mfma16_group_kernel<L, SHB>; }

template <int L, bool SMALL>
polymul_status launch_mfma32_L(const Mfma32Params& P, uint32_t lds, hipStream_t s) {
  if (allow_lds<k_group<L, SMALL>>() != POLYMUL_OK) return POLYMUL_EDEVICE;
  const uint64_t groups = ((P.nprod << P.log2U) + 3) / 4;
  if (groups > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  hipLaunchKernelGGL((mfma32_group_kernel<L, SMALL>), dim3((uint32_t)groups), dim3(kThreads), lds, s, P);
  return launch_status();
}

// The 16x16-tile kernel: `slots` products per workgroup, as many as keep at least
// two rounds of workgroups per CU (at least four, so that every wave has a tile).
template <int L>
polymul_status launch_small_L(Mfma32Params P, hipStream_t s) {
  // one b for every product (one channel): its rows are staged once per workgroup
  const bool shb = P.b_shared && P.lc == 1 && P.lrep == 1;
  if (shb ? allow_lds<k_small<L, true>>() != POLYMUL_OK : allow_lds<k_small<L, false>>() != POLYMUL_OK)
    return POLYMUL_EDEVICE;
  const uint64_t per_slot = shb ? (uint64_t)L * P.a_plane : P.slot_bytes;
  const uint64_t fixed = (shb ? (uint64_t)L * P.b_plane : 0) + kSlots16 * sizeof(Slot16);
  uint32_t slots = kSlots16;
  while (slots > 4 && (P.nprod + slots - 1) / slots < 2ull * device_cus()) slots /= 2;
  while (slots > 1 && slots * per_slot + fixed > kMaxLds / 2) slots /= 2;
  P.slots = slots;
  const uint64_t groups = (P.nprod + slots - 1) / slots;
  if (groups > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  const uint32_t lds = (uint32_t)(slots * per_slot + fixed);  // planes, then the slot table
  if (shb) hipLaunchKernelGGL((mfma16_group_kernel<L, true>), dim3((uint32_t)groups), dim3(kThreads), lds, s, P);
  else hipLaunchKernelGGL((mfma16_group_kernel<L, false>), dim3((uint32_t)groups), dim3(kThreads), lds, s, P);
  return launch_status();
}

// One b per channel for the whole batch: workgroups take chunks of groups of one
// channel and tile position and stage that b once.
template <int L>
polymul_status launch_shared_L(const Mfma32Params& P, const SharedChunks& C, uint32_t grid, uint32_t lds,
                               hipStream_t s) {
  if (allow_lds<k_shared<L>>() != POLYMUL_OK) return POLYMUL_EDEVICE;
  hipLaunchKernelGGL((mfma32_shared_kernel<L>), dim3(grid), dim3(kThreads), lds, s, P, C);
  return launch_status();
}

polymul_status launch_shared(const Mfma32Params& P, int L, uint64_t batch, hipStream_t s) {
  const uint32_t U = 1u << P.log2U;
  SharedChunks C{};
  C.batch = batch;
  C.npos = U >= 4 ? U / 4 : 1;
  const uint64_t gpc = U >= 4 ? batch : (batch + P.slots - 1) / P.slots;
  if (gpc > 0xFFFFFFFFull) return POLYMUL_EUNSUPPORTED;
  C.groups_per_class = (uint32_t)gpc;
  const uint64_t classes = (uint64_t)P.lc * C.npos;
  const uint64_t total = classes * gpc;
  const uint64_t target = 2ull * device_cus();  // one round of two workgroups per CU
  uint64_t chunk = (total + target - 1) / target;
  if (chunk < 1) chunk = 1;
  if (chunk > gpc) chunk = gpc;
  C.chunk = (uint32_t)chunk;
  C.chunks_per_class = (uint32_t)((gpc + chunk - 1) / chunk);
  const uint64_t grid = classes * C.chunks_per_class;
  if (grid > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  const uint64_t lds = (uint64_t)L * P.b_plane + (uint64_t)P.slots * L * P.a_plane;
  if (lds > kMaxLds) return POLYMUL_EUNSUPPORTED;
  switch (L) {
    case 2: return launch_shared_L<2>(P, C, (uint32_t)grid, (uint32_t)lds, s);
    case 3: return launch_shared_L<3>(P, C, (uint32_t)grid, (uint32_t)lds, s);
    default: return launch_shared_L<4>(P, C, (uint32_t)grid, (uint32_t)lds, s);
  }
}

// ------------------------------------------- small-modulus RNS with CRT
// ExtractModuli (Algorithm 1, RNS base rules of Sec. 2.6): co-prime integers
// <= 256 taken largest first until their product exceeds 2 B (1 + 2^-16),
// B = n floor(qmax / 2)^2 the largest |X_j| of a centred negacyclic sum.
// `pad` > 0 keeps taking moduli up to that count.  Returns the count, 0 if
// kMaxCh moduli are not enough.
uint32_t crt_moduli(uint64_t n, uint32_t qmax, uint32_t* m, uint32_t pad = 0) {
  const unsigned __int128 h = qmax / 2;
  const unsigned __int128 B = (unsigned __int128)n * h * h;
  const unsigned __int128 bound = 2 * B + ((2 * B) >> 16) + 1;
  unsigned __int128 prod = 1;
  uint32_t C = 0;
  for (uint32_t cand = 256; cand >= 2 && C < (uint32_t)kMaxCh; --cand) {
    bool coprime = true;
    for (uint32_t i = 0; i < C && coprime; ++i) {
      uint32_t x = cand, y = m[i];
      while (y) { const uint32_t t = x % y; x = y; y = t; }
      coprime = x == 1;
    }
    if (!coprime) continue;
    if (prod > bound && C >= pad) break;
    m[C++] = cand;
    prod *= cand;
  }
  return prod > bound ? C : 0;
}

polymul_status fill_crt(CrtConsts& K, const uint32_t* qs, uint32_t lc, uint64_t n, uint32_t pad) {
  if (lc > (uint32_t)kMaxQC) return POLYMUL_EUNSUPPORTED;
  uint32_t qmax = 0;
  for (uint32_t i = 0; i < lc; ++i) qmax = std::max(qmax, qs[i]);
  K = CrtConsts{};
  K.C = crt_moduli(n, qmax, K.m, pad);
  if (K.C == 0) return POLYMUL_EUNSUPPORTED;
  unsigned __int128 M = 1;
  for (uint32_t c = 0; c < K.C; ++c) M *= K.m[c];
  for (uint32_t c = 0; c < K.C; ++c) {
    const uint32_t mc = K.m[c];
    const unsigned __int128 Mc = M / mc;
    const uint32_t r = (uint32_t)(Mc % mc);
    uint32_t y = 0;
    for (uint32_t k = 1; k < mc; ++k)
      if ((uint64_t)r * k % mc == 1) { y = k; break; }
    if (y == 0 && mc > 1) return POLYMUL_EDEVICE;  // unreachable for co-prime moduli
    K.y[c] = y;
    K.yp[c] = (uint32_t)(((uint64_t)y << 32) / mc);
    K.oy[c] = (uint32_t)(((uint64_t)1 << 31) * y % mc);
    K.magic[c] = (uint32_t)((1ull << 32) / mc);
    K.off[c] = (uint32_t)((1ull << 31) % mc);
    K.invm[c] = 1.0f / (float)mc;
    K.mf[c] = (float)mc;
    K.r16[c] = (int32_t)((1u << 16) % mc);
    for (uint32_t i = 0; i < lc; ++i) K.w[i][c] = (uint32_t)(Mc % qs[i]);
  }
  for (uint32_t i = 0; i < lc; ++i) K.Mq[i] = (uint32_t)(M % qs[i]);
  return POLYMUL_OK;
}

template <int C, bool SMALL, bool SHARE22> const void* k_crt() {
  return (const void*)crt_wave_kernel<C, SMALL, SHARE22>;
}

template <int C, bool SMALL, bool SHARE22>
polymul_status launch_crt_CS(const Mfma32Params& P, const CrtConsts& K, uint32_t lds, hipStream_t s) {
  if (allow_lds<k_crt<C, SMALL, SHARE22>>() != POLYMUL_OK) return POLYMUL_EDEVICE;
  const uint64_t groups = ((P.nprod << P.log2U) + 3) / 4;
  if (groups > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  hipLaunchKernelGGL((crt_wave_kernel<C, SMALL, SHARE22>), dim3((uint32_t)groups), dim3(CrtWaves<C>::kThreadsW),
                     lds, s, P, K);
  return launch_status();
}

template <int C> const void* k_crt_phase() { return (const void*)crt_phase_kernel<C>; }

template <int C>
polymul_status launch_crt_phase(const Mfma32Params& P, const CrtConsts& K, hipStream_t s) {
  if (allow_lds<k_crt_phase<C>>() != POLYMUL_OK) return POLYMUL_EDEVICE;
  const uint64_t groups = ((P.nprod << P.log2U) + 3) / 4;
  if (groups > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  const uint32_t lds = crt_phase_lds<C>(P.a_plane + P.b_plane);
  hipLaunchKernelGGL((crt_phase_kernel<C>), dim3((uint32_t)groups), dim3(8 * 64), lds, s, P, K);
  return launch_status();
}

// Dynamic LDS: the residue planes, or the combine step's bytes laid over them if larger.
template <int C, bool SMALL>
polymul_status launch_crt_C(const Mfma32Params& P, const CrtConsts& K, uint32_t lds, hipStream_t s) {
  lds = std::max(lds, crt_combine_bytes<C>());
  if (lds > kMaxLds) return POLYMUL_EUNSUPPORTED;
  // one product in 2 x 2 tiles per group: the four tiles share A by row and B by column
  const bool share22 = !SMALL && P.log2U == 2 && P.tz == 2 && P.slots == 1;
  if constexpr (!SMALL && (C == 8 || C == 9)) {
    // all C planes hold a CU alone: stage and multiply the channels in two phases
    // so that two workgroups share a CU
    if (share22 && 2 * lds > kMaxLds && 2 * crt_phase_lds<C>(P.a_plane + P.b_plane) <= kMaxLds)
      return launch_crt_phase<C>(P, K, s);
  }
  return share22 ? launch_crt_CS<C, SMALL, true>(P, K, lds, s) : launch_crt_CS<C, SMALL, false>(P, K, lds, s);
}

// Channel counts with a kernel instance; a product needing fewer moduli takes
// the next count up (the extra moduli only enlarge M).
constexpr uint32_t kCrtCounts[] = {2, 4, 6, 8, 9, 10, 11};

// nprod products (i -> global (i/lc)*nq_total + l0 + i%lc) through the small-modulus RNS.
polymul_status run_crt(const uint32_t* a, const uint32_t* b, uint32_t* c, uint32_t n, const uint32_t* qs,
                       uint32_t lc, uint32_t nq_total, uint32_t l0, uint64_t nprod, hipStream_t s) {
  if (n > 4096) return POLYMUL_EUNSUPPORTED;  // C residue planes of both operands no longer fit in LDS
  const bool small = n < 4;
  CrtConsts K;
  polymul_status st = fill_crt(K, qs, lc, n, 0);
  if (st != POLYMUL_OK) return st;
  uint32_t want = small ? (uint32_t)kMaxCh : K.C;
  for (uint32_t cc : kCrtCounts)
    if (cc >= want) { want = cc; break; }
  if (want != K.C) {
    st = fill_crt(K, qs, lc, n, want);
    if (st != POLYMUL_OK) return st;
    if (K.C != want) return POLYMUL_EUNSUPPORTED;
  }
  const int C = (int)K.C;
  // n = 4096: tile side 64, four tiles of one product in 2 x 2 (fragments shared);
  // otherwise the largest tile side whose planes fit (fewest staged bytes)
  Mfma32Params P;
  uint32_t lds = 0;
  st = POLYMUL_EUNSUPPORTED;
  if (n == 4096) {
    st = fill_mfma32(P, a, b, c, n, qs, lc, nq_total, l0, nprod, 4, 64, &lds, false, 1, false, C);
    if (st == POLYMUL_EINVAL) return st;
  }
  const uint32_t t0 = n <= 32 ? n : std::min<uint32_t>(128, n);
  for (uint32_t t = t0; st != POLYMUL_OK && t >= (n <= 32 ? n : 32u); t /= 2) {
    st = fill_mfma32(P, a, b, c, n, qs, lc, nq_total, l0, nprod, 4, t, &lds, false, 1, false, C);
    if (st == POLYMUL_EINVAL) return st;
    if (st == POLYMUL_OK) break;
    if (n <= 32) break;
  }
  if (st != POLYMUL_OK) return st;
  switch (C) {
    case 2: return launch_crt_C<2, false>(P, K, lds, s);
    case 4: return launch_crt_C<4, false>(P, K, lds, s);
    case 6: return launch_crt_C<6, false>(P, K, lds, s);
    case 8: return launch_crt_C<8, false>(P, K, lds, s);
    case 9: return launch_crt_C<9, false>(P, K, lds, s);
    case 10: return launch_crt_C<10, false>(P, K, lds, s);
    default: return small ? launch_crt_C<11, true>(P, K, lds, s) : launch_crt_C<11, false>(P, K, lds, s);
  }
}

// --------------------------------------------------------- streaming kernel
int limbs64(const uint64_t* qs, uint32_t lc) {
  int L = 2;
  for (uint32_t i = 0; i < lc; ++i) L = std::max(L, limbs_for_q64(qs[i]));
  return L <= 4 ? 4 : 8;  // two instantiations: up to 4 and up to 8 limbs
}

polymul_status fill_stream(StreamParams& P, const void* a, const void* b, void* c, uint32_t n, const uint64_t* qs,
                           uint32_t lc, uint32_t nq_total, uint32_t l0, uint64_t nprod, int L, uint32_t* lds,
                           bool cyclic = false, uint32_t lrep = 1, bool b_shared = false) {
  P = StreamParams{};
  P.a = a; P.b = b; P.c = c;
  P.nprod = nprod;
  P.n = n;
  P.t = n < 64 ? n : 64;
  P.log2t = (uint32_t)ilog2(P.t);
  P.r = n / P.t;
  P.spd = P.t >= 64 ? 2 : 1;
  P.log2spd = P.spd == 2 ? 1 : 0;
  P.rowlen = 32 * P.spd;
  P.rs = ((P.rowlen / 16) & 1) ? P.rowlen : P.rowlen + 16;
  P.tz = (P.t + 31) / 32;
  P.ublocks = (P.r + 63) / 64;
  P.dc = P.r < 16 ? P.r : 16;
  P.nchunks = P.r / P.dc;
  // a class sum holds at most L limb pairs of |product| <= 2^14: exact in int32 for K < 2^17 / L
  const uint32_t kflush = (1u << 17) / (uint32_t)L - 1;
  const uint32_t fe = kflush / (P.dc * P.t);
  P.flush_every = fe < 1 ? 1 : fe;
  P.a_win = ((P.dc - 1) * P.t + 32 * P.tz + P.rowlen + 4 + 15) & ~15u;
  P.lds_b = 2u * (uint32_t)L * P.a_win;
  P.lc = lc; P.nq_total = nq_total; P.l0 = l0; P.lrep = lrep;
  P.cyclic = cyclic ? 1u : 0u;
  P.b_shared = b_shared ? 1u : 0u;
  P.kparts = 1;
  for (uint32_t i = 0; i < lc; ++i) P.mods[i] = make_mod64(qs[i], L);
  P.lds_res = P.lds_b + (uint32_t)L * kRing * P.rs;
  *lds = P.lds_res + (L == 8 ? 16u * kStreamThreads * 8u : 0u);
  return *lds <= kMaxLds ? POLYMUL_OK : POLYMUL_EUNSUPPORTED;
}

template <int L, typename W, int WPE>
polymul_status launch_stream_L(const StreamParams& P, uint32_t lds, hipStream_t s) {
  const uint64_t blocks = P.nprod * P.ublocks * P.kparts;
  if (blocks > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  if constexpr (L == 8) {  // shift classes split by parity over wave pairs
    if (allow_lds<k_stream8<W>>() != POLYMUL_OK) return POLYMUL_EDEVICE;
    hipLaunchKernelGGL((stream8_kernel<W>), dim3((uint32_t)blocks), dim3(kStream8Threads), lds, s, P);
  } else {
    if (allow_lds<k_stream<L, W, WPE>>() != POLYMUL_OK) return POLYMUL_EDEVICE;
    hipLaunchKernelGGL((stream_kernel<L, W, WPE>), dim3((uint32_t)blocks), dim3(kStreamThreads), lds, s, P);
  }
  return launch_status();
}

// nprod products of degree bound n (i -> global (i/lc)*nq_total + l0 + i%lc), moduli qs[0..lc <= kMaxQS).
template <typename W>
polymul_status run_stream(const W* a, const W* b, W* c, uint32_t n, const uint64_t* qs, uint32_t lc,
                          uint32_t nq_total, uint32_t l0, uint64_t nprod, hipStream_t s, bool cyclic = false,
                          uint32_t lrep = 1, bool b_shared = false) {
  const int L = limbs64(qs, lc);
  if (sizeof(W) == 4 && L > 4) return POLYMUL_EINVAL;
  StreamParams P;
  uint32_t lds;
  polymul_status st = fill_stream(P, a, b, c, n, qs, lc, nq_total, l0, nprod, L, &lds, cyclic, lrep, b_shared);
  if (st != POLYMUL_OK) return st;
  if (L == 4) return launch_stream_L<4, W, 2>(P, lds, s);
  if constexpr (sizeof(W) == 8) return launch_stream_L<8, W, 1>(P, lds, s);
  return POLYMUL_EINVAL;
}

// nprod products (i -> global (i/lc)*nq_total + l0 + i%lc) with moduli qs[0..lc <= kMaxQ).
polymul_status run_mfma32(const uint32_t* a, const uint32_t* b, uint32_t* c, uint32_t n, const uint32_t* qs,
                          uint32_t lc, uint32_t nq_total, uint32_t l0, uint64_t nprod, hipStream_t s,
                          bool cyclic = false, uint32_t lrep = 1, bool b_shared = false) {
  if (n > 8192) {
    if (lrep > 1) {
      if (lc > (uint32_t)kMaxQS) return POLYMUL_EUNSUPPORTED;
      uint64_t q64[kMaxQS];
      for (uint32_t i = 0; i < lc; ++i) q64[i] = qs[i];
      return run_stream<uint32_t>(a, b, c, n, q64, lc, nq_total, l0, nprod, s, cyclic, lrep);
    }
    // degree too large for both operands in LDS: K-streaming kernel, moduli in chunks of kMaxQS
    uint64_t q64[kMaxQ];
    for (uint32_t i = 0; i < lc; ++i) q64[i] = qs[i];
    const uint64_t batch = nprod / lc;
    for (uint32_t c0 = 0; c0 < lc; c0 += kMaxQS) {
      const uint32_t cc = std::min(lc - c0, (uint32_t)kMaxQS);
      const uint64_t np = cc == lc ? nprod : batch * cc;
      polymul_status st = run_stream<uint32_t>(a, b, c, n, q64 + c0, cc, nq_total, l0 + c0, np, s, cyclic, 1,
                                               b_shared);
      if (st != POLYMUL_OK) return st;
    }
    return POLYMUL_OK;
  }
  const int L = limbs32(qs, lc);
  Mfma32Params P;
  uint32_t lds;
  polymul_status st =
      fill_mfma32(P, a, b, c, n, qs, lc, nq_total, l0, nprod, L, tile_for(n, L), &lds, cyclic, lrep, b_shared);
  if (st != POLYMUL_OK) return st;
  const bool small = n < 4;
  if (P.t == 16 && n >= 64) {
    switch (L) {
      case 2: return launch_small_L<2>(P, s);
      case 3: return launch_small_L<3>(P, s);
      default: return launch_small_L<4>(P, s);
    }
  }
  if (b_shared && !small && lrep == 1) return launch_shared(P, L, nprod / lc, s);
  switch (L) {
    case 2: return small ? launch_mfma32_L<2, true>(P, lds, s) : launch_mfma32_L<2, false>(P, lds, s);
    case 3: return small ? launch_mfma32_L<3, true>(P, lds, s) : launch_mfma32_L<3, false>(P, lds, s);
    default: return small ? launch_mfma32_L<4, true>(P, lds, s) : launch_mfma32_L<4, false>(P, lds, s);
  }
}

// ---------------------------------------------------------------- Karatsuba
template <typename KP>
polymul_status kara_split(const KP& K, uint32_t depth, uint64_t blocks, hipStream_t s) {
  switch (depth) {
    case 1: hipLaunchKernelGGL((kara_split_kernel<1, KP>), dim3((uint32_t)blocks), dim3(256), 0, s, K); break;
    case 2: hipLaunchKernelGGL((kara_split_kernel<2, KP>), dim3((uint32_t)blocks), dim3(256), 0, s, K); break;
    default: hipLaunchKernelGGL((kara_split_kernel<3, KP>), dim3((uint32_t)blocks), dim3(256), 0, s, K); break;
  }
  return launch_status();
}
template <typename KP>
polymul_status kara_combine(const KP& K, uint32_t depth, uint64_t blocks, hipStream_t s) {
  switch (depth) {
    case 1: hipLaunchKernelGGL((kara_combine_kernel<1, KP>), dim3((uint32_t)blocks), dim3(256), 0, s, K); break;
    case 2: hipLaunchKernelGGL((kara_combine_kernel<2, KP>), dim3((uint32_t)blocks), dim3(256), 0, s, K); break;
    default: hipLaunchKernelGGL((kara_combine_kernel<3, KP>), dim3((uint32_t)blocks), dim3(256), 0, s, K); break;
  }
  return launch_status();
}

// Most K runs a streamed Karatsuba sub-product launch is cut into (whole rounds, see
// below); polymul_tune_param_set can lower the cap.
constexpr uint32_t kKaraRuns = 4;
std::atomic<uint32_t> g_kara_runs_max{kKaraRuns};

// Workspace bytes of one Karatsuba call: sub-operands of a and b and the sub-products
// (3 words per sub-product coefficient), plus kKaraRuns copies of the sub-products for
// runs when `runs` is set.
polymul_status kara_workspace(uint64_t n, uint64_t products, uint32_t depth, uint32_t word, uint64_t* bytes,
                              bool runs = false) {
  if (!bytes || !is_pow2(n) || n > 65536) return POLYMUL_EINVAL;
  if (depth == 0) {  // the tuned depth; the direct route needs no workspace
    depth = kara_depth_for(n, products, word == 8);
    if (depth == 0) { *bytes = 0; return POLYMUL_OK; }
  }
  if (depth > 3 || (n >> depth) < 4) return POLYMUL_EINVAL;
  uint64_t nsub = 1;
  for (uint32_t l = 0; l < depth; ++l) nsub *= 3;
  const unsigned __int128 words = (unsigned __int128)products * nsub * (n >> depth);
  if (words >> 57) return POLYMUL_EINVAL;
  *bytes = (uint64_t)((3 + (runs ? kKaraRuns : 0)) * words * word);
  return POLYMUL_OK;
}

// The RNS Karatsuba route on validated arguments with a workspace of at least
// kara_workspace(n, batch * L, depth, 4) bytes: split, sub-products, combine.
polymul_status run_rns_karatsuba(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n, const uint32_t* q,
                                 uint32_t L, uint64_t batch, uint32_t depth, void* workspace, hipStream_t stream) {
  const uint32_t nsub = depth == 1 ? 3 : depth == 2 ? 9 : 27;
  const uint32_t np = (uint32_t)(n >> depth);
  const uint64_t nprod = batch * L;
  const uint64_t sub_words = nprod * nsub * np;
  KaraParams K{};
  K.a = a; K.b = b; K.c = c;
  K.sa = (uint32_t*)workspace;
  K.sb = K.sa + sub_words;
  uint32_t* sc = K.sb + sub_words;
  K.sc = sc;
  K.nprod = nprod; K.n = (uint32_t)n; K.np = np; K.depth = depth; K.nsub = nsub; K.L = L;
  const int Lq = limbs32(q, L);
  for (uint32_t l = 0; l < L; ++l) K.mods[l] = make_mod32(q[l], Lq);
  const uint64_t threads = nprod * np;
  const uint64_t blocks = (threads + 255) / 256;
  if (blocks > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  polymul_status st = kara_split(K, depth, blocks, stream);
  if (st != POLYMUL_OK) return st;
  // the sub-products: nprod * nsub products of degree bound n' with modulus (i / nsub) % L
  st = run_mfma32(K.sa, K.sb, sc, np, q, L, L, 0, nprod * nsub, stream, false, nsub);
  if (st != POLYMUL_OK) return st;
  return kara_combine(K, depth, blocks, stream);
}

// Validation shared by both RNS Karatsuba entry points; *need gets the workspace bytes.
polymul_status check_rns_karatsuba(const uint32_t* a, const uint32_t* b, const uint32_t* c, uint64_t n,
                                   const uint32_t* q, uint32_t L, uint64_t batch, uint32_t depth, uint64_t* need,
                                   uint64_t* bytes) {
  if (L == 0 || L > 16 || !q || depth == 0) return POLYMUL_EINVAL;  // depth resolved by the caller
  for (uint32_t l = 0; l < L; ++l)
    if (q[l] < 2) return POLYMUL_EINVAL;
  polymul_status st = kara_workspace(n, batch * L, depth, 4, need);
  if (st != POLYMUL_OK) return st;
  return check_arrays(a, b, c, n, batch, L, 4, bytes);
}

}  // namespace

// Scratch of the allocation-free Karatsuba entry point: one copy on every GPU the
// library runs on, set aside when the library's code is loaded there and kept
// until the process ends.  In host code `scratch` names a host-side stand-in,
// never the device memory: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[POLYMUL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device (null: not looked up yet)

// Device address of the current device's scratch, looked up once per device.
polymul_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return POLYMUL_EUNSUPPORTED;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
    if (!p) return POLYMUL_EDEVICE;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return POLYMUL_OK;
}

// c = sum of the kparts runs' residues mod q, 64-bit words.
__global__ __launch_bounds__(256) void split_sum64_kernel(const uint64_t* __restrict__ ws, uint64_t* __restrict__ c,
                                                          uint64_t words, uint32_t kparts, uint64_t q) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= words) return;
  uint64_t acc = 0;
  for (uint32_t p = 0; p < kparts; ++p) acc = addmod64(acc, ws[(uint64_t)p * words + i], q);
  c[i] = acc;
}

}  // namespace

// ------------------------------------------------------------------- plans
struct polymul_plan {
  GroupJob* d_jobs = nullptr;       // device job table
  WorkItem* d_items = nullptr;      // device work list (largest first)
  uint32_t* d_counter = nullptr;    // queue counter and workgroups-left counter (zero between launches)
  void* d_part_ws = nullptr;        // residues of K-split runs
  std::vector<SplitSeg> segs;       // K-split jobs: c = sum of their runs mod q, one launch for all
  SplitSeg* d_segs = nullptr;
  uint32_t sum_blocks = 0;
  uint32_t nitems = 0;
  uint32_t lds = 0;                 // dynamic LDS of the grouped launch
  uint32_t grid = 0;
  // 64-bit groups run as separate streaming launches after the grouped one
  std::vector<StreamParams> wide;
  std::vector<uint32_t> wide_lds;
  std::vector<int> wide_L;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true;
};

namespace {

polymul_status plan_attrs() {
  if (allow_lds<k_grouped>() != POLYMUL_OK) return POLYMUL_EDEVICE;
  if (allow_lds<k_stream<4, uint64_t, 2>>() != POLYMUL_OK) return POLYMUL_EDEVICE;
  if (allow_lds<k_stream8<uint64_t>>() != POLYMUL_OK) return POLYMUL_EDEVICE;
  return POLYMUL_OK;
}

polymul_status plan_launch(const polymul_plan* p, hipStream_t s) {
  if (p->nitems) {
    hipLaunchKernelGGL(grouped_kernel, dim3(p->grid), dim3(kThreads), p->lds, s, p->d_jobs, p->d_items,
                       p->nitems, p->d_counter);
    polymul_status st = launch_status();
    if (st != POLYMUL_OK) return st;
    if (!p->segs.empty()) {
      hipLaunchKernelGGL(split_sum_kernel, dim3(p->sum_blocks), dim3(256), 0, s, p->d_segs,
                         (uint32_t)p->segs.size());
      st = launch_status();
      if (st != POLYMUL_OK) return st;
    }
  }
  for (size_t i = 0; i < p->wide.size(); ++i) {
    polymul_status st = p->wide_L[i] == 4 ? launch_stream_L<4, uint64_t, 2>(p->wide[i], p->wide_lds[i], s)
                                          : launch_stream_L<8, uint64_t, 1>(p->wide[i], p->wide_lds[i], s);
    if (st != POLYMUL_OK) return st;
  }
  return POLYMUL_OK;
}

void plan_free(polymul_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->d_jobs) (void)hipFree(p->d_jobs);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_counter) (void)hipFree(p->d_counter);
  if (p->d_part_ws) (void)hipFree(p->d_part_ws);
  if (p->d_segs) (void)hipFree(p->d_segs);
  delete p;
}

// Plan scheduling knobs (polymul_tune_param_set): the split threshold as a percentage
// of a CU's even share of the plan's work, and the weight of a streamed block's MFMA
// work relative to a resident group's (its chunked staging and 128-bit flushes make
// it slower than its MFMA count says), as a percentage.
std::atomic<uint32_t> g_plan_share_pct{140};
std::atomic<uint32_t> g_plan_stream_pct{125};

// Estimated time of one item (MFMAs per wave of its four tiles, the streamed
// blocks' weighted), for the largest-first order and the split decision.
uint64_t item_cost(const GroupJob& j) {
  if (j.kind == kJobSmall) {  // slots x tiles x K-steps of L^2 MFMAs of half the length
    const uint64_t steps = j.rp.n >> 6;
    return (uint64_t)j.rp.slots * (1u << j.rp.log2U) * steps * j.L * j.L / 2;
  }
  if (j.kind == kJobResident) {
    const uint64_t steps = (uint64_t)j.rp.r << j.rp.log2spd;
    return 4 * steps * j.L * j.L / j.rp.kparts;  // four tiles, L^2 MFMAs per K-step
  }
  const uint64_t steps = (uint64_t)j.sp.r << j.sp.log2spd;
  return 4 * steps * 16 * g_plan_stream_pct.load(std::memory_order_relaxed) / 100 / j.sp.kparts;
}

// The same for one unsplit item of a 32-bit group on its default route (resident for
// n in [4, 8192]: beyond 4096 only as K-split runs, else streamed), and the number of
// such items.
void default_cost(uint32_t n, uint64_t count, int L, uint64_t* items, uint64_t* cost) {
  if (n >= 64 && plan_tile(n, L) == 16) {
    const Geometry32 g = geometry32(n, 16);
    const uint32_t slots = plan_small_slots((uint32_t)L * (g.a_plane + g.b_plane));
    *items = (count + slots - 1) / slots;
    *cost = (uint64_t)slots * g.U * (n >> 6) * L * L / 2;
  } else if (n >= 4 && n <= 8192) {
    const Geometry32 g = geometry32(n, plan_tile(n, L));
    *items = (count * g.U + 3) / 4;
    *cost = 4 * (uint64_t)g.r * g.spd * L * L;
  } else {
    const uint32_t t = n < 64 ? n : 64, r = n / t, spd = t >= 64 ? 2 : 1;
    *items = count * ((r + 63) / 64);
    *cost = 4 * (uint64_t)r * spd * 16 * g_plan_stream_pct.load(std::memory_order_relaxed) / 100;
  }
}

// K-split of a resident job whose item would cost `ci` > `share`: runs of K-steps
// (a power of two of them) until a run costs at most the share.  Each run stages
// only its K window (the K-steps' d range, D = d_hi - d_lo <= Dmax): ext positions
// 0 .. Dmax t + t + 3 and 32 utiles + Dmax - 1 B rows, so the slot shrinks with the
// run.  Groups of one product with a tile per wave (U >= 4, hence t >= 32) and
// n >= 256 (the staging runs of 64 word groups) only.  Returns false (job
// unchanged) when the job cannot or need not be split.
bool k_window_split(GroupJob& job, uint64_t ci, uint64_t share, uint32_t* lds) {
  Mfma32Params& P = job.rp;
  if (P.log2U < 2 || P.n < 256 || P.t < 32) return false;
  const uint32_t steps = P.r << P.log2spd;
  uint32_t k = 1;
  while (2 * k <= steps && ci / k > share) k *= 2;
  if (k == 1) return false;
  uint32_t dmax = 0;
  for (uint32_t part = 0; part < k; ++part) {
    const uint32_t st_lo = part * steps / k, st_hi = (part + 1) * steps / k;
    dmax = std::max(dmax, ((st_hi - 1) >> P.log2spd) + 1 - (st_lo >> P.log2spd));
  }
  const uint32_t utiles = 4 / P.tz;  // the group's u tiles (its four tiles cover every z)
  const uint32_t a_plane = (dmax * P.t + P.rowlen + 4 + 15) & ~15u;
  const uint32_t b_rows = 32 * utiles + dmax - 1;
  const uint32_t b_plane = (b_rows * P.b_rowstride + 15) & ~15u;
  const uint32_t slot = job.L * (a_plane + b_plane);
  if (slot > kMaxLds / 2) return false;
  P.kparts = k;
  P.a_plane = a_plane;
  P.b_rows = b_rows;
  P.b_plane = b_plane;
  P.slot_bytes = slot;
  P.slots = 1;
  *lds = slot;
  return true;
}

}  // namespace

extern "C" {

const char* polymul_status_string(polymul_status s) {
  switch (s) {
    case POLYMUL_OK: return "POLYMUL_OK";
    case POLYMUL_EINVAL: return "POLYMUL_EINVAL: invalid argument";
    case POLYMUL_EALIAS: return "POLYMUL_EALIAS: output overlaps an input";
    case POLYMUL_EUNSUPPORTED: return "POLYMUL_EUNSUPPORTED: not implemented for these arguments";
    case POLYMUL_ENOMEM: return "POLYMUL_ENOMEM: allocation failed";
    case POLYMUL_EDEVICE: return "POLYMUL_EDEVICE: HIP call or kernel launch failed";
    case POLYMUL_ESCRATCH: return "POLYMUL_ESCRATCH: the call needs more scratch than the library holds";
  }
  return "POLYMUL_UNKNOWN_STATUS";
}

polymul_status polymul_negacyclic(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n, uint32_t q,
                                  uint64_t batch, hipStream_t stream) {
  if (q < 2) return POLYMUL_EINVAL;
  uint64_t bytes;
  polymul_status st = check_arrays(a, b, c, n, batch, 1, 4, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  return run_mfma32(a, b, c, (uint32_t)n, &q, 1, 1, 0, batch, stream);
}

polymul_status polymul_negacyclic_rns(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n,
                                      const uint32_t* q, uint32_t L, uint64_t batch, hipStream_t stream) {
  if (L == 0 || !q) return POLYMUL_EINVAL;
  for (uint32_t l = 0; l < L; ++l)
    if (q[l] < 2) return POLYMUL_EINVAL;
  uint64_t bytes;
  polymul_status st = check_arrays(a, b, c, n, batch, L, 4, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  for (uint32_t l0 = 0; l0 < L; l0 += kMaxQ) {
    const uint32_t lc = std::min(L - l0, (uint32_t)kMaxQ);
    st = run_mfma32(a, b, c, (uint32_t)n, q + l0, lc, L, l0, batch * lc, stream);
    if (st != POLYMUL_OK) return st;
  }
  return POLYMUL_OK;
}

polymul_status polymul_negacyclic_plain(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n,
                                        uint32_t q, uint64_t batch, hipStream_t stream) {
  if (q < 2) return POLYMUL_EINVAL;
  uint64_t bytes;
  polymul_status st = check_arrays(a, b, c, n, batch, 1, 4, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  PlainParams P{};
  P.a = a; P.b = b; P.c = c; P.batch = batch; P.n = (uint32_t)n;
  P.blocks_per_prod = (uint32_t)((n + kPlainOut - 1) / kPlainOut);
  P.m = make_mod32(q, 4);
  // lazy sums: after a fold s <= (2^32 - 1)(R + 1) with R = 2^32 mod q, and
  // F = floor((2^64 - 1 - that) / (q - 1)^2) >= 1 more products fit
  P.r32 = (uint32_t)((1ull << 32) % q);
  const uint64_t smax = 0xFFFFFFFFull * ((uint64_t)P.r32 + 1);
  const uint64_t qm1 = q - 1;
  const uint64_t F = (UINT64_MAX - smax) / (qm1 * qm1);
  P.fold_bodies = F >= 16 ? (uint32_t)std::min<uint64_t>(F / 16, 1u << 20) : 0u;
  const uint64_t blocks = batch * P.blocks_per_prod;
  if (blocks > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  hipLaunchKernelGGL(plain_kernel, dim3((uint32_t)blocks), dim3(kPlainThreads), 0, stream, P);
  return launch_status();
}

polymul_status polymul_negacyclic_u64(const uint64_t* a, const uint64_t* b, uint64_t* c, uint64_t n, uint64_t q,
                                      uint64_t batch, hipStream_t stream) {
  if (q < 2) return POLYMUL_EINVAL;
  uint64_t bytes;
  polymul_status st = check_arrays(a, b, c, n, batch, 1, 8, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  return run_stream<uint64_t>(a, b, c, (uint32_t)n, &q, 1, 1, 0, batch, stream);
}

polymul_status polymul_plan_create(polymul_plan** plan, const polymul_group* groups, uint32_t ngroups,
                                   uint32_t flags) {
  if (!plan) return POLYMUL_EINVAL;
  *plan = nullptr;
  if (ngroups && !groups) return POLYMUL_EINVAL;
  if (flags & ~POLYMUL_PLAN_NO_GRAPH) return POLYMUL_EINVAL;
  // ---- validate every group before any HIP call (GenConfig / ExtractDimensions)
  for (uint32_t g = 0; g < ngroups; ++g) {
    const polymul_group& G = groups[g];
    if (G.elem_bytes != 4 && G.elem_bytes != 8) return POLYMUL_EINVAL;
    if (G.q < 2 || (G.elem_bytes == 4 && G.q > 0xFFFFFFFFull)) return POLYMUL_EINVAL;
    uint64_t bytes;
    polymul_status st = check_arrays(G.a, G.b, G.c, G.n, G.count, 1, G.elem_bytes, &bytes);
    if (st != POLYMUL_OK) return st;
  }
  polymul_plan* p = new (std::nothrow) polymul_plan();
  if (!p) return POLYMUL_ENOMEM;
  p->use_graph = !(flags & POLYMUL_PLAN_NO_GRAPH);
  std::vector<GroupJob> jobs;
  std::vector<WorkItem> items;
  // Balance (paper Sec. 3 notes the TPU's lack of fine control): the persistent grid
  // holds two workgroups per CU; the items of a 32-bit group that would cost more
  // than a CU's even share of the total (two workgroups' shares: finer runs pay more
  // staging than they save) have their K range cut into runs (resident groups of one
  // product, or streamed blocks), whose residues a second kernel adds up mod q.
  uint64_t total_cost = 0;
  for (uint32_t g = 0; g < ngroups; ++g) {
    if (groups[g].elem_bytes != 4 || groups[g].count == 0) continue;
    const uint32_t q32 = (uint32_t)groups[g].q;
    uint64_t ni, ci;
    default_cost((uint32_t)groups[g].n, groups[g].count, limbs32(&q32, 1), &ni, &ci);
    total_cost += ni * ci;
  }
  const uint64_t share = std::max<uint64_t>(
      64, total_cost / device_cus() * g_plan_share_pct.load(std::memory_order_relaxed) / 100);
  uint64_t part_words = 0;
  for (uint32_t g = 0; g < ngroups; ++g) {
    const polymul_group& G = groups[g];
    if (G.count == 0) continue;
    const uint32_t n = (uint32_t)G.n;
    if (G.elem_bytes == 8) {
      StreamParams sp;
      uint32_t lds;
      const int L = limbs64(&G.q, 1);
      polymul_status st = fill_stream(sp, G.a, G.b, G.c, n, &G.q, 1, 1, 0, G.count, L, &lds);
      if (st != POLYMUL_OK) { plan_free(p); return st; }
      p->wide.push_back(sp);
      p->wide_lds.push_back(lds);
      p->wide_L.push_back(L);
      continue;
    }
    GroupJob job{};
    const uint32_t q32 = (uint32_t)G.q;
    uint32_t lds = 0;
    polymul_status st;
    uint64_t ni, ci;
    const int Lg = limbs32(&q32, 1);
    default_cost(n, G.count, Lg, &ni, &ci);
    const bool split = ci > share;
    job.L = (uint32_t)Lg;
    if (n >= 64 && plan_tile(n, Lg) == 16) {
      job.kind = kJobSmall;
      st = fill_mfma32(job.rp, (const uint32_t*)G.a, (const uint32_t*)G.b, (uint32_t*)G.c, n, &q32, 1, 1, 0,
                       G.count, Lg, 16, &lds);
      job.rp.slots = plan_small_slots(job.rp.slot_bytes);
      lds = job.rp.slots * job.rp.slot_bytes + kSlots16 * (uint32_t)sizeof(Slot16);
    } else if (n >= 4 && n <= 4096) {
      job.kind = kJobResident;
      st = fill_mfma32(job.rp, (const uint32_t*)G.a, (const uint32_t*)G.b, (uint32_t*)G.c, n, &q32, 1, 1, 0,
                       G.count, Lg, plan_tile(n, Lg), &lds);
      if (st == POLYMUL_OK && split && k_window_split(job, ci, share, &lds)) {
        // an offset for now; turned into a device pointer once the buffer exists
        job.rp.part_ws = (uint32_t*)(uintptr_t)part_words;
        part_words += (uint64_t)job.rp.kparts * G.count * n;
      }
    } else if (split && n <= 8192 &&
               fill_mfma32(job.rp, (const uint32_t*)G.a, (const uint32_t*)G.b, (uint32_t*)G.c, n, &q32, 1, 1, 0,
                           G.count, Lg, plan_tile(n, Lg), &lds) == POLYMUL_OK &&
               k_window_split(job, ci, share, &lds)) {
      // whole products too large for two workgroups per CU, K-split into windowed runs
      job.kind = kJobResident;
      st = POLYMUL_OK;
      job.rp.part_ws = (uint32_t*)(uintptr_t)part_words;
      part_words += (uint64_t)job.rp.kparts * G.count * n;
    } else {
      job.kind = kJobStream;
      const uint64_t q64 = G.q;
      st = fill_stream(job.sp, G.a, G.b, G.c, n, &q64, 1, 1, 0, G.count, 4, &lds);
      if (st == POLYMUL_OK && split) {
        uint32_t k = 1;
        while (k < job.sp.nchunks && ci / k > share) k *= 2;
        job.sp.kparts = k;
        if (k > 1) {
          job.sp.part_ws = (void*)(uintptr_t)part_words;
          part_words += (uint64_t)k * G.count * n;
        }
      }
    }
    if (st != POLYMUL_OK) { plan_free(p); return st; }
    p->lds = std::max(p->lds, lds);
    const uint32_t jid = (uint32_t)jobs.size();
    const uint64_t cnt = job.kind == kJobSmall      ? (G.count + job.rp.slots - 1) / job.rp.slots
                         : job.kind == kJobResident ? ((G.count << job.rp.log2U) + 3) / 4 * job.rp.kparts
                                                    : G.count * job.sp.ublocks * job.sp.kparts;
    if (cnt + items.size() > 0xFFFFFFFFull) { plan_free(p); return POLYMUL_EUNSUPPORTED; }
    for (uint64_t i = 0; i < cnt; ++i) items.push_back(WorkItem{jid, (uint32_t)i});
    jobs.push_back(job);
  }
  // largest items first
  std::stable_sort(items.begin(), items.end(), [&](const WorkItem& x, const WorkItem& y) {
    return item_cost(jobs[x.group]) > item_cost(jobs[y.group]);
  });
  p->nitems = (uint32_t)items.size();
  if (p->nitems) {
    if (hipMalloc((void**)&p->d_jobs, jobs.size() * sizeof(GroupJob)) != hipSuccess ||
        hipMalloc((void**)&p->d_items, items.size() * sizeof(WorkItem)) != hipSuccess ||
        hipMalloc((void**)&p->d_counter, 256) != hipSuccess) {
      plan_free(p);
      return POLYMUL_ENOMEM;
    }
    if (part_words) {
      if (hipMalloc(&p->d_part_ws, part_words * 4) != hipSuccess) {
        plan_free(p);
        return POLYMUL_ENOMEM;
      }
      for (GroupJob& j : jobs) {
        if (j.kind == kJobStream && j.sp.kparts > 1) {
          j.sp.part_ws = (uint32_t*)p->d_part_ws + (uintptr_t)j.sp.part_ws;
          p->segs.push_back({(const uint32_t*)j.sp.part_ws, (uint32_t*)j.sp.c, j.sp.nprod * j.sp.n, j.sp.kparts,
                             0, make_mod32((uint32_t)j.sp.mods[0].q, 4)});
        }
        if (j.kind == kJobResident && j.rp.kparts > 1) {
          j.rp.part_ws = (uint32_t*)p->d_part_ws + (uintptr_t)j.rp.part_ws;
          p->segs.push_back({j.rp.part_ws, j.rp.c, j.rp.nprod * j.rp.n, j.rp.kparts, 0, j.rp.mods[0]});
        }
      }
      uint64_t blocks = 0;
      for (SplitSeg& sg : p->segs) {
        sg.first_block = (uint32_t)blocks;
        blocks += (sg.words / 4 + 255) / 256;
      }
      if (blocks > 0x7FFFFFFFull) { plan_free(p); return POLYMUL_EUNSUPPORTED; }
      p->sum_blocks = (uint32_t)blocks;
      if (!p->segs.empty() && hipMalloc((void**)&p->d_segs, p->segs.size() * sizeof(SplitSeg)) != hipSuccess) {
        plan_free(p);
        return POLYMUL_ENOMEM;
      }
    }
    hipError_t e = hipMemcpy(p->d_jobs, jobs.data(), jobs.size() * sizeof(GroupJob), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
    if (e == hipSuccess && !p->segs.empty())
      e = hipMemcpy(p->d_segs, p->segs.data(), p->segs.size() * sizeof(SplitSeg), hipMemcpyHostToDevice);
    // the grouped kernel leaves its counters at zero; they start there (set outside any
    // capture, and finished before the plan is returned: the caller's stream need not
    // be ordered after the null stream the memset runs on)
    if (e == hipSuccess) e = hipMemset(p->d_counter, 0, 2 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) { plan_free(p); return hip_fail(e, "hipMemcpy (plan tables)"); }
    // persistent grid: as many workgroups as fit at once (two per CU within the register budget)
    const uint32_t per_cu = std::max(1u, std::min(2u, kMaxLds / std::max(p->lds, 1u)));
    p->grid = std::min<uint64_t>(p->nitems, (uint64_t)device_cus() * per_cu);
  }
  if (plan_attrs() != POLYMUL_OK) {
    plan_free(p);
    return POLYMUL_EDEVICE;
  }
  if (p->use_graph && (p->nitems || !p->wide.empty())) {
    hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { plan_free(p); return hip_fail(e, "hipStreamCreateWithFlags"); }
    e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { plan_free(p); return hip_fail(e, "hipStreamBeginCapture"); }
    const polymul_status st = plan_launch(p, p->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &graph);
    p->graph = graph;
    if (st != POLYMUL_OK || e != hipSuccess || !graph) {
      plan_free(p);
      return e != hipSuccess ? hip_fail(e, "hipStreamEndCapture") : POLYMUL_EDEVICE;
    }
    e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { plan_free(p); return hip_fail(e, "hipGraphInstantiate"); }
  }
  *plan = p;
  return POLYMUL_OK;
}

polymul_status polymul_plan_execute(polymul_plan* plan, hipStream_t stream) {
  if (!plan) return POLYMUL_EINVAL;
  if (plan->exec) {
    const hipError_t e = hipGraphLaunch(plan->exec, stream);
    return e == hipSuccess ? POLYMUL_OK : hip_fail(e, "hipGraphLaunch");
  }
  return plan_launch(plan, stream);
}

polymul_status polymul_plan_destroy(polymul_plan* plan) {
  plan_free(plan);
  return POLYMUL_OK;
}

polymul_status polymul_cyclic(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n, uint32_t q,
                              uint64_t batch, hipStream_t stream) {
  if (q < 2) return POLYMUL_EINVAL;
  uint64_t bytes;
  polymul_status st = check_arrays(a, b, c, n, batch, 1, 4, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  return run_mfma32(a, b, c, (uint32_t)n, &q, 1, 1, 0, batch, stream, true);
}

polymul_status polymul_cyclic_u64(const uint64_t* a, const uint64_t* b, uint64_t* c, uint64_t n, uint64_t q,
                                  uint64_t batch, hipStream_t stream) {
  if (q < 2) return POLYMUL_EINVAL;
  uint64_t bytes;
  polymul_status st = check_arrays(a, b, c, n, batch, 1, 8, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  return run_stream<uint64_t>(a, b, c, (uint32_t)n, &q, 1, 1, 0, batch, stream, true);
}

polymul_status polymul_crt_moduli(uint64_t n, uint32_t q, uint32_t* moduli, uint32_t* count) {
  if (!moduli || !count || !is_pow2(n) || n > 65536 || q < 2) return POLYMUL_EINVAL;
  uint32_t m[kMaxCh];
  const uint32_t C = crt_moduli(n, q, m);
  if (C == 0) return POLYMUL_EUNSUPPORTED;
  for (uint32_t i = 0; i < C; ++i) moduli[i] = m[i];
  *count = C;
  return POLYMUL_OK;
}

polymul_status polymul_negacyclic_crt(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n, uint32_t q,
                                      uint64_t batch, hipStream_t stream) {
  if (q < 2) return POLYMUL_EINVAL;
  uint64_t bytes;
  polymul_status st = check_arrays(a, b, c, n, batch, 1, 4, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  return run_crt(a, b, c, (uint32_t)n, &q, 1, 1, 0, batch, stream);
}

polymul_status polymul_negacyclic_rns_crt(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n,
                                          const uint32_t* q, uint32_t L, uint64_t batch, hipStream_t stream) {
  if (L == 0 || !q) return POLYMUL_EINVAL;
  for (uint32_t l = 0; l < L; ++l)
    if (q[l] < 2) return POLYMUL_EINVAL;
  uint64_t bytes;
  polymul_status st = check_arrays(a, b, c, n, batch, L, 4, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  for (uint32_t l0 = 0; l0 < L; l0 += kMaxQC) {
    const uint32_t lc = std::min(L - l0, (uint32_t)kMaxQC);
    st = run_crt(a, b, c, (uint32_t)n, q + l0, lc, L, l0, batch * lc, stream);
    if (st != POLYMUL_OK) return st;
  }
  return POLYMUL_OK;
}

polymul_status polymul_negacyclic_shared(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n,
                                         uint32_t q, uint64_t batch, hipStream_t stream) {
  if (q < 2) return POLYMUL_EINVAL;
  polymul_status st = check_shared(a, b, c, n, batch, 1, 4);
  if (st != POLYMUL_OK || batch == 0) return st;
  return run_mfma32(a, b, c, (uint32_t)n, &q, 1, 1, 0, batch, stream, false, 1, true);
}

polymul_status polymul_negacyclic_rns_shared(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n,
                                             const uint32_t* q, uint32_t L, uint64_t batch, hipStream_t stream) {
  if (L == 0 || !q) return POLYMUL_EINVAL;
  for (uint32_t l = 0; l < L; ++l)
    if (q[l] < 2) return POLYMUL_EINVAL;
  polymul_status st = check_shared(a, b, c, n, batch, L, 4);
  if (st != POLYMUL_OK || batch == 0) return st;
  for (uint32_t l0 = 0; l0 < L; l0 += kMaxQ) {
    const uint32_t lc = std::min(L - l0, (uint32_t)kMaxQ);
    st = run_mfma32(a, b, c, (uint32_t)n, q + l0, lc, L, l0, batch * lc, stream, false, 1, true);
    if (st != POLYMUL_OK) return st;
  }
  return POLYMUL_OK;
}

polymul_status polymul_negacyclic_u64_shared(const uint64_t* a, const uint64_t* b, uint64_t* c, uint64_t n,
                                             uint64_t q, uint64_t batch, hipStream_t stream) {
  if (q < 2) return POLYMUL_EINVAL;
  polymul_status st = check_shared(a, b, c, n, batch, 1, 8);
  if (st != POLYMUL_OK || batch == 0) return st;
  return run_stream<uint64_t>(a, b, c, (uint32_t)n, &q, 1, 1, 0, batch, stream, false, 1, true);
}

polymul_status polymul_karatsuba_workspace_size(uint64_t n, uint32_t L, uint64_t batch, uint32_t depth,
                                                uint64_t* bytes) {
  if (L < 1 || L > 16) return POLYMUL_EINVAL;
  return kara_workspace(n, batch * L, depth, 4, bytes);
}

polymul_status polymul_karatsuba_u64_workspace_size(uint64_t n, uint64_t batch, uint32_t depth, uint64_t* bytes) {
  return kara_workspace(n, batch, depth, 8, bytes, true);
}

polymul_status polymul_negacyclic_u64_karatsuba(const uint64_t* a, const uint64_t* b, uint64_t* c, uint64_t n,
                                                uint64_t q, uint64_t batch, uint32_t depth, void* workspace,
                                                uint64_t workspace_bytes, hipStream_t stream) {
  if (q < 2 || !is_pow2(n) || n > 65536) return POLYMUL_EINVAL;
  if (depth == 0) {
    depth = kara_depth_for(n, batch, true);
    if (depth == 0) return polymul_negacyclic_u64(a, b, c, n, q, batch, stream);
  }
  uint64_t need;
  polymul_status st = kara_workspace(n, batch, depth, 8, &need, true);
  if (st != POLYMUL_OK) return st;
  uint64_t bytes;
  st = check_arrays(a, b, c, n, batch, 1, 8, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  if (!workspace || ((uintptr_t)workspace & 15) || workspace_bytes < need) return POLYMUL_EINVAL;
  if (overlaps(workspace, need, a, bytes) || overlaps(workspace, need, b, bytes) || overlaps(workspace, need, c, bytes))
    return POLYMUL_EALIAS;
  const uint32_t nsub = depth == 1 ? 3 : depth == 2 ? 9 : 27;
  const uint32_t np = (uint32_t)(n >> depth);
  const uint64_t sub_words = batch * nsub * np;
  KaraParams64 K{};
  K.a = a; K.b = b; K.c = c;
  K.sa = (uint64_t*)workspace;
  K.sb = K.sa + sub_words;
  uint64_t* sc = K.sb + sub_words;
  K.sc = sc;
  K.nprod = batch; K.n = (uint32_t)n; K.np = np; K.depth = depth; K.nsub = nsub; K.L = 1;
  K.mods[0] = make_mod64(q, limbs64(&q, 1));
  const uint64_t blocks = (batch * np + 255) / 256;
  if (blocks > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  st = kara_split(K, depth, blocks, stream);
  if (st != POLYMUL_OK) return st;
  // the sub-products: batch * nsub products of degree bound n' (K-streamed, 64-bit words).
  // The streaming kernel runs whole rounds of its workgroups (one per CU at 8 limbs,
  // two at 4); when the blocks fill the last round poorly their K range is cut into
  // runs, whose residues a second kernel adds, if that takes fewer rounds per block.
  const int Ls = limbs64(&q, 1);
  StreamParams SP;
  uint32_t lds;
  st = fill_stream(SP, K.sa, K.sb, sc, np, &q, 1, 1, 0, batch * nsub, Ls, &lds, false, nsub);
  if (st != POLYMUL_OK) return st;
  const uint64_t sblocks = batch * nsub * SP.ublocks;
  const uint64_t per_round = (uint64_t)device_cus() * (Ls == 4 ? 2 : 1);
  uint32_t runs = 1;
  double best = (double)((sblocks + per_round - 1) / per_round);
  const uint32_t runs_max = g_kara_runs_max.load(std::memory_order_relaxed);
  for (uint32_t k = 2; k <= runs_max && k <= SP.nchunks; k *= 2) {
    const double rounds = (double)((sblocks * k + per_round - 1) / per_round) / k;
    if (rounds < best - 1e-9) { best = rounds; runs = k; }
  }
  if (runs > 1) {
    SP.kparts = runs;
    SP.part_ws = sc + sub_words;  // runs * sub_words words after the sub-products
  }
  st = Ls == 4 ? launch_stream_L<4, uint64_t, 2>(SP, lds, stream) : launch_stream_L<8, uint64_t, 1>(SP, lds, stream);
  if (st != POLYMUL_OK) return st;
  if (runs > 1) {
    hipLaunchKernelGGL(split_sum64_kernel, dim3((uint32_t)((sub_words + 255) / 256)), dim3(256), 0, stream,
                       (const uint64_t*)SP.part_ws, sc, sub_words, runs, q);
    st = launch_status();
    if (st != POLYMUL_OK) return st;
  }
  return kara_combine(K, depth, blocks, stream);
}

polymul_status polymul_negacyclic_rns_karatsuba(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n,
                                                const uint32_t* q, uint32_t L, uint64_t batch, uint32_t depth,
                                                void* workspace, uint64_t workspace_bytes, hipStream_t stream) {
  if (!is_pow2(n) || n > 65536 || L == 0 || L > 16) return POLYMUL_EINVAL;
  if (depth == 0) {
    depth = kara_depth_for(n, batch * L, false);
    if (depth == 0) return polymul_negacyclic_rns(a, b, c, n, q, L, batch, stream);
  }
  uint64_t need, bytes;
  polymul_status st = check_rns_karatsuba(a, b, c, n, q, L, batch, depth, &need, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  if (!workspace || ((uintptr_t)workspace & 15) || workspace_bytes < need) return POLYMUL_EINVAL;
  if (overlaps(workspace, need, a, bytes) || overlaps(workspace, need, b, bytes) || overlaps(workspace, need, c, bytes))
    return POLYMUL_EALIAS;
  return run_rns_karatsuba(a, b, c, n, q, L, batch, depth, workspace, stream);
}

polymul_status polymul_negacyclic_rns_karatsuba_noalloc(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                                        uint64_t n, const uint32_t* q, uint32_t L, uint64_t batch,
                                                        uint32_t depth, hipStream_t stream) {
  if (!is_pow2(n) || n > 65536 || L == 0 || L > 16) return POLYMUL_EINVAL;
  if (depth == 0) {
    depth = kara_depth_for(n, batch * L, false);
    if (depth == 0) return polymul_negacyclic_rns(a, b, c, n, q, L, batch, stream);
  }
  uint64_t need, bytes;
  polymul_status st = check_rns_karatsuba(a, b, c, n, q, L, batch, depth, &need, &bytes);
  if (st != POLYMUL_OK || batch == 0) return st;
  if (need > POLYMUL_NOALLOC_SCRATCH_BYTES) {
    if (log_enabled())
      fprintf(stderr, "polymul: the call needs %llu bytes of scratch, the library holds %llu\n",
              (unsigned long long)need, (unsigned long long)POLYMUL_NOALLOC_SCRATCH_BYTES);
    return POLYMUL_ESCRATCH;
  }
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != POLYMUL_OK) return st;
  return run_rns_karatsuba(a, b, c, n, q, L, batch, depth, ws, stream);
}

polymul_status polymul_tune_set(uint64_t n, uint32_t L, uint32_t t) {
  if (!is_pow2(n) || n > 65536 || L < 1 || L > 4) return POLYMUL_EINVAL;
  if (t != 0 && !tile_ok((uint32_t)n, t)) return POLYMUL_EINVAL;
  if (t != 0) {
    // the geometry must fit in LDS at the largest slot count
    const Geometry32 g = geometry32((uint32_t)n, t);
    if ((uint64_t)g.slots * (uint32_t)L * (g.a_plane + g.b_plane) > kMaxLds) return POLYMUL_EUNSUPPORTED;
  }
  g_tile[ilog2(n)][L].store(t, std::memory_order_relaxed);
  return POLYMUL_OK;
}

polymul_status polymul_tune_param_set(uint32_t param, uint64_t value) {
  switch (param) {
    case POLYMUL_TUNE_PLAN_SHARE_PCT:
      if (value < 10 || value > 1000) return POLYMUL_EINVAL;
      g_plan_share_pct.store((uint32_t)value, std::memory_order_relaxed);
      return POLYMUL_OK;
    case POLYMUL_TUNE_PLAN_STREAM_PCT:
      if (value < 50 || value > 400) return POLYMUL_EINVAL;
      g_plan_stream_pct.store((uint32_t)value, std::memory_order_relaxed);
      return POLYMUL_OK;
    case POLYMUL_TUNE_U64_KARATSUBA_RUNS:
      if (value != 1 && value != 2 && value != 4) return POLYMUL_EINVAL;
      g_kara_runs_max.store((uint32_t)value, std::memory_order_relaxed);
      return POLYMUL_OK;
  }
  return POLYMUL_EINVAL;
}

polymul_status polymul_tune_set_karatsuba(uint64_t n, uint64_t products, uint32_t elem_bytes, uint32_t depth) {
  if (!is_pow2(n) || n > 65536 || products == 0 || (elem_bytes != 4 && elem_bytes != 8)) return POLYMUL_EINVAL;
  if (depth != kNotTuned && (depth > 3 || (depth > 0 && (n >> depth) < 4))) return POLYMUL_EINVAL;
  (elem_bytes == 8 ? g_kara64_depth : g_kara_depth)[ilog2(n)][ilog2_floor(products)].store(
      depth, std::memory_order_relaxed);
  return POLYMUL_OK;
}

polymul_status polymul_tune_get_karatsuba(uint64_t n, uint64_t products, uint32_t elem_bytes, uint32_t* depth) {
  if (!is_pow2(n) || n > 65536 || products == 0 || (elem_bytes != 4 && elem_bytes != 8) || !depth)
    return POLYMUL_EINVAL;
  *depth = kara_depth_for(n, products, elem_bytes == 8);
  return POLYMUL_OK;
}

polymul_status polymul_tune_param_get(uint32_t param, uint64_t* value) {
  if (!value) return POLYMUL_EINVAL;
  switch (param) {
    case POLYMUL_TUNE_PLAN_SHARE_PCT: *value = g_plan_share_pct.load(std::memory_order_relaxed); return POLYMUL_OK;
    case POLYMUL_TUNE_PLAN_STREAM_PCT: *value = g_plan_stream_pct.load(std::memory_order_relaxed); return POLYMUL_OK;
    case POLYMUL_TUNE_U64_KARATSUBA_RUNS: *value = g_kara_runs_max.load(std::memory_order_relaxed); return POLYMUL_OK;
  }
  return POLYMUL_EINVAL;
}

polymul_status polymul_tune_get(uint64_t n, uint32_t L, uint32_t* t) {
  if (!is_pow2(n) || n > 65536 || L < 1 || L > 4 || !t) return POLYMUL_EINVAL;
  *t = tile_for((uint32_t)n, (int)L);
  return POLYMUL_OK;
}

}  // extern "C"
