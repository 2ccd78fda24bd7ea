// C-ABI of the GPU library: argument checks, launch geometry, dispatch.
#include <mutex>
#include <new>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/polymul.h"
#include "pm_common.h"
#include "pm_mfma32.h"
#include "pm_plain.h"
#include "pm_stream.h"
#include "pm_wide_host.h"

using namespace pm;

namespace {

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

polymul_status launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? POLYMUL_OK : POLYMUL_EDEVICE;
}

// ----------------------------------------------------------- MFMA, 32-bit q
struct Geometry32 {
  uint32_t t, r, spd, rowlen, tz, tu, U, slots, a_plane, b_rows, b_rowstride, b_plane, E;
};

// Degree split n = t * r (Sec. 2.5): t is the Toeplitz tile side.
Geometry32 geometry32(uint32_t n, int L) {
  Geometry32 g{};
  if (n <= 32) { g.t = n; g.r = 1; }
  else if (n <= 1024) { g.t = 32; g.r = n / 32; }
  else { g.t = 64; g.r = n / 64; }
  g.spd = g.t >= 32 ? g.t / 32 : 1;
  g.rowlen = 32 * g.spd;
  g.tz = (g.t + 31) / 32;
  g.tu = (g.r + 31) / 32;
  g.U = g.tz * g.tu;
  g.slots = g.U >= 4 ? 1 : 4 / g.U;
  g.E = (g.r - 1) * g.t + 32 * g.tz - 1;
  g.a_plane = (g.E + g.rowlen + 4 + 15) & ~15u;
  uint32_t utiles = g.U >= 4 ? 4 / g.tz : g.tu;
  if (utiles == 0) utiles = 1;
  g.b_rows = 32 * utiles + g.r - 1;
  g.b_rowstride = ((g.rowlen / 16) & 1) ? g.rowlen : g.rowlen + 16;
  g.b_plane = (g.b_rows * g.b_rowstride + 15) & ~15u;
  (void)L;
  return g;
}

constexpr uint32_t kMaxLds = 160 * 1024;

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

template <int L, bool SMALL>
polymul_status launch_mfma32_L(Mfma32Params& P, const Geometry32& g, hipStream_t s) {
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute((const void*)mfma32_group_kernel<L, SMALL>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
  });
  if (attr_err != hipSuccess) return POLYMUL_EDEVICE;
  P.slot_bytes = L * (g.a_plane + g.b_plane);
  const uint32_t lds = P.slots * P.slot_bytes;
  if (lds > kMaxLds) return POLYMUL_EUNSUPPORTED;
  const uint64_t units = P.nprod << P.log2U;
  const uint64_t groups = (units + 3) / 4;
  // Persistent grid: as many workgroups as fit at once (LDS- and register-bound).
  uint64_t blocks = groups;
  if (blocks > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  hipLaunchKernelGGL((mfma32_group_kernel<L, SMALL>), dim3((uint32_t)blocks), dim3(kThreads), lds, s, P);
  return launch_status();
}

// nprod products (i -> global (i/lc)*nq_total + l0 + i%lc) with moduli qs[0..lc).
template <typename W>
polymul_status run_stream(const W* a, const W* b, W* c, uint32_t n, const uint64_t* qs, uint32_t lc,
                          uint32_t nq_total, uint32_t l0, uint64_t nprod, hipStream_t s);

polymul_status run_mfma32(const uint32_t* a, const uint32_t* b, uint32_t* c, uint32_t n, const uint32_t* qs,
                          uint32_t lc, uint32_t nq_total, uint32_t l0, uint64_t nprod, hipStream_t s) {
  if (n > 8192) {
    // degree too large for both operands in LDS: K-streaming kernel, moduli in chunks of kMaxQS
    uint64_t q64[kMaxQ];
    for (uint32_t i = 0; i < lc; ++i) q64[i] = qs[i];
    if (lc <= (uint32_t)kMaxQS) return run_stream<uint32_t>(a, b, c, n, q64, lc, nq_total, l0, nprod, s);
    // split the channel range (nprod = batch * lc)
    const uint64_t batch = nprod / lc;
    for (uint32_t c0 = 0; c0 < lc; c0 += kMaxQS) {
      const uint32_t cc = lc - c0 < (uint32_t)kMaxQS ? lc - c0 : (uint32_t)kMaxQS;
      polymul_status st = run_stream<uint32_t>(a, b, c, n, q64 + c0, cc, nq_total, l0 + c0, batch * cc, s);
      if (st != POLYMUL_OK) return st;
    }
    return POLYMUL_OK;
  }
  int L = 1;
  for (uint32_t i = 0; i < lc; ++i) L = L > limbs_for_q32(qs[i]) ? L : limbs_for_q32(qs[i]);
  if (L < 2) L = 2;
  Geometry32 g = geometry32(n, L);
  Mfma32Params P{};
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
  P.lc = lc; P.nq_total = nq_total; P.l0 = l0;
  // Epilogue choice: the one-reduction form needs sum_s P_s * n * 2^14 * |rcent_s| < 2^62,
  // P_s = number of limb pairs (i, j) with i + j = s.
  bool fast = true;
  for (uint32_t i = 0; i < lc; ++i) {
    P.mods[i] = make_mod32(qs[i], L);
    unsigned __int128 bound = 0;
    uint64_t pw = 1 % qs[i];
    for (int s = 0; s < 2 * L - 1; ++s) {
      int64_t c = (int64_t)pw;
      if (pw > qs[i] / 2) c -= (int64_t)qs[i];
      P.rcent[i][s] = (int32_t)c;
      uint64_t pairs = (uint64_t)((s < L ? s : 2 * L - 2 - s) + 1);
      bound += (unsigned __int128)pairs * n * 16384u * (uint64_t)(c < 0 ? -c : c);
      pw = (pw * 256) % qs[i];
    }
    if (bound >= ((unsigned __int128)1 << 62)) fast = false;
  }
  P.fast_epilogue = fast ? 1u : 0u;
  const bool small = n < 4;
  switch (L) {
    case 2: return small ? launch_mfma32_L<2, true>(P, g, s) : launch_mfma32_L<2, false>(P, g, s);
    case 3: return small ? launch_mfma32_L<3, true>(P, g, s) : launch_mfma32_L<3, false>(P, g, s);
    default: return small ? launch_mfma32_L<4, true>(P, g, s) : launch_mfma32_L<4, false>(P, g, s);
  }
}

// ------------------------------------------------------- streaming kernel
template <int L, typename W, int WPE>
polymul_status launch_stream_L(const StreamParams& P, uint32_t lds, uint64_t blocks, hipStream_t s) {
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute((const void*)stream_kernel<L, W, WPE>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
  });
  if (attr_err != hipSuccess) return POLYMUL_EDEVICE;
  hipLaunchKernelGGL((stream_kernel<L, W, WPE>), dim3((uint32_t)blocks), dim3(kStreamThreads), lds, s, P);
  return launch_status();
}

// nprod products of degree bound n (i -> global (i/lc)*nq_total + l0 + i%lc), moduli qs[0..lc).
template <typename W>
polymul_status run_stream(const W* a, const W* b, W* c, uint32_t n, const uint64_t* qs, uint32_t lc,
                          uint32_t nq_total, uint32_t l0, uint64_t nprod, hipStream_t s) {
  int L = 1;
  for (uint32_t i = 0; i < lc; ++i) {
    const int li = limbs_for_q64(qs[i]);
    L = L > li ? L : li;
  }
  if (L < 2) L = 2;
  if (sizeof(W) == 4 && L > 4) return POLYMUL_EINVAL;
  L = L <= 4 ? 4 : 8;  // two instantiations: up to 4 and up to 8 limbs
  StreamParams P{};
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
  const uint32_t kflush = L <= 4 ? 16384u : 8192u;  // K values per exact int32 class sum
  uint32_t fe = kflush / (P.dc * P.t);
  P.flush_every = fe < 1 ? 1 : fe;
  P.a_win = ((P.dc - 1) * P.t + 32 * P.tz + P.rowlen + 4 + 15) & ~15u;
  P.lds_b = 2u * (uint32_t)L * P.a_win;
  const uint32_t lds = P.lds_b + (uint32_t)L * kRing * P.rs;
  if (lds > kMaxLds) return POLYMUL_EUNSUPPORTED;
  P.lc = lc; P.nq_total = nq_total; P.l0 = l0;
  for (uint32_t i = 0; i < lc; ++i) P.mods[i] = make_mod64(qs[i], L);
  const uint64_t blocks = nprod * P.ublocks;
  if (blocks > 0x7FFFFFFFull) return POLYMUL_EUNSUPPORTED;
  if (L == 4) return launch_stream_L<4, W, 2>(P, lds, blocks, s);
  return launch_stream_L<8, W, 1>(P, lds, blocks, s);
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
    uint32_t lc = L - l0 < (uint32_t)kMaxQ ? L - l0 : (uint32_t)kMaxQ;
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
  uint64_t blocks = batch * P.blocks_per_prod;
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

struct polymul_plan {
  int unused;
};

polymul_status polymul_plan_create(polymul_plan** plan, const polymul_group* groups, uint32_t ngroups,
                                   uint32_t flags) {
  (void)groups; (void)ngroups; (void)flags;
  if (!plan) return POLYMUL_EINVAL;
  *plan = nullptr;
  return POLYMUL_EUNSUPPORTED;
}
polymul_status polymul_plan_execute(polymul_plan* plan, hipStream_t stream) {
  (void)stream;
  return plan ? POLYMUL_EUNSUPPORTED : POLYMUL_EINVAL;
}
polymul_status polymul_plan_destroy(polymul_plan* plan) {
  delete plan;
  return POLYMUL_OK;
}

}  // extern "C"
