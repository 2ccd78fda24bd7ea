// Host-side construction of the 64-bit-modulus constants.
#pragma once
#include "pm_common.h"
#include "pm_wide.h"

namespace pm {

inline ModQ64 make_mod64(uint64_t q, int L) {
  ModQ64 m{};
  m.q = q;
  const uint64_t top = limb_top(L);
  m.thr = top;
  m.sh = (uint32_t)__builtin_clzll(q);
  m.d = q << m.sh;
  const unsigned __int128 all = ~(unsigned __int128)0;
  m.v = (uint64_t)(all / m.d - ((unsigned __int128)1 << 64));
  unsigned __int128 pw = 1 % q;
  for (int s = 0; s < 16; ++s) {
    m.r[s] = (uint64_t)pw;
    pw = (pw * 256) % q;
  }
  const int groups = (2 * L - 1 + 3) / 4;
  unsigned __int128 rsum = 0;
  for (int j = 0; j < groups; ++j) rsum = (rsum + m.r[4 * j]) % q;
  m.foff = (uint64_t)((((unsigned __int128)1 << 56) % q) * rsum % q);
  return m;
}

}  // namespace pm
