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
  return m;
}

}  // namespace pm
