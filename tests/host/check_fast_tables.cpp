// Host-side checks of the register-phase kernel's tables (built by
// paper_2601_01903_amd/csrc/fsi_tables.cpp), run on the CPU by
// tests/test_host_tables.py. Prints "ok" or the first violation.
#include <cstdio>
#include <set>
#include <string>
#include <vector>

#include "fsi_internal.h"
#include "fsi_kernels.h"
#include "fsi_tile11.h"

using namespace fsi;
using namespace fsi::t11;

static int fails = 0;
#define CHECK(c, ...)                      \
  do {                                     \
    if (!(c)) {                            \
      if (fails++ < 10) {                  \
        std::printf("FAIL: " __VA_ARGS__); \
        std::printf("\n");                 \
      }                                    \
    }                                      \
  } while (0)

int main() {
  // unit order of phase C: a permutation of the units, each wave's units at
  // or above its compile-time bound on |sigma_AB|
  for (int L = 1; L <= 4; ++L) {
    const UnitOrder o = mk_unit_order(L);
    std::set<int> seen;
    int last_pop = -1;
    for (int t = 0; t < n3(L); ++t) {
      seen.insert(o.v[t]);
      int pop = -1;
      for (int sb = 0; sb < NB; ++sb)
        for (int sa = 0; sa < NA; ++sa)
          if (unit_index(L, sa, sb) == o.v[t]) pop = cpop(sa) + cpop(sb);
      CHECK(pop >= 0, "L=%d thread %d: not a unit", L, t);
      CHECK(pop >= last_pop, "L=%d: units not in order of |sigma_AB|", L);
      CHECK(pop >= o.kmin[t / 64], "L=%d thread %d: |sigma_AB| %d below the wave bound %d", L, t,
            pop, o.kmin[t / 64]);
      last_pop = pop;
    }
    CHECK((int)seen.size() == n3(L), "L=%d: unit order is not a permutation", L);
  }
  // every eligible (d, l): tables build, each canonical output decodes to its
  // own mask from the metadata word, and the slots are a bijection
  for (int l = 1; l <= 4; ++l)
    for (int d = 11; d <= 30; ++d) {
      const int slots = fast_output_slots(d, l);
      const bool eligible = slots >= 0 && d - 11 <= fast_max_high_bits(l);
      if (!eligible) continue;
      ClassHost C;
      FastClassHost F;
      std::string e = build_class(d, l, 11, ALGO_FUSED, 0, 0, &C);
      CHECK(e.empty(), "d=%d l=%d build_class: %s", d, l, e.c_str());
      if (!e.empty()) continue;
      e = build_fast_class(C, &F);
      CHECK(e.empty(), "d=%d l=%d build_fast_class: %s", d, l, e.c_str());
      if (!e.empty()) continue;
      CHECK(F.ngroups == (slots + kFastKmax - 1) / kFastKmax, "d=%d l=%d: %d output groups", d, l,
            F.ngroups);
      int sum = 0;
      for (int g = 0; g < F.ngroups; ++g) {
        CHECK(F.gnkk[g] >= 1 && F.gnkk[g] <= kFastKmax, "d=%d l=%d group %d: %d slots", d, l, g,
              F.gnkk[g]);
        sum += F.gnkk[g];
      }
      CHECK(sum == slots, "d=%d l=%d: %d slots over the groups, %d needed", d, l, sum, slots);
      const uint32_t omask = (1u << F.mshift) - 1u;
      std::set<int> used;
      for (size_t k = 0; k < C.out_masks.size(); ++k) {
        const int p = F.pidx[k], g = F.pgroup[k];
        CHECK(g >= 0 && g < F.ngroups, "d=%d l=%d output %zu: group out of range", d, l, k);
        if (g < 0 || g >= F.ngroups) continue;
        CHECK(p >= 0 && p < F.gnkk[g] * kFastThreads, "d=%d l=%d output %zu: slot out of range", d, l, k);
        CHECK(used.insert(g * kFastKmax * kFastThreads + p).second, "d=%d l=%d: slot used twice", d, l);
        const int kk = p / kFastThreads, t = p % kFastThreads;
        const uint32_t m = F.meta[((size_t)g * kFastThreads + t) * kFastMetaStride + kk];
        const uint32_t S = C.out_masks[k];
        const uint32_t SL = S & 0x7FFu, SH = S >> 11;
        CHECK((m >> F.mshift) == SH, "d=%d l=%d output %zu: S_H decodes wrongly", d, l, k);
        // the Y offset at j = 0 addresses (S_L, s_H): its group base plus the
        // rank of S_L, in units of the group's row count
        const int sL = cpop((int)SL), sH = cpop((int)SH);
        const uint32_t want = (uint32_t)(ybase(l, sL) + (sH * (sH + 1) / 2) * cbinom(B, sL) +
                                         rank_colex(SL)) * 8u;
        CHECK((m & omask) == want, "d=%d l=%d output %zu: Y offset decodes wrongly", d, l, k);
        const uint32_t gs = F.gs8[(size_t)g * kFastMetaStride + kk];
        CHECK(gs == (uint32_t)cbinom(B, sL) * 8u, "d=%d l=%d: j stride of slot %d", d, l, kk);
        CHECK((m & omask) + (uint32_t)sH * gs < (uint32_t)ysize(l) * 8u,
              "d=%d l=%d output %zu: Y offset past the tile's results", d, l, k);
      }
      CHECK((int)F.lam.size() == (F.h + 1) * lamblock(l), "d=%d l=%d: weight block size", d, l);
    }
  std::printf(fails ? "failures: %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
