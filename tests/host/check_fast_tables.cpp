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
  // phase-C thread map: every unit once in the whole-tree waves, or (heavy
  // units) on the same lane of the two half-tree waves; each wave's units
  // within its compile-time bounds on |sigma_AB|; heavy units have
  // |sigma_AB| <= L - 2
  for (int L = 1; L <= 4; ++L) {
    const UnitOrder o = mk_unit_order(L);
    int half[2] = {-1, -1};
    for (int w = 0; w < NT / 64; ++w) {
      CHECK(o.part[w] >= 0 && o.part[w] <= 2, "L=%d wave %d: part %d", L, w, o.part[w]);
      if (o.part[w] < 2) half[o.part[w]] = w;
    }
    CHECK(half[0] >= 0 && half[1] >= 0, "L=%d: the two half-tree waves are missing", L);
    if (half[0] < 0 || half[1] < 0) continue;
    std::vector<int> count(n3(L), 0);
    int last_pop = -1;
    for (int t = 0; t < NT; ++t) {
      const int w = t / 64, u = o.v[t];
      if (u < 0) continue;
      CHECK(u < n3(L), "L=%d thread %d: unit %d out of range", L, t, u);
      if (u >= n3(L)) continue;
      int pop = -1;
      for (int sb = 0; sb < NB; ++sb)
        for (int sa = 0; sa < NA; ++sa)
          if (unit_index(L, sa, sb) == u) pop = cpop(sa) + cpop(sb);
      CHECK(pop >= o.kmin[w] && pop <= o.kmax[w],
            "L=%d thread %d: |sigma_AB| %d outside the wave bounds [%d, %d]", L, t, pop,
            o.kmin[w], o.kmax[w]);
      if (o.part[w] < 2) {
        CHECK(pop <= L - 2, "L=%d thread %d: split unit with |sigma_AB| %d", L, t, pop);
        const int partner = 64 * half[1 - o.part[w]] + t % 64;
        CHECK(o.v[partner] == u, "L=%d thread %d: half without its partner", L, t);
        if (o.part[w] == 0) ++count[u];
      } else {
        CHECK(pop > L - 2, "L=%d thread %d: heavy unit not split", L, t);
        ++count[u];
      }
    }
    // whole-tree units in order of |sigma_AB| across the two waves
    for (int q = 0; q < 2; ++q)
      for (int w = 0; w < NT / 64; ++w)
        if (o.part[w] == 2 && ((q == 0) == (w == kCWaveR0)))
          for (int t = 64 * w; t < 64 * w + 64; ++t) {
            if (o.v[t] < 0) continue;
            int pop = -1;
            for (int sb = 0; sb < NB; ++sb)
              for (int sa = 0; sa < NA; ++sa)
                if (unit_index(L, sa, sb) == o.v[t]) pop = cpop(sa) + cpop(sb);
            CHECK(pop >= last_pop, "L=%d: units not in order of |sigma_AB|", L);
            last_pop = pop;
          }
    for (int u = 0; u < n3(L); ++u) CHECK(count[u] == 1, "L=%d unit %d taken %d times", L, u, count[u]);
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
      // runs of two outputs: 2 slots per gather position, kRuns positions per group
      const int npos = slots / 2;
      CHECK(slots % 2 == 0 && npos == positions_needed(l, d - 11), "d=%d l=%d: %d slots", d, l, slots);
      CHECK(F.ngroups == (npos + kRuns - 1) / kRuns, "d=%d l=%d: %d output groups", d, l, F.ngroups);
      CHECK(l == 4 || npos <= np_order(l), "d=%d l=%d: %d positions, kernel unrolls %d", d, l, npos,
            np_order(l));
      for (int g = 0; g < F.ngroups; ++g)
        CHECK(F.gnkk[g] >= 2 && F.gnkk[g] <= 2 * kRuns && F.gnkk[g] % 2 == 0,
              "d=%d l=%d group %d: %d slots", d, l, g, F.gnkk[g]);
      const uint32_t omask = (1u << F.mshift) - 1u;
      std::set<int> used;
      for (size_t k = 0; k < C.out_masks.size(); ++k) {
        const int p = F.pidx[k], g = F.pgroup[k];
        CHECK(g >= 0 && g < F.ngroups, "d=%d l=%d output %zu: group out of range", d, l, k);
        if (g < 0 || g >= F.ngroups) continue;
        CHECK(p >= 0 && p < F.gnkk[g] * kFastThreads, "d=%d l=%d output %zu: slot out of range", d, l, k);
        CHECK(used.insert(g * kFastKmax * kFastThreads + p).second, "d=%d l=%d: slot used twice", d, l);
        const int kk = p / kFastThreads, t = p % kFastThreads;
        const int pos = kk / 2, e = kk % 2, w = t / 64;
        const uint32_t m = F.meta[((size_t)g * kFastThreads + t) * kFastMetaStride + pos];
        const uint32_t S = C.out_masks[k];
        const uint32_t SL = S & 0x7FFu, SH = S >> 11;
        CHECK((m >> F.mshift) == SH, "d=%d l=%d output %zu: S_H decodes wrongly", d, l, k);
        // the run's Y offset at j = 0 addresses (S_L of the even rank, s_H):
        // group base plus the pair's first rank; this output is element e
        const int sL = cpop((int)SL), sH = cpop((int)SH);
        const int rk = rank_colex(SL);
        CHECK(rk % 2 == e, "d=%d l=%d output %zu: rank parity %d in element %d", d, l, k, rk, e);
        const uint32_t want =
            (uint32_t)(ybase(l, sL) + (sH * (sH + 1) / 2) * nrp(sL) + rk - e) * 8u;
        CHECK((m & omask) == want, "d=%d l=%d output %zu: Y offset decodes wrongly", d, l, k);
        CHECK(want % 16 == 0, "d=%d l=%d output %zu: read not 16-byte aligned", d, l, k);
        const uint32_t gs = F.gs8[((size_t)g * kRuns + pos) * 4 + w];
        CHECK(gs == (uint32_t)nrp(sL) * 8u, "d=%d l=%d: j stride of position %d wave %d", d, l, pos, w);
        CHECK((m & omask) + (uint32_t)sH * gs + 16 <= (uint32_t)ysize(l) * 8u,
              "d=%d l=%d output %zu: Y read past the tile's results", d, l, k);
      }
      // every run's read (real or dummy) stays inside Y for every j
      for (int g = 0; g < F.ngroups; ++g)
        for (int t = 0; t < kFastThreads; ++t)
          for (int pos = 0; pos < kRuns; ++pos) {
            const uint32_t m = F.meta[((size_t)g * kFastThreads + t) * kFastMetaStride + pos];
            const uint32_t gs = F.gs8[((size_t)g * kRuns + pos) * 4 + t / 64];
            const int sH = cpop((int)(m >> F.mshift));
            CHECK((m & omask) % 16 == 0 && (m & omask) + (uint32_t)sH * gs + 16 <= (uint32_t)ysize(l) * 8u,
                  "d=%d l=%d group %d thread %d position %d: read out of Y", d, l, g, t, pos);
          }
      CHECK((int)F.lam.size() == (F.h + 1) * lamblock(l), "d=%d l=%d: weight block size", d, l);
    }
  std::printf(fails ? "failures: %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
