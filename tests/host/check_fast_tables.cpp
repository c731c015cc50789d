// Host-side checks of the register-phase kernel's tables (built by
// paper_2601_01903_amd/csrc/fsi_tables.cpp), run on the CPU by
// tests/test_host_tables.py. Prints "ok" or the first violation.
#include <cstdio>
#include <map>
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
  // every (d, l): tables build; each canonical output's slots (j2 = 0 ..
  // |S_H2|; whole instances: j2 = 0) decode from the metadata word to its
  // own S_L, S_H1 and Y offset; distinct (S_L, S_H1, s_H2, j2) take distinct
  // slots; every read stays inside Y
  for (int l = 1; l <= 4; ++l)
    for (int d = 11; d <= 30; ++d) {
      const int kb = fast_block_bits(d, l), h = d - 11;
      CHECK(kb >= 0 && kb <= h, "d=%d l=%d: no block size", d, l);
      if (kb < 0) continue;
      const int slots = fast_output_slots(d, l);
      const bool blocked = kb < h;
      if (blocked)
        CHECK(positions_needed(l, h) > np_order(l) || h > 32 - meta_shift(l),
              "d=%d l=%d: blocked although the outputs fit", d, l);
      ClassHost C;
      FastClassHost F;
      std::string e = build_class(d, l, 11, ALGO_FUSED, 0, 0, &C);
      CHECK(e.empty(), "d=%d l=%d build_class: %s", d, l, e.c_str());
      if (!e.empty()) continue;
      e = build_fast_class(C, &F);
      CHECK(e.empty(), "d=%d l=%d build_fast_class: %s", d, l, e.c_str());
      if (!e.empty()) continue;
      const int npos = slots / 2;
      CHECK(F.kb == kb, "d=%d l=%d: block bits %d, expected %d", d, l, F.kb, kb);
      CHECK(slots % 2 == 0 && npos == (blocked ? positions_blocked(l, kb) : positions_needed(l, h)),
            "d=%d l=%d: %d slots", d, l, slots);
      CHECK(npos <= np_order(l), "d=%d l=%d: %d positions, kernel unrolls %d", d, l, npos, np_order(l));
      CHECK(F.nkk >= 2 && F.nkk <= 2 * npos && F.nkk % 2 == 0, "d=%d l=%d: %d slots in use", d, l, F.nkk);
      const uint32_t omask = (1u << F.mshift) - 1u;
      const uint32_t lowhigh = (uint32_t)((1ull << kb) - 1);
      std::map<int, uint64_t> owner;   // slot -> (S_L, S_H1, s_H2, j2)
      for (size_t k = 0; k < C.out_masks.size(); ++k) {
        const uint32_t S = C.out_masks[k];
        const uint32_t SL = S & 0x7FFu, SH = S >> 11;
        const uint32_t S1 = SH & lowhigh, S2 = blocked ? SH >> kb : 0u;
        CHECK(F.osh2[k] == S2, "d=%d l=%d output %zu: S_H2 %u", d, l, k, F.osh2[k]);
        const int sL = cpop((int)SL), s1 = cpop((int)S1), s2 = cpop((int)S2);
        const int rk = rank_colex(SL);
        for (int j2 = 0; j2 <= l; ++j2) {
          const int jj = j2 < s2 ? j2 : s2;
          const int p = F.pidx[k * (size_t)(l + 1) + j2];
          CHECK(p >= 0 && p < F.nkk * kFastThreads, "d=%d l=%d output %zu: slot out of range", d, l, k);
          if (p < 0 || p >= F.nkk * kFastThreads) continue;
          const uint64_t key = (uint64_t)SL | ((uint64_t)S1 << 11) | ((uint64_t)(s2 * 8 + jj) << 40);
          auto it = owner.find(p);
          if (it == owner.end()) owner[p] = key;
          else CHECK(it->second == key, "d=%d l=%d: slot %d shared by two partial sums", d, l, p);
          const int kk = p / kFastThreads, t = p % kFastThreads;
          const int pos = kk / 2, el = kk % 2, w = t / 64;
          const uint32_t m = F.meta[(size_t)t * kFastMetaStride + pos];
          CHECK((m >> F.mshift) == S1, "d=%d l=%d output %zu: S_H1 decodes wrongly", d, l, k);
          CHECK(rk % 2 == el, "d=%d l=%d output %zu: rank parity %d in element %d", d, l, k, rk, el);
          const int sH = s1 + s2;
          const uint32_t want =
              (uint32_t)(ybase(l, sL) + (sH * (sH + 1) / 2 + jj) * nrp(sL) + rk - el) * 8u;
          CHECK((m & omask) == want, "d=%d l=%d output %zu: Y offset decodes wrongly", d, l, k);
          CHECK(want % 16 == 0, "d=%d l=%d output %zu: read not 16-byte aligned", d, l, k);
          const uint32_t gs = F.gs8[(size_t)pos * 4 + w];
          CHECK(gs == (uint32_t)nrp(sL) * 8u, "d=%d l=%d: j stride of position %d wave %d", d, l, pos, w);
        }
      }
      // every run's read (real or dummy) stays inside Y for every j1 <= |S_H1|
      for (int t = 0; t < kFastThreads; ++t)
        for (int pos = 0; pos < kRuns; ++pos) {
          const uint32_t m = F.meta[(size_t)t * kFastMetaStride + pos];
          const uint32_t gs = F.gs8[(size_t)pos * 4 + t / 64];
          const int s1 = cpop((int)(m >> F.mshift));
          CHECK((m & omask) % 16 == 0 && (m & omask) + (uint32_t)s1 * gs + 16 <= (uint32_t)ysize(l) * 8u,
                "d=%d l=%d thread %d position %d: read out of Y", d, l, t, pos);
        }
      CHECK((int)F.lam.size() == (F.h + 1) * lamblock(l), "d=%d l=%d: weight block size", d, l);
    }
  std::printf(fails ? "failures: %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
