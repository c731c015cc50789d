// Host-side plan tables for the FSI operator: exact weights, the counter
// state tables of the in-tile MPO sweep, the per-tile weight tables of the
// final core, and the output bookkeeping.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>

#include "../../include/fsi.h"
#include "fsi_internal.h"
#include "fsi_kernels.h"
#include "fsi_tile11.h"

namespace fsi {

namespace {

int64_t binom(int n, int k) {
  if (k < 0 || n < 0 || k > n) return 0;
  if (k > n - k) k = n - k;
  __int128 r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;  // exact at each step
  return (int64_t)r;
}

// FSI weight of Eq. 3 + Eq. 4: the coefficient of a(T) in E_S for |S| = s,
// |T| = t, T superset of S:
//   1                 if t == s      (the Moebius term a(S))
//   w(s, t) of Eq. 7  if t > l, s >= 1
//   0                 otherwise.
// w(s, t) = (-1)^(l-s) * s/(l+s) * C(l,s) * C(t-1,l) / C(t+l-1,l+s), whose
// numerator and denominator are exact 64-bit integers for d, l <= 30; the
// quotient is taken in binary128 (113-bit significand).
__float128 weight_fsi(int s, int t, int l) {
  if (t == s) return 1;
  if (!(t > l && s >= 1)) return 0;
  __int128 num = (__int128)s * binom(l, s) * binom(t - 1, l);
  __int128 den = (__int128)(l + s) * binom(t + l - 1, l + s);
  __float128 q = (__float128)num / (__float128)den;
  return ((l - s) & 1) ? -q : q;
}

// Bernoulli number B_j (B_1 = -1/2) from sum_{i=0}^{m} C(m+1, i) B_i = 0,
// in binary128; j <= 30 (B_30 is about 6e8, far inside its exact range).
__float128 bernoulli_q(int j) {
  __float128 B[kMaxD + 1];
  B[0] = 1;
  for (int m = 1; m <= j; ++m) {
    __float128 acc = 0;
    for (int i = 0; i < m; ++i) acc += (__float128)binom(m + 1, i) * B[i];
    B[m] = -acc / (__float128)(m + 1);
  }
  return B[j];
}

// W(s, t) of the plan's interaction index on the Moebius transform (the
// cardinal weights of Appendix A's indices; fsi.h lists them), for t >= s.
__float128 weight_q(int s, int t, int l, int index) {
  if (t < s) return 0;
  switch (index) {
    case FSI_INDEX_STII:
      if (s < l) return t == s ? 1 : 0;
      return (__float128)1 / (__float128)binom(t, l);
    case FSI_INDEX_SII:
      return (__float128)1 / (__float128)(t - s + 1);
    case FSI_INDEX_BII: {
      __float128 w = 1;
      for (int i = 0; i < t - s; ++i) w *= (__float128)0.5;
      return w;
    }
    case FSI_INDEX_KSII: {
      if (s == 0) return t == 0 ? 1 : 0;
      const int n = t - s;
      __float128 acc = 0;
      for (int j = 0; j <= std::min(l - s, n); ++j)
        acc += bernoulli_q(j) * (__float128)binom(n, j) / (__float128)(n - j + 1);
      return acc;
    }
    default:
      return weight_fsi(s, t, l);
  }
}

// Precontracted high-site weight (the Moebius cores of the h high sites
// composed into the final weight core, Sec. 4.5): for a tile whose raw high
// index U_H has popcount u, an output whose high part S_H gives
// q = |S_H union U_H|, and a low superset of popcount t_L:
//   lambda = sum_{m=0}^{h-q} C(h-q, m) (-1)^(q+m-u) W(s, t_L + q + m),
// i.e. the sum over all high supersets T_H of S_H union U_H of
// (-1)^(|T_H|-|U_H|) W(s, t_L + |T_H|).
__float128 lambda_q(int s, int tL, int q, int u, int h, int l, int index) {
  __float128 acc = 0;
  for (int m = 0; m <= h - q; ++m) {
    __float128 term = (__float128)binom(h - q, m) * weight_q(s, tL + q + m, l, index);
    acc += ((q + m - u) & 1) ? -term : term;
  }
  return acc;
}

int popc(uint64_t x) { return __builtin_popcountll(x); }

}  // namespace

double weight_full(int s, int t, int l, int index) { return (double)weight_q(s, t, l, index); }

int64_t num_outputs(int d, int l) {
  if (!(1 <= l && l <= d && d <= kMaxD)) return -1;
  int64_t m = 0;
  for (int s = 0; s <= l; ++s) m += binom(d, s);
  return m;
}

std::vector<uint32_t> canonical_masks(int d, int l) {
  // ascending popcount, then ascending mask value
  std::vector<uint32_t> out;
  for (int s = 0; s <= std::min(l, d); ++s) {
    if (s == 0) { out.push_back(0); continue; }
    // Gosper's hack enumerates same-popcount masks in ascending order
    uint64_t m = (1ull << s) - 1;
    const uint64_t lim = 1ull << d;
    while (m < lim) {
      out.push_back((uint32_t)m);
      uint64_t c = m & (~m + 1), r = m + c;
      m = (((r ^ m) >> 2) / c) | r;
    }
  }
  return out;
}

int64_t sweep_peak_entries(int b, int l) {
  // after k sites: sum_{s <= min(k,l)} C(k,s) (k-s+1) patterns, each holding
  // a suffix of 2^(b-k) inputs (Sec. 4.4, intermediate tensor with the
  // output prefix compressed to |sigma| <= l).
  int64_t peak = 0;
  for (int k = 0; k <= b; ++k) {
    int64_t p = 0;
    for (int s = 0; s <= std::min(k, l); ++s) p += binom(k, s) * (k - s + 1);
    peak = std::max(peak, p << (b - k));
  }
  return peak;
}

std::string build_class(int d, int l, int b, int algo, int index, int mobius_in, ClassHost* C) {
  if (!(1 <= l && l <= d && d <= kMaxD)) return "invalid (d, l)";
  if (!(1 <= b && b <= kMaxTileBits && b <= d)) return "invalid tile bits";
  const int h = d - b;
  C->d = d; C->l = l; C->b = b; C->h = h; C->algo = algo; C->mobius_in = mobius_in;
  if (mobius_in && algo != ALGO_FUSED) return "Moebius input needs the fused algorithm";
  C->M = (int)num_outputs(d, l);

  // ---- counter states of the in-tile sweep (Sec. 4.3 state space) ----
  // Site k (k = 1..b) consumes tile bit b-k (most significant first). After
  // site k a pattern is (sigma, t): sigma the output bits of the consumed
  // sites read as a k-bit number (first site most significant), s =
  // popcount(sigma) <= l, and t in [s, k] the running |T| counter.
  // Patterns are stored sigma-major (ascending), t-minor; each holds the
  // 2^(b-k) inputs of the unconsumed suffix.
  std::vector<uint32_t> sig_prev{0};
  std::vector<int32_t> base_prev{0};  // index of (sigma, t = s)
  C->step_off.assign(b + 1, 0);
  C->step_np.assign(b + 1, 0);
  C->step_np[0] = 1;
  C->pat.clear();
  int64_t lds = 1ll << b;
  for (int k = 1; k <= b; ++k) {
    C->step_off[k] = (int32_t)C->pat.size();
    std::vector<uint32_t> sig_next;
    std::vector<int32_t> base_next;
    int32_t np = 0;
    for (size_t i = 0; i < sig_prev.size(); ++i) {
      const uint32_t sg = sig_prev[i];
      const int s = popc(sg);
      const int32_t bp = base_prev[i];
      auto idx_in = [&](int t) { return bp + (t - s); };  // t in [s, k-1]
      for (int c = 0; c <= 1; ++c) {
        const int s2 = s + c;
        if (s2 > l) continue;
        sig_next.push_back((sg << 1) | (uint32_t)c);
        base_next.push_back(np);
        for (int t2 = s2; t2 <= k; ++t2) {
          int32_t src0 = -1, src1 = -1;  // (sigma, tau) = (c, 0) and (c, 1)
          if (c == 0 && t2 <= k - 1) src0 = idx_in(t2);   // tau = 0: t kept
          if (t2 - 1 >= s && t2 - 1 <= k - 1) src1 = idx_in(t2 - 1);  // tau = 1
          if (src0 >= 0xFFFF || src1 >= 0xFFFF) return "sweep table too large";
          C->pat.push_back((uint32_t)(src0 + 1) | ((uint32_t)(src1 + 1) << 16));
          ++np;
        }
      }
    }
    C->step_np[k] = np;
    lds = std::max<int64_t>(lds, (int64_t)np << (b - k));
    sig_prev.swap(sig_next);
    base_prev.swap(base_next);
  }
  C->lds_elems = (int)lds;
  C->nfinal = C->step_np[b];
  std::map<uint32_t, int32_t> final_base;  // S_L -> index of (S_L, t = s_L)
  for (size_t i = 0; i < sig_prev.size(); ++i) final_base[sig_prev[i]] = base_prev[i];

  // ---- slots of the per-tile partial results ----
  // fused:    (s_H, j_H), s_H in [0, min(l - s_L, h)], j_H in [0, s_H],
  //           slot = s_H (s_H + 1) / 2 + j_H   (j_H = |S_H & U_H|)
  // two-pass: s_H in [0, min(l - s_L, h)], slot = s_H
  auto nslot = [&](int sL) {
    const int top = std::min(l - sL, h);
    if (top < 0) return 0;
    return algo == ALGO_FUSED ? (top + 1) * (top + 2) / 2 : top + 1;
  };
  const std::vector<uint32_t> low_masks = canonical_masks(b, std::min(l, b));
  std::map<uint32_t, int32_t> yoff;
  C->ytab.clear();
  for (uint32_t SL : low_masks) {
    const int sL = popc(SL);
    yoff[SL] = (int32_t)C->ytab.size();
    for (int sl = 0; sl < nslot(sL); ++sl) {
      const int32_t fb = final_base.at(SL);
      if (fb >= (1 << 16) || sl >= (1 << 10) || sL >= 64) return "Y table too large";
      C->ytab.push_back((uint32_t)fb | ((uint32_t)sl << 16) | ((uint32_t)sL << 26));
    }
  }
  C->Ysize = (int)C->ytab.size();
  if (C->Ysize >= (1 << 24)) return "Y table too large";

  // ---- final-core weights per high popcount u ----
  C->lam_soff.assign(l + 1, 0);
  int off = 0;
  for (int sL = 0; sL <= l; ++sL) {
    C->lam_soff[sL] = off;
    if (sL <= b) off += nslot(sL) * (b + 1);
  }
  C->lam_ublock = off;
  C->lam.assign((size_t)(h + 1) * off, 0.0);
  // two-pass: the weights also as double-doubles (their rounding error,
  // for the compensated FP64 weight core)
  if (algo != ALGO_FUSED) C->lam_lo.assign((size_t)(h + 1) * off, 0.0);
  for (int u = 0; u <= h; ++u) {
    for (int sL = 0; sL <= std::min(l, b); ++sL) {
      double* blk = &C->lam[(size_t)u * off + C->lam_soff[sL]];
      const int top = std::min(l - sL, h);
      for (int sH = 0; sH <= top; ++sH) {
        const int s = sL + sH;
        if (algo == ALGO_FUSED) {
          for (int j = 0; j <= sH; ++j) {
            const int slot = sH * (sH + 1) / 2 + j;
            if (mobius_in) {
              // input already transformed: a tile with high index U_H feeds
              // the outputs with S_H inside U_H (j = s_H) at t = t_L + |U_H|
              const bool ok = j == sH && sH <= u;
              for (int tL = sL; tL <= b; ++tL)
                blk[slot * (b + 1) + tL] = ok ? (double)weight_q(s, tL + u, l, index) : 0.0;
              continue;
            }
            const bool ok = j <= u && (sH - j) <= (h - u);
            const int q = u + sH - j;
            for (int tL = sL; tL <= b; ++tL)
              blk[slot * (b + 1) + tL] = ok ? (double)lambda_q(s, tL, q, u, h, l, index) : 0.0;
          }
        } else {
          double* blo = &C->lam_lo[(size_t)u * off + C->lam_soff[sL]];
          for (int tL = sL; tL <= b; ++tL) {
            const __float128 w = weight_q(s, tL + u, l, index);
            blk[sH * (b + 1) + tL] = (double)w;
            blo[sH * (b + 1) + tL] = (double)(w - (__float128)(double)w);
          }
        }
      }
    }
  }

  // ---- outputs ----
  C->out_masks = canonical_masks(d, l);
  C->oinfo.resize(C->out_masks.size());
  C->osh.resize(C->out_masks.size());
  const uint32_t lowmask = (b >= 32) ? 0xFFFFFFFFu : ((1u << b) - 1);
  for (size_t k = 0; k < C->out_masks.size(); ++k) {
    const uint32_t S = C->out_masks[k];
    const uint32_t SL = S & lowmask, SH = S >> b;
    C->oinfo[k] = (uint32_t)yoff.at(SL) | ((uint32_t)popc(SH) << 24);
    C->osh[k] = SH;
  }
  return "";
}

int fast_block_bits(int d, int l) {
  using namespace t11;
  if (d < B || l < 1 || l > 4 || l > d) return -1;
  const int h = d - B, hmax = 32 - meta_shift(l);
  if (h <= hmax && positions_needed(l, h) <= np_order(l)) return h;
  for (int k = std::min(h - 1, hmax); k >= 0; --k)
    if (positions_blocked(l, k) <= np_order(l)) return k;
  return -1;
}

int fast_output_slots(int d, int l) {
  const int k = fast_block_bits(d, l);
  if (k < 0) return -1;
  const int h = d - t11::B;
  return (int)(2 * (k == h ? t11::positions_needed(l, h) : t11::positions_blocked(l, k)));
}

std::string build_fast_class(const ClassHost& C, FastClassHost* F) {
  using namespace t11;
  const int l = C.l, b = C.b, h = C.h;
  if (b != B) return "register-phase kernel needs 11-bit tiles";
  if (C.algo != ALGO_FUSED) return "register-phase kernel needs the fused algorithm";
  if (l > 4) return "register-phase kernel needs l <= 4";
  F->mshift = meta_shift(l);
  F->d = C.d; F->l = l; F->h = h; F->M = C.M; F->mobius_in = C.mobius_in;
  // phase-C units and their maps
  const int nu = n3(l);
  F->unit_mask.assign(nu, -1);
  for (int sa = 0; sa < NA; ++sa)
    for (int sb = 0; sb < NB; ++sb) {
      const int u = unit_index(l, sa, sb);
      if (u < 0) continue;
      if (u >= nu || F->unit_mask[u] != -1) return "unit order is not a bijection";
      F->unit_mask[u] = sa | (sb << PA);
    }
  for (int u = 0; u < nu; ++u)
    if (F->unit_mask[u] < 0) return "unit order has a hole";
  F->uperm.assign(kFastThreads, 0);
  {
    const UnitOrder uo = mk_unit_order(l);
    for (int t = 0; t < kFastThreads; ++t) {
      F->uperm[t] = uo.v[t];
      if (uo.v[t] < -1 || uo.v[t] >= nu) return "phase-C unit order out of range";
    }
  }
  F->zrow.assign((size_t)nu * NC, 0);
  for (int u = 0; u < nu; ++u)
    for (int sc = 0; sc < NC; ++sc)
      F->zrow[(size_t)u * NC + sc] = zrow_of(l, (uint32_t)F->unit_mask[u] | ((uint32_t)sc << KAB));
  // weights: entry (u, s_L, slot, r) = the class's precontracted weight of
  // counter t = s_L + r (zero past t = 11 and for slots the class lacks)
  const int lb = lamblock(l);
  F->lam.assign((size_t)(h + 1) * lb, 0.0);
  for (int u = 0; u <= h; ++u)
    for (int sL = 0; sL <= l; ++sL) {
      const int top = std::min(l - sL, h);
      for (int sH = 0; sH <= top; ++sH)
        for (int j = 0; j <= sH; ++j) {
          const int slot = sH * (sH + 1) / 2 + j;
          for (int r = 0; sL + r <= b; ++r)
            F->lam[(size_t)u * lb + lamoff(l, sL) + slot * ZROW + r] =
                C.lam[(size_t)u * C.lam_ublock + C.lam_soff[sL] + slot * (b + 1) + sL + r];
        }
    }
  // partial sums: runs of two (S_L of ranks 2r and 2r + 1 among the S_L of
  // one size), taken by |S_L| (descending), then by what the run sums over
  // the high bits, then r, and dealt to wave units: unit u is position u / 4
  // of wave u % 4 of the workgroup, 64 runs of one |S_L| (so the j-stride is
  // uniform in a wave); a unit left short by its |S_L| is filled with dummy
  // runs (offset 0, S_H = 0: a valid read whose sums nothing uses).
  //  - whole instance (kb = h): a run is one S_H; it sums, over the tiles,
  //    Y[S_L, |S_H|, |S_H & U_H|], an output.
  //  - blocks (kb < h): a run is (S_H1 over the kb low high bits, s_H2, j2);
  //    it sums Y[S_L, |S_H1| + s_H2, |S_H1 & U_H| + j2] over the block.
  const int kb = fast_block_bits(C.d, l);
  if (kb < 0) return "register-phase kernel does not apply";
  F->kb = kb;
  const bool blocked = kb < h;
  const int npos = fast_output_slots(C.d, l) / 2;
  if (npos > np_order(l)) return "gather positions exceed the kernel's";
  if (kRuns != kFastRuns) return "gather position count mismatch";
  const size_t M = C.out_masks.size();
  const uint32_t lowmask = (1u << b) - 1;
  // S_L of each size in colex rank order
  std::vector<std::vector<uint32_t>> low(l + 1);
  for (uint32_t m = 0; m <= lowmask; ++m) {
    const int sL = popc(m);
    if (sL <= l) low[sL].push_back(m);
  }
  for (int sL = 0; sL <= l; ++sL) {
    std::sort(low[sL].begin(), low[sL].end(),
              [](uint32_t x, uint32_t y) { return rank_colex(x) < rank_colex(y); });
    if ((int)low[sL].size() != cbinom(B, sL)) return "low output count mismatch";
  }
  // high masks (over the kb low high bits) of each size
  std::vector<std::vector<uint32_t>> high(l + 1);
  for (uint32_t m = 0; m < (1u << kb); ++m) {
    const int sH = popc(m);
    if (sH <= l) high[sH].push_back(m);
  }
  F->meta.assign((size_t)kFastThreads * kFastMetaStride, 0u);
  F->gs8.assign((size_t)kRuns * 4, 0u);
  F->nkk = 0;
  // slot of (S_L, S_H1, s_H2, j2), key S_L | S_H1 << 11 | (s_H2 * 8 + j2) << 40
  std::unordered_map<uint64_t, int32_t> slot_of;
  slot_of.reserve((size_t)npos * 4 * 64 * 2);
  auto key = [](uint32_t SL, uint32_t S1, int s2, int j2) {
    return (uint64_t)SL | ((uint64_t)S1 << 11) | ((uint64_t)(s2 * 8 + j2) << 40);
  };
  int64_t unit = 0;
  for (int sL = l; sL >= 0; --sL) {
    const uint32_t nr = (uint32_t)cbinom(B, sL);
    int lane = 64;   // start a new unit for each |S_L|
    for (int a = 0; a <= std::min(l - sL, kb); ++a)
      for (uint32_t S1 : high[a])
        for (int s2 = 0; s2 <= (blocked ? l - sL - a : 0); ++s2)
          for (int j2 = 0; j2 <= s2; ++j2)
            for (uint32_t r0 = 0; r0 < nr; r0 += 2) {
              if (lane == 64) {
                lane = 0;
                ++unit;
              }
              const int64_t u = unit - 1;
              const int pos = (int)(u / 4), w = (int)(u % 4), t = 64 * w + lane;
              if (pos >= npos) return "gather unit past the last position";
              F->gs8[(size_t)pos * 4 + w] = (uint32_t)nrp(sL) * 8u;
              F->nkk = std::max(F->nkk, 2 * (pos + 1));
              const int sH = a + s2;
              const uint32_t A =
                  (uint32_t)(ybase(l, sL) + (sH * (sH + 1) / 2 + j2) * nrp(sL) + (int)r0);
              if (A * 8 >= (1u << F->mshift) || (uint64_t)S1 >= (1ull << (32 - F->mshift)))
                return "output metadata overflow";
              F->meta[(size_t)t * kFastMetaStride + pos] = (A * 8) | (S1 << F->mshift);
              for (uint32_t e = 0; e < 2 && r0 + e < nr; ++e)
                slot_of[key(low[sL][r0 + e], S1, s2, j2)] = (int32_t)((2 * pos + e) * kFastThreads + t);
              ++lane;
            }
  }
  // each canonical output's slots, j2 = 0 .. l (whole instances: j2 = 0)
  F->pidx.assign(M * (size_t)(l + 1), -1);
  F->osh2.assign(M, 0u);
  const uint32_t lowhigh = (uint32_t)((1ull << kb) - 1);
  for (size_t k = 0; k < M; ++k) {
    const uint32_t S = C.out_masks[k];
    const uint32_t SL = S & lowmask, SH = S >> b;
    const uint32_t S1 = SH & lowhigh, S2 = blocked ? SH >> kb : 0u;
    const int s2 = popc(S2);
    F->osh2[k] = S2;
    for (int j2 = 0; j2 <= l; ++j2) {
      auto it = slot_of.find(key(SL, S1, s2, std::min(j2, s2)));
      if (it == slot_of.end()) return "an output has no slot";
      F->pidx[k * (size_t)(l + 1) + j2] = it->second;
    }
  }
  if (!blocked) {
    F->sinv.assign((size_t)F->nkk * kFastThreads, -1);
    for (size_t k = 0; k < M; ++k) {
      const int32_t slot = F->pidx[k * (size_t)(l + 1)];
      if (slot < 0 || (size_t)slot >= F->sinv.size() || F->sinv[slot] != -1)
        return "output slots are not one to one";
      F->sinv[slot] = (int32_t)k;
    }
  }
  return "";
}

}  // namespace fsi
