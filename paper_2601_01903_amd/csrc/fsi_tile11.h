// Compile-time layout of the 2^11-value register-phase tile (fused algorithm,
// l <= 4), shared by the kernel (fsi_tile11.hip) and the host tables
// (fsi_tables.cpp). Everything here depends only on l: the tile splits its
// 11 low bits into phase A (bits 0-3), phase B (bits 4-7), phase C (bits 8-10).
//
// Counter states are stored by their counter RELATIVE to the popcount of
// their output prefix sigma (entry r holds t = |sigma| + r), so an output
// prefix owns the entries r = 0 .. (sites so far) - |sigma|.
//
//  S1  phase-A states (sigma_A, r): row off1(r) + rankA(sigma_A), one column
//      per phase-B/C input (b + 16 c); a row is padded by one 16-byte chunk.
//  S2  phase-B states (sigma_AB, i): for each relative counter i and each
//      half of the 8 phase-C inputs, one 4-input chunk per unit sigma_AB
//      (|sigma_AB| <= l); entries past a unit's counter range hold zeros.
//  Z   final states (S_L, r), one row of 12 entries per S_L; rows grouped by
//      |S_L| and ranked in colex order inside a group; one dump row.
//  Y   per-tile partial results Y[S_L, s_H, j]: group (s_L, slot) holds every
//      S_L of that size in rank order; slot = s_H (s_H + 1) / 2 + j.
#pragma once
#include <cstdint>

namespace fsi {
namespace t11 {

constexpr int PA = 4, PB = 4, PC = 3, B = 11;
constexpr int NA = 1 << PA, NB = 1 << PB, NC = 1 << PC;
constexpr int KAB = PA + PB;
constexpr int NT = 256;      // threads per workgroup
constexpr int ZROW = 12;     // entries per Z row (B + 1)

constexpr int cbinom(int n, int k) {
  if (k < 0 || n < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int)r;
}
constexpr int cpop(int x) {
  int c = 0;
  while (x) { c += x & 1; x >>= 1; }
  return c;
}
// 4-bit masks in (popcount, value) order
constexpr int orderA(int k) {
  int idx = 0;
  for (int s = 0; s <= 4; ++s)
    for (int m = 0; m < 16; ++m)
      if (cpop(m) == s) {
        if (idx == k) return m;
        ++idx;
      }
  return -1;
}
constexpr int rankA(int mask) {
  int idx = 0;
  for (int s = 0; s <= 4; ++s)
    for (int m = 0; m < 16; ++m)
      if (cpop(m) == s) {
        if (m == mask) return idx;
        ++idx;
      }
  return -1;
}
// orderA(k) for a run-time k: nibble k of this constant
constexpr uint64_t kOrderANibbles = 0xfedb7ca965384210ull;
// number of 4-bit masks with popcount <= m
constexpr int N4(int m) {
  int n = 0;
  for (int s = 0; s <= m && s <= 4; ++s) n += cbinom(4, s);
  return n;
}
// colex rank of a mask among the masks of the same popcount
constexpr int rank_colex(uint32_t mask) {
  int r = 0, k = 0;
  for (int p = 0; p < 32; ++p)
    if ((mask >> p) & 1u) {
      r += cbinom(p, k + 1);
      ++k;
    }
  return r;
}
constexpr int imin(int a, int b) { return a < b ? a : b; }

// ---- S1 ----
constexpr int off1(int L, int r) {
  int o = 0;
  for (int q = 0; q < r; ++q) o += N4(imin(L, PA - q));
  return o;
}
constexpr int rows1(int L) { return off1(L, PA + 1); }
template <typename T> constexpr int row1_stride() { return 128 + 16 / (int)sizeof(T); }

// ---- phase-C units sigma_AB = sigma_A | sigma_B << 4, |sigma_AB| <= L,
// ordered by sigma_B, then rankA(sigma_A): the valid sigma_A of a sigma_B
// are a prefix of the rankA order, so unit = ubase(sigma_B) + rankA ----
constexpr int ubase(int L, int sb) {
  int u = 0;
  for (int q = 0; q < sb; ++q) u += N4(L - cpop(q));
  return u;
}
constexpr int n3(int L) { return ubase(L, NB); }
constexpr int unit_index(int L, int sa, int sb) {
  return cpop(sa) + cpop(sb) > L ? -1 : ubase(L, sb) + rankA(sa);
}
// element (i, unit, c) at ((2 i + c / 4) * s2u + unit) * 4 + c % 4, with the
// unit count padded to s2u, a multiple of 8: the counter rows of one
// (unit, c) lie a multiple of 64 elements apart, so their stores pair up
// (two per instruction), and the two c-halves of a phase-B wave fall on
// disjoint LDS banks
constexpr int s2u(int L) { return (n3(L) + 7) & ~7; }
// phase B writes the leaves of prefixes past the order to a padding unit
// (n3 .. s2u - 1), which phase C never reads
static_assert(s2u(1) > n3(1) && s2u(2) > n3(2) && s2u(3) > n3(3) && s2u(4) > n3(4),
              "S2 needs a padding unit");
constexpr int s2_elems(int L) { return (KAB + 1) * s2u(L) * NC; }

// Phase-C thread map. Units in order of |sigma_AB| (stable). The heavy units
// (|sigma_AB| <= L - 2: most output prefixes over the C bits) are split at the
// first C output site: wave kCWaveH0 walks their sigma = 0 subtree, wave
// kCWaveH1 (same lane) their sigma = 1 subtree. The other units fill waves
// kCWaveR0 and kCWaveR1 whole. Thread t takes unit v[t] (-1: idle); every
// unit of wave w has kmin[w] <= |sigma_AB| <= kmax[w] (kmin = L + 1 for a
// wave without units) and wave w walks part[w] of the C-site tree (0: sigma
// = 0 subtree, 1: sigma = 1 subtree, 2: all). The roles are placed so that
// each SIMD's share of the per-tile work (one wave of each workgroup per
// SIMD) comes out about even over the phases.
constexpr int kCWaveH0 = 1, kCWaveH1 = 3, kCWaveR0 = 0, kCWaveR1 = 2;
struct UnitOrder {
  int v[NT];
  int kmin[NT / 64], kmax[NT / 64], part[NT / 64];
  int nheavy;
};
constexpr UnitOrder mk_unit_order(int L) {
  UnitOrder o{};
  int units[NT] = {}, pop[NT] = {};
  int n = 0;
  for (int k = 0; k <= L; ++k)
    for (int sb = 0; sb < NB; ++sb)
      for (int r = 0; r < NA; ++r) {
        const int sa = orderA(r);
        if (cpop(sa) + cpop(sb) == k) {
          units[n] = ubase(L, sb) + r;
          pop[n] = k;
          ++n;
        }
      }
  int nh = 0;
  while (nh < n && pop[nh] <= L - 2) ++nh;
  for (int t = 0; t < NT; ++t) o.v[t] = -1;
  for (int i = 0; i < nh; ++i) o.v[64 * kCWaveH0 + i] = o.v[64 * kCWaveH1 + i] = units[i];
  for (int i = nh; i < n; ++i)
    o.v[64 * (i - nh < 64 ? kCWaveR0 : kCWaveR1) + (i - nh) % 64] = units[i];
  o.nheavy = nh;
  o.part[kCWaveH0] = 0;
  o.part[kCWaveH1] = 1;
  o.part[kCWaveR0] = o.part[kCWaveR1] = 2;
  o.kmin[kCWaveH0] = o.kmin[kCWaveH1] = nh ? 0 : L + 1;
  o.kmax[kCWaveH0] = o.kmax[kCWaveH1] = nh ? pop[nh - 1] : L + 1;
  for (int q = 0; q < 2; ++q) {
    const int w = q ? kCWaveR1 : kCWaveR0;
    const int i0 = nh + 64 * q, i1 = imin(n, i0 + 64);
    o.kmin[w] = i0 < n ? pop[i0] : L + 1;
    o.kmax[w] = i0 < n ? pop[i1 - 1] : L + 1;
  }
  return o;
}
// the map fits the workgroup at every order the kernel runs
constexpr bool unit_order_fits(int L) {
  int heavy = 0, rest = 0;
  for (int k = 0; k <= L; ++k) (k <= L - 2 ? heavy : rest) += cbinom(KAB, k);
  return heavy <= 64 && rest <= 128;
}
static_assert(unit_order_fits(1) && unit_order_fits(2) && unit_order_fits(3) &&
              unit_order_fits(4), "phase-C units exceed the workgroup");

// ---- Z rows ----
constexpr int zbase(int s) {
  int o = 0;
  for (int q = 0; q < s; ++q) o += cbinom(B, q);
  return o;
}
constexpr int nzrows(int L) { return zbase(L + 1); }        // the dump row follows
constexpr int zrow_of(int L, uint32_t SL) {
  const int s = cpop((int)SL);
  return s > L ? nzrows(L) : zbase(s) + rank_colex(SL);
}

// ---- Y ----
// Group (s_L, slot) holds the S_L of size s_L in rank order, padded to an
// even count so that every pair of ranks (2r, 2r + 1) is one aligned
// 16-byte read of the gather.
constexpr int nslots(int L, int s) { return s > L ? 0 : (L - s + 1) * (L - s + 2) / 2; }
constexpr int nrp(int s) { return (cbinom(B, s) + 1) & ~1; }
constexpr int ybase(int L, int s) {
  int o = 0;
  for (int q = 0; q < s; ++q) o += nslots(L, q) * nrp(q);
  return o;
}
constexpr int ysize(int L) { return ybase(L, L + 1); }

// ---- cross-tile gather ----
// A run is two outputs (S_L of ranks 2r and 2r + 1 among the S_L of one
// size, one S_H): one popcount |S_H & U_H| and one 16-byte read of Y per
// tile. A thread holds up to kFastRuns runs ("positions"); at each position
// the 64 runs of a wave share s_L, so the j-stride of Y is wave-uniform.
// Runs of one (s_L, S_H) for the outputs of order L with h high bits:
constexpr int64_t runs_of(int L, int h, int sL) {
  int64_t nh = 0;
  for (int sH = 0; sH <= L - sL && sH <= h; ++sH) nh += cbinom(h, sH);
  return (int64_t)((cbinom(B, sL) + 1) / 2) * nh;
}
// positions of 4 waves x 64 runs the outputs need (all groups together)
constexpr int64_t positions_needed(int L, int h) {
  int64_t units = 0;
  for (int sL = 0; sL <= L; ++sL) units += (runs_of(L, h, sL) + 63) / 64;
  return (units + 3) / 4;
}

// ---- final-core weights (FP64, global memory), per high popcount u:
// entry (s_L, slot, r) at lamoff(s_L) + slot * 12 + r (zero for r > 11 - s_L) ----
constexpr int lamoff(int L, int s) {
  int o = 0;
  for (int q = 0; q < s; ++q) o += nslots(L, q) * ZROW;
  return o;
}
constexpr int lamblock(int L) { return lamoff(L, L + 1); }

// ---- weight-core work of one tile: 64-lane tasks. For |S_L| >= 2 a lane
// owns one Z row and computes all its slots; the (|S_L| <= 1) rows are few,
// so there a lane owns one (row, slot) pair ----
constexpr int row_tasks(int s) { return (cbinom(B, s) + 63) / 64; }
constexpr int npairs(int L) {
  int n = 0;
  for (int s = 0; s <= imin(1, L); ++s) n += cbinom(B, s) * nslots(L, s);
  return n;
}
constexpr int ntasks(int L) {
  int n = (npairs(L) + 63) / 64;
  for (int s = 2; s <= L; ++s) n += row_tasks(s);
  return n;
}
// output metadata word: byte offset of Y(S_L, s_H, j = 0) | S_H << mshift,
// mshift = the bits the largest Y byte offset of the order needs; S_H gets
// the other 32 - mshift bits (19 high bits for l <= 3, 18 for l = 4)
constexpr int meta_shift(int L) {
  int s = 1;
  while ((1 << s) <= ysize(L) * 8) ++s;
  return s;
}

// ---- blocked outputs: when an instance has more outputs than the
// workgroup's accumulators hold, a work item covers a block of 2^k tiles
// sharing their top h - k high bits H2 = U_H >> k, and its partial sums are
//   Y2[S_L, S_H1, s_H2, j2] = sum over the block's tiles of
//                             Y[S_L, |S_H1| + s_H2, |S_H1 & U_H| + j2]
// for S_H1 within the k low high bits; the reduction picks j2 = |S_H2 & H2|
// for an output with S_H = S_H1 | S_H2 << k and s_H2 = |S_H2|. The gather
// is the same as for whole instances: S_H1 in the metadata word, the
// (s_H2, j2) part folded into the Y offset.
constexpr int64_t tri(int n) { return (int64_t)(n + 1) * (n + 2) / 2; }
constexpr int64_t runs_blocked(int L, int k, int sL) {
  int64_t c = 0;
  for (int a = 0; a <= L - sL && a <= k; ++a) c += (int64_t)cbinom(k, a) * tri(L - sL - a);
  return (int64_t)((cbinom(B, sL) + 1) / 2) * c;
}
constexpr int64_t positions_blocked(int L, int k) {
  int64_t units = 0;
  for (int sL = 0; sL <= L; ++sL) units += (runs_blocked(L, k, sL) + 63) / 64;
  return (units + 3) / 4;
}

// gather positions per thread; the kernel of order L unrolls np_order(L) of
// them (the most its outputs need at any h the metadata word holds, at most
// kRuns; past that the outputs are blocked)
constexpr int kRuns = 14;
constexpr int np_order(int L) {
  int64_t m = 0;
  for (int h = 0; h <= 32 - meta_shift(L); ++h) {
    const int64_t p = positions_needed(L, h);
    m = p > m ? p : m;
  }
  return m > kRuns ? kRuns : (int)m;
}

}  // namespace t11
}  // namespace fsi
