// Register-phase tile kernel of the fused FSI algorithm (gfx950), tiles of
// 2^11 values, l <= 4.
//
// A workgroup of 256 threads owns a work item: a run of tiles of one
// instance (raw v, high index U_H) and one group of its outputs. Per tile it
// computes
//   - the in-tile Moebius butterfly (Sec. 4.2) over the 11 low bits: bits
//     8-10 in registers straight from the coalesced loads, bits 4-7 and 0-3
//     through two LDS transposes;
//   - the left-to-right counter sweep (Sec. 4.3 - 4.4) in three phases of 4,
//     4 and 3 sites. Within a phase a thread owns one output prefix with all
//     its counters and the phase's 2^P inputs in registers and walks the
//     phase's output bits depth first: each output state adds its tau = 0
//     and tau = 1 predecessors (the sparse MPO cores). Between phases the
//     (sigma, t) states go through LDS, truncated to |sigma| <= l (the
//     compressed output prefix). Phase B splits its first output site
//     between the two halves of the workgroup (sigma = 0 and sigma = 1
//     subtrees); phase C splits it for its heavy prefixes only. Threads are
//     ordered so that each wave's prefixes share bounds on their popcount,
//     and each wave runs code compiled for those bounds;
//   - the final weight core with the Moebius cores of the high sites
//     precontracted into it (Sec. 4.5 applied to the high sites), in FP64:
//     Y[S_L, s_H, j] = sum_t lambda_u(s_L + s_H, t, s_H + u - j) Z[S_L, t],
//     u = |U_H|; a wave first loads the Z rows of all its tasks, then
//     computes them; rows of one |S_L| take wave-uniform weights through
//     scalar loads, the (row, slot) pairs of |S_L| <= 1 per-lane weights
//     staged in LDS;
//   - the cross-tile sum E_S += Y[S_L, |S_H|, |S_H & U_H|] in FP64 registers
//     for the outputs of the item's group.
// At the end of the item the FP64 partial sums go to a workspace; the
// reduction kernel adds the items of an instance in a fixed order.
//
// Every LDS layout is a compile-time function of l (fsi_tile11.h), so the
// hot loops address LDS with one per-thread base register and immediate
// offsets. LDS regions:
//   region 1: raw-tile transposes and, after them, the partial results Y;
//             phase-B states S2 overlay both (no barrier between a tile's
//             gather and the next tile's loads)
//   region 2: phase-A states S1 -> final states Z
//   region 3: the final-core weights of the current |U_H| (per-lane reads
//             of the |S_L| <= 1 pairs)
//   a zero row read in place of counter rows past a unit's range
#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

#include "fsi_kernels.h"
#include "fsi_tile11.h"

namespace fsi {
namespace t11 {

// ----------------------------------------------------------------- numerics
struct TwoF {
  float hi, lo;
};
// Two-float subtraction: Knuth's TwoSum of the high parts (exact error e),
// the low parts and e added into the low word. The pair is not renormalised
// (hi + lo still holds the value; the low word stays within a few ulps of the
// operands over the 11 butterfly levels) and is rounded once, to FP32, when
// the sweep takes it.
__device__ __forceinline__ TwoF sub(TwoF a, TwoF b) {
  const float s = a.hi - b.hi;
  const float bb = s - a.hi;
  const float e = (a.hi - (s - bb)) + (-b.hi - bb);
  return TwoF{s, e + (a.lo - b.lo)};
}
__device__ __forceinline__ float sub(float a, float b) { return a - b; }
__device__ __forceinline__ double sub(double a, double b) { return a - b; }

template <typename M> __device__ __forceinline__ M mob_from(float x);
template <> __device__ __forceinline__ float mob_from<float>(float x) { return x; }
template <> __device__ __forceinline__ double mob_from<double>(float x) { return x; }
template <> __device__ __forceinline__ TwoF mob_from<TwoF>(float x) { return TwoF{x, 0.f}; }
template <typename M> __device__ __forceinline__ M mob_from_d(double x);
template <> __device__ __forceinline__ double mob_from_d<double>(double x) { return x; }

template <typename S> __device__ __forceinline__ S to_sw(float x) { return (S)x; }
template <typename S> __device__ __forceinline__ S to_sw(double x) { return (S)x; }
template <typename S> __device__ __forceinline__ S to_sw(TwoF x);
template <> __device__ __forceinline__ float to_sw<float>(TwoF x) { return x.hi + x.lo; }
template <> __device__ __forceinline__ double to_sw<double>(TwoF x) {
  return (double)x.hi + (double)x.lo;
}

// ------------------------------------------------- in-register counter sweep
// Node of the depth-first walk over the output bits of one phase: X[t][r]
// holds the states with counter t in [LO, LO + RC) for the 2^REM inputs r of
// the bits still to consume. The most significant remaining bit is consumed
// first: the sigma = 1 child keeps the tau = 1 half with t + 1; the sigma = 0
// child adds the tau = 0 half at t and the tau = 1 half at t - 1. At a leaf
// SIG is the output mask over the phase's bits and X[i] holds counter LO + i,
// i.e. the counter relative to the prefix's popcount (LO = |SIG|).
template <int REM, int LO, int RC, int SIG, typename T, typename Emit>
__device__ __forceinline__ void rsweep(const T (&X)[RC][1 << REM], Emit& emit) {
  if constexpr (REM == 0) {
    emit.template leaf<SIG, LO, RC>(X);
  } else {
    constexpr int H = 1 << (REM - 1);
    {
      T Y0[RC + 1][H];
#pragma unroll
      for (int r = 0; r < H; ++r) {
        Y0[0][r] = X[0][r];
#pragma unroll
        for (int t = 1; t < RC; ++t) Y0[t][r] = X[t][r] + X[t - 1][H + r];
        Y0[RC][r] = X[RC - 1][H + r];
      }
      rsweep<REM - 1, LO, RC + 1, SIG>(Y0, emit);
    }
    {
      T Y1[RC][H];
#pragma unroll
      for (int t = 0; t < RC; ++t)
#pragma unroll
        for (int r = 0; r < H; ++r) Y1[t][r] = X[t][H + r];
      rsweep<REM - 1, LO + 1, RC, SIG | H>(Y1, emit);
    }
  }
}

// Raw-tile transposes: element (a, b, c) of the tile (index a + 16 b + 256 c)
// at a + 17 b + 272 c. Affine in each coordinate, so every access is a
// per-thread base plus an immediate; the three access patterns (fixed c,
// fixed b, fixed a across a wave) hit distinct banks (fixed c: 3 of 64
// banks shared).
constexpr int RB = 17, RC_ = 272;
constexpr int r_elems = RC_ * NC;

// Weights are read-only for the whole launch: addressed through the constant
// address space, so wave-uniform reads become scalar loads.
typedef const __attribute__((address_space(4))) double* cdptr;
typedef const __attribute__((address_space(4))) uint32_t* cdptr_u;

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec4<double> { using type = double2; static constexpr int n = 2; };

// Compile-time tables of one order l (indexed with unrolled loop counters,
// so every use folds into an immediate).
struct A5 { int v[PA + 1]; };
struct A16 { int v[16]; };
constexpr A5 mk_off1(int L) {
  A5 a{};
  for (int r = 0; r <= PA; ++r) a.v[r] = off1(L, r);
  return a;
}
constexpr A16 mk_ubase(int L) {
  A16 a{};
  for (int b = 0; b < NB; ++b) a.v[b] = ubase(L, b);
  return a;
}
constexpr A16 mk_rank() {
  A16 a{};
  for (int m = 0; m < NA; ++m) a.v[m] = rankA(m);
  return a;
}
template <int L>
struct K {
  static constexpr A5 off1v = mk_off1(L);
  static constexpr A16 ub = mk_ubase(L);
  static constexpr A16 rk = mk_rank();
  static constexpr int N3 = n3(L);
  static constexpr int S2U = s2u(L);
  static constexpr int LB = lamblock(L);
  static constexpr int NTASK = ntasks(L);
  static constexpr int NPAIR = npairs(L);
  static constexpr int LAM0 = lamoff(L, 0), LAM1 = lamoff(L, 1);
  static constexpr int YB0 = ybase(L, 0), YB1 = ybase(L, 1);
};

// ----------------------------------------------------------------- emitters
// Phase A -> S1 row off1(i) + rankA(sigma_A), column = this thread's input.
template <typename SwT, int L>
struct EmitS1 {
  SwT* S1;   // already offset by the thread's column
  template <int SIG, int LO, int RC>
  __device__ __forceinline__ void leaf(const SwT (&X)[RC][1]) {
    if constexpr (cpop(SIG) <= L) {
      constexpr int R1 = row1_stride<SwT>();
      constexpr int RK = K<L>::rk.v[SIG];
#pragma unroll
      for (int i = 0; i < RC; ++i) S1[(K<L>::off1v.v[i] + RK) * R1] = X[i][0];
    }
  }
};

// Phase B -> S2 entries (i, unit of (sigma_A, sigma_B), c) for the leaf's
// counters i < RC (entries past this unit's range hold zeros), for the
// prefixes with |sigma_A| + |sigma_B| <= L. Phase C reads only i <= 8 - |sigma_AB|,
// all written here.
template <typename SwT, int L, int SAMIN, int SAMAX>
struct EmitS2 {
  SwT* S2;   // offset by ((c / 4) * s2u + rankA) * 4 + c % 4
  int sA;    // in [SAMIN, SAMAX]
  int rkA;   // rankA
  template <int SIG, int LO, int RC>
  __device__ __forceinline__ void leaf(const SwT (&X)[RC][1]) {
    constexpr int sB = cpop(SIG);
    if constexpr (sB <= L - SAMIN) {
      constexpr int UB = K<L>::ub.v[SIG];
      constexpr int S2U = K<L>::S2U;
      if constexpr (sB <= L - SAMAX) {
#pragma unroll
        for (int i = 0; i < RC; ++i) S2[(2 * i * S2U + UB) * 4] = X[i][0];
      } else {
        // a prefix past the order writes a padding unit (n3 .. s2u - 1),
        // which phase C never reads
        const int ub = sA <= L - sB ? UB : K<L>::N3 - rkA;
#pragma unroll
        for (int i = 0; i < RC; ++i) S2[(2 * i * S2U + ub) * 4] = X[i][0];
      }
    }
  }
};

// Phase C -> Z row of S_L = sigma_AB | sigma_C << 8 (12 entries, zero padded).
template <typename SwT, int L, int KMIN, int KMAX>
struct EmitZ {
  SwT* Z;
  const int (&zr)[NC];   // Z row per sigma_C (dump row where |S_L| > L)
  int sAB;               // in [KMIN, KMAX] for every unit of the wave
  template <int SIG, int LO, int RC>
  __device__ __forceinline__ void leaf(const SwT (&X)[RC][1]) {
    constexpr int sC = cpop(SIG);
    if constexpr (sC <= L - KMIN) {
      {   // leaves past the order write the dump row (zr)
        using V = typename Vec4<SwT>::type;
        constexpr int VN = Vec4<SwT>::n;
        V* p = reinterpret_cast<V*>(Z + zr[SIG] * ZROW);
        // the weight core reads a row's counters only (the first 12 - |S_L|
        // entries, at most RC here): the padding past them is not stored
#pragma unroll
        for (int q = 0; q < (RC + VN - 1) / VN; ++q) {
          SwT e[VN];
#pragma unroll
          for (int k = 0; k < VN; ++k) e[k] = q * VN + k < RC ? X[q * VN + k][0] : SwT(0);
          if constexpr (VN == 4) p[q] = V{e[0], e[1], e[2], e[3]};
          else p[q] = V{e[0], e[1]};
        }
      }
    }
  }
};

// --------------------------------------------------------------- LDS plan
constexpr int align256(int x) { return (x + 255) & ~255; }
constexpr int imax2(int a, int b) { return a > b ? a : b; }
template <int L, typename SwT, typename MobT>
struct Lds {
  // region 1: the raw-tile transposes at 0 and the partial results Y after
  // them (disjoint, so the next tile's loads and first transpose may start
  // while slower waves still gather this tile's Y); phase B's states S2
  // overlay both
  static constexpr int yoff = align256((int)(r_elems * sizeof(MobT)));
  static constexpr int reg1 = align256(imax2((int)(s2_elems(L) * sizeof(SwT)), yoff + ysize(L) * 8));
  static constexpr int reg2 = align256(
      imax2(rows1(L) * row1_stride<SwT>() * (int)sizeof(SwT),
            (nzrows(L) + 1) * ZROW * (int)sizeof(SwT)));
  static constexpr int reg3 = align256(lamblock(L) * 8);   // weights of the current |U_H|
  // zeros, read in place of the counter rows past a prefix's range by the
  // waves that run the general sweep code (their row loads then need no
  // branch and issue back to back)
  static constexpr int zeros = 128;
  static constexpr int bytes = reg1 + reg2 + reg3 + zeros;
};
// The zero row sits at one offset past the regions of every order, so one
// kernel can run items of different orders (each item uses its order's
// regions below that offset) and the row is written once per workgroup.
template <typename SwT, typename MobT>
struct LdsAll {
  static constexpr int zoff =
      imax2(imax2(Lds<1, SwT, MobT>::reg1 + Lds<1, SwT, MobT>::reg2 + Lds<1, SwT, MobT>::reg3,
                  Lds<2, SwT, MobT>::reg1 + Lds<2, SwT, MobT>::reg2 + Lds<2, SwT, MobT>::reg3),
            imax2(Lds<3, SwT, MobT>::reg1 + Lds<3, SwT, MobT>::reg2 + Lds<3, SwT, MobT>::reg3,
                  Lds<4, SwT, MobT>::reg1 + Lds<4, SwT, MobT>::reg2 + Lds<4, SwT, MobT>::reg3));
  static constexpr int zeros = 128;
  static constexpr int bytes = zoff + zeros;
};

// ------------------------------------------------------------ weight core
// Row task: 64 lanes, each owning one Z row of |S_L| = S (S >= 2) and
// producing the slots [K0, K1) of it; the weights are the same for every
// lane. Pair task: the (row, slot) pairs of |S_L| <= 1, 64 per task, with
// per-lane weights.
// Compile-time schedule of the weight-core tasks of one tile over the four
// waves (longest task first to the least loaded wave). Row tasks of rows
// with many slots are split into two slot ranges.
struct LamTask { int kind, S, chunk, k0, k1, cost, wave; };
struct LamPlan { LamTask t[40]; int n; };
constexpr LamPlan make_lam_plan(int L) {
  LamPlan p{};
  p.n = 0;
  for (int S = L; S >= 2; --S) {
    const int RC = ZROW - S, NS = nslots(L, S);
    for (int c = 0; c < row_tasks(S); ++c) {
      const int parts = NS * RC > 40 ? 2 : 1;
      for (int q = 0; q < parts; ++q) {
        const int k0 = NS * q / parts, k1 = NS * (q + 1) / parts;
        p.t[p.n++] = LamTask{0, S, c, k0, k1, (k1 - k0) * RC + RC + 8, -1};
      }
    }
  }
  for (int c = 0; c < (npairs(L) + 63) / 64; ++c) p.t[p.n++] = LamTask{1, 0, c, 0, 0, 2 * ZROW + 8, -1};
  int load[NT / 64] = {0, 0, 0, 0};
  for (int done = 0; done < p.n; ++done) {
    int best = -1;
    for (int i = 0; i < p.n; ++i)
      if (p.t[i].wave < 0 && (best < 0 || p.t[i].cost > p.t[best].cost)) best = i;
    int w = 0;
    for (int q = 1; q < NT / 64; ++q)
      if (load[q] < load[w]) w = q;
    p.t[best].wave = w;
    load[w] += p.t[best].cost;
  }
  return p;
}
template <int L> struct LP { static constexpr LamPlan plan = make_lam_plan(L); };


// Tasks of one wave in plan order, with the offset of each task's Z row in
// the wave's register buffer.
struct WaveList { int idx[40]; int n; };
constexpr WaveList make_wave_list(int L, int W) {
  WaveList w{};
  w.n = 0;
  const LamPlan p = make_lam_plan(L);
  for (int i = 0; i < p.n; ++i)
    if (p.t[i].wave == W) w.idx[w.n++] = i;
  return w;
}
template <int L, int W> struct WL { static constexpr WaveList w = make_wave_list(L, W); };

// Pass 1: every Z row (and the per-lane weights of pair tasks) of the
// wave's tasks is loaded before any arithmetic, so the LDS latency is paid
// once per tile.
template <int L, int W, int J, typename SwT>
__device__ __forceinline__ void lam_load(int lane, const SwT* Z, const double* lam,
                                         SwT (&zb)[ZROW * (WL<L, W>::w.n > 0 ? WL<L, W>::w.n : 1)],
                                         double (&pw)[ZROW * 2]) {
  if constexpr (J < WL<L, W>::w.n) {
    constexpr LamTask T = LP<L>::plan.t[WL<L, W>::w.idx[J]];
    using V = typename Vec4<SwT>::type;
    constexpr int VN = Vec4<SwT>::n;
    const SwT* zr;
    if constexpr (T.kind == 0) {
      constexpr int NR = cbinom(B, T.S);
      constexpr bool full = (T.chunk + 1) * 64 <= NR;
      const int row = T.chunk * 64 + lane;
      zr = Z + (zbase(T.S) + (full || row < NR ? row : 0)) * ZROW;
    } else {
      constexpr int N0 = nslots(L, 0), N1 = nslots(L, 1);
      const int p0 = T.chunk * 64 + lane;
      const int p = p0 < K<L>::NPAIR ? p0 : 0;
      const bool z0 = p < N0;
      const int row = (p - N0) / N1, slot = (p - N0) - row * N1;
      zr = Z + (z0 ? 0 : 1 + row) * ZROW;
      const int lofs = z0 ? K<L>::LAM0 + p * ZROW : K<L>::LAM1 + slot * ZROW;
      const double2* lw = reinterpret_cast<const double2*>(lam + lofs);
      constexpr int PB = (T.chunk & 1) * ZROW;   // at most two pair tasks per wave
#pragma unroll
      for (int q = 0; q < ZROW / 2; ++q) {
        const double2 w = lw[q];
        pw[PB + 2 * q] = w.x;
        pw[PB + 2 * q + 1] = w.y;
      }
    }
    const V* zv = reinterpret_cast<const V*>(zr);
    // a row task reads only its counters (12 - |S_L| entries)
    constexpr int NV = T.kind == 0 ? (ZROW - T.S + VN - 1) / VN : ZROW / VN;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const V v = zv[q];
      if constexpr (VN == 4) {
        zb[J * ZROW + 4 * q] = v.x; zb[J * ZROW + 4 * q + 1] = v.y;
        zb[J * ZROW + 4 * q + 2] = v.z; zb[J * ZROW + 4 * q + 3] = v.w;
      } else {
        zb[J * ZROW + 2 * q] = v.x; zb[J * ZROW + 2 * q + 1] = v.y;
      }
    }
    lam_load<L, W, J + 1, SwT>(lane, Z, lam, zb, pw);
  }
}

// Pass 2: the slots of every task. Row tasks take their weights from the
// constant address space (wave-uniform: scalar loads); lanes past the last
// row write to a dump word.
template <int L, int W, int J, typename SwT>
__device__ __forceinline__ void lam_comp(int lane, double* Y, cdptr lamg, double* dump,
                                         const SwT (&zb)[ZROW * (WL<L, W>::w.n > 0 ? WL<L, W>::w.n : 1)],
                                         const double (&pw)[ZROW * 2]) {
  if constexpr (J < WL<L, W>::w.n) {
    constexpr LamTask T = LP<L>::plan.t[WL<L, W>::w.idx[J]];
    if constexpr (T.kind == 0) {
      constexpr int S = T.S, K0 = T.k0, K1 = T.k1;
      constexpr int NR = cbinom(B, S);
      constexpr int RC = ZROW - S;
      constexpr int LO = lamoff(L, S), YB = ybase(L, S);
      constexpr bool full = (T.chunk + 1) * 64 <= NR;
      const int row = T.chunk * 64 + lane;
      double z[RC];
#pragma unroll
      for (int r = 0; r < RC; ++r) z[r] = (double)zb[J * ZROW + r];
      double a[K1 - K0];
#pragma unroll
      for (int k = K0; k < K1; ++k) a[k - K0] = 0.0;
#pragma unroll
      for (int r = 0; r < RC; ++r)
#pragma unroll
        for (int k = K0; k < K1; ++k) a[k - K0] = fma(lamg[LO + k * ZROW + r], z[r], a[k - K0]);
      const bool ok = full || row < NR;
#pragma unroll
      for (int k = K0; k < K1; ++k) *(ok ? Y + YB + k * nrp(S) + row : dump) = a[k - K0];
    } else {
      constexpr int N0 = nslots(L, 0), N1 = nslots(L, 1);
      constexpr int PB = (T.chunk & 1) * ZROW;
      const int p0 = T.chunk * 64 + lane;
      const bool ok = p0 < K<L>::NPAIR;
      const int p = ok ? p0 : 0;
      const bool z0 = p < N0;
      const int row = (p - N0) / N1, slot = (p - N0) - row * N1;
      const int yidx = z0 ? K<L>::YB0 + p * nrp(0) : K<L>::YB1 + slot * nrp(1) + row;
      double a = 0.0;
#pragma unroll
      for (int r = 0; r < ZROW; ++r) {
        // entry 11 of an |S_L| = 1 row lies past its counters (weight 0)
        const double zz = (r < ZROW - 1 || z0) ? (double)zb[J * ZROW + r] : 0.0;
        a = fma(pw[PB + r], zz, a);
      }
      *(ok ? Y + yidx : dump) = a;
    }
    lam_comp<L, W, J + 1, SwT>(lane, Y, lamg, dump, zb, pw);
  }
}

template <int L, int W, typename SwT>
__device__ __forceinline__ void lam_wave(int lane, const SwT* Z, double* Y, const double* lam,
                                         cdptr lamg, double* dump) {
  SwT zb[ZROW * (WL<L, W>::w.n > 0 ? WL<L, W>::w.n : 1)];
  double pw[ZROW * 2];
  lam_load<L, W, 0, SwT>(lane, Z, lam, zb, pw);
  lam_comp<L, W, 0, SwT>(lane, Y, lamg, dump, zb, pw);
}

// Phase B of one wave: every sigma_A of the wave has SAMIN <= |sigma_A| <=
// SAMAX, so its counter rows past PA - SAMIN are zero and its leaves with
// |sigma_B| > L - SAMIN are never written (both dropped at compile time),
// while rows up to PA - SAMAX and leaves with |sigma_B| <= L - SAMAX need no
// run-time test. HALF 0 walks the sigma = 0 subtree of the first output site
// (all 16 inputs), HALF 1 the sigma = 1 subtree (the 8 tau = 1 inputs).
constexpr int kSALoMax = cpop(orderA(7));   // |sigma_A| of rank 7
constexpr int kSAHi = cpop(orderA(8));      // |sigma_A| of rank 8
constexpr int kSAHiMax = cpop(orderA(15));  // |sigma_A| of rank 15
template <int L, int SAMIN, int SAMAX, int HALF, typename SwT>
__device__ __forceinline__ void phase_b(const SwT* S1, SwT* S2w, int sA, int p2r, int p2c) {
  if constexpr (SAMIN <= L) {
    if (SAMAX > L && sA > L) return;
    using V = typename Vec4<SwT>::type;
    constexpr int VN = Vec4<SwT>::n;
    constexpr int H = NB / 2;
    constexpr int R1 = row1_stride<SwT>();
    constexpr int NRB = PA + 1 - SAMIN;
    constexpr int W = HALF == 0 ? NB : H;       // inputs this half reads
    EmitS2<SwT, L, SAMIN, SAMAX> e2{S2w, sA, p2r};
    const SwT* src0 = S1 + p2r * R1 + NB * p2c + (HALF == 0 ? 0 : H);
    SwT X[NRB][W];
#pragma unroll
    for (int r = 0; r < NRB; ++r) {
      if (r <= PA - SAMAX || r <= PA - sA) {
        const V* src = reinterpret_cast<const V*>(src0 + K<L>::off1v.v[r] * R1);
#pragma unroll
        for (int q = 0; q < W / VN; ++q) {
          const V v = src[q];
          if constexpr (VN == 4) {
            X[r][4 * q] = v.x; X[r][4 * q + 1] = v.y; X[r][4 * q + 2] = v.z; X[r][4 * q + 3] = v.w;
          } else {
            X[r][2 * q] = v.x; X[r][2 * q + 1] = v.y;
          }
        }
      } else {
#pragma unroll
        for (int b = 0; b < W; ++b) X[r][b] = SwT(0);
      }
    }
    if constexpr (HALF == 0) {
      SwT Y0[NRB + 1][H];
#pragma unroll
      for (int j = 0; j < H; ++j) {
        Y0[0][j] = X[0][j];
#pragma unroll
        for (int t = 1; t < NRB; ++t) Y0[t][j] = X[t][j] + X[t - 1][H + j];
        Y0[NRB][j] = X[NRB - 1][H + j];
      }
      rsweep<PB - 1, 0, NRB + 1, 0>(Y0, e2);
    } else {
      rsweep<PB - 1, 1, NRB, H>(X, e2);
    }
  }
}

template <int L> struct UO { static constexpr UnitOrder o = mk_unit_order(L); };

// Phase C of one wave: its units have KMIN <= |sigma_AB| <= KMAX. Counter
// rows past KAB - |sigma_AB| are zero: dropped at compile time past
// KAB - KMIN, and below that read as zeros (a zeroed LDS row where KMIN = 0,
// so the loads issue without branches). PART 2 walks all output prefixes over
// the C bits; PART 0 the sigma = 0 subtree of the first C site (all 8
// inputs), PART 1 its sigma = 1 subtree (the 4 tau = 1 inputs).
template <int L, int KMIN, int KMAX, int PART, typename SwT>
__device__ __forceinline__ void phase_c(const SwT* S2, SwT* Z, const int (&zr)[NC], int sAB,
                                        int u3, const SwT* zrow) {
  if constexpr (KMIN <= L) {
    using V = typename Vec4<SwT>::type;
    constexpr int VN = Vec4<SwT>::n;
    constexpr int S2U = K<L>::S2U;
    constexpr int NR = KAB + 1 - KMIN;
    constexpr int H0 = PART == 1 ? 1 : 0;       // first half (c / 4) read
    constexpr int W = PART == 1 ? NC / 2 : NC;  // inputs read
    SwT X3[NR][W];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const bool in = i <= KAB - KMAX || i <= KAB - sAB;
      if (KMIN > 0 && !in) {   // past this unit's counters: zero, not read
#pragma unroll
        for (int c = 0; c < W; ++c) X3[i][c] = SwT(0);
        continue;
      }
#pragma unroll
      for (int h = H0; h < 2; ++h) {
        const V* src = reinterpret_cast<const V*>(
            KMIN > 0 || in ? S2 + ((2 * i + h) * S2U + u3) * 4 : zrow);
#pragma unroll
        for (int q = 0; q < 4 / VN; ++q) {
          const V v = src[q];
          const int c0 = 4 * (h - H0) + VN * q;
          if constexpr (VN == 4) {
            X3[i][c0] = v.x; X3[i][c0 + 1] = v.y; X3[i][c0 + 2] = v.z; X3[i][c0 + 3] = v.w;
          } else {
            X3[i][c0] = v.x; X3[i][c0 + 1] = v.y;
          }
        }
      }
    }
    EmitZ<SwT, L, KMIN, KMAX> ez{Z, zr, sAB};
    if constexpr (PART == 2) {
      rsweep<PC, 0, NR, 0>(X3, ez);
    } else if constexpr (PART == 0) {
      constexpr int H = NC / 2;
      SwT Y0[NR + 1][H];
#pragma unroll
      for (int j = 0; j < H; ++j) {
        Y0[0][j] = X3[0][j];
#pragma unroll
        for (int t = 1; t < NR; ++t) Y0[t][j] = X3[t][j] + X3[t - 1][H + j];
        Y0[NR][j] = X3[NR - 1][H + j];
      }
      rsweep<PC - 1, 0, NR + 1, 0>(Y0, ez);
    } else {
      rsweep<PC - 1, 1, NR, NC / 2>(X3, ez);
    }
  }
}

// ---------------------------------------------------------- wave priority
// Two workgroups share each SIMD (one wave of each). Within a step separated
// by barriers the waves' shares of the work differ; the wave with the
// longest share is issued first (s_setprio), so the other workgroup's waves
// fill the idle cycles instead of delaying that step's slowest wave.
template <int P> __device__ __forceinline__ void wave_prio() { __builtin_amdgcn_s_setprio(P); }
// phase B: (half 0, low |sigma_A|) > (half 0, high) > (half 1, low) > (half 1, high)
constexpr int kPrioB[NT / 64] = {3, 2, 1, 0};
// phase C: heavy sigma = 0 subtrees > low-|sigma_AB| whole trees > heavy
// sigma = 1 subtrees > the rest
constexpr int prio_c(int w) {
  return w == kCWaveH0 ? 3 : w == kCWaveR0 ? 2 : w == kCWaveH1 ? 1 : 0;
}
// the two-wave Moebius steps run ahead of the idle waves' next step; the
// weight core and the gather (every wave an equal share) stay at 0, behind
// the sweep steps of the other workgroup
constexpr int kPrioTwoWave = 1;

// ------------------------------------------------------------------ item
template <int L, typename SwT, typename MobT, bool IN64, bool MOBIN>
__device__ __forceinline__ void run_item(const FastClassDev* __restrict__ C, const InstDev& I,
                                         const FastItem& W, const float* __restrict__ vals32,
                                         const double* __restrict__ vals64,
                                         const int32_t* __restrict__ torder,
                                         double* __restrict__ partial, unsigned char* smem) {
  static_assert(kFastRuns == kRuns, "gather positions");
  constexpr int NP = np_order(L);     // gather positions of this order
  constexpr int KMAX = 2 * NP;        // output slots
  constexpr int LB = K<L>::LB;
  using LD = Lds<L, SwT, MobT>;
  MobT* R = reinterpret_cast<MobT*>(smem);
  SwT* S2 = reinterpret_cast<SwT*>(smem);
  double* Y = reinterpret_cast<double*>(smem + LD::yoff);
  SwT* S1 = reinterpret_cast<SwT*>(smem + LD::reg1);
  SwT* Z = reinterpret_cast<SwT*>(smem + LD::reg1);
  double* lamL = reinterpret_cast<double*>(smem + LD::reg1 + LD::reg2);
  const SwT* zrow = reinterpret_cast<const SwT*>(smem + LdsAll<SwT, MobT>::zoff);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  // ---- per-item thread constants ----
  // phase B: thread (half, rankA, c); half = tid / 128 is wave-uniform
  // (waves 0, 2: sigma_A ranks 0-7; waves 1, 3: ranks 8-15)
  const int p2r = (((tid & 127) >> 6) << 3) | (tid & 7), p2c = (tid >> 3) & 7;
  const int sA_mask = (int)((kOrderANibbles >> (4 * p2r)) & 15u);
  const int sA = __popc(sA_mask);
  const int wb = ((p2c >> 2) * K<L>::S2U + p2r) * 4 + (p2c & 3);
  // phase C: thread = unit
  const int u3r = C->uperm[tid];
  const bool c_on = u3r >= 0;   // this thread has a phase-C unit
  const int u3 = c_on ? u3r : 0;
  const int sAB = __popc(C->unit_mask[u3]);
  int zr[NC];
#pragma unroll
  for (int sc = 0; sc < NC; ++sc) zr[sc] = C->zrow[u3 * NC + sc];
  // cross-tile sum (the output metadata is re-read per tile from L1/L2 so it
  // holds no registers during the sweep phases)
  double acc[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) acc[k] = 0.0;
  const uint4* meta_g = reinterpret_cast<const uint4*>(C->meta + (size_t)tid * kFastMetaStride);
  // j-stride of Y per (position, wave)
  const cdptr_u gs8 = (cdptr_u)(C->gs8 + wave);
  const int nkk = C->nkk;
  // input already Moebius-transformed (a separate instantiation): the
  // butterflies are skipped
  constexpr bool mob = !MOBIN;
  const int mshift = C->mshift;
  const uint32_t omask = (1u << mshift) - 1u;
  int u_prev = -1;

  const int64_t vbase = I.voff;
  using RawT = typename std::conditional<IN64, double, float>::type;
  RawT xraw[NC];   // next tile's raw values (converted when its butterfly starts)
  // an instance with d < 11 (lowmask = 2^d - 1) runs as d = 11: the value
  // of U is v(U & lowmask), and its Moebius coefficients past bit d - 1
  // are zero (Moebius input)
  const int lowmask = I.lowmask;
  auto load_tile = [&](int UH) {
    const int64_t base = vbase + ((int64_t)UH << B);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int idx = tid + (c << 8);
      const int64_t at = base + (idx & lowmask);
      if constexpr (MOBIN) {
        if constexpr (IN64) xraw[c] = idx <= lowmask ? vals64[at] : 0.0;
        else xraw[c] = idx <= lowmask ? vals32[at] : 0.f;
      } else {
        if constexpr (IN64) xraw[c] = vals64[at];
        else xraw[c] = vals32[at];
      }
    }
  };
  int UH = torder[I.tofs + W.tb];
  load_tile(UH);

  for (int k = W.tb; k < W.te; ++k) {
    const int UHn = k + 1 < W.te ? torder[I.tofs + k + 1] : 0;
    const int u = __builtin_amdgcn_readfirstlane(__popc(UH));
    if (u != u_prev) {
      // tiles run in order of |U_H|: the weights change at most h + 1 times
      const double* src = C->lam + (int64_t)u * LB;
      for (int i = tid; i < LB; i += NT) lamL[i] = src[i];
      u_prev = u;
    }

    // ---- Moebius over bits 8-10 in registers, then transpose (ahead of
    // the other workgroup's weight core and gather) ----
    wave_prio<1>();
    MobT xr[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if constexpr (IN64) xr[c] = mob_from_d<MobT>(xraw[c]);
      else xr[c] = mob_from<MobT>(xraw[c]);
    }
    if (mob) {
#pragma unroll
      for (int bit = 0; bit < PC; ++bit)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c & (1 << bit)) xr[c] = sub(xr[c], xr[c ^ (1 << bit)]);
    }
    {
      MobT* rp = R + (tid & 15) + RB * (tid >> 4);
#pragma unroll
      for (int c = 0; c < NC; ++c) rp[RC_ * c] = xr[c];
    }
    wave_prio<0>();
    __syncthreads();
    // ---- Moebius over bits 4-7: thread (a, c) holds the 16 b values ----
    if (tid < NA * NC) {
      wave_prio<kPrioTwoWave>();
      MobT* rp = R + (tid & 15) + RC_ * (tid >> 4);
      MobT y[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) y[b] = rp[RB * b];
      if (mob) {
#pragma unroll
        for (int bit = 0; bit < PB; ++bit)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            if (b & (1 << bit)) y[b] = sub(y[b], y[b ^ (1 << bit)]);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) rp[RB * b] = y[b];
      wave_prio<0>();
    }
    __syncthreads();
    // ---- Moebius over bits 0-3 + phase A: thread (b, c) of waves 2-3 holds
    // the 16 a values (waves 0-1 ran the B bits: the two-wave steps are
    // spread over all four SIMDs) ----
    if (tid >= NT - NB * NC) {
      wave_prio<kPrioTwoWave>();
      const int ta = tid - (NT - NB * NC);
      const MobT* rp = R + RB * (ta & 15) + RC_ * (ta >> 4);
      MobT y[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) y[a] = rp[a];
      if (mob) {
#pragma unroll
        for (int bit = 0; bit < PA; ++bit)
#pragma unroll
          for (int a = 0; a < NA; ++a)
            if (a & (1 << bit)) y[a] = sub(y[a], y[a ^ (1 << bit)]);
      }
      SwT X1[1][NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) X1[0][a] = to_sw<SwT>(y[a]);
      EmitS1<SwT, L> e1{S1 + ta};
      rsweep<PA, 0, 1, 0>(X1, e1);
      wave_prio<0>();
    }
    __syncthreads();
    // ---- phase B: thread (half, sigma_A, c), counters relative to |sigma_A|;
    // the first output site (b bit 3) is split between the two halves of the
    // workgroup: half 0 walks the sigma = 0 subtree, half 1 the sigma = 1
    // subtree (which needs only the tau = 1 inputs); in each half the second
    // wave holds the sigma_A with |sigma_A| >= 2 ----
    switch (wave) {
      case 0:
        wave_prio<kPrioB[0]>();
        phase_b<L, 0, kSALoMax, 0, SwT>(S1, S2 + wb, sA, p2r, p2c);
        break;
      case 1:
        wave_prio<kPrioB[1]>();
        phase_b<L, kSAHi, kSAHiMax, 0, SwT>(S1, S2 + wb, sA, p2r, p2c);
        break;
      case 2:
        wave_prio<kPrioB[2]>();
        phase_b<L, 0, kSALoMax, 1, SwT>(S1, S2 + wb, sA, p2r, p2c);
        break;
      default:
        wave_prio<kPrioB[3]>();
        phase_b<L, kSAHi, kSAHiMax, 1, SwT>(S1, S2 + wb, sA, p2r, p2c);
        break;
    }
    wave_prio<0>();
    __syncthreads();
    // ---- phase C: thread per unit sigma_AB (units in order of |sigma_AB|,
    // the heavy ones split between two waves), counters relative to
    // |sigma_AB| ----
    if (c_on) {
      using O = UO<L>;
      switch (wave) {
        case 0:
          wave_prio<prio_c(0)>();
          phase_c<L, O::o.kmin[0], O::o.kmax[0], O::o.part[0], SwT>(S2, Z, zr, sAB, u3, zrow);
          break;
        case 1:
          wave_prio<prio_c(1)>();
          phase_c<L, O::o.kmin[1], O::o.kmax[1], O::o.part[1], SwT>(S2, Z, zr, sAB, u3, zrow);
          break;
        case 2:
          wave_prio<prio_c(2)>();
          phase_c<L, O::o.kmin[2], O::o.kmax[2], O::o.part[2], SwT>(S2, Z, zr, sAB, u3, zrow);
          break;
        default:
          wave_prio<prio_c(3)>();
          phase_c<L, O::o.kmin[3], O::o.kmax[3], O::o.part[3], SwT>(S2, Z, zr, sAB, u3, zrow);
          break;
      }
      wave_prio<0>();
    }
    // prefetch the next tile and this tile's output metadata while the
    // weight core runs
    if (k + 1 < W.te) load_tile(UHn);
    uint32_t meta[(NP + 3) & ~3];
#pragma unroll
    for (int q = 0; q < (NP + 3) / 4; ++q) {
      const uint4 v = meta_g[q];
      meta[4 * q] = v.x; meta[4 * q + 1] = v.y; meta[4 * q + 2] = v.z; meta[4 * q + 3] = v.w;
    }
    __syncthreads();
    // ---- final weight core -> Y ----
    {
      const cdptr lamg = (cdptr)(C->lam + (int64_t)u_prev * LB);
      // lanes past a task's rows write here: the transpose region, dead
      // between phase C and the next tile
      double* dump = reinterpret_cast<double*>(smem);
      switch (wave) {
        case 0: lam_wave<L, 0, SwT>(lane, Z, Y, lamL, lamg, dump); break;
        case 1: lam_wave<L, 1, SwT>(lane, Z, Y, lamL, lamg, dump); break;
        case 2: lam_wave<L, 2, SwT>(lane, Z, Y, lamL, lamg, dump); break;
        default: lam_wave<L, 3, SwT>(lane, Z, Y, lamL, lamg, dump); break;
      }
    }
    __syncthreads();
    // ---- cross-tile sum: E_S += Y[S_L, s_H, |S_H & U_H|] ----
    // position p holds a run of two outputs (ranks 2r, 2r + 1 of one |S_L|,
    // one S_H): one popcount and one 16-byte read; the j-stride is uniform
    // in the wave
    {
      const uint32_t UHs = (uint32_t)UH << mshift;
      const unsigned char* Yb = reinterpret_cast<const unsigned char*>(Y);
      constexpr int GB = 5;   // runs per batch of reads
#pragma unroll
      for (int p0 = 0; p0 < NP; p0 += GB) {
        double2 v[GB];
#pragma unroll
        for (int q = 0; q < GB; ++q) {
          if (p0 + q < NP) {
            const uint32_t m = meta[p0 + q];
            const uint32_t off = (m & omask) + (uint32_t)__popc(m & UHs) * gs8[(p0 + q) * 4];
            v[q] = *reinterpret_cast<const double2*>(Yb + off);
          }
        }
#pragma unroll
        for (int q = 0; q < GB; ++q)
          if (p0 + q < NP) {
            acc[2 * (p0 + q)] += v[q].x;
            acc[2 * (p0 + q) + 1] += v[q].y;
          }
      }
    }
    UH = UHn;
    // no barrier: the next tile's first writes (the transpose region, and
    // the weights once every wave has passed the barrier before this
    // gather) do not touch Y
  }
  double* P = partial + W.pofs + tid;
#pragma unroll
  for (int kk = 0; kk < KMAX; ++kk)
    if (kk < nkk) P[kk * NT] = acc[kk];
}

// Work queue of a launch: workgroup b runs item b first, then takes the
// next unclaimed item (from gridDim.x on) each time it is done, so items of
// unequal cost (instances of different d and l in one batch) spread over the
// machine as they finish (items are sorted by decreasing cost). queue[0]
// counts the items taken after the first round, queue[1] the workgroups
// that found the queue empty; the last of those clears both for the next
// launch on the stream. A launch with no more items than workgroups does
// not touch the queue.
__device__ __forceinline__ int next_item(uint32_t* queue, int n_items) {
  if (n_items <= (int)gridDim.x) return n_items;
  __shared__ int s_item;
  if (threadIdx.x == 0) s_item = (int)(gridDim.x + atomicAdd(queue, 1u));
  __syncthreads();
  return s_item;
}
__device__ __forceinline__ void queue_done(uint32_t* queue, int n_items) {
  if (n_items > (int)gridDim.x && threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(queue + 1, 1u) == gridDim.x - 1) {
      __threadfence();
      atomicExch(queue, 0u);
      atomicExch(queue + 1, 0u);
    }
  }
}

// One kernel per order l (the items of a launch all have that order).
// FP32 sweep: two workgroups per CU (2 waves per SIMD), so at most 256 VGPRs
// per thread; the FP64 sweep's LDS allows one workgroup per CU.
template <int L, typename SwT, typename MobT, bool IN64, int WPE, bool MOBIN>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
tile11_kernel(const FastClassDev* __restrict__ classes, const InstDev* __restrict__ insts,
              const FastItem* __restrict__ items, int n_items,
              const float* __restrict__ vals32, const double* __restrict__ vals64,
              const int32_t* __restrict__ torder, double* __restrict__ partial,
              uint32_t* __restrict__ queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  {
    using LA = LdsAll<SwT, MobT>;
    uint32_t* z = reinterpret_cast<uint32_t*>(smem + LA::zoff);
    if (threadIdx.x < LA::zeros / 4) z[threadIdx.x] = 0u;
    __syncthreads();
  }
  for (int item = blockIdx.x; item < n_items; item = next_item(queue, n_items)) {
    const FastItem W = items[item];
    const InstDev I = insts[W.inst];
    run_item<L, SwT, MobT, IN64, MOBIN>(classes + I.fcls, I, W, vals32, vals64, torder, partial,
                                        smem);
    __syncthreads();
  }
  queue_done(queue, n_items);
}

// Items of every order in one launch (a batch of instances with different
// l): each item runs the code compiled for its instance's order; the
// regions of all orders share one allocation (LdsAll).
template <typename SwT, typename MobT, bool IN64, int WPE, bool MOBIN>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
tile11_mixed_kernel(const FastClassDev* __restrict__ classes, const InstDev* __restrict__ insts,
                    const FastItem* __restrict__ items, int n_items,
                    const float* __restrict__ vals32, const double* __restrict__ vals64,
                    const int32_t* __restrict__ torder, double* __restrict__ partial,
                    uint32_t* __restrict__ queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  {
    using LA = LdsAll<SwT, MobT>;
    uint32_t* z = reinterpret_cast<uint32_t*>(smem + LA::zoff);
    if (threadIdx.x < LA::zeros / 4) z[threadIdx.x] = 0u;
    __syncthreads();
  }
  for (int item = blockIdx.x; item < n_items; item = next_item(queue, n_items)) {
    const FastItem W = items[item];
    const InstDev I = insts[W.inst];
    const FastClassDev* C = classes + I.fcls;
    const int l = __builtin_amdgcn_readfirstlane(C->l);
    switch (l) {
      case 1: run_item<1, SwT, MobT, IN64, MOBIN>(C, I, W, vals32, vals64, torder, partial, smem); break;
      case 2: run_item<2, SwT, MobT, IN64, MOBIN>(C, I, W, vals32, vals64, torder, partial, smem); break;
      case 3: run_item<3, SwT, MobT, IN64, MOBIN>(C, I, W, vals32, vals64, torder, partial, smem); break;
      default: run_item<4, SwT, MobT, IN64, MOBIN>(C, I, W, vals32, vals64, torder, partial, smem); break;
    }
    __syncthreads();
  }
  queue_done(queue, n_items);
}

// Every order's kernel places the zero row past the regions of all orders
// (LdsAll), so each allocates the same size.
template <typename SwT, typename MobT>
constexpr int lds_bytes_for(int) {
  return LdsAll<SwT, MobT>::bytes;
}

}  // namespace t11

// ------------------------------------------------------------------ launcher
template <typename SwT> constexpr int wpe_for() { return sizeof(SwT) == 4 ? 2 : 1; }

// Plans whose input is already the Moebius transform run their own
// instantiations.
template <int L, typename SwT, typename MobT, bool IN64, bool MOBIN>
static hipError_t launch_t11_m(const FastLaunch& f, hipStream_t st) {
  const int ib = f.lbeg[L], n = f.lbeg[L + 1] - f.lbeg[L];
  if (n <= 0) return hipSuccess;
  auto k = t11::tile11_kernel<L, SwT, MobT, IN64, wpe_for<SwT>(), MOBIN>;
  hipLaunchKernelGGL(k, dim3(f.grid[L]), dim3(t11::NT), f.lds[L], st, f.classes, f.insts,
                     f.items + ib, n, static_cast<const float*>(f.vals32),
                     static_cast<const double*>(f.vals64), f.torder, f.partial, f.queue);
  return hipGetLastError();
}

template <int L, typename SwT, typename MobT, bool IN64>
static hipError_t launch_t11(const FastLaunch& f, hipStream_t st) {
  return f.mobius_in ? launch_t11_m<L, SwT, MobT, IN64, true>(f, st)
                     : launch_t11_m<L, SwT, MobT, IN64, false>(f, st);
}

template <int L, typename SwT, typename MobT, bool IN64, bool MOBIN>
static hipError_t config_t11_m(size_t lds) {
  auto k = t11::tile11_kernel<L, SwT, MobT, IN64, wpe_for<SwT>(), MOBIN>;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int L, typename SwT, typename MobT, bool IN64>
static hipError_t config_t11(size_t lds) {
  hipError_t e = config_t11_m<L, SwT, MobT, IN64, false>(lds);
  if (e != hipSuccess) return e;
  return config_t11_m<L, SwT, MobT, IN64, true>(lds);
}

// One launch over the items of every order (the plan has several orders).
template <typename SwT, typename MobT, bool IN64, bool MOBIN>
static hipError_t launch_mixed_m(const FastLaunch& f, hipStream_t st) {
  auto k = t11::tile11_mixed_kernel<SwT, MobT, IN64, wpe_for<SwT>(), MOBIN>;
  hipLaunchKernelGGL(k, dim3(f.grid_mixed), dim3(t11::NT), f.lds_mixed, st, f.classes, f.insts,
                     f.items, f.n_items, static_cast<const float*>(f.vals32),
                     static_cast<const double*>(f.vals64), f.torder, f.partial, f.queue);
  return hipGetLastError();
}

template <typename SwT, typename MobT, bool IN64>
static hipError_t launch_mixed_t(const FastLaunch& f, hipStream_t st) {
  return f.mobius_in ? launch_mixed_m<SwT, MobT, IN64, true>(f, st)
                     : launch_mixed_m<SwT, MobT, IN64, false>(f, st);
}

template <typename SwT, typename MobT, bool IN64, bool MOBIN>
static hipError_t config_mixed_m(size_t lds) {
  auto k = t11::tile11_mixed_kernel<SwT, MobT, IN64, wpe_for<SwT>(), MOBIN>;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename SwT, typename MobT, bool IN64>
static hipError_t config_mixed_t(size_t lds) {
  hipError_t e = config_mixed_m<SwT, MobT, IN64, false>(lds);
  if (e != hipSuccess) return e;
  return config_mixed_m<SwT, MobT, IN64, true>(lds);
}

template <typename SwT, typename MobT, bool IN64>
static hipError_t launch_group_t(const FastLaunch& f, int l, hipStream_t st) {
  switch (l) {
    case 1: return launch_t11<1, SwT, MobT, IN64>(f, st);
    case 2: return launch_t11<2, SwT, MobT, IN64>(f, st);
    case 3: return launch_t11<3, SwT, MobT, IN64>(f, st);
    case 4: return launch_t11<4, SwT, MobT, IN64>(f, st);
  }
  return hipErrorInvalidValue;
}

template <typename SwT, typename MobT, bool IN64>
static hipError_t config_all_t(const size_t* lds) {
  hipError_t e = hipSuccess;
  size_t mx = 0;
  int orders = 0;
  for (int l = 1; l <= kFastMaxL; ++l)
    if (lds[l]) { mx = std::max(mx, lds[l]); ++orders; }
  if (orders > 1 && (e = config_mixed_t<SwT, MobT, IN64>(mx)) != hipSuccess) return e;
  if (lds[1] && (e = config_t11<1, SwT, MobT, IN64>(lds[1])) != hipSuccess) return e;
  if (lds[2] && (e = config_t11<2, SwT, MobT, IN64>(lds[2])) != hipSuccess) return e;
  if (lds[3] && (e = config_t11<3, SwT, MobT, IN64>(lds[3])) != hipSuccess) return e;
  if (lds[4] && (e = config_t11<4, SwT, MobT, IN64>(lds[4])) != hipSuccess) return e;
  return e;
}

hipError_t configure_fast(int prec, const size_t* lds) {
  switch (prec) {
    case PREC_F32: return config_all_t<float, float, false>(lds);
    case PREC_F32_COMP: return config_all_t<float, t11::TwoF, false>(lds);
    case PREC_F32_FP64MOB: return config_all_t<float, double, false>(lds);
    case PREC_F64: return config_all_t<double, double, true>(lds);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fast_mixed(const FastLaunch& f, hipStream_t st) {
  switch (f.prec) {
    case PREC_F32: return launch_mixed_t<float, float, false>(f, st);
    case PREC_F32_COMP: return launch_mixed_t<float, t11::TwoF, false>(f, st);
    case PREC_F32_FP64MOB: return launch_mixed_t<float, double, false>(f, st);
    case PREC_F64: return launch_mixed_t<double, double, true>(f, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fast_group(const FastLaunch& f, int l, hipStream_t st) {
  switch (f.prec) {
    case PREC_F32: return launch_group_t<float, float, false>(f, l, st);
    case PREC_F32_COMP: return launch_group_t<float, t11::TwoF, false>(f, l, st);
    case PREC_F32_FP64MOB: return launch_group_t<float, double, false>(f, l, st);
    case PREC_F64: return launch_group_t<double, double, true>(f, l, st);
  }
  return hipErrorInvalidValue;
}

int fast_groups(const FastLaunch& f, int* ls) {
  int n = 0;
  for (int l = 1; l <= kFastMaxL; ++l)
    if (f.lbeg[l + 1] > f.lbeg[l]) {
      if (ls) ls[n] = l;
      ++n;
    }
  return n;
}

int fast_launches(const FastLaunch& f) {
  const int g = fast_groups(f, nullptr);
  return g > 1 ? 1 : g;
}

bool fast_supported(int prec) {
  return prec == PREC_F32 || prec == PREC_F32_COMP || prec == PREC_F32_FP64MOB ||
         prec == PREC_F64;
}

size_t fast_lds_bytes(int prec, int l) {
  switch (prec) {
    case PREC_F32: return t11::lds_bytes_for<float, float>(l);
    case PREC_F32_COMP: return t11::lds_bytes_for<float, t11::TwoF>(l);
    case PREC_F32_FP64MOB: return t11::lds_bytes_for<float, double>(l);
    case PREC_F64: return t11::lds_bytes_for<double, double>(l);
  }
  return 0;
}

// Workgroups of the register-phase kernel that fit on one CU.
int fast_wgs_per_cu(int prec, int l) {
  const size_t lds = fast_lds_bytes(prec, l);
  const int by_lds = lds ? (int)((160 * 1024) / lds) : 1;
  const int by_regs = prec == PREC_F64 ? 1 : 2;
  return std::max(1, std::min(by_lds, by_regs));
}

}  // namespace fsi
