// Register-phase tile kernel of the fused FSI algorithm (gfx950).
//
// One workgroup of 256 threads owns a work item: a run of tiles of one
// instance. For each tile of b = PA + PB + PC low bits (raw v, high index
// U_H) it computes
//   - the in-tile Moebius butterfly (Sec. 3.2) over all b bits: the PC bits
//     in registers straight from the coalesced global loads, then two LDS
//     transposes for the PB and PA bits;
//   - the left-to-right counter sweep (Sec. 4.3 - 4.4) in three phases of
//     PA, PB, PC sites. Within a phase a thread holds one output-prefix
//     pattern with ALL its |T| counter values and its 2^P inputs in
//     registers and walks the 2^P output bits depth first (the sparse cores:
//     per site an output state adds its tau = 0 and tau = 1 predecessors).
//     Between phases the (sigma, t) states go through LDS, truncated to
//     |sigma| <= l (the compressed output prefix);
//   - the final weight core with the high-site Moebius cores precontracted
//     (Sec. 4.5), FP64, into per-tile partial results Y;
//   - the cross-tile sum E_S += Y[S_L, s_H, |S_H & U_H|], kept in FP64
//     registers across the tiles of the work item.
// At the end of the item the FP64 partial sums go to a workspace; the
// reduction kernel adds the items of an instance and writes the outputs.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "fsi_kernels.h"

namespace fsi {
namespace fast {

constexpr int NT = kFastThreads;

// ----------------------------------------------------------------- numerics
struct TwoF {
  float hi, lo;
};
__device__ __forceinline__ TwoF sub(TwoF a, TwoF b) {
  // TwoSum of the high parts, then the low parts, renormalised (Dekker)
  const float s = a.hi - b.hi;
  const float bb = s - a.hi;
  const float e = (a.hi - (s - bb)) + (-b.hi - bb);
  const float t = e + (a.lo - b.lo);
  const float hi = s + t;
  return TwoF{hi, t - (hi - s)};
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

constexpr int cpopc(int x) { return x == 0 ? 0 : (x & 1) + cpopc(x >> 1); }

// ------------------------------------------------- in-register counter sweep
// Node of the depth-first walk over the output bits of one phase: X[t][r]
// holds the states with counter t in [LO, LO + RC) for the 2^REM inputs r of
// the bits still to consume. The most significant remaining bit is consumed
// first: the sigma = 1 child keeps the tau = 1 half with t + 1; the sigma = 0
// child adds the tau = 0 half at t and the tau = 1 half at t - 1. At a leaf
// SIG is the output mask over the phase's bits.
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

// state index of (sigma_A, t = |sigma_A|) after phase 1 (all 2^PA prefixes)
template <int PA>
constexpr int base1(int sig) {
  int b = 0;
  for (int s = 0; s < sig; ++s) b += PA + 1 - cpopc(s);
  return b;
}

// --------------------------------------------------------------- LDS layouts
// Raw-tile transposes: element (a, b, c) of the tile (index a + 16 b + 256 c)
// at row = (b + c) & 15, 16-byte chunk swizzled with row >> 2; conflict-free
// for the column (b) and row (a) accesses used below.
__device__ __forceinline__ int r_addr(int a, int b, int c) {
  const int row = (b + c) & 15;
  return (c << 8) + (row << 4) + ((((a >> 2) ^ (row >> 2)) & 3) << 2) + (a & 3);
}
// Phase-1 states: S1[p1][c][b], b chunk swizzled with c for the b128 reads.
template <int ROW1>
__device__ __forceinline__ int s1_addr(int p1, int c, int b) {
  return p1 * ROW1 + (c << 4) + ((((b >> 2) ^ (c >> 2)) & 3) << 2) + (b & 3);
}
// Phase-2 states: S2[p2][c] (2^PC counters per state), chunk swizzled by p2.
template <int NC>
__device__ __forceinline__ int s2_addr(int p2, int c) {
  if constexpr (NC >= 16)
    return p2 * NC + ((((c >> 2) ^ (p2 >> 2)) & 3) << 2) + (c & 3);
  else
    return p2 * NC + c;
}

// ----------------------------------------------------------------- emitters
// Phase 1 -> S1[p1][c][b]: p1 = base1(sigma_A) + r, r the counter relative
// to |sigma_A| (the leaf's array index).
template <typename SwT, int PA, int ROW1>
struct EmitS1 {
  SwT* S1;
  int c, b;
  template <int SIG, int LO, int RC>
  __device__ __forceinline__ void leaf(const SwT (&X)[RC][1]) {
    constexpr int base = base1<PA>(SIG);
#pragma unroll
    for (int i = 0; i < RC; ++i) S1[s1_addr<ROW1>(base + i, c, b)] = X[i][0];
  }
};

// Phase 2 -> S2[row2[r] + unit][c]. Phase 2 runs on counters relative to
// |sigma_A| (top-padded with zeros), so a leaf's array index i is the counter
// relative to |sigma_AB|. Rows past the unit's range and prefixes with
// |sigma_AB| > l go to a per-thread spare slot.
template <typename SwT, int NB, int NC>
struct EmitS2 {
  SwT* S2;
  const int* u3row;  // LDS: unit of sigma_A | sigma_B << PA, for this sigma_A
  const int* row2;   // LDS: first row of relative counter r
  int sA, n3, spare, c, kAB;
  template <int SIG, int LO, int RC>
  __device__ __forceinline__ void leaf(const SwT (&X)[RC][1]) {
    constexpr int sB = cpopc(SIG);
    const int unit = u3row[SIG];
    const int lim = kAB - sA - sB;  // last valid relative counter
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      const bool ok = unit < n3 && i <= lim;
      const int a = ok ? (row2[i] + unit) * NC + c : spare;
      S2[a] = X[i][0];
    }
  }
};

// Phase 3 -> Z[r][zbase[sigma_C] + unit] (r relative to |S_L|).
template <typename SwT, int NC>
struct EmitZ {
  SwT* Z;
  const int* zb;     // LDS: zbase[sigma_C]
  int unit, sAB, l, nzi, spare;
  template <int SIG, int LO, int RC>
  __device__ __forceinline__ void leaf(const SwT (&X)[RC][1]) {
    constexpr int sC = cpopc(SIG);
    const bool ok = sAB + sC <= l;
    const int col = ok ? zb[SIG] + unit : spare;
#pragma unroll
    for (int i = 0; i < RC; ++i) Z[i * nzi + col] = X[i][0];
  }
};

// ------------------------------------------------------------------- kernel
template <typename SwT, typename MobT, bool IN64, int PA, int PB, int PC, int KMAX, int KY>
__global__ void __launch_bounds__(NT)
fast_tile_kernel(const FastClassDev* __restrict__ classes, const InstDev* __restrict__ insts,
                 const FastItem* __restrict__ items, int n_items,
                 const float* __restrict__ vals32, const double* __restrict__ vals64,
                 const int32_t* __restrict__ torder, double* __restrict__ partial) {
  static_assert(PA == 4 && PB == 4, "phase split");
  constexpr int NA = 1 << PA, NB = 1 << PB, NC = 1 << PC;
  constexpr int B = PA + PB + PC;
  constexpr int KAB = PA + PB;
  constexpr int ROW1 = NB * NC;              // S1 row: all (c, b) of one state
  constexpr int P1 = base1<PA>(NA);          // states after phase 1 (48)
  constexpr int RC2 = PA + 1;                // relative counters entering phase 2
  constexpr int RC3 = KAB + 1;               // relative counters entering phase 3

  extern __shared__ __align__(16) unsigned char smem[];
  // region A: S1 (phase-1 states), later Z (final states)
  // region B: raw-tile transposes, S2 (phase-2 states), later Y
  SwT* regA = reinterpret_cast<SwT*>(smem);
  const int tid = threadIdx.x;

  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    const FastItem W = items[item];
    const InstDev I = insts[W.inst];
    const FastClassDev* C = classes + I.fcls;
    const int l = C->l;
    const int M = C->M;
    const int n3 = C->n3;
    const int nzi = C->nzi;
    const int regA_bytes = (int)(((size_t)(P1 * ROW1 > (B + 1) * nzi ? P1 * ROW1 : (B + 1) * nzi) *
                                  sizeof(SwT) + 255) & ~(size_t)255);
    unsigned char* regB = smem + regA_bytes;
    // per-item LDS tables (offsets from FastClassDev::tabo):
    //   u3tab [NA*NB] | row2 [16] | zbase [NC] | lam_soff [8] | gsize [8] | weights
    int* u3L = reinterpret_cast<int*>(regB + C->tabo);
    int* row2L = u3L + NA * NB;
    int* zbL = row2L + 16;
    int* lsoffL = zbL + NC;
    int* gsL = lsoffL + 8;
    double* lamL = reinterpret_cast<double*>(regB + C->tabo + C->lamo);
    SwT* S2 = reinterpret_cast<SwT*>(regB);
    double* Y = reinterpret_cast<double*>(regB);
    MobT* R = reinterpret_cast<MobT*>(regB);
    SwT* S1 = regA;
    SwT* Z = regA;
    for (int i = tid; i < NA * NB; i += NT) u3L[i] = C->u3tab[i];
    if (tid <= KAB) row2L[tid] = C->row2[tid];
    if (tid < NC) zbL[tid] = C->zbase[tid];
    if (tid <= l) { lsoffL[tid] = C->lam_soff[tid]; gsL[tid] = C->gsize[tid]; }
    // phase-3 unit of this thread, final-core entries of this thread
    const int sAB3 = tid < n3 ? C->unit_s[tid] : 0;
    uint32_t ytabR[KY];
#pragma unroll
    for (int j = 0; j < KY; ++j) ytabR[j] = C->ytab[tid + j * NT];
    // spare slots (discarded writes): per thread, past the live data
    const int spare2 = (C->row2[KAB] + 1) * NC + tid;   // in S2 (row2[KAB] = last row start)
    const int spareZ = nzi - 1;                          // spare Z column

    double acc[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) acc[k] = 0.0;
    uint32_t meta[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int g = tid + k * NT;
      // outputs past M read the spare Y slot Ysize - 1 (a padding entry)
      meta[k] = g < M ? C->ometa[g] : (uint32_t)(C->Ysize - 1);
    }

    const int64_t vbase = I.voff;
    int u_prev = -1;
    // raw tile registers: thread (a, b) = tid holds c = 0 .. NC-1
    MobT xr[NC];
    auto load_tile = [&](int UH) {
      const int64_t base = vbase + ((int64_t)UH << B);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if constexpr (IN64)
          xr[c] = mob_from_d<MobT>(vals64[base + tid + (c << 8)]);
        else
          xr[c] = mob_from<MobT>(vals32[base + tid + (c << 8)]);
      }
    };
    int UH = torder[I.tofs + W.tb];
    load_tile(UH);
    __syncthreads();   // tables visible

    for (int k = W.tb; k < W.te; ++k) {
      const int UHn = k + 1 < W.te ? torder[I.tofs + k + 1] : 0;
      const int u = __popc(UH);
      if (u != u_prev) {
        const double* src = C->lam + (int64_t)u * C->lam_ublock;
        for (int i = tid; i < C->lam_ublock; i += NT) lamL[i] = src[i];
        u_prev = u;
      }
      // ---- in-tile Moebius: C bits in registers ----
#pragma unroll
      for (int bit = 0; bit < PC; ++bit)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c & (1 << bit)) xr[c] = sub(xr[c], xr[c ^ (1 << bit)]);
      {
        const int a = tid & 15, b = tid >> 4;
#pragma unroll
        for (int c = 0; c < NC; ++c) R[r_addr(a, b, c)] = xr[c];
      }
      __syncthreads();
      // ---- B bits: thread (a, c) holds the 16 b values ----
      if (tid < NA * NC) {
        const int a = tid & 15, c = tid >> 4;
        MobT y[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) y[b] = R[r_addr(a, b, c)];
#pragma unroll
        for (int bit = 0; bit < PB; ++bit)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            if (b & (1 << bit)) y[b] = sub(y[b], y[b ^ (1 << bit)]);
#pragma unroll
        for (int b = 0; b < NB; ++b) R[r_addr(a, b, c)] = y[b];
      }
      __syncthreads();
      // ---- A bits + phase 1: thread (b, c) holds the 16 a values ----
      if (tid < NB * NC) {
        const int b = tid & 15, c = tid >> 4;
        MobT y[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) y[a] = R[r_addr(a, b, c)];
#pragma unroll
        for (int bit = 0; bit < PA; ++bit)
#pragma unroll
          for (int a = 0; a < NA; ++a)
            if (a & (1 << bit)) y[a] = sub(y[a], y[a ^ (1 << bit)]);
        SwT X1[1][NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) X1[0][a] = to_sw<SwT>(y[a]);
        EmitS1<SwT, PA, ROW1> e1{S1, c, b};
        rsweep<PA, 0, 1, 0>(X1, e1);
      }
      // prefetch the next tile while the sweep runs
      if (k + 1 < W.te) load_tile(UHn);
      __syncthreads();
      // ---- phase 2: thread (sigma_A, c), counters relative to |sigma_A| ----
      if (tid < NA * NC) {
        const int c = tid % NC, sA_mask = tid / NC;
        const int sA = __popc(sA_mask);
        const int p1b = [&] {
          int bb = 0;
          for (int s = 0; s < sA_mask; ++s) bb += PA + 1 - __popc(s);
          return bb;
        }();
        const int rmax = PA - sA;          // last valid relative counter
        SwT X2[RC2][NB];
#pragma unroll
        for (int r = 0; r < RC2; ++r) {
          const int rr = r <= rmax ? r : rmax;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const SwT v = S1[s1_addr<ROW1>(p1b + rr, c, b)];
            X2[r][b] = r <= rmax ? v : SwT(0);
          }
        }
        EmitS2<SwT, NB, NC> e2{S2, u3L + sA_mask * NB, row2L, sA, n3, spare2, c, KAB};
        rsweep<PB, 0, RC2, 0>(X2, e2);
      }
      __syncthreads();
      // ---- phase 3: thread per unit sigma_AB, counters relative to |sigma_AB| ----
      if (tid < n3) {
        const int rmax = KAB - sAB3;
        SwT X3[RC3][NC];
#pragma unroll
        for (int r = 0; r < RC3; ++r) {
          const int rr = r <= rmax ? r : rmax;
          const int base = (row2L[rr] + tid) * NC;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const SwT v = S2[base + c];
            X3[r][c] = r <= rmax ? v : SwT(0);
          }
        }
        EmitZ<SwT, NC> ez{Z, zbL, tid, sAB3, l, nzi, spareZ};
        rsweep<PC, 0, RC3, 0>(X3, ez);
      }
      __syncthreads();
      // ---- final weight core: Y[e] = sum_r lambda_u[s_L][slot][r] Z[r][col] ----
      // (weights are zero past the last counter of the entry; the row index is
      // clamped so every load stays inside written data)
#pragma unroll
      for (int j = 0; j < KY; ++j) {
        const uint32_t q = ytabR[j];
        const int col = (int)(q & 0xFFFFu);
        const int sL = (int)((q >> 16) & 31u);
        const int slot = (int)(q >> 21);
        const double* lw = lamL + lsoffL[sL] + slot * (B + 1);
        const int rl = B - sL;
        double zv[B + 1], lv[B + 1];
#pragma unroll
        for (int r = 0; r <= B; ++r) {
          const int rr = r <= rl ? r : rl;
          zv[r] = (double)Z[rr * nzi + col];
          lv[r] = lw[r];
        }
        double a = 0.0;
#pragma unroll
        for (int r = 0; r <= B; ++r) a = fma(lv[r], zv[r], a);
        Y[tid + j * NT] = a;
      }
      __syncthreads();
      // ---- cross-tile sum: E_S += Y[S_L, s_H, |S_H & U_H|] ----
#pragma unroll
      for (int kk = 0; kk < KMAX; ++kk) {
        const uint32_t m = meta[kk];
        const int sl = (int)((m >> 16) & 7u);
        const int j = __popc((m >> 19) & (uint32_t)UH);
        acc[kk] += Y[(m & 0xFFFFu) + j * gsL[sl]];
      }
      UH = UHn;
      __syncthreads();
    }
    double* P = partial + W.pofs;
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) {
      const int g = tid + kk * NT;
      if (g < M) P[g] = acc[kk];
    }
    __syncthreads();
  }
}

}  // namespace fast

// ------------------------------------------------------------------ launcher
template <typename SwT, typename MobT, bool IN64, int PC>
static hipError_t launch_fast_t(const FastLaunch& f, hipStream_t st) {
  auto k = fast::fast_tile_kernel<SwT, MobT, IN64, 4, 4, PC, kFastKmax, kFastKy>;
  hipLaunchKernelGGL(k, dim3(f.grid), dim3(kFastThreads), f.lds, st, f.classes, f.insts,
                     f.items, f.n_items, static_cast<const float*>(f.vals32),
                     static_cast<const double*>(f.vals64), f.torder, f.partial);
  return hipGetLastError();
}

template <typename SwT, typename MobT, bool IN64, int PC>
static hipError_t config_fast_t(size_t lds) {
  auto k = fast::fast_tile_kernel<SwT, MobT, IN64, 4, 4, PC, kFastKmax, kFastKy>;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t configure_fast(int prec, size_t lds) {
  switch (prec) {
    case PREC_F32: return config_fast_t<float, float, false, 3>(lds);
    case PREC_F32_COMP: return config_fast_t<float, fast::TwoF, false, 3>(lds);
    case PREC_F32_FP64MOB: return config_fast_t<float, double, false, 3>(lds);
    case PREC_F64: return config_fast_t<double, double, true, 3>(lds);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fast(const FastLaunch& f, hipStream_t st) {
  switch (f.prec) {
    case PREC_F32: return launch_fast_t<float, float, false, 3>(f, st);
    case PREC_F32_COMP: return launch_fast_t<float, fast::TwoF, false, 3>(f, st);
    case PREC_F32_FP64MOB: return launch_fast_t<float, double, false, 3>(f, st);
    case PREC_F64: return launch_fast_t<double, double, true, 3>(f, st);
  }
  return hipErrorInvalidValue;
}

int fast_pc(int prec) { (void)prec; return 3; }
bool fast_supported(int prec) {
  return prec == PREC_F32 || prec == PREC_F32_COMP || prec == PREC_F32_FP64MOB ||
         prec == PREC_F64;
}

// Region A holds the phase-1 states (48 states x 2^(PB+PC) inputs), later
// the final (S_L, t) states; region B (after it) holds the raw-tile
// transposes, then the phase-2 states, then the partial results, followed by
// the per-item tables at byte offset FastClassDev::tabo.
size_t fast_regA_bytes(int prec, int nzi) {
  const size_t sw = prec == PREC_F64 ? 8 : 4;
  const size_t NC = (size_t)1 << fast_pc(prec);
  const size_t B = 8 + fast_pc(prec);
  const size_t cells = std::max<size_t>(48 * 16 * NC, (B + 1) * (size_t)nzi);
  return (cells * sw + 255) & ~(size_t)255;
}

}  // namespace fsi
