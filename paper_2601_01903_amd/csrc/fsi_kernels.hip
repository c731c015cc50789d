// HIP kernels (gfx950) of the FSI operator.
//
//   tile kernel    : per tile of the low b bits of one instance, the in-tile
//                    Moebius butterfly (fused algorithm), the left-to-right
//                    counter sweep over the b tile sites (Sec. 4.3 - 4.4,
//                    Algorithm 1 with the output prefix compressed to
//                    |sigma| <= l), and the final weight core -> per-tile
//                    partial results Y (FP64).
//   reduce kernel  : E_S = sum over tiles of the partial result selected by
//                    the tile's high index (FP64 accumulation, fixed order).
//   Moebius kernels: the in-place butterfly of the two-pass algorithm:
//                    low bits staged in LDS, high bits as strided passes.
//
// All kernels are persistent: a grid sized to the machine walks a work list.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "fsi_kernels.h"

namespace fsi {

// ---------------------------------------------------------------- numerics
// Two-float value hi + lo (|lo| <= ulp(hi)/2), used for the compensated
// Moebius butterfly. Subtraction follows Knuth's TwoSum followed by a
// Fast2Sum renormalisation (Dekker's double-length arithmetic).
struct TwoFloat {
  float hi, lo;
};

__device__ __forceinline__ TwoFloat tf_sub(TwoFloat a, TwoFloat b) {
  const float s = a.hi - b.hi;
  const float bb = s - a.hi;
  const float e = (a.hi - (s - bb)) + (-b.hi - bb);   // exact error of s
  const float t = e + (a.lo - b.lo);
  const float hi = s + t;
  const float lo = t - (hi - s);
  return TwoFloat{hi, lo};
}

template <typename T> struct Num;
template <> struct Num<float> {
  __device__ static float from_in(float x) { return x; }
  __device__ static float from_in(double x) { return (float)x; }
  __device__ static float sub(float a, float b) { return a - b; }
  __device__ static float zero() { return 0.f; }
};
template <> struct Num<double> {
  __device__ static double from_in(float x) { return (double)x; }
  __device__ static double from_in(double x) { return x; }
  __device__ static double sub(double a, double b) { return a - b; }
  __device__ static double zero() { return 0.0; }
};
template <> struct Num<TwoFloat> {
  __device__ static TwoFloat from_in(float x) { return TwoFloat{x, 0.f}; }
  __device__ static TwoFloat from_in(double x) {
    const float hi = (float)x;
    return TwoFloat{hi, (float)(x - (double)hi)};
  }
  __device__ static TwoFloat from_in(TwoFloat x) { return x; }
  __device__ static TwoFloat sub(TwoFloat a, TwoFloat b) { return tf_sub(a, b); }
  __device__ static TwoFloat zero() { return TwoFloat{0.f, 0.f}; }
};

// conversion of a Moebius-stage value to the sweep type
__device__ __forceinline__ float to_sweep(float x, float*) { return x; }
__device__ __forceinline__ float to_sweep(double x, float*) { return (float)x; }
__device__ __forceinline__ float to_sweep(TwoFloat x, float*) { return x.hi + x.lo; }
__device__ __forceinline__ double to_sweep(float x, double*) { return (double)x; }
__device__ __forceinline__ double to_sweep(double x, double*) { return x; }
__device__ __forceinline__ double to_sweep(TwoFloat x, double*) {
  return (double)x.hi + (double)x.lo;
}

__device__ __forceinline__ float load_as(const float* p, float*) { return *p; }
__device__ __forceinline__ double load_as(const double* p, double*) { return *p; }
__device__ __forceinline__ TwoFloat load_as(const TwoFloat* p, TwoFloat*) { return *p; }

// ---------------------------------------------------------------- tile kernel
template <typename SrcT, typename MobT, typename SwT, bool kMobius>
__global__ void __launch_bounds__(kTileThreads)
tile_kernel(const ClassDev* __restrict__ classes, const InstDev* __restrict__ insts,
            const TileItem* __restrict__ items, int n_items, const SrcT* __restrict__ src,
            double* __restrict__ Y, double* __restrict__ Ylo) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  constexpr int NT = kTileThreads;
  constexpr int kPer = (1 << kMaxTileBits) / NT;

  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const TileItem w = items[it];
    const InstDev I = insts[w.inst];
    const ClassDev* C = classes + I.cls;
    const int b = C->b;
    const int nt = 1 << b;
    const int lds_elems = C->lds_elems;
    SwT* cur = reinterpret_cast<SwT*>(smem);
    SwT* nxt = cur + lds_elems;

    if constexpr (kMobius) {
      // in-tile Moebius butterfly over the b low bits (Kronecker factors
      // [[1, 0], [-1, 1]], Sec. 4.2), staged in LDS in the Moebius type
      MobT* m = reinterpret_cast<MobT*>(smem);
      const SrcT* v = src + I.voff + ((int64_t)w.tile << b);
      for (int i = tid; i < nt; i += NT) m[i] = Num<MobT>::from_in(v[i]);
      __syncthreads();
      // (input already Moebius-transformed: no butterfly)
      for (int bit = 0; bit < (C->mobius_in ? 0 : b); ++bit) {
        const int half = nt >> 1;
        for (int p = tid; p < half; p += NT) {
          const int lo = ((p >> bit) << (bit + 1)) | (p & ((1 << bit) - 1));
          const int hi = lo | (1 << bit);
          m[hi] = Num<MobT>::sub(m[hi], m[lo]);
        }
        __syncthreads();
      }
      SwT tmp[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int i = tid + j * NT;
        if (i < nt) tmp[j] = to_sweep(m[i], (SwT*)nullptr);
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int i = tid + j * NT;
        if (i < nt) cur[i] = tmp[j];
      }
    } else {
      // two-pass: src is the already Moebius-transformed workspace
      const SrcT* a = src + I.woff + ((int64_t)w.tile << b);
      for (int i = tid; i < nt; i += NT) cur[i] = to_sweep(load_as(a + i, (SrcT*)nullptr), (SwT*)nullptr);
    }
    __syncthreads();

    // counter sweep: site k consumes tile bit b-k; each output pattern adds
    // its (tau = 0) and (tau = 1) predecessors (at most 2 nonzeros per
    // output state, Sec. 4.4 sparse cores)
    for (int k = 1; k <= b; ++k) {
      const int lg = b - k;
      const int L = 1 << lg;
      const int np = C->step_np[k];
      const uint32_t* __restrict__ pk = C->pat + C->step_off[k];
      const int total = np << lg;
      for (int e = tid; e < total; e += NT) {
        const int p = e >> lg;
        const int r = e & (L - 1);
        const uint32_t q = pk[p];
        const int s0 = (int)(q & 0xFFFFu) - 1;
        const int s1 = (int)(q >> 16) - 1;
        SwT acc = SwT(0);
        if (s0 >= 0) acc = cur[(s0 << (lg + 1)) + r];
        if (s1 >= 0) acc += cur[(s1 << (lg + 1)) + L + r];
        nxt[e] = acc;
      }
      __syncthreads();
      SwT* t = cur; cur = nxt; nxt = t;
    }

    // final weight core (FP64 weights, FP64 accumulation)
    const int u = __popc(w.tile);
    const double* __restrict__ lamu = C->lam + (int64_t)u * C->lam_ublock;
    double* __restrict__ Yt = Y + I.yoff + (int64_t)w.tile * C->Ysize;
    const int Ysize = C->Ysize;
    for (int e = tid; e < Ysize; e += NT) {
      const uint32_t q = C->ytab[e];
      const int fp = (int)(q & 0xFFFFu);
      const int slot = (int)((q >> 16) & 0x3FFu);
      const int sl = (int)(q >> 26);
      const double* lw = lamu + C->lam_soff[sl] + slot * (b + 1);
      if (Ylo) {
        // compensated dot product with double-double weights (the
        // error-free product of the high word by FMA and Knuth's TwoSum,
        // their errors and the low word's product summed apart): the result
        // as a double-double; no contraction, so every sum and product is
        // rounded as written
#pragma clang fp contract(off)
        const double* lwlo = C->lam_lo + (int64_t)u * C->lam_ublock + C->lam_soff[sl] + slot * (b + 1);
        double s = 0.0, c = 0.0;
        for (int t = sl; t <= b; ++t) {
          const double z = (double)cur[fp + t - sl];
          const double p = lw[t] * z;
          const double pe = fma(lw[t], z, -p);
          const double s1 = s + p;
          const double bb = s1 - s;
          c += ((s - (s1 - bb)) + (p - bb)) + (pe + lwlo[t] * z);
          s = s1;
        }
        const double hi = s + c;
        const double bb = hi - s;
        Yt[e] = hi;
        Ylo[I.yoff + (int64_t)w.tile * C->Ysize + e] = (s - (hi - bb)) + (c - bb);
      } else {
        double acc = 0.0;
        for (int t = sl; t <= b; ++t) acc = fma(lw[t], (double)cur[fp + t - sl], acc);
        Yt[e] = acc;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- reduce kernel
template <typename OutT>
__global__ void __launch_bounds__(256)
reduce_kernel(const ClassDev* __restrict__ classes, const InstDev* __restrict__ insts,
              int n_inst, const int64_t* __restrict__ out_offset, int64_t total,
              const double* __restrict__ Y, const double* __restrict__ Ylo,
              const double* __restrict__ partial, OutT* __restrict__ out) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = n_inst;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (out_offset[mid] <= g) lo = mid; else hi = mid;
    }
    const InstDev I = insts[lo];
    const int k = (int)(g - out_offset[lo]);
    if (I.fast || I.wide) continue;   // written by fast_reduce_kernel / wide_final_kernel
    const ClassDev* C = classes + I.cls;
    const uint32_t oi = C->oinfo[k];
    const uint32_t SH = C->osh[k];
    const int yo = (int)(oi & 0xFFFFFFu);
    const int sH = (int)(oi >> 24);
    const double* __restrict__ Yi = Y + I.yoff + yo;
    const int64_t Ys = C->Ysize;
    const uint32_t nt = 1u << C->h;
    double acc = 0.0;
    if (C->algo == ALGO_FUSED) {
      const int base = sH * (sH + 1) / 2;
      for (uint32_t UH = 0; UH < nt; ++UH) acc += Yi[(int64_t)UH * Ys + base + __popc(SH & UH)];
    } else if (Ylo) {
      // compensated sum of double-doubles (Knuth's TwoSum on the high words,
      // their errors and the low words summed apart)
      const double* __restrict__ Li = Ylo + I.yoff + yo;
      const uint32_t comp = (nt - 1u) & ~SH;
      uint32_t sub = 0;
      double c = 0.0;
      for (;;) {
        const int64_t o = (int64_t)(SH | sub) * Ys + sH;
        const double h = Yi[o];
        const double s1 = acc + h;
        const double bb = s1 - acc;
        c += ((acc - (s1 - bb)) + (h - bb)) + Li[o];
        acc = s1;
        if (sub == comp) break;
        sub = (sub - comp) & comp;
      }
      acc += c;
    } else {
      const uint32_t comp = (nt - 1u) & ~SH;
      uint32_t sub = 0;
      for (;;) {
        acc += Yi[(int64_t)(SH | sub) * Ys + sH];
        if (sub == comp) break;
        sub = (sub - comp) & comp;
      }
    }
    out[I.ooff + k] = (OutT)acc;
  }
}

// Wide gather: thread t of a work item owns outputs group * kWideOuts + t +
// 256 q (q < kWideK) and adds, for every tile U of the item's range, the
// per-tile result its output selects (slot |S_H & U| of its s_H block).
// Outputs past M read entry 0 of the tile (in range) and are never stored
// by the final pass.
// For a register-phase instance of several blocks the range is one of
// blocks: each output adds, for every block H2 and every work item of the
// block, the partial sum of its (S_L, S_H1, |S_H2|) at j2 = |S_H2 & H2|.
__device__ __forceinline__ void wide_gather_blocks(const InstDev& I, const WideItem& w, int M,
                                                   const double* __restrict__ fpart,
                                                   double* __restrict__ partial) {
  int32_t pj[kWideK][5];
  uint32_t s2[kWideK];
  double acc[kWideK];
#pragma unroll
  for (int q = 0; q < kWideK; ++q) {
    const int k = w.group * kWideOuts + q * 256 + (int)threadIdx.x;
    const int kk = k < M ? k : 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) pj[q][j] = I.pidx[(int64_t)kk * I.pw + (j < I.pw ? j : 0)];
    s2[q] = I.osh2[kk];
    acc[q] = 0.0;
  }
  for (int blk = w.t0; blk < w.t1; ++blk) {
    for (int r = 0; r < I.ipb; ++r) {
      const double* __restrict__ Pb = fpart + I.pbase + ((int64_t)blk * I.ipb + r) * I.pstride;
#pragma unroll
      for (int q = 0; q < kWideK; ++q) {
        const int j = __popc(s2[q] & (uint32_t)blk);
        const int32_t o = j == 0 ? pj[q][0] : j == 1 ? pj[q][1] : j == 2 ? pj[q][2]
                        : j == 3 ? pj[q][3] : pj[q][4];
        acc[q] += Pb[o];
      }
    }
  }
  double* P = partial + w.pofs;
#pragma unroll
  for (int q = 0; q < kWideK; ++q) P[q * 256 + threadIdx.x] = acc[q];
}

__global__ void __launch_bounds__(256)
wide_gather_kernel(const ClassDev* __restrict__ classes, const InstDev* __restrict__ insts,
                   const WideItem* __restrict__ items, int n_items,
                   const int64_t* __restrict__ out_offset, const double* __restrict__ Y,
                   const double* __restrict__ fpart, double* __restrict__ partial) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WideItem w = items[it];
    const InstDev I = insts[w.inst];
    const ClassDev* C = classes + I.cls;
    const int M = (int)(out_offset[w.inst + 1] - out_offset[w.inst]);
    if (I.fast) {
      wide_gather_blocks(I, w, M, fpart, partial);
      continue;
    }
    const int64_t Ys = C->Ysize;
    uint32_t yo[kWideK], sh[kWideK];
    double acc[kWideK];
#pragma unroll
    for (int q = 0; q < kWideK; ++q) {
      const int k = w.group * kWideOuts + q * 256 + (int)threadIdx.x;
      const uint32_t oi = k < M ? C->oinfo[k] : 0u;
      const uint32_t sH = oi >> 24;
      yo[q] = (oi & 0xFFFFFFu) + sH * (sH + 1) / 2;
      sh[q] = k < M ? C->osh[k] : 0u;
      acc[q] = 0.0;
    }
    const double* __restrict__ Yb = Y + I.yoff;
    for (int U = w.t0; U < w.t1; ++U) {
      const double* __restrict__ Yt = Yb + (int64_t)U * Ys;
#pragma unroll
      for (int q = 0; q < kWideK; ++q) acc[q] += Yt[yo[q] + __popc(sh[q] & (uint32_t)U)];
    }
    double* P = partial + w.pofs;
#pragma unroll
    for (int q = 0; q < kWideK; ++q) P[q * 256 + threadIdx.x] = acc[q];
  }
}

template <typename OutT>
__global__ void __launch_bounds__(256)
wide_final_kernel(const WideGroup* __restrict__ groups, int n_groups,
                  const InstDev* __restrict__ insts, const int64_t* __restrict__ out_offset,
                  const double* __restrict__ partial, OutT* __restrict__ out) {
  // a workgroup takes 256 consecutive outputs of one group
  constexpr int kChunks = kWideOuts / 256;
  for (int ci = blockIdx.x; ci < n_groups * kChunks; ci += gridDim.x) {
    const WideGroup G = groups[ci / kChunks];
    const InstDev I = insts[G.inst];
    const int M = (int)(out_offset[G.inst + 1] - out_offset[G.inst]);
    const int j = (ci % kChunks) * 256 + (int)threadIdx.x;
    const int k = G.group * kWideOuts + j;
    if (k < M) {
      double acc = 0.0;
      for (int r = 0; r < G.nr; ++r) acc += partial[G.pofs + (int64_t)r * kWideOuts + j];
      out[I.ooff + k] = (OutT)acc;
    }
  }
}

// Sum of the register-phase kernel's per-item partial results, in slot
// order: a workgroup owns 256 / ROWS consecutive slots of one instance (so
// a row of threads reads consecutive words of an item's partial sums), and
// writes each slot's sum to the output the slot holds (none for an unused
// slot). Thread (o, r) adds the items j = r mod ROWS in increasing order,
// then the ROWS sums are combined in a fixed order, so the result is bitwise
// repeatable (and, for at most ROWS items, the plain sum in item order).
// ROWS = 1 when every instance has at most two items (the usual batched
// case: one slot per thread, no LDS step), 4 up to 64 items, else 16.
template <typename OutT, int ROWS>
__global__ void __launch_bounds__(256)
fast_reduce_kernel(const InstDev* __restrict__ insts, const int2* __restrict__ chunks,
                   int n_chunks, const double* __restrict__ partial, OutT* __restrict__ out) {
  constexpr int W = 256 / ROWS;
  __shared__ double part[ROWS][W];
  const int o = threadIdx.x % W, r = threadIdx.x / W;
  for (int ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
    const int2 c = chunks[ch];
    const InstDev I = insts[c.x];
    const int s = c.y + o;
    const int k = s < I.pstride ? I.sinv[s] : -1;
    double acc = 0.0;
    if (k >= 0) {
      const double* P = partial + I.pbase + s;
#pragma unroll 4
      for (int j = r; j < I.nitems; j += ROWS) acc += P[(int64_t)j * I.pstride];
    }
    if constexpr (ROWS == 1) {
      if (k >= 0) out[I.ooff + k] = (OutT)acc;
    } else {
      part[r][o] = acc;
      __syncthreads();
      if (r == 0 && k >= 0) {
        double t = part[0][o];
#pragma unroll
        for (int q = 1; q < ROWS; ++q) t += part[q][o];
        out[I.ooff + k] = (OutT)t;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- Moebius (two-pass)
// Low pass: each work item is a tile of 2^b consecutive values; butterflies
// over the b low bits in LDS; the result goes to dst (in place allowed).
template <typename InT, typename MobT>
__global__ void __launch_bounds__(kTileThreads)
mobius_low_kernel(const ClassDev* __restrict__ classes, const InstDev* __restrict__ insts,
                  const TileItem* __restrict__ items, int n_items, const InT* src,
                  MobT* dst, int src_is_values) {
  extern __shared__ __align__(16) unsigned char smem[];
  MobT* m = reinterpret_cast<MobT*>(smem);
  const int tid = threadIdx.x;
  constexpr int NT = kTileThreads;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const TileItem w = items[it];
    const InstDev I = insts[w.inst];
    const int b = classes[I.cls].b;
    const int nt = 1 << b;
    const InT* s = src + (src_is_values ? I.voff : I.woff) + ((int64_t)w.tile << b);
    MobT* o = dst + I.woff + ((int64_t)w.tile << b);
    for (int i = tid; i < nt; i += NT) m[i] = Num<MobT>::from_in(s[i]);
    __syncthreads();
    for (int bit = 0; bit < b; ++bit) {
      for (int p = tid; p < (nt >> 1); p += NT) {
        const int lo = ((p >> bit) << (bit + 1)) | (p & ((1 << bit) - 1));
        const int hi = lo | (1 << bit);
        m[hi] = Num<MobT>::sub(m[hi], m[lo]);
      }
      __syncthreads();
    }
    for (int i = tid; i < nt; i += NT) o[i] = m[i];
    __syncthreads();
  }
}

// High pass: bits [lo, lo + G) of one instance. A work item is a block of
// 2^G x 2^cb values: 2^cb consecutive low indices (coalesced) for each of
// the 2^G settings of the group bits, for one setting of the other bits.
template <typename MobT>
__global__ void __launch_bounds__(kTileThreads)
mobius_high_kernel(const InstDev* __restrict__ insts, const MobItem* __restrict__ items,
                   int n_items, MobT* data) {
  extern __shared__ __align__(16) unsigned char smem[];
  MobT* m = reinterpret_cast<MobT*>(smem);
  const int tid = threadIdx.x;
  constexpr int NT = kTileThreads;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const MobItem w = items[it];
    const InstDev I = insts[w.inst];
    const int G = w.G, lo = w.lo, cb = w.cb;
    const int n = 1 << (G + cb);
    const int64_t nchunk = (int64_t)1 << (lo - cb);
    const int64_t cl = w.block % nchunk;          // which chunk of low indices
    const int64_t rest = w.block / nchunk;        // the bits above the group
    MobT* base = data + I.woff + (rest << (lo + G)) + (cl << cb);
    for (int i = tid; i < n; i += NT) {
      const int g = i >> cb, c = i & ((1 << cb) - 1);
      m[i] = base[((int64_t)g << lo) + c];
    }
    __syncthreads();
    for (int bit = 0; bit < G; ++bit) {
      for (int p = tid; p < (n >> 1); p += NT) {
        const int bb = bit + cb;
        const int lo2 = ((p >> bb) << (bb + 1)) | (p & ((1 << bb) - 1));
        const int hi2 = lo2 | (1 << bb);
        m[hi2] = Num<MobT>::sub(m[hi2], m[lo2]);
      }
      __syncthreads();
    }
    for (int i = tid; i < n; i += NT) {
      const int g = i >> cb, c = i & ((1 << cb) - 1);
      base[((int64_t)g << lo) + c] = m[i];
    }
    __syncthreads();
  }
}

// Convert a Moebius-type buffer back to the storage type (fsi_mobius).
template <typename MobT, typename OutT>
__global__ void convert_kernel(const MobT* __restrict__ a, OutT* __restrict__ o, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    o[i] = (OutT)to_sweep(a[i], (double*)nullptr);
}

// ---------------------------------------------------------------- launchers
namespace {
template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
}  // namespace

template <typename InT, typename MobT, typename SwT>
hipError_t configure_path(int algo, size_t tile_lds, size_t mob_lds) {
  hipError_t e;
  if (algo == ALGO_FUSED) return set_lds(tile_kernel<InT, MobT, SwT, true>, tile_lds);
  if ((e = set_lds(mobius_low_kernel<InT, MobT>, mob_lds)) != hipSuccess) return e;
  if ((e = set_lds(mobius_high_kernel<MobT>, mob_lds)) != hipSuccess) return e;
  return set_lds(tile_kernel<MobT, MobT, SwT, false>, tile_lds);
}

hipError_t configure_kernels(int prec, int algo, size_t tile_lds, size_t mob_lds) {
  hipError_t e;
  // fsi_mobius runs in the storage type
  if ((e = set_lds(mobius_low_kernel<double, double>, mob_lds)) != hipSuccess) return e;
  if ((e = set_lds(mobius_low_kernel<float, float>, mob_lds)) != hipSuccess) return e;
  if ((e = set_lds(mobius_high_kernel<double>, mob_lds)) != hipSuccess) return e;
  if ((e = set_lds(mobius_high_kernel<float>, mob_lds)) != hipSuccess) return e;
  switch (prec) {
    case PREC_F64: return configure_path<double, double, double>(algo, tile_lds, mob_lds);
    case PREC_F32: return configure_path<float, float, float>(algo, tile_lds, mob_lds);
    case PREC_F32_COMP: return configure_path<float, TwoFloat, float>(algo, tile_lds, mob_lds);
    case PREC_F32_FP64MOB: return configure_path<float, double, float>(algo, tile_lds, mob_lds);
    case PREC_F32_FP64REG: return configure_path<float, double, double>(algo, tile_lds, mob_lds);
  }
  return hipErrorInvalidValue;
}

int num_stages(const LaunchArgs& a) {
  // fused: [register-phase kernel per order l], [generic tile kernel],
  //        [generic reduce], [wide gather, wide final], [register-phase reduce]
  // two-pass: Moebius low pass, high passes, tile, reduce
  if (a.algo == ALGO_FUSED)
    return fast_launches(a.fast) + (a.n_tile_items > 0) + (a.n_generic > 0) +
           2 * (a.n_wide_items > 0) + (a.n_red_chunks > 0);
  return 3 + a.n_mob_passes;
}

template <typename InT, typename MobT, typename SwT>
hipError_t launch_stage_t(const LaunchArgs& a, int stage, hipStream_t st) {
  const int last = num_stages(a) - 1;
  if (stage < 0 || stage > last) return hipErrorInvalidValue;
  if (a.algo == ALGO_FUSED && a.n_red_chunks > 0 && stage == last) {
    if (a.red_rows == 1)
      hipLaunchKernelGGL((fast_reduce_kernel<InT, 1>), dim3(a.grid_red_chunks), dim3(256), 0, st,
                         a.insts, a.red_chunks, a.n_red_chunks, a.partial,
                         static_cast<InT*>(a.out));
    else if (a.red_rows == 4)
      hipLaunchKernelGGL((fast_reduce_kernel<InT, 4>), dim3(a.grid_red_chunks), dim3(256), 0, st,
                         a.insts, a.red_chunks, a.n_red_chunks, a.partial,
                         static_cast<InT*>(a.out));
    else
      hipLaunchKernelGGL((fast_reduce_kernel<InT, 16>), dim3(a.grid_red_chunks), dim3(256), 0, st,
                         a.insts, a.red_chunks, a.n_red_chunks, a.partial,
                         static_cast<InT*>(a.out));
    return hipGetLastError();
  }
  if (a.algo == ALGO_FUSED && a.n_wide_items > 0) {
    const int wfin = last - (a.n_red_chunks > 0);
    if (stage == wfin - 1) {
      hipLaunchKernelGGL(wide_gather_kernel, dim3(a.grid_wide), dim3(256), 0, st, a.classes,
                         a.insts, a.wide_items, a.n_wide_items, a.out_offset, a.Y,
                         a.partial, a.wide_partial);
      return hipGetLastError();
    }
    if (stage == wfin) {
      hipLaunchKernelGGL(wide_final_kernel<InT>, dim3(a.grid_wide_groups), dim3(256), 0, st,
                         a.wide_groups, a.n_wide_groups, a.insts, a.out_offset, a.wide_partial,
                         static_cast<InT*>(a.out));
      return hipGetLastError();
    }
  }
  if (a.algo != ALGO_FUSED
          ? stage == last
          : (a.n_generic > 0 &&
             stage == last - (a.n_red_chunks > 0) - 2 * (a.n_wide_items > 0))) {
    hipLaunchKernelGGL(reduce_kernel<InT>, dim3(a.grid_reduce), dim3(256), 0, st, a.classes,
                       a.insts, a.n_inst, a.out_offset, a.total_out, a.Y, a.Ylo, a.partial,
                       static_cast<InT*>(a.out));
    return hipGetLastError();
  }
  if (a.algo == ALGO_FUSED) {
    int ls[kFastMaxL];
    const int ng = fast_groups(a.fast, ls);
    if (stage < fast_launches(a.fast)) {
      FastLaunch f = a.fast;
      f.vals32 = a.values;
      f.vals64 = a.values;
      return ng > 1 ? launch_fast_mixed(f, st) : launch_fast_group(f, ls[0], st);
    }
  }
  if (a.algo == ALGO_FUSED) {
    hipLaunchKernelGGL((tile_kernel<InT, MobT, SwT, true>), dim3(a.grid_tile), dim3(kTileThreads),
                       a.tile_lds, st, a.classes, a.insts, a.tile_items, a.n_tile_items,
                       static_cast<const InT*>(a.values), a.Y, nullptr);
    return hipGetLastError();
  }
  if (stage == 0) {
    hipLaunchKernelGGL((mobius_low_kernel<InT, MobT>), dim3(a.grid_tile), dim3(kTileThreads),
                       a.mob_lds, st, a.classes, a.insts, a.tile_items, a.n_tile_items,
                       static_cast<const InT*>(a.values), static_cast<MobT*>(a.work), 1);
    return hipGetLastError();
  }
  if (stage <= a.n_mob_passes) {
    const int p = stage - 1;
    if (a.n_mob_items[p] == 0) return hipSuccess;
    hipLaunchKernelGGL(mobius_high_kernel<MobT>, dim3(a.grid_tile), dim3(kTileThreads), a.mob_lds,
                       st, a.insts, a.mob_items[p], a.n_mob_items[p], static_cast<MobT*>(a.work));
    return hipGetLastError();
  }
  hipLaunchKernelGGL((tile_kernel<MobT, MobT, SwT, false>), dim3(a.grid_tile), dim3(kTileThreads),
                     a.tile_lds, st, a.classes, a.insts, a.tile_items, a.n_tile_items,
                     static_cast<const MobT*>(a.work), a.Y, a.Ylo);
  return hipGetLastError();
}

hipError_t launch_stage(const LaunchArgs& a, int stage, hipStream_t st) {
  switch (a.prec) {
    case PREC_F64: return launch_stage_t<double, double, double>(a, stage, st);
    case PREC_F32: return launch_stage_t<float, float, float>(a, stage, st);
    case PREC_F32_COMP: return launch_stage_t<float, TwoFloat, float>(a, stage, st);
    case PREC_F32_FP64MOB: return launch_stage_t<float, double, float>(a, stage, st);
    case PREC_F32_FP64REG: return launch_stage_t<float, double, double>(a, stage, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_apply(const LaunchArgs& a, hipStream_t st) {
  const int n = num_stages(a);
  for (int i = 0; i < n; ++i) {
    const hipError_t e = launch_stage(a, i, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_mobius_t(const LaunchArgs& a, hipStream_t st) {
  hipError_t e;
  auto km = mobius_low_kernel<T, T>;
  // in place on the caller's buffer: the instance's work offset is 0 and
  // the source is the buffer itself (src_is_values = 0 -> offset woff)
  hipLaunchKernelGGL(km, dim3(a.grid_tile), dim3(kTileThreads), a.mob_lds, st, a.classes,
                     a.insts, a.all_tiles, a.n_all_tiles, static_cast<const T*>(a.work),
                     static_cast<T*>(a.work), 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  auto kh = mobius_high_kernel<T>;
  for (int p = 0; p < a.n_mob_passes; ++p) {
    if (a.n_mob_items[p] == 0) continue;
    hipLaunchKernelGGL(kh, dim3(a.grid_tile), dim3(kTileThreads), a.mob_lds, st, a.insts,
                       a.mob_items[p], a.n_mob_items[p], static_cast<T*>(a.work));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_mobius(const LaunchArgs& a, hipStream_t st) {
  return a.prec == PREC_F64 ? launch_mobius_t<double>(a, st) : launch_mobius_t<float>(a, st);
}

size_t mob_elem_bytes(int prec) {
  switch (prec) {
    case PREC_F64: return 8;
    case PREC_F32: return 4;
    case PREC_F32_COMP: return sizeof(TwoFloat);
    case PREC_F32_FP64MOB: return 8;
    case PREC_F32_FP64REG: return 8;
  }
  return 8;
}
size_t sweep_elem_bytes(int prec) {
  return (prec == PREC_F64 || prec == PREC_F32_FP64REG) ? 8 : 4;
}
size_t store_elem_bytes(int prec) { return prec == PREC_F64 ? 8 : 4; }

}  // namespace fsi
