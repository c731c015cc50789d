// Launch interface between the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstdint>

#include "fsi_internal.h"

namespace fsi {

constexpr int kTileThreads = 512;
constexpr int kMaxMobPasses = 4;   // high-bit groups of the two-pass butterfly

struct TileItem {
  int32_t inst, tile;       // instance, high index U_H of the tile
};

struct MobItem {
  int32_t inst, lo, G, cb;  // group bits [lo, lo+G); 2^cb consecutive low indices
  int64_t block;            // (bits above the group) * 2^(lo-cb) + low chunk
};

// Register-phase kernel (fsi_tile11.hip)
constexpr int kFastThreads = 256;
constexpr int kFastRuns = 14;      // gather positions (runs of two outputs) per thread
constexpr int kFastKmax = 2 * kFastRuns;  // output slots per thread
constexpr int kFastMetaStride = 16;  // per-thread metadata words (4 x 16 bytes)
constexpr int kFastTileBits = 11;
constexpr int kFastMaxL = 4;

struct FastItem {
  int32_t inst, tb, te, pad;       // tiles [tb, te) of the instance's tile order
  int64_t pofs;                    // partial sums of this item
};

// Work items are sorted by order l; items [lbeg[l], lbeg[l+1]) have order l
// and go to the kernel compiled for that l (one launch per order present).
struct FastLaunch {
  int prec;
  const FastClassDev* classes;
  const InstDev* insts;
  const FastItem* items;
  int n_items;
  int lbeg[kFastMaxL + 2];
  int grid[kFastMaxL + 1];
  size_t lds[kFastMaxL + 1];
  int grid_mixed;                 // grid of the one launch over every order's items
  size_t lds_mixed;               // its dynamic LDS (the largest order's)
  int mobius_in;                  // 1: the input is already the Moebius transform
  const void* vals32;
  const void* vals64;
  const int32_t* torder;
  double* partial;
  // work queue of a launch: [0] next item, [1] workgroups done; zero before
  // every launch (the last workgroup of a launch to finish resets both)
  uint32_t* queue;
};

// lds[l]: dynamic LDS of the order-l kernel, 0 = not used by the plan.
hipError_t configure_fast(int prec, const size_t* lds);
hipError_t launch_fast_group(const FastLaunch& f, int l, hipStream_t st);
// One launch over the items of every order (plans with more than one order).
hipError_t launch_fast_mixed(const FastLaunch& f, hipStream_t st);
// Register-phase launches of one apply: 0, or 1 (one order, or several
// orders in one mixed launch).
int fast_launches(const FastLaunch& f);
// Orders l with work items, ascending; returns their number.
int fast_groups(const FastLaunch& f, int* ls);
bool fast_supported(int prec);
// Dynamic LDS of the register-phase kernel for items of order l.
size_t fast_lds_bytes(int prec, int l);
int fast_wgs_per_cu(int prec, int l);

// Wide gather (generic fused instances with many tiles): a work item is a
// range of tiles and a group of up to kWideOuts outputs; each thread keeps
// kWideK output accumulators in registers across the range. The partial
// sums of a group's ranges are then added in range order.
constexpr int kWideK = 16;
constexpr int kWideOuts = 256 * kWideK;
constexpr int kWideMinH = 10;      // instances with at least 2^10 tiles

struct WideItem {
  int32_t inst, group, t0, t1;     // outputs [group * kWideOuts, ...), tiles [t0, t1)
  int64_t pofs;                    // its kWideOuts partial sums
};
struct WideGroup {
  int32_t inst, group, nr, pad;    // nr ranges, partial sums at pofs + r * kWideOuts
  int64_t pofs;
};

struct LaunchArgs {
  int prec, algo;
  const ClassDev* classes;
  const InstDev* insts;
  int n_inst;
  const TileItem* tile_items;     // tiles of the generic tile kernel
  int n_tile_items;
  const TileItem* all_tiles;      // every tile (standalone Moebius)
  int n_all_tiles;
  const MobItem* mob_items[kMaxMobPasses];
  int n_mob_items[kMaxMobPasses];
  int n_mob_passes;
  const int64_t* out_offset;  // device, n_inst + 1
  int64_t total_out;
  const void* values;
  void* out;
  void* work;                 // Moebius workspace (two-pass, fsi_mobius)
  double* Y;
  double* Ylo;                // two-pass FP64: low words of the per-tile results (else null)
  int grid_tile, grid_reduce;
  size_t tile_lds, mob_lds;
  const double* partial;      // register-phase kernel partial sums
  FastLaunch fast;            // n_items == 0: no register-phase stage
  int n_generic;              // instances of the generic (or two-pass) path outside the wide gather
  const WideItem* wide_items;
  int n_wide_items, grid_wide;
  const WideGroup* wide_groups;
  int n_wide_groups, grid_wide_groups;
  double* wide_partial;
  const int2* red_chunks;     // (instance, first slot) per 256 / red_rows slots of fast instances
  int n_red_chunks, grid_red_chunks;
  int red_rows;               // 1, 4 or 16: item rows per slot in the reduction
};

// Sets the dynamic-LDS limits of the kernels a plan will launch (call once
// per plan, outside any graph capture).
hipError_t configure_kernels(int prec, int algo, size_t tile_lds, size_t mob_lds);
hipError_t launch_apply(const LaunchArgs& a, hipStream_t st);
// Kernel launches of one apply, in order; launch_apply runs all of them.
int num_stages(const LaunchArgs& a);
hipError_t launch_stage(const LaunchArgs& a, int stage, hipStream_t st);
hipError_t launch_mobius(const LaunchArgs& a, hipStream_t st);
size_t mob_elem_bytes(int prec);
size_t sweep_elem_bytes(int prec);
size_t store_elem_bytes(int prec);

}  // namespace fsi
