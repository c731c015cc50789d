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

struct LaunchArgs {
  int prec, algo;
  const ClassDev* classes;
  const InstDev* insts;
  int n_inst;
  const TileItem* tile_items;
  int n_tile_items;
  const MobItem* mob_items[kMaxMobPasses];
  int n_mob_items[kMaxMobPasses];
  int n_mob_passes;
  const int64_t* out_offset;  // device, n_inst + 1
  int64_t total_out;
  const void* values;
  void* out;
  void* work;                 // Moebius workspace (two-pass, fsi_mobius)
  double* Y;
  int grid_tile, grid_reduce;
  size_t tile_lds, mob_lds;
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
