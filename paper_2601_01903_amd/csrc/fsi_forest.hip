// Value function of a tree ensemble on the GPU (include/fsi_forest.h):
// v(S) = (1/B) sum_b sum_k f_k(z_b(S)) for all 2^d coalitions S, the input
// the FSI operator consumes (Sec. 2.1 value function; the paper's appendix
// times this step separately in its bottleneck analysis).
//
// Per call, a small kernel folds the explained point and the background
// points into every internal node: the node's decision when its feature is
// in S (x_f >= threshold, one bit) and, for each background b, when it is not
// (bg_b,f >= threshold, one bit per background in a 32-bit word). A walk
// then needs no feature values: at a node with feature f, coalition S goes
// right iff (S >> f & 1) ? dx : (bits >> b & 1).
//
// The walk kernel gives each lane a few coalitions (independent paths
// interleaved so their node loads overlap) and walks every (background,
// tree) pair in ascending order, summing leaf outputs in FP64. Node records
// are 16 bytes; the records of the top levels are shared by all lanes of a
// wave, the deeper ones sit in L1/L2 (a 200-tree depth-6 forest is 400 KB).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fsi_forest.h"
#include "fsi_abi.h"
#include "fsi_internal.h"

namespace fsi {
namespace forest {

constexpr int kThreads = 256;
constexpr int kBgChunk = 32;     // backgrounds per decision word
constexpr int kMaxBg = 4096;
constexpr int kMaxDepth = 64;

// code: feature | (x_f >= threshold) << 8 for an internal node, -1 for a leaf
struct alignas(16) Node {
  int32_t code, left, right;
  uint32_t bits;                 // bit j: background (32 c + j) goes right
};

__global__ void __launch_bounds__(kThreads)
prep_kernel(const int32_t* __restrict__ feature, const double* __restrict__ threshold,
            const int32_t* __restrict__ left, const int32_t* __restrict__ right,
            int n_nodes, int d, const double* __restrict__ x, const double* __restrict__ bg,
            int n_bg, Node* __restrict__ out) {
  const int n_chunks = (n_bg + kBgChunk - 1) / kBgChunk;
  const int64_t total = (int64_t)n_chunks * n_nodes;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    const int c = (int)(i / n_nodes);
    const int node = (int)(i - (int64_t)c * n_nodes);
    const int f = feature[node];
    Node p;
    if (f < 0) {
      p.code = -1; p.left = 0; p.right = 0; p.bits = 0;
    } else {
      const double th = threshold[node];
      const int b0 = c * kBgChunk;
      const int nb = min(kBgChunk, n_bg - b0);
      uint32_t bits = 0;
      for (int j = 0; j < nb; ++j)
        bits |= (uint32_t)(bg[(int64_t)(b0 + j) * d + f] >= th) << j;
      p.code = f | ((x[f] >= th) ? 256 : 0);
      p.left = left[node];
      p.right = right[node];
      p.bits = bits;
    }
    out[i] = p;
  }
}

// KP coalitions per lane: S = (block * KP + j) * kThreads + lane-in-block.
template <typename OutT, int KP>
__global__ void __launch_bounds__(kThreads)
walk_kernel(const Node* __restrict__ prep, const double* __restrict__ value,
            const int32_t* __restrict__ roots, int n_trees, int n_nodes, int n_bg,
            int max_depth, int d, OutT* __restrict__ v) {
  const uint32_t n_coal = 1u << d;
  uint32_t S[KP];
  double acc[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    S[j] = ((uint32_t)blockIdx.x * KP + j) * kThreads + threadIdx.x;
    acc[j] = 0.0;
  }
  const uint32_t S_any = S[0] < n_coal ? S[0] : 0;
#pragma unroll
  for (int j = 0; j < KP; ++j)
    if (S[j] >= n_coal) S[j] = S_any;          // walk a valid coalition, store nothing
  const int n_chunks = (n_bg + kBgChunk - 1) / kBgChunk;
  for (int c = 0; c < n_chunks; ++c) {
    const Node* P = prep + (int64_t)c * n_nodes;
    const int nb = min(kBgChunk, n_bg - c * kBgChunk);
    for (int jb = 0; jb < nb; ++jb) {
      for (int t = 0; t < n_trees; ++t) {
        const int r = roots[t];
        int n[KP];
#pragma unroll
        for (int j = 0; j < KP; ++j) n[j] = r;
        for (int lv = 0; lv < max_depth; ++lv) {
          Node w[KP];
#pragma unroll
          for (int j = 0; j < KP; ++j) w[j] = P[n[j]];
          bool inner = false;
#pragma unroll
          for (int j = 0; j < KP; ++j) {
            if (w[j].code >= 0) {
              const uint32_t f = (uint32_t)w[j].code & 255u;
              const uint32_t go = ((S[j] >> f) & 1u) ? ((uint32_t)w[j].code >> 8) & 1u
                                                     : (w[j].bits >> jb) & 1u;
              n[j] = go ? w[j].right : w[j].left;
              inner = true;
            }
          }
          if (!__any(inner)) break;
        }
#pragma unroll
        for (int j = 0; j < KP; ++j) acc[j] += value[n[j]];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const uint32_t s = ((uint32_t)blockIdx.x * KP + j) * kThreads + threadIdx.x;
    if (s < n_coal) v[s] = (OutT)(acc[j] / (double)n_bg);
  }
}

constexpr int kWalkKP = 2;

// ---- Moebius route ----
// A leaf of a tree is reached at z_b(S) iff every test on its root path
// passes. With alpha_f (beta_f) = [x (bg_b) passes every test on feature f of
// the path], the leaf's indicator is prod_f (beta_f + [f in S](alpha_f -
// beta_f)), whose Moebius coefficients sit on R = I u Q: I = {f: beta_f = 0}
// (unreachable if some f in I has alpha_f = 0), Q any subset of
// Fr = {f: beta_f = 1, alpha_f = 0}, with sign (-1)^|Q|. One thread per
// (background, path) adds value / B * (-1)^|Q| at every such R.
__global__ void __launch_bounds__(kThreads)
fill_kernel(double* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    a[i] = 0.0;
}

__global__ void __launch_bounds__(kThreads)
mobius_scatter_kernel(const int32_t* __restrict__ path_off, const int32_t* __restrict__ steps,
                      const int32_t* __restrict__ path_leaf, int n_paths,
                      const int32_t* __restrict__ feature, const double* __restrict__ threshold,
                      const double* __restrict__ value, int d, const double* __restrict__ x,
                      const double* __restrict__ bg, int n_bg, double* __restrict__ a) {
  const int64_t total = (int64_t)n_bg * n_paths;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    const int b = (int)(i / n_paths);
    const int p = (int)(i - (int64_t)b * n_paths);
    const double* z = bg + (int64_t)b * d;
    uint32_t seen = 0, aok = ~0u, bok = ~0u;
    for (int s = path_off[p]; s < path_off[p + 1]; ++s) {
      const int e = steps[s];
      const int node = e >> 1;
      const bool dir = e & 1;
      const int f = feature[node];
      const double th = threshold[node];
      const uint32_t bit = 1u << f;
      seen |= bit;
      if ((x[f] >= th) != dir) aok &= ~bit;
      if ((z[f] >= th) != dir) bok &= ~bit;
    }
    const uint32_t I = seen & ~bok;
    if (I & ~aok) continue;                        // never reached
    const uint32_t Fr = seen & bok & ~aok;
    const double c = value[path_leaf[p]] / (double)n_bg;
    uint32_t Q = 0;
    do {
      atomicAdd(a + (I | Q), (__popc(Q) & 1) ? -c : c);
      Q = (Q - Fr) & Fr;
    } while (Q != 0);
  }
}

// Subset sums (zeta transform, the inverse of the Moebius butterfly) over
// the NB bits [bit0, bit0 + NB) of the index: each thread owns the 2^NB
// entries of one column in registers. The last pass may write the result in
// the output dtype instead of in place.
// Small workgroups: a pass has only 2^(d-5) columns (32768 at d = 20), which
// must still spread over every CU.
constexpr int kZetaThreads = 64;

template <int NB, typename OutT>
__global__ void __launch_bounds__(kZetaThreads)
zeta_pass_kernel(double* a, int d, int bit0, OutT* out) {   // out may equal a
  const int64_t cols = (int64_t)1 << (d - NB);
  const int64_t low = ((int64_t)1 << bit0) - 1;
  for (int64_t t = (int64_t)blockIdx.x * kZetaThreads + threadIdx.x; t < cols;
       t += (int64_t)gridDim.x * kZetaThreads) {
    const int64_t base = (t & low) | ((t >> bit0) << (bit0 + NB));
    double v[1 << NB];
#pragma unroll
    for (int k = 0; k < (1 << NB); ++k) v[k] = a[base + ((int64_t)k << bit0)];
#pragma unroll
    for (int bit = 0; bit < NB; ++bit)
#pragma unroll
      for (int k = 0; k < (1 << NB); ++k)
        if (k & (1 << bit)) v[k] += v[k ^ (1 << bit)];
#pragma unroll
    for (int k = 0; k < (1 << NB); ++k) out[base + ((int64_t)k << bit0)] = (OutT)v[k];
  }
}

// The low kZetaLow bits (or all d if fewer) in one pass: a workgroup loads a
// contiguous tile of 2^lb entries into LDS, runs the lb butterfly levels
// there and writes the tile back (coalesced both ways).
constexpr int kZetaLow = 10;

template <typename OutT>
__global__ void __launch_bounds__(kThreads)
zeta_low_kernel(const double* a, int lb, OutT* out) {        // out may equal a
  __shared__ double t[1 << kZetaLow];
  const int n = 1 << lb;
  const int64_t base = (int64_t)blockIdx.x << lb;
  for (int i = threadIdx.x; i < n; i += kThreads) t[i] = a[base + i];
  __syncthreads();
  for (int bit = 0; bit < lb; ++bit) {
    for (int k = threadIdx.x; k < n / 2; k += kThreads) {
      const int i0 = ((k >> bit) << (bit + 1)) | (k & ((1 << bit) - 1));
      t[i0 | (1 << bit)] += t[i0];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += kThreads) out[base + i] = (OutT)t[i];
}

template <typename OutT>
void launch_zeta(double* a, int d, int bit0, int nb, OutT* out, hipStream_t st) {
  const int64_t cols = (int64_t)1 << (d - nb);
  const int grid = (int)std::min<int64_t>((cols + kZetaThreads - 1) / kZetaThreads, 32768);
  switch (nb) {
    case 1: zeta_pass_kernel<1, OutT><<<grid, kZetaThreads, 0, st>>>(a, d, bit0, out); break;
    case 2: zeta_pass_kernel<2, OutT><<<grid, kZetaThreads, 0, st>>>(a, d, bit0, out); break;
    case 3: zeta_pass_kernel<3, OutT><<<grid, kZetaThreads, 0, st>>>(a, d, bit0, out); break;
    case 4: zeta_pass_kernel<4, OutT><<<grid, kZetaThreads, 0, st>>>(a, d, bit0, out); break;
    default: zeta_pass_kernel<5, OutT><<<grid, kZetaThreads, 0, st>>>(a, d, bit0, out); break;
  }
}

constexpr int kZetaBits = 5;        // bits per zeta pass
constexpr int kMaxFreeSplits = 24;  // longest path the Moebius route expands
constexpr int64_t kMaxPathSteps = (int64_t)1 << 26;

}  // namespace forest
}  // namespace fsi

using namespace fsi;
using namespace fsi::forest;

struct fsi_forest_s {
  int d = 0, n_trees = 0, n_nodes = 0, max_bg = 0, max_depth = 0, device = 0;
  int32_t* feature = nullptr;
  int32_t* left = nullptr;
  int32_t* right = nullptr;
  int32_t* roots = nullptr;
  double* threshold = nullptr;
  double* value = nullptr;
  Node* prep = nullptr;
  // root-to-leaf paths for the Moebius route (n_paths < 0: not available)
  int n_paths = 0, max_path = 0;
  int32_t* path_off = nullptr;
  int32_t* steps = nullptr;        // node << 1 | went right
  int32_t* path_leaf = nullptr;
};

namespace {

fsi_status ffail(fsi_status st, const std::string& msg) {
  record_error(msg);
  return st;
}

void free_forest(fsi_forest_s* F) {
  if (!F) return;
  for (void* p : {(void*)F->feature, (void*)F->left, (void*)F->right, (void*)F->roots,
                  (void*)F->threshold, (void*)F->value, (void*)F->prep,
                  (void*)F->path_off, (void*)F->steps, (void*)F->path_leaf})
    if (p) (void)hipFree(p);
  delete F;
}

// Longest root-to-leaf path of the forest in internal nodes, or -1 on a cycle
// or a path longer than kMaxDepth (iterative depth-first search, memoised per
// node; a node is marked while its subtree is open, so meeting a marked node
// means a cycle).
int forest_depth(int n_nodes, const int32_t* feature, const int32_t* left,
                 const int32_t* right, const int32_t* roots, int n_trees) {
  std::vector<int> depth(n_nodes, -2);   // -2 unvisited, -3 on the stack
  int best = 0;
  std::vector<std::pair<int, int>> stack;  // (node, state)
  for (int k = 0; k < n_trees; ++k) {
    stack.push_back({roots[k], 0});
    while (!stack.empty()) {
      auto& [node, state] = stack.back();
      if (feature[node] < 0) { depth[node] = 0; stack.pop_back(); continue; }
      if (state == 0) {
        if (depth[node] >= 0) { stack.pop_back(); continue; }
        if (depth[node] == -3) return -1;          // cycle
        depth[node] = -3;
        state = 1;
        const int l = left[node], r = right[node];
        if (depth[l] == -3 || depth[r] == -3) return -1;
        if (depth[l] == -2) stack.push_back({l, 0});
        if (depth[r] == -2) stack.push_back({r, 0});
        continue;
      }
      const int dl = depth[left[node]], dr = depth[right[node]];
      if (dl < 0 || dr < 0) return -1;
      depth[node] = 1 + std::max(dl, dr);
      if (depth[node] > kMaxDepth) return -1;
      stack.pop_back();
    }
    best = std::max(best, depth[roots[k]]);
  }
  return best;
}

// Every root-to-leaf path (a leaf reached from several roots or along several
// routes counts once per path). Returns false if the paths exceed the caps.
bool enumerate_paths(const int32_t* feature, const int32_t* left, const int32_t* right,
                     const int32_t* roots, int n_trees, std::vector<int32_t>* off,
                     std::vector<int32_t>* steps, std::vector<int32_t>* leaf) {
  off->assign(1, 0);
  steps->clear();
  leaf->clear();
  std::vector<int32_t> path;
  // explicit DFS: (node, next child to visit: 0 left, 1 right, 2 done)
  std::vector<std::pair<int, int>> st;
  for (int k = 0; k < n_trees; ++k) {
    st.assign(1, {roots[k], 0});
    path.clear();
    while (!st.empty()) {
      auto& top = st.back();
      const int node = top.first;
      if (feature[node] < 0) {
        steps->insert(steps->end(), path.begin(), path.end());
        off->push_back((int32_t)steps->size());
        leaf->push_back(node);
        if ((int64_t)steps->size() > kMaxPathSteps || (int64_t)leaf->size() >= ((int64_t)1 << 26))
          return false;
        st.pop_back();
        if (!path.empty()) path.pop_back();
        continue;
      }
      if (top.second == 2) {
        st.pop_back();
        if (!path.empty()) path.pop_back();
        continue;
      }
      const int dir = top.second++;
      path.push_back((node << 1) | dir);
      st.push_back({dir ? right[node] : left[node], 0});
    }
  }
  return true;
}

template <typename T>
hipError_t upload(T** dst, const T* src, size_t n) {
  hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

extern "C" {

fsi_status fsi_forest_create(int d, int n_trees, const int32_t* roots, int n_nodes,
                             const int32_t* feature, const double* threshold,
                             const int32_t* left, const int32_t* right, const double* value,
                             int max_bg, fsi_forest_t* out) {
  FSI_ABI_TRY
  if (!out) return ffail(FSI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!(1 <= d && d <= kMaxD)) return ffail(FSI_ERR_INVALID_ARG, "need 1 <= d <= 30");
  if (n_trees < 1 || n_nodes < 1) return ffail(FSI_ERR_INVALID_ARG, "need n_trees >= 1 and n_nodes >= 1");
  if (max_bg < 1 || max_bg > kMaxBg) return ffail(FSI_ERR_INVALID_ARG, "need 1 <= max_bg <= 4096");
  if (!roots || !feature || !threshold || !left || !right || !value)
    return ffail(FSI_ERR_INVALID_ARG, "null forest array");
  for (int k = 0; k < n_trees; ++k)
    if (roots[k] < 0 || roots[k] >= n_nodes)
      return ffail(FSI_ERR_INVALID_ARG, "root " + std::to_string(k) + " out of range");
  for (int i = 0; i < n_nodes; ++i) {
    if (feature[i] >= d)
      return ffail(FSI_ERR_INVALID_ARG, "node " + std::to_string(i) + ": feature >= d");
    if (feature[i] >= 0) {
      if (left[i] < 0 || left[i] >= n_nodes || right[i] < 0 || right[i] >= n_nodes)
        return ffail(FSI_ERR_INVALID_ARG, "node " + std::to_string(i) + ": child out of range");
      if (!std::isfinite(threshold[i]))
        return ffail(FSI_ERR_INVALID_ARG, "node " + std::to_string(i) + ": threshold not finite");
    }
  }
  const int depth = forest_depth(n_nodes, feature, left, right, roots, n_trees);
  if (depth < 0)
    return ffail(FSI_ERR_INVALID_ARG, "forest has a cycle or a path of more than 64 splits");
  int dev = 0, n_cu = 0;
  std::string why;
  if (!gfx950_device(&dev, &n_cu, &why)) return ffail(FSI_ERR_UNSUPPORTED, why);

  auto* F = new (std::nothrow) fsi_forest_s();
  if (!F) return ffail(FSI_ERR_OUT_OF_MEMORY, "host allocation failed");
  // frees the partly built forest on every failure below, thrown or returned
  struct Guard {
    fsi_forest_s* f;
    ~Guard() { free_forest(f); }
  } guard{F};
  F->d = d; F->n_trees = n_trees; F->n_nodes = n_nodes; F->max_bg = max_bg;
  F->max_depth = depth; F->device = dev;
  // leaves keep feature -1 on the device whatever negative value they had
  std::vector<int32_t> feat(feature, feature + n_nodes);
  for (auto& f : feat) f = f < 0 ? -1 : f;
  hipError_t e = upload(&F->feature, feat.data(), (size_t)n_nodes);
  if (e == hipSuccess) e = upload(&F->left, left, (size_t)n_nodes);
  if (e == hipSuccess) e = upload(&F->right, right, (size_t)n_nodes);
  if (e == hipSuccess) e = upload(&F->roots, roots, (size_t)n_trees);
  if (e == hipSuccess) e = upload(&F->threshold, threshold, (size_t)n_nodes);
  if (e == hipSuccess) e = upload(&F->value, value, (size_t)n_nodes);
  if (e == hipSuccess) {
    const size_t chunks = (size_t)((max_bg + kBgChunk - 1) / kBgChunk);
    e = hipMalloc((void**)&F->prep, chunks * (size_t)n_nodes * sizeof(Node));
  }
  if (e == hipSuccess) {
    std::vector<int32_t> poff, psteps, pleaf;
    if (enumerate_paths(feat.data(), left, right, roots, n_trees, &poff, &psteps, &pleaf)) {
      F->n_paths = (int)pleaf.size();
      for (size_t p = 0; p + 1 < poff.size(); ++p)
        F->max_path = std::max(F->max_path, poff[p + 1] - poff[p]);
      if (std::min(F->max_path, d) > kMaxFreeSplits) F->n_paths = -1;
    } else {
      F->n_paths = -1;
    }
    if (F->n_paths > 0) {
      e = upload(&F->path_off, poff.data(), poff.size());
      if (e == hipSuccess) e = upload(&F->steps, psteps.data(), std::max<size_t>(psteps.size(), 1));
      if (e == hipSuccess) e = upload(&F->path_leaf, pleaf.data(), pleaf.size());
    }
  }
  if (e != hipSuccess) {
    return ffail(e == hipErrorOutOfMemory ? FSI_ERR_OUT_OF_MEMORY : FSI_ERR_HIP,
                 std::string("forest upload: ") + hipGetErrorString(e));
  }
  guard.f = nullptr;
  *out = F;
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_forest_destroy(fsi_forest_t forest) {
  FSI_ABI_TRY
  free_forest(forest);
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_forest_values(fsi_forest_t F, const double* x_dev, int n_bg, const double* bg_dev,
                             int dtype, void* v_dev, hipStream_t stream) {
  FSI_ABI_TRY
  if (!F) return ffail(FSI_ERR_INVALID_ARG, "forest is NULL");
  if (!x_dev || !bg_dev || !v_dev) return ffail(FSI_ERR_INVALID_ARG, "null device pointer");
  if (n_bg < 1 || n_bg > F->max_bg)
    return ffail(FSI_ERR_INVALID_ARG, "need 1 <= n_bg <= the forest's max_bg");
  if (dtype != FSI_DTYPE_F64 && dtype != FSI_DTYPE_F32)
    return ffail(FSI_ERR_INVALID_ARG, "dtype must be FSI_DTYPE_F64 or FSI_DTYPE_F32");
  if (((uintptr_t)v_dev | (uintptr_t)x_dev | (uintptr_t)bg_dev) & 15u)
    return ffail(FSI_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
  const int n_chunks = (n_bg + kBgChunk - 1) / kBgChunk;
  const int64_t prep_total = (int64_t)n_chunks * F->n_nodes;
  const int prep_grid = (int)std::min<int64_t>((prep_total + kThreads - 1) / kThreads, 4096);
  prep_kernel<<<prep_grid, kThreads, 0, stream>>>(F->feature, F->threshold, F->left, F->right,
                                                  F->n_nodes, F->d, x_dev, bg_dev, n_bg, F->prep);
  const int64_t n_coal = (int64_t)1 << F->d;
  const int64_t per_block = (int64_t)kThreads * kWalkKP;
  const int grid = (int)((n_coal + per_block - 1) / per_block);
  if (dtype == FSI_DTYPE_F64)
    walk_kernel<double, kWalkKP><<<grid, kThreads, 0, stream>>>(
        F->prep, F->value, F->roots, F->n_trees, F->n_nodes, n_bg, F->max_depth, F->d,
        (double*)v_dev);
  else
    walk_kernel<float, kWalkKP><<<grid, kThreads, 0, stream>>>(
        F->prep, F->value, F->roots, F->n_trees, F->n_nodes, n_bg, F->max_depth, F->d,
        (float*)v_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ffail(FSI_ERR_HIP, std::string("forest launch: ") + hipGetErrorString(e));
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_forest_mobius(fsi_forest_t F, const double* x_dev, int n_bg, const double* bg_dev,
                             double* a_dev, hipStream_t stream) {
  FSI_ABI_TRY
  if (!F) return ffail(FSI_ERR_INVALID_ARG, "forest is NULL");
  if (!x_dev || !bg_dev || !a_dev) return ffail(FSI_ERR_INVALID_ARG, "null device pointer");
  if (n_bg < 1 || n_bg > F->max_bg)
    return ffail(FSI_ERR_INVALID_ARG, "need 1 <= n_bg <= the forest's max_bg");
  if (((uintptr_t)a_dev | (uintptr_t)x_dev | (uintptr_t)bg_dev) & 15u)
    return ffail(FSI_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
  if (F->n_paths < 0)
    return ffail(FSI_ERR_UNSUPPORTED, "the Moebius route needs at most 2^26 root-to-leaf paths "
                                      "of at most 24 splits (or d <= 24)");
  const int64_t n_coal = (int64_t)1 << F->d;
  fill_kernel<<<(int)std::min<int64_t>((n_coal + kThreads - 1) / kThreads, 8192), kThreads, 0,
                stream>>>(a_dev, n_coal);
  const int64_t work = (int64_t)n_bg * F->n_paths;
  mobius_scatter_kernel<<<(int)std::min<int64_t>((work + kThreads - 1) / kThreads, 65535),
                          kThreads, 0, stream>>>(F->path_off, F->steps, F->path_leaf, F->n_paths,
                                                 F->feature, F->threshold, F->value, F->d, x_dev,
                                                 bg_dev, n_bg, a_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ffail(FSI_ERR_HIP, std::string("forest launch: ") + hipGetErrorString(e));
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_forest_values_mobius(fsi_forest_t F, const double* x_dev, int n_bg,
                                    const double* bg_dev, double* work_dev, int dtype,
                                    void* v_dev, hipStream_t stream) {
  FSI_ABI_TRY
  if (!F) return ffail(FSI_ERR_INVALID_ARG, "forest is NULL");
  if (!v_dev) return ffail(FSI_ERR_INVALID_ARG, "null device pointer");
  if (dtype != FSI_DTYPE_F64 && dtype != FSI_DTYPE_F32)
    return ffail(FSI_ERR_INVALID_ARG, "dtype must be FSI_DTYPE_F64 or FSI_DTYPE_F32");
  if ((uintptr_t)v_dev & 15u) return ffail(FSI_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
  if (dtype == FSI_DTYPE_F32 && (void*)work_dev == v_dev)
    return ffail(FSI_ERR_INVALID_ARG, "an FP32 output needs its own FP64 workspace");
  fsi_status st = fsi_forest_mobius(F, x_dev, n_bg, bg_dev, work_dev, stream);
  if (st != FSI_OK) return st;
  const int d = F->d;
  const int lb = std::min(d, kZetaLow);
  if (lb == d) {
    if (dtype == FSI_DTYPE_F32)
      zeta_low_kernel<float><<<1, kThreads, 0, stream>>>(work_dev, lb, (float*)v_dev);
    else
      zeta_low_kernel<double><<<1, kThreads, 0, stream>>>(work_dev, lb, (double*)v_dev);
  } else {
    zeta_low_kernel<double><<<1 << (d - lb), kThreads, 0, stream>>>(work_dev, lb, work_dev);
  }
  for (int bit0 = lb; bit0 < d; bit0 += kZetaBits) {
    const int nb = std::min(kZetaBits, d - bit0);
    const bool last = bit0 + nb >= d;
    if (last && dtype == FSI_DTYPE_F32)
      launch_zeta<float>(work_dev, d, bit0, nb, (float*)v_dev, stream);
    else if (last)
      launch_zeta<double>(work_dev, d, bit0, nb, (double*)v_dev, stream);
    else
      launch_zeta<double>(work_dev, d, bit0, nb, work_dev, stream);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ffail(FSI_ERR_HIP, std::string("forest launch: ") + hipGetErrorString(e));
  return FSI_OK;
  FSI_ABI_CATCH
}

}  // extern "C"
