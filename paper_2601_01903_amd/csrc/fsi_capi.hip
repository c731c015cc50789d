// C ABI of the FSI operator (declarations and contracts: include/fsi.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <queue>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <utility>
#include <vector>

#include "../../include/fsi.h"
#include "fsi_abi.h"
#include "fsi_internal.h"
#include "fsi_kernels.h"

using namespace fsi;

namespace {

thread_local std::string g_err;

fsi_status fail(fsi_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(call)                                                            \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(e_ == hipErrorOutOfMemory ? FSI_ERR_OUT_OF_MEMORY : FSI_ERR_HIP, \
                  std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

bool device_is_gfx950(int* dev, int* n_cu, std::string* why) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    *why = "no HIP device";
    return false;
  }
  if (hipGetDevice(dev) != hipSuccess) {
    *why = "hipGetDevice failed";
    return false;
  }
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, *dev) != hipSuccess) {
    *why = "hipGetDeviceProperties failed";
    return false;
  }
  if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) {
    *why = std::string("device is ") + p.gcnArchName + ", this library is built for gfx950";
    return false;
  }
  *n_cu = p.multiProcessorCount;
  return true;
}

}  // namespace

namespace fsi {
void record_error(const std::string& msg) { g_err = msg; }
void record_error_noexcept(const char* msg) noexcept {
  try {
    g_err = msg;
  } catch (...) {
  }
}
void record_error_noexcept2(const char* a, const char* b) noexcept {
  try {
    g_err = std::string(a) + b;
  } catch (...) {
  }
}
bool test_fail_alloc(const char* site) {
  const char* v = std::getenv("FSI_TEST_FAIL_ALLOC");
  return v && std::strcmp(v, site) == 0;
}
bool gfx950_device(int* dev, int* n_cu, std::string* why) { return device_is_gfx950(dev, n_cu, why); }
}  // namespace fsi

struct fsi_batch_plan_s {
  int n = 0, dtype = FSI_DTYPE_F64, prec = PREC_F64, algo = ALGO_FUSED;
  int in_place = 0;                // two-pass: the input buffer is the Moebius workspace
  int device = 0, n_cu = 256;
  std::vector<int> d, l, cls_of;
  std::vector<int64_t> voff, ooff;
  std::vector<ClassHost> classes;
  // device memory
  void* arena = nullptr;           // tables, descriptors, work lists
  double* Y = nullptr;
  void* work = nullptr;            // two-pass Moebius workspace
  double* partial = nullptr;       // register-phase kernel partial sums
  double* wide_partial = nullptr;  // wide gather partial sums
  std::vector<FastClassHost> fclasses;
  std::vector<int> fast_of;        // per class: index into fclasses or -1
  LaunchArgs args{};
  // bytes of each device workspace an apply writes and reads back (partial
  // sums, per-tile results, wide-gather partials, two-pass Moebius
  // workspace): the no-allocation entry point carves them from its static
  // scratch array instead
  size_t partial_bytes = 0, y_bytes = 0, wide_bytes = 0, work_bytes = 0;
  int64_t ylo_off = -1;            // two-pass FP64: low words at Y + ylo_off
  // recorded after every apply on the caller's stream (outside stream
  // capture): destroying the plan waits for it, not for the whole device
  hipEvent_t done = nullptr;
  int tile_bits_reported = 0;
  fsi_schedule sched{};            // the schedule this plan was built with
  // graph cache
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* g_in = nullptr;
  void* g_out = nullptr;
};

struct fsi_plan_s {
  fsi_batch_plan_s* bp = nullptr;
  int d = 0, l = 0;
  std::vector<TileItem> dummy;
};

namespace {

void free_batch(fsi_batch_plan_s* p) {
  if (!p) return;
  if (p->done) {
    (void)hipEventSynchronize(p->done);
    (void)hipEventDestroy(p->done);
  }
  // an apply still replaying on the plan's capture stream, or a launch on a
  // stream the completion event did not see (one being captured by the
  // caller): the plan's own stream and the kernels it replayed finish first
  if (p->cap_stream) (void)hipStreamSynchronize(p->cap_stream);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->arena) (void)hipFree(p->arena);
  if (p->Y) (void)hipFree(p->Y);
  if (p->work) (void)hipFree(p->work);
  if (p->partial) (void)hipFree(p->partial);
  if (p->wide_partial) (void)hipFree(p->wide_partial);
  delete p;
}

int resolve_prec(int dtype, int prec) {
  if (prec == FSI_PREC_AUTO) return dtype == FSI_DTYPE_F64 ? PREC_F64 : PREC_F32_FP64MOB;
  return prec;
}

// Largest tile (b <= 12, b <= d) whose sweep state double-buffers in LDS.
int choose_tile_bits(int d, int l, int prec, int requested) {
  if (requested > 0) return requested;
  for (int b = std::min(d, kMaxTileBits); b >= 1; --b) {
    const int64_t need = std::max<int64_t>(2 * sweep_peak_entries(b, l) * (int64_t)sweep_elem_bytes(prec),
                                           ((int64_t)1 << b) * (int64_t)mob_elem_bytes(prec));
    if (need <= kLdsBudget) return b;
  }
  return 1;
}

// Appends an aligned block to a host staging buffer and returns its offset.
template <typename T>
size_t stage(std::vector<unsigned char>& buf, const T* data, size_t count) {
  size_t off = (buf.size() + 255) & ~(size_t)255;
  buf.resize(off + count * sizeof(T));
  if (count) std::memcpy(buf.data() + off, data, count * sizeof(T));
  return off;
}

// Schedule knobs the autotuner varies (the defaults are the heuristics).
struct Sched {
  int kernel = -1;      // fsi_kernel to use, -1: the option's
  int tb_shift = 0;     // generic tile: bits relative to the largest that fits LDS (<= 0)
  int chunk_shift = 0;  // register-phase kernel: log2 tiles per item relative to the default
  int mob_group = 0;    // two-pass: bits per strided high Moebius pass (0: 6)
  int algo = 0;         // FSI_ALGO_FUSED or FSI_ALGO_TWO_PASS; 0: the option's
};

// FSI_ALGO_AUTO without the autotuner: the fused algorithm, unless every
// instance has an order of at least kAutoTwoPassL (value input, no kernel
// named: a named kernel is one of the fused algorithm's). Such
// instances run on the generic kernel, whose per-tile results feed a gather
// over M outputs x 2^h tiles; the two-pass algorithm's counter sweep over
// the Moebius transform does not grow that way with M (32 x d = 20 at
// l = 8: 7.6 against 29 ms in FP32, 16 against 32 ms in FP64; at l = 6 the
// two are within 15% either way, at l = 5 the fused one is faster).
constexpr int kAutoTwoPassL = 7;
int auto_algo(int n, const int* lh, const fsi_plan_opts& o) {
  if (o.input != FSI_INPUT_VALUES || o.kernel != FSI_KERNEL_AUTO) return ALGO_FUSED;
  for (int i = 0; i < n; ++i)
    if (lh[i] < kAutoTwoPassL) return ALGO_FUSED;
  return ALGO_TWO_PASS;
}

fsi_status build_batch(int n, const int* dh, const int* lh, const fsi_plan_opts* opts_in,
                       bool single, fsi_batch_plan_s** out, const Sched& sc = Sched{}) {
  *out = nullptr;
  if (n < 1) return fail(FSI_ERR_INVALID_ARG, "n must be >= 1");
  if (!dh || !lh) return fail(FSI_ERR_INVALID_ARG, "null d or l array");
  fsi_plan_opts opts;
  fsi_default_opts(&opts);
  if (opts_in) opts = *opts_in;
  if (opts.allow_input_overwrite != 0 && opts.allow_input_overwrite != 1)
    return fail(FSI_ERR_INVALID_ARG, "allow_input_overwrite must be 0 or 1");
  if (opts.input != FSI_INPUT_VALUES && opts.input != FSI_INPUT_MOBIUS)
    return fail(FSI_ERR_INVALID_ARG, "unknown input kind");
  if (opts.input == FSI_INPUT_MOBIUS && opts.algo == FSI_ALGO_TWO_PASS)
    return fail(FSI_ERR_INVALID_ARG, "Moebius input needs the fused algorithm");
  if (opts.index < FSI_INDEX_FSI || opts.index > FSI_INDEX_BII)
    return fail(FSI_ERR_INVALID_ARG, "unknown interaction index");
  if (opts.kernel < FSI_KERNEL_AUTO || opts.kernel > FSI_KERNEL_REGISTER)
    return fail(FSI_ERR_INVALID_ARG, "unknown kernel");
  if (opts.dtype != FSI_DTYPE_F64 && opts.dtype != FSI_DTYPE_F32)
    return fail(FSI_ERR_INVALID_ARG, "dtype must be FSI_DTYPE_F64 or FSI_DTYPE_F32");
  if (opts.precision < 0 || opts.precision > FSI_PREC_AUTO)
    return fail(FSI_ERR_INVALID_ARG, "unknown precision");
  const int prec = resolve_prec(opts.dtype, opts.precision);
  if (opts.dtype == FSI_DTYPE_F64 && prec != PREC_F64)
    return fail(FSI_ERR_INVALID_ARG, "FP64 storage supports FSI_PREC_F64 only");
  if (opts.dtype == FSI_DTYPE_F32 && prec == PREC_F64)
    return fail(FSI_ERR_INVALID_ARG, "FP32 storage needs an FP32 precision mode");
  if (opts.algo < 0 || opts.algo > FSI_ALGO_TWO_PASS)
    return fail(FSI_ERR_INVALID_ARG, "unknown algo");
  // FSI_ALGO_AUTO: the autotuner's choice (a schedule's algorithm), else the
  // heuristic; an explicit algorithm is never overridden
  const bool sched_algo = opts.algo == FSI_ALGO_AUTO && opts.input == FSI_INPUT_VALUES &&
                          (sc.algo == FSI_ALGO_FUSED || sc.algo == FSI_ALGO_TWO_PASS);
  const int algo = sched_algo ? sc.algo
                   : opts.algo == FSI_ALGO_AUTO ? auto_algo(n, lh, opts) : opts.algo;
  if (opts.block_threads != 0)
    return fail(FSI_ERR_INVALID_ARG, "block_threads is reserved and must be 0");
  if (opts.tile_bits < 0 || opts.tile_bits > kMaxTileBits)
    return fail(FSI_ERR_INVALID_ARG, "tile_bits must be in [0, 12]");
  for (int i = 0; i < n; ++i) {
    if (!(1 <= dh[i] && dh[i] <= kMaxD && 1 <= lh[i] && lh[i] <= dh[i]))
      return fail(FSI_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": need 1 <= l <= d <= 30");
    if (opts.tile_bits > dh[i])
      return fail(FSI_ERR_INVALID_ARG, "tile_bits larger than d");
  }
  // test hook: a host allocation failure while the plan is built (before
  // any device call, so it is reachable without a GPU)
  if (test_fail_alloc("host")) throw std::bad_alloc();
  int dev = 0, n_cu = 0;
  std::string why;
  if (!device_is_gfx950(&dev, &n_cu, &why)) return fail(FSI_ERR_UNSUPPORTED, why);

  auto* P = new (std::nothrow) fsi_batch_plan_s();
  if (!P) return fail(FSI_ERR_OUT_OF_MEMORY, "host allocation failed");
  // frees the partly built plan if a host allocation below throws
  struct Guard {
    fsi_batch_plan_s* p;
    ~Guard() { free_batch(p); }
  } guard{P};
  P->n = n; P->dtype = opts.dtype; P->prec = prec; P->algo = algo;
  // the input buffer can hold the Moebius transform in place when the
  // butterfly runs in the storage type
  P->in_place = opts.allow_input_overwrite && algo == ALGO_TWO_PASS &&
                mob_elem_bytes(prec) == (opts.dtype == FSI_DTYPE_F64 ? 8u : 4u);
  P->device = dev; P->n_cu = n_cu;
  P->d.assign(dh, dh + n);
  P->l.assign(lh, lh + n);

  // ---- classes ----
  std::map<std::pair<int, int>, int> cls_index;
  P->cls_of.resize(n);
  for (int i = 0; i < n; ++i) {
    auto key = std::make_pair(dh[i], lh[i]);
    auto it = cls_index.find(key);
    if (it == cls_index.end()) {
      ClassHost C;
      // register-phase kernel: fused algorithm, l <= 4, tile of 11 bits. An
      // instance with d < 11 runs as the d = 11 instance of the game that
      // ignores the players past d: its Moebius coefficients vanish on every
      // set holding one of them and the weights W(s, t) do not depend on d,
      // so the outputs of the sets inside [d] are the instance's own
      const int fb = kFastTileBits;
      const int kern = sc.kernel >= 0 ? sc.kernel : opts.kernel;
      const int dfast = std::max(dh[i], fb);
      const bool want_fast = kern != FSI_KERNEL_GENERIC && algo == ALGO_FUSED &&
                             fast_supported(prec) && lh[i] <= kFastMaxL &&
                             fast_block_bits(dfast, lh[i]) >= 0 &&
                             (opts.tile_bits == 0 || opts.tile_bits == fb);
      if (kern == FSI_KERNEL_REGISTER && !want_fast) {
        return fail(FSI_ERR_UNSUPPORTED, "register-phase kernel does not apply to instance " +
                                             std::to_string(i));
      }
      int b = want_fast ? fb : choose_tile_bits(dh[i], lh[i], prec, opts.tile_bits);
      if (!want_fast && opts.tile_bits == 0) b = std::max(1, b + sc.tb_shift);
      std::string err = build_class(want_fast ? dfast : dh[i], lh[i], b, algo, opts.index,
                                    opts.input, &C);
      if (!err.empty()) { return fail(FSI_ERR_INTERNAL, err); }
      if (want_fast && dh[i] < fb) {
        // the outputs are those of the instance's own d
        C.out_masks = canonical_masks(dh[i], lh[i]);
        C.M = (int)C.out_masks.size();
      }
      const int64_t need = std::max<int64_t>(2 * (int64_t)C.lds_elems * (int64_t)sweep_elem_bytes(prec),
                                             ((int64_t)1 << b) * (int64_t)mob_elem_bytes(prec));
      if (!want_fast && need > kLdsBudget) {
        return fail(FSI_ERR_INVALID_ARG, "tile_bits too large for LDS at this l and precision");
      }
      int fidx = -1;
      if (want_fast) {
        FastClassHost F;
        err = build_fast_class(C, &F);
        if (!err.empty()) { return fail(FSI_ERR_INTERNAL, err); }
        fidx = (int)P->fclasses.size();
        P->fclasses.push_back(std::move(F));
      }
      P->fast_of.push_back(fidx);
      cls_index[key] = (int)P->classes.size();
      P->classes.push_back(std::move(C));
      it = cls_index.find(key);
    }
    P->cls_of[i] = it->second;
  }
  P->tile_bits_reported = P->classes[0].b;
  if (n_cu <= 0) n_cu = 1;

  // ---- instances, offsets, work lists ----
  std::vector<InstDev> insts(n);
  P->voff.assign(n + 1, 0);
  P->ooff.assign(n + 1, 0);
  int64_t ytot = 0, wtot = 0;
  for (int i = 0; i < n; ++i) {
    const ClassHost& C = P->classes[P->cls_of[i]];
    P->voff[i + 1] = P->voff[i] + ((int64_t)1 << dh[i]);
    P->ooff[i + 1] = P->ooff[i] + C.M;
    insts[i].cls = P->cls_of[i];
    insts[i].d = dh[i];
    insts[i].voff = P->voff[i];
    insts[i].ooff = P->ooff[i];
    insts[i].yoff = ytot;
    insts[i].woff = single ? 0 : wtot;
    // per-tile results in HBM only for the generic kernel (the register-phase
    // kernel keeps them in LDS)
    if (P->fast_of[P->cls_of[i]] < 0) ytot += ((int64_t)1 << C.h) * C.Ysize;
    wtot += (int64_t)1 << dh[i];
  }
  // register-phase work items: runs of tiles of one instance, in the order of
  // the class's tile list: block by block (blocks of 2^kb tiles sharing
  // their top h - kb high bits; one block when kb = h), the tiles of a block
  // sorted by popcount, so the final weights change at most kb + 1 times
  // per block
  std::vector<int32_t> torder;
  std::vector<int32_t> tofs_of_fast(P->fclasses.size(), 0);
  for (size_t f = 0; f < P->fclasses.size(); ++f) {
    tofs_of_fast[f] = (int32_t)torder.size();
    const int h = P->fclasses[f].h, kb = P->fclasses[f].kb;
    std::vector<int32_t> ord((size_t)1 << kb);
    for (size_t t = 0; t < ord.size(); ++t) ord[t] = (int32_t)t;
    std::stable_sort(ord.begin(), ord.end(), [](int32_t x, int32_t y) {
      return __builtin_popcount(x) < __builtin_popcount(y);
    });
    for (int64_t blk = 0; blk < ((int64_t)1 << (h - kb)); ++blk)
      for (int32_t t : ord) torder.push_back((int32_t)((blk << kb) | t));
  }
  // tiles the register-phase kernel walks
  int64_t fast_tiles = 0;
  for (int i = 0; i < n; ++i)
    if (P->fast_of[P->cls_of[i]] >= 0) fast_tiles += (int64_t)1 << P->classes[P->cls_of[i]].h;
  // tiles per work item: the candidate size (powers of two and 1.5 times
  // them) whose simulated launch ends first. The model: an item costs its
  // tiles at the order's measured cost per tile plus a fixed cost (the first
  // tile's loads, which nothing prefetches, and the partial-sum write);
  // workgroup b runs item b, then the workgroups take the items in order of
  // decreasing cost as they finish (the kernel's work queue); the reduction
  // reads every item's partial sums. Small items balance the end of the
  // launch, large ones write fewer partial sums.
  int slots = n_cu;
  for (size_t f = 0; f < P->fclasses.size(); ++f)
    slots = std::max(slots, n_cu * fast_wgs_per_cu(prec, P->fclasses[f].l));
  // tiles of one item of instance i at a nominal size c: any size inside a
  // one-block instance (its last item takes the rest), a power of two
  // dividing the block for an instance of several blocks
  auto item_tiles = [&](int i, int64_t c) {
    const FastClassHost& F = P->fclasses[P->fast_of[P->cls_of[i]]];
    const int64_t ntile = (int64_t)1 << F.h, bsize = (int64_t)1 << F.kb;
    if (F.kb >= F.h) return std::min<int64_t>(c, ntile);
    int64_t cs = std::min<int64_t>(c, bsize);
    while (cs & (cs - 1)) cs &= cs - 1;
    return cs;
  };
  int64_t chunk = 1;
  {
    static const double kTileUs[kFastMaxL + 1] = {0.0, 2.47, 3.03, 3.65, 3.79};
    const double tile_scale = prec == PREC_F64 ? 2.3 : 1.0;
    const double item_us = 6.0, red_base_us = 4.0, red_bytes_per_us = 3.0e6;
    int64_t max_tiles = 1;
    for (int i = 0; i < n; ++i)
      if (P->fast_of[P->cls_of[i]] >= 0)
        max_tiles = std::max<int64_t>(max_tiles, (int64_t)1 << P->classes[P->cls_of[i]].h);
    std::vector<int64_t> cand;
    for (int64_t c2 = 1; c2 <= max_tiles; c2 *= 2) {
      cand.push_back(c2);
      if (c2 >= 2 && c2 + c2 / 2 <= max_tiles) cand.push_back(c2 + c2 / 2);
    }
    double best = -1.0;
    std::vector<double> cost;
    for (int64_t c : cand) {
      // sizes that cut the batch into far more items than workgroups only
      // add partial sums (the largest size is always simulated)
      int64_t items = 0;
      for (int i = 0; i < n; ++i)
        if (P->fast_of[P->cls_of[i]] >= 0) {
          const int64_t ntile = (int64_t)1 << P->classes[P->cls_of[i]].h;
          items += (ntile + item_tiles(i, c) - 1) / item_tiles(i, c);
        }
      if (items > 64 * (int64_t)slots && c != cand.back()) continue;
      cost.clear();
      double part_bytes = 0.0;
      for (int i = 0; i < n; ++i) {
        const int f = P->fast_of[P->cls_of[i]];
        if (f < 0) continue;
        const FastClassHost& F = P->fclasses[f];
        const int64_t ntile = (int64_t)1 << F.h, cs = item_tiles(i, c);
        for (int64_t tb = 0; tb < ntile; tb += cs) {
          const int64_t nt = std::min<int64_t>(cs, ntile - tb);
          cost.push_back((double)nt * kTileUs[F.l] * tile_scale + item_us);
          part_bytes += (double)F.nkk * kFastThreads * 8.0;
        }
      }
      std::sort(cost.begin(), cost.end(), std::greater<double>());
      std::priority_queue<double, std::vector<double>, std::greater<double>> busy;
      for (double x : cost) {
        if ((int)busy.size() < slots) {
          busy.push(x);
        } else {
          const double t = busy.top();
          busy.pop();
          busy.push(t + x);
        }
      }
      double end = 0.0;
      while (!busy.empty()) { end = std::max(end, busy.top()); busy.pop(); }
      const double total = end + red_base_us + part_bytes / red_bytes_per_us;
      if (best < 0.0 || total < best) { best = total; chunk = c; }
    }
    if (sc.chunk_shift > 0) chunk <<= sc.chunk_shift;
    if (sc.chunk_shift < 0) chunk = std::max<int64_t>(1, chunk >> -sc.chunk_shift);
  }
  // work items: tile ranges of an instance's tile order (inside a block for
  // instances of several blocks); item j of an instance covers block j / ipb
  // and has its partial sums at pbase + j * pstride
  std::vector<FastItem> fitems;
  int64_t ptot = 0;
  for (int i = 0; i < n; ++i) {
    const int f = P->fast_of[P->cls_of[i]];
    if (f < 0) continue;
    const FastClassHost& F = P->fclasses[f];
    const int64_t ntile = (int64_t)1 << F.h, bsize = (int64_t)1 << F.kb;
    const int64_t cs = item_tiles(i, chunk);
    const int64_t nit = (ntile + cs - 1) / cs;
    insts[i].fast = 1;
    insts[i].fcls = f;
    insts[i].tofs = tofs_of_fast[f];
    insts[i].pbase = ptot;
    insts[i].pstride = F.nkk * kFastThreads;
    insts[i].nitems = (int32_t)nit;
    insts[i].ipb = (int32_t)(F.kb >= F.h ? nit : bsize / cs);
    insts[i].pw = F.l + 1;
    insts[i].lowmask = dh[i] < kFastTileBits ? (1 << dh[i]) - 1 : (1 << kFastTileBits) - 1;
    for (int64_t tb = 0; tb < ntile; tb += cs) {
      fitems.push_back(FastItem{i, (int32_t)tb, (int32_t)std::min<int64_t>(tb + cs, ntile), 0, ptot});
      ptot += (int64_t)F.nkk * kFastThreads;
    }
  }
  // reduction of the register-phase partial sums of one-block instances, in
  // slot order (consecutive threads read consecutive slots of an item): one
  // slot per thread when no instance has more than two items, four item rows
  // up to 64 items, sixteen past that (a small instance split into one-tile
  // items); instances of several blocks go to the wide gather
  int red_rows = 1;
  for (int i = 0; i < n; ++i)
    if (insts[i].fast && insts[i].nitems == insts[i].ipb) {
      if (insts[i].nitems > 64) red_rows = std::max(red_rows, 16);
      else if (insts[i].nitems > 2) red_rows = std::max(red_rows, 4);
    }
  const int red_width = kFastThreads / red_rows;
  std::vector<int2> red_chunks;
  int n_generic = 0;
  for (int i = 0; i < n; ++i) {
    if (!insts[i].fast) {
      // generic fused instances with many tiles: the wide gather
      insts[i].wide = (algo == ALGO_FUSED && P->classes[P->cls_of[i]].h >= kWideMinH) ? 1 : 0;
      if (!insts[i].wide) ++n_generic;
      continue;
    }
    if (insts[i].nitems > insts[i].ipb) {
      insts[i].wide = 1;
      continue;
    }
    const int nslot = insts[i].pstride;
    for (int s0 = 0; s0 < nslot; s0 += red_width) red_chunks.push_back(make_int2(i, s0));
  }
  // wide gather items: per instance, output groups x ranges of tiles
  // (generic instances) or blocks (register-phase instances); the ranges (a
  // power of two) give the machine about two items per CU
  std::vector<WideItem> witems;
  std::vector<WideGroup> wgroups;
  int64_t wptot = 0;
  {
    int64_t total_groups = 0;
    for (int i = 0; i < n; ++i)
      if (insts[i].wide) total_groups += (P->classes[P->cls_of[i]].M + kWideOuts - 1) / kWideOuts;
    int64_t nr_target = 1;
    while (total_groups > 0 && nr_target * total_groups < 2 * (int64_t)n_cu) nr_target *= 2;
    for (int i = 0; i < n; ++i) {
      if (!insts[i].wide) continue;
      const ClassHost& C = P->classes[P->cls_of[i]];
      const int64_t ntile =
          insts[i].fast ? (int64_t)insts[i].nitems / insts[i].ipb : (int64_t)1 << C.h;
      const int64_t nr = std::min(nr_target, ntile);
      const int64_t per = ntile / nr;
      const int G = (C.M + kWideOuts - 1) / kWideOuts;
      for (int g = 0; g < G; ++g) {
        wgroups.push_back(WideGroup{i, g, (int32_t)nr, 0, wptot});
        for (int64_t r = 0; r < nr; ++r)
          witems.push_back(WideItem{i, g, (int32_t)(r * per), (int32_t)((r + 1) * per),
                                    wptot + r * kWideOuts});
        wptot += nr * kWideOuts;
      }
    }
  }
  // the items of each order l counted (a plan with one order launches the
  // kernel compiled for it)
  auto item_l = [&](const FastItem& it) { return P->fclasses[P->fast_of[P->cls_of[it.inst]]].l; };
  std::stable_sort(fitems.begin(), fitems.end(),
                   [&](const FastItem& x, const FastItem& y) { return item_l(x) < item_l(y); });
  int lbeg[kFastMaxL + 2];
  for (int l = 0; l <= kFastMaxL + 1; ++l) lbeg[l] = 0;
  {
    int cnt[kFastMaxL + 2] = {0};
    for (const FastItem& it : fitems) ++cnt[item_l(it)];
    int acc = 0;
    for (int l = 1; l <= kFastMaxL; ++l) { lbeg[l] = acc; acc += cnt[l]; }
    lbeg[kFastMaxL + 1] = acc;
  }
  // several orders run as one launch over all items (the kernel dispatches
  // per item): the costliest items first, so that the launch's work queue
  // ends evenly. Cost = tiles x the order's relative cost per tile (measured
  // on 256 x d = 20: 2.5, 3.0, 3.6 and 3.8 us per tile and workgroup at
  // l = 1 .. 4).
  int n_orders = 0;
  for (int l = 1; l <= kFastMaxL; ++l) n_orders += lbeg[l + 1] > lbeg[l];
  if (n_orders >= 1) {
    static const int64_t kTileCost[kFastMaxL + 1] = {0, 65, 80, 96, 100};
    auto item_cost = [&](const FastItem& it) { return (int64_t)(it.te - it.tb) * kTileCost[item_l(it)]; };
    std::stable_sort(fitems.begin(), fitems.end(), [&](const FastItem& x, const FastItem& y) {
      const int64_t cx = item_cost(x), cy = item_cost(y);
      if (cx != cy) return cx > cy;
      return item_l(x) > item_l(y);
    });
  }

  // every tile of every instance (standalone Moebius low pass)
  std::vector<TileItem> all_tiles;
  for (int i = 0; i < n; ++i) {
    const ClassHost& C = P->classes[P->cls_of[i]];
    for (int64_t t = 0; t < ((int64_t)1 << C.h); ++t) all_tiles.push_back(TileItem{i, (int32_t)t});
  }
  // generic tiles: larger tiles first, so a persistent grid finishes evenly
  std::vector<TileItem> tiles;
  for (int i = 0; i < n; ++i) {
    if (insts[i].fast) continue;
    const ClassHost& C = P->classes[P->cls_of[i]];
    for (int64_t t = 0; t < ((int64_t)1 << C.h); ++t) tiles.push_back(TileItem{i, (int32_t)t});
  }
  std::stable_sort(tiles.begin(), tiles.end(), [&](const TileItem& a, const TileItem& b) {
    return P->classes[P->cls_of[a.inst]].b > P->classes[P->cls_of[b.inst]].b;
  });
  // strided high-bit passes of the two-pass butterfly (also fsi_mobius)
  std::vector<MobItem> mob[kMaxMobPasses];
  int n_passes = 0;
  for (int i = 0; i < n; ++i) {
    const ClassHost& C = P->classes[P->cls_of[i]];
    int lo = C.b, p = 0;
    while (lo < dh[i]) {
      const int G = std::min(sc.mob_group > 0 ? sc.mob_group : 6, dh[i] - lo);
      const int cb = std::min(lo, kMaxTileBits - G);
      if (p >= kMaxMobPasses) { return fail(FSI_ERR_INTERNAL, "too many passes"); }
      const int64_t nblk = (int64_t)1 << (dh[i] - G - cb);
      for (int64_t bk = 0; bk < nblk; ++bk) mob[p].push_back(MobItem{i, lo, G, cb, bk});
      lo += G;
      ++p;
    }
    n_passes = std::max(n_passes, p);
  }

  // ---- device arena ----
  std::vector<unsigned char> buf;
  std::vector<ClassDev> cdev(P->classes.size());
  struct Offs { size_t step_off, step_np, pat, ytab, lam, lam_lo, lam_soff, oinfo, osh; };
  std::vector<Offs> co(P->classes.size());
  for (size_t c = 0; c < P->classes.size(); ++c) {
    const ClassHost& C = P->classes[c];
    co[c].step_off = stage(buf, C.step_off.data(), C.step_off.size());
    co[c].step_np = stage(buf, C.step_np.data(), C.step_np.size());
    co[c].pat = stage(buf, C.pat.data(), C.pat.size());
    co[c].ytab = stage(buf, C.ytab.data(), C.ytab.size());
    co[c].lam = stage(buf, C.lam.data(), C.lam.size());
    co[c].lam_lo = stage(buf, C.lam_lo.data(), C.lam_lo.size());
    co[c].lam_soff = stage(buf, C.lam_soff.data(), C.lam_soff.size());
    co[c].oinfo = stage(buf, C.oinfo.data(), C.oinfo.size());
    co[c].osh = stage(buf, C.osh.data(), C.osh.size());
  }
  std::vector<FastClassDev> fdev(P->fclasses.size());
  struct FOffs { size_t lam, meta, gs8, unit_mask, zrow, pidx, uperm, osh2, sinv; };
  std::vector<FOffs> fo(P->fclasses.size());
  for (size_t f = 0; f < P->fclasses.size(); ++f) {
    const FastClassHost& F = P->fclasses[f];
    fo[f].lam = stage(buf, F.lam.data(), F.lam.size());
    fo[f].meta = stage(buf, F.meta.data(), F.meta.size());
    fo[f].gs8 = stage(buf, F.gs8.data(), F.gs8.size());
    fo[f].pidx = stage(buf, F.pidx.data(), F.pidx.size());
    fo[f].osh2 = stage(buf, F.osh2.data(), F.osh2.size());
    fo[f].sinv = stage(buf, F.sinv.data(), F.sinv.size());
    fo[f].unit_mask = stage(buf, F.unit_mask.data(), F.unit_mask.size());
    fo[f].zrow = stage(buf, F.zrow.data(), F.zrow.size());
    fo[f].uperm = stage(buf, F.uperm.data(), F.uperm.size());
  }
  const size_t o_fcls = stage(buf, fdev.data(), fdev.size());
  const size_t o_fitems = stage(buf, fitems.data(), fitems.size());
  const size_t o_red = stage(buf, red_chunks.data(), red_chunks.size());
  const size_t o_witems = stage(buf, witems.data(), witems.size());
  const size_t o_wgroups = stage(buf, wgroups.data(), wgroups.size());
  const size_t o_torder = stage(buf, torder.data(), torder.size());
  const size_t o_cls = stage(buf, cdev.data(), cdev.size());
  const size_t o_inst = stage(buf, insts.data(), insts.size());
  const size_t o_tiles = stage(buf, tiles.data(), tiles.size());
  const size_t o_all_tiles = stage(buf, all_tiles.data(), all_tiles.size());
  size_t o_mob[kMaxMobPasses] = {0, 0, 0, 0};
  for (int p = 0; p < n_passes; ++p) o_mob[p] = stage(buf, mob[p].data(), mob[p].size());
  const size_t o_ooff = stage(buf, P->ooff.data(), P->ooff.size());
  // work queue of the register-phase launches: zero here, and every launch
  // leaves it zero
  const uint32_t queue0[4] = {0u, 0u, 0u, 0u};
  const size_t o_queue = stage(buf, queue0, 4);

  hipError_t e = hipMalloc(&P->arena, buf.size());
  if (e != hipSuccess) { return fail(FSI_ERR_OUT_OF_MEMORY, "hipMalloc(tables) failed"); }
  auto* A = static_cast<unsigned char*>(P->arena);
  for (size_t c = 0; c < P->classes.size(); ++c) {
    const ClassHost& C = P->classes[c];
    ClassDev& D = cdev[c];
    D.d = C.d; D.l = C.l; D.b = C.b; D.h = C.h; D.algo = C.algo;
    D.M = C.M; D.Ysize = C.Ysize; D.lam_ublock = C.lam_ublock;
    D.lds_elems = C.lds_elems; D.nfinal = C.nfinal; D.mobius_in = C.mobius_in;
    D.step_off = reinterpret_cast<const int32_t*>(A + co[c].step_off);
    D.step_np = reinterpret_cast<const int32_t*>(A + co[c].step_np);
    D.pat = reinterpret_cast<const uint32_t*>(A + co[c].pat);
    D.ytab = reinterpret_cast<const uint32_t*>(A + co[c].ytab);
    D.lam = reinterpret_cast<const double*>(A + co[c].lam);
    D.lam_lo = C.lam_lo.empty() ? nullptr : reinterpret_cast<const double*>(A + co[c].lam_lo);
    D.lam_soff = reinterpret_cast<const int32_t*>(A + co[c].lam_soff);
    D.oinfo = reinterpret_cast<const uint32_t*>(A + co[c].oinfo);
    D.osh = reinterpret_cast<const uint32_t*>(A + co[c].osh);
  }
  std::memcpy(buf.data() + o_cls, cdev.data(), cdev.size() * sizeof(ClassDev));
  size_t fast_lds[kFastMaxL + 1] = {0, 0, 0, 0, 0};
  size_t fast_lds_max = 0;
  for (size_t f = 0; f < P->fclasses.size(); ++f) {
    const FastClassHost& F = P->fclasses[f];
    FastClassDev& D = fdev[f];
    D.d = F.d; D.l = F.l; D.h = F.h; D.M = F.M; D.nkk = F.nkk; D.mshift = F.mshift; D.kb = F.kb;
    fast_lds[F.l] = fast_lds_bytes(prec, F.l);
    fast_lds_max = std::max(fast_lds_max, fast_lds[F.l]);
    D.lam = reinterpret_cast<const double*>(A + fo[f].lam);
    D.meta = reinterpret_cast<const uint32_t*>(A + fo[f].meta);
    D.gs8 = reinterpret_cast<const uint32_t*>(A + fo[f].gs8);
    D.unit_mask = reinterpret_cast<const int32_t*>(A + fo[f].unit_mask);
    D.zrow = reinterpret_cast<const int32_t*>(A + fo[f].zrow);
    D.uperm = reinterpret_cast<const int32_t*>(A + fo[f].uperm);
  }
  if (fast_lds_max > 160 * 1024) {
    return fail(FSI_ERR_INTERNAL, "register-phase kernel does not fit in LDS");
  }
  std::memcpy(buf.data() + o_fcls, fdev.data(), fdev.size() * sizeof(FastClassDev));
  for (int i = 0; i < n; ++i)
    if (insts[i].fast) {
      insts[i].pidx = reinterpret_cast<const int32_t*>(A + fo[insts[i].fcls].pidx);
      insts[i].osh2 = reinterpret_cast<const uint32_t*>(A + fo[insts[i].fcls].osh2);
      insts[i].sinv = P->fclasses[insts[i].fcls].sinv.empty()
                          ? nullptr
                          : reinterpret_cast<const int32_t*>(A + fo[insts[i].fcls].sinv);
    }
  // instance descriptors carry the fast fields filled above
  std::memcpy(buf.data() + o_inst, insts.data(), insts.size() * sizeof(InstDev));
  e = hipMemcpy(P->arena, buf.data(), buf.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { return fail(FSI_ERR_HIP, "hipMemcpy(tables) failed"); }

  // the two-pass FP64 path keeps each per-tile result as a double-double
  // (high words, then low words)
  const bool ycomp = algo == ALGO_TWO_PASS && prec == PREC_F64;
  const int64_t ywords = std::max<int64_t>(ytot, 1) * (ycomp ? 2 : 1);
  P->ylo_off = ycomp ? std::max<int64_t>(ytot, 1) : -1;
  e = hipMalloc(reinterpret_cast<void**>(&P->Y), ywords * sizeof(double));
  if (e != hipSuccess) { return fail(FSI_ERR_OUT_OF_MEMORY, "hipMalloc(Y) failed"); }
  if (algo == ALGO_TWO_PASS && !P->in_place) {
    const size_t wbytes = (size_t)wtot *
                          std::max(mob_elem_bytes(prec), (size_t)8);
    e = hipMalloc(&P->work, wbytes);
    if (e != hipSuccess) { return fail(FSI_ERR_OUT_OF_MEMORY, "hipMalloc(work) failed"); }
  }

  if (ptot > 0) {
    e = test_fail_alloc("device") ? hipErrorOutOfMemory
                                  : hipMalloc(reinterpret_cast<void**>(&P->partial), ptot * sizeof(double));
    if (e != hipSuccess) { return fail(FSI_ERR_OUT_OF_MEMORY, "hipMalloc(partial) failed"); }
  }
  if (wptot > 0) {
    e = hipMalloc(reinterpret_cast<void**>(&P->wide_partial), wptot * sizeof(double));
    if (e != hipSuccess) { return fail(FSI_ERR_OUT_OF_MEMORY, "hipMalloc(wide partial) failed"); }
  }

  // ---- schedule ----
  // Moebius passes stage at most 2^12 elements of at most 8 bytes
  const size_t mob_lds = ((size_t)1 << kMaxTileBits) * 8;
  size_t tile_lds = 0;
  for (size_t c = 0; c < P->classes.size(); ++c) {
    const ClassHost& C = P->classes[c];
    if (P->fast_of[c] >= 0) continue;
    tile_lds = std::max<size_t>(tile_lds, std::max<size_t>(2 * (size_t)C.lds_elems * sweep_elem_bytes(prec),
                                                           ((size_t)1 << C.b) * mob_elem_bytes(prec)));
  }
  e = configure_kernels(prec, algo, tile_lds, mob_lds);
  if (e != hipSuccess) { return fail(FSI_ERR_HIP, std::string("configure_kernels: ") + hipGetErrorString(e)); }
  if (tile_lds == 0) tile_lds = 1024;
  const int per_cu = std::max(1, std::min<int>(4, (int)((160 * 1024) / std::max<size_t>(tile_lds, 1))));
  LaunchArgs& a = P->args;
  a.prec = prec; a.algo = algo;
  a.classes = reinterpret_cast<const ClassDev*>(A + o_cls);
  a.insts = reinterpret_cast<const InstDev*>(A + o_inst);
  a.n_inst = n;
  a.tile_items = reinterpret_cast<const TileItem*>(A + o_tiles);
  a.n_tile_items = (int)tiles.size();
  a.all_tiles = reinterpret_cast<const TileItem*>(A + o_all_tiles);
  a.n_all_tiles = (int)all_tiles.size();
  a.n_mob_passes = n_passes;
  for (int p = 0; p < kMaxMobPasses; ++p) {
    a.mob_items[p] = p < n_passes ? reinterpret_cast<const MobItem*>(A + o_mob[p]) : nullptr;
    a.n_mob_items[p] = p < n_passes ? (int)mob[p].size() : 0;
  }
  a.out_offset = reinterpret_cast<const int64_t*>(A + o_ooff);
  a.total_out = P->ooff[n];
  a.Y = P->Y;
  a.Ylo = P->ylo_off >= 0 ? P->Y + P->ylo_off : nullptr;
  a.work = P->work;
  a.grid_tile = std::max(1, std::min<int>((int)std::max(tiles.size(), all_tiles.size()), n_cu * per_cu));
  a.grid_reduce = (int)std::max<int64_t>(1, std::min<int64_t>((a.total_out + 255) / 256, (int64_t)n_cu * 8));
  a.tile_lds = tile_lds;
  a.mob_lds = mob_lds;
  a.partial = P->partial;
  a.n_generic = n_generic;
  a.wide_items = reinterpret_cast<const WideItem*>(A + o_witems);
  a.n_wide_items = (int)witems.size();
  a.grid_wide = std::max(1, std::min<int>((int)witems.size(), n_cu * 4));
  a.wide_groups = reinterpret_cast<const WideGroup*>(A + o_wgroups);
  a.n_wide_groups = (int)wgroups.size();
  a.grid_wide_groups = std::max(1, std::min<int>((int)wgroups.size() * (kWideOuts / 256), n_cu * 4));
  a.wide_partial = P->wide_partial;
  a.red_chunks = reinterpret_cast<const int2*>(A + o_red);
  a.n_red_chunks = (int)red_chunks.size();
  a.red_rows = red_rows;
  a.grid_red_chunks = std::max(1, std::min<int>((int)red_chunks.size(), n_cu * 8));
  a.fast = FastLaunch{};
  a.fast.n_items = (int)fitems.size();
  if (!fitems.empty()) {
    e = configure_fast(prec, fast_lds);
    if (e != hipSuccess) { return fail(FSI_ERR_HIP, std::string("configure_fast: ") + hipGetErrorString(e)); }
    a.fast.prec = prec;
    a.fast.classes = reinterpret_cast<const FastClassDev*>(A + o_fcls);
    a.fast.insts = a.insts;
    a.fast.items = reinterpret_cast<const FastItem*>(A + o_fitems);
    a.fast.torder = reinterpret_cast<const int32_t*>(A + o_torder);
    a.fast.partial = P->partial;
    a.fast.queue = reinterpret_cast<uint32_t*>(A + o_queue);
    for (int l = 0; l <= kFastMaxL + 1; ++l) a.fast.lbeg[l] = lbeg[l];
    a.fast.mobius_in = 0;
    for (const FastClassHost& F : P->fclasses)
      if (F.mobius_in) a.fast.mobius_in = 1;
    int wgs = 1;
    a.fast.lds_mixed = 0;
    for (int l = 0; l <= kFastMaxL; ++l) {
      a.fast.lds[l] = fast_lds[l];
      const int nl = l >= 1 ? lbeg[l + 1] - lbeg[l] : 0;
      a.fast.grid[l] = nl > 0 ? std::max(1, std::min(nl, n_cu * fast_wgs_per_cu(prec, l))) : 0;
      if (nl > 0) {
        wgs = std::max(wgs, fast_wgs_per_cu(prec, l));
        a.fast.lds_mixed = std::max(a.fast.lds_mixed, fast_lds[l]);
      }
    }
    a.fast.grid_mixed = std::max(1, std::min((int)fitems.size(), n_cu * wgs));
  }
  P->sched.autotuned = 0;
  P->sched.fast_instances = 0;
  for (int i = 0; i < n; ++i) P->sched.fast_instances += insts[i].fast;
  P->sched.tiles_per_item = fitems.empty() ? 0 : (int)chunk;
  P->sched.tile_shift = sc.tb_shift;
  P->sched.mob_group = algo == ALGO_TWO_PASS ? (sc.mob_group > 0 ? sc.mob_group : 6) : 0;
  P->sched.tuned_ms = 0.f;
  P->partial_bytes = (size_t)ptot * sizeof(double);
  P->y_bytes = (size_t)ywords * sizeof(double);
  P->wide_bytes = (size_t)wptot * sizeof(double);
  P->work_bytes = (algo == ALGO_TWO_PASS && !P->in_place)
                      ? (size_t)wtot * std::max(mob_elem_bytes(prec), (size_t)8)
                      : 0;
  e = hipEventCreateWithFlags(&P->done, hipEventDisableTiming);
  if (e != hipSuccess) { P->done = nullptr; return fail(FSI_ERR_HIP, "hipEventCreate failed"); }
  guard.p = nullptr;
  *out = P;
  return FSI_OK;
}

// ---------------------------------------------------------------- autotuner
// With fsi_plan_opts.autotune = 1 the plan is built for each candidate
// schedule, each candidate is timed on zero-filled device buffers of the
// plan's size (the kernels' work does not depend on the values), and the
// fastest is kept. Results are cached per (device architecture and compute
// units, dtype, precision, algo, kernel, tile_bits, input, multiset of
// (d, l)): in the process, and in a JSON file that later processes read
// (the path in FSI_TUNE_CACHE, an empty value for none; by default
// $HOME/.cache/fsi_mi355x/autotune.json). The file is an optimisation
// only: a missing, unreadable or unwritable file changes nothing else.
std::mutex g_tune_mu;
std::map<std::string, Sched>& tune_cache() {
  static std::map<std::string, Sched> m;
  return m;
}

std::string tune_file_path() {
  const char* env = std::getenv("FSI_TUNE_CACHE");
  if (env) return std::string(env);
  const char* home = std::getenv("HOME");
  if (!home || !*home) return "";
  return std::string(home) + "/.cache/fsi_mi355x/autotune.json";
}

// One entry per line:
//   {"key": "...", "kernel": K, "tb_shift": T, "chunk_shift": C, "mob_group": G, "algo": A},
// (entries without "algo" read as A = 0, the option's algorithm)
// inside {"format": "fsi-autotune-1", "entries": [ ... ]}. Keys hold only
// [0-9a-z/;,x-], so no escapes are needed; lines that do not parse are
// skipped.
void tune_file_load(std::map<std::string, Sched>& m) {
  const std::string path = tune_file_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[4096];
  while (std::fgets(line, sizeof line, f)) {
    const char* k = std::strstr(line, "\"key\": \"");
    if (!k) continue;
    k += 8;
    const char* ke = std::strchr(k, '"');
    if (!ke) continue;
    Sched sc;
    const int got = std::sscanf(
        ke + 1, ", \"kernel\": %d, \"tb_shift\": %d, \"chunk_shift\": %d, \"mob_group\": %d, \"algo\": %d",
        &sc.kernel, &sc.tb_shift, &sc.chunk_shift, &sc.mob_group, &sc.algo);
    if (got != 4 && got != 5) continue;
    if (got == 4) sc.algo = 0;
    if (sc.algo != 0 && sc.algo != FSI_ALGO_FUSED && sc.algo != FSI_ALGO_TWO_PASS) continue;
    m.emplace(std::string(k, ke), sc);
  }
  std::fclose(f);
}

void tune_file_save(const std::map<std::string, Sched>& m) {
  const std::string path = tune_file_path();
  if (path.empty()) return;
  // create the default directory (two levels below $HOME) if needed
  for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1))
    (void)mkdir(path.substr(0, p).c_str(), 0755);
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  bool ok = std::fprintf(f, "{\"format\": \"fsi-autotune-1\", \"entries\": [\n") > 0;
  size_t i = 0;
  for (const auto& e : m) {
    ok = ok && std::fprintf(f,
                            "{\"key\": \"%s\", \"kernel\": %d, \"tb_shift\": %d, "
                            "\"chunk_shift\": %d, \"mob_group\": %d, \"algo\": %d}%s\n",
                            e.first.c_str(), e.second.kernel, e.second.tb_shift,
                            e.second.chunk_shift, e.second.mob_group, e.second.algo,
                            ++i < m.size() ? "," : "") > 0;
  }
  ok = ok && std::fprintf(f, "]}\n") > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) (void)std::remove(tmp.c_str());
}

std::string tune_key(int n, const int* dh, const int* lh, const fsi_plan_opts& o) {
  std::map<std::pair<int, int>, int> cnt;
  for (int i = 0; i < n; ++i) ++cnt[{dh[i], lh[i]}];
  std::string k = std::to_string(o.dtype) + "/" + std::to_string(o.precision) + "/" +
                  std::to_string(o.algo) + "/" + std::to_string(o.kernel) + "/" +
                  std::to_string(o.tile_bits) + "/" + std::to_string(o.input);
  for (auto& e : cnt)
    k += ";" + std::to_string(e.first.first) + "," + std::to_string(e.first.second) + "x" +
         std::to_string(e.second);
  return k;
}

// Launch arguments of one apply on the given buffers (an in-place two-pass
// plan runs its Moebius passes on the input buffer).
LaunchArgs apply_args(const fsi_batch_plan_s* P, const void* values, void* out) {
  LaunchArgs a = P->args;
  a.values = values;
  a.out = out;
  if (P->in_place) a.work = const_cast<void*>(values);
  return a;
}

// Median device time of launch_apply over a few runs, in ms (< 0 on error).
float time_plan(fsi_batch_plan_s* P, void* vin, void* vout, hipStream_t st) {
  LaunchArgs a = apply_args(P, vin, vout);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1.f; }
  std::vector<float> t;
  bool ok = true;
  for (int r = 0; r < 7 && ok; ++r) {
    ok = hipEventRecord(e0, st) == hipSuccess && launch_apply(a, st) == hipSuccess &&
         hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && r >= 2) t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok || t.empty()) return -1.f;
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

fsi_status build_tuned(int n, const int* dh, const int* lh, const fsi_plan_opts* opts_in,
                       bool single, fsi_batch_plan_s** out) {
  fsi_plan_opts opts;
  fsi_default_opts(&opts);
  if (opts_in) opts = *opts_in;
  if (!opts.autotune) return build_batch(n, dh, lh, opts_in, single, out);
  if (n < 1 || !dh || !lh) return build_batch(n, dh, lh, opts_in, single, out);
  std::string key = tune_key(n, dh, lh, opts);
  {
    int dev = 0, ncu = 0;
    std::string why;
    // without a gfx950 device the plain build reports why
    if (!device_is_gfx950(&dev, &ncu, &why)) return build_batch(n, dh, lh, opts_in, single, out);
    key = "gfx950-" + std::to_string(ncu) + "cu/" + key;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    static bool loaded = false;
    if (!loaded) {
      loaded = true;
      tune_file_load(tune_cache());
    }
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      fsi_status st = build_batch(n, dh, lh, opts_in, single, out, it->second);
      if (st == FSI_OK) (*out)->sched.autotuned = 1;
      return st;
    }
  }
  // candidates
  std::vector<Sched> cand;
  // FSI_ALGO_AUTO times both algorithms when no instance can take the
  // register-phase kernel (every order above 4, value input, no kernel
  // named); otherwise the algorithm it resolves to without the autotuner
  bool all_generic = opts.input == FSI_INPUT_VALUES && opts.kernel == FSI_KERNEL_AUTO;
  for (int i = 0; i < n && all_generic; ++i) all_generic = lh[i] > kFastMaxL;
  const bool both = opts.algo == FSI_ALGO_AUTO && all_generic;
  const int fused_algo = both ? FSI_ALGO_FUSED : 0;
  const bool fused = opts.algo == FSI_ALGO_FUSED || (opts.algo == FSI_ALGO_AUTO &&
                                                     (both || auto_algo(n, lh, opts) == ALGO_FUSED));
  const bool two_pass = opts.algo == FSI_ALGO_TWO_PASS || both ||
                        (opts.algo == FSI_ALGO_AUTO && auto_algo(n, lh, opts) == ALGO_TWO_PASS);
  if (fused) {
    if (opts.kernel != FSI_KERNEL_GENERIC)
      for (int cs = -1; cs <= 2; ++cs) {
        Sched s; s.kernel = opts.kernel; s.chunk_shift = cs; s.algo = fused_algo; cand.push_back(s);
      }
    if (opts.kernel != FSI_KERNEL_REGISTER)
      for (int tb = 0; tb >= (opts.tile_bits ? 0 : -2); --tb) {
        Sched s; s.kernel = FSI_KERNEL_GENERIC; s.tb_shift = tb; s.algo = fused_algo; cand.push_back(s);
      }
  }
  if (two_pass) {
    for (int g = 4; g <= 6; ++g)
      for (int tb = 0; tb >= (opts.tile_bits ? 0 : -1); --tb) {
        Sched s; s.mob_group = g; s.tb_shift = tb; s.algo = both ? FSI_ALGO_TWO_PASS : 0;
        cand.push_back(s);
      }
  }
  fsi_batch_plan_s* best = nullptr;
  float best_ms = 0.f;
  Sched best_s;
  fsi_status first_err = FSI_OK;
  std::string first_msg;
  void* vin = nullptr;
  void* vout = nullptr;
  hipStream_t st = nullptr;
  for (const Sched& sc : cand) {
    fsi_batch_plan_s* P = nullptr;
    fsi_status s = build_batch(n, dh, lh, opts_in, single, &P, sc);
    if (s != FSI_OK) {
      if (first_err == FSI_OK) { first_err = s; first_msg = g_err; }
      continue;
    }
    if (!st) {
      const size_t elem = opts.dtype == FSI_DTYPE_F64 ? 8 : 4;
      const size_t nin = (size_t)P->voff[n] * elem, nout = (size_t)P->ooff[n] * elem;
      if (hipMalloc(&vin, nin) != hipSuccess || hipMalloc(&vout, nout) != hipSuccess ||
          hipMemset(vin, 0, nin) != hipSuccess ||
          hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        free_batch(P);
        if (vin) (void)hipFree(vin);
        if (vout) (void)hipFree(vout);
        return fail(FSI_ERR_OUT_OF_MEMORY, "autotune: scratch buffers");
      }
    }
    const float ms = time_plan(P, vin, vout, st);
    if (ms >= 0.f && (!best || ms < best_ms)) {
      if (best) free_batch(best);
      best = P; best_ms = ms; best_s = sc;
    } else {
      free_batch(P);
    }
  }
  if (st) (void)hipStreamDestroy(st);
  if (vin) (void)hipFree(vin);
  if (vout) (void)hipFree(vout);
  if (!best) {
    if (first_err != FSI_OK) { g_err = first_msg; return first_err; }
    return fail(FSI_ERR_INTERNAL, "autotune: no candidate could be timed");
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache()[key] = best_s;
    tune_file_save(tune_cache());
  }
  best->sched.autotuned = 1;
  best->sched.tuned_ms = best_ms;
  *out = best;
  return FSI_OK;
}

}  // namespace

// ------------------------------------------------ no-allocation scratch
// Device scratch of fsi_apply_batched_noalloc: a fixed-size array in the
// library's code object, one copy per GPU the library runs on (held until
// the process ends). In host code the array's name is only a host-side
// stand-in: its device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is passed to
// kernels. Every no-allocation apply on a GPU carves its workspaces from the
// same array, so such calls that overlap on one GPU race; the array keeps
// the last call's contents (no kernel of an apply reads a workspace word
// before the same apply has written it, so nothing needs clearing).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchMaxDevices] = {};

// Device address of this device's scratch array (current device = dev).
fsi_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kScratchMaxDevices)
    return fail(FSI_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FSI_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return FSI_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t scratch_need(const fsi_batch_plan_s* P) {
  return align256(P->partial_bytes) + align256(P->y_bytes) + align256(P->wide_bytes) +
         align256(P->work_bytes);
}

// Marks the plan's work on `stream` as issued: destroying the plan waits
// for this event. Not recorded while the stream is being captured (the
// caller's graph then owns the ordering).
void mark_done(fsi_batch_plan_s* P, hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
    (void)hipEventRecord(P->done, stream);
}

fsi_status check_ptr(const void* p, const char* what) {
  if (!p) return fail(FSI_ERR_INVALID_ARG, std::string(what) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) & 15)
    return fail(FSI_ERR_INVALID_ARG, std::string(what) + " is not 16-byte aligned");
  return FSI_OK;
}

}  // namespace

extern "C" {

fsi_status fsi_default_opts(fsi_plan_opts* opts) {
  if (!opts) return fail(FSI_ERR_INVALID_ARG, "opts is NULL");
  std::memset(opts, 0, sizeof(*opts));
  opts->dtype = FSI_DTYPE_F64;
  opts->precision = FSI_PREC_AUTO;
  opts->algo = FSI_ALGO_AUTO;
  return FSI_OK;
}

int64_t fsi_num_outputs(int d, int l) { return num_outputs(d, l); }

fsi_status fsi_plan(int d, int l, fsi_plan_t* out) { return fsi_plan_ex(d, l, nullptr, out); }

fsi_status fsi_plan_ex(int d, int l, const fsi_plan_opts* opts, fsi_plan_t* out) {
  FSI_ABI_TRY
  if (!out) return fail(FSI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!(1 <= d && d <= kMaxD && 1 <= l && l <= d))
    return fail(FSI_ERR_INVALID_ARG, "need 1 <= l <= d <= 30");
  fsi_batch_plan_s* bp = nullptr;
  fsi_status st = build_tuned(1, &d, &l, opts, true, &bp);
  if (st != FSI_OK) return st;
  auto* p = new (std::nothrow) fsi_plan_s();
  if (!p) { free_batch(bp); return fail(FSI_ERR_OUT_OF_MEMORY, "host allocation failed"); }
  p->bp = bp; p->d = d; p->l = l;
  *out = p;
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_plan_destroy(fsi_plan_t plan) {
  FSI_ABI_TRY
  if (!plan) return FSI_OK;
  free_batch(plan->bp);
  delete plan;
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_output_masks(fsi_plan_t plan, uint32_t* host_masks) {
  if (!plan || !host_masks) return fail(FSI_ERR_INVALID_ARG, "null plan or output");
  const ClassHost& C = plan->bp->classes[0];
  std::memcpy(host_masks, C.out_masks.data(), C.out_masks.size() * sizeof(uint32_t));
  return FSI_OK;
}

fsi_status fsi_plan_info(fsi_plan_t plan, int* tile_bits, int* block_threads, int* algo,
                         int* precision) {
  if (!plan) return fail(FSI_ERR_INVALID_ARG, "null plan");
  const bool fast = plan->bp->sched.fast_instances > 0;
  if (tile_bits) *tile_bits = plan->bp->classes[0].b;
  if (block_threads) *block_threads = fast ? kFastThreads : kTileThreads;
  if (algo) *algo = plan->bp->algo;
  if (precision) *precision = plan->bp->prec;
  return FSI_OK;
}

fsi_status fsi_apply(fsi_plan_t plan, const void* v_dev, void* out_dev, hipStream_t stream) {
  FSI_ABI_TRY
  if (!plan) return fail(FSI_ERR_INVALID_ARG, "null plan");
  fsi_status st;
  if ((st = check_ptr(v_dev, "v_dev")) != FSI_OK) return st;
  if ((st = check_ptr(out_dev, "out_dev")) != FSI_OK) return st;
  LaunchArgs a = apply_args(plan->bp, v_dev, out_dev);
  HIP_TRY(launch_apply(a, stream));
  mark_done(plan->bp, stream);
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_mobius(fsi_plan_t plan, void* a_dev, hipStream_t stream) {
  FSI_ABI_TRY
  if (!plan) return fail(FSI_ERR_INVALID_ARG, "null plan");
  fsi_status st;
  if ((st = check_ptr(a_dev, "a_dev")) != FSI_OK) return st;
  LaunchArgs a = plan->bp->args;
  a.work = a_dev;
  a.prec = plan->bp->dtype == FSI_DTYPE_F64 ? PREC_F64 : PREC_F32;
  HIP_TRY(launch_mobius(a, stream));
  mark_done(plan->bp, stream);
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_plan_batched(int n, const int* d_host, const int* l_host,
                            const fsi_plan_opts* opts, fsi_batch_plan_t* out) {
  FSI_ABI_TRY
  if (!out) return fail(FSI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  fsi_batch_plan_s* bp = nullptr;
  fsi_status st = build_tuned(n, d_host, l_host, opts, false, &bp);
  if (st != FSI_OK) return st;
  *out = bp;
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_batch_plan_destroy(fsi_batch_plan_t plan) {
  FSI_ABI_TRY
  free_batch(plan);
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_batch_offsets(fsi_batch_plan_t plan, int64_t* value_offset, int64_t* out_offset) {
  if (!plan) return fail(FSI_ERR_INVALID_ARG, "null plan");
  if (value_offset) std::memcpy(value_offset, plan->voff.data(), (plan->n + 1) * sizeof(int64_t));
  if (out_offset) std::memcpy(out_offset, plan->ooff.data(), (plan->n + 1) * sizeof(int64_t));
  return FSI_OK;
}

fsi_status fsi_apply_batched_nograph(fsi_batch_plan_t plan, const void* values_dev,
                                     void* out_dev, hipStream_t stream) {
  FSI_ABI_TRY
  if (!plan) return fail(FSI_ERR_INVALID_ARG, "null plan");
  fsi_status st;
  if ((st = check_ptr(values_dev, "values_dev")) != FSI_OK) return st;
  if ((st = check_ptr(out_dev, "out_dev")) != FSI_OK) return st;
  LaunchArgs a = apply_args(plan, values_dev, out_dev);
  HIP_TRY(launch_apply(a, stream));
  mark_done(plan, stream);
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_apply_batched_noalloc(fsi_batch_plan_t plan, const void* values_dev,
                                     void* out_dev, hipStream_t stream) {
  FSI_ABI_TRY
  if (!plan) return fail(FSI_ERR_INVALID_ARG, "null plan");
  fsi_status st;
  if ((st = check_ptr(values_dev, "values_dev")) != FSI_OK) return st;
  if ((st = check_ptr(out_dev, "out_dev")) != FSI_OK) return st;
  const size_t need = scratch_need(plan);
  if (need > kScratchBytes)
    return fail(FSI_ERR_INVALID_ARG,
                "the plan's workspaces need " + std::to_string(need) +
                    " bytes; the no-allocation scratch holds " + std::to_string(kScratchBytes));
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != plan->device)
    return fail(FSI_ERR_INVALID_ARG, "the current HIP device is not the plan's device");
  unsigned char* base = nullptr;
  if ((st = scratch_address(dev, &base)) != FSI_OK) return st;
  LaunchArgs a = apply_args(plan, values_dev, out_dev);
  size_t off = 0;
  double* part = plan->partial_bytes ? reinterpret_cast<double*>(base + off) : nullptr;
  a.partial = part;
  a.fast.partial = part;
  off += align256(plan->partial_bytes);
  a.Y = reinterpret_cast<double*>(base + off);
  a.Ylo = plan->ylo_off >= 0 ? a.Y + plan->ylo_off : nullptr;
  off += align256(plan->y_bytes);
  a.wide_partial = plan->wide_bytes ? reinterpret_cast<double*>(base + off) : nullptr;
  off += align256(plan->wide_bytes);
  if (plan->work_bytes) a.work = base + off;
  HIP_TRY(launch_apply(a, stream));
  mark_done(plan, stream);
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_apply_batched(fsi_batch_plan_t plan, const void* values_dev, void* out_dev,
                             hipStream_t stream) {
  FSI_ABI_TRY
  if (!plan) return fail(FSI_ERR_INVALID_ARG, "null plan");
  fsi_status st;
  if ((st = check_ptr(values_dev, "values_dev")) != FSI_OK) return st;
  if ((st = check_ptr(out_dev, "out_dev")) != FSI_OK) return st;
  if (!plan->exec || plan->g_in != values_dev || plan->g_out != out_dev) {
    if (!plan->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
    LaunchArgs a = apply_args(plan, values_dev, out_dev);
    HIP_TRY(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_apply(a, plan->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(plan->cap_stream, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(FSI_ERR_HIP, std::string("launch during capture: ") + hipGetErrorString(le));
    }
    if (ce != hipSuccess) return fail(FSI_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    // the launch sequence does not depend on the pointers: a new pointer
    // pair updates the kernel arguments of the instantiated graph in place
    // (re-instantiated only if the update is refused)
    bool updated = false;
    if (plan->exec) {
      hipGraphExecUpdateResult ur = hipGraphExecUpdateError;
      hipGraphNode_t bad = nullptr;
      updated = hipGraphExecUpdate(plan->exec, g, &bad, &ur) == hipSuccess &&
                ur == hipGraphExecUpdateSuccess;
      if (!updated) {
        (void)hipGetLastError();
        HIP_TRY(hipGraphExecDestroy(plan->exec));
        plan->exec = nullptr;
      }
    }
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->graph = g;
    if (!updated) HIP_TRY(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
    plan->g_in = values_dev;
    plan->g_out = out_dev;
  }
  HIP_TRY(hipGraphLaunch(plan->exec, stream));
  mark_done(plan, stream);
  return FSI_OK;
  FSI_ABI_CATCH
}

int fsi_batch_num_stages(fsi_batch_plan_t plan) {
  if (!plan) { fail(FSI_ERR_INVALID_ARG, "null plan"); return -1; }
  return num_stages(plan->args);
}

fsi_status fsi_apply_batched_stage(fsi_batch_plan_t plan, const void* values_dev, void* out_dev,
                                   int stage, hipStream_t stream) {
  FSI_ABI_TRY
  if (!plan) return fail(FSI_ERR_INVALID_ARG, "null plan");
  fsi_status st;
  if ((st = check_ptr(values_dev, "values_dev")) != FSI_OK) return st;
  if ((st = check_ptr(out_dev, "out_dev")) != FSI_OK) return st;
  if (stage < 0 || stage >= num_stages(plan->args))
    return fail(FSI_ERR_INVALID_ARG, "stage out of range");
  LaunchArgs a = apply_args(plan, values_dev, out_dev);
  HIP_TRY(launch_stage(a, stage, stream));
  mark_done(plan, stream);
  return FSI_OK;
  FSI_ABI_CATCH
}

fsi_status fsi_batch_schedule(fsi_batch_plan_t plan, fsi_schedule* out) {
  if (!plan || !out) return fail(FSI_ERR_INVALID_ARG, "null plan or output");
  *out = plan->sched;
  return FSI_OK;
}

fsi_status fsi_plan_schedule(fsi_plan_t plan, fsi_schedule* out) {
  if (!plan || !out) return fail(FSI_ERR_INVALID_ARG, "null plan or output");
  *out = plan->bp->sched;
  return FSI_OK;
}

const char* fsi_last_error(void) { return g_err.c_str(); }

}  // extern "C"
