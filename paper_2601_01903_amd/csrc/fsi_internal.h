// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace fsi {

constexpr int kMaxD = 30;
constexpr int kMaxTileBits = 12;   // LDS-staged tile: 2^b values
constexpr int kLdsBudget = 150 * 1024;

enum Algo : int32_t { ALGO_FUSED = 1, ALGO_TWO_PASS = 2 };
enum Prec : int32_t {
  PREC_F64 = 0, PREC_F32 = 1, PREC_F32_COMP = 2, PREC_F32_FP64MOB = 3,
  PREC_F32_FP64REG = 4
};

// Per (d, l, b, algo) tables, as seen by the kernels (device pointers).
struct ClassDev {
  int32_t d, l, b, h, algo;
  int32_t M;            // outputs per instance
  int32_t Ysize;        // per-tile partial results (doubles)
  int32_t lam_ublock;   // doubles per high-popcount block of the weight table
  int32_t lds_elems;    // largest sweep state (entries) of one step
  int32_t nfinal;       // final patterns (S_L, t_L)
  int32_t mobius_in;    // 1: the input is already the Moebius transform
  int32_t pad0;
  const int32_t* step_off;  // [b+1] start of step k's entries in pat
  const int32_t* step_np;   // [b+1] number of patterns after step k
  const uint32_t* pat;      // (src0+1) | (src1+1) << 16 per output pattern
  const uint32_t* ytab;     // [Ysize] final-pattern base | slot << 16 | s_L << 26
  const double* lam;        // [(h+1) * lam_ublock]
  const double* lam_lo;     // two-pass: [(h+1) * lam_ublock] low words of the weights, else null
  const int32_t* lam_soff;  // [l+1] offset of the s_L block inside a u block
  const uint32_t* oinfo;    // [M] Y offset of S_L | s_H << 24
  const uint32_t* osh;      // [M] S_H (mask over the h high bits)
};

// Tables of the register-phase tile kernel (fsi_tile11.hip): tiles of 11
// low bits, l <= 4. The in-tile layouts are compile-time functions of l; the
// tables here hold what depends on d (weights, output metadata) and the
// per-thread unit maps of the sweep phases.
// Partial sums are held by the kernel in slots: thread t owns the slots
// (kk, t), kk = 0 .. nkk-1; slot kk holds sums of one |S_L| only, so the
// stride between the j-variants of its per-tile results is uniform. An
// instance whose outputs all fit the slots is one block (kb = h: a slot sums
// an output); otherwise a work item covers a block of 2^kb tiles and its
// slots hold the block's partial sums over (S_L, S_H1, s_H2, j2), from which
// the reduction picks j2 = |S_H2 & block| per output.
struct FastClassDev {
  int32_t d, l, h, M;
  int32_t nkk;                // slots per thread in use
  int32_t mshift;             // bits of the Y byte offset in a metadata word
  int32_t kb, pad1;           // low high bits per block (h: the whole instance)
  const double* lam;          // [(h+1) * lamblock(l)] final-core weights per high popcount
  const uint32_t* meta;       // [256 * kFastMetaStride] per thread and position:
                              // Y byte offset | S_H (blocked: S_H1) << mshift
  const uint32_t* gs8;        // [kFastRuns * 4] byte stride between j-variants per position and wave
  const int32_t* unit_mask;   // [n3(l)] sigma_A | sigma_B << 4 of a phase-C unit
  const int32_t* zrow;        // [n3(l) * 8] Z row of (unit, sigma_C)
  const int32_t* uperm;       // [256] phase-C unit of thread t, -1 for none (heavy units on two lanes)
};

struct FastClassHost {
  int d = 0, l = 0, h = 0, M = 0, nkk = 0, mshift = 16, kb = 0, mobius_in = 0;
  std::vector<double> lam;
  std::vector<uint32_t> meta, gs8;
  std::vector<int32_t> unit_mask, zrow, uperm;
  // [M * (l + 1)] slot index kk * 256 + t of canonical output k's partial
  // sum for j2 = 0 .. l (whole instances: every entry the j2 = 0 slot)
  std::vector<int32_t> pidx;
  std::vector<uint32_t> osh2;   // [M] S_H2 = S_H >> kb of canonical output k
  // [nkk * 256] canonical output of slot kk * 256 + t for one-block classes
  // (its j2 = 0 slot), -1 for an unused slot; empty for blocked classes
  std::vector<int32_t> sinv;
};

struct InstDev {
  int32_t cls;       // index into the class array
  int32_t d;
  int64_t voff;      // first value
  int64_t ooff;      // first output
  int64_t yoff;      // first partial result (doubles) in the Y workspace
  int64_t woff;      // first element of the Moebius workspace (two-pass)
  int32_t fast;      // 1: handled by the register-phase kernel
  int32_t nitems;    // its work items (partial sums at pbase + j * pstride)
  int32_t tofs;      // first entry of its class's tile order
  int32_t fcls;      // index into the register-phase class array
  int64_t pbase;     // first partial sum (doubles)
  int32_t pstride;   // partial sums per work item
  int32_t wide;      // 1: reduced by the wide gather (generic instances with
                     // many tiles, register-phase instances of several blocks)
  int32_t pw;        // row width of pidx (l + 1)
  int32_t ipb;       // work items per block (item j covers block j / ipb)
  int32_t lowmask;   // register-phase kernel: 2^d - 1 for d < 11 (the tile's
                     // value U is v(U & lowmask)), else 2^11 - 1
  int32_t pad2;
  const int32_t* pidx;   // [M * pw] position of canonical output k's partial sum for j2
  const uint32_t* osh2;  // [M] S_H2 of canonical output k
  const int32_t* sinv;   // [pstride] canonical output whose partial sum a slot holds
                         // (one-block instances), -1 for an unused slot
};

// Host-side tables of one class (built once, uploaded into a device arena).
struct ClassHost {
  int d = 0, l = 0, b = 0, h = 0, algo = ALGO_FUSED, mobius_in = 0;
  int M = 0, Ysize = 0, lam_ublock = 0, lds_elems = 0, nfinal = 0;
  std::vector<int32_t> step_off, step_np;
  std::vector<uint32_t> pat, ytab, oinfo, osh, out_masks;
  std::vector<double> lam, lam_lo;
  std::vector<int32_t> lam_soff;
};

int64_t num_outputs(int d, int l);
std::vector<uint32_t> canonical_masks(int d, int l);
// Message behind fsi_last_error() (thread-local), for entry points outside
// the main C-ABI source.
void record_error(const std::string& msg);
// True if the current HIP device is a gfx950; else *why says what it is.
bool gfx950_device(int* dev, int* n_cu, std::string* why);
// Exact W(s, t) of the operator, rounded once to double (see fsi_tables.cpp).
double weight_full(int s, int t, int l, int index);
// Largest sweep state of an in-tile sweep over b bits, in entries.
int64_t sweep_peak_entries(int b, int l);
// Builds all tables for one class; returns "" or an error message.
std::string build_class(int d, int l, int b, int algo, int index, int mobius_in, ClassHost* out);
// Low high bits per block of the register-phase kernel for (d, l): h = d - 11
// when every output fits the workgroup's slots, else the most that fit; -1
// when the kernel does not apply.
int fast_block_bits(int d, int l);
// Slots per thread the register-phase kernel uses for (d, l), or -1.
int fast_output_slots(int d, int l);
// Builds the register-phase kernel tables from an already built fused class
// with b = 11 and l <= 4 (its final weights and output order).
std::string build_fast_class(const ClassHost& C, FastClassHost* out);

}  // namespace fsi
