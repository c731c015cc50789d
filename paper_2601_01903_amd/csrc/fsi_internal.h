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
  const int32_t* lam_soff;  // [l+1] offset of the s_L block inside a u block
  const uint32_t* oinfo;    // [M] Y offset of S_L | s_H << 24
  const uint32_t* osh;      // [M] S_H (mask over the h high bits)
};

// Tables of the register-phase tile kernel (fsi_tile11.hip): tiles of 11
// low bits, l <= 4. The in-tile layouts are compile-time functions of l; the
// tables here hold what depends on d (weights, output metadata) and the
// per-thread unit maps of the sweep phases.
// Outputs are held by the kernel in slots: thread t owns the outputs
// (kk, t), kk = 0 .. nkk-1; slot kk holds outputs of one |S_L| only, so the
// stride between the j-variants of its partial results is uniform.
struct FastClassDev {
  int32_t d, l, h, M;
  int32_t nkk;                // slots per thread in use (largest over the output groups)
  int32_t mshift;             // bits of the Y byte offset in a metadata word
  int32_t pad0, pad1;
  const double* lam;          // [(h+1) * lamblock(l)] final-core weights per high popcount
  const uint32_t* meta;       // [groups * 256 * kFastMetaStride] per group and thread:
                              // Y byte offset | S_H << mshift
  const uint32_t* gs8;        // [groups * kFastMetaStride] byte stride between j-variants per slot
  const int32_t* gnkk;        // [groups] slots per thread in use in each output group
  const int32_t* unit_mask;   // [n3(l)] sigma_A | sigma_B << 4 of a phase-C unit
  const int32_t* zrow;        // [n3(l) * 8] Z row of (unit, sigma_C)
  const int32_t* uperm;       // [256] phase-C unit of thread t, -1 for none (heavy units on two lanes)
};

struct FastClassHost {
  int d = 0, l = 0, h = 0, M = 0, nkk = 0, mshift = 16, ngroups = 1, mobius_in = 0;
  std::vector<double> lam;
  std::vector<uint32_t> meta, gs8;
  std::vector<int32_t> gnkk;
  std::vector<int32_t> unit_mask, zrow, uperm;
  std::vector<int32_t> pidx;    // [M] slot index kk * 256 + t of canonical output k in its group
  std::vector<int32_t> pgroup;  // [M] output group of canonical output k
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
  int32_t wide;      // 1: generic instance reduced by the wide gather
  const int32_t* pidx;  // [M] position of canonical output k in an item's partial sums
};

// Host-side tables of one class (built once, uploaded into a device arena).
struct ClassHost {
  int d = 0, l = 0, b = 0, h = 0, algo = ALGO_FUSED, mobius_in = 0;
  int M = 0, Ysize = 0, lam_ublock = 0, lds_elems = 0, nfinal = 0;
  std::vector<int32_t> step_off, step_np;
  std::vector<uint32_t> pat, ytab, oinfo, osh, out_masks;
  std::vector<double> lam;
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
// Output slots per thread the register-phase kernel needs for (d, l), or -1.
int fast_output_slots(int d, int l);
// Most high bits (d - 11) the register-phase kernel's output metadata holds at order l.
int fast_max_high_bits(int l);
// Builds the register-phase kernel tables from an already built fused class
// with b = 11 and l <= 4 (its final weights and output order).
std::string build_fast_class(const ClassHost& C, FastClassHost* out);

}  // namespace fsi
