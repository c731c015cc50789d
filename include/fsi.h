/*
 * fsi.h - C ABI of the MI355X (gfx950) Faithful Shapley Interaction operator.
 *
 * The operator maps a value vector v over all 2^d coalitions of d players to
 * the FSI scores E_S of every coalition S with |S| <= l (paper: "TT-FSI:
 * Scalable Faithful Shapley Interactions via Tensor-Train"):
 *
 *   E_S = a(S) + sum_{T superset of S, |T| > l} w(|S|, |T|) a(T)
 *
 * with a the Moebius transform of v (Sec. 2.2, Eq. 3 and Eq. 4; Sec. 4.1,
 * Eq. 5) and w the cardinality-only weight of Sec. 4.3, Eq. 7. The GPU
 * computes it as a Moebius butterfly (Sec. 4.2, the Moebius transform as a
 * rank-1 MPO; Appendix B) followed by the left-to-right MPO sweep over
 * (|S|, |T|) counter states (Sec. 4.3 - 4.4, Algorithm 1), with the Moebius
 * cores of the high sites precontracted into the final weight core
 * (Sec. 4.5) in the fused algorithm.
 *
 * Conventions (all entry points):
 *  - v is indexed by a d-bit mask: bit i set <=> player i in the coalition.
 *    v(empty) need not be 0; then E_empty = v(empty).
 *  - Outputs are in canonical order: ascending |S|, then ascending mask value
 *    (slot 0 is the empty set). fsi_output_masks() returns that order.
 *  - Device pointers are caller-owned HIP device memory, 16-byte aligned,
 *    holding elements of the plan's storage dtype (FP64 or FP32). The library
 *    never frees them. Outputs are always written in the storage dtype.
 *  - Calls are asynchronous on the given HIP stream (NULL = default stream).
 *    Bad arguments are rejected on the host before anything is launched and
 *    leave the outputs untouched. HIP faults surface on the next call or on
 *    the caller's synchronization.
 *  - A plan owns its device tables and workspace; it is immutable after
 *    creation. Concurrent applies of ONE plan on different streams race on
 *    its workspace; use one plan per stream.
 *  - No C++ exception crosses this ABI: a failed host allocation returns
 *    FSI_ERR_OUT_OF_MEMORY, any other internal exception FSI_ERR_INTERNAL,
 *    and the partly built object is freed. Every non-OK status sets a
 *    thread-local message readable with fsi_last_error().
 *  - Test hook: with the environment variable FSI_TEST_FAIL_ALLOC=host a
 *    plan's host-table allocation fails (std::bad_alloc, before any device
 *    call), with FSI_TEST_FAIL_ALLOC=device its device workspace allocation
 *    fails; both return FSI_ERR_OUT_OF_MEMORY and free what was built.
 */
#ifndef FSI_MI355X_H
#define FSI_MI355X_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FSI_OK = 0,
  FSI_ERR_INVALID_ARG = 1,   /* a size, pointer, alignment or option is wrong */
  FSI_ERR_UNSUPPORTED = 2,   /* no gfx950 device, or a combination not built */
  FSI_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed */
  FSI_ERR_HIP = 4,           /* a HIP runtime call failed */
  FSI_ERR_INTERNAL = 5
} fsi_status;

typedef enum { FSI_DTYPE_F64 = 0, FSI_DTYPE_F32 = 1 } fsi_dtype;

/* Arithmetic of the path (the storage dtype is fsi_plan_opts.dtype).
 * Correction weights (Eq. 7 and their precontracted forms) and the final
 * cross-tile reduction are FP64 in every mode. */
typedef enum {
  FSI_PREC_F64 = 0,             /* FP64 storage, FP64 everywhere            */
  FSI_PREC_F32 = 1,             /* FP32 Moebius, FP32 sweep accumulation    */
  FSI_PREC_F32_COMPENSATED = 2, /* two-float Moebius, FP32 sweep            */
  FSI_PREC_F32_FP64MOB = 3,     /* FP64 Moebius, FP32 sweep                 */
  FSI_PREC_F32_FP64REG = 4,     /* FP32 storage, FP64 Moebius and sweep     */
  FSI_PREC_AUTO = 5             /* F64 for FP64 storage; F32_FP64MOB for    */
                                /* FP32 storage (on gfx950 an FP64 add      */
                                /* issues at the rate of an unpacked FP32   */
                                /* add, so the FP64 butterfly costs one     */
                                /* instruction per step against about eight */
                                /* for the two-float one, and is at least   */
                                /* as accurate)                             */
} fsi_precision;

typedef enum {
  /* The fused algorithm, except for plans whose instances all have l >= 7
   * (value input, kernel FSI_KERNEL_AUTO): there the two-pass one, whose
   * sweep does not grow with the number of outputs the way the fused gather
   * does. With the autotuner, such a plan whose instances all have l > 4
   * times both. */
  FSI_ALGO_AUTO = 0,
  /* One read of v: per tile of the low b bits, the in-tile Moebius and the
   * counter sweep; the high-site Moebius cores are precontracted into the
   * final weights (Sec. 4.5 applied to the high sites); a small cross-tile
   * reduction finishes. */
  FSI_ALGO_FUSED = 1,
  /* Literal Eq. 5 order: the full Moebius butterfly (low bits in LDS, high
   * bits as strided passes) into the workspace, then the counter sweep with
   * the weights of each tile's known high popcount, then the reduction. */
  FSI_ALGO_TWO_PASS = 2
} fsi_algo;

/* Interaction index computed by a plan. Every index here is linear in v and,
 * on the Moebius transform a, weights each superset T of S by a number that
 * depends only on s = |S| and t = |T| (Appendix A), so all of them run through
 * the same Moebius butterfly, counter sweep and final weight core:
 *
 *   I_S = sum_{T superset of S} W(s, t) a(T),   |S| <= l,
 *
 *   FSI   W = 1 at t = s; w(s, t) of Eq. 7 for t > l, s >= 1; else 0
 *   STII  W = [t = s] for s < l; 1 / C(t, l) for s = l (Shapley-Taylor,
 *         the cited definition: higher-order Moebius mass split evenly over
 *         the top-order subsets)
 *   SII   W = 1 / (t - s + 1)     (Shapley interaction index)
 *   KSII  W = [t = 0] for s = 0; for s >= 1
 *         sum_{j=0}^{min(l-s, t-s)} B_j C(t-s, j) / (t-s-j+1), B_j the
 *         Bernoulli numbers with B_1 = -1/2 (k-Shapley interaction index)
 *   BII   W = 2^-(t - s)          (Banzhaf interaction index)
 *
 * The weights are evaluated in binary128 and rounded once to FP64. */
typedef enum {
  FSI_INDEX_FSI = 0,
  FSI_INDEX_STII = 1,
  FSI_INDEX_SII = 2,
  FSI_INDEX_KSII = 3,
  FSI_INDEX_BII = 4
} fsi_index;

/* What the input buffer holds. FSI_INPUT_MOBIUS: the Moebius transform a
 * of the value vector (a(S) = sum over subsets T of S of (-1)^|S - T| v(T),
 * Sec. 2.2), so the plan applies only the correction of Eq. 3 - 4,
 * I_S = sum_{T superset of S} W(s, |T|) a(T) (the MPO on a, Sec. 4.4; for
 * callers that already hold Moebius coefficients, e.g. fsi_forest_mobius).
 * Needs the fused algorithm (FSI_ALGO_AUTO or FSI_ALGO_FUSED). */
typedef enum { FSI_INPUT_VALUES = 0, FSI_INPUT_MOBIUS = 1 } fsi_input;

typedef struct {
  int32_t dtype;                 /* fsi_dtype, default FSI_DTYPE_F64         */
  int32_t precision;             /* fsi_precision, default FSI_PREC_AUTO     */
  int32_t algo;                  /* fsi_algo, default FSI_ALGO_AUTO          */
  int32_t tile_bits;             /* b, 0 = choose (autotuned if enabled)     */
  int32_t block_threads;         /* reserved, must be 0: each kernel has a   */
                                 /* fixed workgroup size (fsi_plan_info)    */
  int32_t autotune;              /* 1 = time candidate schedules at plan     */
                                 /* time (see fsi_schedule), keep the best   */
  int32_t kernel;                /* fsi_kernel, default FSI_KERNEL_AUTO      */
  int32_t index;                 /* fsi_index, default FSI_INDEX_FSI         */
  int32_t input;                 /* fsi_input, default FSI_INPUT_VALUES      */
  int32_t allow_input_overwrite; /* 0 or 1, default 0; see below            */
} fsi_plan_opts;

/* allow_input_overwrite = 1 lets a two-pass plan (FSI_ALGO_TWO_PASS) run its
 * Moebius butterfly in place on the input buffer instead of a workspace of
 * 2^d elements per instance: no workspace is allocated, and after an apply
 * the input buffer holds the Moebius transform a of v (Sec. 2.2; the same
 * array fsi_mobius writes). It is honoured when the butterfly runs in the
 * storage type (FSI_PREC_F64, FSI_PREC_F32); with a wider butterfly type
 * (compensated, FP64 butterfly or FP64 sweep on FP32 storage) the plan keeps
 * its workspace and leaves the input unmodified. The fused algorithm reads v
 * once, never writes it and needs no such workspace, so it ignores the flag.
 * Values other than 0 and 1 give FSI_ERR_INVALID_ARG. */

/* Tile kernel of the fused algorithm. The register-phase kernel (tiles of
 * 11 low bits) covers every storage dtype and precision except
 * F32_FP64REG, at l <= 4 for every d <= 30: an instance with d < 11 runs as
 * the d = 11 instance of the game that ignores the players past d (its
 * scores on the first d players are the same, the weights not depending on
 * d), and past d = 20 at l = 4 the outputs outnumber a workgroup's
 * accumulators: a work item then covers a block of 2^6 tiles sharing their
 * top high bits, and the wide gather combines the blocks' partial sums;
 * every tile is still read and swept once. The generic LDS kernel covers
 * every (d, l). AUTO picks the register-phase kernel where it applies. */
typedef enum {
  FSI_KERNEL_AUTO = 0,
  FSI_KERNEL_GENERIC = 1,
  FSI_KERNEL_REGISTER = 2   /* FSI_ERR_UNSUPPORTED where it does not apply */
} fsi_kernel;

typedef struct fsi_plan_s* fsi_plan_t;
typedef struct fsi_batch_plan_s* fsi_batch_plan_t;

/* The schedule a plan runs (fsi_plan_schedule / fsi_batch_schedule).
 * With fsi_plan_opts.autotune = 1, plan creation builds the plan for each
 * candidate schedule, times one apply of each on zero-filled scratch
 * buffers of the plan's size (allocated and freed inside the call) on a
 * private stream, and keeps the fastest. Candidates: for the fused
 * algorithm the register-phase kernel at 1/2x, 1x, 2x and 4x the default
 * tiles per work item and the generic kernel at the largest tile that fits
 * LDS and 1 or 2 bits less; for the two-pass algorithm 4, 5 or 6 bits per
 * strided high Moebius pass, with the largest tile or 1 bit less;
 * FSI_ALGO_AUTO takes the candidates of both algorithms when every instance
 * has l > 4, else those of the algorithm it resolves to. The
 * choice is cached per (device architecture and compute-unit count, dtype,
 * precision, algo, kernel, tile_bits, input, multiset of (d, l)) in the
 * process and in a JSON file read by later processes: the path in the
 * environment variable FSI_TUNE_CACHE (empty: no file), by default
 * $HOME/.cache/fsi_mi355x/autotune.json. A plan whose schedule comes from
 * the cache reports autotuned = 1 and tuned_ms = 0. The file only saves
 * plan time: when it is missing, unreadable or unwritable, plans are timed
 * as without it. */
typedef struct {
  int32_t autotuned;        /* 1 if chosen by timing                         */
  int32_t fast_instances;   /* instances on the register-phase kernel       */
  int32_t tiles_per_item;   /* register-phase kernel: tiles per work item   */
  int32_t tile_shift;       /* generic tile: bits below the largest fitting */
  int32_t mob_group;        /* two-pass: bits per strided high pass; 0 for  */
                            /* the fused algorithm                          */
  float tuned_ms;           /* measured time of the chosen schedule (ms)    */
} fsi_schedule;

/* Fill opts with the defaults listed above. */
fsi_status fsi_default_opts(fsi_plan_opts* opts);

/* M(d, l) = sum_{s=0..l} C(d, s): number of outputs, one per coalition S with
 * |S| <= l (the output set of Eq. 3, Sec. 2.2; the empty set counts), or -1
 * if not 1 <= l <= d <= 30. Host only. */
int64_t fsi_num_outputs(int d, int l);

/* Plan for one instance size of the operator of Sec. 4.1, Eq. 5 (Eq. 3 - 4
 * with the weights of Eq. 7, Sec. 4.3): the exact weight tables, the sweep's
 * counter-state tables and the launch schedule. Requires 1 <= d <= 30 and
 * 1 <= l <= d (else FSI_ERR_INVALID_ARG; l = 0 is rejected). Uses the
 * current HIP device, which must be gfx950 (else FSI_ERR_UNSUPPORTED).
 * fsi_plan uses FP64 storage and defaults. *out receives the plan (NULL on
 * failure); the caller destroys it with fsi_plan_destroy. */
fsi_status fsi_plan(int d, int l, fsi_plan_t* out);
fsi_status fsi_plan_ex(int d, int l, const fsi_plan_opts* opts, fsi_plan_t* out);

/* Frees the plan's host tables, device tables and workspace. NULL is a
 * no-op. Waits first for the plan's work issued by the apply calls (an
 * event recorded on the apply's stream after each call, outside stream
 * capture), not for the whole device. */
fsi_status fsi_plan_destroy(fsi_plan_t plan);

/* Writes the M output masks of the plan (the coalitions S, |S| <= l, of
 * Eq. 3, Sec. 2.2), in canonical order, to host_masks (caller-owned host
 * memory, length fsi_num_outputs(d, l)). Host only. */
fsi_status fsi_output_masks(fsi_plan_t plan, uint32_t* host_masks);

/* Schedule actually chosen, for reporting: tile bits b, the workgroup size
 * of the plan's tile kernel (256 on the register-phase kernel, 512 on the
 * generic one), algorithm, precision. Any pointer may be NULL. */
fsi_status fsi_plan_info(fsi_plan_t plan, int* tile_bits, int* block_threads,
                         int* algo, int* precision);

/* out_dev[k] = E_{S_k} for the plan's (d, l): the operator of Sec. 4.1,
 * Eq. 5 (Moebius transform, then the correction of Eq. 4 with the weights
 * of Eq. 7). v_dev has 2^d elements and is not modified (except by an
 * in-place two-pass plan, see allow_input_overwrite); out_dev has M
 * elements; both are caller-owned device memory in the storage dtype.
 * Asynchronous on stream. */
fsi_status fsi_apply(fsi_plan_t plan, const void* v_dev, void* out_dev,
                     hipStream_t stream);

/* Moebius transform alone (Sec. 4.2, Appendix B), in place on a_dev
 * (2^d elements of the plan's storage dtype): for every bit i and every mask
 * m with bit i set, a[m] -= a[m with bit i cleared]. Low bits are staged in
 * LDS, high bits run as coalesced strided passes. */
fsi_status fsi_mobius(fsi_plan_t plan, void* a_dev, hipStream_t stream);

/* Batched plan over n instances of possibly different (d_i, l_i)
 * (1 <= l_i <= d_i <= 30, n >= 1). Instance i reads values
 * [value_offset[i], value_offset[i+1]) of one concatenated device array and
 * writes outputs [out_offset[i], out_offset[i+1]) of another; both offset
 * tables are prefix sums of 2^d_i and M(d_i, l_i) starting at 0. One apply
 * is a fixed sequence of persistent kernel launches over a device work list,
 * replayed from a captured HIP graph. The register-phase kernel's work items
 * are sorted by decreasing cost; past the first round its workgroups take
 * them from a queue in the plan's tables as they finish, and each launch
 * leaves that queue as it found it (zero). */
fsi_status fsi_plan_batched(int n, const int* d_host, const int* l_host,
                            const fsi_plan_opts* opts, fsi_batch_plan_t* out);
fsi_status fsi_batch_plan_destroy(fsi_batch_plan_t plan);

/* Copies the offset tables (n + 1 int64 each) to host memory; either pointer
 * may be NULL. */
fsi_status fsi_batch_offsets(fsi_batch_plan_t plan, int64_t* value_offset,
                             int64_t* out_offset);

/* Applies the batched plan: values_dev holds value_offset[n] elements,
 * out_dev out_offset[n] elements (storage dtype). Asynchronous on stream.
 * The first call for a given (values_dev, out_dev) pair captures the
 * launch sequence into a HIP graph; later calls with the same pointers
 * replay it. */
fsi_status fsi_apply_batched(fsi_batch_plan_t plan, const void* values_dev,
                             void* out_dev, hipStream_t stream);

/* Same as fsi_apply_batched but launches the kernels directly (no graph). */
fsi_status fsi_apply_batched_nograph(fsi_batch_plan_t plan,
                                     const void* values_dev, void* out_dev,
                                     hipStream_t stream);

/* For callers that cannot allocate device memory at apply time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * fsi_apply_batched_nograph with the plan's device workspaces (partial sums,
 * per-tile results, two-pass Moebius workspace) taken from a static device
 * scratch array of 64 MiB per GPU instead of the plan's own buffers. It
 * calls no hipMalloc, hipFree or other allocating routine. Plans whose
 * workspaces need more than 64 MiB (e.g. d above about 24 at l = 4 on the
 * generic kernel) get FSI_ERR_INVALID_ARG; so does a call whose current HIP
 * device is not the plan's. Every such call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (other streams, other
 * threads) race, and the array keeps the last call's contents (no kernel
 * reads a word the same call has not written). Same outputs as
 * fsi_apply_batched_nograph. */
fsi_status fsi_apply_batched_noalloc(fsi_batch_plan_t plan,
                                     const void* values_dev, void* out_dev,
                                     hipStream_t stream);

/* The kernel launches of one batched apply, for per-kernel timing. The
 * fused algorithm launches, in this order and each only if the plan has
 * such work: the register-phase tile kernel once (in-tile Moebius + counter
 * sweep + final weights + cross-tile sums per work item; one launch over
 * the items of every order l present), the generic tile kernel, the generic
 * per-output reduction, the wide gather and its final pass (generic
 * instances with at least 2^10 tiles, register-phase instances of several
 * blocks), and the reduction of the register-phase partial sums of
 * one-block instances. A batch whose instances all take the register-phase
 * kernel (l <= 4) and fit one block each (l <= 3, or d <= 20 at l = 4) has
 * two stages. The
 * two-pass algorithm has 3 + (number of strided high-bit Moebius passes)
 * stages (low pass, high passes, tile kernel, reduction). Running stages
 * 0 .. n-1 in order on one stream equals fsi_apply_batched_nograph.
 * fsi_batch_num_stages returns -1 for a NULL plan. */
int fsi_batch_num_stages(fsi_batch_plan_t plan);
fsi_status fsi_apply_batched_stage(fsi_batch_plan_t plan, const void* values_dev,
                                   void* out_dev, int stage, hipStream_t stream);

/* Schedule of a plan (host struct filled by the call). */
fsi_status fsi_plan_schedule(fsi_plan_t plan, fsi_schedule* out);
fsi_status fsi_batch_schedule(fsi_batch_plan_t plan, fsi_schedule* out);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* fsi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FSI_MI355X_H */
