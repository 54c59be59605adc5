/*
 * cqsim -- compressed full-amplitude quantum circuit simulation on one MI355X.
 *
 * C ABI of the library libcqsim.so.  It implements the per-gate, per-slice
 * loop of Algorithm 1 of Wu, Di, Cappello, Finkel, Alexeev and Chong,
 * "Memory-Efficient Quantum Circuit Simulation by Using Lossy Data
 * Compression" (Section II): the state vector of 2^n complex amplitudes
 * (Section I: 2^(n+4) bytes in FP64) is cut into slices; every slice stays
 * compressed in device memory (HBM) with an error-bounded lossy codec, and
 * each gate is applied as
 *     for each slice: Decompress -> Normalize -> GateComputation -> Compress.
 *
 * Conventions shared by all entry points
 *   - Return value: 0 on success, a negative SIM_E* code on failure.  The text
 *     of the last failure on the calling thread is sim_last_error().
 *   - Amplitude index i = sum_q b_q 2^q (qubit 0 is the least significant bit).
 *   - Pointers named "host" are ordinary CPU memory owned by the caller; the
 *     library never keeps them after the call returns.  All device memory is
 *     owned by the handle (or obtained through sim_set_allocator).
 *   - One handle must not be used from two threads at once.  Work is ordered
 *     on the handle's HIP stream; calls that return data synchronise it.
 *   - No CPU fallback exists: without a usable gfx950 device sim_create fails
 *     with SIM_EDEVICE.
 */
#ifndef CQSIM_H
#define CQSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes */
#define SIM_OK 0
#define SIM_EINVAL (-1)   /* invalid argument or gate */
#define SIM_ENOMEM (-2)   /* device memory could not be obtained */
#define SIM_EBOUND (-3)   /* a value cannot be coded within the error bound */
#define SIM_ECORRUPT (-4) /* a slice record failed its consistency checks */
#define SIM_EDEVICE (-5)  /* HIP runtime or device failure */

/* ---- mode bits of sim_create (Section II: the user sets the error bound) */
#define SIM_EB_ABS 0x0u  /* |a - a'| <= error_bound for every real and imaginary part */
#define SIM_EB_REL 0x1u  /* per slice: error_bound * max(max - min, 2^-24 max|a|) over its 2L values */
#define SIM_FP64 0x0u    /* amplitudes and gate arithmetic in FP64 */
#define SIM_FP32 0x2u    /* amplitudes, gate matrices, initial factors and every product and sum
                            of the gate arithmetic rounded to FP32 (an extension: the paper
                            works in FP64); quantisation, the bound check and the norm stay
                            FP64, applied to the FP32 values; raw bytes are 8 per amplitude.
                            The bound holds for the stored value q*step; the working value
                            read back is that value rounded to FP32, so it lies within
                            error_bound + 2^-24 |a| of the gate output */
#define SIM_PLAIN 0x0u   /* one pass per gate, exactly as in Algorithm 1 */
#define SIM_FUSED 0x4u   /* runs of consecutive gates on at most SIM_FUSE_MAX qubits are applied
                            as one dense block per pass (see sim_plan); blocks of 3 or more
                            qubits run on FP64 matrix cores */

#define SIM_ZERO_CHUNKS 0x8u /* a chunk whose codes are all zero is stored with no words (an
                                extension for sparse states; header word 14 bit 0 marks such
                                records).  Codes, amplitudes and norms are those of the mode
                                without it; only record sizes shrink */
#define SIM_CONST_CHUNKS 0x10u /* a chunk whose values all equal its first keeps only the first
                                  one's code; bit 31 of its word offset marks it, header word 14
                                  bit 1 marks such records (an extension for states with flat
                                  stretches).  With SIM_ZERO_CHUNKS an all-zero chunk stays a zero
                                  chunk.  Codes, amplitudes and norms are unchanged */

#define SIM_EB_PWREL 0x20u /* pointwise-relative bound: |a - a'| <= error_bound |a| for every real and
                               imaginary part (an extension, one reading of Section II's bound for each
                               amplitude number): each value is stored as the nearest FP64 number with
                               b mantissa bits, b the least with 2^-(b+1) <= error_bound (0 < error_bound
                               < 0.5, b <= 20); zeros stay zero.  Header word 14 bit 2 and word 15 = b
                               mark such records, whose step is 1 and whose sum field holds the slice's
                               squared norm as an FP64 value (a pairwise tree over its 2L values).
                               Excludes SIM_EB_REL */

#define SIM_CHUNK_RUNS 0x40u /* chunk runs (an extension: a run-length stage over the Huffman output, one
                                of the compression variants Section IV leaves to future work):
                                consecutive chunks whose stored streams are identical (the same words and
                                constant mark) form a run whose stream is stored once.  Where that makes
                                a record smaller and the slice has at most 4096 runs, the chunk offsets
                                are replaced by u32 R, R run ends (cumulative chunk counts) and R + 1 word
                                offsets of the runs' streams; header word 14 bit 3 marks such records.
                                Codes, amplitudes and norms are unchanged; only record sizes shrink */

#define SIM_OPT 0x80u    /* optimised passes (an extension, off for Algorithm 1 as written; not with
                            SIM_FUSED, not through sim_apply_noalloc): a gate controlled on slice-index
                            qubits leaves the slice groups whose index bits fail those controls as they
                            are (records not decoded, renormalised or re-encoded), and a SWAP of two
                            slice-index qubits without controls relabels the slices (record j becomes
                            the record of j with the two index bits exchanged) without touching a value */

#define SIM_FUSE_MAX 5   /* widest fused block, in qubits */

/* ---- gate kinds (Section II: the circuit is a sequence of gates applied one
 * by one).  Every kind also takes the extra controls ctrl_mask / ctrl_vals: it
 * acts only on amplitudes i with (i & ctrl_mask) == ctrl_vals.  Named kinds
 * are turned into a matrix or a phase on the host, in FP64, before a pass
 * runs; they give the same records as the DENSE or PHASE gate with that
 * matrix or phase. */
#define SIM_GATE_DENSE 1u /* 2^k x 2^k complex `matrix` on targets[0..k), k = n_targets = 1..5 */
#define SIM_GATE_PHASE 2u /* n_targets = 0: amplitude i times (params[0] + i params[1]) */
#define SIM_GATE_H 3u     /* Hadamard on targets[0]: sqrt(1/2) [[1, 1], [1, -1]] */
#define SIM_GATE_X 4u     /* NOT on targets[0] */
#define SIM_GATE_Z 5u     /* -1 where bit targets[0] is 1 */
#define SIM_GATE_P 6u     /* e^{i params[0]} where bit targets[0] is 1 */
#define SIM_GATE_CP 7u    /* e^{i params[0]} where bits targets[0] and targets[1] are both 1 */
#define SIM_GATE_CZ 8u    /* -1 where bits targets[0] and targets[1] are both 1 */
#define SIM_GATE_SWAP 9u  /* exchange of qubits targets[0] and targets[1] */
#define SIM_GATE_U3 10u   /* OpenQASM 2 u3(theta, phi, lambda) = (params[0], params[1], params[2]) on
                             targets[0]: [[c, -e^{i lambda} s], [e^{i phi} s, e^{i(phi+lambda)} c]],
                             c = cos(theta/2), s = sin(theta/2) (each entry one FP64 product) */
#define SIM_GATE_MCZ 11u  /* -1 where every bit of targets[0..n_targets) is 1 (n_targets = 1..5);
                             wider multi-controlled Z: SIM_GATE_PHASE with params (-1, 0) and the
                             qubits in ctrl_mask and ctrl_vals */
#define SIM_GATE_U1Q 12u  /* one-qubit gate: the 2 x 2 complex `matrix` on targets[0] */

typedef struct sim_s sim_t;

/* One gate of the program (Section II: the program is processed gate by gate).
 * DENSE (and U1Q): local index m = sum_k bit(i, targets[k]) << k selects the
 *   row and column of `matrix` (row-major, 2^k x 2^k complex, interleaved
 *   re, im; host memory, copied by sim_apply).
 * PHASE: amplitude i is multiplied by (params[0] + i params[1]) where
 *   (i & ctrl_mask) == ctrl_vals (Z, CZ, controlled phases, oracles).
 * The other kinds are listed above.  Controls must not overlap targets.
 * Layout is fixed: 80 bytes, naturally aligned. */
typedef struct sim_gate {
  uint32_t kind;
  uint32_t n_targets;
  uint32_t targets[5];
  uint32_t reserved;
  uint64_t ctrl_mask;
  uint64_t ctrl_vals;
  double params[3];
  const double *matrix;
} sim_gate;

/* One pass of a fused program (sim_plan).  Gates [first_gate, first_gate +
 * n_gates) of the program form the pass.  fused == 0: a single gate, applied
 * as in plain mode.  fused == 1: two or more gates whose qubits (targets and
 * control bits) together are qubits[0..n_qubits), ascending; they are applied
 * as the one 2^n_qubits x 2^n_qubits matrix U = G_last ... G_first, each
 * gate embedded in the block's space (local bit i is qubits[i]) and the
 * product formed left to right, U <- G U, with every term of every sum
 * included in ascending order and the complex multiply-add of the gate
 * kernels.  Layout is fixed: 40 bytes. */
typedef struct sim_pass {
  uint32_t first_gate;
  uint32_t n_gates;
  uint32_t fused;
  uint32_t n_qubits;
  uint32_t qubits[5];
  uint32_t reserved;
} sim_pass;

/* Extended creation parameters; zero fields take the defaults. */
typedef struct sim_config {
  int n_qubits;             /* 1..40 */
  int slice_log2;           /* L = 2^slice_log2 amplitudes per slice, 1..26, <= n_qubits */
  int chunk_log2;           /* B = 2^chunk_log2 values per coded chunk (0: 10), clipped to slice_log2 */
  double error_bound;       /* > 0 */
  uint32_t mode;            /* SIM_EB_* | SIM_FP64 or SIM_FP32 | SIM_PLAIN or SIM_FUSED */
  uint64_t workspace_bytes; /* budget for decompressed slices in flight (0: up to 16 GiB) */
  /* optional device-memory hooks used for every allocation of the handle
   * (e.g. a framework's caching allocator); both NULL: hipMalloc / hipFree */
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free_fn)(void *ptr, void *ctx);
  void *alloc_ctx;
  void *stream;             /* hipStream_t to enqueue on (NULL: a stream of the handle) */
  uint64_t arena_bytes;     /* initial capacity of each of the two record arenas (0: sized
                               from the slice count); arenas grow by doubling when a pass
                               overflows, and the pass is run again */
} sim_config;

/* Statistics (Section III measures compression ratio, fidelity and time). */
typedef struct sim_stats_t {
  uint64_t raw_bytes;           /* 16 * 2^n: the uncompressed FP64 state (8 * 2^n with SIM_FP32) */
  uint64_t compressed_bytes;    /* sum of the slice records now stored */
  uint64_t peak_compressed;     /* largest total after any pass (sets the minimum ratio) */
  double ratio;                 /* raw_bytes / compressed_bytes */
  double min_ratio;             /* raw_bytes / peak_compressed */
  uint64_t passes;              /* gates applied since creation */
  uint64_t escapes;             /* escape symbols coded since creation */
  double last_norm;             /* squared norm of the stored state before the last pass */
  double max_abs_codec_err;     /* largest |a - p*step| seen by the quantiser */
  double elapsed_s;             /* device time spent in sim_apply */
  uint64_t arena_bytes;         /* device bytes held for compressed records (both buffers) */
  uint64_t workspace_slots;     /* slices decompressed at once */
  uint64_t device_bytes;        /* every device byte the handle holds now */
  double min_slice_ratio;       /* smallest ratio of one slice now: raw slice bytes (16 L, or 8 L with
                                   SIM_FP32) / its record bytes */
  uint64_t gates;               /* gates of the program applied since creation (passes count the
                                   passes; in SIM_FUSED mode a pass applies one or more gates) */
} sim_stats_t;

/* Create a simulator holding |0...0>, compressed (Algorithm 1 starts from a
 * compressed state).  Arguments as in sim_config; error_bound is absolute or
 * relative according to `mode`.  *out receives the handle.  Errors: SIM_EINVAL
 * (range), SIM_ENOMEM, SIM_EDEVICE, SIM_EBOUND (the bound is too fine for the
 * codes to stay below 2^48 in magnitude). */
int sim_create(int n_qubits, int slice_log2, double error_bound, uint32_t mode, sim_t **out);
int sim_create_ex(const sim_config *cfg, sim_t **out);

/* Device bytes that sim_create_ex(cfg) would hold once the initial state is
 * built (every buffer of the handle, both record arenas at their initial
 * capacity and the slot order of slice-local gates); later growth (arena
 * doubling, gate groups on slice-index qubits, fused-block matrices, readout
 * staging) is not included.  Host-only: touches no device.  Errors: as
 * sim_create_ex for the configuration's fields (allocator and stream ignored). */
int sim_footprint(const sim_config *cfg, uint64_t *bytes);

/* Release all device memory of the handle.  NULL is ignored. */
void sim_destroy(sim_t *sim);

/* Text of the last failure on this thread (never NULL). */
const char *sim_last_error(void);

/* Replace the state by the basis state |x> (x < 2^n) and compress it
 * (Algorithm 1 starts from a compressed state: its first step is Decompress). */
int sim_init_basis(sim_t *sim, uint64_t x);

/* Replace the state by the product state prod_q f_q(b_q) (compressed, as
 * sim_init_basis) with
 * f_q(0) = cos(theta_q / 2), f_q(1) = e^{i phi_q} sin(theta_q / 2); `factors`
 * is host memory of n_qubits * 4 doubles (f_q(0).re, f_q(0).im, f_q(1).re,
 * f_q(1).im), computed by the caller.  The product is formed from (1, 0) with
 * qubit 0 first. */
int sim_init_product(sim_t *sim, const double *factors);

/* Use caller-provided device memory for allocations made from now on (arena
 * growth, staging buffers).  alloc(bytes, ctx) returns device memory or NULL;
 * free(ptr, ctx) releases it.  Memory already held is released through the
 * functions that allocated it.  To cover the initial allocations as well,
 * pass the hooks in sim_config. */
int sim_set_allocator(sim_t *sim, void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *), void *ctx);

/* Enqueue all work of the handle on `hip_stream` (a hipStream_t) from now on. */
int sim_set_stream(sim_t *sim, void *hip_stream);

/* Apply gates[0..n) in order, one pass of Algorithm 1 per gate (Section II),
 * or in SIM_FUSED mode one pass per block of sim_plan's partition of the n
 * gates (then *n_applied counts the gates of the completed passes):
 * for every slice group, decompress, normalise by the norm of the stored
 * state, apply the gate, recompress.  Gates whose targets are slice-index
 * qubits couple 2^m slices, which are processed together.  The gate array
 * and matrices are host memory read during the call.  Passes are
 * transactional: on failure the state is the one after the last completed
 * pass, and *n_applied (may be NULL) counts completed passes.  Errors:
 * SIM_EINVAL (bad gate; nothing after it runs), SIM_EBOUND, SIM_ENOMEM,
 * SIM_EDEVICE. */
int sim_apply(sim_t *sim, const sim_gate *gates, size_t n, size_t *n_applied);

/* The partition of gates[0..n) into passes that sim_apply uses in SIM_FUSED
 * mode (an extension: Algorithm 1 makes one pass per gate, and fused mode
 * groups gates into passes; host computation, nothing is enqueued).  Greedy,
 * in program order: a pass collects consecutive gates while the union of
 * their qubits (targets and control bits of each gate; a phase gate's qubits
 * are its control bits) has at most SIM_FUSE_MAX members; a gate that alone
 * touches more qubits is a pass of its own.  A pass of one gate is plain.
 * The gates must be valid for the handle's qubits (SIM_EINVAL otherwise).
 * out (host memory, `cap` entries, may be NULL to count) receives the passes;
 * *n_pass their number.  Returns SIM_ENOMEM if cap is too small (n_pass is
 * still set). */
int sim_plan(const sim_t *sim, const sim_gate *gates, size_t n, sim_pass *out, size_t cap, size_t *n_pass);

/* sim_plan for n_qubits qubits without a handle (the same partition). */
int sim_plan_qubits(int n_qubits, const sim_gate *gates, size_t n, sim_pass *out, size_t cap, size_t *n_pass);

/* Normalised amplitudes [begin, begin + count) into host memory `out`
 * (2 * count doubles, interleaved re, im): the stored state decompressed and
 * scaled by the same normalisation a pass would use (Section III compares
 * the final amplitudes with the uncompressed simulation to measure fidelity). */
int sim_amplitudes(sim_t *sim, uint64_t begin, uint64_t count, double *out);

/* |a_i|^2 of the same normalised amplitudes into host memory (count doubles):
 * the measurement probabilities (Section III: Grover's success probability). */
int sim_probabilities(sim_t *sim, uint64_t begin, uint64_t count, double *out);

/* Fill *out (host memory).  Synchronises the stream. */
int sim_stats(sim_t *sim, sim_stats_t *out);

/* Size in bytes of the stored record of slice j (0 if j is out of range). */
uint64_t sim_record_size(sim_t *sim, uint64_t j);

/* Copy the stored record of slice j (its exact bytes) into host memory `buf`
 * of `cap` bytes; *len receives the size.  The record format is fixed and
 * self-describing: header, symbol table, chunk word offsets, bit stream. */
int sim_export_slice(sim_t *sim, uint64_t j, void *buf, uint64_t cap, uint64_t *len);

/* The 64-byte headers of the stored records of slices [first, first + count)
 * into host memory `out` (64 * count bytes, caller-owned): per slice the
 * step, the exact sum p^2 of its codes and its sizes -- what Normalize needs
 * from every slice (Algorithm 1; the norm of the stored state), without the
 * bit streams.  Synchronises the stream.  Errors: SIM_EINVAL (range). */
int sim_record_headers(sim_t *sim, uint64_t first, uint64_t count, void *out);

/* Replace the stored record of slice j by `len` bytes from host memory
 * (checkpoint restore).  The record is checked for consistency (SIM_ECORRUPT)
 * and must have the handle's slice and chunk sizes. */
int sim_import_slice(sim_t *sim, uint64_t j, const void *buf, uint64_t len);

/* ---- allocation-free apply
 * For callers that cannot allocate device memory once the handle exists
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): sim_apply's passes with the same results (the same kernels,
 * byte-identical records), calling no hipMalloc, hipFree or allocator hook.
 * The decompressed slots, per-slot partial results, slot orders and gate
 * matrices of the passes live in a scratch array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends, instead of the
 * handle's workspace; slices are processed in as many batches as the array
 * needs.  Differences from sim_apply:
 *   - the whole program is checked first; an invalid gate runs nothing;
 *   - a pass needing a group of slices (2^m slices for m slice-index targets)
 *     larger than the array holds is refused with SIM_ENOMEM before anything
 *     runs (one slot of 2^k amplitudes takes about 52 x 2^k bytes: slices of
 *     2^21 amplitudes never fit, slices of 2^20 only one at a time);
 *   - the record arenas do not grow: a pass that overflows its output arena
 *     fails with SIM_ENOMEM, leaving the state of the last completed pass
 *     (*n_applied counts its gates); create the handle with enough
 *     arena_bytes, or let sim_apply grow the arenas first.
 * The array is shared by every call on one GPU and keeps the last call's
 * contents (each call clears what it counts into): calls that overlap in
 * time on one GPU, from any handles or threads, race and must not be made. */
int sim_apply_noalloc(sim_t *sim, const sim_gate *gates, size_t n, size_t *n_applied);

/* ---- captured gate programs (HIP graphs)
 * For callers that apply one gate program many times (a Grover iteration, a
 * circuit served repeatedly) and want no per-pass host work.
 * sim_graph_create records the passes of gates[0..n) (plain or fused, as
 * sim_apply would run them) into a HIP graph without running them; the
 * matrices are copied, the gates need not outlive the call.  Every gate must
 * be valid (SIM_EINVAL otherwise, no graph).  sim_graph_launch applies the
 * program to the current state with the same result as sim_apply and the
 * same failure semantics; *n_applied counts the gates of completed passes.
 * The graph replays as captured only from the arena parity and arena
 * allocations it was captured on: after an odd number of other passes the
 * program runs through the ordinary launches, and after an arena has grown
 * it is captured again first (both automatic).  A graph belongs to its
 * handle: destroy it before sim_destroy; launches on one handle must not
 * overlap. */
typedef struct sim_graph_s sim_graph_t;
int sim_graph_create(sim_t *sim, const sim_gate *gates, size_t n, sim_graph_t **out);
int sim_graph_launch(sim_t *sim, sim_graph_t *graph, size_t *n_applied);
void sim_graph_destroy(sim_graph_t *graph);

/* Chunk-length autotuning (B = 2^chunk_log2 values per coded chunk is a format
 * parameter, recorded in every record header).  For each chunk_log2 in
 * [lo, hi] (within 1..10) a fresh handle of configuration *cfg (its
 * chunk_log2 ignored) applies gates[0..n): the first n/4 untimed, the rest
 * timed on the device as in sim_apply.  *best receives the fastest (ties: the
 * smaller record total); ms_per_gate[k] and bytes[k] (each hi - lo + 1
 * entries, or NULL) receive the timed milliseconds per gate and the record
 * total after the program for chunk_log2 = lo + k.  Every handle is destroyed
 * before the call returns.  Errors: SIM_EINVAL (range, n < 2), and any error
 * of creating or running a candidate. */
int sim_tune_chunk(const sim_config *cfg, const sim_gate *gates, size_t n, int lo, int hi, int *best,
                   double *ms_per_gate, uint64_t *bytes);

/* Device time (milliseconds, summed since the last reset) spent in each of
 * the library's kernel classes, measured with HIP events on the handle's
 * stream when enabled.  `names` receives a static comma-separated list of the
 * class names in order; out has room for `cap` values: out[k] is class k's
 * milliseconds and, when cap >= 2 * classes, out[classes + k] the number of
 * its launches that were timed.  Returns the number of classes.  enable != 0
 * turns the per-kernel events on and resets the sums, enable == 0 turns them
 * off, enable < 0 only reads. */
int sim_kernel_times(sim_t *sim, int enable, double *out, int cap, const char **names);

/* ---- job server (an extension: the paper simulates one circuit at a time)
 * For callers that run many independent circuits on one device (a request
 * queue of simulation jobs).  Each admitted job gets its own handle and one
 * of `max_active` HIP streams, driven by a host worker thread, so the passes
 * of different jobs run on the device at the same time; jobs stay compressed
 * in device memory while they run.
 * Admission is first come, first served: the job at the head of the queue
 * starts when fewer than max_active jobs run and the projected footprints of
 * the running jobs plus its own fit `budget_bytes` (or nothing runs).  The
 * projected footprint is sim_footprint() of the job's configuration with
 * each record arena sized by a per-family ratio model: 8 bytes per amplitude
 * (int32 codes for both components) until a job of the family has finished,
 * afterwards 1.25 x raw bytes / (the smallest minimum ratio seen in the
 * family), never above 8 bytes per amplitude.  A job whose records outgrow
 * the projection still completes (its arenas double).  Device memory of
 * finished jobs is cached for later jobs (requests are rounded up to
 * multiples of 64 KiB and of an eighth of their largest power of two; the
 * cache holds at most `budget_bytes`).
 * Jobs share nothing but the device: a job's records, amplitudes and
 * statistics do not depend on the jobs that run beside it. */
#define SRV_INIT_ZERO 0u    /* start from |0...0> */
#define SRV_INIT_BASIS 1u   /* start from |basis> */
#define SRV_INIT_PRODUCT 2u /* start from the product state of `factors` */
#define SRV_FAMILIES 16u    /* ratio-model classes */

typedef struct srv_s srv_t;

typedef struct srv_job {
  sim_config cfg;         /* alloc, free_fn and stream must be NULL (the server provides
                             them); arena_bytes 0: sized by the ratio model */
  uint32_t family;        /* ratio-model class, < SRV_FAMILIES (e.g. one per circuit family) */
  uint32_t init;          /* SRV_INIT_* */
  uint64_t basis;         /* SRV_INIT_BASIS: the basis index */
  const double *factors;  /* SRV_INIT_PRODUCT: 4 * n_qubits doubles as for sim_init_product;
                             host memory, copied by srv_submit */
  const sim_gate *gates;  /* the program; host memory, copied (matrices too) by srv_submit */
  size_t n_gates;
  double *out;            /* host buffer for amplitudes [out_begin, out_begin + out_count) as
                             sim_amplitudes writes them, filled when the job ends; NULL: none.
                             Owned by the caller; must stay valid until srv_wait reports the job */
  uint64_t out_begin;
  uint64_t out_count;
} srv_job;

typedef struct srv_done {
  uint64_t id;               /* as returned by srv_submit */
  int status;                /* SIM_OK or the code of the first failing call */
  uint32_t family;
  uint64_t applied;          /* gates applied */
  uint64_t projected_bytes;  /* footprint the job was admitted with */
  uint64_t device_bytes;     /* device bytes its handle held at the end */
  double t_submit, t_start, t_end; /* seconds on the server clock (srv_clock) */
  sim_stats_t stats;         /* final statistics (zero if the handle was never created) */
  char error[160];           /* sim_last_error() of the failing call, or empty */
} srv_done;

/* Start a server with `max_active` (1..64) workers and streams.  Errors:
 * SIM_EINVAL, SIM_EDEVICE (no gfx950 device). */
int srv_create(uint64_t budget_bytes, int max_active, srv_t **out);

/* Queue a job; *id receives its number (1, 2, ...).  Errors: SIM_EINVAL
 * (configuration, family, init or pointers), SIM_ENOMEM (the projected
 * footprint alone exceeds the budget).  The job's gates are validated when it
 * runs (the status reports a bad gate). */
int srv_submit(srv_t *srv, const srv_job *job, uint64_t *id);

/* Move up to `cap` finished jobs not yet reported into out[0..*n_out), in
 * completion order.  Waits up to timeout_s seconds for the first one (0: do
 * not wait); returns at once with *n_out = 0 when no job is queued or
 * running. */
int srv_wait(srv_t *srv, srv_done *out, size_t cap, size_t *n_out, double timeout_s);

/* Seconds since srv_create (the clock of srv_done's times). */
double srv_clock(srv_t *srv);

/* The footprint the job would be admitted with now (the model changes as
 * jobs finish). */
int srv_projected_bytes(srv_t *srv, const srv_job *job, uint64_t *bytes);

/* Cancel queued jobs, wait for running ones, release everything.  Finished
 * jobs not yet reported are dropped.  NULL is ignored. */
void srv_destroy(srv_t *srv);

#ifdef __cplusplus
}
#endif

#endif /* CQSIM_H */
