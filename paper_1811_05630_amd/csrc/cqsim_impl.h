// Internal declarations of libcqsim: the slice-record format constants, the
// device control block, kernel parameter blocks and the launch wrappers that
// the host scheduler (api.hip) calls.  Everything runs on gfx950; there is no
// CPU path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cq {

// ---------------------------------------------------------------- record format
// A slice of L = 2^slice_log2 amplitudes is coded as one stream of 2L values
// (the real plane, then the imaginary plane), cut into chunks of
// B = 2^chunk_log2 values.  Record layout (little-endian, 4-byte fields):
//   0  u32 magic 0x31535143         32 f64 step (quantisation step)
//   4  u32 slice_log2                40 u64 sum p^2, low 64 bits
//   8  u32 chunk_log2                48 u64 sum p^2, high 64 bits
//  12  u32 n_used (coded symbols)    56 u32 flags: bit 0 zero chunks, bit 1 constant chunks,
//                                       bit 2 pointwise-relative codes (step 1, the sum field
//                                       an FP64 squared norm), bit 3 chunk runs
//                                    60 u32 pointwise-relative mantissa bits, else 0
//  16  u32 n_chunks = 2L/B
//  20  u32 n_words (bit stream)
//  24  u32 n_escapes
//  28  u32 total bytes of the record
//  64  n_used x u16 (symbol | length << 10) ordered by (length, symbol), padded to 4 bytes
//      (n_chunks + 1) x u32 word offset of each chunk in the bit stream
//      n_words x u32 bit stream, most significant bit first, chunks word-aligned
// With chunk runs (flags bit 3), consecutive chunks with identical streams
// share one stored stream, and the offsets table is instead: u32 R (at most
// kMaxRuns), R x u32 run ends (cumulative chunk counts, the last n_chunks),
// (R + 1) x u32 word offsets of the runs' streams (the last n_words).  A
// chunk's word offset (or its run's) carries the constant mark in bit 31.
constexpr uint32_t kMagic = 0x31535143u;
constexpr int kHdr = 64;
constexpr int kR = 512;       // quantisation radius: symbol d + R for |d| < R
constexpr int kNSym = 1024;   // alphabet; symbol 0 is the escape
constexpr int kLMax = 12;     // longest code; also the decoder's lookup width
constexpr int kEscBits = 6;   // escape payload: 6-bit length, then zigzag(d)
constexpr double kPMax = 281474976710656.0;  // 2^48: |p| must stay below
constexpr uint64_t kRecAlign = 256;          // records start on 256-byte boundaries

// Decoder table entry for a 12-bit peek at the stream: the first code's
// symbol and length, and -- when the next code also lies inside the 12 bits
// and neither symbol is the escape -- the second symbol and length.
//   bits 0-9 symbol 1, 10-13 length 1, 14-23 symbol 2, 24-27 length 2, 28 second present
inline __host__ __device__ uint32_t dtab_entry(uint32_t s1, uint32_t l1, uint32_t s2, uint32_t l2, bool two) {
  return s1 | (l1 << 10) | (two ? (s2 << 14) | (l2 << 24) | (1u << 28) : 0u);
}

// ------------------------------------------------------------- control block
enum : uint32_t { kFlagBound = 1u, kFlagOverflow = 2u, kFlagCorrupt = 4u };

struct Ctl {
  uint64_t bump;          // aligned bytes used in the output arena by this pass
  uint64_t cur_bytes;     // exact record bytes of the stored state
  uint64_t peak_bytes;    // largest cur_bytes at the end of any pass
  uint64_t max_err_bits;  // largest |a - p step| (non-negative FP64 bits)
  uint64_t escapes;       // escape symbols coded
  uint32_t flags;         // kFlag* bits; any set bit turns later kernels into no-ops
  uint32_t fail_pass;     // pass counter value of the first failure
  double N;               // norm of the stored state at the start of this pass
  double s;               // 1 / sqrt(N)
  uint64_t pending_bump;  // aligned bytes of the last batch written; added to bump and
  uint64_t pending_bytes; // cur_bytes by the next launch that starts a batch or a pass
  uint32_t wide;          // 1: the records of this pass may hold |q| >= 2^31 (the decoded
                          // workspace is FP64); 0: every q fits int32 (compact workspace)
  uint32_t wide_next;     // set by any quantisation of this pass that produced |q| >= 2^31;
                          // moved to `wide` by the next pass's begin
  uint64_t pad[3];
};

// ---------------------------------------------------------------- gate block
// A gate acting on a group of 2^m slices (m = targets at slice-index qubits).
// Inside a group the local index is gl = (member << slice_log2) | offset;
// target k sits at local bit tloc[k] (targets below slice_log2 keep their bit,
// slice-bit targets are renumbered slice_log2, slice_log2 + 1, ... in order).
struct GateDesc {
  int kind;               // 0: identity, 1: dense, 2: phase, 4: fused dense block of 3..5
                          // qubits on matrix cores (mat: its 2^(k+1) square real embedding)
  int k;                  // number of targets
  int m;                  // slice-bit targets
  int pad0;
  int tloc[5];
  int pad1;
  uint64_t tmask_loc;     // OR of 1 << tloc[k]
  uint64_t ctrl_mask, ctrl_vals;
  double ph_re, ph_im;
  const double *mat;      // device, 2^k x 2^k complex, row-major, interleaved
  double m2[8];           // one-target gates: the 2x2 matrix itself
  uint64_t dep[32];       // local offset of column c: bits of c deposited at tloc
};

struct QuantParams {
  int rel;                // 0: absolute bound, 1: value-range-relative bound
  double eb;              // absolute bound, or the relative factor
  double step, recip;     // absolute mode: step = 2 eb (1 - 2^-20), recip = 1/step
  int pw;                 // 1: pointwise-relative bound eb: each value rounded to pw_bits mantissa bits
  int pw_bits;            // the least b with 2^-(b+1) <= eb (pointwise-relative mode)
};

struct Geo {
  int n;
  int slice_log2;
  int chunk_log2;
  uint32_t nchunks;       // 2L / B
  uint64_t L;
  uint32_t zero_chunks;   // SIM_ZERO_CHUNKS: all-zero chunks are stored with no words
  uint32_t const_chunks;  // SIM_CONST_CHUNKS: constant chunks keep their head only (offset bit 31)
  uint32_t fmt_in;        // the stored records may hold zero chunks (bit 0) or constant chunks (bit 1):
                          // the modes, or imported records
  int pw_bits;            // -1, or pointwise-relative records: a code is a value's bit pattern without
                          // the sign, rounded to pw_bits mantissa bits and shifted right by 52 - pw_bits
  uint32_t chunk_runs;    // SIM_CHUNK_RUNS: runs of chunks with identical streams store the stream once
  uint32_t run_tiles;     // tiles of kRunTile chunks per slice (the runs kernels' grid)
};

// Per-slot scratch of one batch of decompressed slices.
// Every gate_quant workgroup overwrites its partial results (hpart, part)
// whole, and the codebook kernel reads only those of the current launch.
// words is cleared by the codebook kernel before encode adds to it; minmax
// is cleared by the relative-step kernel after reading it.
struct Slots {
  double *ws;             // [W][2L] decompressed values (re plane, im plane)
  uint16_t *sym;          // [W][2L] symbols
  int64_t *esc;           // [W][2L] exact differences of escaped values
  uint32_t *codes;        // [W][1024] code << 8 | length
  uint16_t *symtab;       // [W][1024] canonical symbol table
  uint32_t *nused;        // [W]
  uint32_t *chunk_words;  // [W][nchunks] word offset of each chunk inside its encode block
  uint32_t *words;        // [W] total words (zeroed by the codebook kernel, added by encode)
  uint32_t *blk_words;    // [W][kMaxEncBlocks] words of each encode block
  uint64_t *sq;           // [W][2] sum p^2 (lo, hi)
  uint32_t *nesc;         // [W]
  uint64_t *minmax;       // [W][2] ordered keys of min and max (relative bound)
  double *qstep;          // [W][3] step, recip, bound (relative bound)
  uint32_t *stage;        // [W][nchunks][stage_words]: each encode block's chunks, packed from the
                          // start of the block's region, before they move into the record
  uint32_t stage_words;   // capacity of one chunk: ceil(B * 68 / 32) words
  // gate_quant writes, per slot, up to kGqParts partial results (one per
  // workgroup and tile role) without atomics; the codebook kernel adds them
  uint32_t *hpart;        // [W][kGqParts][1024] partial histograms
  uint64_t *part;         // [W][kGqParts][4] sum p^2 lo, hi, escapes, max error bits
  double *csum;           // [W][nchunks] pointwise-relative mode: each chunk's sum of squared stored
                          // values as a pairwise tree in index order (the codebook sums the slice)
  // chunk runs (SIM_CHUNK_RUNS), written by the runs kernel after encode
  uint8_t *run_start;     // [W][nchunks] 1 where a chunk starts a run
  uint32_t *run_tile;     // [W][run_tiles][2] runs starting in each tile of kRunTile chunks, their words
  uint32_t *blk_run;      // [W][kMaxEncBlocks] index of the first run starting in each encode block
  uint32_t *run_src;      // [W][kMaxRuns] first chunk of each run
  uint32_t *run_woff;     // [W][kMaxRuns + 1] word offset of each run's stream in the record | mark
  uint32_t *nruns;        // [W] number of runs (may exceed kMaxRuns: then the plain layout)
  uint32_t *run_words;    // [W] words of the runs' streams
};

// Per-slice stored-state metadata (one copy per arena).
struct StateMeta {
  uint64_t *rec_off;      // [S] byte offset of the record in the arena
  uint32_t *rec_len;      // [S] exact record bytes
  double *step;           // [S]
  uint64_t *sq;           // [S][2]
  uint32_t *dtab;         // [S][4096] decoder table derived from the record's symbol table (dtab_entry)
};

// ---------------------------------------------------------------- timing
// Events that the next kernel launch of this thread records when the kernel
// starts and when it ends (both null: none).  The host scheduler sets them
// around one launch to time it.
struct LaunchTimer {
  hipEvent_t start = nullptr, stop = nullptr;
};
LaunchTimer &launch_timer();

// -------------------------------------------------------------- launchers
// All launches go to `st`; `pass` is the global pass counter (for failure
// reporting); `slot_slice` lists the slice held by every slot of the batch.
//
// The kernels that compute amplitudes exist twice: in namespace f64 (every
// value and operation in FP64) and in namespace f32 (the same source compiled
// with every value of the working form and every gate operation rounded to
// FP32; SIM_FP32).  The kernels that only count, code and move bits exist in
// f64 only and serve both.
#define CQ_AMPLITUDE_LAUNCHERS                                                                                  \
  void launch_init(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,      \
                   int kind, uint64_t x, const double *factors, const Ctl *ctl);                                \
  /* compact: the gate_quant launch of this pass reads a compact workspace when ctl->wide is clear          \
     (gq_compact below); decode then writes int32 codes q instead of the values q * kscale */                 \
  void launch_decode(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,    \
                     const uint8_t *arena, const StateMeta &cur, const double *kscale, Ctl *ctl,               \
                     uint32_t pass, bool compact);                                                             \
  void launch_gate_minmax(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice,           \
                          int nslots, const GateDesc &gd, const Ctl *ctl);                                     \
  /* returns the number of partial results per slot that the launch writes */                                 \
  uint32_t launch_gate_quant(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice,        \
                             int nslots, const GateDesc &gd, const QuantParams &qp, Ctl *ctl, uint32_t pass,   \
                             bool compact, const double *kscale);                                              \
  /* whether the gate_quant kernel chosen for gd can read a compact workspace */                               \
  bool gq_compact(const Geo &g, const GateDesc &gd);                                                           \
  /* fused block (kind 4) applied in place to the decompressed slots; minmax: also each slot's min/max   */ \
  /* of the outputs (relative bound; only where dense_minmax_ok)                                         */ \
  void launch_dense_mfma(hipStream_t st, const Slots &sl, const Geo &g, int nslots, const GateDesc &gd,        \
                         const Ctl *ctl, bool minmax);                                                         \
  bool dense_minmax_ok(const Geo &g, const GateDesc &gd);                                                      \
  void launch_readout(hipStream_t st, const Slots &sl, const Geo &g, uint64_t first_amp, uint64_t count,       \
                      int probabilities, double *out);

namespace f64 {
CQ_AMPLITUDE_LAUNCHERS
// with_norm: 0 = a pass that builds an initial state, 1 = a gate pass,
// 2 = read-out only (scales without touching the pass counters), 3 = only
// count the records of the last batch written.  Every mode first counts
// the last batch.
// pw: the records' sum fields hold FP64 squared norms (pointwise-relative mode)
void launch_begin_pass(hipStream_t st, Ctl *ctl, const StateMeta &cur, uint64_t nslices, double *kscale,
                       int with_norm, bool pw = false);
void launch_reset_slots(hipStream_t st, const Slots &sl, int nslots);
void launch_rel_step(hipStream_t st, const Slots &sl, int nslots, double rel, const Ctl *ctl);
// nparts: partial results per slot written by the preceding gate_quant launch
// pw_nchunks: pointwise-relative mode, the slice's squared norm from its nchunks chunk sums (0: off)
void launch_codebook(hipStream_t st, const Slots &sl, const uint64_t *slot_slice, int nslots, const StateMeta &nxt,
                     uint32_t nparts, Ctl *ctl, uint32_t pw_nchunks = 0);
void launch_encode(hipStream_t st, const Slots &sl, const Geo &g, int nslots, const Ctl *ctl);
// SIM_OPT: the records of slices src[0..count) copied unchanged into the output
// arena as slices dst[...] (after the arena position), with their metadata
void launch_carry(hipStream_t st, Ctl *ctl, const StateMeta &cur, const StateMeta &nxt, const uint8_t *in,
                  uint8_t *out, uint64_t cap, const uint64_t *src, const uint64_t *dst, uint64_t count, uint64_t *off,
                  uint32_t pass);
// chunk runs of each slot of the batch (SIM_CHUNK_RUNS), between encode and finish
void launch_runs(hipStream_t st, const Slots &sl, const Geo &g, int nslots, const Ctl *ctl);
// records of the batch: offsets in the output arena, headers, symbol tables,
// chunk offsets, bit streams, per-slice metadata
void launch_finish(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                   const QuantParams &qp, uint8_t *arena, uint64_t arena_cap, const StateMeta &nxt, Ctl *ctl,
                   uint32_t pass);
}  // namespace f64

namespace f32 {
CQ_AMPLITUDE_LAUNCHERS
}  // namespace f32

// amplitudes per gate_quant tile (a power of two, at most L, a multiple of
// the chunk length); workgroups per slot and partial results per slot
inline uint64_t gq_tile(uint64_t L) { return L < 1024 ? L : 1024; }
constexpr uint32_t kGqWgs = 16;
constexpr uint32_t kMaxEncBlocks = 1024;  // encode (and finish) workgroups per slot, at most
constexpr uint32_t kMaxRuns = 4096;       // chunk runs of a record, at most
constexpr uint32_t kRunTile = 1024;       // chunks per workgroup of the runs kernels
constexpr uint32_t kGqParts = 2 * kGqWgs;

// words of one chunk's staging slot
inline uint32_t stage_words_for(int chunk_log2) {
  return (uint32_t)((((uint64_t)1 << chunk_log2) * (kLMax + kEscBits + 50) + 31) / 32 + 1);
}

// Sets the calling thread's sim_last_error() text; returns `code`.
int fail(int code, const char *msg);

}  // namespace cq
