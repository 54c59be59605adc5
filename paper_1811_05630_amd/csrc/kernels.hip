// Device kernels of libcqsim for gfx950 (CDNA4, 64-wide wavefronts).
//
// One pass of Algorithm 1 (Section II of the paper) over a batch of slices:
//   begin_pass  norm of the stored state -> normalisation scale per slice
//   decode      Decompress(S) + Normalize(S): canonical-Huffman decode with a
//               4096-entry LDS table, exact escapes, prefix sum inside each
//               chunk: the codes q, or a = q * (step * s); stores staged
//               through LDS so that every wavefront writes whole 128-byte lines
//   gate_quant  GateComputation(G, S) and the first half of Compress(S):
//               error-bounded quantisation, chunked Lorenzo difference,
//               symbols, escapes, histogram, exact sum of p^2
//   codebook    package-merge code lengths (limit 12), canonical codes, the
//               decoder table of the new record
//   encode      bit packing, most significant bit first, one wavefront per
//               chunk, packed per encode block into staging
//   finish      record sizes -> offsets in the output arena; record header,
//               symbol table, chunk word offsets and bit streams
// FP64 arithmetic is never contracted into FMAs (the pragma below), so every
// rounding happens exactly as in the stream definition.
//
// This file is compiled twice: as namespace f64, and with CQ_FP32 = 1 (from
// kernels_fp32.hip) as namespace f32, where every value of the working form
// and every result of the gate arithmetic is rounded to FP32 (rw below).  The
// kernels that do not compute amplitudes are built in f64 only.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include "cqsim_impl.h"

#ifndef CQ_FP32
#define CQ_FP32 0
#endif
#if CQ_FP32
#define CQ_PREC f32
#else
#define CQ_PREC f64
#endif

namespace cq {

#if !CQ_FP32
LaunchTimer &launch_timer() {
  static thread_local LaunchTimer t;
  return t;
}
#endif

namespace CQ_PREC {

// A value of the working form: FP64, or FP32 held in an FP64 register.  One
// FP64 +, - or * of two FP32 numbers rounded once to FP32 is the FP32 result
// itself (53 >= 2 * 24 + 2 bits make the double rounding innocuous), so the
// FP32 build computes FP32 arithmetic exactly by rounding every result.
__device__ __forceinline__ double rw(double x) { return CQ_FP32 ? (double)(float)x : x; }

// a launch that is being timed goes through the AMD launch call that records
// the thread's timing events at kernel start and end; other launches take the
// ordinary (cheaper) path
#define CQ_LAUNCH(K, G, B, S, ST, ...)                                                                    \
  do {                                                                                                    \
    if (launch_timer().start)                                                                             \
      hipExtLaunchKernelGGL(K, G, B, S, ST, launch_timer().start, launch_timer().stop, 0, __VA_ARGS__);   \
    else                                                                                                  \
      hipLaunchKernelGGL(K, G, B, S, ST, __VA_ARGS__);                                                    \
  } while (0)

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ void cmac(double ur, double ui, double ar, double ai, double &cr, double &ci) {
  // c += u * a with the fixed operation order of every gate
  double pr = rw(ur * ar);
  double pi = rw(ui * ai);
  double qr = rw(ur * ai);
  double qi = rw(ui * ar);
  cr = rw(cr + rw(pr - pi));
  ci = rw(ci + rw(qr + qi));
}

// u * a as the first term of a sum: equal to cmac from c = 0 except for the
// sign of an exact zero, which no quantisation code can see
__device__ __forceinline__ void cmul(double ur, double ui, double ar, double ai, double &cr, double &ci) {
  double pr = rw(ur * ar);
  double pi = rw(ui * ai);
  double qr = rw(ur * ai);
  double qi = rw(ui * ar);
  cr = rw(pr - pi);
  ci = rw(qr + qi);
}

__device__ __forceinline__ uint64_t zigzag(int64_t d) { return ((uint64_t)d << 1) ^ (uint64_t)(d >> 63); }
__device__ __forceinline__ int64_t unzigzag(uint64_t z) { return (int64_t)(z >> 1) ^ -(int64_t)(z & 1); }
__device__ __forceinline__ int bitlen64(uint64_t z) { return z ? 64 - __clzll((long long)z) : 0; }

__device__ __forceinline__ uint64_t dkey(double x) {
  // order-preserving map of FP64 to unsigned integers
  uint64_t b = (uint64_t)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_inv(uint64_t k) {
  uint64_t b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __longlong_as_double((long long)b);
}

__device__ __forceinline__ void fail(Ctl *ctl, uint32_t bit, uint32_t pass) {
  if (atomicOr(&ctl->flags, bit) == 0u) ctl->fail_pass = pass;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

// Workgroup barrier for phases that share only LDS: waits for this
// wavefront's LDS operations (s_waitcnt lgkmcnt(0)), not for its global loads
// and stores, so prefetched loads and earlier stores stay in flight.  The
// asm clobbers keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_sync() {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt and expcnt at their maximum, lgkmcnt 0
  __builtin_amdgcn_s_barrier();
  __asm__ __volatile__("" ::: "memory");
}

// inclusive scan of a u32 over one (full) wavefront with DPP: a scan inside
// every row of 16 lanes (shifts by 1, 2, 4 and 8, lanes shifted in from
// outside the row read 0), then lane 15 of each row added to the next row
// (rows 1 and 3) and lane 31 added to rows 2 and 3
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111 /* row_shr:1 */, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112 /* row_shr:2 */, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114 /* row_shr:4 */, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118 /* row_shr:8 */, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142 /* row_bcast:15 */, 0xA, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143 /* row_bcast:31 */, 0xC, 0xF, false);
  return x;
}

// exclusive scan of one u32 per thread over a block of up to 1024 threads
// (whole wavefronts); returns the prefix, *total gets the block sum.
__device__ uint32_t block_excl_scan(uint32_t x, uint32_t *scratch, uint32_t *total) {
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t nw = (blockDim.x + 63) >> 6;
  uint32_t inc = wave_incl_scan(x);
  if (lane == 63) scratch[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t w = 0; w < nw; w++) {
      uint32_t t = scratch[w];
      scratch[w] = run;
      run += t;
    }
    scratch[16] = run;
  }
  __syncthreads();
  uint32_t r = scratch[wave] + inc - x;
  *total = scratch[16];
  __syncthreads();
  return r;
}

// block-wide sum of a u64 (whole wavefronts, up to 16 of them)
__device__ uint64_t block_sum64(uint64_t x, uint64_t *scratch) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  if (lane_id() == 0) scratch[threadIdx.x >> 6] = x;
  __syncthreads();
  uint64_t t = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; w++) t += scratch[w];
  __syncthreads();
  return t;
}

__device__ __forceinline__ uint64_t rec_bytes(uint32_t n_used, uint32_t nchunks, uint32_t words) {
  return (uint64_t)kHdr + ((2ull * n_used + 3) & ~3ull) + 4ull * (nchunks + 1) + 4ull * words;
}

__device__ __forceinline__ uint32_t ld32(const uint8_t *p) { return *(const uint32_t *)p; }

#if !CQ_FP32  // kernels that do not compute amplitudes: f64 build only
// ----------------------------------------------------------- begin pass

// The records of the last batch are counted by the launch that starts the
// next batch or pass (the batch's own workgroups all read the arena position
// it started from, so none of them may move it).
__device__ __forceinline__ void settle(Ctl *ctl) {
  ctl->bump += ctl->pending_bump;
  ctl->cur_bytes += ctl->pending_bytes;
  ctl->pending_bump = 0;
  ctl->pending_bytes = 0;
}

// A slice's term of N: step^2 x its exact sum p^2, or (pointwise-relative
// records) the FP64 squared norm its sum field holds.
__device__ __forceinline__ double norm_leaf(const double *step, const uint64_t *sq, uint64_t j, bool pw) {
  if (pw) return __longlong_as_double((long long)sq[2 * j]);
  double s = step[j];
  double p = (double)sq[2 * j + 1] * 0x1p64 + (double)sq[2 * j];
  return (s * s) * p;
}

// Pairwise sum of `b` (a power of two) consecutive leaves: the same balanced
// tree as adding neighbours level by level.
__device__ double pairwise_block(const double *step, const uint64_t *sq, uint64_t first, uint64_t b, bool pw) {
  double stk[48];
  int top = 0;
  for (uint64_t i = 0; i < b; i++) {
    double v = norm_leaf(step, sq, first + i, pw);
    uint64_t k = i;
    while (k & 1) {
      v = stk[--top] + v;
      k >>= 1;
    }
    stk[top++] = v;
  }
  return stk[0];
}

__global__ void __launch_bounds__(1024) k_begin_pass(Ctl *ctl, const double *step, const uint64_t *sq, uint64_t S,
                                                     double *kscale, int with_norm, int pw) {
  if (ctl->flags) return;
  __shared__ double part[1024];
  __shared__ double s_sh;
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  if (tid == 0) settle(ctl);
  if ((with_norm == 0 || with_norm == 1) && tid == 0) {  // a pass starts writing the other arena
    if (ctl->cur_bytes > ctl->peak_bytes) ctl->peak_bytes = ctl->cur_bytes;
    ctl->bump = 0;
    ctl->cur_bytes = 0;
    ctl->wide = ctl->wide_next;  // the codes this pass decodes came from the last quantisation
    ctl->wide_next = 0;
  }
  if (with_norm == 0 || with_norm == 3) return;
  uint64_t active;
  if (S <= T) {
    part[tid] = tid < S ? norm_leaf(step, sq, tid, pw) : 0.0;
    active = S;
  } else {
    uint64_t b = S / T;
    part[tid] = pairwise_block(step, sq, (uint64_t)tid * b, b, pw);
    active = T;
  }
  __syncthreads();
  for (uint64_t m = active; m > 1; m >>= 1) {
    double v = 0.0;
    if (tid < m / 2) v = part[2 * tid] + part[2 * tid + 1];
    __syncthreads();
    if (tid < m / 2) part[tid] = v;
    __syncthreads();
  }
  if (tid == 0) {
    double N = part[0];
    double h = 0.5 * N;  // 1/sqrt(N): ten Newton steps from 1
    double y = 1.0;
    for (int k = 0; k < 10; k++) {
      double t = h * y;
      t = t * y;
      t = 1.5 - t;
      y = y * t;
    }
    if (with_norm == 1) {
      ctl->N = N;
      ctl->s = y;
    }
    s_sh = y;
  }
  __syncthreads();
  for (uint64_t j = tid; j < S; j += T) kscale[j] = step[j] * s_sh;
}

// zero every per-slot accumulator (creation and recovery after a failure)
__global__ void k_reset_slots(Slots sl, int nslots) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (uint64_t)nslots * kGqParts * kNSym) sl.hpart[i] = 0;
  if (i < (uint64_t)nslots * kGqParts * 4) sl.part[i] = 0;
  if (i < (uint64_t)nslots) {
    sl.sq[2 * i] = 0;
    sl.sq[2 * i + 1] = 0;
    sl.nesc[i] = 0;
    sl.words[i] = 0;
    sl.minmax[2 * i] = ~0ull;
    sl.minmax[2 * i + 1] = 0ull;
  }
}

#endif  // !CQ_FP32

// ------------------------------------------------------------------ init

__global__ void k_init(Slots sl, Geo g, const uint64_t *slot_slice, uint64_t total, int kind, uint64_t x,
                       const double *f, const Ctl *ctl) {
  if (ctl->flags) return;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint64_t u = i >> g.slice_log2, o = i & (g.L - 1);
  const uint64_t gi = (slot_slice[u] << g.slice_log2) | o;
  double re = 0.0, im = 0.0;
  if (kind == 0) {
    re = gi == 0 ? 1.0 : 0.0;
  } else if (kind == 1) {
    re = gi == x ? 1.0 : 0.0;
  } else {
    double ar = 1.0, ai = 0.0;
    for (int q = 0; q < g.n; q++) {
      int b = (int)((gi >> q) & 1);
      double cr = 0.0, ci = 0.0;
      cmac(f[4 * q + 2 * b], f[4 * q + 2 * b + 1], ar, ai, cr, ci);
      ar = cr;
      ai = ci;
    }
    re = ar;
    im = ai;
  }
  double *w = sl.ws + u * 2 * g.L;
  w[o] = re;
  w[g.L + o] = im;
}

// ------------------------------------------------------------------ decode
// One lane per chunk: the lane walks its chunk's bit stream serially (12-bit
// peek into the decoder table, escapes carry the exact difference) and keeps
// the running sum p.  It writes the FP64 value a = p * k, or in a compact
// workspace the int32 code p itself.  Four wavefronts share one decoder
// table.  Values go out in rounds through an LDS tile (16 FP64 or 32 int32
// values per lane and round), so that every store instruction writes whole
// 128-byte lines.
// Stream words come from a per-lane LDS slot that holds the next PF words of
// the chunk, loaded while the previous round's values were being stored: the
// loads are issued before those stores, so waiting for them never waits for
// the stores (one in-order counter covers both on CDNA).  A round that needs
// more words than the slot holds reads them from global memory.

constexpr int kDecWaves = 4;       // wavefronts per workgroup

// Two decoder configurations.  The wide one, for passes that decode FP64
// values (relative and pointwise-relative bounds, fused blocks), stages 16
// FP64 values per lane and round and prefetches up to 12 words; its 63.5 KB
// of LDS per workgroup allow two workgroups per CU.  The narrow one, for
// passes that decode int32 codes, stages 32 codes per round and prefetches 4
// words (53 KB): three workgroups per CU, more chains to hide the table
// lookups' latency.  Its FP64 fallback (a pass whose codes may not fit int32)
// stages 8 values per round.
template <bool SMALL>
struct DecCfg {
  static constexpr int kPfMax = SMALL ? 4 : 12;                    // largest slot (words per lane)
  static constexpr int kStage = SMALL ? 64 * 33 * 4 : 64 * 17 * 8;  // tile bytes per wavefront, rows padded
};

// The running sum p: FP64 (exact below 2^53) for the FP64 workspace; for
// the compact one, whose codes all lie below 2^31 in magnitude, uint32
// arithmetic modulo 2^32, which is exact for every partial sum as each of
// them is such a code (an escaped difference may be larger, its sum is not).
template <bool C32, bool SMALL = false>
struct DecFmt {  // FP64 workspace
  using T = double;
  using P = double;
  static constexpr int R = SMALL ? 8 : 16, PITCH = R + 1, PF = SMALL ? 4 : 8;
  static __device__ __forceinline__ double add(double p, int d) { return p + (double)d; }
  static __device__ __forceinline__ double add_esc(double p, int64_t d) { return p + (double)d; }
  static __device__ __forceinline__ double val(double p, double k) { return rw(p * k); }
};
template <bool SMALL>
struct DecFmt<true, SMALL> {  // compact workspace: the code itself
  using T = int32_t;
  using P = uint32_t;
  static constexpr int R = 32, PITCH = 33, PF = SMALL ? 4 : 12;
  static __device__ __forceinline__ uint32_t add(uint32_t p, int d) { return p + (uint32_t)d; }
  static __device__ __forceinline__ uint32_t add_esc(uint32_t p, int64_t d) { return p + (uint32_t)(uint64_t)d; }
  static __device__ __forceinline__ int32_t val(uint32_t p, double) { return (int32_t)p; }
};
template <bool SMALL>
constexpr bool dec_fits() {
  return 64 * DecFmt<true, SMALL>::PITCH * 4 <= DecCfg<SMALL>::kStage &&
         64 * DecFmt<false, SMALL>::PITCH * 8 <= DecCfg<SMALL>::kStage &&
         DecFmt<true, SMALL>::PF <= DecCfg<SMALL>::kPfMax && DecFmt<false, SMALL>::PF <= DecCfg<SMALL>::kPfMax;
}
static_assert(dec_fits<false>() && dec_fits<true>(), "tile and slot sizes");

template <int PF>
struct BitReader {
  const uint32_t *w;  // the chunk's words (global)
  uint32_t nw;        // number of words
  uint32_t wi;        // next word to enter buf
  uint32_t wbase;     // first word held in the LDS slot
  uint64_t buf;       // bits not yet consumed, most significant first
  int nbits;
  __device__ __forceinline__ void refill(const uint32_t (*pf)[64 * kDecWaves], uint32_t tid) {
    while (nbits <= 32) {
      uint32_t word = 0;
      const uint32_t d = wi - wbase;
      if (wi < nw) {
        if (d < (uint32_t)PF) {
          word = pf[d][tid];
        } else {  // past the prefetched words: wait for this load here, so
                  // that the common path after the join waits for LDS only
          word = w[wi];
          __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        }
      }
      buf |= (uint64_t)word << (32 - nbits);
      nbits += 32;
      wi++;
    }
  }
  // one word when at most 32 bits are left: a step consumes at most kLMax
  // bits, so calling this before every step keeps at least 20 in buf
  __device__ __forceinline__ void refill1(const uint32_t (*pf)[64 * kDecWaves], uint32_t tid) {
    if (nbits <= 32) {
      const uint32_t d = wi - wbase;
      uint32_t word;
      if (d < (uint32_t)PF) {  // past the chunk's end the slot holds words that are never consumed
        word = pf[d][tid];
      } else {
        word = wi < nw ? w[wi] : 0u;
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), as in refill
      }
      buf |= (uint64_t)word << (32 - nbits);
      nbits += 32;
      wi++;
    }
  }
  __device__ __forceinline__ uint64_t take(int n) {  // 0 <= n <= 32, needs nbits >= n
    if (n == 0) return 0;
    uint64_t v = buf >> (64 - n);
    buf <<= n;
    nbits -= n;
    return v;
  }
};

// The chunks of one workgroup (after the record checks).  FULL: chunks of at
// least 32 values and a whole number of workgroups of chunks per slot (every
// lane active, whole rounds).  FMT: the records may hold zero chunks (bit 0)
// or constant chunks (bit 1).
// The value of a pointwise-relative code q (an integer held in a double):
// the bit pattern |q| << (52 - b) with q's sign.
__device__ __forceinline__ double pw_value(double q, int b) {
  const uint64_t m = (uint64_t)fabs(q) << (52 - b);
  const double x = __longlong_as_double((long long)m);
  return q < 0.0 ? -x : x;
}

// A decoded value: the code itself (compact workspace), else p k, or (PW:
// records of pointwise-relative codes) the pointwise-relative value of p
// times k.  PW is a template parameter of the decode kernels, so that the
// other FP64 loops carry no trace of it.
template <bool C32, bool PW>
__device__ __forceinline__ typename DecFmt<C32>::T dec_val(typename DecFmt<C32>::P p, double k, int pwb) {
  if constexpr (C32 || !PW) {
    return DecFmt<C32>::val(p, k);
  } else {
    return rw(pw_value(p, pwb) * k);
  }
}

template <bool FULL, bool C32, int FMT, bool SMALL, bool PW>
__device__ __forceinline__ void decode_chunks(const Slots &sl, const Geo &g, const StateMeta &cur, uint64_t slice,
                                              uint32_t u, const uint32_t *offs, uint32_t nchunks, uint32_t n_words,
                                              uint32_t n_used, uint32_t nruns, double k, uint32_t *dtab,
                                              uint8_t *stg, uint32_t (*pf)[64 * kDecWaves], Ctl *ctl,
                                              uint32_t pass) {
  using F = DecFmt<C32, SMALL>;
  using T = typename F::T;
  constexpr int PF = F::PF, RMAX = F::R, PITCH = F::PITCH;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
  const uint32_t c0 = (blockIdx.x * kDecWaves + wave) * 64u;  // first chunk of this wavefront
  const uint32_t c = c0 + lane;
  const bool active = FULL || c < nchunks;
  BitReader<PF> br;
  uint32_t w0 = 0;
  br.nw = 0;
  constexpr bool ZC = (FMT & 1) != 0, CC = (FMT & 2) != 0;
  bool cconst = false;  // a constant chunk: its head, then the zero difference
  const uint32_t *stream = offs + (nchunks + 1);  // the bit stream
  if (active) {
    uint32_t w1;
    if (nruns) {  // chunk runs: the run holding chunk c, by binary search over the run ends
      const uint32_t *ends = offs + 1, *wo = offs + 1 + nruns;
      uint32_t lo = 0, hi = nruns - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ends[mid] > c)
          hi = mid;
        else
          lo = mid + 1;
      }
      w0 = wo[lo];
      w1 = wo[lo + 1];
      stream = wo + nruns + 1;
    } else {
      w0 = offs[c];
      w1 = offs[c + 1];
    }
    if (CC) {
      cconst = (w0 >> 31) != 0;
      w0 &= 0x7FFFFFFFu;
      w1 &= 0x7FFFFFFFu;
    }
    if (w1 < w0 || w1 > n_words) {
      fail(ctl, kFlagCorrupt, pass);
      w0 = 0;
    } else {
      br.nw = w1 - w0;
    }
  }
  // an empty chunk under a code of two or more symbols is a zero chunk (a
  // one-symbol code has no bits: its chunks are empty and decode normally)
  const bool zero = ZC && active && !cconst && br.nw == 0 && n_used > 1;
  constexpr uint32_t kZeroPair = (uint32_t)kR | ((uint32_t)kR << 14) | (1u << 28);  // dtab_entry(R, 0, R, 0, true)
  br.w = stream + w0;
  br.wi = 0;
  br.buf = 0;
  br.nbits = 0;
  // words [from, from + PF) of the chunk; the address of a word past the
  // end is replaced by a valid one (the load is always issued)
  uint32_t nx[PF];
  auto prefetch = [&](uint32_t from) {
#pragma unroll
    for (int i = 0; i < PF; i++) nx[i] = *(from + i < br.nw ? br.w + from + i : offs);
  };
  auto to_slot = [&]() {
    br.wbase = br.wi;
#pragma unroll
    for (int i = 0; i < PF; i++) pf[i][tid] = nx[i];  // words past the chunk's end are never read
  };
  prefetch(0);
  __syncthreads();  // decoder table in LDS
  to_slot();
  const uint64_t B = 1ull << g.chunk_log2;
  const uint32_t R = FULL ? (uint32_t)RMAX : (B < (uint64_t)RMAX ? (uint32_t)B : (uint32_t)RMAX);
  T *out = (T *)(sl.ws + (uint64_t)u * 2 * g.L);
  T *st = (T *)(stg + wave * DecCfg<SMALL>::kStage);
  typename F::P p = 0;  // running sum
  // nothing is in flight when the rounds start, so no load issued here is
  // waited for inside them (where a wait would also wait for the stores)
  __builtin_amdgcn_s_waitcnt(0);
  for (uint64_t j0 = 0; j0 < B; j0 += R) {
    if (active) {
      for (uint32_t q = 0; q < R;) {
        br.refill1(pf, tid);
        // a zero chunk reads two zero differences of no bits per step, and
        // so does a constant chunk after its head
        const bool fill = (ZC && zero) || (CC && cconst && (j0 > 0 || q > 0));
        const uint32_t e = fill ? kZeroPair : dtab[(uint32_t)(br.buf >> (64 - kLMax))];
        const uint32_t sym = e & 1023u;
        if (sym == 0) {  // escape (never part of a two-symbol entry)
          const uint32_t len = (e >> 10) & 15u;
          br.buf <<= len;
          br.nbits -= (int)len;
          if (br.nbits < kEscBits) br.refill(pf, tid);
          const int nb = (int)br.take(kEscBits);
          uint64_t z;
          if (nb > 32) {
            if (br.nbits < 32) br.refill(pf, tid);
            const uint64_t hi = br.take(nb - 32);
            if (br.nbits < 32) br.refill(pf, tid);
            z = (hi << 32) | br.take(32);
          } else {
            if (br.nbits < nb) br.refill(pf, tid);
            z = br.take(nb);
          }
          p = F::add_esc(p, unzigzag(z));
          st[lane * PITCH + q] = dec_val<C32, PW>(p, k, g.pw_bits);
          q++;
          continue;
        }
        // one or two symbols on one path for every lane; the second value
        // is written in any case (at q + 1 <= R, inside the padded row) and
        // overwritten later when it was not decoded
        const bool two = (e >> 28) && q + 1 < R && !(CC && cconst && j0 == 0 && q == 0);  // a lone head
        const uint32_t len = ((e >> 10) & 15u) + (two ? ((e >> 24) & 15u) : 0u);
        br.buf <<= len;
        br.nbits -= (int)len;
        p = F::add(p, (int)sym - kR);
        st[lane * PITCH + q] = dec_val<C32, PW>(p, k, g.pw_bits);
        const typename F::P p2 = F::add(p, (int)((e >> 14) & 1023u) - kR);
        st[lane * PITCH + q + 1] = dec_val<C32, PW>(p2, k, g.pw_bits);
        p = two ? p2 : p;
        q += two ? 2u : 1u;
      }
    }
    prefetch(br.wi);  // the next round's words, ahead of this round's stores
    // the tile is private to the wavefront: its LDS operations complete in
    // order, so waiting for them is enough before other lanes read
    __asm__ __volatile__("s_waitcnt lgkmcnt(0)" ::: "memory");
    // streaming stores: the workspace is read once, by the next kernel, and
    // is larger than the L2 caches
    if (FULL) {
#pragma unroll
      for (int i = 0; i < RMAX; i++) {
        const uint32_t idx = (uint32_t)i * 64u + lane, row = idx / RMAX, col = idx % RMAX;
        __builtin_nontemporal_store(st[row * PITCH + col], &out[(uint64_t)(c0 + row) * B + j0 + col]);
      }
    } else {
      for (uint32_t idx = lane; idx < 64u * R; idx += 64u) {
        const uint32_t row = idx / R, col = idx % R;
        if (c0 + row < nchunks)
          __builtin_nontemporal_store(st[row * PITCH + col], &out[(uint64_t)(c0 + row) * B + j0 + col]);
      }
    }
    // the next round's slot; its words were loaded before the stores above,
    // so the wait for them leaves the stores in flight
    to_slot();
    __asm__ __volatile__("s_waitcnt lgkmcnt(0)" ::: "memory");  // tile read before the next round writes it
  }
}

// SMALL: the narrow configuration (launched for passes that may decode int32
// codes); PW: records of pointwise-relative codes
template <bool FULL, int FMT, bool SMALL, bool PW>
__global__ void __launch_bounds__(64 * kDecWaves, SMALL ? 3 : 1) k_decode(Slots sl, Geo g, const uint64_t *slot_slice,
                                                                       const uint8_t *arena, StateMeta cur,
                                                                       const double *kscale, Ctl *ctl, uint32_t pass,
                                                                       int compact_ok) {
  if (ctl->flags) return;
  // compact workspace: the int32 codes q themselves (every |q| < 2^31), the
  // gate kernel multiplies by the slice's scale; else the FP64 values q * k
  const bool c32 = compact_ok && !ctl->wide;
  __shared__ __align__(16) uint32_t dtab[1 << kLMax];
  __shared__ __align__(16) uint8_t stg[kDecWaves * DecCfg<SMALL>::kStage];
  __shared__ uint32_t pf[DecCfg<SMALL>::kPfMax][64 * kDecWaves];
  const uint32_t u = blockIdx.y, tid = threadIdx.x;
  const uint64_t slice = slot_slice[u];
  // the slice's decoder table (16 KiB, its own buffer): its loads go out
  // with the record header's, and reach LDS before decode_chunks' barrier
  constexpr uint32_t kT = 64 * kDecWaves, kN = (1u << kLMax) / 4 / kT;
  static_assert(kN * kT == (1u << kLMax) / 4, "whole uint4 rows per thread");
  uint4 dt[kN];
  {
    const uint4 *src = (const uint4 *)(cur.dtab + slice * (1u << kLMax));
#pragma unroll
    for (uint32_t k = 0; k < kN; k++) dt[k] = src[tid + k * kT];
  }
  const uint8_t *rec = arena + cur.rec_off[slice];
  const uint32_t n_used = ld32(rec + 12);
  const uint32_t nchunks = ld32(rec + 16);
  const uint32_t n_words = ld32(rec + 20);
  if (ld32(rec) != kMagic || n_used < 1 || n_used > (uint32_t)kNSym || nchunks != g.nchunks ||
      ld32(rec + 8) != (uint32_t)g.chunk_log2) {
    if (tid == 0) fail(ctl, kFlagCorrupt, pass);
    return;
  }
#pragma unroll
  for (uint32_t k = 0; k < kN; k++) ((uint4 *)dtab)[tid + k * kT] = dt[k];
  const uint32_t sym_bytes = (2 * n_used + 3) & ~3u;
  const uint32_t *offs = (const uint32_t *)(rec + kHdr + sym_bytes);
  // chunk runs (flags bit 3): the table starts with the number of runs
  const uint32_t nruns = (ld32(rec + 56) & 8u) ? offs[0] : 0u;
  if ((ld32(rec + 56) & 8u) && (nruns < 1 || nruns > nchunks || nruns > kMaxRuns)) {
    if (tid == 0) fail(ctl, kFlagCorrupt, pass);
    return;
  }
  if (c32)
    decode_chunks<FULL, true, FMT, SMALL, false>(sl, g, cur, slice, u, offs, nchunks, n_words, n_used, nruns, 0.0, dtab,
                                          stg, pf, ctl, pass);
  else
    decode_chunks<FULL, false, FMT, SMALL, PW>(sl, g, cur, slice, u, offs, nchunks, n_words, n_used, nruns,
                                           kscale[slice], dtab, stg, pf, ctl, pass);
}

// ------------------------------------------------------------ gate + quantise

// Output amplitude (re, im) of the gate at slot u, offset o.
// KIND: 0 identity, 1 dense on one target, 2 phase, 3 dense on 2..5 targets.
template <int KIND>
__device__ __forceinline__ void eval_amp(const double *__restrict__ ws, const Geo &g, const uint64_t *slot_slice,
                                         const GateDesc &gd, uint32_t u, uint64_t o, double &re, double &im) {
  const uint64_t twoL = 2 * g.L;
  const double *w = ws + (uint64_t)u * twoL;
  if (KIND == 0) {
    re = w[o];
    im = w[g.L + o];
    return;
  }
  const uint64_t gi = (slot_slice[u] << g.slice_log2) | o;
  if ((gi & gd.ctrl_mask) != gd.ctrl_vals) {
    re = w[o];
    im = w[g.L + o];
    return;
  }
  if (KIND == 2) {
    double cr = 0.0, ci = 0.0;
    cmac(gd.ph_re, gd.ph_im, w[o], w[g.L + o], cr, ci);
    re = cr;
    im = ci;
    return;
  }
  const uint32_t mm = (1u << gd.m) - 1u;
  const uint32_t gbase = u & ~mm;
  const uint64_t gl = ((uint64_t)(u & mm) << g.slice_log2) | o;
  if (KIND == 1) {
    const int t = gd.tloc[0];
    const uint64_t g0 = gl & ~(1ull << t), g1 = g0 | (1ull << t);
    const double *w0 = ws + (uint64_t)(gbase + (uint32_t)(g0 >> g.slice_log2)) * twoL;
    const double *w1 = ws + (uint64_t)(gbase + (uint32_t)(g1 >> g.slice_log2)) * twoL;
    const uint64_t o0 = g0 & (g.L - 1), o1 = g1 & (g.L - 1);
    const bool row = (gl >> t) & 1;
    const double u0r = row ? gd.m2[4] : gd.m2[0], u0i = row ? gd.m2[5] : gd.m2[1];
    const double u1r = row ? gd.m2[6] : gd.m2[2], u1i = row ? gd.m2[7] : gd.m2[3];
    double cr = 0.0, ci = 0.0;
    cmac(u0r, u0i, w0[o0], w0[g.L + o0], cr, ci);
    cmac(u1r, u1i, w1[o1], w1[g.L + o1], cr, ci);
    re = cr;
    im = ci;
    return;
  }
  int row = 0;
  for (int t = 0; t < gd.k; t++) row |= (int)((gl >> gd.tloc[t]) & 1) << t;
  const uint64_t bl = gl & ~gd.tmask_loc;
  const int dim = 1 << gd.k;
  const double *mrow = gd.mat + 2 * (row * dim);
  double cr = 0.0, ci = 0.0;
  for (int c = 0; c < dim; c++) {
    const uint64_t glc = bl | gd.dep[c];
    const double *wc = ws + (uint64_t)(gbase + (uint32_t)(glc >> g.slice_log2)) * twoL;
    const uint64_t oc = glc & (g.L - 1);
    cmac(mrow[2 * c], mrow[2 * c + 1], wc[oc], wc[g.L + oc], cr, ci);
  }
  re = cr;
  im = ci;
}

// q = rint(v / step) as an integer-valued double; false if |q| >= 2^48 or
// the reconstruction q * step misses v by more than the bound.
__device__ __forceinline__ bool quantise(double v, double step, double recip, double ebj, double &q, double &err) {
  double t = v * recip;
  q = rint(t);
  if (!(fabs(q) < kPMax)) {
    q = 0.0;
    err = 0.0;
    return false;
  }
  double back = q * step;
  err = fabs(v - back);
  return err <= ebj;
}

// Pointwise-relative bound: v rounded to b mantissa bits (half to even on its
// bit pattern); q = the rounded bit pattern without the sign, shifted right by
// 52 - b, with v's sign; back = the stored value.  False if v is not finite
// (or rounds to infinity) or |v - back| > eb |v|.
__device__ __forceinline__ bool quantise_pw(double v, int b, double eb, double &q, double &err, double &back) {
  const uint64_t bits = (uint64_t)__double_as_longlong(v);
  const uint64_t mag = bits & 0x7FFFFFFFFFFFFFFFull;
  const int sh = 52 - b;
  const uint64_t half = 1ull << (sh - 1);
  const uint64_t c = (mag + (half - 1) + ((mag >> sh) & 1)) >> sh;
  if (c >= (2047ull << b)) {
    q = 0.0;
    err = 0.0;
    back = 0.0;
    return false;
  }
  const double x = __longlong_as_double((long long)(c << sh));
  const bool neg = (bits >> 63) != 0;
  back = neg ? -x : x;
  q = neg ? -(double)c : (double)c;
  err = fabs(v - back);
  return err <= eb * fabs(v);
}

// Pairwise sum of b (a power of two) consecutive values: the same balanced
// tree as adding neighbours level by level.
__device__ double tree_sum(const double *x, uint64_t first, uint64_t b) {
  double stk[48];
  int top = 0;
  for (uint64_t i = 0; i < b; i++) {
    double v = x[first + i];
    uint64_t k = i;
    while (k & 1) {
      v = stk[--top] + v;
      k >>= 1;
    }
    stk[top++] = v;
  }
  return stk[0];
}

// relative bound: min/max of the gate's output over every slot.  Workgroup
// (x, u) of G per slot takes amplitudes x * T + tid, stepping by G * T,
// reduces them, and adds its result with one atomic per workgroup (the
// keys are order-preserving integers, so min/max are exact).
template <int KIND>
__global__ void __launch_bounds__(256) k_gate_minmax(Slots sl, Geo g, const uint64_t *slot_slice, GateDesc gd,
                                                     const Ctl *ctl) {
  if (ctl->flags) return;
  const uint32_t u = blockIdx.y, T = blockDim.x;
  uint64_t kmin = ~0ull, kmax = 0ull;
  for (uint64_t o = (uint64_t)blockIdx.x * T + threadIdx.x; o < g.L; o += (uint64_t)gridDim.x * T) {
    double re, im;
    eval_amp<KIND>(sl.ws, g, slot_slice, gd, u, o, re, im);
    const uint64_t a = dkey(re), b = dkey(im);
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    kmin = lo < kmin ? lo : kmin;
    kmax = hi > kmax ? hi : kmax;
  }
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t a = __shfl_xor(kmin, off, 64), b = __shfl_xor(kmax, off, 64);
    kmin = a < kmin ? a : kmin;
    kmax = b > kmax ? b : kmax;
  }
  __shared__ uint64_t smin[4], smax[4];
  if (lane_id() == 0) {
    smin[threadIdx.x >> 6] = kmin;
    smax[threadIdx.x >> 6] = kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < T / 64; w++) {
      kmin = smin[w] < kmin ? smin[w] : kmin;
      kmax = smax[w] > kmax ? smax[w] : kmax;
    }
    atomicMin((unsigned long long *)&sl.minmax[2 * u], (unsigned long long)kmin);
    atomicMax((unsigned long long *)&sl.minmax[2 * u + 1], (unsigned long long)kmax);
  }
}

// relative bound: eb_j = rel * max(max - min, 2^-24 max|a|); step = largest
// power of two <= 2 eb_j (1 when eb_j is 0)
#if !CQ_FP32
__global__ void k_rel_step(Slots sl, int nslots, double rel, const Ctl *ctl) {
  if (ctl->flags) return;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nslots) return;
  double lo = dkey_inv(sl.minmax[2 * u]), hi = dkey_inv(sl.minmax[2 * u + 1]);
  sl.minmax[2 * u] = ~0ull;  // consumed
  sl.minmax[2 * u + 1] = 0ull;
  double range = hi - lo;
  double m = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
  double fl = m * 0x1p-24;
  double e = rel * (range > fl ? range : fl);
  double step = 1.0, recip = 1.0;
  if (e > 0.0) {
    int ex;
    frexp(2.0 * e, &ex);
    step = ldexp(1.0, ex - 1);
    recip = ldexp(1.0, 1 - ex);
  }
  sl.qstep[3 * u] = step;
  sl.qstep[3 * u + 1] = recip;
  sl.qstep[3 * u + 2] = e;
}
#endif  // !CQ_FP32

// Sum of q^2 over a thread's integer-valued doubles |q| < 2^48, added to a
// 128-bit (lo, hi) sum.  When every value of the wavefront is below 2^31 the
// squares come from 32-bit multiplies; otherwise from 64-bit ones.
template <int V>
__device__ __forceinline__ void add_squares(const double (&qr)[V], const double (&qi)[V], uint64_t &lo,
                                            uint64_t &hi) {
  bool small = true;
#pragma unroll
  for (int v = 0; v < V; v++) small = small && fabs(qr[v]) < 2147483648.0 && fabs(qi[v]) < 2147483648.0;
  if (__ballot(!small) == 0) {
#pragma unroll
    for (int v = 0; v < V; v++) {
      const uint32_t a = (uint32_t)abs((int)qr[v]), b = (uint32_t)abs((int)qi[v]);
      const uint64_t s = (uint64_t)a * a, t = (uint64_t)b * b;
      uint64_t x = lo + s;
      hi += x < lo;
      lo = x + t;
      hi += lo < x;
    }
  } else {
#pragma unroll
    for (int v = 0; v < V; v++) {
      const uint64_t a = (uint64_t)fabs(qr[v]), b = (uint64_t)fabs(qi[v]);
      uint64_t x = lo + a * a;
      hi += __umul64hi(a, a) + (x < lo);
      lo = x + b * b;
      hi += __umul64hi(b, b) + (lo < x);
    }
  }
}

// Per-slot output pointers of gate_quant.
struct SlotOut {
  uint16_t *symr, *symi;
  int64_t *escr, *esci;
};

__device__ __forceinline__ SlotOut slot_out(const Slots &sl, const Geo &g, uint32_t u) {
  SlotOut t;
  t.symr = sl.sym + (uint64_t)u * 2 * g.L;
  t.symi = t.symr + g.L;
  t.escr = sl.esc + (uint64_t)u * 2 * g.L;
  t.esci = t.escr + g.L;
  return t;
}

// ------------------------------------------------ buffer memory operations
// The gate kernels address slot memory through buffer resources: a
// descriptor in scalar registers plus a 32-bit offset per lane, so that no
// 64-bit address arithmetic runs per lane, and an access past the
// descriptor's size is dropped by the hardware (reads return zero).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufWord3 = 0x00020000;  // descriptor word 3 for untyped 32-bit access on gfx9-family chips

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufWord3);
}
__device__ __forceinline__ double buf_ld_f64(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return __longlong_as_double((long long)(((uint64_t)x.y << 32) | x.x));
}
__device__ __forceinline__ void buf_st_u16(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, off, 0, 0);
}
__device__ __forceinline__ void buf_st_i64(__amdgpu_buffer_rsrc_t r, uint32_t off, int64_t v) {
  u32x2 x;
  x.x = (uint32_t)(uint64_t)v;
  x.y = (uint32_t)((uint64_t)v >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(x, r, off, 0, 0);
}

// Escape buffer layout.  gate_quant writes each escaped difference to the
// escape buffer and encode reads it back.  Within every aligned group of
// G = min(B, 256) positions of a plane (B the chunk length) the group's
// escapes fill its first entries, in position order, so that sparse escapes
// touch few cache lines (a scattered 8-byte store makes the memory read and
// rewrite its whole line).
__device__ __forceinline__ uint32_t esc_group(const Geo &g) { return g.chunk_log2 < 8 ? 1u << g.chunk_log2 : 256u; }

// set bits of m in the lanes below this one
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// set bits of m in the lanes below this one inside its aligned segment of G < 64 lanes
__device__ __forceinline__ uint32_t seg_below(uint64_t m, uint32_t G) {
  const uint32_t lane = lane_id();
  const uint64_t before_seg = (1ull << (lane & ~(G - 1))) - 1;
  return (uint32_t)__popcll(m & ((1ull << lane) - 1) & ~before_seg);
}

// Escapes of a tile whose element e = v * T + tid sits at position ob + e
// (T = 64 nwv threads, ob a multiple of G): the escape's rank in its group
// counts the group's escapes in earlier rows and wavefronts (through cnt in
// LDS, written before a workgroup barrier and read after it) and in lower
// lanes.  Step 1, before the barrier: each wavefront's counts per row.
template <int V>
__device__ __forceinline__ void esc_count_tile(const bool (&er)[V], const bool (&ei)[V], uint32_t G, uint32_t *cnt) {
  const uint32_t wave = threadIdx.x >> 6, nwv = blockDim.x >> 6;
#pragma unroll
  for (int v = 0; v < V; v++) {
    const uint64_t mr = __ballot(er[v]), mi = __ballot(ei[v]);
    if (G >= 64 && lane_id() == 0) {
      cnt[2 * (v * nwv + wave)] = (uint32_t)__popcll(mr);
      cnt[2 * (v * nwv + wave) + 1] = (uint32_t)__popcll(mi);
    }
  }
}
// Step 2, after the barrier: ranks and stores, through a buffer resource
// over the slot's escape buffer (re plane, then im plane of L entries each).
template <int V>
__device__ __forceinline__ void esc_store_tile(const bool (&er)[V], const bool (&ei)[V], const int64_t (&dr)[V],
                                               const int64_t (&di)[V], uint32_t G, const uint32_t *cnt, uint32_t ob,
                                               __amdgpu_buffer_rsrc_t esc, uint32_t L) {
  const uint32_t tid = threadIdx.x, wave = tid >> 6, nwv = blockDim.x >> 6, T = blockDim.x;
#pragma unroll
  for (int v = 0; v < V; v++) {
    const uint64_t mr = __ballot(er[v]), mi = __ballot(ei[v]);
    if ((mr | mi) == 0) continue;
    uint32_t rr, ri;
    if (G >= 64) {
      const uint32_t f = v * nwv + wave, f0 = f & ~((G >> 6) - 1);
      uint32_t br = 0, bi = 0;
      for (uint32_t x = f0; x < f; x++) {
        br += cnt[2 * x];
        bi += cnt[2 * x + 1];
      }
      rr = br + lanes_below(mr);
      ri = bi + lanes_below(mi);
    } else {
      rr = seg_below(mr, G);
      ri = seg_below(mi, G);
    }
    const uint32_t gb = (ob + v * T + tid) & ~(G - 1);
    if (er[v]) buf_st_i64(esc, 8 * (gb + rr), dr[v]);
    if (ei[v]) buf_st_i64(esc, 8 * (L + gb + ri), di[v]);
  }
}

// Running sums of one thread over the tiles it handles.
struct Acc {
  uint64_t lo, hi;  // sum p^2
  uint32_t nesc;
  double emax;
  bool ok;
  bool wide;  // some |q| >= 2^31: the next pass needs an FP64 workspace
  __device__ __forceinline__ void zero() {
    lo = hi = 0;
    nesc = 0;
    emax = 0.0;
    ok = true;
    wide = false;
  }
  __device__ __forceinline__ void merge(const Acc &o) {  // exact: integer sums, max, flags
    const uint64_t x = lo + o.lo;
    hi += o.hi + (x < lo);
    lo = x;
    nesc += o.nesc;
    emax = fmax(emax, o.emax);
    ok = ok && o.ok;
    wide = wide || o.wide;
  }
};

// codes outside int32 (only on the paths taken when some |q| >= 2^24)
template <int V>
__device__ __forceinline__ void note_wide(const double (&qr)[V], const double (&qi)[V], Acc &acc) {
#pragma unroll
  for (int v = 0; v < V; v++) acc.wide = acc.wide || !(fabs(qr[v]) < 0x1p31) || !(fabs(qi[v]) < 0x1p31);
}

// Symbols of one tile of C consecutive amplitudes from offset ob (a chunk
// head: C is a multiple of the chunk length): Lorenzo differences inside
// chunks -- the predecessor of tile element e = v * blockDim + tid comes
// from the lane below, or across a wavefront boundary through LDS --,
// symbols, escapes, the LDS histogram h and the running sums.
template <int V, bool FULL>
__device__ __forceinline__ void tile_symbols(const double (&qr)[V], const double (&qi)[V], uint32_t *h,
                                             double (*bnd)[V][4], const Geo &g, const SlotOut &so, uint32_t ob,
                                             uint32_t C, Acc &acc) {
  const uint32_t tid = threadIdx.x, T = blockDim.x, lane = lane_id(), wave = tid >> 6, nwv = T >> 6;
  const uint32_t Bm = (1u << g.chunk_log2) - 1;
  if (lane == 63) {
#pragma unroll
    for (int v = 0; v < V; v++) {
      bnd[0][v][wave] = qr[v];
      bnd[1][v][wave] = qi[v];
    }
  }
  lds_sync();
  uint32_t sr[V], si[V];
  uint32_t nval = 0;
  bool uni = true;
  bool esr[V], esi[V];
  int64_t edr[V], edi[V];
#pragma unroll
  for (int v = 0; v < V; v++) {
    const uint32_t e = v * T + tid;
    const double up_r = __shfl_up(qr[v], 1, 64), up_i = __shfl_up(qi[v], 1, 64);
    sr[v] = si[v] = 0;
    esr[v] = esi[v] = false;
    edr[v] = edi[v] = 0;
    if (!FULL && e >= C) continue;
    const uint32_t o = ob + e;
    double pr = 0.0, pi = 0.0;  // predecessor in the chunk (0 at a chunk head)
    if ((o & Bm) != 0) {
      if (lane > 0) {
        pr = up_r;
        pi = up_i;
      } else if (wave > 0) {
        pr = bnd[0][v][wave - 1];
        pi = bnd[1][v][wave - 1];
      } else {  // e > 0 here: the tile starts at a chunk head
        pr = bnd[0][v - 1][nwv - 1];
        pi = bnd[1][v - 1][nwv - 1];
      }
    }
    const double dr = qr[v] - pr, di = qi[v] - pi;  // exact: integers below 2^49
    const bool er = !(fabs(dr) < (double)kR), ei = !(fabs(di) < (double)kR);
    sr[v] = er ? 0u : (uint32_t)((int)dr + kR);
    si[v] = ei ? 0u : (uint32_t)((int)di + kR);
    esr[v] = er;
    esi[v] = ei;
    edr[v] = (int64_t)dr;
    edi[v] = (int64_t)di;
    acc.nesc += (uint32_t)er + (uint32_t)ei;
    so.symr[o] = (uint16_t)sr[v];
    so.symi[o] = (uint16_t)si[v];
    uni &= (sr[v] == sr[0]) & (si[v] == sr[0]);
    nval += 2;
  }
  add_squares<V>(qr, qi, acc.lo, acc.hi);  // values past C are zero
  note_wide<V>(qr, qi, acc);
  // histogram: a wavefront whose values all share one symbol adds once
  const bool any = nval != 0;
  const uint32_t s0 = (uint32_t)__shfl((int)sr[0], 0, 64);
  const uint64_t act = __ballot(any);
  const bool wave_uni = __ballot(any && uni && sr[0] == s0) == act;
  if (wave_uni) {
    uint32_t cnt;
    if (FULL) {
      cnt = 2u * V * (uint32_t)__popcll(act);
    } else {
      cnt = nval;
      for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    }
    if (lane == 0 && cnt) atomicAdd(&h[s0], cnt);
  } else if (any) {
    uint32_t cs = sr[0], cn = 0;
#pragma unroll
    for (int v = 0; v < V; v++) {
      if (!FULL && v * T + tid >= C) break;
      if (sr[v] != cs) { atomicAdd(&h[cs], cn); cs = sr[v]; cn = 0; }
      cn++;
      if (si[v] != cs) { atomicAdd(&h[cs], cn); cs = si[v]; cn = 0; }
      cn++;
    }
    atomicAdd(&h[cs], cn);
  }
  __shared__ uint32_t ecnt[2 * V * 4];
  const uint32_t G = esc_group(g);
  esc_count_tile<V>(esr, esi, G, ecnt);
  lds_sync();  // bnd is reused by the next tile; ecnt is read below and rewritten after the next tile's barrier
  esc_store_tile<V>(esr, esi, edr, edi, G, ecnt, ob, buf_rsrc(so.escr, (uint32_t)(16 * g.L)), (uint32_t)g.L);
}

// LDS histogram update of one thread's 2V symbols of a whole tile.  The
// real and the imaginary parts are counted apart (their differences follow
// different patterns): a wavefront whose symbols of one part are all equal
// adds them once, otherwise every thread adds its runs of equal symbols.
template <int V>
__device__ __forceinline__ void hist_part(const uint32_t (&sv)[V], uint32_t *h) {
  bool uni = true;
#pragma unroll
  for (int v = 1; v < V; v++) uni &= sv[v] == sv[0];
  const uint32_t s0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)sv[0]);
  if (__ballot(!(uni && sv[0] == s0)) == 0) {
    if (lane_id() == 0) atomicAdd(&h[s0], (uint32_t)V * 64u);
  } else {
    uint32_t cs = sv[0], cn = 1;
#pragma unroll
    for (int v = 1; v < V; v++) {
      if (sv[v] != cs) {
        atomicAdd(&h[cs], cn);
        cs = sv[v];
        cn = 0;
      }
      cn++;
    }
    atomicAdd(&h[cs], cn);
  }
}

template <int V>
__device__ __forceinline__ void hist_full(const uint32_t (&sr)[V], const uint32_t (&si)[V], uint32_t *h) {
  hist_part<V>(sr, h);
  hist_part<V>(si, h);
}

// the value of the lane below (0 in lane 0): a DPP shift of the wavefront
__device__ __forceinline__ int lane_below(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}

// Output of a slot's gate_quant over whole tiles: symbols and escapes.
struct SlotBuf {
  __amdgpu_buffer_rsrc_t sym, esc;  // [2L] u16, [2L] i64 (re plane, then im plane)
  uint32_t L;
};

__device__ __forceinline__ SlotBuf slot_buf(const Slots &sl, const Geo &g, uint32_t u) {
  SlotBuf b;
  b.sym = buf_rsrc(sl.sym + (uint64_t)u * 2 * g.L, (uint32_t)(4 * g.L));
  b.esc = buf_rsrc(sl.esc + (uint64_t)u * 2 * g.L, (uint32_t)(16 * g.L));
  b.L = (uint32_t)g.L;
  return b;
}

// tile_symbols for whole tiles of 256 V amplitudes (256 threads), with an
// integer path: when every |q| of the tile is below 2^24 -- decided for the
// whole workgroup at the first barrier, so that all wavefronts take the same
// barriers and exchange boundary values in one form -- differences, symbols
// and squares are computed in 32/64-bit integers (q^2 < 2^48, and a tile adds
// at most 2V of them per thread before they join the 128-bit sum).
// Otherwise the FP64 path runs, which also refuses |q| >= 2^48.  Results are
// identical on both paths.
template <int V>
__device__ __forceinline__ void tile_symbols_full(const double (&qr)[V], const double (&qi)[V], uint32_t *h,
                                                  double (*bnd)[V][4], uint32_t *bigw, const Geo &g,
                                                  const SlotBuf &sb, uint32_t ob, Acc &acc) {
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  constexpr uint32_t T = 256, nwv = 4;
  const uint32_t Bm = (1u << g.chunk_log2) - 1;
  bool small = true;
#pragma unroll
  for (int v = 0; v < V; v++) small = small && fabs(qr[v]) < 0x1p24 && fabs(qi[v]) < 0x1p24;
  const bool wbig = __ballot(!small) != 0;
  if (lane == 63) {
#pragma unroll
    for (int v = 0; v < V; v++) {
      bnd[0][v][wave] = qr[v];
      bnd[1][v][wave] = qi[v];
    }
  }
  if (lane == 0) bigw[wave] = wbig ? 1u : 0u;
  lds_sync();
  const bool big = (bigw[0] | bigw[1] | bigw[2] | bigw[3]) != 0;
  uint32_t sr[V], si[V];
  int64_t edr[V], edi[V];  // escaped differences, stored after the barrier below
  if (big) {
    bool any_esc = false;
    double dr[V], di[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
      acc.ok = acc.ok && fabs(qr[v]) < kPMax && fabs(qi[v]) < kPMax;
      const uint32_t o = ob + v * T + tid;
      const double up_r = __shfl_up(qr[v], 1, 64), up_i = __shfl_up(qi[v], 1, 64);
      double pr = 0.0, pi = 0.0;  // predecessor in the chunk (0 at a chunk head)
      if ((o & Bm) != 0) {
        if (lane > 0) {
          pr = up_r;
          pi = up_i;
        } else if (wave > 0) {
          pr = bnd[0][v][wave - 1];
          pi = bnd[1][v][wave - 1];
        } else {  // the tile starts at a chunk head, so v > 0 here
          pr = bnd[0][v - 1][nwv - 1];
          pi = bnd[1][v - 1][nwv - 1];
        }
      }
      dr[v] = qr[v] - pr;  // exact: integers below 2^49
      di[v] = qi[v] - pi;
      const bool er = !(fabs(dr[v]) < (double)kR), ei = !(fabs(di[v]) < (double)kR);
      sr[v] = er ? 0u : (uint32_t)((int)dr[v] + kR);
      si[v] = ei ? 0u : (uint32_t)((int)di[v] + kR);
      any_esc |= er | ei;
      acc.nesc += (uint32_t)er + (uint32_t)ei;
      buf_st_u16(sb.sym, 2 * o, sr[v]);
      buf_st_u16(sb.sym, 2 * (sb.L + o), si[v]);
    }
    if (__ballot(any_esc)) {
#pragma unroll
      for (int v = 0; v < V; v++) {
        edr[v] = (int64_t)dr[v];
        edi[v] = (int64_t)di[v];
      }
    }
    add_squares<V>(qr, qi, acc.lo, acc.hi);
    note_wide<V>(qr, qi, acc);
  } else {
    int ir[V], ii[V], dr[V], di[V];
    bool any_esc = false;
    int64_t t = 0;  // sum of q^2 over the tile's 2V values of this thread, below 2^52
#pragma unroll
    for (int v = 0; v < V; v++) {
      ir[v] = (int)qr[v];  // exact: |q| < 2^24
      ii[v] = (int)qi[v];
      const uint32_t o = ob + v * T + tid;
      int pr = lane_below(ir[v]), pi = lane_below(ii[v]);
      if (lane == 0) {
        if (wave > 0) {
          pr = (int)bnd[0][v][wave - 1];
          pi = (int)bnd[1][v][wave - 1];
        } else if (v > 0) {
          pr = (int)bnd[0][v - 1][nwv - 1];
          pi = (int)bnd[1][v - 1][nwv - 1];
        }
      }
      if ((o & Bm) == 0) pr = pi = 0;  // chunk head: predictor 0
      dr[v] = ir[v] - pr;  // |d| < 2^25
      di[v] = ii[v] - pi;
      const bool er = (uint32_t)(dr[v] + (kR - 1)) > (uint32_t)(2 * kR - 2);  // !(|d| < R)
      const bool ei = (uint32_t)(di[v] + (kR - 1)) > (uint32_t)(2 * kR - 2);
      sr[v] = er ? 0u : (uint32_t)(dr[v] + kR);
      si[v] = ei ? 0u : (uint32_t)(di[v] + kR);
      any_esc |= er | ei;
      acc.nesc += (uint32_t)er + (uint32_t)ei;
      buf_st_u16(sb.sym, 2 * o, sr[v]);
      buf_st_u16(sb.sym, 2 * (sb.L + o), si[v]);
      t += (int64_t)ir[v] * ir[v];
      t += (int64_t)ii[v] * ii[v];
    }
    if (__ballot(any_esc)) {
#pragma unroll
      for (int v = 0; v < V; v++) {
        edr[v] = (int64_t)dr[v];
        edi[v] = (int64_t)di[v];
      }
    }
    const uint64_t x = acc.lo + (uint64_t)t;
    acc.hi += x < acc.lo;
    acc.lo = x;
  }
  hist_full<V>(sr, si, h);
  __shared__ uint32_t ecnt[2 * V * 4];
  const uint32_t G = esc_group(g);
  bool esr[V], esi[V];
#pragma unroll
  for (int v = 0; v < V; v++) {
    esr[v] = sr[v] == 0;
    esi[v] = si[v] == 0;
  }
  esc_count_tile<V>(esr, esi, G, ecnt);
  lds_sync();  // bnd and bigw are reused by the next tile; ecnt is read below and rewritten after the next tile's barrier
  esc_store_tile<V>(esr, esi, edr, edi, G, ecnt, ob, sb.esc, sb.L);
}

// Reduce the workgroup's sums and write them, with the LDS histogram h (then
// cleared), to partial result `pidx` of slot u.
__device__ __forceinline__ void write_partial(Acc &acc, uint32_t *h, uint64_t (*wred)[4], const Slots &sl,
                                              uint32_t u, uint32_t pidx, Ctl *ctl, uint32_t pass) {
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, nwv = blockDim.x >> 6;
  uint64_t lo = acc.lo, hi = acc.hi, ne = acc.nesc;
  double em = acc.emax;
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t ol = __shfl_xor(lo, off, 64), oh = __shfl_xor(hi, off, 64);
    uint64_t t = lo + ol;
    hi += oh + (t < lo);
    lo = t;
    em = fmax(em, __shfl_xor(em, off, 64));
    ne += __shfl_xor(ne, off, 64);
  }
  if (lane == 0) {
    wred[wave][0] = lo;
    wred[wave][1] = hi;
    wred[wave][2] = ne;
    wred[wave][3] = (uint64_t)__double_as_longlong(em);
  }
  if (__ballot(!acc.ok) && lane == 0) fail(ctl, kFlagBound, pass);
  if (__ballot(acc.wide) && lane == 0) atomicOr(&ctl->wide_next, 1u);
  __syncthreads();
  if (pidx >= kGqParts) return;  // launches never exceed the partial count
  uint32_t *hp = sl.hpart + ((uint64_t)u * kGqParts + pidx) * kNSym;
  for (uint32_t s = tid; s < (uint32_t)kNSym; s += blockDim.x) {
    hp[s] = h[s];
    h[s] = 0;
  }
  if (tid == 0) {
    uint64_t l2 = wred[0][0], h2 = wred[0][1], n2 = wred[0][2], eb = wred[0][3];
    for (uint32_t w = 1; w < nwv; w++) {
      uint64_t t = l2 + wred[w][0];
      h2 += wred[w][1] + (t < l2);
      l2 = t;
      n2 += wred[w][2];
      eb = wred[w][3] > eb ? wred[w][3] : eb;
    }
    uint64_t *pp = sl.part + ((uint64_t)u * kGqParts + pidx) * 4;
    pp[0] = l2;
    pp[1] = h2;
    pp[2] = n2;
    pp[3] = eb;
  }
  __syncthreads();
}

__device__ __forceinline__ void slot_quant(const Slots &sl, const QuantParams &qp, uint32_t u, double &step,
                                           double &recip, double &ebj) {
  step = qp.step;
  recip = qp.recip;
  ebj = qp.eb;
  if (qp.rel) {
    step = sl.qstep[3 * u];
    recip = sl.qstep[3 * u + 1];
    ebj = sl.qstep[3 * u + 2];
  }
}

// gate_quant: workgroup (x, u) takes tiles x, x + G, ... of slot u, each of C
// = min(256 V, L) consecutive amplitudes; tile element e = v * blockDim + tid
// belongs to thread tid, so every load and store instruction is contiguous
// across the wavefront.  The LDS histogram and the sums run over all the
// workgroup's tiles and leave once, as partial result x of the slot.
// KIND 0: identity; 1: one target inside the tile (partner through the
// cache); 2: phase; 3: dense on several targets (general indexing).
template <int KIND, int V, bool FULL>
__global__ void __launch_bounds__(256, 2) k_gate_quant(Slots sl, Geo g, const uint64_t *slot_slice, GateDesc gd,
                                                       QuantParams qp, Ctl *ctl, uint32_t pass) {
  if (ctl->flags) return;
  __shared__ uint32_t h[kNSym];
  __shared__ double bnd[2][V][4];
  __shared__ uint64_t wred[4][4];
  const uint32_t tid = threadIdx.x, T = FULL ? 256u : blockDim.x;
  for (uint32_t s = tid; s < (uint32_t)kNSym; s += T) h[s] = 0;
  const uint32_t C = FULL ? 256u * V : (uint32_t)((uint64_t)T * V < g.L ? (uint64_t)T * V : g.L);
  const uint32_t u = blockIdx.y, G = gridDim.x;
  const uint32_t ntiles = (uint32_t)(g.L / C);
  const double *wre = sl.ws + (uint64_t)u * 2 * g.L, *wim = wre + g.L;
  const SlotOut so = slot_out(sl, g, u);
  // controls: slice-index bits are uniform, offset bits are checked per lane
  const uint64_t gi_hi = slot_slice[u] << g.slice_log2;
  const uint64_t mask_hi = gd.ctrl_mask & ~(g.L - 1);
  const bool hi_ok = (gi_hi & mask_hi) == (gd.ctrl_vals & mask_hi);
  const uint32_t mask_lo = (uint32_t)(gd.ctrl_mask & (g.L - 1)), vals_lo = (uint32_t)(gd.ctrl_vals & (g.L - 1));
  const uint32_t bit = KIND == 1 ? 1u << gd.tloc[0] : 0u;
  double step, recip, ebj;
  slot_quant(sl, qp, u, step, recip, ebj);
  // pointwise-relative mode: the tile's squared stored values (real plane,
  // imaginary plane), 2 C doubles of dynamic LDS (none otherwise)
  extern __shared__ double pws[];
  Acc acc;
  acc.zero();
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += G) {
    const uint32_t ob = tile * C;
    double sr[V], si[V];  // pointwise-relative mode: the stored values
    double ar[V], ai[V], br[V], bi[V];  // own amplitude; partner (one-target gates)
    // all loads first (whole tiles need no bounds checks), then arithmetic
#pragma unroll
    for (int v = 0; v < V; v++) {
      const uint32_t e = v * T + tid;
      ar[v] = ai[v] = br[v] = bi[v] = 0.0;
      if (KIND != 3 && (FULL || e < C)) {
        ar[v] = wre[ob + e];
        ai[v] = wim[ob + e];
        if (KIND == 1) {
          br[v] = wre[(ob + e) ^ bit];
          bi[v] = wim[(ob + e) ^ bit];
        }
      }
    }
    double qr[V], qi[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
      const uint32_t e = v * T + tid;
      qr[v] = qi[v] = 0.0;
      if (!FULL && e >= C) continue;
      const uint32_t o = ob + e;
      double re = ar[v], im = ai[v];
      if (KIND == 3) {
        eval_amp<3>(sl.ws, g, slot_slice, gd, u, o, re, im);
      } else {
        const bool on = hi_ok && (o & mask_lo) == vals_lo;
        if (KIND == 2 && on) {
          cmul(gd.ph_re, gd.ph_im, ar[v], ai[v], re, im);
        } else if (KIND == 1 && on) {
          // column 0 is the amplitude with the target bit clear
          const bool row = (o & bit) != 0;
          const double a0r = row ? br[v] : ar[v], a0i = row ? bi[v] : ai[v];
          const double a1r = row ? ar[v] : br[v], a1i = row ? ai[v] : bi[v];
          const double u0r = row ? gd.m2[4] : gd.m2[0], u0i = row ? gd.m2[5] : gd.m2[1];
          const double u1r = row ? gd.m2[6] : gd.m2[2], u1i = row ? gd.m2[7] : gd.m2[3];
          double cr, ci;
          cmul(u0r, u0i, a0r, a0i, cr, ci);
          cmac(u1r, u1i, a1r, a1i, cr, ci);
          re = cr;
          im = ci;
        }
      }
      double e1, e2;
      if (qp.pw) {
        acc.ok &= quantise_pw(re, qp.pw_bits, qp.eb, qr[v], e1, sr[v]);
        acc.ok &= quantise_pw(im, qp.pw_bits, qp.eb, qi[v], e2, si[v]);
      } else {
        acc.ok &= quantise(re, step, recip, ebj, qr[v], e1);
        acc.ok &= quantise(im, step, recip, ebj, qi[v], e2);
      }
      acc.emax = fmax(acc.emax, fmax(e1, e2));
    }
    if (qp.pw) {  // each chunk's sum of squared stored values, a pairwise tree in index order
#pragma unroll
      for (int v = 0; v < V; v++) {
        const uint32_t e = v * T + tid;
        if (FULL || e < C) {
          pws[e] = sr[v] * sr[v];
          pws[C + e] = si[v] * si[v];
        }
      }
      __syncthreads();
      const uint32_t B = 1u << g.chunk_log2;
      for (uint32_t m = C; m > C / B; m >>= 1) {  // m values per plane -> m / 2: x[i] = x[2i] + x[2i+1]
        double t[8];
        const uint32_t h2 = m / 2;
#pragma unroll
        for (int k = 0; k < 8; k++) {
          const uint32_t i = k * T + tid;
          t[k] = 0.0;
          if (i < m) {
            const uint32_t base = i < h2 ? 0u : C, j = i < h2 ? i : i - h2;
            t[k] = pws[base + 2 * j] + pws[base + 2 * j + 1];
          }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; k++) {
          const uint32_t i = k * T + tid;
          if (i < m) pws[(i < h2 ? 0u : C) + (i < h2 ? i : i - h2)] = t[k];
        }
        __syncthreads();
      }
      const uint32_t nc = C / B;  // chunks of this tile per plane
      double *cs = sl.csum + (uint64_t)u * g.nchunks;
      for (uint32_t i = tid; i < 2 * nc; i += T) {
        const uint32_t plane = i / nc, k = i - plane * nc;
        cs[(uint64_t)plane * (g.L / B) + ob / B + k] = pws[plane * C + k];
      }
      __syncthreads();  // pws is refilled by the next tile
    }
    tile_symbols<V, FULL>(qr, qi, h, bnd, g, so, ob, C, acc);
  }
  write_partial(acc, h, wred, sl, u, blockIdx.x, ctl, pass);
}

// ------------------------------------------- gate + quantise, whole tiles
// Slices of at least 1024 amplitudes run through software-pipelined variants
// of the kernels above.  Vector memory operations of a wavefront complete in
// issue order on CDNA (one counter for loads and stores), so a wait for a
// tile's loads also waits for every store issued before them.  The pipelines
// below keep, at the top of every tile step, the pending operations in the
// order [loads of this tile] [stores of the previous tile] [loads of the next
// tile]: waiting for this tile never waits for the previous tile's stores.
// Every load is issued unconditionally (past the last tile a valid tile is
// loaded again and ignored), so the count of operations in flight is the
// same on every path into a step.  The number of tiles per workgroup is 1 or
// even (slice and tile sizes are powers of two).

constexpr int kGqV = 4;                      // amplitudes per thread per tile
constexpr uint32_t kGqTile = 256 * kGqV;     // amplitudes per tile
constexpr int kGpV = 2;                      // the same for the paired kernel (two tiles per step)
constexpr uint32_t kGpTile = 256 * kGpV;

template <int V>
struct GqTile {  // one tile of one slot, in registers
  double r[V], i[V];
};

// tile at offset ob of a slot whose planes are addressed by `ws` (re plane,
// then im plane, L values each)
template <int V>
__device__ __forceinline__ void gq_load(GqTile<V> &x, __amdgpu_buffer_rsrc_t ws, uint32_t L, uint32_t ob) {
#pragma unroll
  for (int v = 0; v < V; v++) {
    x.r[v] = buf_ld_f64(ws, 8 * (ob + v * 256 + threadIdx.x));
    x.i[v] = buf_ld_f64(ws, 8 * (L + ob + v * 256 + threadIdx.x));
  }
}

// Per-workgroup constants of gate_quant for one slot.
struct GqSlot {
  __amdgpu_buffer_rsrc_t ws;  // decompressed planes of the slot
  SlotBuf out;
  uint32_t mask_lo, vals_lo;  // control bits inside the slice
  bool hi_ok;                 // control bits of the slice index hold
  double step, recip, ebj;
};

__device__ __forceinline__ GqSlot gq_slot(const Slots &sl, const Geo &g, const uint64_t *slot_slice,
                                          const GateDesc &gd, const QuantParams &qp, uint32_t u) {
  GqSlot s;
  s.ws = buf_rsrc(sl.ws + (uint64_t)u * 2 * g.L, (uint32_t)(16 * g.L));
  s.out = slot_buf(sl, g, u);
  const uint64_t gi_hi = slot_slice[u] << g.slice_log2;
  const uint64_t mask_hi = gd.ctrl_mask & ~(g.L - 1);
  s.hi_ok = (gi_hi & mask_hi) == (gd.ctrl_vals & mask_hi);
  s.mask_lo = (uint32_t)(gd.ctrl_mask & (g.L - 1));
  s.vals_lo = (uint32_t)(gd.ctrl_vals & (g.L - 1));
  slot_quant(sl, qp, u, s.step, s.recip, s.ebj);
  return s;
}

// q = rint(v / step) as an integer-valued double and the check of the bound;
// the range of q is checked by the tile's symbol step
__device__ __forceinline__ void quant_tile(double v, const GqSlot &s, double &q, Acc &acc) {
  q = rint(v * s.recip);
  const double err = fabs(v - q * s.step);
  acc.ok &= err <= s.ebj;
  acc.emax = fmax(acc.emax, err);
}

// Gate, quantisation and symbols of one tile at offset ob.  KIND 0:
// identity; 1: one target t inside the tile (partner amplitude from the same
// thread when 2^t >= 256, else through the LDS exchange buffer xch); 2: phase.
template <int KIND>
__device__ __forceinline__ void gq_tile_step(const GqTile<kGqV> &x, uint32_t ob, const GqSlot &s, const GateDesc &gd,
                                             const Geo &g, double (*xch)[kGqTile], uint32_t *h,
                                             double (*bnd)[kGqV][4], uint32_t *bigw, Acc &acc) {
  const uint32_t tid = threadIdx.x;
  double qr[kGqV], qi[kGqV];
  double pr[kGqV], pi[kGqV];  // partner amplitudes (KIND 1)
  uint32_t bit = 0;
  if (KIND == 1) {
    const int tb = gd.tloc[0];
    bit = 1u << tb;
    if (tb >= 8) {  // partner element (v ^ 2^(t-8)) * 256 + tid: same thread
#pragma unroll
      for (int v = 0; v < kGqV; v++) {
        pr[v] = tb == 8 ? x.r[v ^ 1] : x.r[v ^ 2];
        pi[v] = tb == 8 ? x.i[v ^ 1] : x.i[v ^ 2];
      }
    } else {
#pragma unroll
      for (int v = 0; v < kGqV; v++) {
        xch[0][v * 256 + tid] = x.r[v];
        xch[1][v * 256 + tid] = x.i[v];
      }
      lds_sync();
#pragma unroll
      for (int v = 0; v < kGqV; v++) {
        pr[v] = xch[0][(v * 256 + tid) ^ bit];
        pi[v] = xch[1][(v * 256 + tid) ^ bit];
      }
      // the tile's symbols start with a barrier; xch is written again only
      // after the barrier that ends them
    }
  }
#pragma unroll
  for (int v = 0; v < kGqV; v++) {
    const uint32_t o = ob + v * 256 + tid;
    double re = x.r[v], im = x.i[v];
    const bool on = s.hi_ok && (o & s.mask_lo) == s.vals_lo;
    if (KIND == 2 && on) {
      cmul(gd.ph_re, gd.ph_im, x.r[v], x.i[v], re, im);
    } else if (KIND == 1 && on) {
      const bool row = (o & bit) != 0;  // column 0: the amplitude with the target bit clear
      const double a0r = row ? pr[v] : x.r[v], a0i = row ? pi[v] : x.i[v];
      const double a1r = row ? x.r[v] : pr[v], a1i = row ? x.i[v] : pi[v];
      const double u0r = row ? gd.m2[4] : gd.m2[0], u0i = row ? gd.m2[5] : gd.m2[1];
      const double u1r = row ? gd.m2[6] : gd.m2[2], u1i = row ? gd.m2[7] : gd.m2[3];
      double cr, ci;
      cmul(u0r, u0i, a0r, a0i, cr, ci);
      cmac(u1r, u1i, a1r, a1i, cr, ci);
      re = cr;
      im = ci;
    }
    quant_tile(re, s, qr[v], acc);
    quant_tile(im, s, qi[v], acc);
  }
  tile_symbols_full<kGqV>(qr, qi, h, bnd, bigw, g, s.out, ob, acc);
}

// gate_quant over whole tiles: workgroup (x, u) takes tiles x, x + G, ... of
// slot u (n = ntiles / G of them), two tiles in flight.
template <int KIND>
__global__ void __launch_bounds__(256, 2) k_gate_quant_pipe(Slots sl, Geo g, const uint64_t *slot_slice,
                                                            GateDesc gd, QuantParams qp, Ctl *ctl, uint32_t pass) {
  if (ctl->flags) return;
  __shared__ uint32_t h[kNSym];
  __shared__ double bnd[2][kGqV][4];
  __shared__ uint64_t wred[4][4];
  __shared__ double xch[KIND == 1 ? 2 : 1][kGqTile];
  __shared__ uint32_t bigw[4];
  for (uint32_t s = threadIdx.x; s < (uint32_t)kNSym; s += 256) h[s] = 0;
  const uint32_t u = blockIdx.y, G = gridDim.x, t0 = blockIdx.x;
  const uint32_t ntiles = (uint32_t)(g.L / kGqTile), n = ntiles / G, L = (uint32_t)g.L;
  const GqSlot s = gq_slot(sl, g, slot_slice, gd, qp, u);
  Acc acc;
  acc.zero();
  auto tile_of = [&](uint32_t k) { return k < n ? t0 + k * G : t0; };  // past the end: tile t0 again
  GqTile<kGqV> A, B;
  gq_load(A, s.ws, L, t0 * kGqTile);
  if (n == 1) {
    gq_tile_step<KIND>(A, t0 * kGqTile, s, gd, g, xch, h, bnd, bigw, acc);
  } else {
    gq_load(B, s.ws, L, tile_of(1) * kGqTile);
    gq_tile_step<KIND>(A, t0 * kGqTile, s, gd, g, xch, h, bnd, bigw, acc);
    gq_load(A, s.ws, L, tile_of(2) * kGqTile);
    for (uint32_t k = 1; k + 1 < n; k += 2) {
      gq_tile_step<KIND>(B, tile_of(k) * kGqTile, s, gd, g, xch, h, bnd, bigw, acc);
      gq_load(B, s.ws, L, tile_of(k + 2) * kGqTile);
      gq_tile_step<KIND>(A, tile_of(k + 1) * kGqTile, s, gd, g, xch, h, bnd, bigw, acc);
      gq_load(A, s.ws, L, tile_of(k + 3) * kGqTile);
    }
    gq_tile_step<KIND>(B, tile_of(n - 1) * kGqTile, s, gd, g, xch, h, bnd, bigw, acc);
  }
  write_partial(acc, h, wred, sl, u, blockIdx.x, ctl, pass);
}

// One tile pair of a one-target gate whose partner lies in another tile.
struct GqPair {
  GqTile<kGpV> a, b;
};

__device__ __forceinline__ void gq_pair_step(const GqPair &x, uint32_t obA, uint32_t obB, const GqSlot &sA,
                                             const GqSlot &sB, const GateDesc &gd, const Geo &g, uint32_t *hA,
                                             uint32_t *hB, double (*bnd)[kGpV][4], uint32_t *bigw, Acc &accA,
                                             Acc &accB) {
  const uint32_t tid = threadIdx.x;
  double qar[kGpV], qai[kGpV], qbr[kGpV], qbi[kGpV];
#pragma unroll
  for (int v = 0; v < kGpV; v++) {
    const uint32_t e = v * 256 + tid;
    const double a0r = x.a.r[v], a0i = x.a.i[v], a1r = x.b.r[v], a1i = x.b.i[v];
    double outAr = a0r, outAi = a0i, outBr = a1r, outBi = a1i;
    // controls never include the target bit: A's index decides for the pair
    if (sA.hi_ok && ((obA + e) & sA.mask_lo) == sA.vals_lo) {
      cmul(gd.m2[0], gd.m2[1], a0r, a0i, outAr, outAi);
      cmac(gd.m2[2], gd.m2[3], a1r, a1i, outAr, outAi);
      cmul(gd.m2[4], gd.m2[5], a0r, a0i, outBr, outBi);
      cmac(gd.m2[6], gd.m2[7], a1r, a1i, outBr, outBi);
    }
    quant_tile(outAr, sA, qar[v], accA);
    quant_tile(outAi, sA, qai[v], accA);
    quant_tile(outBr, sB, qbr[v], accB);
    quant_tile(outBi, sB, qbi[v], accB);
  }
  tile_symbols_full<kGpV>(qar, qai, hA, bnd, bigw, g, sA.out, obA, accA);
  tile_symbols_full<kGpV>(qbr, qbi, hB, bnd, bigw, g, sB.out, obB, accB);
}

// A one-target gate whose partner lies in another tile (target bit t at or
// above the tile size): a workgroup takes both tiles of a pair, so every
// amplitude is read once.  In the batch's flat index (slot * L + offset) the
// partner of amplitude f is f ^ 2^t.  Slice-index targets pair slot uA (bit
// clear) with uB = uA + 2^(t - slice_log2), tile for tile; in-slice targets
// pair tiles of one slot.  Two tile pairs are in flight.
__global__ void __launch_bounds__(256, 2) k_gate_quant_pair_pipe(Slots sl, Geo g, const uint64_t *slot_slice,
                                                                 GateDesc gd, QuantParams qp, Ctl *ctl,
                                                                 uint32_t pass) {
  if (ctl->flags) return;
  __shared__ uint32_t hA[kNSym], hB[kNSym];
  __shared__ double bnd[2][kGpV][4];
  __shared__ uint64_t wred[4][4];
  __shared__ uint32_t bigw[4];
  for (uint32_t s = threadIdx.x; s < (uint32_t)kNSym; s += 256) hA[s] = hB[s] = 0;
  const uint32_t ntiles = (uint32_t)(g.L / kGpTile), L = (uint32_t)g.L;
  const int t = gd.tloc[0];
  const bool cross = t >= g.slice_log2;
  uint32_t uA, uB, npairs;
  int b = 0;
  if (cross) {
    const uint32_t sb = t - g.slice_log2, y = blockIdx.y;
    uA = ((y >> sb) << (sb + 1)) | (y & ((1u << sb) - 1));
    uB = uA | (1u << sb);
    npairs = ntiles;
  } else {
    uA = uB = blockIdx.y;
    b = t - 9;  // log2 of the tile size
    npairs = ntiles / 2;
  }
  const uint32_t G = gridDim.x, w0 = blockIdx.x, n = npairs / G;
  const GqSlot sA = gq_slot(sl, g, slot_slice, gd, qp, uA), sB = gq_slot(sl, g, slot_slice, gd, qp, uB);
  Acc accA, accB;
  accA.zero();
  accB.zero();
  auto pair_of = [&](uint32_t k) { return k < n ? w0 + k * G : w0; };  // past the end: pair w0 again
  auto tA_of = [&](uint32_t w) { return cross ? w : ((w >> b) << (b + 1)) | (w & ((1u << b) - 1)); };
  auto tB_of = [&](uint32_t w) { return cross ? w : tA_of(w) | (1u << b); };
  auto load = [&](GqPair &x, uint32_t w) {
    gq_load(x.a, sA.ws, L, tA_of(w) * kGpTile);
    gq_load(x.b, sB.ws, L, tB_of(w) * kGpTile);
  };
  auto step = [&](const GqPair &x, uint32_t w) {
    gq_pair_step(x, tA_of(w) * kGpTile, tB_of(w) * kGpTile, sA, sB, gd, g, hA, hB, bnd, bigw, accA, accB);
  };
  GqPair P, Q;
  load(P, w0);
  if (n == 1) {
    step(P, w0);
  } else {
    load(Q, pair_of(1));
    step(P, w0);
    load(P, pair_of(2));
    for (uint32_t k = 1; k + 1 < n; k += 2) {
      step(Q, pair_of(k));
      load(Q, pair_of(k + 2));
      step(P, pair_of(k + 1));
      load(P, pair_of(k + 3));
    }
    step(Q, pair_of(n - 1));
  }
  // partial results: x for both slots of a cross-slice pair; x and G + x
  // when both tiles belong to one slot
  write_partial(accA, hA, wred, sl, uA, blockIdx.x, ctl, pass);
  write_partial(accB, hB, wred, sl, uB, cross ? blockIdx.x : gridDim.x + blockIdx.x, ctl, pass);
}

// ------------------------------------------ gate + quantise, wave ranges
// For chunks of at most 256 values, every wavefront works alone on ranges of
// 256 consecutive amplitudes of a slot (element v * 64 + lane, v < 4).  A
// range starts at a chunk head, so the Lorenzo predecessor of an element is
// in the same wavefront (the lane below, or lane 63 at v - 1): the range loop
// has no workgroup barrier, and the workgroup shares only the LDS histogram.
// Loads are pipelined as in the whole-tile kernels: [loads of this range]
// [stores of the previous range] [loads of the next range].

constexpr uint32_t kWr = 256;  // amplitudes per wavefront range

struct WRange {  // FP64 workspace: the values
  double r[4], i[4];
};
struct WRange32 {  // compact workspace: the int32 codes, times the slice's scale on use
  int32_t r[4], i[4];
};

__device__ __forceinline__ void wr_load(WRange &x, __amdgpu_buffer_rsrc_t ws, uint32_t L, uint32_t ob) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int v = 0; v < 4; v++) {
    x.r[v] = buf_ld_f64(ws, 8 * (ob + v * 64 + lane));
    x.i[v] = buf_ld_f64(ws, 8 * (L + ob + v * 64 + lane));
  }
}
// (streaming loads, cache policy bit 1: the codes are read once)
__device__ __forceinline__ void wr_load(WRange32 &x, __amdgpu_buffer_rsrc_t ws, uint32_t L, uint32_t ob) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int v = 0; v < 4; v++) {
    x.r[v] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(ws, 4 * (ob + v * 64 + lane), 0, 2);
    x.i[v] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(ws, 4 * (L + ob + v * 64 + lane), 0, 2);
  }
}
// the values of a loaded range: (double)q * k rounds exactly like the FP64
// workspace's q * k
__device__ __forceinline__ const WRange &wr_val(const WRange &x, double) { return x; }
__device__ __forceinline__ WRange wr_val(const WRange32 &x, double k) {
  WRange y;
#pragma unroll
  for (int v = 0; v < 4; v++) {
    y.r[v] = rw((double)x.r[v] * k);
    y.i[v] = rw((double)x.i[v] * k);
  }
  return y;
}

__device__ __forceinline__ double lane63(double x) {  // the value of lane 63, in every lane
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Escapes of a wavefront range (position ob + v * 64 + lane, ob a multiple
// of 256): each one's rank in its group counts the group's escapes in earlier
// rows and lower lanes.
template <typename D>
__device__ __forceinline__ void wr_store_escs(const SlotBuf &sb, uint32_t ob, uint32_t G, const uint32_t (&sr)[4],
                                              const uint32_t (&si)[4], const D (&dr)[4], const D (&di)[4]) {
  const uint32_t lane = lane_id();
  const uint32_t rows = G >= 64 ? G >> 6 : 1u;  // rows per group
  uint32_t br = 0, bi = 0;                       // the group's escapes in earlier rows
#pragma unroll
  for (int v = 0; v < 4; v++) {
    const uint64_t mr = __ballot(sr[v] == 0), mi = __ballot(si[v] == 0);
    if (((uint32_t)v & (rows - 1)) == 0) br = bi = 0;
    uint32_t rr, ri;
    if (G >= 64) {
      rr = br + lanes_below(mr);
      ri = bi + lanes_below(mi);
    } else {
      rr = seg_below(mr, G);
      ri = seg_below(mi, G);
    }
    br += (uint32_t)__popcll(mr);
    bi += (uint32_t)__popcll(mi);
    const uint32_t gb = (ob + v * 64 + lane) & ~(G - 1);
    if (sr[v] == 0) buf_st_i64(sb.esc, 8 * (gb + rr), (int64_t)dr[v]);
    if (si[v] == 0) buf_st_i64(sb.esc, 8 * (sb.L + gb + ri), (int64_t)di[v]);
  }
}

// Symbols, escapes, squares and histogram of one range at offset ob (a
// chunk head).  Integer path when every |q| of the wavefront is below 2^24
// (the choice only changes the arithmetic, not the result).
__device__ __forceinline__ void wr_symbols(const double (&qr)[4], const double (&qi)[4], uint32_t *h, const Geo &g,
                                           const SlotBuf &sb, uint32_t ob, Acc &acc) {
  const uint32_t lane = lane_id();
  const uint32_t Bm = (1u << g.chunk_log2) - 1;
  bool small = true;
#pragma unroll
  for (int v = 0; v < 4; v++) small = small && fabs(qr[v]) < 0x1p24 && fabs(qi[v]) < 0x1p24;
  uint32_t sr[4], si[4];
  bool any_esc = false;
  if (__ballot(!small) != 0) {
    double dr[4], di[4];
#pragma unroll
    for (int v = 0; v < 4; v++) {
      acc.ok = acc.ok && fabs(qr[v]) < kPMax && fabs(qi[v]) < kPMax;
      const uint32_t o = ob + v * 64 + lane;
      double pr = __shfl_up(qr[v], 1, 64), pi = __shfl_up(qi[v], 1, 64);
      if (v > 0) {
        const double lr = lane63(qr[v - 1]), li = lane63(qi[v - 1]);
        if (lane == 0) {
          pr = lr;
          pi = li;
        }
      }
      if ((o & Bm) == 0) pr = pi = 0.0;  // chunk head: predictor 0
      dr[v] = qr[v] - pr;  // exact: integers below 2^49
      di[v] = qi[v] - pi;
      const bool er = !(fabs(dr[v]) < (double)kR), ei = !(fabs(di[v]) < (double)kR);
      sr[v] = er ? 0u : (uint32_t)((int)dr[v] + kR);
      si[v] = ei ? 0u : (uint32_t)((int)di[v] + kR);
      any_esc = any_esc || er || ei;
      acc.nesc += (uint32_t)er + (uint32_t)ei;
      buf_st_u16(sb.sym, 2 * o, sr[v]);
      buf_st_u16(sb.sym, 2 * (sb.L + o), si[v]);
    }
    if (__ballot(any_esc)) wr_store_escs(sb, ob, esc_group(g), sr, si, dr, di);
    add_squares<4>(qr, qi, acc.lo, acc.hi);
    note_wide<4>(qr, qi, acc);
  } else {
    int ir[4], ii[4], dr[4], di[4];
    int64_t t = 0;  // sum of q^2 of this thread's 8 values, below 2^51
#pragma unroll
    for (int v = 0; v < 4; v++) {
      ir[v] = (int)qr[v];  // exact: |q| < 2^24
      ii[v] = (int)qi[v];
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const uint32_t o = ob + v * 64 + lane;
      int pr = lane_below(ir[v]), pi = lane_below(ii[v]);
      if (v > 0) {
        const int lr = __builtin_amdgcn_readlane(ir[v - 1], 63), li = __builtin_amdgcn_readlane(ii[v - 1], 63);
        if (lane == 0) {
          pr = lr;
          pi = li;
        }
      }
      if ((o & Bm) == 0) pr = pi = 0;  // chunk head (lane 0 at v = 0 always is one)
      dr[v] = ir[v] - pr;  // |d| < 2^25
      di[v] = ii[v] - pi;
      const bool er = (uint32_t)(dr[v] + (kR - 1)) > (uint32_t)(2 * kR - 2);  // !(|d| < R)
      const bool ei = (uint32_t)(di[v] + (kR - 1)) > (uint32_t)(2 * kR - 2);
      sr[v] = er ? 0u : (uint32_t)(dr[v] + kR);
      si[v] = ei ? 0u : (uint32_t)(di[v] + kR);
      any_esc = any_esc || er || ei;
      acc.nesc += (uint32_t)er + (uint32_t)ei;
      buf_st_u16(sb.sym, 2 * o, sr[v]);
      buf_st_u16(sb.sym, 2 * (sb.L + o), si[v]);
      t += (int64_t)ir[v] * ir[v];
      t += (int64_t)ii[v] * ii[v];
    }
    if (__ballot(any_esc)) wr_store_escs(sb, ob, esc_group(g), sr, si, dr, di);
    const uint64_t x = acc.lo + (uint64_t)t;
    acc.hi += x < acc.lo;
    acc.lo = x;
  }
  hist_full<4>(sr, si, h);
}

// Coefficients of a one-target gate for the element itself and for its
// partner.  Row 0 (target bit clear) gives u00 a + u01 b, row 1 gives
// u10 b + u11 a; the sum of the two products is commutative, so both rows
// compute cs a + co b with cs the diagonal and co the off-diagonal entry of
// the element's row, bit for bit like the product in column order.
struct GateCoef {
  double sr, si, pr, pi;
  bool real;  // the gate's matrix has no imaginary parts (the same for every lane)
};
// whether a one-target gate's 2 x 2 matrix is real
__device__ __forceinline__ bool real_m2(const GateDesc &gd) {
  return gd.m2[1] == 0.0 && gd.m2[3] == 0.0 && gd.m2[5] == 0.0 && gd.m2[7] == 0.0;
}
__device__ __forceinline__ GateCoef gate_coef(const GateDesc &gd, bool row) {
  GateCoef c;
  c.sr = row ? gd.m2[6] : gd.m2[0];
  c.si = row ? gd.m2[7] : gd.m2[1];
  c.pr = row ? gd.m2[4] : gd.m2[2];
  c.pi = row ? gd.m2[5] : gd.m2[3];
  c.real = real_m2(gd);
  return c;
}
// The complex multiply-adds of u0 a + u1 b.  With real coefficients the
// products with a zero imaginary part are exact zeros, and adding them
// changes at most the sign of an exact zero: the real path below gives the
// same values with half the operations.
__device__ __forceinline__ void gate_pair(const GateCoef &c, double ar, double ai, double br, double bi, double &re,
                                          double &im) {
  if (c.real) {
    re = rw(rw(c.sr * ar) + rw(c.pr * br));
    im = rw(rw(c.sr * ai) + rw(c.pr * bi));
    return;
  }
  double cr, ci;
  cmul(c.sr, c.si, ar, ai, cr, ci);
  cmac(c.pr, c.pi, br, bi, cr, ci);
  re = cr;
  im = ci;
}

// The loaded values of a range, and the value of lane ^ m (a partner in
// another lane): compact ranges exchange the int32 codes before conversion.
__device__ __forceinline__ void wr_vals(const WRange &x, double, double (&ar)[4], double (&ai)[4]) {
#pragma unroll
  for (int v = 0; v < 4; v++) {
    ar[v] = x.r[v];
    ai[v] = x.i[v];
  }
}
__device__ __forceinline__ void wr_vals(const WRange32 &x, double k, double (&ar)[4], double (&ai)[4]) {
#pragma unroll
  for (int v = 0; v < 4; v++) {
    ar[v] = rw((double)x.r[v] * k);
    ai[v] = rw((double)x.i[v] * k);
  }
}
// The value of lane l ^ 2^T (T < 6) without going through LDS: DPP inside
// rows of 16 lanes (quad permutations, row rotations), the row swaps of
// gfx950 across rows.  A swap of x with itself leaves x's lower row (half) in
// the first result and its upper one in the second, each in both positions.
template <int T>
__device__ __forceinline__ int xor_lanes(int x) {
  static_assert(T >= 0 && T < 6, "a partner inside the wavefront");
  if constexpr (T == 0) {
    return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);  // quad_perm [1, 0, 3, 2]
  } else if constexpr (T == 1) {
    return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);  // quad_perm [2, 3, 0, 1]
  } else if constexpr (T == 2) {
    const int a = __builtin_amdgcn_mov_dpp(x, 0x124, 0xF, 0xF, false);  // row_ror 4: lane i <- (i - 4) mod 16
    const int b = __builtin_amdgcn_mov_dpp(x, 0x12C, 0xF, 0xF, false);  // row_ror 12: lane i <- (i + 4) mod 16
    return (lane_id() & 4u) ? a : b;
  } else if constexpr (T == 3) {
    return __builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false);  // row_ror 8: lane i <- i ^ 8
  } else if constexpr (T == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
    return (int)((lane_id() & 16u) ? r[0] : r[1]);
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
    return (int)((lane_id() & 32u) ? r[0] : r[1]);
  }
}
template <int T>
__device__ __forceinline__ double xor_lanes(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)xor_lanes<T>((int)(uint32_t)b), hi = (uint32_t)xor_lanes<T>((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
template <int T>
__device__ __forceinline__ void wr_lane_partner(const WRange &x, double, double (&br)[4], double (&bi)[4]) {
#pragma unroll
  for (int v = 0; v < 4; v++) {
    br[v] = xor_lanes<T>(x.r[v]);
    bi[v] = xor_lanes<T>(x.i[v]);
  }
}
template <int T>
__device__ __forceinline__ void wr_lane_partner(const WRange32 &x, double k, double (&br)[4], double (&bi)[4]) {
#pragma unroll
  for (int v = 0; v < 4; v++) {
    br[v] = rw((double)xor_lanes<T>(x.r[v]) * k);
    bi[v] = rw((double)xor_lanes<T>(x.i[v]) * k);
  }
}
// KIND 10 + t of the wavefront-range kernels: one target t < 6, the partner in lane ^ 2^t
constexpr bool lane_x(int kind) { return kind >= 10 && kind <= 15; }

// Gate and quantisation of one range.  KIND 0: identity; 10 + t: one target
// t < 6, partner element e ^ 2^t in another lane (c0 holds this lane's
// coefficients); 6 and 7: one target t = 6 or 7, partner at v ^ 2^(t-6) in
// the same lane (c0, c1: the coefficients of rows 0 and 1); 2: phase.
// ALLON: no control bit inside the slice (every element takes the gate);
// otherwise elements whose control bits do not hold keep their value.
template <int KIND, bool ALLON>
__device__ __forceinline__ void wr_gate_quant(const double (&ar)[4], const double (&ai)[4], const double (&br)[4],
                                              const double (&bi)[4], const GateCoef &c0, const GateCoef &c1,
                                              uint32_t ob, const GqSlot &s, const GateDesc &gd, const Geo &g,
                                              uint32_t *h, Acc &acc) {
  const uint32_t lane = lane_id();
  double qr[4], qi[4];
#pragma unroll
  for (int v = 0; v < 4; v++) {
    double re = ar[v], im = ai[v];
    if (KIND != 0) {
      double gr, gi;
      if (KIND == 2) {
        if (gd.ph_im == 0.0) {  // a real phase: u a with u_i = 0 (see gate_pair)
          gr = rw(gd.ph_re * ar[v]);
          gi = rw(gd.ph_re * ai[v]);
        } else {
          cmul(gd.ph_re, gd.ph_im, ar[v], ai[v], gr, gi);
        }
      } else if (lane_x(KIND)) {
        gate_pair(c0, ar[v], ai[v], br[v], bi[v], gr, gi);
      } else {  // row of element v: bit t - 6 of v
        const bool row = ((v >> (KIND - 6)) & 1) != 0;
        gate_pair(row ? c1 : c0, ar[v], ai[v], br[v], bi[v], gr, gi);
      }
      if (ALLON) {
        re = gr;
        im = gi;
      } else {
        const bool on = s.hi_ok && ((ob + v * 64 + lane) & s.mask_lo) == s.vals_lo;
        re = on ? gr : re;
        im = on ? gi : im;
      }
    }
    quant_tile(re, s, qr[v], acc);
    quant_tile(im, s, qi[v], acc);
  }
  wr_symbols(qr, qi, h, g, s.out, ob, acc);
}

template <int KIND, typename R>
__device__ __forceinline__ void wr_step(const R &x, double k, const GateCoef &c0, const GateCoef &c1, uint32_t ob,
                                        const GqSlot &s, const GateDesc &gd, const Geo &g, uint32_t *h, Acc &acc) {
  double ar[4], ai[4], br[4], bi[4];
  wr_vals(x, k, ar, ai);
  if constexpr (lane_x(KIND)) wr_lane_partner<KIND - 10>(x, k, br, bi);
#pragma unroll
  for (int v = 0; v < 4; v++) {
    if (KIND == 6 || KIND == 7) {
      br[v] = ar[v ^ (1 << (KIND - 6))];
      bi[v] = ai[v ^ (1 << (KIND - 6))];
    } else if (!lane_x(KIND)) {
      br[v] = bi[v] = 0.0;
    }
  }
  if (KIND == 0 || (s.hi_ok && s.mask_lo == 0))
    wr_gate_quant<KIND, true>(ar, ai, br, bi, c0, c1, ob, s, gd, g, h, acc);
  else
    wr_gate_quant<KIND, false>(ar, ai, br, bi, c0, c1, ob, s, gd, g, h, acc);
}

// Wavefront w of workgroup (x, u) takes ranges x * 4 + w + k * 4G of slot u.
// R: WRange (FP64 workspace) or WRange32 (compact workspace).
template <int KIND, typename R>
__device__ __forceinline__ void gq_wave_ranges(const GqSlot &s, double k, const GateDesc &gd, const Geo &g,
                                               uint32_t *h, Acc &acc) {
  const uint32_t L = (uint32_t)g.L;
  const uint32_t nwv = gridDim.x * 4, w0 = blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t n = (L / kWr) / nwv;  // ranges per wavefront: 1 or even
  auto range_of = [&](uint32_t j) { return (j < n ? w0 + j * nwv : w0) * kWr; };  // past the end: w0 again
  // KIND 10 + t: this lane's row (bit t of the lane); KIND 6, 7: rows 0 and 1
  const GateCoef c0 = gate_coef(gd, lane_x(KIND) && ((lane_id() >> (KIND - 10)) & 1) != 0);
  const GateCoef c1 = gate_coef(gd, KIND == 6 || KIND == 7);
  R A, B;
  wr_load(A, s.ws, L, range_of(0));
  if (n == 1) {
    wr_step<KIND>(A, k, c0, c1, range_of(0), s, gd, g, h, acc);
  } else {
    wr_load(B, s.ws, L, range_of(1));
    wr_step<KIND>(A, k, c0, c1, range_of(0), s, gd, g, h, acc);
    wr_load(A, s.ws, L, range_of(2));
    for (uint32_t j = 1; j + 1 < n; j += 2) {
      wr_step<KIND>(B, k, c0, c1, range_of(j), s, gd, g, h, acc);
      wr_load(B, s.ws, L, range_of(j + 2));
      wr_step<KIND>(A, k, c0, c1, range_of(j + 1), s, gd, g, h, acc);
      wr_load(A, s.ws, L, range_of(j + 3));
    }
    wr_step<KIND>(B, k, c0, c1, range_of(n - 1), s, gd, g, h, acc);
  }
}

// The same ranges from an FP64 workspace one at a time (no loads ahead):
// the compact kernels' path for a pass whose codes do not fit int32.
template <int KIND>
__device__ __forceinline__ void gq_wave_ranges_fp64(const GqSlot &s, const GateDesc &gd, const Geo &g, uint32_t *h,
                                                    Acc &acc) {
  const uint32_t L = (uint32_t)g.L;
  const uint32_t nwv = gridDim.x * 4, w0 = blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t n = (L / kWr) / nwv;
  const GateCoef c0 = gate_coef(gd, lane_x(KIND) && ((lane_id() >> (KIND - 10)) & 1) != 0);
  const GateCoef c1 = gate_coef(gd, KIND == 6 || KIND == 7);
  for (uint32_t j = 0; j < n; j++) {
    WRange A;
    wr_load(A, s.ws, L, (w0 + j * nwv) * kWr);
    wr_step<KIND>(A, 0.0, c0, c1, (w0 + j * nwv) * kWr, s, gd, g, h, acc);
  }
}

// C32: the workspace is compact unless ctl->wide (decode was told so); else
// it is FP64.  The compact identity kernel fits three workgroups per CU
// without spilling.
template <int KIND, bool C32>
__global__ void __launch_bounds__(256, C32 && KIND == 0 ? 3 : 2) k_gq_wave(Slots sl, Geo g, const uint64_t *slot_slice,
                                                              GateDesc gd, QuantParams qp, Ctl *ctl, uint32_t pass,
                                                              const double *kscale) {
  if (ctl->flags) return;
  __shared__ uint32_t h[kNSym];
  __shared__ uint64_t wred[4][4];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kNSym; i += 256) h[i] = 0;
  __syncthreads();
  const uint32_t u = blockIdx.y;
  const GqSlot s = gq_slot(sl, g, slot_slice, gd, qp, u);
  Acc acc;
  acc.zero();
  if (!C32)
    gq_wave_ranges<KIND, WRange>(s, 0.0, gd, g, h, acc);
  else if (!ctl->wide)
    gq_wave_ranges<KIND, WRange32>(s, kscale[slot_slice[u]], gd, g, h, acc);
  else
    gq_wave_ranges_fp64<KIND>(s, gd, g, h, acc);
  write_partial(acc, h, wred, sl, u, blockIdx.x, ctl, pass);
}

// One-target gate whose partner is in another range (2^t >= 256): a
// wavefront takes range pairs.  In-slice targets pair ranges rA (range bit
// t - 8 clear) and rB = rA | 2^(t-8) of one slot, whose results share one
// histogram; slice-index targets pair the same range of slots uA and uB.
// One pair in registers: the gate and quantisation of a pair free its
// registers, the next pair's loads go there, then the symbols are stored --
// so at every step the pending operations are [next loads][these stores].
__device__ __forceinline__ void wr_pair_quant(const WRange &a, const WRange &b, uint32_t obA, const GqSlot &sA,
                                              const GqSlot &sB, const GateDesc &gd, double (&qar)[4],
                                              double (&qai)[4], double (&qbr)[4], double (&qbi)[4], Acc &accA,
                                              Acc &accB) {
  const uint32_t lane = lane_id();
  const bool real = real_m2(gd);
#pragma unroll
  for (int v = 0; v < 4; v++) {
    const double a0r = a.r[v], a0i = a.i[v], a1r = b.r[v], a1i = b.i[v];
    double outAr = a0r, outAi = a0i, outBr = a1r, outBi = a1i;
    if (sA.hi_ok && ((obA + v * 64 + lane) & sA.mask_lo) == sA.vals_lo) {
      if (real) {  // real matrix: the same values with half the operations (see gate_pair)
        outAr = rw(rw(gd.m2[0] * a0r) + rw(gd.m2[2] * a1r));
        outAi = rw(rw(gd.m2[0] * a0i) + rw(gd.m2[2] * a1i));
        outBr = rw(rw(gd.m2[4] * a0r) + rw(gd.m2[6] * a1r));
        outBi = rw(rw(gd.m2[4] * a0i) + rw(gd.m2[6] * a1i));
      } else {
        cmul(gd.m2[0], gd.m2[1], a0r, a0i, outAr, outAi);
        cmac(gd.m2[2], gd.m2[3], a1r, a1i, outAr, outAi);
        cmul(gd.m2[4], gd.m2[5], a0r, a0i, outBr, outBi);
        cmac(gd.m2[6], gd.m2[7], a1r, a1i, outBr, outBi);
      }
    }
    quant_tile(outAr, sA, qar[v], accA);
    quant_tile(outAi, sA, qai[v], accA);
    quant_tile(outBr, sB, qbr[v], accB);
    quant_tile(outBi, sB, qbi[v], accB);
  }
}

template <typename R>
__device__ __forceinline__ void gq_wave_pairs(const GqSlot &sA, const GqSlot &sB, double kA, double kB, bool cross,
                                              int b, uint32_t n, const GateDesc &gd, const Geo &g, uint32_t *hA,
                                              uint32_t *hb, Acc &accA, Acc &accB) {
  const uint32_t L = (uint32_t)g.L;
  const uint32_t nwv = gridDim.x * 4, w0 = blockIdx.x * 4 + (threadIdx.x >> 6);
  auto pair_of = [&](uint32_t j) { return j < n ? w0 + j * nwv : w0; };  // past the end: pair w0 again
  auto rA = [&](uint32_t w) { return (cross ? w : ((w >> b) << (b + 1)) | (w & ((1u << b) - 1))) * kWr; };
  auto rB = [&](uint32_t w) { return cross ? w * kWr : rA(w) | (kWr << b); };
  R xa, xb;
  double qar[4], qai[4], qbr[4], qbi[4];
  auto step = [&](uint32_t j) {  // quantise pair j (in xa, xb), load pair j + 1, store pair j's symbols
    const uint32_t w = pair_of(j), wn = pair_of(j + 1);
    wr_pair_quant(wr_val(xa, kA), wr_val(xb, kB), rA(w), sA, sB, gd, qar, qai, qbr, qbi, accA, accB);
    wr_load(xa, sA.ws, L, rA(wn));
    wr_load(xb, sB.ws, L, rB(wn));
    wr_symbols(qar, qai, hA, g, sA.out, rA(w), accA);
    wr_symbols(qbr, qbi, hb, g, sB.out, rB(w), accB);
  };
  wr_load(xa, sA.ws, L, rA(w0));
  wr_load(xb, sB.ws, L, rB(w0));
  step(0);
  for (uint32_t j = 1; j < n; j++) step(j);
}

// The range pairs from an FP64 workspace one pair at a time (no loads
// ahead): the compact kernel's path for a pass whose codes do not fit int32.
__device__ __forceinline__ void gq_wave_pairs_fp64(const GqSlot &sA, const GqSlot &sB, bool cross, int b, uint32_t n,
                                                   const GateDesc &gd, const Geo &g, uint32_t *hA, uint32_t *hb,
                                                   Acc &accA, Acc &accB) {
  const uint32_t L = (uint32_t)g.L;
  const uint32_t nwv = gridDim.x * 4, w0 = blockIdx.x * 4 + (threadIdx.x >> 6);
  for (uint32_t j = 0; j < n; j++) {
    const uint32_t w = w0 + j * nwv;
    const uint32_t ra = (cross ? w : ((w >> b) << (b + 1)) | (w & ((1u << b) - 1))) * kWr;
    const uint32_t rb = cross ? w * kWr : ra | (kWr << b);
    WRange xa, xb;
    double qar[4], qai[4], qbr[4], qbi[4];
    wr_load(xa, sA.ws, L, ra);
    wr_load(xb, sB.ws, L, rb);
    wr_pair_quant(xa, xb, ra, sA, sB, gd, qar, qai, qbr, qbi, accA, accB);
    wr_symbols(qar, qai, hA, g, sA.out, ra, accA);
    wr_symbols(qbr, qbi, hb, g, sB.out, rb, accB);
  }
}

template <bool C32>
__global__ void __launch_bounds__(256, 2) k_gq_wave_pair(Slots sl, Geo g, const uint64_t *slot_slice,
                                                                   GateDesc gd, QuantParams qp, Ctl *ctl,
                                                                   uint32_t pass, const double *kscale) {
  if (ctl->flags) return;
  __shared__ uint32_t hA[kNSym], hB[kNSym];
  __shared__ uint64_t wred[4][4];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kNSym; i += 256) hA[i] = hB[i] = 0;
  __syncthreads();
  const uint32_t L = (uint32_t)g.L, nr = L / kWr;
  const int t = gd.tloc[0];
  const bool cross = t >= g.slice_log2;
  uint32_t uA, uB, npairs;
  int b = 0;
  if (cross) {
    const uint32_t sb = t - g.slice_log2, y = blockIdx.y;
    uA = ((y >> sb) << (sb + 1)) | (y & ((1u << sb) - 1));
    uB = uA | (1u << sb);
    npairs = nr;
  } else {
    uA = uB = blockIdx.y;
    b = t - 8;  // log2 of the range size
    npairs = nr / 2;
  }
  const uint32_t n = npairs / (gridDim.x * 4);
  const GqSlot sA = gq_slot(sl, g, slot_slice, gd, qp, uA), sB = gq_slot(sl, g, slot_slice, gd, qp, uB);
  // one slot: both ranges' results go to one histogram and one sum
  uint32_t *hb = cross ? hB : hA;
  Acc accA, accB;
  accA.zero();
  accB.zero();
  if (!C32)
    gq_wave_pairs<WRange>(sA, sB, 0.0, 0.0, cross, b, n, gd, g, hA, hb, accA, accB);
  else if (!ctl->wide)
    gq_wave_pairs<WRange32>(sA, sB, kscale[slot_slice[uA]], kscale[slot_slice[uB]], cross, b, n, gd, g, hA, hb,
                            accA, accB);
  else
    gq_wave_pairs_fp64(sA, sB, cross, b, n, gd, g, hA, hb, accA, accB);
  if (!cross) accA.merge(accB);
  write_partial(accA, hA, wred, sl, uA, blockIdx.x, ctl, pass);
  if (cross) write_partial(accB, hB, wred, sl, uB, blockIdx.x, ctl, pass);
}

// The paired gate_quant without pipelining, on tiles of 1024 amplitudes: used
// when chunks are longer than the pipelined kernel's tile (a tile must start
// at a chunk head).  Partial results are numbered as in the pipelined kernel.
template <int V>
__global__ void __launch_bounds__(256, 2) k_gate_quant_pair(Slots sl, Geo g, const uint64_t *slot_slice, GateDesc gd,
                                                            QuantParams qp, Ctl *ctl, uint32_t pass) {
  if (ctl->flags) return;
  __shared__ uint32_t hA[kNSym], hB[kNSym];
  __shared__ double bnd[2][V][4];
  __shared__ uint64_t wred[4][4];
  const uint32_t tid = threadIdx.x, T = 256;
  for (uint32_t s = tid; s < (uint32_t)kNSym; s += T) hA[s] = hB[s] = 0;
  const uint32_t C = T * V;  // pairs are only formed when L >= C
  const uint32_t ntiles = (uint32_t)(g.L / C);
  const int t = gd.tloc[0];
  const bool cross = t >= g.slice_log2;
  uint32_t uA, uB, npairs;
  int b = 0;
  if (cross) {
    const uint32_t sb = t - g.slice_log2, y = blockIdx.y;
    uA = ((y >> sb) << (sb + 1)) | (y & ((1u << sb) - 1));
    uB = uA | (1u << sb);
    npairs = ntiles;
  } else {
    uA = uB = blockIdx.y;
    b = t - (31 - __clz((int)C));
    npairs = ntiles / 2;
  }
  const double *aRe = sl.ws + (uint64_t)uA * 2 * g.L, *aIm = aRe + g.L;
  const double *bRe = sl.ws + (uint64_t)uB * 2 * g.L, *bIm = bRe + g.L;
  const SlotOut soA = slot_out(sl, g, uA), soB = slot_out(sl, g, uB);
  // controls never include the target bit: A's index decides for the pair
  const uint64_t gi_hi = slot_slice[uA] << g.slice_log2;
  const uint64_t mask_hi = gd.ctrl_mask & ~(g.L - 1);
  const bool hi_ok = (gi_hi & mask_hi) == (gd.ctrl_vals & mask_hi);
  const uint32_t mask_lo = (uint32_t)(gd.ctrl_mask & (g.L - 1)), vals_lo = (uint32_t)(gd.ctrl_vals & (g.L - 1));
  double sa, ra, ba, sb2, rb, bb;
  slot_quant(sl, qp, uA, sa, ra, ba);
  slot_quant(sl, qp, uB, sb2, rb, bb);
  Acc accA, accB;
  accA.zero();
  accB.zero();
  for (uint32_t w = blockIdx.x; w < npairs; w += gridDim.x) {
    uint32_t tA = w, tB = w;
    if (!cross) {
      tA = ((w >> b) << (b + 1)) | (w & ((1u << b) - 1));
      tB = tA | (1u << b);
    }
    const uint32_t obA = tA * C, obB = tB * C;
    double x0r[V], x0i[V], x1r[V], x1i[V];
#pragma unroll
    for (int v = 0; v < V; v++) {  // all loads first
      const uint32_t e = v * T + tid;
      x0r[v] = aRe[obA + e];
      x0i[v] = aIm[obA + e];
      x1r[v] = bRe[obB + e];
      x1i[v] = bIm[obB + e];
    }
    double qar[V], qai[V], qbr[V], qbi[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
      const uint32_t e = v * T + tid;
      const double a0r = x0r[v], a0i = x0i[v], a1r = x1r[v], a1i = x1i[v];
      double outAr = a0r, outAi = a0i, outBr = a1r, outBi = a1i;
      if (hi_ok && ((obA + e) & mask_lo) == vals_lo) {
        cmul(gd.m2[0], gd.m2[1], a0r, a0i, outAr, outAi);
        cmac(gd.m2[2], gd.m2[3], a1r, a1i, outAr, outAi);
        cmul(gd.m2[4], gd.m2[5], a0r, a0i, outBr, outBi);
        cmac(gd.m2[6], gd.m2[7], a1r, a1i, outBr, outBi);
      }
      double e1, e2;
      accA.ok &= quantise(outAr, sa, ra, ba, qar[v], e1);
      accA.ok &= quantise(outAi, sa, ra, ba, qai[v], e2);
      accA.emax = fmax(accA.emax, fmax(e1, e2));
      accB.ok &= quantise(outBr, sb2, rb, bb, qbr[v], e1);
      accB.ok &= quantise(outBi, sb2, rb, bb, qbi[v], e2);
      accB.emax = fmax(accB.emax, fmax(e1, e2));
    }
    tile_symbols<V, true>(qar, qai, hA, bnd, g, soA, obA, C, accA);
    tile_symbols<V, true>(qbr, qbi, hB, bnd, g, soB, obB, C, accB);
  }
  write_partial(accA, hA, wred, sl, uA, blockIdx.x, ctl, pass);
  write_partial(accB, hB, wred, sl, uB, cross ? blockIdx.x : gridDim.x + blockIdx.x, ctl, pass);
}

#if !CQ_FP32  // coding kernels: f64 build only
// ---------------------------------------------------------------- codebook
// One workgroup per slot.  Package-merge (Larmore & Hirschberg) in its
// coin-collector form: level 12 holds the leaves (sorted by count, then
// symbol); level l is the merge of the leaves with the pairwise packages of
// level l+1, a leaf first on equal weights.  The 2n-2 cheapest items of
// level 1 are selected.  A selected prefix of m items at level l holds the
// q_l lightest leaves and m - q_l packages, i.e. the first 2(m - q_l) items of
// level l+1; a leaf of rank i gets the length #{l : i < q_l}.  Canonical codes
// are the left-aligned starts of intervals of size 2^(12 - len) that tile
// [0, 4096) in (length, symbol) order; the same intervals fill the decoder
// table of the new record.

// Orders the LDS accesses of one wavefront's lanes around this point: the
// wavefront's LDS instructions execute in program order, so only the
// compiler has to be kept from moving accesses across it.
__device__ __forceinline__ void lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ void bitonic_sort(uint64_t *key, uint32_t P) {
  if (P <= 64) {  // one wavefront, in registers: no barrier between stages
    if (threadIdx.x < 64) {
      const uint32_t lane = threadIdx.x;
      uint64_t a = lane < P ? key[lane] : ~0ull;
      for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
          const uint64_t b = __shfl_xor(a, (int)j, 64);
          const bool asc = (lane & k) == 0, lower = (lane & j) == 0;
          a = (lower == asc) ? (a < b ? a : b) : (a < b ? b : a);
        }
      }
      if (lane < P) key[lane] = a;
    }
    __syncthreads();
    return;
  }
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t p = threadIdx.x; p < P / 2; p += blockDim.x) {
        uint32_t i = 2 * p - (p & (j - 1));  // (p / j) * 2j + p % j, j a power of two
        uint32_t ixj = i + j;
        bool asc = (i & k) == 0;
        uint64_t a = key[i], b = key[ixj];
        if ((a > b) == asc) {
          key[i] = b;
          key[ixj] = a;
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(256) k_codebook(Slots sl, const uint64_t *slot_slice, StateMeta nxt,
                                                  uint32_t nparts, Ctl *ctl, uint32_t pw_nchunks) {
  if (ctl->flags) return;
  __shared__ uint64_t key[kNSym];
  __shared__ uint32_t wgt[kNSym];
  __shared__ uint32_t LA[2 * kNSym], LB[2 * kNSym];
  __shared__ uint16_t LP[kLMax][kNSym];
  __shared__ uint8_t lens[kNSym];
  __shared__ uint32_t lav[kNSym];
  __shared__ uint16_t ent[kNSym];
  __shared__ __align__(16) uint16_t one[1 << kLMax];  // one-symbol decoder table
  __shared__ uint32_t q[kLMax + 1];
  __shared__ uint32_t chg[kLMax];
  __shared__ uint32_t scratch[20];
  __shared__ uint64_t s64[16];
  const uint32_t u = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) {
    if (u == 0) settle(ctl);
    sl.words[u] = 0;  // encode adds the slot's words
  }
  // the first 16 partial histograms (loaded now, summed below): every load
  // is issued before the sums' loads are waited for
  const uint4 *hp = (const uint4 *)(sl.hpart + (uint64_t)u * kGqParts * kNSym) + tid;
  uint4 x0[16];
#pragma unroll
  for (int i = 0; i < 16; i++) x0[i] = hp[i * (kNSym / 4)];  // i < kGqParts: in bounds
  {  // sums of the gate_quant workgroups of this slot (partials [0, nparts))
    uint64_t lo = 0, hi = 0, ne = 0, eb = 0;
    const uint64_t *pp = sl.part + (uint64_t)u * kGqParts * 4;
    if (tid < nparts) {
      lo = pp[4 * tid];
      hi = pp[4 * tid + 1];
      ne = pp[4 * tid + 2];
      eb = pp[4 * tid + 3];
    }
    for (int off = 32; off > 0; off >>= 1) {
      uint64_t ol = __shfl_xor(lo, off, 64), oh = __shfl_xor(hi, off, 64);
      uint64_t t = lo + ol;
      hi += oh + (t < lo);
      lo = t;
      ne += __shfl_xor(ne, off, 64);
      uint64_t oe = __shfl_xor(eb, off, 64);
      eb = oe > eb ? oe : eb;
    }
    if (lane_id() == 0) {
      s64[4 * (tid >> 6)] = lo;
      s64[4 * (tid >> 6) + 1] = hi;
      s64[4 * (tid >> 6) + 2] = ne;
      s64[4 * (tid >> 6) + 3] = eb;
    }
    __syncthreads();
    if (tid == 0) {
      for (uint32_t w = 1; w < blockDim.x / 64; w++) {
        uint64_t t = lo + s64[4 * w];
        hi += s64[4 * w + 1] + (t < lo);
        lo = t;
        ne += s64[4 * w + 2];
        eb = s64[4 * w + 3] > eb ? s64[4 * w + 3] : eb;
      }
      sl.sq[2 * u] = lo;
      sl.sq[2 * u + 1] = hi;
      sl.nesc[u] = (uint32_t)ne;
      atomicMax((unsigned long long *)&ctl->max_err_bits, (unsigned long long)eb);
      if (ne) atomicAdd((unsigned long long *)&ctl->escapes, (unsigned long long)ne);
    }
  }
  if (pw_nchunks) {  // pointwise-relative records: the slice's squared norm, a pairwise tree over its chunks
    __shared__ double ptree[256];
    const uint32_t T = blockDim.x;
    const double *cs = sl.csum + (uint64_t)u * pw_nchunks;
    uint32_t active;
    if (pw_nchunks >= T) {
      const uint32_t b = pw_nchunks / T;
      ptree[tid] = tree_sum(cs, (uint64_t)tid * b, b);
      active = T;
    } else {
      ptree[tid] = tid < pw_nchunks ? cs[tid] : 0.0;
      active = pw_nchunks;
    }
    __syncthreads();
    for (uint32_t m = active; m > 1; m >>= 1) {
      const double v = tid < m / 2 ? ptree[2 * tid] + ptree[2 * tid + 1] : 0.0;
      __syncthreads();
      if (tid < m / 2) ptree[tid] = v;
      __syncthreads();
    }
    if (tid == 0) {
      sl.sq[2 * u] = (uint64_t)__double_as_longlong(ptree[0]);
      sl.sq[2 * u + 1] = 0;
    }
  }
  // used symbols, compacted in symbol order (4 consecutive symbols per thread)
  uint32_t hv[4], cnt = 0;
  {  // histogram = sum of the partial histograms; all loads of a group of 16
     // partials are issued before the first add
    uint4 acc4 = make_uint4(0, 0, 0, 0);
    for (uint32_t p0 = 0; p0 < nparts; p0 += 16) {
      uint4 x[16];
#pragma unroll
      for (int i = 0; i < 16; i++) x[i] = p0 == 0 ? x0[i] : hp[(p0 + i) * (kNSym / 4)];  // p0 + i < kGqParts
#pragma unroll
      for (int i = 0; i < 16; i++) {
        if (p0 + i >= nparts) x[i] = make_uint4(0, 0, 0, 0);  // not written by this pass
        acc4.x += x[i].x;
        acc4.y += x[i].y;
        acc4.z += x[i].z;
        acc4.w += x[i].w;
      }
    }
    hv[0] = acc4.x;
    hv[1] = acc4.y;
    hv[2] = acc4.z;
    hv[3] = acc4.w;
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    cnt += hv[k] ? 1u : 0u;
    lens[tid * 4 + k] = 0;
  }
  uint32_t n;
  uint32_t pos = block_excl_scan(cnt, scratch, &n);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t s = tid * 4 + k;
    if (hv[k]) key[pos++] = ((uint64_t)hv[k] << 10) | s;
  }
  uint32_t P = 1;
  while (P < n) P <<= 1;
  for (uint32_t i = n + tid; i < P; i += blockDim.x) key[i] = ~0ull;
  __syncthreads();
  bitonic_sort(key, P);
  for (uint32_t i = tid; i < n; i += blockDim.x) wgt[i] = (uint32_t)(key[i] >> 10);
  __syncthreads();
  // Up to 64 leaves the levels are built by wavefront 0 alone, synchronised
  // by lds_order() (its LDS instructions run in program order) instead of
  // workgroup barriers; the other wavefronts wait at the barrier below.  Up
  // to 32 leaves a level has at most 63 items, one per lane: the merge ranks
  // are counted over broadcast lanes, in registers.
  const bool one_wave = n <= 64;
  if (n >= 2 && n <= 32 && tid < 64) {
    const uint32_t lane = tid;
    const uint32_t w = lane < n ? wgt[lane] : 0u;
    uint32_t cur = w, len_cur = n;
    int lfix = 1;
    for (int l = kLMax - 1; l >= 1; l--) {
      const uint32_t np = len_cur / 2;
      const uint32_t a = (uint32_t)__shfl((int)cur, (int)((2 * lane) & 63), 64);
      const uint32_t b = (uint32_t)__shfl((int)cur, (int)((2 * lane + 1) & 63), 64);
      const uint32_t pk = a + b;  // package `lane` (lane < np)
      uint32_t cl = 0, cp = 0;    // packages lighter than leaf `lane`; leaves not heavier than package `lane`
      for (uint32_t j = 0; j < n; j++) {
        const uint32_t wj = (uint32_t)__builtin_amdgcn_readlane((int)w, (int)j);
        cp += wj <= pk ? 1u : 0u;
        if (j < np) {
          const uint32_t pj = (uint32_t)__builtin_amdgcn_readlane((int)pk, (int)j);
          cl += pj < w ? 1u : 0u;
        }
      }
      if (lane < n) {
        LA[lane + cl] = w;
        LP[l][lane] = (uint16_t)(lane + cl);
      }
      if (lane < np) LA[lane + cp] = pk;
      const uint32_t len_nx = n + np;
      lds_order();
      const uint32_t nxv = lane < len_nx ? LA[lane] : 0u;
      lds_order();  // every lane has read LA before the next level writes it
      const bool same = len_nx == len_cur && __ballot(nxv != cur) == 0;
      cur = nxv;
      len_cur = len_nx;
      if (same) {
        lfix = l;
        break;
      }
    }
    uint32_t m = 2 * n - 2;  // the leaves before position m, counted by ballots
    for (int l = 1; l < kLMax; l++) {
      const int lp = l < lfix ? lfix : l;
      const uint32_t lo = (uint32_t)__popcll(__ballot(lane < n && LP[lp][lane] < m));
      if (lane == 0) q[l] = lo;
      m = 2 * (m - lo);
    }
    if (lane == 0) q[kLMax] = m;
  } else if (n >= 2 && (!one_wave || tid < 64)) {
    const uint32_t nthr = one_wave ? 64u : blockDim.x;
    uint32_t *cur = LA, *nx = LB;
    for (uint32_t i = tid; i < n; i += nthr) cur[i] = wgt[i];
    uint32_t len_cur = n;
    if (tid < kLMax) chg[tid] = 0;
    if (one_wave) lds_order(); else __syncthreads();
    // Level l is a function of level l + 1 alone, and so are the leaves'
    // positions in it.  Once a level equals the one above, every lower level
    // equals it too and has the same leaf positions: the loop stops there and
    // the levels below read LP[lfix].
    int lfix = 1;
    for (int l = kLMax - 1; l >= 1; l--) {
      const uint32_t np = len_cur / 2;
      const bool same_len = len_cur == n + np;
      bool diff = false;
      for (uint32_t i = tid; i < n; i += nthr) {
        const uint32_t wi = wgt[i];
        uint32_t lo = 0, hi = np;  // packages lighter than the leaf
        while (lo < hi) {
          uint32_t mid = (lo + hi) >> 1;
          if (cur[2 * mid] + cur[2 * mid + 1] < wi) lo = mid + 1; else hi = mid;
        }
        nx[i + lo] = wi;
        LP[l][i] = (uint16_t)(i + lo);
        diff |= !same_len || cur[i + lo] != wi;
      }
      for (uint32_t k = tid; k < np; k += nthr) {
        const uint32_t pv = cur[2 * k] + cur[2 * k + 1];
        uint32_t lo = 0, hi = n;  // leaves not heavier than the package
        while (lo < hi) {
          uint32_t mid = (lo + hi) >> 1;
          if (wgt[mid] <= pv) lo = mid + 1; else hi = mid;
        }
        nx[k + lo] = pv;
        diff |= !same_len || cur[k + lo] != pv;
      }
      if (diff) chg[l] = 1;
      if (one_wave) lds_order(); else __syncthreads();
      uint32_t *t = cur;
      cur = nx;
      nx = t;
      len_cur = n + np;
      if (!chg[l]) {  // the same value in every thread after the barrier
        lfix = l;
        break;
      }
    }
    if (tid < 64) {  // one wavefront: the leaves before position m, counted by ballots
      uint32_t m = 2 * n - 2;
      for (int l = 1; l < kLMax; l++) {
        const int lp = l < lfix ? lfix : l;
        uint32_t lo = 0;  // LP[lp][.] increases with the leaf index
        for (uint32_t i0 = 0; i0 < n; i0 += 64) {
          const uint32_t i = i0 + tid;
          lo += (uint32_t)__popcll(__ballot(i < n && LP[lp][i] < m));
        }
        if (tid == 0) q[l] = lo;
        m = 2 * (m - lo);
      }
      if (tid == 0) q[kLMax] = m;
    }
  }
  __syncthreads();
  if (n >= 2)
    for (uint32_t i = tid; i < n; i += blockDim.x) {
      uint32_t len = 0;
      for (int l = 1; l <= kLMax; l++) len += i < q[l] ? 1u : 0u;
      lens[key[i] & 1023] = (uint8_t)len;
    }
  __syncthreads();
  // canonical order (length, symbol)
  for (uint32_t i = tid; i < n; i += blockDim.x) {
    const uint32_t s = (uint32_t)(key[i] & 1023);
    key[i] = ((uint64_t)lens[s] << 10) | s;
  }
  __syncthreads();
  bitonic_sort(key, P);
  uint32_t sz[4], loc = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    uint32_t i = tid * 4 + k;
    sz[k] = i < n ? (1u << (kLMax - (uint32_t)(key[i] >> 10))) : 0u;
    loc += sz[k];
  }
  uint32_t tot;
  uint32_t pre = block_excl_scan(loc, scratch, &tot);
  uint32_t *codes = sl.codes + (uint64_t)u * kNSym;
  uint16_t *tab = sl.symtab + (uint64_t)u * kNSym;
  for (uint32_t s = tid; s < (uint32_t)kNSym; s += blockDim.x) codes[s] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; k++) {
    uint32_t i = tid * 4 + k;
    if (i < n) {
      uint32_t len = (uint32_t)(key[i] >> 10), sym = (uint32_t)(key[i] & 1023);
      uint32_t code = pre >> (kLMax - len);
      codes[sym] = (code << 8) | len;
      const uint16_t e = (uint16_t)(sym | (len << 10));
      tab[i] = e;
      ent[i] = e;
      lav[i] = pre;
    }
    pre += sz[k];
  }
  __syncthreads();
  // decoder table of the new record: the one-symbol table first (in LDS),
  // then entries with a second symbol where both codes fit the 12 bits.
  // Entry e belongs to the last code whose interval starts at or before e:
  // every code marks its first entry with its index, a prefix maximum
  // spreads the marks (starts increase with the index; code 0 starts at 0).
  {
    constexpr uint32_t kPer = (1u << kLMax) / 256;  // entries per thread: two uint4
    uint4 *one4 = (uint4 *)one + 2 * tid;
    one4[0] = make_uint4(0, 0, 0, 0);
    one4[1] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    for (uint32_t i = tid; i < n; i += blockDim.x)
      if (lav[i] < (1u << kLMax)) one[lav[i]] = (uint16_t)i;
    __syncthreads();
    uint32_t m[kPer], run = 0;
    {
      const uint4 a = one4[0], b = one4[1];
      const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
      for (uint32_t k = 0; k < kPer; k++) {
        const uint32_t x = (w[k >> 1] >> (16 * (k & 1))) & 0xffffu;
        run = x > run ? x : run;
        m[k] = run;
      }
    }
    // exclusive prefix maximum of the threads' maxima
    uint32_t inc = run;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)inc, off, 64);
      if (lane_id() >= (uint32_t)off) inc = y > inc ? y : inc;
    }
    if (lane_id() == 63) scratch[tid >> 6] = inc;
    uint32_t before = (uint32_t)__shfl_up((int)inc, 1, 64);
    if (lane_id() == 0) before = 0;
    __syncthreads();
    for (uint32_t w = 0; w < (tid >> 6); w++) before = scratch[w] > before ? scratch[w] : before;
    uint32_t w[8];
#pragma unroll
    for (uint32_t k = 0; k < kPer; k += 2) {
      const uint32_t x0 = m[k] > before ? m[k] : before, x1 = m[k + 1] > before ? m[k + 1] : before;
      w[k >> 1] = (uint32_t)ent[x0] | ((uint32_t)ent[x1] << 16);
    }
    one4[0] = make_uint4(w[0], w[1], w[2], w[3]);
    one4[1] = make_uint4(w[4], w[5], w[6], w[7]);
  }
  __syncthreads();
  uint32_t *dt = nxt.dtab + slot_slice[u] * (1u << kLMax);
#pragma unroll
  for (uint32_t k = 0; k < (1u << kLMax) / 256; k++) {  // all LDS reads issued before the stores
    const uint32_t e = k * 256 + tid;
    const uint32_t s1 = one[e] & 1023u, l1 = one[e] >> 10;
    const uint32_t e2 = (e << l1) & ((1u << kLMax) - 1);
    const uint32_t s2 = one[e2] & 1023u, l2 = one[e2] >> 10;
    dt[e] = dtab_entry(s1, l1, s2, l2, s1 != 0 && s2 != 0 && l1 + l2 <= (uint32_t)kLMax);
  }
  if (tid == 0) sl.nused[u] = n;
}

// ------------------------------------------------------------------ encode
// One wavefront per chunk, four consecutive symbols per lane per step: code
// lengths -> wavefront prefix sum -> bit positions; a lane's codes are joined
// into one 64-bit field and OR-ed into the chunk's words staged in LDS.
// Four wavefronts only load and code (a chunk each per round); a fifth only
// stores the previous round's chunks to their fixed-size staging slots.  So
// no wavefront mixes loads and stores (a wait for a load would otherwise
// also wait for earlier stores), and the LDS chunk buffers are double-buffered
// between rounds.

// A field of n <= 64 bits at bit position pos: at most three words, each
// touched only where the field has bits in it.
__device__ __forceinline__ void put_field(uint32_t *lw, uint64_t v, int n, uint32_t pos) {
  if (n <= 0) return;
  const uint32_t w = (uint32_t)(pos >> 5);
  const int off = (int)(pos & 31);
  const uint64_t f = v << (64 - n);  // left-aligned
  atomicOr(&lw[w], (uint32_t)(f >> (32 + off)));
  if (off + n > 32) atomicOr(&lw[w + 1], (uint32_t)(f >> off));
  if (off + n > 64) atomicOr(&lw[w + 2], (uint32_t)(f << (32 - off)));
}

constexpr int kEncWaves = 4;  // coding wavefronts; one more stores

// Symbols j .. j + 3 of a chunk of B values (the zero difference R past the end, never coded).
__device__ __forceinline__ uint2 enc_syms(const uint16_t *sym, uint64_t j, uint64_t B) {
  if (j + 3 < B) return *(const uint2 *)(sym + j);  // four aligned symbols in one load
  uint32_t t[4];
#pragma unroll
  for (int k = 0; k < 4; k++) t[k] = j + k < B ? sym[j + k] : (uint32_t)kR;
  return make_uint2(t[0] | (t[1] << 16), t[2] | (t[3] << 16));
}

// The store wavefront's work for one round: the round's NCH chunks (those
// below ce) are packed after the block's earlier words.  Lane k < NCH holds
// chunk k's word count, a prefix over those lanes places the chunks, and one
// flat loop copies every word and clears it for the round after next, so
// the chunks do not form a chain of LDS round trips.
template <uint32_t NCH, bool CC>
__device__ __forceinline__ void enc_store_round(const Slots &sl, const Geo &g, uint32_t u, uint32_t c0, uint32_t ce,
                                                uint32_t *lw_round, const uint32_t *cnw_round, uint32_t W,
                                                uint32_t *blk, uint32_t &packed) {
  static_assert(NCH >= 1 && NCH <= 8, "one row of lanes");
  const uint32_t lane = lane_id();
  const uint32_t nch = c0 < ce ? (ce - c0 < NCH ? ce - c0 : NCH) : 0u;
  const uint32_t v = lane < nch ? cnw_round[lane] : 0u;
  const uint32_t nw = CC ? v & 0x7FFFFFFFu : v;
  uint32_t inc = nw;  // inclusive prefix over lanes 0..7 (row 0)
  inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x111 /* row_shr:1 */, 0xF, 0xF, true);
  inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x112 /* row_shr:2 */, 0xF, 0xF, true);
  inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x114 /* row_shr:4 */, 0xF, 0xF, true);
  const uint32_t pre = inc - nw;
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)inc, (int)NCH - 1);
  if (lane < nch) sl.chunk_words[(uint64_t)u * g.nchunks + c0 + lane] = (packed + pre) | (CC ? v & 0x80000000u : 0u);
  uint32_t pk[NCH];
#pragma unroll
  for (uint32_t k = 0; k < NCH; k++) pk[k] = (uint32_t)__builtin_amdgcn_readlane((int)pre, (int)k);
  for (uint32_t i = lane; i < total; i += 64) {
    uint32_t off = i;  // word i of the round lies in the last chunk whose prefix is at most i
#pragma unroll
    for (uint32_t k = 1; k < NCH; k++)
      if (i >= pk[k]) off = k * W + (i - pk[k]);
    blk[packed + i] = lw_round[off];
    lw_round[off] = 0;
  }
  packed += total;
}

// Chunks [cb, ce) of slot blockIdx.y; coding wavefront w takes chunks cb + w,
// cb + w + 4, ...; every wavefront runs the same number of rounds so that
// barriers line up.  STEPS = ceil(B / 256) steps of 256 symbols per chunk.
// FMT: bit 0 zero chunks (no words), bit 1 constant chunks (the head only,
// marked by bit 31 of the chunk's word offset).
template <int STEPS, int FMT>
__global__ void __launch_bounds__(64 * (kEncWaves + 1), STEPS > 2 ? 2 : 4) k_encode(Slots sl, Geo g, uint32_t chunks_per_block,
                                                                    const Ctl *ctl) {
  constexpr bool ZC = (FMT & 1) != 0, CC = (FMT & 2) != 0;
  if (ctl->flags) return;
  extern __shared__ uint32_t lw_all[];  // [2][kEncWaves][stage_words]
  __shared__ __align__(16) uint32_t codes[kNSym];
  __shared__ uint32_t cnw[2][kEncWaves];  // words of each coded chunk
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  const uint32_t u = blockIdx.y;
  const uint32_t cb = blockIdx.x * chunks_per_block;
  const uint32_t ce = cb + chunks_per_block < g.nchunks ? cb + chunks_per_block : g.nchunks;
  const uint32_t W = sl.stage_words;
  static_assert(64 * (kEncWaves + 1) >= kNSym / 4, "one uint4 of the code table per thread");
  if (threadIdx.x < (uint32_t)kNSym / 4)  // the code table with one load per thread
    ((uint4 *)codes)[threadIdx.x] = ((const uint4 *)(sl.codes + (uint64_t)u * kNSym))[threadIdx.x];
  // chunk buffers start cleared; afterwards the store wavefront clears the
  // words it copies out
  for (uint32_t i = threadIdx.x; i < 2u * kEncWaves * sl.stage_words; i += blockDim.x) lw_all[i] = 0;
  const uint64_t Bc = 1ull << g.chunk_log2;
  const uint32_t rounds = (chunks_per_block + kEncWaves - 1) / kEncWaves;
  const uint64_t slot0 = (uint64_t)u * 2 * g.L;
  // the block's chunks, packed from the start of its staging region
  // (store wavefront only; capacity W words per chunk)
  uint32_t *blk = sl.stage + ((uint64_t)u * g.nchunks + cb) * W;
  uint32_t packed = 0;
  // symbols arrive two rounds ahead, escaped differences one round ahead:
  // round r issues the symbol loads of round r + 2 and the escape loads of
  // round r + 1 (whose symbols are already there), then codes round r.  An
  // escape load is issued by every lane through a buffer resource; lanes
  // without an escape use an offset past the end, which reads nothing.
  const __amdgpu_buffer_rsrc_t escb = buf_rsrc(sl.esc + slot0, (uint32_t)(16 * g.L));
  uint2 cur[STEPS], nxt[STEPS], nn[STEPS];
  int64_t ecur[STEPS][4] = {}, enxt[STEPS][4] = {};
  auto load_syms = [&](uint2 (&d)[STEPS], uint32_t r) {
    const uint32_t c = cb + r * kEncWaves + wave;
    const bool live = c < ce && r < rounds;
    const uint16_t *sym = sl.sym + slot0 + (uint64_t)(c < ce ? c : 0) * Bc;
    if (live && Bc >= 256) {  // whole steps of 256: every lane's four symbols lie inside the chunk
#pragma unroll
      for (int i = 0; i < STEPS; i++) d[i] = *(const uint2 *)(sym + i * 256 + 4 * lane);
    } else {
      const uint64_t B = live ? Bc : 0;
#pragma unroll
      for (int i = 0; i < STEPS; i++) d[i] = enc_syms(sym, (uint64_t)i * 256 + 4 * (uint64_t)lane, B);
    }
  };
  // escaped differences of a round whose symbols are in d; nothing is loaded
  // (and e is never read) when no lane of the wavefront holds an escape
  auto load_escs = [&](int64_t (&e)[STEPS][4], const uint2 (&d)[STEPS], uint32_t r) {
    const uint32_t c = cb + r * kEncWaves + wave;
    const uint64_t B = c < ce && r < rounds ? Bc : 0;
    bool zsym = false;
#pragma unroll
    for (int i = 0; i < STEPS; i++)
      zsym = zsym || (d[i].x & 0xffffu) == 0 || (d[i].x >> 16) == 0 || (d[i].y & 0xffffu) == 0 || (d[i].y >> 16) == 0;
    if (__ballot(zsym) == 0) return;
#pragma unroll
    for (int i = 0; i < STEPS; i++) {
      const uint32_t sv[4] = {d[i].x & 0xffffu, d[i].x >> 16, d[i].y & 0xffffu, d[i].y >> 16};
      bool is_esc[4];
#pragma unroll
      for (int k = 0; k < 4; k++) is_esc[k] = (uint64_t)i * 256 + 4 * (uint64_t)lane + k < B && sv[k] == 0;
      // the group is step i's 256 positions (or the chunk, below 256): escapes
      // of lower lanes come first, then this lane's in order
      uint32_t r = lanes_below(__ballot(is_esc[0])) + lanes_below(__ballot(is_esc[1])) +
                   lanes_below(__ballot(is_esc[2])) + lanes_below(__ballot(is_esc[3]));
      const uint64_t gb = (uint64_t)c * Bc + (uint64_t)i * 256;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const uint32_t off = is_esc[k] ? (uint32_t)(8 * (gb + r)) : 0xFFFFFFF0u;
        r += is_esc[k] ? 1u : 0u;
        const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(escb, off, 0, 0);
        e[i][k] = (int64_t)(((uint64_t)x.y << 32) | x.x);
      }
    }
  };
  if (wave < kEncWaves) {
    load_syms(cur, 0);
    load_syms(nxt, 1);
    load_escs(ecur, cur, 0);
  }
  __syncthreads();  // code table in LDS, chunk buffers cleared
  for (uint32_t r = 0; r <= rounds; r++) {  // one more round: the store wavefront drains the last one
    const uint32_t buf = r & 1u;
    if (wave < kEncWaves && r < rounds) {
      load_syms(nn, r + 2);
      load_escs(enxt, nxt, r + 1);
      const uint32_t c = cb + r * kEncWaves + wave;
      const bool active = c < ce;
      const uint32_t B = active ? (uint32_t)Bc : 0u;
      const bool full = B == 256u * STEPS;  // every position of every step lies inside the chunk
      uint32_t *lw = lw_all + (uint64_t)(buf * kEncWaves + wave) * W;
      uint32_t run = 0;  // the buffer lw is all zero (cleared by the store wavefront)
      bool nz = false;   // zero-chunk records: a symbol other than the zero difference
      bool cchunk = false;  // constant-chunk records: every symbol after the head is the zero difference
      if (CC) {  // positions past the chunk's end hold the zero difference
        bool rest = false;
#pragma unroll
        for (int i = 0; i < STEPS; i++) {
          const uint32_t x = (i == 0 && lane == 0) ? ((cur[i].x & 0xffff0000u) | (uint32_t)kR) : cur[i].x;
          rest = rest || x != ((uint32_t)kR | ((uint32_t)kR << 16)) || cur[i].y != ((uint32_t)kR | ((uint32_t)kR << 16));
        }
        cchunk = active && __ballot(rest) == 0;
      }
#pragma unroll
      for (int i = 0; i < STEPS; i++) {
        const uint32_t j = (uint32_t)i * 256u + 4u * lane;
        uint32_t sv[4], cw[4], bl = 0;
        sv[0] = cur[i].x & 0xffffu;
        sv[1] = cur[i].x >> 16;
        sv[2] = cur[i].y & 0xffffu;
        sv[3] = cur[i].y >> 16;
        uint64_t z[4];   // zigzag code of an escaped difference
        uint32_t nb[4];  // its bit length (0: no escape)
        bool esc[4], any = false;
#pragma unroll
        for (int k = 0; k < 4; k++) cw[k] = codes[sv[k]];  // every symbol is a table index
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const bool valid = (full || j + k < B) && !(CC && cchunk && j + k > 0);  // a constant chunk codes its head only
          cw[k] = valid ? cw[k] : 0u;
          bl += cw[k] & 0xffu;
          esc[k] = valid && sv[k] == 0;
          any = any || esc[k];
          z[k] = 0;
          nb[k] = 0;
        }
        if (ZC) {  // positions past the chunk's end hold the zero difference
          constexpr uint32_t kRR = (uint32_t)kR | ((uint32_t)kR << 16);
          nz = nz || cur[i].x != kRR || cur[i].y != kRR;
        }
        const bool wave_esc = __ballot(any) != 0;
        if (wave_esc) {
#pragma unroll
          for (int k = 0; k < 4; k++) {
            if (esc[k]) {
              z[k] = zigzag(ecur[i][k]);
              nb[k] = (uint32_t)bitlen64(z[k]);
              bl += kEscBits + nb[k];
            }
          }
        }
        const uint32_t inc = wave_incl_scan(bl);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        uint32_t pos = run + inc - bl;
        run += tot;
        if (pos + bl > 32u * W) continue;  // cannot happen for a consistent codebook
        if (!wave_esc) {  // four codes of at most 12 bits: one field
          uint64_t acc = 0;
#pragma unroll
          for (int k = 0; k < 4; k++) acc = (acc << (cw[k] & 0xffu)) | (cw[k] >> 8);
          put_field(lw, acc, (int)bl, pos);
        } else if (bl <= 64) {  // the lane's codes and escape payloads as one field (every part below 64 bits)
          uint64_t acc = 0;
#pragma unroll
          for (int k = 0; k < 4; k++) {
            acc = (acc << (cw[k] & 0xffu)) | (cw[k] >> 8);
            if (nb[k]) {  // an escape: 6-bit length, then the payload (|d| >= R: never empty)
              acc = (acc << kEscBits) | nb[k];
              acc = (acc << nb[k]) | z[k];
            }
          }
          put_field(lw, acc, (int)bl, pos);
        } else {  // two symbols per field where they fit in 64 bits, else a field per code and per payload
#pragma unroll
          for (int k = 0; k < 4; k += 2) {
            const uint32_t l0 = (cw[k] & 0xffu) + (nb[k] ? kEscBits + nb[k] : 0u);
            const uint32_t l1 = (cw[k + 1] & 0xffu) + (nb[k + 1] ? kEscBits + nb[k + 1] : 0u);
            if (l0 + l1 <= 64) {
              uint64_t acc = 0;
#pragma unroll
              for (int kk = k; kk < k + 2; kk++) {
                acc = (acc << (cw[kk] & 0xffu)) | (cw[kk] >> 8);
                if (nb[kk]) {
                  acc = (acc << kEscBits) | nb[kk];
                  acc = (acc << nb[kk]) | z[kk];
                }
              }
              put_field(lw, acc, (int)(l0 + l1), pos);
              pos += l0 + l1;
            } else {
#pragma unroll
              for (int kk = k; kk < k + 2; kk++) {
                const uint32_t len = cw[kk] & 0xffu;
                put_field(lw, cw[kk] >> 8, (int)len, pos);
                pos += len;
                if (nb[kk]) {  // 6-bit length and payload: at most 54 bits
                  put_field(lw, ((uint64_t)nb[kk] << nb[kk]) | z[kk], kEscBits + (int)nb[kk], pos);
                  pos += kEscBits + nb[kk];
                }
              }
            }
          }
        }
      }
      uint32_t nw = (uint32_t)((run + 31) >> 5);
      if (nw > W) nw = W;  // at most 68 bits per value: never reached by a consistent codebook
      bool zchunk = false;
      if (ZC && __ballot(nz) == 0) {  // zero-chunk records: an all-zero chunk keeps no words
        for (uint32_t i = lane; i < nw; i += 64) lw[i] = 0;  // after the lanes' writes (LDS in order)
        nw = 0;
        zchunk = true;
      }
      const uint32_t mark = (CC && cchunk && !zchunk) ? 0x80000000u : 0u;
      if (lane == 0) cnw[buf][wave] = active ? (nw | mark) : 0u;
#pragma unroll
      for (int i = 0; i < STEPS; i++) {
        cur[i] = nxt[i];
        nxt[i] = nn[i];
#pragma unroll
        for (int k = 0; k < 4; k++) ecur[i][k] = enxt[i][k];
      }
    } else if (wave == kEncWaves && r > 0) {  // store the previous round's chunks, packed
      const uint32_t pb = buf ^ 1u;
      enc_store_round<kEncWaves, CC>(sl, g, u, cb + (r - 1) * kEncWaves, ce, lw_all + (uint64_t)pb * kEncWaves * W,
                                     cnw[pb], W, blk, packed);
    }
    lds_sync();  // round r coded; round r - 1 read out of LDS
  }
  if (wave == kEncWaves && lane == 0) {
    sl.blk_words[(uint64_t)u * kMaxEncBlocks + blockIdx.x] = packed;
    if (packed) atomicAdd(&sl.words[u], packed);
  }
}

// ------------------------------------------------------------------ carried records
// SIM_OPT passes that leave slices as they are: record j of the input arena
// becomes record dst[i] = src[i] (groups where the gate is the identity) or a
// relabelled slice of the output arena, copied byte for byte with its
// metadata and decoder table.  A plan launch (one workgroup) places the
// records after the arena position begin_pass left, as one batch whose size
// the next batch's codebook (or the next pass) settles; a copy launch moves
// them.  Carried records keep the input's code width.
__global__ void __launch_bounds__(1024) k_carry_plan(Ctl *ctl, StateMeta cur, const uint64_t *src, uint64_t count,
                                                     uint64_t cap, uint64_t *off, uint32_t pass) {
  if (ctl->flags) return;
  __shared__ uint64_t wsum[16][2];
  const uint32_t tid = threadIdx.x, T = blockDim.x, lane = lane_id(), wave = tid >> 6;
  const uint64_t base = ctl->bump;
  uint64_t run = 0, exact = 0;  // bytes placed by earlier rounds (uniform)
  for (uint64_t i0 = 0; i0 < count; i0 += T) {
    const uint64_t i = i0 + tid;
    const uint64_t len = i < count ? cur.rec_len[src[i]] : 0u;
    const uint64_t ba = (len + kRecAlign - 1) & ~(kRecAlign - 1);
    // 64-bit exclusive scan of the aligned sizes (and sum of the exact ones) over the block
    uint64_t inc = ba, le = len;
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(inc, d, 64);
      if (lane >= (uint32_t)d) inc += y;
    }
    for (int d = 32; d > 0; d >>= 1) le += __shfl_xor(le, d, 64);
    if (lane == 63) wsum[wave][0] = inc;
    if (lane == 0) wsum[wave][1] = le;
    __syncthreads();
    uint64_t before = 0, tot = 0, tlen = 0;
    for (uint32_t w = 0; w < T / 64; w++) {
      if (w < wave) before += wsum[w][0];
      tot += wsum[w][0];
      tlen += wsum[w][1];
    }
    __syncthreads();
    if (i < count) off[i] = base + run + before + inc - ba;
    run += tot;
    exact += tlen;
  }
  if (tid == 0) {
    if (base + run > cap) {
      fail(ctl, kFlagOverflow, pass);
      return;
    }
    ctl->pending_bump = run;
    ctl->pending_bytes = exact;
    if (ctl->wide) ctl->wide_next = 1;
  }
}

__global__ void __launch_bounds__(256) k_carry_copy(const Ctl *ctl, StateMeta cur, StateMeta nxt, const uint8_t *in,
                                                    uint8_t *out, const uint64_t *src, const uint64_t *dst,
                                                    uint64_t count, const uint64_t *off) {
  if (ctl->flags) return;
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  for (uint64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const uint64_t j = src[i], t = dst[i];
    const uint32_t len = cur.rec_len[j];
    const uint8_t *a = in + cur.rec_off[j];
    uint8_t *b = out + off[i];
    // records start on 256-byte boundaries and hold whole 4-byte words
    for (uint32_t k = tid; k < len / 16; k += T) ((uint4 *)b)[k] = ((const uint4 *)a)[k];
    for (uint32_t k = (len / 16) * 4 + tid; k < len / 4; k += T) ((uint32_t *)b)[k] = ((const uint32_t *)a)[k];
    const uint4 *dt = (const uint4 *)(cur.dtab + j * (1u << kLMax));
    uint4 *dn = (uint4 *)(nxt.dtab + t * (1u << kLMax));
    for (uint32_t k = tid; k < (1u << kLMax) / 4; k += T) dn[k] = dt[k];
    if (tid == 0) {
      nxt.rec_off[t] = off[i];
      nxt.rec_len[t] = len;
      nxt.step[t] = cur.step[j];
      nxt.sq[2 * t] = cur.sq[2 * j];
      nxt.sq[2 * t + 1] = cur.sq[2 * j + 1];
    }
  }
}

// ------------------------------------------------------------------ chunk runs
// SIM_CHUNK_RUNS: chunk c starts a run unless its staged stream -- word
// count, constant mark and words -- equals chunk c - 1's.  Two launches over
// tiles of kRunTile chunks (grid: tiles x slots): the first marks the run
// starts and counts each tile's runs and their words; the second adds the
// counts of the tiles before its own and numbers its runs with block scans.
// The first kMaxRuns runs get their first chunk and the word offset of their
// stream (with the mark); nruns and run_words hold the slot's totals, from
// which finish chooses the record layout.
struct ChunkSpan {  // a chunk's staged words (offset from the slot's staging region), count and mark
  uint64_t w0;
  uint32_t n, mark;
};
// chunk c's words: staged at block b's region (b * cpb chunks in) plus its
// packed offset; they end at the next chunk's offset or the block's total
__device__ __forceinline__ ChunkSpan chunk_span(const uint32_t *cw, const uint32_t *bw, uint32_t nch, uint32_t cpb,
                                                uint32_t W, uint32_t c) {
  const uint32_t b = c / cpb, x = cw[c], off = x & 0x7FFFFFFFu;
  const uint32_t end = (c + 1 < nch && (c + 1) / cpb == b) ? (cw[c + 1] & 0x7FFFFFFFu) : bw[b];
  return ChunkSpan{(uint64_t)b * cpb * W + off, end - off, x & 0x80000000u};
}

__global__ void __launch_bounds__(kRunTile) k_runs_mark(Slots sl, Geo g, uint32_t cpb, const Ctl *ctl) {
  if (ctl->flags) return;
  __shared__ uint32_t scan[17];
  const uint32_t t = blockIdx.x, u = blockIdx.y, tid = threadIdx.x;
  const uint32_t nch = g.nchunks, W = sl.stage_words, c = t * kRunTile + tid;
  const uint32_t *cw = sl.chunk_words + (uint64_t)u * nch;
  const uint32_t *bw = sl.blk_words + (uint64_t)u * kMaxEncBlocks;
  const uint32_t *stage = sl.stage + (uint64_t)u * nch * W;
  uint32_t start = 0, nw = 0;
  if (c < nch) {
    const ChunkSpan a = chunk_span(cw, bw, nch, cpb, W, c);
    nw = a.n;
    start = 1;
    if (c > 0) {
      const ChunkSpan p = chunk_span(cw, bw, nch, cpb, W, c - 1);
      if (p.n == a.n && p.mark == a.mark) {
        uint32_t i = 0;
        while (i < a.n && stage[a.w0 + i] == stage[p.w0 + i]) i++;
        start = i == a.n ? 0u : 1u;
      }
    }
    sl.run_start[(uint64_t)u * nch + c] = (uint8_t)start;
  }
  uint32_t runs, words;
  block_excl_scan(start, scan, &runs);
  block_excl_scan(start ? nw : 0u, scan, &words);
  if (tid == 0) {
    const uint64_t k = (uint64_t)u * g.run_tiles + t;
    sl.run_tile[2 * k] = runs;
    sl.run_tile[2 * k + 1] = words;
  }
}

__global__ void __launch_bounds__(kRunTile) k_runs_number(Slots sl, Geo g, uint32_t cpb, const Ctl *ctl) {
  if (ctl->flags) return;
  __shared__ uint32_t scan[17];
  const uint32_t t = blockIdx.x, u = blockIdx.y, tid = threadIdx.x;
  const uint32_t nch = g.nchunks, c = t * kRunTile + tid;
  const uint32_t *tiles = sl.run_tile + 2ull * u * g.run_tiles;
  // runs and words of the tiles before this one (and, for the last tile, of all)
  const uint32_t upto = t + 1 == g.run_tiles ? g.run_tiles : t;
  uint32_t r0 = 0, w0 = 0, rall = 0, wall = 0;
  for (uint32_t i = tid; i < upto; i += kRunTile) {
    if (i < t) {
      r0 += tiles[2 * i];
      w0 += tiles[2 * i + 1];
    }
    rall += tiles[2 * i];
    wall += tiles[2 * i + 1];
  }
  uint32_t x;
  block_excl_scan(r0, scan, &x);
  r0 = x;
  block_excl_scan(w0, scan, &x);
  w0 = x;
  block_excl_scan(rall, scan, &x);
  rall = x;
  block_excl_scan(wall, scan, &x);
  wall = x;
  uint32_t *src = sl.run_src + (uint64_t)u * kMaxRuns;
  uint32_t *woff = sl.run_woff + (uint64_t)u * (kMaxRuns + 1);
  // every tile, also past kMaxRuns runs: a slot of exactly kMaxRuns runs
  // still takes the run layout, and finish reads every block's first run
  uint32_t start = 0, nw = 0, mark = 0;
  if (c < nch) {
    start = sl.run_start[(uint64_t)u * nch + c];
    const ChunkSpan a = chunk_span(sl.chunk_words + (uint64_t)u * nch, sl.blk_words + (uint64_t)u * kMaxEncBlocks,
                                   nch, cpb, sl.stage_words, c);
    nw = a.n;
    mark = a.mark;
  }
  uint32_t tr, tw;
  const uint32_t r = r0 + block_excl_scan(start, scan, &tr);
  const uint32_t w = w0 + block_excl_scan(start ? nw : 0u, scan, &tw);
  if (start && r < kMaxRuns) {
    src[r] = c;
    woff[r] = w | mark;
  }
  // the first run of each encode block: the runs starting before its first chunk
  if (c < nch && c % cpb == 0) sl.blk_run[(uint64_t)u * kMaxEncBlocks + c / cpb] = r;
  if (t + 1 == g.run_tiles && tid == 0) {
    sl.nruns[u] = rall;
    sl.run_words[u] = wall;
    if (rall <= kMaxRuns) woff[rall] = wall;
  }
}

// The layout of slot v's record: chunk runs when the mode is on, the slot
// has at most kMaxRuns runs and that layout is the smaller; its bytes.
__device__ __forceinline__ uint64_t slot_rec_bytes(const Slots &sl, const Geo &g, uint32_t v, uint32_t n_used,
                                                   uint32_t words, bool &runs) {
  const uint64_t nch = g.nchunks, plain = rec_bytes(n_used, g.nchunks, words);
  runs = false;
  if (!g.chunk_runs) return plain;
  const uint64_t R = sl.nruns[v], Wr = sl.run_words[v];
  if (R > kMaxRuns || 8 * R + 8 + 4 * Wr >= 4 * (nch + 1) + 4ull * words) return plain;
  runs = true;
  return plain - 4 * (nch + 1) - 4ull * words + 8 * R + 8 + 4 * Wr;
}

// ------------------------------------------------------------------ finish
// Workgroup (b, u) takes encode block b of slot u.  Every workgroup sizes all
// records of the batch (slot order), so it knows its record's offset and the
// batch total, which must fit the arena (else the pass fails with an overflow
// flag); the words before its block are the totals of the slot's earlier
// blocks.  It writes its chunks' offsets and copies their packed words into
// the record; block 0 also writes the header, symbol table and last offset
// and the slice's metadata.  The batch total becomes pending and is counted
// by the next launch that starts a batch or pass.

__global__ void __launch_bounds__(256) k_finish(Slots sl, Geo g, const uint64_t *slot_slice, int nslots,
                                                QuantParams qp, uint8_t *arena, uint64_t cap, StateMeta nxt,
                                                uint32_t cpb, Ctl *ctl, uint32_t pass) {
  if (ctl->flags) return;
  __shared__ uint64_t s64[16];
  const uint32_t u = blockIdx.y, b = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
  const uint32_t nch = g.nchunks;
  const uint32_t cb = b * cpb, ce = cb + cpb < nch ? cb + cpb : nch;
  // Every load whose address is known at entry goes out before the first
  // wait: the first element of each loop below, this block's first staged
  // words (up to kU per thread, within the block's staging region), the arena
  // position and, for block 0, the slot's header fields and symbol table.
  constexpr uint32_t kU = 8;
  const uint32_t *src = sl.stage + ((uint64_t)u * nch + cb) * sl.stage_words;
  const uint64_t region = (uint64_t)(ce - cb) * sl.stage_words;
  uint32_t sw[kU];
#pragma unroll
  for (uint32_t k = 0; k < kU; k++) {
    const uint64_t i = (uint64_t)k * T + tid;
    sw[k] = i < region ? src[i] : 0u;
  }
  const uint32_t nu0 = tid < (uint32_t)nslots ? sl.nused[tid] : 0u;
  const uint32_t wd0 = tid < (uint32_t)nslots ? sl.words[tid] : 0u;
  const uint32_t *bw = sl.blk_words + (uint64_t)u * kMaxEncBlocks;
  const uint32_t bw0 = tid < b ? bw[tid] : 0u;
  const uint32_t *cw = sl.chunk_words + (uint64_t)u * nch;
  const uint32_t cw0 = cb + tid < ce ? cw[cb + tid] : 0u;
  const uint32_t nw = bw[b];
  const uint64_t base = ctl->bump;
  const uint32_t n_used = sl.nused[u], words = sl.words[u];
  uint2 tab0 = make_uint2(0, 0);  // symbol table entries 4 tid .. 4 tid + 3 (block 0)
  uint32_t nesc = 0;
  uint64_t sq_lo = 0, sq_hi = 0, slice = 0;
  double qstep = 0.0;
  if (b == 0) {
    if (4 * tid < (uint32_t)kNSym) tab0 = ((const uint2 *)(sl.symtab + (uint64_t)u * kNSym))[tid];
    if (tid == 0) {
      nesc = sl.nesc[u];
      sq_lo = sl.sq[2 * u];
      sq_hi = sl.sq[2 * u + 1];
      slice = slot_slice[u];
      if (qp.rel) qstep = sl.qstep[3 * u];
    }
  }
  // record sizes of the batch (slot order) and this slot's offset among them
  uint64_t pre = 0, tot = 0, ex = 0;
  for (uint32_t v = tid; v < (uint32_t)nslots; v += T) {
    bool rv;
    const uint64_t bytes = v == tid ? slot_rec_bytes(sl, g, v, nu0, wd0, rv)
                                    : slot_rec_bytes(sl, g, v, sl.nused[v], sl.words[v], rv);
    const uint64_t ba = (bytes + kRecAlign - 1) & ~(kRecAlign - 1);
    tot += ba;
    ex += bytes;
    if (v < u) pre += ba;
  }
  uint64_t bp = 0;  // words of the slot's earlier blocks
  for (uint32_t i = tid; i < b; i += T) bp += i == tid ? bw0 : bw[i];
  {  // the four block sums at once (4 wavefronts x 4 values in s64)
    uint64_t x[4] = {pre, tot, ex, bp};
#pragma unroll
    for (int k = 0; k < 4; k++)
      for (int off = 32; off > 0; off >>= 1) x[k] += __shfl_xor(x[k], off, 64);
    if (lane_id() == 0)
      for (int k = 0; k < 4; k++) s64[4 * (tid >> 6) + k] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; k++) {
      x[k] = 0;
      for (uint32_t w = 0; w < T / 64; w++) x[k] += s64[4 * w + k];
    }
    pre = x[0];
    tot = x[1];
    ex = x[2];
    bp = x[3];
  }
  if (base + tot > cap) {
    if (tid == 0 && b == 0 && u == 0) fail(ctl, kFlagOverflow, pass);
    return;
  }
  if (tid == 0 && b == 0 && u == 0) {
    ctl->pending_bump = tot;
    ctl->pending_bytes = ex;
  }
  const uint64_t off = base + pre;
  uint8_t *rec = arena + off;
  bool ru;  // chunk-run layout
  const uint64_t rbytes = slot_rec_bytes(sl, g, u, n_used, words, ru);
  uint32_t *offs = (uint32_t *)(rec + kHdr + ((2 * n_used + 3) & ~3u));
  const uint32_t R = ru ? sl.nruns[u] : 0u;
  const uint32_t *rsrc = sl.run_src + (uint64_t)u * kMaxRuns;
  const uint32_t *rwoff = sl.run_woff + (uint64_t)u * (kMaxRuns + 1);
  if (ru) {  // the streams of the runs that start in this block
    uint32_t *rstream = offs + 2 * R + 2;
    const uint32_t lo = sl.blk_run[(uint64_t)u * kMaxEncBlocks + b];  // the first run starting at or after cb
    for (uint32_t r = lo + tid; r < R && rsrc[r] < ce; r += T) {  // a thread per run
      const uint32_t from = cw[rsrc[r]] & 0x7FFFFFFFu;  // in this block's packed words
      const uint32_t to = rwoff[r] & 0x7FFFFFFFu, n = (rwoff[r + 1] & 0x7FFFFFFFu) - to;
      uint32_t i = 0;
      for (; i + 8 <= n; i += 8) {  // eight loads in flight, then their stores
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) v[k] = src[from + i + k];
#pragma unroll
        for (int k = 0; k < 8; k++) rstream[to + i + k] = v[k];
      }
      for (; i < n; i++) rstream[to + i] = src[from + i];
    }
  } else {
    uint32_t *stream = offs + nch + 1;
    for (uint32_t c = cb + tid; c < ce; c += T) {  // a constant chunk's mark (bit 31) travels with its offset
      const uint32_t x = c == cb + tid ? cw0 : cw[c];
      offs[c] = ((uint32_t)bp + (x & 0x7FFFFFFFu)) | (x & 0x80000000u);
    }
#pragma unroll
    for (uint32_t k = 0; k < kU; k++) {
      const uint32_t i = k * T + tid;
      if (i < nw) stream[bp + i] = sw[k];
    }
    // the rest in steps of kB words per thread: every load of a step is issued
    // before its stores, so a step waits for memory once, not once per word
    constexpr uint32_t kB = 32;
    for (uint32_t i0 = kU * T; i0 < nw; i0 += kB * T) {
      uint32_t v[kB];
#pragma unroll
      for (uint32_t k = 0; k < kB; k++) {
        const uint32_t i = i0 + k * T + tid;
        v[k] = i < nw ? src[i] : 0u;
      }
#pragma unroll
      for (uint32_t k = 0; k < kB; k++) {
        const uint32_t i = i0 + k * T + tid;
        if (i < nw) stream[bp + i] = v[k];
      }
    }
  }
  if (b != 0) return;
  const double step = qp.pw ? 1.0 : qp.rel ? qstep : qp.step;
  if (tid == 0) {
    uint32_t *h32 = (uint32_t *)rec;
    h32[0] = kMagic;
    h32[1] = (uint32_t)g.slice_log2;
    h32[2] = (uint32_t)g.chunk_log2;
    h32[3] = n_used;
    h32[4] = nch;
    h32[5] = ru ? sl.run_words[u] : words;
    h32[6] = nesc;
    h32[7] = (uint32_t)rbytes;
    *(double *)(rec + 32) = step;
    *(uint64_t *)(rec + 40) = sq_lo;
    *(uint64_t *)(rec + 48) = sq_hi;
    // zero chunks; constant chunks; pointwise-relative codes and their mantissa bits; chunk runs
    h32[14] = (g.zero_chunks ? 1u : 0u) | (g.const_chunks ? 2u : 0u) | (qp.pw ? 4u : 0u) | (ru ? 8u : 0u);
    h32[15] = qp.pw ? (uint32_t)qp.pw_bits : 0u;
    nxt.rec_off[slice] = off;
    nxt.rec_len[slice] = h32[7];
    nxt.step[slice] = step;
    nxt.sq[2 * slice] = sq_lo;
    nxt.sq[2 * slice + 1] = sq_hi;
    if (ru) {
      offs[0] = R;
      offs[1 + 2 * R] = rwoff[R];
    } else {
      offs[nch] = words;
    }
  }
  if (ru) {  // run ends and the runs' word offsets
    for (uint32_t r = tid; r < R; r += T) {
      offs[1 + r] = r + 1 < R ? rsrc[r + 1] : nch;
      offs[1 + R + r] = rwoff[r];
    }
  }
  // the symbol table, padded with a zero entry to 4 bytes
  uint16_t *tab = (uint16_t *)(rec + kHdr);
  const uint32_t e[4] = {tab0.x & 0xffffu, tab0.x >> 16, tab0.y & 0xffffu, tab0.y >> 16};
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) {
    const uint32_t i = 4 * tid + k;
    if (i < n_used) tab[i] = (uint16_t)e[k];
  }
  if (tid == 0 && (n_used & 1)) tab[n_used] = 0;
}

#endif  // !CQ_FP32

// ------------------------------------------------------------ fused blocks
// A dense block of K = 3..5 qubits (several gates fused on the host) applied
// in place to the decompressed slots on FP64 matrix cores.  With the real
// embedding M = [[Ur, -Ui], [Ui, Ur]] (D = 2^(K+1) rows) and, for a base
// amplitude b (all target bits clear), x_b = (re of its 2^K members, im of
// its 2^K members), the outputs are y_b = M x_b.  A wavefront takes 16 bases
// at a time: Y (D x 16) = M (D x D) X (D x 16) in (D / 16) x (D / 4)
// v_mfma_f64_16x16x4f64 steps.  Operand layouts of that instruction: A
// (16 x 4): lane l holds A[l % 16][l / 16]; B (4 x 16): lane l holds
// B[l / 16][l % 16]; C and D (16 x 16): register i of lane l holds
// D[4 i + l / 16][l % 16] for i = 0..3.  Member c of base b has the flat batch index f_b | dep[c],
// where f_b is the base counter with a zero inserted at every target bit.
// A wavefront reads all inputs of its 16 bases before it writes their
// outputs, and no two wavefronts share a base, so updating in place is safe.
// MM (relative bound, every target inside the slice, whole groups of 16
// bases per slot): the block also takes each slot's min/max of its outputs,
// as the min/max kernel would from the workspace afterwards.  Then every
// wavefront walks one contiguous range of bases, whose 16-base groups each
// lie in one slot, keeps the keys of the slot it is in, and folds them into
// the slot's with one atomic pair per slot it leaves.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int K, bool MM>
__global__ void __launch_bounds__(256) k_dense_mfma(Slots sl, Geo g, GateDesc gd, uint64_t nbases, const Ctl *ctl) {
  if (ctl->flags) return;
  constexpr int NM = 1 << K, D = 2 * NM, RB = D / 16, KS = D / 4;
  const uint32_t lane = lane_id(), col = lane & 15u, quad = lane >> 4;
  double a[RB][KS];  // this lane's entries of M for every step
#pragma unroll
  for (int R = 0; R < RB; R++)
#pragma unroll
    for (int s = 0; s < KS; s++) a[R][s] = gd.mat[(uint64_t)(16 * R + col) * D + 4 * s + quad];
  const uint64_t L = g.L;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwv = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  // MM: bases [wave * per, (wave + 1) * per) in steps of 16; otherwise every nwv-th group of 16
  const uint64_t per = MM ? ((nbases + nwv - 1) / nwv + 15) & ~15ull : 16;
  const uint64_t j0 = MM ? wave * per : wave * 16, jend = MM ? (j0 + per < nbases ? j0 + per : nbases) : nbases;
  const uint64_t jstep = MM ? 16 : nwv * 16;
  uint64_t kmin = ~0ull, kmax = 0ull, mslot = ~0ull;  // MM: this lane's keys for slot mslot
  auto flush = [&]() {  // wavefront-uniform: the keys of every lane into slot mslot's
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t x = __shfl_xor(kmin, off, 64), y = __shfl_xor(kmax, off, 64);
      kmin = x < kmin ? x : kmin;
      kmax = y > kmax ? y : kmax;
    }
    if (lane == 0 && kmin <= kmax) {
      atomicMin((unsigned long long *)&sl.minmax[2 * mslot], (unsigned long long)kmin);
      atomicMax((unsigned long long *)&sl.minmax[2 * mslot + 1], (unsigned long long)kmax);
    }
    kmin = ~0ull;
    kmax = 0ull;
  };
  for (uint64_t jb = j0; jb < jend; jb += jstep) {
    const uint64_t j = jb + col;
    const bool valid = j < nbases;
    uint64_t f = valid ? j : jb;  // lanes past the last base read base jb and store nothing
#pragma unroll
    for (int t = 0; t < K; t++) {  // target positions ascend
      const int p = gd.tloc[t];
      f = ((f >> p) << (p + 1)) | (f & ((1ull << p) - 1));
    }
    double x[KS];
#pragma unroll
    for (int s = 0; s < KS; s++) {
      const uint32_t r = 4 * s + quad;
      const uint64_t fm = f | gd.dep[r & (NM - 1)];
      x[s] = sl.ws[(fm >> g.slice_log2) * 2 * L + (r >= (uint32_t)NM ? L : 0) + (fm & (L - 1))];
    }
    dbl4 acc[RB];
#pragma unroll
    for (int R = 0; R < RB; R++) acc[R] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KS; s++)
#pragma unroll
      for (int R = 0; R < RB; R++) acc[R] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[R][s], x[s], acc[R], 0, 0, 0);
    if (MM) {  // the group's slot (uniform: 16 bases of one slot)
      const uint64_t slot = (uint64_t)__builtin_amdgcn_readfirstlane((int)(f >> g.slice_log2));
      if (slot != mslot) {
        if (mslot != ~0ull) flush();
        mslot = slot;
      }
    }
    if (valid) {
#pragma unroll
      for (int R = 0; R < RB; R++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const uint32_t r = 16 * R + 4 * i + quad;
          const uint64_t fm = f | gd.dep[r & (NM - 1)];
          const double y = rw(acc[R][i]);
          sl.ws[(fm >> g.slice_log2) * 2 * L + (r >= (uint32_t)NM ? L : 0) + (fm & (L - 1))] = y;
          if (MM) {
            const uint64_t key = dkey(y);
            kmin = key < kmin ? key : kmin;
            kmax = key > kmax ? key : kmax;
          }
        }
    }
  }
  if (MM && mslot != ~0ull) flush();
}

bool dense_minmax_ok(const Geo &g, const GateDesc &gd) {
  for (int t = 0; t < gd.k; t++)
    if (gd.tloc[t] >= g.slice_log2) return false;
  return ((g.L >> gd.k) & 15) == 0;  // whole groups of 16 bases per slot
}

void launch_dense_mfma(hipStream_t st, const Slots &sl, const Geo &g, int nslots, const GateDesc &gd,
                       const Ctl *ctl, bool minmax) {
  const uint64_t nbases = ((uint64_t)nslots * g.L) >> gd.k;
  const uint64_t waves = (nbases + 15) / 16;
  uint64_t blocks = (waves + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  const dim3 grid((unsigned)blocks), block(256);
#define CQ_DM(K_)                                                                     \
  do {                                                                                \
    if (minmax)                                                                       \
      CQ_LAUNCH((k_dense_mfma<K_, true>), grid, block, 0, st, sl, g, gd, nbases, ctl); \
    else                                                                              \
      CQ_LAUNCH((k_dense_mfma<K_, false>), grid, block, 0, st, sl, g, gd, nbases, ctl); \
  } while (0)
  switch (gd.k) {
    case 3: CQ_DM(3); break;
    case 4: CQ_DM(4); break;
    default: CQ_DM(5); break;
  }
#undef CQ_DM
}

// ----------------------------------------------------------------- readout

__global__ void k_readout(Slots sl, Geo g, uint64_t first, uint64_t count, int probabilities, double *out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t f = first + i;
  const uint64_t u = f >> g.slice_log2, o = f & (g.L - 1);
  const double re = sl.ws[u * 2 * g.L + o], im = sl.ws[u * 2 * g.L + g.L + o];
  if (probabilities) {
    double a = re * re;
    double b = im * im;
    out[i] = a + b;
  } else {
    out[2 * i] = re;
    out[2 * i + 1] = im;
  }
}

// =============================================================== launchers


static inline unsigned grid1(uint64_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

#if !CQ_FP32
void launch_begin_pass(hipStream_t st, Ctl *ctl, const StateMeta &cur, uint64_t nslices, double *kscale,
                       int with_norm, bool pw) {
  CQ_LAUNCH(k_begin_pass, dim3(1), dim3(1024), 0, st, ctl, cur.step, cur.sq, nslices, kscale, with_norm,
            pw ? 1 : 0);
}

void launch_reset_slots(hipStream_t st, const Slots &sl, int nslots) {
  uint64_t n = (uint64_t)nslots * kGqParts * kNSym;
  CQ_LAUNCH(k_reset_slots, dim3(grid1(n, 256)), dim3(256), 0, st, sl, nslots);
}

#endif  // !CQ_FP32

void launch_init(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots, int kind,
                 uint64_t x, const double *factors, const Ctl *ctl) {
  uint64_t total = (uint64_t)nslots * g.L;
  CQ_LAUNCH(k_init, dim3(grid1(total, 256)), dim3(256), 0, st, sl, g, slot_slice, total, kind, x, factors,
                     ctl);
}

void launch_decode(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                   const uint8_t *arena, const StateMeta &cur, const double *kscale, Ctl *ctl, uint32_t pass,
                   bool compact) {
  const uint32_t per_wg = 64u * kDecWaves;
  dim3 grid(grid1(g.nchunks, per_wg), (unsigned)nslots);
  const bool full = (1ull << g.chunk_log2) >= (uint64_t)DecFmt<true>::R && g.nchunks % per_wg == 0;
  const int c = compact ? 1 : 0;
#define CQ_DEC2(FULL_, FMT_, SMALL_, PW_)                                                                       \
  CQ_LAUNCH((k_decode<FULL_, FMT_, SMALL_, PW_>), grid, dim3(per_wg), 0, st, sl, g, slot_slice, arena, cur, kscale, \
            ctl, pass, c)
#define CQ_DEC1(FULL_, FMT_, SMALL_)         \
  do {                                       \
    if (g.pw_bits >= 0)                      \
      CQ_DEC2(FULL_, FMT_, SMALL_, true);    \
    else                                     \
      CQ_DEC2(FULL_, FMT_, SMALL_, false);   \
  } while (0)
#define CQ_DEC(FULL_, FMT_)                 \
  do {                                      \
    if (compact)                            \
      CQ_DEC1(FULL_, FMT_, true);           \
    else                                    \
      CQ_DEC1(FULL_, FMT_, false);          \
  } while (0)
  switch (g.fmt_in & 3u) {
    case 0: if (full) CQ_DEC(true, 0); else CQ_DEC(false, 0); break;
    case 1: if (full) CQ_DEC(true, 1); else CQ_DEC(false, 1); break;
    case 2: if (full) CQ_DEC(true, 2); else CQ_DEC(false, 2); break;
    default: if (full) CQ_DEC(true, 3); else CQ_DEC(false, 3); break;
  }
#undef CQ_DEC
#undef CQ_DEC1
#undef CQ_DEC2
}

static int gate_kind(const GateDesc &gd) {
  if (gd.kind == 0) return 0;
  if (gd.kind == 2) return 2;
  return gd.k == 1 ? 1 : 3;
}

template <int KIND>
static void launch_minmax_k(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *ss, int nslots,
                            const GateDesc &gd, const Ctl *ctl) {
  const int threads = g.L >= 256 ? 256 : 64;
  const uint64_t per_wg = (uint64_t)threads * 16;  // at least 16 amplitudes per thread
  uint64_t G = (g.L + per_wg - 1) / per_wg;
  if (G > 64) G = 64;
  CQ_LAUNCH(k_gate_minmax<KIND>, dim3((unsigned)G, (unsigned)nslots), dim3(threads), 0, st, sl, g, ss, gd,
                     ctl);
}

void launch_gate_minmax(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                        const GateDesc &gd, const Ctl *ctl) {
  switch (gate_kind(gd)) {
    case 0: launch_minmax_k<0>(st, sl, g, slot_slice, nslots, gd, ctl); break;
    case 1: launch_minmax_k<1>(st, sl, g, slot_slice, nslots, gd, ctl); break;
    case 2: launch_minmax_k<2>(st, sl, g, slot_slice, nslots, gd, ctl); break;
    default: launch_minmax_k<3>(st, sl, g, slot_slice, nslots, gd, ctl); break;
  }
}

#if !CQ_FP32
void launch_rel_step(hipStream_t st, const Slots &sl, int nslots, double rel, const Ctl *ctl) {
  CQ_LAUNCH(k_rel_step, dim3(grid1((uint64_t)nslots, 256)), dim3(256), 0, st, sl, nslots, rel, ctl);
}
#endif  // !CQ_FP32

// Kernels over wavefront ranges (chunks of at most 256 values, slices of at
// least 1024 amplitudes): 1 for one range at a time (identity, phase, or a
// one-target gate whose partner is in the range), 2 for range pairs (a
// one-target gate with its partner in another range of the slice or in
// another slice), 0 when neither applies.
static int wave_route(const Geo &g, const GateDesc &gd, int kind) {
  if (g.chunk_log2 > 8 || g.L < 4 * kWr) return 0;
  if (kind == 0 || kind == 2) return 1;
  if (kind != 1) return 0;
  if ((1ull << gd.tloc[0]) < kWr) return 1;
  const bool cross = gd.tloc[0] >= g.slice_log2;
  const uint32_t nr = (uint32_t)(g.L / kWr);
  return (cross ? nr : nr / 2) >= 4 ? 2 : 0;
}

template <bool C32>
static void launch_gq_wave(int kind, dim3 grid, hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *ss,
                           const GateDesc &gd, const QuantParams &qp, Ctl *ctl, uint32_t pass, const double *kscale) {
#define CQ_GQW(K) CQ_LAUNCH((k_gq_wave<K, C32>), grid, dim3(256), 0, st, sl, g, ss, gd, qp, ctl, pass, kscale)
  switch (kind) {
    case 0: CQ_GQW(0); break;
    case 2: CQ_GQW(2); break;
    case 6: CQ_GQW(6); break;
    case 7: CQ_GQW(7); break;
    case 10: CQ_GQW(10); break;
    case 11: CQ_GQW(11); break;
    case 12: CQ_GQW(12); break;
    case 13: CQ_GQW(13); break;
    case 14: CQ_GQW(14); break;
    case 15: CQ_GQW(15); break;
    default: break;
  }
#undef CQ_GQW
}

// Returns the number of partial results per slot that the launch writes.
template <int KIND>
static uint32_t launch_gq_k(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *ss, int nslots,
                            const GateDesc &gd, const QuantParams &qp, Ctl *ctl, uint32_t pass, bool compact,
                            const double *kscale) {
  if (KIND != 3 && wave_route(g, gd, KIND) == 1) {
    const uint32_t nr = (uint32_t)(g.L / kWr);
    const uint32_t G = nr / 4 < kGqWgs ? nr / 4 : kGqWgs;
    constexpr int K = KIND == 3 ? 0 : KIND;
    const dim3 grid(G, (unsigned)nslots);
    // one target: t < 6 partner in another lane (kernel 10 + t), 6 and 7 in the same lane
    const int kk = KIND == 1 ? (gd.tloc[0] < 6 ? 10 + gd.tloc[0] : gd.tloc[0]) : K;
    if (compact)
      launch_gq_wave<true>(kk, grid, st, sl, g, ss, gd, qp, ctl, pass, kscale);
    else
      launch_gq_wave<false>(kk, grid, st, sl, g, ss, gd, qp, ctl, pass, kscale);
    return G;
  }
  const uint64_t C = gq_tile(g.L);
  const uint32_t ntiles = (uint32_t)(g.L / C);
  const uint32_t G = ntiles < kGqWgs ? ntiles : kGqWgs;
  const dim3 grid(G, (unsigned)nslots);
  if (C == kGqTile) {  // whole tiles of 256 threads x 4 amplitudes
    if (KIND == 3)
      CQ_LAUNCH((k_gate_quant<3, 4, true>), grid, dim3(256), 0, st, sl, g, ss, gd, qp, ctl, pass);
    else
      CQ_LAUNCH((k_gate_quant_pipe<KIND == 3 ? 0 : KIND>), grid, dim3(256), 0, st, sl, g, ss, gd, qp, ctl,
                         pass);
    return G;
  }
  const int threads = g.L >= 256 ? 256 : 64;
  CQ_LAUNCH((k_gate_quant<KIND, 4, false>), grid, dim3(threads), 0, st, sl, g, ss, gd, qp, ctl, pass);
  return G;
}

bool gq_compact(const Geo &g, const GateDesc &gd) { return wave_route(g, gd, gate_kind(gd)) != 0; }

// compact: read a compact workspace when ctl->wide is clear (only the
// wavefront-range kernels can; gq_compact tells whether gd goes there)
// Pointwise-relative mode: the tiled kernel with its general gate path
// (identity, phase, or any dense gate through eval_amp) and 2 C doubles of
// dynamic LDS for the chunk sums.
static uint32_t launch_gq_pw(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *ss, int nslots,
                             const GateDesc &gd, const QuantParams &qp, Ctl *ctl, uint32_t pass, int kind) {
  const uint64_t C = gq_tile(g.L);
  const uint32_t ntiles = (uint32_t)(g.L / C);
  const uint32_t G = ntiles < kGqWgs ? ntiles : kGqWgs;
  const dim3 grid(G, (unsigned)nslots);
  const size_t shm = 16 * C;
  if (C == kGqTile) {
    if (kind == 0)
      CQ_LAUNCH((k_gate_quant<0, 4, true>), grid, dim3(256), shm, st, sl, g, ss, gd, qp, ctl, pass);
    else if (kind == 2)
      CQ_LAUNCH((k_gate_quant<2, 4, true>), grid, dim3(256), shm, st, sl, g, ss, gd, qp, ctl, pass);
    else
      CQ_LAUNCH((k_gate_quant<3, 4, true>), grid, dim3(256), shm, st, sl, g, ss, gd, qp, ctl, pass);
    return G;
  }
  const int threads = g.L >= 256 ? 256 : 64;
  if (kind == 0)
    CQ_LAUNCH((k_gate_quant<0, 4, false>), grid, dim3(threads), shm, st, sl, g, ss, gd, qp, ctl, pass);
  else if (kind == 2)
    CQ_LAUNCH((k_gate_quant<2, 4, false>), grid, dim3(threads), shm, st, sl, g, ss, gd, qp, ctl, pass);
  else
    CQ_LAUNCH((k_gate_quant<3, 4, false>), grid, dim3(threads), shm, st, sl, g, ss, gd, qp, ctl, pass);
  return G;
}

uint32_t launch_gate_quant(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                           const GateDesc &gd, const QuantParams &qp, Ctl *ctl, uint32_t pass, bool compact,
                           const double *kscale) {
  const int kind = gate_kind(gd);
  if (qp.pw) return launch_gq_pw(st, sl, g, slot_slice, nslots, gd, qp, ctl, pass, kind);
  if (kind == 1) {
    const uint64_t C = gq_tile(g.L);
    const int wr = wave_route(g, gd, kind);
    if (wr == 1) return launch_gq_k<1>(st, sl, g, slot_slice, nslots, gd, qp, ctl, pass, compact, kscale);
    if (wr == 2) {
      const bool cross = gd.tloc[0] >= g.slice_log2;
      const uint32_t nr = (uint32_t)(g.L / kWr);
      const uint32_t npairs = cross ? nr : nr / 2;
      const uint32_t G = npairs / 4 < kGqWgs ? npairs / 4 : kGqWgs;
      const dim3 grid(G, (unsigned)(cross ? nslots / 2 : nslots));
      if (compact)
        CQ_LAUNCH(k_gq_wave_pair<true>, grid, dim3(256), 0, st, sl, g, slot_slice, gd, qp, ctl, pass, kscale);
      else
        CQ_LAUNCH(k_gq_wave_pair<false>, grid, dim3(256), 0, st, sl, g, slot_slice, gd, qp, ctl, pass, kscale);
      return G;
    }
    if ((1ull << gd.tloc[0]) < C)  // partner inside the tile
      return launch_gq_k<1>(st, sl, g, slot_slice, nslots, gd, qp, ctl, pass, false, kscale);
    if (g.L >= kGqTile) {  // partner in the paired tile (2^t >= 1024)
      const bool cross = gd.tloc[0] >= g.slice_log2;
      if ((1ull << g.chunk_log2) > kGpTile) {  // tiles of 1024, no pipelining
        const uint32_t ntiles = (uint32_t)(g.L / kGqTile);
        const uint32_t npairs = cross ? ntiles : ntiles / 2;
        const uint32_t G = npairs < kGqWgs ? npairs : kGqWgs;
        const dim3 grid(G, (unsigned)(cross ? nslots / 2 : nslots));
        CQ_LAUNCH(k_gate_quant_pair<kGqV>, grid, dim3(256), 0, st, sl, g, slot_slice, gd, qp, ctl, pass);
        return cross ? G : 2 * G;
      }
      const uint32_t ntiles = (uint32_t)(g.L / kGpTile);
      const uint32_t npairs = cross ? ntiles : ntiles / 2;
      const uint32_t G = npairs < kGqWgs ? npairs : kGqWgs;
      const dim3 grid(G, (unsigned)(cross ? nslots / 2 : nslots));
      CQ_LAUNCH(k_gate_quant_pair_pipe, grid, dim3(256), 0, st, sl, g, slot_slice, gd, qp, ctl, pass);
      return cross ? G : 2 * G;
    }
    return launch_gq_k<3>(st, sl, g, slot_slice, nslots, gd, qp, ctl, pass, false, kscale);  // short slices
  }
  switch (kind) {
    case 0: return launch_gq_k<0>(st, sl, g, slot_slice, nslots, gd, qp, ctl, pass, compact, kscale);
    case 2: return launch_gq_k<2>(st, sl, g, slot_slice, nslots, gd, qp, ctl, pass, compact, kscale);
    default: return launch_gq_k<3>(st, sl, g, slot_slice, nslots, gd, qp, ctl, pass, false, kscale);
  }
}

#if !CQ_FP32
void launch_codebook(hipStream_t st, const Slots &sl, const uint64_t *slot_slice, int nslots, const StateMeta &nxt,
                     uint32_t nparts, Ctl *ctl, uint32_t pw_nchunks) {
  CQ_LAUNCH(k_codebook, dim3((unsigned)nslots), dim3(256), 0, st, sl, slot_slice, nxt, nparts, ctl, pw_nchunks);
}

// chunks per encode (and finish) workgroup: about four workgroups per CU over
// the batch, at least one chunk per coding wavefront, at most kMaxEncBlocks
// workgroups per slot
static uint32_t enc_chunks_per_block(const Geo &g, int nslots) {
  const uint64_t total = (uint64_t)nslots * g.nchunks;
  uint64_t cpb = total / 1024;
  if (cpb < kEncWaves) cpb = kEncWaves;
  const uint64_t least = (g.nchunks + kMaxEncBlocks - 1) / kMaxEncBlocks;
  if (cpb < least) cpb = least;
  if (cpb > g.nchunks) cpb = g.nchunks;
  return (uint32_t)cpb;
}

template <int FMT>
void launch_encode_fmt(hipStream_t st, const Slots &sl, const Geo &g, int nslots, const Ctl *ctl) {
  const uint32_t cpb = enc_chunks_per_block(g, nslots);
  dim3 grid(grid1(g.nchunks, cpb), (unsigned)nslots);
  const size_t shm = (size_t)2 * kEncWaves * sl.stage_words * 4;
  const dim3 block(64 * (kEncWaves + 1));
  if (g.chunk_log2 <= 8) {
    CQ_LAUNCH((k_encode<1, FMT>), grid, block, shm, st, sl, g, cpb, ctl);
    return;
  }
  // dynamic LDS above the default needs the attribute: set once to the
  // largest request (chunks of 1024 values, ~70 KB)
  static const bool attrs = [] {
    const int most = (int)(2 * kEncWaves * stage_words_for(10) * 4);
    (void)hipFuncSetAttribute((const void *)k_encode<4, FMT>, hipFuncAttributeMaxDynamicSharedMemorySize, most);
    (void)hipFuncSetAttribute((const void *)k_encode<2, FMT>, hipFuncAttributeMaxDynamicSharedMemorySize, most);
    return true;
  }();
  (void)attrs;
  if (g.chunk_log2 == 9)
    CQ_LAUNCH((k_encode<2, FMT>), grid, block, shm, st, sl, g, cpb, ctl);
  else
    CQ_LAUNCH((k_encode<4, FMT>), grid, block, shm, st, sl, g, cpb, ctl);
}

void launch_encode(hipStream_t st, const Slots &sl, const Geo &g, int nslots, const Ctl *ctl) {
  switch ((g.zero_chunks ? 1 : 0) | (g.const_chunks ? 2 : 0)) {
    case 0: launch_encode_fmt<0>(st, sl, g, nslots, ctl); break;
    case 1: launch_encode_fmt<1>(st, sl, g, nslots, ctl); break;
    case 2: launch_encode_fmt<2>(st, sl, g, nslots, ctl); break;
    default: launch_encode_fmt<3>(st, sl, g, nslots, ctl); break;
  }
}

void launch_carry(hipStream_t st, Ctl *ctl, const StateMeta &cur, const StateMeta &nxt, const uint8_t *in,
                  uint8_t *out, uint64_t cap, const uint64_t *src, const uint64_t *dst, uint64_t count, uint64_t *off,
                  uint32_t pass) {
  CQ_LAUNCH(k_carry_plan, dim3(1), dim3(1024), 0, st, ctl, cur, src, count, cap, off, pass);
  const uint32_t wgs = (uint32_t)(count < 2048 ? count : 2048);
  CQ_LAUNCH(k_carry_copy, dim3(wgs), dim3(256), 0, st, ctl, cur, nxt, in, out, src, dst, count, off);
}

void launch_runs(hipStream_t st, const Slots &sl, const Geo &g, int nslots, const Ctl *ctl) {
  const uint32_t cpb = enc_chunks_per_block(g, nslots);
  const dim3 grid(g.run_tiles, (unsigned)nslots);
  CQ_LAUNCH(k_runs_mark, grid, dim3(kRunTile), 0, st, sl, g, cpb, ctl);
  CQ_LAUNCH(k_runs_number, grid, dim3(kRunTile), 0, st, sl, g, cpb, ctl);
}

void launch_finish(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                   const QuantParams &qp, uint8_t *arena, uint64_t arena_cap, const StateMeta &nxt, Ctl *ctl,
                   uint32_t pass) {
  const uint32_t cpb = enc_chunks_per_block(g, nslots);
  dim3 grid(grid1(g.nchunks, cpb), (unsigned)nslots);
  CQ_LAUNCH(k_finish, grid, dim3(256), 0, st, sl, g, slot_slice, nslots, qp, arena, arena_cap, nxt, cpb,
                     ctl, pass);
}

#endif  // !CQ_FP32

void launch_readout(hipStream_t st, const Slots &sl, const Geo &g, uint64_t first_amp, uint64_t count,
                    int probabilities, double *out) {
  CQ_LAUNCH(k_readout, dim3(grid1(count, 256)), dim3(256), 0, st, sl, g, first_amp, count, probabilities,
                     out);
}

}  // namespace CQ_PREC
}  // namespace cq
