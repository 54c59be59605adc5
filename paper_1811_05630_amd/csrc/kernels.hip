// Device kernels of libcqsim for gfx950 (CDNA4, 64-wide wavefronts).
//
// One pass of Algorithm 1 (Section II of the paper) over a batch of slices is
//   decode      Decompress(S): canonical-Huffman decode, exact escapes, prefix
//               sum inside each chunk, a = p * (step * s)  -- Normalize(S) folded in
//   gate_quant  GateComputation(G, S) and the first half of Compress(S):
//               error-bounded quantisation, chunked Lorenzo difference, symbols,
//               escapes, histogram, exact sum of p^2
//   codebook    package-merge code lengths (limit 12), canonical codes
//   chunkbits   coded size of every chunk
//   layout      record sizes -> offsets in the output arena
//   header      record header, symbol table, chunk word offsets
//   encode      bit packing, most significant bit first, one wavefront per chunk
// FP64 arithmetic is never contracted into FMAs (the pragma below), so that
// every rounding happens exactly as in the stream definition.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cqsim_impl.h"

namespace cq {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ void cmac(double ur, double ui, double ar, double ai, double &cr, double &ci) {
  // c += u * a with the fixed operation order of every gate
  double pr = ur * ar;
  double pi = ui * ai;
  double qr = ur * ai;
  double qi = ui * ar;
  cr = cr + (pr - pi);
  ci = ci + (qr + qi);
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

// inclusive scan of a u32 over one wavefront
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= (uint32_t)off) x += y;
  }
  return x;
}

// exclusive scan of one u32 per thread over a block of up to 1024 threads;
// returns the prefix, *total gets the block sum.  Uses `scratch` (>= 16 u32).
__device__ uint32_t block_excl_scan(uint32_t x, uint32_t *scratch, uint32_t *total) {
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t nw = (blockDim.x + 63) >> 6;
  uint32_t inc = wave_incl_scan(x);
  if (lane == 63 || threadIdx.x == blockDim.x - 1) scratch[wave] = inc;
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

// ----------------------------------------------------------- begin / end pass

__device__ __forceinline__ double norm_leaf(const double *step, const uint64_t *sq, uint64_t j) {
  double s = step[j];
  double p = (double)sq[2 * j + 1] * 0x1p64 + (double)sq[2 * j];
  return (s * s) * p;
}

// Pairwise sum of `b` (a power of two) consecutive leaves: the same balanced
// tree as adding neighbours level by level.
__device__ double pairwise_block(const double *step, const uint64_t *sq, uint64_t first, uint64_t b) {
  double stk[48];
  int top = 0;
  for (uint64_t i = 0; i < b; i++) {
    double v = norm_leaf(step, sq, first + i);
    uint64_t k = i;
    while (k & 1) {
      v = stk[--top] + v;
      k >>= 1;
    }
    stk[top++] = v;
  }
  return stk[0];
}

// with_norm: 0 = initial state (no norm), 1 = a pass, 2 = read-out only
__global__ void __launch_bounds__(1024) k_begin_pass(Ctl *ctl, const double *step, const uint64_t *sq, uint64_t S,
                                                     double *kscale, int with_norm) {
  if (ctl->flags) return;
  __shared__ double part[1024];
  __shared__ double s_sh;
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  if (!with_norm) {
    if (tid == 0) {
      ctl->bump = 0;
      ctl->cur_bytes = 0;
    }
    return;
  }
  uint64_t active;
  if (S <= T) {
    part[tid] = tid < S ? norm_leaf(step, sq, tid) : 0.0;
    active = S;
  } else {
    uint64_t b = S / T;
    part[tid] = pairwise_block(step, sq, (uint64_t)tid * b, b);
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
    if (with_norm == 1) {  // a pass starts writing the other arena
      ctl->N = N;
      ctl->s = y;
      ctl->bump = 0;
      ctl->cur_bytes = 0;
    }
    s_sh = y;
  }
  __syncthreads();
  for (uint64_t j = tid; j < S; j += T) kscale[j] = step[j] * s_sh;
}

__global__ void k_end_pass(Ctl *ctl) {
  if (ctl->flags) return;
  if (ctl->cur_bytes > ctl->peak_bytes) ctl->peak_bytes = ctl->cur_bytes;
}

__global__ void k_reset_slots(Slots sl, uint32_t nchunks, int nslots) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (uint64_t)nslots * kNSym) sl.hist[i] = 0;
  if (i < (uint64_t)nslots) {
    sl.sq[2 * i] = 0;
    sl.sq[2 * i + 1] = 0;
    sl.nesc[i] = 0;
    sl.words[i] = 0;
    sl.minmax[2 * i] = ~0ull;
    sl.minmax[2 * i + 1] = 0ull;
  }
}

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
// One lane decodes one chunk serially; the workgroup first expands the
// record's canonical symbol table into a 4096-entry lookup table in LDS
// (entry = symbol | length << 10, indexed by the next 12 stream bits).

__device__ __forceinline__ uint32_t ld32(const uint8_t *p) { return *(const uint32_t *)p; }

struct BitReader {
  const uint32_t *w;
  uint32_t nw, wi;
  uint64_t buf;
  int nbits;
  __device__ __forceinline__ void refill() {
    while (nbits <= 32) {
      uint32_t x = wi < nw ? w[wi] : 0u;
      wi++;
      buf |= (uint64_t)x << (32 - nbits);
      nbits += 32;
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

__global__ void __launch_bounds__(256) k_decode(Slots sl, Geo g, const uint64_t *slot_slice, const uint8_t *arena,
                                                StateMeta cur, const double *kscale, Ctl *ctl, uint32_t pass) {
  if (ctl->flags) return;
  __shared__ uint16_t dtab[1 << kLMax];
  __shared__ uint16_t ent[kNSym];
  __shared__ uint32_t lav[kNSym];
  __shared__ uint32_t scratch[20];
  __shared__ int bad;
  const uint32_t u = blockIdx.y;
  const uint64_t slice = slot_slice[u];
  const uint8_t *rec = arena + cur.rec_off[slice];
  const uint32_t tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  const uint32_t n_used = ld32(rec + 12);
  const uint32_t nchunks = ld32(rec + 16);
  const uint32_t n_words = ld32(rec + 20);
  if (tid == 0) {
    if (ld32(rec) != kMagic || n_used < 1 || n_used > (uint32_t)kNSym || nchunks != g.nchunks ||
        ld32(rec + 8) != (uint32_t)g.chunk_log2)
      bad = 1;
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) fail(ctl, kFlagCorrupt, pass);
    return;
  }
  // canonical table: code intervals of size 2^(12 - len) tile [0, 4096) in order
  const uint16_t *st = (const uint16_t *)(rec + kHdr);
  uint32_t sz[4], loc = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    uint32_t i = tid * 4 + k;
    uint32_t s = 0;
    if (i < n_used) {
      uint16_t e = st[i];
      ent[i] = e;
      uint32_t len = e >> 10;
      s = len <= (uint32_t)kLMax ? (1u << (kLMax - len)) : 0x10000u;
    }
    sz[k] = s;
    loc += s;
  }
  uint32_t tot;
  uint32_t pre = block_excl_scan(loc, scratch, &tot);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    uint32_t i = tid * 4 + k;
    if (i < n_used) lav[i] = pre;
    pre += sz[k];
  }
  if (tot != (1u << kLMax)) {
    if (tid == 0) fail(ctl, kFlagCorrupt, pass);
    return;
  }
  __syncthreads();
  for (uint32_t e = tid; e < (1u << kLMax); e += blockDim.x) {
    uint32_t lo = 0, hi = n_used;  // last k with lav[k] <= e
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (lav[mid] <= e) lo = mid; else hi = mid;
    }
    dtab[e] = ent[lo];
  }
  __syncthreads();

  const uint32_t c = blockIdx.x * blockDim.x + tid;
  if (c >= nchunks) return;
  const uint32_t sym_bytes = (2 * n_used + 3) & ~3u;
  const uint32_t *offs = (const uint32_t *)(rec + kHdr + sym_bytes);
  const uint32_t w0 = offs[c], w1 = offs[c + 1];
  if (w1 < w0 || w1 > n_words) {
    fail(ctl, kFlagCorrupt, pass);
    return;
  }
  BitReader br;
  br.w = offs + (nchunks + 1) + w0;
  br.nw = w1 - w0;
  br.wi = 0;
  br.buf = 0;
  br.nbits = 0;
  br.refill();
  const uint64_t B = 1ull << g.chunk_log2;
  const double k = kscale[slice];
  double *out = sl.ws + (uint64_t)u * 2 * g.L + (uint64_t)c * B;
  int64_t p = 0;
  for (uint64_t j = 0; j < B; j++) {
    if (br.nbits < kLMax) br.refill();
    uint32_t e = dtab[(uint32_t)(br.buf >> (64 - kLMax))];
    uint32_t sym = e & 1023u, len = e >> 10;
    br.buf <<= len;
    br.nbits -= (int)len;
    int64_t d;
    if (sym == 0) {
      if (br.nbits < kEscBits) br.refill();
      int nb = (int)br.take(kEscBits);
      uint64_t z;
      if (nb > 32) {
        if (br.nbits < 32) br.refill();
        uint64_t hi = br.take(nb - 32);
        if (br.nbits < 32) br.refill();
        z = (hi << 32) | br.take(32);
      } else {
        if (br.nbits < nb) br.refill();
        z = br.take(nb);
      }
      d = unzigzag(z);
    } else {
      d = (int64_t)sym - kR;
    }
    p += d;
    out[j] = (double)p * k;
  }
}

// ------------------------------------------------------------ gate + quantise

// Output amplitude (re, im) of the gate at slot u, offset o.
__device__ __forceinline__ void eval_amp(const double *__restrict__ ws, const Geo &g, const uint64_t *slot_slice,
                                         const GateDesc &gd, uint32_t u, uint64_t o, double &re, double &im) {
  const uint64_t twoL = 2 * g.L;
  const double *w = ws + (uint64_t)u * twoL;
  if (gd.kind == 0) {
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
  if (gd.kind == 2) {
    double cr = 0.0, ci = 0.0;
    cmac(gd.ph_re, gd.ph_im, w[o], w[g.L + o], cr, ci);
    re = cr;
    im = ci;
    return;
  }
  const uint32_t mm = (1u << gd.m) - 1u;
  const uint32_t gbase = u & ~mm;
  const uint64_t gl = ((uint64_t)(u & mm) << g.slice_log2) | o;
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

__device__ __forceinline__ bool quantise(double v, double step, double recip, double ebj, int64_t &p, double &err) {
  double t = v * recip;
  double q = rint(t);
  if (!(fabs(q) < kPMax)) {
    p = 0;
    err = 0.0;
    return false;
  }
  p = (int64_t)q;
  double back = (double)p * step;
  err = fabs(v - back);
  return err <= ebj;
}

// relative bound: min/max of the gate's output over every slot.  Workgroups
// are whole wavefronts; a workgroup covers C = min(blockDim, L) amplitudes of
// one slot and threads past C only take part in the reductions.
__global__ void __launch_bounds__(256) k_gate_minmax(Slots sl, Geo g, const uint64_t *slot_slice, GateDesc gd,
                                                     const Ctl *ctl) {
  if (ctl->flags) return;
  const uint64_t C = (uint64_t)blockDim.x < g.L ? (uint64_t)blockDim.x : g.L;
  const uint64_t i = (uint64_t)blockIdx.x * C + threadIdx.x;
  const uint32_t u = (uint32_t)(((uint64_t)blockIdx.x * C) >> g.slice_log2);
  uint64_t kmin = ~0ull, kmax = 0ull;
  if (threadIdx.x < C) {
    double re, im;
    eval_amp(sl.ws, g, slot_slice, gd, u, i & (g.L - 1), re, im);
    kmin = dkey(re) < dkey(im) ? dkey(re) : dkey(im);
    kmax = dkey(re) < dkey(im) ? dkey(im) : dkey(re);
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
    for (uint32_t w = 1; w < blockDim.x / 64; w++) {
      kmin = smin[w] < kmin ? smin[w] : kmin;
      kmax = smax[w] > kmax ? smax[w] : kmax;
    }
    atomicMin((unsigned long long *)&sl.minmax[2 * u], (unsigned long long)kmin);
    atomicMax((unsigned long long *)&sl.minmax[2 * u + 1], (unsigned long long)kmax);
  }
}

// relative bound: eb_j = rel * max(max - min, 2^-24 max|a|); step = largest
// power of two <= 2 eb_j (1 when eb_j is 0)
__global__ void k_rel_step(Slots sl, int nslots, double rel, const Ctl *ctl) {
  if (ctl->flags) return;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nslots) return;
  double lo = dkey_inv(sl.minmax[2 * u]), hi = dkey_inv(sl.minmax[2 * u + 1]);
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

template <int V>
__global__ void __launch_bounds__(256) k_gate_quant(Slots sl, Geo g, const uint64_t *slot_slice, GateDesc gd,
                                                    QuantParams qp, Ctl *ctl, uint32_t pass) {
  if (ctl->flags) return;
  __shared__ uint32_t h[kNSym];
  __shared__ int64_t last[2][256];
  __shared__ uint64_t wsq[4][2];
  __shared__ uint64_t werr[4];
  __shared__ uint32_t nesc_sh;
  __shared__ uint32_t bad_sh;
  const uint32_t tid = threadIdx.x;
  for (uint32_t s = tid; s < (uint32_t)kNSym; s += blockDim.x) h[s] = 0;
  if (tid == 0) {
    nesc_sh = 0;
    bad_sh = 0;
  }
  // the workgroup (whole wavefronts) covers C = min(blockDim * V, L)
  // consecutive amplitudes of one slot; threads past C only take part in
  // the reductions
  const uint64_t C = (uint64_t)blockDim.x * V < g.L ? (uint64_t)blockDim.x * V : g.L;
  const uint64_t flat0 = (uint64_t)blockIdx.x * C;
  const uint32_t u = (uint32_t)(flat0 >> g.slice_log2);
  const bool active = (uint64_t)tid * V < C;
  const uint64_t o0 = (flat0 & (g.L - 1)) + (active ? (uint64_t)tid * V : 0);
  const uint64_t Bm = (1ull << g.chunk_log2) - 1;
  double step = qp.step, recip = qp.recip, ebj = qp.eb;
  if (qp.rel) {
    step = sl.qstep[3 * u];
    recip = sl.qstep[3 * u + 1];
    ebj = sl.qstep[3 * u + 2];
  }
  int64_t pr[V], pim[V];
  double emax = 0.0;
  bool ok = true;
#pragma unroll
  for (int v = 0; v < V; v++) {
    pr[v] = 0;
    pim[v] = 0;
    if (active) {
      double re, im, e1, e2;
      eval_amp(sl.ws, g, slot_slice, gd, u, o0 + v, re, im);
      ok &= quantise(re, step, recip, ebj, pr[v], e1);
      ok &= quantise(im, step, recip, ebj, pim[v], e2);
      emax = fmax(emax, fmax(e1, e2));
    }
  }
  last[0][tid] = pr[V - 1];
  last[1][tid] = pim[V - 1];
  __syncthreads();
  int64_t prev_r = 0, prev_i = 0;
  if (active && (o0 & Bm) != 0) {
    if (tid > 0) {
      prev_r = last[0][tid - 1];
      prev_i = last[1][tid - 1];
    } else {
      double re, im, e1, e2;
      eval_amp(sl.ws, g, slot_slice, gd, u, o0 - 1, re, im);
      quantise(re, step, recip, ebj, prev_r, e1);
      quantise(im, step, recip, ebj, prev_i, e2);
    }
  }
  uint16_t *sym_r = sl.sym + (uint64_t)u * 2 * g.L;
  uint16_t *sym_i = sym_r + g.L;
  int64_t *esc_r = sl.esc + (uint64_t)u * 2 * g.L;
  int64_t *esc_i = esc_r + g.L;
  uint32_t sr[V], si[V];
  uint32_t nesc = 0;
  uint64_t sq_lo = 0, sq_hi = 0;
#pragma unroll
  for (int v = 0; v < V; v++) {
    sr[v] = si[v] = 0;
    if (!active) continue;
    const uint64_t o = o0 + v;
    if ((o & Bm) == 0) {
      prev_r = 0;
      prev_i = 0;
    }
    int64_t dr = pr[v] - prev_r, di = pim[v] - prev_i;
    prev_r = pr[v];
    prev_i = pim[v];
    bool er = !(dr > -kR && dr < kR), ei = !(di > -kR && di < kR);
    sr[v] = er ? 0u : (uint32_t)(dr + kR);
    si[v] = ei ? 0u : (uint32_t)(di + kR);
    if (er) esc_r[o] = dr;
    if (ei) esc_i[o] = di;
    nesc += (uint32_t)er + (uint32_t)ei;
    uint64_t a = (uint64_t)(pr[v] < 0 ? -pr[v] : pr[v]);
    uint64_t b = (uint64_t)(pim[v] < 0 ? -pim[v] : pim[v]);
    uint64_t l1 = a * a, h1 = __umul64hi(a, a), l2 = b * b, h2 = __umul64hi(b, b);
    uint64_t t = sq_lo + l1;
    sq_hi += h1 + (t < sq_lo);
    sq_lo = t;
    t = sq_lo + l2;
    sq_hi += h2 + (t < sq_lo);
    sq_lo = t;
  }
  // symbols out: V consecutive u16 per plane
  if (active) {
#pragma unroll
    for (int v = 0; v < V; v++) {
      sym_r[o0 + v] = (uint16_t)sr[v];
      sym_i[o0 + v] = (uint16_t)si[v];
    }
  }
  // histogram: a wavefront whose values all share one symbol adds once
  bool uni = true;
#pragma unroll
  for (int v = 0; v < V; v++) uni &= (sr[v] == sr[0]) & (si[v] == sr[0]);
  const uint32_t s0 = (uint32_t)__shfl((int)sr[0], 0, 64);
  const uint64_t act = __ballot(active);
  const bool wave_uni = __ballot(active && uni && sr[0] == s0) == act;
  if (wave_uni) {
    if (lane_id() == 0 && act) atomicAdd(&h[s0], (uint32_t)(2 * V * __popcll(act)));
  } else if (active) {
    uint32_t cs = sr[0], cn = 0;
#pragma unroll
    for (int v = 0; v < V; v++) {
      if (sr[v] != cs) { atomicAdd(&h[cs], cn); cs = sr[v]; cn = 0; }
      cn++;
    }
#pragma unroll
    for (int v = 0; v < V; v++) {
      if (si[v] != cs) { atomicAdd(&h[cs], cn); cs = si[v]; cn = 0; }
      cn++;
    }
    atomicAdd(&h[cs], cn);
  }
  // wavefront reductions of sum p^2, max error, escapes
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t ol = __shfl_xor(sq_lo, off, 64), oh = __shfl_xor(sq_hi, off, 64);
    uint64_t t = sq_lo + ol;
    sq_hi += oh + (t < sq_lo);
    sq_lo = t;
    emax = fmax(emax, __shfl_xor(emax, off, 64));
  }
  if (nesc) atomicAdd(&nesc_sh, nesc);
  if (!ok) atomicOr(&bad_sh, 1u);
  const uint32_t wave = tid >> 6;
  if (lane_id() == 0) {
    wsq[wave][0] = sq_lo;
    wsq[wave][1] = sq_hi;
    werr[wave] = (uint64_t)__double_as_longlong(emax);
  }
  __syncthreads();
  for (uint32_t s = tid; s < (uint32_t)kNSym; s += blockDim.x)
    if (h[s]) atomicAdd(&sl.hist[(uint64_t)u * kNSym + s], h[s]);
  if (tid == 0) {
    uint64_t lo = wsq[0][0], hi = wsq[0][1], eb = werr[0];
    for (uint32_t w = 1; w < blockDim.x / 64; w++) {
      uint64_t t = lo + wsq[w][0];
      hi += wsq[w][1] + (t < lo);
      lo = t;
      eb = werr[w] > eb ? werr[w] : eb;
    }
    unsigned long long old = atomicAdd((unsigned long long *)&sl.sq[2 * u], (unsigned long long)lo);
    if (old + lo < old) hi += 1;
    atomicAdd((unsigned long long *)&sl.sq[2 * u + 1], (unsigned long long)hi);
    atomicMax((unsigned long long *)&ctl->max_err_bits, (unsigned long long)eb);
    if (nesc_sh) {
      atomicAdd(&sl.nesc[u], nesc_sh);
      atomicAdd((unsigned long long *)&ctl->escapes, (unsigned long long)nesc_sh);
    }
    if (bad_sh) fail(ctl, kFlagBound, pass);
  }
}

// ---------------------------------------------------------------- codebook
// One workgroup per slot.  Package-merge (Larmore & Hirschberg) in its
// coin-collector form: level 12 holds the leaves (sorted by count, then
// symbol); level l is the merge of the leaves with the pairwise packages of
// level l+1, a leaf first on equal weights.  The 2n-2 cheapest items of
// level 1 are selected.  A selected prefix of m items at level l holds the
// q_l lightest leaves and m - q_l packages, i.e. the first 2(m - q_l) items of
// level l+1; a leaf of rank i gets the length #{l : i < q_l}.

__device__ void bitonic_sort_1024(uint64_t *key) {
  for (uint32_t k = 2; k <= 1024; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t p = threadIdx.x; p < 512; p += blockDim.x) {
        uint32_t i = (p / j) * 2 * j + (p % j);
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

__global__ void __launch_bounds__(256) k_codebook(Slots sl, const Ctl *ctl) {
  if (ctl->flags) return;
  __shared__ uint64_t key[kNSym];
  __shared__ uint32_t wgt[kNSym];
  __shared__ uint32_t LA[2 * kNSym], LB[2 * kNSym];
  __shared__ uint16_t LP[kLMax][kNSym];
  __shared__ uint8_t lens[kNSym];
  __shared__ uint32_t q[kLMax + 1];
  __shared__ uint32_t scratch[20];
  const uint32_t u = blockIdx.x, tid = threadIdx.x;
  const uint32_t *hist = sl.hist + (uint64_t)u * kNSym;
  uint32_t cnt = 0;
  for (uint32_t s = tid; s < (uint32_t)kNSym; s += blockDim.x) {
    uint32_t hv = hist[s];
    key[s] = hv ? (((uint64_t)hv << 10) | s) : ~0ull;
    lens[s] = 0;
    cnt += hv ? 1u : 0u;
  }
  uint32_t n;
  block_excl_scan(cnt, scratch, &n);
  bitonic_sort_1024(key);
  for (uint32_t i = tid; i < n; i += blockDim.x) wgt[i] = (uint32_t)(key[i] >> 10);
  __syncthreads();
  if (n >= 2) {
    uint32_t *cur = LA, *nxt = LB;
    for (uint32_t i = tid; i < n; i += blockDim.x) cur[i] = wgt[i];
    uint32_t len_cur = n;
    __syncthreads();
    for (int l = kLMax - 1; l >= 1; l--) {
      const uint32_t np = len_cur / 2;
      for (uint32_t i = tid; i < n; i += blockDim.x) {
        const uint32_t wi = wgt[i];
        uint32_t lo = 0, hi = np;  // packages lighter than the leaf
        while (lo < hi) {
          uint32_t mid = (lo + hi) >> 1;
          if (cur[2 * mid] + cur[2 * mid + 1] < wi) lo = mid + 1; else hi = mid;
        }
        nxt[i + lo] = wi;
        LP[l][i] = (uint16_t)(i + lo);
      }
      for (uint32_t k = tid; k < np; k += blockDim.x) {
        const uint32_t pv = cur[2 * k] + cur[2 * k + 1];
        uint32_t lo = 0, hi = n;  // leaves not heavier than the package
        while (lo < hi) {
          uint32_t mid = (lo + hi) >> 1;
          if (wgt[mid] <= pv) lo = mid + 1; else hi = mid;
        }
        nxt[k + lo] = pv;
      }
      __syncthreads();
      uint32_t *t = cur;
      cur = nxt;
      nxt = t;
      len_cur = n + np;
    }
    if (tid == 0) {
      uint32_t m = 2 * n - 2;
      for (int l = 1; l < kLMax; l++) {
        uint32_t lo = 0, hi = n;  // leaves placed before position m
        while (lo < hi) {
          uint32_t mid = (lo + hi) >> 1;
          if (LP[l][mid] < m) lo = mid + 1; else hi = mid;
        }
        q[l] = lo;
        m = 2 * (m - lo);
      }
      q[kLMax] = m;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += blockDim.x) {
      uint32_t len = 0;
      for (int l = 1; l <= kLMax; l++) len += i < q[l] ? 1u : 0u;
      lens[key[i] & 1023] = (uint8_t)len;
    }
  }
  __syncthreads();
  // canonical order (length, symbol); codes are the left-aligned interval
  // starts shifted back: intervals of size 2^(12 - len) tile [0, 4096)
  for (uint32_t s = tid; s < (uint32_t)kNSym; s += blockDim.x)
    key[s] = hist[s] ? (((uint64_t)lens[s] << 10) | s) : ~0ull;
  bitonic_sort_1024(key);
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
      tab[i] = (uint16_t)(sym | (len << 10));
    }
    pre += sz[k];
  }
  if (tid == 0) sl.nused[u] = n;
}

// --------------------------------------------------------------- chunk bits

__global__ void __launch_bounds__(256) k_chunkbits(Slots sl, Geo g, uint64_t total_chunks, const Ctl *ctl) {
  if (ctl->flags) return;
  const uint64_t cg = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (cg >= total_chunks) return;
  const uint32_t u = (uint32_t)(cg / g.nchunks), c = (uint32_t)(cg % g.nchunks);
  const uint64_t B = 1ull << g.chunk_log2;
  const uint64_t base = (uint64_t)u * 2 * g.L + (uint64_t)c * B;
  const uint32_t *codes = sl.codes + (uint64_t)u * kNSym;
  uint64_t bits = 0;
  for (uint64_t j = lane_id(); j < B; j += 64) {
    uint32_t s = sl.sym[base + j];
    bits += codes[s] & 0xffu;
    if (s == 0) bits += kEscBits + bitlen64(zigzag(sl.esc[base + j]));
  }
  for (int off = 32; off > 0; off >>= 1) bits += __shfl_xor(bits, off, 64);
  if (lane_id() == 0) {
    uint32_t w = (uint32_t)((bits + 31) >> 5);
    sl.chunk_words[(uint64_t)u * g.nchunks + c] = w;
    atomicAdd(&sl.words[u], w);
  }
}

// ------------------------------------------------------------------ layout

__device__ __forceinline__ uint64_t rec_bytes(uint32_t n_used, uint32_t nchunks, uint32_t words) {
  return (uint64_t)kHdr + ((2ull * n_used + 3) & ~3ull) + 4ull * (nchunks + 1) + 4ull * words;
}

__global__ void __launch_bounds__(1024) k_layout(Slots sl, Geo g, const uint64_t *slot_slice, int nslots,
                                                 StateMeta nxt, uint64_t cap, Ctl *ctl, uint32_t pass) {
  if (ctl->flags) return;
  __shared__ unsigned long long tot_al, tot_ex;
  __shared__ unsigned long long carry;
  __shared__ unsigned long long wpart[16];
  const uint32_t tid = threadIdx.x;
  if (tid == 0) {
    tot_al = 0;
    tot_ex = 0;
    carry = 0;
  }
  __syncthreads();
  unsigned long long a = 0, e = 0;
  for (int u = tid; u < nslots; u += blockDim.x) {
    uint64_t b = rec_bytes(sl.nused[u], g.nchunks, sl.words[u]);
    e += b;
    a += (b + kRecAlign - 1) & ~(kRecAlign - 1);
  }
  atomicAdd(&tot_al, a);
  atomicAdd(&tot_ex, e);
  __syncthreads();
  const uint64_t base = ctl->bump;
  if (base + tot_al > cap) {
    if (tid == 0) fail(ctl, kFlagOverflow, pass);
    return;
  }
  // exclusive scan of aligned sizes in slot order, tile by tile
  for (int t0 = 0; t0 < nslots; t0 += blockDim.x) {
    const int u = t0 + (int)tid;
    uint64_t b = 0, ba = 0;
    if (u < nslots) {
      b = rec_bytes(sl.nused[u], g.nchunks, sl.words[u]);
      ba = (b + kRecAlign - 1) & ~(kRecAlign - 1);
    }
    uint64_t x = ba;
    const uint32_t lane = lane_id(), wave = tid >> 6;
    for (int off = 1; off < 64; off <<= 1) {
      uint64_t y = __shfl_up(x, off, 64);
      if (lane >= (uint32_t)off) x += y;
    }
    if (lane == 63) wpart[wave] = x;
    __syncthreads();
    uint64_t wpre = 0;
    for (uint32_t w = 0; w < wave; w++) wpre += wpart[w];
    const uint64_t excl = carry + wpre + x - ba;
    if (u < nslots) {
      const uint64_t slice = slot_slice[u];
      nxt.rec_off[slice] = base + excl;
      nxt.rec_len[slice] = (uint32_t)b;
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t s = 0;
      for (uint32_t w = 0; w < (blockDim.x >> 6); w++) s += wpart[w];
      carry += s;
    }
    __syncthreads();
  }
  if (tid == 0) {
    ctl->bump = base + tot_al;
    ctl->cur_bytes += tot_ex;
  }
}

// ------------------------------------------------------------------ header

__global__ void __launch_bounds__(256) k_header(Slots sl, Geo g, const uint64_t *slot_slice, QuantParams qp,
                                                uint8_t *arena, StateMeta nxt, const Ctl *ctl) {
  if (ctl->flags) return;
  __shared__ uint32_t scratch[20];
  __shared__ uint32_t carry;
  const uint32_t u = blockIdx.x, tid = threadIdx.x;
  const uint64_t slice = slot_slice[u];
  uint8_t *rec = arena + nxt.rec_off[slice];
  const uint32_t n_used = sl.nused[u], words = sl.words[u], nch = g.nchunks;
  const double step = qp.rel ? sl.qstep[3 * u] : qp.step;
  if (tid == 0) {
    uint32_t *h32 = (uint32_t *)rec;
    h32[0] = kMagic;
    h32[1] = (uint32_t)g.slice_log2;
    h32[2] = (uint32_t)g.chunk_log2;
    h32[3] = n_used;
    h32[4] = nch;
    h32[5] = words;
    h32[6] = sl.nesc[u];
    h32[7] = (uint32_t)rec_bytes(n_used, nch, words);
    *(double *)(rec + 32) = step;
    *(uint64_t *)(rec + 40) = sl.sq[2 * u];
    *(uint64_t *)(rec + 48) = sl.sq[2 * u + 1];
    h32[14] = 0;
    h32[15] = 0;
    nxt.step[slice] = step;
    nxt.sq[2 * slice] = sl.sq[2 * u];
    nxt.sq[2 * slice + 1] = sl.sq[2 * u + 1];
    carry = 0;
  }
  uint16_t *tab = (uint16_t *)(rec + kHdr);
  for (uint32_t i = tid; i < n_used; i += blockDim.x) tab[i] = sl.symtab[(uint64_t)u * kNSym + i];
  if (tid == 0 && (n_used & 1)) tab[n_used] = 0;
  uint32_t *offs = (uint32_t *)(rec + kHdr + ((2 * n_used + 3) & ~3u));
  const uint32_t *cw = sl.chunk_words + (uint64_t)u * nch;
  __syncthreads();
  for (uint32_t t0 = 0; t0 < nch; t0 += blockDim.x) {
    uint32_t c = t0 + tid;
    uint32_t x = c < nch ? cw[c] : 0u, tot;
    uint32_t pre = block_excl_scan(x, scratch, &tot);
    if (c < nch) offs[c] = carry + pre;
    __syncthreads();
    if (tid == 0) carry += tot;
    __syncthreads();
  }
  if (tid == 0) offs[nch] = words;
}

// ------------------------------------------------------------------ encode
// One wavefront per chunk: code lengths -> wavefront prefix sum -> bit
// positions; codes are OR-ed into the chunk's words staged in LDS, which are
// then written out with coalesced stores.

__device__ __forceinline__ void put_bits(uint32_t *lw, uint64_t v, int n, uint64_t pos) {
  while (n > 0) {
    const uint32_t w = (uint32_t)(pos >> 5);
    const int off = (int)(pos & 31);
    const int take = n < 32 - off ? n : 32 - off;
    const uint32_t piece = (uint32_t)((v >> (n - take)) & ((1ull << take) - 1));
    atomicOr(&lw[w], piece << (32 - off - take));
    n -= take;
    pos += take;
  }
}

__global__ void __launch_bounds__(256) k_encode(Slots sl, Geo g, const uint64_t *slot_slice, uint64_t total_chunks,
                                                uint32_t lds_words, uint8_t *arena, StateMeta nxt, const Ctl *ctl) {
  if (ctl->flags) return;
  extern __shared__ uint32_t lw_all[];
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  const uint64_t cg = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  const bool active = cg < total_chunks;  // inactive wavefronts still meet the barriers
  uint32_t *lw = lw_all + (uint64_t)wave * lds_words;
  const uint32_t u = active ? (uint32_t)(cg / g.nchunks) : 0u;
  const uint32_t c = active ? (uint32_t)(cg % g.nchunks) : 0u;
  const uint64_t slice = slot_slice[u];
  uint8_t *rec = arena + nxt.rec_off[slice];
  const uint32_t n_used = sl.nused[u];
  const uint32_t *offs = (const uint32_t *)(rec + kHdr + ((2 * n_used + 3) & ~3u));
  const uint32_t w0 = active ? offs[c] : 0u;
  const uint32_t nw = active ? offs[c + 1] - w0 : 0u;
  uint32_t *out = (uint32_t *)(offs + g.nchunks + 1) + w0;
  for (uint32_t i = lane; i < nw && i < lds_words; i += 64) lw[i] = 0;
  __syncthreads();
  const uint64_t B = active ? (1ull << g.chunk_log2) : 0;
  const uint64_t base = (uint64_t)u * 2 * g.L + (uint64_t)c * (1ull << g.chunk_log2);
  const uint32_t *codes = sl.codes + (uint64_t)u * kNSym;
  uint64_t run = 0;
  for (uint64_t j0 = 0; j0 < B; j0 += 64) {
    const uint64_t j = j0 + lane;
    uint32_t bl = 0, code = 0, len = 0, s = 1;
    int nb = 0;
    uint64_t z = 0;
    if (j < B) {
      s = sl.sym[base + j];
      uint32_t cwv = codes[s];
      len = cwv & 0xffu;
      code = cwv >> 8;
      bl = len;
      if (s == 0) {
        z = zigzag(sl.esc[base + j]);
        nb = bitlen64(z);
        bl += kEscBits + (uint32_t)nb;
      }
    }
    const uint32_t inc = wave_incl_scan(bl);
    const uint64_t pos = run + inc - bl;
    run += (uint32_t)__shfl((int)inc, 63, 64);
    if (j < B && pos + bl <= 32ull * (nw < lds_words ? nw : lds_words)) {
      put_bits(lw, code, (int)len, pos);
      if (s == 0) {
        put_bits(lw, (uint64_t)nb, kEscBits, pos + len);
        put_bits(lw, z, nb, pos + len + kEscBits);
      }
    }
  }
  __syncthreads();
  for (uint32_t i = lane; i < nw && i < lds_words; i += 64) out[i] = lw[i];
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

void launch_begin_pass(hipStream_t st, Ctl *ctl, const StateMeta &cur, uint64_t nslices, double *tmp,
                       double *kscale, int with_norm) {
  (void)tmp;
  hipLaunchKernelGGL(k_begin_pass, dim3(1), dim3(1024), 0, st, ctl, cur.step, cur.sq, nslices, kscale, with_norm);
}

void launch_end_pass(hipStream_t st, Ctl *ctl) { hipLaunchKernelGGL(k_end_pass, dim3(1), dim3(1), 0, st, ctl); }

void launch_reset_slots(hipStream_t st, const Slots &sl, const Geo &g, int nslots) {
  uint64_t n = (uint64_t)nslots * kNSym;
  hipLaunchKernelGGL(k_reset_slots, dim3(grid1(n, 256)), dim3(256), 0, st, sl, g.nchunks, nslots);
}

void launch_init(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots, int kind,
                 uint64_t x, const double *factors, const Ctl *ctl) {
  uint64_t total = (uint64_t)nslots * g.L;
  hipLaunchKernelGGL(k_init, dim3(grid1(total, 256)), dim3(256), 0, st, sl, g, slot_slice, total, kind, x, factors,
                     ctl);
}

void launch_decode(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                   const uint8_t *arena, const StateMeta &cur, const double *kscale, Ctl *ctl, uint32_t pass) {
  dim3 grid(grid1(g.nchunks, 256), (unsigned)nslots);
  hipLaunchKernelGGL(k_decode, grid, dim3(256), 0, st, sl, g, slot_slice, arena, cur, kscale, ctl, pass);
}

// Gate kernels: workgroups of whole wavefronts, each covering
// C = min(threads * V, L) amplitudes of one slot.
void launch_gate_minmax(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                        const GateDesc &gd, const Ctl *ctl) {
  const int threads = g.L >= 256 ? 256 : 64;
  const uint64_t C = (uint64_t)threads < g.L ? (uint64_t)threads : g.L;
  const uint64_t total = (uint64_t)nslots * g.L;
  hipLaunchKernelGGL(k_gate_minmax, dim3((unsigned)(total / C)), dim3(threads), 0, st, sl, g, slot_slice, gd, ctl);
}

void launch_rel_step(hipStream_t st, const Slots &sl, int nslots, double rel, const Ctl *ctl) {
  hipLaunchKernelGGL(k_rel_step, dim3(grid1((uint64_t)nslots, 256)), dim3(256), 0, st, sl, nslots, rel, ctl);
}

void launch_gate_quant(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                       const GateDesc &gd, const QuantParams &qp, Ctl *ctl, uint32_t pass) {
  const uint64_t total = (uint64_t)nslots * g.L;
  if (g.L >= 1024) {
    hipLaunchKernelGGL(k_gate_quant<4>, dim3((unsigned)(total / 1024)), dim3(256), 0, st, sl, g, slot_slice, gd, qp,
                       ctl, pass);
  } else {
    const int threads = g.L >= 256 ? 256 : (g.L >= 64 ? (int)g.L : 64);
    const uint64_t C = (uint64_t)threads < g.L ? (uint64_t)threads : g.L;
    hipLaunchKernelGGL(k_gate_quant<1>, dim3((unsigned)(total / C)), dim3(threads), 0, st, sl, g, slot_slice, gd, qp,
                       ctl, pass);
  }
}

void launch_codebook(hipStream_t st, const Slots &sl, int nslots, const Ctl *ctl) {
  hipLaunchKernelGGL(k_codebook, dim3((unsigned)nslots), dim3(256), 0, st, sl, ctl);
}

void launch_chunkbits(hipStream_t st, const Slots &sl, const Geo &g, int nslots, const Ctl *ctl) {
  uint64_t tc = (uint64_t)nslots * g.nchunks;
  hipLaunchKernelGGL(k_chunkbits, dim3(grid1(tc, 4)), dim3(256), 0, st, sl, g, tc, ctl);
}

void launch_layout(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                   const StateMeta &nxt, uint64_t arena_cap, Ctl *ctl, uint32_t pass) {
  hipLaunchKernelGGL(k_layout, dim3(1), dim3(1024), 0, st, sl, g, slot_slice, nslots, nxt, arena_cap, ctl, pass);
}

void launch_header(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                   const QuantParams &qp, uint8_t *arena, const StateMeta &nxt, const Ctl *ctl) {
  hipLaunchKernelGGL(k_header, dim3((unsigned)nslots), dim3(256), 0, st, sl, g, slot_slice, qp, arena, nxt, ctl);
}

void launch_encode(hipStream_t st, const Slots &sl, const Geo &g, const uint64_t *slot_slice, int nslots,
                   uint8_t *arena, const StateMeta &nxt, const Ctl *ctl) {
  const uint64_t B = 1ull << g.chunk_log2;
  const uint32_t lds_words = (uint32_t)((B * (kLMax + kEscBits + 50) + 31) / 32 + 1);
  int waves = 4;
  while (waves > 1 && (uint64_t)waves * lds_words * 4 > 64 * 1024) waves >>= 1;
  uint64_t tc = (uint64_t)nslots * g.nchunks;
  size_t shm = (size_t)waves * lds_words * 4;
  hipLaunchKernelGGL(k_encode, dim3(grid1(tc, (unsigned)waves)), dim3(64 * waves), shm, st, sl, g, slot_slice, tc,
                     lds_words, arena, nxt, ctl);
}

void launch_readout(hipStream_t st, const Slots &sl, const Geo &g, int nslots, uint64_t first_amp, uint64_t count,
                    int probabilities, double *out) {
  (void)nslots;
  hipLaunchKernelGGL(k_readout, dim3(grid1(count, 256)), dim3(256), 0, st, sl, g, first_amp, count, probabilities,
                     out);
}

}  // namespace cq
