/*
 * CPU ORACLE: test infrastructure only.  Nothing in the simulator library may
 * include, link or call this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg use it (through oracle/__init__.py).
 *
 * A plain, slow FP64 reference of the paper's Algorithm 1 (Section II): the
 * state vector of 2^n complex amplitudes is cut into slices, every slice is
 * kept compressed, and for each gate every slice goes through
 *     Decompress -> Normalize -> GateComputation -> Compress.
 * The compressor is an SZ-style error-bounded lossy codec (Section I names SZ;
 * Section II lets the user set the per-amplitude error bound):
 *     prequantise p = rint(a / step)  (error-bounded quantisation)
 *     Lorenzo difference d = p_i - p_{i-1} inside chunks of B values
 *     symbols d + R for |d| < R, else an escape carrying d exactly
 *     length-limited Huffman code (package-merge, Larmore & Hirschberg 1990)
 *     canonical codes (as in RFC 1951), MSB-first 32-bit words.
 * Everything here follows the stream definition directly, one value at a time;
 * no blocking or fusion.  Compiled with -ffp-contract=off: every FP64
 * operation is rounded on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ format */

#define ORC_MAGIC 0x31535143u /* "CQS1" little-endian */
#define ORC_HDR 64
#define ORC_R 512             /* quantisation radius: symbols 1..1023 hold d + R */
#define ORC_NSYM 1024         /* alphabet size; symbol 0 is the escape */
#define ORC_LMAX 12           /* longest Huffman code */
#define ORC_ESC_LEN_BITS 6    /* escape payload: 6-bit length, then the zigzag value */
#define ORC_PMAX ((int64_t)1 << 48) /* |p| must stay below this */

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EBOUND = -3, ORC_ECORRUPT = -4 };

enum { ORC_DENSE = 1, ORC_PHASE = 2 };

typedef struct {
  uint32_t kind;
  uint32_t n_targets;
  uint32_t targets[5];
  uint32_t pad;
  uint64_t ctrl_mask;
  uint64_t ctrl_vals;
  double phase_re, phase_im;
  const double *matrix; /* row-major 2^k x 2^k, interleaved (re, im) */
} orc_gate;

/* ------------------------------------------------------- complex arithmetic */

/* c += u * a, in the fixed order used by every gate:
   pr = ur*ar, pi = ui*ai, qr = ur*ai, qi = ui*ar; cr += (pr - pi); ci += (qr + qi). */
static void cmac(double ur, double ui, double ar, double ai, double *cr, double *ci) {
  double pr = ur * ar;
  double pi = ui * ai;
  double qr = ur * ai;
  double qi = ui * ar;
  *cr = *cr + (pr - pi);
  *ci = *ci + (qr + qi);
}

/* FP32 mode (mode bit ORC_FP32; an extension, the paper works in FP64): every
 * value of the working form -- decoded amplitudes, gate matrix entries and
 * phases, initial factors -- is an FP32 number, and every product and sum of
 * the gate arithmetic is rounded to FP32.  One FP64 operation on two FP32
 * numbers rounded once to FP32 is the FP32 result itself, since 53 >= 2*24 + 2
 * bits make the double rounding innocuous (Figueroa, 1995).  Quantisation,
 * the bound check and the norm stay FP64, applied to the FP32 values. */
#define ORC_FP32 2u

/* Zero chunks (mode bit ORC_ZERO_CHUNKS; an extension toward the paper's
 * remark that other compressors may suit the state better, Section IV): a
 * chunk whose codes p are all zero -- every symbol the zero difference R --
 * is stored with no words; its offset repeats.  The histogram, and so the
 * code, still counts its symbols.  Header word 14 bit 0 marks such records.
 * (A one-symbol code has no bits at all, so there every chunk is empty and
 * decodes to that symbol.) */
#define ORC_ZERO_CHUNKS 8u

/* Constant chunks (mode bit ORC_CONST_CHUNKS; an extension of the same kind):
 * a chunk of two or more values whose differences after the head are all zero
 * (every value equals the head's) keeps only the head's code (and escape);
 * bit 31 of its word offset marks it, and header word 14 bit 1 marks records
 * that may hold such chunks.  The histogram still counts every symbol.  With
 * ORC_ZERO_CHUNKS as well, an all-zero chunk is a zero chunk (no words, no
 * mark). */
#define ORC_CONST_CHUNKS 16u
#define ORC_CONST_MARK 0x80000000u

/* Pointwise-relative bound (mode bit ORC_PWREL; an extension, one reading of
 * the bound Section II sets for each amplitude number): every real and
 * imaginary value v is stored as the FP64 number nearest to it that has b
 * mantissa bits, b the least integer with 2^-(b+1) <= eb, so that
 * |v - v'| <= eb |v| and zero stays zero.  The integer code of v is its IEEE
 * bit pattern without the sign, rounded to b mantissa bits (half to even) and
 * shifted right by 52 - b, negated for negative v: a monotone, logarithm-like
 * integer that the Lorenzo difference and the Huffman code take like any
 * other code.  Such records have step 1.0, header word 15 = b and flags
 * bit 2; their 16-byte sum field holds, in its low 8 bytes, the FP64 squared
 * norm of the slice's decoded values, summed as a pairwise tree over the 2L
 * values in order (the codes' squares are no norm here). */
#define ORC_PWREL 32u
#define ORC_PW_MAXBITS 20

/* Chunk runs (mode bit ORC_CHUNK_RUNS; an extension: the run-length stage
 * over the Huffman output that ratios far beyond one bit per value need, one
 * of the codec variants Section IV leaves to future work): consecutive chunks
 * whose stored streams are identical (the same words and the same constant
 * mark) form a run, whose stream is stored once.  Where that makes the record
 * smaller and the slice has at most ORC_MAX_RUNS runs, the table of chunk
 * offsets is replaced by: u32 R; R u32 run ends (cumulative chunk counts,
 * strictly increasing, the last equal to n_chunks); R + 1 u32 word offsets of
 * the runs' streams (non-decreasing; bit 31 of all but the last is the
 * constant mark; the last equals n_words).  Header word 14 bit 3 marks such
 * records.  Codes, amplitudes and norms are those of the mode without it. */
#define ORC_CHUNK_RUNS 64u
#define ORC_MAX_RUNS 4096u

/* Optimised passes (mode bit ORC_OPT; an extension, off for Algorithm 1 as
 * written, plain mode only): a pass whose gate is controlled on slice-index
 * qubits leaves the slice groups whose index bits fail those controls as
 * they are (their records are not decoded, renormalised or re-encoded), and
 * a SWAP of two slice-index qubits without controls relabels the slices
 * (record j becomes record sigma(j), sigma exchanging the two index bits)
 * without touching a value.  The norm of the next pass is that of all stored
 * records, as always. */
#define ORC_OPT 128u

/* b for a pointwise-relative bound eb, or -1 when eb is out of range. */
static int pw_bits(double eb) {
  if (!(eb > 0.0) || !(eb < 0.5)) return -1;
  int b = 0;
  while (b <= ORC_PW_MAXBITS && ldexp(1.0, -(b + 1)) > eb) b++;
  return b <= ORC_PW_MAXBITS ? b : -1;
}

/* The value of pointwise-relative code c with b mantissa bits. */
static double pw_value(int64_t c, int b) {
  uint64_t m = (uint64_t)(c < 0 ? -c : c) << (52 - b);
  double x;
  memcpy(&x, &m, 8);
  return c < 0 ? -x : x;
}

static double r32(double x) { return (double)(float)x; }

static void cmac_m(int fp32, double ur, double ui, double ar, double ai, double *cr, double *ci) {
  if (!fp32) {
    cmac(ur, ui, ar, ai, cr, ci);
    return;
  }
  double pr = r32(ur * ar);
  double pi = r32(ui * ai);
  double qr = r32(ur * ai);
  double qi = r32(ui * ar);
  *cr = r32(*cr + r32(pr - pi));
  *ci = r32(*ci + r32(qr + qi));
}

/* ------------------------------------------------------------ gate on a group
 * A group is a set of M = 2^m slices whose indices differ only in the slice
 * bits of the gate's targets.  amp_re[u] / amp_im[u] hold slice slices[u],
 * L = 2^slice_log2 amplitudes each.  The gate is applied to every tuple of
 * amplitudes it couples inside the group. */

static double *locate(int nmem, const uint64_t *slices, double **planes, int slice_log2, uint64_t gi) {
  uint64_t j = gi >> slice_log2;
  uint64_t o = gi & (((uint64_t)1 << slice_log2) - 1);
  for (int u = 0; u < nmem; u++)
    if (slices[u] == j) return planes[u] + o;
  return NULL;
}

static int apply_gate_group(const orc_gate *g, int slice_log2, int nmem, const uint64_t *slices,
                            double **re, double **im, int fp32) {
  uint64_t L = (uint64_t)1 << slice_log2;
  if (g->kind == ORC_PHASE) {
    const double phr = fp32 ? r32(g->phase_re) : g->phase_re, phi = fp32 ? r32(g->phase_im) : g->phase_im;
    for (int u = 0; u < nmem; u++) {
      for (uint64_t o = 0; o < L; o++) {
        uint64_t gi = (slices[u] << slice_log2) | o;
        if ((gi & g->ctrl_mask) != g->ctrl_vals) continue;
        double cr = 0.0, ci = 0.0;
        cmac_m(fp32, phr, phi, re[u][o], im[u][o], &cr, &ci);
        re[u][o] = cr;
        im[u][o] = ci;
      }
    }
    return ORC_OK;
  }
  if (g->kind != ORC_DENSE || g->n_targets < 1 || g->n_targets > 5) return ORC_EINVAL;
  int k = (int)g->n_targets;
  int dim = 1 << k;
  uint64_t tmask = 0;
  for (int t = 0; t < k; t++) tmask |= (uint64_t)1 << g->targets[t];
  double in_r[32], in_i[32], out_r[32], out_i[32];
  double *pr_[32], *pi_[32];
  /* every amplitude of the group whose target bits are all zero is a base */
  for (int u = 0; u < nmem; u++) {
    for (uint64_t o = 0; o < L; o++) {
      uint64_t base = (slices[u] << slice_log2) | o;
      if (base & tmask) continue;
      if ((base & g->ctrl_mask) != g->ctrl_vals) continue;
      for (int m = 0; m < dim; m++) {
        uint64_t gi = base;
        for (int t = 0; t < k; t++)
          if ((m >> t) & 1) gi |= (uint64_t)1 << g->targets[t];
        pr_[m] = locate(nmem, slices, re, slice_log2, gi);
        pi_[m] = locate(nmem, slices, im, slice_log2, gi);
        if (!pr_[m]) return ORC_EINVAL;
        in_r[m] = *pr_[m];
        in_i[m] = *pi_[m];
      }
      for (int r = 0; r < dim; r++) {
        double cr = 0.0, ci = 0.0;
        for (int c = 0; c < dim; c++) {
          const double *u2 = g->matrix + 2 * (r * dim + c);
          if (fp32)
            cmac_m(1, r32(u2[0]), r32(u2[1]), in_r[c], in_i[c], &cr, &ci);
          else
            cmac(u2[0], u2[1], in_r[c], in_i[c], &cr, &ci);
        }
        out_r[r] = cr;
        out_i[r] = ci;
      }
      for (int m = 0; m < dim; m++) {
        *pr_[m] = out_r[m];
        *pi_[m] = out_i[m];
      }
    }
  }
  return ORC_OK;
}

/* The gate on one group of slices given as raw planes (no compression). */
int orc_group_apply(const orc_gate *g, int slice_log2, int nmem, const uint64_t *slices, double **re, double **im) {
  return apply_gate_group(g, slice_log2, nmem, slices, re, im, 0);
}

/* Uncompressed state vector: the whole state is one slice of 2^n amplitudes
 * (mode: ORC_FP32 or 0). */
int orc_sv_apply_mode(int n, double *re, double *im, const orc_gate *g, uint32_t mode) {
  uint64_t zero = 0;
  return apply_gate_group(g, n, 1, &zero, &re, &im, (mode & ORC_FP32) != 0);
}

int orc_sv_apply(int n, double *re, double *im, const orc_gate *g) { return orc_sv_apply_mode(n, re, im, g, 0); }

/* -------------------------------------------------------------- quantiser */

/* Absolute bound eb: step = 2*eb*(1 - 2^-20), r = 1/step. */
void orc_abs_step(double eb, double *step, double *recip) {
  double s = (2.0 * eb) * (1.0 - 0x1p-20);
  *step = s;
  *recip = 1.0 / s;
}

/* Relative bound rel over one slice's 2L values (value-range based): the
 * bound is eb_j = rel * max(max - min, 2^-24 * max|a|) -- the floor keeps
 * nearly constant slices codable -- and the step is the largest power of two
 * not above 2*eb_j (1 if eb_j is zero), so that a*r, rint and p*step are all
 * exact. */
void orc_rel_step(double rel, const double *v, uint64_t count, double *step, double *recip, double *ebj) {
  double lo = v[0], hi = v[0];
  for (uint64_t i = 1; i < count; i++) {
    if (v[i] < lo) lo = v[i];
    if (v[i] > hi) hi = v[i];
  }
  double range = hi - lo;
  double m = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
  double fl = m * 0x1p-24;
  double e = rel * (range > fl ? range : fl);
  *ebj = e;
  if (!(e > 0.0)) {
    *step = 1.0;
    *recip = 1.0;
    return;
  }
  int ex;
  frexp(2.0 * e, &ex); /* 2e = f * 2^ex, f in [0.5, 1) */
  *step = ldexp(1.0, ex - 1);
  *recip = ldexp(1.0, 1 - ex);
}

/* ----------------------------------------------------------- package-merge */

typedef struct {
  uint64_t w;
  int leaf; /* >= 0: leaf rank; -1: package of items a and b of the next deeper level */
  int a, b;
} pm_item;

static void pm_count(pm_item **lev, int l, int lmax, int idx, int *len) {
  pm_item *it = &lev[l][idx];
  if (it->leaf >= 0) {
    len[it->leaf]++;
    return;
  }
  pm_count(lev, l + 1, lmax, it->a, len);
  pm_count(lev, l + 1, lmax, it->b, len);
}

/* Optimal code lengths bounded by lmax for n weights sorted ascending.
 * Coin-collector form: level lmax holds the leaves; each shallower level is
 * the merge of the leaves with the pairwise packages of the level below (a
 * leaf goes first when weights tie); the 2n-2 cheapest items of level 1 are
 * selected and a leaf's code length is the number of times it occurs in them.
 * One leaf gets length 0 (no bits are needed to name the only symbol). */
static int package_merge(const uint64_t *w, int n, int lmax, int *len) {
  for (int i = 0; i < n; i++) len[i] = 0;
  if (n <= 1) return ORC_OK;
  if (lmax < 1 || lmax > 30 || (uint64_t)n > ((uint64_t)1 << lmax)) return ORC_EINVAL;
  pm_item *lev[33];
  int cnt[33];
  for (int l = 0; l <= lmax; l++) lev[l] = NULL;
  int rc = ORC_OK;
  lev[lmax] = (pm_item *)malloc(sizeof(pm_item) * (size_t)n);
  if (!lev[lmax]) return ORC_ENOMEM;
  for (int i = 0; i < n; i++) {
    lev[lmax][i].w = w[i];
    lev[lmax][i].leaf = i;
    lev[lmax][i].a = lev[lmax][i].b = -1;
  }
  cnt[lmax] = n;
  for (int l = lmax - 1; l >= 1; l--) {
    int np = cnt[l + 1] / 2;
    lev[l] = (pm_item *)malloc(sizeof(pm_item) * (size_t)(n + np));
    if (!lev[l]) {
      rc = ORC_ENOMEM;
      goto done;
    }
    int i = 0, p = 0, o = 0;
    while (i < n || p < np) {
      uint64_t pw = 0;
      if (p < np) pw = lev[l + 1][2 * p].w + lev[l + 1][2 * p + 1].w;
      if (i < n && (p >= np || w[i] <= pw)) {
        lev[l][o].w = w[i];
        lev[l][o].leaf = i;
        lev[l][o].a = lev[l][o].b = -1;
        i++;
      } else {
        lev[l][o].w = pw;
        lev[l][o].leaf = -1;
        lev[l][o].a = 2 * p;
        lev[l][o].b = 2 * p + 1;
        p++;
      }
      o++;
    }
    cnt[l] = o;
  }
  for (int s = 0; s < 2 * n - 2; s++) pm_count(lev, 1, lmax, s, len);
done:
  for (int l = 1; l <= lmax; l++) free(lev[l]);
  return rc;
}

typedef struct {
  uint64_t count;
  int sym;
} sym_count;

static int cmp_sym_count(const void *x, const void *y) {
  const sym_count *a = (const sym_count *)x, *b = (const sym_count *)y;
  if (a->count != b->count) return a->count < b->count ? -1 : 1;
  return a->sym < b->sym ? -1 : (a->sym > b->sym ? 1 : 0);
}

/* Code lengths per symbol from a histogram: leaves ordered by (count, symbol). */
int orc_huffman_lengths(const uint64_t *hist, int nsym, int lmax, uint8_t *lens) {
  sym_count *sc = (sym_count *)malloc(sizeof(sym_count) * (size_t)nsym);
  uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nsym);
  int *len = (int *)malloc(sizeof(int) * (size_t)nsym);
  if (!sc || !w || !len) {
    free(sc); free(w); free(len);
    return ORC_ENOMEM;
  }
  int n = 0;
  for (int s = 0; s < nsym; s++) {
    lens[s] = 0;
    if (hist[s]) {
      sc[n].count = hist[s];
      sc[n].sym = s;
      n++;
    }
  }
  qsort(sc, (size_t)n, sizeof(sym_count), cmp_sym_count);
  for (int i = 0; i < n; i++) w[i] = sc[i].count;
  int rc = package_merge(w, n, lmax, len);
  if (rc == ORC_OK)
    for (int i = 0; i < n; i++) lens[sc[i].sym] = (uint8_t)len[i];
  free(sc); free(w); free(len);
  return rc;
}

/* Canonical codes: for each length, consecutive values in symbol order,
 * shorter codes first (RFC 1951, section 3.2.2). */
void orc_canonical_codes(const uint8_t *lens, int nsym, int lmax, uint32_t *codes) {
  uint32_t bl_count[33] = {0}, next_code[33] = {0};
  for (int s = 0; s < nsym; s++)
    if (lens[s]) bl_count[lens[s]]++;
  uint32_t code = 0;
  bl_count[0] = 0;
  for (int b = 1; b <= lmax; b++) {
    code = (code + bl_count[b - 1]) << 1;
    next_code[b] = code;
  }
  for (int s = 0; s < nsym; s++) {
    codes[s] = 0;
    if (lens[s]) codes[s] = next_code[lens[s]]++;
  }
}

/* -------------------------------------------------------------- bit writer */

typedef struct {
  uint32_t *words;
  uint64_t pos; /* bits written */
} bitw;

static void put_bits(bitw *bw, uint64_t v, int nbits) {
  for (int k = nbits - 1; k >= 0; k--) {
    uint64_t bit = (v >> k) & 1;
    if (bit) bw->words[bw->pos >> 5] |= 0x80000000u >> (bw->pos & 31);
    bw->pos++;
  }
}

static uint64_t zigzag(int64_t d) { return ((uint64_t)d << 1) ^ (uint64_t)(d >> 63); }
static int64_t unzigzag(uint64_t z) { return (int64_t)(z >> 1) ^ -(int64_t)(z & 1); }
static int bitlen(uint64_t z) {
  int b = 0;
  while (z) {
    b++;
    z >>= 1;
  }
  return b;
}

static uint32_t rd32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t rd64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
static double rdf64(const uint8_t *p) { double v; memcpy(&v, p, 8); return v; }
static void wr32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void wr64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static void wrf64(uint8_t *p, double v) { memcpy(p, &v, 8); }

/* ------------------------------------------------------------- compressor */

typedef struct {
  double max_err;        /* max |a - p*step| over the slice */
  uint64_t n_escapes;
  uint64_t sumsq_lo, sumsq_hi;
  double step;
} orc_cstats;

/* Error-bounded quantisation, the first stage of Compress: the step from the
 * bound (absolute, or relative to the values' range when mode bit 0 is set),
 * then p = rint(v * r) for every value, refused (ORC_EBOUND) when |p| reaches
 * 2^48 or |v - p * step| exceeds the bound.  *sumsq receives sum p^2 exactly. */
static int quantise(const double *v, uint64_t nv, double eb, uint32_t mode, int64_t *p, double *step_out,
                    double *max_err_out, unsigned __int128 *sumsq_out) {
  double step, r, ebj;
  if (mode & 1) {
    orc_rel_step(eb, v, nv, &step, &r, &ebj);
  } else {
    orc_abs_step(eb, &step, &r);
    ebj = eb;
  }
  double max_err = 0.0;
  unsigned __int128 sumsq = 0;
  for (uint64_t i = 0; i < nv; i++) {
    double t = v[i] * r;
    double q = rint(t);
    if (!(fabs(q) < (double)ORC_PMAX)) return ORC_EBOUND;
    p[i] = (int64_t)q;
    double back = (double)p[i] * step;
    double err = fabs(v[i] - back);
    if (err > ebj) return ORC_EBOUND;
    if (err > max_err) max_err = err;
    unsigned __int128 sq = (unsigned __int128)((__int128)p[i] * (__int128)p[i]);
    sumsq += sq;
  }
  *step_out = step;
  *max_err_out = max_err;
  *sumsq_out = sumsq;
  return ORC_OK;
}

/* Pointwise-relative quantisation (ORC_PWREL) of nv values, nv a power of
 * two: the codes, the largest |v - v'| and the pairwise-tree sum of v'^2. */
static int quantise_pw(const double *v, uint64_t nv, double eb, int64_t *p, double *max_err_out, double *norm_out) {
  const int b = pw_bits(eb);
  if (b < 0) return ORC_EINVAL;
  const int sh = 52 - b;
  double *x = (double *)malloc(sizeof(double) * nv);
  if (!x) return ORC_ENOMEM;
  double max_err = 0.0;
  for (uint64_t i = 0; i < nv; i++) {
    uint64_t bits;
    memcpy(&bits, &v[i], 8);
    const uint64_t mag = bits & 0x7FFFFFFFFFFFFFFFull;
    const uint64_t half = (uint64_t)1 << (sh - 1);
    const uint64_t c = (mag + (half - 1) + ((mag >> sh) & 1)) >> sh; /* round half to even */
    if (c >= ((uint64_t)2047 << b)) { /* infinite or not a number, or rounds to infinity */
      free(x);
      return ORC_EBOUND;
    }
    p[i] = (bits >> 63) ? -(int64_t)c : (int64_t)c;
    const double back = pw_value(p[i], b);
    const double err = fabs(v[i] - back);
    if (!(err <= eb * fabs(v[i]))) {
      free(x);
      return ORC_EBOUND;
    }
    if (err > max_err) max_err = err;
    x[i] = back * back;
  }
  for (uint64_t m = nv; m > 1; m /= 2)
    for (uint64_t i = 0; i < m / 2; i++) x[i] = x[2 * i] + x[2 * i + 1];
  *norm_out = x[0];
  *max_err_out = max_err;
  free(x);
  return ORC_OK;
}

/* Compress one slice (Re plane then Im plane, L values each).
 * mode bit 0: 0 = absolute bound eb, 1 = relative bound eb (bit 1, ORC_FP32, does not
 * change the compressor: the values it gets are then FP32 numbers); ORC_ZERO_CHUNKS:
 * all-zero chunks take no words.
 * On success *out is a malloc'ed record of *out_len bytes. */
int orc_compress_slice(const double *re, const double *im, int slice_log2, int chunk_log2, double eb,
                       uint32_t mode, uint8_t **out, uint64_t *out_len, orc_cstats *st) {
  if (slice_log2 < 0 || slice_log2 > 26 || chunk_log2 < 0) return ORC_EINVAL;
  if (chunk_log2 > slice_log2) chunk_log2 = slice_log2;
  uint64_t L = (uint64_t)1 << slice_log2;
  uint64_t nv = 2 * L;
  uint64_t B = (uint64_t)1 << chunk_log2;
  uint64_t nchunks = nv / B;
  double *v = (double *)malloc(sizeof(double) * nv);
  int64_t *p = (int64_t *)malloc(sizeof(int64_t) * nv);
  int64_t *d = (int64_t *)malloc(sizeof(int64_t) * nv);
  uint32_t *sym = (uint32_t *)malloc(sizeof(uint32_t) * nv);
  if (!v || !p || !d || !sym) {
    free(v); free(p); free(d); free(sym);
    return ORC_ENOMEM;
  }
  memcpy(v, re, sizeof(double) * L);
  memcpy(v + L, im, sizeof(double) * L);

  double step, max_err;
  unsigned __int128 sumsq;
  const int pw = (mode & ORC_PWREL) != 0;
  int rc;
  if (pw) {
    double pn;
    rc = quantise_pw(v, nv, eb, p, &max_err, &pn);
    uint64_t pb;
    memcpy(&pb, &pn, 8);
    sumsq = pb;
    step = 1.0;
  } else {
    rc = quantise(v, nv, eb, mode, p, &step, &max_err, &sumsq);
  }
  if (rc != ORC_OK) {
    free(v); free(p); free(d); free(sym);
    return rc;
  }
  /* Lorenzo difference inside each chunk, predictor 0 at the chunk head */
  uint64_t hist[ORC_NSYM];
  memset(hist, 0, sizeof(hist));
  uint64_t nesc = 0;
  for (uint64_t c = 0; c < nchunks; c++) {
    int64_t prev = 0;
    for (uint64_t j = 0; j < B; j++) {
      uint64_t i = c * B + j;
      d[i] = p[i] - prev;
      prev = p[i];
      if (d[i] > -ORC_R && d[i] < ORC_R) {
        sym[i] = (uint32_t)(d[i] + ORC_R);
      } else {
        sym[i] = 0;
        nesc++;
      }
      hist[sym[i]]++;
    }
  }
  uint8_t lens[ORC_NSYM];
  uint32_t codes[ORC_NSYM];
  rc = orc_huffman_lengths(hist, ORC_NSYM, ORC_LMAX, lens);
  if (rc != ORC_OK) {
    free(v); free(p); free(d); free(sym);
    return rc;
  }
  orc_canonical_codes(lens, ORC_NSYM, ORC_LMAX, codes);
  uint32_t n_used = 0;
  for (int s = 0; s < ORC_NSYM; s++)
    if (hist[s]) n_used++;
  /* bits per chunk, then the stream */
  uint64_t *cbits = (uint64_t *)calloc(nchunks, sizeof(uint64_t));
  uint64_t *coff = (uint64_t *)calloc(nchunks + 1, sizeof(uint64_t));
  if (!cbits || !coff) {
    free(v); free(p); free(d); free(sym); free(cbits); free(coff);
    return ORC_ENOMEM;
  }
  const int zc = (mode & ORC_ZERO_CHUNKS) != 0;
  const int cc = (mode & ORC_CONST_CHUNKS) != 0;
  uint8_t *cconst = (uint8_t *)calloc(nchunks, 1);
  if (!cconst) {
    free(v); free(p); free(d); free(sym); free(cbits); free(coff);
    return ORC_ENOMEM;
  }
  for (uint64_t c = 0; c < nchunks; c++) {
    uint64_t bits = 0, head_bits = 0;
    int all_zero = 1, rest_zero = 1;
    for (uint64_t j = 0; j < B; j++) {
      uint64_t i = c * B + j;
      uint64_t b = lens[sym[i]];
      if (sym[i] == 0) b += ORC_ESC_LEN_BITS + (uint64_t)bitlen(zigzag(d[i]));
      bits += b;
      if (j == 0) head_bits = b;
      if (sym[i] != ORC_R) {
        all_zero = 0;
        if (j > 0) rest_zero = 0;
      }
    }
    if (zc && all_zero) {
      bits = 0;
    } else if (cc && B > 1 && rest_zero) {
      cconst[c] = 1;
      bits = head_bits;
    }
    cbits[c] = bits;
    coff[c + 1] = coff[c] + (bits + 31) / 32;
  }
  uint64_t n_words = coff[nchunks];
  uint64_t symtab_bytes = ((2 * (uint64_t)n_used) + 3) & ~(uint64_t)3;
  uint32_t *words = (uint32_t *)calloc(n_words ? n_words : 1, sizeof(uint32_t));
  if (!words) {
    free(v); free(p); free(d); free(sym); free(cbits); free(coff); free(cconst);
    return ORC_ENOMEM;
  }
  for (uint64_t c = 0; c < nchunks; c++) {
    if (cbits[c] == 0) continue; /* a zero chunk, or a one-symbol code */
    bitw bw;
    bw.words = words + coff[c];
    bw.pos = 0;
    for (uint64_t j = 0; j < (cconst[c] ? 1 : B); j++) { /* a constant chunk: the head only */
      uint64_t i = c * B + j;
      put_bits(&bw, codes[sym[i]], lens[sym[i]]);
      if (sym[i] == 0) {
        uint64_t z = zigzag(d[i]);
        int nb = bitlen(z);
        put_bits(&bw, (uint64_t)nb, ORC_ESC_LEN_BITS);
        put_bits(&bw, z, nb);
      }
    }
  }
  /* chunk runs: a chunk starts a run unless its stream (words and constant
   * mark) equals its predecessor's */
  uint64_t nruns = 0, run_words = 0;
  uint32_t *run_src = NULL;
  if (mode & ORC_CHUNK_RUNS) {
    run_src = (uint32_t *)malloc(sizeof(uint32_t) * (ORC_MAX_RUNS + 1));
    if (!run_src) {
      free(words); free(v); free(p); free(d); free(sym); free(cbits); free(coff); free(cconst);
      return ORC_ENOMEM;
    }
    for (uint64_t c = 0; c < nchunks; c++) {
      uint64_t nw = coff[c + 1] - coff[c];
      int same = c > 0 && cconst[c] == cconst[c - 1] && nw == coff[c] - coff[c - 1] &&
                 memcmp(words + coff[c], words + coff[c - 1], 4 * nw) == 0;
      if (same) continue;
      if (nruns < ORC_MAX_RUNS) {
        run_src[nruns] = (uint32_t)c;
        run_words += nw;
      }
      nruns++;
    }
  }
  const int use_runs = (mode & ORC_CHUNK_RUNS) && nruns <= ORC_MAX_RUNS &&
                       8 * nruns + 8 + 4 * run_words < 4 * (nchunks + 1) + 4 * n_words;
  uint64_t table_bytes = use_runs ? 8 * nruns + 8 : 4 * (nchunks + 1);
  uint64_t stored_words = use_runs ? run_words : n_words;
  uint64_t total = ORC_HDR + symtab_bytes + table_bytes + 4 * stored_words;
  if (total > 0xFFFFFFFFull) {
    free(words); free(run_src); free(v); free(p); free(d); free(sym); free(cbits); free(coff); free(cconst);
    return ORC_EINVAL;
  }
  uint8_t *rec = (uint8_t *)calloc(total, 1);
  if (!rec) {
    free(words); free(run_src); free(v); free(p); free(d); free(sym); free(cbits); free(coff); free(cconst);
    return ORC_ENOMEM;
  }
  wr32(rec + 0, ORC_MAGIC);
  wr32(rec + 4, (uint32_t)slice_log2);
  wr32(rec + 8, (uint32_t)chunk_log2);
  wr32(rec + 12, n_used);
  wr32(rec + 16, (uint32_t)nchunks);
  wr32(rec + 20, (uint32_t)stored_words);
  wr32(rec + 24, (uint32_t)nesc);
  wr32(rec + 28, (uint32_t)total);
  wrf64(rec + 32, step);
  wr64(rec + 40, (uint64_t)sumsq);
  wr64(rec + 48, (uint64_t)(sumsq >> 64));
  wr32(rec + 56, (zc ? 1u : 0u) | (cc ? 2u : 0u) | (pw ? 4u : 0u) | (use_runs ? 8u : 0u));
  wr32(rec + 60, pw ? (uint32_t)pw_bits(eb) : 0u);
  /* symbol table in canonical order: by code length, then by symbol */
  uint8_t *tab = rec + ORC_HDR;
  uint32_t k = 0;
  for (int l = 0; l <= ORC_LMAX; l++) {
    for (int s = 0; s < ORC_NSYM; s++) {
      if (!hist[s] || lens[s] != l) continue;
      uint16_t e = (uint16_t)((unsigned)s | ((unsigned)lens[s] << 10));
      memcpy(tab + 2 * k, &e, 2);
      k++;
    }
  }
  uint8_t *offs = tab + symtab_bytes;
  if (use_runs) {
    uint8_t *ends = offs + 4, *woff = ends + 4 * nruns, *stream = woff + 4 * (nruns + 1);
    wr32(offs, (uint32_t)nruns);
    uint64_t w = 0;
    for (uint64_t r = 0; r < nruns; r++) {
      uint64_t c = run_src[r], nw = coff[c + 1] - coff[c];
      wr32(ends + 4 * r, r + 1 < nruns ? run_src[r + 1] : (uint32_t)nchunks);
      wr32(woff + 4 * r, (uint32_t)w | (cconst[c] ? ORC_CONST_MARK : 0u));
      memcpy(stream + 4 * w, words + coff[c], 4 * nw);
      w += nw;
    }
    wr32(woff + 4 * nruns, (uint32_t)w);
  } else {
    for (uint64_t c = 0; c <= nchunks; c++)
      wr32(offs + 4 * c, (uint32_t)coff[c] | (c < nchunks && cconst[c] ? ORC_CONST_MARK : 0u));
    memcpy(offs + 4 * (nchunks + 1), words, 4 * n_words);
  }
  free(words);
  free(run_src);
  if (st) {
    st->max_err = max_err;
    st->n_escapes = nesc;
    st->sumsq_lo = (uint64_t)sumsq;
    st->sumsq_hi = (uint64_t)(sumsq >> 64);
    st->step = step;
  }
  *out = rec;
  *out_len = total;
  free(v); free(p); free(d); free(sym); free(cbits); free(coff); free(cconst);
  return ORC_OK;
}

/* ----------------------------------------------------------- decompressor */

typedef struct {
  uint32_t slice_log2, chunk_log2, n_used, n_chunks, n_words, n_escapes, total, flags, pw_bits;
  uint32_t nruns;  /* chunk-run records: the number of runs (0 otherwise) */
  double step;
  uint64_t sumsq_lo, sumsq_hi;
  const uint8_t *symtab;
  const uint8_t *offs;  /* chunk offsets, or (chunk-run records) the run ends */
  const uint8_t *woff;  /* chunk-run records: the runs' word offsets */
  const uint8_t *words;
} orc_rec;

int orc_parse(const uint8_t *rec, uint64_t len, orc_rec *h) {
  if (len < ORC_HDR || rd32(rec) != ORC_MAGIC) return ORC_ECORRUPT;
  h->slice_log2 = rd32(rec + 4);
  h->chunk_log2 = rd32(rec + 8);
  h->n_used = rd32(rec + 12);
  h->n_chunks = rd32(rec + 16);
  h->n_words = rd32(rec + 20);
  h->n_escapes = rd32(rec + 24);
  h->total = rd32(rec + 28);
  h->step = rdf64(rec + 32);
  h->sumsq_lo = rd64(rec + 40);
  h->sumsq_hi = rd64(rec + 48);
  h->flags = rd32(rec + 56);
  h->pw_bits = rd32(rec + 60);
  if (h->flags > 15) return ORC_ECORRUPT;
  if (h->flags & 4 ? (h->pw_bits > ORC_PW_MAXBITS || h->step != 1.0 || h->sumsq_hi != 0) : h->pw_bits != 0)
    return ORC_ECORRUPT;
  if (h->slice_log2 > 26 || h->chunk_log2 > h->slice_log2) return ORC_ECORRUPT;
  if (h->n_chunks != (uint32_t)((2ull << h->slice_log2) >> h->chunk_log2)) return ORC_ECORRUPT;
  if (h->n_used < 1 || h->n_used > ORC_NSYM) return ORC_ECORRUPT;
  uint64_t symtab_bytes = ((2 * (uint64_t)h->n_used) + 3) & ~(uint64_t)3;
  h->symtab = rec + ORC_HDR;
  uint64_t table_bytes = 4 * ((uint64_t)h->n_chunks + 1);
  h->nruns = 0;
  h->woff = NULL;
  if (h->flags & 8) {
    if (len < ORC_HDR + symtab_bytes + 4) return ORC_ECORRUPT;
    h->nruns = rd32(h->symtab + symtab_bytes);
    if (h->nruns < 1 || h->nruns > h->n_chunks || h->nruns > ORC_MAX_RUNS) return ORC_ECORRUPT;
    table_bytes = 8 * (uint64_t)h->nruns + 8;
  }
  uint64_t total = ORC_HDR + symtab_bytes + table_bytes + 4 * (uint64_t)h->n_words;
  if (total != h->total || total > len) return ORC_ECORRUPT;
  if (h->flags & 8) {
    h->offs = h->symtab + symtab_bytes + 4;
    h->woff = h->offs + 4 * (uint64_t)h->nruns;
    /* run ends strictly increasing up to n_chunks; word offsets non-decreasing
     * up to n_words, the last without a mark */
    uint32_t prev_end = 0, prev_w = 0;
    for (uint32_t r = 0; r < h->nruns; r++) {
      uint32_t e = rd32(h->offs + 4 * (uint64_t)r), w = rd32(h->woff + 4 * (uint64_t)r) & ~ORC_CONST_MARK;
      if (e <= prev_end || w < prev_w) return ORC_ECORRUPT;
      prev_end = e;
      prev_w = w;
    }
    uint32_t wl = rd32(h->woff + 4 * (uint64_t)h->nruns);
    if (prev_end != h->n_chunks || wl != h->n_words || wl < prev_w) return ORC_ECORRUPT;
  } else {
    h->offs = h->symtab + symtab_bytes;
  }
  h->words = h->symtab + symtab_bytes + table_bytes;
  return ORC_OK;
}

typedef struct {
  const uint32_t *w; /* chunk words, read as little-endian u32 */
  uint64_t nw;
  uint64_t pos;
} bitr;

static int get_bit(bitr *br, int *bit) {
  uint64_t wi = br->pos >> 5;
  if (wi >= br->nw) return ORC_ECORRUPT;
  uint32_t word;
  memcpy(&word, (const uint8_t *)br->w + 4 * wi, 4);
  *bit = (int)((word >> (31 - (br->pos & 31))) & 1);
  br->pos++;
  return ORC_OK;
}

static int get_bits(bitr *br, int n, uint64_t *v) {
  uint64_t x = 0;
  for (int k = 0; k < n; k++) {
    int b;
    if (get_bit(br, &b)) return ORC_ECORRUPT;
    x = (x << 1) | (uint64_t)b;
  }
  *v = x;
  return ORC_OK;
}

/* Decode a record into integer codes p (2L values, Re plane then Im plane).
 * Canonical decoding one bit at a time: a code of length l with value c is
 * symbol number c - first[l] among the symbols of length l in symbol order. */
int orc_decode_p(const uint8_t *rec, uint64_t len, int64_t *p) {
  orc_rec h;
  int rc = orc_parse(rec, len, &h);
  if (rc) return rc;
  uint32_t lens_count[ORC_LMAX + 1] = {0};
  uint16_t syms[ORC_NSYM];
  uint8_t lens[ORC_NSYM];
  int prev_key = -1;
  for (uint32_t k = 0; k < h.n_used; k++) {
    uint16_t e;
    memcpy(&e, h.symtab + 2 * k, 2);
    int s = e & 1023, l = e >> 10;
    int key = (l << 10) | s; /* entries are ordered by (length, symbol) */
    if (key <= prev_key || l > ORC_LMAX) return ORC_ECORRUPT;
    prev_key = key;
    if (h.n_used > 1 && l == 0) return ORC_ECORRUPT;
    if (h.n_used == 1 && l != 0) return ORC_ECORRUPT;
    syms[k] = (uint16_t)s;
    lens[k] = (uint8_t)l;
    lens_count[l]++;
  }
  if (h.n_used > 1) { /* a complete prefix code: sum of 2^-l equals 1 */
    uint64_t kraft = 0;
    for (int l = 1; l <= ORC_LMAX; l++) kraft += (uint64_t)lens_count[l] << (ORC_LMAX - l);
    if (kraft != ((uint64_t)1 << ORC_LMAX)) return ORC_ECORRUPT;
  }
  /* symbols sorted by (length, symbol), and the first code of each length */
  uint16_t by_len[ORC_NSYM];
  uint32_t first[ORC_LMAX + 2] = {0}, start[ORC_LMAX + 2] = {0};
  {
    uint32_t o = 0;
    for (int l = 1; l <= ORC_LMAX; l++) {
      start[l] = o;
      for (uint32_t k = 0; k < h.n_used; k++)
        if (lens[k] == l) by_len[o++] = syms[k];
    }
    uint32_t code = 0;
    for (int l = 1; l <= ORC_LMAX; l++) {
      code = (code + (l > 1 ? lens_count[l - 1] : 0)) << 1;
      first[l] = code;
    }
  }
  uint64_t B = (uint64_t)1 << h.chunk_log2;
  uint32_t run = 0, run_begin = 0; /* chunk-run records: the run holding chunk c */
  for (uint64_t c = 0; c < h.n_chunks; c++) {
    uint32_t o0, o1;
    if (h.flags & 8) {
      uint32_t end = rd32(h.offs + 4 * run);
      while (end <= c) { /* the next run: its end must lie beyond the previous one */
        run_begin = end;
        if (++run >= h.nruns) return ORC_ECORRUPT;
        end = rd32(h.offs + 4 * run);
        if (end <= run_begin) return ORC_ECORRUPT;
      }
      if (run + 1 == h.nruns && end != h.n_chunks) return ORC_ECORRUPT;
      o0 = rd32(h.woff + 4 * run);
      o1 = rd32(h.woff + 4 * (run + 1));
      if (run + 1 == h.nruns && (o1 & ~ORC_CONST_MARK) != h.n_words) return ORC_ECORRUPT;
      if (run + 1 == h.nruns && (o1 & ORC_CONST_MARK)) return ORC_ECORRUPT;
    } else {
      o0 = rd32(h.offs + 4 * c);
      o1 = rd32(h.offs + 4 * (c + 1));
      if (c + 1 == h.n_chunks && (o1 & ORC_CONST_MARK)) return ORC_ECORRUPT;
    }
    const int cconst = (o0 & ORC_CONST_MARK) != 0;
    if (cconst && !(h.flags & 2)) return ORC_ECORRUPT;
    uint32_t w0 = o0 & ~ORC_CONST_MARK, w1 = o1 & ~ORC_CONST_MARK;
    if (w1 < w0 || w1 > h.n_words) return ORC_ECORRUPT;
    if (!cconst && w1 == w0 && h.n_used > 1) { /* an empty chunk under a real code: all zero */
      if (!(h.flags & 1)) return ORC_ECORRUPT;
      for (uint64_t j = 0; j < B; j++) p[c * B + j] = 0;
      continue;
    }
    bitr br;
    br.w = (const uint32_t *)(h.words + 4 * (uint64_t)w0);
    br.nw = w1 - w0;
    br.pos = 0;
    int64_t prev = 0;
    for (uint64_t j = 0; j < B; j++) {
      if (cconst && j > 0) { /* a constant chunk: every value is the head's */
        p[c * B + j] = prev;
        continue;
      }
      int sym;
      if (h.n_used == 1) {
        sym = syms[0];
      } else {
        uint32_t code = 0;
        int l = 0;
        sym = -1;
        while (l < ORC_LMAX) {
          int b;
          if (get_bit(&br, &b)) return ORC_ECORRUPT;
          code = (code << 1) | (uint32_t)b;
          l++;
          if (code - first[l] < lens_count[l]) {
            sym = by_len[start[l] + (code - first[l])];
            break;
          }
        }
        if (sym < 0) return ORC_ECORRUPT;
      }
      int64_t dv;
      if (sym == 0) {
        uint64_t nb, z;
        if (get_bits(&br, ORC_ESC_LEN_BITS, &nb)) return ORC_ECORRUPT;
        if (get_bits(&br, (int)nb, &z)) return ORC_ECORRUPT;
        dv = unzigzag(z);
      } else {
        dv = (int64_t)sym - ORC_R;
      }
      prev = prev + dv;
      p[c * B + j] = prev;
    }
  }
  return ORC_OK;
}

/* Decompress into planes, a = p * kscale (kscale = step * normalisation). */
/* a = p * kscale, rounded to FP32 in FP32 mode */
int orc_decompress_slice_mode(const uint8_t *rec, uint64_t len, double kscale, uint32_t mode, double *re,
                              double *im) {
  orc_rec h;
  int rc = orc_parse(rec, len, &h);
  if (rc) return rc;
  uint64_t L = (uint64_t)1 << h.slice_log2;
  int64_t *p = (int64_t *)malloc(sizeof(int64_t) * 2 * L);
  if (!p) return ORC_ENOMEM;
  rc = orc_decode_p(rec, len, p);
  const int pw = (h.flags & 4) != 0;
  if (rc == ORC_OK) {
    for (uint64_t i = 0; i < L; i++) {
      re[i] = (pw ? pw_value(p[i], (int)h.pw_bits) : (double)p[i]) * kscale;
      im[i] = (pw ? pw_value(p[L + i], (int)h.pw_bits) : (double)p[L + i]) * kscale;
      if (mode & ORC_FP32) {
        re[i] = r32(re[i]);
        im[i] = r32(im[i]);
      }
    }
  }
  free(p);
  return rc;
}

int orc_decompress_slice(const uint8_t *rec, uint64_t len, double kscale, double *re, double *im) {
  return orc_decompress_slice_mode(rec, len, kscale, 0, re, im);
}

/* ----------------------------------------------------------- normalisation */

/* sum of p^2 as FP64: hi * 2^64 + lo, each half converted with one rounding */
static double sumsq_to_double(uint64_t lo, uint64_t hi) { return (double)hi * 0x1p64 + (double)lo; }

/* N = sum_j step_j^2 * P_j over the stored state, added as a pairwise tree over
 * slice indices (x_i <- x_2i + x_2i+1 level by level; count a power of two). */
double orc_norm_mode(int nslices, const double *step, const uint64_t *lo, const uint64_t *hi, uint32_t mode) {
  double *x = (double *)malloc(sizeof(double) * (size_t)nslices);
  for (int j = 0; j < nslices; j++) {
    if (mode & ORC_PWREL) /* the record holds the slice's squared norm itself */
      memcpy(&x[j], &lo[j], 8);
    else
      x[j] = (step[j] * step[j]) * sumsq_to_double(lo[j], hi[j]);
  }
  int m = nslices;
  while (m > 1) {
    for (int i = 0; i < m / 2; i++) x[i] = x[2 * i] + x[2 * i + 1];
    m /= 2;
  }
  double N = x[0];
  free(x);
  return N;
}

double orc_norm(int nslices, const double *step, const uint64_t *lo, const uint64_t *hi) {
  return orc_norm_mode(nslices, step, lo, hi, 0);
}

/* 1/sqrt(N) by ten Newton steps y <- y * (1.5 - (0.5 N y) y) from y = 1
 * (converged to the last bit for 0.25 <= N <= 2.5). */
double orc_rsqrt(double N) {
  double h = 0.5 * N;
  double y = 1.0;
  for (int k = 0; k < 10; k++) {
    double t = h * y;
    t = t * y;
    t = 1.5 - t;
    y = y * t;
  }
  return y;
}

/* ------------------------------------------------------ compressed simulator */

typedef struct {
  int n, slice_log2, chunk_log2;
  double eb;
  uint32_t mode;
  uint64_t nslices;
  uint8_t **rec;
  uint64_t *rec_len;
  double *step;
  uint64_t *sq_lo, *sq_hi;
  double max_err;
  uint64_t passes;
  uint64_t min_total_inv; /* largest total compressed bytes seen after any pass */
} orc_sim;

static uint64_t total_bytes(const orc_sim *s) {
  uint64_t t = 0;
  for (uint64_t j = 0; j < s->nslices; j++) t += s->rec_len[j];
  return t;
}

orc_sim *orc_sim_create(int n, int slice_log2, int chunk_log2, double eb, uint32_t mode) {
  if (n < 1 || n > 40 || slice_log2 < 1 || slice_log2 > n || slice_log2 > 26) return NULL;
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  if (!s) return NULL;
  s->n = n;
  s->slice_log2 = slice_log2;
  s->chunk_log2 = chunk_log2 > slice_log2 ? slice_log2 : chunk_log2;
  s->eb = eb;
  s->mode = mode;
  s->nslices = (uint64_t)1 << (n - slice_log2);
  s->rec = (uint8_t **)calloc(s->nslices, sizeof(uint8_t *));
  s->rec_len = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
  s->step = (double *)calloc(s->nslices, sizeof(double));
  s->sq_lo = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
  s->sq_hi = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
  return s;
}

void orc_sim_destroy(orc_sim *s) {
  if (!s) return;
  for (uint64_t j = 0; j < s->nslices; j++) free(s->rec[j]);
  free(s->rec); free(s->rec_len); free(s->step); free(s->sq_lo); free(s->sq_hi);
  free(s);
}

static void note_total(orc_sim *s) {
  uint64_t t = total_bytes(s);
  if (t > s->min_total_inv) s->min_total_inv = t;
}

/* Initial state: kind 0 = |0..0>, 1 = basis |x>, 2 = product state with
 * per-qubit factors f[q] = (f0re, f0im, f1re, f1im): psi_i = prod_q f_q(b_q),
 * multiplied from (1, 0) with qubit 0 first. */
int orc_sim_init(orc_sim *s, int kind, uint64_t x, const double *f) {
  uint64_t L = (uint64_t)1 << s->slice_log2;
  int rc_all = ORC_OK;
  uint8_t **nrec = (uint8_t **)calloc(s->nslices, sizeof(uint8_t *));
  uint64_t *nlen = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
  orc_cstats *st = (orc_cstats *)calloc(s->nslices, sizeof(orc_cstats));
#pragma omp parallel for schedule(dynamic)
  for (int64_t j = 0; j < (int64_t)s->nslices; j++) {
    double *re = (double *)calloc(L, sizeof(double));
    double *im = (double *)calloc(L, sizeof(double));
    for (uint64_t o = 0; o < L; o++) {
      uint64_t gi = ((uint64_t)j << s->slice_log2) | o;
      if (kind == 0) {
        re[o] = gi == 0 ? 1.0 : 0.0;
      } else if (kind == 1) {
        re[o] = gi == x ? 1.0 : 0.0;
      } else {
        const int fp32 = (s->mode & ORC_FP32) != 0;
        double ar = 1.0, ai = 0.0;
        for (int q = 0; q < s->n; q++) {
          int b = (int)((gi >> q) & 1);
          double cr = 0.0, ci = 0.0;
          const double fr = f[4 * q + 2 * b], fi = f[4 * q + 2 * b + 1];
          cmac_m(fp32, fp32 ? r32(fr) : fr, fp32 ? r32(fi) : fi, ar, ai, &cr, &ci);
          ar = cr;
          ai = ci;
        }
        re[o] = ar;
        im[o] = ai;
      }
    }
    int rc = orc_compress_slice(re, im, s->slice_log2, s->chunk_log2, s->eb, s->mode, &nrec[j], &nlen[j], &st[j]);
    if (rc) {
#pragma omp critical
      rc_all = rc;
    }
    free(re);
    free(im);
  }
  if (rc_all == ORC_OK) {
    for (uint64_t j = 0; j < s->nslices; j++) {
      if (!nrec[j]) continue; /* a group left as it was (ORC_OPT) */
      free(s->rec[j]);
      s->rec[j] = nrec[j];
      s->rec_len[j] = nlen[j];
      s->step[j] = st[j].step;
      s->sq_lo[j] = st[j].sumsq_lo;
      s->sq_hi[j] = st[j].sumsq_hi;
      if (st[j].max_err > s->max_err) s->max_err = st[j].max_err;
    }
    note_total(s);
  } else {
    for (uint64_t j = 0; j < s->nslices; j++) free(nrec[j]);
  }
  free(nrec); free(nlen); free(st);
  return rc_all;
}

double orc_sim_scale(const orc_sim *s) {
  return orc_rsqrt(orc_norm_mode((int)s->nslices, s->step, s->sq_lo, s->sq_hi, s->mode));
}

/* Slices whose index bits coincide except at the gate's target slice bits
 * form one group; return the members of the group led by j0 (ascending in
 * the local index of those bits). */
static int group_of(const orc_sim *s, const orc_gate *g, uint64_t j0, uint64_t *mem) {
  int m = 0;
  int bits[5];
  if (g->kind == ORC_DENSE)
    for (uint32_t t = 0; t < g->n_targets; t++)
      if ((int)g->targets[t] >= s->slice_log2) bits[m++] = (int)g->targets[t] - s->slice_log2;
  for (int u = 0; u < (1 << m); u++) {
    uint64_t j = j0;
    for (int b = 0; b < m; b++)
      if ((u >> b) & 1) j |= (uint64_t)1 << bits[b];
    mem[u] = j;
  }
  return 1 << m;
}

static uint64_t group_mask(const orc_sim *s, const orc_gate *g) {
  uint64_t mk = 0;
  if (g->kind == ORC_DENSE)
    for (uint32_t t = 0; t < g->n_targets; t++)
      if ((int)g->targets[t] >= s->slice_log2) mk |= (uint64_t)1 << (g->targets[t] - s->slice_log2);
  return mk;
}

static int check_gate(const orc_sim *s, const orc_gate *g) {
  uint64_t top = s->n >= 64 ? ~0ull : (((uint64_t)1 << s->n) - 1);
  if (g->ctrl_mask & ~top) return ORC_EINVAL;
  if (g->ctrl_vals & ~g->ctrl_mask) return ORC_EINVAL;
  if (g->kind == ORC_PHASE) return ORC_OK;
  if (g->kind != ORC_DENSE || g->n_targets < 1 || g->n_targets > 5 || !g->matrix) return ORC_EINVAL;
  uint64_t tm = 0;
  for (uint32_t t = 0; t < g->n_targets; t++) {
    if ((int)g->targets[t] >= s->n) return ORC_EINVAL;
    if (tm & ((uint64_t)1 << g->targets[t])) return ORC_EINVAL;
    tm |= (uint64_t)1 << g->targets[t];
  }
  if (tm & g->ctrl_mask) return ORC_EINVAL;
  return ORC_OK;
}

/* One pass of Algorithm 1 for one group: decompress each member, normalise
 * with the global scale, apply the gate, compress each member. */
static int process_group(const orc_sim *s, const orc_gate *g, double scale, int nmem, const uint64_t *mem,
                         uint8_t **orec, uint64_t *olen, orc_cstats *ost) {
  uint64_t L = (uint64_t)1 << s->slice_log2;
  double *re[32], *im[32];
  int rc = ORC_OK;
  for (int u = 0; u < nmem; u++) {
    re[u] = (double *)malloc(sizeof(double) * L);
    im[u] = (double *)malloc(sizeof(double) * L);
  }
  for (int u = 0; u < nmem && rc == ORC_OK; u++) {
    uint64_t j = mem[u];
    double k = s->step[j] * scale;                                          /* Normalize */
    rc = orc_decompress_slice_mode(s->rec[j], s->rec_len[j], k, s->mode, re[u], im[u]); /* Decompress */
  }
  if (rc == ORC_OK)
    rc = apply_gate_group(g, s->slice_log2, nmem, mem, re, im, (s->mode & ORC_FP32) != 0); /* GateComputation */
  for (int u = 0; u < nmem && rc == ORC_OK; u++)                              /* Compress */
    rc = orc_compress_slice(re[u], im[u], s->slice_log2, s->chunk_log2, s->eb, s->mode, &orec[u], &olen[u], &ost[u]);
  for (int u = 0; u < nmem; u++) {
    free(re[u]);
    free(im[u]);
  }
  return rc;
}

/* ORC_OPT: whether g is a SWAP of two slice-index qubits without controls
 * (a two-target dense gate whose matrix is exactly the exchange); *a, *b get
 * the two index bits. */
static int slice_swap(const orc_sim *s, const orc_gate *g, int *a, int *b) {
  if (g->kind != ORC_DENSE || g->n_targets != 2 || g->ctrl_mask) return 0;
  if ((int)g->targets[0] < s->slice_log2 || (int)g->targets[1] < s->slice_log2) return 0;
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 4; c++) {
      int one = (r == 0 && c == 0) || (r == 1 && c == 2) || (r == 2 && c == 1) || (r == 3 && c == 3);
      if (g->matrix[2 * (4 * r + c)] != (one ? 1.0 : 0.0) || g->matrix[2 * (4 * r + c) + 1] != 0.0) return 0;
    }
  *a = (int)g->targets[0] - s->slice_log2;
  *b = (int)g->targets[1] - s->slice_log2;
  return 1;
}

/* Apply gates one by one (one pass each).  A pass that fails leaves the state
 * as it was before that pass; *applied counts the completed passes. */
int orc_sim_apply(orc_sim *s, const orc_gate *gates, uint64_t ngates, uint64_t *applied) {
  *applied = 0;
  const int opt = (s->mode & ORC_OPT) != 0;
  for (uint64_t gi = 0; gi < ngates; gi++) {
    const orc_gate *g = &gates[gi];
    int rc = check_gate(s, g);
    if (rc) return rc;
    int sa, sb;
    if (opt && slice_swap(s, g, &sa, &sb)) { /* relabel: record j moves to sigma(j) */
      uint8_t **nrec = (uint8_t **)malloc(sizeof(uint8_t *) * s->nslices);
      uint64_t *nlen = (uint64_t *)malloc(sizeof(uint64_t) * s->nslices);
      double *nstep = (double *)malloc(sizeof(double) * s->nslices);
      uint64_t *nlo = (uint64_t *)malloc(sizeof(uint64_t) * s->nslices);
      uint64_t *nhi = (uint64_t *)malloc(sizeof(uint64_t) * s->nslices);
      if (!nrec || !nlen || !nstep || !nlo || !nhi) {
        free(nrec); free(nlen); free(nstep); free(nlo); free(nhi);
        return ORC_ENOMEM;
      }
      for (uint64_t j = 0; j < s->nslices; j++) {
        uint64_t ba = (j >> sa) & 1, bb = (j >> sb) & 1;
        uint64_t t = ba == bb ? j : j ^ (((uint64_t)1 << sa) | ((uint64_t)1 << sb));
        nrec[t] = s->rec[j];
        nlen[t] = s->rec_len[j];
        nstep[t] = s->step[j];
        nlo[t] = s->sq_lo[j];
        nhi[t] = s->sq_hi[j];
      }
      memcpy(s->rec, nrec, sizeof(uint8_t *) * s->nslices);
      memcpy(s->rec_len, nlen, sizeof(uint64_t) * s->nslices);
      memcpy(s->step, nstep, sizeof(double) * s->nslices);
      memcpy(s->sq_lo, nlo, sizeof(uint64_t) * s->nslices);
      memcpy(s->sq_hi, nhi, sizeof(uint64_t) * s->nslices);
      free(nrec); free(nlen); free(nstep); free(nlo); free(nhi);
      s->passes++;
      note_total(s);
      *applied = gi + 1;
      continue;
    }
    /* controls on slice-index qubits: the slice bits a group must have */
    const uint64_t lo_bits = ((uint64_t)1 << s->slice_log2) - 1;
    const uint64_t smask = opt ? (g->ctrl_mask & ~lo_bits) >> s->slice_log2 : 0;
    const uint64_t svals = opt ? (g->ctrl_vals & ~lo_bits) >> s->slice_log2 : 0;
    double scale = orc_sim_scale(s);
    uint64_t gm = group_mask(s, g);
    uint8_t **nrec = (uint8_t **)calloc(s->nslices, sizeof(uint8_t *));
    uint64_t *nlen = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
    orc_cstats *st = (orc_cstats *)calloc(s->nslices, sizeof(orc_cstats));
    int rc_all = ORC_OK;
#pragma omp parallel for schedule(dynamic)
    for (int64_t j0 = 0; j0 < (int64_t)s->nslices; j0++) {
      if ((uint64_t)j0 & gm) continue; /* not a group leader */
      if (((uint64_t)j0 & smask) != svals) continue; /* ORC_OPT: the gate is the identity here */
      uint64_t mem[32];
      uint8_t *orec[32];
      uint64_t olen[32];
      orc_cstats ost[32];
      memset(orec, 0, sizeof(orec));
      int nmem = group_of(s, g, (uint64_t)j0, mem);
      int rc2 = process_group(s, g, scale, nmem, mem, orec, olen, ost);
      if (rc2) {
#pragma omp critical
        rc_all = rc2;
        for (int u = 0; u < nmem; u++) free(orec[u]);
        continue;
      }
      for (int u = 0; u < nmem; u++) {
        nrec[mem[u]] = orec[u];
        nlen[mem[u]] = olen[u];
        st[mem[u]] = ost[u];
      }
    }
    if (rc_all) {
      for (uint64_t j = 0; j < s->nslices; j++) free(nrec[j]);
      free(nrec); free(nlen); free(st);
      return rc_all;
    }
    for (uint64_t j = 0; j < s->nslices; j++) {
      if (!nrec[j]) continue; /* a group left as it was (ORC_OPT) */
      free(s->rec[j]);
      s->rec[j] = nrec[j];
      s->rec_len[j] = nlen[j];
      s->step[j] = st[j].step;
      s->sq_lo[j] = st[j].sumsq_lo;
      s->sq_hi[j] = st[j].sumsq_hi;
      if (st[j].max_err > s->max_err) s->max_err = st[j].max_err;
    }
    free(nrec); free(nlen); free(st);
    s->passes++;
    note_total(s);
    *applied = gi + 1;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------ fused passes
 * Fused mode (an extension of Algorithm 1 that changes only how gates are
 * grouped into passes).  Walking the program in order, a pass takes
 * consecutive gates for as long as the qubits they involve together number
 * at most ORC_FUSE_MAX; a gate involves its target qubits and the qubits of
 * its control mask (a phase gate only the latter).  A gate that by itself
 * involves more qubits forms a pass alone.  A pass of one gate applies that
 * gate; a pass of several applies, as one dense gate on its qubits in
 * ascending order, the product U = G_last ... G_first of the gates written
 * as matrices over those qubits (block index bit i is the i-th qubit). */
#define ORC_FUSE_MAX 5

typedef struct {
  uint32_t first, count, fused, k;
  uint32_t qubits[5];
  uint32_t pad;
} orc_pass;

static uint64_t involved_qubits(const orc_gate *g) {
  uint64_t q = g->ctrl_mask;
  if (g->kind == ORC_DENSE)
    for (uint32_t t = 0; t < g->n_targets; t++) q |= (uint64_t)1 << g->targets[t];
  return q;
}

static int count_bits(uint64_t x) {
  int c = 0;
  while (x) {
    x &= x - 1;
    c++;
  }
  return c;
}

/* The pass partition; *npass receives the number of passes (out may be NULL
 * to count only; ORC_ENOMEM if cap is too small). */
int orc_plan(const orc_gate *gates, uint64_t n, orc_pass *out, uint64_t cap, uint64_t *npass) {
  uint64_t np = 0, i = 0;
  while (i < n) {
    uint64_t q = involved_qubits(&gates[i]);
    uint64_t end = i + 1;
    while (count_bits(q) <= ORC_FUSE_MAX && end < n) {
      uint64_t wider = q | involved_qubits(&gates[end]);
      if (count_bits(wider) > ORC_FUSE_MAX) break;
      q = wider;
      end++;
    }
    if (out && np < cap) {
      orc_pass *p = &out[np];
      memset(p, 0, sizeof(*p));
      p->first = (uint32_t)i;
      p->count = (uint32_t)(end - i);
      p->fused = p->count > 1;
      if (p->fused)
        for (uint32_t b = 0; b < 64; b++)
          if (q & ((uint64_t)1 << b)) p->qubits[p->k++] = b;
    }
    np++;
    i = end;
  }
  *npass = np;
  return out && np > cap ? ORC_ENOMEM : ORC_OK;
}

/* Entry (row r, column c) of gate g written over the block qubits q[0..k):
 * the amplitude that basis state c sends to basis state r. */
static void gate_entry(const orc_gate *g, const uint32_t *q, uint32_t k, uint32_t r, uint32_t c, double *er,
                       double *ei) {
  /* block bit of each qubit of the gate */
  int ctrl_ok = 1;
  for (uint32_t i = 0; i < k; i++) {
    uint64_t qb = (uint64_t)1 << q[i];
    if (g->ctrl_mask & qb) ctrl_ok &= (((c >> i) & 1u) == ((g->ctrl_vals & qb) ? 1u : 0u));
  }
  *er = 0.0;
  *ei = 0.0;
  if (!ctrl_ok || g->kind == ORC_PHASE) {
    if (r == c) {
      if (ctrl_ok) {
        *er = g->phase_re;
        *ei = g->phase_im;
      } else {
        *er = 1.0;
      }
    }
    return;
  }
  /* dense: the gate's row/column indices from the target bits, the other bits unchanged */
  uint32_t gr = 0, gc = 0, rest_r = r, rest_c = c;
  for (uint32_t t = 0; t < g->n_targets; t++) {
    uint32_t pos = 0;
    while (q[pos] != g->targets[t]) pos++;
    gr |= ((r >> pos) & 1u) << t;
    gc |= ((c >> pos) & 1u) << t;
    rest_r &= ~(1u << pos);
    rest_c &= ~(1u << pos);
  }
  if (rest_r != rest_c) return;
  uint32_t gdim = 1u << g->n_targets;
  *er = g->matrix[2 * (gr * gdim + gc)];
  *ei = g->matrix[2 * (gr * gdim + gc) + 1];
}

/* U (2^k x 2^k, row-major, interleaved) of a fused pass. */
int orc_block_matrix(const orc_gate *gates, const orc_pass *p, double *U) {
  uint32_t k = p->k, dim = 1u << k;
  double *G = (double *)malloc(sizeof(double) * 2 * dim * dim);
  double *T = (double *)malloc(sizeof(double) * 2 * dim * dim);
  if (!G || !T) {
    free(G);
    free(T);
    return ORC_ENOMEM;
  }
  for (uint32_t r = 0; r < dim; r++)
    for (uint32_t c = 0; c < dim; c++) {
      U[2 * (r * dim + c)] = r == c ? 1.0 : 0.0;
      U[2 * (r * dim + c) + 1] = 0.0;
    }
  for (uint32_t gi = p->first; gi < p->first + p->count; gi++) {
    for (uint32_t r = 0; r < dim; r++)
      for (uint32_t c = 0; c < dim; c++)
        gate_entry(&gates[gi], p->qubits, k, r, c, &G[2 * (r * dim + c)], &G[2 * (r * dim + c) + 1]);
    /* T = G U: every term, in ascending order */
    for (uint32_t r = 0; r < dim; r++)
      for (uint32_t c = 0; c < dim; c++) {
        double tr = 0.0, ti = 0.0;
        for (uint32_t m = 0; m < dim; m++)
          cmac(G[2 * (r * dim + m)], G[2 * (r * dim + m) + 1], U[2 * (m * dim + c)], U[2 * (m * dim + c) + 1], &tr,
               &ti);
        T[2 * (r * dim + c)] = tr;
        T[2 * (r * dim + c) + 1] = ti;
      }
    memcpy(U, T, sizeof(double) * 2 * dim * dim);
  }
  free(G);
  free(T);
  return ORC_OK;
}

/* Apply a program in fused mode; *applied counts the gates of completed
 * passes. */
int orc_sim_apply_fused(orc_sim *s, const orc_gate *gates, uint64_t ngates, uint64_t *applied) {
  *applied = 0;
  if (s->mode & ORC_OPT) return ORC_EINVAL; /* optimised passes are a plain-mode option */
  uint64_t np = 0;
  orc_plan(gates, ngates, NULL, 0, &np);
  orc_pass *plan = (orc_pass *)calloc(np ? np : 1, sizeof(orc_pass));
  double *U = (double *)malloc(sizeof(double) * 2 * 32 * 32);
  if (!plan || !U) {
    free(plan);
    free(U);
    return ORC_ENOMEM;
  }
  orc_plan(gates, ngates, plan, np, &np);
  int rc = ORC_OK;
  for (uint64_t i = 0; i < np && rc == ORC_OK; i++) {
    const orc_pass *p = &plan[i];
    uint64_t one = 0;
    if (!p->fused) {
      rc = orc_sim_apply(s, &gates[p->first], 1, &one);
    } else {
      rc = orc_block_matrix(gates, p, U);
      if (rc) break;
      orc_gate g;
      memset(&g, 0, sizeof(g));
      if (p->k == 0) { /* global phases only */
        g.kind = ORC_PHASE;
        g.phase_re = U[0];
        g.phase_im = U[1];
      } else {
        g.kind = ORC_DENSE;
        g.n_targets = p->k;
        for (uint32_t t = 0; t < p->k; t++) g.targets[t] = p->qubits[t];
        g.matrix = U;
      }
      rc = orc_sim_apply(s, &g, 1, &one);
    }
    if (rc == ORC_OK) *applied += p->count;
  }
  free(plan);
  free(U);
  return rc;
}

/* Recompute one group's pass from given input records (used to check single
 * slices of a large state).  in_rec[u] belongs to slice mem[u]; scale is the
 * normalisation of the whole input state. */
int orc_pass_group(int n, int slice_log2, int chunk_log2, double eb, uint32_t mode, const orc_gate *g, double scale,
                   int nmem, const uint64_t *mem, const uint8_t *const *in_rec, const uint64_t *in_len,
                   uint8_t **out_rec, uint64_t *out_len) {
  orc_sim s;
  memset(&s, 0, sizeof(s));
  s.n = n;
  s.slice_log2 = slice_log2;
  s.chunk_log2 = chunk_log2 > slice_log2 ? slice_log2 : chunk_log2;
  s.eb = eb;
  s.mode = mode;
  s.nslices = (uint64_t)1 << (n - slice_log2);
  int rc = check_gate(&s, g);
  if (rc) return rc;
  /* a private view holding only the group's records, indexed by slice */
  uint8_t *recs[32];
  uint64_t lens[32];
  double steps[32];
  for (int u = 0; u < nmem; u++) {
    orc_rec h;
    rc = orc_parse(in_rec[u], in_len[u], &h);
    if (rc) return rc;
    recs[u] = (uint8_t *)in_rec[u];
    lens[u] = in_len[u];
    steps[u] = h.step;
  }
  uint64_t L = (uint64_t)1 << slice_log2;
  double *re[32], *im[32];
  for (int u = 0; u < nmem; u++) {
    re[u] = (double *)malloc(sizeof(double) * L);
    im[u] = (double *)malloc(sizeof(double) * L);
  }
  for (int u = 0; u < nmem && rc == ORC_OK; u++)
    rc = orc_decompress_slice_mode(recs[u], lens[u], steps[u] * scale, mode, re[u], im[u]);
  if (rc == ORC_OK) rc = apply_gate_group(g, slice_log2, nmem, mem, re, im, (mode & ORC_FP32) != 0);
  for (int u = 0; u < nmem && rc == ORC_OK; u++) {
    orc_cstats st;
    rc = orc_compress_slice(re[u], im[u], slice_log2, s.chunk_log2, eb, mode, &out_rec[u], &out_len[u], &st);
  }
  for (int u = 0; u < nmem; u++) {
    free(re[u]);
    free(im[u]);
  }
  return rc;
}

/* Replace the stored record of slice j by a copy of rec (a state built
 * elsewhere, e.g. to recompute one pass from given records).  The record
 * must parse and have the simulator's geometry. */
int orc_sim_set_record(orc_sim *s, uint64_t j, const uint8_t *rec, uint64_t len) {
  orc_rec h;
  if (j >= s->nslices) return ORC_EINVAL;
  int rc = orc_parse(rec, len, &h);
  if (rc) return rc;
  if ((int)h.slice_log2 != s->slice_log2 || (int)h.chunk_log2 != s->chunk_log2) return ORC_EINVAL;
  uint8_t *c = (uint8_t *)malloc(len);
  if (!c) return ORC_ENOMEM;
  memcpy(c, rec, len);
  free(s->rec[j]);
  s->rec[j] = c;
  s->rec_len[j] = len;
  s->step[j] = h.step;
  s->sq_lo[j] = h.sumsq_lo;
  s->sq_hi[j] = h.sumsq_hi;
  return ORC_OK;
}

uint64_t orc_sim_nslices(const orc_sim *s) { return s->nslices; }
uint64_t orc_sim_record_len(const orc_sim *s, uint64_t j) { return j < s->nslices ? s->rec_len[j] : 0; }
int orc_sim_record(const orc_sim *s, uint64_t j, uint8_t *buf, uint64_t cap) {
  if (j >= s->nslices || cap < s->rec_len[j]) return ORC_EINVAL;
  memcpy(buf, s->rec[j], s->rec_len[j]);
  return ORC_OK;
}
uint64_t orc_sim_total_bytes(const orc_sim *s) { return total_bytes(s); }
uint64_t orc_sim_peak_bytes(const orc_sim *s) { return s->min_total_inv; }
double orc_sim_max_err(const orc_sim *s) { return s->max_err; }

/* Normalised amplitudes [begin, begin + count), interleaved (re, im). */
int orc_sim_amplitudes(const orc_sim *s, uint64_t begin, uint64_t count, double *out) {
  uint64_t N = (uint64_t)1 << s->n;
  if (begin > N || count > N - begin) return ORC_EINVAL;
  double scale = orc_sim_scale(s);
  uint64_t L = (uint64_t)1 << s->slice_log2;
  double *re = (double *)malloc(sizeof(double) * L);
  double *im = (double *)malloc(sizeof(double) * L);
  int rc = ORC_OK;
  uint64_t i = begin;
  while (i < begin + count && rc == ORC_OK) {
    uint64_t j = i >> s->slice_log2;
    rc = orc_decompress_slice_mode(s->rec[j], s->rec_len[j], s->step[j] * scale, s->mode, re, im);
    uint64_t end = (j + 1) << s->slice_log2;
    if (end > begin + count) end = begin + count;
    for (; i < end && rc == ORC_OK; i++) {
      uint64_t o = i & (L - 1);
      out[2 * (i - begin)] = re[o];
      out[2 * (i - begin) + 1] = im[o];
    }
  }
  free(re);
  free(im);
  return rc;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* ------------------------------------------------------- code-level runner
 * The stages of Compress after the quantiser -- Lorenzo difference, symbols,
 * escapes, Huffman code, record layout -- are lossless: Decompress returns
 * exactly the codes p that Compress was given.  The amplitudes of a run of
 * Algorithm 1 therefore depend only on the codes, the steps and the norm, and
 * this runner keeps just those: the codes p of every slice (as int32; a pass
 * that makes a code of magnitude 2^31 or more is refused with ORC_EBOUND),
 * and the step and sum p^2 of every slice.  A pass is the full simulator's
 * pass without the lossless stages: the global scale s from the norm of the
 * stored state, a = p * (step_j * s), the gate on each group of slices, the
 * quantiser.  It can follow runs far too long for the full codec (hundreds of
 * thousands of passes over 2^24 amplitudes); tests check that it reproduces
 * the full simulator's codes and amplitudes. */

/* The gate on one group, as apply_gate_group computes it -- the same
 * operations on the same operands in the same order -- with the amplitudes
 * addressed by a local index u * L + o (member u, offset o): target bits
 * below slice_log2 keep their position, the slice-bit targets take bits
 * slice_log2, slice_log2 + 1, ... in the order group_of gives the members. */
static int apply_gate_local(const orc_gate *g, int slice_log2, int nmem, const uint64_t *mem, double **re,
                            double **im, int fp32) {
  if (g->kind == ORC_PHASE) return apply_gate_group(g, slice_log2, nmem, mem, re, im, fp32);
  if (g->kind != ORC_DENSE || g->n_targets < 1 || g->n_targets > 5) return ORC_EINVAL;
  const uint64_t L = (uint64_t)1 << slice_log2, omask = L - 1;
  const int k = (int)g->n_targets, dim = 1 << k;
  uint64_t off[32], tl = 0;
  int lb[5], nslice = 0;
  for (int t = 0; t < k; t++) {
    lb[t] = (int)g->targets[t] < slice_log2 ? (int)g->targets[t] : slice_log2 + nslice++;
    tl |= (uint64_t)1 << lb[t];
  }
  if ((1 << nslice) != nmem) return ORC_EINVAL;
  for (int m = 0; m < dim; m++) {
    off[m] = 0;
    for (int t = 0; t < k; t++)
      if ((m >> t) & 1) off[m] |= (uint64_t)1 << lb[t];
  }
  double ur[1024], ui[1024];
  for (int e = 0; e < dim * dim; e++) {
    ur[e] = fp32 ? r32(g->matrix[2 * e]) : g->matrix[2 * e];
    ui[e] = fp32 ? r32(g->matrix[2 * e + 1]) : g->matrix[2 * e + 1];
  }
  double in_r[32], in_i[32], out_r[32], out_i[32];
  const uint64_t total = (uint64_t)nmem << slice_log2;
  if (k == 1) { /* the loop below written out for one target */
    for (uint64_t li = 0; li < total; li++) {
      if (li & tl) continue;
      const uint64_t gi = (mem[li >> slice_log2] << slice_log2) | (li & omask);
      if ((gi & g->ctrl_mask) != g->ctrl_vals) continue;
      const uint64_t x1 = li | off[1];
      double *r0 = &re[li >> slice_log2][li & omask], *i0 = &im[li >> slice_log2][li & omask];
      double *r1 = &re[x1 >> slice_log2][x1 & omask], *i1 = &im[x1 >> slice_log2][x1 & omask];
      const double a0r = *r0, a0i = *i0, a1r = *r1, a1i = *i1;
      double c0r = 0.0, c0i = 0.0, c1r = 0.0, c1i = 0.0;
      cmac_m(fp32, ur[0], ui[0], a0r, a0i, &c0r, &c0i);
      cmac_m(fp32, ur[1], ui[1], a1r, a1i, &c0r, &c0i);
      cmac_m(fp32, ur[2], ui[2], a0r, a0i, &c1r, &c1i);
      cmac_m(fp32, ur[3], ui[3], a1r, a1i, &c1r, &c1i);
      *r0 = c0r;
      *i0 = c0i;
      *r1 = c1r;
      *i1 = c1i;
    }
    return ORC_OK;
  }
  for (uint64_t li = 0; li < total; li++) {
    if (li & tl) continue;
    const uint64_t gi = (mem[li >> slice_log2] << slice_log2) | (li & omask);
    if ((gi & g->ctrl_mask) != g->ctrl_vals) continue;
    for (int m = 0; m < dim; m++) {
      const uint64_t x = li | off[m];
      in_r[m] = re[x >> slice_log2][x & omask];
      in_i[m] = im[x >> slice_log2][x & omask];
    }
    for (int r = 0; r < dim; r++) {
      double cr = 0.0, ci = 0.0;
      for (int c = 0; c < dim; c++) cmac_m(fp32, ur[r * dim + c], ui[r * dim + c], in_r[c], in_i[c], &cr, &ci);
      out_r[r] = cr;
      out_i[r] = ci;
    }
    for (int m = 0; m < dim; m++) {
      const uint64_t x = li | off[m];
      re[x >> slice_log2][x & omask] = out_r[m];
      im[x >> slice_log2][x & omask] = out_i[m];
    }
  }
  return ORC_OK;
}

/* The same gate through both addressings (tests compare them). */
int orc_group_apply_local(const orc_gate *g, int slice_log2, int nmem, const uint64_t *slices, double **re,
                          double **im, int fp32) {
  return apply_gate_local(g, slice_log2, nmem, slices, re, im, fp32);
}

typedef struct {
  int n, slice_log2;
  double eb;
  uint32_t mode;
  uint64_t nslices, L;
  int32_t *p; /* [nslices][2L]: real plane, then imaginary plane */
  double *step;
  uint64_t *sq_lo, *sq_hi;
  int32_t *p2; /* the same for the output of a pass */
  double *step2;
  uint64_t *lo2, *hi2;
  double max_err;
  uint64_t passes;
} orc_vsim;

void orc_vsim_destroy(orc_vsim *s);

orc_vsim *orc_vsim_create(int n, int slice_log2, double eb, uint32_t mode) {
  if (n < 1 || n > 40 || slice_log2 < 1 || slice_log2 > n || slice_log2 > 26) return NULL;
  if (mode & ORC_PWREL) return NULL; /* codes only: the pointwise-relative norm needs the values */
  if (mode & ORC_OPT) return NULL;   /* Algorithm 1 as written only */
  orc_vsim *s = (orc_vsim *)calloc(1, sizeof(orc_vsim));
  if (!s) return NULL;
  s->n = n;
  s->slice_log2 = slice_log2;
  s->eb = eb;
  s->mode = mode;
  s->nslices = (uint64_t)1 << (n - slice_log2);
  s->L = (uint64_t)1 << slice_log2;
  s->p = (int32_t *)calloc(s->nslices * 2 * s->L, sizeof(int32_t));
  s->step = (double *)calloc(s->nslices, sizeof(double));
  s->sq_lo = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
  s->sq_hi = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
  s->p2 = (int32_t *)calloc(s->nslices * 2 * s->L, sizeof(int32_t));
  s->step2 = (double *)calloc(s->nslices, sizeof(double));
  s->lo2 = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
  s->hi2 = (uint64_t *)calloc(s->nslices, sizeof(uint64_t));
  if (!s->p || !s->step || !s->sq_lo || !s->sq_hi || !s->p2 || !s->step2 || !s->lo2 || !s->hi2) {
    orc_vsim_destroy(s);
    return NULL;
  }
  return s;
}

void orc_vsim_destroy(orc_vsim *s) {
  if (!s) return;
  free(s->p); free(s->step); free(s->sq_lo); free(s->sq_hi);
  free(s->p2); free(s->step2); free(s->lo2); free(s->hi2);
  free(s);
}

/* Quantise one slice's 2L values into codes; fills the slice's step and
 * sum p^2 into the given outputs. */
static int vsim_quantise(const orc_vsim *s, const double *v, int32_t *codes, int64_t *tmp, double *step,
                         uint64_t *lo, uint64_t *hi, double *max_err) {
  unsigned __int128 sq;
  int rc = quantise(v, 2 * s->L, s->eb, s->mode, tmp, step, max_err, &sq);
  if (rc) return rc;
  for (uint64_t i = 0; i < 2 * s->L; i++) {
    if (tmp[i] > INT32_MAX || tmp[i] < -INT32_MAX) return ORC_EBOUND;
    codes[i] = (int32_t)tmp[i];
  }
  *lo = (uint64_t)sq;
  *hi = (uint64_t)(sq >> 64);
  return ORC_OK;
}

/* Initial states as orc_sim_init builds them. */
int orc_vsim_init(orc_vsim *s, int kind, uint64_t x, const double *f) {
  const uint64_t L = s->L;
  const int fp32 = (s->mode & ORC_FP32) != 0;
  int rc_all = ORC_OK;
  double err_all = 0.0;
#pragma omp parallel for schedule(dynamic)
  for (int64_t j = 0; j < (int64_t)s->nslices; j++) {
    double *v = (double *)calloc(2 * L, sizeof(double));
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * 2 * L);
    int rc = v && tmp ? ORC_OK : ORC_ENOMEM;
    for (uint64_t o = 0; o < L && rc == ORC_OK; o++) {
      uint64_t gi = ((uint64_t)j << s->slice_log2) | o;
      if (kind == 0) {
        v[o] = gi == 0 ? 1.0 : 0.0;
      } else if (kind == 1) {
        v[o] = gi == x ? 1.0 : 0.0;
      } else {
        double ar = 1.0, ai = 0.0;
        for (int q = 0; q < s->n; q++) {
          int b = (int)((gi >> q) & 1);
          double cr = 0.0, ci = 0.0;
          const double fr = f[4 * q + 2 * b], fi = f[4 * q + 2 * b + 1];
          cmac_m(fp32, fp32 ? r32(fr) : fr, fp32 ? r32(fi) : fi, ar, ai, &cr, &ci);
          ar = cr;
          ai = ci;
        }
        v[o] = ar;
        v[L + o] = ai;
      }
    }
    double err = 0.0;
    if (rc == ORC_OK)
      rc = vsim_quantise(s, v, s->p + (uint64_t)j * 2 * L, tmp, &s->step[j], &s->sq_lo[j], &s->sq_hi[j], &err);
#pragma omp critical
    {
      if (rc) rc_all = rc;
      if (err > err_all) err_all = err;
    }
    free(v);
    free(tmp);
  }
  if (err_all > s->max_err) s->max_err = err_all;
  return rc_all;
}

double orc_vsim_scale(const orc_vsim *s) {
  return orc_rsqrt(orc_norm((int)s->nslices, s->step, s->sq_lo, s->sq_hi));
}

/* One pass of one gate.  The new codes go to a second buffer, so a failing
 * pass leaves the state as it was. */
static int vsim_pass(orc_vsim *s, const orc_gate *g, int32_t *np, double *nstep, uint64_t *nlo, uint64_t *nhi) {
  const uint64_t L = s->L;
  const int fp32 = (s->mode & ORC_FP32) != 0;
  const double scale = orc_vsim_scale(s);
  orc_sim view; /* for the group helpers: geometry only */
  memset(&view, 0, sizeof(view));
  view.n = s->n;
  view.slice_log2 = s->slice_log2;
  view.nslices = s->nslices;
  int rc = check_gate(&view, g);
  if (rc) return rc;
  const uint64_t gm = group_mask(&view, g);
  int rc_all = ORC_OK;
  double err_all = 0.0;
#pragma omp parallel for schedule(dynamic)
  for (int64_t j0 = 0; j0 < (int64_t)s->nslices; j0++) {
    if ((uint64_t)j0 & gm) continue; /* not a group leader */
    uint64_t mem[32];
    const int nmem = group_of(&view, g, (uint64_t)j0, mem);
    double *buf = (double *)malloc(sizeof(double) * 2 * L * (uint64_t)nmem);
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * 2 * L);
    int rc2 = buf && tmp ? ORC_OK : ORC_ENOMEM;
    double *re[32], *im[32];
    double err = 0.0;
    for (int u = 0; u < nmem && rc2 == ORC_OK; u++) { /* Decompress + Normalize */
      const uint64_t j = mem[u];
      const double k = s->step[j] * scale;
      const int32_t *c = s->p + j * 2 * L;
      double *v = buf + (uint64_t)u * 2 * L;
      for (uint64_t i = 0; i < 2 * L; i++) {
        double a = (double)c[i] * k;
        v[i] = fp32 ? r32(a) : a;
      }
      re[u] = v;
      im[u] = v + L;
    }
    if (rc2 == ORC_OK) rc2 = apply_gate_local(g, s->slice_log2, nmem, mem, re, im, fp32); /* GateComputation */
    for (int u = 0; u < nmem && rc2 == ORC_OK; u++) {                                    /* Compress */
      const uint64_t j = mem[u];
      double e = 0.0;
      rc2 = vsim_quantise(s, buf + (uint64_t)u * 2 * L, np + j * 2 * L, tmp, &nstep[j], &nlo[j], &nhi[j], &e);
      if (e > err) err = e;
    }
#pragma omp critical
    {
      if (rc2) rc_all = rc2;
      if (err > err_all) err_all = err;
    }
    free(buf);
    free(tmp);
  }
  if (rc_all == ORC_OK && err_all > s->max_err) s->max_err = err_all;
  return rc_all;
}

/* ABS mode with a one-target dense gate or a phase gate: Decompress,
 * Normalize, GateComputation and the quantiser in one sweep over each group
 * of one or two slices, with the operations of the general pass on every
 * value (apply_gate_group's complex multiply-adds, quantise's steps and
 * checks; sum p^2 is exact, so its order does not matter).  Returns 1 when
 * the gate is not of this kind (the general pass runs instead). */
static int vsim_pass_abs1(orc_vsim *s, const orc_gate *g, int32_t *np, double *nstep, uint64_t *nlo,
                          uint64_t *nhi, int *rc_out) {
  if ((s->mode & 1) || !(g->kind == ORC_PHASE || (g->kind == ORC_DENSE && g->n_targets == 1))) return 1;
  const uint64_t L = s->L, sl2 = (uint64_t)s->slice_log2;
  const int fp32 = (s->mode & ORC_FP32) != 0;
  const double scale = orc_vsim_scale(s);
  double step, r;
  orc_abs_step(s->eb, &step, &r);
  const double eb = s->eb;
  const int dense = g->kind == ORC_DENSE;
  const uint64_t t = dense ? g->targets[0] : 0;
  const int cross = dense && t >= sl2;            /* pairs across two slices */
  const uint64_t gm = cross ? (uint64_t)1 << (t - sl2) : 0;
  const uint64_t tb = dense && !cross ? (uint64_t)1 << t : 0;
  double u[8];
  if (dense)
    for (int e = 0; e < 8; e++) u[e] = fp32 ? r32(g->matrix[e]) : g->matrix[e];
  const double phr = fp32 ? r32(g->phase_re) : g->phase_re, phi = fp32 ? r32(g->phase_im) : g->phase_im;
  int rc_all = ORC_OK;
  double err_all = 0.0;
#pragma omp parallel for schedule(dynamic)
  for (int64_t j0 = 0; j0 < (int64_t)s->nslices; j0++) {
    if ((uint64_t)j0 & gm) continue;
    const uint64_t ja = (uint64_t)j0, jb = ja | gm;
    const double ka = s->step[ja] * scale, kb = s->step[jb] * scale;
    const int32_t *pa = s->p + ja * 2 * L, *pb = s->p + jb * 2 * L;
    int32_t *oa = np + ja * 2 * L, *ob = np + jb * 2 * L;
    unsigned __int128 sqa = 0, sqb = 0;
    double err = 0.0;
    int bad = 0;
#define CQ_DEC(c, k) (fp32 ? r32((double)(c) * (k)) : (double)(c) * (k))
#define CQ_QUANT(v, dst, sq)                                                     \
  do {                                                                           \
    const double q_ = rint((v) * r);                                             \
    if (!(fabs(q_) < 2147483648.0)) {                                            \
      bad = 1;                                                                   \
      (dst) = 0;                                                                 \
    } else {                                                                     \
      const int64_t p_ = (int64_t)q_;                                            \
      const double e_ = fabs((v) - (double)p_ * step);                           \
      if (e_ > eb) bad = 1;                                                      \
      if (e_ > err) err = e_;                                                    \
      (dst) = (int32_t)p_;                                                       \
      (sq) += (unsigned __int128)((__int128)p_ * (__int128)p_);                  \
    }                                                                            \
  } while (0)
    if (!dense) { /* phase gate: one slice */
      for (uint64_t o = 0; o < L; o++) {
        const uint64_t gi = (ja << sl2) | o;
        double ar = CQ_DEC(pa[o], ka), ai = CQ_DEC(pa[L + o], ka);
        if ((gi & g->ctrl_mask) == g->ctrl_vals) {
          double cr = 0.0, ci = 0.0;
          cmac_m(fp32, phr, phi, ar, ai, &cr, &ci);
          ar = cr;
          ai = ci;
        }
        CQ_QUANT(ar, oa[o], sqa);
        CQ_QUANT(ai, oa[L + o], sqa);
      }
    } else {
      /* pairs (x0, x1): x1 = x0 | tb inside slice ja, or offset o of slices ja and jb */
      const uint64_t npair = cross ? L : L / 2;
      for (uint64_t i = 0; i < npair; i++) {
        const uint64_t o0 = cross ? i : ((i & ~(tb - 1)) << 1) | (i & (tb - 1));
        const uint64_t o1 = cross ? i : (o0 | tb);
        const int32_t *p1 = cross ? pb : pa;
        int32_t *q1 = cross ? ob : oa;
        const double k1 = cross ? kb : ka;
        const uint64_t g0 = (ja << sl2) | o0;  /* controls never touch the target bit */
        double a0r = CQ_DEC(pa[o0], ka), a0i = CQ_DEC(pa[L + o0], ka);
        double a1r = CQ_DEC(p1[o1], k1), a1i = CQ_DEC(p1[L + o1], k1);
        if ((g0 & g->ctrl_mask) == g->ctrl_vals) {
          double c0r = 0.0, c0i = 0.0, c1r = 0.0, c1i = 0.0;
          cmac_m(fp32, u[0], u[1], a0r, a0i, &c0r, &c0i);
          cmac_m(fp32, u[2], u[3], a1r, a1i, &c0r, &c0i);
          cmac_m(fp32, u[4], u[5], a0r, a0i, &c1r, &c1i);
          cmac_m(fp32, u[6], u[7], a1r, a1i, &c1r, &c1i);
          a0r = c0r;
          a0i = c0i;
          a1r = c1r;
          a1i = c1i;
        }
        CQ_QUANT(a0r, oa[o0], sqa);
        CQ_QUANT(a0i, oa[L + o0], sqa);
        if (cross) {
          CQ_QUANT(a1r, q1[o1], sqb);
          CQ_QUANT(a1i, q1[L + o1], sqb);
        } else {
          CQ_QUANT(a1r, q1[o1], sqa);
          CQ_QUANT(a1i, q1[L + o1], sqa);
        }
      }
    }
#undef CQ_DEC
#undef CQ_QUANT
    nstep[ja] = step;
    nlo[ja] = (uint64_t)sqa;
    nhi[ja] = (uint64_t)(sqa >> 64);
    if (cross) {
      nstep[jb] = step;
      nlo[jb] = (uint64_t)sqb;
      nhi[jb] = (uint64_t)(sqb >> 64);
    }
#pragma omp critical
    {
      if (bad) rc_all = ORC_EBOUND;
      if (err > err_all) err_all = err;
    }
  }
  if (rc_all == ORC_OK && err_all > s->max_err) s->max_err = err_all;
  *rc_out = rc_all;
  return 0;
}

static int vsim_run(orc_vsim *s, const orc_gate *g) {
  int rc = ORC_OK;
  orc_sim view; /* geometry for check_gate */
  memset(&view, 0, sizeof(view));
  view.n = s->n;
  view.slice_log2 = s->slice_log2;
  view.nslices = s->nslices;
  if ((rc = check_gate(&view, g))) return rc;
  if (vsim_pass_abs1(s, g, s->p2, s->step2, s->lo2, s->hi2, &rc)) rc = vsim_pass(s, g, s->p2, s->step2, s->lo2, s->hi2);
  if (rc == ORC_OK) {
    int32_t *t = s->p; s->p = s->p2; s->p2 = t;
    double *ts = s->step; s->step = s->step2; s->step2 = ts;
    uint64_t *tl = s->sq_lo; s->sq_lo = s->lo2; s->lo2 = tl;
    uint64_t *th = s->sq_hi; s->sq_hi = s->hi2; s->hi2 = th;
    s->passes++;
  }
  return rc;
}

/* Plain mode: one pass per gate; *applied counts completed passes. */
int orc_vsim_apply(orc_vsim *s, const orc_gate *gates, uint64_t ngates, uint64_t *applied) {
  *applied = 0;
  for (uint64_t i = 0; i < ngates; i++) {
    int rc = vsim_run(s, &gates[i]);
    if (rc) return rc;
    *applied = i + 1;
  }
  return ORC_OK;
}

/* Fused mode, with the partition and block matrices of orc_sim_apply_fused;
 * *applied counts the gates of completed passes. */
int orc_vsim_apply_fused(orc_vsim *s, const orc_gate *gates, uint64_t ngates, uint64_t *applied) {
  *applied = 0;
  uint64_t np = 0;
  orc_plan(gates, ngates, NULL, 0, &np);
  orc_pass *plan = (orc_pass *)calloc(np ? np : 1, sizeof(orc_pass));
  double *U = (double *)malloc(sizeof(double) * 2 * 32 * 32);
  if (!plan || !U) {
    free(plan);
    free(U);
    return ORC_ENOMEM;
  }
  orc_plan(gates, ngates, plan, np, &np);
  int rc = ORC_OK;
  for (uint64_t i = 0; i < np && rc == ORC_OK; i++) {
    const orc_pass *p = &plan[i];
    if (!p->fused) {
      rc = vsim_run(s, &gates[p->first]);
    } else {
      rc = orc_block_matrix(gates, p, U);
      if (rc) break;
      orc_gate g;
      memset(&g, 0, sizeof(g));
      if (p->k == 0) {
        g.kind = ORC_PHASE;
        g.phase_re = U[0];
        g.phase_im = U[1];
      } else {
        g.kind = ORC_DENSE;
        g.n_targets = p->k;
        for (uint32_t t = 0; t < p->k; t++) g.targets[t] = p->qubits[t];
        g.matrix = U;
      }
      rc = vsim_run(s, &g);
    }
    if (rc == ORC_OK) *applied += p->count;
  }
  free(plan);
  free(U);
  return rc;
}

/* Normalised amplitudes [begin, begin + count), interleaved (re, im), as
 * orc_sim_amplitudes reads them out. */
int orc_vsim_amplitudes(const orc_vsim *s, uint64_t begin, uint64_t count, double *out) {
  const uint64_t N = (uint64_t)1 << s->n, L = s->L;
  if (begin > N || count > N - begin) return ORC_EINVAL;
  const double scale = orc_vsim_scale(s);
  const int fp32 = (s->mode & ORC_FP32) != 0;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < (int64_t)count; t++) {
    const uint64_t i = begin + (uint64_t)t, j = i >> s->slice_log2, o = i & (L - 1);
    const double k = s->step[j] * scale;
    double ar = (double)s->p[j * 2 * L + o] * k, ai = (double)s->p[j * 2 * L + L + o] * k;
    out[2 * t] = fp32 ? r32(ar) : ar;
    out[2 * t + 1] = fp32 ? r32(ai) : ai;
  }
  return ORC_OK;
}

/* The whole state: codes [nslices][2L], steps, sum p^2 (low, high words);
 * get copies it out, set replaces it (a checkpoint of a long run). */
void orc_vsim_get(const orc_vsim *s, int32_t *codes, double *step, uint64_t *lo, uint64_t *hi) {
  memcpy(codes, s->p, sizeof(int32_t) * s->nslices * 2 * s->L);
  memcpy(step, s->step, sizeof(double) * s->nslices);
  memcpy(lo, s->sq_lo, sizeof(uint64_t) * s->nslices);
  memcpy(hi, s->sq_hi, sizeof(uint64_t) * s->nslices);
}

void orc_vsim_set(orc_vsim *s, const int32_t *codes, const double *step, const uint64_t *lo, const uint64_t *hi,
                  uint64_t passes, double max_err) {
  memcpy(s->p, codes, sizeof(int32_t) * s->nslices * 2 * s->L);
  memcpy(s->step, step, sizeof(double) * s->nslices);
  memcpy(s->sq_lo, lo, sizeof(uint64_t) * s->nslices);
  memcpy(s->sq_hi, hi, sizeof(uint64_t) * s->nslices);
  s->passes = passes;
  s->max_err = max_err;
}

uint64_t orc_vsim_passes(const orc_vsim *s) { return s->passes; }
double orc_vsim_max_err(const orc_vsim *s) { return s->max_err; }
