// Host side of libcqsim: the C ABI declared in include/cqsim.h.
//
// The handle owns the compressed state: two arenas of slice records (the
// input and output of a pass, swapped after every pass), per-slice metadata
// for each arena, and a workspace of W slots into which slices are
// decompressed.  A pass enqueues, for every batch of whole slice groups that
// fits the workspace, the kernel chain of kernels.hip; nothing returns to the
// host between passes.  Failures raise a flag in device memory that turns all
// later kernels into no-ops; the host reads it once per sim_apply call, rolls
// back to the input arena of the failed pass and, when the output arena was
// too small, grows it and runs the remaining passes again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "cqsim.h"
#include "cqsim_impl.h"

using namespace cq;
using cq::f64::launch_begin_pass;
using cq::f64::launch_codebook;
using cq::f64::launch_encode;
using cq::f64::launch_finish;
using cq::f64::launch_runs;
using cq::f64::launch_carry;
using cq::f64::launch_rel_step;
using cq::f64::launch_reset_slots;

// the amplitude launcher of the simulator's precision (SIM_FP32: namespace f32)
#define AMP(sim, fn) ((sim)->fp32 ? cq::f32::fn : cq::f64::fn)

namespace {

thread_local std::string g_last_error = "no error";

int set_err(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int set_err(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace

int cq::fail(int code, const char *msg) { return set_err(code, "%s", msg); }

namespace {

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_err(SIM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

enum KClass { K_BEGIN, K_RESET, K_INIT, K_DECODE, K_MINMAX, K_RELSTEP, K_GATEQ, K_CODEBOOK, K_ENCODE, K_FINISH,
              K_READOUT, K_DENSE, K_RUNS, K_COUNT };
const char *kClassNames =
    "begin_pass,reset_slots,init,decode,gate_minmax,rel_step,gate_quant,codebook,encode,finish,readout,dense_mfma,"
    "runs";

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

uint64_t rec_bytes_host(uint32_t n_used, uint32_t nchunks, uint64_t words) {
  return (uint64_t)kHdr + ((2ull * n_used + 3) & ~3ull) + 4ull * (nchunks + 1) + 4ull * words;
}

}  // namespace

struct sim_s {
  Geo geo{};
  double eb = 0;
  uint32_t mode = 0;
  bool fp32 = false;  // SIM_FP32: working values, gate matrices and factors rounded to FP32
  uint64_t nslices = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void *(*al_fn)(size_t, void *) = nullptr;
  void (*al_free)(void *, void *) = nullptr;
  void *al_ctx = nullptr;
  struct Owner {
    void (*free_fn)(void *, void *);  // NULL: hipFree
    void *ctx;
    size_t bytes;
  };
  std::map<void *, Owner> owned;
  uint64_t dev_bytes = 0;  // sum over `owned`
  bool dry = false;        // count the bytes of every dalloc, allocate nothing (sim_footprint)

  Ctl *ctl = nullptr;
  Ctl *h_ctl = nullptr;  // pinned host copy
  uint8_t *arena[2] = {nullptr, nullptr};
  uint64_t arena_cap[2] = {0, 0};
  StateMeta meta[2]{};
  int cur = 0;
  double *kscale = nullptr;
  Slots slots{};
  int W = 0;
  std::map<uint64_t, uint64_t *> tables;  // group mask -> slot order of all slices
  // SIM_OPT: slices a pass processes and those it carries over unchanged, per
  // (group mask, slice-index control mask, values), or, for a relabelling
  // SWAP, per (all ones, bit a, bit b); and the carried records' offsets
  struct OptLists {
    uint64_t *active = nullptr, n_active = 0;
    uint64_t *src = nullptr, *dst = nullptr, n_carry = 0;
  };
  std::map<std::array<uint64_t, 3>, OptLists> opt_lists;
  uint64_t *carry_off = nullptr;
  // The workspace that passes run on: the handle's own (slots, W, tables),
  // or, during sim_apply_noalloc, one carved from the scratch array, with
  // every slot table present and no device allocation allowed.
  const Slots *wslots = nullptr;
  int wW = 0;
  const std::map<uint64_t, uint64_t *> *wtables = nullptr;
  bool no_alloc = false;
  const Slots &run_slots() const { return wslots ? *wslots : slots; }
  int run_W() const { return wslots ? wW : W; }
  double *dmat = nullptr;
  size_t dmat_cap = 0;  // doubles
  GateDesc ident{};     // the identity (kind 0): quantisation step of fused passes
  double *dfactors = nullptr;
  double *dstage = nullptr;
  size_t dstage_cap = 0;  // doubles
  uint32_t pass_counter = 0;
  uint64_t passes = 0;
  uint64_t gates = 0;  // program gates applied (a fused pass applies one or more)
  double elapsed = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream on which gate programs are captured into graphs

  bool kt_on = false;
  std::vector<hipEvent_t> kt_pool;
  std::vector<int> kt_cls;
  size_t kt_used = 0;
  double kt_ms[K_COUNT] = {0};
  double kt_n[K_COUNT] = {0};  // launches timed per class

  int dalloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (dry) {
      dev_bytes += bytes;
      return SIM_OK;
    }
    if (al_fn) {
      *p = al_fn(bytes, al_ctx);
      if (!*p) return set_err(SIM_ENOMEM, "allocator hook returned NULL for %zu bytes", bytes);
      owned[*p] = Owner{al_free, al_ctx, bytes};
      dev_bytes += bytes;
      return SIM_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return set_err(SIM_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    owned[*p] = Owner{nullptr, nullptr, bytes};
    dev_bytes += bytes;
    return SIM_OK;
  }
  void dfree(void *p) {
    if (!p) return;
    auto it = owned.find(p);
    if (it == owned.end()) return;
    if (it->second.free_fn)
      it->second.free_fn(p, it->second.ctx);
    else
      hipFree(p);
    dev_bytes -= it->second.bytes;
    owned.erase(it);
  }

  // per-kernel-class event timing (off unless requested)
  void kt_flush() {
    if (!kt_used) return;
    hipStreamSynchronize(stream);
    for (size_t i = 0; i + 1 < kt_used; i += 2) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, kt_pool[i], kt_pool[i + 1]) == hipSuccess) {
        kt_ms[kt_cls[i / 2]] += ms;
        kt_n[kt_cls[i / 2]] += 1;
      }
    }
    kt_used = 0;
  }
  // the next launch records its own start and end (kernel time only)
  void kt_begin(int cls) {
    if (!kt_on) return;
    if (kt_used + 2 > kt_pool.size()) kt_flush();
    kt_cls[kt_used / 2] = cls;
    launch_timer().start = kt_pool[kt_used++];
    launch_timer().stop = kt_pool[kt_used++];
  }
  void kt_end() {
    if (!kt_on) return;
    launch_timer() = LaunchTimer{};
  }
};

namespace {

int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(SIM_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
  return SIM_OK;
}

int alloc_meta(sim_t *s, StateMeta &m) {
  int rc;
  if ((rc = s->dalloc((void **)&m.rec_off, 8 * s->nslices))) return rc;
  if ((rc = s->dalloc((void **)&m.rec_len, 4 * s->nslices))) return rc;
  if ((rc = s->dalloc((void **)&m.step, 8 * s->nslices))) return rc;
  if ((rc = s->dalloc((void **)&m.sq, 16 * s->nslices))) return rc;
  if ((rc = s->dalloc((void **)&m.dtab, 4ull * (1u << kLMax) * s->nslices))) return rc;
  return SIM_OK;
}

int alloc_slots(sim_t *s) {
  const uint64_t W = (uint64_t)s->W, L2 = 2 * s->geo.L;
  Slots &sl = s->slots;
  int rc;
  if ((rc = s->dalloc((void **)&sl.ws, 8 * W * L2))) return rc;
  if ((rc = s->dalloc((void **)&sl.sym, 2 * W * L2))) return rc;
  if ((rc = s->dalloc((void **)&sl.esc, 8 * W * L2))) return rc;
  if ((rc = s->dalloc((void **)&sl.codes, 4 * W * kNSym))) return rc;
  if ((rc = s->dalloc((void **)&sl.symtab, 2 * W * kNSym))) return rc;
  if ((rc = s->dalloc((void **)&sl.nused, 4 * W))) return rc;
  if ((rc = s->dalloc((void **)&sl.chunk_words, 4 * W * s->geo.nchunks))) return rc;
  if ((rc = s->dalloc((void **)&sl.words, 4 * W))) return rc;
  if ((rc = s->dalloc((void **)&sl.blk_words, 4 * W * kMaxEncBlocks))) return rc;
  if ((rc = s->dalloc((void **)&sl.sq, 16 * W))) return rc;
  if ((rc = s->dalloc((void **)&sl.nesc, 4 * W))) return rc;
  if ((rc = s->dalloc((void **)&sl.minmax, 16 * W))) return rc;
  if ((rc = s->dalloc((void **)&sl.qstep, 24 * W))) return rc;
  if ((rc = s->dalloc((void **)&sl.part, 32ull * W * kGqParts))) return rc;
  if ((rc = s->dalloc((void **)&sl.hpart, 4ull * W * kGqParts * kNSym))) return rc;
  sl.stage_words = stage_words_for(s->geo.chunk_log2);
  if ((rc = s->dalloc((void **)&sl.stage, 4ull * W * s->geo.nchunks * sl.stage_words))) return rc;
  if ((rc = s->dalloc((void **)&sl.csum, 8ull * W * s->geo.nchunks))) return rc;
  if ((rc = s->dalloc((void **)&sl.run_start, 1ull * W * s->geo.nchunks))) return rc;
  if ((rc = s->dalloc((void **)&sl.run_tile, 8ull * W * s->geo.run_tiles))) return rc;
  if ((rc = s->dalloc((void **)&sl.blk_run, 4ull * W * kMaxEncBlocks))) return rc;
  if ((rc = s->dalloc((void **)&sl.run_src, 4ull * W * kMaxRuns))) return rc;
  if ((rc = s->dalloc((void **)&sl.run_woff, 4ull * W * (kMaxRuns + 1)))) return rc;
  if ((rc = s->dalloc((void **)&sl.nruns, 4 * W))) return rc;
  if ((rc = s->dalloc((void **)&sl.run_words, 4 * W))) return rc;
  return SIM_OK;
}

// The fields of a W-slot workspace laid out from `base` (each 256-byte
// aligned), with the sizes alloc_slots gives them; base == nullptr only
// measures.  Returns the bytes used.
uint64_t carve_slots(const Geo &g, uint64_t W, uint8_t *base, Slots *sl) {
  const uint64_t L2 = 2 * g.L;
  uint64_t off = 0;
  auto take = [&](auto **ptr, uint64_t bytes) {
    using T = std::remove_reference_t<decltype(**ptr)>;
    *ptr = base ? (T *)(base + off) : nullptr;
    off = align_up(off + bytes, 256);
  };
  Slots t{};
  Slots &o = sl ? *sl : t;
  take(&o.ws, 8 * W * L2);
  take(&o.sym, 2 * W * L2);
  take(&o.esc, 8 * W * L2);
  take(&o.codes, 4 * W * kNSym);
  take(&o.symtab, 2 * W * kNSym);
  take(&o.nused, 4 * W);
  take(&o.chunk_words, 4 * W * g.nchunks);
  take(&o.words, 4 * W);
  take(&o.blk_words, 4 * W * kMaxEncBlocks);
  take(&o.sq, 16 * W);
  take(&o.nesc, 4 * W);
  take(&o.minmax, 16 * W);
  take(&o.qstep, 24 * W);
  take(&o.part, 32ull * W * kGqParts);
  take(&o.hpart, 4ull * W * kGqParts * kNSym);
  o.stage_words = stage_words_for(g.chunk_log2);
  take(&o.stage, 4ull * W * g.nchunks * o.stage_words);
  take(&o.csum, 8ull * W * g.nchunks);
  take(&o.run_start, 1ull * W * g.nchunks);
  take(&o.run_tile, 8ull * W * g.run_tiles);
  take(&o.blk_run, 4ull * W * kMaxEncBlocks);
  take(&o.run_src, 4ull * W * kMaxRuns);
  take(&o.run_woff, 4ull * W * (kMaxRuns + 1));
  take(&o.nruns, 4 * W);
  take(&o.run_words, 4 * W);
  return off;
}

uint64_t per_slot_bytes(const Geo &g) {
  return 2 * g.L * (8 + 2 + 8) + (uint64_t)kNSym * (4 + 2) + 4ull * kGqParts * (kNSym + 8) + 12ull * g.nchunks +
         4ull * g.nchunks * stage_words_for(g.chunk_log2) + 4ull * kMaxEncBlocks + 8ull * kMaxRuns + 140 +
         g.nchunks + 8ull * g.run_tiles + 4ull * kMaxEncBlocks;
}

// Slot order of every slice for gates whose slice-index targets form `gm`:
// groups (slices equal outside gm) are contiguous, members ordered by the
// bits of gm in ascending order.
int slot_table(sim_t *s, uint64_t gm, const uint64_t **out) {
  if (s->wtables) {  // the scratch workspace: every table was placed before the passes
    auto it = s->wtables->find(gm);
    if (it == s->wtables->end()) return set_err(SIM_EINVAL, "no slot order for group mask 0x%llx", (unsigned long long)gm);
    *out = it->second;
    return SIM_OK;
  }
  auto it = s->tables.find(gm);
  if (it != s->tables.end()) {
    *out = it->second;
    return SIM_OK;
  }
  std::vector<int> bits;
  for (int b = 0; b < 64; b++)
    if ((gm >> b) & 1) bits.push_back(b);
  std::vector<uint64_t> h;
  h.reserve(s->nslices);
  for (uint64_t j0 = 0; j0 < s->nslices; j0++) {
    if (j0 & gm) continue;
    for (uint64_t r = 0; r < (1ull << bits.size()); r++) {
      uint64_t j = j0;
      for (size_t b = 0; b < bits.size(); b++)
        if ((r >> b) & 1) j |= 1ull << bits[b];
      h.push_back(j);
    }
  }
  uint64_t *d;
  int rc = s->dalloc((void **)&d, 8 * s->nslices);
  if (rc) return rc;
  HIP_TRY(hipMemcpy(d, h.data(), 8 * s->nslices, hipMemcpyHostToDevice));
  s->tables[gm] = d;
  *out = d;
  return SIM_OK;
}

// ------------------------------------------------------------- fused passes
// Qubits a gate acts on or depends on: targets and control bits (a phase
// gate: its control bits).
uint64_t gate_qubits(const sim_gate &g) {
  uint64_t q = g.ctrl_mask;
  if (g.kind == SIM_GATE_DENSE)
    for (uint32_t k = 0; k < g.n_targets && k < 5; k++) q |= 1ull << g.targets[k];
  return q;
}

struct PlanPass {
  uint32_t first, count;
  bool fused;
  int k;          // block width (fused)
  int qubits[5];  // ascending (fused)
};

// Greedy partition of a gate list into passes (the rule sim_plan documents).
void plan_gates(const sim_gate *gates, size_t n, std::vector<PlanPass> &out) {
  out.clear();
  size_t i = 0;
  while (i < n) {
    uint64_t q = gate_qubits(gates[i]);
    size_t j = i + 1;
    if (__builtin_popcountll(q) <= SIM_FUSE_MAX) {
      while (j < n) {
        const uint64_t q2 = q | gate_qubits(gates[j]);
        if (__builtin_popcountll(q2) > SIM_FUSE_MAX) break;
        q = q2;
        j++;
      }
    }
    PlanPass p{};
    p.first = (uint32_t)i;
    p.count = (uint32_t)(j - i);
    p.fused = p.count >= 2;
    if (p.fused) {
      for (int b = 0; b < 64; b++)
        if ((q >> b) & 1) p.qubits[p.k++] = b;
    }
    out.push_back(p);
    i = j;
  }
}

// c += u * a in the order of the gate kernels
inline void host_cmac(double ur, double ui, double ar, double ai, double &cr, double &ci) {
  double pr = ur * ar;
  double pi = ui * ai;
  double qr = ur * ai;
  double qi = ui * ar;
  cr = cr + (pr - pi);
  ci = ci + (qr + qi);
}

// U = G_last ... G_first of a fused pass, 2^k x 2^k complex, row-major,
// interleaved; local bit i of a block index is qubit p.qubits[i].
void block_matrix(const sim_gate *gates, const PlanPass &p, std::vector<double> &U) {
  const uint32_t dim = 1u << p.k;
  int loc[64];
  for (int b = 0; b < 64; b++) loc[b] = -1;
  for (int i = 0; i < p.k; i++) loc[p.qubits[i]] = i;
  U.assign(2ull * dim * dim, 0.0);
  for (uint32_t r = 0; r < dim; r++) U[2 * (r * dim + r)] = 1.0;
  std::vector<double> G(2ull * dim * dim), T(2ull * dim * dim);
  for (uint32_t gi = p.first; gi < p.first + p.count; gi++) {
    const sim_gate &g = gates[gi];
    std::fill(G.begin(), G.end(), 0.0);
    // control bits as a local mask and values
    uint32_t cmask = 0, cvals = 0;
    for (int b = 0; b < 64; b++)
      if ((g.ctrl_mask >> b) & 1) {
        cmask |= 1u << loc[b];
        if ((g.ctrl_vals >> b) & 1) cvals |= 1u << loc[b];
      }
    for (uint32_t c = 0; c < dim; c++) {
      const bool on = (c & cmask) == cvals;
      if (!on) {
        G[2 * (c * dim + c)] = 1.0;
        continue;
      }
      if (g.kind == SIM_GATE_PHASE) {
        G[2 * (c * dim + c)] = g.params[0];
        G[2 * (c * dim + c) + 1] = g.params[1];
        continue;
      }
      const uint32_t kg = g.n_targets, gd = 1u << kg;
      uint32_t tmask = 0, cm = 0;
      for (uint32_t t = 0; t < kg; t++) {
        const int lb = loc[g.targets[t]];
        tmask |= 1u << lb;
        cm |= ((c >> lb) & 1u) << t;
      }
      for (uint32_t rm = 0; rm < gd; rm++) {
        uint32_t r = c & ~tmask;
        for (uint32_t t = 0; t < kg; t++) r |= ((rm >> t) & 1u) << loc[g.targets[t]];
        G[2 * (r * dim + c)] = g.matrix[2 * (rm * gd + cm)];
        G[2 * (r * dim + c) + 1] = g.matrix[2 * (rm * gd + cm) + 1];
      }
    }
    for (uint32_t r = 0; r < dim; r++)
      for (uint32_t c = 0; c < dim; c++) {
        double cr = 0.0, ci = 0.0;
        for (uint32_t m = 0; m < dim; m++)
          host_cmac(G[2 * (r * dim + m)], G[2 * (r * dim + m) + 1], U[2 * (m * dim + c)], U[2 * (m * dim + c) + 1],
                    cr, ci);
        T[2 * (r * dim + c)] = cr;
        T[2 * (r * dim + c) + 1] = ci;
      }
    U.swap(T);
  }
}

// A named gate kind written as the DENSE or PHASE gate it stands for (host
// FP64 arithmetic; each U3 entry is one product of libm values, in the form
// the header gives).  mat receives up to 32 doubles (a 4 x 4 complex matrix)
// and must outlive `out`.  DENSE and PHASE pass through.
int expand_gate(const sim_gate &g, size_t idx, sim_gate &out, double *mat) {
  out = g;
  auto need = [&](uint32_t k) {
    return g.n_targets == k ? SIM_OK : set_err(SIM_EINVAL, "gate %zu: kind %u takes %u targets, not %u", idx, g.kind, k,
                                                g.n_targets);
  };
  auto phase_on = [&](uint64_t bits, double re, double im) {
    if (g.ctrl_mask & bits) return set_err(SIM_EINVAL, "gate %zu: controls overlap targets", idx);
    out.kind = SIM_GATE_PHASE;
    out.n_targets = 0;
    out.ctrl_mask = g.ctrl_mask | bits;
    out.ctrl_vals = g.ctrl_vals | bits;
    out.params[0] = re;
    out.params[1] = im;
    out.params[2] = 0.0;
    out.matrix = nullptr;
    return SIM_OK;
  };
  auto bit = [&](uint32_t k) { return g.targets[k] < 64 ? 1ull << g.targets[k] : 0ull; };
  auto dense = [&](uint32_t k, const double *m) {
    const size_t cnt = 2ull << (2 * k);
    std::copy(m, m + cnt, mat);
    out.kind = SIM_GATE_DENSE;
    out.n_targets = k;
    out.matrix = mat;
    return SIM_OK;
  };
  int rc;
  switch (g.kind) {
    case SIM_GATE_DENSE:
    case SIM_GATE_PHASE:
      return SIM_OK;
    case SIM_GATE_U1Q:
      if ((rc = need(1))) return rc;
      if (!g.matrix) return set_err(SIM_EINVAL, "gate %zu: no matrix", idx);
      return dense(1, g.matrix);
    case SIM_GATE_H: {
      if ((rc = need(1))) return rc;
      const double h = std::sqrt(0.5);
      const double m[8] = {h, 0.0, h, 0.0, h, 0.0, -h, 0.0};
      return dense(1, m);
    }
    case SIM_GATE_X: {
      if ((rc = need(1))) return rc;
      const double m[8] = {0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0};
      return dense(1, m);
    }
    case SIM_GATE_Z:
      if ((rc = need(1))) return rc;
      return phase_on(bit(0), -1.0, 0.0);
    case SIM_GATE_P:
      if ((rc = need(1))) return rc;
      return phase_on(bit(0), std::cos(g.params[0]), std::sin(g.params[0]));
    case SIM_GATE_CP:
      if ((rc = need(2))) return rc;
      if (g.targets[0] == g.targets[1]) return set_err(SIM_EINVAL, "gate %zu: repeated target", idx);
      return phase_on(bit(0) | bit(1), std::cos(g.params[0]), std::sin(g.params[0]));
    case SIM_GATE_CZ:
      if ((rc = need(2))) return rc;
      if (g.targets[0] == g.targets[1]) return set_err(SIM_EINVAL, "gate %zu: repeated target", idx);
      return phase_on(bit(0) | bit(1), -1.0, 0.0);
    case SIM_GATE_MCZ: {
      if (g.n_targets < 1 || g.n_targets > 5) return set_err(SIM_EINVAL, "gate %zu: MCZ on %u targets", idx, g.n_targets);
      uint64_t b = 0;
      for (uint32_t k = 0; k < g.n_targets; k++) {
        if (b & bit(k)) return set_err(SIM_EINVAL, "gate %zu: repeated target", idx);
        b |= bit(k);
      }
      return phase_on(b, -1.0, 0.0);
    }
    case SIM_GATE_SWAP: {
      if ((rc = need(2))) return rc;
      double m[32] = {0.0};
      m[2 * (0 * 4 + 0)] = m[2 * (1 * 4 + 2)] = m[2 * (2 * 4 + 1)] = m[2 * (3 * 4 + 3)] = 1.0;
      return dense(2, m);
    }
    case SIM_GATE_U3: {
      if ((rc = need(1))) return rc;
      const double th = g.params[0], ph = g.params[1], la = g.params[2];
      const double c = std::cos(th / 2), sn = std::sin(th / 2);
      const double m[8] = {c, 0.0, -std::cos(la) * sn, -std::sin(la) * sn,
                           std::cos(ph) * sn, std::sin(ph) * sn, std::cos(ph + la) * c, std::sin(ph + la) * c};
      return dense(1, m);
    }
    default:
      return set_err(SIM_EINVAL, "gate %zu: unknown kind %u", idx, g.kind);
  }
}

// The gates with every named kind expanded; stops at the first gate that
// cannot be expanded (its status is returned, *n_ok counts the gates before it).
int expand_gates(const sim_gate *gates, size_t n, std::vector<sim_gate> &out, std::vector<double> &mats,
                 size_t *n_ok) {
  out.assign(n, sim_gate{});
  mats.assign(32 * n, 0.0);  // never reallocated: gates point into it
  for (size_t i = 0; i < n; i++) {
    const int rc = expand_gate(gates[i], i, out[i], mats.data() + 32 * i);
    if (rc) {
      *n_ok = i;
      out.resize(i);
      return rc;
    }
  }
  *n_ok = n;
  return SIM_OK;
}

int validate_gate(const sim_t *s, const sim_gate &g, size_t idx) {
  const int n = s->geo.n;
  const uint64_t top = n >= 64 ? ~0ull : ((1ull << n) - 1);
  if (g.ctrl_mask & ~top) return set_err(SIM_EINVAL, "gate %zu: control mask beyond %d qubits", idx, n);
  if (g.ctrl_vals & ~g.ctrl_mask) return set_err(SIM_EINVAL, "gate %zu: control values outside the mask", idx);
  if (g.kind == SIM_GATE_PHASE) return SIM_OK;
  if (g.kind != SIM_GATE_DENSE) return set_err(SIM_EINVAL, "gate %zu: unknown kind %u", idx, g.kind);
  if (g.n_targets < 1 || g.n_targets > 5) return set_err(SIM_EINVAL, "gate %zu: %u targets", idx, g.n_targets);
  if (!g.matrix) return set_err(SIM_EINVAL, "gate %zu: no matrix", idx);
  uint64_t tm = 0;
  int m = 0;
  for (uint32_t k = 0; k < g.n_targets; k++) {
    if ((int)g.targets[k] >= n) return set_err(SIM_EINVAL, "gate %zu: target %u beyond %d qubits", idx, g.targets[k], n);
    if (tm & (1ull << g.targets[k])) return set_err(SIM_EINVAL, "gate %zu: repeated target", idx);
    tm |= 1ull << g.targets[k];
    if ((int)g.targets[k] >= s->geo.slice_log2) m++;
  }
  if (tm & g.ctrl_mask) return set_err(SIM_EINVAL, "gate %zu: controls overlap targets", idx);
  if ((1 << m) > s->W) return set_err(SIM_ENOMEM, "gate %zu: group of %d slices exceeds the workspace", idx, 1 << m);
  return SIM_OK;
}

GateDesc make_desc(const sim_t *s, const sim_gate &g, const double *dmat, uint64_t *gm_out) {
  GateDesc d;
  memset(&d, 0, sizeof(d));
  d.ctrl_mask = g.ctrl_mask;
  d.ctrl_vals = g.ctrl_vals;
  *gm_out = 0;
  if (g.kind == SIM_GATE_PHASE) {
    d.kind = 2;
    d.ph_re = s->fp32 ? (double)(float)g.params[0] : g.params[0];
    d.ph_im = s->fp32 ? (double)(float)g.params[1] : g.params[1];
    return d;
  }
  const int sl2 = s->geo.slice_log2;
  d.kind = 1;
  d.k = (int)g.n_targets;
  uint64_t gm = 0;
  for (int k = 0; k < d.k; k++)
    if ((int)g.targets[k] >= sl2) gm |= 1ull << (g.targets[k] - sl2);
  for (int k = 0; k < d.k; k++) {
    int t = (int)g.targets[k];
    if (t < sl2) {
      d.tloc[k] = t;
    } else {
      int rank = __builtin_popcountll(gm & ((1ull << (t - sl2)) - 1));
      d.tloc[k] = sl2 + rank;
    }
    d.tmask_loc |= 1ull << d.tloc[k];
  }
  d.m = __builtin_popcountll(gm);
  if (d.k == 1)
    for (int i = 0; i < 8; i++) d.m2[i] = g.matrix[i];
  for (int c = 0; c < (1 << d.k); c++) {
    uint64_t off = 0;
    for (int k = 0; k < d.k; k++)
      if ((c >> k) & 1) off |= 1ull << d.tloc[k];
    d.dep[c] = off;
  }
  d.mat = dmat;
  *gm_out = gm;
  return d;
}

QuantParams quant_params(const sim_t *s) {
  QuantParams q;
  q.rel = (s->mode & SIM_EB_REL) ? 1 : 0;
  q.pw = s->geo.pw_bits >= 0 ? 1 : 0;
  q.pw_bits = s->geo.pw_bits;
  q.eb = s->eb;
  double step = (2.0 * s->eb) * (1.0 - 0x1p-20);
  q.step = step;
  q.recip = 1.0 / step;
  return q;
}

// Enqueue one pass.  init_kind >= 0: build that initial state instead of
// decompressing (no normalisation, identity gate).
// SIM_OPT decisions of one pass: a SWAP of slice-index bits sa and sb (a
// relabelling), or controls on slice-index bits (smask, svals in slice-index
// bits) that leave the other groups untouched; neither: an ordinary pass.
struct PassOpt {
  int sa = -1, sb = -1;
  uint64_t smask = 0, svals = 0;
};

// SIM_OPT lists of a pass (built on the host and copied to the device once,
// before any graph capture that uses them).
int opt_lists(sim_t *s, uint64_t gm, const PassOpt &po, const sim_t::OptLists **out) {
  const std::array<uint64_t, 3> key = po.sa >= 0 ? std::array<uint64_t, 3>{~0ull, (uint64_t)po.sa, (uint64_t)po.sb}
                                                 : std::array<uint64_t, 3>{gm, po.smask, po.svals};
  auto it = s->opt_lists.find(key);
  if (it != s->opt_lists.end()) {
    *out = &it->second;
    return SIM_OK;
  }
  if (s->no_alloc) return set_err(SIM_EINVAL, "SIM_OPT passes are not available without allocation");
  int rc;
  if (!s->carry_off && (rc = s->dalloc((void **)&s->carry_off, 8 * s->nslices))) return rc;
  std::vector<uint64_t> act, src, dst;
  if (po.sa >= 0) {  // relabel: slice j becomes the slice with index bits sa and sb exchanged
    for (uint64_t j = 0; j < s->nslices; j++) {
      const uint64_t ba = (j >> po.sa) & 1, bb = (j >> po.sb) & 1;
      src.push_back(j);
      dst.push_back(ba == bb ? j : j ^ ((1ull << po.sa) | (1ull << po.sb)));
    }
  } else {  // whole groups (slot order of gm) whose index bits meet the controls; the rest carried
    const uint64_t *table;
    if ((rc = slot_table(s, gm, &table))) return rc;
    std::vector<uint64_t> order(s->nslices);
    HIP_TRY(hipMemcpy(order.data(), table, 8 * s->nslices, hipMemcpyDeviceToHost));
    for (uint64_t j : order) {
      if ((j & po.smask) == po.svals)
        act.push_back(j);
      else
        src.push_back(j);
    }
    dst = src;
  }
  sim_t::OptLists L;
  auto put = [&](const std::vector<uint64_t> &h, uint64_t **d) -> int {
    if (h.empty()) return SIM_OK;
    int r = s->dalloc((void **)d, 8 * h.size());
    if (r) return r;
    HIP_TRY(hipMemcpy(*d, h.data(), 8 * h.size(), hipMemcpyHostToDevice));
    return SIM_OK;
  };
  if ((rc = put(act, &L.active)) || (rc = put(src, &L.src)) || (rc = put(dst, &L.dst))) return rc;
  L.n_active = act.size();
  L.n_carry = src.size();
  *out = &(s->opt_lists[key] = L);
  return SIM_OK;
}

int enqueue_pass(sim_t *s, const GateDesc &gd, uint64_t gm, int init_kind, uint64_t x, const PassOpt *po = nullptr) {
  const int c = s->cur;
  const StateMeta &cur = s->meta[c];
  const StateMeta &nxt = s->meta[1 - c];
  const uint32_t pass = s->pass_counter++;
  hipStream_t st = s->stream;
  const QuantParams qp = quant_params(s);
  const uint64_t *table;
  int rc = slot_table(s, init_kind >= 0 ? 0 : gm, &table);
  if (rc) return rc;
  uint64_t count = s->nslices;  // slices the batches process
  const sim_t::OptLists *ol = nullptr;
  if (init_kind < 0 && po && (po->sa >= 0 || po->smask)) {
    if ((rc = opt_lists(s, gm, *po, &ol))) return rc;
    if (po->sa >= 0) {  // a relabelling SWAP: every record carried to its new slice, nothing decoded
      s->kt_begin(K_BEGIN);
      launch_begin_pass(st, s->ctl, cur, s->nslices, s->kscale, 0, s->geo.pw_bits >= 0);
      s->kt_end();
      launch_carry(st, s->ctl, cur, nxt, s->arena[c], s->arena[1 - c], s->arena_cap[1 - c], ol->src, ol->dst,
                   ol->n_carry, s->carry_off, pass);
      s->cur = 1 - c;
      return check_launch("relabel");
    }
    table = ol->active;
    count = ol->n_active;
  }
  s->kt_begin(K_BEGIN);
  launch_begin_pass(st, s->ctl, cur, s->nslices, s->kscale, init_kind >= 0 ? 0 : 1, s->geo.pw_bits >= 0);
  s->kt_end();
  if (ol && ol->n_carry)  // groups where the gate is the identity keep their records
    launch_carry(st, s->ctl, cur, nxt, s->arena[c], s->arena[1 - c], s->arena_cap[1 - c], ol->src, ol->dst,
                 ol->n_carry, s->carry_off, pass);
  const GateDesc &gq = gd.kind == 4 ? s->ident : gd;
  // compact workspace (int32 codes) when decode feeds the quantising kernel
  // directly and that kernel reads it; the device still falls back to FP64
  // for a pass whose codes may not fit
  const bool compact = init_kind < 0 && !qp.rel && !qp.pw && gd.kind != 4 && AMP(s, gq_compact)(s->geo, gq);
  const Slots &slots = s->run_slots();
  const uint64_t W = (uint64_t)s->run_W();
  for (uint64_t b0 = 0; b0 < count; b0 += W) {
    const int ns = (int)std::min<uint64_t>(W, count - b0);
    const uint64_t *ss = table + b0;
    if (init_kind >= 0) {
      s->kt_begin(K_INIT);
      AMP(s, launch_init)(st, slots, s->geo, ss, ns, init_kind, x, s->dfactors, s->ctl);
      s->kt_end();
    } else {
      s->kt_begin(K_DECODE);
      AMP(s, launch_decode)(st, slots, s->geo, ss, ns, s->arena[c], cur, s->kscale, s->ctl, pass, compact);
      s->kt_end();
    }
    // fused block on matrix cores, in place; then quantised as the identity.
    // With the relative bound the block kernel can take the min/max itself.
    const bool mm_fused = gd.kind == 4 && qp.rel && AMP(s, dense_minmax_ok)(s->geo, gd);
    if (gd.kind == 4) {
      s->kt_begin(K_DENSE);
      AMP(s, launch_dense_mfma)(st, slots, s->geo, ns, gd, s->ctl, mm_fused);
      s->kt_end();
    }
    if (qp.rel && !mm_fused) {
      s->kt_begin(K_MINMAX);
      AMP(s, launch_gate_minmax)(st, slots, s->geo, ss, ns, gd.kind == 4 ? s->ident : gd, s->ctl);
      s->kt_end();
    }
    if (qp.rel) {
      s->kt_begin(K_RELSTEP);
      launch_rel_step(st, slots, ns, qp.eb, s->ctl);
      s->kt_end();
    }
    s->kt_begin(K_GATEQ);
    const uint32_t nparts = AMP(s, launch_gate_quant)(st, slots, s->geo, ss, ns, gq, qp, s->ctl, pass, compact, s->kscale);
    s->kt_end();
    s->kt_begin(K_CODEBOOK);
    launch_codebook(st, slots, ss, ns, nxt, nparts, s->ctl, qp.pw ? s->geo.nchunks : 0u);
    s->kt_end();
    s->kt_begin(K_ENCODE);
    launch_encode(st, slots, s->geo, ns, s->ctl);
    s->kt_end();
    if (s->geo.chunk_runs) {
      s->kt_begin(K_RUNS);
      launch_runs(st, slots, s->geo, ns, s->ctl);
      s->kt_end();
    }
    s->kt_begin(K_FINISH);
    launch_finish(st, slots, s->geo, ss, ns, qp, s->arena[1 - c], s->arena_cap[1 - c], nxt, s->ctl, pass);
    s->kt_end();
  }
  s->cur = 1 - c;
  return check_launch("pass");
}

int read_ctl(sim_t *s) {
  HIP_TRY(hipMemcpyAsync(s->h_ctl, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return SIM_OK;
}

// After a failure the per-slot accumulators may hold partial sums: clear
// them together with the flags.
int clear_flags(sim_t *s) {
  s->h_ctl->flags = 0;
  s->h_ctl->fail_pass = 0;
  s->h_ctl->pending_bump = 0;  // a failed batch's records are not counted
  s->h_ctl->pending_bytes = 0;
  s->h_ctl->wide = 1;  // the failed pass may have changed the flag: the replay decodes to FP64
  s->h_ctl->wide_next = 1;
  HIP_TRY(hipMemcpyAsync(&s->ctl->flags, &s->h_ctl->flags, 8, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(&s->ctl->pending_bump, &s->h_ctl->pending_bump, 16, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(&s->ctl->wide, &s->h_ctl->wide, 8, hipMemcpyHostToDevice, s->stream));
  launch_reset_slots(s->stream, s->run_slots(), s->run_W());
  HIP_TRY(hipStreamSynchronize(s->stream));
  return check_launch("reset_slots");
}

uint64_t min_record_total(const sim_t *s);

// Replace arena `which` (its contents are dead: the output of the next pass)
// by one of at least max(2 x its capacity, min_cap, the smallest possible
// state) bytes.  The old block is freed first, so that the peak stays low;
// when the larger one cannot be had, the old capacity is requested again
// and SIM_ENOMEM returned.  An arena that cannot be restored either is left
// empty (capacity 0), and ensure_arenas refuses the next pass.
int grow_arena(sim_t *s, int which, uint64_t min_cap) {
  const uint64_t old = s->arena_cap[which];
  const uint64_t cap = std::max<uint64_t>(std::max<uint64_t>(2 * old, min_cap), 4 * min_record_total(s));
  s->dfree(s->arena[which]);
  s->arena[which] = nullptr;
  s->arena_cap[which] = 0;
  int rc = s->dalloc((void **)&s->arena[which], cap);
  if (rc == SIM_OK) {
    s->arena_cap[which] = cap;
    return SIM_OK;
  }
  const std::string why = g_last_error;
  if (old && s->dalloc((void **)&s->arena[which], old) == SIM_OK) s->arena_cap[which] = old;
  return set_err(SIM_ENOMEM, "record arena could not grow to %llu bytes: %s", (unsigned long long)cap, why.c_str());
}

// Both arenas must exist before passes are enqueued (a failed growth may
// have left one empty): allocate a missing one at the initial size.
int ensure_arenas(sim_t *s) {
  for (int a = 0; a < 2; a++)
    if (!s->arena[a]) {
      if (s->no_alloc) return set_err(SIM_ENOMEM, "a record arena is missing (an earlier growth failed)");
      int rc = grow_arena(s, a, std::max<uint64_t>(s->arena_cap[1 - a], 16ull << 20));
      if (rc) return rc;
    }
  return SIM_OK;
}

// Run gates (or an init pass when gates == nullptr) with failure handling.
int run_passes(sim_t *s, const GateDesc *descs, const uint64_t *gms, size_t n, int init_kind, uint64_t x,
               size_t *applied_out, const PassOpt *opts = nullptr) {
  size_t applied = 0;
  int rc = SIM_OK;
  size_t total = descs ? n : 1;
  if (applied_out) *applied_out = 0;
  if ((rc = ensure_arenas(s))) return rc;
  for (int attempt = 0; applied < total; attempt++) {
    if (attempt == 64) {
      rc = set_err(SIM_ENOMEM, "a pass overflowed its record arena 64 times in a row");
      break;
    }
    const uint32_t start_pass = s->pass_counter;
    const int cur_start = s->cur;
    for (size_t i = applied; i < total; i++) {
      if (descs)
        rc = enqueue_pass(s, descs[i], gms[i], -1, 0, opts ? opts + i : nullptr);
      else
        rc = enqueue_pass(s, GateDesc{}, 0, init_kind, x, nullptr);
      if (rc) return rc;
    }
    // count the records of the last batch (settle only)
    launch_begin_pass(s->stream, s->ctl, s->meta[s->cur], s->nslices, s->kscale, 3, s->geo.pw_bits >= 0);
    if ((rc = read_ctl(s))) return rc;
    const uint32_t flags = s->h_ctl->flags;
    if (!flags) {
      applied = total;
      // the next pass writes the other arena: give it a quarter above the
      // stored state's size now, since an overflow inside a later batch
      // costs a device synchronisation, a reallocation and a replay.  This
      // growth is optional: when it fails the arena keeps its size, and an
      // overflow later grows it then (or reports SIM_ENOMEM)
      const int tgt = 1 - s->cur;
      const uint64_t want = s->h_ctl->bump + s->h_ctl->bump / 4;
      if (want > s->arena_cap[tgt] && !s->no_alloc) (void)grow_arena(s, tgt, want);
      break;
    }
    const uint32_t done = s->h_ctl->fail_pass - start_pass;  // passes that completed
    s->cur = cur_start ^ (int)(done & 1);
    s->pass_counter = start_pass + done;
    applied += done;
    if ((rc = clear_flags(s))) break;
    if (flags & kFlagOverflow) {
      if (s->no_alloc) {
        rc = set_err(SIM_ENOMEM, "a pass needs more than the %llu bytes of its record arena, which the "
                     "allocation-free entry point cannot grow", (unsigned long long)s->arena_cap[1 - s->cur]);
        break;
      }
      if ((rc = grow_arena(s, 1 - s->cur, 0))) break;
      continue;
    }
    if (flags & kFlagCorrupt) {
      rc = set_err(SIM_ECORRUPT, "a stored slice record failed its consistency checks");
    } else {
      rc = set_err(SIM_EBOUND, "a value could not be coded within the error bound (|p| >= 2^48 or bound check)");
    }
    break;
  }
  if (applied_out) *applied_out = applied;
  return rc;
}

uint64_t min_record_total(const sim_t *s) {
  return s->nslices * align_up(rec_bytes_host(1, s->geo.nchunks, 0), kRecAlign);
}

}  // namespace

// =================================================================== C ABI

extern "C" {

const char *sim_last_error(void) { return g_last_error.c_str(); }

int sim_create(int n_qubits, int slice_log2, double error_bound, uint32_t mode, sim_t **out) {
  sim_config c;
  memset(&c, 0, sizeof(c));
  c.n_qubits = n_qubits;
  c.slice_log2 = slice_log2;
  c.error_bound = error_bound;
  c.mode = mode;
  return sim_create_ex(&c, out);
}

}  // extern "C"

namespace {

// Geometry, workspace slots and arena capacity of a configuration; shared by
// sim_create_ex and sim_footprint.
int configure(const sim_config *cfg, sim_t *s, uint64_t *arena_cap) {
  const int n = cfg->n_qubits, sl2 = cfg->slice_log2;
  if (n < 1 || n > 40) return set_err(SIM_EINVAL, "n_qubits %d outside 1..40", n);
  if (sl2 < 1 || sl2 > n || sl2 > 26) return set_err(SIM_EINVAL, "slice_log2 %d outside 1..min(26, n)", sl2);
  if (!(cfg->error_bound > 0.0) || !std::isfinite(cfg->error_bound))
    return set_err(SIM_EINVAL, "error bound must be positive and finite");
  if (cfg->mode & ~(SIM_EB_REL | SIM_FP32 | SIM_FUSED | SIM_ZERO_CHUNKS | SIM_CONST_CHUNKS | SIM_EB_PWREL |
                    SIM_CHUNK_RUNS | SIM_OPT))
    return set_err(SIM_EINVAL, "unsupported mode bits 0x%x", cfg->mode);
  if ((cfg->mode & SIM_OPT) && (cfg->mode & SIM_FUSED))
    return set_err(SIM_EINVAL, "SIM_OPT is a plain-mode option (not with SIM_FUSED)");
  if ((cfg->mode & SIM_EB_REL) && (cfg->mode & SIM_EB_PWREL))
    return set_err(SIM_EINVAL, "SIM_EB_REL and SIM_EB_PWREL exclude each other");
  int pwb = -1;
  if (cfg->mode & SIM_EB_PWREL) {  // the least b with 2^-(b+1) <= eb, at most 20
    if (!(cfg->error_bound < 0.5)) return set_err(SIM_EINVAL, "a pointwise-relative bound must be below 0.5");
    pwb = 0;
    while (pwb <= 20 && std::ldexp(1.0, -(pwb + 1)) > cfg->error_bound) pwb++;
    if (pwb > 20) return set_err(SIM_EINVAL, "a pointwise-relative bound below 2^-21 needs more than 20 mantissa bits");
  }
  int cl2 = cfg->chunk_log2 > 0 ? cfg->chunk_log2 : 10;
  if (cl2 > sl2) cl2 = sl2;
  if (cl2 > 10) return set_err(SIM_EINVAL, "chunk_log2 %d above 10", cl2);
  s->geo.n = n;
  s->geo.slice_log2 = sl2;
  s->geo.chunk_log2 = cl2;
  s->geo.L = 1ull << sl2;
  s->geo.nchunks = (uint32_t)((2ull << sl2) >> cl2);
  s->geo.zero_chunks = (cfg->mode & SIM_ZERO_CHUNKS) ? 1u : 0u;
  s->geo.const_chunks = (cfg->mode & SIM_CONST_CHUNKS) ? 1u : 0u;
  s->geo.fmt_in = s->geo.zero_chunks | (s->geo.const_chunks << 1);
  s->geo.pw_bits = pwb;
  s->geo.chunk_runs = (cfg->mode & SIM_CHUNK_RUNS) ? 1u : 0u;
  s->geo.run_tiles = (s->geo.nchunks + kRunTile - 1) / kRunTile;
  s->eb = cfg->error_bound;
  s->mode = cfg->mode;
  s->fp32 = (cfg->mode & SIM_FP32) != 0;
  s->nslices = 1ull << (n - sl2);
  // workspace: a power of two number of slots within the budget; the default
  // budget always holds one full 32-slice group (a dense gate on five
  // slice-index qubits); an explicit budget is honoured and gates whose group
  // does not fit are refused with SIM_ENOMEM
  const uint64_t budget = cfg->workspace_bytes ? cfg->workspace_bytes : (16ull << 30);
  uint64_t W = 1;
  while (W * 2 <= s->nslices && W * 2 * per_slot_bytes(s->geo) <= budget) W *= 2;
  if (!cfg->workspace_bytes) W = std::max<uint64_t>(W, std::min<uint64_t>(s->nslices, 32));
  s->W = (int)W;
  *arena_cap = cfg->arena_bytes ? std::max<uint64_t>(cfg->arena_bytes, 4096)
                                : std::max<uint64_t>(4 * min_record_total(s), 16ull << 20);
  return SIM_OK;
}

// Every device buffer of a new handle (in dry mode: only their sizes).
int alloc_state(sim_t *s, uint64_t cap) {
  int rc;
  if ((rc = s->dalloc((void **)&s->ctl, sizeof(Ctl))) || (rc = alloc_meta(s, s->meta[0])) ||
      (rc = alloc_meta(s, s->meta[1])) || (rc = s->dalloc((void **)&s->kscale, 8 * s->nslices)) ||
      (rc = alloc_slots(s)) || (rc = s->dalloc((void **)&s->dfactors, 32 * (size_t)s->geo.n)))
    return rc;
  for (int a = 0; a < 2; a++) {
    if ((rc = s->dalloc((void **)&s->arena[a], cap))) return rc;
    s->arena_cap[a] = cap;
  }
  return SIM_OK;
}

}  // namespace

extern "C" {

int sim_footprint(const sim_config *cfg, uint64_t *bytes) {
  if (!cfg || !bytes) return set_err(SIM_EINVAL, "null argument");
  *bytes = 0;
  sim_t s;
  s.dry = true;
  uint64_t cap = 0;
  int rc = configure(cfg, &s, &cap);
  if (rc) return rc;
  alloc_state(&s, cap);
  // plus the slot order of slice-local gates, made by the pass that builds
  // the initial state
  *bytes = s.dev_bytes + 8 * s.nslices;
  return SIM_OK;
}

int sim_create_ex(const sim_config *cfg, sim_t **out) {
  if (!cfg || !out) return set_err(SIM_EINVAL, "null argument");
  *out = nullptr;
  {
    sim_t probe;
    uint64_t cap;
    int rc = configure(cfg, &probe, &cap);
    if (rc) return rc;
  }
  if ((cfg->alloc == nullptr) != (cfg->free_fn == nullptr)) return set_err(SIM_EINVAL, "allocator needs both functions");

  int ndev = 0;
  hipError_t de = hipGetDeviceCount(&ndev);
  if (de != hipSuccess || ndev < 1)
    return set_err(SIM_EDEVICE, "no HIP device (hipGetDeviceCount: %d %s, count %d)", (int)de, hipGetErrorString(de),
                   ndev);
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return set_err(SIM_EDEVICE, "no device properties");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_err(SIM_EDEVICE, "device %s is not gfx950", prop.gcnArchName);

  sim_t *s = new sim_t();
  uint64_t cap = 0;
  configure(cfg, s, &cap);
  s->al_fn = cfg->alloc;
  s->al_free = cfg->free_fn;
  s->al_ctx = cfg->alloc_ctx;
  if (cfg->stream) {
    s->stream = (hipStream_t)cfg->stream;
    s->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return set_err(SIM_EDEVICE, "stream creation failed");
    }
    s->own_stream = true;
  }
  hipEventCreate(&s->ev0);
  hipEventCreate(&s->ev1);
  int rc;
  if ((rc = alloc_state(s, cap))) {
    sim_destroy(s);
    return rc;
  }
  if (hipHostMalloc((void **)&s->h_ctl, sizeof(Ctl), 0) != hipSuccess) {
    sim_destroy(s);
    return set_err(SIM_ENOMEM, "pinned host allocation failed");
  }
  memset(s->h_ctl, 0, sizeof(Ctl));
  s->h_ctl->wide = s->h_ctl->wide_next = 1;
  if (hipMemcpy(s->ctl, s->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice) != hipSuccess) {
    sim_destroy(s);
    return set_err(SIM_EDEVICE, "control block upload failed");
  }
  launch_reset_slots(s->stream, s->slots, s->W);
  rc = run_passes(s, nullptr, nullptr, 0, 0, 0, nullptr);
  if (rc) {
    sim_destroy(s);
    return rc;
  }
  *out = s;
  return SIM_OK;
}

void sim_destroy(sim_t *s) {
  if (!s) return;
  if (s->stream) hipStreamSynchronize(s->stream);
  std::vector<void *> ptrs;
  for (auto &kv : s->owned) ptrs.push_back(kv.first);
  for (void *p : ptrs) s->dfree(p);
  if (s->h_ctl) hipHostFree(s->h_ctl);
  for (hipEvent_t e : s->kt_pool) hipEventDestroy(e);
  if (s->ev0) hipEventDestroy(s->ev0);
  if (s->ev1) hipEventDestroy(s->ev1);
  if (s->cap_stream) hipStreamDestroy(s->cap_stream);
  if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
  delete s;
}

int sim_set_allocator(sim_t *s, void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *), void *ctx) {
  if (!s) return set_err(SIM_EINVAL, "null handle");
  if ((alloc == nullptr) != (free_fn == nullptr)) return set_err(SIM_EINVAL, "allocator needs both functions");
  s->al_fn = alloc;
  s->al_free = free_fn;
  s->al_ctx = ctx;
  return SIM_OK;
}

int sim_set_stream(sim_t *s, void *hip_stream) {
  if (!s) return set_err(SIM_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (s->own_stream) hipStreamDestroy(s->stream);
  s->own_stream = false;
  s->stream = (hipStream_t)hip_stream;
  return SIM_OK;
}

int sim_init_basis(sim_t *s, uint64_t x) {
  if (!s) return set_err(SIM_EINVAL, "null handle");
  if (s->geo.n < 64 && x >= (1ull << s->geo.n)) return set_err(SIM_EINVAL, "basis index out of range");
  return run_passes(s, nullptr, nullptr, 0, 1, x, nullptr);
}

int sim_init_product(sim_t *s, const double *factors) {
  if (!s || !factors) return set_err(SIM_EINVAL, "null argument");
  std::vector<double> f(factors, factors + 4 * (size_t)s->geo.n);
  if (s->fp32)
    for (double &v : f) v = (double)(float)v;
  HIP_TRY(hipMemcpy(s->dfactors, f.data(), 32 * (size_t)s->geo.n, hipMemcpyHostToDevice));
  return run_passes(s, nullptr, nullptr, 0, 2, 0, nullptr);
}

// The passes of a gate program: the plan (one pass per gate, or the fused
// partition), the gate each pass applies and its host matrices (FP32-rounded
// in FP32 mode).  Gates from the first invalid one on are dropped (vrc, verr).
struct PassSet {
  std::vector<sim_gate> eg;  // the program with named kinds expanded
  std::vector<double> emat;  // matrices of expanded named kinds (eg points here)
  size_t n_valid = 0;
  int vrc = SIM_OK;
  std::string verr;
  std::vector<PlanPass> plan;
  std::vector<double> hm;
  std::vector<size_t> moff;
  std::vector<sim_gate> pg;
  std::vector<int> kind4;
  std::vector<PassOpt> opts;  // SIM_OPT: per pass (empty otherwise)
  size_t n_pass = 0;
};

static void prepare_passes(sim_t *s, const sim_gate *gates_in, size_t n_in, PassSet &P) {
  size_t &n_valid = P.n_valid;
  int &vrc = P.vrc;
  size_t n = 0;
  vrc = expand_gates(gates_in, n_in, P.eg, P.emat, &n);
  const sim_gate *gates = P.eg.data();
  for (; n_valid < n; n_valid++) {
    const int rc = validate_gate(s, gates[n_valid], n_valid);
    if (rc) {
      vrc = rc;
      break;
    }
  }
  P.verr = vrc ? g_last_error : std::string();
  std::string &verr = P.verr;
  // passes: one per gate, or the fused partition of the valid gates
  std::vector<PlanPass> &plan = P.plan;
  if (s->mode & SIM_FUSED) {
    plan_gates(gates, n_valid, plan);
  } else {
    plan.resize(n_valid);
    for (size_t i = 0; i < n_valid; i++) plan[i] = PlanPass{(uint32_t)i, 1u, false, 0, {0, 0, 0, 0, 0}};
  }
  // host matrices of all passes, then one copy to the device
  std::vector<double> &hm = P.hm;
  std::vector<size_t> &moff = P.moff;
  std::vector<sim_gate> &pg = P.pg;  // the gate each pass applies
  std::vector<int> &kind4 = P.kind4;
  moff.assign(plan.size(), 0);
  pg.assign(plan.size(), sim_gate{});
  kind4.assign(plan.size(), 0);
  std::vector<double> U;
  size_t &n_pass = P.n_pass;
  n_pass = 0;
  for (; n_pass < plan.size(); n_pass++) {
    const PlanPass &p = plan[n_pass];
    if (!p.fused) {
      pg[n_pass] = gates[p.first];
      if (pg[n_pass].kind == SIM_GATE_DENSE) {
        const size_t cnt = 2ull << (2 * pg[n_pass].n_targets);
        moff[n_pass] = hm.size();
        hm.insert(hm.end(), pg[n_pass].matrix, pg[n_pass].matrix + cnt);
      }
      continue;
    }
    block_matrix(gates, p, U);
    sim_gate g{};
    if (p.k == 0) {  // global phases only
      g.kind = SIM_GATE_PHASE;
      g.params[0] = U[0];
      g.params[1] = U[1];
      pg[n_pass] = g;
      continue;
    }
    g.kind = SIM_GATE_DENSE;
    g.n_targets = (uint32_t)p.k;
    for (int i = 0; i < p.k; i++) g.targets[i] = (uint32_t)p.qubits[i];
    int m = 0;
    for (int i = 0; i < p.k; i++) m += p.qubits[i] >= s->geo.slice_log2;
    if ((1 << m) > s->W) {
      vrc = set_err(SIM_ENOMEM, "fused pass %zu: group of %d slices exceeds the workspace", n_pass, 1 << m);
      verr = g_last_error;
      break;
    }
    moff[n_pass] = hm.size();
    if (p.k <= 2) {  // narrow blocks run through the plain kernels
      hm.insert(hm.end(), U.begin(), U.end());
    } else {  // real embedding [[Ur, -Ui], [Ui, Ur]] for the matrix cores
      const uint32_t dim = 1u << p.k, D = 2 * dim;
      const size_t base = hm.size();
      hm.resize(base + (size_t)D * D);
      for (uint32_t r = 0; r < dim; r++)
        for (uint32_t c = 0; c < dim; c++) {
          const double ur = U[2 * (r * dim + c)], ui = U[2 * (r * dim + c) + 1];
          hm[base + (size_t)r * D + c] = ur;
          hm[base + (size_t)r * D + dim + c] = -ui;
          hm[base + (size_t)(dim + r) * D + c] = ui;
          hm[base + (size_t)(dim + r) * D + dim + c] = ur;
        }
      kind4[n_pass] = 1;
    }
    pg[n_pass] = g;
  }
  if (s->fp32)  // FP32 gate arithmetic takes FP32 matrix entries
    for (double &v : hm) v = (double)(float)v;
}

// Descriptors of the passes, their matrices at dev (a device copy of P.hm).
static void pass_descs(const sim_t *s, PassSet &P, double *dev, std::vector<GateDesc> &descs,
                       std::vector<uint64_t> &gms) {
  descs.resize(P.n_pass);
  gms.resize(P.n_pass);
  for (size_t i = 0; i < P.n_pass; i++) {
    const bool dense = P.pg[i].kind == SIM_GATE_DENSE;
    if (dense && !P.kind4[i]) P.pg[i].matrix = P.hm.data() + P.moff[i];  // host copy, read by make_desc
    descs[i] = make_desc(s, P.pg[i], dense ? dev + P.moff[i] : nullptr, &gms[i]);
    if (P.kind4[i]) descs[i].kind = 4;
  }
  P.opts.clear();
  if (!(s->mode & SIM_OPT)) return;
  P.opts.resize(P.n_pass);
  const int sl2 = s->geo.slice_log2;
  const uint64_t lo = (1ull << sl2) - 1;
  for (size_t i = 0; i < P.n_pass; i++) {
    const sim_gate &g = P.pg[i];
    PassOpt &o = P.opts[i];
    bool swap = g.kind == SIM_GATE_DENSE && g.n_targets == 2 && g.ctrl_mask == 0 && (int)g.targets[0] >= sl2 &&
                (int)g.targets[1] >= sl2;
    for (int r = 0; swap && r < 4; r++)  // exactly the exchange of the two targets
      for (int c = 0; c < 4; c++) {
        const bool one = (r == 0 && c == 0) || (r == 1 && c == 2) || (r == 2 && c == 1) || (r == 3 && c == 3);
        if (g.matrix[2 * (4 * r + c)] != (one ? 1.0 : 0.0) || g.matrix[2 * (4 * r + c) + 1] != 0.0) swap = false;
      }
    if (swap) {
      o.sa = (int)g.targets[0] - sl2;
      o.sb = (int)g.targets[1] - sl2;
    } else {
      o.smask = (g.ctrl_mask & ~lo) >> sl2;
      o.svals = (g.ctrl_vals & ~lo) >> sl2;
    }
  }
}

int sim_apply(sim_t *s, const sim_gate *gates, size_t n, size_t *n_applied) {
  if (n_applied) *n_applied = 0;
  if (!s) return set_err(SIM_EINVAL, "null handle");
  if (n && !gates) return set_err(SIM_EINVAL, "null gate array");
  PassSet P;
  prepare_passes(s, gates, n, P);
  std::vector<double> &hm = P.hm;
  std::vector<PlanPass> &plan = P.plan;
  const size_t n_pass = P.n_pass;
  int vrc = P.vrc;
  std::string verr = P.verr;
  if (hm.size() > s->dmat_cap) {
    s->dfree(s->dmat);
    s->dmat = nullptr;
    s->dmat_cap = 0;
    int rc = s->dalloc((void **)&s->dmat, 8 * hm.size());
    if (rc) return rc;
    s->dmat_cap = hm.size();
  }
  std::vector<GateDesc> descs;
  std::vector<uint64_t> gms;
  pass_descs(s, P, s->dmat, descs, gms);
  if (!hm.empty()) HIP_TRY(hipMemcpy(s->dmat, hm.data(), 8 * hm.size(), hipMemcpyHostToDevice));
  size_t applied = 0;
  HIP_TRY(hipEventRecord(s->ev0, s->stream));
  int rc = n_pass ? run_passes(s, descs.data(), gms.data(), n_pass, -1, 0, &applied,
                               P.opts.empty() ? nullptr : P.opts.data())
                  : SIM_OK;
  HIP_TRY(hipEventRecord(s->ev1, s->stream));
  HIP_TRY(hipEventSynchronize(s->ev1));
  float ms = 0;
  hipEventElapsedTime(&ms, s->ev0, s->ev1);
  s->elapsed += ms * 1e-3;
  s->passes += applied;
  if (s->kt_on) s->kt_flush();
  size_t gates_done = 0;
  for (size_t i = 0; i < applied; i++) gates_done += plan[i].count;
  s->gates += gates_done;
  if (n_applied) *n_applied = gates_done;
  if (rc) return rc;
  if (vrc) {
    g_last_error = verr;
    return vrc;
  }
  return SIM_OK;
}

// ------------------------------------------------------------ gate graphs

struct sim_graph_s {
  sim_t *sim = nullptr;
  PassSet P;                        // the program's passes and host matrices
  double *dmat = nullptr;           // device copy of the matrices (the handle's allocator)
  std::vector<GateDesc> descs;
  std::vector<uint64_t> gms;
  hipGraphExec_t exec = nullptr;    // the passes as captured
  int start_cur = 0;                // arena parity they start from
  uint32_t start_pass = 0;          // pass numbers [start_pass, start_pass + n) baked into the kernels
  uint8_t *arena[2] = {nullptr, nullptr};
  uint64_t cap[2] = {0, 0};
  uint32_t fmt_in = 0;              // the decoder variant captured (record formats it reads)
};

static bool graph_current(const sim_graph_t *G) {
  const sim_t *s = G->sim;
  return G->exec && s->cur == G->start_cur && s->arena[0] == G->arena[0] && s->arena[1] == G->arena[1] &&
         s->arena_cap[0] == G->cap[0] && s->arena_cap[1] == G->cap[1] && s->geo.fmt_in == G->fmt_in;
}

// Record the program's passes from the current arena parity.  Nothing runs:
// the state and parity are unchanged, the pass numbers are reserved.
static int graph_capture(sim_graph_t *G) {
  sim_t *s = G->sim;
  if (G->exec) {
    hipGraphExecDestroy(G->exec);
    G->exec = nullptr;
  }
  int rc;
  const PassOpt *opts = G->P.opts.empty() ? nullptr : G->P.opts.data();
  for (size_t i = 0; i < G->P.n_pass; i++) {  // slot tables exist before the capture (they copy to the device)
    const uint64_t *t;
    if ((rc = slot_table(s, G->gms[i], &t))) return rc;
    const sim_t::OptLists *ol;
    if (opts && (opts[i].sa >= 0 || opts[i].smask) && (rc = opt_lists(s, G->gms[i], opts[i], &ol))) return rc;
  }
  if (!s->cap_stream && hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return set_err(SIM_EDEVICE, "capture stream creation failed");
  const bool kt = s->kt_on;  // launches in a graph record no timing events
  s->kt_on = false;
  const int cur0 = s->cur;
  const uint32_t pc0 = s->pass_counter;
  hipStream_t saved = s->stream;
  s->stream = s->cap_stream;
  hipGraph_t graph = nullptr;
  rc = SIM_OK;
  hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    rc = set_err(SIM_EDEVICE, "graph capture could not start: %s", hipGetErrorString(e));
  } else {
    for (size_t i = 0; i < G->P.n_pass && rc == SIM_OK; i++)
      rc = enqueue_pass(s, G->descs[i], G->gms[i], -1, 0, opts ? opts + i : nullptr);
    e = hipStreamEndCapture(s->cap_stream, &graph);
    if (rc == SIM_OK && e != hipSuccess) rc = set_err(SIM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  }
  s->stream = saved;
  s->cur = cur0;
  s->pass_counter = pc0 + (uint32_t)G->P.n_pass;
  s->kt_on = kt;
  if (rc == SIM_OK && (e = hipGraphInstantiate(&G->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
    G->exec = nullptr;
    rc = set_err(SIM_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  if (graph) hipGraphDestroy(graph);
  (void)hipGetLastError();
  if (rc) return rc;
  G->start_cur = cur0;
  G->start_pass = pc0;
  for (int a = 0; a < 2; a++) {
    G->arena[a] = s->arena[a];
    G->cap[a] = s->arena_cap[a];
  }
  G->fmt_in = s->geo.fmt_in;
  return SIM_OK;
}

void sim_graph_destroy(sim_graph_t *G) {
  if (!G) return;
  if (G->exec) hipGraphExecDestroy(G->exec);
  if (G->dmat) G->sim->dfree(G->dmat);
  delete G;
}

int sim_tune_chunk(const sim_config *cfg, const sim_gate *gates, size_t n, int lo, int hi, int *best,
                   double *ms_per_gate, uint64_t *bytes) {
  if (!cfg || !best || (n && !gates)) return set_err(SIM_EINVAL, "null argument");
  if (n < 2) return set_err(SIM_EINVAL, "tuning needs at least two gates");
  if (lo < 1 || hi > 10 || lo > hi) return set_err(SIM_EINVAL, "chunk range %d..%d outside 1..10", lo, hi);
  *best = 0;
  double best_ms = 0.0;
  uint64_t best_bytes = 0;
  const size_t warm = n / 4 ? n / 4 : 1;  // first passes untimed (arena growth, first launches)
  for (int cl = lo; cl <= hi; cl++) {
    sim_config c = *cfg;
    c.chunk_log2 = cl;
    sim_t *s = nullptr;
    int rc = sim_create_ex(&c, &s);
    size_t done = 0;
    if (!rc) rc = sim_apply(s, gates, warm, &done);
    double t0 = s ? s->elapsed : 0.0;
    if (!rc) rc = sim_apply(s, gates + warm, n - warm, &done);
    sim_stats_t st;
    if (!rc) rc = sim_stats(s, &st);
    const double ms = rc ? 0.0 : (s->elapsed - t0) * 1e3 / (double)(n - warm);
    sim_destroy(s);
    if (rc) return rc;
    if (ms_per_gate) ms_per_gate[cl - lo] = ms;
    if (bytes) bytes[cl - lo] = st.compressed_bytes;
    if (*best == 0 || ms < best_ms || (ms == best_ms && st.compressed_bytes < best_bytes)) {
      *best = cl;
      best_ms = ms;
      best_bytes = st.compressed_bytes;
    }
  }
  return SIM_OK;
}

int sim_graph_create(sim_t *s, const sim_gate *gates, size_t n, sim_graph_t **out) {
  if (!out) return set_err(SIM_EINVAL, "null argument");
  *out = nullptr;
  if (!s) return set_err(SIM_EINVAL, "null handle");
  if (n && !gates) return set_err(SIM_EINVAL, "null gate array");
  sim_graph_t *G = new sim_graph_s();
  G->sim = s;
  prepare_passes(s, gates, n, G->P);
  int rc = G->P.vrc;
  if (rc) {
    g_last_error = G->P.verr;
    delete G;
    return rc;
  }
  if (!G->P.hm.empty()) {
    if ((rc = s->dalloc((void **)&G->dmat, 8 * G->P.hm.size()))) {
      delete G;
      return rc;
    }
  }
  pass_descs(s, G->P, G->dmat, G->descs, G->gms);
  if (!G->P.hm.empty() &&
      hipMemcpy(G->dmat, G->P.hm.data(), 8 * G->P.hm.size(), hipMemcpyHostToDevice) != hipSuccess) {
    sim_graph_destroy(G);
    return set_err(SIM_EDEVICE, "matrix upload failed");
  }
  if ((rc = graph_capture(G))) {
    sim_graph_destroy(G);
    return rc;
  }
  *out = G;
  return SIM_OK;
}

int sim_graph_launch(sim_t *s, sim_graph_t *G, size_t *n_applied) {
  if (n_applied) *n_applied = 0;
  if (!s || !G || G->sim != s) return set_err(SIM_EINVAL, "graph does not belong to this handle");
  const size_t n = G->P.n_pass;
  if (n == 0) return SIM_OK;
  size_t applied = 0;
  int rc = SIM_OK;
  if ((rc = ensure_arenas(s))) return rc;
  HIP_TRY(hipEventRecord(s->ev0, s->stream));
  if (s->cur != G->start_cur) {  // the other parity: ordinary launches of the same passes
    rc = run_passes(s, G->descs.data(), G->gms.data(), n, -1, 0, &applied,
                    G->P.opts.empty() ? nullptr : G->P.opts.data());
  } else {
    if (!graph_current(G)) rc = graph_capture(G);  // an arena has been reallocated since
    if (rc == SIM_OK) {
      HIP_TRY(hipGraphLaunch(G->exec, s->stream));
      // count the records of the last batch, then check the passes
      const int end_cur = G->start_cur ^ (int)(n & 1);
      launch_begin_pass(s->stream, s->ctl, s->meta[end_cur], s->nslices, s->kscale, 3, s->geo.pw_bits >= 0);
      if ((rc = read_ctl(s)) == SIM_OK) {
        const uint32_t flags = s->h_ctl->flags;
        if (!flags) {
          applied = n;
          s->cur = end_cur;
          const int tgt = 1 - s->cur;  // as after every batch: room for the next pass
          const uint64_t want = s->h_ctl->bump + s->h_ctl->bump / 4;
          if (want > s->arena_cap[tgt]) (void)grow_arena(s, tgt, want);
        } else {
          const uint32_t done = s->h_ctl->fail_pass - G->start_pass;  // passes that completed
          s->cur = G->start_cur ^ (int)(done & 1);
          applied = done;
          if ((rc = clear_flags(s)) == SIM_OK) {
            if (flags & kFlagOverflow) {  // the rest through ordinary launches, into a larger arena
              if ((rc = grow_arena(s, 1 - s->cur, 0)) == SIM_OK) {
                size_t more = 0;
                rc = run_passes(s, G->descs.data() + done, G->gms.data() + done, n - done, -1, 0, &more,
                                G->P.opts.empty() ? nullptr : G->P.opts.data() + done);
                applied += more;
              }
            } else if (flags & kFlagCorrupt) {
              rc = set_err(SIM_ECORRUPT, "a stored slice record failed its consistency checks");
            } else {
              rc = set_err(SIM_EBOUND, "a value could not be coded within the error bound (|p| >= 2^48 or bound check)");
            }
          }
        }
      }
    }
  }
  HIP_TRY(hipEventRecord(s->ev1, s->stream));
  HIP_TRY(hipEventSynchronize(s->ev1));
  float ms = 0;
  hipEventElapsedTime(&ms, s->ev0, s->ev1);
  s->elapsed += ms * 1e-3;
  s->passes += applied;
  if (s->kt_on) s->kt_flush();
  size_t gates_done = 0;
  for (size_t i = 0; i < applied; i++) gates_done += G->P.plan[i].count;
  s->gates += gates_done;
  if (n_applied) *n_applied = gates_done;
  return rc;
}

// validity of a gate for n qubits (no handle: no workspace limits)
static int check_gate_n(int n, const sim_gate &g, size_t idx) {
  const uint64_t top = n >= 64 ? ~0ull : ((1ull << n) - 1);
  if (g.ctrl_mask & ~top) return set_err(SIM_EINVAL, "gate %zu: control mask beyond %d qubits", idx, n);
  if (g.ctrl_vals & ~g.ctrl_mask) return set_err(SIM_EINVAL, "gate %zu: control values outside the mask", idx);
  if (g.kind == SIM_GATE_PHASE) return SIM_OK;
  if (g.kind != SIM_GATE_DENSE) return set_err(SIM_EINVAL, "gate %zu: unknown kind %u", idx, g.kind);
  if (g.n_targets < 1 || g.n_targets > 5) return set_err(SIM_EINVAL, "gate %zu: %u targets", idx, g.n_targets);
  if (!g.matrix) return set_err(SIM_EINVAL, "gate %zu: no matrix", idx);
  uint64_t tm = 0;
  for (uint32_t k = 0; k < g.n_targets; k++) {
    if ((int)g.targets[k] >= n) return set_err(SIM_EINVAL, "gate %zu: target %u beyond %d qubits", idx, g.targets[k], n);
    if (tm & (1ull << g.targets[k])) return set_err(SIM_EINVAL, "gate %zu: repeated target", idx);
    tm |= 1ull << g.targets[k];
  }
  if (tm & g.ctrl_mask) return set_err(SIM_EINVAL, "gate %zu: controls overlap targets", idx);
  return SIM_OK;
}

int sim_plan_qubits(int n_qubits, const sim_gate *gates_in, size_t n, sim_pass *out, size_t cap, size_t *n_pass) {
  if (n_pass) *n_pass = 0;
  if (n_qubits < 1 || n_qubits > 40) return set_err(SIM_EINVAL, "n_qubits %d out of range", n_qubits);
  if (n && !gates_in) return set_err(SIM_EINVAL, "null gate array");
  std::vector<sim_gate> eg;
  std::vector<double> emat;
  size_t n_ok = 0;
  int rc = expand_gates(gates_in, n, eg, emat, &n_ok);
  if (rc) return rc;
  const sim_gate *gates = eg.data();
  for (size_t i = 0; i < n; i++) {
    rc = check_gate_n(n_qubits, gates[i], i);
    if (rc) return rc;
  }
  std::vector<PlanPass> plan;
  plan_gates(gates, n, plan);
  if (n_pass) *n_pass = plan.size();
  if (!out) return SIM_OK;
  if (cap < plan.size()) return set_err(SIM_ENOMEM, "%zu passes do not fit %zu entries", plan.size(), cap);
  for (size_t i = 0; i < plan.size(); i++) {
    sim_pass &o = out[i];
    memset(&o, 0, sizeof(o));
    o.first_gate = plan[i].first;
    o.n_gates = plan[i].count;
    o.fused = plan[i].fused ? 1u : 0u;
    o.n_qubits = plan[i].fused ? (uint32_t)plan[i].k : 0u;
    for (int k = 0; k < plan[i].k; k++) o.qubits[k] = (uint32_t)plan[i].qubits[k];
  }
  return SIM_OK;
}

int sim_plan(const sim_t *s, const sim_gate *gates, size_t n, sim_pass *out, size_t cap, size_t *n_pass) {
  if (n_pass) *n_pass = 0;
  if (!s) return set_err(SIM_EINVAL, "null handle");
  return sim_plan_qubits(s->geo.n, gates, n, out, cap, n_pass);
}

static int readout(sim_t *s, uint64_t begin, uint64_t count, double *out, int probs) {
  if (!s || (!out && count)) return set_err(SIM_EINVAL, "null argument");
  const uint64_t N = 1ull << s->geo.n;
  if (begin > N || count > N - begin) return set_err(SIM_EINVAL, "amplitude range out of bounds");
  if (!count) return SIM_OK;
  int rc;
  const uint64_t *table;
  if ((rc = slot_table(s, 0, &table))) return rc;
  launch_begin_pass(s->stream, s->ctl, s->meta[s->cur], s->nslices, s->kscale, 2, s->geo.pw_bits >= 0);
  const uint64_t L = s->geo.L;
  const uint64_t per = probs ? 1 : 2;
  const uint64_t stage_amps = std::min<uint64_t>(count, std::max<uint64_t>(L, 1ull << 24));
  if (stage_amps * per > s->dstage_cap) {
    s->dfree(s->dstage);
    s->dstage = nullptr;
    s->dstage_cap = 0;
    if ((rc = s->dalloc((void **)&s->dstage, 8 * stage_amps * per))) return rc;
    s->dstage_cap = stage_amps * per;
  }
  uint64_t i = begin;
  const uint64_t end = begin + count;
  while (i < end) {
    const uint64_t j0 = i / L;
    const uint64_t j1 = std::min<uint64_t>((end + L - 1) / L, j0 + (uint64_t)s->W);
    const int ns = (int)(j1 - j0);
    AMP(s, launch_decode)(s->stream, s->slots, s->geo, table + j0, ns, s->arena[s->cur], s->meta[s->cur], s->kscale, s->ctl,
                  s->pass_counter, false);
    const uint64_t bend = std::min<uint64_t>(end, j1 * L);
    uint64_t k = i;
    while (k < bend) {
      const uint64_t cnt = std::min<uint64_t>(bend - k, stage_amps);
      AMP(s, launch_readout)(s->stream, s->slots, s->geo, k - j0 * L, cnt, probs, s->dstage);
      HIP_TRY(hipMemcpyAsync(out + (k - begin) * per, s->dstage, 8 * cnt * per, hipMemcpyDeviceToHost, s->stream));
      HIP_TRY(hipStreamSynchronize(s->stream));
      k += cnt;
    }
    i = bend;
  }
  if ((rc = check_launch("readout"))) return rc;
  if ((rc = read_ctl(s))) return rc;
  if (s->h_ctl->flags) {
    clear_flags(s);
    return set_err(SIM_ECORRUPT, "a stored slice record failed its consistency checks");
  }
  return SIM_OK;
}

int sim_amplitudes(sim_t *s, uint64_t begin, uint64_t count, double *out) { return readout(s, begin, count, out, 0); }

int sim_probabilities(sim_t *s, uint64_t begin, uint64_t count, double *out) {
  return readout(s, begin, count, out, 1);
}

int sim_stats(sim_t *s, sim_stats_t *out) {
  if (!s || !out) return set_err(SIM_EINVAL, "null argument");
  int rc = read_ctl(s);
  if (rc) return rc;
  const Ctl &c = *s->h_ctl;
  memset(out, 0, sizeof(*out));
  out->raw_bytes = (s->fp32 ? 8ull : 16ull) << s->geo.n;
  out->compressed_bytes = c.cur_bytes;
  out->peak_compressed = std::max(c.peak_bytes, c.cur_bytes);
  out->ratio = c.cur_bytes ? (double)out->raw_bytes / (double)c.cur_bytes : 0.0;
  out->min_ratio = out->peak_compressed ? (double)out->raw_bytes / (double)out->peak_compressed : 0.0;
  out->passes = s->passes;
  out->escapes = c.escapes;
  out->last_norm = c.N;
  double me;
  memcpy(&me, &c.max_err_bits, 8);
  out->max_abs_codec_err = me;
  out->elapsed_s = s->elapsed;
  out->arena_bytes = s->arena_cap[0] + s->arena_cap[1];
  out->workspace_slots = (uint64_t)s->W;
  out->device_bytes = s->dev_bytes;
  out->gates = s->gates;
  std::vector<uint32_t> len(s->nslices);
  HIP_TRY(hipMemcpy(len.data(), s->meta[s->cur].rec_len, 4 * s->nslices, hipMemcpyDeviceToHost));
  const uint32_t big = *std::max_element(len.begin(), len.end());
  out->min_slice_ratio = big ? (double)((s->fp32 ? 8ull : 16ull) << s->geo.slice_log2) / (double)big : 0.0;
  return SIM_OK;
}

static int record_loc(sim_t *s, uint64_t j, uint64_t *off, uint32_t *len) {
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemcpy(off, s->meta[s->cur].rec_off + j, 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(len, s->meta[s->cur].rec_len + j, 4, hipMemcpyDeviceToHost));
  return SIM_OK;
}

uint64_t sim_record_size(sim_t *s, uint64_t j) {
  if (!s || j >= s->nslices) return 0;
  uint64_t off;
  uint32_t len;
  if (record_loc(s, j, &off, &len)) return 0;
  return len;
}

int sim_export_slice(sim_t *s, uint64_t j, void *buf, uint64_t cap, uint64_t *len_out) {
  if (!s || !buf) return set_err(SIM_EINVAL, "null argument");
  if (j >= s->nslices) return set_err(SIM_EINVAL, "slice %llu out of range", (unsigned long long)j);
  uint64_t off;
  uint32_t len;
  int rc = record_loc(s, j, &off, &len);
  if (rc) return rc;
  if (len_out) *len_out = len;
  if (cap < len) return set_err(SIM_EINVAL, "buffer of %llu bytes is smaller than the record (%u)",
                                (unsigned long long)cap, len);
  HIP_TRY(hipMemcpy(buf, s->arena[s->cur] + off, len, hipMemcpyDeviceToHost));
  return SIM_OK;
}

int sim_record_headers(sim_t *s, uint64_t first, uint64_t count, void *out) {
  if (!s || (count && !out)) return set_err(SIM_EINVAL, "null argument");
  if (first > s->nslices || count > s->nslices - first) return set_err(SIM_EINVAL, "slice range out of bounds");
  if (!count) return SIM_OK;
  HIP_TRY(hipStreamSynchronize(s->stream));
  std::vector<uint64_t> off(count);
  HIP_TRY(hipMemcpy(off.data(), s->meta[s->cur].rec_off + first, 8 * count, hipMemcpyDeviceToHost));
  uint8_t *o = (uint8_t *)out;
  for (uint64_t i = 0; i < count; i++)
    HIP_TRY(hipMemcpy(o + (uint64_t)kHdr * i, s->arena[s->cur] + off[i], kHdr, hipMemcpyDeviceToHost));
  return SIM_OK;
}

// Host check of a record's structure (everything a decoder relies on).
static int check_record(const sim_t *s, const uint8_t *r, uint64_t len, double *step, uint64_t sq[2]) {
  auto rd32 = [&](uint64_t o) { uint32_t v; memcpy(&v, r + o, 4); return v; };
  if (len < (uint64_t)kHdr || rd32(0) != kMagic) return set_err(SIM_ECORRUPT, "bad magic or short record");
  const uint32_t sl2 = rd32(4), cl2 = rd32(8), n_used = rd32(12), nch = rd32(16), nw = rd32(20), tot = rd32(28);
  if ((int)sl2 != s->geo.slice_log2 || (int)cl2 != s->geo.chunk_log2 || nch != s->geo.nchunks)
    return set_err(SIM_ECORRUPT, "record geometry does not match the simulator");
  if (n_used < 1 || n_used > (uint32_t)kNSym) return set_err(SIM_ECORRUPT, "bad symbol count");
  const uint32_t flags = rd32(56);
  if (flags > 15) return set_err(SIM_ECORRUPT, "unknown header flags");
  const uint64_t ooff = kHdr + ((2ull * n_used + 3) & ~3ull);
  uint32_t nruns = 0;  // chunk runs (flags bit 3)
  if (flags & 8) {
    if (len < ooff + 4) return set_err(SIM_ECORRUPT, "short record");
    nruns = rd32(ooff);
    if (nruns < 1 || nruns > nch || nruns > kMaxRuns) return set_err(SIM_ECORRUPT, "bad run count");
    if (ooff + 8ull * nruns + 8 + 4ull * nw != tot || tot != len) return set_err(SIM_ECORRUPT, "inconsistent size");
  } else if (rec_bytes_host(n_used, nch, nw) != tot || tot != len) {
    return set_err(SIM_ECORRUPT, "inconsistent size");
  }
  uint64_t kraft = 0;
  int prev = -1;
  for (uint32_t k = 0; k < n_used; k++) {
    uint16_t e;
    memcpy(&e, r + kHdr + 2 * k, 2);
    uint32_t l = e >> 10;
    int key = (int)e;
    if (l > (uint32_t)kLMax || key <= prev) return set_err(SIM_ECORRUPT, "bad symbol table");
    prev = key;
    kraft += 1ull << (kLMax - l);
  }
  if (kraft != (1ull << kLMax)) return set_err(SIM_ECORRUPT, "symbol table is not a complete prefix code");
  // pointwise-relative records (flags bit 2, word 15 their mantissa bits) only in that mode, with its bits
  const bool pw = (flags & 4) != 0;
  if (pw != (s->geo.pw_bits >= 0) || rd32(60) != (pw ? (uint32_t)s->geo.pw_bits : 0u))
    return set_err(SIM_ECORRUPT, "record's bound kind does not match the simulator");
  // the streams' word offsets (per chunk, or per run after the run ends):
  // non-decreasing from 0 to n_words, constant marks only where allowed, an
  // empty stream only with zero chunks (or as a constant chunk)
  const uint32_t nent = nruns ? nruns : nch;
  const uint64_t woff = nruns ? ooff + 4 + 4ull * nruns : ooff;
  uint32_t prevw = 0, prev_end = 0;
  bool prev_const = false;
  for (uint32_t c = 0; c <= nent; c++) {
    const uint32_t x = rd32(woff + 4ull * c);
    const bool cst = (x >> 31) != 0;
    const uint32_t w = x & 0x7FFFFFFFu;
    if (cst && (!(flags & 2) || c == nent)) return set_err(SIM_ECORRUPT, "bad constant-chunk mark");
    if (w < prevw || w > nw || (c == 0 && w != 0) || (c == nent && w != nw))
      return set_err(SIM_ECORRUPT, "bad chunk offsets");
    if (c > 0 && w == prevw && n_used > 1 && !prev_const && !(flags & 1))
      return set_err(SIM_ECORRUPT, "empty chunk in a record without zero chunks");
    if (nruns && c < nent) {  // run ends: strictly increasing, the last n_chunks
      const uint32_t e = rd32(ooff + 4 + 4ull * c);
      if (e <= prev_end || (c + 1 == nent && e != nch)) return set_err(SIM_ECORRUPT, "bad chunk runs");
      prev_end = e;
    }
    prevw = w;
    prev_const = cst;
  }
  memcpy(step, r + 32, 8);
  memcpy(sq, r + 40, 16);
  if (!(*step > 0.0) || !std::isfinite(*step)) return set_err(SIM_ECORRUPT, "bad step");
  if (pw) {  // step 1, and the sum field an FP64 squared norm
    double nrm;
    memcpy(&nrm, &sq[0], 8);
    if (*step != 1.0 || sq[1] != 0 || !(nrm >= 0.0) || !std::isfinite(nrm))
      return set_err(SIM_ECORRUPT, "bad pointwise-relative header");
  }
  return SIM_OK;
}

int sim_import_slice(sim_t *s, uint64_t j, const void *buf, uint64_t len) {
  if (!s || !buf) return set_err(SIM_EINVAL, "null argument");
  if (j >= s->nslices) return set_err(SIM_EINVAL, "slice out of range");
  double step;
  uint64_t sq[2];
  int rc = check_record(s, (const uint8_t *)buf, len, &step, sq);
  if (rc) return rc;
  if ((rc = read_ctl(s))) return rc;
  const int a = s->cur;
  uint64_t off = align_up(s->h_ctl->bump, kRecAlign);
  if (off + len > s->arena_cap[a]) {
    // move the arena into a larger buffer (records keep their offsets)
    uint64_t cap = std::max<uint64_t>(2 * s->arena_cap[a], off + len + (16ull << 20));
    uint8_t *na;
    if ((rc = s->dalloc((void **)&na, cap))) return rc;
    HIP_TRY(hipMemcpy(na, s->arena[a], s->h_ctl->bump, hipMemcpyDeviceToDevice));
    s->dfree(s->arena[a]);
    s->arena[a] = na;
    s->arena_cap[a] = cap;
  }
  uint64_t old_off;
  uint32_t old_len;
  if ((rc = record_loc(s, j, &old_off, &old_len))) return rc;
  const uint32_t len32 = (uint32_t)len;
  HIP_TRY(hipMemcpy(s->arena[a] + off, buf, len, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->meta[a].rec_off + j, &off, 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->meta[a].rec_len + j, &len32, 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->meta[a].step + j, &step, 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->meta[a].sq + 2 * j, sq, 16, hipMemcpyHostToDevice));
  {  // decoder table: code intervals of size 2^(12 - len) in table order tile [0, 4096)
    const uint8_t *r = (const uint8_t *)buf;
    uint32_t n_used;
    memcpy(&n_used, r + 12, 4);
    std::vector<uint16_t> one(1u << kLMax);
    uint32_t at = 0;
    for (uint32_t k = 0; k < n_used; k++) {
      uint16_t e;
      memcpy(&e, r + kHdr + 2 * k, 2);
      const uint32_t size = 1u << (kLMax - (e >> 10));
      for (uint32_t i = 0; i < size; i++) one[at + i] = e;
      at += size;
    }
    std::vector<uint32_t> dt(1u << kLMax);
    for (uint32_t e = 0; e < (1u << kLMax); e++) {
      const uint32_t s1 = one[e] & 1023u, l1 = one[e] >> 10;
      const uint32_t e2 = (e << l1) & ((1u << kLMax) - 1);
      const uint32_t s2 = one[e2] & 1023u, l2 = one[e2] >> 10;
      dt[e] = dtab_entry(s1, l1, s2, l2, s1 != 0 && s2 != 0 && l1 + l2 <= (uint32_t)kLMax);
    }
    HIP_TRY(hipMemcpy(s->meta[a].dtab + j * (1u << kLMax), dt.data(), 4u << kLMax, hipMemcpyHostToDevice));
  }
  s->h_ctl->bump = off + align_up(len, kRecAlign);
  s->h_ctl->cur_bytes = s->h_ctl->cur_bytes - old_len + len;
  HIP_TRY(hipMemcpy(&s->ctl->bump, &s->h_ctl->bump, 16, hipMemcpyHostToDevice));
  // a record with zero chunks: from now on the decoder handles them
  uint32_t flags;
  memcpy(&flags, (const uint8_t *)buf + 56, 4);
  s->geo.fmt_in |= flags & 3u;
  // the record's codes are not known to fit int32: the next pass decodes to FP64
  s->h_ctl->wide_next = 1;
  HIP_TRY(hipMemcpy(&s->ctl->wide_next, &s->h_ctl->wide_next, 4, hipMemcpyHostToDevice));
  return SIM_OK;
}

}  // extern "C"

// ------------------------------------------------- allocation-free apply
// Scratch of sim_apply_noalloc: the decompressed slots and per-slot
// partial results of a pass, the slot order of every slice group and the
// pass's gate matrices.  One array per GPU, held until the process ends;
// every call on that GPU uses it, so calls that overlap on one GPU race.
constexpr uint64_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, uint8_t *> g_scratch_ptr;  // device -> device address of `scratch`

// The device address of the scratch array on the current device, looked up
// once per device.
int scratch_address(uint8_t **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_err(SIM_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, (uint8_t *)p).first;
  }
  *out = it->second;
  return SIM_OK;
}

// Host slot order of all slices for group mask gm (as slot_table builds it).
void slot_order(uint64_t nslices, uint64_t gm, std::vector<uint64_t> &h) {
  std::vector<int> bits;
  for (int b = 0; b < 64; b++)
    if ((gm >> b) & 1) bits.push_back(b);
  h.clear();
  for (uint64_t j0 = 0; j0 < nslices; j0++) {
    if (j0 & gm) continue;
    for (uint64_t r = 0; r < (1ull << bits.size()); r++) {
      uint64_t j = j0;
      for (size_t b = 0; b < bits.size(); b++)
        if ((r >> b) & 1) j |= 1ull << bits[b];
      h.push_back(j);
    }
  }
}

}  // namespace

extern "C" {

int sim_apply_noalloc(sim_t *s, const sim_gate *gates, size_t n, size_t *n_applied) {
  if (n_applied) *n_applied = 0;
  if (!s) return set_err(SIM_EINVAL, "null handle");
  if (n && !gates) return set_err(SIM_EINVAL, "null gate array");
  if (s->mode & SIM_OPT) return set_err(SIM_EINVAL, "SIM_OPT handles apply through sim_apply");
  uint8_t *base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  PassSet P;
  prepare_passes(s, gates, n, P);
  if (P.vrc) {  // nothing runs: the whole program is checked first
    g_last_error = P.verr;
    return P.vrc;
  }
  const size_t n_pass = P.n_pass;
  if (n_pass == 0) return SIM_OK;
  // slice groups of the passes and their slot orders
  std::vector<GateDesc> descs;
  std::vector<uint64_t> gms;
  pass_descs(s, P, nullptr, descs, gms);
  std::vector<uint64_t> masks(gms.begin(), gms.end());
  std::sort(masks.begin(), masks.end());
  masks.erase(std::unique(masks.begin(), masks.end()), masks.end());
  int mmax = 0;
  for (uint64_t gm : masks) mmax = std::max(mmax, __builtin_popcountll(gm));
  // layout: [slots][one slot order per group mask][matrices]
  const uint64_t tab_bytes = align_up(8 * s->nslices, 256);
  const uint64_t fixed = masks.size() * tab_bytes + align_up(8 * P.hm.size(), 256);
  uint64_t W = 0;
  for (uint64_t w = 1; w <= s->nslices; w *= 2)
    if (carve_slots(s->geo, w, nullptr, nullptr) + fixed <= kScratchBytes) W = w;
  if (W < (1ull << mmax))
    return set_err(SIM_ENOMEM,
                   "the allocation-free entry point holds %llu bytes of scratch; a group of %d slices of 2^%d "
                   "amplitudes needs %llu",
                   (unsigned long long)kScratchBytes, 1 << mmax, s->geo.slice_log2,
                   (unsigned long long)(carve_slots(s->geo, 1ull << mmax, nullptr, nullptr) + fixed));
  Slots sl{};
  uint64_t off = carve_slots(s->geo, W, base, &sl);
  std::map<uint64_t, uint64_t *> tables;
  std::vector<std::vector<uint64_t>> host_tables(masks.size());
  for (size_t i = 0; i < masks.size(); i++) {
    slot_order(s->nslices, masks[i], host_tables[i]);
    uint64_t *d = (uint64_t *)(base + off);
    off += tab_bytes;
    HIP_TRY(hipMemcpyAsync(d, host_tables[i].data(), 8 * s->nslices, hipMemcpyHostToDevice, s->stream));
    tables[masks[i]] = d;
  }
  double *dmat = (double *)(base + off);
  if (!P.hm.empty())
    HIP_TRY(hipMemcpyAsync(dmat, P.hm.data(), 8 * P.hm.size(), hipMemcpyHostToDevice, s->stream));
  pass_descs(s, P, dmat, descs, gms);
  // the array keeps the last call's contents: clear what the passes count into
  launch_reset_slots(s->stream, sl, (int)W);
  if ((rc = check_launch("reset_slots"))) return rc;
  s->wslots = &sl;
  s->wW = (int)W;
  s->wtables = &tables;
  s->no_alloc = true;
  size_t applied = 0;
  HIP_TRY(hipEventRecord(s->ev0, s->stream));
  rc = run_passes(s, descs.data(), gms.data(), n_pass, -1, 0, &applied);
  s->wslots = nullptr;
  s->wW = 0;
  s->wtables = nullptr;
  s->no_alloc = false;
  // the host copies of tables and matrices stay alive until the stream has
  // passed them (run_passes synchronises)
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipEventRecord(s->ev1, s->stream));
  HIP_TRY(hipEventSynchronize(s->ev1));
  float ms = 0;
  hipEventElapsedTime(&ms, s->ev0, s->ev1);
  s->elapsed += ms * 1e-3;
  s->passes += applied;
  if (s->kt_on) s->kt_flush();
  size_t gates_done = 0;
  for (size_t i = 0; i < applied; i++) gates_done += P.plan[i].count;
  s->gates += gates_done;
  if (n_applied) *n_applied = gates_done;
  return rc;
}

int sim_kernel_times(sim_t *s, int enable, double *out, int cap, const char **names) {
  if (!s) return set_err(SIM_EINVAL, "null handle");
  if (names) *names = kClassNames;
  if (s->kt_on) s->kt_flush();
  if (out) {
    for (int k = 0; k < K_COUNT && k < cap; k++) out[k] = s->kt_ms[k];
    for (int k = 0; k < K_COUNT && K_COUNT + k < cap; k++) out[K_COUNT + k] = s->kt_n[k];
  }
  if (enable >= 0) {
    const bool on = enable != 0;
    if (on && s->kt_pool.empty()) {
      s->kt_pool.resize(8192);
      s->kt_cls.resize(4096);
      for (auto &e : s->kt_pool) hipEventCreate(&e);
    }
    s->kt_on = on;
    for (double &v : s->kt_ms) v = 0;
    for (double &v : s->kt_n) v = 0;
    s->kt_used = 0;
  }
  return K_COUNT;
}

}  // extern "C"
