// Job server: many independent compressed simulations on one device at once.
//
// Host code only.  It drives the public entry points of the library (one
// handle per job) from worker threads, one HIP stream per worker, so the
// passes of different jobs overlap on the device.  Admission, the ratio model
// and the memory cache are described with the srv_* declarations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "cqsim.h"
#include "cqsim_impl.h"

namespace {

// Device memory cache.  Requests are rounded up to a size class: multiples of
// an eighth of the largest power of two not above the request, and of 64 KiB,
// so a class of 512 KiB or more is at most 12.5% above its requests.  Freed
// blocks stay
// cached for later requests of the same class while the cache holds at most
// `limit` bytes; the rest go back to the device.  Blocks are handed back only
// after their handle's stream has drained (sim_destroy synchronises it).
class Pool {
 public:
  explicit Pool(uint64_t limit) : limit_(limit) {}
  ~Pool() { trim(0); }

  static size_t size_class(size_t b) {
    const size_t min_cls = 64u << 10;
    if (b <= min_cls) return min_cls;
    size_t p = 1;
    while (p <= b / 2) p <<= 1;  // largest power of two <= b
    const size_t step = std::max<size_t>(p / 8, min_cls);
    return (b + step - 1) / step * step;
  }

  void *alloc(size_t bytes) {
    const size_t c = size_class(bytes);
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = free_.find(c);
      if (it != free_.end() && !it->second.empty()) {
        void *p = it->second.back();
        it->second.pop_back();
        cached_ -= c;
        live_[p] = c;
        return p;
      }
    }
    void *p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
      (void)hipGetLastError();
      trim(0);  // give the cache back and try once more
      if (hipMalloc(&p, c) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    std::lock_guard<std::mutex> lk(mu_);
    live_[p] = c;
    return p;
  }

  void release(void *p) {
    size_t c = 0;
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = live_.find(p);
      if (it == live_.end()) return;
      c = it->second;
      live_.erase(it);
      if (cached_ + c <= limit_) {
        free_[c].push_back(p);
        cached_ += c;
        return;
      }
    }
    hipFree(p);
  }

  // Free cached blocks until at most `keep` bytes stay cached.
  void trim(uint64_t keep) {
    std::vector<void *> out;
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto it = free_.rbegin(); it != free_.rend() && cached_ > keep; ++it) {
        while (!it->second.empty() && cached_ > keep) {
          out.push_back(it->second.back());
          it->second.pop_back();
          cached_ -= it->first;
        }
      }
    }
    for (void *p : out) hipFree(p);
  }

  static void *alloc_hook(size_t bytes, void *ctx) { return static_cast<Pool *>(ctx)->alloc(bytes); }
  static void free_hook(void *p, void *ctx) { static_cast<Pool *>(ctx)->release(p); }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void *>> free_;
  std::map<void *, size_t> live_;
  uint64_t cached_ = 0;
  uint64_t limit_;
};

struct Job {
  srv_job spec{};
  std::vector<sim_gate> gates;
  std::vector<double> mats;     // every DENSE gate's matrix, gates[i].matrix points here
  std::vector<double> factors;  // SRV_INIT_PRODUCT
  srv_done done{};
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct srv_s {
  uint64_t budget = 0;
  int max_active = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  Pool pool;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job *> queue;
  std::vector<Job *> finished;
  uint64_t next_id = 1;
  uint64_t in_use = 0;  // projected bytes of running jobs
  int active = 0;
  bool stop = false;
  double model[SRV_FAMILIES] = {0};  // smallest minimum ratio seen per family; 0: none yet

  explicit srv_s(uint64_t b) : budget(b), pool(b) {}

  // Arena capacity (each of the two) for a job under the current model.
  uint64_t arena_for(const srv_job &j) const {
    const uint64_t amps = 1ull << j.cfg.n_qubits;
    const uint64_t cap = 8 * amps;  // int32 codes of both components
    const double raw = (double)(((j.cfg.mode & SIM_FP32) ? 8ull : 16ull) << j.cfg.n_qubits);
    const double r = model[j.family];
    uint64_t a = cap;
    if (r > 0) a = std::min<uint64_t>(cap, (uint64_t)(1.25 * raw / r));
    return std::max<uint64_t>(a, 64u << 10);
  }

  int project(const srv_job &j, uint64_t *bytes) const {
    sim_config c = j.cfg;
    if (!c.arena_bytes) c.arena_bytes = arena_for(j);
    return sim_footprint(&c, bytes);
  }

  void run(Job *J, hipStream_t st) {
    srv_done &d = J->done;
    sim_config c = J->spec.cfg;
    if (!c.arena_bytes) c.arena_bytes = arena_for(J->spec);
    c.stream = st;
    c.alloc = &Pool::alloc_hook;
    c.free_fn = &Pool::free_hook;
    c.alloc_ctx = &pool;
    sim_t *s = nullptr;
    int rc = sim_create_ex(&c, &s);
    if (!rc && J->spec.init == SRV_INIT_BASIS) rc = sim_init_basis(s, J->spec.basis);
    if (!rc && J->spec.init == SRV_INIT_PRODUCT) rc = sim_init_product(s, J->factors.data());
    size_t applied = 0;
    if (!rc && !J->gates.empty()) rc = sim_apply(s, J->gates.data(), J->gates.size(), &applied);
    if (!rc && J->spec.out) rc = sim_amplitudes(s, J->spec.out_begin, J->spec.out_count, J->spec.out);
    if (rc) snprintf(d.error, sizeof(d.error), "%s", sim_last_error());
    if (s) {
      sim_stats_t st_out;
      if (sim_stats(s, &st_out) == SIM_OK) {
        d.stats = st_out;
        d.device_bytes = st_out.device_bytes;
      }
      sim_destroy(s);
    }
    d.status = rc;
    d.applied = applied;
  }

  void worker(int w) {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      Job *J = nullptr;
      uint64_t proj = 0;
      cv_work.wait(lk, [&] {
        if (stop) return true;
        if (queue.empty() || active >= max_active) return false;
        if (project(queue.front()->spec, &proj)) proj = 0;  // refused later by sim_create_ex
        return active == 0 || in_use + proj <= budget;
      });
      if (stop) return;
      J = queue.front();
      queue.pop_front();
      active++;
      in_use += proj;
      J->done.projected_bytes = proj;
      J->done.t_start = seconds_since(t0);
      cv_work.notify_all();  // the next job may fit beside this one
      lk.unlock();
      run(J, streams[w]);
      lk.lock();
      J->done.t_end = seconds_since(t0);
      active--;
      in_use -= proj;
      const double r = J->done.stats.min_ratio;
      if (J->done.status == SIM_OK && r > 0) {
        double &m = model[J->spec.family];
        m = m > 0 ? std::min(m, r) : r;
      }
      finished.push_back(J);
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

namespace {

int check_job(const srv_job *j) {
  if (!j) return cq::fail(SIM_EINVAL, "null job");
  if (j->cfg.alloc || j->cfg.free_fn || j->cfg.stream)
    return cq::fail(SIM_EINVAL, "a job's allocator and stream are the server's");
  if (j->family >= SRV_FAMILIES) return cq::fail(SIM_EINVAL, "family outside 0..SRV_FAMILIES-1");
  if (j->init > SRV_INIT_PRODUCT) return cq::fail(SIM_EINVAL, "unknown init");
  if (j->init == SRV_INIT_PRODUCT && !j->factors) return cq::fail(SIM_EINVAL, "product init without factors");
  if (j->n_gates && !j->gates) return cq::fail(SIM_EINVAL, "null gate array");
  if (j->out && j->out_count == 0) return cq::fail(SIM_EINVAL, "output buffer for no amplitudes");
  uint64_t b;
  return sim_footprint(&j->cfg, &b);
}

}  // namespace

extern "C" {

int srv_create(uint64_t budget_bytes, int max_active, srv_t **out) {
  if (!out || max_active < 1 || max_active > 64 || budget_bytes == 0) return cq::fail(SIM_EINVAL, "max_active outside 1..64, zero budget or null handle");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return cq::fail(SIM_EDEVICE, "no HIP device");
  }
  srv_s *S = new srv_s(budget_bytes);
  hipGetDevice(&S->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, S->device) != hipSuccess || strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete S;
    return cq::fail(SIM_EDEVICE, "device is not gfx950");
  }
  S->max_active = max_active;
  S->t0 = std::chrono::steady_clock::now();
  for (int w = 0; w < max_active; w++) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : S->streams) hipStreamDestroy(x);
      delete S;
      return cq::fail(SIM_EDEVICE, "stream creation failed");
    }
    S->streams.push_back(st);
  }
  for (int w = 0; w < max_active; w++) S->workers.emplace_back(&srv_s::worker, S, w);
  *out = S;
  return SIM_OK;
}

int srv_submit(srv_t *S, const srv_job *job, uint64_t *id) {
  if (!S || !id) return cq::fail(SIM_EINVAL, "null argument");
  int rc = check_job(job);
  if (rc) return rc;
  uint64_t proj = 0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    rc = S->project(*job, &proj);
  }
  if (rc) return rc;
  if (proj > S->budget) return cq::fail(SIM_ENOMEM, "projected footprint exceeds the server's budget");
  Job *J = new Job();
  J->spec = *job;
  size_t nm = 0;
  for (size_t i = 0; i < job->n_gates; i++)
    if ((job->gates[i].kind == SIM_GATE_DENSE || job->gates[i].kind == SIM_GATE_U1Q) && job->gates[i].matrix &&
        job->gates[i].n_targets <= 5)
      nm += 2ull << (2 * job->gates[i].n_targets);
  J->mats.resize(nm);
  J->gates.assign(job->gates, job->gates + job->n_gates);
  size_t off = 0;
  for (sim_gate &g : J->gates) {
    if ((g.kind == SIM_GATE_DENSE || g.kind == SIM_GATE_U1Q) && g.matrix && g.n_targets <= 5) {
      const size_t m = 2ull << (2 * g.n_targets);
      std::copy(g.matrix, g.matrix + m, J->mats.begin() + off);
      g.matrix = J->mats.data() + off;
      off += m;
    }
  }
  J->spec.gates = nullptr;
  J->spec.factors = nullptr;
  if (job->init == SRV_INIT_PRODUCT) J->factors.assign(job->factors, job->factors + 4 * (size_t)job->cfg.n_qubits);
  J->done.family = job->family;
  std::lock_guard<std::mutex> lk(S->mu);
  J->done.id = S->next_id++;
  J->done.t_submit = seconds_since(S->t0);
  *id = J->done.id;
  S->queue.push_back(J);
  S->cv_work.notify_all();
  return SIM_OK;
}

int srv_wait(srv_t *S, srv_done *out, size_t cap, size_t *n_out, double timeout_s) {
  if (!S || !n_out || (cap && !out)) return cq::fail(SIM_EINVAL, "null argument");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(S->mu);
  auto ready = [&] { return !S->finished.empty() || (S->queue.empty() && S->active == 0); };
  if (timeout_s > 0)
    S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
  const size_t n = std::min(cap, S->finished.size());
  for (size_t i = 0; i < n; i++) {
    out[i] = S->finished[i]->done;
    delete S->finished[i];
  }
  S->finished.erase(S->finished.begin(), S->finished.begin() + n);
  *n_out = n;
  return SIM_OK;
}

double srv_clock(srv_t *S) { return S ? seconds_since(S->t0) : 0.0; }

int srv_projected_bytes(srv_t *S, const srv_job *job, uint64_t *bytes) {
  if (!S || !bytes) return cq::fail(SIM_EINVAL, "null argument");
  int rc = check_job(job);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(S->mu);
  return S->project(*job, bytes);
}

void srv_destroy(srv_t *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (Job *J : S->queue) delete J;
    S->queue.clear();
    S->cv_work.notify_all();
  }
  for (std::thread &t : S->workers) t.join();  // running jobs finish first
  for (Job *J : S->finished) delete J;
  for (hipStream_t st : S->streams) hipStreamDestroy(st);
  S->pool.trim(0);
  delete S;
}

}  // extern "C"
