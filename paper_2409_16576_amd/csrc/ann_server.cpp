// Served form of the search: continuous batching on one GPU.
//
// Requests (a few queries each, host memory) are queued by ann_server_submit.
// A scheduler thread coalesces consecutive waiting requests with the same
// (k, rerank_n) into one launch of at most max_batch queries, and starts it as
// soon as a slot (a stream with its pinned staging buffers) is free and the
// launch's device footprint fits in what is left of the HBM budget.  Launches
// on different slots overlap on the device; a finished launch frees its slot
// and its bytes at once, so requests that arrived meanwhile are admitted
// without waiting for a whole batch to drain.
//
// Device memory for in-flight work is one arena allocated at start and carved
// per launch (queries, per-query nprobe, outputs, the search's working
// buffers); the serving loop itself never calls hipMalloc.  Each query's result
// does not depend on which requests share its launch: the search treats every
// query independently (per-query nprobe, top-n and re-rank), so a request
// gives the same bits alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ann.h"
#include "ann_internal.h"

using namespace ann;

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;

size_t aup(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing frees.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      free_.erase(it);
      if (rest) free_[roff] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  void clear_peak() { peak_ = used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

struct Request {
  uint64_t ticket;
  int nq, k, n, np_max;
  std::vector<float> q;         // [nq, dim]
  std::vector<int32_t> np;      // [nq]
  std::vector<int64_t> ids;     // [nq, k]
  std::vector<float> dists;     // [nq, k]
  Clock::time_point t_submit, t_done;
  int state = 0;                // 0 waiting, 1 on the device, 2 done
  int status = ANN_OK;
};
using ReqPtr = std::shared_ptr<Request>;

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  float* h_q = nullptr;         // pinned [max_batch, dim]
  int32_t* h_np = nullptr;      // pinned [max_batch]
  int64_t* h_ids = nullptr;     // pinned [max_batch, max_k]
  float* h_d = nullptr;         // pinned [max_batch, max_k]
  bool busy = false;
  // the launch occupying the slot
  std::vector<ReqPtr> reqs;
  size_t off = 0, bytes = 0;
  int qc = 0, k = 0;
};

// Device bytes of one launch, laid out as: queries, nprobe, ids, dists, work.
struct Footprint {
  size_t q, np, ids, d, work, total;
};

Footprint footprint(const DevIndex& dv, int qc, int np_max, int n, int k) {
  Footprint f;
  f.q = aup((size_t)qc * dv.dim * 4);
  f.np = aup((size_t)qc * 4);
  f.ids = aup((size_t)qc * k * 8);
  f.d = aup((size_t)qc * k * 4);
  f.work = work_bytes(dv, qc, np_max, n);
  f.total = f.q + f.np + f.ids + f.d + f.work;
  return f;
}

}  // namespace

struct ann_server {
  ann_index* ix = nullptr;
  int device = 0;
  ann_server_cfg cfg{};
  void* arena_base = nullptr;
  Arena arena;
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_submit, cv_done;
  std::deque<ReqPtr> waiting;
  std::unordered_map<uint64_t, ReqPtr> live;  // submitted, not yet collected
  uint64_t next_ticket = 1;
  bool stopping = false;
  int fatal = ANN_OK;
  std::thread worker;

  // statistics (guarded by mu)
  std::vector<double> lat_ms;
  int64_t req_done = 0, q_done = 0, launches = 0;
  int in_flight = 0, max_in_flight = 0;

  ~ann_server() {
    for (Slot& s : slots) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.stream) (void)hipStreamDestroy(s.stream);
      if (s.h_q) (void)hipHostFree(s.h_q);
      if (s.h_np) (void)hipHostFree(s.h_np);
      if (s.h_ids) (void)hipHostFree(s.h_ids);
      if (s.h_d) (void)hipHostFree(s.h_d);
    }
    if (arena_base) (void)hipFree(arena_base);
  }

  // Start every waiting launch that a free slot and the arena allow.  Called
  // by the worker only.  Returns true if anything was launched.
  bool admit() {
    bool any = false;
    const DevIndex& dv = index_dev(ix);
    for (;;) {
      int si = -1;
      for (int i = 0; i < (int)slots.size(); ++i)
        if (!slots[i].busy) {
          si = i;
          break;
        }
      if (si < 0) return any;
      std::vector<ReqPtr> batch;
      int qc = 0, np_max = 0;
      Footprint fp{};
      size_t off = 0;
      {
        std::lock_guard<std::mutex> g(mu);
        if (waiting.empty()) return any;
        const int k = waiting.front()->k, n = waiting.front()->n;
        for (const ReqPtr& r : waiting) {
          if (r->k != k || r->n != n || qc + r->nq > cfg.max_batch) break;
          batch.push_back(r);
          qc += r->nq;
          np_max = std::max(np_max, r->np_max);
        }
        fp = footprint(dv, qc, np_max, n, k);
        if (!arena.alloc(fp.total, &off)) return any;  // wait for a launch to finish
        waiting.erase(waiting.begin(), waiting.begin() + (long)batch.size());
        for (const ReqPtr& r : batch) r->state = 1;
        ++in_flight;
        max_in_flight = std::max(max_in_flight, in_flight);
        ++launches;
      }
      Slot& s = slots[si];
      s.busy = true;
      s.reqs = std::move(batch);
      s.off = off;
      s.bytes = fp.total;
      s.qc = qc;
      s.k = s.reqs.front()->k;
      const int n = s.reqs.front()->n;
      // stage the queries and per-query nprobe in pinned memory
      int row = 0;
      for (const ReqPtr& r : s.reqs) {
        std::memcpy(s.h_q + (size_t)row * dv.dim, r->q.data(), r->q.size() * 4);
        std::memcpy(s.h_np + row, r->np.data(), r->np.size() * 4);
        row += r->nq;
      }
      char* base = static_cast<char*>(arena_base) + off;
      float* d_q = reinterpret_cast<float*>(base);
      int32_t* d_np = reinterpret_cast<int32_t*>(base + fp.q);
      int64_t* d_ids = reinterpret_cast<int64_t*>(base + fp.q + fp.np);
      float* d_d = reinterpret_cast<float*>(base + fp.q + fp.np + fp.ids);
      Work w = work_carve(dv, qc, np_max, n, base + fp.q + fp.np + fp.ids + fp.d);
      int st = ANN_OK;
      if (hipMemcpyAsync(d_q, s.h_q, (size_t)qc * dv.dim * 4, hipMemcpyHostToDevice, s.stream) !=
              hipSuccess ||
          hipMemcpyAsync(d_np, s.h_np, (size_t)qc * 4, hipMemcpyHostToDevice, s.stream) !=
              hipSuccess)
        st = set_error(ANN_EDEVICE, "server: query upload failed");
      if (st == ANN_OK)
        st = search_on(ix, w, d_q, qc, d_np, np_max, s.k, n, d_ids, d_d, s.stream);
      if (st == ANN_OK &&
          (hipMemcpyAsync(s.h_ids, d_ids, (size_t)qc * s.k * 8, hipMemcpyDeviceToHost, s.stream) !=
               hipSuccess ||
           hipMemcpyAsync(s.h_d, d_d, (size_t)qc * s.k * 4, hipMemcpyDeviceToHost, s.stream) !=
               hipSuccess))
        st = set_error(ANN_EDEVICE, "server: result download failed");
      if (hipEventRecord(s.done, s.stream) != hipSuccess && st == ANN_OK)
        st = set_error(ANN_EDEVICE, "server: event record failed");
      if (st != ANN_OK) {
        // the launch did not start cleanly: wait for what was enqueued, fail its requests
        (void)hipStreamSynchronize(s.stream);
        finish(s, st);
      }
      any = true;
    }
  }

  // Hand the slot's results to its requests and free the slot and its bytes.
  void finish(Slot& s, int st) {
    const auto now = Clock::now();
    std::lock_guard<std::mutex> g(mu);
    int row = 0;
    for (const ReqPtr& r : s.reqs) {
      if (st == ANN_OK) {
        for (int i = 0; i < r->nq; ++i) {
          std::memcpy(r->ids.data() + (size_t)i * r->k, s.h_ids + (size_t)(row + i) * s.k,
                      (size_t)r->k * 8);
          std::memcpy(r->dists.data() + (size_t)i * r->k, s.h_d + (size_t)(row + i) * s.k,
                      (size_t)r->k * 4);
        }
      }
      row += r->nq;
      r->status = st;
      r->t_done = now;
      r->state = 2;
      if (st == ANN_OK) {
        lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
        ++req_done;
        q_done += r->nq;
      }
    }
    // a device failure stops the server; any other failure (a request the
    // kernels cannot take) fails only that launch's requests
    if (st == ANN_EDEVICE) fatal = st;
    arena.release(s.off, s.bytes);
    --in_flight;
    s.reqs.clear();
    s.busy = false;
    cv_done.notify_all();
  }

  // Retire finished launches.  Returns true if any finished.
  bool retire() {
    bool any = false;
    for (Slot& s : slots) {
      if (!s.busy) continue;
      const hipError_t e = hipEventQuery(s.done);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) set_error(ANN_EDEVICE, "server: launch failed: %s", hipGetErrorString(e));
      finish(s, e == hipSuccess ? ANN_OK : ANN_EDEVICE);
      any = true;
    }
    return any;
  }

  void run() {
    (void)hipSetDevice(device);
    for (;;) {
      bool progress = retire();
      progress = admit() || progress;
      if (progress) continue;
      std::unique_lock<std::mutex> g(mu);
      const bool busy = in_flight > 0;
      if (stopping && waiting.empty() && !busy) return;
      if (busy) {
        // work on the device: poll its events again shortly
        g.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      } else {
        cv_submit.wait_for(g, std::chrono::milliseconds(2),
                           [&] { return stopping || !waiting.empty(); });
      }
    }
  }
};

extern "C" ann_status ann_server_start(ann_index* ix, const ann_server_cfg* cfg_in,
                                       ann_server** out) {
  if (!ix || !out) return (ann_status)set_error(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  ann_server_cfg c{};
  if (cfg_in) c = *cfg_in;
  const DevIndex& dv = index_dev(ix);
  if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = (int64_t)2 << 30;
  if (c.max_slots == 0) c.max_slots = 4;
  if (c.max_batch == 0) c.max_batch = std::min(1024, max_chunk(dv));
  if (c.max_nprobe == 0) c.max_nprobe = 256;
  if (c.max_k == 0) c.max_k = 64;
  if (c.max_rerank_n == 0) c.max_rerank_n = kMaxRerank;
  if (c.max_slots < 1 || c.max_slots > 16)
    return (ann_status)set_error(ANN_EINVAL, "max_slots must be in [1, 16]");
  if (c.max_batch < 1 || c.max_batch > max_chunk(dv))
    return (ann_status)set_error(ANN_EINVAL, "max_batch must be in [1, %d]", max_chunk(dv));
  if (c.max_nprobe < 1 || c.max_nprobe > 4096)
    return (ann_status)set_error(ANN_EINVAL, "max_nprobe must be in [1, 4096]");
  if (c.max_rerank_n < 1 || c.max_rerank_n > kMaxRerank)
    return (ann_status)set_error(ANN_EINVAL, "max_rerank_n must be in [1, %d]", kMaxRerank);
  if (c.max_k < 1 || c.max_k > c.max_rerank_n)
    return (ann_status)set_error(ANN_EINVAL, "max_k must be in [1, max_rerank_n]");
  // every admissible request must fit the scan's LDS (the largest request
  // needs the most: LDS grows with nprobe and rerank_n) and the raw tier
  int max_lds = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            index_device(ix)) != hipSuccess)
    return (ann_status)set_error(ANN_EDEVICE, "hipDeviceGetAttribute failed");
  const size_t lds = scan_lds_bytes(dv, c.max_nprobe, c.max_rerank_n, false);
  if ((int64_t)lds > (int64_t)max_lds)
    return (ann_status)set_error(ANN_EINVAL,
                                 "max_nprobe %d with max_rerank_n %d needs %zu bytes of scan LDS "
                                 "per block; the device allows %d",
                                 c.max_nprobe, c.max_rerank_n, lds, max_lds);
  if (dv.hpages && c.max_rerank_n > kHostMaxRerank)
    return (ann_status)set_error(ANN_EINVAL,
                                 "max_rerank_n must be <= %d with the host-memory raw tier",
                                 kHostMaxRerank);
  // the budget must admit one launch of the largest kind
  size_t biggest = 0;
  for (int n = 1; n <= c.max_rerank_n; ++n)
    biggest = std::max(biggest, footprint(dv, c.max_batch, c.max_nprobe, n, std::min(c.max_k, n)).total);
  if ((size_t)c.hbm_budget_bytes < biggest)
    return (ann_status)set_error(ANN_EINVAL,
                                 "hbm_budget_bytes %lld cannot hold one launch of max_batch "
                                 "queries (%zu bytes)", (long long)c.hbm_budget_bytes, biggest);
  if (hipSetDevice(index_device(ix)) != hipSuccess)
    return (ann_status)set_error(ANN_EDEVICE, "hipSetDevice failed");
  std::unique_ptr<ann_server> s(new ann_server());
  s->ix = ix;
  s->device = index_device(ix);
  s->cfg = c;
  if (hipMalloc(&s->arena_base, (size_t)c.hbm_budget_bytes) != hipSuccess)
    return (ann_status)set_error(ANN_ENOMEM, "server arena of %lld bytes", (long long)c.hbm_budget_bytes);
  s->arena.reset((size_t)c.hbm_budget_bytes);
  s->slots.resize(c.max_slots);
  for (Slot& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
      return (ann_status)set_error(ANN_EDEVICE, "server: stream/event creation failed");
    if (hipHostMalloc((void**)&sl.h_q, (size_t)c.max_batch * dv.dim * 4, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&sl.h_np, (size_t)c.max_batch * 4, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&sl.h_ids, (size_t)c.max_batch * c.max_k * 8, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&sl.h_d, (size_t)c.max_batch * c.max_k * 4, hipHostMallocDefault) !=
            hipSuccess)
      return (ann_status)set_error(ANN_ENOMEM, "server: pinned staging buffers");
  }
  ann_server* raw = s.get();
  s->worker = std::thread([raw] { raw->run(); });
  *out = s.release();
  return ANN_OK;
}

extern "C" ann_status ann_server_submit(ann_server* s, const float* queries, int32_t nq,
                                        const int32_t* nprobe, int32_t nprobe_max, int32_t k,
                                        int32_t rerank_n, uint64_t* ticket) {
  if (!s || !ticket) return (ann_status)set_error(ANN_EINVAL, "NULL argument");
  const ann_server_cfg& c = s->cfg;
  if (nq < 1 || nq > c.max_batch)
    return (ann_status)set_error(ANN_EINVAL, "nq must be in [1, %d]", c.max_batch);
  if (!queries) return (ann_status)set_error(ANN_EINVAL, "queries pointer is NULL");
  if (nprobe_max < 1 || nprobe_max > c.max_nprobe)
    return (ann_status)set_error(ANN_EINVAL, "nprobe_max must be in [1, %d]", c.max_nprobe);
  if (index_dev(s->ix).nav_beam > 0 && nprobe_max > kNavMaxBeam)
    return (ann_status)set_error(ANN_EINVAL, "nprobe_max above %d with the graph probe", kNavMaxBeam);
  if (k < 1 || k > c.max_k) return (ann_status)set_error(ANN_EINVAL, "k must be in [1, %d]", c.max_k);
  if (rerank_n < k || rerank_n > c.max_rerank_n)
    return (ann_status)set_error(ANN_EINVAL, "rerank_n must be in [k, %d]", c.max_rerank_n);
  const int dim = index_dev(s->ix).dim;
  ReqPtr r = std::make_shared<Request>();
  r->nq = nq;
  r->k = k;
  r->n = rerank_n;
  r->np_max = nprobe_max;
  r->q.assign(queries, queries + (size_t)nq * dim);
  r->np.resize(nq);
  for (int i = 0; i < nq; ++i)
    r->np[i] = nprobe ? std::max(0, std::min(nprobe[i], nprobe_max)) : nprobe_max;
  r->ids.resize((size_t)nq * k);
  r->dists.resize((size_t)nq * k);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stopping) return (ann_status)set_error(ANN_EINVAL, "server is stopping");
    if (s->fatal != ANN_OK)
      return (ann_status)set_error(s->fatal, "server: an earlier launch failed");
    r->ticket = s->next_ticket++;
    r->t_submit = Clock::now();
    s->waiting.push_back(r);
    s->live[r->ticket] = r;
  }
  s->cv_submit.notify_one();
  *ticket = r->ticket;
  return ANN_OK;
}

extern "C" ann_status ann_server_poll(ann_server* s, uint64_t ticket, int64_t* ids, float* dists,
                                      int32_t* done, int32_t wait) {
  if (!s || !done) return (ann_status)set_error(ANN_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> g(s->mu);
  auto it = s->live.find(ticket);
  if (it == s->live.end()) return (ann_status)set_error(ANN_EINVAL, "unknown ticket %llu",
                                                         (unsigned long long)ticket);
  ReqPtr r = it->second;
  if (wait) s->cv_done.wait(g, [&] { return r->state == 2; });
  if (r->state != 2) {
    *done = 0;
    return ANN_OK;
  }
  *done = 1;
  s->live.erase(it);
  if (r->status != ANN_OK) return (ann_status)set_error(r->status, "server: the launch failed");
  if (ids) std::memcpy(ids, r->ids.data(), r->ids.size() * 8);
  if (dists) std::memcpy(dists, r->dists.data(), r->dists.size() * 4);
  return ANN_OK;
}

extern "C" ann_status ann_server_get_stats(ann_server* s, ann_server_stats* out, int reset) {
  if (!s || !out) return (ann_status)set_error(ANN_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  ann_server_stats r{};
  r.requests_done = s->req_done;
  r.queries_done = s->q_done;
  r.launches = s->launches;
  r.max_in_flight = s->max_in_flight;
  r.peak_bytes = (int64_t)s->arena.peak();
  r.budget_bytes = s->cfg.hbm_budget_bytes;
  std::vector<double> v = s->lat_ms;
  if (!v.empty()) {
    auto pct = [&](double p) {
      const size_t i = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
      std::nth_element(v.begin(), v.begin() + (long)i, v.end());
      return v[i];
    };
    r.latency_p50_ms = pct(0.50);
    r.latency_p99_ms = pct(0.99);
    r.latency_max_ms = *std::max_element(v.begin(), v.end());
  }
  if (reset) {
    s->lat_ms.clear();
    s->req_done = s->q_done = s->launches = 0;
    s->max_in_flight = s->in_flight;
    s->arena.clear_peak();
  }
  *out = r;
  return ANN_OK;
}

extern "C" ann_status ann_server_stop(ann_server* s) {
  if (!s) return ANN_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
  }
  s->cv_submit.notify_all();
  if (s->worker.joinable()) s->worker.join();
  const int fatal = s->fatal;
  delete s;
  return fatal == ANN_OK ? ANN_OK
                         : (ann_status)set_error(fatal, "server: a launch failed before stop");
}
