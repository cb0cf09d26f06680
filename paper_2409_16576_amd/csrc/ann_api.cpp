// C ABI of the filtering stage: index loading, HBM layout, working-memory
// pool and the plain search pipeline.  Declarations and contracts: include/ann.h.
#include "ann.h"

#include <zlib.h>

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ann_internal.h"

using namespace ann;

namespace {

thread_local std::string g_err;

ann_status fail(ann_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

}  // namespace

int ann::set_error(int s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

namespace {

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ANN_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));            \
  } while (0)

// Working memory for one in-flight call: one block of the index's pool (the
// paper's per-query working-memory blocks, Sec. 5).  A block is reused only
// after the stream work of its previous user has completed (event order).
struct Workspace {
  Work w;
  void* lm_buf = nullptr;  // the list-major pass's buffers (carved per call)
  size_t cap_qc = 0, cap_np = 0, cap_nlist = 0, cap_keys = 0, cap_items = 0, cap_lut = 0,
         cap_cand = 0, cap_lm = 0;
  std::vector<void*> allocs;
  hipEvent_t done = nullptr;
  bool recorded = false;

  void release_memory() {
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
    w = Work{};
    lm_buf = nullptr;
    cap_qc = cap_np = cap_nlist = cap_keys = cap_items = cap_lut = cap_cand = cap_lm = 0;
  }
  ~Workspace() {
    if (recorded) (void)hipEventSynchronize(done);
    release_memory();
    if (done) (void)hipEventDestroy(done);
  }
};

struct Need {
  size_t qc, np, nlist, keys, items, lut, cand, lm = 0;
};

}  // namespace

struct ProfMark {
  int stage;
  hipEvent_t a, b;
};

struct ann_index {
  int device = 0;
  DevIndex d{};
  ann_index_desc desc{};
  std::vector<void*> allocs;
  std::mutex mu;
  std::vector<std::unique_ptr<Workspace>> pool;
  std::vector<Workspace*> free_ws;
  // tuning (ann_set_option); never changes results
  int64_t opt_tile = 0;  // 0: the tile follows the launch size (default_tile)
  int64_t opt_split = 16;
  int64_t opt_lut16 = 0;
  int64_t opt_order = 0;
  int64_t opt_lmajor = 0;  // list-major pass for large batches (integer-grid indexes)
  int64_t opt_lm_alpha = 2;
  int64_t opt_lm_tile = 4096;
  int64_t opt_lm_blocks = 0;
  int64_t opt_lm_cap = 0;
  int64_t opt_lm_min_rows = 0;
  int num_cu = 256;
  void* host_pages = nullptr;  // host-memory raw tier (pinned), freed with the index
  // stage timing
  bool profiling = false;
  std::mutex prof_mu;
  std::vector<ProfMark> marks;
  std::vector<hipEvent_t> spare_events;

  ~ann_index() {
    pool.clear();
    for (auto& m : marks) {
      (void)hipEventSynchronize(m.b);
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    for (auto e : spare_events) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
    if (host_pages) (void)hipHostFree(host_pages);
  }
};

namespace {

template <class T>
ann_status dev_upload(ann_index* ix, const T* host, size_t count, const T** out) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
  if (hipMalloc(&p, bytes) != hipSuccess)
    return fail(ANN_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  ix->allocs.push_back(p);
  ix->desc.hbm_bytes += (int64_t)bytes;
  if (count) HIP_TRY(hipMemcpy(p, host, count * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<const T*>(p);
  return ANN_OK;
}

ann_status ws_alloc(Workspace* ws, size_t bytes, void** out) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess)
    return fail(ANN_ENOMEM, "workspace hipMalloc of %zu bytes failed", bytes);
  ws->allocs.push_back(p);
  *out = p;
  return ANN_OK;
}

ann_status ws_ensure(Workspace* ws, const Need& n) {
  if (ws->cap_qc >= n.qc && ws->cap_np >= n.np && ws->cap_nlist >= n.nlist &&
      ws->cap_keys >= n.keys && ws->cap_items >= n.items && ws->cap_lut >= n.lut &&
      ws->cap_cand >= n.cand && ws->cap_lm >= n.lm)
    return ANN_OK;
  if (ws->recorded) HIP_TRY(hipEventSynchronize(ws->done));
  Need g{std::max(n.qc, ws->cap_qc), std::max(n.np, ws->cap_np), std::max(n.nlist, ws->cap_nlist),
         std::max(n.keys, ws->cap_keys), std::max(n.items, ws->cap_items),
         std::max(n.lut, ws->cap_lut), std::max(n.cand, ws->cap_cand),
         std::max(n.lm, ws->cap_lm)};
  ws->release_memory();
  Work& w = ws->w;
  ann_status s;
#define WS(ptr, bytes)                                                  \
  if ((s = ws_alloc(ws, (bytes), reinterpret_cast<void**>(&(ptr)))) != ANN_OK) { \
    ws->release_memory();                                               \
    return s;                                                           \
  }
  WS(w.dist, g.qc * g.nlist * 4);
  WS(w.lists, g.qc * g.np * 4);
  WS(w.np_eff, g.qc * 4);
  WS(w.lut, g.lut * 4);
  WS(w.perm, g.qc * 4);
  WS(w.sq, g.qc * 4);
  WS(w.pkeys, g.keys * 8);
  WS(w.pcount, g.items * 4);
  WS(w.pscan, g.items * 8);
  WS(w.cand, g.cand * 4);
  if (g.lm) WS(ws->lm_buf, g.lm);
#undef WS
  ws->cap_qc = g.qc; ws->cap_np = g.np; ws->cap_nlist = g.nlist; ws->cap_keys = g.keys;
  ws->cap_items = g.items; ws->cap_lut = g.lut; ws->cap_cand = g.cand; ws->cap_lm = g.lm;
  return ANN_OK;
}

// Take a pool block for this call and order it after its previous user.
ann_status ws_acquire(ann_index* ix, const Need& need, hipStream_t st, Workspace** out) {
  Workspace* ws = nullptr;
  {
    std::lock_guard<std::mutex> g(ix->mu);
    if (!ix->free_ws.empty()) {
      ws = ix->free_ws.back();
      ix->free_ws.pop_back();
    } else {
      ix->pool.emplace_back(new Workspace());
      ws = ix->pool.back().get();
    }
  }
  ann_status s = ANN_OK;
  if (!ws->done && hipEventCreateWithFlags(&ws->done, hipEventDisableTiming) != hipSuccess)
    s = fail(ANN_EDEVICE, "hipEventCreate failed");
  if (s == ANN_OK) s = ws_ensure(ws, need);
  if (s == ANN_OK && ws->recorded && hipStreamWaitEvent(st, ws->done, 0) != hipSuccess)
    s = fail(ANN_EDEVICE, "hipStreamWaitEvent failed");
  if (s != ANN_OK) {
    std::lock_guard<std::mutex> g(ix->mu);
    ix->free_ws.push_back(ws);
    return s;
  }
  *out = ws;
  return ANN_OK;
}

void ws_release(ann_index* ix, Workspace* ws, hipStream_t st) {
  if (hipEventRecord(ws->done, st) == hipSuccess) ws->recorded = true;
  std::lock_guard<std::mutex> g(ix->mu);
  ix->free_ws.push_back(ws);
}

struct WsGuard {
  ann_index* ix;
  Workspace* ws;
  hipStream_t st;
  ~WsGuard() {
    if (ws) ws_release(ix, ws, st);
  }
};

// Set while a search is captured into a HIP graph: no stage events then.
thread_local bool g_capturing = false;

// Brackets one kernel stage with an event pair when profiling is enabled.
struct StageMark {
  ann_index* ix;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;

  static hipEvent_t take(ann_index* ix) {
    std::lock_guard<std::mutex> g(ix->prof_mu);
    hipEvent_t e = nullptr;
    if (!ix->spare_events.empty()) {
      e = ix->spare_events.back();
      ix->spare_events.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  StageMark(ann_index* ix_, int stage_, hipStream_t st_) : ix(ix_), stage(stage_), st(st_) {
    if (!ix->profiling || g_capturing) return;
    a = take(ix);
    b = take(ix);
    if (a) (void)hipEventRecord(a, st);
  }
  ~StageMark() {
    if (!a || !b) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> g(ix->prof_mu);
    ix->marks.push_back({stage, a, b});
  }
};

// ---------------------------------------------------------------------------
// Index file parsing.

struct Section {
  uint64_t off, bytes;
  uint32_t crc;
};

uint32_t crc32_of(const uint8_t* p, size_t n) {
  uLong c = crc32(0L, Z_NULL, 0);
  while (n) {
    const uInt chunk = (uInt)std::min<size_t>(n, 1u << 30);
    c = crc32(c, p, chunk);
    p += chunk;
    n -= chunk;
  }
  return (uint32_t)c;
}

template <class T>
T rd(const std::vector<uint8_t>& b, size_t off) {
  T v;
  std::memcpy(&v, b.data() + off, sizeof(T));
  return v;
}

int elem_size(int dtype) { return dtype == F32 ? 4 : 1; }

size_t align_up_sz(size_t x, size_t a) { return (x + a - 1) / a * a; }

ann_status validate_args(ann_index* ix, const void* q, int64_t nq, int32_t np_max) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  if (nq < 0) return fail(ANN_EINVAL, "nq < 0");
  if (nq > 0 && !q) return fail(ANN_EINVAL, "queries pointer is NULL");
  if (np_max < 1 || np_max > 4096) return fail(ANN_EINVAL, "nprobe_max must be in [1, 4096]");
  if (ix->d.nav_beam > 0 && np_max > kNavMaxBeam)
    return fail(ANN_EINVAL, "nprobe_max above %d with the graph probe", kNavMaxBeam);
  return ANN_OK;
}

int chunk_queries(const DevIndex& d, int64_t nq) {
  // the coarse-distance matrix of a chunk is the largest working buffer; 4 GiB
  // (1.4% of HBM) keeps a 16k-query chunk up to 65536 lists, so a batch of
  // that size is one probe, one scan and one merge launch
  const size_t budget = size_t(4) << 30;
  size_t by_dist = budget / ((size_t)d.nlist * 4);
  size_t qc = std::min<size_t>({(size_t)nq, by_dist, size_t(16384)});
  return (int)std::max<size_t>(qc, 1);
}

// The list-major pass's buffers for a chunk of qc queries, carved from one
// 256-aligned block (sizes grow with every argument, so a block sized for
// larger arguments also holds smaller ones).
template <class F>
void lm_layout(const DevIndex& d, int qc, int np_max, int cap2, F&& take) {
  take(0, (size_t)qc * 4);                          // walkp
  take(1, (size_t)qc * 8);                          // thr
  take(2, (size_t)qc * 4);                          // cnt2
  take(3, (size_t)qc * cap2 * 8);                   // out2
  take(4, (size_t)qc);                              // flag
  take(5, (size_t)d.nlist * 4);                     // lcnt
  take(6, (size_t)d.nlist * 4);                     // lfill
  take(7, (size_t)(d.nlist + 1) * 4);               // loff
  take(8, (size_t)(d.nlist + 1) * 4);               // ioff
  take(9, (size_t)qc * np_max * 4);                 // invq
  take(10, (size_t)16 + (size_t)8 * ((d.nlist + 1023) / 1024));  // ctr + per-block totals
  take(11, lmajor_mfma(d) ? 0 : (size_t)qc * d.M * kKsub * 4);  // lut (float indexes)
}

size_t lm_bytes(const DevIndex& d, int qc, int np_max, int cap2) {
  size_t t = 0;
  lm_layout(d, qc, np_max, cap2,
            [&](int, size_t b) { t += align_up_sz(std::max<size_t>(b, 16), 256); });
  return t;
}

LmWork lm_carve(const DevIndex& d, int qc, int np_max, int cap2, void* base) {
  LmWork w;
  char* p = static_cast<char*>(base);
  void* ptr[12];
  lm_layout(d, qc, np_max, cap2, [&](int i, size_t b) {
    ptr[i] = p;
    p += align_up_sz(std::max<size_t>(b, 16), 256);
  });
  w.walkp = static_cast<int32_t*>(ptr[0]);
  w.thr = static_cast<unsigned long long*>(ptr[1]);
  w.cnt2 = static_cast<int32_t*>(ptr[2]);
  w.out2 = static_cast<uint64_t*>(ptr[3]);
  w.flag = static_cast<uint8_t*>(ptr[4]);
  w.lcnt = static_cast<int32_t*>(ptr[5]);
  w.lfill = static_cast<int32_t*>(ptr[6]);
  w.loff = static_cast<int32_t*>(ptr[7]);
  w.ioff = static_cast<int32_t*>(ptr[8]);
  w.invq = static_cast<int32_t*>(ptr[9]);
  w.ctr = static_cast<int32_t*>(ptr[10]);
  w.lut = lmajor_mfma(d) ? nullptr : static_cast<float*>(ptr[11]);
  w.cap2 = cap2;
  return w;
}

Need need_for(const DevIndex& d, int qc, int np_max, int n, int smax) {
  Need r;
  r.qc = (size_t)qc;
  r.np = (size_t)np_max;
  r.nlist = (size_t)d.nlist;
  r.items = (size_t)qc * smax;
  r.keys = r.items * (size_t)std::max(n, 1);
  r.lut = 0;  // the scan builds each query's table in LDS
  r.cand = 0;
  return r;
}

// Unless set: 65536 entries per work item from 1024 queries a launch on,
// proportionally fewer below (at least 4096), so that a small launch still
// has enough work items to fill the GPU.
int64_t default_tile(int qc) {
  return qc >= 1024 ? 65536 : std::max<int64_t>(4096, (int64_t)65536 * qc / 1024 / 64 * 64);
}

// Items of up to `tile` entries (default 64k: one per query at typical probe
// sizes, so the table is loaded once per query and the threshold filter sees
// long streams); very long queries are split across up to smax items.
LaunchCfg cfg_for(int qc, int np_max, int n, int k, int64_t tile, int64_t split) {
  LaunchCfg c;
  c.qc = qc;
  c.np_max = np_max;
  c.n = n;
  c.k = k;
  c.smax = std::max(1, std::min<int>((int)split, scan_smax(n)));
  c.tile = (int)tile;
  return c;
}

ann_status check_lds(ann_index* ix, int np_max, int n) {
  int max_lds = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device) !=
      hipSuccess)
    return fail(ANN_EDEVICE, "hipDeviceGetAttribute failed");
  const size_t need = scan_lds_bytes(ix->d, np_max, n, ix->opt_lut16 != 0);
  if ((int64_t)need > (int64_t)max_lds)
    return fail(ANN_EUNSUPPORTED, "scan needs %zu bytes of LDS per block, device allows %d", need,
                max_lds);
  return ANN_OK;
}

}  // namespace

// ===========================================================================

extern "C" const char* ann_last_error(void) { return g_err.c_str(); }

// Raw vectors on pages (Sec. 4.3, optimized storage layout).  Vectors are
// bucketed by nearest list; a bucket's whole pages are laid out first (bucket
// order, ascending ID); the remainders are packed onto shared pages: each new
// page starts with the largest remainder left and keeps adding the largest
// one that still fits its free slots (equal sizes: lower bucket first).
extern "C" int64_t ann_page_layout(const int32_t* bucket_of, int64_t n, int32_t nbuckets,
                                   int32_t row_bytes, int32_t page_bytes, int32_t* page,
                                   int32_t* slot) {
  if (!bucket_of || !page || !slot || n < 0 || nbuckets < 1 || row_bytes < 1 ||
      page_bytes < row_bytes) {
    fail(ANN_EINVAL, "page layout: bad arguments");
    return -1;
  }
  const int per = page_bytes / row_bytes;
  std::vector<std::vector<int32_t>> members(nbuckets);
  for (int64_t v = 0; v < n; ++v) {
    if (bucket_of[v] < 0 || bucket_of[v] >= nbuckets) {
      fail(ANN_EINVAL, "page layout: bucket out of range");
      return -1;
    }
    members[bucket_of[v]].push_back((int32_t)v);
  }
  int64_t next_page = 0;
  for (int b = 0; b < nbuckets; ++b) {
    const size_t whole = members[b].size() / per * per;
    for (size_t i = 0; i < whole; ++i) {
      page[members[b][i]] = (int32_t)(next_page + (int64_t)(i / per));
      slot[members[b][i]] = (int32_t)(i % per);
    }
    next_page += (int64_t)(whole / per);
  }
  // remainders by size: for each size, the buckets that have it, ascending
  std::vector<std::vector<int>> by_size(per);
  std::vector<size_t> taken(per, 0);
  int64_t left = 0;
  for (int b = 0; b < nbuckets; ++b) {
    const int r = (int)(members[b].size() % per);
    if (r) {
      by_size[r].push_back(b);
      ++left;
    }
  }
  auto largest_fitting = [&](int room) {
    for (int r = std::min(room, per - 1); r > 0; --r)
      if (taken[r] < by_size[r].size()) return r;
    return 0;
  };
  while (left > 0) {
    int room = per, filled = 0;
    for (int r; (r = largest_fitting(room)) > 0;) {
      const int b = by_size[r][taken[r]++];
      const size_t base = members[b].size() - r;
      for (int i = 0; i < r; ++i) {
        page[members[b][base + i]] = (int32_t)next_page;
        slot[members[b][base + i]] = filled + i;
      }
      filled += r;
      room -= r;
      --left;
    }
    ++next_page;
  }
  return next_page;
}

extern "C" ann_status ann_load_index(const char* path, int device, ann_index** out) {
  return ann_load_index_ex(path, device, nullptr, out);
}

extern "C" ann_status ann_load_index_ex(const char* path, int device, const ann_load_cfg* cfg,
                                        ann_index** out) {
  if (!path || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  const int raw_tier = cfg ? cfg->raw_tier : 0;
  const int page_bytes = cfg && cfg->page_bytes ? cfg->page_bytes : 4096;
  if (raw_tier != 0 && raw_tier != 1) return fail(ANN_EINVAL, "raw_tier must be 0 or 1");
  if (raw_tier && (page_bytes < 16 || page_bytes % 16 != 0 || page_bytes > 65536))
    return fail(ANN_EINVAL, "page_bytes must be a multiple of 16 in [16, 65536]");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(ANN_EIO, "cannot open %s", path);
  std::fseek(f, 0, SEEK_END);
  const long fsz = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  if (fsz < 512) {
    std::fclose(f);
    return fail(ANN_EFORMAT, "file too small");
  }
  std::vector<uint8_t> b((size_t)fsz);
  const size_t got = std::fread(b.data(), 1, b.size(), f);
  std::fclose(f);
  if (got != b.size()) return fail(ANN_EIO, "short read of %s", path);

  if (std::memcmp(b.data(), "FANNIDX1", 8) != 0) return fail(ANN_EFORMAT, "bad magic");
  if (rd<uint32_t>(b, 8) != 1 || rd<uint32_t>(b, 12) != 512 || rd<uint32_t>(b, 60) != 7)
    return fail(ANN_EFORMAT, "unsupported version");
  if (crc32_of(b.data(), 508) != rd<uint32_t>(b, 508)) return fail(ANN_EFORMAT, "header checksum");
  const int dtype = (int)rd<uint32_t>(b, 16);
  const int dim = (int)rd<uint32_t>(b, 20);
  const uint64_t n = rd<uint64_t>(b, 24);
  const int nlist = (int)rd<uint32_t>(b, 32);
  const int M = (int)rd<uint32_t>(b, 36);
  const int ksub = (int)rd<uint32_t>(b, 40);
  const int dsub = (int)rd<uint32_t>(b, 44);
  const int R = (int)rd<uint32_t>(b, 48);
  const uint32_t flags = rd<uint32_t>(b, 52);
  const uint64_t E = rd<uint64_t>(b, 64);
  if (dtype < 0 || dtype > 2) return fail(ANN_EFORMAT, "bad dtype %d", dtype);
  if (dim < 1 || nlist < 1 || M < 1 || R < 1 || n < 1 || dsub < 1 || (int64_t)dsub * M != dim)
    return fail(ANN_EFORMAT, "bad sizes");
  if (ksub != kKsub) return fail(ANN_EUNSUPPORTED, "ksub %d (only 256)", ksub);
  if (M > kMaxM) return fail(ANN_EUNSUPPORTED, "M %d > %d", M, kMaxM);
  if (dim > kMaxDim) return fail(ANN_EUNSUPPORTED, "dim %d > %d", dim, kMaxDim);
  if (R > 15) return fail(ANN_EUNSUPPORTED, "R %d > 15", R);
  if (n >= (1ull << kRankShift)) return fail(ANN_EUNSUPPORTED, "N >= 2^28");
  if (E > (uint64_t)INT32_MAX) return fail(ANN_EUNSUPPORTED, "more than 2^31 list entries");

  Section sec[7];
  const uint64_t want[7] = {(uint64_t)nlist * dim * 4, (uint64_t)M * ksub * dsub * 4,
                            n * (uint64_t)M,           n * (uint64_t)dim * elem_size(dtype),
                            (uint64_t)(nlist + 1) * 8, E * 4,
                            n * (uint64_t)R * 4};
  for (int i = 0; i < 7; ++i) {
    sec[i].off = rd<uint64_t>(b, 128 + 24 * i);
    sec[i].bytes = rd<uint64_t>(b, 128 + 24 * i + 8);
    sec[i].crc = rd<uint32_t>(b, 128 + 24 * i + 16);
    if (sec[i].bytes != want[i] || sec[i].off + sec[i].bytes > (uint64_t)fsz)
      return fail(ANN_EFORMAT, "section %d size/offset", i);
    if (crc32_of(b.data() + sec[i].off, sec[i].bytes) != sec[i].crc)
      return fail(ANN_EFORMAT, "section %d checksum", i);
  }
  const float* cent = reinterpret_cast<const float*>(b.data() + sec[0].off);
  const float* cb = reinterpret_cast<const float*>(b.data() + sec[1].off);
  const uint8_t* codes = b.data() + sec[2].off;
  const uint8_t* vecs = b.data() + sec[3].off;
  std::vector<int64_t> offs(nlist + 1);
  std::memcpy(offs.data(), b.data() + sec[4].off, sec[4].bytes);
  const int32_t* ent = reinterpret_cast<const int32_t*>(b.data() + sec[5].off);
  const int32_t* asg = reinterpret_cast<const int32_t*>(b.data() + sec[6].off);

  // Structural checks.
  if (offs[0] != 0 || offs[nlist] != (int64_t)E) return fail(ANN_EFORMAT, "list offsets");
  for (int l = 0; l < nlist; ++l) {
    if (offs[l + 1] < offs[l]) return fail(ANN_EFORMAT, "list offsets decrease");
    for (int64_t e = offs[l]; e < offs[l + 1]; ++e) {
      if (ent[e] < 0 || (uint64_t)ent[e] >= n) return fail(ANN_EFORMAT, "list entry out of range");
      if (e > offs[l] && ent[e] <= ent[e - 1]) return fail(ANN_EFORMAT, "list entries not ascending");
    }
  }
  uint64_t nassign = 0;
  std::vector<int32_t> primary(n);
  for (uint64_t v = 0; v < n; ++v) {
    const int32_t* a = asg + v * R;
    if (a[0] < 0 || a[0] >= nlist) return fail(ANN_EFORMAT, "vector %" PRIu64 " has no list", v);
    primary[v] = a[0];
    bool ended = false;
    for (int r = 0; r < R; ++r) {
      if (a[r] < 0) {
        ended = true;
        continue;
      }
      if (ended || a[r] >= nlist) return fail(ANN_EFORMAT, "bad assignment of vector %" PRIu64, v);
      for (int s = 0; s < r; ++s)
        if (a[s] == a[r]) return fail(ANN_EFORMAT, "duplicate list in assignment");
      ++nassign;
    }
  }
  if (nassign != E) return fail(ANN_EFORMAT, "assignment and lists disagree");
  const bool int_grid = (flags & 1u) && dtype != F32;
  if (int_grid) {
    const float lo = dtype == U8 ? 0.f : -128.f, hi = dtype == U8 ? 255.f : 127.f;
    auto ok = [&](const float* p, size_t cnt) {
      for (size_t i = 0; i < cnt; ++i)
        if (!(p[i] == std::nearbyint(p[i]) && p[i] >= lo && p[i] <= hi)) return false;
      return true;
    };
    if (!ok(cent, (size_t)nlist * dim) || !ok(cb, (size_t)M * ksub * dsub))
      return fail(ANN_EFORMAT, "integer-grid flag set but centroids/codebooks are not integers");
  }

  // Row order: vectors grouped by first list, ascending external id inside.
  std::vector<int32_t> pstart(nlist + 1, 0);
  for (uint64_t v = 0; v < n; ++v) pstart[primary[v] + 1]++;
  for (int l = 0; l < nlist; ++l) pstart[l + 1] += pstart[l];
  std::vector<int32_t> fill(pstart.begin(), pstart.end() - 1);
  std::vector<int32_t> row2ext(n), ext2row(n);
  for (uint64_t v = 0; v < n; ++v) {
    const int32_t row = fill[primary[v]]++;
    row2ext[row] = (int32_t)v;
    ext2row[v] = row;
  }
  // Replica entries and list / assignment consistency.
  std::vector<int32_t> rstart(nlist + 1, 0);
  std::vector<int2> rep;
  rep.reserve(E - n);
  for (int l = 0; l < nlist; ++l) {
    rstart[l] = (int32_t)rep.size();
    int64_t nprim = 0;
    for (int64_t e = offs[l]; e < offs[l + 1]; ++e) {
      const int32_t v = ent[e];
      const int32_t* a = asg + (uint64_t)v * R;
      int rank = -1;
      for (int r = 0; r < R; ++r)
        if (a[r] == l) rank = r;
      if (rank < 0) return fail(ANN_EFORMAT, "list %d holds vector %d not assigned to it", l, v);
      if (rank == 0) {
        ++nprim;
      } else {
        rep.push_back(make_int2((int)((uint32_t)ext2row[v] | ((uint32_t)rank << kRankShift)), a[0]));
      }
    }
    if (nprim != pstart[l + 1] - pstart[l])
      return fail(ANN_EFORMAT, "list %d misses some of its first-list vectors", l);
    // group this list's replica entries by their vector's first list (then row)
    std::sort(rep.begin() + rstart[l], rep.end(), [](const int2& x, const int2& y) {
      const uint32_t rx = (uint32_t)x.x & kRowMask, ry = (uint32_t)y.x & kRowMask;
      return x.y < y.y || (x.y == y.y && rx < ry);
    });
  }
  rstart[nlist] = (int32_t)rep.size();
  std::vector<int32_t> lseg(nlist + 1, 0);
  std::vector<int4> segs;
  int max_segs = 0;
  for (int l = 0; l < nlist; ++l) {
    lseg[l] = (int32_t)segs.size();
    for (int32_t r = rstart[l]; r < rstart[l + 1];) {
      int32_t e = r;
      while (e < rstart[l + 1] && rep[e].y == rep[r].y) ++e;
      segs.push_back(make_int4(rep[r].y, r, e, 0));
      r = e;
    }
    max_segs = std::max(max_segs, (int)(segs.size() - lseg[l]));
  }
  lseg[nlist] = (int32_t)segs.size();

  const int row_bytes = (M + 3) / 4 * 4;
  const int es = elem_size(dtype);
  std::vector<uint8_t> codes_rows((n + rep.size()) * row_bytes + kCodeSlack, 0);
  std::vector<int32_t> asg_rows((size_t)n * R);
  for (uint64_t row = 0; row < n; ++row) {
    const uint64_t v = (uint64_t)row2ext[row];
    std::memcpy(&codes_rows[row * row_bytes], codes + v * M, M);
    std::memcpy(&asg_rows[row * R], asg + v * R, (size_t)R * 4);
  }
  // rows n + e: replica entry e's code row and ID, in entry order
  row2ext.resize(n + rep.size());
  for (size_t e = 0; e < rep.size(); ++e) {
    const uint32_t row = (uint32_t)rep[e].x & kRowMask;
    std::memcpy(&codes_rows[(n + e) * row_bytes], &codes_rows[(size_t)row * row_bytes], row_bytes);
    row2ext[n + e] = row2ext[row];
  }
  std::vector<float> cent_t((size_t)dim * nlist);
  for (int l = 0; l < nlist; ++l)
    for (int t = 0; t < dim; ++t) cent_t[(size_t)t * nlist + l] = cent[(size_t)l * dim + t];
  int64_t max_list = 0;
  for (int l = 0; l < nlist; ++l) max_list = std::max<int64_t>(max_list, offs[l + 1] - offs[l]);

  std::unique_ptr<ann_index> ix(new ann_index());
  ix->device = device;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(ANN_EDEVICE, "device %d not available", device);
  HIP_TRY(hipSetDevice(device));
  if (noalloc_setup(device) != ANN_OK) return ANN_EDEVICE;  // message already set
  HIP_TRY(hipDeviceGetAttribute(&ix->num_cu, hipDeviceAttributeMultiprocessorCount, device));
  DevIndex& d = ix->d;
  d.dtype = dtype; d.dim = dim; d.nlist = nlist; d.M = M; d.row_bytes = row_bytes; d.dsub = dsub;
  d.R = R; d.int_grid = int_grid ? 1 : 0; d.n = (int64_t)n;
  ann_status s;
  const uint8_t* pc = nullptr;
  const uint8_t* pv = nullptr;
  const int2* prep = nullptr;
  if ((s = dev_upload(ix.get(), codes_rows.data(), codes_rows.size(), &pc)) != ANN_OK) return s;
  if (!raw_tier) {
    // raw vectors stay in external-ID order: the re-rank reads them by ID
    if ((s = dev_upload(ix.get(), vecs, (size_t)n * dim * es, &pv)) != ANN_OK) return s;
  } else {
    // host-memory raw tier: pages of pinned host memory, bucketed by nearest list
    const int rowb = dim * es;
    if (rowb > page_bytes) return fail(ANN_EINVAL, "a raw vector (%d bytes) exceeds a page", rowb);
    std::vector<int32_t> vpage(n), vslot(n);
    const int64_t npages = ann_page_layout(primary.data(), (int64_t)n, nlist, rowb, page_bytes,
                                           vpage.data(), vslot.data());
    if (npages < 0) return ANN_EINVAL;
    const size_t hbytes = std::max<size_t>((size_t)npages * page_bytes, 16);
    if (hipHostMalloc(&ix->host_pages, hbytes, hipHostMallocMapped) != hipSuccess) {
      ix->host_pages = nullptr;
      return fail(ANN_ENOMEM, "hipHostMalloc of %zu bytes (raw pages) failed", hbytes);
    }
    uint8_t* hp = static_cast<uint8_t*>(ix->host_pages);
    std::memset(hp, 0, hbytes);
    for (uint64_t v = 0; v < n; ++v)
      std::memcpy(hp + (size_t)vpage[v] * page_bytes + (size_t)vslot[v] * rowb,
                  vecs + v * (size_t)rowb, rowb);
    void* dp = nullptr;
    HIP_TRY(hipHostGetDevicePointer(&dp, ix->host_pages, 0));
    d.hpages = static_cast<const uint8_t*>(dp);
    d.page_bytes = page_bytes;
    if ((s = dev_upload(ix.get(), vpage.data(), vpage.size(), &d.vpage)) != ANN_OK) return s;
    if ((s = dev_upload(ix.get(), vslot.data(), vslot.size(), &d.vslot)) != ANN_OK) return s;
    ix->desc.host_bytes = (int64_t)hbytes;
    ix->desc.pages = npages;
  }
  d.codes = pc;
  d.vecs = pv;
  if ((s = dev_upload(ix.get(), row2ext.data(), row2ext.size(), &d.row2ext)) != ANN_OK) return s;
  if ((s = dev_upload(ix.get(), cent, (size_t)nlist * dim, &d.centroids)) != ANN_OK) return s;
  if ((s = dev_upload(ix.get(), cent_t.data(), cent_t.size(), &d.centroids_t)) != ANN_OK) return s;
  if ((s = dev_upload(ix.get(), cb, (size_t)M * ksub * dsub, &d.codebooks)) != ANN_OK) return s;
  if ((s = dev_upload(ix.get(), pstart.data(), pstart.size(), &d.pstart)) != ANN_OK) return s;
  if ((s = dev_upload(ix.get(), rstart.data(), rstart.size(), &d.rstart)) != ANN_OK) return s;
  if ((s = dev_upload(ix.get(), rep.data(), rep.size(), &prep)) != ANN_OK) return s;
  d.rep = prep;
  if ((s = dev_upload(ix.get(), asg_rows.data(), asg_rows.size(), &d.assign_rows)) != ANN_OK)
    return s;
  const int4* pseg = nullptr;
  if ((s = dev_upload(ix.get(), segs.data(), segs.size(), &pseg)) != ANN_OK) return s;
  d.segs = pseg;
  if ((s = dev_upload(ix.get(), lseg.data(), lseg.size(), &d.lseg)) != ANN_OK) return s;
  d.max_segs = max_segs;
  // Integer-grid indexes probe on the int8 matrix cores: shifted, padded centroids.
  d.dim_pad = (dim + 63) / 64 * 64;
  d.shift8 = dtype == U8 ? 128 : 0;
  if (int_grid && d.dim_pad <= 512) {
    std::vector<int8_t> c8((size_t)nlist * d.dim_pad, 0);
    std::vector<int32_t> cn(nlist, 0);
    for (int l = 0; l < nlist; ++l) {
      int32_t acc = 0;
      for (int t = 0; t < dim; ++t) {
        const int v = (int)cent[(size_t)l * dim + t] - d.shift8;
        c8[(size_t)l * d.dim_pad + t] = (int8_t)v;
        acc += v * v;
      }
      cn[l] = acc;
    }
    if ((s = dev_upload(ix.get(), c8.data(), c8.size(), &d.cent8)) != ANN_OK) return s;
    if ((s = dev_upload(ix.get(), cn.data(), cn.size(), &d.cnorm8)) != ANN_OK) return s;
    // the codebooks shifted the same way (decoding for the list-major scan),
    // padded to a multiple of 16 bytes
    std::vector<int8_t> b8(((size_t)M * ksub * dsub + 15) / 16 * 16, 0);
    for (size_t i = 0; i < (size_t)M * ksub * dsub; ++i) b8[i] = (int8_t)((int)cb[i] - d.shift8);
    if ((s = dev_upload(ix.get(), b8.data(), b8.size(), &d.cb8)) != ANN_OK) return s;
  }

  ann_index_desc& ds = ix->desc;
  ds.n = (int64_t)n; ds.dim = dim; ds.dtype = dtype; ds.nlist = nlist; ds.m = M; ds.ksub = ksub;
  ds.dsub = dsub; ds.r = R; ds.int_grid = d.int_grid; ds.entries = (int64_t)E;
  ds.replica_entries = (int64_t)rep.size(); ds.max_list = max_list; ds.device = device;
  ds.max_rerank_n = raw_tier ? kHostMaxRerank : kMaxRerank;
  ds.raw_tier = raw_tier;
  ds.page_bytes = raw_tier ? page_bytes : 0;
  *out = ix.release();
  return ANN_OK;
}

extern "C" ann_status ann_index_info(const ann_index* ix, ann_index_desc* out) {
  if (!ix || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = ix->desc;
  return ANN_OK;
}

extern "C" void ann_free_index(ann_index* ix) { delete ix; }

namespace {

// Heuristic re-ranking parameters (Alg. 1); batch 0 = the fixed-n re-rank.
struct Heur {
  int batch = 0;
  double eps = 0.0;
  int beta = 1;
  int32_t* reranked = nullptr;    // [nq] candidates re-ranked, or NULL
  int32_t* page_reads = nullptr;  // [nq] raw pages read (host-memory raw tier), or NULL
};

// Steps 1-8 (or 1-7 with topn_ids) for qc <= chunk_queries(...) queries, on
// the given working buffers.
ann_status run_chunk(ann_index* ix, Work& w, const float* q, int qc, const int32_t* nprobe,
                     int32_t np_max, int32_t k, int32_t n, int64_t* out_ids, float* out_d,
                     int32_t* topn_ids, float* topn_adc, int64_t* ncand, hipStream_t st,
                     const Heur& h = Heur(), int64_t* nwalk = nullptr) {
  const DevIndex& d = ix->d;
  LaunchCfg c = cfg_for(qc, np_max, n, k, ix->opt_tile ? ix->opt_tile : default_tile(qc),
                        ix->opt_split);
  c.lut16 = ix->opt_lut16 != 0;
  c.order = ix->opt_order != 0;
  c.hb = h.batch;
  c.h_eps = h.eps;
  c.h_beta = h.beta;
  {
    StageMark m(ix, 0, st);
    HIP_TRY(launch_probe(d, q, nprobe, np_max, qc, w, nullptr, w.lists, st));
  }
  if (w.lm.thr && lmajor_cap(ix, n) > 0) {
    // batched form: per-query part, list-major pass, per-query selection;
    // stages: per-query part 2, the persistent launch 4, the rest (split,
    // work list, selection, overflow fallback) 5
    LmCfg lc;
    lc.alpha = (int)ix->opt_lm_alpha;
    lc.tile_rows = (int)ix->opt_lm_tile;
    lc.blocks = (int)ix->opt_lm_blocks;
    lc.min_rows = (int)ix->opt_lm_min_rows;
    static const int stage_of[kLmPhases] = {5, 2, 5, 4, 5, 5};
    for (int ph = 0; ph < kLmPhases; ++ph) {
      StageMark m(ix, stage_of[ph], st);
      HIP_TRY(launch_lmajor(d, q, c, w, w.lm, lc, ix->num_cu, ph, st));
    }
  } else {
    StageMark m(ix, 2, st);  // steps 1, 3, 5, 6, 7: the table is built inside the scan
    HIP_TRY(launch_scan(d, w.lists, w.np_eff, q, c, w, st));
  }
  {
    StageMark m(ix, 3, st);
    HIP_TRY(launch_merge(d, q, c, w, topn_ids, topn_adc, ncand, nwalk, out_ids, out_d, h.reranked,
                         h.page_reads, st));
  }
  return ANN_OK;
}

ann_status run_pipeline(ann_index* ix, const float* Q, int64_t nq, const int32_t* nprobe,
                        int32_t np_max, int32_t k, int32_t n, int64_t* out_ids, float* out_d,
                        int32_t* topn_ids, float* topn_adc, int64_t* ncand, hipStream_t st,
                        const Heur& h = Heur(), int64_t* nwalk = nullptr) {
  HIP_TRY(hipSetDevice(ix->device));
  ann_status s;
  if ((s = check_lds(ix, np_max, n)) != ANN_OK) return s;
  const DevIndex& d = ix->d;
  if (d.hpages && out_ids && n > kHostMaxRerank)
    return fail(ANN_EINVAL, "rerank_n must be <= %d with the host-memory raw tier", kHostMaxRerank);
  const int qc_max = chunk_queries(d, nq);
  const LaunchCfg c0 = cfg_for(qc_max, np_max, n, k, ix->opt_tile, ix->opt_split);
  Workspace* ws = nullptr;
  Need need = need_for(d, qc_max, np_max, n, c0.smax);
  const int cap2 = lmajor_cap(ix, n);
  if (cap2) need.lm = lm_bytes(d, qc_max, np_max, cap2);
  if ((s = ws_acquire(ix, need, st, &ws)) != ANN_OK) return s;
  WsGuard guard{ix, ws, st};
  Work w = ws->w;
  if (cap2) w.lm = lm_carve(d, qc_max, np_max, cap2, ws->lm_buf);
  for (int64_t q0 = 0; q0 < nq; q0 += qc_max) {
    const int qc = (int)std::min<int64_t>(qc_max, nq - q0);
    s = run_chunk(ix, w, Q + q0 * d.dim, qc, nprobe ? nprobe + q0 : nullptr, np_max, k, n,
                  out_ids ? out_ids + q0 * k : nullptr, out_d ? out_d + q0 * k : nullptr,
                  topn_ids ? topn_ids + q0 * n : nullptr, topn_adc ? topn_adc + q0 * n : nullptr,
                  ncand ? ncand + q0 : nullptr, st,
                  Heur{h.batch, h.eps, h.beta, h.reranked ? h.reranked + q0 : nullptr,
                       h.page_reads ? h.page_reads + q0 : nullptr},
                  nwalk ? nwalk + q0 : nullptr);
    if (s != ANN_OK) return s;
  }
  return ANN_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Helpers for the serving loop (ann_server.cpp).

const DevIndex& ann::index_dev(const ann_index* ix) { return ix->d; }
int ann::index_device(const ann_index* ix) { return ix->device; }

size_t ann::work_bytes(const DevIndex& d, int qc, int np_max, int n, int lm_cap2) {
  const int smax = cfg_for(qc, np_max, n, 1, 65536, 16).smax;
  const Need g = need_for(d, qc, np_max, n, smax);
  auto a = [](size_t b) { return align_up_sz(std::max<size_t>(b, 16), 256); };
  return a(g.qc * g.nlist * 4) + a(g.qc * g.np * 4) + a(g.qc * 4) + a(g.qc * 8) + a(g.qc * 4) +
         a(g.keys * 8) + a(g.items * 4) + a(g.items * 8) +
         (lm_cap2 > 0 ? lm_bytes(d, qc, np_max, lm_cap2) : 0);
}

Work ann::work_carve(const DevIndex& d, int qc, int np_max, int n, void* base, int lm_cap2) {
  const int smax = cfg_for(qc, np_max, n, 1, 65536, 16).smax;
  const Need g = need_for(d, qc, np_max, n, smax);
  char* p = static_cast<char*>(base);
  auto take = [&](size_t b) {
    void* r = p;
    p += align_up_sz(std::max<size_t>(b, 16), 256);
    return r;
  };
  Work w;
  w.dist = static_cast<float*>(take(g.qc * g.nlist * 4));
  w.lists = static_cast<int32_t*>(take(g.qc * g.np * 4));
  w.np_eff = static_cast<int32_t*>(take(g.qc * 4));
  w.perm = static_cast<int32_t*>(take(g.qc * 4));
  w.sq = static_cast<int32_t*>(take(g.qc * 4));
  w.pkeys = static_cast<uint64_t*>(take(g.keys * 8));
  w.pcount = static_cast<int32_t*>(take(g.items * 4));
  w.pscan = static_cast<int32_t*>(take(g.items * 8));
  if (lm_cap2 > 0) w.lm = lm_carve(d, qc, np_max, lm_cap2, p);
  return w;
}

int ann::lmajor_cap(const ann_index* ix, int n) {
  if (!ix->opt_lmajor || !lmajor_supported(ix->d)) return 0;
  return ix->opt_lm_cap > 0 ? (int)ix->opt_lm_cap : lmajor_cap2(n);
}

int ann::search_on(ann_index* ix, Work& w, const float* d_q, int qc, const int32_t* d_nprobe,
                   int np_max, int k, int n, int64_t* d_ids, float* d_dists, hipStream_t st) {
  ann_status s = check_lds(ix, np_max, n);
  if (s != ANN_OK) return s;
  if (ix->d.hpages && n > kHostMaxRerank)
    return fail(ANN_EINVAL, "rerank_n must be <= %d with the host-memory raw tier", kHostMaxRerank);
  return run_chunk(ix, w, d_q, qc, d_nprobe, np_max, k, n, d_ids, d_dists, nullptr, nullptr,
                   nullptr, st);
}

int ann::max_chunk(const DevIndex& d) { return chunk_queries(d, INT32_MAX); }

bool ann::set_capturing(bool on) {
  const bool was = g_capturing;
  g_capturing = on;
  return was;
}

int ann::get_opt(const ann_index* ix, int option, int64_t* v) {
  switch (option) {
    case ANN_OPT_SCAN_TILE: *v = ix->opt_tile; return ANN_OK;
    case ANN_OPT_SCAN_SPLIT: *v = ix->opt_split; return ANN_OK;
    case ANN_OPT_LUT_F16: *v = ix->opt_lut16; return ANN_OK;
    case ANN_OPT_SCAN_ORDER: *v = ix->opt_order; return ANN_OK;
    case ANN_OPT_LIST_MAJOR: *v = ix->opt_lmajor; return ANN_OK;
    case ANN_OPT_LM_ALPHA: *v = ix->opt_lm_alpha; return ANN_OK;
    case ANN_OPT_LM_TILE: *v = ix->opt_lm_tile; return ANN_OK;
    case ANN_OPT_LM_BLOCKS: *v = ix->opt_lm_blocks; return ANN_OK;
    case ANN_OPT_LM_CAP: *v = ix->opt_lm_cap; return ANN_OK;
    case ANN_OPT_LM_MIN_ROWS: *v = ix->opt_lm_min_rows; return ANN_OK;
    case ANN_OPT_PROBE_BEAM: *v = ix->d.nav_beam; return ANN_OK;
    default: return ANN_EINVAL;
  }
}

namespace {

}  // namespace

extern "C" ann_status ann_search(ann_index* ix, const float* d_queries, int64_t nq,
                                 const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                                 int32_t rerank_n, int64_t* d_out_ids, float* d_out_dists,
                                 void* stream) {
  ann_status s = validate_args(ix, d_queries, nq, nprobe_max);
  if (s != ANN_OK) return s;
  if (k < 1) return fail(ANN_EINVAL, "k must be >= 1");
  if (rerank_n < k || rerank_n > kMaxRerank)
    return fail(ANN_EINVAL, "rerank_n must be in [k, %d]", kMaxRerank);
  if (nq > 0 && (!d_out_ids || !d_out_dists)) return fail(ANN_EINVAL, "output pointer is NULL");
  if (nq == 0) return ANN_OK;
  return run_pipeline(ix, d_queries, nq, d_nprobe, nprobe_max, k, rerank_n, d_out_ids,
                      d_out_dists, nullptr, nullptr, nullptr, (hipStream_t)stream);
}

extern "C" ann_status ann_search_heuristic(ann_index* ix, const float* d_queries, int64_t nq,
                                           const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                                           int32_t rerank_n, int32_t batch_size, double eps,
                                           int32_t beta, int64_t* d_out_ids, float* d_out_dists,
                                           int32_t* d_out_reranked, void* stream) {
  ann_status s = validate_args(ix, d_queries, nq, nprobe_max);
  if (s != ANN_OK) return s;
  if (k < 1 || k > 64) return fail(ANN_EINVAL, "k must be in [1, 64] for the heuristic re-rank");
  if (rerank_n < k || rerank_n > kMaxRerank)
    return fail(ANN_EINVAL, "rerank_n must be in [k, %d]", kMaxRerank);
  if (batch_size < 1) return fail(ANN_EINVAL, "batch_size must be >= 1");
  if (beta < 1) return fail(ANN_EINVAL, "beta must be >= 1");
  if (!(eps >= 0.0)) return fail(ANN_EINVAL, "eps must be >= 0");
  if (nq > 0 && (!d_out_ids || !d_out_dists)) return fail(ANN_EINVAL, "output pointer is NULL");
  if (nq == 0) return ANN_OK;
  Heur h;
  h.batch = batch_size;
  h.eps = eps;
  h.beta = beta;
  h.reranked = d_out_reranked;
  return run_pipeline(ix, d_queries, nq, d_nprobe, nprobe_max, k, rerank_n, d_out_ids,
                      d_out_dists, nullptr, nullptr, nullptr, (hipStream_t)stream, h);
}

extern "C" ann_status ann_search_pages(ann_index* ix, const float* d_queries, int64_t nq,
                                       const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                                       int32_t rerank_n, int32_t batch_size, double eps,
                                       int32_t beta, int64_t* d_out_ids, float* d_out_dists,
                                       int32_t* d_out_reranked, int32_t* d_out_page_reads,
                                       void* stream) {
  ann_status s = validate_args(ix, d_queries, nq, nprobe_max);
  if (s != ANN_OK) return s;
  if (!ix->d.hpages)
    return fail(ANN_EUNSUPPORTED, "the index keeps its raw vectors in HBM (no pages to count)");
  if (k < 1) return fail(ANN_EINVAL, "k must be >= 1");
  if (batch_size > 0 && k > 64)
    return fail(ANN_EINVAL, "k must be in [1, 64] for the heuristic re-rank");
  if (rerank_n < k || rerank_n > kHostMaxRerank)
    return fail(ANN_EINVAL, "rerank_n must be in [k, %d]", kHostMaxRerank);
  if (batch_size < 0) return fail(ANN_EINVAL, "batch_size must be >= 0");
  if (batch_size > 0 && beta < 1) return fail(ANN_EINVAL, "beta must be >= 1");
  if (batch_size > 0 && !(eps >= 0.0)) return fail(ANN_EINVAL, "eps must be >= 0");
  if (nq > 0 && (!d_out_ids || !d_out_dists)) return fail(ANN_EINVAL, "output pointer is NULL");
  if (nq == 0) return ANN_OK;
  Heur h;
  h.batch = batch_size;
  h.eps = eps;
  h.beta = beta;
  h.reranked = d_out_reranked;
  h.page_reads = d_out_page_reads;
  return run_pipeline(ix, d_queries, nq, d_nprobe, nprobe_max, k, rerank_n, d_out_ids,
                      d_out_dists, nullptr, nullptr, nullptr, (hipStream_t)stream, h);
}

extern "C" ann_status ann_search_topn(ann_index* ix, const float* d_queries, int64_t nq,
                                      const int32_t* d_nprobe, int32_t nprobe_max,
                                      int32_t rerank_n, int32_t* d_out_ids, float* d_out_adc,
                                      int64_t* d_out_ncand, int64_t* d_out_nwalk,
                                      void* stream) {
  ann_status s = validate_args(ix, d_queries, nq, nprobe_max);
  if (s != ANN_OK) return s;
  if (rerank_n < 1 || rerank_n > kMaxRerank)
    return fail(ANN_EINVAL, "rerank_n must be in [1, %d]", kMaxRerank);
  if (nq > 0 && (!d_out_ids || !d_out_adc)) return fail(ANN_EINVAL, "output pointer is NULL");
  if (nq == 0) return ANN_OK;
  return run_pipeline(ix, d_queries, nq, d_nprobe, nprobe_max, 1, rerank_n, nullptr, nullptr,
                      d_out_ids, d_out_adc, d_out_ncand, (hipStream_t)stream, Heur(), d_out_nwalk);
}

extern "C" ann_status ann_probe(ann_index* ix, const float* d_queries, int64_t nq,
                                const int32_t* d_nprobe, int32_t nprobe_max, int32_t* d_out_lists,
                                float* d_out_dists, void* stream) {
  ann_status s = validate_args(ix, d_queries, nq, nprobe_max);
  if (s != ANN_OK) return s;
  if (nq > 0 && !d_out_lists) return fail(ANN_EINVAL, "output pointer is NULL");
  if (nq == 0) return ANN_OK;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ix->device));
  const int qc_max = chunk_queries(ix->d, nq);
  Workspace* ws = nullptr;
  if ((s = ws_acquire(ix, need_for(ix->d, qc_max, nprobe_max, 1, 1), st, &ws)) != ANN_OK) return s;
  WsGuard guard{ix, ws, st};
  for (int64_t q0 = 0; q0 < nq; q0 += qc_max) {
    const int qc = (int)std::min<int64_t>(qc_max, nq - q0);
    HIP_TRY(launch_probe(ix->d, d_queries + q0 * ix->d.dim, d_nprobe ? d_nprobe + q0 : nullptr,
                         nprobe_max, qc, ws->w, d_out_dists ? d_out_dists + q0 * nprobe_max : nullptr,
                         d_out_lists + q0 * nprobe_max, st));
  }
  return ANN_OK;
}

extern "C" ann_status ann_lut(ann_index* ix, const float* d_queries, int64_t nq, float* d_out_lut,
                              void* stream) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  if (nq < 0) return fail(ANN_EINVAL, "nq < 0");
  if (nq > 0 && (!d_queries || !d_out_lut)) return fail(ANN_EINVAL, "NULL pointer");
  HIP_TRY(hipSetDevice(ix->device));
  const int64_t step = 65535;
  for (int64_t q0 = 0; q0 < nq; q0 += step) {
    const int qc = (int)std::min<int64_t>(step, nq - q0);
    HIP_TRY(launch_lut(ix->d, d_queries + q0 * ix->d.dim, qc,
                       d_out_lut + q0 * (int64_t)ix->d.M * kKsub, (hipStream_t)stream));
  }
  return ANN_OK;
}

extern "C" ann_status ann_scan_trace(ann_index* ix, const int32_t* d_lists, int64_t nq,
                                     int32_t nprobe_max, const float* d_lut, int64_t capacity,
                                     int32_t* d_out_ids, float* d_out_adc, int64_t* d_out_count,
                                     void* stream) {
  ann_status s = validate_args(ix, d_lists, nq, nprobe_max);
  if (s != ANN_OK) return s;
  if (capacity < 0) return fail(ANN_EINVAL, "capacity < 0");
  if (nq > 0 && (!d_lut || !d_out_count || (capacity > 0 && (!d_out_ids || !d_out_adc))))
    return fail(ANN_EINVAL, "NULL pointer");
  if (nq == 0) return ANN_OK;
  if (nq > (1 << 24)) return fail(ANN_EINVAL, "nq too large for the trace form");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ix->device));
  if ((s = check_lds(ix, nprobe_max, 1)) != ANN_OK) return s;
  Workspace* ws = nullptr;
  Need nd = need_for(ix->d, (int)nq, nprobe_max, 1, 16);
  nd.nlist = 0;
  nd.lut = 0;
  if ((s = ws_acquire(ix, nd, st, &ws)) != ANN_OK) return s;
  WsGuard guard{ix, ws, st};
  HIP_TRY(launch_scan_trace(ix->d, d_lists, d_lut, (int)nq, nprobe_max, capacity, d_out_ids,
                            d_out_adc, d_out_count, ws->w, st));
  return ANN_OK;
}

extern "C" ann_status ann_rerank(ann_index* ix, const float* d_queries, int64_t nq,
                                 const int32_t* d_cand_ids, int32_t n, int32_t k,
                                 int64_t* d_out_ids, float* d_out_dists, void* stream) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  if (nq < 0) return fail(ANN_EINVAL, "nq < 0");
  if (k < 1 || n < k || n > kMaxRerank) return fail(ANN_EINVAL, "need 1 <= k <= n <= %d", kMaxRerank);
  if (nq > 0 && (!d_queries || !d_cand_ids || !d_out_ids || !d_out_dists))
    return fail(ANN_EINVAL, "NULL pointer");
  if (ix->d.hpages)
    return fail(ANN_EUNSUPPORTED, "ann_rerank reads raw vectors from HBM; this index keeps them "
                                  "in host memory (use ann_search_pages)");
  HIP_TRY(hipSetDevice(ix->device));
  const int64_t step = 1 << 20;
  for (int64_t q0 = 0; q0 < nq; q0 += step) {
    const int qc = (int)std::min<int64_t>(step, nq - q0);
    HIP_TRY(launch_rerank_only(ix->d, d_queries + q0 * ix->d.dim, d_cand_ids + q0 * n, qc, n, k,
                               d_out_ids + q0 * k, d_out_dists + q0 * k, (hipStream_t)stream));
  }
  return ANN_OK;
}

extern "C" ann_status ann_set_profiling(ann_index* ix, int enable) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  ix->profiling = enable != 0;
  return ANN_OK;
}

extern "C" ann_status ann_get_profile(ann_index* ix, ann_profile* out, int reset) {
  if (!ix || !out) return fail(ANN_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(ix->prof_mu);
  *out = ann_profile{};
  for (auto& m : ix->marks) {
    HIP_TRY(hipEventSynchronize(m.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, m.a, m.b));
    out->ms[m.stage] += ms;
    out->launches[m.stage] += 1;
  }
  if (reset) {
    for (auto& m : ix->marks) {
      ix->spare_events.push_back(m.a);
      ix->spare_events.push_back(m.b);
    }
    ix->marks.clear();
  }
  return ANN_OK;
}

extern "C" ann_status ann_set_option(ann_index* ix, int option, int64_t value) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  switch (option) {
    case ANN_OPT_SCAN_TILE:
      if (value != 0 && (value < 64 || value > (int64_t)1 << 30))
        return fail(ANN_EINVAL, "tile must be 0 or in [64, 2^30]");
      ix->opt_tile = value;
      return ANN_OK;
    case ANN_OPT_SCAN_SPLIT:
      if (value < 1 || value > 16) return fail(ANN_EINVAL, "split must be in [1, 16]");
      ix->opt_split = value;
      return ANN_OK;
    case ANN_OPT_LUT_F16:
      if (value != 0 && value != 1) return fail(ANN_EINVAL, "lut_f16 must be 0 or 1");
      ix->opt_lut16 = value;
      return ANN_OK;
    case ANN_OPT_SCAN_ORDER:
      if (value != 0 && value != 1) return fail(ANN_EINVAL, "scan order must be 0 or 1");
      ix->opt_order = value;
      return ANN_OK;
    case ANN_OPT_LIST_MAJOR:
      if (value != 0 && value != 1) return fail(ANN_EINVAL, "list-major must be 0 or 1");
      ix->opt_lmajor = value;
      return ANN_OK;
    case ANN_OPT_LM_ALPHA:
      if (value < 1 || value > 64) return fail(ANN_EINVAL, "list-major alpha must be in [1, 64]");
      ix->opt_lm_alpha = value;
      return ANN_OK;
    case ANN_OPT_LM_TILE:
      if (value < 64 || value > (int64_t)1 << 24)
        return fail(ANN_EINVAL, "list-major tile must be in [64, 2^24] rows");
      ix->opt_lm_tile = value;
      return ANN_OK;
    case ANN_OPT_LM_BLOCKS:
      if (value < 0 || value > 65536) return fail(ANN_EINVAL, "list-major blocks must be in [0, 65536]");
      ix->opt_lm_blocks = value;
      return ANN_OK;
    case ANN_OPT_LM_CAP:
      if (value < 0 || value > (1 << 20))
        return fail(ANN_EINVAL, "list-major capacity must be in [0, 2^20] keys");
      ix->opt_lm_cap = value;
      return ANN_OK;
    case ANN_OPT_LM_MIN_ROWS:
      if (value < 0 || value > (1 << 30))
        return fail(ANN_EINVAL, "list-major minimum rows must be in [0, 2^30]");
      ix->opt_lm_min_rows = value;
      return ANN_OK;
    case ANN_OPT_PROBE_BEAM:
      if (value < 0 || value > kNavMaxBeam)
        return fail(ANN_EINVAL, "probe beam must be in [0, %d]", kNavMaxBeam);
      if (value > 0 && !ix->d.nav_adj) return fail(ANN_EINVAL, "no navigation graph (ann_set_nav_graph)");
      ix->d.nav_beam = (int)value;
      return ANN_OK;
    default:
      return fail(ANN_EINVAL, "unknown option %d", option);
  }
}

namespace {
void free_dev(ann_index* ix, const void* p) {
  if (!p) return;
  auto it = std::find(ix->allocs.begin(), ix->allocs.end(), const_cast<void*>(p));
  if (it != ix->allocs.end()) {
    ix->allocs.erase(it);
    (void)hipFree(const_cast<void*>(p));
  }
}
}  // namespace

extern "C" ann_status ann_set_nav_graph(ann_index* ix, const int32_t* adj, int32_t deg,
                                        const int32_t* entry, int32_t n_entry) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  DevIndex& d = ix->d;
  if (!adj) {  // remove the graph: the probe is exact again
    HIP_TRY(hipSetDevice(ix->device));
    HIP_TRY(hipDeviceSynchronize());
    free_dev(ix, d.nav_adj);
    free_dev(ix, d.nav_entry);
    d.nav_adj = d.nav_entry = nullptr;
    d.nav_deg = d.nav_nentry = d.nav_beam = 0;
    return ANN_OK;
  }
  if (deg < 1 || deg > 1024) return fail(ANN_EINVAL, "degree must be in [1, 1024]");
  if (!entry || n_entry < 1 || n_entry > d.nlist)
    return fail(ANN_EINVAL, "need 1 to nlist entry vertices");
  std::vector<int32_t> row(deg);
  for (int v = 0; v < d.nlist; ++v) {
    int c = 0;
    for (int j = 0; j < deg; ++j) {
      const int32_t u = adj[(size_t)v * deg + j];
      if (u < -1 || u >= d.nlist) return fail(ANN_EINVAL, "vertex %d: neighbour %d out of range", v, u);
      if (u >= 0) row[c++] = u;
    }
    std::sort(row.begin(), row.begin() + c);
    if (std::adjacent_find(row.begin(), row.begin() + c) != row.begin() + c)
      return fail(ANN_EINVAL, "vertex %d lists a neighbour twice", v);
  }
  std::vector<int32_t> es(entry, entry + n_entry);
  std::sort(es.begin(), es.end());
  if (es.front() < 0 || es.back() >= d.nlist) return fail(ANN_EINVAL, "entry vertex out of range");
  if (std::adjacent_find(es.begin(), es.end()) != es.end())
    return fail(ANN_EINVAL, "an entry vertex is listed twice");
  HIP_TRY(hipSetDevice(ix->device));
  HIP_TRY(hipDeviceSynchronize());  // no search may still read the old graph
  free_dev(ix, d.nav_adj);
  free_dev(ix, d.nav_entry);
  d.nav_adj = d.nav_entry = nullptr;
  d.nav_deg = d.nav_nentry = d.nav_beam = 0;
  ann_status s;
  const int32_t* pa = nullptr;
  const int32_t* pe = nullptr;
  if ((s = dev_upload(ix, adj, (size_t)d.nlist * deg, &pa)) != ANN_OK) return s;
  if ((s = dev_upload(ix, entry, (size_t)n_entry, &pe)) != ANN_OK) {
    free_dev(ix, pa);
    return s;
  }
  d.nav_adj = pa;
  d.nav_entry = pe;
  d.nav_deg = deg;
  d.nav_nentry = n_entry;
  return ANN_OK;
}

extern "C" ann_status ann_get_option(ann_index* ix, int option, int64_t* value) {
  if (!ix || !value) return fail(ANN_EINVAL, "NULL argument");
  if (get_opt(ix, option, value) == ANN_OK) return ANN_OK;
  switch (option) {
    default: return fail(ANN_EINVAL, "unknown option %d", option);
  }
}
