// Batched form: a whole query batch's search captured once into a HIP graph
// (one graph launch replays probe, scan and merge for every chunk), and an
// autotuner that picks the scan's work split for a batch by timing it.
//
// The graph owns its working memory, so a launch neither allocates nor takes
// a block from the index's pool; successive launches of one graph are ordered
// by an event (they share that memory).  Results are those of ann_search on
// the same buffers: the captured kernels are the same launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <memory>
#include <vector>

#include "ann.h"
#include "ann_internal.h"

using namespace ann;

struct ann_graph {
  ann_index* ix = nullptr;
  void* work = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t last = nullptr;
  bool launched = false;

  ~ann_graph() {
    if (last) {
      if (launched) (void)hipEventSynchronize(last);
      (void)hipEventDestroy(last);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (work) (void)hipFree(work);
  }
};

namespace {

ann_status err(ann_status s, const char* what, hipError_t e) {
  return (ann_status)set_error(s, "%s: %s", what, hipGetErrorString(e));
}

// Enqueue the search of nq queries on st with the given working memory
// (chunks of at most max_chunk queries share it in stream order).
ann_status enqueue_search(ann_index* ix, void* work, const float* q, int64_t nq,
                          const int32_t* nprobe, int np_max, int k, int n, int64_t* ids,
                          float* dists, hipStream_t st) {
  const DevIndex& d = index_dev(ix);
  const int chunk = max_chunk(d);
  const int lm_cap2 = lmajor_cap(ix, n);
  for (int64_t q0 = 0; q0 < nq; q0 += chunk) {
    const int qc = (int)std::min<int64_t>(chunk, nq - q0);
    Work w = work_carve(d, qc, np_max, n, work, lm_cap2);
    const int s = search_on(ix, w, q + q0 * d.dim, qc, nprobe ? nprobe + q0 : nullptr, np_max, k,
                            n, ids + q0 * k, dists + q0 * k, st);
    if (s != ANN_OK) return (ann_status)s;
  }
  return ANN_OK;
}

ann_status check_search_args(ann_index* ix, const float* q, int64_t nq, int32_t np_max, int32_t k,
                             int32_t n, const void* ids, const void* dists) {
  if (!ix) return (ann_status)set_error(ANN_EINVAL, "index is NULL");
  if (nq < 1) return (ann_status)set_error(ANN_EINVAL, "nq must be >= 1");
  if (!q || !ids || !dists) return (ann_status)set_error(ANN_EINVAL, "NULL pointer");
  if (np_max < 1 || np_max > 4096)
    return (ann_status)set_error(ANN_EINVAL, "nprobe_max must be in [1, 4096]");
  if (k < 1) return (ann_status)set_error(ANN_EINVAL, "k must be >= 1");
  if (n < k || n > kMaxRerank)
    return (ann_status)set_error(ANN_EINVAL, "rerank_n must be in [k, %d]", kMaxRerank);
  return ANN_OK;
}

}  // namespace

extern "C" ann_status ann_graph_create(ann_index* ix, const float* d_queries, int64_t nq,
                                       const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                                       int32_t rerank_n, int64_t* d_out_ids, float* d_out_dists,
                                       ann_graph** out) {
  if (!out) return (ann_status)set_error(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  ann_status s = check_search_args(ix, d_queries, nq, nprobe_max, k, rerank_n, d_out_ids,
                                   d_out_dists);
  if (s != ANN_OK) return s;
  hipError_t e = hipSetDevice(index_device(ix));
  if (e != hipSuccess) return err(ANN_EDEVICE, "hipSetDevice", e);
  const DevIndex& d = index_dev(ix);
  const int chunk = (int)std::min<int64_t>(nq, max_chunk(d));
  std::unique_ptr<ann_graph> g(new ann_graph());
  g->ix = ix;
  if ((e = hipMalloc(&g->work, work_bytes(d, chunk, nprobe_max, rerank_n,
                                           lmajor_cap(ix, rerank_n)))) != hipSuccess)
    return err(ANN_ENOMEM, "graph working memory", e);
  if ((e = hipEventCreateWithFlags(&g->last, hipEventDisableTiming)) != hipSuccess)
    return err(ANN_EDEVICE, "hipEventCreate", e);
  hipStream_t cs = nullptr;
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
    return err(ANN_EDEVICE, "hipStreamCreate", e);
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return err(ANN_EDEVICE, "hipStreamBeginCapture", e);
  }
  set_capturing(true);
  s = enqueue_search(ix, g->work, d_queries, nq, d_nprobe, nprobe_max, k, rerank_n, d_out_ids,
                     d_out_dists, cs);
  set_capturing(false);
  e = hipStreamEndCapture(cs, &g->graph);
  (void)hipStreamDestroy(cs);
  if (s != ANN_OK) return s;
  if (e != hipSuccess) return err(ANN_EDEVICE, "hipStreamEndCapture", e);
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
    return err(ANN_EDEVICE, "hipGraphInstantiate", e);
  *out = g.release();
  return ANN_OK;
}

extern "C" ann_status ann_graph_launch(ann_graph* g, void* stream) {
  if (!g) return (ann_status)set_error(ANN_EINVAL, "graph is NULL");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSetDevice(index_device(g->ix));
  if (e != hipSuccess) return err(ANN_EDEVICE, "hipSetDevice", e);
  if (g->launched && (e = hipStreamWaitEvent(st, g->last, 0)) != hipSuccess)
    return err(ANN_EDEVICE, "hipStreamWaitEvent", e);
  if ((e = hipGraphLaunch(g->exec, st)) != hipSuccess) return err(ANN_EDEVICE, "hipGraphLaunch", e);
  if ((e = hipEventRecord(g->last, st)) != hipSuccess) return err(ANN_EDEVICE, "hipEventRecord", e);
  g->launched = true;
  return ANN_OK;
}

extern "C" void ann_graph_free(ann_graph* g) { delete g; }

extern "C" ann_status ann_autotune(ann_index* ix, const float* d_queries, int64_t nq,
                                   const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                                   int32_t rerank_n, int32_t reps, ann_tune_result* out) {
  if (!out) return (ann_status)set_error(ANN_EINVAL, "NULL argument");
  if (reps < 1 || reps > 100) return (ann_status)set_error(ANN_EINVAL, "reps must be in [1, 100]");
  int64_t* ids = nullptr;
  float* dists = nullptr;
  ann_status s = check_search_args(ix, d_queries, nq, nprobe_max, k, rerank_n, d_queries,
                                   d_queries);
  if (s != ANN_OK) return s;
  hipError_t e = hipSetDevice(index_device(ix));
  if (e != hipSuccess) return err(ANN_EDEVICE, "hipSetDevice", e);
  // the options this search may change, restored on error
  const int opts[] = {ANN_OPT_SCAN_TILE, ANN_OPT_SCAN_SPLIT, ANN_OPT_LIST_MAJOR, ANN_OPT_LM_ALPHA,
                      ANN_OPT_LM_TILE, ANN_OPT_LM_BLOCKS, ANN_OPT_LM_MIN_ROWS};
  constexpr int kOpts = 7;
  int64_t saved[kOpts];
  for (int i = 0; i < kOpts; ++i) get_opt(ix, opts[i], &saved[i]);
  hipStream_t st = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  auto cleanup = [&]() {
    if (st) (void)hipStreamSynchronize(st);
    if (ids) (void)hipFree(ids);
    if (dists) (void)hipFree(dists);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (st) (void)hipStreamDestroy(st);
  };
  if ((e = hipMalloc(&ids, (size_t)nq * k * 8)) != hipSuccess ||
      (e = hipMalloc(&dists, (size_t)nq * k * 4)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
    cleanup();
    return err(ANN_ENOMEM, "autotune buffers", e);
  }
  // median of `reps` timed searches after one warm-up, with the options set
  auto time_it = [&](double* med) -> ann_status {
    std::vector<float> t;
    for (int r = 0; r <= reps; ++r) {  // r = 0: warm-up
      (void)hipEventRecord(a, st);
      ann_status s2 = ann_search(ix, d_queries, nq, d_nprobe, nprobe_max, k, rerank_n, ids, dists, st);
      if (s2 != ANN_OK) return s2;
      (void)hipEventRecord(b, st);
      if ((e = hipEventSynchronize(b)) != hipSuccess) return err(ANN_EDEVICE, "autotune run", e);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      if (r > 0) t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    *med = t[t.size() / 2];
    return ANN_OK;
  };
  ann_tune_result best{};
  best.ms = -1.0;
  int tried = 0;
  // 1. the per-query scan's work split
  ann_set_option(ix, ANN_OPT_LIST_MAJOR, 0);
  for (int64_t tile : {4096LL, 8192LL, 16384LL, 32768LL, 65536LL, 131072LL, 1LL << 30}) {
    for (int split : {1, 2, 4, 8, 16}) {
      if (tile == (1LL << 30) && split > 1) continue;  // one item per query whatever the split
      ann_set_option(ix, ANN_OPT_SCAN_TILE, tile);
      ann_set_option(ix, ANN_OPT_SCAN_SPLIT, split);
      double med = 0;
      if ((s = time_it(&med)) != ANN_OK) break;
      ++tried;
      if (best.ms < 0 || med < best.ms) {
        best.tile = tile;
        best.split = split;
        best.ms = med;
      }
    }
    if (s != ANN_OK) break;
  }
  // 2. list-major: its split of each query (alpha, shortest list taken),
  //    rows per work item and persistent blocks, with the best split above
  if (s == ANN_OK && lmajor_supported(index_dev(ix))) {
    ann_set_option(ix, ANN_OPT_SCAN_TILE, best.tile);
    ann_set_option(ix, ANN_OPT_SCAN_SPLIT, best.split);
    ann_set_option(ix, ANN_OPT_LIST_MAJOR, 1);
    int cu = 256;
    (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, index_device(ix));
    const int64_t ncu = std::max(1, cu);
    struct LmCand {
      int alpha, rows, min_rows;
      int64_t blocks;
    };
    std::vector<LmCand> lm;
    if (lmajor_mfma(index_dev(ix))) {  // int8 MFMA groups of 16 (several blocks per CU fit)
      for (int alpha : {1, 2, 4, 8})
        for (int rows : {1024, 4096, 16384})
          for (int64_t blocks : {(int64_t)0, 2 * ncu, 8 * ncu})  // 0: all resident at once
            lm.push_back({alpha, rows, 0, blocks});
    } else {  // tables in LDS: one block per CU; short lists stay per query
      for (int alpha : {1, 2, 8})
        for (int min_rows : {0, 2048, 16384})
          for (int rows : {16384, 1 << 24}) lm.push_back({alpha, rows, min_rows, ncu});
    }
    for (const LmCand& cd : lm) {
      ann_set_option(ix, ANN_OPT_LM_ALPHA, cd.alpha);
      ann_set_option(ix, ANN_OPT_LM_TILE, cd.rows);
      ann_set_option(ix, ANN_OPT_LM_BLOCKS, cd.blocks);
      ann_set_option(ix, ANN_OPT_LM_MIN_ROWS, cd.min_rows);
      double med = 0;
      if ((s = time_it(&med)) != ANN_OK) break;
      ++tried;
      if (med < best.ms) {
        best.list_major = 1;
        best.lm_alpha = cd.alpha;
        best.lm_tile = cd.rows;
        best.lm_blocks = (int32_t)cd.blocks;
        best.lm_min_rows = cd.min_rows;
        best.ms = med;
      }
    }
  }
  cleanup();
  if (s != ANN_OK) {
    for (int i = 0; i < kOpts; ++i) ann_set_option(ix, opts[i], saved[i]);
    return s;
  }
  ann_set_option(ix, ANN_OPT_SCAN_TILE, best.tile);
  ann_set_option(ix, ANN_OPT_SCAN_SPLIT, best.split);
  ann_set_option(ix, ANN_OPT_LIST_MAJOR, best.list_major);
  if (best.list_major) {
    ann_set_option(ix, ANN_OPT_LM_ALPHA, best.lm_alpha);
    ann_set_option(ix, ANN_OPT_LM_TILE, best.lm_tile);
    ann_set_option(ix, ANN_OPT_LM_BLOCKS, best.lm_blocks);
    ann_set_option(ix, ANN_OPT_LM_MIN_ROWS, best.lm_min_rows);
  }
  best.tried = tried;
  *out = best;
  return ANN_OK;
}
