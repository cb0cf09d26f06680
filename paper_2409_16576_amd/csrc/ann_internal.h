// Internal declarations shared by the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct ann_index;

namespace ann {

enum DType : int { F32 = 0, U8 = 1, I8 = 2 };

constexpr int kKsub = 256;
constexpr int kBlock = 256;           // threads per block (all kernels but the scan)
constexpr int kScanBlock = 1024;      // threads per block of the scan kernel
constexpr int kMergeBlock = 1024;     // threads per block of the merge / re-rank kernels
constexpr int kLdsPerCu = 160 * 1024;  // LDS bytes per compute unit (gfx950)
constexpr int kScanRT = 1;            // entries per scan thread per round (one: the top-n
                                      // buffer keeps a round's worth of room, and a smaller
                                      // round leaves more of it between cut-backs)
constexpr int kMaxRerank = 4096;      // largest rerank_n
constexpr int kMaxM = 64;             // largest number of PQ subspaces
constexpr int kMaxDim = 2048;
constexpr int kRankShift = 28;        // replica entry: row | rank << 28
constexpr uint32_t kRowMask = (1u << kRankShift) - 1;

// Device view of a loaded index.  Rows are the vectors reordered by their
// first (nearest) posting list (codes and list data are by row, raw vectors
// by external ID); a list's first-list members are one
// contiguous row range, its other members ("replica entries") are explicit.
struct DevIndex {
  int dtype, dim, nlist, M, row_bytes, dsub, R, int_grid;
  int64_t n;
  // Codes and IDs by row.  Rows n + e (e < replica entries) repeat the row
  // of replica entry e, so a run of replica entries reads its code rows and
  // IDs contiguously instead of gathering them from the vectors' first lists.
  const uint8_t* codes;       // [n + replica entries, row_bytes] PQ codes (M used bytes),
                              // then kCodeSlack zero bytes
  const void* vecs;           // [n, dim] raw vectors by external ID
  const int32_t* row2ext;     // [n + replica entries]
  const float* centroids;     // [nlist, dim]
  const float* centroids_t;   // [dim, nlist]
  const float* codebooks;     // [M, 256, dsub]
  const int32_t* pstart;      // [nlist + 1] first-list row ranges
  const int32_t* rstart;      // [nlist + 1] replica entry ranges
  const int2* rep;            // [replica entries] {row | rank << 28, first list of the vector}
  const int32_t* assign_rows; // [n, R] lists of each row, nearest first, -1 padded
  // integer-grid indexes only (else null): centroids shifted to int8, zero-padded
  const int8_t* cent8;        // [nlist, dim_pad], value - shift8
  const int32_t* cnorm8;      // [nlist] sum of squares of the shifted centroid
  int dim_pad;                // dim rounded up to 64
  int shift8;                 // 128 for uint8, 0 for int8
  const int8_t* cb8;          // [M, 256, dsub] codebooks shifted to int8 (16-byte padded)
  // replica entries of each list grouped by their vector's first list: group s
  // of list l (s in [lseg[l], lseg[l+1])) is {first list, rep begin, rep end, 0}
  const int4* segs;
  const int32_t* lseg;        // [nlist + 1]
  int max_segs;               // most groups of one list
  // host-memory raw tier (vecs is then null): the raw vectors on pages in
  // pinned host memory (device-accessible address), laid out by ann_page_layout
  const uint8_t* hpages;      // [pages, page_bytes]
  const int32_t* vpage;       // [n] page of each vector (by external ID)
  const int32_t* vslot;       // [n] its position on the page
  int page_bytes;
  // navigation graph over the list centroids (null: none); nav_beam > 0 makes
  // step 2 a beam walk of it instead of the exact probe
  const int32_t* nav_adj;     // [nlist, nav_deg] neighbour lists, -1 padded
  const int32_t* nav_entry;   // [nav_nentry] entry vertices
  int nav_deg, nav_nentry, nav_beam;
};

// Working buffers of the list-major pass of the batched form (integer-grid
// indexes; all null when the pass is not used).
struct LmWork {
  int32_t* walkp = nullptr;           // [qc] first probed slot left to the list-major pass
  unsigned long long* thr = nullptr;  // [qc] bound of each query's n-th smallest key
  int32_t* cnt2 = nullptr;            // [qc] keys the list-major pass appended
  uint64_t* out2 = nullptr;           // [qc, cap2] those keys
  uint8_t* flag = nullptr;            // [qc] overflowed: searched by the per-query scan
  int32_t* lcnt = nullptr;            // [nlist] queries per list
  int32_t* lfill = nullptr;           // [nlist]
  int32_t* loff = nullptr;            // [nlist + 1]
  int32_t* ioff = nullptr;            // [nlist + 1] work items per list (prefix)
  int32_t* invq = nullptr;            // [qc * np_max] queries by list
  int32_t* ctr = nullptr;             // [4 + 2 ceil(nlist / 1024)] work items, next item,
                                      // then the work list's per-block totals
  float* lut = nullptr;               // [qc, M, 256] distance tables (float indexes)
  int cap2 = 0;
};

// Tuning of the list-major pass (never changes results).
struct LmCfg {
  int alpha = 2;          // the per-query part walks leading lists up to alpha * n rows
  int tile_rows = 4096;   // first-list rows per work item
  int blocks = 0;         // persistent blocks (0: per compute unit, 4 (MFMA) or 1 (tables))
  int min_rows = 0;       // lists with fewer first-list rows stay with the per-query part
};

// Per-call working buffers (one block of the memory pool).
struct Work {
  float* dist = nullptr;        // [qc, nlist] coarse distances
  int32_t* lists = nullptr;     // [qc, np_max]
  int32_t* np_eff = nullptr;    // [qc]
  float* lut = nullptr;         // [qc, M, 256]
  int32_t* perm = nullptr;      // [qc] scan order of the queries (locality order)
  int32_t* sq = nullptr;        // [qc] work items per query
  uint64_t* pkeys = nullptr;    // [qc, smax, n] partial top-n keys
  int32_t* pcount = nullptr;    // [qc, smax]
  int32_t* pscan = nullptr;     // [qc, smax, 2] candidates scored, entries walked per item
  int32_t* cand = nullptr;      // [qc, n] (rerank-only entry point)
  LmWork lm;                    // list-major pass (batched form)
};

struct LaunchCfg {
  int qc;          // queries in this chunk
  int np_max;
  int n;           // rerank_n (top-n size)
  int k;
  int smax;        // work items per query (max)
  int tile;        // target entries per work item
  bool lut16 = false;  // half-precision distance table in the scan
  bool order = false;  // scan queries in locality order (by nearest list)
  // heuristic re-ranking (Alg. 1): mini-batch size (0: fixed-n re-rank), eps, beta
  int hb = 0;
  double h_eps = 0.0;
  int h_beta = 1;
};

// Kernel launchers (ann_kernels.hip).  All enqueue on `st` and return hipError_t.
hipError_t launch_probe(const DevIndex& ix, const float* q, const int32_t* nprobe, int np_max,
                        int qc, Work& w, float* out_dists_opt, int32_t* out_lists,
                        hipStream_t st);
hipError_t launch_lut(const DevIndex& ix, const float* q, int qc, float* out_lut, hipStream_t st);
// The scan computes each query's distance table itself (step 1 fused).
hipError_t launch_scan(const DevIndex& ix, const int32_t* lists, const int32_t* np_eff,
                       const float* q, const LaunchCfg& c, Work& w, hipStream_t st);
hipError_t launch_scan_trace(const DevIndex& ix, const int32_t* lists, const float* lut, int qc,
                             int np_max, int64_t capacity, int32_t* out_ids, float* out_adc,
                             int64_t* out_count, Work& w, hipStream_t st);
// page_reads (host-memory raw tier only, may be null): pages read per query
hipError_t launch_merge(const DevIndex& ix, const float* q, const LaunchCfg& c, Work& w,
                        int32_t* topn_ids, float* topn_adc, int64_t* ncand, int64_t* nwalk,
                        int64_t* out_ids, float* out_dists, int32_t* reranked,
                        int32_t* page_reads, hipStream_t st);
constexpr int kHostMaxRerank = 2048;  // largest rerank_n with the host-memory raw tier
// Bytes after the last code row: a kernel may read whole dwords up to
// dim_pad / dsub (<= 256) bytes from a row's start.
constexpr int kCodeSlack = 256;
constexpr int kNavMaxBeam = 1024;     // largest beam (and nprobe) of the graph walk
// Batched form on integer-grid indexes: after launch_probe, in place of
// launch_scan (same outputs for launch_merge, one item per query).
bool lmajor_supported(const DevIndex& ix);
bool lmajor_mfma(const DevIndex& ix);  // integer-grid form (else table lookups)
int lmajor_cap2(int n);
// Phases, in order: 0 split and counters, 1 per-query part, 2 work list,
// 3 persistent list-major launch, 4 per-query selection, 5 overflow fallback.
constexpr int kLmPhases = 6;
hipError_t launch_lmajor(const DevIndex& ix, const float* q, const LaunchCfg& c, Work& w,
                         const LmWork& lw, const LmCfg& lc, int num_cu, int phase,
                         hipStream_t st);
hipError_t launch_rerank_only(const DevIndex& ix, const float* q, const int32_t* cand, int qc,
                              int n, int k, int64_t* out_ids, float* out_dists, hipStream_t st);

// Serving-loop helpers (ann_api.cpp): the pipeline of ann_search for one
// chunk of queries on caller-carved working buffers (no allocation).
const DevIndex& index_dev(const ann_index* ix);
int index_device(const ann_index* ix);
// lm_cap2 > 0: include the list-major pass's buffers with that many keys per
// query (the pass runs only when they are there)
size_t work_bytes(const DevIndex& d, int qc, int np_max, int n, int lm_cap2 = 0);  // 256-aligned
Work work_carve(const DevIndex& d, int qc, int np_max, int n, void* base, int lm_cap2 = 0);
// list-major keys per query for this index's options, 0 when the pass is off
// (option unset or the index not supported)
int lmajor_cap(const ann_index* ix, int n);
int search_on(ann_index* ix, Work& w, const float* d_q, int qc, const int32_t* d_nprobe,
              int np_max, int k, int n, int64_t* d_ids, float* d_dists, hipStream_t st);
int max_chunk(const DevIndex& d);  // most queries one search_on call may take
bool set_capturing(bool on);       // this thread records no stage events (graph capture,
                                   // no-alloc calls); returns the previous setting
int get_opt(const ann_index* ix, int option, int64_t* v);

// Allocation-free search (ann_noalloc.cpp): looks up this device's scratch
// array once (the device must be current); called at index load.
int noalloc_setup(int device);

// Records the thread's last error message (ann_last_error) and returns s.
int set_error(int s, const char* fmt, ...);

// Sizes of the dynamic LDS areas (bytes) for the scan kernel.
size_t scan_lds_bytes(const DevIndex& ix, int np_max, int n, bool lut16);
int scan_smax(int n);

}  // namespace ann
