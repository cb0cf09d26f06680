// Allocation-free search (ann_search_noalloc): the plain pipeline of
// ann_search run on a fixed device array instead of the index's memory pool.
//
// The working buffers of a chunk of queries (coarse distances, probed lists,
// per-item top-n keys and counts) are carved from `scratch`, a file-scope
// device array of kScratchBytes.  Host code never passes the array's name to
// a kernel: its device address is looked up once per device with
// hipGetSymbolAddress (at index load, with the index's device current) and
// that address is what the carved buffers point into.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "ann.h"
#include "ann_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;  // 128 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace ann {

// Device address of this device's scratch array; the device must be current.
// Looked up once per device and kept until the process ends.
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return set_error(ANN_EUNSUPPORTED, "device %d: at most %d devices", device, kMaxDevices);
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch_ptr[device]) return ANN_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(ANN_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return ANN_OK;
}

}  // namespace ann

extern "C" size_t ann_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" ann_status ann_search_noalloc(ann_index* ix, const float* d_queries, int64_t nq,
                                         const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                                         int32_t rerank_n, int64_t* d_out_ids, float* d_out_dists,
                                         void* stream) {
  using namespace ann;
  if (!ix) return (ann_status)set_error(ANN_EINVAL, "index is NULL");
  if (nq < 0) return (ann_status)set_error(ANN_EINVAL, "nq < 0");
  if (nq > 0 && !d_queries) return (ann_status)set_error(ANN_EINVAL, "queries pointer is NULL");
  if (nprobe_max < 1 || nprobe_max > 4096)
    return (ann_status)set_error(ANN_EINVAL, "nprobe_max must be in [1, 4096]");
  if (k < 1) return (ann_status)set_error(ANN_EINVAL, "k must be >= 1");
  if (rerank_n < k || rerank_n > kMaxRerank)
    return (ann_status)set_error(ANN_EINVAL, "rerank_n must be in [k, %d]", kMaxRerank);
  if (nq > 0 && (!d_out_ids || !d_out_dists))
    return (ann_status)set_error(ANN_EINVAL, "output pointer is NULL");
  if (nq == 0) return ANN_OK;
  const int dev = index_device(ix);
  if (hipSetDevice(dev) != hipSuccess)
    return (ann_status)set_error(ANN_EDEVICE, "hipSetDevice(%d) failed", dev);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    base = dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr;
  }
  if (!base) return (ann_status)set_error(ANN_EDEVICE, "scratch of device %d not set up", dev);
  const DevIndex& d = index_dev(ix);
  // largest chunk whose working buffers fit the scratch array
  const size_t one = work_bytes(d, 1, nprobe_max, rerank_n);
  if (one > kScratchBytes)
    return (ann_status)set_error(ANN_EINVAL,
                                 "one query needs %zu bytes of working memory; the scratch "
                                 "array holds %zu",
                                 one, kScratchBytes);
  int lo = 1, hi = std::max(1, (int)std::min<int64_t>(nq, max_chunk(d)));
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (work_bytes(d, mid, nprobe_max, rerank_n) <= kScratchBytes) lo = mid;
    else hi = mid - 1;
  }
  const int qc_max = lo;
  Work w = work_carve(d, qc_max, nprobe_max, rerank_n, base);
  hipStream_t st = (hipStream_t)stream;
  const bool was = set_capturing(true);  // no stage-timing events on this path
  int s = ANN_OK;
  for (int64_t q0 = 0; q0 < nq && s == ANN_OK; q0 += qc_max) {
    const int qc = (int)std::min<int64_t>(qc_max, nq - q0);
    s = search_on(ix, w, d_queries + q0 * d.dim, qc, d_nprobe ? d_nprobe + q0 : nullptr,
                  nprobe_max, k, rerank_n, d_out_ids + q0 * k, d_out_dists + q0 * k, st);
  }
  set_capturing(was);
  return (ann_status)s;
}
