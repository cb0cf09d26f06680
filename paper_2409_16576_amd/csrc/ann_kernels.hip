// HIP kernels (gfx950) of the IVF-PQ filtering stage.
//
//   k_probe_dist   step 2: squared distances of each query to every list centroid
//   k_probe_select step 2: the nprobe nearest lists, ascending by (distance, list)
//   k_lut          step 1: per-query distance table, entry = ||q_m - c_{m,j}||^2 (Sec. 2.2)
//   k_scan         steps 1, 3, 5, 6, 7 fused: build the query's table in LDS,
//                  walk the probed lists, drop replica entries owned by an
//                  earlier probed list (dedup), Eq. 1 by table lookups, keep
//                  the n best (distance, id) keys; splits long queries into
//                  work items
//   k_merge        step 7 across a query's work items, then step 8: exact
//                  squared L2 of the n survivors, top-k
//
// Arithmetic contract (what makes the results bit-identical to the CPU
// oracle): every distance that decides a selection is a float32 value that is
// either an exact integer (uint8/int8 data on an integer-grid index: all
// partial sums are integers below 2^24) or a float64 sum over dimensions in
// ascending order, rounded once to float32; the Eq. 1 sum is a float32 sum
// over subspaces m = 0..M-1 in order from +0.0f.  No fused multiply-add is
// formed anywhere in this file.  Selections order by 64-bit keys
// (order-preserving bits of the float32 distance, id), so ties go to the
// lower id.
#pragma clang fp contract(off)

#include <hip/hip_fp16.h>

#include <algorithm>
#include <climits>
#include <type_traits>
#include <utility>

#include "ann_internal.h"

namespace ann {
namespace {

__device__ __forceinline__ uint32_t ord32(float f) {
  const uint32_t b = __float_as_uint(f + 0.0f);  // -0 -> +0
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float unord32(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ float conv_query(float v, int dtype) {
  if (dtype == U8) return fminf(fmaxf(rintf(v), 0.f), 255.f);
  if (dtype == I8) return fminf(fmaxf(rintf(v), -128.f), 127.f);
  return v;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(v, d, 64);
    if (lane_id() >= d) v += t;
  }
  return v;
}

__host__ __device__ inline int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Block-wide selection of the want-th smallest of cnt distinct 64-bit keys
// (MSD radix, 8-bit digits, early exit once the digit bucket holds one key).

struct SelScratch {
  uint32_t hist[256];
  uint64_t prefix;
  uint64_t found;
  uint64_t lo, hi;
  int want;
  int done;
};

template <class G>
__device__ __forceinline__ uint64_t block_kth(G get, int cnt, int want, SelScratch* s,
                                               int min_shift = 0) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    s->want = want;
    s->done = 0;
    s->lo = ~0ull;
    s->hi = 0ull;
  }
  // Bytes shared by every key need no histogram pass: start below them.
  {
    uint64_t lo = ~0ull, hi = 0ull;
    for (int i = tid; i < cnt; i += blockDim.x) {
      const uint64_t k = get(i);
      lo = k < lo ? k : lo;
      hi = k > hi ? k : hi;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      const uint64_t a = __shfl_xor(lo, d, 64), b = __shfl_xor(hi, d, 64);
      lo = a < lo ? a : lo;
      hi = b > hi ? b : hi;
    }
    __syncthreads();
    if ((tid & 63) == 0) {
      atomicMin(&s->lo, lo);
      atomicMax(&s->hi, hi);
    }
    __syncthreads();
  }
  const uint64_t diff = s->lo ^ s->hi;
  if (diff == 0) {  // a single distinct key
    const uint64_t r = s->lo;
    __syncthreads();
    return r;
  }
  const int top_shift = ((63 - __clzll((long long)diff)) / 8) * 8;
  uint64_t mask = top_shift >= 56 ? 0ull : ~((1ull << (top_shift + 8)) - 1ull);
  if (tid == 0) s->prefix = s->lo & mask;
  // digits below min_shift are not resolved (keys equal above it count as one)
  for (int shift = top_shift; shift >= min_shift; shift -= 8) {
    for (int i = tid; i < 256; i += blockDim.x) s->hist[i] = 0;
    __syncthreads();
    const uint64_t prefix = s->prefix;
    // Histogram of the digit.  Keys cluster on few digits (nearby distances
    // share their high bits), so lanes holding the same digit first combine
    // into one atomic per digit (a few rounds), the rest add one by one.
    for (int i0 = 0; i0 < cnt; i0 += blockDim.x) {  // trip count uniform per wave
      const int i = i0 + tid;
      uint64_t k = 0;
      bool act = false;
      if (i < cnt) {
        k = get(i);
        act = (k & mask) == prefix;
      }
      const uint32_t dig = (uint32_t)(k >> shift) & 255u;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        if (act) {
          const uint32_t d = __builtin_amdgcn_readfirstlane(dig);  // first active lane's digit
          const uint64_t same = __ballot(dig == d);                  // active lanes only
          if (dig == d) {
            if ((tid & 63) == __ffsll((unsigned long long)same) - 1)
              atomicAdd(&s->hist[d], (uint32_t)__popcll(same));
            act = false;
          }
        }
      }
      if (act) atomicAdd(&s->hist[dig], 1u);
    }
    __syncthreads();
    const uint32_t w = (uint32_t)s->want;
    if (tid < 64) {
      const uint32_t h0 = s->hist[4 * tid], h1 = s->hist[4 * tid + 1];
      const uint32_t h2 = s->hist[4 * tid + 2], h3 = s->hist[4 * tid + 3];
      const uint32_t sum = h0 + h1 + h2 + h3;
      const uint32_t incl = wave_incl_scan(sum);
      const uint32_t excl = incl - sum;
      if (excl < w && w <= incl) {
        uint32_t r = w - excl;
        int b = 4 * tid;
        uint32_t hb = h0;
        if (r > h0) {
          r -= h0; b += 1; hb = h1;
          if (r > h1) {
            r -= h1; b += 1; hb = h2;
            if (r > h2) { r -= h2; b += 1; hb = h3; }
          }
        }
        s->want = (int)r;
        s->prefix = prefix | ((uint64_t)b << shift);
        s->done = (hb == 1u);
      }
    }
    __syncthreads();
    mask |= (255ull << shift);
    if (s->done) break;
  }
  const uint64_t prefix = s->prefix;
  for (int i = tid; i < cnt; i += blockDim.x) {
    const uint64_t k = get(i);
    if ((k & mask) == prefix) s->found = k;
  }
  __syncthreads();
  const uint64_t r = s->found;
  __syncthreads();
  return r;
}

// Ascending bitonic sort of s[0..p), p a power of two.
// Ascending sort of s[0..p) (p a power of two) by the bitonic network.  The
// stages whose partners lie within 64 consecutive elements run in registers,
// one element per lane, exchanging through cross-lane shuffles, so a block
// barrier is needed only per stage of stride >= 64 and per register pass.
// The caller synchronises before (s complete) and the sort ends with a
// barrier.
__device__ void block_bitonic(uint64_t* s, int p) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // stages (k, j) for k in [k0, k1], j from min(k/2, 32) down to 1, on
  // aligned 64-element blocks (lanes past p carry a sentinel and never store)
  auto regs = [&](int k0, int k1) {
    for (int b0 = w * 64; b0 < p; b0 += nw * 64) {  // wave-uniform
      const int i = b0 + lane;
      uint64_t a = i < p ? s[i] : ~0ull;
      for (int k = k0; k <= k1; k <<= 1)
        for (int j = min(k >> 1, 32); j > 0; j >>= 1) {
          const uint64_t o = __shfl_xor(a, j, 64);
          const bool lower = (i & j) == 0, up = (i & k) == 0;
          a = (lower == up) ? (o < a ? o : a) : (o > a ? o : a);
        }
      if (i < p) s[i] = a;
    }
  };
  regs(2, min(p, 64));
  __syncthreads();
  for (int k = 128; k <= p; k <<= 1) {
    for (int j = k >> 1; j >= 64; j >>= 1) {
      for (int t = threadIdx.x; t < (p >> 1); t += blockDim.x) {
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const uint64_t a = s[i], b = s[i + j];
        if ((a > b) == ((i & k) == 0)) {
          s[i] = b;
          s[i + j] = a;
        }
      }
      __syncthreads();
    }
    regs(k, k);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Step 2a: coarse distances.  One thread per list, QT queries per block; the
// centroids are read transposed so consecutive threads read consecutive
// addresses.  EXACT64: float64 sum over t in order (float data); otherwise
// float32, exact on integer-grid indexes.

constexpr int kProbeQT = 8;

template <bool EXACT64>
__global__ __launch_bounds__(kBlock) void k_probe_dist(DevIndex ix, const float* __restrict__ Q,
                                                        int qc, float* __restrict__ dist) {
  extern __shared__ float s_q[];  // [kProbeQT, dim]
  const int D = ix.dim;
  const int q0 = blockIdx.y * kProbeQT;
  for (int i = threadIdx.x; i < kProbeQT * D; i += kBlock) {
    const int qq = q0 + i / D;
    s_q[i] = qq < qc ? conv_query(Q[(size_t)qq * D + (i % D)], ix.dtype) : 0.f;
  }
  __syncthreads();
  const int l = blockIdx.x * kBlock + threadIdx.x;
  if (l >= ix.nlist) return;
  const float* ct = ix.centroids_t + l;
  if (EXACT64) {
    double acc[kProbeQT];
#pragma unroll
    for (int i = 0; i < kProbeQT; ++i) acc[i] = 0.0;
    for (int t = 0; t < D; ++t) {
      const double c = (double)ct[(size_t)t * ix.nlist];
#pragma unroll
      for (int i = 0; i < kProbeQT; ++i) {
        const double u = (double)s_q[i * D + t] - c;
        const double sq = u * u;
        acc[i] = acc[i] + sq;
      }
    }
#pragma unroll
    for (int i = 0; i < kProbeQT; ++i)
      if (q0 + i < qc) dist[(size_t)(q0 + i) * ix.nlist + l] = (float)acc[i];
  } else {
    float acc[kProbeQT];
#pragma unroll
    for (int i = 0; i < kProbeQT; ++i) acc[i] = 0.f;
    for (int t = 0; t < D; ++t) {
      const float c = ct[(size_t)t * ix.nlist];
#pragma unroll
      for (int i = 0; i < kProbeQT; ++i) {
        const float u = s_q[i * D + t] - c;
        acc[i] = acc[i] + u * u;
      }
    }
#pragma unroll
    for (int i = 0; i < kProbeQT; ++i)
      if (q0 + i < qc) dist[(size_t)(q0 + i) * ix.nlist + l] = acc[i];
  }
}

// Step 2a on integer-grid indexes, as an int8 contraction on the matrix cores:
// ||q - c||^2 = ||q'||^2 + ||c'||^2 - 2 q'.c' with q' = q - s, c' = c - s
// (s = 128 for uint8, 0 for int8) so both operands fit int8; every term is an
// exact int32, hence the float32 result equals the oracle's exact value.
// Block: 64 queries x 256 lists; wave w: all 64 queries x lists
// [64w, 64w + 64) as 4 x 4 tiles of v_mfma_i32_16x16x64_i8 (K = 64 per step).
typedef int v4i_t __attribute__((ext_vector_type(4)));
constexpr int kPM = 64;   // queries per probe block
constexpr int kPN = 256;  // lists per probe block

__global__ __launch_bounds__(kBlock) void k_probe_mfma(DevIndex ix, const float* __restrict__ Q,
                                                        int qc, float* __restrict__ dist) {
  extern __shared__ __align__(16) int8_t s_q8[];  // [kPM, dim_pad] then int32 norms [kPM]
  const int Dp = ix.dim_pad, D = ix.dim;
  int* s_qn = reinterpret_cast<int*>(s_q8 + kPM * Dp);
  const int q0 = blockIdx.y * kPM;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the block's queries as shifted int8: 8 loads in flight per thread (clamped
  // addresses, so no branch sits between them), then the conversions
  constexpr int U = 8;
  for (int i0 = tid; i0 < kPM * Dp; i0 += kBlock * U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kBlock;
      v[u] = Q[(size_t)min(q0 + i / Dp, qc - 1) * D + min(i % Dp, D - 1)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kBlock;
      const int qq = q0 + i / Dp, t = i % Dp;
      if (i < kPM * Dp)
        s_q8[i] = (int8_t)(qq < qc && t < D ? (int)conv_query(v[u], ix.dtype) - ix.shift8 : 0);
    }
  }
  __syncthreads();
  if (tid < kPM) {
    int s = 0;
    for (int t = 0; t < Dp; ++t) {
      const int v = s_q8[tid * Dp + t];
      s += v * v;
    }
    s_qn[tid] = s;
  }
  const int l0 = blockIdx.x * kPN + w * 64;
  const int r16 = lane & 15, g = lane >> 4;
  v4i_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4i_t{0, 0, 0, 0};
  for (int k0 = 0; k0 < Dp; k0 += 64) {
    v4i_t fa[4], fb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      fa[a] = *reinterpret_cast<const v4i_t*>(s_q8 + (a * 16 + r16) * Dp + k0 + 16 * g);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int l = l0 + b * 16 + r16;
      fb[b] = l < ix.nlist
                  ? *reinterpret_cast<const v4i_t*>(ix.cent8 + (size_t)l * Dp + k0 + 16 * g)
                  : v4i_t{0, 0, 0, 0};
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
  }
  __syncthreads();  // s_qn
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int l = l0 + b * 16 + r16;  // output column = lane % 16
    if (l >= ix.nlist) continue;
    const int cn = ix.cnorm8[l];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = a * 16 + 4 * g + r;  // output row = 4 * (lane / 16) + r
        if (q0 + m < qc)
          dist[(size_t)(q0 + m) * ix.nlist + l] = (float)(s_qn[m] + cn - 2 * acc[a][b][r]);
      }
    }
  }
}

// Step 2b: per query, the np smallest (distance, list) keys, sorted.
// Fast path (np <= kBlock): each thread takes the minimum key of its strided
// share of the row; the np-th smallest of those minima is a threshold with at
// least np keys at or below it, usually only a few more.  Those keys are
// collected and sorted.  Otherwise (or if too many keys tie below the
// threshold) a block radix select finds the exact np-th key.
constexpr int kSelCand = 1024;
constexpr int kSelU = 8;

__global__ __launch_bounds__(kBlock) void k_probe_select(const float* __restrict__ dist, int nlist,
                                                          const int32_t* __restrict__ nprobe,
                                                          int np_max, int32_t* __restrict__ lists,
                                                          float* __restrict__ out_d,
                                                          int32_t* __restrict__ np_eff) {
  extern __shared__ __align__(16) uint64_t s_sel[];  // [max(pow2(np_max), kSelCand)]
  __shared__ SelScratch ss;
  __shared__ uint64_t s_min[kBlock];
  __shared__ int s_cnt;
  const int q = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  int np = nprobe ? nprobe[q] : np_max;
  np = max(0, min(np, min(np_max, nlist)));
  const float* row = dist + (size_t)q * nlist;
  auto get = [&](int i) -> uint64_t { return ((uint64_t)ord32(row[i]) << 32) | (uint32_t)i; };
  int P = pow2_at_least(max(np, 1));
  if (np > 0) {
    bool done = false;
    if (np < nlist && np <= kBlock) {
      // both passes load kSelU distances per thread before using any, so a
      // thread has kSelU loads in flight instead of one
      uint64_t mn = ~0ull;
      for (int i0 = tid; i0 < nlist; i0 += kBlock * kSelU) {
        float v[kSelU];
#pragma unroll
        for (int u = 0; u < kSelU; ++u)  // (clamped index: no branch between the loads)
          v[u] = row[min(i0 + u * kBlock, nlist - 1)];
#pragma unroll
        for (int u = 0; u < kSelU; ++u) {
          const int i = i0 + u * kBlock;
          const uint64_t k = ((uint64_t)ord32(v[u]) << 32) | (uint32_t)i;
          if (i < nlist) mn = k < mn ? k : mn;
        }
      }
      s_min[tid] = mn;
      if (tid == 0) s_cnt = 0;
      __syncthreads();
      block_bitonic(s_min, kBlock);
      const uint64_t tau = s_min[np - 1];
      for (int i0 = 0; i0 < nlist; i0 += kBlock * kSelU) {  // block-uniform trip count
        float v[kSelU];
#pragma unroll
        for (int u = 0; u < kSelU; ++u) v[u] = row[min(i0 + u * kBlock + tid, nlist - 1)];
#pragma unroll
        for (int u = 0; u < kSelU; ++u) {
          const int i = i0 + u * kBlock + tid;
          const uint64_t k = ((uint64_t)ord32(v[u]) << 32) | (uint32_t)i;
          const bool take = i < nlist && k <= tau;
          const uint64_t m = __ballot(take);
          if (m) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_cnt, (int)__popcll(m));
            base = __shfl(base, 0, 64);
            const int pos = base + (int)__popcll(m & ((1ull << lane) - 1ull));
            if (take && pos < kSelCand) s_sel[pos] = k;
          }
        }
      }
      __syncthreads();
      const int cnt = s_cnt;
      if (cnt <= kSelCand) {
        P = pow2_at_least(cnt);
        for (int i = cnt + tid; i < P; i += kBlock) s_sel[i] = ~0ull;
        __syncthreads();
        block_bitonic(s_sel, P);
        done = true;
      }
    }
    if (!done) {
      P = pow2_at_least(np);
      const uint64_t K = (np == nlist) ? ~0ull : block_kth(get, nlist, np, &ss);
      if (tid == 0) s_cnt = 0;
      for (int i = np + tid; i < P; i += kBlock) s_sel[i] = ~0ull;
      __syncthreads();
      for (int i = tid; i < nlist; i += kBlock) {
        const uint64_t k = get(i);
        if (k <= K) {
          const int pos = atomicAdd(&s_cnt, 1);
          if (pos < P) s_sel[pos] = k;
        }
      }
      __syncthreads();
      block_bitonic(s_sel, P);
    }
  }
  for (int p = tid; p < np_max; p += kBlock) {
    const bool v = p < np;
    lists[(size_t)q * np_max + p] = v ? (int32_t)(uint32_t)s_sel[p] : -1;
    if (out_d) out_d[(size_t)q * np_max + p] = v ? unord32((uint32_t)(s_sel[p] >> 32)) : INFINITY;
  }
  if (tid == 0) np_eff[q] = np;
}

__global__ void k_zero_i64(int64_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Number of leading non-negative list ids (for caller-provided list arrays).
__global__ void k_count_lists(const int32_t* __restrict__ lists, int qc, int np_max, int nlist,
                              int32_t* __restrict__ np_eff) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= qc) return;
  int c = 0;
  while (c < np_max) {
    const int l = lists[(size_t)q * np_max + c];
    if (l < 0 || l >= nlist) break;
    ++c;
  }
  np_eff[q] = c;
}

// ---------------------------------------------------------------------------
// Step 1: distance table entry [m][j] of one query (qrow = the query's raw
// float32 values).  Integer-grid indexes: float32, exact; otherwise a float64
// sum over t in order, rounded once.

__device__ __forceinline__ float lut_entry(const DevIndex& ix, const float* __restrict__ qrow,
                                           int m, int j) {
  const float* qs = qrow + (size_t)m * ix.dsub;
  const float* c = ix.codebooks + ((size_t)m * kKsub + j) * ix.dsub;
  if (!ix.int_grid) {
    double acc = 0.0;
    for (int t = 0; t < ix.dsub; ++t) {
      const double u = (double)conv_query(qs[t], ix.dtype) - (double)c[t];
      const double sq = u * u;
      acc = acc + sq;
    }
    return (float)acc;
  }
  float acc = 0.f;
  for (int t = 0; t < ix.dsub; ++t) {
    const float u = conv_query(qs[t], ix.dtype) - c[t];
    acc = acc + u * u;
  }
  return acc;
}

// Entry [m][j] from the already converted subvector m of the query (qs),
// same arithmetic and order as lut_entry.
__device__ __forceinline__ float lut_entry_conv(const DevIndex& ix, const float* qs, int m, int j) {
  const float* c = ix.codebooks + ((size_t)m * kKsub + j) * ix.dsub;
  if (!ix.int_grid) {
    double acc = 0.0;
    for (int t = 0; t < ix.dsub; ++t) {
      const double u = (double)qs[t] - (double)c[t];
      const double sq = u * u;
      acc = acc + sq;
    }
    return (float)acc;
  }
  float acc = 0.f;
  for (int t = 0; t < ix.dsub; ++t) {
    const float u = qs[t] - c[t];
    acc = acc + u * u;
  }
  return acc;
}

// The same with dsub a multiple of 4: the codeword is read as float4 vectors.
__device__ __forceinline__ float lut_entry_v4(const DevIndex& ix, const float* qs, int m, int j) {
  const float4* c4 = reinterpret_cast<const float4*>(ix.codebooks + ((size_t)m * kKsub + j) * ix.dsub);
  if (!ix.int_grid) {
    double acc = 0.0;
    auto add = [&](float qv, float cv) {
      const double u = (double)qv - (double)cv;
      const double sq = u * u;
      acc = acc + sq;
    };
    for (int t4 = 0; t4 < ix.dsub / 4; ++t4) {
      const float4 c = c4[t4];
      const float* qq = qs + 4 * t4;
      add(qq[0], c.x); add(qq[1], c.y); add(qq[2], c.z); add(qq[3], c.w);
    }
    return (float)acc;
  }
  float acc = 0.f;
  auto add = [&](float qv, float cv) {
    const float u = qv - cv;
    acc = acc + u * u;
  };
  for (int t4 = 0; t4 < ix.dsub / 4; ++t4) {
    const float4 c = c4[t4];
    const float* qq = qs + 4 * t4;
    add(qq[0], c.x); add(qq[1], c.y); add(qq[2], c.z); add(qq[3], c.w);
  }
  return acc;
}

// The entry of a 4-dimensional subspace from its codeword c (same arithmetic
// and order as lut_entry_v4).
__device__ __forceinline__ float lut_entry_d4(const DevIndex& ix, const float* qs, float4 c) {
  if (!ix.int_grid) {
    double acc = 0.0;
    const double u0 = (double)qs[0] - (double)c.x, u1 = (double)qs[1] - (double)c.y;
    const double u2 = (double)qs[2] - (double)c.z, u3 = (double)qs[3] - (double)c.w;
    const double s0 = u0 * u0, s1 = u1 * u1, s2 = u2 * u2, s3 = u3 * u3;
    acc = acc + s0;
    acc = acc + s1;
    acc = acc + s2;
    acc = acc + s3;
    return (float)acc;
  }
  const float u0 = qs[0] - c.x, u1 = qs[1] - c.y, u2 = qs[2] - c.z, u3 = qs[3] - c.w;
  float acc = 0.f;
  acc = acc + u0 * u0;
  acc = acc + u1 * u1;
  acc = acc + u2 * u2;
  acc = acc + u3 * u3;
  return acc;
}

// One block per query, thread = codeword, loop over subspaces.
__global__ __launch_bounds__(kBlock) void k_lut(DevIndex ix, const float* __restrict__ Q, int qc,
                                                 float* __restrict__ lut) {
  const int q = blockIdx.x, j = threadIdx.x;
  const float* qrow = Q + (size_t)q * ix.dim;
  for (int m = 0; m < ix.M; ++m) lut[((size_t)q * ix.M + m) * kKsub + j] = lut_entry(ix, qrow, m, j);
}

// ---------------------------------------------------------------------------
// Steps 3, 5, 6, 7: the fused scan.

// A query's gathered entries are enumerated as "runs": per probed list, its
// first-list rows (one contiguous row range) and its replica entries.  With
// segmented replicas, a list's replica entries are grouped by their vector's
// first list and only groups whose first list is NOT probed become runs (the
// others are all duplicates of entries scanned from that first list).
struct ScanLayout {
  size_t lut, bits, list, rstart, pre, buf, tmp, sel, misc, total;
};

// Most runs a query can have: per probed list, one row run plus one run per
// replica group (segmented) or one replica run (not segmented).
__host__ __device__ inline int scan_max_runs(int np_max, int max_segs, bool segmented) {
  return np_max * (1 + (segmented ? max_segs : 1));
}

// The scan's set of a query's probed lists (for the ownership rule): a
// bitmap over all lists while that is small, else the probed lists sorted
// ascending (membership by halving), so that large list counts leave the
// LDS to the run slots.
__host__ __device__ inline bool probe_set_sorted(int nlist, int np_max) {
  const int words = (nlist + 31) / 32;
  return words > 512 && words > np_max;
}

__host__ __device__ inline ScanLayout scan_layout(int M, int nlist, int R, int np_max,
                                                  int max_runs, int cap, int lut_elem) {
  ScanLayout L;
  size_t o = 0;
  L.lut = o; o += (size_t)M * kKsub * lut_elem; o = align_up(o, 16);
  L.bits = o;
  o += R > 1 ? (probe_set_sorted(nlist, np_max) ? (size_t)pow2_at_least(np_max) * 4
                                                : (size_t)((nlist + 31) / 32) * 4)
             : 0;
  o = align_up(o, 16);
  L.list = o; o += (size_t)np_max * 4; o = align_up(o, 16);
  L.rstart = o; o += (size_t)max_runs * 4; o = align_up(o, 16);
  L.pre = o; o += (size_t)(max_runs + 1) * 4; o = align_up(o, 16);
  L.buf = o; o += (size_t)cap * 8; o = align_up(o, 16);
  L.tmp = o; o += (size_t)(kScanBlock / 64 + 1) * 4; o = align_up(o, 16);  // per-wave sums + total
  L.sel = o; o += sizeof(SelScratch); o = align_up(o, 16);
  L.misc = o; o += 32;
  L.total = align_up(o, 16);
  return L;
}

struct ScanMisc {
  uint64_t thr;
  int count;
  int ncount;
  int scanned;
  int done;  // waves that have walked all their entries
  int seg;   // the query's replica entries are laid out as surviving groups
};

// Exclusive prefix sum of v over the block (in thread order); s_wsum holds
// one int per wave.  All threads must call.
__device__ __forceinline__ int block_excl_scan(int v, int* s_wsum) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) s_wsum[wv] = incl;
  __syncthreads();
  int before = 0;
  for (int i = 0; i < wv; ++i) before += s_wsum[i];
  (void)nw;
  return before + incl - v;
}

__device__ __forceinline__ bool testbit(const uint32_t* bits, int l) {
  return (bits[l >> 5] >> (l & 31)) & 1u;
}

// (probed lists up to 2^13 for the sorted form: nprobe is at most 4096)
struct ProbeSet {
  const uint32_t* bits;  // bitmap over all lists, or
  const int32_t* set;    // the probed lists ascending, padded with INT_MAX to p2
  int p2;                // a power of two >= the probed lists
  __device__ __forceinline__ bool has(int l) const {
    if (!set) return testbit(bits, l);
    // branchless lower bound with a fixed number of steps, so that several
    // lookups of a thread can overlap their LDS reads
    int pos = 0;
#pragma unroll
    for (int step = 4096; step >= 1; step >>= 1)
      if (step < p2 && set[pos + step - 1] < l) pos += step;
    return set[pos] == l;
  }
};

// Code row -> W dwords (natural alignment: rows are 4*W bytes apart).
template <int W>
__device__ __forceinline__ void load_row(const uint8_t* __restrict__ rowp, uint32_t (&w)[W]) {
  if constexpr (W % 4 == 0) {
#pragma unroll
    for (int i = 0; i < W / 4; ++i) {
      const uint4 v = reinterpret_cast<const uint4*>(rowp)[i];
      w[4 * i] = v.x; w[4 * i + 1] = v.y; w[4 * i + 2] = v.z; w[4 * i + 3] = v.w;
    }
  } else if constexpr (W % 2 == 0) {
#pragma unroll
    for (int i = 0; i < W / 2; ++i) {
      const uint2 v = reinterpret_cast<const uint2*>(rowp)[i];
      w[2 * i] = v.x; w[2 * i + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = reinterpret_cast<const uint32_t*>(rowp)[i];
  }
}

__device__ __forceinline__ float lut_val(float v) { return v; }
__device__ __forceinline__ float lut_val(__half v) { return __half2float(v); }  // exact

// Eq. 1 for one code row: float32 sum over m = 0..M-1 in order.  The table
// holds float32 entries, or binary16 entries (the half-precision variant,
// widened exactly before the float32 sum).
// Byte B of w times sizeof(T), the code's byte offset inside its subspace's
// table: one VALU instruction (sub-dword operand select) instead of a
// bit-field extract and a shift.  The scan issues one per code, so this is
// most of its address arithmetic.
#define ANN_BYTE_SCALED(SH, B)                                                            \
  asm("v_lshlrev_b32_sdwa %0, " #SH ", %1 dst_sel:DWORD dst_unused:UNUSED_PAD "         \
      "src0_sel:DWORD src1_sel:BYTE_" #B                                                   \
      : "=v"(r)                                                                           \
      : "v"(w))
template <class T, int B>
__device__ __forceinline__ uint32_t code_offset(uint32_t w) {
  uint32_t r;
  if constexpr (sizeof(T) == 4) {
    if constexpr (B == 0) ANN_BYTE_SCALED(2, 0);
    else if constexpr (B == 1) ANN_BYTE_SCALED(2, 1);
    else if constexpr (B == 2) ANN_BYTE_SCALED(2, 2);
    else ANN_BYTE_SCALED(2, 3);
  } else {
    if constexpr (B == 0) ANN_BYTE_SCALED(1, 0);
    else if constexpr (B == 1) ANN_BYTE_SCALED(1, 1);
    else if constexpr (B == 2) ANN_BYTE_SCALED(1, 2);
    else ANN_BYTE_SCALED(1, 3);
  }
  return r;
}
#undef ANN_BYTE_SCALED

template <class T, int B>
__device__ __forceinline__ float table_at(const T* __restrict__ s_lut, int m, uint32_t w) {
  const char* base = reinterpret_cast<const char*>(s_lut) + (size_t)m * kKsub * sizeof(T);
  return lut_val(*reinterpret_cast<const T*>(base + code_offset<T, B>(w)));
}

template <int W, class T>
__device__ __forceinline__ float adc_words(const uint32_t (&w)[W], const T* __restrict__ s_lut,
                                           int M) {
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const int m = 4 * i;
    if (i < W - 1 || m < M) acc = acc + table_at<T, 0>(s_lut, m, w[i]);
    if (i < W - 1 || m + 1 < M) acc = acc + table_at<T, 1>(s_lut, m + 1, w[i]);
    if (i < W - 1 || m + 2 < M) acc = acc + table_at<T, 2>(s_lut, m + 2, w[i]);
    if (i < W - 1 || m + 3 < M) acc = acc + table_at<T, 3>(s_lut, m + 3, w[i]);
  }
  return acc;
}

// Reduce s_buf[0..count) to its n smallest keys; threshold = the n-th key.
// In place: each thread stages a contiguous chunk of the buffer in registers,
// the survivors' positions come from a block prefix sum, and every survivor
// moves to a position no later than its own (all reads precede all writes).
constexpr int kCompactChunk = 8;  // cap <= kCompactChunk * kScanBlock

// loose: keep every key whose distance is at most the n-th smallest distance
// (n or a few more keys: ties at that distance are not broken by id), which
// resolves only the distance half of the keys; the threshold stays valid (it
// is never below the n-th smallest key).  Exact: keep exactly the n smallest.
// Returns the buffer's count afterwards, the same value in every thread (read
// between two barriers, before any wave can insert again).  Call with every
// wave of the block present and none inserting.
__device__ __forceinline__ int scan_compact(uint64_t* s_buf, int* s_wsum, SelScratch* ss, ScanMisc* mc, int n,
                                            bool loose = false) {
  const int cnt = mc->count;
  if (cnt <= n) return cnt;
  const uint64_t K =
      loose ? (block_kth([&](int i) { return s_buf[i] & 0xffffffff00000000ull; }, cnt, n, ss, 32) |
               0xffffffffull)
            : block_kth([&](int i) { return s_buf[i]; }, cnt, n, ss);
  const int ch = (cnt + (int)blockDim.x - 1) / (int)blockDim.x;
  const int b0 = threadIdx.x * ch;
  uint64_t r[kCompactChunk];
  int c = 0;
#pragma unroll
  for (int i = 0; i < kCompactChunk; ++i) {
    uint64_t k = ~0ull;
    if (i < ch && b0 + i < cnt) {
      k = s_buf[b0 + i];
      if (k > K) k = ~0ull;
    }
    r[i] = k;
    c += k != ~0ull ? 1 : 0;
  }
  int pos = block_excl_scan(c, s_wsum);  // contains a barrier: all reads are done
  if (threadIdx.x == blockDim.x - 1) mc->ncount = pos + c;  // survivors
#pragma unroll
  for (int i = 0; i < kCompactChunk; ++i)
    if (r[i] != ~0ull) s_buf[pos++] = r[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    mc->count = mc->ncount;
    mc->thr = K;
  }
  __syncthreads();
  const int out = mc->count;
  __syncthreads();
  return out;
}

// One block = one work item (a contiguous range of one query's gathered
// entries).  Each round, every thread takes kScanRT entries (stride
// kScanBlock), resolves them to code rows, issues all row loads, then scores
// them; keys below the current threshold go to the LDS buffer, which is cut
// back to the n best whenever it holds more than n.
constexpr uint32_t kRunReplica = 0x80000000u;  // run start flag: replica-entry run

// Splitting a query's entries between the per-query scan and the list-major
// pass of the batched form (defaults: the whole query here).
//   walkp    [qc] probed slots >= walkp[q] leave the first-list rows of their
//            lists (those with at least min_rows of them) to the list-major
//            pass; replica entries of every probed list are walked here
//   active   [qc] nonzero: scan this query; zero: the block does nothing
//   thr_out  [qc] atomically lowered to each item's n-th smallest key
struct ScanSplit {
  const int32_t* walkp = nullptr;
  const uint8_t* active = nullptr;
  unsigned long long* thr_out = nullptr;
  int min_rows = 0;
};

// Whether probed slot p of a query (list with `rows` first-list rows) leaves
// those rows to the list-major pass.
__host__ __device__ inline bool lm_slot(int p, int walkp, int rows, int min_rows) {
  return p >= walkp && rows > 0 && rows >= min_rows;
}

// Runs of up to 64 probed lists laid out by one wave (lane p: list p): run
// starts in s_rstart, exclusive entry offsets in s_pre[0..nruns], and
// s_pre[nruns] = the query's entries; *s_nruns = nruns, *s_seg = whether the
// replica runs are surviving groups.
__device__ __forceinline__ void runs_wave(const DevIndex& ix, const int32_t* s_list, int np,
                          int walk_np, int min_rows, const ProbeSet& ps, int segmented,
                          int max_runs, uint32_t* s_rstart, int32_t* s_pre, int* s_nruns,
                          int* s_seg) {
  const int lane = threadIdx.x & 63;
  int cnt = 0, l = 0, s0 = 0, s1 = 0;
  // group descriptors are read kSegU at a time, their loads in flight together
  constexpr int kSegU = 8;
  if (lane < np) {
    l = s_list[lane];
    cnt = 1;
    if (segmented) {
      s0 = ix.lseg[l];
      s1 = ix.lseg[l + 1];
      for (int s = s0; s < s1; s += kSegU) {
        int fl[kSegU];
#pragma unroll
        for (int u = 0; u < kSegU; ++u) fl[u] = s + u < s1 ? ix.segs[s + u].x : -1;
#pragma unroll
        for (int u = 0; u < kSegU; ++u) cnt += (fl[u] >= 0 && !ps.has(fl[u])) ? 1 : 0;
      }
    }
  }
  int incl = (int)wave_incl_scan((uint32_t)cnt);
  int nruns = __shfl(incl, 63, 64);
  // groups that survive go in as runs of their own while they fit; otherwise
  // each list's replica entries form one run, tested entry by entry
  const bool seg = segmented && nruns <= max_runs;  // wave-uniform
  if (!seg) {
    cnt = lane < np ? 1 + (ix.rstart[l + 1] > ix.rstart[l] ? 1 : 0) : 0;
    incl = (int)wave_incl_scan((uint32_t)cnt);
    nruns = __shfl(incl, 63, 64);
  }
  if (lane < np) {
    const int off = incl - cnt;
    s_rstart[off] = (uint32_t)ix.pstart[l];
    // entry counts first; first-list rows left to the list-major pass make an
    // empty run
    const int rows = ix.pstart[l + 1] - ix.pstart[l];
    s_pre[off] = lm_slot(lane, walk_np, rows, min_rows) ? 0 : rows;
    int r = off + 1;
    if (seg) {
      for (int s = s0; s < s1; s += kSegU / 2) {
        int4 gg[kSegU / 2];
#pragma unroll
        for (int u = 0; u < kSegU / 2; ++u)
          gg[u] = s + u < s1 ? ix.segs[s + u] : make_int4(-1, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < kSegU / 2; ++u) {
          if (gg[u].x >= 0 && !ps.has(gg[u].x)) {
            s_rstart[r] = (uint32_t)gg[u].y | kRunReplica;
            s_pre[r] = gg[u].z - gg[u].y;
            ++r;
          }
        }
      }
    } else if (cnt > 1) {
      s_rstart[r] = (uint32_t)ix.rstart[l] | kRunReplica;
      s_pre[r] = ix.rstart[l + 1] - ix.rstart[l];
    }
  }
  __threadfence_block();  // other lanes read these counts below
  int total = 0;
  for (int r0 = 0; r0 < nruns; r0 += 64) {
    const int r = r0 + lane;
    const int c = r < nruns ? s_pre[r] : 0;
    const int in = (int)wave_incl_scan((uint32_t)c);
    if (r < nruns) s_pre[r] = total + in - c;
    total += __shfl(in, 63, 64);
  }
  if (lane == 0) {
    s_pre[nruns] = total;
    *s_nruns = nruns;
    *s_seg = seg ? 1 : 0;
  }
}

template <int W, bool TRACE, bool H>
__global__ __launch_bounds__(kScanBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_scan(
    DevIndex ix, const int32_t* __restrict__ lists, const int32_t* __restrict__ np_eff, int np_max,
    int qc, const float* __restrict__ Q, const float* __restrict__ lut,
    int32_t* __restrict__ sq, int smax, int tile, int segmented, int max_runs, int n, int cap,
    uint64_t* __restrict__ pkeys, int32_t* __restrict__ pcount, int32_t* __restrict__ pscan,
    const int32_t* __restrict__ perm, int64_t t_capacity, int32_t* __restrict__ t_ids, float* __restrict__ t_adc,
    unsigned long long* __restrict__ t_count, ScanSplit sp) {
  // Block -> (query, item).  Blocks are dispatched round-robin over the 8
  // XCDs (each with its own L2): block b runs on XCD b % 8.  With a locality
  // order, XCD x takes the contiguous share x of the ordered queries, so the
  // queries running side by side on one XCD probe overlapping lists; all
  // items of a query stay on one XCD.
  const int b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int j = slot % smax;
  int q;
  if (perm) {
    const int per = (qc + 7) / 8;
    const int pos = xcd * per + slot / smax;
    if (slot / smax >= per || pos >= qc) return;
    q = perm[pos];
  } else {
    q = (slot / smax) * 8 + xcd;
    if (q >= qc) return;
  }
  if (sp.active && !sp.active[q]) return;  // only the flagged queries (block-uniform)
  const int tid = threadIdx.x;
  const int M = ix.M;

  extern __shared__ __align__(16) unsigned char smem[];
  using LutT = std::conditional_t<H, __half, float>;
  // The table is a static array sized for 4W subspaces, so its LDS address
  // is a compile-time constant: every lookup's subspace offset folds into the
  // load's immediate field and the code byte's offset is its whole address.
  __shared__ __align__(16) LutT s_lut_st[4 * W * kKsub];
  const ScanLayout L = scan_layout(M, ix.nlist, ix.R, np_max, max_runs, cap, 0);
  LutT* s_lut = s_lut_st;
  uint32_t* s_bits = reinterpret_cast<uint32_t*>(smem + L.bits);
  int32_t* s_list = reinterpret_cast<int32_t*>(smem + L.list);
  uint32_t* s_rstart = reinterpret_cast<uint32_t*>(smem + L.rstart);
  int32_t* s_pre = reinterpret_cast<int32_t*>(smem + L.pre);
  uint64_t* s_buf = reinterpret_cast<uint64_t*>(smem + L.buf);
  int* s_wsum = reinterpret_cast<int*>(smem + L.tmp);
  SelScratch* ss = reinterpret_cast<SelScratch*>(smem + L.sel);
  ScanMisc* mc = reinterpret_cast<ScanMisc*>(smem + L.misc);

  // Probed lists and their set (bitmap, or sorted for large list counts).
  const int nwords = (ix.nlist + 31) / 32;
  const bool use_bits = ix.R > 1;
  const bool sorted_set = probe_set_sorted(ix.nlist, np_max);
  if (use_bits && !sorted_set)
    for (int i = tid; i < nwords; i += kScanBlock) s_bits[i] = 0u;
  const int np = np_eff[q];
  const int walk_np = sp.walkp ? min(np, sp.walkp[q]) : np;  // slots walked whole
  for (int p = tid; p < np; p += kScanBlock) s_list[p] = lists[(size_t)q * np_max + p];
  if (tid == 0) {
    mc->thr = ~0ull;
    mc->count = 0;
    mc->scanned = 0;
    mc->done = 0;
  }
  // The distance table is computed here (step 1 fused into the scan) unless
  // the caller passed one in; the converted query is staged in the (still
  // unused) top-n buffer so every table entry reads it from LDS.
  const bool own_table = !TRACE;
  float* s_qv = reinterpret_cast<float*>(s_buf);  // dim floats <= cap keys
  if (own_table)
    for (int t = tid; t < ix.dim; t += kScanBlock)
      s_qv[t] = conv_query(Q[(size_t)q * ix.dim + t], ix.dtype);
  __syncthreads();
  if (use_bits) {
    if (sorted_set) {  // rank of each probed list among them (lists are distinct)
      int32_t* s_set = reinterpret_cast<int32_t*>(s_bits);
      for (int p = tid; p < np; p += kScanBlock) {
        const int l = s_list[p];
        int r = 0;
        for (int j = 0; j < np; ++j) r += s_list[j] < l ? 1 : 0;
        s_set[r] = l;
      }
      for (int p = np + tid; p < pow2_at_least(max(np, 1)); p += kScanBlock) s_set[p] = INT_MAX;
    } else {
      for (int p = tid; p < np; p += kScanBlock) {
        const int l = s_list[p];
        atomicOr(&s_bits[l >> 5], 1u << (l & 31));
      }
    }
  }
  __syncthreads();
  const ProbeSet ps{s_bits, sorted_set ? reinterpret_cast<const int32_t*>(s_bits) : nullptr,
                    pow2_at_least(max(np, 1))};

  // Table entry i of the query (or its copy from the caller's table).
  auto table_entry = [&](int i) {
    if constexpr (H) {
      const int m = i >> 8;
      const float* qs = s_qv + m * ix.dsub;
      const float e = ix.dsub % 4 == 0 ? lut_entry_v4(ix, qs, m, i & 255)
                                       : lut_entry_conv(ix, qs, m, i & 255);
      s_lut[i] = __float2half_rn(e);  // half-precision variant: nearest binary16, ties to even
    } else if (TRACE) {  // the trace form takes the caller's table
      s_lut[i] = lut[(size_t)q * M * kKsub + i];
    } else {
      const int m = i >> 8;
      const float* qs = s_qv + m * ix.dsub;
      s_lut[i] = ix.dsub % 4 == 0 ? lut_entry_v4(ix, qs, m, i & 255)
                                  : lut_entry_conv(ix, qs, m, i & 255);
    }
  };

  // Table entries i0, i0 + stride, ...: with 4-dimensional subspaces the
  // codewords of four entries are loaded before any is computed.
  auto build_table = [&](int i0, int stride) {
    const int total = M * kKsub;
    if (!TRACE && ix.dsub == 4) {
      const float4* cb4 = reinterpret_cast<const float4*>(ix.codebooks);
      for (int i = i0; i < total; i += 4 * stride) {
        float4 c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = i + u * stride;
          c[u] = k < total ? cb4[k] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = i + u * stride;
          if (k < total) {
            const float e = lut_entry_d4(ix, s_qv + (k >> 8) * 4, c[u]);
            if constexpr (H) s_lut[k] = __float2half_rn(e);  // nearest binary16, ties to even
            else s_lut[k] = e;
          }
        }
      }
    } else {
      for (int i = i0; i < total; i += stride) table_entry(i);
    }
  };

  // Runs of every probed list (slot order), then their entry prefix sums.
  // Up to 64 probed lists: wave 0 lays the runs out (one list per lane) while
  // the other waves build the table; otherwise the whole block does both in turn.
  int nruns = 0;
  const bool wave_setup = np <= 64;
  if (wave_setup) {
    if (tid < 64) {
      runs_wave(ix, s_list, np, walk_np, sp.min_rows, ps, segmented, max_runs, s_rstart,
                s_pre, &s_wsum[kScanBlock / 64], &mc->seg);
    } else {
      build_table(tid - 64, kScanBlock - 64);
    }
    __syncthreads();
    nruns = s_wsum[kScanBlock / 64];
  }
  bool seg = segmented != 0;  // as in runs_wave: surviving groups as runs while they fit
  bool seg_all;
  if (!wave_setup && seg) {
    int tot = 0;
    for (int p0 = 0; p0 < np; p0 += kScanBlock) {  // uniform trip count
      const int p = p0 + tid;
      int cnt = 0;
      if (p < np) {
        const int l = s_list[p];
        cnt = 1;
        for (int s = ix.lseg[l]; s < ix.lseg[l + 1]; ++s) cnt += ps.has(ix.segs[s].x) ? 0 : 1;
      }
      const int off = block_excl_scan(cnt, s_wsum);
      if (tid == kScanBlock - 1) s_wsum[kScanBlock / 64] = off + cnt;
      __syncthreads();
      tot += s_wsum[kScanBlock / 64];
      __syncthreads();
    }
    seg = tot <= max_runs;
  }
  if (!wave_setup) seg_all = seg;
  else seg_all = mc->seg != 0;  // runs_wave's decision (read after its barrier)
  // With at most two lists per vector, every entry of a surviving group is
  // kept (its vector's only earlier list is the group's, not probed), so
  // the entries themselves need not be read.
  const bool grp = seg_all && ix.R == 2;
  for (int p0 = 0; !wave_setup && p0 < np; p0 += kScanBlock) {  // uniform trip count
    const int p = p0 + tid;
    int cnt = 0, l = 0;
    if (p < np) {
      l = s_list[p];
      cnt = 1;
      if (seg) {
        for (int s = ix.lseg[l]; s < ix.lseg[l + 1]; ++s) cnt += ps.has(ix.segs[s].x) ? 0 : 1;
      } else {
        cnt += ix.rstart[l + 1] > ix.rstart[l] ? 1 : 0;
      }
    }
    const int off = nruns + block_excl_scan(cnt, s_wsum);
    if (p < np) {
      s_rstart[off] = (uint32_t)ix.pstart[l];
      // entry count, turned into offsets below (empty when left to the
      // list-major pass, as in runs_wave)
      const int rows = ix.pstart[l + 1] - ix.pstart[l];
      s_pre[off] = lm_slot(p, walk_np, rows, sp.min_rows) ? 0 : rows;
      int r = off + 1;
      if (seg) {
        for (int s = ix.lseg[l]; s < ix.lseg[l + 1]; ++s) {
          const int4 g = ix.segs[s];
          if (!ps.has(g.x)) {
            s_rstart[r] = (uint32_t)g.y | kRunReplica;
            s_pre[r] = g.z - g.y;
            ++r;
          }
        }
      } else if (cnt > 1) {
        s_rstart[r] = (uint32_t)ix.rstart[l] | kRunReplica;
        s_pre[r] = ix.rstart[l + 1] - ix.rstart[l];
      }
    }
    if (tid == kScanBlock - 1) s_wsum[kScanBlock / 64] = off + cnt;  // running total
    __syncthreads();
    nruns = s_wsum[kScanBlock / 64];
    __syncthreads();
  }
  // entry counts -> exclusive offsets (runs are at most a few thousand)
  int total = wave_setup ? s_pre[nruns] : 0;
  for (int r0 = 0; !wave_setup && r0 < nruns; r0 += kScanBlock) {
    const int r = r0 + tid;
    const int c = r < nruns ? s_pre[r] : 0;
    const int off = total + block_excl_scan(c, s_wsum);
    if (tid == kScanBlock - 1) s_wsum[kScanBlock / 64] = off + c;
    __syncthreads();
    if (r < nruns) s_pre[r] = off;
    total = s_wsum[kScanBlock / 64];
    __syncthreads();
  }
  if (!wave_setup && tid == 0) s_pre[nruns] = total;

  // Work items of this query: ceil(E / tile), at most smax.
  const int E = total;
  const int S = (int)max(1, min(smax, (E + tile - 1) / tile));
  if (j == 0 && tid == 0) sq[q] = S;
  if (j >= S) return;

  if (!wave_setup) {
    build_table(tid, kScanBlock);
    __syncthreads();
  }

  const int e0 = (int)((int64_t)E * j / S), e1 = (int)((int64_t)E * (j + 1) / S);
  const int lane = tid & 63;
  const uint64_t lanemask = (1ull << lane) - 1ull;
  int scanned = 0;
  int cur = 0;  // run of this thread's current entry (entries only increase)
  int run_lo = 0, run_hi = -1;  // entries [run_lo, run_hi) of run cur (none yet)
  uint32_t run_rs = 0;
  // Each wave walks its part of every round (kScanRT entries per lane) at its
  // own pace; the block meets only when some wave has seen the buffer above
  // T = cap - kRound, or has finished.  A wave inserts at most kScanRT * 64
  // keys per round and checks the count after each round, so once the count
  // passes T every wave adds at most one more round before it meets: the
  // count never exceeds cap.  At a meeting the decision (cut back? all
  // done?) is read between two barriers, so every wave takes the same path
  // and every meeting is reached by every wave.
  constexpr int kRound = kScanBlock * kScanRT;
  const int T = cap - kRound;
  int base = e0;
  bool wdone = base >= e1;
  bool counted = false;

  for (;;) {
    if (!wdone) {
      const uint64_t thr = mc->thr;
      const uint32_t thr_hi = (uint32_t)(thr >> 32);
      int rows[kScanRT];
      bool keep[kScanRT];
      // resolve entries -> rows; replica entries owned by an earlier probed list are dropped
#pragma unroll
      for (int u = 0; u < kScanRT; ++u) {
        const int e = base + u * kScanBlock + tid;
        keep[u] = false;
        rows[u] = 0;
        if (e < e1) {
          if (e >= run_hi) {
            // the run holding e: the last r in [cur, nruns) with s_pre[r] <= e
            // (s_pre[nruns] = E > e); a step or two linearly, else by halving
            if (s_pre[cur + 1] <= e) {
              ++cur;
              if (s_pre[cur + 1] <= e) {
                int lo = cur + 1, hi = nruns;  // s_pre[lo] <= e < s_pre[hi]
                while (hi - lo > 1) {
                  const int mid = (lo + hi) >> 1;
                  if (s_pre[mid] <= e) lo = mid;
                  else hi = mid;
                }
                cur = lo;
              }
            }
            run_lo = s_pre[cur];
            run_hi = s_pre[cur + 1];
            run_rs = s_rstart[cur];
          }
          const int o = e - run_lo;
          const uint32_t rs = run_rs;
          if (!(rs & kRunReplica)) {
            rows[u] = (int)rs + o;
            keep[u] = true;
          } else {
            // replica entry ei: its code row and ID are row n + ei
            const int ei = (int)(rs & ~kRunReplica) + o;
            bool k = true;
            if (!grp) {
              const int2 r = ix.rep[ei];
              const int row = (int)((uint32_t)r.x & kRowMask);
              const int rank = (int)((uint32_t)r.x >> kRankShift);
              k = !ps.has(r.y);
              for (int i = 1; i < rank && k; ++i)
                k = !ps.has(ix.assign_rows[(size_t)row * ix.R + i]);
            }
            rows[u] = (int)ix.n + ei;
            keep[u] = k;
          }
        }
      }
      // all code-row loads of the round in flight together (an entry not
      // kept reads row 0, a valid row whose sum is then ignored)
      uint32_t cw[kScanRT][W];
#pragma unroll
      for (int u = 0; u < kScanRT; ++u)
        load_row<W>(ix.codes + (size_t)(keep[u] ? rows[u] : 0) * ix.row_bytes, cw[u]);
#pragma unroll
      for (int u = 0; u < kScanRT; ++u) {
        const float acc = adc_words<W, LutT>(cw[u], s_lut, M);
        scanned += keep[u] ? 1 : 0;
        if constexpr (TRACE) {
          const uint64_t m = __ballot(keep[u]);
          if (m) {
            unsigned long long bpos = 0;
            if (lane == 0) bpos = atomicAdd(&t_count[q], (unsigned long long)__popcll(m));
            bpos = __shfl(bpos, 0, 64);
            if (keep[u]) {
              const unsigned long long pos = bpos + __popcll(m & lanemask);
              if ((int64_t)pos < t_capacity) {
                t_ids[(size_t)q * t_capacity + pos] = ix.row2ext[rows[u]];
                t_adc[(size_t)q * t_capacity + pos] = acc;
              }
            }
          }
        } else {
          bool pass = false;
          uint64_t key = 0;
          if (keep[u]) {
            const uint32_t h = ord32(acc);
            if (h <= thr_hi) {
              key = ((uint64_t)h << 32) | (uint32_t)ix.row2ext[rows[u]];
              pass = key < thr;
            }
          }
          const uint64_t m = __ballot(pass);
          if (m) {
            int bpos = 0;
            if (lane == 0) bpos = atomicAdd(&mc->count, (int)__popcll(m));
            bpos = __shfl(bpos, 0, 64);
            const int pos = bpos + __popcll(m & lanemask);
            if (pass && pos < cap) s_buf[pos] = key;  // (pos < cap always holds, see above)
          }
        }
      }
      base += kRound;
      wdone = base >= e1;
    }
    bool meet = wdone;
    if constexpr (!TRACE)
      meet = meet || __hip_atomic_load(&mc->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > T;
    if (meet) {  // wave-uniform
      if (wdone && !counted) {
        if (lane == 0) atomicAdd(&mc->done, 1);
        counted = true;
      }
      __syncthreads();
      const bool all = mc->done == kScanBlock / 64;
      const bool cut = !TRACE && !all && mc->count > T;
      __syncthreads();
      if (all) break;
      if constexpr (!TRACE) {
        // cut back to about the n best (by distance alone; exactly when ties
        // at the cut would still leave the count above T)
        if (cut && scan_compact(s_buf, s_wsum, ss, mc, n, true) > T)
          scan_compact(s_buf, s_wsum, ss, mc, n);
      }
    }
  }
  // candidates scored by this item
  {
    int v = scanned;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) atomicAdd(&mc->scanned, v);
  }
  __syncthreads();
  if constexpr (!TRACE) {
    scan_compact(s_buf, s_wsum, ss, mc, n);
    const int cnt = min(mc->count, n);
    uint64_t* dst = pkeys + ((size_t)q * smax + j) * n;
    for (int i = tid; i < cnt; i += kScanBlock) dst[i] = s_buf[i];
    if (tid == 0) {
      pcount[(size_t)q * smax + j] = cnt;
      pscan[2 * ((size_t)q * smax + j)] = mc->scanned;
      pscan[2 * ((size_t)q * smax + j) + 1] = e1 - e0;  // entries walked
    }
    if (sp.thr_out && cnt == n) {  // block-uniform
      // this item's n-th smallest key (the largest it keeps) bounds the
      // query's n-th smallest key from above
      uint64_t mx = 0;
      for (int i = tid; i < cnt; i += kScanBlock) mx = s_buf[i] > mx ? s_buf[i] : mx;
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) {
        const uint64_t o = __shfl_xor(mx, d, 64);
        mx = o > mx ? o : mx;
      }
      __syncthreads();
      if (tid == 0) mc->thr = 0;
      __syncthreads();
      if (lane == 0) atomicMax(reinterpret_cast<unsigned long long*>(&mc->thr), (unsigned long long)mx);
      __syncthreads();
      if (tid == 0) atomicMin(&sp.thr_out[q], (unsigned long long)mc->thr);
    }
  }
}

// ---------------------------------------------------------------------------
// Step 8: exact squared distance of one raw vector, addressed by its external
// ID (float64 in order for float data, exact integers for uint8/int8).

__device__ __forceinline__ float exact_row(const DevIndex& ix, const float* __restrict__ s_q,
                                           uint32_t id) {
  const int D = ix.dim;
  if (ix.dtype == F32) {
    const float* x = static_cast<const float*>(ix.vecs) + (size_t)id * D;
    double acc = 0.0;
    auto add = [&](float qv, float xv) {
      const double u = (double)qv - (double)xv;
      const double sq = u * u;
      acc = acc + sq;
    };
    if (D % 4 == 0) {  // rows are 16-byte aligned: float4 loads, same order of sums
      const float4* x4 = reinterpret_cast<const float4*>(x);
#pragma unroll 4
      for (int t4 = 0; t4 < D / 4; ++t4) {
        const float4 v = x4[t4];
        add(s_q[4 * t4], v.x);
        add(s_q[4 * t4 + 1], v.y);
        add(s_q[4 * t4 + 2], v.z);
        add(s_q[4 * t4 + 3], v.w);
      }
    } else {
      for (int t = 0; t < D; ++t) add(s_q[t], x[t]);
    }
    return (float)acc;
  }
  int acc = 0;
  if (ix.dtype == U8) {
    const uint8_t* x = static_cast<const uint8_t*>(ix.vecs) + (size_t)id * D;
    for (int t = 0; t < D; ++t) {
      const int u = (int)s_q[t] - (int)x[t];
      acc += u * u;
    }
  } else {
    const int8_t* x = static_cast<const int8_t*>(ix.vecs) + (size_t)id * D;
    for (int t = 0; t < D; ++t) {
      const int u = (int)s_q[t] - (int)x[t];
      acc += u * u;
    }
  }
  return (float)acc;
}

// Integer rows of 16*G bytes: G lanes per candidate, one 16-byte chunk per
// lane, 4 candidates per lane group in flight.  Exact integer sums: per chunk
// ||q - x||^2 = ||q||^2 + ||x||^2 - 2 q.x with the byte dot products done by
// v_dot4 (unsigned bytes for uint8 data, signed for int8).
template <int G>
__device__ void rerank_int16(const DevIndex& ix, const float* s_q, const uint64_t* s_top, int nn,
                             uint64_t* s_key2, int P) {
  const int lg = threadIdx.x % G, grp = threadIdx.x / G, ngrp = blockDim.x / G;
  const bool u8 = ix.dtype == U8;
  uint32_t qw[4];
  int qq = 0;
#pragma unroll
  for (int b4 = 0; b4 < 4; ++b4) {
    uint32_t wv = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int v = (int)s_q[lg * 16 + 4 * b4 + b];
      qq += v * v;
      wv |= ((uint32_t)v & 255u) << (8 * b);
    }
    qw[b4] = wv;
  }
  constexpr int U = 4;
  for (int i0 = 0; i0 < P; i0 += ngrp * U) {
    uint4 v[U];
    uint32_t id[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * ngrp + grp;
      ok[u] = i < nn;
      id[u] = ok[u] ? (uint32_t)s_top[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = make_uint4(0u, 0u, 0u, 0u);
      if (ok[u])
        v[u] = *reinterpret_cast<const uint4*>(static_cast<const uint8_t*>(ix.vecs) +
                                               (size_t)id[u] * ix.dim + lg * 16);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int xx, qx;
      if (u8) {
        uint32_t a = __builtin_amdgcn_udot4(v[u].x, v[u].x, 0u, false);
        a = __builtin_amdgcn_udot4(v[u].y, v[u].y, a, false);
        a = __builtin_amdgcn_udot4(v[u].z, v[u].z, a, false);
        a = __builtin_amdgcn_udot4(v[u].w, v[u].w, a, false);
        uint32_t c = __builtin_amdgcn_udot4(qw[0], v[u].x, 0u, false);
        c = __builtin_amdgcn_udot4(qw[1], v[u].y, c, false);
        c = __builtin_amdgcn_udot4(qw[2], v[u].z, c, false);
        c = __builtin_amdgcn_udot4(qw[3], v[u].w, c, false);
        xx = (int)a;
        qx = (int)c;
      } else {
        int a = __builtin_amdgcn_sdot4((int)v[u].x, (int)v[u].x, 0, false);
        a = __builtin_amdgcn_sdot4((int)v[u].y, (int)v[u].y, a, false);
        a = __builtin_amdgcn_sdot4((int)v[u].z, (int)v[u].z, a, false);
        a = __builtin_amdgcn_sdot4((int)v[u].w, (int)v[u].w, a, false);
        int c = __builtin_amdgcn_sdot4((int)qw[0], (int)v[u].x, 0, false);
        c = __builtin_amdgcn_sdot4((int)qw[1], (int)v[u].y, c, false);
        c = __builtin_amdgcn_sdot4((int)qw[2], (int)v[u].z, c, false);
        c = __builtin_amdgcn_sdot4((int)qw[3], (int)v[u].w, c, false);
        xx = a;
        qx = c;
      }
      int acc = qq + xx - 2 * qx;
#pragma unroll
      for (int d = 1; d < G; d <<= 1) acc += __shfl_xor(acc, d, 64);
      const int i = i0 + u * ngrp + grp;
      if (lg == 0 && i < P)
        s_key2[i] = ok[u] ? (((uint64_t)ord32((float)acc) << 32) | id[u]) : ~0ull;
    }
  }
}

// Wave-aggregated append: lanes with take set get consecutive slots counted
// by *cnt (LDS); returns this lane's slot (undefined where take is false).
__device__ __forceinline__ int wave_append(bool take, int* cnt) {
  const uint64_t m = __ballot(take);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0 && m) base = atomicAdd(cnt, __popcll(m));
  base = __shfl(base, 0, 64);
  return base + __popcll(m & ((1ull << lane) - 1ull));
}

// Ascending bitonic sort of the 64 R keys a wave holds in registers (element
// r * 64 + lane in a[r]): strides below 64 exchange across lanes, larger ones
// between a lane's own registers.  Stage (K, J) is a template so every
// register index is a constant (the keys stay in registers).
template <int R, int K, int J>
__device__ __forceinline__ void wave_sort_stage(uint64_t (&a)[R], int lane) {
  if constexpr (J >= 64) {
    constexpr int RJ = J / 64;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((r & RJ) == 0) {
        const bool up = ((r * 64 + lane) & K) == 0;
        const uint64_t x = a[r], y = a[r | RJ];
        const bool sw = (x > y) == up;
        a[r] = sw ? y : x;
        a[r | RJ] = sw ? x : y;
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t o = __shfl_xor(a[r], J, 64);
      const bool lower = (lane & J) == 0, up = ((r * 64 + lane) & K) == 0;
      a[r] = (lower == up) ? (o < a[r] ? o : a[r]) : (o > a[r] ? o : a[r]);
    }
  }
  if constexpr (J > 1) wave_sort_stage<R, K, J / 2>(a, lane);
}

template <int R, int K = 2>
__device__ __forceinline__ void wave_sort_regs(uint64_t (&a)[R]) {
  if constexpr (K <= 64 * R) {
    wave_sort_stage<R, K, K / 2>(a, threadIdx.x & 63);
    wave_sort_regs<R, K * 2>(a);
  }
}

// Exact keys (distance << 32 | external ID) of the candidates s_top[0..nn)
// (external ID in the low half); s_key2[nn..P) = ~0.
__device__ void exact_keys(const DevIndex& ix, const float* s_q, const uint64_t* s_top, int nn,
                           uint64_t* s_key2, int P) {
  const int g16 = ix.dim % 16 == 0 ? ix.dim / 16 : 0;
  if (ix.dtype != F32 && (g16 == 1 || g16 == 2 || g16 == 4 || g16 == 8 || g16 == 16)) {
    switch (g16) {
      case 1: rerank_int16<1>(ix, s_q, s_top, nn, s_key2, P); break;
      case 2: rerank_int16<2>(ix, s_q, s_top, nn, s_key2, P); break;
      case 4: rerank_int16<4>(ix, s_q, s_top, nn, s_key2, P); break;
      case 8: rerank_int16<8>(ix, s_q, s_top, nn, s_key2, P); break;
      default: rerank_int16<16>(ix, s_q, s_top, nn, s_key2, P); break;
    }
  } else if (ix.dtype != F32 && ix.dim % 4 == 0) {
    // integer data: 8 lanes per candidate, each summing every 8th dword of
    // the row (exact integers, so the summation order is free)
    const int g = threadIdx.x >> 3, jl = threadIdx.x & 7, ng = blockDim.x >> 3;
    const int nd = ix.dim >> 2;
    for (int i0 = 0; i0 < P; i0 += ng) {
      const int i = i0 + g;
      int acc = 0;
      uint32_t id = 0;
      if (i < nn) {
        id = (uint32_t)s_top[i];
        const uint32_t* x = reinterpret_cast<const uint32_t*>(
            static_cast<const uint8_t*>(ix.vecs) + (size_t)id * ix.dim);
        for (int t = jl; t < nd; t += 8) {
          const uint32_t v = x[t];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int xv = ix.dtype == U8 ? (int)((v >> (8 * b)) & 255u)
                                          : (int)(int8_t)(uint8_t)((v >> (8 * b)) & 255u);
            const int u = (int)s_q[4 * t + b] - xv;
            acc += u * u;
          }
        }
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      acc += __shfl_xor(acc, 4, 64);
      if (jl == 0 && i < P)
        s_key2[i] = i < nn ? (((uint64_t)ord32((float)acc) << 32) | id) : ~0ull;
    }
  } else {
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
      uint64_t key = ~0ull;
      if (i < nn) {
        const uint32_t id = (uint32_t)s_top[i];
        const float e = exact_row(ix, s_q, id);
        key = ((uint64_t)ord32(e) << 32) | id;
      }
      s_key2[i] = key;
    }
  }
}

// Host-memory raw tier (Sec. 4.3): the raw vectors lie on pages in pinned
// host memory, bucketed by nearest list.  A query's candidates are scored a
// page at a time: a page is read whole (over PCIe, into the reading wave's
// LDS buffer) the first time one of the candidates being re-ranked lies on
// it, and every candidate of the query on that page is scored from that one
// read -- so requests for one page within a mini-batch are merged, and a
// later mini-batch finds its candidates on already-read pages scored (the
// page buffer across mini-batches).  Pages read = distinct pages of the
// candidates re-ranked, counted in the mini-batch that first needs them.
struct PageScratch {
  uint64_t* pg;         // [P] (page << 32 | candidate index), ascending
  int32_t* first;       // [P] candidate i: start of its page's run in pg if i is
                        //     the run's lowest index, else -1
  int32_t* list;        // [P] runs to read now
  uint64_t* ex;         // [P] exact key of each candidate once scored
  unsigned char* buf;   // [waves, page_bytes] one page per wave
  int* cnt;
};

// Layout (base 16-byte aligned): pg, ex, first, list, cnt, then the page
// buffers at a 16-byte aligned offset.
__host__ __device__ inline size_t page_scratch_head(int P) {
  return align_up((size_t)P * (8 + 8 + 4 + 4) + 16, 16);
}

__host__ __device__ inline size_t page_scratch_bytes(int P, int waves, int page_bytes) {
  return page_scratch_head(P) + (size_t)waves * page_bytes;
}

__device__ inline PageScratch page_scratch(unsigned char* base, int P) {
  PageScratch ps;
  ps.pg = reinterpret_cast<uint64_t*>(base);
  ps.ex = ps.pg + P;
  ps.first = reinterpret_cast<int32_t*>(ps.ex + P);
  ps.list = ps.first + P;
  ps.cnt = ps.list + P;
  ps.buf = base + page_scratch_head(P);
  return ps;
}

// Runs of candidates s_top[0..nn) by page.  Ends with a barrier.
__device__ void pages_prepare(const DevIndex& ix, const uint64_t* s_top, int nn, int P,
                              const PageScratch& ps) {
  for (int i = threadIdx.x; i < P; i += blockDim.x)
    ps.pg[i] = i < nn ? ((uint64_t)(uint32_t)ix.vpage[(uint32_t)s_top[i]] << 32) | (uint32_t)i
                      : ~0ull;
  __syncthreads();
  block_bitonic(ps.pg, P);
  for (int i = threadIdx.x; i < nn; i += blockDim.x) ps.first[i] = -1;
  __syncthreads();
  for (int j = threadIdx.x; j < nn; j += blockDim.x)
    if (j == 0 || (ps.pg[j] >> 32) != (ps.pg[j - 1] >> 32)) ps.first[(uint32_t)ps.pg[j]] = j;
  __syncthreads();
}

// Exact squared distance of a raw row held in LDS (same arithmetic and order
// as exact_row).
__device__ __forceinline__ float exact_row_lds(const DevIndex& ix, const float* __restrict__ s_q,
                                               const unsigned char* row) {
  const int D = ix.dim;
  if (ix.dtype == F32) {
    const float* x = reinterpret_cast<const float*>(row);
    double acc = 0.0;
    for (int t = 0; t < D; ++t) {
      const double u = (double)s_q[t] - (double)x[t];
      const double sq = u * u;
      acc = acc + sq;
    }
    return (float)acc;
  }
  int acc = 0;
  for (int t = 0; t < D; ++t) {
    const int xv = ix.dtype == U8 ? (int)row[t] : (int)(int8_t)row[t];
    const int u = (int)s_q[t] - xv;
    acc += u * u;
  }
  return (float)acc;
}

// Read the pages first needed by candidates [c0, c1) and score every
// candidate on them.  Returns the pages read (the same in every thread).
__device__ int pages_read(const DevIndex& ix, const float* s_q, const uint64_t* s_top, int nn,
                          int c0, int c1, const PageScratch& ps) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  if (tid == 0) *ps.cnt = 0;
  __syncthreads();
  for (int i0 = c0; i0 < c1; i0 += blockDim.x) {  // uniform trip count
    const int i = i0 + tid;
    const bool take = i < c1 && ps.first[i] >= 0;
    const int pos = wave_append(take, ps.cnt);
    if (take) ps.list[pos] = ps.first[i];
  }
  __syncthreads();
  const int nr = *ps.cnt;
  const int row_bytes = ix.dim * (ix.dtype == F32 ? 4 : 1);
  unsigned char* mine = ps.buf + (size_t)wv * ix.page_bytes;
  for (int r0 = 0; r0 < nr; r0 += nw) {  // uniform trip count: one page per wave and round
    const int r = r0 + wv;
    uint64_t page = 0;
    int j0 = 0;
    if (r < nr) {
      j0 = ps.list[r];
      page = ps.pg[j0] >> 32;
      const uint4* src = reinterpret_cast<const uint4*>(ix.hpages + page * (uint64_t)ix.page_bytes);
      for (int t = lane; t < ix.page_bytes / 16; t += 64) reinterpret_cast<uint4*>(mine)[t] = src[t];
    }
    __syncthreads();  // the round's pages are in LDS
    if (r < nr) {
      for (int j = j0 + lane; j < nn && (ps.pg[j] >> 32) == page; j += 64) {
        const uint32_t ci = (uint32_t)ps.pg[j];
        const uint32_t id = (uint32_t)s_top[ci];
        const float e = exact_row_lds(ix, s_q, mine + (size_t)ix.vslot[id] * row_bytes);
        ps.ex[ci] = ((uint64_t)ord32(e) << 32) | id;
      }
    }
    __syncthreads();  // before the next round overwrites the buffers
  }
  return nr;
}

// Re-rank s_top[0..nn) (external IDs in the low halves) by exact distance
// and write the top-k, sorted.  s_key2 holds
// P >= nn keys; s_top is reused for the result (it needs
// max(128, pow2_at_least(min(k, nn))) slots).
__device__ void rerank_write(const DevIndex& ix, const float* s_q, uint64_t* s_top, int nn,
                             uint64_t* s_key2, int P, int k, int64_t* out_ids, float* out_d,
                             SelScratch* ss, int* s_cnt, bool keys_ready = false) {
  if (!keys_ready) exact_keys(ix, s_q, s_top, nn, s_key2, P);
  __syncthreads();
  const int kk = min(k, nn);
  const int lane = threadIdx.x & 63;
  auto write_out = [&](int i, uint64_t key) {  // output slot i < k
    const bool v = i < kk;
    out_ids[i] = v ? (int64_t)(uint32_t)key : -1;
    out_d[i] = v ? unord32((uint32_t)(key >> 32)) : INFINITY;
  };
  if (kk <= 64 && k <= 64) {
    // The first min(nn, 256) keys sorted by one wave: the answer if they are
    // all, else their kk-th smallest bounds the kk-th smallest of all, and
    // the keys up to it (at least kk) are usually few enough for one wave.
    if (threadIdx.x < 64) {
      uint64_t a[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = r * 64 + lane < nn ? s_key2[r * 64 + lane] : ~0ull;
      wave_sort_regs<4>(a);
      const uint64_t t = __shfl(a[0], max(kk, 1) - 1, 64);
      if (nn <= 256) {
        if (lane < k) write_out(lane, a[0]);
      } else if (lane == 0) {
        ss->lo = t;
        *s_cnt = 0;
      }
    }
    if (nn <= 256) return;  // uniform
    __syncthreads();
    const uint64_t T = ss->lo;
    for (int i0 = 0; i0 < nn; i0 += blockDim.x) {  // uniform trip count
      const int i = i0 + threadIdx.x;
      const uint64_t key = i < nn ? s_key2[i] : ~0ull;
      const bool take = i < nn && key <= T;
      const int pos = wave_append(take, s_cnt);
      if (take && pos < 128) s_top[pos] = key;
    }
    __syncthreads();
    const int ns = *s_cnt;
    if (ns <= 128) {  // uniform
      if (threadIdx.x < 64) {
        uint64_t a[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) a[r] = r * 64 + lane < ns ? s_top[r * 64 + lane] : ~0ull;
        wave_sort_regs<2>(a);
        if (lane < k) write_out(lane, a[0]);
      }
      return;
    }
    __syncthreads();  // (rare) too many keys up to the bound: select exactly
  }
  // the kk smallest keys, ascending: select the kk-th, collect, sort kk
  if (kk > 0) {
    const int pk = pow2_at_least(kk);
    const uint64_t K = kk == nn ? ~0ull : block_kth([&](int i) { return s_key2[i]; }, nn, kk, ss);
    if (threadIdx.x == 0) *s_cnt = 0;
    for (int i = threadIdx.x; i < pk; i += blockDim.x) s_top[i] = ~0ull;
    __syncthreads();
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
      const uint64_t key = s_key2[i];
      if (key <= K) {
        const int pos = atomicAdd(s_cnt, 1);
        if (pos < pk) s_top[pos] = key;
      }
    }
    __syncthreads();
    block_bitonic(s_top, pk);
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) write_out(i, s_top[i]);
}


// Step 8 by the heuristic re-ranking (Alg. 1, change rate of Eq. 3): the
// candidates s_top[0..nn), sorted ascending by (adc, id), are re-ranked in
// mini-batches of hb; after each mini-batch the k best (distance, id) pairs
// so far are the k smallest of (previous best, this mini-batch), and the
// change rate is the number of their IDs absent from the previous best,
// divided by k.  The loop stops once the rate has been <= eps for beta
// mini-batches in a row; *reranked counts the candidates of the mini-batches
// used.  Exact distances are gathered a chunk of whole mini-batches (about
// 1024 candidates) at a time so that the loads of several mini-batches are in
// flight together; the rule itself is evaluated mini-batch by mini-batch.
// Per mini-batch, only keys below the current k-th best can enter the best;
// they are merged with the best by counting ranks (after a radix select of
// the k smallest when they are many).  k <= 64.  s_key2 holds >= nn keys;
// s_best 64 keys; s_cand >= 256 keys; s_misc 3 ints.
__device__ void rerank_heuristic(const DevIndex& ix, const float* s_q, uint64_t* s_top, int nn,
                                 uint64_t* s_key2, uint64_t* s_best, uint64_t* s_cand,
                                 int* s_misc, SelScratch* ss, int k, int hb, double eps, int beta,
                                 int64_t* out_ids, float* out_d, int32_t* reranked,
                                 const PageScratch* ps = nullptr, int* page_reads = nullptr) {
  constexpr int kU = 256;  // merge set: the previous best and at most kU - cur entrants
  const int tid = threadIdx.x;
  int cur = 0, stable = 0, done = 0, preads = 0;
  bool stop = false;
  // candidates gathered per chunk; from host pages one mini-batch at a time
  // (a page is read only when a mini-batch that is re-ranked needs it)
  const int per = ps ? hb : hb * max(1, 1024 / hb);
  for (int c0 = 0; c0 < nn && !stop; c0 += per) {
    const int cn = min(per, nn - c0);
    __syncthreads();  // the previous chunk's exact keys have been read
    if (ps) {
      preads += pages_read(ix, s_q, s_top, nn, c0, c0 + cn, *ps);
      for (int i = tid; i < cn; i += blockDim.x) s_key2[i] = ps->ex[c0 + i];
    } else {
      exact_keys(ix, s_q, s_top + c0, cn, s_key2, cn);
    }
    __syncthreads();
    // s_top[c0..c0+cn) has been read: it holds the entrants of each mini-batch
    uint64_t* s_in = s_top + c0;
    for (int i = c0; i < c0 + cn && !stop; i += hb) {  // block-uniform
      const int b = min(hb, nn - i);
      const uint64_t* seg = s_key2 + (i - c0);
      const uint64_t T = cur == k ? s_best[k - 1] : ~0ull;
      for (int t = tid; t < cur; t += blockDim.x) s_cand[t] = s_best[t];
      if (tid == 0) s_misc[0] = s_misc[1] = s_misc[2] = 0;
      __syncthreads();
      for (int t0 = 0; t0 < b; t0 += blockDim.x) {  // entrants: keys below the k-th best
        const int t = t0 + tid;
        const uint64_t x = t < b ? seg[t] : ~0ull;
        const bool take = x < T;
        const int pos = wave_append(take, s_misc);
        if (take) {
          s_in[pos] = x;
          if (cur + pos < kU) s_cand[cur + pos] = x;
        }
      }
      __syncthreads();
      int m = cur + s_misc[0];
      if (m > kU) {  // many entrants (the first mini-batches): keep their k smallest
        const int ne = s_misc[0];
        const uint64_t K = block_kth([&](int u) { return s_in[u]; }, ne, k, ss);
        for (int t0 = 0; t0 < ne; t0 += blockDim.x) {
          const int t = t0 + tid;
          const uint64_t x = t < ne ? s_in[t] : ~0ull;
          const bool take = t < ne && x <= K;
          const int pos = wave_append(take, s_misc + 2);
          if (take && cur + pos < kU) s_cand[cur + pos] = x;
        }
        __syncthreads();
        m = min(kU, cur + s_misc[2]);  // k entrants when the keys are distinct
      }
      const int kk = min(k, m);
      // rank of each member of the merge set (ties broken by position)
      uint64_t x = ~0ull;
      int r = kU;
      if (tid < m) {
        x = s_cand[tid];
        r = 0;
        for (int u = 0; u < m; ++u) {
          const uint64_t y = s_cand[u];
          r += (y < x) | ((y == x) & (u < tid));
        }
      }
      bool fresh = false;  // an entrant in the new best whose ID the previous best lacks
      if (tid >= cur && r < kk) {
        fresh = true;
        for (int u = 0; u < cur; ++u) fresh = fresh && (uint32_t)s_cand[u] != (uint32_t)x;
      }
      (void)wave_append(fresh, s_misc + 1);
      __syncthreads();
      if (r < kk) s_best[r] = x;
      const int changed = s_misc[1];
      cur = kk;
      done = i + b;
      __syncthreads();
      const double delta = (double)changed / (double)k;  // Eq. 3
      if (delta <= eps) {
        if (++stable >= beta) stop = true;
      } else {
        stable = 0;
      }
    }
  }
  for (int t = tid; t < k; t += blockDim.x) {
    const bool v = t < cur;
    out_ids[t] = v ? (int64_t)(uint32_t)s_best[t] : -1;
    out_d[t] = v ? unord32((uint32_t)(s_best[t] >> 32)) : INFINITY;
  }
  if (tid == 0 && reranked) *reranked = done;
  if (tid == 0 && page_reads) *page_reads = preads;
}

struct MergeLayout {
  size_t keys, top, key2, q, sel, cand, best, misc, total;
};

__host__ __device__ inline MergeLayout merge_layout(int smax, int n, int dim) {
  MergeLayout L;
  const int P = pow2_at_least(n);
  size_t o = 0;
  // the re-rank keys reuse the partial-key area once the top-n is selected
  L.keys = o; L.key2 = o; o += (size_t)std::max(smax * n, P) * 8;
  L.top = o; o += (size_t)P * 8;
  L.q = o; o += (size_t)dim * 4; o = align_up(o, 16);
  L.sel = o; o += sizeof(SelScratch); o = align_up(o, 16);
  L.cand = o; o += (size_t)256 * 8;  // the heuristic re-ranking's merge set
  L.best = o; o += 64 * 8;
  L.misc = o; o += 16 + 4 * 18;
  L.total = align_up(o, 16);
  return L;
}

// HEUR: step 8 by the heuristic re-ranking (a kernel of its own, so the
// plain form's registers are not sized for it).  HOSTP: the raw vectors are
// read from host-memory pages (page scratch after the merge layout).
template <int BS, bool HEUR, bool HOSTP = false>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_merge(
    DevIndex ix, const float* __restrict__ Q, int qc, const int32_t* __restrict__ sq, int smax,
    int n, int k, const uint64_t* __restrict__ pkeys, const int32_t* __restrict__ pcount,
    const int32_t* __restrict__ pscan, int32_t* __restrict__ topn_ids, float* __restrict__ topn_adc,
    int64_t* __restrict__ ncand, int64_t* __restrict__ nwalk, int64_t* __restrict__ out_ids,
    float* __restrict__ out_dists,
    int hb, double h_eps, int h_beta, int32_t* __restrict__ reranked,
    int32_t* __restrict__ page_reads) {
  extern __shared__ __align__(16) unsigned char smem[];
  const MergeLayout L = merge_layout(smax, n, ix.dim);
  uint64_t* s_keys = reinterpret_cast<uint64_t*>(smem + L.keys);
  uint64_t* s_top = reinterpret_cast<uint64_t*>(smem + L.top);
  uint64_t* s_key2 = reinterpret_cast<uint64_t*>(smem + L.key2);
  float* s_q = reinterpret_cast<float*>(smem + L.q);
  SelScratch* ss = reinterpret_cast<SelScratch*>(smem + L.sel);
  uint64_t* s_cand = reinterpret_cast<uint64_t*>(smem + L.cand);
  int* s_cnt = reinterpret_cast<int*>(smem + L.misc);
  int* s_off = s_cnt + 1;  // [smax + 1] (smax <= 16)
  const int q = blockIdx.x, tid = threadIdx.x;
  const int S = sq[q];
  const int P = pow2_at_least(n);
  for (int t = tid; t < ix.dim; t += BS) s_q[t] = conv_query(Q[(size_t)q * ix.dim + t], ix.dtype);
  if (tid < 64) {  // one wave: the items' offsets (S <= 16) and the work counts
    int c = 0;
    int64_t sc = 0, sw = 0;
    if (tid < S) {
      c = pcount[(size_t)q * smax + tid];
      sc = pscan[2 * ((size_t)q * smax + tid)];
      sw = pscan[2 * ((size_t)q * smax + tid) + 1];
    }
    const int incl = (int)wave_incl_scan((uint32_t)c);
    if (tid < S) s_off[tid] = incl - c;
    if (tid == S - 1) s_off[S] = incl;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      sc += __shfl_xor(sc, d, 64);
      sw += __shfl_xor(sw, d, 64);
    }
    if (tid == 0) {
      *s_cnt = 0;
      if (ncand) ncand[q] = sc;
      if (nwalk) nwalk[q] = sw;
    }
  }
  __syncthreads();
  const int total = s_off[S];
  const int nn = min(n, total);
  // No selection needed: the keys go straight to s_top.
  const bool direct = total <= n;
  uint64_t* dst = direct ? s_top : s_keys;
  auto fetch = [&](int i) -> uint64_t {  // key i of the query's items, in item order
    int j = 0;
    while (j + 1 < S && s_off[j + 1] <= i) ++j;
    return pkeys[((size_t)q * smax + j) * n + (i - s_off[j])];
  };
  for (int i0 = 0; i0 < total; i0 += 2 * BS) {  // two keys per thread in flight
    const int ia = i0 + tid, ib = ia + BS;
    const bool oa = ia < total, ob = ib < total;
    const uint64_t ka = oa ? fetch(ia) : 0ull, kb = ob ? fetch(ib) : 0ull;
    if (oa) dst[ia] = ka;
    if (ob) dst[ib] = kb;
  }
  for (int i = nn + tid; i < P; i += BS) s_top[i] = ~0ull;
  __syncthreads();
  if (!direct) {
    const uint64_t K = block_kth([&](int i) { return s_keys[i]; }, total, n, ss);
    for (int i = tid; i < total; i += BS) {
      const uint64_t key = s_keys[i];
      if (key <= K) {
        const int pos = atomicAdd(s_cnt, 1);
        if (pos < P) s_top[pos] = key;
      }
    }
  }
  __syncthreads();
  if (topn_ids) {
    block_bitonic(s_top, P);
    for (int i = tid; i < n; i += BS) {
      const bool v = i < nn;
      topn_ids[(size_t)q * n + i] = v ? (int32_t)(uint32_t)s_top[i] : -1;
      topn_adc[(size_t)q * n + i] = v ? unord32((uint32_t)(s_top[i] >> 32)) : INFINITY;
    }
  }
  if (!out_ids) return;
  if constexpr (HOSTP) {
    const PageScratch ps = page_scratch(smem + L.total, P);
    if constexpr (HEUR) {
      if (!topn_ids) block_bitonic(s_top, P);
      __syncthreads();  // s_key2 aliases s_keys
      pages_prepare(ix, s_top, nn, P, ps);
      int preads = 0;
      rerank_heuristic(ix, s_q, s_top, nn, s_key2, reinterpret_cast<uint64_t*>(smem + L.best),
                       s_cand, s_cnt + 18, ss, k, hb, h_eps, h_beta, out_ids + (size_t)q * k,
                       out_dists + (size_t)q * k, reranked ? reranked + q : nullptr, &ps,
                       &preads);
      if (tid == 0 && page_reads) page_reads[q] = preads;
    } else {  // fixed re-rank: one mini-batch of all nn candidates
      __syncthreads();  // s_key2 aliases s_keys
      pages_prepare(ix, s_top, nn, P, ps);
      const int preads = pages_read(ix, s_q, s_top, nn, 0, nn, ps);
      for (int i = tid; i < P; i += BS) s_key2[i] = i < nn ? ps.ex[i] : ~0ull;
      if (tid == 0 && page_reads) page_reads[q] = preads;
      if (tid == 0 && reranked) reranked[q] = nn;
      rerank_write(ix, s_q, s_top, nn, s_key2, P, k, out_ids + (size_t)q * k,
                   out_dists + (size_t)q * k, ss, s_cnt, true);
    }
  } else if constexpr (HEUR) {  // heuristic re-ranking: candidates in ascending ADC order
    if (!topn_ids) block_bitonic(s_top, P);  // (already sorted when the top-n was written)
    __syncthreads();  // s_key2 aliases s_keys
    rerank_heuristic(ix, s_q, s_top, nn, s_key2, reinterpret_cast<uint64_t*>(smem + L.best),
                     s_cand, s_cnt + 18, ss, k, hb, h_eps, h_beta, out_ids + (size_t)q * k,
                     out_dists + (size_t)q * k, reranked ? reranked + q : nullptr);
  } else {
    __syncthreads();  // s_key2 aliases s_keys
    rerank_write(ix, s_q, s_top, nn, s_key2, P, k, out_ids + (size_t)q * k,
                 out_dists + (size_t)q * k, ss, s_cnt);
  }
}

// Step 8 for caller-provided candidates.
template <int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_rerank_only(DevIndex ix, const float* __restrict__ Q,
                                                         const int32_t* __restrict__ cand, int n,
                                                         int k, int64_t* __restrict__ out_ids,
                                                         float* __restrict__ out_dists) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int P = pow2_at_least(n);
  uint64_t* s_top = reinterpret_cast<uint64_t*>(smem);
  uint64_t* s_key2 = s_top + P;
  float* s_q = reinterpret_cast<float*>(s_key2 + P);
  int* s_cnt = reinterpret_cast<int*>(s_q + ix.dim);
  const int q = blockIdx.x, tid = threadIdx.x;
  for (int t = tid; t < ix.dim; t += BS) s_q[t] = conv_query(Q[(size_t)q * ix.dim + t], ix.dtype);
  if (tid == 0) *s_cnt = 0;
  __syncthreads();
  for (int i = tid; i < n; i += BS) {
    const int id = cand[(size_t)q * n + i];
    if (id >= 0 && id < ix.n) s_top[atomicAdd(s_cnt, 1)] = (uint32_t)id;
  }
  __syncthreads();
  const int nn = *s_cnt;
  __shared__ SelScratch ss;
  rerank_write(ix, s_q, s_top, nn, s_key2, P, k, out_ids + (size_t)q * k, out_dists + (size_t)q * k,
               &ss, s_cnt);
}

// Step 2 on integer-grid indexes without materialising the distance matrix:
// a block takes kFQ = 16 queries (the rows of one MFMA tile) through every
// list tile of 128 lists (int8 MFMA, same exact arithmetic as k_probe_mfma),
// keeps each query's keys (ordered distance bits, list) below its running
// threshold in an LDS buffer, and cuts a buffer back to its NP smallest keys
// when another tile might not fit.  At the end the NP smallest of each query
// come out ascending.  16 queries per block keep a 10k-query batch within
// one round of resident blocks (3 per CU at NP = 64).
constexpr int kFQ = 16;
constexpr int kFTile = 128;
constexpr int kFCols = kFTile / 4 / 16;  // 16-list MFMA column blocks per wave and tile
constexpr int kFusedMinQueries = 4096;

template <int NP>
__host__ __device__ constexpr int fused_cap() { return NP + kFTile + 128; }

// The want-th smallest (1-based) of the distinct keys s_key[0..c), found by
// one wave: MSD radix over 8-bit digits below the bits all keys share, with a
// private 256-bin histogram (hist), stopping once the digit bucket holds one
// key.  LDS traffic of the wave is ordered with workgroup fences.
__device__ uint64_t wave_kth(const uint64_t* s_key, int c, int want, uint32_t* hist) {
  const int lane = threadIdx.x & 63;
  uint64_t lo = ~0ull, hi = 0ull;
  for (int i = lane; i < c; i += 64) {
    const uint64_t k = s_key[i];
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const uint64_t a = __shfl_xor(lo, d, 64), b = __shfl_xor(hi, d, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  const uint64_t diff = lo ^ hi;
  if (diff == 0) return lo;
  const int top = ((63 - __clzll((long long)diff)) / 8) * 8;
  uint64_t mask = top >= 56 ? 0ull : ~((1ull << (top + 8)) - 1ull);
  uint64_t prefix = lo & mask;
  for (int shift = top; shift >= 0; shift -= 8) {
#pragma unroll
    for (int b = 0; b < 4; ++b) hist[4 * lane + b] = 0u;
    __threadfence_block();
    for (int i = lane; i < c; i += 64) {
      const uint64_t k = s_key[i];
      if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
    }
    __threadfence_block();
    const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1];
    const uint32_t h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
    const uint32_t sum = h0 + h1 + h2 + h3;
    const uint32_t incl = wave_incl_scan(sum);
    const uint32_t excl = incl - sum;
    const bool mine = excl < (uint32_t)want && (uint32_t)want <= incl;
    uint32_t r = (uint32_t)want - excl, hb = h0;
    int b = 4 * lane;
    if (r > h0) {
      r -= h0; b += 1; hb = h1;
      if (r > h1) {
        r -= h1; b += 1; hb = h2;
        if (r > h2) { r -= h2; b += 1; hb = h3; }
      }
    }
    const int owner = __ffsll((unsigned long long)__ballot(mine)) - 1;
    want = __shfl((int)r, owner, 64);
    b = __shfl(b, owner, 64);
    hb = (uint32_t)__shfl((int)hb, owner, 64);
    prefix |= (uint64_t)b << shift;
    mask |= 255ull << shift;
    if (hb == 1u) break;
  }
  uint64_t found = 0;
  for (int i = lane; i < c; i += 64) {
    const uint64_t k = s_key[i];
    if ((k & mask) == prefix) found = k;
  }
  // one key matches: the largest over lanes is it (others hold 0)
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const uint64_t o = __shfl_xor(found, d, 64);
    found = o > found ? o : found;
  }
  return found;
}

// Keys of s_key[0..c) that are <= K, appended to out by one wave; returns
// how many.
__device__ int wave_collect_le(const uint64_t* s_key, int c, uint64_t K, uint64_t* out) {
  const int lane = threadIdx.x & 63;
  int n = 0;
  for (int i0 = 0; i0 < c; i0 += 64) {
    const int i = i0 + lane;
    const uint64_t k = i < c ? s_key[i] : ~0ull;
    const bool take = i < c && k <= K;
    const uint64_t m = __ballot(take);
    if (take) out[n + __popcll(m & ((1ull << lane) - 1ull))] = k;
    n += __popcll(m);
  }
  __threadfence_block();
  return n;
}

// Ascending bitonic sort of s[0..P) (P a power of two, <= 4096) by one wave.
__device__ void wave_bitonic(uint64_t* s, int P) {
  const int lane = threadIdx.x & 63;
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < P; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = s[i], b = s[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __threadfence_block();
    }
  }
}

template <int NP, int KS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_probe_fused(DevIndex ix, const float* __restrict__ Q,
                                                         int qc, const int32_t* __restrict__ nprobe,
                                                         int np_max, int32_t* __restrict__ lists,
                                                         float* __restrict__ out_d,
                                                         int32_t* __restrict__ np_eff) {
  constexpr int CAP = fused_cap<NP>();
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* s_buf = reinterpret_cast<uint64_t*>(smem);        // [kFQ][CAP]
  uint64_t* s_tmp = s_buf + kFQ * CAP;                         // [4 waves][NP]
  uint64_t* s_thr = s_tmp + 4 * NP;                            // [kFQ]
  uint32_t* s_hist = reinterpret_cast<uint32_t*>(s_thr + kFQ); // [4 waves][256]
  int* s_cnt = reinterpret_cast<int*>(s_hist + 4 * 256);      // [kFQ]
  int* s_qn = s_cnt + kFQ;                                     // [kFQ]
  int8_t* s_q8 = reinterpret_cast<int8_t*>(s_qn + kFQ);       // [16][dim_pad]
  const int Dp = ix.dim_pad, D = ix.dim;
  const int q0 = blockIdx.x * kFQ;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  {  // the block's queries as shifted int8, 8 loads in flight per thread
    constexpr int U = 8;
    for (int i0 = tid; i0 < 16 * Dp; i0 += kBlock * U) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kBlock;
        v[u] = Q[(size_t)min(q0 + i / Dp, qc - 1) * D + min(i % Dp, D - 1)];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kBlock;
        const int qi = i / Dp, qq = q0 + qi, t = i % Dp;
        if (i < 16 * Dp)
          s_q8[i] = (int8_t)(qi < kFQ && qq < qc && t < D
                                 ? (int)conv_query(v[u], ix.dtype) - ix.shift8
                                 : 0);
      }
    }
  }
  if (tid < kFQ) {
    s_thr[tid] = ~0ull;
    s_cnt[tid] = 0;
  }
  __syncthreads();
  if (tid < kFQ) {
    int sum = 0;
    for (int t = 0; t < Dp; ++t) {
      const int v = s_q8[tid * Dp + t];
      sum += v * v;
    }
    s_qn[tid] = sum;
  }
  __syncthreads();
  const int r16 = lane & 15, g = lane >> 4;
  int qn[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) qn[r] = s_qn[4 * g + r];
  // KS = dim_pad / 64 K-steps.  The query fragments stay in registers; the
  // centroid fragments and norms of the next list tile are in flight while
  // this one is being filtered (software pipelining across tiles).
  v4i_t fa[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k)
    fa[k] = *reinterpret_cast<const v4i_t*>(s_q8 + r16 * Dp + 64 * k + 16 * g);
  v4i_t fn[KS][kFCols], fn2[KS][kFCols];
  int cnn[kFCols], cnn2[kFCols];
  // this lane's centroid fragment and norm addresses for list column 0 of a
  // tile (column b adds 16 lists); tiles wholly inside nlist load unguarded
  const int8_t* cbase = ix.cent8 + (size_t)(w * (kFTile / 4) + r16) * Dp + 16 * g;
  const int32_t* nbase = ix.cnorm8 + w * (kFTile / 4) + r16;
  auto load_tile = [&](int t0, v4i_t (&dst)[KS][kFCols], int (&dn)[kFCols]) {
    const int8_t* cp = cbase + (size_t)t0 * Dp;
    if (t0 + kFTile <= ix.nlist) {  // tile-uniform
#pragma unroll
      for (int b = 0; b < kFCols; ++b) {
#pragma unroll
        for (int k = 0; k < KS; ++k)
          dst[k][b] = *reinterpret_cast<const v4i_t*>(cp + (size_t)b * 16 * Dp + 64 * k);
        dn[b] = nbase[t0 + b * 16];
      }
    } else {
#pragma unroll
      for (int b = 0; b < kFCols; ++b) {
        const bool in = t0 + w * (kFTile / 4) + b * 16 + r16 < ix.nlist;
#pragma unroll
        for (int k = 0; k < KS; ++k)
          dst[k][b] = in ? *reinterpret_cast<const v4i_t*>(cp + (size_t)b * 16 * Dp + 64 * k)
                         : v4i_t{0, 0, 0, 0};
        dn[b] = in ? nbase[t0 + b * 16] : 0;
      }
    }
  };
  // A list l passes row r's filter when cn(l) - 2 q.c(l) <= lim[r] =
  // (distance of the row's threshold key) - |q|^2, i.e. when its distance is
  // at most the threshold's: a tie with the threshold distance is admitted
  // (the key may be larger than the threshold key; cut-backs and the final
  // selection keep exactly the smallest keys).  lim changes only at cut-backs.
  int lim[4];
  auto load_lim = [&]() {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint64_t t = s_thr[4 * g + r];
      lim[r] = t == ~0ull ? INT_MAX : (int)unord32((uint32_t)(t >> 32)) - qn[r];
    }
  };
  load_lim();
  // one tile: its MFMAs (fragments fb, norms cnb), the filter into the
  // buffers, and the cut-backs of buffers that might not take another tile
  auto process = [&](int t0, const v4i_t (&fb)[KS][kFCols], const int (&cnb)[kFCols]) {
    const int l0 = t0 + w * (kFTile / 4);
    v4i_t acc[kFCols];
#pragma unroll
    for (int b = 0; b < kFCols; ++b) acc[b] = v4i_t{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < KS; ++k)
#pragma unroll
      for (int b = 0; b < kFCols; ++b)
        acc[b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[k], fb[k][b], acc[b], 0, 0, 0);
    const bool whole = t0 + kFTile <= ix.nlist;  // tile-uniform
#pragma unroll
    for (int b = 0; b < kFCols; ++b) {
      const int l = l0 + b * 16 + r16;  // output column = lane % 16
      const bool in = whole || l < ix.nlist;
      const int cn = cnb[b];
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // output row = 4 * (lane / 16) + r
        const int v = cn - 2 * acc[b][r];
        if (in && v <= lim[r]) {
          const int m = 4 * g + r;
          const int d = v + qn[r];
          s_buf[m * CAP + atomicAdd(&s_cnt[m], 1)] =
              ((uint64_t)ord32((float)d) << 32) | (uint32_t)l;
        }
      }
    }
    __syncthreads();
    // cut back the buffers that might not take another tile; the cuts are
    // dealt round-robin to the waves (the full set is read by every wave
    // before any cut rewrites a count)
    const uint64_t full = __ballot(lane < kFQ && s_cnt[lane] > CAP - kFTile);
    __syncthreads();
    int job = 0;
    for (uint64_t f = full; f; f &= f - 1, ++job) {
      if ((job & 3) != w) continue;
      const int m = __ffsll((unsigned long long)f) - 1;
      const int c = s_cnt[m];
      const uint64_t K = wave_kth(s_buf + m * CAP, c, NP, s_hist + w * 256);
      wave_collect_le(s_buf + m * CAP, c, K, s_tmp + w * NP);  // exactly NP keys
      for (int i = lane; i < NP; i += 64) s_buf[m * CAP + i] = s_tmp[w * NP + i];
      if (lane == 0) {
        s_cnt[m] = NP;
        s_thr[m] = K;
      }
    }
    __syncthreads();
    if (full) load_lim();  // block-uniform: the thresholds changed
  };
  // two register sets, alternating: the next tile loads while this one runs
  load_tile(0, fn, cnn);
  for (int t0 = 0; t0 < ix.nlist; t0 += 2 * kFTile) {
    if (t0 + kFTile < ix.nlist) load_tile(t0 + kFTile, fn2, cnn2);
    process(t0, fn, cnn);
    if (t0 + kFTile >= ix.nlist) break;
    if (t0 + 2 * kFTile < ix.nlist) load_tile(t0 + 2 * kFTile, fn, cnn);
    process(t0 + kFTile, fn2, cnn2);
  }
  // the np smallest of each query, ascending
  for (int m = w; m < kFQ; m += 4) {
    const int q = q0 + m;
    if (q >= qc) continue;
    int np = nprobe ? nprobe[q] : np_max;
    np = max(0, min(np, min(np_max, ix.nlist)));
    const int c = s_cnt[m];
    const int kk = min(NP, c);
    uint64_t* t = s_tmp + w * NP;
    if (kk > 0) {
      const uint64_t K = kk == c ? ~0ull : wave_kth(s_buf + m * CAP, c, kk, s_hist + w * 256);
      const int got = wave_collect_le(s_buf + m * CAP, c, K, t);
      const int P = pow2_at_least(got);
      for (int i = got + lane; i < P; i += 64) t[i] = ~0ull;
      __threadfence_block();
      wave_bitonic(t, P);
    }
    for (int p = lane; p < np_max; p += 64) {
      const bool v = p < np;
      const uint64_t key = v ? s_tmp[w * NP + p] : ~0ull;
      lists[(size_t)q * np_max + p] = v ? (int32_t)(uint32_t)key : -1;
      if (out_d) out_d[(size_t)q * np_max + p] = v ? unord32((uint32_t)(key >> 32)) : INFINITY;
    }
    if (lane == 0) np_eff[q] = np;
  }
}

template <int NP>
size_t fused_lds(const DevIndex& ix) {
  return (size_t)kFQ * fused_cap<NP>() * 8 + (size_t)4 * NP * 8 + kFQ * 8 + 4 * 256 * 4 +
         kFQ * 8 + (size_t)16 * ix.dim_pad;
}

// ---------------------------------------------------------------------------
// Step 2 through the navigation graph over the list centroids (Sec. 4.1).
//
// One wave per query walks the graph best first: the candidate set C holds
// the query's `beam` nearest (distance, list) keys found so far, ascending,
// each marked expanded or not; the nearest not-yet-expanded one is expanded
// by scoring its neighbours (one lane each) and merging those that are new
// and below C's last key into C; the walk ends when all of C is expanded and
// the first np keys are the probe.  Offering a list twice changes nothing (a
// key already in C is dropped as a duplicate, and a key once dropped from a
// full C can never re-enter, because C's last key only decreases), so a
// lossy visited cache (a list whose slot holds it was scored before) only
// saves distances.  Distances are the exact probe's.
constexpr int kNavVis = 1024;  // visited-cache slots per query

__host__ __device__ inline size_t nav_wave_bytes(int dim, int dim_pad, int cap) {
  size_t o = (size_t)cap * 16;                 // two key buffers
  o += (size_t)cap * 2;                        // two flag buffers
  o = (o + 15) / 16 * 16;
  o += 64 * 8 + 64 * 4;                        // new keys and their ranks in C
  o += (size_t)kNavVis * 4;                    // visited cache
  const size_t qb = (size_t)dim * 8 > (size_t)dim_pad ? (size_t)dim * 8 : (size_t)dim_pad;
  o += (qb + 15) / 16 * 16;                    // the query (float64 or shifted int8)
  return o;
}

__device__ __forceinline__ uint32_t nav_slot(int u) {
  return ((uint32_t)u * 2654435761u) >> (32 - 10);  // kNavVis = 2^10
}

template <bool INT>
__global__ __launch_bounds__(kBlock) void k_probe_graph(DevIndex ix, const float* __restrict__ Q,
                                                      int qc, const int32_t* __restrict__ nprobe,
                                                      int np_max, int cap,
                                                      int32_t* __restrict__ lists,
                                                      float* __restrict__ out_d,
                                                      int32_t* __restrict__ np_eff) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = blockIdx.x * (blockDim.x >> 6) + w;
  if (q >= qc) return;  // wave-uniform; the waves of a block never synchronise
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* base = smem + (size_t)w * nav_wave_bytes(ix.dim, ix.dim_pad, cap);
  uint64_t* keys[2] = {reinterpret_cast<uint64_t*>(base), reinterpret_cast<uint64_t*>(base) + cap};
  uint8_t* flg[2] = {reinterpret_cast<uint8_t*>(keys[1] + cap),
                     reinterpret_cast<uint8_t*>(keys[1] + cap) + cap};
  size_t off = ((size_t)cap * 18 + 15) / 16 * 16;
  uint64_t* nk = reinterpret_cast<uint64_t*>(base + off);
  int32_t* nr = reinterpret_cast<int32_t*>(nk + 64);
  int32_t* vis = nr + 64;
  unsigned char* qv = reinterpret_cast<unsigned char*>(vis + kNavVis);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));

  int np = nprobe ? nprobe[q] : np_max;
  np = max(0, min(np, min(np_max, ix.nlist)));
  const int B = max(max(ix.nav_beam, np), 1);  // <= cap

  // the query: shifted int8 (integer grid) or float64 values
  int qn = 0;
  if constexpr (INT) {
    int8_t* q8 = reinterpret_cast<int8_t*>(qv);
    for (int t = lane; t < ix.dim_pad; t += 64) {
      const int v = t < ix.dim ? (int)conv_query(Q[(size_t)q * ix.dim + t], ix.dtype) - ix.shift8 : 0;
      q8[t] = (int8_t)v;
      qn += v * v;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) qn += __shfl_xor(qn, d, 64);
  } else {
    double* qd = reinterpret_cast<double*>(qv);
    for (int t = lane; t < ix.dim; t += 64) qd[t] = (double)conv_query(Q[(size_t)q * ix.dim + t], ix.dtype);
  }
  for (int i = lane; i < kNavVis; i += 64) vis[i] = -1;
  __threadfence_block();

  // key of list u: (ordered distance bits << 32) | u, the exact probe's distance
  auto key_of = [&](int u) -> uint64_t {
    float dist;
    if constexpr (INT) {
      const int4* cr = reinterpret_cast<const int4*>(ix.cent8 + (size_t)u * ix.dim_pad);
      const int4* qr = reinterpret_cast<const int4*>(qv);
      int dot = 0;
      for (int c = 0; c < ix.dim_pad / 16; ++c) {
        const int4 a = cr[c], b = qr[c];
        dot = __builtin_amdgcn_sdot4(a.x, b.x, dot, false);
        dot = __builtin_amdgcn_sdot4(a.y, b.y, dot, false);
        dot = __builtin_amdgcn_sdot4(a.z, b.z, dot, false);
        dot = __builtin_amdgcn_sdot4(a.w, b.w, dot, false);
      }
      dist = (float)(qn + ix.cnorm8[u] - 2 * dot);
    } else {
      const double* qd = reinterpret_cast<const double*>(qv);
      const float* c = ix.centroids + (size_t)u * ix.dim;
      double acc = 0.0;
      for (int t = 0; t < ix.dim; ++t) {
        const double x = qd[t] - (double)c[t];
        const double sq = x * x;
        acc = acc + sq;
      }
      dist = (float)acc;
    }
    return ((uint64_t)ord32(dist) << 32) | (uint32_t)u;
  };

  int cur = 0, cnt = 0;
  // Merge each lane's key (if `valid`) into C: drop duplicates and keys that
  // would land at or past B; every key's new position is its old position
  // plus the number of keys of the other side below it.
  auto merge = [&](uint64_t kk, bool valid) {
    int r = 0;
    if (valid) {
      int lo = 0, hi = cnt;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[cur][mid] < kk) lo = mid + 1;
        else hi = mid;
      }
      r = lo;
      if ((r < cnt && keys[cur][r] == kk) || r >= B) valid = false;
    }
    const uint64_t m = __ballot(valid);
    if (m == 0) return;
    const int nv = __popcll(m);
    if (valid) {
      const int slot = __popcll(m & below);
      nk[slot] = kk;
      nr[slot] = r;
    }
    __threadfence_block();
    const int dst = cur ^ 1;
    for (int i = lane; i < cnt; i += 64) {
      const uint64_t ki = keys[cur][i];
      int sb = 0;
      for (int t = 0; t < nv; ++t) sb += nk[t] < ki ? 1 : 0;
      const int pos = i + sb;
      if (pos < B) {
        keys[dst][pos] = ki;
        flg[dst][pos] = flg[cur][i];
      }
    }
    if (lane < nv) {
      const uint64_t kj = nk[lane];
      int sb = 0;
      for (int t = 0; t < nv; ++t) sb += nk[t] < kj ? 1 : 0;
      const int pos = nr[lane] + sb;
      if (pos < B) {
        keys[dst][pos] = kj;
        flg[dst][pos] = 0;
      }
    }
    __threadfence_block();
    cur = dst;
    cnt = min(B, cnt + nv);
  };

  for (int e0 = 0; e0 < ix.nav_nentry; e0 += 64) {
    const int e = e0 + lane;
    const bool valid = e < ix.nav_nentry;
    const int u = valid ? ix.nav_entry[e] : 0;
    if (valid) vis[nav_slot(u)] = u;
    merge(valid ? key_of(u) : ~0ull, valid);
  }
  // at most nlist expansions: a list enters C at most once
  for (int it = 0; it <= ix.nlist; ++it) {
    int i = -1;
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      const int c = c0 + lane;
      const uint64_t m = __ballot(c < cnt && flg[cur][c] == 0);
      if (m) {
        i = c0 + __ffsll((unsigned long long)m) - 1;
        break;
      }
    }
    if (i < 0) break;
    const int v = (int)(uint32_t)keys[cur][i];
    __threadfence_block();
    if (lane == 0) flg[cur][i] = 1;
    __threadfence_block();
    for (int j0 = 0; j0 < ix.nav_deg; j0 += 64) {
      const int j = j0 + lane;
      const int u = j < ix.nav_deg ? ix.nav_adj[(size_t)v * ix.nav_deg + j] : -1;
      bool valid = u >= 0 && u < ix.nlist;
      if (valid) {
        const uint32_t h = nav_slot(u);
        valid = vis[h] != u;
        __threadfence_block();
        if (valid) vis[h] = u;
      }
      merge(valid ? key_of(u) : ~0ull, valid);
    }
  }
  const int got = min(np, cnt);
  for (int p = lane; p < np_max; p += 64) {
    const uint64_t k = p < got ? keys[cur][p] : ~0ull;
    lists[(size_t)q * np_max + p] = p < got ? (int32_t)(uint32_t)k : -1;
    if (out_d) out_d[(size_t)q * np_max + p] = p < got ? unord32((uint32_t)(k >> 32)) : INFINITY;
  }
  if (lane == 0) np_eff[q] = got;
}

// Locality order of a chunk's queries: ascending (nearest probed list, query).
// One block; bitonic sort of 64-bit keys in LDS (qc <= kOrderMax).
constexpr int kOrderMax = 16384;

__global__ __launch_bounds__(kScanBlock) void k_order(const int32_t* __restrict__ lists,
                                                       const int32_t* __restrict__ np_eff,
                                                       int np_max, int qc,
                                                       int32_t* __restrict__ perm) {
  extern __shared__ __align__(16) uint64_t s_key[];
  const int P = pow2_at_least(qc);
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    uint64_t key = ~0ull;
    if (i < qc) {
      const uint32_t l = np_eff[i] > 0 ? (uint32_t)lists[(size_t)i * np_max] : 0xffffffffu;
      key = ((uint64_t)l << 32) | (uint32_t)i;
    }
    s_key[i] = key;
  }
  __syncthreads();
  block_bitonic(s_key, P);
  for (int i = threadIdx.x; i < qc; i += blockDim.x) perm[i] = (int32_t)(uint32_t)s_key[i];
}

// Segmented replica runs when their LDS bound stays small.
constexpr int kMaxSegRuns = 1024;

// Run slots of a scan block: room for every list's surviving replica groups
// when that worst case is small, else two runs per probed list, in which case
// a query's groups become runs only when they fit (the block checks).
inline bool scan_segmented(const DevIndex& ix, int) { return ix.segs != nullptr; }

// The scan kernel's static table: 4 * ceil(M / 4) subspaces of 256 entries.
inline size_t scan_table_bytes(const DevIndex& ix, bool lut16) {
  return (size_t)((ix.M + 3) / 4) * 4 * kKsub * (lut16 ? 2 : 4);
}
constexpr size_t kScanTwoPerCU = 80 * 1024;  // LDS of a scan block that still fits twice in a CU

// Past the worst-case bound, as many run slots as keep two blocks per CU next
// to the smallest top-n buffer (n + one round): at least two per probed list.
inline int scan_runs(const DevIndex& ix, int np_max, int n, bool lut16) {
  const int floor_runs = scan_max_runs(np_max, 0, false);
  if (ix.segs == nullptr) return floor_runs;
  const int worst = scan_max_runs(np_max, ix.max_segs, true);
  if (worst <= kMaxSegRuns) return worst;
  const size_t fixed = scan_table_bytes(ix, lut16) +
                       scan_layout(ix.M, ix.nlist, ix.R, np_max, 0, n + kScanBlock * kScanRT, 0).total;
  const int fit = fixed + 64 < kScanTwoPerCU ? (int)((kScanTwoPerCU - 64 - fixed) / 8) - 8 : 0;
  return std::max(floor_runs, std::min(worst, fit / 64 * 64));
}

template <int W>
hipError_t launch_scan_w(const DevIndex& ix, const int32_t* lists, const int32_t* np_eff,
                         int np_max, int qc, const float* Q, const float* lut, int32_t* sq,
                         int smax, int tile, int n, int cap, uint64_t* pkeys, int32_t* pcount,
                         int32_t* pscan, const int32_t* perm, bool trace, bool lut16,
                         int64_t t_capacity, int32_t* t_ids, float* t_adc, int64_t* t_count,
                         ScanSplit sp, hipStream_t st) {
  const int seg = scan_segmented(ix, np_max) ? 1 : 0;
  const int max_runs = scan_runs(ix, np_max, n, lut16);
  const ScanLayout L = scan_layout(ix.M, ix.nlist, ix.R, np_max, max_runs, cap, 0);
  const int qpad = (qc + 7) / 8 * 8;
  const dim3 grid((unsigned)((size_t)qpad * smax));
  if (trace) {
    auto kern = k_scan<W, true, false>;
    if (L.total > 65536)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
    hipLaunchKernelGGL(kern, grid, dim3(kScanBlock), L.total, st, ix, lists, np_eff, np_max, qc,
                       Q, lut, sq, smax, tile, seg, max_runs, n, cap, pkeys, pcount, pscan,
                       perm, t_capacity, t_ids, t_adc,
                       reinterpret_cast<unsigned long long*>(t_count), sp);
  } else {
    auto kern = lut16 ? k_scan<W, false, true> : k_scan<W, false, false>;
    if (L.total > 65536)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
    hipLaunchKernelGGL(kern, grid, dim3(kScanBlock), L.total, st, ix, lists, np_eff, np_max, qc,
                       Q, lut, sq, smax, tile, seg, max_runs, n, cap, pkeys, pcount, pscan,
                       perm, t_capacity, t_ids, t_adc,
                       reinterpret_cast<unsigned long long*>(t_count), sp);
  }
  return hipGetLastError();
}

using ScanFn = hipError_t (*)(const DevIndex&, const int32_t*, const int32_t*, int, int,
                              const float*, const float*, int32_t*, int, int, int, int, uint64_t*,
                              int32_t*, int32_t*, const int32_t*, bool, bool, int64_t, int32_t*,
                              float*, int64_t*, ScanSplit, hipStream_t);

template <int... Ws>
constexpr ScanFn scan_table_entry(int w, std::integer_sequence<int, Ws...>) {
  ScanFn f = nullptr;
  ((f = (w == Ws + 1) ? &launch_scan_w<Ws + 1> : f), ...);
  return f;
}

ScanFn scan_fn(int W) {
  return scan_table_entry(W, std::make_integer_sequence<int, kMaxM / 4>{});
}

// ---------------------------------------------------------------------------
// Batched form, list-major pass (integer-grid indexes).
//
// The per-query scan reads a list's code rows once for every query probing
// it.  In a large batch each list is probed by many queries, so here the
// chunk's (query, probed list) pairs are inverted into per-list groups of up
// to 16 queries, and a work item is (list, group, tile of the list's
// first-list rows).  One persistent launch pulls items from a device counter;
// an item reads each code row of its tile once, decodes it through the int8
// codebook in LDS, and scores it for the whole group on the int8 matrix
// cores:
//   Eq. 1 sum = ||q - dec(v)||^2 = ||q'||^2 + ||dec'(v)||^2 - 2 q'.dec'(v)
// (' = shifted to int8 as for the probe).  On an integer-grid index every
// term is an exact integer below 2^24, so the float32 value is bit-identical
// to the per-query table sum.
//
// The split of a query's entries: the per-query scan takes the first-list
// rows of its leading probed lists (until alpha * n rows) and the replica
// entries of all its probed lists (the ownership test needs the whole probe
// set); the list-major pass takes the first-list rows of the other probed
// lists, which are kept for every query (a vector's first list owns it).
// The per-query scan's n-th smallest key bounds the query's n-th smallest key
// from above, so the list-major pass keeps only keys below it, appended to
// the query's output area; a final per-query selection takes the n smallest
// of both parts.  A query whose area overflows is searched again by the plain
// per-query scan.  Every step is exact, so results equal the plain form's.

constexpr int kLmG = 16;       // queries per group (rows of the MFMA tile)
constexpr int kLmBlock = 256;  // threads per list-major block (4 waves)
constexpr int kLmU = 4;        // 16-row tiles per wave with loads in flight together

struct LmArgs {
  const int32_t* loff;   // [nlist + 1] start of each list's queries in invq
  const int32_t* ioff;   // [nlist + 1] start of each list's work items
  const int32_t* lcnt;   // [nlist] queries per list
  const int32_t* invq;   // queries by list
  const unsigned long long* thr;  // [qc] key bound per query
  int32_t* cnt2;         // [qc] keys appended (may exceed cap2: overflow)
  uint64_t* out2;        // [qc, cap2]
  int cap2;
  int32_t* ctr;          // [0] work items, [1] next item
  int tile_rows;
  int group;             // queries per group
};

// Per query: the first probed slot whose first-list rows may go to the
// list-major pass (the leading slots hold >= need rows, or all slots); its
// bound (none yet) and counters; per-list counters; the item counters.
__global__ void k_lm_prep(DevIndex ix, const int32_t* __restrict__ lists,
                          const int32_t* __restrict__ np_eff, int np_max, int qc, int64_t need,
                          int32_t* __restrict__ walkp, unsigned long long* __restrict__ thr,
                          int32_t* __restrict__ cnt2, uint8_t* __restrict__ flag,
                          int32_t* __restrict__ lcnt, int32_t* __restrict__ lfill,
                          int32_t* __restrict__ ctr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ix.nlist) {
    lcnt[i] = 0;
    lfill[i] = 0;
  }
  if (i < 4) ctr[i] = 0;
  if (i < qc) {
    const int np = np_eff[i];
    int P = np;
    int64_t acc = 0;
    for (int p = 0; p < np; ++p) {
      const int l = lists[(size_t)i * np_max + p];
      acc += ix.pstart[l + 1] - ix.pstart[l];
      if (acc >= need) {
        P = p + 1;
        break;
      }
    }
    walkp[i] = P;
    thr[i] = ~0ull;
    cnt2[i] = 0;
    flag[i] = 0;
  }
}

// (query, slot) pairs of the list-major pass: count per list, then fill.
__device__ __forceinline__ int lm_pair_list(const DevIndex& ix, const int32_t* lists,
                                            const int32_t* np_eff, const int32_t* walkp,
                                            int np_max, int qc, int min_rows, int i, int* q_out) {
  const int q = i / np_max, p = i % np_max;
  if (q >= qc || p >= np_eff[q]) return -1;
  const int l = lists[(size_t)q * np_max + p];
  if (!lm_slot(p, walkp[q], ix.pstart[l + 1] - ix.pstart[l], min_rows)) return -1;
  *q_out = q;
  return l;
}

__global__ void k_lm_count(DevIndex ix, const int32_t* __restrict__ lists,
                           const int32_t* __restrict__ np_eff, const int32_t* __restrict__ walkp,
                           int np_max, int qc, int min_rows, int32_t* __restrict__ lcnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int q;
  const int l = lm_pair_list(ix, lists, np_eff, walkp, np_max, qc, min_rows, i, &q);
  if (l >= 0) atomicAdd(&lcnt[l], 1);
}

__global__ void k_lm_fill(DevIndex ix, const int32_t* __restrict__ lists,
                          const int32_t* __restrict__ np_eff, const int32_t* __restrict__ walkp,
                          int np_max, int qc, int min_rows, const int32_t* __restrict__ loff,
                          int32_t* __restrict__ lfill, int32_t* __restrict__ invq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int q;
  const int l = lm_pair_list(ix, lists, np_eff, walkp, np_max, qc, min_rows, i, &q);
  if (l >= 0) invq[loff[l] + atomicAdd(&lfill[l], 1)] = q;
}

// Per-list query offsets and work-item offsets (exclusive prefix sums) and
// the item count, in two launches over blocks of 1024 lists: k_lm_offsets
// scans each block's lists and records the block's totals after ctr[4];
// k_lm_offsets_add adds the totals of the blocks before it.
__device__ __forceinline__ int lm_items(const DevIndex& ix, int l, int c, int group, int tile_rows) {
  if (c == 0) return 0;
  const int len = ix.pstart[l + 1] - ix.pstart[l];
  return ((c + group - 1) / group) * ((len + tile_rows - 1) / tile_rows);
}

__global__ __launch_bounds__(1024) void k_lm_offsets(DevIndex ix, const int32_t* __restrict__ lcnt,
                                                     int tile_rows, int group,
                                                     int32_t* __restrict__ loff,
                                                     int32_t* __restrict__ ioff,
                                                     int32_t* __restrict__ ctr) {
  __shared__ int s_a[17], s_b[17];
  const int nblk = (ix.nlist + 1023) / 1024;
  const int l = blockIdx.x * 1024 + threadIdx.x;
  const int c = l < ix.nlist ? lcnt[l] : 0;
  const int it = l < ix.nlist ? lm_items(ix, l, c, group, tile_rows) : 0;
  const int a = block_excl_scan(c, s_a);
  const int b = block_excl_scan(it, s_b);
  if (l < ix.nlist) {
    loff[l] = a;
    ioff[l] = b;
  }
  if (threadIdx.x == 1023) {
    ctr[4 + blockIdx.x] = a + c;
    ctr[4 + nblk + blockIdx.x] = b + it;
  }
}

__global__ __launch_bounds__(1024) void k_lm_offsets_add(DevIndex ix, int32_t* __restrict__ loff,
                                                         int32_t* __restrict__ ioff,
                                                         int32_t* __restrict__ ctr) {
  const int nblk = (ix.nlist + 1023) / 1024;  // <= 1024 (lmajor_supported)
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // totals of the blocks before this one (ta) and of all blocks (tot)
  int ta = 0, tb = 0, aa = 0, ab = 0;
  if (t < nblk) {
    aa = ctr[4 + t];
    ab = ctr[4 + nblk + t];
    if (t < (int)blockIdx.x) {
      ta = aa;
      tb = ab;
    }
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    ta += __shfl_xor(ta, d, 64);
    tb += __shfl_xor(tb, d, 64);
    aa += __shfl_xor(aa, d, 64);
    ab += __shfl_xor(ab, d, 64);
  }
  __shared__ int s_t[4][16];
  if (lane == 0) {
    s_t[0][w] = ta;
    s_t[1][w] = tb;
    s_t[2][w] = aa;
    s_t[3][w] = ab;
  }
  __syncthreads();
  ta = tb = aa = ab = 0;
  for (int i = 0; i < 16; ++i) {
    ta += s_t[0][i];
    tb += s_t[1][i];
    aa += s_t[2][i];
    ab += s_t[3][i];
  }
  const int l = blockIdx.x * 1024 + t;
  if (l < ix.nlist) {
    loff[l] += ta;
    ioff[l] += tb;
  }
  if (blockIdx.x == 0 && t == 0) {
    loff[ix.nlist] = aa;
    ioff[ix.nlist] = ab;
    ctr[0] = ab;
  }
}

// Work item `it`: its list (largest l with ioff[l] <= it), query group and
// row tile -> s_it[1..4] = queries in the group, first row, end row, first
// slot of the group in invq.  Groups of one tile are adjacent items.  Called
// by every lane of one wave: the list is found by a 64-way search (each
// round probes 64 points of the remaining range at once, so 65,536 lists
// take three dependent loads), lane 0 writes the result.
__device__ __forceinline__ void lm_item(const DevIndex& ix, const LmArgs& a, int it, int G,
                                        int* s_it) {
  const int lane = threadIdx.x & 63;
  int lo = 0, hi = ix.nlist - 1;  // the list is in [lo, hi]; ioff[0] = 0 <= it
  while (hi > lo) {                // wave-uniform
    // probes in (lo, hi], nondecreasing with the lane, the last at hi: the
    // lanes whose probe passes form a prefix
    const int pr = lo + (int)(((int64_t)(hi - lo) * (lane + 1) + 63) / 64);
    const int np = __popcll(__ballot(a.ioff[pr] <= it));
    const int nlo = np > 0 ? __shfl(pr, np - 1, 64) : lo;
    const int nhi = np < 64 ? __shfl(pr, np, 64) - 1 : hi;
    lo = nlo;
    hi = nhi;
  }
  if (lane != 0) return;
  const int l = lo, local = it - a.ioff[l], nql = a.lcnt[l];
  const int ng = (nql + G - 1) / G;
  const int grp = local % ng, tile = local / ng;
  const int r0 = ix.pstart[l] + tile * a.tile_rows;
  s_it[1] = min(G, nql - grp * G);
  s_it[2] = r0;
  s_it[3] = min(ix.pstart[l + 1], r0 + a.tile_rows);
  s_it[4] = a.loff[l] + grp * G;
}

// The code dwords a lane needs for K chunk kc of a row: codes (kc*64 + 16g)/DS
// onward, 16/DS of them.  Offsets past the row (padding subspaces) are
// clamped to the row's first dword: those codes look up the zero codewords
// of the padded LDS codebook whatever their value.
template <int DS>
struct LmCodes {
  static constexpr int NC = 16 / DS;            // codes per lane and chunk
  static constexpr int ND = NC >= 4 ? NC / 4 : 1;  // code dwords per lane and chunk
};

// Decoded bytes [kb, kb + 16) from the code dwords w (first code at byte
// b0 of w[0]); cb: this lane's LDS codebook base for the chunk (subspace
// kb / DS).  Padded subspaces are all-zero codewords.
template <int DS>
__device__ __forceinline__ v4i_t lm_decode(const unsigned char* __restrict__ cb,
                                           const uint32_t (&w)[LmCodes<DS>::ND], int b0) {
  constexpr int NC = LmCodes<DS>::NC;
  constexpr int kSub = kKsub * DS;  // bytes per subspace
  auto code = [&](int j) -> uint32_t {  // byte j of the lane's codes
    const int b = (DS == 8 ? b0 : 0) + j;
    return (w[b >> 2] >> (8 * (b & 3))) & 255u;
  };
  v4i_t out;
  if constexpr (DS == 1) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v |= (uint32_t)cb[(4 * d + j) * kSub + code(4 * d + j)] << (8 * j);
      out[d] = (int)v;
    }
  } else if constexpr (DS == 2) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const uint32_t lo = *reinterpret_cast<const uint16_t*>(cb + (2 * d) * kSub + 2 * code(2 * d));
      const uint32_t hi =
          *reinterpret_cast<const uint16_t*>(cb + (2 * d + 1) * kSub + 2 * code(2 * d + 1));
      out[d] = (int)(lo | (hi << 16));
    }
  } else if constexpr (DS == 4) {
#pragma unroll
    for (int d = 0; d < 4; ++d)
      out[d] = *reinterpret_cast<const int*>(cb + d * kSub + 4 * code(d));
  } else {  // DS == 8
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const uint2 v = *reinterpret_cast<const uint2*>(cb + d * kSub + 8 * code(d));
      out[2 * d] = (int)v.x;
      out[2 * d + 1] = (int)v.y;
    }
  }
  (void)NC;
  return out;
}

__device__ __forceinline__ int sq_bytes(v4i_t v, int acc) {
  acc = __builtin_amdgcn_sdot4(v[0], v[0], acc, false);
  acc = __builtin_amdgcn_sdot4(v[1], v[1], acc, false);
  acc = __builtin_amdgcn_sdot4(v[2], v[2], acc, false);
  return __builtin_amdgcn_sdot4(v[3], v[3], acc, false);
}

// Sum of x over the four 16-lane groups (lanes l, l ^ 16, l ^ 32, l ^ 48),
// in every lane: each swap exchanges a half (a pair of rows) of two copies
// of x, so the two copies' sum holds both halves.
__device__ __forceinline__ int sum_lane_groups(int x) {
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
  const int y = (int)h[0] + (int)h[1];
  const auto r = __builtin_amdgcn_permlane16_swap((unsigned)y, (unsigned)y, false, false);
  return (int)r[0] + (int)r[1];
}

// Largest integer distance d >= 0 whose key's high word (the bits of
// (float)d with the sign bit set) is <= hi, capped at 2^26 (the distances
// of an integer-grid index stay below 2^24); -1 if there is none.
__device__ __forceinline__ int lm_dist_limit(uint32_t hi) {
  if (hi < 0x80000000u) return -1;
  const uint32_t b = hi & 0x7fffffffu;
  if (b >= 0x4c800000u) return 1 << 26;  // (float)2^26 and above, inf, NaN patterns
  return (int)floorf(__uint_as_float(b));
}

// LDS codebook bytes of the list-major kernel: the lane groups (16 bytes of
// a K chunk: 16 / dsub subspaces of 256 codewords of dsub bytes, 4096 bytes)
// that hold at least one of the M subspaces; the subspaces past M inside
// them are all zero.
__host__ __device__ inline int lm_cb_bytes(int M, int dsub) {
  const int per = 16 / dsub;
  return (M + per - 1) / per * 16 * kKsub;
}

// The persistent list-major kernel.  KC = dim_pad / 64 (K chunks of one
// MFMA), DS = dsub.  Wave w of a block takes 16-row tiles w, w + 4, ... of
// the item, kLmU of them per round with all their loads (code dwords and
// external IDs) in flight together.  Lane (r, g) (r = lane % 16, g =
// lane / 16) holds query row r's and candidate r's bytes [16g, 16g + 16) of
// each K chunk, and after the MFMA the products of queries 4g..4g+3 with
// candidate r.
// Least waves per SIMD the list-major kernel is compiled for: five (at most
// 96 registers) where that needs no spill, else no bound.
constexpr int lm_waves(int kc, int ds) {
  return kc == 1 || (kc == 2 && ds >= 2) || (kc == 3 && ds >= 4) ? 5 : 1;
}

template <int KC, int DS>
__global__ __launch_bounds__(kLmBlock) __attribute__((amdgpu_waves_per_eu(lm_waves(KC, DS))))
void k_lm_mfma(DevIndex ix, const float* __restrict__ Q,
                                                      LmArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int Dp = KC * 64;
  constexpr int ND = LmCodes<DS>::ND;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int cb_bytes = lm_cb_bytes(ix.M, DS);
  unsigned char* s_cb = smem;
  int8_t* s_q8 = reinterpret_cast<int8_t*>(smem + cb_bytes);  // [16][Dp]
  unsigned long long* s_thr =
      reinterpret_cast<unsigned long long*>(smem + cb_bytes + kLmG * Dp);  // [16]
  int* s_qid = reinterpret_cast<int*>(s_thr + kLmG);                      // [16]
  int* s_it = s_qid + kLmG;  // item, queries, first row, end row, first query slot
  {  // codebook, zero-padded to whole lane groups
    const int real16 = (ix.M * kKsub * DS + 15) / 16;
    for (int i = tid; i < cb_bytes / 16; i += kLmBlock)
      reinterpret_cast<int4*>(s_cb)[i] =
          i < real16 ? reinterpret_cast<const int4*>(ix.cb8)[i] : int4{0, 0, 0, 0};
  }
  // Per lane: the code dwords of chunk kc sit at lane_off + 64 kc / DS + 4 i
  // in a row (the lane's first code at byte b0[kc] of the first dword);
  // cbk[kc]: the LDS codebook of that first code's subspace.  Dwords past
  // the row's M codes read the next row's bytes (the buffer keeps slack
  // after its last row).  In a lane group that holds a real subspace those
  // codes index padded subspaces, whose LDS codewords are all zero; a lane
  // group past the M subspaces (real[kc] false) decodes through the first
  // group's codewords instead: its query bytes are zero, so it adds nothing
  // to the product, and its bytes are left out of the norm.
  const uint32_t lane_off = (uint32_t)((16 * g / DS) & ~3);
  int b0[KC];
  bool real[KC];
  const unsigned char* cbk[KC];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    const int m0 = (kc * 64 + 16 * g) / DS;
    b0[kc] = m0 & 3;
    real[kc] = m0 < ix.M;
    cbk[kc] = s_cb + (real[kc] ? m0 * kKsub * DS : 0);
  }
  const int nitems = a.ctr[0];
  for (;;) {
    if (tid < 64) {  // wave 0 takes the next item and looks it up
      int it = 0;
      if (tid == 0) it = atomicAdd(&a.ctr[1], 1);
      it = __shfl(it, 0, 64);
      if (tid == 0) s_it[0] = it;
      if (it < nitems) lm_item(ix, a, it, kLmG, s_it);
    }
    __syncthreads();
    if (s_it[0] >= nitems) break;  // block-uniform
    const int gcnt = s_it[1], row0 = s_it[2], row1 = s_it[3], qbase = s_it[4];
    if (tid < kLmG) {
      const int qid = tid < gcnt ? a.invq[qbase + tid] : -1;
      s_qid[tid] = qid;
      s_thr[tid] = qid >= 0 ? a.thr[qid] : 0ull;  // 0: an empty row never passes
    }
    __syncthreads();
    for (int i = tid; i < kLmG * Dp; i += kLmBlock) {  // queries as shifted int8, zero-padded
      const int qi = i / Dp, t = i % Dp, qid = s_qid[qi];
      int v = 0;
      if (qid >= 0 && t < ix.dim)
        v = (int)conv_query(Q[(size_t)qid * ix.dim + t], ix.dtype) - ix.shift8;
      s_q8[i] = (int8_t)v;
    }
    __syncthreads();
    v4i_t fa[KC];
    int qn_r = 0;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      fa[kc] = *reinterpret_cast<const v4i_t*>(s_q8 + r16 * Dp + kc * 64 + 16 * g);
      qn_r = sq_bytes(fa[kc], qn_r);
    }
    qn_r += __shfl_xor(qn_r, 16, 64);
    qn_r += __shfl_xor(qn_r, 32, 64);  // ||q'||^2 of query row r16
    int qn[4], qid[4];
    unsigned long long th[4];
    int lim[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      qn[r] = __shfl(qn_r, 4 * g + r, 64);
      qid[r] = s_qid[4 * g + r];
      th[r] = s_thr[4 * g + r];
      // rn - 2 acc <= lim[r] exactly when the key's high word is within the
      // bound's (lm_dist_limit); qn <= 2^23 and 2 |acc| <= 2^23 keep the
      // per-row test free of overflow
      lim[r] = lm_dist_limit((uint32_t)(th[r] >> 32)) - qn[r];
    }
    constexpr int kStep = 16 * (kLmBlock / 64);
    // the item's rows from block-uniform bases, so that every load takes a
    // 32-bit lane offset (rows per item <= 2^24, row_bytes <= 256)
    const int nrows = __builtin_amdgcn_readfirstlane(row1 - row0);
    const int r0u = __builtin_amdgcn_readfirstlane(row0);
    const unsigned char* icodes = ix.codes + (size_t)r0u * ix.row_bytes;
    const unsigned char* iext = reinterpret_cast<const unsigned char*>(ix.row2ext + r0u);
    for (int rel0 = 16 * wv; rel0 < nrows; rel0 += kStep * kLmU) {
      uint32_t cw[kLmU][KC][ND];
      uint32_t ext[kLmU];
      uint32_t voff[kLmU];
#pragma unroll
      for (int u = 0; u < kLmU; ++u) {  // every load of the round first, external IDs leading
        const int rel = rel0 + u * kStep + r16;
        const uint32_t rc = rel < nrows ? (uint32_t)rel : 0u;  // past the item: its first row
        ext[u] = *reinterpret_cast<const uint32_t*>(iext + 4u * rc);
        voff[u] = __umul24(rc, (uint32_t)ix.row_bytes) + lane_off;
      }
#pragma unroll
      for (int u = 0; u < kLmU; ++u)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
          for (int i = 0; i < ND; ++i)
            cw[u][kc][i] =
                *reinterpret_cast<const uint32_t*>(icodes + voff[u] + (kc * 64 / DS + 4 * i));
      __builtin_amdgcn_sched_barrier(0);  // every load issued before the first decode
      // the IDs are used only when a key may pass; keep their loads here (in
      // flight with the codes) rather than issued late on that rare path
#pragma unroll
      for (int u = 0; u < kLmU; ++u) asm volatile("" ::"v"(ext[u]));
#pragma unroll
      for (int u = 0; u < kLmU; ++u) {
        const int rel = rel0 + u * kStep + r16;
        int rn = 0;
        v4i_t acc = v4i_t{0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
          const v4i_t fb = lm_decode<DS>(cbk[kc], cw[u][kc], b0[kc]);
          const int rs = sq_bytes(fb, rn);
          rn = real[kc] ? rs : rn;
          acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[kc], fb, acc, 0, 0, 0);
        }
        rn = sum_lane_groups(rn);  // ||dec'||^2 of candidate r16
        uint64_t may = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) may |= __ballot(rn <= lim[r] + 2 * acc[r]);
        if (may == 0) continue;  // wave-uniform: no key can pass
        const bool rv = rel < nrows;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // d >= 0 is an exact integer: its order-preserving bits are bits | 2^31
          const uint32_t h = __float_as_uint((float)(qn[r] + rn - 2 * acc[r])) | 0x80000000u;
          const uint64_t key = ((uint64_t)h << 32) | ext[u];
          const bool pass = rv && key < th[r];
          const uint64_t m = __ballot(pass);
          if (m) {  // wave-uniform; append: one atomic per (query, 16-lane group)
            const uint32_t seg = (uint32_t)(m >> (16 * g)) & 0xffffu;
            const int leader = seg ? 16 * g + __ffs(seg) - 1 : lane;
            int pos0 = 0;
            if (pass && lane == leader) pos0 = atomicAdd(&a.cnt2[qid[r]], __popc(seg));
            pos0 = __shfl(pos0, leader, 64);
            if (pass) {
              const int pos = pos0 + __popc(seg & ((1u << (lane - 16 * g)) - 1u));
              if (pos < a.cap2) a.out2[(size_t)qid[r] * a.cap2 + pos] = key;
            }
          }
        }
      }
    }
    __syncthreads();  // the next item restages the queries
  }
}

// The persistent list-major kernel for float indexes: Eq. 1 by table
// lookups, as in the per-query scan.  The group's G distance tables (taken
// from the chunk's table buffer) are staged in LDS interleaved by query --
// entry (m, j) of the G queries is one 16-byte word: G = 4 float32 entries,
// or G = 8 binary16 entries in the half-precision variant -- so each code of
// a row is one LDS read for the whole group.  A thread scores kLutU rows per
// round for all G queries, each sum in float32 over m = 0..M-1 from +0.0f
// (the per-query scan's order, hence its bits).
constexpr int kLutBlock = 1024;  // threads per block (one block per CU: tables take most of LDS)
constexpr int kLutU = 2;         // rows per thread and round
constexpr int kLutMaxW = 9;      // up to 36 subspaces (4 * 9 * 256 * 16 bytes of tables)

template <int W, bool H>
__global__ __launch_bounds__(kLutBlock) void k_lm_lut(DevIndex ix, const float* __restrict__ lut,
                                                      LmArgs a) {
  constexpr int G = H ? 8 : 4;
  constexpr int MS = 4 * W;  // table subspaces (those past M unused)
  extern __shared__ __align__(16) unsigned char smem[];
  uint4* s_t = reinterpret_cast<uint4*>(smem);  // [MS * 256]
  unsigned long long* s_thr = reinterpret_cast<unsigned long long*>(smem + MS * kKsub * 16);
  int* s_qid = reinterpret_cast<int*>(s_thr + G);  // [G]
  int* s_it = s_qid + G;
  const int tid = threadIdx.x, lane = tid & 63;
  const int M = ix.M;
  const uint64_t lanemask = (1ull << lane) - 1ull;
  const int nitems = a.ctr[0];
  for (;;) {
    if (tid < 64) {  // wave 0 takes the next item and looks it up
      int it = 0;
      if (tid == 0) it = atomicAdd(&a.ctr[1], 1);
      it = __shfl(it, 0, 64);
      if (tid == 0) s_it[0] = it;
      if (it < nitems) lm_item(ix, a, it, G, s_it);
    }
    __syncthreads();
    if (s_it[0] >= nitems) break;  // block-uniform
    const int gcnt = s_it[1], row0 = s_it[2], row1 = s_it[3], qbase = s_it[4];
    if (tid < G) {
      const int qid = tid < gcnt ? a.invq[qbase + tid] : -1;
      s_qid[tid] = qid;
      s_thr[tid] = qid >= 0 ? a.thr[qid] : 0ull;  // 0: an empty slot never passes
    }
    __syncthreads();
    int qid[G];
#pragma unroll
    for (int g = 0; g < G; ++g) qid[g] = s_qid[g];
    for (int i = tid; i < M * kKsub; i += kLutBlock) {  // the group's tables, interleaved
      float v[G];
#pragma unroll
      for (int g = 0; g < G; ++g) v[g] = qid[g] >= 0 ? lut[(size_t)qid[g] * M * kKsub + i] : 0.f;
      uint4 wv;
      if constexpr (H) {  // nearest binary16, ties to even (as the per-query scan's variant)
        uint32_t hw[4];
#pragma unroll
        for (int d = 0; d < 4; ++d)
          hw[d] = (uint32_t)__half_as_ushort(__float2half_rn(v[2 * d])) |
                  ((uint32_t)__half_as_ushort(__float2half_rn(v[2 * d + 1])) << 16);
        wv = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      } else {
        wv = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                        __float_as_uint(v[3]));
      }
      s_t[i] = wv;
    }
    unsigned long long th[G];
    uint32_t th_hi[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      th[g] = s_thr[g];
      th_hi[g] = (uint32_t)(th[g] >> 32);
    }
    __syncthreads();
    for (int base = row0; base < row1; base += kLutBlock * kLutU) {  // uniform trip count
      uint32_t cw[kLutU][W];
      uint32_t ext[kLutU];
      int rr[kLutU];
#pragma unroll
      for (int u = 0; u < kLutU; ++u) {
        const int row = base + u * kLutBlock + tid;
        rr[u] = row < row1 ? row : row0;
        ext[u] = (uint32_t)ix.row2ext[rr[u]];
      }
#pragma unroll
      for (int u = 0; u < kLutU; ++u) load_row<W>(ix.codes + (size_t)rr[u] * ix.row_bytes, cw[u]);
#pragma unroll
      for (int u = 0; u < kLutU; ++u) asm volatile("" ::"v"(ext[u]));
#pragma unroll
      for (int u = 0; u < kLutU; ++u) {
        const bool rv = base + u * kLutBlock + tid < row1;
        float acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0.f;
#pragma unroll
        for (int i = 0; i < W; ++i) {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int m = 4 * i + b;
            if (i < W - 1 || m < M) {
              const uint4 e = s_t[m * kKsub + ((cw[u][i] >> (8 * b)) & 255u)];
              const uint32_t ew[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
              for (int g = 0; g < G; ++g) {
                float x;
                if constexpr (H)
                  x = __half2float(__ushort_as_half((unsigned short)(ew[g >> 1] >> (16 * (g & 1)))));
                else
                  x = __uint_as_float(ew[g]);
                acc[g] = acc[g] + x;
              }
            }
          }
        }
        uint32_t h[G];
        bool c = false;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          h[g] = ord32(acc[g]);
          c = c || h[g] <= th_hi[g];
        }
        if (__ballot(c) == 0) continue;  // wave-uniform: no key can pass
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const uint64_t key = ((uint64_t)h[g] << 32) | ext[u];
          const bool pass = rv && key < th[g];
          const uint64_t m = __ballot(pass);
          if (m) {  // wave-uniform: one atomic per query and wave
            int pos0 = 0;
            if (lane == __ffsll((unsigned long long)m) - 1)
              pos0 = atomicAdd(&a.cnt2[qid[g]], __popcll(m));
            pos0 = __shfl(pos0, __ffsll((unsigned long long)m) - 1, 64);
            if (pass) {
              const int pos = pos0 + __popcll(m & lanemask);
              if (pos < a.cap2) a.out2[(size_t)qid[g] * a.cap2 + pos] = key;
            }
          }
        }
      }
    }
    __syncthreads();  // the next item restages the tables
  }
}

// Per query: the n smallest of the per-query scan's item keys and the
// list-major keys, into item 0 (sq = 1), with the work counts; a query whose
// list-major area overflowed is flagged for a full per-query scan instead.
__global__ __launch_bounds__(kBlock) void k_lm_select(
    DevIndex ix, const int32_t* __restrict__ lists, const int32_t* __restrict__ np_eff,
    int np_max, const int32_t* __restrict__ walkp, int min_rows, int smax, int n,
    uint64_t* __restrict__ pkeys,
    int32_t* __restrict__ pcount, int32_t* __restrict__ pscan, int32_t* __restrict__ sq,
    const int32_t* __restrict__ cnt2, const uint64_t* __restrict__ out2, int cap2,
    uint8_t* __restrict__ flag) {
  extern __shared__ __align__(16) uint64_t s_top[];  // [n]
  __shared__ SelScratch ss;
  __shared__ int s_off[17];
  __shared__ int s_cnt, s_sc, s_sw;
  const int q = blockIdx.x, tid = threadIdx.x;
  const int c2 = cnt2[q];
  if (c2 > cap2) {
    if (tid == 0) flag[q] = 1;
    return;
  }
  const int S = sq[q];
  const size_t it0 = (size_t)q * smax;
  if (tid < 64) {
    int c = 0, sc = 0, sw = 0;
    if (tid < S) {
      c = pcount[it0 + tid];
      sc = pscan[2 * (it0 + tid)];
      sw = pscan[2 * (it0 + tid) + 1];
    }
    const int incl = (int)wave_incl_scan((uint32_t)c);
    if (tid < S) s_off[tid] = incl - c;
    if (tid == S - 1) s_off[S] = incl;
    const int np = np_eff[q], wp = walkp[q];
    for (int p = min(np, wp) + tid; p < np; p += 64) {  // rows of the list-major part
      const int l = lists[(size_t)q * np_max + p];
      const int r = ix.pstart[l + 1] - ix.pstart[l];
      if (lm_slot(p, wp, r, min_rows)) {
        sc += r;
        sw += r;
      }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      sc += __shfl_xor(sc, d, 64);
      sw += __shfl_xor(sw, d, 64);
    }
    if (tid == 0) {
      s_sc = sc;
      s_sw = sw;
      s_cnt = 0;
    }
  }
  __syncthreads();
  const int t1 = s_off[S], total = t1 + c2;
  auto get = [&](int i) -> uint64_t {
    if (i < t1) {
      int j = 0;
      while (j + 1 < S && s_off[j + 1] <= i) ++j;
      return pkeys[(it0 + j) * n + (i - s_off[j])];
    }
    return out2[(size_t)q * cap2 + (i - t1)];
  };
  const uint64_t K = total > n ? block_kth(get, total, n, &ss) : ~0ull;
  for (int i = tid; i < total; i += kBlock) {
    const uint64_t k = get(i);
    if (k <= K) {
      const int pos = atomicAdd(&s_cnt, 1);
      if (pos < n) s_top[pos] = k;
    }
  }
  __syncthreads();  // every read of item 0 is done
  const int cnt = min(s_cnt, n);
  for (int i = tid; i < cnt; i += kBlock) pkeys[it0 * n + i] = s_top[i];
  if (tid == 0) {
    pcount[it0] = cnt;
    pscan[2 * it0] = s_sc;
    pscan[2 * it0 + 1] = s_sw;
    sq[q] = 1;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

int scan_smax(int n) { return std::max(1, std::min(16, 4096 / std::max(n, 1))); }

// Top-n buffer slots of a scan block: n + one round of entries at least;
// more slack (fewer cut-backs) while the block still fits twice in a CU's LDS.
int scan_cap(const DevIndex& ix, int np_max, int n, bool lut16) {
  constexpr size_t kTwoPerCU = kScanTwoPerCU;
  constexpr int kRound = kScanBlock * kScanRT;
  const int base = n + kRound;
  const size_t fixed = scan_table_bytes(ix, lut16) +
                       scan_layout(ix.M, ix.nlist, ix.R, np_max, scan_runs(ix, np_max, n, lut16), 0,
                                   0).total;
  int extra = 0;
  if (fixed + (size_t)base * 8 + 64 < kTwoPerCU)
    extra = (int)((kTwoPerCU - 64 - fixed - (size_t)base * 8) / 8) / 64 * 64;
  return std::min(base + std::min(extra, 2 * kRound), kCompactChunk * kScanBlock);
}

size_t scan_lds_bytes(const DevIndex& ix, int np_max, int n, bool lut16) {
  return scan_table_bytes(ix, lut16) + scan_layout(ix.M, ix.nlist, ix.R, np_max,
                                                   scan_runs(ix, np_max, n, lut16),
                                                   scan_cap(ix, np_max, n, lut16), 0).total;
}

static bool exact64(const DevIndex& ix) { return !ix.int_grid; }

hipError_t launch_probe(const DevIndex& ix, const float* q, const int32_t* nprobe, int np_max,
                        int qc, Work& w, float* out_dists_opt, int32_t* out_lists,
                        hipStream_t st) {
  if (qc <= 0) return hipSuccess;
  if (ix.nav_beam > 0) {  // beam walk of the navigation graph
    if (!ix.nav_adj || np_max > kNavMaxBeam || ix.nav_beam > kNavMaxBeam) return hipErrorInvalidValue;
    const int cap = (std::max(ix.nav_beam, np_max) + 63) / 64 * 64;
    const int wpb = cap <= 256 ? 4 : 1;  // waves (queries) per block
    const size_t lds = (size_t)wpb * nav_wave_bytes(ix.dim, ix.dim_pad, cap);
    auto kern = ix.cent8 ? k_probe_graph<true> : k_probe_graph<false>;
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
    hipLaunchKernelGGL(kern, dim3((qc + wpb - 1) / wpb), dim3(64 * wpb), lds, st, ix, q, qc,
                       nprobe, np_max, cap, out_lists, out_dists_opt, w.np_eff);
    return hipGetLastError();
  }
  if (ix.cent8 && np_max <= 128 && ix.dim_pad <= 128 && qc >= kFusedMinQueries) {
    // integer grid, large batch: fused distances + selection, no distance
    // matrix in HBM (a block walks all lists for its 8 queries, so small
    // batches would leave most of the GPU idle: they take the two-kernel path)
    const dim3 g((qc + kFQ - 1) / kFQ);
    auto kern = np_max <= 64 ? (ix.dim_pad == 64 ? k_probe_fused<64, 1> : k_probe_fused<64, 2>)
                             : (ix.dim_pad == 64 ? k_probe_fused<128, 1> : k_probe_fused<128, 2>);
    const size_t lds = np_max <= 64 ? fused_lds<64>(ix) : fused_lds<128>(ix);
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
    hipLaunchKernelGGL(kern, g, dim3(kBlock), lds, st, ix, q, qc, nprobe, np_max, out_lists,
                       out_dists_opt, w.np_eff);
    return hipGetLastError();
  }
  if (ix.cent8) {
    const dim3 g((ix.nlist + kPN - 1) / kPN, (qc + kPM - 1) / kPM);
    const size_t lds = (size_t)kPM * ix.dim_pad + kPM * 4;
    hipLaunchKernelGGL(k_probe_mfma, g, dim3(kBlock), lds, st, ix, q, qc, w.dist);
  } else {
    const dim3 g1((ix.nlist + kBlock - 1) / kBlock, (qc + kProbeQT - 1) / kProbeQT);
    const size_t lds1 = (size_t)kProbeQT * ix.dim * 4;
    if (exact64(ix))
      hipLaunchKernelGGL(k_probe_dist<true>, g1, dim3(kBlock), lds1, st, ix, q, qc, w.dist);
    else
      hipLaunchKernelGGL(k_probe_dist<false>, g1, dim3(kBlock), lds1, st, ix, q, qc, w.dist);
  }
  const size_t lds2 = (size_t)std::max(pow2_at_least(np_max), kSelCand) * 8;
  if (lds2 > 65536)
    (void)hipFuncSetAttribute((const void*)k_probe_select,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
  hipLaunchKernelGGL(k_probe_select, dim3(qc), dim3(kBlock), lds2, st, w.dist, ix.nlist, nprobe,
                     np_max, out_lists, out_dists_opt, w.np_eff);
  return hipGetLastError();
}

hipError_t launch_lut(const DevIndex& ix, const float* q, int qc, float* out_lut, hipStream_t st) {
  if (qc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lut, dim3(qc), dim3(kKsub), 0, st, ix, q, qc, out_lut);
  return hipGetLastError();
}

hipError_t launch_scan(const DevIndex& ix, const int32_t* lists, const int32_t* np_eff,
                       const float* q, const LaunchCfg& c, Work& w, hipStream_t st) {
  if (c.qc <= 0) return hipSuccess;
  const int W = (ix.M + 3) / 4;
  const int cap = scan_cap(ix, c.np_max, c.n, c.lut16);
  const int32_t* perm = nullptr;
  if (c.order && c.qc > 8 && c.qc <= kOrderMax) {
    const int P = pow2_at_least(c.qc);
    const size_t lds = (size_t)P * 8;
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void*)k_order, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
    hipLaunchKernelGGL(k_order, dim3(1), dim3(kScanBlock), lds, st, lists, np_eff, c.np_max, c.qc,
                       w.perm);
    perm = w.perm;
  }
  return scan_fn(W)(ix, lists, np_eff, c.np_max, c.qc, q, nullptr, w.sq, c.smax, c.tile, c.n, cap,
                    w.pkeys, w.pcount, w.pscan, perm, false, c.lut16, 0, nullptr, nullptr, nullptr,
                    ScanSplit{}, st);
}

hipError_t launch_scan_trace(const DevIndex& ix, const int32_t* lists, const float* lut, int qc,
                             int np_max, int64_t capacity, int32_t* out_ids, float* out_adc,
                             int64_t* out_count, Work& w, hipStream_t st) {
  if (qc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_lists, dim3((qc + 255) / 256), dim3(256), 0, st, lists, qc, np_max,
                     ix.nlist, w.np_eff);
  const int smax = 16, tile = 4096;
  hipLaunchKernelGGL(k_zero_i64, dim3((qc + 255) / 256), dim3(256), 0, st, out_count, qc);
  const int W = (ix.M + 3) / 4;
  return scan_fn(W)(ix, lists, w.np_eff, np_max, qc, nullptr, lut, w.sq, smax, tile, 1, 1, nullptr,
                    nullptr, nullptr, nullptr, true, false, capacity, out_ids, out_adc, out_count,
                    ScanSplit{}, st);
}

hipError_t launch_merge(const DevIndex& ix, const float* q, const LaunchCfg& c, Work& w,
                        int32_t* topn_ids, float* topn_adc, int64_t* ncand, int64_t* nwalk,
                        int64_t* out_ids, float* out_dists, int32_t* reranked,
                        int32_t* page_reads, hipStream_t st) {
  if (c.qc <= 0) return hipSuccess;
  const MergeLayout L = merge_layout(c.smax, c.n, ix.dim);
  const bool heur = c.hb > 0 && out_ids;
  if (ix.hpages && out_ids) {
    // raw vectors in host memory: 256-thread blocks, a page buffer per wave
    const size_t lds = L.total + page_scratch_bytes(pow2_at_least(c.n), 256 / 64, ix.page_bytes);
    auto kern = heur ? k_merge<256, true, true> : k_merge<256, false, true>;
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
    hipLaunchKernelGGL(kern, dim3(c.qc), dim3(256), lds, st, ix, q, c.qc, w.sq, c.smax, c.n, c.k,
                       w.pkeys, w.pcount, w.pscan, topn_ids, topn_adc, ncand, nwalk, out_ids,
                       out_dists, c.hb, c.h_eps, c.h_beta, reranked, page_reads);
    return hipGetLastError();
  }
  // More threads only pay off when there are many candidates to re-rank.
  // Then four 512-thread blocks per CU, where their LDS fits, beat two of
  // 1024: while one block sits in its barrier-bound selection and sort, the
  // others' row gathers keep memory busy (rerank_n 600: 0.34 -> 0.26 ms;
  // heuristic rerank_n 2000: 1.73 -> 1.25 ms).
  const int bs = c.n <= 512 ? 256 : 4 * L.total <= (size_t)kLdsPerCu ? 512 : kMergeBlock;
  auto kern = heur ? (bs == 256   ? k_merge<256, true>
                      : bs == 512 ? k_merge<512, true>
                                  : k_merge<kMergeBlock, true>)
                   : (bs == 256   ? k_merge<256, false>
                      : bs == 512 ? k_merge<512, false>
                                  : k_merge<kMergeBlock, false>);
  if (L.total > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
  hipLaunchKernelGGL(kern, dim3(c.qc), dim3(bs), L.total, st, ix, q, c.qc, w.sq, c.smax,
                     c.n, c.k, w.pkeys, w.pcount, w.pscan, topn_ids, topn_adc, ncand, nwalk, out_ids,
                     out_dists, c.hb, c.h_eps, c.h_beta, reranked, nullptr);
  return hipGetLastError();
}

hipError_t launch_rerank_only(const DevIndex& ix, const float* q, const int32_t* cand, int qc,
                              int n, int k, int64_t* out_ids, float* out_dists, hipStream_t st) {
  if (qc <= 0) return hipSuccess;
  const int P = pow2_at_least(n);
  const size_t lds = (size_t)P * 16 + (size_t)ix.dim * 4 + 16;
  const bool big = n > 512;
  auto kern = big ? k_rerank_only<kMergeBlock> : k_rerank_only<256>;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(kern, dim3(qc), dim3(big ? kMergeBlock : 256), lds, st, ix, q, cand, n, k, out_ids,
                     out_dists);
  return hipGetLastError();
}

}  // namespace ann

namespace ann {

// ---------------------------------------------------------------------------
// Batched form: the list-major pass (see k_lm_mfma).

// Integer-grid indexes: decode + int8 MFMA (k_lm_mfma); float indexes:
// interleaved tables (k_lm_lut).
bool lmajor_mfma(const DevIndex& ix) {
  return ix.int_grid && ix.cb8 && ix.cent8 &&
         (ix.dsub == 1 || ix.dsub == 2 || ix.dsub == 4 || ix.dsub == 8) && ix.dim_pad <= 256;
}

bool lmajor_supported(const DevIndex& ix) {
  if (ix.nlist > (1 << 20)) return false;  // the work list's offsets take 1024 blocks of lists
  return lmajor_mfma(ix) || (!ix.int_grid && (ix.M + 3) / 4 <= kLutMaxW);
}

int lmajor_group(const DevIndex& ix, bool lut16) { return lmajor_mfma(ix) ? kLmG : lut16 ? 8 : 4; }

int lmajor_cap2(int n) { return std::min(32768, std::max(4096, 16 * n)); }

namespace {

using LmFn = void (*)(DevIndex, const float*, LmArgs);

template <int KC>
LmFn lm_kernel_ds(int ds) {
  switch (ds) {
    case 1: return k_lm_mfma<KC, 1>;
    case 2: return k_lm_mfma<KC, 2>;
    case 4: return k_lm_mfma<KC, 4>;
    default: return k_lm_mfma<KC, 8>;
  }
}

using LutFn = void (*)(DevIndex, const float*, LmArgs);

template <int... Ws>
constexpr LutFn lut_kernel_entry(int w, bool h, std::integer_sequence<int, Ws...>) {
  LutFn f = nullptr;
  ((f = (w == Ws + 1) ? (h ? k_lm_lut<Ws + 1, true> : k_lm_lut<Ws + 1, false>) : f), ...);
  return f;
}

LutFn lut_kernel(const DevIndex& ix, bool h) {
  return lut_kernel_entry((ix.M + 3) / 4, h, std::make_integer_sequence<int, kLutMaxW>{});
}

LmFn lm_kernel(const DevIndex& ix) {
  switch (ix.dim_pad / 64) {
    case 1: return lm_kernel_ds<1>(ix.dsub);
    case 2: return lm_kernel_ds<2>(ix.dsub);
    case 3: return lm_kernel_ds<3>(ix.dsub);
    default: return lm_kernel_ds<4>(ix.dsub);
  }
}

}  // namespace

hipError_t launch_lmajor(const DevIndex& ix, const float* q, const LaunchCfg& c, Work& w,
                         const LmWork& lw, const LmCfg& lc, int num_cu, int phase,
                         hipStream_t st) {
  if (c.qc <= 0) return hipSuccess;
  const int W = (ix.M + 3) / 4;
  const int cap = scan_cap(ix, c.np_max, c.n, c.lut16);
  const int pairs = c.qc * c.np_max;
  const dim3 gp((pairs + 255) / 256);
  switch (phase) {
    case 0: {  // which slots each query leaves to the list-major pass; counters
      const int nprep = std::max({c.qc, ix.nlist, 4});
      hipLaunchKernelGGL(k_lm_prep, dim3((nprep + 255) / 256), dim3(256), 0, st, ix, w.lists,
                         w.np_eff, c.np_max, c.qc, (int64_t)lc.alpha * c.n, lw.walkp, lw.thr,
                         lw.cnt2, lw.flag, lw.lcnt, lw.lfill, lw.ctr);
      return hipGetLastError();
    }
    case 1: {  // per-query part: leading lists, short lists, replica entries; the bound
      ScanSplit sp;
      sp.walkp = lw.walkp;
      sp.thr_out = lw.thr;
      sp.min_rows = lc.min_rows;
      return scan_fn(W)(ix, w.lists, w.np_eff, c.np_max, c.qc, q, nullptr, w.sq, c.smax, c.tile,
                        c.n, cap, w.pkeys, w.pcount, w.pscan, nullptr, false, c.lut16, 0, nullptr,
                        nullptr, nullptr, sp, st);
    }
    case 2: {  // the work list
      const int G = lmajor_group(ix, c.lut16);
      hipLaunchKernelGGL(k_lm_count, gp, dim3(256), 0, st, ix, w.lists, w.np_eff, lw.walkp,
                         c.np_max, c.qc, lc.min_rows, lw.lcnt);
      const int nblk = (ix.nlist + 1023) / 1024;
      hipLaunchKernelGGL(k_lm_offsets, dim3(nblk), dim3(1024), 0, st, ix, lw.lcnt, lc.tile_rows,
                         G, lw.loff, lw.ioff, lw.ctr);
      hipLaunchKernelGGL(k_lm_offsets_add, dim3(nblk), dim3(1024), 0, st, ix, lw.loff, lw.ioff,
                         lw.ctr);
      hipLaunchKernelGGL(k_lm_fill, gp, dim3(256), 0, st, ix, w.lists, w.np_eff, lw.walkp,
                         c.np_max, c.qc, lc.min_rows, lw.loff, lw.lfill, lw.invq);
      return hipGetLastError();
    }
    case 3: {  // the persistent list-major launch
      const int G = lmajor_group(ix, c.lut16);
      LmArgs a{lw.loff, lw.ioff, lw.lcnt, lw.invq, lw.thr, lw.cnt2, lw.out2, lw.cap2, lw.ctr,
               lc.tile_rows, G};
      if (lmajor_mfma(ix)) {
        const size_t lds = (size_t)lm_cb_bytes(ix.M, ix.dsub) + (size_t)kLmG * ix.dim_pad +
                           kLmG * 8 + kLmG * 4 + 8 * 4;
        const LmFn kern = lm_kernel(ix);
        if (lds > 65536)
          (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds);
        int blocks = lc.blocks;
        if (blocks <= 0) {  // every block resident at once
          int per_cu = 0;
          if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, kLmBlock,
                                                           lds) != hipSuccess || per_cu < 1)
            per_cu = 4;
          blocks = per_cu * std::max(1, num_cu);
        }
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kLmBlock), lds, st, ix, q, a);
        return hipGetLastError();
      }
      // float index: the chunk's tables, then the table-lookup kernel
      hipLaunchKernelGGL(k_lut, dim3(c.qc), dim3(kBlock), 0, st, ix, q, c.qc, lw.lut);
      const size_t lds = (size_t)4 * ((ix.M + 3) / 4) * kKsub * 16 + G * 8 + G * 4 + 8 * 4;
      const LutFn kern = lut_kernel(ix, c.lut16);
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      const int blocks = lc.blocks > 0 ? lc.blocks : std::max(1, num_cu);
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(kLutBlock), lds, st, ix, lw.lut, a);
      return hipGetLastError();
    }
    case 4: {  // both parts' n best per query
      const size_t lds_sel = (size_t)c.n * 8;
      if (lds_sel > 65536)
        (void)hipFuncSetAttribute((const void*)k_lm_select,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_sel);
      hipLaunchKernelGGL(k_lm_select, dim3(c.qc), dim3(kBlock), lds_sel, st, ix, w.lists,
                         w.np_eff, c.np_max, lw.walkp, lc.min_rows, c.smax, c.n, w.pkeys,
                         w.pcount, w.pscan, w.sq, lw.cnt2, lw.out2, lw.cap2, lw.flag);
      return hipGetLastError();
    }
    default: {  // queries whose list-major output overflowed: the whole query per query
      ScanSplit sp;
      sp.active = lw.flag;
      return scan_fn(W)(ix, w.lists, w.np_eff, c.np_max, c.qc, q, nullptr, w.sq, c.smax, c.tile,
                        c.n, cap, w.pkeys, w.pcount, w.pscan, nullptr, false, c.lut16, 0, nullptr,
                        nullptr, nullptr, sp, st);
    }
  }
}

}  // namespace ann
