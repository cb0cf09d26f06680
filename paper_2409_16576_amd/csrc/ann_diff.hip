// Differentiable PQ distance (codes fixed) on gfx950.
//
// Forward, for queries Q [B, D], codebooks CB [M, 256, dsub] and fixed codes
// [C, M]:   Dhat[b][c] = sum_m || q_b,m - CB[m][code[c][m]] ||^2   (Eq. 1 with
// dist = squared L2 of sub-vectors), float32.
//
// Backward, given G = dL/dDhat [B, C]:
//   dQ[b]       = 2 * ( rowsum(G)_b * q_b - (G . Dec)_b )          Dec[c] = decoded code c
//   dCB[m][j]   = -2 * ( sum_{c: code[c][m] = j} (G^T . Q)[c]_m  -  (sum_{c: code[c][m] = j} colsum(G)_c) * CB[m][j] )
// The two products run on the fp32 matrix cores (v_mfma_f32_16x16x4f32); the
// scatter into the codebook is a deterministic segmented sum: one thread per
// (subspace, codeword) adds its members in increasing candidate order.
#include <algorithm>
#include <cstdint>

#include "ann.h"
#include "ann_internal.h"

namespace ann {
namespace {

typedef float v4f_t __attribute__((ext_vector_type(4)));

// Forward: block per query; table in LDS, threads over candidates.
__global__ __launch_bounds__(kBlock) void k_adc_fwd(const float* __restrict__ Q,
                                                     const float* __restrict__ CB,
                                                     const uint8_t* __restrict__ codes, int B,
                                                     int C, int D, int M, int dsub,
                                                     float* __restrict__ out) {
  extern __shared__ float s_lut[];  // [M, 256]
  const int b = blockIdx.x;
  const float* q = Q + (size_t)b * D;
  for (int e = threadIdx.x; e < M * kKsub; e += kBlock) {
    const int m = e >> 8, j = e & 255;
    const float* c = CB + ((size_t)m * kKsub + j) * dsub;
    float acc = 0.f;
    for (int t = 0; t < dsub; ++t) {
      const float u = q[m * dsub + t] - c[t];
      acc = acc + u * u;
    }
    s_lut[e] = acc;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += kBlock) {
    const uint8_t* code = codes + (size_t)c * M;
    float acc = 0.f;
    for (int m = 0; m < M; ++m) acc = acc + s_lut[m * kKsub + code[m]];
    out[(size_t)b * C + c] = acc;
  }
}


// Exact squared distances in direct form (no expansion into norms and a
// product, so no cancellation): out[b][c] = sum_t (q_bt - x_ct)^2 summed in
// float64 over t in order and rounded once to float32.  Block: 16 x 16 pairs,
// Q and X staged 64 dimensions at a time.
__global__ __launch_bounds__(kBlock) void k_exact_sq(const float* __restrict__ Q,
                                                      const float* __restrict__ X, int B, int C,
                                                      int D, float* __restrict__ out) {
  __shared__ float s_q[16][65], s_x[16][65];
  const int tb = threadIdx.x >> 4, tc = threadIdx.x & 15;
  const int b = blockIdx.y * 16 + tb, c = blockIdx.x * 16 + tc;
  double acc = 0.0;
  for (int t0 = 0; t0 < D; t0 += 64) {
    for (int i = threadIdx.x; i < 16 * 64; i += kBlock) {
      const int r = i >> 6, t = t0 + (i & 63);
      const int qb = blockIdx.y * 16 + r, xc = blockIdx.x * 16 + r;
      s_q[r][i & 63] = qb < B && t < D ? Q[(size_t)qb * D + t] : 0.f;
      s_x[r][i & 63] = xc < C && t < D ? X[(size_t)xc * D + t] : 0.f;
    }
    __syncthreads();
    const int tn = min(64, D - t0);
    for (int t = 0; t < tn; ++t) {
      const double u = (double)s_q[tb][t] - (double)s_x[tc][t];
      const double sq = u * u;
      acc = acc + sq;
    }
    __syncthreads();
  }
  if (b < B && c < C) out[(size_t)b * C + c] = (float)acc;
}

// Out[i][j] = sum over k in [k0, k1) of A(i, k) * Bm(k, j), fp32 MFMA
// 16x16x4.  A(i, k) = A[i * lda_i + k * lda_k] (a transposed operand is
// just other strides), Bm(k, j) = Bm[k * ldb + j], Out row-major [rows,
// cols].  Block: 64 x 64 output tile, 4 waves of 32 x 32 (2 x 2 MFMA tiles);
// K staged 16 at a time, loads coalesced along whichever index of A is
// contiguous.  blockIdx.z picks the K slice [z * kslice, (z + 1) * kslice)
// and the partial tile goes to out + z * rows * cols (split K; the slices are
// summed afterwards in a fixed order, so results do not depend on timing).
__global__ __launch_bounds__(kBlock) void k_gemm_f32(const float* __restrict__ A, int64_t lda_i,
                                                      int64_t lda_k, const float* __restrict__ Bm,
                                                      int64_t ldb, int rows, int cols, int K,
                                                      int kslice, float* __restrict__ out) {
  __shared__ float sA[64][17];
  __shared__ float sB[16][65];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kslice, ke = min(K, kb + kslice);
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  const bool a_rows_contig = lda_i == 1;  // A(i, k) contiguous along i (a transposed operand)
  v4f_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = v4f_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += kBlock) {
      const int r = a_rows_contig ? e % 64 : e / 16, kk = a_rows_contig ? e / 64 : e % 16;
      const int gi = i0 + r, gk = k0 + kk;
      sA[r][kk] = (gi < rows && gk < ke) ? A[(int64_t)gi * lda_i + (int64_t)gk * lda_k] : 0.f;
    }
    for (int e = tid; e < 16 * 64; e += kBlock) {
      const int kk = e / 64, c = e % 64;
      const int gk = k0 + kk, gj = j0 + c;
      sB[kk][c] = (gk < ke && gj < cols) ? Bm[(int64_t)gk * ldb + gj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float fa = sA[wi + a * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const float fb = sB[ks + (lane >> 4)][wj + c * 16 + (lane & 15)];
          acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa, fb, acc[a][c], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  float* o = out + (size_t)blockIdx.z * rows * cols;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wi + a * 16 + 4 * (lane >> 4) + r;
        const int gj = j0 + wj + c * 16 + (lane & 15);
        if (gi < rows && gj < cols) o[(size_t)gi * cols + gj] = acc[a][c][r];
      }
}

// out[i] = sum over s = 0..S-1, in that order, of part[s][i].
__global__ void k_sum_slices(const float* __restrict__ part, int S, size_t n,
                             float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = part[i];
  for (int s = 1; s < S; ++s) acc = acc + part[(size_t)s * n + i];
  out[i] = acc;
}

// Q1 [B, D + 1] = [Q | 1]: the extra column makes G^T Q1 carry colsum(G).
__global__ void k_ones_col(const float* __restrict__ Q, int B, int D, float* __restrict__ q1) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)B * (D + 1)) return;
  const int b = (int)(i / (D + 1)), d = (int)(i % (D + 1));
  q1[i] = d < D ? Q[(size_t)b * D + d] : 1.f;
}

// dQ = 2 * (rowsum(G) * Q - G Dec), both read from GD1 = G [Dec | 1].
__global__ void k_dq(const float* __restrict__ Q, const float* __restrict__ gd1, int B, int D,
                     float* __restrict__ dq) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)B * D) return;
  const int b = (int)(i / D), d = (int)(i % D);
  const float* row = gd1 + (size_t)b * (D + 1);
  dq[i] = 2.f * (row[D] * Q[i] - row[d]);
}

// dCB[m][j][t] = -2 * (sum_{c in S_mj} T[c][m*dsub+t] - (sum_{c in S_mj} colsum_c) * CB[m][j][t])
// with T1 = G^T [Q | 1] (its last column is colsum).  Block per subspace m,
// thread per codeword j; the subspace's codes are staged in LDS in chunks and
// every thread walks them in increasing c (broadcast reads), adding the rows
// of its members in that order.
constexpr int kDcbChunk = 16384;

__global__ __launch_bounds__(kKsub) void k_dcb(const float* __restrict__ CB,
                                                const uint8_t* __restrict__ codes,
                                                const float* __restrict__ T1, int C, int D, int M,
                                                int dsub, float* __restrict__ dcb) {
  __shared__ uint8_t s_code[kDcbChunk];
  const int m = blockIdx.x, j = threadIdx.x;
  float s_cs = 0.f;
  float s_t[16];
  for (int t = 0; t < 16; ++t) s_t[t] = 0.f;
  for (int c0 = 0; c0 < C; c0 += kDcbChunk) {
    const int cn = min(kDcbChunk, C - c0);
    __syncthreads();
    for (int c = j; c < cn; c += kKsub) s_code[c] = codes[(size_t)(c0 + c) * M + m];
    __syncthreads();
    for (int c = 0; c < cn; ++c) {
      if (s_code[c] != j) continue;
      const float* row = T1 + (size_t)(c0 + c) * (D + 1);
      s_cs += row[D];
      for (int t = 0; t < dsub; ++t) s_t[t] += row[m * dsub + t];
    }
  }
  for (int t = 0; t < dsub; ++t) {
    const float cb = CB[((size_t)m * kKsub + j) * dsub + t];
    dcb[((size_t)m * kKsub + j) * dsub + t] = -2.f * (s_t[t] - s_cs * cb);
  }
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_prefix(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// The members of every codeword, in increasing candidate order: one wave per
// subspace m counts the codes, turns the counts into starts
// (starts[m][j] .. starts[m][j + 1]) and places the candidates 64 at a time,
// a candidate's rank among the lanes holding the same code coming from eight
// ballots (one per code bit), so the order within a codeword is stable.
__global__ __launch_bounds__(64) void k_dcb_order(const uint8_t* __restrict__ codes, int C, int M,
                                                  int32_t* __restrict__ order,
                                                  int32_t* __restrict__ starts) {
  __shared__ int s_cur[kKsub];
  const int m = blockIdx.x, lane = threadIdx.x;
  for (int j = lane; j < kKsub; j += 64) s_cur[j] = 0;
  __threadfence_block();
  for (int c = lane; c < C; c += 64) atomicAdd(&s_cur[codes[(size_t)c * M + m]], 1);
  __threadfence_block();
  int v[4], sum = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    v[b] = s_cur[4 * lane + b];
    sum += v[b];
  }
  int run = wave_prefix(sum) - sum;
  int32_t* st = starts + (size_t)m * (kKsub + 1);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    s_cur[4 * lane + b] = run;
    st[4 * lane + b] = run;
    run += v[b];
  }
  if (lane == 63) st[kKsub] = run;  // = C
  __threadfence_block();
  const uint64_t below = (1ull << lane) - 1ull;
  for (int c0 = 0; c0 < C; c0 += 64) {
    const int c = c0 + lane;
    const bool ok = c < C;
    const int code = ok ? codes[(size_t)c * M + m] : 0;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (code >> b) & 1;
      const uint64_t ones = __ballot(ok && bit);
      peers &= bit ? ones : ~ones;
    }
    const int base = ok ? s_cur[code] : 0;
    const int rank = __popcll(peers & below);
    if (ok) order[(size_t)m * C + base + rank] = c;
    __threadfence_block();  // every lane has read its cursor
    if (ok && rank == 0) s_cur[code] = base + __popcll(peers);
    __threadfence_block();
  }
}

// dCB as k_dcb, one thread per (subspace, codeword): the members' rows of T1
// are read four at a time (loads in flight together) and added in increasing
// candidate order, so every sum is the same float sequence as k_dcb's.
template <int DS>
__global__ __launch_bounds__(kKsub) void k_dcb_sum(const float* __restrict__ CB,
                                                    const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ starts,
                                                    const float* __restrict__ T1, int C, int D,
                                                    float* __restrict__ dcb) {
  const int m = blockIdx.x, j = threadIdx.x;
  const int32_t* st = starts + (size_t)m * (kKsub + 1);
  const int32_t* mem = order + (size_t)m * C;
  const int e = st[j + 1];
  float s_cs = 0.f;
  float s_t[DS];
#pragma unroll
  for (int t = 0; t < DS; ++t) s_t[t] = 0.f;
  int i = st[j];
  for (; i + 4 <= e; i += 4) {
    float r[4][DS + 1];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float* row = T1 + (size_t)mem[i + u] * (D + 1);
      r[u][DS] = row[D];
#pragma unroll
      for (int t = 0; t < DS; ++t) r[u][t] = row[m * DS + t];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s_cs += r[u][DS];
#pragma unroll
      for (int t = 0; t < DS; ++t) s_t[t] += r[u][t];
    }
  }
  for (; i < e; ++i) {
    const float* row = T1 + (size_t)mem[i] * (D + 1);
    s_cs += row[D];
#pragma unroll
    for (int t = 0; t < DS; ++t) s_t[t] += row[m * DS + t];
  }
#pragma unroll
  for (int t = 0; t < DS; ++t) {
    const float cb = CB[((size_t)m * kKsub + j) * DS + t];
    dcb[((size_t)m * kKsub + j) * DS + t] = -2.f * (s_t[t] - s_cs * cb);
  }
}

// Decoded candidates with a ones column: Dec1 [C, D + 1] = [Dec | 1].
__global__ void k_decode1(const float* __restrict__ CB, const uint8_t* __restrict__ codes, int C,
                          int D, int M, int dsub, float* __restrict__ dec1) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)C * (D + 1)) return;
  const int c = (int)(i / (D + 1)), d = (int)(i % (D + 1));
  if (d == D) {
    dec1[i] = 1.f;
    return;
  }
  const int m = d / dsub, t = d % dsub;
  dec1[i] = CB[((size_t)m * kKsub + codes[(size_t)c * M + m]) * dsub + t];
}

// K slices for a GEMM with `tiles` output tiles: about 1024 blocks in all,
// slices of at least 64.
int kslices(int tiles, int K) {
  int s = std::max(1, 1024 / std::max(1, tiles));
  s = std::min(s, std::max(1, K / 64));
  return std::min(s, 64);
}

ann_status diff_fail(ann_status s, const char* msg) { return (ann_status)set_error(s, "%s", msg); }

bool diff_shapes_ok(int64_t B, int64_t C, int D, int M, int dsub) {
  return B >= 0 && C >= 0 && M >= 1 && dsub >= 1 && dsub <= 16 && D == M * dsub &&
         (int64_t)M * kKsub * 4 <= 65536 && B < (1ll << 31) && C < (1ll << 31);
}

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" ann_status ann_adc_forward(const float* d_queries, int64_t B, const float* d_codebooks,
                                      int32_t M, int32_t dsub, const uint8_t* d_codes, int64_t C,
                                      float* d_out, void* stream) {
  const int D = M * dsub;
  if (!diff_shapes_ok(B, C, D, M, dsub)) return diff_fail(ANN_EINVAL, "bad shapes");
  if (B == 0 || C == 0) return ANN_OK;
  if (!d_queries || !d_codebooks || !d_codes || !d_out) return diff_fail(ANN_EINVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_adc_fwd, dim3((unsigned)B), dim3(kBlock), (size_t)M * kKsub * 4, st,
                     d_queries, d_codebooks, d_codes, (int)B, (int)C, D, M, dsub, d_out);
  return hipGetLastError() == hipSuccess ? ANN_OK : diff_fail(ANN_EDEVICE, "launch failed");
}

extern "C" ann_status ann_exact_sq(const float* d_queries, int64_t B, const float* d_vectors,
                                    int64_t C, int32_t D, float* d_out, void* stream) {
  if (B < 0 || C < 0 || D < 1 || B >= (1ll << 31) || C >= (1ll << 31))
    return diff_fail(ANN_EINVAL, "bad shapes");
  if (B == 0 || C == 0) return ANN_OK;
  if (!d_queries || !d_vectors || !d_out) return diff_fail(ANN_EINVAL, "NULL pointer");
  if ((C + 15) / 16 > INT32_MAX || (B + 15) / 16 > 65535)
    return diff_fail(ANN_EINVAL, "too many queries for one call (at most 1048560)");
  const dim3 grid((unsigned)((C + 15) / 16), (unsigned)((B + 15) / 16));
  hipLaunchKernelGGL(k_exact_sq, grid, dim3(kBlock), 0, (hipStream_t)stream, d_queries,
                     d_vectors, (int)B, (int)C, D, d_out);
  return hipGetLastError() == hipSuccess ? ANN_OK : diff_fail(ANN_EDEVICE, "launch failed");
}

extern "C" size_t ann_adc_backward_workspace(int64_t B, int64_t C, int32_t M, int32_t dsub) {
  const size_t D1 = (size_t)M * dsub + 1;
  const int t1 = (int)(((D1 + 63) / 64) * ((B + 63) / 64)), t2 = (int)(((D1 + 63) / 64) * ((C + 63) / 64));
  const size_t s1 = (size_t)kslices(t1, (int)C), s2 = (size_t)kslices(t2, (int)B);
  // Dec1 [C, D1], Q1 [B, D1], GD1 [B, D1], T1 [C, D1], K-slice partials
  // + the members of every codeword: order [M, C] and starts [M, 257] (int32)
  return sizeof(float) * ((size_t)C * D1 + 2 * (size_t)B * D1 + (size_t)C * D1 +
                          std::max(s1 * (size_t)B * D1, s2 * (size_t)C * D1)) +
         sizeof(int32_t) * ((size_t)M * C + (size_t)M * (kKsub + 1)) + 256;
}

extern "C" ann_status ann_adc_backward(const float* d_queries, int64_t B, const float* d_codebooks,
                                       int32_t M, int32_t dsub, const uint8_t* d_codes, int64_t C,
                                       const float* d_grad, float* d_dq, float* d_dcb,
                                       void* d_workspace, size_t workspace_bytes, void* stream) {
  const int D = M * dsub;
  if (!diff_shapes_ok(B, C, D, M, dsub)) return diff_fail(ANN_EINVAL, "bad shapes");
  if (workspace_bytes < ann_adc_backward_workspace(B, C, M, dsub))
    return diff_fail(ANN_EINVAL, "workspace too small");
  if (!d_queries || !d_codebooks || !d_codes || !d_grad || !d_workspace)
    return diff_fail(ANN_EINVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  const int D1 = D + 1;
  float* ws = static_cast<float*>(d_workspace);
  float* dec1 = ws;                          // [C, D1]
  float* q1 = dec1 + (size_t)C * D1;         // [B, D1]
  float* gd1 = q1 + (size_t)B * D1;          // [B, D1] = G [Dec | 1]
  float* t1 = gd1 + (size_t)B * D1;          // [C, D1] = G^T [Q | 1]
  float* part = t1 + (size_t)C * D1;         // K-slice partials
  const int thr = 256;
  const int ct = (D1 + 63) / 64;
  if (d_dq && B > 0) {
    if (C > 0)
      hipLaunchKernelGGL(k_decode1, dim3((unsigned)(((size_t)C * D1 + thr - 1) / thr)), dim3(thr),
                         0, st, d_codebooks, d_codes, (int)C, D, M, dsub, dec1);
    const int rt = (int)((B + 63) / 64), S = kslices(ct * rt, (int)C);
    hipLaunchKernelGGL(k_gemm_f32, dim3(ct, rt, S), dim3(kBlock), 0, st, d_grad, (int64_t)C,
                       (int64_t)1, dec1, (int64_t)D1, (int)B, D1, (int)C,
                       (int)((C + S - 1) / S + 15) / 16 * 16, part);
    const size_t nb = (size_t)B * D1;
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((nb + thr - 1) / thr)), dim3(thr), 0, st,
                       part, S, nb, gd1);
    hipLaunchKernelGGL(k_dq, dim3((unsigned)(((size_t)B * D + thr - 1) / thr)), dim3(thr), 0, st,
                       d_queries, gd1, (int)B, D, d_dq);
  }
  if (d_dcb) {
    if (C > 0) {
      hipLaunchKernelGGL(k_ones_col, dim3((unsigned)(((size_t)B * D1 + thr - 1) / thr)), dim3(thr),
                         0, st, d_queries, (int)B, D, q1);
      const int rt = (int)((C + 63) / 64), S = kslices(ct * rt, (int)B);
      hipLaunchKernelGGL(k_gemm_f32, dim3(ct, rt, S), dim3(kBlock), 0, st, d_grad, (int64_t)1,
                         (int64_t)C, q1, (int64_t)D1, (int)C, D1, (int)B,
                         (int)((B + S - 1) / S + 15) / 16 * 16, part);
      const size_t nc = (size_t)C * D1;
      hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((nc + thr - 1) / thr)), dim3(thr), 0, st,
                         part, S, nc, t1);
    }
    const int t1c = (int)(((size_t)D1 + 63) / 64) * (int)((C + 63) / 64);
    const int t2c = (int)(((size_t)D1 + 63) / 64) * (int)((B + 63) / 64);
    const size_t part_n = std::max((size_t)kslices(t2c, (int)C) * (size_t)B * D1,
                                   (size_t)kslices(t1c, (int)B) * (size_t)C * D1);
    int32_t* order = reinterpret_cast<int32_t*>(part + part_n);  // [M, C]
    int32_t* starts = order + (size_t)M * C;                      // [M, 257]
    if (dsub <= 8 && C > 0)
      hipLaunchKernelGGL(k_dcb_order, dim3(M), dim3(64), 0, st, d_codes, (int)C, M, order, starts);
    switch (dsub) {
#define ANN_DCB(DS)                                                                            \
  case DS:                                                                                     \
    if (C > 0)                                                                                 \
      hipLaunchKernelGGL(k_dcb_sum<DS>, dim3(M), dim3(kKsub), 0, st, d_codebooks, order,       \
                         starts, t1, (int)C, D, d_dcb);                                        \
    else                                                                                       \
      hipLaunchKernelGGL(k_dcb, dim3(M), dim3(kKsub), 0, st, d_codebooks, d_codes, t1, (int)C, \
                         D, M, dsub, d_dcb);                                                   \
    break;
      ANN_DCB(1) ANN_DCB(2) ANN_DCB(3) ANN_DCB(4) ANN_DCB(5) ANN_DCB(6) ANN_DCB(7) ANN_DCB(8)
#undef ANN_DCB
      default:
        hipLaunchKernelGGL(k_dcb, dim3(M), dim3(kKsub), 0, st, d_codebooks, d_codes, t1, (int)C,
                           D, M, dsub, d_dcb);
    }
  }
  return hipGetLastError() == hipSuccess ? ANN_OK : diff_fail(ANN_EDEVICE, "launch failed");
}
