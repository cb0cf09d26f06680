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

// Decoded candidates Dec [C, D].
__global__ void k_decode(const float* __restrict__ CB, const uint8_t* __restrict__ codes, int C,
                         int D, int M, int dsub, float* __restrict__ dec) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)C * D) return;
  const int c = (int)(i / D), d = (int)(i % D);
  const int m = d / dsub, t = d % dsub;
  dec[i] = CB[((size_t)m * kKsub + codes[(size_t)c * M + m]) * dsub + t];
}

// Row sums and column sums of G [B, C].
__global__ void k_rowsum(const float* __restrict__ G, int B, int C, float* __restrict__ rs) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float acc = 0.f;
  for (int c = 0; c < C; ++c) acc += G[(size_t)b * C + c];
  rs[b] = acc;
}

__global__ void k_colsum(const float* __restrict__ G, int B, int C, float* __restrict__ cs) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  float acc = 0.f;
  for (int b = 0; b < B; ++b) acc += G[(size_t)b * C + c];
  cs[c] = acc;
}

// Out[i][j] = sum_k A(i, k) * Bm(k, j), fp32 MFMA 16x16x4.  A(i, k) =
// A[i * lda_i + k * lda_k] (so a transposed operand is just other strides),
// Bm(k, j) = Bm[k * ldb + j], Out row-major [rows, cols].  Block: 64 x 64
// output tile, 4 waves of 32 x 32 (2 x 2 MFMA tiles); K staged 16 at a time.
__global__ __launch_bounds__(kBlock) void k_gemm_f32(const float* __restrict__ A, int64_t lda_i,
                                                      int64_t lda_k, const float* __restrict__ Bm,
                                                      int64_t ldb, int rows, int cols, int K,
                                                      float* __restrict__ out) {
  __shared__ float sA[64][17];
  __shared__ float sB[16][65];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  v4f_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = v4f_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += kBlock) {
      const int r = e / 16, kk = e % 16;
      const int gi = i0 + r, gk = k0 + kk;
      sA[r][kk] = (gi < rows && gk < K) ? A[(int64_t)gi * lda_i + (int64_t)gk * lda_k] : 0.f;
    }
    for (int e = tid; e < 16 * 64; e += kBlock) {
      const int kk = e / 64, c = e % 64;
      const int gk = k0 + kk, gj = j0 + c;
      sB[kk][c] = (gk < K && gj < cols) ? Bm[(int64_t)gk * ldb + gj] : 0.f;
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
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wi + a * 16 + 4 * (lane >> 4) + r;
        const int gj = j0 + wj + c * 16 + (lane & 15);
        if (gi < rows && gj < cols) out[(size_t)gi * cols + gj] = acc[a][c][r];
      }
}

// dQ = 2 * (rowsum(G) * Q - GDec)
__global__ void k_dq(const float* __restrict__ Q, const float* __restrict__ rs,
                     const float* __restrict__ gdec, int B, int D, float* __restrict__ dq) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)B * D) return;
  const int b = (int)(i / D);
  dq[i] = 2.f * (rs[b] * Q[i] - gdec[i]);
}

// dCB[m][j][t] = -2 * (sum_{c in S_mj} T[c][m*dsub+t] - (sum_{c in S_mj} cs[c]) * CB[m][j][t])
// One thread per (m, j); members added in increasing c.
__global__ void k_dcb(const float* __restrict__ CB, const uint8_t* __restrict__ codes,
                      const float* __restrict__ T, const float* __restrict__ cs, int C, int D,
                      int M, int dsub, float* __restrict__ dcb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * kKsub) return;
  const int m = e >> 8, j = e & 255;
  float s_cs = 0.f;
  float s_t[16];
  for (int t = 0; t < 16; ++t) s_t[t] = 0.f;
  for (int c = 0; c < C; ++c) {
    if (codes[(size_t)c * M + m] != j) continue;
    s_cs += cs[c];
    for (int t = 0; t < dsub; ++t) s_t[t] += T[(size_t)c * D + m * dsub + t];
  }
  for (int t = 0; t < dsub; ++t) {
    const float cb = CB[((size_t)m * kKsub + j) * dsub + t];
    dcb[((size_t)m * kKsub + j) * dsub + t] = -2.f * (s_t[t] - s_cs * cb);
  }
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

extern "C" size_t ann_adc_backward_workspace(int64_t B, int64_t C, int32_t M, int32_t dsub) {
  const size_t D = (size_t)M * dsub;
  // Dec [C, D], GDec [B, D], T [C, D], rowsum [B], colsum [C]
  return sizeof(float) * ((size_t)C * D + (size_t)B * D + (size_t)C * D + (size_t)B + (size_t)C) +
         256;
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
  float* ws = static_cast<float*>(d_workspace);
  float* dec = ws;
  float* gdec = dec + (size_t)C * D;
  float* T = gdec + (size_t)B * D;
  float* rs = T + (size_t)C * D;
  float* cs = rs + B;
  const int thr = 256;
  if (C > 0 && D > 0)
    hipLaunchKernelGGL(k_decode, dim3((unsigned)(((size_t)C * D + thr - 1) / thr)), dim3(thr), 0,
                       st, d_codebooks, d_codes, (int)C, D, M, dsub, dec);
  if (B > 0)
    hipLaunchKernelGGL(k_rowsum, dim3((unsigned)((B + thr - 1) / thr)), dim3(thr), 0, st, d_grad,
                       (int)B, (int)C, rs);
  if (C > 0)
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((C + thr - 1) / thr)), dim3(thr), 0, st, d_grad,
                       (int)B, (int)C, cs);
  if (d_dq && B > 0) {
    // GDec [B, D] = G [B, C] . Dec [C, D]
    hipLaunchKernelGGL(k_gemm_f32, dim3((D + 63) / 64, (unsigned)((B + 63) / 64)), dim3(kBlock), 0,
                       st, d_grad, (int64_t)C, (int64_t)1, dec, (int64_t)D, (int)B, D, (int)C, gdec);
    hipLaunchKernelGGL(k_dq, dim3((unsigned)(((size_t)B * D + thr - 1) / thr)), dim3(thr), 0, st,
                       d_queries, rs, gdec, (int)B, D, d_dq);
  }
  if (d_dcb) {
    if (C > 0)  // T [C, D] = G^T [C, B] . Q [B, D]
      hipLaunchKernelGGL(k_gemm_f32, dim3((D + 63) / 64, (unsigned)((C + 63) / 64)), dim3(kBlock),
                         0, st, d_grad, (int64_t)1, (int64_t)C, d_queries, (int64_t)D, (int)C, D,
                         (int)B, T);
    hipLaunchKernelGGL(k_dcb, dim3((M * kKsub + thr - 1) / thr), dim3(thr), 0, st, d_codebooks,
                       d_codes, T, cs, (int)C, D, M, dsub, d_dcb);
  }
  return hipGetLastError() == hipSuccess ? ANN_OK : diff_fail(ANN_EDEVICE, "launch failed");
}
