// Offline index construction (CPU): IVF clustering, boundary replication and
// product-quantisation training/encoding.
//
// This is the offline half of the multi-tiered index (paper Sec. 4.1): the
// dataset is partitioned into posting lists by (hierarchical) k-means, each
// vector is replicated into every list that satisfies the boundary rule of
// Eq. 2 (up to R lists), and every vector gets one M-byte PQ code (Sec. 2.2).
// The online search never runs this code; it only reads the index file the
// Python driver writes from these results.
//
// Plain scalar C++ with OpenMP over rows.  Distances use the direct form
// sum_t (x_t - c_t)^2 in fp32; on integer-valued data and integer-valued
// centroids every partial sum is an exact integer below 2^24.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include <omp.h>

namespace {

inline float sqdist(const float* a, const float* b, int d) {
  float s = 0.f;
  for (int t = 0; t < d; ++t) {
    float u = a[t] - b[t];
    s += u * u;
  }
  return s;
}

// Distances from one row to a block of centroids stored transposed
// (ct[t * ldc + j]); vectorises over j.
inline void sqdist_block(const float* x, const float* ct, int64_t ldc, int nb, int d,
                         float* out) {
  for (int j = 0; j < nb; ++j) out[j] = 0.f;
  for (int t = 0; t < d; ++t) {
    const float xt = x[t];
    const float* c = ct + (int64_t)t * ldc;
#pragma omp simd
    for (int j = 0; j < nb; ++j) {
      float u = xt - c[j];
      out[j] += u * u;
    }
  }
}

std::vector<float> transpose(const float* c, int k, int d) {
  std::vector<float> ct((size_t)k * d);
  for (int j = 0; j < k; ++j)
    for (int t = 0; t < d; ++t) ct[(size_t)t * k + j] = c[(size_t)j * d + t];
  return ct;
}

// Nearest centroid (ties: lower index) of every row.
void nearest(const float* X, int64_t n, int d, const float* C, int k, int32_t* lab,
             float* dist) {
  std::vector<float> ct = transpose(C, k, d);
#pragma omp parallel
  {
    std::vector<float> buf(k);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      sqdist_block(X + i * d, ct.data(), k, k, d, buf.data());
      int best = 0;
      float bd = buf[0];
      for (int j = 1; j < k; ++j)
        if (buf[j] < bd) { bd = buf[j]; best = j; }
      lab[i] = best;
      if (dist) dist[i] = bd;
    }
  }
}

}  // namespace

extern "C" {

int bld_num_threads(void) { return omp_get_max_threads(); }

// Lloyd iterations. C (k x d) holds the initial centroids on entry and the
// result on exit. A cluster that becomes empty keeps its previous centroid.
void bld_kmeans(const float* X, int64_t n, int d, float* C, int k, int iters) {
  std::vector<int32_t> lab(n);
  std::vector<double> sum((size_t)k * d);
  std::vector<int64_t> cnt(k);
  for (int it = 0; it < iters; ++it) {
    nearest(X, n, d, C, k, lab.data(), nullptr);
    std::fill(sum.begin(), sum.end(), 0.0);
    std::fill(cnt.begin(), cnt.end(), 0);
    int nt = omp_get_max_threads();
    std::vector<std::vector<double>> ps(nt, std::vector<double>((size_t)k * d, 0.0));
    std::vector<std::vector<int64_t>> pc(nt, std::vector<int64_t>(k, 0));
#pragma omp parallel
    {
      int tid = omp_get_thread_num();
      double* s = ps[tid].data();
      int64_t* c = pc[tid].data();
#pragma omp for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        const float* x = X + i * d;
        double* sj = s + (size_t)lab[i] * d;
        for (int t = 0; t < d; ++t) sj[t] += x[t];
        c[lab[i]] += 1;
      }
    }
    for (int t = 0; t < nt; ++t) {
      for (size_t u = 0; u < sum.size(); ++u) sum[u] += ps[t][u];
      for (int j = 0; j < k; ++j) cnt[j] += pc[t][j];
    }
    for (int j = 0; j < k; ++j) {
      if (cnt[j] == 0) continue;
      for (int t = 0; t < d; ++t) C[(size_t)j * d + t] = (float)(sum[(size_t)j * d + t] / cnt[j]);
    }
  }
}

// Balanced assignment (the balance constraint of hierarchical balanced
// clustering, Sec. 4.1): every row goes to its nearest centroid that still
// has room, each centroid holding at most `cap` rows.  Rows are placed in
// order of how much they lose if their nearest centroid is full (the gap
// between their nearest and second-nearest of T candidates, largest first;
// ties: lower row), so rows far from any other centroid keep their nearest.
// A row whose T candidates are all full takes the nearest centroid with room.
void bld_balanced_assign(const float* X, int64_t n, int d, const float* C, int k, int64_t cap,
                         int T, int32_t* lab) {
  T = std::max(1, std::min(T, k));
  std::vector<float> ct = transpose(C, k, d);
  std::vector<int32_t> cidx((size_t)n * T);
  std::vector<float> cdist((size_t)n * T);
  std::vector<float> gap(n);
#pragma omp parallel
  {
    std::vector<float> buf(k);
    std::vector<int32_t> idx(k);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      sqdist_block(X + i * d, ct.data(), k, k, d, buf.data());
      for (int j = 0; j < k; ++j) idx[j] = j;
      std::partial_sort(idx.begin(), idx.begin() + T, idx.end(), [&](int a, int b) {
        return buf[a] < buf[b] || (buf[a] == buf[b] && a < b);
      });
      for (int t = 0; t < T; ++t) {
        cidx[(size_t)i * T + t] = idx[t];
        cdist[(size_t)i * T + t] = buf[idx[t]];
      }
      gap[i] = T > 1 ? buf[idx[1]] - buf[idx[0]] : 0.f;
    }
  }
  std::vector<int64_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return gap[a] > gap[b]; });
  std::vector<int64_t> fill(k, 0);
  std::vector<float> row(k);
  for (int64_t i : order) {
    int got = -1;
    for (int t = 0; t < T && got < 0; ++t) {
      const int c = cidx[(size_t)i * T + t];
      if (fill[c] < cap) got = c;
    }
    if (got < 0) {
      sqdist_block(X + i * d, ct.data(), k, k, d, row.data());
      float best = std::numeric_limits<float>::infinity();
      for (int c = 0; c < k; ++c)
        if (fill[c] < cap && row[c] < best) {
          best = row[c];
          got = c;
        }
    }
    lab[i] = got;
    fill[got] += 1;
  }
}

// Nearest centroid of every row (exported for the driver).
void bld_nearest(const float* X, int64_t n, int d, const float* C, int k, int32_t* lab,
                 float* dist) {
  nearest(X, n, d, C, k, lab, dist);
}

// Eq. 2 assignment over a flat centroid set: list i is kept for row v iff
// Dist(v, C_i) <= (1 + eps) * Dist(v, C_1), C_1 the nearest list, Dist plain
// Euclidean.  At most R lists are kept, nearest first (ties: lower list id);
// unused slots are -1.
void bld_assign_flat(const float* X, int64_t n, int d, const float* C, int k, int R,
                     float eps, int32_t* assign) {
  std::vector<float> ct = transpose(C, k, d);
  const double lim = (1.0 + (double)eps) * (1.0 + (double)eps);
#pragma omp parallel
  {
    std::vector<float> buf(k);
    std::vector<int32_t> idx(k);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      sqdist_block(X + i * d, ct.data(), k, k, d, buf.data());
      int r = std::min(R, k);
      for (int j = 0; j < k; ++j) idx[j] = j;
      std::partial_sort(idx.begin(), idx.begin() + r, idx.end(), [&](int a, int b) {
        return buf[a] < buf[b] || (buf[a] == buf[b] && a < b);
      });
      int32_t* out = assign + i * R;
      double d1 = buf[idx[0]];
      int w = 0;
      for (int s = 0; s < r; ++s) {
        if (s == 0 || (double)buf[idx[s]] <= lim * d1) out[w++] = idx[s];
      }
      for (; w < R; ++w) out[w] = -1;
    }
  }
}

// Eq. 2 assignment inside a two-level hierarchy.  The candidate lists of a
// row are the sub-lists of its T nearest top-level clusters; the rule of
// bld_assign_flat is applied over those candidates.  Sub-centroids of top
// cluster a are rows sub_off[a] .. sub_off[a+1]-1 of Csub (their list ids).
void bld_assign_hier(const float* X, int64_t n, int d, const float* Ctop, int ktop,
                     const float* Csub, const int32_t* sub_off, int T, int R, float eps,
                     int32_t* assign) {
  std::vector<float> ctt = transpose(Ctop, ktop, d);
  const int ksub_total = sub_off[ktop];
  std::vector<float> cst = transpose(Csub, ksub_total, d);
  int maxsub = 0;
  for (int a = 0; a < ktop; ++a) maxsub = std::max(maxsub, sub_off[a + 1] - sub_off[a]);
  T = std::min(T, ktop);
  const double lim = (1.0 + (double)eps) * (1.0 + (double)eps);
#pragma omp parallel
  {
    std::vector<float> tb(ktop);
    std::vector<int32_t> tidx(ktop);
    std::vector<float> cand_d((size_t)T * maxsub);
    std::vector<int32_t> cand_l((size_t)T * maxsub);
    std::vector<int32_t> order((size_t)T * maxsub);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const float* x = X + i * d;
      sqdist_block(x, ctt.data(), ktop, ktop, d, tb.data());
      for (int a = 0; a < ktop; ++a) tidx[a] = a;
      std::partial_sort(tidx.begin(), tidx.begin() + T, tidx.end(), [&](int a, int b) {
        return tb[a] < tb[b] || (tb[a] == tb[b] && a < b);
      });
      int nc = 0;
      for (int s = 0; s < T; ++s) {
        int a = tidx[s];
        int b0 = sub_off[a], nb = sub_off[a + 1] - b0;
        sqdist_block(x, cst.data() + b0, ksub_total, nb, d, cand_d.data() + nc);
        for (int j = 0; j < nb; ++j) cand_l[nc + j] = b0 + j;
        nc += nb;
      }
      int r = std::min(R, nc);
      for (int j = 0; j < nc; ++j) order[j] = j;
      std::partial_sort(order.begin(), order.begin() + r, order.begin() + nc, [&](int a, int b) {
        return cand_d[a] < cand_d[b] || (cand_d[a] == cand_d[b] && cand_l[a] < cand_l[b]);
      });
      int32_t* out = assign + i * R;
      double d1 = cand_d[order[0]];
      int w = 0;
      for (int s = 0; s < r; ++s) {
        if (s == 0 || (double)cand_d[order[s]] <= lim * d1) out[w++] = cand_l[order[s]];
      }
      for (; w < R; ++w) out[w] = -1;
    }
  }
}

// PQ encoding: code[i][m] = argmin_j || x_i[m*dsub:(m+1)*dsub] - CB[m][j] ||^2
// (ties: lower j).  CB is M x ksub x dsub.
void bld_pq_encode(const float* X, int64_t n, int d, const float* CB, int M, int ksub,
                   int dsub, uint8_t* codes) {
  std::vector<std::vector<float>> cbt(M);
  for (int m = 0; m < M; ++m) cbt[m] = transpose(CB + (size_t)m * ksub * dsub, ksub, dsub);
#pragma omp parallel
  {
    std::vector<float> buf(ksub);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const float* x = X + i * d;
      for (int m = 0; m < M; ++m) {
        sqdist_block(x + m * dsub, cbt[m].data(), ksub, ksub, dsub, buf.data());
        int best = 0;
        float bd = buf[0];
        for (int j = 1; j < ksub; ++j)
          if (buf[j] < bd) { bd = buf[j]; best = j; }
        codes[i * M + m] = (uint8_t)best;
      }
    }
  }
}

// Navigation graph over the list centroids (Sec. 4.1): every centroid is
// joined to up to `deg` other centroids, as when vertices are added one at a
// time, each taking edges to its nearest neighbours, and those neighbours
// updating their own edge lists.  Candidates of vertex v are the centroids of
// the `gprobe` groups nearest to v (groups: a k-means of the centroids, gof[v]
// = v's group, members listed in gmem[goff[g] .. goff[g+1])), the `pool`
// nearest of them kept.  With `rng` the edges are chosen by the relative
// neighbourhood rule first (a candidate u is taken only if no edge already
// taken, w, is nearer to u than v is: the edges fan out instead of all
// pointing into v's own cluster), then the remaining slots take the nearest
// candidates left.  A vertex chosen by v is offered v as a candidate too
// (reverse edges), and the final lists are chosen the same way from both.
// adj: k x deg, -1 padded.
namespace {
void choose_edges(const float* C, int d, int v, std::vector<std::pair<float, int32_t>>& cand,
                  int deg, bool rng, int32_t* row) {
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end(),
                         [](const std::pair<float, int32_t>& a, const std::pair<float, int32_t>& b) {
                           return a.second == b.second;
                         }),
             cand.end());
  std::vector<char> taken(cand.size(), 0);
  int w = 0;
  if (rng) {
    std::vector<int32_t> kept;
    for (size_t i = 0; i < cand.size() && w < deg; ++i) {
      const int32_t u = cand[i].second;
      const float duv = cand[i].first;
      bool ok = true;
      for (int32_t x : kept)
        if (sqdist(C + (size_t)u * d, C + (size_t)x * d, d) < duv) {
          ok = false;
          break;
        }
      if (ok) {
        kept.push_back(u);
        taken[i] = 1;
        row[w++] = u;
      }
    }
  }
  for (size_t i = 0; i < cand.size() && w < deg; ++i)
    if (!taken[i]) row[w++] = cand[i].second;
  for (; w < deg; ++w) row[w] = -1;
  (void)v;
}
}  // namespace

void bld_nav_graph(const float* C, int k, int d, int deg, const float* G, int ng,
                   const int32_t* goff, const int32_t* gmem, int gprobe, int pool, int rng,
                   int32_t* adj) {
  gprobe = std::min(gprobe, ng);
  pool = std::max(pool, deg);
  std::vector<float> gt = transpose(G, ng, d);
  // 1. each vertex's nearest among its candidate groups, then its edges
  std::vector<std::vector<std::pair<float, int32_t>>> near(k);
#pragma omp parallel
  {
    std::vector<float> gd(ng);
    std::vector<int32_t> gi(ng);
    std::vector<std::pair<float, int32_t>> cand;
#pragma omp for schedule(dynamic, 64)
    for (int v = 0; v < k; ++v) {
      const float* cv = C + (size_t)v * d;
      sqdist_block(cv, gt.data(), ng, ng, d, gd.data());
      for (int g = 0; g < ng; ++g) gi[g] = g;
      std::partial_sort(gi.begin(), gi.begin() + gprobe, gi.end(), [&](int a, int b) {
        return gd[a] < gd[b] || (gd[a] == gd[b] && a < b);
      });
      cand.clear();
      for (int s = 0; s < gprobe; ++s) {
        const int g = gi[s];
        for (int32_t j = goff[g]; j < goff[g + 1]; ++j) {
          const int32_t u = gmem[j];
          if (u != v) cand.emplace_back(sqdist(cv, C + (size_t)u * d, d), u);
        }
      }
      const size_t r = std::min<size_t>(pool, cand.size());
      std::partial_sort(cand.begin(), cand.begin() + r, cand.end());
      cand.resize(r);
      near[v] = cand;
      choose_edges(C, d, v, cand, deg, rng != 0, adj + (size_t)v * deg);
    }
  }
  // 2. reverse edges: u chosen by v is offered v as well
  std::vector<std::vector<std::pair<float, int32_t>>> rev(k);
  for (int v = 0; v < k; ++v)
    for (int j = 0; j < deg; ++j) {
      const int32_t u = adj[(size_t)v * deg + j];
      if (u >= 0) rev[u].emplace_back(sqdist(C + (size_t)v * d, C + (size_t)u * d, d), v);
    }
#pragma omp parallel for schedule(dynamic, 64)
  for (int v = 0; v < k; ++v) {
    std::vector<std::pair<float, int32_t>> all = near[v];
    all.insert(all.end(), rev[v].begin(), rev[v].end());
    choose_edges(C, d, v, all, deg, rng != 0, adj + (size_t)v * deg);
  }
}

}  // extern "C"
