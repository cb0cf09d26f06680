/*
 * CPU oracle for the GPU filtering stage of the multi-tiered IVF-PQ index.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU search path
 * never links, loads or calls it, and it shares no code with that path.
 *
 * Plain scalar C, one query at a time, in the order the paper describes the
 * online search (Sec. 3, steps 1-8):
 *   probe   the top-m nearest posting lists                   (Sec. 2.1, step 2)
 *   lut     the per-query distance table                      (Sec. 2.2, step 1)
 *   gather  the vector IDs of the probed lists (a multiset)   (Sec. 4.1, step 3)
 *   dedup   remove the duplicates left by replication         (step 5, Sec. 5)
 *   adc     approximate distance by table lookups             (Eq. 1, step 6)
 *   topn    the n best approximate distances                  (step 7)
 *   rerank  exact distance on raw vectors, keep the top-k     (step 8, fixed n)
 * plus brute-force exact kNN for recall.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - dist() of Eq. 1 is the squared Euclidean distance of the subvectors, so
 *    the table sum equals the squared distance to the decoded vector.
 *  - Non-residual PQ: one table per query, built before the lists are known.
 *  - The probe is exact over all centroids, or a best-first beam search over
 *    a navigation graph of the centroids when one is given.
 *  - Every distance that decides a selection is a float32 value: exact
 *    squared distances are evaluated in float64 (sequential over dimensions)
 *    or in integers, then rounded to nearest-even float32.  The table sum of
 *    Eq. 1 is a float32 sum over subspaces m = 0..M-1 in that order, starting
 *    from +0.0f, with plain additions (no fused multiply-add anywhere; build
 *    with -ffp-contract=off).
 *  - Every selection orders by (distance, id) lexicographically: ties go to
 *    the lower list ID / lower external vector ID.
 *  - For uint8/int8 datasets the float32 queries are first converted to the
 *    data type: round half to even, then saturate to the type's range.
 *  - Fewer candidates than n (or k): all are kept; outputs are padded with
 *    id -1 and distance +inf.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_F32 = 0, ORC_U8 = 1, ORC_I8 = 2 };

/* The index as the oracle sees it: external vector order, arrays owned by the
 * caller (read from the index file by the oracle's own reader). */
typedef struct {
  int32_t dtype; /* ORC_F32 / ORC_U8 / ORC_I8 */
  int32_t dim;
  int64_t n;
  int32_t nlist;
  int32_t m;
  int32_t ksub;
  int32_t dsub;
  int32_t r;
  int32_t pad_;
  const float* centroids;   /* nlist x dim */
  const float* codebooks;   /* m x ksub x dsub */
  const uint8_t* codes;     /* n x m */
  const void* vectors;      /* n x dim of dtype */
  const int64_t* offsets;   /* nlist + 1 */
  const int32_t* entries;   /* offsets[nlist] external ids */
} orc_index;

/* ------------------------------------------------------------------------ */
/* Query conversion (reading: integer datasets take integer queries).        */

static void convert_query(const orc_index* ix, const float* q, double* out) {
  for (int t = 0; t < ix->dim; ++t) {
    double v = (double)q[t];
    if (ix->dtype == ORC_U8) {
      v = nearbyint(v);
      if (v < 0.0) v = 0.0;
      if (v > 255.0) v = 255.0;
    } else if (ix->dtype == ORC_I8) {
      v = nearbyint(v);
      if (v < -128.0) v = -128.0;
      if (v > 127.0) v = 127.0;
    }
    out[t] = v;
  }
}

/* Squared Euclidean distance in float64, sequential over t, rounded once to
 * float32.  Exact for integer-valued inputs (every partial sum < 2^53). */
static float sqdist_f64(const double* q, const float* c, int d) {
  double acc = 0.0;
  for (int t = 0; t < d; ++t) {
    double u = q[t] - (double)c[t];
    double sq = u * u;
    acc = acc + sq;
  }
  return (float)acc;
}

/* Exact squared distance between the converted query and raw vector v.
 * Integer datasets: exact in 32-bit integers (|q_t - x_t| <= 255, so the sum
 * stays below 2^31 for dim < 33025), then converted to float32. */
static float exact_dist(const orc_index* ix, const double* q, const int32_t* qi, int64_t v) {
  const int d = ix->dim;
  if (ix->dtype == ORC_F32) return sqdist_f64(q, (const float*)ix->vectors + v * d, d);
  int32_t acc = 0;
  if (ix->dtype == ORC_U8) {
    const uint8_t* x = (const uint8_t*)ix->vectors + v * d;
    for (int t = 0; t < d; ++t) {
      int32_t u = qi[t] - (int32_t)x[t];
      acc += u * u;
    }
  } else {
    const int8_t* x = (const int8_t*)ix->vectors + v * d;
    for (int t = 0; t < d; ++t) {
      int32_t u = qi[t] - (int32_t)x[t];
      acc += u * u;
    }
  }
  return (float)acc;
}

static void int_query(const orc_index* ix, const double* q, int32_t* qi) {
  for (int t = 0; t < ix->dim; ++t) qi[t] = (int32_t)q[t];
}

/* ------------------------------------------------------------------------ */
/* (distance, id) pairs and their lexicographic order.                       */

typedef struct {
  float d;
  int32_t id;
} pair_t;

static int pair_cmp(const void* a, const void* b) {
  const pair_t* x = (const pair_t*)a;
  const pair_t* y = (const pair_t*)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

static int i32_cmp(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* Step 2: top-m nearest posting lists (exact probe over all centroids).     */

static int probe_one(const orc_index* ix, const double* q, int np, int32_t* out_l, float* out_d,
                     pair_t* scratch) {
  for (int l = 0; l < ix->nlist; ++l) {
    scratch[l].d = sqdist_f64(q, ix->centroids + (int64_t)l * ix->dim, ix->dim);
    scratch[l].id = l;
  }
  qsort(scratch, (size_t)ix->nlist, sizeof(pair_t), pair_cmp);
  if (np > ix->nlist) np = ix->nlist;
  for (int p = 0; p < np; ++p) {
    out_l[p] = scratch[p].id;
    if (out_d) out_d[p] = scratch[p].d;
  }
  return np;
}

/* ------------------------------------------------------------------------ */
/* Step 2 through a navigation graph over the list centroids (Sec. 4.1: the  */
/* host traverses an in-memory graph whose vertices are the posting-list    */
/* centroids, each joined to its nearest neighbours, to find the top-m      */
/* lists).  The traversal read here is a best-first beam search:            */
/*   - the candidate set C holds at most `beam` (distance, list) pairs,      */
/*     ascending, each marked expanded or not; every centroid whose          */
/*     distance has been computed is "visited" and never computed again;     */
/*   - C starts with the entry vertices (their `beam` smallest);             */
/*   - repeatedly the smallest member of C not yet expanded is expanded:     */
/*     each unvisited neighbour is visited and offered to C, which keeps its */
/*     `beam` smallest pairs; the search ends when every member of C has     */
/*     been expanded;                                                        */
/*   - the result is C's first m pairs.                                      */
/* beam is raised to m when smaller.  Distances are those of the exact      */
/* probe (float64 sums rounded once), ties to the lower list.  Pairs are     */
/* never re-admitted once dropped (C's largest member only decreases once C  */
/* is full), so each list is expanded at most once and the search ends.      */

typedef struct {
  pair_t p;
  int expanded;
} beam_t;

/* Offer pair x to the ascending candidate set c[0..*cnt) of capacity cap. */
static void beam_offer(beam_t* c, int* cnt, int cap, pair_t x) {
  if (*cnt == cap && pair_cmp(&x, &c[cap - 1].p) >= 0) return;
  int pos = *cnt < cap ? *cnt : cap - 1;
  while (pos > 0 && pair_cmp(&x, &c[pos - 1].p) < 0) {
    c[pos] = c[pos - 1];
    --pos;
  }
  c[pos].p = x;
  c[pos].expanded = 0;
  if (*cnt < cap) ++*cnt;
}

/* One query's graph walk; returns the lists found (<= np) and adds the
 * distances it computed to *ndist. */
static int graph_probe_one(const orc_index* ix, const double* q, const int32_t* adj, int deg,
                           const int32_t* entry, int n_entry, int beam, int np, int32_t* out_l,
                           float* out_d, beam_t* c, uint8_t* visited, int64_t* ndist) {
  if (np > ix->nlist) np = ix->nlist;
  if (np < 0) np = 0;
  if (beam < np) beam = np;
  if (beam < 1) beam = 1;
  memset(visited, 0, (size_t)ix->nlist);
  int cnt = 0;
  for (int i = 0; i < n_entry; ++i) {
    const int32_t e = entry[i];
    if (e < 0 || e >= ix->nlist || visited[e]) continue;
    visited[e] = 1;
    ++*ndist;
    pair_t x;
    x.d = sqdist_f64(q, ix->centroids + (int64_t)e * ix->dim, ix->dim);
    x.id = e;
    beam_offer(c, &cnt, beam, x);
  }
  for (;;) {
    int i = 0;
    while (i < cnt && c[i].expanded) ++i;
    if (i == cnt) break;
    c[i].expanded = 1;
    const int32_t v = c[i].p.id;
    for (int j = 0; j < deg; ++j) {
      const int32_t u = adj[(int64_t)v * deg + j];
      if (u < 0 || u >= ix->nlist || visited[u]) continue;
      visited[u] = 1;
      ++*ndist;
      pair_t x;
      x.d = sqdist_f64(q, ix->centroids + (int64_t)u * ix->dim, ix->dim);
      x.id = u;
      beam_offer(c, &cnt, beam, x);
    }
  }
  const int got = cnt < np ? cnt : np;
  for (int p = 0; p < got; ++p) {
    out_l[p] = c[p].p.id;
    if (out_d) out_d[p] = c[p].p.d;
  }
  return got;
}

/* A navigation graph: adj[nlist][deg] neighbour lists (-1 padded), the entry
 * vertices, and the beam width of the walk. */
typedef struct {
  const int32_t* adj;
  int32_t deg;
  int32_t n_entry;
  const int32_t* entry;
  int32_t beam;
  int32_t pad_;
} orc_graph;

/* The binary16 value nearest to x, ties to the even significand, as a float
 * (exact: every binary16 value is a float).  binary16 has 10 fraction bits,
 * normal magnitudes in [2^-14, 65504] and subnormal spacing 2^-24; magnitudes
 * from 65520 (half-way to the first power of two it cannot hold) overflow to
 * infinity.  Computed from that definition in float64: the spacing of x's
 * binade divides x exactly, nearbyint rounds half to even. */
static float round_to_half(float x) {
  if (isnan(x)) return x;
  const double a = fabs((double)x);
  if (a >= 65520.0) return copysignf(INFINITY, x);
  double quantum = 0x1p-24;
  if (a >= 0x1p-14) {
    int e;
    (void)frexp(a, &e); /* a = f 2^e with f in [0.5, 1): the binade starts at 2^(e-1) */
    quantum = ldexp(1.0, e - 1 - 10);
  }
  const double r = nearbyint(a / quantum) * quantum;
  return copysignf((float)r, x);
}

/* Step 1: distance table L[m][j] = sum_t (q[m*dsub+t] - CB[m][j][t])^2.
 * With f16 the float32 entry is then rounded to binary16 (the half-precision
 * table variant) and kept widened back to float32. */
static void lut_one(const orc_index* ix, const double* q, float* lut32, double* lut64, int f16) {
  for (int m = 0; m < ix->m; ++m) {
    for (int j = 0; j < ix->ksub; ++j) {
      const float* c = ix->codebooks + ((int64_t)m * ix->ksub + j) * ix->dsub;
      double acc = 0.0;
      for (int t = 0; t < ix->dsub; ++t) {
        double u = q[m * ix->dsub + t] - (double)c[t];
        double sq = u * u;
        acc = acc + sq;
      }
      lut32[m * ix->ksub + j] = f16 ? round_to_half((float)acc) : (float)acc;
      if (lut64) lut64[m * ix->ksub + j] = acc;
    }
  }
}

/* Steps 3 and 5: the multiset of IDs of the probed lists, then its set of
 * distinct IDs in ascending order.  Returns the multiset size. */
static int64_t gather_dedup(const orc_index* ix, const int32_t* probe, int np, int32_t* buf,
                            int64_t* n_unique) {
  int64_t g = 0;
  for (int p = 0; p < np; ++p) {
    int32_t l = probe[p];
    for (int64_t e = ix->offsets[l]; e < ix->offsets[l + 1]; ++e) buf[g++] = ix->entries[e];
  }
  qsort(buf, (size_t)g, sizeof(int32_t), i32_cmp);
  int64_t u = 0;
  for (int64_t i = 0; i < g; ++i)
    if (u == 0 || buf[u - 1] != buf[i]) buf[u++] = buf[i];
  *n_unique = u;
  return g;
}

/* Step 6, Eq. 1: float32 sum of table entries over m = 0..M-1. */
static float adc_one(const orc_index* ix, const float* lut32, int64_t v) {
  const uint8_t* code = ix->codes + v * ix->m;
  float a = 0.0f;
  for (int m = 0; m < ix->m; ++m) a = a + lut32[m * ix->ksub + code[m]];
  return a;
}

/* ------------------------------------------------------------------------ */
/* Step 8, heuristic form: re-ranking in mini-batches that stops once the    */
/* exact top-k has settled (Alg. 1; change rate of Eq. 3).                   */
/*                                                                           */
/* The candidates are visited in ascending (ADC distance, id) order, `batch` */
/* at a time.  `best` holds the k smallest (exact distance, id) pairs of the */
/* candidates visited so far, ascending, each with its candidate's position  */
/* in the visiting order.  A pair that drops out of `best` never returns     */
/* (the k-th smallest pair only decreases), so the IDs that are in `best`    */
/* after a mini-batch but were not before it are exactly the members whose   */
/* position lies inside that mini-batch.  Their number divided by k is the   */
/* change rate.  Re-ranking ends once the change rate has been <= eps after  */
/* beta mini-batches in a row, or when the candidates run out.  Returns the  */
/* number of candidates whose exact distance was computed.                   */

typedef struct {
  pair_t p;
  int64_t pos;
} member_t;

static int64_t heuristic_rerank(const orc_index* ix, const double* q, const int32_t* qi,
                                const pair_t* tasks, int64_t ntask, int k, int batch, double eps,
                                int beta, member_t* best, int* out_n) {
  int nbest = 0, quiet = 0;
  int64_t pos = 0;
  while (pos < ntask) {
    const int64_t start = pos;
    const int64_t end = ntask - pos > batch ? pos + batch : ntask;
    for (; pos < end; ++pos) {
      member_t c;
      c.p.id = tasks[pos].id;
      c.p.d = exact_dist(ix, q, qi, c.p.id);
      c.pos = pos;
      if (nbest == k && pair_cmp(&c.p, &best[k - 1].p) >= 0) continue;
      int at = nbest < k ? nbest++ : k - 1; /* when full, the largest pair drops out */
      while (at > 0 && pair_cmp(&c.p, &best[at - 1].p) < 0) {
        best[at] = best[at - 1];
        --at;
      }
      best[at] = c;
    }
    int joined = 0;
    for (int t = 0; t < nbest; ++t) joined += best[t].pos >= start;
    const double rate = (double)joined / (double)k; /* Eq. 3: over k, however full */
    quiet = rate <= eps ? quiet + 1 : 0;
    if (quiet >= beta) break;
  }
  *out_n = nbest;
  return pos;
}

/* ------------------------------------------------------------------------ */
/* Raw vectors on pages (Sec. 4.3, optimized storage layout): one bucket per */
/* posting list holding the vectors whose nearest list it is (no vector in  */
/* two buckets), ascending ID.  A page holds floor(page_bytes / row_bytes)   */
/* whole vectors.  Each bucket's full pages come first, bucket by bucket;   */
/* the leftover tails (fewer vectors than a page) are then combined onto    */
/* shared pages: a new page takes the largest remaining tail, then keeps     */
/* taking the largest remaining tail that still fits its free slots (ties:  */
/* lower bucket), until none fits.  Reading of the paper's max-min          */
/* combination of unaligned bucket portions.                                 */

typedef struct {
  int32_t* head; /* per tail size: first bucket on that size's list, ascending bucket */
  int32_t* next;
} tail_lists;

int64_t orc_page_layout(const int32_t* bucket_of, int64_t n, int32_t nbuckets, int32_t row_bytes,
                        int32_t page_bytes, int32_t* page, int32_t* slot) {
  const int P = page_bytes / row_bytes;
  if (P < 1) return -1;
  int64_t* cnt = (int64_t*)calloc((size_t)nbuckets + 1, sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) cnt[bucket_of[v] + 1]++;
  for (int b = 0; b < nbuckets; ++b) cnt[b + 1] += cnt[b]; /* bucket starts */
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nbuckets);
  int32_t* members = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int b = 0; b < nbuckets; ++b) fill[b] = cnt[b];
  for (int64_t v = 0; v < n; ++v) members[fill[bucket_of[v]]++] = (int32_t)v; /* ascending ID */
  int64_t pages = 0;
  for (int b = 0; b < nbuckets; ++b) { /* full pages */
    const int64_t c = cnt[b + 1] - cnt[b];
    for (int64_t i = 0; i < c / P * P; ++i) {
      const int32_t v = members[cnt[b] + i];
      page[v] = (int32_t)(pages + i / P);
      slot[v] = (int32_t)(i % P);
    }
    pages += c / P;
  }
  /* tails, largest first; per size a list of buckets in ascending order */
  tail_lists tl;
  tl.head = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
  tl.next = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nbuckets > 0 ? nbuckets : 1));
  int32_t* tail = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
  for (int t = 0; t < P; ++t) tl.head[t] = tail[t] = -1;
  int64_t left = 0;
  for (int b = 0; b < nbuckets; ++b) {
    const int t = (int)((cnt[b + 1] - cnt[b]) % P);
    tl.next[b] = -1;
    if (t == 0) continue;
    if (tail[t] < 0) tl.head[t] = b;
    else tl.next[tail[t]] = b;
    tail[t] = b;
    ++left;
  }
  while (left > 0) {
    int free_slots = P, used = 0;
    for (;;) {
      int t = free_slots < P - 1 ? free_slots : P - 1;
      while (t > 0 && tl.head[t] < 0) --t;
      if (t == 0) break;
      const int b = tl.head[t];
      tl.head[t] = tl.next[b];
      const int64_t c = cnt[b + 1] - cnt[b];
      for (int i = 0; i < t; ++i) {
        const int32_t v = members[cnt[b] + c - t + i];
        page[v] = (int32_t)pages;
        slot[v] = used + i;
      }
      used += t;
      free_slots -= t;
      --left;
    }
    ++pages;
  }
  free(cnt);
  free(fill);
  free(members);
  free(tl.head);
  free(tl.next);
  free(tail);
  return pages;
}

/* Pages read for one query's re-ranking with intra- and inter-mini-batch
 * de-duplication (Sec. 4.3): the candidates are re-ranked in mini-batches
 * (the fixed re-rank is one mini-batch of all of them); a mini-batch reads
 * each page its candidates lie on once, and none that an earlier mini-batch
 * of the same query has already read (those stay in the buffer).  `order`:
 * the candidates in visiting order, of which the first `used` were re-ranked
 * in mini-batches of `batch`.  `seen` has room for `used` page IDs. */
static int64_t count_page_reads(const int32_t* page, const pair_t* order, int64_t used,
                                int64_t batch, int32_t* seen) {
  int64_t nseen = 0, reads = 0;
  for (int64_t b0 = 0; b0 < used; b0 += batch) {
    const int64_t b1 = used - b0 > batch ? b0 + batch : used;
    const int64_t before = nseen; /* pages held when the mini-batch starts */
    for (int64_t i = b0; i < b1; ++i) {
      const int32_t pg = page[order[i].id];
      int have = 0;
      for (int64_t j = 0; j < nseen && !have; ++j) have = seen[j] == pg;
      if (!have) seen[nseen++] = pg;
    }
    reads += nseen - before;
  }
  return reads;
}

/* ------------------------------------------------------------------------ */
/* Public entry points.  All arrays are host arrays owned by the caller.     */

/* Step 2 for a batch.  probe/pdist: nq x nprobe_max, padded with -1/+inf. */
void orc_probe(const orc_index* ix, const float* Q, int64_t nq, const int32_t* nprobe,
               int32_t nprobe_max, int32_t* probe, float* pdist, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double* q = (double*)malloc(sizeof(double) * ix->dim);
    pair_t* scratch = (pair_t*)malloc(sizeof(pair_t) * ix->nlist);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
    for (int64_t i = 0; i < nq; ++i) {
      convert_query(ix, Q + i * ix->dim, q);
      int np = nprobe[i];
      int32_t* pl = probe + i * nprobe_max;
      float* pd = pdist ? pdist + i * nprobe_max : NULL;
      int got = probe_one(ix, q, np, pl, pd, scratch);
      for (int p = got; p < nprobe_max; ++p) {
        pl[p] = -1;
        if (pd) pd[p] = INFINITY;
      }
    }
    free(q);
    free(scratch);
  }
}

/* Step 2 for a batch through a navigation graph.  probe/pdist: nq x
 * nprobe_max, padded with -1/+inf; ndist (optional, nq): centroid distances
 * computed by each query's walk. */
void orc_graph_probe(const orc_index* ix, const orc_graph* g, const float* Q, int64_t nq,
                     const int32_t* nprobe, int32_t nprobe_max, int32_t* probe, float* pdist,
                     int64_t* ndist, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double* q = (double*)malloc(sizeof(double) * ix->dim);
    int cap = g->beam > nprobe_max ? g->beam : nprobe_max;
    if (cap < 1) cap = 1;
    beam_t* c = (beam_t*)malloc(sizeof(beam_t) * cap);
    uint8_t* visited = (uint8_t*)malloc((size_t)ix->nlist);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
    for (int64_t i = 0; i < nq; ++i) {
      convert_query(ix, Q + i * ix->dim, q);
      int32_t* pl = probe + i * nprobe_max;
      float* pd = pdist ? pdist + i * nprobe_max : NULL;
      int64_t nd = 0;
      int np = nprobe[i] < nprobe_max ? nprobe[i] : nprobe_max;
      int got = graph_probe_one(ix, q, g->adj, g->deg, g->entry, g->n_entry, g->beam, np, pl, pd,
                                c, visited, &nd);
      for (int p = got; p < nprobe_max; ++p) {
        pl[p] = -1;
        if (pd) pd[p] = INFINITY;
      }
      if (ndist) ndist[i] = nd;
    }
    free(q);
    free(c);
    free(visited);
  }
}

/* Step 1 for a batch.  lut32: nq x M x ksub; lut64 optional (same shape);
 * f16: round the float32 entries to binary16. */
void orc_lut(const orc_index* ix, const float* Q, int64_t nq, float* lut32, double* lut64,
             int f16) {
  double* q = (double*)malloc(sizeof(double) * ix->dim);
  int64_t per = (int64_t)ix->m * ix->ksub;
  for (int64_t i = 0; i < nq; ++i) {
    convert_query(ix, Q + i * ix->dim, q);
    lut_one(ix, q, lut32 + i * per, lut64 ? lut64 + i * per : NULL, f16);
  }
  free(q);
}

/* binary16 rounding of explicit values (exposed for its pins). */
void orc_round_half(const float* x, int64_t n, float* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = round_to_half(x[i]);
}

/* Steps 3+5 for one probe list: writes the distinct IDs (ascending) into
 * out (capacity >= multiset size), returns the multiset size. */
int64_t orc_gather_dedup(const orc_index* ix, const int32_t* probe, int32_t np, int32_t* out,
                         int64_t* n_unique) {
  return gather_dedup(ix, probe, np, out, n_unique);
}

/* Step 6 for explicit IDs with a given table (M x ksub): float32 sums and,
 * optionally, float64 sums of the float64 table. */
void orc_adc(const orc_index* ix, const float* lut32, const double* lut64, const int32_t* ids,
             int64_t n, float* adc32, double* adc64) {
  for (int64_t i = 0; i < n; ++i) {
    adc32[i] = adc_one(ix, lut32, ids[i]);
    if (adc64) {
      const uint8_t* code = ix->codes + (int64_t)ids[i] * ix->m;
      double a = 0.0;
      for (int m = 0; m < ix->m; ++m) a = a + lut64[m * ix->ksub + code[m]];
      adc64[i] = a;
    }
  }
}

/* Exact squared distances of explicit IDs to one query (after conversion). */
void orc_exact(const orc_index* ix, const float* q32, const int32_t* ids, int64_t n, float* out) {
  double* q = (double*)malloc(sizeof(double) * ix->dim);
  int32_t* qi = (int32_t*)malloc(sizeof(int32_t) * ix->dim);
  convert_query(ix, q32, q);
  int_query(ix, q, qi);
  for (int64_t i = 0; i < n; ++i) out[i] = exact_dist(ix, q, qi, ids[i]);
  free(q);
  free(qi);
}

/*
 * Steps 1-8 for a batch of queries.
 *   nprobe[i]            lists probed by query i (clamped to nlist)
 *   ids, dists           nq x k final results (-1 / +inf padded)
 *   topn_ids, topn_adc   optional nq x rerank_n: the step-7 selection, ascending
 *   ncand                optional nq: distinct candidates scored by Eq. 1
 *   nentries             optional nq: list entries gathered (with duplicates)
 *   lut_f16              1: the half-precision table variant (entries rounded
 *                        to binary16, summed in float32 as in Eq. 1)
 *   h_batch              > 0: step 8 is the heuristic re-ranking (Alg. 1) with
 *                        mini-batches of h_batch, threshold h_eps, count h_beta;
 *                        0: the fixed-n re-rank
 *   reranked             optional nq: candidates whose exact distance was computed
 *   page, page_reads     optional: the page of every vector (orc_page_layout) and,
 *                        per query, the pages its re-ranking reads (Sec. 4.3)
 */
void orc_search(const orc_index* ix, const float* Q, int64_t nq, const int32_t* nprobe,
                int32_t k, int32_t rerank_n, int64_t* ids, float* dists, int32_t* topn_ids,
                float* topn_adc, int64_t* ncand, int64_t* nentries, int nthreads, int lut_f16,
                int32_t h_batch, double h_eps, int32_t h_beta, int64_t* reranked,
                const int32_t* page, int64_t* page_reads, const orc_graph* graph) {
  int64_t maxg = ix->offsets[ix->nlist];
  if (maxg < 1) maxg = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double* q = (double*)malloc(sizeof(double) * ix->dim);
    int32_t* qi = (int32_t*)malloc(sizeof(int32_t) * ix->dim);
    pair_t* scratch = (pair_t*)malloc(sizeof(pair_t) * (ix->nlist > maxg ? ix->nlist : maxg));
    int32_t* probe = (int32_t*)malloc(sizeof(int32_t) * ix->nlist);
    float* lut = (float*)malloc(sizeof(float) * ix->m * ix->ksub);
    int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * maxg);
    pair_t* rr = (pair_t*)malloc(sizeof(pair_t) * (rerank_n > 0 ? rerank_n : 1));
    member_t* best = (member_t*)malloc(sizeof(member_t) * (k > 0 ? k : 1));
    int32_t* seen = (int32_t*)malloc(sizeof(int32_t) * (rerank_n > 0 ? rerank_n : 1));
    beam_t* gc = NULL;
    uint8_t* visited = NULL;
    if (graph) {
      int cap = graph->beam > ix->nlist ? graph->beam : ix->nlist;
      gc = (beam_t*)malloc(sizeof(beam_t) * (cap > 0 ? cap : 1));
      visited = (uint8_t*)malloc((size_t)ix->nlist);
    }
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < nq; ++i) {
      convert_query(ix, Q + i * ix->dim, q);
      int_query(ix, q, qi);
      lut_one(ix, q, lut, NULL, lut_f16);                          /* step 1 */
      int np;                                                      /* step 2 */
      if (graph) {
        int64_t nd = 0;
        np = graph_probe_one(ix, q, graph->adj, graph->deg, graph->entry, graph->n_entry,
                             graph->beam, nprobe[i], probe, NULL, gc, visited, &nd);
      } else {
        np = probe_one(ix, q, nprobe[i], probe, NULL, scratch);
      }
      int64_t nu = 0;
      int64_t g = gather_dedup(ix, probe, np, buf, &nu);           /* steps 3, 5 */
      for (int64_t c = 0; c < nu; ++c) {                           /* step 6 */
        scratch[c].d = adc_one(ix, lut, buf[c]);
        scratch[c].id = buf[c];
      }
      qsort(scratch, (size_t)nu, sizeof(pair_t), pair_cmp);        /* step 7 */
      int64_t nn = nu < rerank_n ? nu : rerank_n;
      if (topn_ids) {
        for (int64_t c = 0; c < rerank_n; ++c) {
          topn_ids[i * rerank_n + c] = c < nn ? scratch[c].id : -1;
          topn_adc[i * rerank_n + c] = c < nn ? scratch[c].d : INFINITY;
        }
      }
      int64_t nout = nn, nre = nn;
      if (h_batch > 0) {                                           /* step 8, Alg. 1 */
        int hn = 0;
        nre = heuristic_rerank(ix, q, qi, scratch, nn, k, h_batch, h_eps, h_beta, best, &hn);
        for (int c = 0; c < hn; ++c) rr[c] = best[c].p;
        nout = hn;
      } else {                                                     /* step 8, fixed n */
        for (int64_t c = 0; c < nn; ++c) {
          rr[c].id = scratch[c].id;
          rr[c].d = exact_dist(ix, q, qi, scratch[c].id);
        }
        qsort(rr, (size_t)nn, sizeof(pair_t), pair_cmp);
      }
      for (int c = 0; c < k; ++c) {
        ids[i * k + c] = c < nout ? (int64_t)rr[c].id : -1;
        dists[i * k + c] = c < nout ? rr[c].d : INFINITY;
      }
      if (reranked) reranked[i] = nre;
      if (page && page_reads)
        page_reads[i] = count_page_reads(page, scratch, nre, h_batch > 0 ? h_batch : (nn > 0 ? nn : 1),
                                         seen);
      if (ncand) ncand[i] = nu;
      if (nentries) nentries[i] = g;
    }
    free(q);
    free(qi);
    free(scratch);
    free(probe);
    free(lut);
    free(buf);
    free(rr);
    free(best);
    free(seen);
    free(gc);
    free(visited);
  }
}

/* Exact k nearest neighbours over all N vectors, ordered by (distance, id). */
void orc_bruteforce(const orc_index* ix, const float* Q, int64_t nq, int32_t k, int64_t* ids,
                    float* dists, int nthreads) {
  if (k <= 0) return;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double* q = (double*)malloc(sizeof(double) * ix->dim);
    int32_t* qi = (int32_t*)malloc(sizeof(int32_t) * ix->dim);
    pair_t* best = (pair_t*)malloc(sizeof(pair_t) * (k + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < nq; ++i) {
      convert_query(ix, Q + i * ix->dim, q);
      int_query(ix, q, qi);
      int cnt = 0;
      for (int64_t v = 0; v < ix->n; ++v) {
        pair_t p;
        p.d = exact_dist(ix, q, qi, v);
        p.id = (int32_t)v;
        if (cnt == k && pair_cmp(&p, &best[k - 1]) >= 0) continue;
        /* insertion into the sorted best list */
        int pos = cnt < k ? cnt : k - 1;
        while (pos > 0 && pair_cmp(&p, &best[pos - 1]) < 0) {
          best[pos] = best[pos - 1];
          --pos;
        }
        best[pos] = p;
        if (cnt < k) ++cnt;
      }
      for (int c = 0; c < k; ++c) {
        ids[i * k + c] = c < cnt ? (int64_t)best[c].id : -1;
        dists[i * k + c] = c < cnt ? best[c].d : INFINITY;
      }
    }
    free(q);
    free(qi);
    free(best);
  }
}
