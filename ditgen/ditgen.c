/*
 * ditgen — seeded synthetic web-like directed graphs in CSC form.
 *
 * This module produces inputs only. It holds none of the D-iteration
 * arithmetic; both the FP64 oracle and the GPU library consume its output.
 *
 * Model (one reading of the paper's workload, whose web-crawl dataset of
 * Section 3 is replaced by a synthetic stand-in):
 *   - every node is dangling (no out-link) with probability p_dangling;
 *   - other nodes draw an out-degree k in [deg_min, deg_max] from a
 *     Zipf-Mandelbrot law P(k) ~ (k + s)^-zipf_exponent, with the offset s
 *     solved so that the mean out-degree over all nodes is mean_outdeg;
 *   - each out-link is "local" with probability p_local: uniform over the
 *     other ids of the source's block of `block` consecutive ids; otherwise
 *     it is preferential: drawn from static Chung-Lu weights
 *     w_v ~ (v+1)^(-1/(gamma-1)), so the in-degree tail has exponent ~gamma
 *     and hubs sit at low ids, as in a crawl order;
 *   - targets of one source are distinct and never the source itself; local
 *     links beyond the block's capacity become preferential ones;
 *   - each column (the out-link list of a source) is emitted sorted.
 *
 * Randomness is SplitMix64 keyed by (seed, node, stream), so the result does
 * not depend on the thread count. Built without fast-math.
 *
 * Column j of the CSC holds the out-neighbours of node j: col_ptr[j] ..
 * col_ptr[j+1]-1 index row_idx. int32 throughout (edge count < 2^31).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n;            /* number of nodes */
  int32_t block;        /* locality block size (consecutive ids) */
  int32_t deg_min;      /* smallest out-degree of a non-dangling node */
  int32_t deg_max;      /* largest out-degree */
  double zipf_exponent; /* tail exponent of the out-degree law */
  double mean_outdeg;   /* target mean out-degree over ALL nodes */
  double p_dangling;    /* probability that a node has no out-link */
  double p_local;       /* probability that a link stays in the block */
  double gamma;         /* in-degree power-law exponent of the preferential part */
  uint64_t seed;
} ditgen_params;

enum { DITGEN_OK = 0, DITGEN_EINVAL = -1, DITGEN_ENOMEM = -2, DITGEN_ETOOBIG = -3 };

/* ---------- SplitMix64 (Steele, Lea, Flood 2014) ---------- */
static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t sm_next(uint64_t* s) {
  *s += 0x9E3779B97F4A7C15ULL;
  return sm_mix(*s);
}
static inline double sm_u01(uint64_t* s) { return (double)(sm_next(s) >> 11) * 0x1.0p-53; }
/* uniform integer in [0, m), m >= 1, by rejection (no modulo bias) */
static inline uint64_t sm_below(uint64_t* s, uint64_t m) {
  uint64_t lim = UINT64_MAX - (UINT64_MAX % m);
  uint64_t x;
  do { x = sm_next(s); } while (x >= lim);
  return x % m;
}
static inline uint64_t stream_state(uint64_t seed, uint64_t node, uint64_t stream) {
  return sm_mix(sm_mix(seed ^ 0xD1B54A32D192ED03ULL) ^ sm_mix(node * 4 + stream + 0x8CB92BA72F3D8DD7ULL));
}

static int check_params(const ditgen_params* p) {
  if (!p || p->n < 0 || p->n >= ((int64_t)1 << 31) || p->block < 1 || p->deg_min < 1 ||
      p->deg_max < p->deg_min || !(p->zipf_exponent > 0) || !(p->mean_outdeg >= 0) ||
      !(p->p_dangling >= 0 && p->p_dangling <= 1) || !(p->p_local >= 0 && p->p_local <= 1) ||
      !(p->gamma > 1.0))
    return DITGEN_EINVAL;
  return DITGEN_OK;
}

/* mean of P(k) ~ (k+s)^-a on [lo, hi] */
static double zm_mean(double s, double a, int lo, int hi) {
  double num = 0, den = 0;
  for (int k = lo; k <= hi; ++k) {
    double w = pow(k + s, -a);
    num += k * w;
    den += w;
  }
  return num / den;
}

/* Offset s with mean over non-dangling nodes = mean_outdeg / (1 - p_dangling).
 * The mean grows with s; s is searched in (1 - lo, 1e6]. The target is clamped
 * to the reachable range. */
int ditgen_zipf_offset(const ditgen_params* p, double* s_out) {
  int rc = check_params(p);
  if (rc) return rc;
  double want = p->p_dangling < 1 ? p->mean_outdeg / (1.0 - p->p_dangling) : 0;
  double a = p->zipf_exponent;
  double lo = 1.0 - p->deg_min + 1e-9, hi = 1e6;
  if (want <= zm_mean(lo, a, p->deg_min, p->deg_max)) { *s_out = lo; return DITGEN_OK; }
  if (want >= zm_mean(hi, a, p->deg_min, p->deg_max)) { *s_out = hi; return DITGEN_OK; }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (zm_mean(mid, a, p->deg_min, p->deg_max) < want) lo = mid; else hi = mid;
  }
  *s_out = 0.5 * (lo + hi);
  return DITGEN_OK;
}

/* out-degree of every node, before the N-1 cap */
static int32_t draw_degree(const ditgen_params* p, const double* dcdf, int nk, int64_t v) {
  uint64_t st = stream_state(p->seed, (uint64_t)v, 0);
  if (sm_u01(&st) < p->p_dangling) return 0;
  double u = sm_u01(&st);
  int lo = 0, hi = nk - 1; /* first index with dcdf > u */
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (dcdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  int32_t k = p->deg_min + lo;
  if (p->n - 1 < k) k = (int32_t)(p->n - 1);
  return k;
}

static double* degree_cdf(const ditgen_params* p, int* nk_out) {
  double s;
  ditgen_zipf_offset(p, &s);
  int nk = p->deg_max - p->deg_min + 1;
  double* c = (double*)malloc(sizeof(double) * nk);
  if (!c) return NULL;
  double acc = 0;
  for (int i = 0; i < nk; ++i) { acc += pow(p->deg_min + i + s, -p->zipf_exponent); c[i] = acc; }
  for (int i = 0; i < nk; ++i) c[i] /= acc;
  c[nk - 1] = 1.0 + 1e-12; /* u < 1 always lands inside */
  *nk_out = nk;
  return c;
}

/* Total edge count for these parameters (runs the degree draw). */
int64_t ditgen_count_edges(const ditgen_params* p) {
  int rc = check_params(p);
  if (rc) return rc;
  int nk;
  double* dcdf = degree_cdf(p, &nk);
  if (!dcdf) return DITGEN_ENOMEM;
  int64_t total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
  for (int64_t v = 0; v < p->n; ++v) total += draw_degree(p, dcdf, nk, v);
  free(dcdf);
  return total;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}
static inline int contains(const int32_t* t, int cnt, int32_t x) {
  for (int i = 0; i < cnt; ++i)
    if (t[i] == x) return 1;
  return 0;
}

/* Fill col_ptr[n+1] and row_idx[nnz]; nnz must equal ditgen_count_edges(p). */
int ditgen_build(const ditgen_params* p, int32_t* col_ptr, int32_t* row_idx, int64_t nnz) {
  int rc = check_params(p);
  if (rc) return rc;
  if (nnz >= ((int64_t)1 << 31)) return DITGEN_ETOOBIG;
  const int64_t n = p->n;
  int nk;
  double* dcdf = degree_cdf(p, &nk);
  double* wcdf = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  if (!dcdf || !wcdf) { free(dcdf); free(wcdf); return DITGEN_ENOMEM; }
  /* Chung-Lu weights, cumulative (sequential: fixed summation order) */
  {
    double e = -1.0 / (p->gamma - 1.0), acc = 0;
    for (int64_t v = 0; v < n; ++v) { acc += pow((double)(v + 1), e); wcdf[v] = acc; }
    for (int64_t v = 0; v < n; ++v) wcdf[v] /= acc;
    if (n > 0) wcdf[n - 1] = 1.0 + 1e-12;
  }
  /* degrees -> col_ptr (prefix sum) */
  col_ptr[0] = 0;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) col_ptr[v + 1] = draw_degree(p, dcdf, nk, v);
  for (int64_t v = 0; v < n; ++v) col_ptr[v + 1] += col_ptr[v];
  if (col_ptr[n] != nnz) { free(dcdf); free(wcdf); return DITGEN_EINVAL; }

#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    int32_t k = col_ptr[v + 1] - col_ptr[v];
    if (k == 0) continue;
    int32_t* t = row_idx + col_ptr[v];
    uint64_t st = stream_state(p->seed, (uint64_t)v, 1);
    int64_t blo = (v / p->block) * (int64_t)p->block;
    int64_t bhi = blo + p->block < n ? blo + p->block : n;
    int64_t avail = bhi - blo - 1;
    int nloc = 0;
    for (int i = 0; i < k; ++i) nloc += sm_u01(&st) < p->p_local;
    if (nloc > avail) nloc = (int)avail;
    int cnt = 0;
    /* local: Floyd's sampling of nloc distinct offsets from [0, avail) */
    for (int64_t jj = avail - nloc; jj < avail; ++jj) {
      int64_t c = (int64_t)sm_below(&st, (uint64_t)jj + 1);
      int32_t id = (int32_t)(blo + c + (blo + c >= v ? 1 : 0));
      if (contains(t, cnt, id)) id = (int32_t)(blo + jj + (blo + jj >= v ? 1 : 0));
      t[cnt++] = id;
    }
    /* preferential: Chung-Lu draws, rejecting self and repeats */
    int tries = 0;
    while (cnt < k) {
      int32_t id;
      if (tries < 64 * k) {
        ++tries;
        double u = sm_u01(&st);
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
          int64_t mid = (lo + hi) >> 1;
          if (wcdf[mid] > u) hi = mid; else lo = mid + 1;
        }
        id = (int32_t)lo;
        if (id == v || contains(t, cnt, id)) continue;
      } else { /* fallback for tiny graphs: first unused id from a random start */
        int64_t start = (int64_t)sm_below(&st, (uint64_t)n);
        id = -1;
        for (int64_t q = 0; q < n; ++q) {
          int32_t c = (int32_t)((start + q) % n);
          if (c != v && !contains(t, cnt, c)) { id = c; break; }
        }
      }
      t[cnt++] = id;
    }
    qsort(t, (size_t)k, sizeof(int32_t), cmp_i32);
  }
  free(dcdf);
  free(wcdf);
  return DITGEN_OK;
}
