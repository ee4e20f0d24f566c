/*
 * dref — plain sequential FP64 D-iteration: the ORACLE.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing but the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load or call this library; the GPU
 * library never does, and the two share no code.
 *
 * What it computes (Hong, "D-iteration: evaluation of the asynchronous
 * distributed computation", arXiv:1202.6168):
 *   - the fluid recursion F_n = (I - J_{i_n} + P J_{i_n}) F_{n-1}, F_0 = B
 *     (Section 2, equation defF) and the history H_n = sum_k J_{i_k} F_{k-1}
 *     (equation defH), run in the order of the Section 2.1 pseudo-code:
 *     take the fluid of node i, add it to H_i, zero F_i, give sent * p_ji to
 *     every child j;
 *   - node choice by the cyclic threshold test of Section 2.4: scan ids in
 *     ascending order, diffuse every node with |F_i| > T, then T <- T / alpha;
 *   - PageRank matrix of Section 2.2: p_ji = d / #out_i for each out-link
 *     i -> j; a node without out-link (dangling) only moves F_i into H_i;
 *   - partitions of Section 2.3: uniform and cost-balanced (CB), and the
 *     alternative the paper proposes there, blocks of equal internal p mass;
 *   - the general matrix of Section 2: a weighted graph whose link j -> i
 *     carries p_ij of either sign (one value per CSC entry), solved when P is
 *     strictly contractive (Section 1, equation affine);
 *   - the normalized node priority of Section 2.4, F_i / ((#in_i + 1)(#out_i + 1)),
 *     used by the threshold test in place of F_i when asked for.
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - stop when ||F||_1 <= rel_tol * ||B||_1 (the paper's r/(1-d) test with
 *     a relative target); r is recomputed once per sweep (Remark after the
 *     pseudo-code), as an FP64 sum in index order;
 *   - T_0 = max_i |F_i| / alpha; strict test |F_i| > T; if a sweep diffuses
 *     nothing, T <- min(T, max|F| / alpha) so the run never stalls;
 *   - a warm start H_0 gives F_0 = B + P H_0 - H_0, which follows from the two
 *     recursions (F_n - F_{n-1} = (P - I)(H_n - H_{n-1})).
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef struct {
  int64_t edges;       /* elementary diffusions (one per out-link of a diffused node) */
  int64_t diffusions;  /* node diffusions */
  int64_t sweeps;      /* cyclic passes over all ids */
  int64_t increases;   /* sweeps after which ||F||_1 grew (expected 0) */
  double resid_l1;     /* final ||F||_1 */
  double b_l1;         /* ||B||_1 */
  double seconds;      /* wall time of the iteration (steady clock) */
  int32_t converged;   /* 1 if resid_l1 <= rel_tol * b_l1 */
  int32_t pad;
} dref_stats;

enum { DREF_OK = 0, DREF_NOT_CONVERGED = 1, DREF_EINVAL = -1, DREF_EGRAPH = -2, DREF_ENOMEM = -3 };

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* CSC sanity: col_ptr[0] = 0, non-decreasing, col_ptr[n] = nnz, rows in [0, n). */
int dref_check_csc(int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx) {
  if (n < 0 || nnz < 0) return DREF_EINVAL;
  if (col_ptr[0] != 0 || col_ptr[n] != nnz) return DREF_EGRAPH;
  for (int64_t i = 0; i < n; ++i)
    if (col_ptr[i + 1] < col_ptr[i]) return DREF_EGRAPH;
  for (int64_t e = 0; e < nnz; ++e)
    if (row_idx[e] < 0 || row_idx[e] >= n) return DREF_EGRAPH;
  return DREF_OK;
}

/* Column norm bound of a general matrix: max over columns of sum |p_ji|.
 * The bound ||X - H||_1 <= ||F||_1 / (1 - c) of Section 2 holds with c = this
 * norm when it is below 1 (||P||_1 <= c). */
double dref_col_norm(int64_t n, const int32_t* col_ptr, const double* val) {
  double c = 0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0;
    for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) s += fabs(val[e]);
    if (s > c) c = s;
  }
  return c;
}

/* F = B + P H - H for a general matrix: entry e of column i carries val[e]. */
int dref_fluid_from_history_w(int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx,
                              const double* val, const double* b, const double* h, double* f) {
  (void)nnz;
  for (int64_t i = 0; i < n; ++i) f[i] = b[i] - h[i];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[row_idx[e]] += val[e] * h[i];
  return DREF_OK;
}

/* F = B + P H - H, straight from the definition of P (column i spreads
 * d / #out_i on each of its entries). */
int dref_fluid_from_history(int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx,
                            double d, const double* b, const double* h, double* f) {
  (void)nnz;
  for (int64_t i = 0; i < n; ++i) f[i] = b[i] - h[i];
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = col_ptr[i + 1] - col_ptr[i];
    if (k == 0) continue;
    double p = d / (double)k;
    for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[row_idx[e]] += p * h[i];
  }
  return DREF_OK;
}

static double norm1(const double* x, int64_t n) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += fabs(x[i]);
  return s;
}
/* largest |F_i| / c_i (c = NULL: all c_i = 1) */
static double max_scaled(const double* x, const double* c, int64_t n) {
  double m = 0;
  for (int64_t i = 0; i < n; ++i) {
    double v = c ? fabs(x[i]) / c[i] : fabs(x[i]);
    if (v > m) m = v;
  }
  return m;
}

/*
 * Sequential D-iteration until ||F||_1 <= rel_tol * ||B||_1.
 *   val      NULL: the PageRank matrix (p_ji = d / #out_i, Section 2.2);
 *            else the general matrix whose CSC entry e carries val[e]
 *            (Section 2; d is then only the contraction factor of the bound)
 *   priority 0: diffuse i when |F_i| > T (Section 2.4 cyclic test on F_i);
 *            1: when |F_i| / ((#in_i + 1)(#out_i + 1)) > T, the normalized
 *            priority of the argmax rule of Section 2.4 under the same cyclic
 *            threshold (T_0 and the no-pass rule use the same ratio)
 *   h0       optional warm start (NULL = zero history)
 *   h, f     outputs [n]: history and remaining fluid
 *   r_hist   optional [r_hist_cap] record of ||F||_1 after each sweep
 * Returns DREF_OK, DREF_NOT_CONVERGED (max_sweeps hit; h, f still valid) or
 * a negative error.
 */
int dref_solve_ex(int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx, double d,
                  const double* val, int priority, const double* b, const double* h0, double rel_tol,
                  double alpha, int64_t max_sweeps, double* h, double* f, dref_stats* st,
                  double* r_hist, int64_t r_hist_cap) {
  memset(st, 0, sizeof(*st));
  if (!(d > 0 && d < 1) || !(alpha > 1) || !(rel_tol >= 0)) return DREF_EINVAL;
  int rc = dref_check_csc(n, nnz, col_ptr, row_idx);
  if (rc) return rc;
  double* c = NULL; /* (#in_i + 1)(#out_i + 1), priority only */
  if (priority) {
    c = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!c) return DREF_ENOMEM;
    for (int64_t e = 0; e < nnz; ++e) c[row_idx[e]] += 1.0; /* #in */
    for (int64_t i = 0; i < n; ++i) c[i] = (c[i] + 1.0) * (double)(col_ptr[i + 1] - col_ptr[i] + 1);
  }

  double t_start = now_s();
  if (h0) {
    memcpy(h, h0, sizeof(double) * n);
    if (val) dref_fluid_from_history_w(n, nnz, col_ptr, row_idx, val, b, h, f);
    else dref_fluid_from_history(n, nnz, col_ptr, row_idx, d, b, h, f);
  } else {
    memset(h, 0, sizeof(double) * n);
    memcpy(f, b, sizeof(double) * n);
  }
  st->b_l1 = norm1(b, n);
  const double target = rel_tol * st->b_l1;
  double r = norm1(f, n);
  double T = max_scaled(f, c, n) / alpha;

  while (r > target && st->sweeps < max_sweeps) {
    int64_t passed = 0;
    for (int64_t i = 0; i < n; ++i) {
      const double Ti = c ? T * c[i] : T;
      if (!(fabs(f[i]) > Ti)) continue;
      double sent = f[i];
      h[i] += sent;
      f[i] = 0.0;
      int64_t k = col_ptr[i + 1] - col_ptr[i];
      if (val) {
        for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[row_idx[e]] += sent * val[e];
      } else if (k > 0) {
        double p = d / (double)k; /* p_ji for every child j of i */
        for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) f[row_idx[e]] += sent * p;
      }
      st->edges += k;
      st->diffusions += 1;
      ++passed;
    }
    st->sweeps += 1;
    double r_new = norm1(f, n);
    if (r_new > r) st->increases += 1;
    r = r_new;
    if (r_hist && st->sweeps <= r_hist_cap) r_hist[st->sweeps - 1] = r;
    T /= alpha;
    if (passed == 0) {
      double m = max_scaled(f, c, n) / alpha;
      if (m < T) T = m;
    }
  }
  free(c);
  st->resid_l1 = r;
  st->converged = r <= target;
  st->seconds = now_s() - t_start;
  return st->converged ? DREF_OK : DREF_NOT_CONVERGED;
}

/* The PageRank matrix with the plain |F_i| test. */
int dref_solve(int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx, double d,
               const double* b, const double* h0, double rel_tol, double alpha, int64_t max_sweeps,
               double* h, double* f, dref_stats* st, double* r_hist, int64_t r_hist_cap) {
  return dref_solve_ex(n, nnz, col_ptr, row_idx, d, NULL, 0, b, h0, rel_tol, alpha, max_sweeps, h, f,
                       st, r_hist, r_hist_cap);
}

/* Uniform partition (Section 2.3): K contiguous ranges of floor(n/K) ids, the
 * last one also taking the remainder. ptr has K+1 entries. */
int dref_partition_uniform(int64_t n, int64_t K, int64_t* ptr) {
  if (K < 1 || K > (n > 0 ? n : 1)) return DREF_EINVAL;
  int64_t q = n / K;
  for (int64_t k = 0; k < K; ++k) ptr[k] = k * q;
  ptr[K] = n;
  return DREF_OK;
}

/* Cost-balanced partition (Section 2.3): contiguous ranges whose out-link
 * counts equal L/K as nearly as integers allow. omega_k is the first id whose
 * out-link prefix reaches k L / K, i.e. the smallest j with
 * K * col_ptr[j] >= k * L (exact integer comparison, so the K = 2 split
 * reappears among the K = 4 boundaries). */
int dref_partition_cb(int64_t n, const int32_t* col_ptr, int64_t K, int64_t* ptr) {
  if (K < 1 || K > (n > 0 ? n : 1)) return DREF_EINVAL;
  int64_t L = col_ptr[n];
  int64_t j = 0;
  ptr[0] = 0;
  for (int64_t k = 1; k < K; ++k) {
    while (j < n && (int64_t)col_ptr[j] * K < k * L) ++j;
    ptr[k] = j;
  }
  ptr[K] = n;
  return DREF_OK;
}

/* Cost-balanced partition on in+out links: the CB rule above with the cost of
 * a prefix [0, j) taken as its out-links plus its in-links (in-links counted
 * here from the row indices). omega_k = min { j : K cost(j) >= k 2L }. */
int dref_partition_cb_inout(int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx,
                            int64_t K, int64_t* ptr) {
  if (K < 1 || K > (n > 0 ? n : 1)) return DREF_EINVAL;
  int64_t* cost = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cost) return DREF_ENOMEM;
  for (int64_t e = 0; e < nnz; ++e) cost[row_idx[e] + 1] += 1;   /* in-links of each node */
  for (int64_t j = 0; j < n; ++j) cost[j + 1] += cost[j];         /* in-link prefix */
  for (int64_t j = 0; j <= n; ++j) cost[j] += col_ptr[j];          /* + out-link prefix */
  const int64_t total = cost[n];
  int64_t j = 0;
  ptr[0] = 0;
  for (int64_t k = 1; k < K; ++k) {
    while (j < n && cost[j] * K < k * total) ++j;
    ptr[k] = j;
  }
  ptr[K] = n;
  free(cost);
  return DREF_OK;
}

/* Partition of equal internal p mass (the alternative balance proposed in
 * Section 2.3): the mass of a block [a, b) is the sum of |p_ji| over the links
 * i -> j with both ends in [a, b). Readings (the paper gives no rule):
 *   - each link weighs floor(|p_ji| 2^32) integer units, so that block masses
 *     are exact integers whatever order they are summed in;
 *   - "equal" is taken as the contiguous K-block partition whose largest
 *     block mass is smallest (t*), and among those the one whose blocks take,
 *     from the left, as many nodes as they can: omega_{k+1} is the largest j
 *     with m(omega_k, j) <= t*. When fewer than K blocks cover all nodes, the
 *     remaining boundaries are n (empty blocks).
 * val = NULL: PageRank weights d / #out_i. ptr has K+1 entries. */
static int64_t link_units(const double* val, double d, const int32_t* col_ptr, int64_t i, int64_t e) {
  double p = val ? fabs(val[e]) : d / (double)(col_ptr[i + 1] - col_ptr[i]);
  return (int64_t)floor(p * 4294967296.0);
}

/* greedy blocks under the bound t; writes up to K+1 boundaries into ptr when
 * ptr != NULL; returns the number of blocks needed to cover [0, n) */
static int64_t pmass_greedy(int64_t n, const int32_t* col_ptr, const int32_t* row_idx,
                            const int64_t* wout, const int32_t* in_ptr, const int32_t* in_src,
                            const int64_t* win, int64_t t, int64_t K, int64_t* ptr) {
  int64_t blocks = 1, a = 0, cur = 0;
  if (ptr) ptr[0] = 0;
  for (int64_t j = 0; j < n; ++j) {
    /* mass node j adds to the block [a, j): its links to [a, j] plus the links
       from [a, j) into it */
    int64_t inc = 0, self = 0;
    for (int64_t e = col_ptr[j]; e < col_ptr[j + 1]; ++e) {
      if (row_idx[e] >= a && row_idx[e] <= j) inc += wout[e];
      if (row_idx[e] == j) self += wout[e];
    }
    for (int64_t q = in_ptr[j]; q < in_ptr[j + 1]; ++q)
      if (in_src[q] >= a && in_src[q] < j) inc += win[q];
    if (j > a && cur + inc > t) { /* close [a, j), start [j, ...) */
      if (ptr && blocks < K) ptr[blocks] = j;
      ++blocks;
      a = j;
      cur = self;
    } else {
      cur += inc;
    }
  }
  if (ptr) {
    for (int64_t k = blocks; k <= K; ++k) ptr[k] = n;
  }
  return blocks;
}

int dref_partition_pmass(int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx,
                         const double* val, double d, int64_t K, int64_t* ptr) {
  if (K < 1 || K > (n > 0 ? n : 1)) return DREF_EINVAL;
  int64_t* wout = (int64_t*)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(int64_t));
  int32_t* in_ptr = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  int32_t* in_src = (int32_t*)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(int32_t));
  int64_t* win = (int64_t*)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(int64_t));
  int32_t* fill = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  if (!wout || !in_ptr || !in_src || !win || !fill) {
    free(wout), free(in_ptr), free(in_src), free(win), free(fill);
    return DREF_ENOMEM;
  }
  /* link weights, and the in-links of every node (source and weight) */
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) wout[e] = link_units(val, d, col_ptr, i, e);
  for (int64_t e = 0; e < nnz; ++e) in_ptr[row_idx[e] + 1] += 1;
  for (int64_t j = 0; j < n; ++j) in_ptr[j + 1] += in_ptr[j];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) {
      int64_t q = in_ptr[row_idx[e]] + fill[row_idx[e]]++;
      in_src[q] = (int32_t)i;
      win[q] = wout[e];
    }
  /* t* by bisection on the integers: feasible(t) = greedy needs <= K blocks;
     a single node's block holds its self-links, so t >= their largest mass */
  int64_t lo = 0, hi = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t self = 0;
    for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e)
      if (row_idx[e] == i) self += wout[e];
    if (self > lo) lo = self;
  }
  for (int64_t e = 0; e < nnz; ++e) hi += wout[e];
  if (hi < lo) hi = lo;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (pmass_greedy(n, col_ptr, row_idx, wout, in_ptr, in_src, win, mid, K, NULL) <= K) hi = mid;
    else lo = mid + 1;
  }
  pmass_greedy(n, col_ptr, row_idx, wout, in_ptr, in_src, win, lo, K, ptr);
  free(wout), free(in_ptr), free(in_src), free(win), free(fill);
  return DREF_OK;
}

/* Cut-minimizing cost-balanced partition: the CB boundaries slide, each within
 * a window and under a balance slack, to where the fewest short links cross.
 * It keeps more links inside their sets, the aim behind the internal-mass
 * balance of Section 2.3, while the sets stay contiguous and balanced.
 * Readings (the paper gives no rule; all of them are listed in the design
 * notes):
 *   - cost of node i: 1 + #out_i + min(#in_i, h) with h = max(1, floor(3L/N)):
 *     a node's own work, its pushes, and its inflow up to h links (the inflow
 *     of a row with more in-links is summed by all workgroups together);
 *   - CB targets t_k: the smallest j with K C(j) >= k C(n), C the cost prefix;
 *   - balance: every set costs at most cmax = cB + floor(cB / 10) and holds
 *     at most smax = sB + floor(sB / 10) nodes, where cB and sB are the
 *     largest cost and node count among the sets of the CB targets;
 *   - a link i -> j (i != j) is short when |i - j| < 2 ceil(N/K); cross(b)
 *     is the p mass of the short links with min(i, j) < b <= max(i, j), each
 *     link weighing floor(p_ji 2^32) units, p_ji = d / #out_i with d = 0.85
 *     (only the ratios matter: the weights rank positions, they move no fluid);
 *   - boundary k moves within [t_k - w_k, t_k + w_k], w_k = min(ceil(N/K)/2,
 *     half of each neighbouring target gap less one), so the windows are
 *     disjoint and the CB targets stay feasible;
 *   - no boundary falls inside a short tight cycle when a plan exists
 *     without that: a directed cycle of two or three distinct nodes whose
 *     out-degrees multiply to at most 2 (it hands back at least 0.85^len / 2
 *     of its fluid per round, so split across two sets its fluid would cross
 *     back and forth one level per hop), spanning fewer than 2 ceil(N/K) ids;
 *     a boundary b lies inside the cycle when min < b <= max of its ids;
 *   - the plan minimizes the sum of cross(b_k) over the inner boundaries;
 *     among plans of equal sum, b_{K-1} is the smallest possible, then
 *     b_{K-2}, and so on (a dynamic programme over the windows whose
 *     back-pointers take the smallest of equal predecessors).
 * ptr has K+1 entries. */
int dref_partition_mincut(int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx,
                          int64_t K, int64_t* ptr) {
  if (K < 1 || K > (n > 0 ? n : 1)) return DREF_EINVAL;
  int64_t* C = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t* indeg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t* cross = (int64_t*)calloc((size_t)n + 2, sizeof(int64_t));
  int64_t* t = (int64_t*)calloc((size_t)K + 1, sizeof(int64_t));
  int64_t* lo = (int64_t*)calloc((size_t)K + 1, sizeof(int64_t));
  int64_t* hi = (int64_t*)calloc((size_t)K + 1, sizeof(int64_t));
  int64_t* off = (int64_t*)calloc((size_t)K + 2, sizeof(int64_t));
  if (!C || !indeg || !cross || !t || !lo || !hi || !off) {
    free(C), free(indeg), free(cross), free(t), free(lo), free(hi), free(off);
    return DREF_ENOMEM;
  }
  /* node costs and their prefix */
  const int64_t h = nnz * 3 / (n > 0 ? n : 1) > 1 ? nnz * 3 / n : 1;
  for (int64_t e = 0; e < nnz; ++e) indeg[row_idx[e]] += 1;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t out = col_ptr[i + 1] - col_ptr[i];
    C[i + 1] = C[i] + 1 + out + (indeg[i] < h ? indeg[i] : h);
  }
  /* CB targets */
  int64_t j = 0;
  t[0] = 0;
  for (int64_t k = 1; k < K; ++k) {
    while (j < n && C[j] * K < k * C[n]) ++j;
    t[k] = j;
  }
  t[K] = n;
  /* balance limits */
  int64_t cstar = 0, sstar = 0;
  for (int64_t k = 0; k < K; ++k) {
    if (C[t[k + 1]] - C[t[k]] > cstar) cstar = C[t[k + 1]] - C[t[k]];
    if (t[k + 1] - t[k] > sstar) sstar = t[k + 1] - t[k];
  }
  const int64_t cmax = cstar + cstar / 10, smax = sstar + sstar / 10;
  /* p mass of the short links crossing each position: cross[b] for b = 0..n */
  const int64_t mean = (n + K - 1) / K, span = 2 * mean;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) {
      const int64_t r = row_idx[e];
      const int64_t a = r < i ? r : i, z = r < i ? i : r;
      if (a == z || z - a >= span) continue;
      const int64_t u = link_units(NULL, 0.85, col_ptr, i, e);
      cross[a + 1] += u; /* the link crosses b = a+1 .. z: a difference array */
      cross[z + 1] -= u;
    }
  for (int64_t b = 1; b <= n; ++b) cross[b] += cross[b - 1];
  /* positions inside a short tight cycle: a directed cycle of two or three
     distinct nodes whose out-degrees multiply to at most 2, so that it hands
     back at least 0.85^len / 2 of its fluid per round */
  int64_t* tight = (int64_t*)calloc((size_t)n + 2, sizeof(int64_t));
  if (!tight) {
    free(C), free(indeg), free(cross), free(t), free(lo), free(hi), free(off);
    return DREF_ENOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    const int64_t oi = col_ptr[i + 1] - col_ptr[i];
    if (oi < 1 || oi > 2) continue;
    for (int64_t e1 = col_ptr[i]; e1 < col_ptr[i + 1]; ++e1) {
      const int64_t j = row_idx[e1], oj = col_ptr[j + 1] - col_ptr[j];
      if (j <= i || oi * oj > 2) continue;
      for (int64_t e2 = col_ptr[j]; e2 < col_ptr[j + 1]; ++e2) {
        const int64_t k = row_idx[e2];
        if (k == i) { /* i -> j -> i */
          if (j - i < span) tight[i + 1] += 1, tight[j + 1] -= 1;
          continue;
        }
        const int64_t ok = col_ptr[k + 1] - col_ptr[k];
        if (k <= i || k == j || oi * oj * ok > 2) continue;
        for (int64_t e3 = col_ptr[k]; e3 < col_ptr[k + 1]; ++e3)
          if (row_idx[e3] == i) { /* i -> j -> k -> i */
            const int64_t z = j > k ? j : k;
            if (z - i < span) tight[i + 1] += 1, tight[z + 1] -= 1;
          }
      }
    }
  }
  for (int64_t b = 1; b <= n; ++b) tight[b] += tight[b - 1];
  /* windows */
  const int64_t W = mean / 2;
  for (int64_t k = 1; k < K; ++k) {
    int64_t w = W;
    const int64_t gl = (t[k] - t[k - 1] - 1) / 2, gr = (t[k + 1] - t[k] - 1) / 2;
    if (gl < w) w = gl;
    if (gr < w) w = gr;
    if (w < 0) w = 0;
    lo[k] = t[k] - w;
    hi[k] = t[k] + w;
  }
  lo[0] = hi[0] = 0;
  lo[K] = hi[K] = n;
  for (int64_t k = 0; k <= K; ++k) off[k + 1] = off[k] + (hi[k] - lo[k] + 1);
  int64_t* V = (int64_t*)malloc(sizeof(int64_t) * (size_t)off[K + 1]);
  int64_t* P = (int64_t*)malloc(sizeof(int64_t) * (size_t)off[K + 1]);
  if (!V || !P) {
    free(V), free(P), free(C), free(indeg), free(cross), free(t), free(lo), free(hi), free(off), free(tight);
    return DREF_ENOMEM;
  }
  const int64_t INF = INT64_MAX / 4;
  /* V[k][b]: least sum of cross over boundaries 1..k with b_k = b; the first
     pass admits no boundary inside a tight cycle, the second (only when the
     first finds no plan) admits every position */
  for (int pass = 0; pass < 2; ++pass) {
    V[0] = 0;
    P[0] = -1;
    for (int64_t k = 1; k <= K; ++k) {
      for (int64_t b = lo[k]; b <= hi[k]; ++b) {
        int64_t best = INF, arg = -1;
        for (int64_t q = lo[k - 1]; q <= hi[k - 1]; ++q) {
          const int64_t v = V[off[k - 1] + q - lo[k - 1]];
          if (v >= INF || b - q > smax || C[b] - C[q] > cmax) continue;
          if (v < best) best = v, arg = q; /* strict: the smallest q among equals */
        }
        if (pass == 0 && k < K && tight[b] > 0) best = INF;
        V[off[k] + b - lo[k]] = best >= INF ? INF : best + (k < K ? cross[b] : 0);
        P[off[k] + b - lo[k]] = arg;
      }
    }
    if (V[off[K]] < INF) break;
  }
  /* back from b_K = n (the CB targets are feasible, so V[K][n] is finite) */
  ptr[K] = n;
  for (int64_t k = K; k >= 1; --k) ptr[k - 1] = P[off[k] + ptr[k] - lo[k]];
  free(V), free(P), free(C), free(indeg), free(cross), free(t), free(lo), free(hi), free(off), free(tight);
  return ptr[0] == 0 ? DREF_OK : DREF_EINVAL;
}
