// Partition adaptation (Section 3.4): the paper moves the boundary between
// two PIDs towards the one that does more work for less progress. Here every
// boundary of the partition plan moves, from a measured cost per partition:
// each partition's own work per threshold level, averaged over the levels of
// a traced solve. The nodes of a partition share its cost evenly, and the
// boundaries move a fraction omega of the way to the points that split the
// total cost into K equal parts. A new plan is kept only when the solve gets
// faster; otherwise the previous plan comes back and the adaptation stops.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "common.h"

namespace {

double wall_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Run {
  ditr_ctx* c;
  ditr_graph* g;
  const double* b;
  double* h;
  float* f;
  double tol;
  ditr_opts o;
};

// best wall time to tolerance of `reps` solves
int best_time(const Run& r, int reps, double* secs) {
  *secs = INFINITY;
  for (int i = 0; i < reps; ++i) {
    ditr_stats st;
    const double t0 = wall_now();
    const int rc = ditr_solve(r.c, r.g, r.b, r.h, r.f, 0, r.tol, &r.o, &st);
    const double dt = wall_now() - t0;
    if (rc != DITR_OK) return rc < 0 ? rc : set_error(DITR_NOT_CONVERGED, "a solve did not converge");
    *secs = std::min(*secs, dt);
  }
  return DITR_OK;
}

// one traced solve: each partition's mean work per level (seconds), and the
// slowest one's over the mean
int measure_costs(const Run& r, std::vector<double>& cost, double* spread) {
  const int64_t K = r.g->K;
  const int64_t levels_cap = std::max<int64_t>(8, std::min<int64_t>(4096, ((int64_t)1 << 27) / (K * DITR_TRACE_FIELDS)));
  const int64_t cap = levels_cap * K;
  double* d_trace = nullptr;
  HIP_TRY(hipMalloc((void**)&d_trace, sizeof(double) * DITR_TRACE_FIELDS * cap));
  double* const prev = r.c->trace;
  const int64_t prev_cap = r.c->trace_cap;
  r.c->trace = d_trace;
  r.c->trace_cap = cap;
  ditr_stats st;
  int rc = ditr_solve(r.c, r.g, r.b, r.h, r.f, 0, r.tol, &r.o, &st);
  r.c->trace = prev;
  r.c->trace_cap = prev_cap;
  std::vector<double> rec;
  const int64_t L = std::min<int64_t>(st.sweeps, levels_cap);
  if (rc == DITR_OK && L > 0) {
    rec.resize((size_t)(L * K * DITR_TRACE_FIELDS));
    const hipError_t e = hipMemcpy(rec.data(), d_trace, sizeof(double) * rec.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = set_error(DITR_EHIP, "hipMemcpy failed: %s", hipGetErrorString(e));
  }
  (void)hipFree(d_trace);
  if (rc != DITR_OK) return rc < 0 ? rc : set_error(DITR_NOT_CONVERGED, "the traced solve did not converge");
  if (L < 1) return set_error(DITR_EINVAL, "the traced solve ran no level");
  // the first level has no wait and the last one only finishes the stage
  const int64_t l0 = L > 2 ? 1 : 0, l1 = L > 2 ? L - 1 : L;
  cost.assign((size_t)K, 0.0);
  for (int64_t l = l0; l < l1; ++l)
    for (int64_t k = 0; k < K; ++k) cost[k] += rec[(size_t)((l * K + k) * DITR_TRACE_FIELDS + 5)];
  double mean = 0, mx = 0;
  for (int64_t k = 0; k < K; ++k) {
    cost[k] /= (double)(l1 - l0);
    mean += cost[k];
    mx = std::max(mx, cost[k]);
  }
  mean /= (double)K;
  *spread = mean > 0 ? mx / mean : 1.0;
  return DITR_OK;
}

// boundaries moved omega of the way to equal cost (nodes share their
// partition's cost evenly), each part at least one node and at most cap;
// false if no such plan exists
bool equal_cost_plan(const int64_t* ptr, int64_t K, int64_t n, const std::vector<double>& cost, double omega,
                     int64_t cap, std::vector<int64_t>& out) {
  double total = 0;
  for (double x : cost) total += x;
  out.assign((size_t)K + 1, 0);
  out[K] = n;
  if (!(total > 0)) {
    std::copy(ptr, ptr + K + 1, out.begin());
    return true;
  }
  int64_t k = 0;
  double before = 0;  // cost of the partitions left of k
  for (int64_t j = 1; j < K; ++j) {
    const double t = total * (double)j / (double)K;
    while (k < K - 1 && before + cost[k] <= t) before += cost[k++];
    const double np = (double)(ptr[k + 1] - ptr[k]);
    const double frac = cost[k] > 0 ? std::min(1.0, std::max(0.0, (t - before) / cost[k])) : 0.0;
    const double x = (double)ptr[k] + frac * np;
    out[j] = (int64_t)std::llround((double)ptr[j] + omega * (x - (double)ptr[j]));
  }
  // each part at least one node and at most cap nodes (two passes each way;
  // the plan on entry satisfies both, so a plan between it and the target can)
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t j = 1; j < K; ++j) out[j] = std::min(std::max(out[j], out[j - 1] + 1), out[j - 1] + cap);
    for (int64_t j = K - 1; j >= 1; --j) out[j] = std::max(std::min(out[j], out[j + 1] - 1), out[j + 1] - cap);
  }
  for (int64_t j = 1; j <= K; ++j)
    if (out[j] - out[j - 1] < 1 || out[j] - out[j - 1] > cap) return false;
  return true;
}

}  // namespace

extern "C" {

int ditr_graph_set_partitions(ditr_ctx* c, ditr_graph* g, const int64_t* h_ptr, int64_t K) {
  return graph_set_plan(c, g, h_ptr, K);
}

int ditr_graph_adapt(ditr_ctx* c, ditr_graph* g, const double* d_b, double* d_h, float* d_f, double rel_tol,
                     int rounds, double omega, ditr_adapt_info* info) {
  const double t_start = wall_now();
  if (!c || !g || !d_b || !d_h || !d_f) return set_error(DITR_EINVAL, "NULL argument");
  if (g->val) return set_error(DITR_EINVAL, "a general matrix is solved by the pull sweep, which has no partitions");
  if (g->arena.base)
    return set_error(DITR_EINVAL, "a graph in a caller workspace keeps the plan it was uploaded with");
  if (rounds < 0 || rounds > 64) return set_error(DITR_EINVAL, "rounds must lie in [0, 64]");
  if (!(omega > 0 && omega <= 1)) return set_error(DITR_EINVAL, "omega must lie in (0, 1]");
  if (!(rel_tol > 0) || !std::isfinite(rel_tol)) return set_error(DITR_EINVAL, "rel_tol must be > 0");
  ditr_adapt_info inf;
  memset(&inf, 0, sizeof(inf));
  Run r{c, g, d_b, d_h, d_f, rel_tol, {}};
  ditr_opts_default(&r.o);
  r.o.mode = DITR_MODE_PARTITION;
  r.o.flags = 0;
  const int reps = 3;
  {
    ditr_stats st;  // warm-up
    const int rc = ditr_solve(c, g, d_b, d_h, d_f, 0, rel_tol, &r.o, &st);
    if (rc != DITR_OK) return rc < 0 ? rc : set_error(DITR_NOT_CONVERGED, "the solve does not converge");
  }
  double t_best;
  int rc = best_time(r, reps, &t_best);
  if (rc) return rc;
  inf.seconds_before = t_best;
  std::vector<double> cost;
  double spread = 1;
  rc = measure_costs(r, cost, &spread);
  if (rc) return rc;
  inf.spread_before = spread;
  const int64_t K = g->K, n = g->n;
  std::vector<int64_t> keep(g->part_ptr_host, g->part_ptr_host + K + 1), next;
  for (int it = 0; it < rounds; ++it) {
    inf.rounds += 1;
    if (!equal_cost_plan(keep.data(), K, n, cost, omega, g->cap_nodes, next) || next == keep) break;
    rc = graph_set_plan(c, g, next.data(), K);
    double t = INFINITY;
    if (!rc) rc = best_time(r, reps, &t);
    if (rc < 0 && rc != DITR_EINVAL) return rc;
    if (rc == DITR_OK && t < 0.995 * t_best) {  // kept: at least half a percent faster
      inf.kept += 1;
      t_best = t;
      keep = next;
      rc = measure_costs(r, cost, &spread);
      if (rc) return rc;
      continue;
    }
    rc = graph_set_plan(c, g, keep.data(), K);  // back to the previous plan
    if (rc) return rc;
    break;
  }
  inf.seconds_after = t_best;
  rc = measure_costs(r, cost, &spread);
  if (rc) return rc;
  inf.spread_after = spread;
  inf.seconds = wall_now() - t_start;
  if (info) *info = inf;
  return DITR_OK;
}

}  // extern "C"
