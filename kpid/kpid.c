/*
 * kpid — time-stepped simulation of the K-PID asynchronous D-iteration on
 * one CPU (Hong, arXiv:1202.6168, Sections 2.3-2.6 and 3): the model the
 * paper's own evaluation runs, rebuilt for synthetic graphs. CPU only; its
 * figures are operation counts, not times.
 *
 * Model (Section 2.4, PID modelling): K PIDs own contiguous node ranges
 * Omega_k = [omega_k, omega_{k+1}). Time advances in steps; in each step every
 * PID may spend PID_Speed_k = speed elementary operations, one per diffusion
 * from a node to one child (a dangling node's diffusion costs nothing).
 * Inside a step a PID
 *   1. takes the fluid of the messages that have arrived (Section 2.6): adds
 *      it node by node and raises its threshold T_k by the factor
 *      (r_k + m) / r_k, capped so that T_k never exceeds the largest |F_i| of
 *      Omega_k (m = received L1 mass; if r_k = 0, T_k = that largest |F_i|);
 *   2. if r_k = sum_{i in Omega_k} |F_i| is below its share of the target,
 *      sleeps (the rest of the step is idle time, Section 3.3);
 *   3. otherwise runs the local algorithm (*) of Section 2.5: a cyclic scan of
 *      Omega_k diffusing every node with |F_i| > T_k, children inside Omega_k
 *      served at once, T_k /= alpha after each full scan (Section 2.4);
 *   4. whenever the fluid owed to outside nodes, s_k = sum over outside links
 *      of |p_ji (H_i - Hold_i)|, exceeds r_k / K (equation send, Section 2.5),
 *      sends P (H - Hold) restricted to each other PID's nodes and sets
 *      Hold = H. A message is delivered at each later step with probability
 *      1 - delay_proba (Section 3.3: mean delay delay_proba / (1 - delay_proba)
 *      steps of speed operations).
 * The run stops once every PID sleeps, no message is in flight and
 * ||F||_1 / (1 - d) <= target_error (the paper's error bound), or at max_steps.
 * Cost: normalized iterations = steps * speed / L (the slowest PID sets the
 * time: every PID's clock advances together), elementary operations, idle
 * proportion idle / (elementary + idle) (Section 3.3).
 *
 * Partition adaptation (Section 3.4, K = 2): every adapt_every steps, if one
 * PID's residual is more than twice the other's and its operation count more
 * than 1.2 times the other's, omega_1 moves by 10% towards it, handing over
 * the moved nodes' F, H and Hold (the other PID owes nothing for them).
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t steps;          /* time steps simulated */
  int64_t ops;            /* elementary operations, all PIDs */
  int64_t idle;           /* idle operation slots, all PIDs */
  int64_t messages;       /* messages sent */
  int64_t adaptations;    /* boundary moves (K = 2 adaptation) */
  double norm_iters;      /* steps * speed / L */
  double idle_frac;       /* idle / (ops + idle) */
  double resid_l1;        /* final ||F||_1 including fluid in flight */
  int32_t converged;
  int32_t pad;
} kpid_stats;

typedef struct {
  double* F;      /* [n] fluid of every node (each PID touches only its own) */
  double* H;      /* [n] history */
  double* Hold;   /* [n] history at the last send */
  double* T;      /* [K] thresholds */
  int64_t* cur;   /* [K] scan cursor inside Omega_k */
  int64_t* kops;  /* [K] operations done */
  int32_t* scanned_any; /* [K] a node passed since the cursor last wrapped */
  double* pend;   /* [n] fluid sent to node j, waiting for delivery to its owner */
  double* pend_mass; /* [K] */
  int32_t* has_pend; /* [K] */
} state;

static uint64_t sm64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double unif(uint64_t* s) { return (double)(sm64(s) >> 11) * (1.0 / 9007199254740992.0); }

static int owner(const int64_t* omega, int K, int64_t j) {
  int lo = 0, hi = K - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (omega[mid] <= j) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static double range_l1(const double* x, int64_t a, int64_t b) {
  double s = 0;
  for (int64_t i = a; i < b; ++i) s += fabs(x[i]);
  return s;
}
static double range_max(const double* x, int64_t a, int64_t b) {
  double m = 0;
  for (int64_t i = a; i < b; ++i)
    if (fabs(x[i]) > m) m = fabs(x[i]);
  return m;
}

/* fluid owed by PID k to outside nodes: sum over links i -> j leaving Omega_k of
 * |p_ji (H_i - Hold_i)| */
static double owed(const int32_t* cp, const int32_t* ri, double d, const int64_t* omega, int k,
                   const state* S) {
  double s = 0;
  for (int64_t i = omega[k]; i < omega[k + 1]; ++i) {
    const double dh = S->H[i] - S->Hold[i];
    const int64_t deg = cp[i + 1] - cp[i];
    if (dh == 0 || deg == 0) continue;
    int64_t out = 0;
    for (int64_t e = cp[i]; e < cp[i + 1]; ++e) out += ri[e] < omega[k] || ri[e] >= omega[k + 1];
    s += fabs(dh) * d / (double)deg * (double)out;
  }
  return s;
}

static void send(const int32_t* cp, const int32_t* ri, double d, const int64_t* omega, int K, int k,
                 state* S, kpid_stats* st) {
  for (int64_t i = omega[k]; i < omega[k + 1]; ++i) {
    const double dh = S->H[i] - S->Hold[i];
    const int64_t deg = cp[i + 1] - cp[i];
    S->Hold[i] = S->H[i];
    if (dh == 0 || deg == 0) continue;
    const double w = dh * d / (double)deg;
    for (int64_t e = cp[i]; e < cp[i + 1]; ++e) {
      const int64_t j = ri[e];
      if (j >= omega[k] && j < omega[k + 1]) continue;
      const int q = owner(omega, K, j);
      S->pend[j] += w;
      S->pend_mass[q] += fabs(w);
      S->has_pend[q] = 1;
    }
  }
  st->messages += 1;
}

static void deliver(const int64_t* omega, int q, state* S) {
  double m = 0;
  const double r = range_l1(S->F, omega[q], omega[q + 1]);
  for (int64_t j = omega[q]; j < omega[q + 1]; ++j) {
    const double x = S->pend[j];
    if (x == 0) continue;
    S->F[j] += x;
    m += fabs(x);
    S->pend[j] = 0;
  }
  S->pend_mass[q] = 0;
  S->has_pend[q] = 0;
  /* reception rescale of the threshold (Section 2.6) */
  const double fmax = range_max(S->F, omega[q], omega[q + 1]);
  if (r > 0) S->T[q] = fmin(S->T[q] * (r + m) / r, fmax);
  else S->T[q] = fmax;
}

/*
 * omega   [K+1] initial boundaries (updated in place by the adaptation)
 * speed   operations per PID per step (the paper's default L / K)
 * r_trace optional [trace_cap * K * 2]: per step and PID, r_k then s_k
 * h_out, f_out [n]: history and fluid (pending fluid added into f_out)
 */
int kpid_simulate(int64_t n, const int32_t* cp, const int32_t* ri, double d, const double* b, int K,
                  int64_t* omega, int64_t speed, double alpha, double target_error, double delay_proba,
                  int adapt_every, uint64_t seed, int64_t max_steps, double* h_out, double* f_out,
                  kpid_stats* st, double* r_trace, int64_t trace_cap) {
  memset(st, 0, sizeof(*st));
  if (K < 1 || n < 1 || speed < 1 || !(alpha > 1) || !(d > 0 && d < 1) || !(delay_proba >= 0 && delay_proba < 1))
    return -1;
  if (omega[0] != 0 || omega[K] != n) return -1;
  for (int k = 0; k < K; ++k)
    if (omega[k + 1] < omega[k]) return -1;
  state S;
  S.F = f_out;
  S.H = h_out;
  S.Hold = calloc((size_t)n, sizeof(double));
  S.T = calloc((size_t)K, sizeof(double));
  S.cur = calloc((size_t)K, sizeof(int64_t));
  S.kops = calloc((size_t)K, sizeof(int64_t));
  S.scanned_any = calloc((size_t)K, sizeof(int32_t));
  S.pend = calloc((size_t)n, sizeof(double));
  S.pend_mass = calloc((size_t)K, sizeof(double));
  S.has_pend = calloc((size_t)K, sizeof(int32_t));
  if (!S.Hold || !S.T || !S.cur || !S.kops || !S.scanned_any || !S.pend || !S.pend_mass || !S.has_pend) {
    free(S.Hold), free(S.T), free(S.cur), free(S.kops), free(S.scanned_any), free(S.pend), free(S.pend_mass),
        free(S.has_pend);
    return -3;
  }
  memcpy(S.F, b, sizeof(double) * n);
  memset(S.H, 0, sizeof(double) * n);
  const int64_t L = cp[n];
  const double fluid_target = target_error * (1 - d); /* ||F||_1 / (1 - d) <= target_error */
  for (int k = 0; k < K; ++k) {
    S.T[k] = range_max(S.F, omega[k], omega[k + 1]) / alpha;
    S.cur[k] = omega[k];
  }
  uint64_t rng = seed;
  int64_t step = 0;
  int conv = 0;
  while (step < max_steps) {
    /* message delivery: each pending batch arrives with probability 1 - delay_proba */
    for (int q = 0; q < K; ++q)
      if (S.has_pend[q] && unif(&rng) >= delay_proba) deliver(omega, q, &S);
    int all_asleep = 1;
    for (int k = 0; k < K; ++k) {
      const int64_t a = omega[k], e = omega[k + 1];
      int64_t budget = speed;
      double r = range_l1(S.F, a, e);
      const double share = fluid_target / (double)K;
      if (r <= share || a == e) { /* asleep: the whole step is idle */
        st->idle += budget;
        if (trace_cap > step && r_trace) {
          r_trace[((size_t)step * K + k) * 2] = r;
          r_trace[((size_t)step * K + k) * 2 + 1] = owed(cp, ri, d, omega, k, &S);
        }
        continue;
      }
      all_asleep = 0;
      int64_t scans_empty = 0;
      while (budget > 0) {
        const int64_t i = S.cur[k];
        if (fabs(S.F[i]) > S.T[k]) {
          const double sent = S.F[i];
          const int64_t deg = cp[i + 1] - cp[i];
          S.H[i] += sent;
          S.F[i] = 0;
          if (deg > 0) {
            const double w = sent * d / (double)deg;
            for (int64_t q = cp[i]; q < cp[i + 1]; ++q)
              if (ri[q] >= a && ri[q] < e) S.F[ri[q]] += w;
          }
          budget -= deg;
          S.kops[k] += deg;
          st->ops += deg;
          S.scanned_any[k] = 1;
        }
        if (++S.cur[k] == e) { /* a full cyclic scan: lower the threshold */
          S.cur[k] = a;
          S.T[k] /= alpha;
          if (!S.scanned_any[k]) {
            const double m = range_max(S.F, a, e) / alpha;
            if (m < S.T[k]) S.T[k] = m;
            if (++scans_empty > 1) break; /* nothing left locally this step */
          }
          S.scanned_any[k] = 0;
          r = range_l1(S.F, a, e);
          const double s = owed(cp, ri, d, omega, k, &S);
          if (s > r / (double)K) send(cp, ri, d, omega, K, k, &S, st); /* equation send */
          if (r <= share) break;
        }
      }
      if (budget > 0) st->idle += budget;
      r = range_l1(S.F, a, e);
      const double s = owed(cp, ri, d, omega, k, &S);
      if (s > r / (double)K || (r <= share && s > 0)) send(cp, ri, d, omega, K, k, &S, st);
      if (trace_cap > step && r_trace) {
        r_trace[((size_t)step * K + k) * 2] = r;
        r_trace[((size_t)step * K + k) * 2 + 1] = owed(cp, ri, d, omega, k, &S);
      }
    }
    ++step;
    /* adaptation of omega_1 for two PIDs (Section 3.4) */
    if (K == 2 && adapt_every > 0 && step % adapt_every == 0) {
      const double r0 = range_l1(S.F, omega[0], omega[1]), r1 = range_l1(S.F, omega[1], omega[2]);
      const double o0 = (double)S.kops[0] + 1, o1 = (double)S.kops[1] + 1;
      int64_t w = omega[1], nw = w;
      if (r0 > 2 * r1 && o0 > 1.2 * o1) nw = w - (int64_t)(0.1 * (double)w);
      else if (r1 > 2 * r0 && o1 > 1.2 * o0) nw = w + (int64_t)(0.1 * (double)w);
      if (nw < 1) nw = 1;
      if (nw > n - 1) nw = n - 1;
      if (nw != w && n > 1) {
        /* settle what each side owes before the boundary moves */
        send(cp, ri, d, omega, K, 0, &S, st);
        send(cp, ri, d, omega, K, 1, &S, st);
        for (int q = 0; q < 2; ++q)
          if (S.has_pend[q]) deliver(omega, q, &S);
        omega[1] = nw;
        for (int k = 0; k < 2; ++k) {
          S.cur[k] = omega[k];
          S.T[k] = range_max(S.F, omega[k], omega[k + 1]) / alpha;
        }
        st->adaptations += 1;
      }
    }
    if (all_asleep) {
      int pending = 0;
      for (int q = 0; q < K; ++q) pending |= S.has_pend[q];
      if (!pending && range_l1(S.F, 0, n) <= fluid_target) {
        conv = 1;
        break;
      }
    }
  }
  /* fluid still in flight belongs to F */
  for (int64_t j = 0; j < n; ++j) S.F[j] += S.pend[j];
  st->steps = step;
  st->norm_iters = L > 0 ? (double)step * (double)speed / (double)L : 0;
  st->idle_frac = st->ops + st->idle > 0 ? (double)st->idle / (double)(st->ops + st->idle) : 0;
  st->resid_l1 = range_l1(S.F, 0, n);
  st->converged = conv;
  free(S.Hold), free(S.T), free(S.cur), free(S.kops), free(S.scanned_any), free(S.pend), free(S.pend_mass),
      free(S.has_pend);
  return conv ? 0 : 1;
}
