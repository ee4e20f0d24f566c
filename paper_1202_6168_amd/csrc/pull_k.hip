// Grid-synchronous threshold sweep in pull form (no atomics on the fluid).
//
// Sweep k diffuses, all at once, every node whose fluid exceeds T (the cyclic
// threshold test of Section 2.4 applied to a whole set, F <- (I - J + P J) F
// with J the selector of that set, which keeps F = B + P H - H exactly). A
// node's share for its children, sent * p_ji = sent * d / #out_i, is stored in
// S_k; sweep k+1 adds to F_j the sum of S_k over the in-links of j (read over
// the CSR transpose) before testing j. The fluid in S between two sweeps is in
// flight, as the delayed exchange of Section 3.3 allows.
//
// Rows with more than kHeavyRow in-links are summed by chunk workgroups
// (kHeavyChunk in-links each) that add their partial sum into a per-row FP64
// accumulator; the row takes that inflow one sweep later.
#include <algorithm>
#include <vector>

#include "common.h"

namespace {

constexpr int kPullBlock = 256;
constexpr int kStride = 4;                     // doubles per block in ctx->partials

struct PullArgs {
  int64_t n;
  const int32_t* __restrict__ row_ptr;
  const int32_t* __restrict__ csr_col;
  const int32_t* __restrict__ col_ptr;
  const int32_t* __restrict__ heavy_rows;
  const int32_t* __restrict__ chunk_h;
  const int32_t* __restrict__ chunk_beg;
  const int32_t* __restrict__ chunk_end;
  const double* __restrict__ csr_val;  // general matrix: weight of each CSR entry (else nullptr)
  const double* __restrict__ colabs;   // general matrix: sum |p_ji| of each column
  float* F;
  double* H;
  float* S;          // [2][n] PageRank: sent * d / #out_i; general matrix: sent
  double* heavy_in;  // [2][n_heavy]
  double* partials;
  Ctrl* ctrl;
  int n_heavy;
  int n_light_blocks;
  float d;
};

__device__ __forceinline__ int find_heavy(const int32_t* rows, int nh, int j) {
  int lo = 0, hi = nh - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (rows[mid] < j) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// W: general matrix (an in-link's share is its weight times the source's sent
// fluid) instead of the PageRank shares published per source
template <bool W>
__global__ void __launch_bounds__(kPullBlock) k_pull_sweep(PullArgs a, int parity) {
  if (__hip_atomic_load(&a.ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const float* S_in = a.S + (size_t)(parity ^ 1) * a.n;  // written by the previous sweep
  float* S_out = a.S + (size_t)parity * a.n;
  double* hin_prev = a.heavy_in + (size_t)(parity ^ 1) * a.n_heavy;
  double* hin_cur = a.heavy_in + (size_t)parity * a.n_heavy;
  const int tid = threadIdx.x;

  if ((int)blockIdx.x >= a.n_light_blocks) {
    // ---- one chunk of the in-links of a heavy row
    const int c = blockIdx.x - a.n_light_blocks;
    double acc = 0;
    for (int e = a.chunk_beg[c] + tid; e < a.chunk_end[c]; e += kPullBlock)
      acc += W ? a.csr_val[e] * (double)S_in[a.csr_col[e]] : (double)S_in[a.csr_col[e]];
    acc = wave_sum(acc);
    __shared__ double red[kPullBlock / 64];
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      acc = red[0] + red[1] + red[2] + red[3];
      if (acc != 0.0) add_agent(&hin_cur[a.chunk_h[c]], acc);
      double* p = a.partials + (size_t)kStride * blockIdx.x;  // fluid in transit to the row
      p[0] = fabs(acc);
      p[1] = 0.0;
      p[2] = 0.0;
      p[3] = 0.0;
    }
    return;
  }

  const float T = (float)a.ctrl->T;
  const float d = a.d;
  // resid: |F_j| after the sweep plus the in-flight share d |sent| of every
  // diffused node with out-links (an upper bound of its l1 mass once delivered)
  double resid = 0, fmx = 0, edges = 0, diffs = 0;
  const int64_t stride = (int64_t)a.n_light_blocks * kPullBlock;
  for (int64_t j = (int64_t)blockIdx.x * kPullBlock + tid; j < a.n; j += stride) {
    const int32_t r0 = a.row_ptr[j], r1 = a.row_ptr[j + 1];
    const float fj = a.F[j];
    double acc = 0;
    if (r1 - r0 > kHeavyRow) {
      const int h = find_heavy(a.heavy_rows, a.n_heavy, (int)j);
      acc = hin_prev[h];
      hin_prev[h] = 0.0;  // becomes the accumulator of the next sweep
    } else {
      int32_t e = r0;
      if (W) {
        for (; e + 4 <= r1; e += 4) {  // four index and weight loads, then four gathers
          const int32_t c0 = a.csr_col[e], c1 = a.csr_col[e + 1], c2 = a.csr_col[e + 2],
                        c3 = a.csr_col[e + 3];
          const double w0 = a.csr_val[e], w1 = a.csr_val[e + 1], w2 = a.csr_val[e + 2],
                       w3 = a.csr_val[e + 3];
          acc += w0 * (double)S_in[c0] + w1 * (double)S_in[c1] + w2 * (double)S_in[c2] +
                 w3 * (double)S_in[c3];
        }
        for (; e < r1; ++e) acc += a.csr_val[e] * (double)S_in[a.csr_col[e]];
      } else {
        for (; e + 4 <= r1; e += 4) {  // four index loads, then four gathers
          const int32_t c0 = a.csr_col[e], c1 = a.csr_col[e + 1], c2 = a.csr_col[e + 2],
                        c3 = a.csr_col[e + 3];
          acc += (double)S_in[c0] + (double)S_in[c1] + (double)S_in[c2] + (double)S_in[c3];
        }
        for (; e < r1; ++e) acc += S_in[a.csr_col[e]];
      }
    }
    float f = (float)((double)fj + acc);
    float s_out = 0.f;
    if (fabsf(f) > T) {
      const int deg = a.col_ptr[j + 1] - a.col_ptr[j];
      a.H[j] += (double)f;
      if (W) {
        s_out = deg > 0 ? f : 0.f;
        resid += a.colabs[j] * fabs((double)f);  // l1 mass of the shares in flight
      } else {
        s_out = deg > 0 ? f * (d / (float)deg) : 0.f;
        if (deg > 0) resid += (double)d * fabs((double)f);
      }
      edges += deg;
      diffs += 1;
      f = 0.f;
    }
    a.F[j] = f;
    S_out[j] = s_out;
    resid += fabs((double)f);
    fmx = fmx > fabs((double)f) ? fmx : fabs((double)f);
  }
  // block partials (fixed order: deterministic)
  resid = wave_sum(resid);
  edges = wave_sum(edges);
  diffs = wave_sum(diffs);
  fmx = wave_maxd(fmx);
  __shared__ double red[4][kPullBlock / 64];
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0) {
    red[0][wave] = resid;
    red[1][wave] = fmx;
    red[2][wave] = edges;
    red[3][wave] = diffs;
  }
  __syncthreads();
  if (tid == 0) {
    double* p = a.partials + (size_t)kStride * blockIdx.x;
    p[0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    p[1] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    p[2] = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    p[3] = red[3][0] + red[3][1] + red[3][2] + red[3][3];
  }
}

// after a sweep: stop once the fluid (held plus in flight) is below target,
// else T <- T / alpha (or max |F| / alpha if the sweep diffused nothing)
__global__ void __launch_bounds__(256) k_pull_step(const double* partials, int nb, Ctrl* ctrl,
                                                   double alpha) {
  if (ctrl->done) return;
  double D = 0, M = 0, E = 0, P = 0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    const double* p = partials + (size_t)kStride * i;
    D += p[0];
    M = fmax(M, p[1]);
    E += p[2];
    P += p[3];
  }
  D = wave_sum(D);
  E = wave_sum(E);
  P = wave_sum(P);
  M = wave_maxd(M);
  __shared__ double red[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = D;
    red[1][wave] = M;
    red[2][wave] = E;
    red[3][wave] = P;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    D = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    M = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    E = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    P = red[3][0] + red[3][1] + red[3][2] + red[3][3];
    ctrl->sum_abs = D;
    ctrl->edges += (unsigned long long)E;
    ctrl->diffusions += (unsigned long long)P;
    ctrl->sweeps += 1;
    if (D <= ctrl->target) {
      ctrl->done = 1;
    } else {
      double T = ctrl->T / alpha;
      if (P == 0 && M / alpha < T) T = M / alpha;
      ctrl->T = T;
    }
  }
}

__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.f;
}
__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

__global__ void k_gather_heavy_ranges(int32_t nh, const int32_t* __restrict__ rows,
                                      const int32_t* __restrict__ row_ptr, int32_t* out) {
  for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += gridDim.x * blockDim.x) {
    out[2 * h] = row_ptr[rows[h]];
    out[2 * h + 1] = row_ptr[rows[h] + 1];
  }
}

int light_blocks(const ditr_ctx* c, int64_t n) {
  int64_t g = (n + kPullBlock - 1) / kPullBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, (int64_t)c->num_cus * 8));
}

}  // namespace

// Sort the heavy-row list and cut each heavy row's in-links into chunks.
int build_heavy_chunks(ditr_ctx* c, ditr_graph* g) {
  const int nh = g->n_heavy;
  std::vector<int32_t> rows(nh), ranges(2 * (size_t)nh);
  int32_t* d_ranges = nullptr;
  if (nh > 0) {
    HIP_TRY(hipMemcpyAsync(rows.data(), g->heavy_rows, sizeof(int32_t) * nh, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::sort(rows.begin(), rows.end());
    HIP_TRY(hipMemcpyAsync(g->heavy_rows, rows.data(), sizeof(int32_t) * nh, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(g_alloc(g, (void**)&d_ranges, sizeof(int32_t) * 2 * nh));
    k_gather_heavy_ranges<<<std::min(1024, (nh + 255) / 256), 256, 0, c->stream>>>(
        nh, g->heavy_rows, g->row_ptr, d_ranges);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(ranges.data(), d_ranges, sizeof(int32_t) * 2 * nh, hipMemcpyDeviceToHost,
                         c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    g_free(g, d_ranges);
    HIP_TRY(e);
  }
  std::vector<int32_t> ch, cb, ce;
  for (int h = 0; h < nh; ++h)
    for (int32_t b = ranges[2 * h]; b < ranges[2 * h + 1]; b += kHeavyChunk) {
      ch.push_back(h);
      cb.push_back(b);
      ce.push_back(std::min(b + kHeavyChunk, ranges[2 * h + 1]));
    }
  g->n_chunks = (int32_t)ch.size();
  const size_t nc = std::max<size_t>(1, ch.size());
  HIP_TRY(g_alloc(g, (void**)&g->chunk_h, sizeof(int32_t) * nc));
  HIP_TRY(g_alloc(g, (void**)&g->chunk_beg, sizeof(int32_t) * nc));
  HIP_TRY(g_alloc(g, (void**)&g->chunk_end, sizeof(int32_t) * nc));
  if (!ch.empty()) {
    HIP_TRY(hipMemcpy(g->chunk_h, ch.data(), sizeof(int32_t) * ch.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->chunk_beg, cb.data(), sizeof(int32_t) * ch.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->chunk_end, ce.data(), sizeof(int32_t) * ch.size(), hipMemcpyHostToDevice));
  }
  HIP_TRY(g_alloc(g, (void**)&g->chunk_sum, sizeof(double) * nc));
  HIP_TRY(g_alloc(g, (void**)&g->pull_s, sizeof(float) * 2 * g->n));
  HIP_TRY(g_alloc(g, (void**)&g->pull_heavy, sizeof(double) * 2 * std::max(1, nh)));
  HIP_TRY(g_alloc(g, (void**)&g->pull_partials,
                    sizeof(double) * kStride * (light_blocks(c, g->n) + std::max(1, g->n_chunks))));
  return DITR_OK;
}

// start of a round: nothing in flight
int launch_pull_prepare(ditr_ctx* c, const ditr_graph* g) {
  k_zero_f32<<<std::min<int64_t>(4096, (2 * g->n + 255) / 256), 256, 0, c->stream>>>(g->pull_s, 2 * g->n);
  if (g->n_heavy > 0)
    k_zero_f64<<<std::min(1024, (2 * g->n_heavy + 255) / 256), 256, 0, c->stream>>>(
        g->pull_heavy, 2 * (int64_t)g->n_heavy);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

int launch_pull_sweeps(ditr_ctx* c, const ditr_graph* g, float* f, double* h, double alpha,
                       int first_parity, int nsweeps) {
  PullArgs a;
  a.n = g->n;
  a.row_ptr = g->row_ptr;
  a.csr_col = g->csr_col;
  a.col_ptr = g->col_ptr;
  a.heavy_rows = g->heavy_rows;
  a.chunk_h = g->chunk_h;
  a.chunk_beg = g->chunk_beg;
  a.chunk_end = g->chunk_end;
  a.csr_val = g->csr_val;
  a.colabs = g->colabs;
  a.F = f;
  a.H = h;
  a.S = g->pull_s;
  a.heavy_in = g->pull_heavy;
  a.partials = g->pull_partials;
  a.ctrl = c->ctrl;
  a.n_heavy = g->n_heavy;
  a.n_light_blocks = light_blocks(c, g->n);
  a.d = (float)g->d;
  const int grid = a.n_light_blocks + g->n_chunks;
  for (int s = 0; s < nsweeps; ++s) {
    if (a.csr_val) k_pull_sweep<true><<<grid, kPullBlock, 0, c->stream>>>(a, (first_parity + s) & 1);
    else k_pull_sweep<false><<<grid, kPullBlock, 0, c->stream>>>(a, (first_parity + s) & 1);
    k_pull_step<<<1, 256, 0, c->stream>>>(g->pull_partials, grid, c->ctrl, alpha);
  }
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}
