// Batched personalized PageRank: R right-hand sides B_r diffused together.
//
// Every right-hand side runs its own D-iteration (Section 2) with its own
// threshold T_r (Section 2.4) and stop test; they share the graph reads. The
// fluid, history and published shares are node-major: row i holds the R values
// of node i, so one wave reads a row as 64 lanes x 4 values (1 KB for R = 256)
// and one in-link index serves all R right-hand sides.
//
// A sweep is the pull form of the threshold test applied to a node set (as in
// pull_k.hip): row j adds sum_{i -> j} S_in[i, :] to F[j, :], then every lane
// r with |F[j, r]| > T_r diffuses: H[j, r] += F, S_out[j, r] = F p_j, F = 0.
// Rows whose S row is all zero are flagged inactive so their in-links cost a
// byte, not a row. Rows with many in-links are summed by chunk workgroups
// right before the sweep (k_batch_heavy).
#include <string.h>

#include <algorithm>

#include "common.h"

namespace {

constexpr int kBB = 256;          // threads per block (4 waves)
constexpr int kMaxR = 256;        // right-hand sides per call (64 lanes x 4)
constexpr int kFinBlocks = 256;   // blocks finishing the heavy rows of a refresh
constexpr int kSub = 16;          // workgroups per heavy chunk (kHeavyChunk / kSub in-links each)
constexpr int kStepBlocks = 64;   // workgroups of the per-sweep reduction

struct BatchArgs {
  int64_t n;
  int R;                           // right-hand sides (multiple of 4, <= 256)
  const int32_t* __restrict__ row_ptr;
  const int32_t* __restrict__ csr_col;
  const int32_t* __restrict__ col_ptr;
  const int32_t* __restrict__ heavy_rows;
  const int32_t* __restrict__ chunk_h;
  const int32_t* __restrict__ chunk_beg;
  const int32_t* __restrict__ chunk_end;
  int n_heavy;
  int n_chunks;
  const double* B;                 // [n][R]
  float* F;                        // [n][R]
  double* H;                       // [n][R]
  float* G;                        // [n][R] history increments of the current stage (FP32),
                                   //   added into H before each exact refresh
  float* S;                        // [2][n][R]
  uint8_t* act;                    // [2][n] row of S nonzero
  float* heavy_in;                 // [n_heavy][R]
  double* racc;                    // [n_heavy][R] refresh accumulator of heavy rows
  double* part;                    // [nblocks + kFinBlocks + kStepBlocks][R][2]: sum |fluid|, diffused edges
  double* T;                       // [R] thresholds
  double* tol;                     // [R] absolute targets
  int* done;                       // [R] 1 once the right-hand side met its target
  int* all_done;                   // all right-hand sides done
  int* step_count;                 // workgroups of k_batch_step that finished (reset by the last)
  float d;                         // damping, FP32 fluid arithmetic
  double dd;                       // damping, FP64 exact residual
  int nblocks;
};

__device__ __forceinline__ int find_row(const int32_t* rows, int nh, int j) {
  int lo = 0, hi = nh - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (rows[mid] < j) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// init: F = (float)B, H = 0, G = 0, S = 0, activity = 0; per block sum |B| and max |B| per lane
__global__ void __launch_bounds__(kBB) k_batch_init(BatchArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * (kBB / 64);
  const bool on = 4 * lane < a.R;
  double s[4] = {0, 0, 0, 0}, m[4] = {0, 0, 0, 0};
  for (int64_t j = (int64_t)blockIdx.x * (kBB / 64) + wave; j < a.n; j += nw) {
    if (on) {
      const size_t o = (size_t)j * a.R + 4 * lane;
      float4 f;
      double b0 = a.B[o], b1 = a.B[o + 1], b2 = a.B[o + 2], b3 = a.B[o + 3];
      f.x = (float)b0; f.y = (float)b1; f.z = (float)b2; f.w = (float)b3;
      *reinterpret_cast<float4*>(&a.F[o]) = f;
      *reinterpret_cast<double2*>(&a.H[o]) = make_double2(0.0, 0.0);
      *reinterpret_cast<double2*>(&a.H[o + 2]) = make_double2(0.0, 0.0);
      *reinterpret_cast<float4*>(&a.G[o]) = make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(&a.S[o]) = make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(&a.S[(size_t)a.n * a.R + o]) = make_float4(0.f, 0.f, 0.f, 0.f);
      s[0] += fabs(b0); s[1] += fabs(b1); s[2] += fabs(b2); s[3] += fabs(b3);
      m[0] = fmax(m[0], fabs(b0)); m[1] = fmax(m[1], fabs(b1));
      m[2] = fmax(m[2], fabs(b2)); m[3] = fmax(m[3], fabs(b3));
    }
    if (lane == 0) { a.act[j] = 0; a.act[a.n + j] = 0; }
  }
  __shared__ double red[2][kBB / 64][kMaxR];
  if (on)
    for (int k = 0; k < 4; ++k) {
      red[0][wave][4 * lane + k] = s[k];
      red[1][wave][4 * lane + k] = m[k];
    }
  __syncthreads();
  for (int r = threadIdx.x; r < a.R; r += kBB) {
    double S0 = 0, M0 = 0;
    for (int w = 0; w < kBB / 64; ++w) {
      S0 += red[0][w][r];
      M0 = fmax(M0, red[1][w][r]);
    }
    a.part[((size_t)blockIdx.x * a.R + r) * 2 + 0] = S0;
    a.part[((size_t)blockIdx.x * a.R + r) * 2 + 1] = M0;
  }
}

// per lane: b1 = sum of part[.,r,0], fmax = max part[.,r,1]; T_r = fmax / alpha,
// tol_r = rel_tol b1; done_r if b1 == 0. Writes b1 into out_b1.
__global__ void k_batch_setup(BatchArgs a, double alpha, double rel_tol, double* out_b1,
                              double* out_r) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < a.R; r += gridDim.x * blockDim.x) {
    double s = 0, m = 0;
    for (int b = 0; b < a.nblocks; ++b) {
      s += a.part[((size_t)b * a.R + r) * 2 + 0];
      m = fmax(m, a.part[((size_t)b * a.R + r) * 2 + 1]);
    }
    out_b1[r] = s;
    out_r[r] = s;
    a.T[r] = m / alpha;
    a.tol[r] = rel_tol * s;
    a.done[r] = s <= a.tol[r];
  }
}

// inflow of heavy rows: one block per chunk of in-links; 4 waves take 4 links at
// a time, each lane 4 right-hand sides; one FP32 atomic per lane per chunk
__global__ void __launch_bounds__(kBB) k_batch_heavy(BatchArgs a, int parity) {
  if (__hip_atomic_load(a.all_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const float* S_in = a.S + (size_t)(parity ^ 1) * a.n * a.R;
  const uint8_t* act_in = a.act + (size_t)(parity ^ 1) * a.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x / kSub;
  const int sb = a.chunk_beg[c] + (blockIdx.x % kSub) * (kHeavyChunk / kSub);
  const int se = min(a.chunk_end[c], sb + kHeavyChunk / kSub);
  const bool on = 4 * lane < a.R;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  // each wave takes 64 in-links at a time, one per lane (index and activity
  // flag), then reads the active sources' share rows four at a time
  for (int eb = sb + 64 * wave; eb < se; eb += kBB) {
    const int32_t src = eb + lane < se ? a.csr_col[eb + lane] : -1;
    unsigned long long m = __ballot(src >= 0 && act_in[src] != 0);
    while (m) {
      int32_t s4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        s4[q] = -1;
        if (m) {
          const int bit = __ffsll(m) - 1;
          m &= m - 1;
          s4[q] = __builtin_amdgcn_readlane(src, bit);
        }
      }
      float4 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        v[q] = on && s4[q] >= 0 ? *reinterpret_cast<const float4*>(&S_in[(size_t)s4[q] * a.R + 4 * lane])
                                : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc.x += v[q].x; acc.y += v[q].y; acc.z += v[q].z; acc.w += v[q].w;
      }
    }
  }
  __shared__ float4 red[kBB / 64][64];
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && on) {
    float4 t = red[0][lane];
    for (int w = 1; w < kBB / 64; ++w) {
      t.x += red[w][lane].x; t.y += red[w][lane].y; t.z += red[w][lane].z; t.w += red[w][lane].w;
    }
    float* dst = &a.heavy_in[(size_t)a.chunk_h[c] * a.R + 4 * lane];  // sub-chunks of one row add up
    if (t.x != 0.f) add_agent(&dst[0], t.x);
    if (t.y != 0.f) add_agent(&dst[1], t.y);
    if (t.z != 0.f) add_agent(&dst[2], t.z);
    if (t.w != 0.f) add_agent(&dst[3], t.w);
  }
}

// one batched threshold sweep: a wave per row
__global__ void __launch_bounds__(kBB, 8) k_batch_sweep(BatchArgs a, int parity) {
  if (__hip_atomic_load(a.all_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const float* S_in = a.S + (size_t)(parity ^ 1) * a.n * a.R;
  float* S_out = a.S + (size_t)parity * a.n * a.R;
  const uint8_t* act_in = a.act + (size_t)(parity ^ 1) * a.n;
  uint8_t* act_out = a.act + (size_t)parity * a.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool on = 4 * lane < a.R;
  const int r0 = 4 * lane;
  float T[4];
  int dn[4];
  for (int k = 0; k < 4; ++k) {
    T[k] = on ? (float)a.T[r0 + k] : 0.f;
    dn[k] = on ? a.done[r0 + k] : 1;
  }
  double resid[4] = {0, 0, 0, 0}, edges[4] = {0, 0, 0, 0};
  const int64_t nw = (int64_t)gridDim.x * (kBB / 64);
  for (int64_t j = (int64_t)blockIdx.x * (kBB / 64) + wave; j < a.n; j += nw) {
    const int32_t e0 = a.row_ptr[j], e1 = a.row_ptr[j + 1];
    // the row's own fluid and out-degree do not depend on the inflow: their
    // loads go out first and land while the in-links are gathered
    const size_t o = (size_t)j * a.R + r0;
    const float4 f0 = on ? *reinterpret_cast<const float4*>(&a.F[o]) : make_float4(0.f, 0.f, 0.f, 0.f);
    const int deg = a.col_ptr[j + 1] - a.col_ptr[j];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (e1 - e0 > kHeavyRow) {
      if (on) {
        const int h = find_row(a.heavy_rows, a.n_heavy, (int)j);
        float4* hp = reinterpret_cast<float4*>(&a.heavy_in[(size_t)h * a.R + r0]);
        acc = *hp;
        *hp = make_float4(0.f, 0.f, 0.f, 0.f);  // accumulator of the next sweep
      }
    } else {
      // at most kHeavyRow (64) in-links: lane l reads in-link l and its source's
      // activity flag, then the active sources' share rows are read four at a
      // time (three dependent loads in all instead of three per pair of links)
      const int32_t src = lane < e1 - e0 ? a.csr_col[e0 + lane] : -1;
      unsigned long long m = __ballot(src >= 0 && act_in[src] != 0);
      while (m) {
        int32_t s[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          s[q] = -1;
          if (m) {
            const int b = __ffsll(m) - 1;
            m &= m - 1;
            s[q] = __builtin_amdgcn_readlane(src, b);
          }
        }
        float4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          v[q] = on && s[q] >= 0 ? *reinterpret_cast<const float4*>(&S_in[(size_t)s[q] * a.R + r0])
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc.x += v[q].x; acc.y += v[q].y; acc.z += v[q].z; acc.w += v[q].w;
        }
      }
    }
    int any = 0;
    float4 so = make_float4(0.f, 0.f, 0.f, 0.f);
    if (on) {
      float f[4] = {f0.x + acc.x, f0.y + acc.y, f0.z + acc.z, f0.w + acc.w};
      const float p = deg > 0 ? a.d / (float)deg : 0.f;
      float s[4] = {0.f, 0.f, 0.f, 0.f};
      bool sel = false;
      for (int k = 0; k < 4; ++k)
        if (!dn[k] && fabsf(f[k]) > T[k]) {
          s[k] = f[k];
          f[k] = 0.f;
          sel = true;
        }
      if (sel) {  // the stage's history increment: FP32 here, added into the FP64 H before the refresh
        float4 g = *reinterpret_cast<const float4*>(&a.G[o]);
        g.x += s[0]; g.y += s[1]; g.z += s[2]; g.w += s[3];
        *reinterpret_cast<float4*>(&a.G[o]) = g;
      }
      // F is rewritten only where it changed
      const bool inflow = (acc.x != 0.f) | (acc.y != 0.f) | (acc.z != 0.f) | (acc.w != 0.f);
      if (sel || inflow) *reinterpret_cast<float4*>(&a.F[o]) = make_float4(f[0], f[1], f[2], f[3]);
      so = make_float4(s[0] * p, s[1] * p, s[2] * p, s[3] * p);
      any = (so.x != 0.f) | (so.y != 0.f) | (so.z != 0.f) | (so.w != 0.f);
      for (int k = 0; k < 4; ++k) {
        resid[k] += fabs((double)f[k]) + (deg > 0 ? (double)a.d * fabs((double)s[k]) : 0.0);
        if (s[k] != 0.f) edges[k] += deg;
      }
    }
    any = __ballot(any) != 0ull;
    // the S row is read only when some lane of it is active: then every lane
    // writes its part; an inactive row keeps whatever it held
    if (any && on) *reinterpret_cast<float4*>(&S_out[(size_t)j * a.R + r0]) = so;
    if (lane == 0) act_out[j] = (uint8_t)any;
  }
  // per-lane block sums
  __shared__ double red[2][kBB / 64][kMaxR];
  if (on)
    for (int k = 0; k < 4; ++k) {
      red[0][wave][r0 + k] = resid[k];
      red[1][wave][r0 + k] = edges[k];
    }
  __syncthreads();
  for (int r = threadIdx.x; r < a.R; r += kBB) {
    double s0 = 0, s1 = 0;
    for (int w = 0; w < kBB / 64; ++w) {
      s0 += red[0][w][r];
      s1 += red[1][w][r];
    }
    a.part[((size_t)blockIdx.x * a.R + r) * 2 + 0] = s0;
    a.part[((size_t)blockIdx.x * a.R + r) * 2 + 1] = s1;
  }
}

// after a sweep: per right-hand side, fluid (held plus in flight and in the
// heavy accumulators) and edges; stop test; T_r <- T_r / alpha. kStepBlocks
// workgroups each sum a slice of the sweep's block partials and of the heavy
// rows for every right-hand side; the last one to finish adds the slices in a
// fixed order and takes the decisions (its count is reset for the next sweep).
__global__ void __launch_bounds__(kMaxR) k_batch_step(BatchArgs a, double alpha, double* resid_out,
                                                      double* edges_acc, unsigned long long* sweeps) {
  if (__hip_atomic_load(a.all_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ int s_all, s_last;
  const int G = gridDim.x, gb = blockIdx.x;
  double* sp = a.part + (size_t)(a.nblocks + kFinBlocks) * a.R * 2;  // [G][R][2]
  const int b0 = (int)((int64_t)a.nblocks * gb / G), b1 = (int)((int64_t)a.nblocks * (gb + 1) / G);
  const int h0 = (int)((int64_t)a.n_heavy * gb / G), h1 = (int)((int64_t)a.n_heavy * (gb + 1) / G);
  for (int r = threadIdx.x; r < a.R; r += blockDim.x) {
    double s = 0, e = 0;
    for (int b = b0; b < b1; ++b) {
      s += a.part[((size_t)b * a.R + r) * 2 + 0];
      e += a.part[((size_t)b * a.R + r) * 2 + 1];
    }
    for (int h = h0; h < h1; ++h) s += fabs((double)a.heavy_in[(size_t)h * a.R + r]);
    st_agent(&sp[((size_t)gb * a.R + r) * 2 + 0], s);
    st_agent(&sp[((size_t)gb * a.R + r) * 2 + 1], e);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // s_waitcnt vmcnt(0): the slice sums land first
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = __hip_atomic_fetch_add(a.step_count, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == G - 1;
  __syncthreads();
  if (!s_last) return;
  if (threadIdx.x == 0) {
    s_all = 1;
    __hip_atomic_store(a.step_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < a.R; r += blockDim.x) {
    double s = 0, e = 0;
    for (int q = 0; q < G; ++q) {
      s += ld_agent(&sp[((size_t)q * a.R + r) * 2 + 0]);
      e += ld_agent(&sp[((size_t)q * a.R + r) * 2 + 1]);
    }
    resid_out[r] = s;
    edges_acc[r] += e;
    if (!a.done[r]) {
      if (s <= a.tol[r]) a.done[r] = 1;
      else a.T[r] = a.T[r] / alpha;
    }
    if (!a.done[r]) atomicAnd(&s_all, 0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *sweeps += 1;
    if (s_all) __hip_atomic_store(a.all_done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// end of a stage: H += G, G = 0 (before the exact residual reads H)
__global__ void __launch_bounds__(256) k_batch_flush(BatchArgs a) {
  const int64_t total = a.n * (int64_t)a.R / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    const size_t o = (size_t)q * 4;
    const float4 g = *reinterpret_cast<const float4*>(&a.G[o]);
    if (g.x == 0.f && g.y == 0.f && g.z == 0.f && g.w == 0.f) continue;
    double2 h01 = *reinterpret_cast<const double2*>(&a.H[o]);
    double2 h23 = *reinterpret_cast<const double2*>(&a.H[o + 2]);
    h01.x += g.x; h01.y += g.y; h23.x += g.z; h23.y += g.w;
    *reinterpret_cast<double2*>(&a.H[o]) = h01;
    *reinterpret_cast<double2*>(&a.H[o + 2]) = h23;
    *reinterpret_cast<float4*>(&a.G[o]) = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// exact residual F = B + P H - H per right-hand side (FP64), FP32 store; one
// wave per row over its in-links (heavy rows too: a whole wave row by row)
__global__ void __launch_bounds__(kBB) k_batch_refresh(BatchArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool on = 4 * lane < a.R;
  const int r0 = 4 * lane;
  double resid[4] = {0, 0, 0, 0}, mx[4] = {0, 0, 0, 0};
  const int64_t nw = (int64_t)gridDim.x * (kBB / 64);
  for (int64_t j = (int64_t)blockIdx.x * (kBB / 64) + wave; j < a.n; j += nw) {
    if (!on || a.row_ptr[j + 1] - a.row_ptr[j] > kHeavyRow) continue;  // heavy rows: chunks
    double acc[4] = {0, 0, 0, 0};
    for (int32_t e = a.row_ptr[j]; e < a.row_ptr[j + 1]; ++e) {
      const int32_t i = a.csr_col[e];
      const int deg = a.col_ptr[i + 1] - a.col_ptr[i];
      const double p = a.dd / (double)deg;  // deg > 0: i has the out-link i -> j
      const size_t o = (size_t)i * a.R + r0;
      const double2 h01 = *reinterpret_cast<const double2*>(&a.H[o]);
      const double2 h23 = *reinterpret_cast<const double2*>(&a.H[o + 2]);
      acc[0] += p * h01.x; acc[1] += p * h01.y; acc[2] += p * h23.x; acc[3] += p * h23.y;
    }
    const size_t o = (size_t)j * a.R + r0;
    const double2 h01 = *reinterpret_cast<const double2*>(&a.H[o]);
    const double2 h23 = *reinterpret_cast<const double2*>(&a.H[o + 2]);
    const double hv[4] = {h01.x, h01.y, h23.x, h23.y};
    float f[4];
    for (int k = 0; k < 4; ++k) {
      const double v = a.B[o + k] - hv[k] + acc[k];
      f[k] = (float)v;
      resid[k] += fabs(v);
      mx[k] = fmax(mx[k], fabs(v));
    }
    *reinterpret_cast<float4*>(&a.F[o]) = make_float4(f[0], f[1], f[2], f[3]);
  }
  __shared__ double red[2][kBB / 64][kMaxR];
  if (on)
    for (int k = 0; k < 4; ++k) {
      red[0][wave][r0 + k] = resid[k];
      red[1][wave][r0 + k] = mx[k];
    }
  __syncthreads();
  for (int r = threadIdx.x; r < a.R; r += kBB) {
    double s0 = 0, m0 = 0;
    for (int w = 0; w < kBB / 64; ++w) {
      s0 += red[0][w][r];
      m0 = fmax(m0, red[1][w][r]);
    }
    a.part[((size_t)blockIdx.x * a.R + r) * 2 + 0] = s0;
    a.part[((size_t)blockIdx.x * a.R + r) * 2 + 1] = m0;
  }
}

// refresh of heavy rows, part 1: one block per chunk of in-links, FP64 sums of
// p_ji H_i into racc (one FP64 atomic per lane value per chunk)
__global__ void __launch_bounds__(kBB) k_batch_refresh_heavy(BatchArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x / kSub;
  const int sb = a.chunk_beg[c] + (blockIdx.x % kSub) * (kHeavyChunk / kSub);
  const int se = min(a.chunk_end[c], sb + kHeavyChunk / kSub);
  const bool on = 4 * lane < a.R;
  const int r0 = 4 * lane;
  double acc[4] = {0, 0, 0, 0};
  if (on)
    for (int e = sb + wave; e < se; e += kBB / 64) {
      const int32_t i = a.csr_col[e];
      const double p = a.dd / (double)(a.col_ptr[i + 1] - a.col_ptr[i]);
      const size_t o = (size_t)i * a.R + r0;
      const double2 h01 = *reinterpret_cast<const double2*>(&a.H[o]);
      const double2 h23 = *reinterpret_cast<const double2*>(&a.H[o + 2]);
      acc[0] += p * h01.x; acc[1] += p * h01.y; acc[2] += p * h23.x; acc[3] += p * h23.y;
    }
  __shared__ double red[kBB / 64][kMaxR];
  if (on)
    for (int k = 0; k < 4; ++k) red[wave][r0 + k] = acc[k];
  __syncthreads();
  for (int r = threadIdx.x; r < a.R; r += kBB) {
    double t = 0;
    for (int w = 0; w < kBB / 64; ++w) t += red[w][r];
    if (t != 0.0) add_agent(&a.racc[(size_t)a.chunk_h[c] * a.R + r], t);
  }
}

// refresh of heavy rows, part 2: F = B - H + racc, partial sums in part rows
// [nblocks, nblocks + kFinBlocks); racc cleared for the next refresh
__global__ void __launch_bounds__(kBB) k_batch_refresh_fin(BatchArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool on = 4 * lane < a.R;
  const int r0 = 4 * lane;
  double resid[4] = {0, 0, 0, 0}, mx[4] = {0, 0, 0, 0};
  for (int h = blockIdx.x * (kBB / 64) + wave; h < a.n_heavy; h += gridDim.x * (kBB / 64)) {
    if (!on) continue;
    const int64_t j = a.heavy_rows[h];
    const size_t o = (size_t)j * a.R + r0;
    float f[4];
    for (int k = 0; k < 4; ++k) {
      double* ra = &a.racc[(size_t)h * a.R + r0 + k];
      const double v = a.B[o + k] - a.H[o + k] + *ra;
      *ra = 0.0;
      f[k] = (float)v;
      resid[k] += fabs(v);
      mx[k] = fmax(mx[k], fabs(v));
    }
    *reinterpret_cast<float4*>(&a.F[o]) = make_float4(f[0], f[1], f[2], f[3]);
  }
  __shared__ double red[2][kBB / 64][kMaxR];
  if (on)
    for (int k = 0; k < 4; ++k) {
      red[0][wave][r0 + k] = resid[k];
      red[1][wave][r0 + k] = mx[k];
    }
  __syncthreads();
  for (int r = threadIdx.x; r < a.R; r += kBB) {
    double s0 = 0, m0 = 0;
    for (int w = 0; w < kBB / 64; ++w) {
      s0 += red[0][w][r];
      m0 = fmax(m0, red[1][w][r]);
    }
    const size_t row = (size_t)a.nblocks + blockIdx.x;
    a.part[(row * a.R + r) * 2 + 0] = s0;
    a.part[(row * a.R + r) * 2 + 1] = m0;
  }
}

// after a refresh: exact residual per right-hand side; the next round starts
// with nothing in flight, T_r = min(T_r, max|F_r| / alpha) and a stage target
__global__ void k_batch_after_refresh(BatchArgs a, double alpha, const double* b1, double rel_tol,
                                      double stage_rel, double* resid_out, int* remaining) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < a.R; r += gridDim.x * blockDim.x) {
    double s = 0, m = 0;
    for (int b = 0; b < a.nblocks + kFinBlocks; ++b) {
      s += a.part[((size_t)b * a.R + r) * 2 + 0];
      m = fmax(m, a.part[((size_t)b * a.R + r) * 2 + 1]);
    }
    resid_out[r] = s;
    const bool ok = s <= rel_tol * b1[r];
    a.done[r] = ok;
    a.tol[r] = stage_rel * b1[r];
    a.T[r] = fmin(a.T[r], m / alpha);
    if (!ok) atomicAdd(remaining, 1);
  }
}

__global__ void k_batch_clear(BatchArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t total = 2 * a.n * (int64_t)a.R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += stride) a.S[i] = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * a.n; i += stride) a.act[i] = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)a.n_heavy * a.R; i += stride)
    a.heavy_in[i] = 0.f;
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.all_done = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// host driver (called from api.hip)

struct BatchWork {
  float* S = nullptr;
  float* G = nullptr;
  uint8_t* act = nullptr;
  float* heavy_in = nullptr;
  double* racc = nullptr;
  double* part = nullptr;
  double* lane = nullptr;   // T, tol, b1, resid, edges: 5 x R doubles
  int* flags = nullptr;     // done[R], all_done, remaining
  unsigned long long* sweeps = nullptr;
  unsigned char* ws = nullptr;  // caller workspace the buffers are carved from (nothing to free)
  size_t ws_cap = 0, ws_used = 0;
};

static void free_work(BatchWork& w) {
  if (!w.ws)
    for (void* p : {(void*)w.S, (void*)w.G, (void*)w.act, (void*)w.heavy_in, (void*)w.racc, (void*)w.part,
                    (void*)w.lane, (void*)w.flags, (void*)w.sweeps})
      (void)hipFree(p);
  w = BatchWork();
}

// one buffer of the batched solve: carved from the caller's workspace when
// there is one, else hipMalloc
static hipError_t work_alloc(BatchWork& w, void** p, size_t bytes) {
  if (!w.ws) return hipMalloc(p, bytes);
  const size_t need = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
  if (w.ws_used + need > w.ws_cap) return hipErrorOutOfMemory;
  *p = w.ws + w.ws_used;
  w.ws_used += need;
  return hipSuccess;
}

static int batch_blocks(const ditr_ctx* c, int64_t n) {
  return (int)std::min<int64_t>((int64_t)c->num_cus * 8, (n + 3) / 4);
}

// device bytes of the batched solve's buffers (the workspace ditr_solve_batched takes)
size_t batch_workspace_bytes(const ditr_ctx* c, int64_t n, int64_t n_heavy, int R) {
  auto al = [](size_t x) { return (std::max<size_t>(x, 1) + 255) & ~(size_t)255; };
  const size_t N = (size_t)n, r = (size_t)R, nh = (size_t)std::max<int64_t>(1, n_heavy);
  const size_t nb = (size_t)batch_blocks(c, n);
  return al(sizeof(float) * 2 * N * r) + al(sizeof(float) * N * r) + al(2 * N) + al(sizeof(float) * nh * r) +
         al(sizeof(double) * nh * r) + al(sizeof(double) * (nb + kFinBlocks + kStepBlocks) * r * 2) +
         al(sizeof(double) * 5 * r) + al(sizeof(int) * (r + 3)) + al(sizeof(unsigned long long));
}

int batch_solve(ditr_ctx* c, const ditr_graph* g, int R, const double* d_b, double* d_h, float* d_f,
                double rel_tol, const ditr_opts& o, ditr_stats* per_rhs, ditr_stats* total,
                void* d_workspace, size_t ws_bytes) {
  if (R < 4 || R > kMaxR || R % 4) return set_error(DITR_EINVAL, "nrhs must be a multiple of 4 in [4, 256]");
  const int64_t n = g->n;
  const int nblocks = batch_blocks(c, n);
  BatchWork w;
  if (d_workspace) {
    const size_t need = batch_workspace_bytes(c, n, g->n_heavy, R);
    if (ws_bytes < need)
      return set_error(DITR_EINVAL, "batched workspace of %zu bytes is too small (%zu needed)", ws_bytes, need);
    w.ws = static_cast<unsigned char*>(d_workspace);
    w.ws_cap = ws_bytes;
  }
  // the loop is captured as a graph, which the legacy null stream cannot do:
  // run on the context's private stream once the caller's stream has drained
  hipStream_t st = c->work;
  HIP_TRY(hipStreamSynchronize(c->stream));
  auto fail = [&](int code) {
    (void)hipStreamSynchronize(st);
    free_work(w);
    return code;
  };
#define B_TRY(expr)                                                                          \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(set_error(DITR_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e)));      \
  } while (0)
  B_TRY(work_alloc(w, (void**)&w.S, sizeof(float) * 2 * n * R));
  B_TRY(work_alloc(w, (void**)&w.G, sizeof(float) * n * R));
  B_TRY(work_alloc(w, (void**)&w.act, 2 * n));
  B_TRY(work_alloc(w, (void**)&w.heavy_in, sizeof(float) * std::max(1, g->n_heavy) * R));
  B_TRY(work_alloc(w, (void**)&w.racc, sizeof(double) * std::max(1, g->n_heavy) * R));
  B_TRY(hipMemsetAsync(w.racc, 0, sizeof(double) * std::max(1, g->n_heavy) * R, st));
  B_TRY(work_alloc(w, (void**)&w.part, sizeof(double) * (nblocks + kFinBlocks + kStepBlocks) * R * 2));
  B_TRY(hipMemsetAsync(w.part, 0, sizeof(double) * (nblocks + kFinBlocks + kStepBlocks) * R * 2, st));
  B_TRY(work_alloc(w, (void**)&w.lane, sizeof(double) * 5 * R));
  B_TRY(work_alloc(w, (void**)&w.flags, sizeof(int) * (R + 3)));
  B_TRY(work_alloc(w, (void**)&w.sweeps, sizeof(unsigned long long)));
  B_TRY(hipMemsetAsync(w.lane, 0, sizeof(double) * 5 * R, st));
  B_TRY(hipMemsetAsync(w.flags, 0, sizeof(int) * (R + 3), st));
  B_TRY(hipMemsetAsync(w.sweeps, 0, sizeof(unsigned long long), st));

  BatchArgs a;
  a.n = n;
  a.R = R;
  a.row_ptr = g->row_ptr;
  a.csr_col = g->csr_col;
  a.col_ptr = g->col_ptr;
  a.heavy_rows = g->heavy_rows;
  a.chunk_h = g->chunk_h;
  a.chunk_beg = g->chunk_beg;
  a.chunk_end = g->chunk_end;
  a.n_heavy = g->n_heavy;
  a.n_chunks = g->n_chunks;
  a.B = d_b;
  a.F = d_f;
  a.H = d_h;
  a.S = w.S;
  a.G = w.G;
  a.act = w.act;
  a.heavy_in = w.heavy_in;
  a.racc = w.racc;
  a.part = w.part;
  a.T = w.lane;
  a.tol = w.lane + R;
  double* b1 = w.lane + 2 * R;
  double* resid = w.lane + 3 * R;
  double* edges = w.lane + 4 * R;
  a.done = w.flags;
  a.all_done = w.flags + R;
  int* remaining = w.flags + R + 1;
  a.step_count = w.flags + R + 2;
  a.d = (float)g->d;
  a.dd = g->d;
  a.nblocks = nblocks;

  k_batch_init<<<nblocks, kBB, 0, st>>>(a);
  k_batch_clear<<<2048, 256, 0, st>>>(a);
  k_batch_setup<<<1, 256, 0, st>>>(a, o.alpha, std::max(rel_tol, o.refresh_at > 0 ? o.refresh_at : 1e-6), b1, resid);
  B_TRY(hipGetLastError());

  // the sweep loop, captured once as a graph of kBatchSweeps (heavy, sweep, step)
  // triples; the stop flag turns the rest of a replay into no-ops
  constexpr int kBatchSweeps = 16;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct GraphGuard {
    hipGraph_t* g;
    hipGraphExec_t* e;
    ~GraphGuard() {
      if (*e) (void)hipGraphExecDestroy(*e);
      if (*g) (void)hipGraphDestroy(*g);
    }
  } guard{&graph, &exec};
  B_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  for (int s = 0; s < kBatchSweeps; ++s) {
    if (a.n_chunks > 0) k_batch_heavy<<<a.n_chunks * kSub, kBB, 0, st>>>(a, s & 1);
    k_batch_sweep<<<nblocks, kBB, 0, st>>>(a, s & 1);
    k_batch_step<<<kStepBlocks, kMaxR, 0, st>>>(a, o.alpha, resid, edges, w.sweeps);
  }
  hipError_t ce = hipStreamEndCapture(st, &graph);
  if (ce != hipSuccess) return fail(set_error(DITR_EHIP, "graph capture failed: %s", hipGetErrorString(ce)));
  B_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));

  const int max_rounds = o.max_rounds > 0 ? o.max_rounds : 16;
  const int64_t budget = o.max_sweeps > 0 ? o.max_sweeps : 4096;
  int rounds = 0, status = DITR_OK;
  int host_flags[2] = {0, 0};
  for (;;) {
    // diffusion: replay the captured sweeps until every right-hand side stops
    for (int64_t k = 0; k < budget; k += kBatchSweeps) {
      B_TRY(hipGraphLaunch(exec, st));
      B_TRY(hipMemcpyAsync(host_flags, a.all_done, sizeof(int), hipMemcpyDeviceToHost, st));
      B_TRY(hipStreamSynchronize(st));
      if (host_flags[0] || __atomic_load_n(c->abort_host, __ATOMIC_SEQ_CST)) break;
    }
    // exact residual of every right-hand side; stage 2 aims below the target
    ++rounds;
    B_TRY(hipMemsetAsync(remaining, 0, sizeof(int), st));
    k_batch_flush<<<4096, 256, 0, st>>>(a);
    k_batch_refresh<<<nblocks, kBB, 0, st>>>(a);
    if (a.n_chunks > 0) k_batch_refresh_heavy<<<a.n_chunks * kSub, kBB, 0, st>>>(a);
    k_batch_refresh_fin<<<kFinBlocks, kBB, 0, st>>>(a);
    k_batch_after_refresh<<<1, 256, 0, st>>>(a, o.alpha, b1, rel_tol, 0.5 * rel_tol, resid, remaining);
    k_batch_clear<<<2048, 256, 0, st>>>(a);
    B_TRY(hipGetLastError());
    B_TRY(hipMemcpyAsync(&host_flags[1], remaining, sizeof(int), hipMemcpyDeviceToHost, st));
    B_TRY(hipStreamSynchronize(st));
    if (host_flags[1] == 0) break;
    if (__atomic_load_n(c->abort_host, __ATOMIC_SEQ_CST)) { status = DITR_ABORTED; break; }
    if (rounds >= max_rounds) { status = DITR_NOT_CONVERGED; break; }
  }
  // per right-hand side statistics
  double hres[kMaxR], hb1[kMaxR], hedg[kMaxR];
  unsigned long long hsweeps = 0;
  B_TRY(hipMemcpyAsync(hres, resid, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  B_TRY(hipMemcpyAsync(hb1, b1, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  B_TRY(hipMemcpyAsync(hedg, edges, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  B_TRY(hipMemcpyAsync(&hsweeps, w.sweeps, sizeof(hsweeps), hipMemcpyDeviceToHost, st));
  B_TRY(hipStreamSynchronize(st));
  double tot_e = 0, tot_r = 0, tot_b = 0;
  for (int r = 0; r < R; ++r) {
    if (per_rhs) {
      memset(&per_rhs[r], 0, sizeof(ditr_stats));
      per_rhs[r].edges = (int64_t)hedg[r];
      per_rhs[r].resid_l1 = hres[r];
      per_rhs[r].b_l1 = hb1[r];
      per_rhs[r].sweeps = (int64_t)hsweeps;
      per_rhs[r].rounds = rounds;
      per_rhs[r].refreshes = rounds;
      per_rhs[r].status = hres[r] <= rel_tol * hb1[r] ? DITR_OK : status;
    }
    tot_e += hedg[r];
    tot_r += hres[r];
    tot_b += hb1[r];
  }
  if (total) {
    total->edges = (int64_t)tot_e;
    total->resid_l1 = tot_r;
    total->b_l1 = tot_b;
    total->sweeps = (int64_t)hsweeps;
    total->rounds = rounds;
    total->refreshes = rounds;
    total->launches = (int64_t)hsweeps;
    total->status = status;
  }
  free_work(w);
#undef B_TRY
  return status;
}
