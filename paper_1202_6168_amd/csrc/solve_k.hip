// D-iteration kernels for gfx950.
//
// A node diffusion (Section 2, equations defF and defH; Section 2.1
// pseudo-code) takes sent = F_i, adds it to H_i, zeroes F_i and adds
// sent * p_ji = sent * d / #out_i to F_j for every child j. Nodes are chosen by
// the cyclic threshold test of Section 2.4 (diffuse every i with |F_i| > T,
// then T <- T / alpha).
//
// k_persistent runs the asynchronous partitioned scheme of Sections 2.3-2.6 on
// one GPU: a workgroup owns a node range Omega_k, holds its fluid and history
// increment in LDS, diffuses locally (Section 2.5, algorithm (*)), sends fluid
// of outside targets straight into the owner's slot of the global fluid array
// (its inbox) with device-scope atomics, drains its own inbox between sweeps
// (Section 2.6) and idles while its residual is small (Section 2.4, r_k < T).
// No grid-wide barrier. (The grid-synchronous pull sweep is in pull_k.hip.)
// Termination uses the mass each diffusion provably removes from ||F||_1:
// |sent| (1 - d) for a node with out-links, |sent| for a dangling node. The
// launch stops once ||F_start||_1 minus the removed mass reaches its target;
// the host then recomputes the exact residual in FP64 (k_refresh_*).
#include "common.h"

namespace {

constexpr int kRedBlock = 256;
constexpr int kPartialStride = 4;  // doubles per block in ctx->partials

int grid_for(int64_t n, int block, int cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// block-wide sum of (s0, s1) and max of m; thread 0 gets the result.
// Wave 0 combines the per-wave values with shuffles (fixed order: deterministic).
template <int BLOCK>
__device__ __forceinline__ void block_reduce3(double& s0, double& s1, double& m) {
  constexpr int NW = BLOCK / 64;
  __shared__ double r0[NW], r1[NW], r2[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  m = wave_maxd(m);
  if (NW > 1) {
    if (lane == 0) {
      r0[wave] = s0;
      r1[wave] = s1;
      r2[wave] = m;
    }
    __syncthreads();
    if (wave == 0) {
      s0 = wave_sum(lane < NW ? r0[lane] : 0.0);
      s1 = wave_sum(lane < NW ? r1[lane] : 0.0);
      m = wave_maxd(lane < NW ? r2[lane] : -INFINITY);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// init: F = (float)B, H = 0; sums |B|, |(float)B| and max |B| per block;
// err = 1 if B holds a NaN or Inf.
__global__ void __launch_bounds__(kRedBlock) k_init(int64_t n, const double* __restrict__ b,
                                                     double* __restrict__ h, float* __restrict__ f,
                                                     double* partials, int* err) {
  double s = 0, s32 = 0, m = 0;
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * kRedBlock;
  constexpr int U = 4;  // four loads of B in flight per thread
  for (int64_t i0 = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i0 < n; i0 += U * stride) {
    double bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) bv[u] = i0 + u * stride < n ? b[i0 + u * stride] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      if (i >= n) continue;
      const double v = bv[u];
      bad |= !isfinite(v);
      const float v32 = (float)v;
      f[i] = v32;
      h[i] = 0.0;
      s += fabs(v);
      s32 += fabs((double)v32);
      m = fmax(m, fabs(v));
    }
  }
  if (bad) atomicOr(err, 1);
  block_reduce3<kRedBlock>(s, s32, m);
  if (threadIdx.x == 0) {
    partials[kPartialStride * blockIdx.x + 0] = s;
    partials[kPartialStride * blockIdx.x + 1] = m;
    partials[kPartialStride * blockIdx.x + 2] = s32;
  }
}

// sum |x|, max |x| per block; err = 1 on NaN or Inf
__global__ void __launch_bounds__(kRedBlock) k_norm_f64(int64_t n, const double* __restrict__ x,
                                                         double* partials, int* err) {
  double s = 0, unused = 0, m = 0;
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * kRedBlock;
  for (int64_t i = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i < n; i += stride) {
    double v = x[i];
    bad |= !isfinite(v);
    s += fabs(v);
    m = fmax(m, fabs(v));
  }
  if (bad) atomicOr(err, 1);
  block_reduce3<kRedBlock>(s, unused, m);
  if (threadIdx.x == 0) {
    partials[kPartialStride * blockIdx.x + 0] = s;
    partials[kPartialStride * blockIdx.x + 1] = m;
    partials[kPartialStride * blockIdx.x + 2] = 0;
  }
}

// A start whose fluid is given: sums |B| (slot 0), max |F| (slot 1) and
// |F| (slot 2) per block; err = 1 if B, H or F holds a NaN or Inf
__global__ void __launch_bounds__(kRedBlock) k_given_start(int64_t n, const double* __restrict__ b,
                                                           const double* __restrict__ h,
                                                           const float* __restrict__ f, double* partials,
                                                           int* err) {
  double sb = 0, sf = 0, m = 0;
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * kRedBlock;
  for (int64_t i = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i < n; i += stride) {
    const double bv = b[i], hv = h[i], fv = (double)f[i];
    bad |= !isfinite(bv) || !isfinite(hv) || !isfinite(fv);
    sb += fabs(bv);
    sf += fabs(fv);
    m = fmax(m, fabs(fv));
  }
  if (bad) atomicOr(err, 1);
  block_reduce3<kRedBlock>(sb, sf, m);
  if (threadIdx.x == 0) {
    partials[kPartialStride * blockIdx.x + 0] = sb;
    partials[kPartialStride * blockIdx.x + 1] = m;
    partials[kPartialStride * blockIdx.x + 2] = sf;
  }
}

__global__ void __launch_bounds__(kRedBlock) k_check_finite(int64_t n, const double* __restrict__ x,
                                                             int* err) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * kRedBlock;
  for (int64_t i = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i < n; i += stride)
    bad |= !isfinite(x[i]);
  if (bad) atomicOr(err, 1);
}

// reduce partials[0..nb) (sum of slot 0, max of slot 1, sum of slot 2) into ctrl
// (one workgroup of kFinBlock threads, eight partials of each in flight at once:
// a lone workgroup waits out every load it cannot overlap)
constexpr int kFinBlock = 1024;
__global__ void __launch_bounds__(kFinBlock) k_finalize(const double* partials, int nb, Ctrl* ctrl) {
  double s = 0, s2 = 0, m = 0;
#pragma unroll 8
  for (int i = threadIdx.x; i < nb; i += kFinBlock) {
    s += partials[kPartialStride * i + 0];
    m = fmax(m, partials[kPartialStride * i + 1]);
    s2 += partials[kPartialStride * i + 2];
  }
  block_reduce3<kFinBlock>(s, s2, m);
  if (threadIdx.x == 0) {
    ctrl->sum_abs = s;
    ctrl->max_abs = m;
    ctrl->sum_abs_f32 = s2;
  }
}

// ---------------------------------------------------------------------------
// Exact residual F = B + P H - H (the identity of equations defF/defH),
// pulled over the transpose in FP64 and stored as FP32.
// general: the weights sit on the links (wh = H, each in-link multiplies its
// own weight); PageRank: every link of column i carries d / #out_i
__global__ void k_refresh_wh(int64_t n, const int32_t* __restrict__ col_ptr,
                             const double* __restrict__ h, double d, double* __restrict__ wh,
                             int general) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    int32_t k = col_ptr[i + 1] - col_ptr[i];
    if (general) wh[i] = h[i];
    else wh[i] = k > 0 ? d * h[i] / (double)k : 0.0;  // H_i spread over its column: p_ji H_i
  }
}

// Exact residual B + P H - H: blocks [0, nl) take the rows with in-degree <=
// kHeavyRow (8 lanes per row); blocks [nl, nl + n_chunks) sum one kHeavyChunk
// piece of a heavy row each into chunk_sum
template <bool W>
__global__ void __launch_bounds__(kRedBlock) k_refresh_main(
    int64_t n, int nl, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ csr_col,
    const double* __restrict__ csr_val,
    const double* __restrict__ wh, const double* __restrict__ b, const double* __restrict__ h,
    float* __restrict__ f, double* partials, const int32_t* __restrict__ chunk_beg,
    const int32_t* __restrict__ chunk_end, double* __restrict__ chunk_sum) {
  if ((int)blockIdx.x >= nl) {
    // one kHeavyChunk piece of a heavy row: eight gathers in flight per thread
    const int c = (int)blockIdx.x - nl;
    const int32_t e1 = chunk_end[c];
    double acc = 0, unused = 0, um = 0;
    constexpr int U = 8;
    for (int32_t e = chunk_beg[c] + threadIdx.x; e < e1; e += U * kRedBlock) {
      int32_t i[U];
#pragma unroll
      for (int u = 0; u < U; ++u) i[u] = e + u * kRedBlock < e1 ? csr_col[e + u * kRedBlock] : -1;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i[u] >= 0) acc += W ? csr_val[e + u * kRedBlock] * wh[i[u]] : wh[i[u]];
    }
    block_reduce3<kRedBlock>(acc, unused, um);
    if (threadIdx.x == 0) chunk_sum[c] = acc;
    return;
  }
  const int sub = threadIdx.x & 7;
  double s = 0, unused = 0, m = 0;
  const int64_t rows_per_block = kRedBlock / 8;
  for (int64_t base = blockIdx.x * rows_per_block; base < n; base += (int64_t)nl * rows_per_block) {
    const int64_t j = base + (threadIdx.x >> 3);
    bool live = false;
    double acc = 0;
    if (j < n) {
      const int32_t e0 = row_ptr[j], e1 = row_ptr[j + 1];
      live = e1 - e0 <= kHeavyRow;
      if (live)
        for (int32_t e = e0 + sub; e < e1; e += 8) acc += W ? csr_val[e] * wh[csr_col[e]] : wh[csr_col[e]];
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    if (live && sub == 0) {
      double v = b[j] - h[j] + acc;
      f[j] = (float)v;
      s += fabs(v);
      m = fmax(m, fabs(v));
    }
  }
  block_reduce3<kRedBlock>(s, unused, m);
  if (threadIdx.x == 0) {
    partials[kPartialStride * blockIdx.x + 0] = s;
    partials[kPartialStride * blockIdx.x + 1] = m;
    partials[kPartialStride * blockIdx.x + 2] = 0;
  }
}

// heavy rows: chunks are grouped by heavy row, in row order; the thread that
// holds a row's first chunk adds the row's chunk sums in chunk order
__global__ void __launch_bounds__(kRedBlock) k_refresh_heavy_fin(
    const int32_t* __restrict__ rows, const int32_t* __restrict__ chunk_h, int32_t n_chunks,
    const double* __restrict__ chunk_sum, const double* __restrict__ b, const double* __restrict__ h,
    float* __restrict__ f, double* partials) {
  double s = 0, unused = 0, m = 0;
  for (int32_t c = blockIdx.x * kRedBlock + threadIdx.x; c < n_chunks; c += gridDim.x * kRedBlock) {
    const int32_t r = chunk_h[c];
    if (c > 0 && chunk_h[c - 1] == r) continue;
    double acc = 0;
    for (int32_t k = c; k < n_chunks && chunk_h[k] == r; ++k) acc += chunk_sum[k];
    const int32_t j = rows[r];
    const double v = b[j] - h[j] + acc;
    f[j] = (float)v;
    s += fabs(v);
    m = fmax(m, fabs(v));
  }
  block_reduce3<kRedBlock>(s, unused, m);
  if (threadIdx.x == 0) {
    partials[kPartialStride * blockIdx.x + 0] = s;
    partials[kPartialStride * blockIdx.x + 1] = m;
    partials[kPartialStride * blockIdx.x + 2] = 0;
  }
}

__global__ void k_fill_double(double* p, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_reset_ctrl(Ctrl* c) {
  c->destroyed = 0;
  c->edges = c->diffusions = c->sweeps = c->idle_polls = c->passed = 0;
  c->done = 0;
  c->ticket = 0;
  c->err = 0;
  c->stages = 0;
  c->b1 = 0;
}

// start of a diffusion launch: r0 = ||F||_1 (exact), target, T0
__global__ void k_set_launch(Ctrl* c, double r0, double target, double T0) {
  c->destroyed = 0;
  c->r0 = r0;
  c->target = target;
  c->T = T0;
  c->done = 0;
  c->ticket = 0;
  c->passed = 0;
}

// ---------------------------------------------------------------------------
// Wave-level edge expansion. The 64 lanes of a wave test 64 consecutive nodes;
// the out-links of the nodes that pass are laid end to end and each lane then
// pushes every 64th of them, so the CSC column reads are coalesced and no lane
// waits on a long column of another. Index loads of UNROLL windows are issued
// before their pushes.
constexpr int kUnroll = 4;

// lane owning edge slot e: the first lane whose inclusive degree prefix exceeds e
__device__ __forceinline__ int owner_lane(int incl, int e) {
  int k = 0;
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    int v = __shfl(incl, k + s - 1, 64);
    if (v <= e) k += s;
  }
  return k;
}

// Push fluid w to target j: into LDS if j lies in [lo, lo + np), else into the
// global fluid array (the owner's inbox) with a device-scope atomic.
template <bool kLds>
__device__ __forceinline__ void push(float* Fl, float* F, int lo, int np, int j, float w) {
  if (kLds) {
    const int jl = j - lo;
    if ((unsigned)jl < (unsigned)np) {
      atomicAdd(&Fl[jl], w);  // ds_add_f32
      return;
    }
  }
  add_agent(&F[j], w);
}

// One threshold pass over the nodes [lo, lo + np) owned by this caller,
// wave chunks chunk0, chunk0 + chunk_stride, ...
// Fl / Hl: fluid and history of those nodes (LDS, or the global arrays with lo
// already applied); F: the global fluid array for targets outside the range.
template <bool kLds>
__device__ __forceinline__ void sweep_nodes(const int32_t* __restrict__ col_ptr,
                                            const int32_t* __restrict__ row_idx, float* Fl,
                                            double* Hl, float* F, int lo, int np, int chunk0,
                                            int chunk_stride, float T, float d, double& destroyed,
                                            unsigned long long& edges,
                                            unsigned long long& diffs, int& passed) {
  const int lane = threadIdx.x & 63;
  for (int base = chunk0 * 64; base < np; base += chunk_stride * 64) {
    const int i = base + lane;
    float sent = 0.f;
    int deg = 0, src0 = 0;
    if (i < np) {
      const float fi = Fl[i];
      if (fabsf(fi) > T) {
        if (kLds) sent = atomicExch(&Fl[i], 0.f);
        else sent = xchg_agent(&Fl[i], 0.f);
        Hl[i] += (double)sent;
        const int beg = col_ptr[lo + i];
        deg = col_ptr[lo + i + 1] - beg;
        src0 = beg;
        destroyed += fabs((double)sent) * (deg > 0 ? (1.0 - (double)d) : 1.0);
        edges += (unsigned long long)deg;
        diffs += 1;
        passed += 1;
      }
    }
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, 63, 64);
    if (total == 0) continue;
    const float w = deg > 0 ? sent * (d / (float)deg) : 0.f;
    const int base_off = src0 - (incl - deg);  // edge slot e of this lane reads row_idx[base_off + e]
    for (int e0 = 0; e0 < total; e0 += 64 * kUnroll) {
      int tj[kUnroll];
      float tw[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = e0 + u * 64 + lane;
        const int k = owner_lane(incl, e);
        const int off = __shfl(base_off, k, 64);
        tw[u] = __shfl(w, k, 64);
        tj[u] = e < total ? row_idx[off + e] : -1;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        if (tj[u] >= 0) push<kLds>(Fl, F, lo, np, tj[u], tw[u]);
    }
  }
}

// ---------------------------------------------------------------------------
// Persistent partitioned kernel.
struct PArgs {
  int64_t n;
  const int32_t* __restrict__ col_ptr;
  const int32_t* __restrict__ row_idx;
  const int32_t* __restrict__ part_ptr;
  float* F;
  double* H;
  Ctrl* ctrl;
  double* part_T;
  int* part_lock;
  const int* abort_flag;
  int K;
  int static_mode;
  int lds_nodes;
  int max_sweeps;
  int sweeps_per_claim;
  int max_passes;
  int xcd_remap;
  float d;
  float alpha;
  float park_ratio;
  float rescale_cap;
};

enum { kCmdSweep = 0, kCmdPark = 1, kCmdRelease = 2, kCmdExit = 3 };
constexpr int kStallPolls = 400;  // idle polls without global progress before a workgroup leaves

__device__ int claim_partition(const PArgs& a) {
  for (int tries = 0; tries < 2 * a.K + 64; ++tries) {
    if (ld_agent(&a.ctrl->done)) return -1;
    const int t = __hip_atomic_fetch_add(&a.ctrl->ticket, 1, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    if (t >= a.max_passes * a.K) return -1;
    const int p = t % a.K;
    int expect = 0;
    if (__hip_atomic_compare_exchange_strong(&a.part_lock[p], &expect, 1, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return p;
  }
  return -1;
}

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_persistent(PArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = BLOCK / 64;
  float* Fl = reinterpret_cast<float*>(smem);
  double* Hl = reinterpret_cast<double*>(smem + (((size_t)a.lds_nodes * 4 + 15) & ~(size_t)15));
  __shared__ int s_part, s_cmd;
  __shared__ float s_T;
  __shared__ double s_red[4][NW];
  __shared__ int s_redi[NW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double r0 = a.ctrl->r0, target = a.ctrl->target;
  unsigned long long my_edges = 0, my_diffs = 0;
  unsigned long long wg_sweeps = 0, wg_idle = 0;
  int claims = 0;
  int empty_claims = 0;  // consecutive claims without a sweep (dynamic binding)
  bool exit_all = false;

  while (!exit_all) {
    // ---- claim a partition
    if (tid == 0) {
      int p = -1;
      if (a.static_mode) {
        if (claims == 0) {
          p = blockIdx.x;
          if (a.xcd_remap && (gridDim.x & 7) == 0)  // workgroups go round-robin over 8 XCDs
            p = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
        }
        if (ld_agent(&a.ctrl->done)) p = -1;
      } else {
        // two passes' worth of partitions with nothing to diffuse: leave
        p = empty_claims > 2 * (a.K / (int)gridDim.x) + 8 ? -1 : claim_partition(a);
      }
      s_part = p;
    }
    __syncthreads();
    const int p = s_part;
    if (p < 0) break;
    ++claims;
    const int lo = a.part_ptr[p];
    const int np = a.part_ptr[p + 1] - lo;

    // ---- load: take the partition's fluid out of the global array into LDS
    double r = 0, mx = 0, unused = 0;
    for (int i = tid; i < np; i += BLOCK) {
      float v = ld_agent(&a.F[lo + i]);
      if (v != 0.f) v = xchg_agent(&a.F[lo + i], 0.f);
      Fl[i] = v;
      Hl[i] = 0.0;
      r += fabsf(v);
      mx = fmax(mx, (double)fabsf(v));
    }
    block_reduce3<BLOCK>(r, unused, mx);
    if (tid == 0) {
      const double Tp = a.static_mode ? -1.0 : ld_agent(&a.part_T[p]);
      s_T = Tp > 0 ? (float)Tp : (float)(mx / a.alpha);
      s_cmd = kCmdSweep;
      if (np == 0) s_cmd = a.static_mode ? kCmdExit : kCmdRelease;
      else if (!a.static_mode && r <= a.park_ratio * (r0 - ld_agent(&a.ctrl->destroyed)) *
                                            ((double)np / (double)a.n))
        s_cmd = kCmdRelease;  // nothing worth a claim here
    }
    __syncthreads();

    int sweeps_here = 0, idle_streak = 0, backoff = 1;
    double last_tot = -1.0;
    while (s_cmd == kCmdSweep || s_cmd == kCmdPark) {
      double destroyed = 0;
      int passed = 0;
      if (s_cmd == kCmdSweep) {
        sweep_nodes<true>(a.col_ptr, a.row_idx, Fl, Hl, a.F, lo, np, wave, NW, s_T, a.d,
                          destroyed, my_edges, my_diffs, passed);
        ++sweeps_here;
      } else {
        for (int s = 0; s < backoff; ++s) __builtin_amdgcn_s_sleep(127);
      }
      __syncthreads();
      // ---- drain the inbox, measure the partition's residual
      double recv = 0, rr = 0, mxx = 0;
      for (int i = tid; i < np; i += BLOCK) {
        float v = ld_agent(&a.F[lo + i]);
        float fl = Fl[i];
        if (v != 0.f) {
          v = xchg_agent(&a.F[lo + i], 0.f);
          fl += v;
          Fl[i] = fl;
          recv += fabsf(v);
        }
        rr += fabsf(fl);
        mxx = fmax(mxx, (double)fabsf(fl));
      }
      // block reduction of (destroyed, recv, rr, mxx, passed)
      destroyed = wave_sum(destroyed);
      recv = wave_sum(recv);
      rr = wave_sum(rr);
      mxx = wave_maxd(mxx);
      int pw = passed;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) pw += __shfl_xor(pw, o, 64);
      if (lane == 0) {
        s_red[0][wave] = destroyed;
        s_red[1][wave] = recv;
        s_red[2][wave] = rr;
        s_red[3][wave] = mxx;
        s_redi[wave] = pw;
      }
      __syncthreads();
      if (wave == 0) {
        const double D = wave_sum(lane < NW ? s_red[0][lane] : 0.0);
        const double R = wave_sum(lane < NW ? s_red[1][lane] : 0.0);
        const double RR = wave_sum(lane < NW ? s_red[2][lane] : 0.0);
        const double MX = wave_maxd(lane < NW ? s_red[3][lane] : 0.0);
        int PS = lane < NW ? s_redi[lane] : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) PS += __shfl_xor(PS, o, 64);
        if (lane == 0) {
        const bool swept = s_cmd == kCmdSweep;
        if (swept) ++wg_sweeps;
        double tot = D != 0 ? fetch_add_agent(&a.ctrl->destroyed, D) + D
                            : ld_agent(&a.ctrl->destroyed);
        const double rem = r0 - tot;
        int cmd;
        int done = 0;
        if (rem <= target) {
          st_agent(&a.ctrl->done, 1);
          done = 1;
        } else {
          done = ld_agent(&a.ctrl->done);
        }
        if (!done && (wg_sweeps + wg_idle) % 8 == 0 && ld_system(a.abort_flag)) {
          st_agent(&a.ctrl->done, 1);
          done = 1;
        }
        // threshold schedule (Section 2.4) and reception rescale (Section 2.6)
        float T = s_T;
        if (swept) {
          T = T / a.alpha;
          if (PS == 0 && (float)(MX / a.alpha) < T) T = (float)(MX / a.alpha);
        }
        if (R > 0) {
          const double rpre = RR - R;
          if (rpre > 0) {
            double f = (rpre + R) / rpre;
            if (f > a.rescale_cap) f = a.rescale_cap;
            T = (float)fmin((double)T * f, MX);
          } else {
            T = (float)(MX / a.alpha);
          }
        }
        s_T = T;
        const bool small = RR <= a.park_ratio * rem * ((double)np / (double)a.n);
        if (done) {
          cmd = kCmdExit;
        } else if (a.static_mode) {
          if (wg_sweeps >= (unsigned long long)a.max_sweeps) {
            cmd = kCmdExit;
          } else if (small) {
            cmd = kCmdPark;
            ++wg_idle;
            if (tot == last_tot) {
              if (++idle_streak > kStallPolls) cmd = kCmdExit;
              backoff = backoff < 4 ? backoff + 1 : 4;
            } else {
              idle_streak = 0;
              backoff = 1;
            }
            last_tot = tot;
          } else {
            cmd = kCmdSweep;
            idle_streak = 0;
            backoff = 1;
          }
        } else {
          cmd = (small || sweeps_here >= a.sweeps_per_claim) ? kCmdRelease : kCmdSweep;
        }
        s_cmd = cmd;
        }
      }
      __syncthreads();
    }
    if (s_cmd == kCmdExit) exit_all = true;
    if (tid == 0) empty_claims = sweeps_here == 0 ? empty_claims + 1 : 0;

    // ---- write back: remaining fluid to the global array, history increment to H
    for (int i = tid; i < np; i += BLOCK) {
      const float v = Fl[i];
      if (v != 0.f) add_agent(&a.F[lo + i], v);
      const double hv = Hl[i];
      if (hv != 0.0) {
        if (a.static_mode) a.H[lo + i] += hv;  // sole owner for the whole launch
        else add_agent(&a.H[lo + i], hv);
      }
    }
    if (tid == 0 && !a.static_mode) {
      __hip_atomic_store(&a.part_T[p], (double)s_T, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.part_lock[p], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }

  // ---- statistics
  my_edges = wave_sum_u64(my_edges);
  my_diffs = wave_sum_u64(my_diffs);
  if (lane == 0) {
    if (my_edges) add_agent(&a.ctrl->edges, my_edges);
    if (my_diffs) add_agent(&a.ctrl->diffusions, my_diffs);
  }
  if (tid == 0) {
    if (wg_sweeps) add_agent(&a.ctrl->sweeps, wg_sweeps);
    if (wg_idle) add_agent(&a.ctrl->idle_polls, wg_idle);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

static int finalize_partials(ditr_ctx* c, int nb) {
  k_finalize<<<1, kFinBlock, 0, c->stream>>>(c->partials, nb, c->ctrl);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

int launch_reset_ctrl(ditr_ctx* c) {
  k_reset_ctrl<<<1, 1, 0, c->stream>>>(c->ctrl);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

int launch_set_launch_target(ditr_ctx* c, double r0, double target, double T0) {
  k_set_launch<<<1, 1, 0, c->stream>>>(c->ctrl, r0, target, T0);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

int launch_fill_double(ditr_ctx* c, double* p, int64_t n, double v) {
  if (n <= 0) return DITR_OK;
  k_fill_double<<<grid_for(n, 256, 4096), 256, 0, c->stream>>>(p, n, v);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

int launch_init(ditr_ctx* c, int64_t n, const double* b, double* h, float* f) {
  const int nb = grid_for(n, 4 * kRedBlock, (int)c->partials_cap);
  k_init<<<nb, kRedBlock, 0, c->stream>>>(n, b, h, f, c->partials, &c->ctrl->err);
  HIP_TRY(hipGetLastError());
  return finalize_partials(c, nb);
}

int launch_norm_f64(ditr_ctx* c, int64_t n, const double* x) {
  const int nb = grid_for(n, kRedBlock, (int)c->partials_cap);
  k_norm_f64<<<nb, kRedBlock, 0, c->stream>>>(n, x, c->partials, &c->ctrl->err);
  HIP_TRY(hipGetLastError());
  return finalize_partials(c, nb);
}

int launch_given_start(ditr_ctx* c, int64_t n, const double* b, const double* h, const float* f) {
  const int nb = grid_for(n, kRedBlock, (int)c->partials_cap);
  k_given_start<<<nb, kRedBlock, 0, c->stream>>>(n, b, h, f, c->partials, &c->ctrl->err);
  HIP_TRY(hipGetLastError());
  return finalize_partials(c, nb);
}

int launch_check_finite(ditr_ctx* c, int64_t n, const double* x) {
  if (n <= 0) return DITR_OK;
  k_check_finite<<<grid_for(n, kRedBlock, 4096), kRedBlock, 0, c->stream>>>(n, x, &c->ctrl->err);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

int launch_refresh(ditr_ctx* c, const ditr_graph* g, const double* b, const double* h, float* f) {
  return launch_refresh_bufs(c, g, b, h, f, g->wh, g->chunk_sum);
}

// the same with the work arrays wh [n] and chunk_sum [n_chunks] given
int launch_refresh_bufs(ditr_ctx* c, const ditr_graph* g, const double* b, const double* h, float* f,
                        double* wh, double* chunk_sum) {
  const int64_t n = g->n;
  const bool general = g->csr_val != nullptr;
  k_refresh_wh<<<grid_for(n, 256, 8192), 256, 0, c->stream>>>(n, g->col_ptr, h, g->d, wh, general);
  HIP_TRY(hipGetLastError());
  // light rows and the heavy chunks in one launch, then the heavy rows from
  // their chunk sums (every sum in a fixed order)
  const int cap = (int)c->partials_cap;
  const int nf = g->n_heavy > 0 ? std::min(64, (g->n_chunks + kRedBlock - 1) / kRedBlock) : 0;
  const int nl = grid_for(n, kRedBlock / 8, cap - nf);
  const int nc = g->n_heavy > 0 ? g->n_chunks : 0;
  if (general)
    k_refresh_main<true><<<nl + nc, kRedBlock, 0, c->stream>>>(n, nl, g->row_ptr, g->csr_col, g->csr_val,
                                                               wh, b, h, f, c->partials, g->chunk_beg,
                                                               g->chunk_end, chunk_sum);
  else
    k_refresh_main<false><<<nl + nc, kRedBlock, 0, c->stream>>>(n, nl, g->row_ptr, g->csr_col, nullptr,
                                                                wh, b, h, f, c->partials, g->chunk_beg,
                                                                g->chunk_end, chunk_sum);
  HIP_TRY(hipGetLastError());
  if (nf > 0) {
    k_refresh_heavy_fin<<<nf, kRedBlock, 0, c->stream>>>(g->heavy_rows, g->chunk_h, g->n_chunks, chunk_sum,
                                                         b, h, f,
                                                         c->partials + kPartialStride * nl);
    HIP_TRY(hipGetLastError());
  }
  return finalize_partials(c, nl + nf);
}

template <int BLOCK>
static int launch_persistent_t(ditr_ctx* c, const PArgs& a, int grid, size_t lds) {
  k_persistent<BLOCK><<<grid, BLOCK, lds, c->stream>>>(a);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

// Raise the dynamic-LDS limit of one persistent instantiation as far as the
// runtime accepts (whole-CU LDS first, then the per-workgroup default).
template <int BLOCK>
static size_t configure_one(size_t cu_lds, size_t block_lds) {
  hipFuncAttributes attr;
  if (hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_persistent<BLOCK>)) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const size_t stat = attr.sharedSizeBytes;
  for (size_t total : {cu_lds, block_lds}) {
    if (total <= stat + 64) continue;
    const size_t dyn = total - stat;
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_persistent<BLOCK>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) == hipSuccess)
      return dyn;
    (void)hipGetLastError();  // clear the refused request
  }
  return block_lds > stat ? block_lds - stat : 0;
}

int persistent_configure(ditr_ctx* c, size_t cu_lds, size_t block_lds) {
  c->lds_dyn[0] = configure_one<256>(cu_lds, block_lds);
  c->lds_dyn[1] = configure_one<512>(cu_lds, block_lds);
  c->lds_dyn[2] = configure_one<1024>(cu_lds, block_lds);
  return DITR_OK;
}

int launch_persistent(ditr_ctx* c, const ditr_graph* g, float* f, double* h,
                      const PersistentCfg& cfg) {
  PArgs a;
  a.n = g->n;
  a.col_ptr = g->col_ptr;
  a.row_idx = g->row_idx;
  a.part_ptr = g->part_ptr;
  a.F = f;
  a.H = h;
  a.ctrl = c->ctrl;
  a.part_T = g->part_T;
  a.part_lock = g->part_lock;
  a.abort_flag = c->abort_dev;
  a.K = (int)g->K;
  a.static_mode = cfg.static_mode;
  a.lds_nodes = cfg.lds_nodes;
  a.max_sweeps = cfg.max_sweeps;
  a.sweeps_per_claim = cfg.sweeps_per_claim;
  a.max_passes = cfg.max_passes;
  a.xcd_remap = cfg.xcd_remap;
  a.d = (float)g->d;
  a.alpha = (float)cfg.alpha;
  a.park_ratio = (float)cfg.park_ratio;
  a.rescale_cap = (float)cfg.rescale_cap;
  switch (cfg.block) {
    case 256: return launch_persistent_t<256>(c, a, cfg.grid, cfg.lds_bytes);
    case 512: return launch_persistent_t<512>(c, a, cfg.grid, cfg.lds_bytes);
    case 1024: return launch_persistent_t<1024>(c, a, cfg.grid, cfg.lds_bytes);
    default: return set_error(DITR_EINVAL, "persistent block size must be 256, 512 or 1024");
  }
}

// workgroups of `block` threads with `lds` bytes that fit on one CU at once
int persistent_occupancy(ditr_ctx* c, int block, size_t lds, int* per_cu) {
  int nb = 0;
  hipError_t e = hipSuccess;
  switch (block) {
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<256>, 256, lds); break;
    case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<512>, 512, lds); break;
    case 1024: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<1024>, 1024, lds); break;
    default: return set_error(DITR_EINVAL, "bad block size");
  }
  HIP_TRY(e);
  *per_cu = nb;
  return DITR_OK;
}

// static LDS of the persistent kernel (the dynamic part must fit beside it)
int persistent_static_lds_impl(int block, size_t* bytes) {
  hipFuncAttributes attr;
  hipError_t e = hipSuccess;
  switch (block) {
    case 256: e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_persistent<256>)); break;
    case 512: e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_persistent<512>)); break;
    case 1024: e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_persistent<1024>)); break;
    default: return set_error(DITR_EINVAL, "bad block size");
  }
  HIP_TRY(e);
  *bytes = attr.sharedSizeBytes;
  return DITR_OK;
}
