// Cut-minimizing cost-balanced partition. Section 2.3 chooses the sets so
// that the work balances (CB) and proposes sets that keep more of the p mass
// inside them; this plan does both: it starts from CB targets and slides each
// inner boundary, within a window and a balance slack, to where the least p
// mass of short links crosses.
//
// Definition (the oracle's, step for step):
//   * node cost 1 + #out_i + min(#in_i, h), h = max(1, floor(3 L / N)): its own
//     work, its pushes, and its inflow up to h links (a row with more in-links
//     has them summed by all workgroups together); C is the cost prefix;
//   * targets t_k = min { j : K C(j) >= k C(N) };
//   * every set costs at most cB + cB / 10 and holds at most sB + sB / 10 nodes,
//     cB and sB the largest among the sets of the targets;
//   * a link i -> j (i != j) is short when |i - j| < 2 ceil(N/K) (a longer link
//     crosses some boundary wherever the boundaries sit) and weighs
//     floor(0.85 / #out_i 2^32) units; cross(b) sums the short links with
//     min(i, j) < b <= max(i, j);
//   * boundary k lies in [t_k - w_k, t_k + w_k], w_k = min(ceil(N/K) / 2, half
//     of each neighbouring target gap less one): the windows are disjoint and
//     the targets themselves are a feasible plan;
//   * no boundary lies inside a short tight cycle (a directed cycle of two or
//     three distinct nodes whose out-degrees multiply to at most 2, spanning
//     fewer than 2 ceil(N/K) ids; b is inside when min < b <= max) when a
//     plan exists without that: split across two sets, such a cycle hands its
//     fluid back one level per hop;
//   * the plan minimizes the sum of cross(b_k); among equal sums the last
//     boundary is the smallest possible, then the one before, and so on.
//
// Device plan: the costs and their scan, the targets by binary search, the
// crossing mass as a difference array (two atomics per short link, one per
// column for the end at the column's own id) and its scan, the tight cycles
// counted over each position the same way (each found from its smallest
// node, whose out-degree is 1 or 2), then a dynamic programme in one
// workgroup, one window per step: a suffix minimum (value, position) of the
// previous window, and each position of the current window takes the best
// predecessor its balance limits admit (a binary search on C). The previous
// window sits in LDS when it fits. Back-pointers hold the smallest
// predecessor among equals. The programme runs a second time, admitting
// every position, only when the first finds no plan.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "common.h"

namespace {

constexpr int kMcBlock = 1024;
constexpr long long kMcInf = 0x7fffffffffffffffLL / 4;

int mc_grid(int64_t items, int block, int64_t cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((items + block - 1) / block, cap));
}

__global__ void k_mc_cost(int64_t n, const int32_t* __restrict__ col_ptr, const int32_t* __restrict__ in_ptr,
                          long long h, long long* c) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += stride) {
    if (i == n) {
      c[n] = 0;
      continue;
    }
    const long long in = (long long)in_ptr[i + 1] - in_ptr[i];
    c[i] = 1 + ((long long)col_ptr[i + 1] - col_ptr[i]) + (in < h ? in : h);
  }
}

__global__ void k_mc_targets(int64_t n, int64_t K, const long long* __restrict__ C, long long* t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const long long total = C[n];
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= K; k += stride) {
    long long w;
    if (k == 0) w = 0;
    else if (k == K) w = n;
    else {
      int64_t lo = 0, hi = n;  // first j with K C(j) >= k C(n), in [lo, hi]
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (C[mid] * K >= k * total) hi = mid; else lo = mid + 1;
      }
      w = lo;
    }
    t[k] = w;
  }
}

// lim[0] = largest set cost, lim[1] = largest set size of the targets
__global__ void k_mc_limits(int64_t K, const long long* __restrict__ C, const long long* __restrict__ t,
                            unsigned long long* lim) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < K; k += stride) {
    atomicMax(&lim[0], (unsigned long long)(C[t[k + 1]] - C[t[k]]));
    atomicMax(&lim[1], (unsigned long long)(t[k + 1] - t[k]));
  }
}

// windows [lo_k, hi_k] and their sizes (size[K + 1] = 0 closes the scan)
__global__ void k_mc_windows(int64_t n, int64_t K, long long W, const long long* __restrict__ t, long long* lo,
                             long long* hi, long long* size) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= K + 1; k += stride) {
    if (k == K + 1) {
      size[k] = 0;
      continue;
    }
    long long a, z;
    if (k == 0) a = z = 0;
    else if (k == K) a = z = n;
    else {
      long long w = W;
      const long long gl = (t[k] - t[k - 1] - 1) / 2, gr = (t[k + 1] - t[k] - 1) / 2;
      w = gl < w ? gl : w;
      w = gr < w ? gr : w;
      w = w < 0 ? 0 : w;
      a = t[k] - w;
      z = t[k] + w;
    }
    lo[k] = a;
    hi[k] = z;
    size[k] = z - a + 1;
  }
}

// difference array of the crossing mass: diff[a + 1] += u, diff[z + 1] -= u
// for each short link between a < z (modulo 2^64; the scan gives the true
// nonnegative sums)
__global__ void k_mc_cross(int64_t n, long long span, const int32_t* __restrict__ col_ptr,
                           const int32_t* __restrict__ row_idx, unsigned long long* diff) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t e0 = col_ptr[i], e1 = col_ptr[i + 1];
    if (e1 == e0) continue;
    const unsigned long long u = (unsigned long long)floor(0.85 / (double)(e1 - e0) * 4294967296.0);
    unsigned long long own = 0;  // net change at diff[i + 1]
    for (int32_t e = e0; e < e1; ++e) {
      const int64_t r = row_idx[e];
      if (r == i) continue;
      if (r > i) {
        if (r - i >= span) continue;
        own += u;
        atomicAdd(&diff[r + 1], (unsigned long long)0 - u);
      } else {
        if (i - r >= span) continue;
        own -= u;
        atomicAdd(&diff[r + 1], u);
      }
    }
    if (own) atomicAdd(&diff[i + 1], own);
  }
}

// tight cycles: +1 at min + 1, -1 at max + 1 for each one found from its
// smallest node i (every path of CSC entries i -> j -> i or i -> j -> k -> i)
__global__ void k_mc_tight(int64_t n, long long span, const int32_t* __restrict__ col_ptr,
                           const int32_t* __restrict__ row_idx, int* tdiff) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int oi = col_ptr[i + 1] - col_ptr[i];
    if (oi < 1 || oi > 2) continue;
    for (int32_t e1 = col_ptr[i]; e1 < col_ptr[i + 1]; ++e1) {
      const int64_t j = row_idx[e1];
      const int oj = col_ptr[j + 1] - col_ptr[j];
      if (j <= i || oi * oj > 2) continue;
      for (int32_t e2 = col_ptr[j]; e2 < col_ptr[j + 1]; ++e2) {
        const int64_t k = row_idx[e2];
        if (k == i) {  // i -> j -> i
          if (j - i < span) {
            atomicAdd(&tdiff[i + 1], 1);
            atomicAdd(&tdiff[j + 1], -1);
          }
          continue;
        }
        if (k <= i || k == j) continue;
        const int ok = col_ptr[k + 1] - col_ptr[k];
        if (oi * oj * ok > 2) continue;
        for (int32_t e3 = col_ptr[k]; e3 < col_ptr[k + 1]; ++e3)
          if (row_idx[e3] == i) {  // i -> j -> k -> i
            const int64_t z = j > k ? j : k;
            if (z - i < span) {
              atomicAdd(&tdiff[i + 1], 1);
              atomicAdd(&tdiff[z + 1], -1);
            }
          }
      }
    }
  }
}

// The dynamic programme (one workgroup). Va/Vb: values of the previous and
// the current window; smv/smi: suffix minimum of the previous window (value,
// position); back: the chosen predecessor of every window position, at
// off[k] + (b - lo[k]).
__global__ void __launch_bounds__(kMcBlock) k_mc_dp(int64_t n, int64_t K, const long long* __restrict__ C,
                                                  const unsigned long long* __restrict__ cross,
                                                  const long long* __restrict__ lo, const long long* __restrict__ hi,
                                                  const long long* __restrict__ off, long long cmax, long long smax,
                                                  const int* __restrict__ tight, int keep_tight, long long* Va,
                                                  long long* Vb, long long* smv, int32_t* smi, int32_t* back,
                                                  int64_t* out64, int32_t* out32, int* err) {
  __shared__ long long s_val[kMcBlock];
  __shared__ int32_t s_pos[kMcBlock];
  const int tid = threadIdx.x;
  long long* Vp = Va;
  long long* Vc = Vb;
  if (tid == 0) Vp[0] = 0;  // window 0 is {0}
  __syncthreads();
  for (int64_t k = 1; k <= K; ++k) {
    const long long plo = lo[k - 1], pm = hi[k - 1] - plo + 1;
    // suffix minimum of the previous window: each thread a chunk, from its
    // right end (a smaller position wins a tie), then across the chunks
    const long long ch = (pm + kMcBlock - 1) / kMcBlock;
    const long long c0 = (long long)tid * ch, c1 = c0 + ch < pm ? c0 + ch : pm;
    long long bv = kMcInf;
    int32_t bp = -1;
    for (long long i = c1 - 1; i >= c0; --i) {
      const long long v = Vp[i];
      if (v <= bv) {
        bv = v;
        bp = (int32_t)(plo + i);
      }
      smv[i] = bv;
      smi[i] = bp;
    }
    s_val[tid] = bv;
    s_pos[tid] = bp;
    __syncthreads();
    for (int d = 1; d < kMcBlock; d <<= 1) {
      long long ov = kMcInf;
      int32_t op = -1;
      if (tid + d < kMcBlock) {
        ov = s_val[tid + d];
        op = s_pos[tid + d];
      }
      __syncthreads();
      if (ov < s_val[tid]) {  // strict: the left (smaller positions) keeps a tie
        s_val[tid] = ov;
        s_pos[tid] = op;
      }
      __syncthreads();
    }
    const long long rv = tid + 1 < kMcBlock ? s_val[tid + 1] : kMcInf;
    const int32_t rp = tid + 1 < kMcBlock ? s_pos[tid + 1] : -1;
    for (long long i = c0; i < c1; ++i)
      if (rv < smv[i]) {
        smv[i] = rv;
        smi[i] = rp;
      }
    __syncthreads();
    // the current window: each position's best admissible predecessor
    const long long clo = lo[k], cm = hi[k] - clo + 1, phi = hi[k - 1];
    for (long long j = tid; j < cm; j += kMcBlock) {
      const long long b = clo + j;
      long long a = b - smax > plo ? b - smax : plo, z = phi + 1;
      const long long need = C[b] - cmax;  // first q in [a, phi] with C(q) >= C(b) - cmax
      while (a < z) {
        const long long mid = (a + z) >> 1;
        if (C[mid] < need) a = mid + 1; else z = mid;
      }
      long long v = kMcInf;
      int32_t p = -1;
      if (a <= phi && !(keep_tight && k < K && tight[b] > 0)) {
        v = smv[a - plo];
        p = smi[a - plo];
      }
      Vc[j] = v >= kMcInf ? kMcInf : v + (k < K ? (long long)cross[b] : 0);
      back[off[k] + j] = v >= kMcInf ? -1 : p;
    }
    __syncthreads();
    long long* tmp = Vp;
    Vp = Vc;
    Vc = tmp;
  }
  if (tid == 0) {
    long long b = n;
    if (out64) out64[K] = n;
    if (out32) out32[K] = (int32_t)n;
    for (int64_t k = K; k >= 1; --k) {
      const int32_t q = back[off[k] + (b - lo[k])];
      if (q < 0) {
        *err = 1;
        return;
      }
      b = q;
      if (out64) out64[k - 1] = b;
      if (out32) out32[k - 1] = (int32_t)b;
    }
    if (b != 0) *err = 1;
  }
}

// (value, position) with the smaller position first among equal values
struct McMin {
  long long v;
  int32_t p;
};
__device__ __forceinline__ McMin mc_min(McMin a, McMin b) { return (b.v < a.v || (b.v == a.v && b.p < a.p)) ? b : a; }

// The same programme with the previous window staged in LDS (values, cost
// prefix, suffix-minimum positions: 20 bytes per position), for windows of at
// most `wmax` positions. The suffix minimum runs in place: each thread a chunk
// from its right end, then across the chunks with wave shuffles and one LDS
// round for the sixteen waves; the binary searches read the staged prefix.
__global__ void __launch_bounds__(kMcBlock) k_mc_dp_lds(int64_t n, int64_t K, const long long* __restrict__ C,
                                                      const unsigned long long* __restrict__ cross,
                                                      const long long* __restrict__ lo,
                                                      const long long* __restrict__ hi,
                                                      const long long* __restrict__ off, long long cmax,
                                                      long long smax, const int* __restrict__ tight, int keep_tight,
                                                      int wmax, long long* Va, long long* Vb, int32_t* back,
                                                      int64_t* out64, int32_t* out32, int* err) {
  extern __shared__ __align__(16) unsigned char mc_smem[];
  long long* sV = reinterpret_cast<long long*>(mc_smem);
  long long* sC = sV + wmax;
  int32_t* sP = reinterpret_cast<int32_t*>(sC + wmax);
  __shared__ long long w_v[kMcBlock / 64];
  __shared__ int32_t w_p[kMcBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  long long* Vp = Va;
  long long* Vc = Vb;
  if (tid == 0) Vp[0] = 0;  // window 0 is {0}
  __syncthreads();
  for (int64_t k = 1; k <= K; ++k) {
    const long long plo = lo[k - 1], phi = hi[k - 1];
    const int pm = (int)(phi - plo + 1);
    for (int i = tid; i < pm; i += kMcBlock) {
      sV[i] = Vp[i];
      sC[i] = C[plo + i];
    }
    __syncthreads();
    // suffix minimum within each thread's chunk, in place
    const int ch = (pm + kMcBlock - 1) / kMcBlock;
    const int c0 = tid * ch, c1 = c0 + ch < pm ? c0 + ch : pm;
    McMin run{kMcInf, -1};
    for (int i = c1 - 1; i >= c0; --i) {
      run = mc_min(run, McMin{sV[i], (int32_t)(plo + i)});
      sV[i] = run.v;
      sP[i] = run.p;
    }
    // minimum over the chunks to the right: inclusive suffix scan in the wave,
    // shifted by one lane, then the waves to the right
    McMin inc = run;
    for (int d = 1; d < 64; d <<= 1) {
      McMin o;
      o.v = __shfl_down(inc.v, d, 64);
      o.p = __shfl_down(inc.p, d, 64);
      if (lane + d < 64) inc = mc_min(inc, o);
    }
    McMin excl;
    excl.v = __shfl_down(inc.v, 1, 64);
    excl.p = __shfl_down(inc.p, 1, 64);
    if (lane == 63) excl = McMin{kMcInf, -1};
    if (lane == 0) {
      w_v[wave] = inc.v;
      w_p[wave] = inc.p;
    }
    __syncthreads();
    for (int w = wave + 1; w < kMcBlock / 64; ++w) excl = mc_min(excl, McMin{w_v[w], w_p[w]});
    for (int i = c0; i < c1; ++i) {
      const McMin m = mc_min(McMin{sV[i], sP[i]}, excl);
      sV[i] = m.v;
      sP[i] = m.p;
    }
    __syncthreads();
    // the current window
    const long long clo = lo[k], cm = hi[k] - clo + 1;
    for (long long j = tid; j < cm; j += kMcBlock) {
      const long long b = clo + j;
      int a = (int)((b - smax > plo ? b - smax : plo) - plo), z = pm;
      const long long need = C[b] - cmax;  // first q with C(q) >= C(b) - cmax
      while (a < z) {
        const int mid = (a + z) >> 1;
        if (sC[mid] < need) a = mid + 1; else z = mid;
      }
      long long v = kMcInf;
      int32_t q = -1;
      if (a < pm && !(keep_tight && k < K && tight[b] > 0)) {
        v = sV[a];
        q = sP[a];
      }
      Vc[j] = v >= kMcInf ? kMcInf : v + (k < K ? (long long)cross[b] : 0);
      back[off[k] + j] = v >= kMcInf ? -1 : q;
    }
    __syncthreads();
    long long* t = Vp;
    Vp = Vc;
    Vc = t;
  }
  if (tid == 0) {
    long long b = n;
    if (out64) out64[K] = n;
    if (out32) out32[K] = (int32_t)n;
    for (int64_t k = K; k >= 1; --k) {
      const int32_t q = back[off[k] + (b - lo[k])];
      if (q < 0) {
        *err = 1;
        return;
      }
      b = q;
      if (out64) out64[k - 1] = b;
      if (out32) out32[k - 1] = (int32_t)b;
    }
    if (b != 0) *err = 1;
  }
}

struct McSizes {
  size_t scan_n = 0, scan_k = 0, scan_x = 0, scan_t = 0;
};

McSizes mc_scan_sizes(int64_t n, int64_t K) {
  McSizes s;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, s.scan_n, (long long*)nullptr, (long long*)nullptr, (int)(n + 1));
  (void)hipcub::DeviceScan::InclusiveSum(nullptr, s.scan_x, (unsigned long long*)nullptr,
                                         (unsigned long long*)nullptr, (int)(n + 1));
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, s.scan_k, (long long*)nullptr, (long long*)nullptr, (int)(K + 2));
  (void)hipcub::DeviceScan::InclusiveSum(nullptr, s.scan_t, (int*)nullptr, (int*)nullptr, (int)(n + 1));
  return s;
}

}  // namespace

// K+1 boundaries of the cut-minimizing partition into out64 and/or out32
// (device). in_ptr: the in-link prefix (CSR row pointer). Synchronizes.
int launch_partition_mincut(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx,
                            const int32_t* in_ptr, int64_t K, int64_t* out64, int32_t* out32, ditr_graph* g) {
  hipStream_t st = c->stream;
  std::vector<void*> owned;
  auto alloc = [&](void** p, size_t bytes) -> bool {
    bytes = std::max<size_t>(bytes, 16);
    if ((g ? g_alloc(g, p, bytes) : hipMalloc(p, bytes)) != hipSuccess) return false;
    owned.push_back(*p);
    return true;
  };
  auto done = [&](int rc) {
    (void)hipStreamSynchronize(st);
    for (void* p : owned) {
      if (g) g_free(g, p);
      else (void)hipFree(p);
    }
    return rc;
  };
  if (n < 1 || K < 1 || K > n) return set_error(DITR_EINVAL, "need 1 <= K <= n");
  const long long h = std::max<long long>(1, 3 * (long long)nnz / n);
  const long long mean = (n + K - 1) / K, span = 2 * mean, W = mean / 2;
  const size_t win = (size_t)(2 * W + 2);
  const size_t nback = (size_t)(K + 1) * (size_t)(2 * W + 1);
  const McSizes ss = mc_scan_sizes(n, K);
  long long *cst, *C, *t, *lo, *hi, *size, *off, *Va, *Vb, *smv;
  unsigned long long *cross, *lim;
  int32_t *smi, *back;
  int *err, *tdiff, *tight;
  void *tn, *tk, *tx, *tt;
  if (!alloc((void**)&cst, 8 * (n + 1)) || !alloc((void**)&C, 8 * (n + 1)) || !alloc((void**)&cross, 8 * (n + 1)) ||
      !alloc((void**)&t, 8 * (K + 1)) || !alloc((void**)&lo, 8 * (K + 1)) || !alloc((void**)&hi, 8 * (K + 1)) ||
      !alloc((void**)&size, 8 * (K + 2)) || !alloc((void**)&off, 8 * (K + 2)) || !alloc((void**)&lim, 16) ||
      !alloc((void**)&Va, 8 * win) || !alloc((void**)&Vb, 8 * win) || !alloc((void**)&smv, 8 * win) ||
      !alloc((void**)&smi, 4 * win) || !alloc((void**)&back, 4 * nback) || !alloc((void**)&err, 4) ||
      !alloc((void**)&tdiff, 4 * (n + 1)) || !alloc((void**)&tight, 4 * (n + 1)) || !alloc(&tn, ss.scan_n) ||
      !alloc(&tk, ss.scan_k) || !alloc(&tx, ss.scan_x) || !alloc(&tt, ss.scan_t))
    return done(set_error(DITR_ENOMEM, "device allocation failed (cut-minimizing partition)"));
  size_t bn = ss.scan_n, bk = ss.scan_k, bx = ss.scan_x, bt = ss.scan_t;
  // costs, their prefix, the targets, the balance limits and the windows
  k_mc_cost<<<mc_grid(n + 1, 256, 16384), 256, 0, st>>>(n, col_ptr, in_ptr, h, cst);
  if (hipcub::DeviceScan::ExclusiveSum(tn, bn, cst, C, (int)(n + 1), st) != hipSuccess)
    return done(set_error(DITR_EHIP, "cost scan failed"));
  k_mc_targets<<<mc_grid(K + 1, 256, 4096), 256, 0, st>>>(n, K, C, t);
  if (hipMemsetAsync(lim, 0, 16, st) != hipSuccess || hipMemsetAsync(err, 0, 4, st) != hipSuccess)
    return done(set_error(DITR_EHIP, "hipMemsetAsync failed"));
  k_mc_limits<<<mc_grid(K, 256, 4096), 256, 0, st>>>(K, C, t, lim);
  k_mc_windows<<<mc_grid(K + 2, 256, 4096), 256, 0, st>>>(n, K, W, t, lo, hi, size);
  if (hipcub::DeviceScan::ExclusiveSum(tk, bk, size, off, (int)(K + 2), st) != hipSuccess)
    return done(set_error(DITR_EHIP, "window scan failed"));
  // crossing mass of every position (cst is reused as the difference array)
  unsigned long long* diff = reinterpret_cast<unsigned long long*>(cst);
  if (hipMemsetAsync(diff, 0, 8 * (n + 1), st) != hipSuccess)
    return done(set_error(DITR_EHIP, "hipMemsetAsync failed"));
  if (nnz > 0) k_mc_cross<<<mc_grid(n, 256, 16384), 256, 0, st>>>(n, span, col_ptr, row_idx, diff);
  if (hipcub::DeviceScan::InclusiveSum(tx, bx, diff, cross, (int)(n + 1), st) != hipSuccess)
    return done(set_error(DITR_EHIP, "crossing scan failed"));
  // tight cycles over every position
  if (hipMemsetAsync(tdiff, 0, 4 * (n + 1), st) != hipSuccess)
    return done(set_error(DITR_EHIP, "hipMemsetAsync failed"));
  if (nnz > 0) k_mc_tight<<<mc_grid(n, 256, 16384), 256, 0, st>>>(n, span, col_ptr, row_idx, tdiff);
  if (hipcub::DeviceScan::InclusiveSum(tt, bt, tdiff, tight, (int)(n + 1), st) != hipSuccess)
    return done(set_error(DITR_EHIP, "tight-cycle scan failed"));
  unsigned long long hl[2] = {0, 0};
  if (hipGetLastError() != hipSuccess || hipMemcpyAsync(hl, lim, 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return done(set_error(DITR_EHIP, "cut-minimizing partition setup failed"));
  const long long cmax = (long long)hl[0] + (long long)hl[0] / 10, smax = (long long)hl[1] + (long long)hl[1] / 10;
  // the previous window in LDS when it fits (20 bytes per position), else in
  // global memory
  const size_t lds = 20 * win;
  bool in_lds = lds <= 150 * 1024 &&
                hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mc_dp_lds),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
  if (!in_lds) (void)hipGetLastError();
  // first with no boundary inside a tight cycle; when that leaves no plan,
  // again with every position admitted
  int herr = 0;
  for (int keep = 1; keep >= 0; --keep) {
    if (hipMemsetAsync(err, 0, 4, st) != hipSuccess) return done(set_error(DITR_EHIP, "hipMemsetAsync failed"));
    if (in_lds)
      k_mc_dp_lds<<<1, kMcBlock, lds, st>>>(n, K, C, cross, lo, hi, off, cmax, smax, tight, keep, (int)win, Va, Vb,
                                            back, out64, out32, err);
    else
      k_mc_dp<<<1, kMcBlock, 0, st>>>(n, K, C, cross, lo, hi, off, cmax, smax, tight, keep, Va, Vb, smv, smi, back,
                                      out64, out32, err);
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return done(set_error(DITR_EHIP, "cut-minimizing partition failed"));
    if (!herr) break;
  }
  if (herr) return done(set_error(DITR_EINVAL, "cut-minimizing partition found no plan"));
  return done(DITR_OK);
}

// device bytes launch_partition_mincut takes for its temporaries (an upper
// bound, with the scans' own scratch)
// (an upper bound over every partition count in [K_min, K_max], with the
// scans' own scratch)
size_t mincut_temp_bytes(int64_t n, int64_t K_min, int64_t K_max) {
  auto al = [](size_t x) { return (std::max<size_t>(x, 16) + 255) & ~(size_t)255; };
  const McSizes ss = mc_scan_sizes(n, K_max);
  const size_t N = (size_t)n, KK = (size_t)std::max<int64_t>(K_max, 1);
  // the widest windows come with the fewest partitions
  const size_t W = ((N + (size_t)std::max<int64_t>(K_min, 1) - 1) / (size_t)std::max<int64_t>(K_min, 1)) / 2;
  // back-pointers: (K + 1)(2 w + 1) <= (K + 1)(ceil(N/K) + 1) <= 3 (N + 1) for any K in [1, N]
  return 3 * al(8 * (N + 1)) + 2 * al(4 * (N + 1)) + 3 * al(8 * (KK + 1)) + 2 * al(8 * (KK + 2)) + al(16) +
         3 * al(8 * (2 * W + 2)) + al(4 * (2 * W + 2)) + al(12 * (N + 1)) + al(4) + al(ss.scan_n) +
         al(ss.scan_k) + al(ss.scan_x) + al(ss.scan_t) + 4096;
}
