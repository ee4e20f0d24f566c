// Partition of equal internal p mass: the alternative balance Section 2.3
// proposes (make sum_{n,m in Omega_k} p_nm the same for every block).
//
// Readings (the paper gives no rule): a link i -> t weighs floor(|p_ti| 2^32)
// integer units, so block masses are exact whatever order they are summed in;
// "equal" is the contiguous K-block partition whose largest block mass t* is
// smallest, each block taking from the left as many nodes as it can while its
// mass stays <= t*; when fewer than K blocks cover the nodes the remaining
// boundaries are n.
//
// Device plan: every link becomes (hi = max(i, t), lo = min(i, t), units),
// sorted by (hi, lo). The mass node j adds to a block starting at a is then the
// sum over its group hi = j of the links with lo >= a: a binary search in the
// group and a difference of the prefix sums S. A greedy scan for one bound t
// runs in one workgroup over chunks of 1024 nodes: a block-wide scan of the
// increments finds where the running mass first exceeds t, the block closes
// there and the scan resumes after it. t* is found by rounds of 256 bounds
// probed at once (one workgroup each), narrowing the integer interval about
// 255-fold per round, then the exact minimum in a last exhaustive round.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "common.h"

namespace {

constexpr int kProbeBlock = 1024;
constexpr int kProbes = 256;
constexpr long long kNone = 0x7fffffffffffffffLL;

__global__ void k_pm_links(int64_t n, const int32_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
                           const double* __restrict__ val, double d, unsigned long long* key,
                           unsigned long long* w) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t e0 = col_ptr[i], e1 = col_ptr[i + 1];
    for (int32_t e = e0; e < e1; ++e) {
      const int64_t t = row_idx[e];
      const double p = val ? fabs(val[e]) : d / (double)(e1 - e0);
      w[e] = (unsigned long long)floor(p * 4294967296.0);
      const int64_t hi = t > i ? t : i, lo = t > i ? i : t;
      key[e] = ((unsigned long long)hi << 32) | (unsigned long long)lo;
    }
  }
}

// gbeg[j] = first sorted link with hi >= j (j = 0..n)
__global__ void k_pm_groups(int64_t n, int64_t nnz, const unsigned long long* __restrict__ key, int32_t* gbeg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= n; j += stride) {
    const unsigned long long k = (unsigned long long)j << 32;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (key[mid] < k) lo = mid + 1; else hi = mid;
    }
    gbeg[j] = (int32_t)lo;
  }
}

// mass of the links of group j whose lower end is >= a: S[end] - S[first lo >= a]
__device__ __forceinline__ unsigned long long pm_inc(const unsigned long long* __restrict__ key,
                                                     const unsigned long long* __restrict__ S,
                                                     const int32_t* __restrict__ gbeg, int64_t j, int64_t a) {
  int32_t lo = gbeg[j], hi = gbeg[j + 1];
  const int32_t end = hi;
  const unsigned long long k = ((unsigned long long)j << 32) | (unsigned long long)a;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (key[mid] < k) lo = mid + 1; else hi = mid;
  }
  return S[end] - S[lo];
}

// largest self-link mass of one node (a block of one node holds at least that)
__global__ void k_pm_selfmax(int64_t n, const unsigned long long* __restrict__ key,
                             const unsigned long long* __restrict__ S, const int32_t* __restrict__ gbeg,
                             unsigned long long* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long m = 0;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += stride)
    m = max(m, pm_inc(key, S, gbeg, j, j));
  if (m) atomicMax(out, m);
}

// inclusive block scan of 64-bit values over kProbeBlock threads; returns the
// total in *total (valid in every thread)
__device__ __forceinline__ unsigned long long block_scan_u64(unsigned long long v, unsigned long long* sh,
                                                             unsigned long long* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kProbeBlock / 64;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  unsigned long long off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const unsigned long long x = sh[w];
    if (w < wave) off += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return v + off;
}

__device__ __forceinline__ long long block_min_ll(long long v, long long* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kProbeBlock / 64;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (long long)__shfl_xor(v, o, 64));
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  long long m = kNone;
#pragma unroll
  for (int w = 0; w < NW; ++w) m = min(m, sh[w]);
  __syncthreads();
  return m;
}

// One workgroup per bound tcand[blockIdx.x]: the greedy scan. nblocks gets the
// number of blocks it needs (stopping once it exceeds K unless the boundaries
// are wanted); b64 / b32 (one workgroup) get the K+1 boundaries.
__global__ void __launch_bounds__(kProbeBlock) k_pm_probe(int64_t n, int64_t K,
                                                          const unsigned long long* __restrict__ key,
                                                          const unsigned long long* __restrict__ S,
                                                          const int32_t* __restrict__ gbeg,
                                                          const unsigned long long* __restrict__ tcand,
                                                          long long* nblocks, int64_t* b64, int32_t* b32) {
  __shared__ unsigned long long sh_scan[kProbeBlock / 64];
  __shared__ long long sh_min[kProbeBlock / 64];
  const unsigned long long t = tcand[blockIdx.x];
  const bool want = b64 != nullptr || b32 != nullptr;
  int64_t a = 0, j0 = 0, blocks = 1;
  unsigned long long cur = 0;
  if (threadIdx.x == 0) {
    if (b64) b64[0] = 0;
    if (b32) b32[0] = 0;
  }
  while (j0 < n) {
    const int64_t j = j0 + threadIdx.x;
    const unsigned long long inc = j < n ? pm_inc(key, S, gbeg, j, a) : 0ull;
    unsigned long long total;
    const unsigned long long incl = block_scan_u64(inc, sh_scan, &total);
    const long long cand = (j < n && j > a && cur + incl > t) ? (long long)j : kNone;
    const long long js = block_min_ll(cand, sh_min);
    if (js == kNone) {
      cur += total;
      j0 += kProbeBlock;
      continue;
    }
    // close [a, js); js starts the next block with its own self-links
    ++blocks;
    if (want && blocks - 1 <= K && threadIdx.x == 0) {
      if (b64) b64[blocks - 1] = js;
      if (b32) b32[blocks - 1] = (int32_t)js;
    }
    if (!want && blocks > K) break;
    a = js;
    cur = pm_inc(key, S, gbeg, js, js);
    j0 = js + 1;
  }
  if (threadIdx.x == 0) {
    nblocks[blockIdx.x] = blocks;
    for (int64_t k = blocks; k <= K; ++k) {
      if (b64) b64[k] = n;
      if (b32) b32[k] = (int32_t)n;
    }
  }
}

int grid_for(int64_t n, int block, int cap) {
  int64_t g = (n + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

// K+1 boundaries of the equal-internal-mass partition into out64 and/or out32
// (device). val = nullptr: PageRank weights d / #out_i. Synchronizes.
int launch_partition_pmass(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* col_ptr,
                           const int32_t* row_idx, const double* val, double d, int64_t K,
                           int64_t* out64, int32_t* out32, ditr_graph* g) {
  hipStream_t st = c->stream;
  std::vector<void*> owned;
  // temporaries: the graph's own memory when there is a graph (its workspace
  // for an uploaded one), else hipMalloc
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
  const size_t L = (size_t)std::max<int64_t>(nnz, 1);
  unsigned long long *key0, *key1, *w0, *w1, *S, *tc, *smax;
  long long* nb;
  int32_t* gbeg;
  if (!alloc((void**)&key0, 8 * L) || !alloc((void**)&key1, 8 * L) || !alloc((void**)&w0, 8 * L) ||
      !alloc((void**)&w1, 8 * L) || !alloc((void**)&S, 8 * (L + 1)) || !alloc((void**)&gbeg, 4 * (n + 1)) ||
      !alloc((void**)&tc, 8 * kProbes) || !alloc((void**)&nb, 8 * kProbes) || !alloc((void**)&smax, 8))
    return done(set_error(DITR_ENOMEM, "device allocation failed (internal-mass partition)"));
  if (nnz > 0) {
    k_pm_links<<<grid_for(n, 256, 16384), 256, 0, st>>>(n, col_ptr, row_idx, val, d, key0, w0);
    size_t tb = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key0, key1, w0, w1, (int)nnz, 0, 63, st) != hipSuccess)
      return done(set_error(DITR_EHIP, "radix sort size query failed"));
    void* temp = nullptr;
    if (!alloc(&temp, tb)) return done(set_error(DITR_ENOMEM, "device allocation failed (sort)"));
    if (hipcub::DeviceRadixSort::SortPairs(temp, tb, key0, key1, w0, w1, (int)nnz, 0, 63, st) != hipSuccess)
      return done(set_error(DITR_EHIP, "radix sort failed"));
    size_t sb = 0;
    if (hipcub::DeviceScan::InclusiveSum(nullptr, sb, w1, S + 1, (int)nnz, st) != hipSuccess)
      return done(set_error(DITR_EHIP, "scan size query failed"));
    void* stemp = nullptr;
    if (!alloc(&stemp, sb)) return done(set_error(DITR_ENOMEM, "device allocation failed (scan)"));
    if (hipcub::DeviceScan::InclusiveSum(stemp, sb, w1, S + 1, (int)nnz, st) != hipSuccess)
      return done(set_error(DITR_EHIP, "scan failed"));
  }
  if (hipMemsetAsync(S, 0, 8, st) != hipSuccess || hipMemsetAsync(smax, 0, 8, st) != hipSuccess)
    return done(set_error(DITR_EHIP, "hipMemsetAsync failed"));
  k_pm_groups<<<grid_for(n + 1, 256, 16384), 256, 0, st>>>(n, nnz, key1, gbeg);
  k_pm_selfmax<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, key1, S, gbeg, smax);
  unsigned long long lo = 0, hi = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&lo, smax, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&hi, S + std::max<int64_t>(nnz, 0), 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return done(set_error(DITR_EHIP, "internal-mass partition setup failed"));
  if (hi < lo) hi = lo;
  // t* = the least bound whose greedy scan needs <= K blocks (hi, the whole
  // mass, always does)
  std::vector<unsigned long long> cand;
  std::vector<long long> got(kProbes);
  for (;;) {
    cand.clear();
    const unsigned long long span = hi - lo;
    const bool exhaustive = span < (unsigned long long)kProbes;
    if (exhaustive) {
      for (unsigned long long x = lo; x <= hi; ++x) cand.push_back(x);
    } else {
      const unsigned long long step = span / (kProbes - 1);
      for (int p = 0; p < kProbes - 1; ++p) cand.push_back(lo + step * (unsigned long long)p);
      cand.push_back(hi);
    }
    const int np = (int)cand.size();
    if (hipMemcpyAsync(tc, cand.data(), 8 * np, hipMemcpyHostToDevice, st) != hipSuccess)
      return done(set_error(DITR_EHIP, "hipMemcpyAsync failed"));
    k_pm_probe<<<np, kProbeBlock, 0, st>>>(n, K, key1, S, gbeg, tc, nb, nullptr, nullptr);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(got.data(), nb, 8 * np, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return done(set_error(DITR_EHIP, "internal-mass probe failed"));
    int first_ok = np - 1;
    for (int p = 0; p < np; ++p)
      if (got[p] <= K) {
        first_ok = p;
        break;
      }
    if (exhaustive) {
      lo = hi = cand[first_ok];
      break;
    }
    hi = cand[first_ok];
    if (first_ok > 0) lo = cand[first_ok - 1] + 1;
    if (lo >= hi) {
      lo = hi;
      break;
    }
  }
  if (hipMemcpyAsync(tc, &lo, 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return done(set_error(DITR_EHIP, "hipMemcpyAsync failed"));
  k_pm_probe<<<1, kProbeBlock, 0, st>>>(n, K, key1, S, gbeg, tc, nb, out64, out32);
  if (hipGetLastError() != hipSuccess) return done(set_error(DITR_EHIP, "internal-mass boundaries failed"));
  return done(DITR_OK);
}

// device bytes launch_partition_pmass takes for its temporaries (an upper
// bound, with the radix sort's and the scan's own scratch)
size_t pmass_temp_bytes(int64_t n, int64_t nnz) {
  auto al = [](size_t x) { return (std::max<size_t>(x, 16) + 255) & ~(size_t)255; };
  const size_t L = (size_t)std::max<int64_t>(nnz, 1);
  size_t tb = 0, sb = 0;
  if (nnz > 0) {
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                             (unsigned long long*)nullptr, (unsigned long long*)nullptr, (int)nnz,
                                             0, 63);
    (void)hipcub::DeviceScan::InclusiveSum(nullptr, sb, (unsigned long long*)nullptr,
                                           (unsigned long long*)nullptr, (int)nnz);
  }
  return 4 * al(8 * L) + al(8 * (L + 1)) + al(4 * ((size_t)n + 1)) + 2 * al(8 * kProbes) + al(8) + al(tb) +
         al(sb) + 4096;
}
