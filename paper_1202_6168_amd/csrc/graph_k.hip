// Graph preparation kernels: CSC validation, the CSR transpose used by the
// exact residual, and the partition plan of Section 2.3 (uniform and
// cost-balanced node ranges).
#include <string.h>

#include "common.h"

namespace {

constexpr int kBlock = 256;

int grid_for(int64_t n, int block, int cap = 65536) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// err bits: 1 col_ptr[0] != 0 or col_ptr[n] != nnz, 2 col_ptr decreasing, 4 row out of range
__global__ void k_validate_ptr(int64_t n, int64_t nnz, const int32_t* __restrict__ col_ptr,
                               int* err) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
    if (col_ptr[i + 1] < col_ptr[i]) atomicOr(err, 2);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    if (col_ptr[0] != 0 || (int64_t)col_ptr[n] != nnz) atomicOr(err, 1);
}

__global__ void k_validate_rows(int64_t n, int64_t nnz, const int32_t* __restrict__ row_idx,
                                int* err) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride) {
    int32_t r = row_idx[e];
    if (r < 0 || (int64_t)r >= n) atomicOr(err, 4);
  }
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

__global__ void k_count_in(int64_t nnz, const int32_t* __restrict__ row_idx, int32_t* cnt) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride)
    atomicAdd(&cnt[row_idx[e]], 1);
}

// ---- exclusive scan of int32 counts: out[0..n] with out[n] = total ----------
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ int block_excl_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = wave_incl_scan(v);
  if (lane == 63) sh[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    int s = lane < nw ? sh[lane] : 0;
    int si = wave_incl_scan(s);
    if (lane < nw) sh[lane] = si - s;
    if (lane == nw - 1) sh[32] = si;
  }
  __syncthreads();
  int r = sh[wave] + incl - v;
  *total = sh[32];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(const int32_t* in, int64_t n,
                                                            int32_t* tile_sums) {
  __shared__ int sh[40];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in[base + k];
  int tot;
  block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// single workgroup: exclusive scan of the tile sums in place
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int32_t* sums, int64_t ntiles) {
  __shared__ int sh[40];
  int carry = 0;
  for (int64_t base = 0; base < ntiles; base += kScanBlock) {
    int64_t i = base + threadIdx.x;
    int v = i < ntiles ? sums[i] : 0;
    int tot;
    int ex = block_excl_scan(v, sh, &tot);
    if (i < ntiles) sums[i] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const int32_t* in, int64_t n,
                                                            const int32_t* tile_off,
                                                            int32_t* out) {
  __shared__ int sh[40];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  int tot;
  int ex = block_excl_scan(s, sh, &tot) + tile_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (base + kScanItems >= n && base < n) out[n] = ex;  // the thread holding the last item
}

// cursor[j] starts at row_ptr[j]; every CSC entry (j in column i) lands in row j
// (with its weight, for a general matrix)
__global__ void k_fill_csr(int64_t n, const int32_t* __restrict__ col_ptr,
                           const int32_t* __restrict__ row_idx, const double* __restrict__ val,
                           int32_t* cursor, int32_t* csr_col, double* csr_val) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
    for (int32_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) {
      int32_t pos = atomicAdd(&cursor[row_idx[e]], 1);
      csr_col[pos] = (int32_t)i;
      if (val) csr_val[pos] = val[e];
    }
}

// General matrix: colabs[i] = sum |p_ji| over column i, the largest of them
// (the contraction factor of the bound ||X - H||_1 <= ||F||_1 / (1 - c),
// Section 2) as the bits of a non-negative double, err = 1 for a NaN or Inf.
__global__ void k_col_abs(int64_t n, const int32_t* __restrict__ col_ptr, const double* __restrict__ val,
                          double* colabs, unsigned long long* max_bits, int* err) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long m = 0;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    double s = 0;
    for (int32_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) {
      bad |= !isfinite(val[e]);
      s += fabs(val[e]);
    }
    colabs[i] = s;
    if (isfinite(s)) m = max(m, (unsigned long long)__double_as_longlong(s));
  }
  if (bad) atomicOr(err, 1);
  if (m) atomicMax(max_bits, m);
}

__global__ void k_heavy_rows(int64_t n, const int32_t* __restrict__ row_ptr, int32_t* list,
                             int* count) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += stride)
    if (row_ptr[j + 1] - row_ptr[j] > kHeavyRow) list[atomicAdd(count, 1)] = (int32_t)j;
}

// Partition boundaries (Section 2.3). Uniform: omega_k = k floor(n/K), omega_K = n.
// Cost-balanced: omega_k = min { j in [0, n] : K cost(j) >= k cost(n) } with
// cost(j) the out-link prefix col_ptr[j] (CB, the paper's rule) or the in+out
// prefix col_ptr[j] + row_ptr[j] (CB_INOUT, a balance on all links a partition
// touches, after the alternative balance the paper proposes). Binary search.
__global__ void k_partition(int64_t n, const int32_t* __restrict__ col_ptr,
                            const int32_t* __restrict__ row_ptr, int type, int64_t K,
                            int64_t* out64, int32_t* out32) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool inout = type == DITR_PART_CB_INOUT;
  const int64_t L = (int64_t)col_ptr[n] + (inout ? (int64_t)row_ptr[n] : 0);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= K; k += stride) {
    int64_t w;
    if (k == 0) w = 0;
    else if (k == K) w = n;
    else if (type == DITR_PART_UNIFORM) w = k * (n / K);
    else {
      int64_t lo = 0, hi = n;  // answer in [lo, hi]
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        const int64_t cost = (int64_t)col_ptr[mid] + (inout ? (int64_t)row_ptr[mid] : 0);
        if (cost * K >= k * L) hi = mid; else lo = mid + 1;
      }
      w = lo;
    }
    if (out64) out64[k] = w;
    if (out32) out32[k] = (int32_t)w;
  }
}

}  // namespace

int launch_validate_csc(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* col_ptr,
                        const int32_t* row_idx) {
  int* err = &c->ctrl->err;
  HIP_TRY(hipMemsetAsync(err, 0, sizeof(int), c->stream));
  k_validate_ptr<<<grid_for(n, kBlock), kBlock, 0, c->stream>>>(n, nnz, col_ptr, err);
  HIP_TRY(hipGetLastError());
  if (nnz > 0) {
    k_validate_rows<<<grid_for(nnz, kBlock), kBlock, 0, c->stream>>>(n, nnz, row_idx, err);
    HIP_TRY(hipGetLastError());
  }
  return DITR_OK;
}

int scan_exclusive_i32(ditr_ctx* c, const int32_t* in, int64_t n, int32_t* out, ditr_graph* g) {
  int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles < 1) ntiles = 1;
  int32_t* sums = nullptr;
  HIP_TRY(g ? g_alloc(g, (void**)&sums, sizeof(int32_t) * ntiles) : hipMalloc((void**)&sums, sizeof(int32_t) * ntiles));
  k_scan_tiles<<<(unsigned)ntiles, kScanBlock, 0, c->stream>>>(in, n, sums);
  k_scan_sums<<<1, kScanBlock, 0, c->stream>>>(sums, ntiles);
  k_scan_apply<<<(unsigned)ntiles, kScanBlock, 0, c->stream>>>(in, n, sums, out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (g) g_free(g, sums);
  else (void)hipFree(sums);
  HIP_TRY(e);
  if (n == 0) HIP_TRY(hipMemsetAsync(out, 0, sizeof(int32_t), c->stream));
  return DITR_OK;
}

int launch_build_transpose(ditr_ctx* c, ditr_graph* g) {
  const int64_t n = g->n, nnz = g->nnz;
  int32_t* cnt = nullptr;
  HIP_TRY(g_alloc(g, (void**)&cnt, sizeof(int32_t) * (n + 1)));
  k_zero_i32<<<grid_for(n + 1, kBlock), kBlock, 0, c->stream>>>(cnt, n + 1);
  if (nnz > 0) k_count_in<<<grid_for(nnz, kBlock), kBlock, 0, c->stream>>>(nnz, g->row_idx, cnt);
  int rc = scan_exclusive_i32(c, cnt, n, g->row_ptr, g);
  if (rc) {
    g_free(g, cnt);
    return rc;
  }
  // cnt becomes the fill cursor
  HIP_TRY(hipMemcpyAsync(cnt, g->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice,
                         c->stream));
  if (n > 0)
    k_fill_csr<<<grid_for(n, kBlock), kBlock, 0, c->stream>>>(n, g->col_ptr, g->row_idx, g->val, cnt,
                                                              g->csr_col, g->csr_val);
  int* hcount = &c->ctrl->err;
  HIP_TRY(hipMemsetAsync(hcount, 0, sizeof(int), c->stream));
  if (n > 0)
    k_heavy_rows<<<grid_for(n, kBlock), kBlock, 0, c->stream>>>(n, g->row_ptr, g->heavy_rows,
                                                                hcount);
  int hc = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&hc, hcount, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  g_free(g, cnt);
  HIP_TRY(e);
  g->n_heavy = hc;
  return DITR_OK;
}

int launch_partition(ditr_ctx* c, int64_t n, const int32_t* col_ptr, const int32_t* row_ptr,
                     int part_type, int64_t K, int64_t* out64, int32_t* out32) {
  k_partition<<<grid_for(K + 1, kBlock), kBlock, 0, c->stream>>>(n, col_ptr, row_ptr, part_type, K,
                                                                   out64, out32);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

// in-link prefix (CSR row pointer) of a CSC graph, for a standalone CB_INOUT plan
int launch_in_prefix(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* row_idx, int32_t* out) {
  int32_t* cnt = nullptr;
  HIP_TRY(hipMalloc((void**)&cnt, sizeof(int32_t) * (n + 1)));
  k_zero_i32<<<grid_for(n + 1, kBlock), kBlock, 0, c->stream>>>(cnt, n + 1);
  if (nnz > 0) k_count_in<<<grid_for(nnz, kBlock), kBlock, 0, c->stream>>>(nnz, row_idx, cnt);
  int rc = scan_exclusive_i32(c, cnt, n, out);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(cnt);
  return rc;
}

// column l1 norms of a general matrix into g->colabs; the largest into *h_max
// and 1 into *h_bad if a weight is NaN or Inf. Synchronizes.
int launch_col_abs(ditr_ctx* c, ditr_graph* g, double* h_max, int* h_bad) {
  int* err = &c->ctrl->err;
  unsigned long long* mx = reinterpret_cast<unsigned long long*>(&c->ctrl->max_abs);
  HIP_TRY(hipMemsetAsync(err, 0, sizeof(int), c->stream));
  HIP_TRY(hipMemsetAsync(mx, 0, sizeof(unsigned long long), c->stream));
  k_col_abs<<<grid_for(g->n, kBlock), kBlock, 0, c->stream>>>(g->n, g->col_ptr, g->val, g->colabs, mx, err);
  HIP_TRY(hipGetLastError());
  unsigned long long bits = 0;
  int bad = 0;
  HIP_TRY(hipMemcpyAsync(&bits, mx, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double m;
  memcpy(&m, &bits, sizeof(m));
  *h_max = m;
  *h_bad = bad;
  return DITR_OK;
}
