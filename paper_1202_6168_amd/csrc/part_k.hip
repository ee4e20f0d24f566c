// Partitioned sweep: the K-PID scheme of Sections 2.3-2.6 with one
// workgroup per node range Omega_k and a synchronous exchange per launch.
//
// One launch ("macro sweep"), for every partition Omega_k in parallel:
//   1. load F of Omega_k into LDS and add the fluid that outside sources sent
//      during the previous launch: for an external in-link i -> j the amount is
//      p_ji times the increment of H_i over that launch (Section 2.5: external
//      fluid is the diffusion of the increment of H since the last exchange);
//   2. run m threshold sweeps inside Omega_k (local diffusion, algorithm (*) of
//      Section 2.5): diffuse every node with |F_i| > T, push only to targets in
//      Omega_k (LDS atomics), lower T by alpha after each sweep (Section 2.4);
//   3. write F back, add the increment dH_i to H_i and publish p_i dH_i for the
//      outside targets of i, read by step 1 of the next launch.
// Outside fluid is pulled, never pushed: no atomics on the fluid arrays. Heavy
// rows (many external in-links) get their inflow from chunk workgroups one
// launch later, as in the pull sweep.
//
// Graph preprocessing (partition ids, the local CSC with 16-bit local targets,
// the external in-link lists) is built once per graph.
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace {

constexpr int kPB = 1024;     // threads per partition workgroup
constexpr int kStride = 8;    // doubles per block in the partials (sums, abort vote)
constexpr int kCounters = 8;  // launch finish count, level arrivals of the resident sweep

int grid_for(int64_t n, int block, int cap) {
  int64_t g = (n + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// ---------------------------------------------------------------- preprocessing
__global__ void k_fill_pid(int K, const int32_t* __restrict__ part_ptr, int32_t* pid) {
  for (int k = blockIdx.x; k < K; k += gridDim.x)
    for (int32_t j = part_ptr[k] + threadIdx.x; j < part_ptr[k + 1]; j += blockDim.x) pid[j] = k;
}

// per column: number of out-links whose target lies in the same partition
__global__ void k_count_local(int64_t n, const int32_t* __restrict__ col_ptr,
                              const int32_t* __restrict__ row_idx, const int32_t* __restrict__ pid,
                              int32_t* cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    int c = 0;
    const int32_t pi = pid[i];
    for (int32_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) c += pid[row_idx[e]] == pi;
    cnt[i] = c;
  }
}

// sort keys of the visiting order: partition, then falling local out-degree
__global__ void k_order_keys(int64_t n, const int32_t* __restrict__ pid, const int32_t* __restrict__ cnt,
                             unsigned long long* key, int32_t* val) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    key[i] = ((unsigned long long)(uint32_t)pid[i] << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)cnt[i]);
    val[i] = (int32_t)i;
  }
}

// from the sorted order: each node's local id, and the local out-degrees in
// visiting order (partitions are contiguous ranges, so position j of the sort
// lies in the partition of the node it holds)
__global__ void k_inv(int64_t n, const int32_t* __restrict__ ord, const int32_t* __restrict__ pid,
                      const int32_t* __restrict__ part_ptr, const int32_t* __restrict__ cnt, uint16_t* inv,
                      int32_t* degp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += stride) {
    const int32_t i = ord[j];
    inv[i] = (uint16_t)(j - part_ptr[pid[i]]);
    degp[j] = cnt[i];
  }
}

// local targets of node i, as local ids, at the position of i's local id
__global__ void k_fill_local(int64_t n, const int32_t* __restrict__ col_ptr,
                             const int32_t* __restrict__ row_idx, const int32_t* __restrict__ pid,
                             const int32_t* __restrict__ part_ptr, const uint16_t* __restrict__ inv,
                             const int32_t* __restrict__ loc_ptr, uint16_t* loc_idx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t pi = pid[i];
    int32_t w = loc_ptr[part_ptr[pi] + inv[i]];
    for (int32_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) {
      const int32_t j = row_idx[e];
      if (pid[j] == pi) loc_idx[w++] = inv[j];
    }
  }
}

// largest number of local targets of one partition
__global__ void k_part_max_edges(int K, const int32_t* __restrict__ part_ptr, const int32_t* __restrict__ loc_ptr,
                                 int32_t* mx) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x)
    atomicMax(mx, loc_ptr[part_ptr[k + 1]] - loc_ptr[part_ptr[k]]);
}

// per row: external in-links, split into light (partition stream) and heavy
// (chunk kernel). One wave per row, so hub rows do not serialize one thread.
__global__ void k_count_ext(int64_t n, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ csr_col, const int32_t* __restrict__ pid,
                            int32_t* light_cnt, int32_t* heavy_cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t j = wid; j < n; j += nw) {
    const int32_t pj = pid[j];
    int c = 0;
    for (int32_t e = row_ptr[j] + lane; e < row_ptr[j + 1]; e += 64) c += pid[csr_col[e]] != pj;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (lane == 0) {
      const bool heavy = c > kPartHeavy;
      light_cnt[j] = heavy ? 0 : c;
      heavy_cnt[j] = heavy ? c : 0;
    }
  }
}

__global__ void k_fill_ext(int64_t n, const int32_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ csr_col, const int32_t* __restrict__ pid,
                           const uint16_t* __restrict__ inv,
                           const int32_t* __restrict__ light_ptr, const int32_t* __restrict__ heavy_ptr,
                           int32_t* ext_src, uint16_t* ext_row, int32_t* heavy_src) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t j = wid; j < n; j += nw) {
    const int32_t pj = pid[j];
    const bool heavy = heavy_ptr[j + 1] > heavy_ptr[j];
    int32_t w = heavy ? heavy_ptr[j] : light_ptr[j];
    const uint16_t jl = inv[j];  // the row's local id
    const int32_t r1 = row_ptr[j + 1];
    for (int32_t e0 = row_ptr[j]; e0 < r1; e0 += 64) {  // wave-wide, in CSR order
      const int32_t e = e0 + lane;
      int32_t i = -1;
      bool ext = false;
      if (e < r1) {
        i = csr_col[e];
        ext = pid[i] != pj;
      }
      const unsigned long long m = __ballot(ext);
      if (ext) {
        const int32_t pos = w + __popcll(m & ((1ull << lane) - 1ull));
        if (heavy) heavy_src[pos] = i;
        else {
          ext_src[pos] = i;
          ext_row[pos] = jl;
        }
      }
      w += __popcll(m);
    }
  }
}

__global__ void k_gather_ptr(int K, const int32_t* __restrict__ part_ptr,
                             const int32_t* __restrict__ row_scan, int32_t* out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= K; k += gridDim.x * blockDim.x)
    out[k] = row_scan[part_ptr[k]];
}

// out[k] = idx[ptr[k]]: the start of partition k's range in a list indexed by
// a position of ptr
__global__ void k_gather_ptr2(int K, const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                              int32_t* out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= K; k += gridDim.x * blockDim.x) out[k] = idx[ptr[k]];
}

__global__ void k_heavy_flag(int64_t n, const int32_t* __restrict__ heavy_ptr, int32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += stride)
    flag[j] = heavy_ptr[j + 1] > heavy_ptr[j];
}

__global__ void k_heavy_rows(int64_t n, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                             int32_t* rows) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += stride)
    if (flag[j]) rows[pos[j]] = (int32_t)j;
}

// items of kItem links per heavy row
__global__ void k_item_count(int32_t nh, const int32_t* __restrict__ rows, const int32_t* __restrict__ heavy_ptr,
                             int32_t* cnt) {
  for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += gridDim.x * blockDim.x) {
    const int32_t r = rows[h];
    cnt[h] = (heavy_ptr[r + 1] - heavy_ptr[r] + kItem - 1) / kItem;
  }
}

// lanes of an item's group: 2^l, the fewest whose eight slots hold its links
__device__ __forceinline__ int item_lg2(int32_t links) {
  int l = 0;
  while ((8 << l) < links) ++l;
  return l;
}

// every item: its row (local id), link range, and its size class (6 - log2 of
// its lanes, so an ascending sort puts the largest groups first)
__global__ void k_item_fill(int32_t nh, const int32_t* __restrict__ rows, const int32_t* __restrict__ heavy_ptr,
                            const int32_t* __restrict__ ioff, const uint16_t* __restrict__ inv, int32_t* item_row,
                            int32_t* ibeg, int32_t* iend, uint32_t* ikey, int32_t* ival) {
  for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += gridDim.x * blockDim.x) {
    const int32_t r = rows[h], b0 = heavy_ptr[r], b1 = heavy_ptr[r + 1];
    int32_t idx = ioff[h];
    for (int32_t b = b0; b < b1; b += kItem, ++idx) {
      const int32_t e = min(b + kItem, b1);
      item_row[idx] = inv[r];
      ibeg[idx] = b;
      iend[idx] = e;
      ikey[idx] = (uint32_t)(6 - item_lg2(e - b));
      ival[idx] = idx;
    }
  }
}

__global__ void k_unit_lanes(int32_t ni, const int32_t* __restrict__ by, const int32_t* __restrict__ ibeg,
                             const int32_t* __restrict__ iend, int32_t* gl) {
  for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < ni; j += gridDim.x * blockDim.x) {
    const int32_t k = by[j];
    gl[j] = 1 << item_lg2(iend[k] - ibeg[k]);
  }
}

// sorted item j (item by[j]) takes lanes loff[j] .. loff[j] + gl of the unit
// table: lane l of its group sums slots l, l + gl, ..., l + 7 gl of its links;
// the leader's meta word names the item
__global__ void k_unit_fill(int32_t ni, const int32_t* __restrict__ by, const int32_t* __restrict__ loff,
                            const int32_t* __restrict__ ibeg, const int32_t* __restrict__ iend,
                            const int32_t* __restrict__ hsrc, int32_t* usrc, int32_t* umeta) {
  for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < ni; j += gridDim.x * blockDim.x) {
    const int32_t k = by[j], L = loff[j];
    const int32_t gl = loff[j + 1] - L;
    const int lg = __builtin_ctz((unsigned)gl);
    const int64_t u = L >> 6;
    const int lane = L & 63;
    for (int l = 0; l < gl; ++l) {
      umeta[u * 64 + lane + l] = ((l == 0 ? k + 1 : 0) << 3) | lg;
      for (int qq = 0; qq < 8; ++qq) {
        const int32_t e = ibeg[k] + l + gl * qq;
        usrc[u * 512 + (int64_t)qq * 64 + lane + l] = e < iend[k] ? hsrc[e] : -1;
      }
    }
  }
}

__global__ void k_fill_i32p(int32_t* p, int64_t n, int32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_weights(int64_t n, const int32_t* __restrict__ col_ptr, float d, float* pw) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t k = col_ptr[i + 1] - col_ptr[i];
    pw[i] = k > 0 ? d / (float)k : 0.f;  // p_ji for every out-link of i
  }
}

// ---------------------------------------------------------------- the sweep
struct PartArgs {
  int64_t n;
  int K;
  int m;  // local sweeps per threshold level
  const int32_t* __restrict__ part_ptr;
  const int32_t* __restrict__ col_ptr;
  const int32_t* __restrict__ loc_ptr;
  const uint16_t* __restrict__ loc_idx;
  const uint16_t* __restrict__ inv;    // [n] local id of each node in its partition
  const int32_t* __restrict__ ext_ptr;   // [K+1] light external in-links of each partition
  const int32_t* __restrict__ ext_src;
  const uint16_t* __restrict__ ext_row;
  const int32_t* __restrict__ part_items;   // [K+1] heavy items of each partition
  const int32_t* __restrict__ item_row;     // item -> local row
  const int32_t* __restrict__ unit_src;     // [n_units][8][64] sources of the item work units
  const int32_t* __restrict__ unit_meta;    // [n_units][64] lane -> item it leads, group size
  unsigned long long* item_word;            // [2][n_items] item inflow bits | epoch << 32 (resident: by level parity)
  int n_items, n_units;
  int epoch0;        // resident: epoch of level 0 (grows across launches)
  float* F;
  double* H;
  float* S;          // [2][n] published p_i dH_i
  double* partials;  // [2][K][kStride] per-workgroup sums (resident: by level parity)
  int* counters;     // [1] finished workgroups (launches); [6], [7] resident: workgroups done with
                     // the levels of each parity (monotonic within a launch)
  Ctrl* ctrl;
  const int* abort_flag;  // host abort word (mapped)
  int n_heavy;
  int lds_nodes;   // node capacity of the LDS layout
  int prio;        // 1: threshold test on |F_i| / c_i, c_i = (#in_i + 1)(#out_i + 1) (Section 2.4)
  const int32_t* __restrict__ row_ptr;  // transpose row pointer (in-degrees, priority only)
  int lds_edges;   // local-target capacity (a larger partition reads its targets from memory)
  int max_levels;  // resident kernel: threshold levels before it returns
  float alpha;
  float d;
  double dd;  // damping in FP64 for the published shares
  double* trace;      // per-partition trace records (nullptr: off), see ditr_set_trace
  int64_t trace_cap;  // records
  double tick_s;      // seconds per s_memrealtime tick
};

constexpr int kTrace = DITR_TRACE_FIELDS;  // doubles per trace record

// thread 0 writes partition p's record of solve level `level` (if it fits)
__device__ __forceinline__ void trace_write(const PartArgs& a, int64_t level, int p, double held, double sent,
                                            double diffs, double edges, uint64_t idle_ticks,
                                            uint64_t busy_ticks) {
  const int64_t rec = level * a.K + p;
  if (rec >= a.trace_cap) return;
  double* t = a.trace + rec * kTrace;
  t[0] = held;
  t[1] = sent;
  t[2] = diffs;
  t[3] = edges;
  t[4] = (double)idle_ticks * a.tick_s;
  t[5] = (double)busy_ticks * a.tick_s;
}

// Fluid in LDS is fixed point: F = Fq q with q = T 2^-32 for the threshold T
// of the level, so the test |F| > T is |Fq| > 2^32, a push is an integer LDS
// atomic (ds_add_u64, several times the rate of the FP32 one on this chip) and
// the resolution is 2^-32 T (FP32 gives 2^-24 of the value). Signed fluid adds
// in two's complement; conversions saturate at 2^62 q (T never falls 2^30
// below the fluid it tests).
constexpr double kFix = 4294967296.0;  // 2^32
__device__ __forceinline__ long long to_fixed(double x) {
  const double lim = 4611686018427387904.0;  // 2^62
  return __double2ll_rn(fmin(fmax(x, -lim), lim));
}
__device__ __forceinline__ void add_fixed(long long* p, long long v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);  // ds_add_u64
}
// No node holds more than the total absolute fluid D (fluid in flight
// included): diffusion only splits and damps it. T therefore never drops below
// D 2^-28 (kPartTFloor), so no fixed-point value exceeds 2^60. A lower T would
// not diffuse more on graphs below 2^28 nodes, where some node holds at least
// D / n of the fluid; without the floor, fluid that only crosses partitions
// (M = 0 at every level) would let T fall by alpha per level while the fluid
// falls by d.
// quantum of the threshold T (a positive floor keeps 1/q finite when T = 0)
__device__ __forceinline__ double fixed_quantum(double T) { return fmax(T, 1e-280) / kFix; }

// Workgroup barrier for LDS traffic: each wave's LDS accesses complete before
// it, while its global loads stay in flight. __syncthreads and its _or/_and
// forms also wait for every outstanding global load, which would expose the
// latency of the outside gathers at the first barrier after they are issued.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// block-wide OR of a predicate over one LDS slot per wave; callers alternate
// two slot sets between consecutive calls, so one barrier per call suffices
template <int NW>
__device__ __forceinline__ int block_or(int pred, int* slots) {
  const unsigned long long b = __ballot(pred);
  if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = b != 0ull;
  lds_barrier();
  int any = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) any |= slots[w];
  return any;
}

// block-wide sum of one value, valid in thread 0 (its own LDS slots)
template <int BLOCK>
__device__ double block_sum_t0(double x) {
  __shared__ double slot[BLOCK / 64];
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = x;
  lds_barrier();
  double t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < BLOCK / 64; ++w) t += slot[w];
  lds_barrier();  // slot is free again
  return t;
}

// A partition's view of the dynamic LDS, indexed by local id (the partition's
// nodes renumbered in visiting order: node lo + j has local id inv[lo + j]):
// fluid (fixed point), history increment of the level (FP32, added to the
// FP64 H when published), local CSC offsets, out-degrees and, when they fit,
// the local targets.
struct PartView {
  long long* Fq;
  float* dH;
  int32_t* lptr;
  int32_t* odeg;
  uint32_t* lidx_words;
  uint32_t* cq;     // priority: c_i = (#in_i + 1)(#out_i + 1), capped at 2^30
  const uint16_t* lidx;
  int lo, np, lbase, nl;
  bool lidx_in_lds;
};

__device__ __forceinline__ PartView part_view(const PartArgs& a, unsigned char* smem, int p) {
  PartView v;
  const int cap = a.lds_nodes;
  v.Fq = reinterpret_cast<long long*>(smem);
  v.dH = reinterpret_cast<float*>(smem + (size_t)cap * 8);
  v.lptr = reinterpret_cast<int32_t*>(smem + (size_t)cap * 12);
  v.odeg = reinterpret_cast<int32_t*>(smem + (size_t)cap * 16 + 4);
  v.cq = reinterpret_cast<uint32_t*>(smem + (size_t)cap * 20 + 4);
  v.lidx_words = reinterpret_cast<uint32_t*>(smem + (size_t)cap * (a.prio ? 24 : 20) + 4);
  v.lo = a.part_ptr[p];
  v.np = a.part_ptr[p + 1] - v.lo;
  v.lbase = a.loc_ptr[v.lo];
  v.nl = a.loc_ptr[v.lo + v.np] - v.lbase;
  v.lidx_in_lds = v.nl + 2 <= a.lds_edges;
  // the LDS copy keeps the parity of lbase so that it moves whole 32-bit words
  v.lidx = v.lidx_in_lds ? reinterpret_cast<const uint16_t*>(v.lidx_words) + (v.lbase & 1)
                         : a.loc_idx + v.lbase;
  return v;
}

// 1. load the partition into LDS: local CSC offsets in local order, fluid and
// out-degrees in node order through inv (coalesced; eight nodes per thread in
// flight)
template <int BLOCK, bool PRIO>
__device__ void part_load(const PartArgs& a, const PartView& v, double inv_q) {
  const int tid = threadIdx.x;
  {
    // position j of the partition: the local CSC offset of local id j, and
    // the fluid and out-degree of node lo + j (at its local id)
    constexpr int U = 8;
    for (int j0 = tid; j0 < v.np; j0 += U * BLOCK) {
      int r[U], c0[U], c1[U], lp[U];
      float f[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * BLOCK;
        if (j < v.np) {
          lp[u] = a.loc_ptr[v.lo + j];
          r[u] = a.inv[v.lo + j];
          f[u] = a.F[v.lo + j];
          c0[u] = a.col_ptr[v.lo + j];
          c1[u] = a.col_ptr[v.lo + j + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * BLOCK;
        if (j < v.np) {
          v.lptr[j] = lp[u] - v.lbase;
          v.Fq[r[u]] = to_fixed((double)f[u] * inv_q);
          v.dH[r[u]] = 0.f;
          v.odeg[r[u]] = c1[u] - c0[u];
        }
      }
    }
  }
  if (PRIO) {
    // the normalized priority's divisor (#in_i + 1)(#out_i + 1) of Section 2.4
    for (int j = tid; j < v.np; j += BLOCK) {
      const int32_t g = v.lo + j;
      const long long in = a.row_ptr[g + 1] - a.row_ptr[g], out = a.col_ptr[g + 1] - a.col_ptr[g];
      v.cq[a.inv[g]] = (uint32_t)min((in + 1) * (out + 1), 1LL << 30);
    }
  }
  if (tid == 0) v.lptr[v.np] = v.nl;
  if (v.lidx_in_lds) {
    constexpr int U = 8;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.loc_idx) + (v.lbase >> 1);
    const int words = ((v.lbase & 1) + v.nl + 1) >> 1;
    for (int w0 = tid; w0 < words; w0 += U * BLOCK) {
      uint32_t x[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (w0 + u * BLOCK < words) x[u] = src[w0 + u * BLOCK];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (w0 + u * BLOCK < words) v.lidx_words[w0 + u * BLOCK] = x[u];
    }
  }
  __syncthreads();
}

// Sums of heavy items. Rows with more than kPartHeavy external in-links are
// cut in items of at most kItem links. An item is summed by a group of 1..64
// lanes (a power of two, eight links per lane); the plan packs the groups,
// largest first and aligned to their size, into work units of one wave, and
// stores for each unit the sources of every lane's eight slots, so a lane
// loads them from one table row and a butterfly over its group adds them. The
// group leader stores the sum as FP32 bits together with the level's epoch in
// one 64-bit word. Units are spread round-robin over all waves of the grid, so
// a hub's inflow is summed by many workgroups at once.
struct UnitLane {
  int32_t src[8];
  int meta;
};

__device__ __forceinline__ void unit_load(const PartArgs& a, int64_t u, UnitLane& L) {
  const int lane = threadIdx.x & 63;
  const int32_t* t = a.unit_src + (size_t)u * 512 + lane;
#pragma unroll
  for (int q = 0; q < 8; ++q) L.src[q] = t[64 * q];
  L.meta = a.unit_meta[(size_t)u * 64 + lane];
}

template <bool RESIDENT>
__device__ __forceinline__ void unit_gather(const float* S_in, const UnitLane& L, float (&v)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q)
    v[q] = L.src[q] >= 0 ? (RESIDENT ? ld_agent(&S_in[L.src[q]]) : S_in[L.src[q]]) : 0.f;
}

// the whole wave calls this (the butterfly shuffles over all 64 lanes)
template <bool RESIDENT>
__device__ __forceinline__ void unit_finish(const PartArgs& a, const UnitLane& L, const float (&v)[8],
                                            int epoch, int ib = 0) {
  double x = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) x += (double)v[q];
  const int lanes = 1 << (L.meta & 7);
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const double y = __shfl_xor(x, m, 64);
    if (m < lanes) x += y;
  }
  const int item = (L.meta >> 3) - 1;
  if (item >= 0) {
    const unsigned long long w =
        ((unsigned long long)(unsigned)epoch << 32) | (unsigned long long)__float_as_uint((float)x);
    if (RESIDENT) __hip_atomic_store(&a.item_word[ib + item], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else a.item_word[item] = w;
  }
}

template <bool RESIDENT>
__device__ __forceinline__ void unit_sum(const PartArgs& a, const float* S_in, const UnitLane& L,
                                         int epoch, int ib) {
  float v[8];
  unit_gather<RESIDENT>(S_in, L, v);
  unit_finish<RESIDENT>(a, L, v, epoch, ib);
}

// units first, first + stride, ... (the caller's wave)
template <bool RESIDENT>
__device__ void item_sums(const PartArgs& a, const float* S_in, int64_t first, int64_t stride,
                          int epoch, int ib = 0) {
  for (int64_t u = first; u < a.n_units; u += stride) {
    UnitLane L;
    unit_load(a, u, L);
    unit_sum<RESIDENT>(a, S_in, L, epoch, ib);
  }
}

// The resident sweep splits the light inflow: the first kLight links of each
// thread (sources and rows held in registers) have their shares gathered at the
// start of a level, so the loads are in flight during the first local sweep,
// and are added after it; links beyond them take the plain loop.
constexpr int kLight = 8;

// rows go two to a register (local ids are 16-bit)
__device__ __forceinline__ void light_prep(const PartArgs& a, int p, int32_t (&src)[kLight],
                                           uint32_t (&row)[kLight / 2]) {
  const int e0 = a.ext_ptr[p] + threadIdx.x, e1 = a.ext_ptr[p + 1];
#pragma unroll
  for (int u = 0; u < kLight; ++u) {
    const int e = e0 + u * (int)blockDim.x;
    src[u] = e < e1 ? a.ext_src[e] : -1;
  }
#pragma unroll
  for (int u = 0; u < kLight; u += 2) {
    const int e = e0 + u * (int)blockDim.x;
    const uint32_t r0 = e < e1 ? a.ext_row[e] : 0u;
    const uint32_t r1 = e + (int)blockDim.x < e1 ? a.ext_row[e + blockDim.x] : 0u;
    row[u / 2] = r0 | (r1 << 16);
  }
}

__device__ __forceinline__ void light_gather(const float* S_in, const int32_t (&src)[kLight], float (&x)[kLight]) {
#pragma unroll
  for (int u = 0; u < kLight; ++u) x[u] = src[u] >= 0 ? ld_agent(&S_in[src[u]]) : 0.f;
}

__device__ __forceinline__ void light_apply(const PartView& v, const uint32_t (&row)[kLight / 2],
                                            const float (&x)[kLight], double inv_q) {
#pragma unroll
  for (int u = 0; u < kLight; ++u)
    if (x[u] != 0.f) add_fixed(&v.Fq[(row[u / 2] >> (16 * (u & 1))) & 0xFFFFu], to_fixed((double)x[u] * inv_q));
}

// 2. outside fluid, pulled by the partition that owns it: each light external
// in-link (source, local row) adds the source's published share (one thread
// per link, LDS atomics); each heavy item of the partition adds its sum
// (resident: once its flag shows this level's epoch; a wait longer than
// spin_limit polls sets ctrl->err = 2 and ends the wait). RESIDENT: the values
// were published inside the same kernel, so they are read at agent scope.
// Returns false on a timed-out wait.
template <int BLOCK, bool RESIDENT>
__device__ bool part_inflow(const PartArgs& a, const PartView& v, int p, const float* S_in, double inv_q,
                            int epoch, int spin_limit, int skip = 0, int ib = 0) {
  const int tid = threadIdx.x;
  auto ld = [&](int32_t s) { return RESIDENT ? ld_agent(&S_in[s]) : S_in[s]; };
  const int e1 = a.ext_ptr[p + 1];
  constexpr int U = 8;  // eight gathers in flight per thread
  for (int e = a.ext_ptr[p] + skip * BLOCK + tid; e < e1; e += U * BLOCK) {
    // every load unconditional (slots past the end repeat the last link and
    // are dropped): a load under a per-lane branch must land before the
    // branch joins, which would serialize the thread's eight gathers
    int32_t src[U];
    int r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ee = min(e + u * BLOCK, e1 - 1);
      src[u] = a.ext_src[ee];
      r[u] = a.ext_row[ee];
    }
    float x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = ld(src[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e + u * BLOCK < e1 && x[u] != 0.f) add_fixed(&v.Fq[r[u]], to_fixed((double)x[u] * inv_q));
  }
  bool ok = true;
  const int k1 = a.part_items[p + 1];
  constexpr int UI = 4;  // the first polls of four items in flight together
  for (int k0 = a.part_items[p] + tid; k0 < k1 && ok; k0 += UI * BLOCK) {
    int row[UI];
    unsigned long long w[UI];
#pragma unroll
    for (int u = 0; u < UI; ++u) {
      const int k = k0 + u * BLOCK;
      if (k < k1) {
        row[u] = a.item_row[k];
        w[u] = RESIDENT ? __hip_atomic_load(&a.item_word[ib + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : a.item_word[k];
      }
    }
#pragma unroll
    for (int u = 0; u < UI; ++u) {
      const int k = k0 + u * BLOCK;
      if (k >= k1 || !ok) continue;
      if (RESIDENT) {
        int spins = 0;
        while ((w[u] >> 32) != (unsigned long long)(unsigned)epoch) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > spin_limit) {
            ok = false;
            __hip_atomic_store(&a.ctrl->err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          w[u] = __hip_atomic_load(&a.item_word[ib + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!ok) continue;
      }
      const float x = __uint_as_float((unsigned)w[u]);
      if (x != 0.f) add_fixed(&v.Fq[row[u]], to_fixed((double)x * inv_q));
    }
  }
  __shared__ int any_fail[BLOCK / 64];
  return !block_or<BLOCK / 64>(!ok, any_fail);
}

// 3. local threshold sweeps s0..s1-1 at one T until none passes. Each
// thread takes one node at a time in local-id order (consecutive ids have about
// the same local out-degree, so a wave's lanes finish their lists together)
// and pushes its share to every local target with LDS atomics, eight targets
// per step: their loads are issued together, then the adds. TARGETS_LDS: the local targets were copied to LDS (the pointer then has
// a known address space and the loop waits on LDS traffic only).
template <int BLOCK, bool TARGETS_LDS, bool PRIO>
__device__ void part_sweeps_t(const PartArgs& a, const PartView& v, double quantum, double& edges,
                              double& diffs, int s0, int s1) {
  const uint16_t* __restrict__ lidx =
      TARGETS_LDS ? reinterpret_cast<const uint16_t*>(v.lidx_words) + (v.lbase & 1) : a.loc_idx + v.lbase;
  const long long Tq = 1LL << 32;  // T in fixed point
  const float ddf = (float)a.dd;
  __shared__ int any_passed[2][BLOCK / 64];
  for (int s = s0; s < s1; ++s) {
    int passed = 0;
    for (int i = threadIdx.x; i < v.np; i += BLOCK) {
      // everything the step needs is read at once (one LDS round trip)
      const long long f = v.Fq[i];
      const int od = v.odeg[i];
      const int e0 = v.lptr[i], e1 = v.lptr[i + 1];
      const float dh = v.dH[i];
      // priority: node i's own threshold T c_i in the same fixed point
      const long long Ti = PRIO ? (long long)v.cq[i] << 32 : Tq;
      // keeps the compiler from sinking these reads into the branch below,
      // which would cost a second round trip for every node that passes
      asm volatile("" ::"v"(od), "v"(e0), "v"(e1), "v"(dh));
      if (!(f > Ti || f < -Ti)) continue;
      // the fluid read leaves the node; what other threads push meanwhile
      // stays there (an atomic subtract, no returned value to wait for)
      add_fixed(&v.Fq[i], -f);
      v.dH[i] = dh + (float)((double)f * quantum);
      // share per target: FP32 reciprocal (the pushes need not be exact: the
      // exact refresh recomputes F from H when the stage ends)
      const long long w = od > 0 ? to_fixed((double)f * (double)(ddf * __builtin_amdgcn_rcpf((float)od))) : 0;
      edges += (double)od;
      diffs += 1.0;
      passed = 1;
      for (int e = e0; e < e1; e += 8) {
        int t[8];
        if (TARGETS_LDS) {
          // the eight 16-bit targets from five aligned words (three LDS reads
          // instead of eight); the words past the last slot are padding
          const int u = e + (v.lbase & 1);
          const uint32_t* wp = v.lidx_words + (u >> 1);
          const uint32_t sh = (uint32_t)(u & 1) * 16u;
          uint32_t d[5];
#pragma unroll
          for (int k = 0; k < 5; ++k) d[k] = wp[k];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t win = __builtin_amdgcn_alignbit(d[k + 1], d[k], sh);
            t[2 * k] = win & 0xFFFFu;
            t[2 * k + 1] = win >> 16;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) t[q] = lidx[min(e + q, e1 - 1)];  // in range, no per-slot branch
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (e + q < e1) add_fixed(&v.Fq[t[q]], w);  // ds_add_u64
      }
    }
    if (!block_or<BLOCK / 64>(passed, any_passed[s & 1])) break;  // barrier + "did any node pass"
  }
}

template <int BLOCK, bool PRIO>
__device__ void part_sweeps(const PartArgs& a, const PartView& v, double quantum, double& edges,
                            double& diffs, int s0, int s1) {
  if (v.lidx_in_lds) part_sweeps_t<BLOCK, true, PRIO>(a, v, quantum, edges, diffs, s0, s1);
  else part_sweeps_t<BLOCK, false, PRIO>(a, v, quantum, edges, diffs, s0, s1);
}

// 4. H += dH and the shares p_i dH_i published for the outside targets, in node
// order through inv (H, S and F move coalesced; eight nodes per thread in
// flight). Sums |F| plus the fluid in flight to outside targets into resid, the
// fluid in flight alone into sent, and the largest |F| into fmx. RESIDENT: F
// stays in LDS and dH restarts from zero; otherwise F goes back to memory.
template <int BLOCK, bool RESIDENT, bool PRIO, bool SENT = false>
__device__ void part_publish(const PartArgs& a, const PartView& v, double quantum, float* S_out,
                             double& resid, double& sent, double& fmx) {
  constexpr int U = 8;
  for (int j0 = threadIdx.x; j0 < v.np; j0 += U * BLOCK) {
    int r[U];
    double hv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * BLOCK;
      r[u] = j < v.np ? a.inv[v.lo + j] : 0;
      hv[u] = j < v.np ? a.H[v.lo + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * BLOCK;
      if (j >= v.np) continue;
      const int i = r[u];
      const int32_t g = v.lo + j;
      const double f = (double)v.Fq[i] * quantum;
      const double dh = (double)v.dH[i];
      if (!RESIDENT) a.F[g] = (float)f;
      float so = 0.f;
      if (dh != 0.0) {
        a.H[g] = hv[u] + dh;
        if (RESIDENT) v.dH[i] = 0.f;
        const int od = v.odeg[i];
        if (od > 0) {
          so = (float)(a.dd * dh / (double)od);
          const double out = fabs((double)so) * (double)(od - (v.lptr[i + 1] - v.lptr[i]));
          resid += out;
          if (SENT) sent += out;
        }
      }
      if (RESIDENT) st_agent(&S_out[g], so);
      else S_out[g] = so;
      resid += fabs(f);
      // largest priority (|F_i| / c_i under the normalized test)
      fmx = fmax(fmx, PRIO ? fabs(f) / (double)v.cq[i] : fabs(f));
    }
  }
}

// block-wide sums of (resid, edges, diffs) and max of fmx, in a fixed order;
// the result is valid in every thread
template <int BLOCK>
__device__ void block_reduce4(double& r0, double& r1, double& r2, double& r3, double (*red)[BLOCK / 64]) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  r0 = wave_sum(r0);
  r1 = wave_maxd(r1);
  r2 = wave_sum(r2);
  r3 = wave_sum(r3);
  lds_barrier();  // red may still be read by an earlier reduction
  if (lane == 0) {
    red[0][wave] = r0;
    red[1][wave] = r1;
    red[2][wave] = r2;
    red[3][wave] = r3;
  }
  lds_barrier();
  r0 = 0, r1 = 0, r2 = 0, r3 = 0;
  for (int w = 0; w < NW; ++w) {
    r0 += red[0][w];
    r1 = fmax(r1, red[1][w]);
    r2 += red[2][w];
    r3 += red[3][w];
  }
}

// Heavy-item sums as their own kernel, right before a launch of the sweep.
__global__ void __launch_bounds__(256) k_part_items(PartArgs a, int parity) {
  if (__hip_atomic_load(&a.ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  item_sums<false>(a, a.S + (size_t)(parity ^ 1) * a.n, (int64_t)(threadIdx.x >> 6) * gridDim.x + blockIdx.x,
                   (int64_t)gridDim.x * 4, 0);
}

// One launch of the partitioned sweep. Workgroup p:
//   1. loads Omega_p into LDS (fluid, history increment, local CSC);
//   2. pulls the outside fluid S_in over its light external in-links and adds
//      the sums of its heavy items (k_part_items, just before);
//   3. runs up to m threshold sweeps at the launch's T until none passes;
//   4. writes F and H back and publishes S_out = p_i dH_i;
//   5. the last workgroup to finish reduces the per-workgroup sums and sets
//      the next T and the stop flag (no separate step kernel).
template <int BLOCK, bool PRIO>
__global__ void __launch_bounds__(BLOCK) k_part_sweep(PartArgs a, int parity) {
  if (__hip_atomic_load(&a.ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const float* S_in = a.S + (size_t)(parity ^ 1) * a.n;
  float* S_out = a.S + (size_t)parity * a.n;
  const int tid = threadIdx.x;
  constexpr int NW = BLOCK / 64;
  __shared__ double red[4][NW];
  __shared__ int s_last;
  extern __shared__ __align__(16) unsigned char smem[];
  const int p = blockIdx.x;
  const PartView v = part_view(a, smem, p);

  const double quantum = fixed_quantum(a.ctrl->T);
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
  const int64_t level = (int64_t)a.ctrl->sweeps;  // this launch's level of the solve
  part_load<BLOCK, PRIO>(a, v, 1.0 / quantum);
  part_inflow<BLOCK, false>(a, v, p, S_in, 1.0 / quantum, 0, 0);
  double edges = 0, diffs = 0;
  part_sweeps<BLOCK, PRIO>(a, v, quantum, edges, diffs, 0, a.m);

  // ---- 4. write back, publish p_i dH_i, partial sums
  double resid = 0, sent = 0, fmx = 0;
  part_publish<BLOCK, false, PRIO, true>(a, v, quantum, S_out, resid, sent, fmx);

  // ---- 5. per-workgroup sums; the last workgroup finishes the launch
  block_reduce4<BLOCK>(resid, fmx, edges, diffs, red);
  if (a.trace) {
    const double s_tot = block_sum_t0<BLOCK>(sent);
    if (tid == 0)
      trace_write(a, level, p, resid - s_tot, s_tot, diffs, edges, 0,
                  __builtin_amdgcn_s_memrealtime() - t_start);
  }
  if (tid == 0) {
    double* q = a.partials + (size_t)kStride * p;
    __hip_atomic_store(&q[0], resid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q[1], fmx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q[2], edges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q[3], diffs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int t = __hip_atomic_fetch_add(&a.counters[1], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = t == a.K - 1;
  }
  __syncthreads();
  if (!s_last) return;
  double D = 0, M = 0, E = 0, P = 0;
  for (int k = tid; k < a.K; k += BLOCK) {
    const double* q = a.partials + (size_t)kStride * k;
    D += __hip_atomic_load(&q[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    M = fmax(M, __hip_atomic_load(&q[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    E += __hip_atomic_load(&q[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    P += __hip_atomic_load(&q[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  block_reduce4<BLOCK>(D, M, E, P, red);
  if (tid == 0) {
    Ctrl* ctrl = a.ctrl;
    ctrl->sum_abs = D;
    ctrl->edges += (unsigned long long)E;
    ctrl->diffusions += (unsigned long long)P;
    ctrl->sweeps += 1;
    if (D <= ctrl->target) {
      __hip_atomic_store(&ctrl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      double Tn = ctrl->T / (double)a.alpha;  // one threshold level per launch
      if (P == 0 && M / a.alpha < Tn) Tn = M / a.alpha;
      ctrl->T = fmax(Tn, D * kPartTFloor);
    }
    a.counters[1] = 0;  // finish count of the next launch
  }
}

// ---------------------------------------------------- the resident sweep
// Every value one workgroup of the resident sweep hands to another (published
// shares, partial sums, heavy-row sums, the votes) is written and read with
// agent-scope atomics, which bypass the per-XCD L2s, so a level arrival needs
// no cache maintenance: each thread waits until its own stores are
// acknowledged, then thread 0 counts the workgroup in on an agent-scope word.
__device__ __forceinline__ void wait_stores() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // s_waitcnt vmcnt(0)
}

// Wait of a cooperative launch (every workgroup resident) until a monotonic
// arrival counter reaches `target`: thread 0 polls it at agent scope, the
// workgroup meets on the result. A wait longer than spin_limit polls sets
// ctrl->err = 2 and returns false; the caller then leaves the kernel, so every
// wave exits even if some workgroup never arrives. The polls that found the
// count short are added to *polls.
__device__ bool wait_count(const int* cnt, int target, int spin_limit, int* err, int* s_ok,
                           unsigned long long* polls) {
  if (threadIdx.x == 0) {
    int ok = 1, spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > spin_limit) {
        ok = 0;
        __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    if (spins) __hip_atomic_fetch_add(polls, (unsigned long long)spins, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_ok = ok;
  }
  lds_barrier();
  return *s_ok != 0;
}

// The partitioned sweep with every partition resident for a whole stage: the
// partition is loaded into LDS once and stays there across threshold levels.
// Level l of a workgroup: wait until every workgroup has published level l-1
// (an arrival count, not a barrier: the workgroups that finished first do not
// wait for a release); gather the outside shares of level l-1 and run the
// first local sweep while they land; finish the item sums, add the outside
// fluid; read the per-workgroup sums of level l-1; further local sweeps;
// publish H += dH and the shares p_i dH_i of level l and its own sums; arrive.
// The stop, abort and next-threshold decisions come from the sums of level
// l-1, which every workgroup reduces in the same order, so all take them at the
// same level; the run therefore ends one level after the one whose sums met
// the target. Shares, item words and sums alternate between two buffers by
// level parity: a workgroup publishes level l only after every workgroup has
// finished level l-1, so nobody still reads the level l-2 contents it
// replaces. F goes back to memory when the stage ends.
// TRACE: write the per-partition trace records (a separate instantiation, so
// the untraced kernel carries none of its registers)
template <int BLOCK, bool PRIO, bool TRACE>
__global__ void __launch_bounds__(BLOCK) k_part_resident(PartArgs a, int spin_limit) {
  const int tid = threadIdx.x;
  constexpr int NW = BLOCK / 64;
  __shared__ double red[4][NW];
  __shared__ int s_ok;
  extern __shared__ __align__(16) unsigned char smem[];
  // a queued stage the previous one made unnecessary (its start meets the
  // target) returns at once; every workgroup reads the flag before any of them
  // can finish a level, so the end-of-stage write below cannot race with it
  if (a.ctrl->done) return;
  const int p = blockIdx.x;
  const PartView v = part_view(a, smem, p);
  int* arrive = a.counters + 6;
  int* err = &a.ctrl->err;
  const double target = a.ctrl->target;
  double T = a.ctrl->T;
  // TRACE, thread 0: the solve's level count at the launch, the clock before
  // and after the level's wait and at its arrival (in LDS, not in registers)
  __shared__ long long s_tr[4];
  if (TRACE && tid == 0) s_tr[0] = (long long)a.ctrl->sweeps;
  int done = 0, levels = 0, stop = 0;
  double edges_tail = 0, diffs_tail = 0;  // own counts of the last level, added at the end

  double quantum = fixed_quantum(T);
  part_load<BLOCK, PRIO>(a, v, 1.0 / quantum);
  // wave w of workgroup p takes item units w K + p, (w + NW) K + p, ..., so
  // the densest units (packed first) are spread over all CUs; the sources of
  // the first one and of the first light links are loaded at the end of the
  // level before (they are constant), out of the register-heavy publish
  const int64_t unit0 = (int64_t)(tid >> 6) * a.K + p, n_waves = (int64_t)a.K * NW;
  UnitLane L0;
  if (unit0 < a.n_units) unit_load(a, unit0, L0);
  int32_t lsrc[kLight];
  uint32_t lrow[kLight / 2];
  light_prep(a, p, lsrc, lrow);
  for (; levels < a.max_levels; ++levels) {
    const int par = levels & 1;
    const float* S_in = a.S + (size_t)(par ^ 1) * a.n;
    float* S_out = a.S + (size_t)par * a.n;
    const int epoch = a.epoch0 + levels, ib = par * a.n_items;
    // everything of level l-1 is out (shares, sums); level 0 reads the zeroed
    // buffer of parity 1
    if (TRACE && tid == 0) s_tr[1] = (long long)__builtin_amdgcn_s_memrealtime();
    if (levels > 0 && !wait_count(&arrive[par ^ 1], a.K * ((levels - 1) / 2 + 1), spin_limit, err, &s_ok,
                                  &a.ctrl->idle_polls))
      return;
    if (TRACE && tid == 0) s_tr[2] = (long long)__builtin_amdgcn_s_memrealtime();
    // the outside shares are gathered first and land during the first local
    // sweep; they join the fluid before the second one
    float iv[8], lv[kLight];
    if (unit0 < a.n_units) unit_gather<true>(S_in, L0, iv);
    light_gather(S_in, lsrc, lv);
    double edges = 0, diffs = 0;
    part_sweeps<BLOCK, PRIO>(a, v, quantum, edges, diffs, 0, 1);
    // the sums of level l-1, in flight while the outside fluid is added
    const double* prev = a.partials + (size_t)(par ^ 1) * a.K * kStride;
    double D = 0, M = 0, E = 0, P = 0;
    const bool aborted = levels > 0 && ld_agent(&prev[4]) != 0.0;  // workgroup 0's vote
    if (levels > 0)
      for (int k = tid; k < a.K; k += BLOCK) {
        // the four loads first, then the uses (one wait instead of four)
        const double* q = prev + (size_t)kStride * k;
        const double q0 = ld_agent(&q[0]), q1 = ld_agent(&q[1]), q2 = ld_agent(&q[2]), q3 = ld_agent(&q[3]);
        D += q0;
        M = fmax(M, q1);
        E += q2;
        P += q3;
      }
    if (unit0 < a.n_units) unit_finish<true>(a, L0, iv, epoch, ib);
    item_sums<true>(a, S_in, unit0 + n_waves, n_waves, epoch, ib);
    light_apply(v, lrow, lv, 1.0 / quantum);
    if (!part_inflow<BLOCK, true>(a, v, p, S_in, 1.0 / quantum, epoch, spin_limit, kLight, ib)) return;
    // decisions from level l-1, the same in every workgroup
    double Tn = T / (double)a.alpha;
    if (levels > 0) {
      block_reduce4<BLOCK>(D, M, E, P, red);
      if (p == 0 && tid == 0) {
        Ctrl* ctrl = a.ctrl;
        ctrl->sum_abs = D;
        __hip_atomic_fetch_add(&ctrl->edges, (unsigned long long)E, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&ctrl->diffusions, (unsigned long long)P, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
      if (D <= target) done = stop = 1;
      if (aborted) stop = 1;
      if (P == 0 && M / a.alpha < Tn) Tn = M / a.alpha;
      Tn = fmax(Tn, D * kPartTFloor);
    }
    part_sweeps<BLOCK, PRIO>(a, v, quantum, edges, diffs, 1, a.m);

    // H += dH, publish p_i dH_i, partial sums (F stays in LDS)
    double resid = 0, sent = 0, fmx = 0;
    part_publish<BLOCK, true, PRIO>(a, v, quantum, S_out, resid, sent, fmx);
    double* part = a.partials + (size_t)par * a.K * kStride;
    block_reduce4<BLOCK>(resid, fmx, edges, diffs, red);
    edges_tail = edges;
    diffs_tail = diffs;
    if (tid == 0) {
      double* q = part + (size_t)kStride * p;
      st_agent(&q[0], resid);
      st_agent(&q[1], fmx);
      st_agent(&q[2], edges);
      st_agent(&q[3], diffs);
      if (p == 0) st_agent(&q[4], ld_system(a.abort_flag) != 0 ? 1.0 : 0.0);
    }
    // every wave's shares, H and sums are out before the arrival
    wait_stores();
    __syncthreads();
    if (tid == 0) {
      if (TRACE) s_tr[3] = (long long)__builtin_amdgcn_s_memrealtime();
      __hip_atomic_fetch_add(&arrive[par], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (unit0 < a.n_units) unit_load(a, unit0, L0);  // for the next level, after the arrival
    light_prep(a, p, lsrc, lrow);
    if (TRACE) {
      // the fluid held, in a pass of its own after the arrival (the rest of
      // resid is in flight); the record is written off the level's path
      double held = 0;
      for (int i = tid; i < v.np; i += BLOCK) held += fabs((double)v.Fq[i] * quantum);
      held = block_sum_t0<BLOCK>(held);
      if (tid == 0)
        trace_write(a, s_tr[0] + levels, p, held, resid - held, diffs, edges, s_tr[2] - s_tr[1],
                    s_tr[3] - s_tr[2]);
    }
    if (stop) {
      ++levels;
      break;
    }
    // the fluid moves to the quantum of the next threshold
    const double qn = fixed_quantum(Tn), r = quantum / qn;
    for (int i = tid; i < v.np; i += BLOCK) v.Fq[i] = to_fixed((double)v.Fq[i] * r);
    lds_barrier();
    T = Tn;
    quantum = qn;
  }
  for (int j = tid; j < v.np; j += BLOCK) a.F[v.lo + j] = (float)((double)v.Fq[a.inv[v.lo + j]] * quantum);
  // the counts of the last level were not in any decision: each workgroup adds its own
  if (tid == 0) {
    __hip_atomic_fetch_add(&a.ctrl->edges, (unsigned long long)edges_tail, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&a.ctrl->diffusions, (unsigned long long)diffs_tail, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
  if (p == 0 && tid == 0) {
    a.ctrl->sweeps += (unsigned long long)levels;
    a.ctrl->T = T;
    a.ctrl->done = done;
    a.ctrl->stages += 1;
  }
}

__global__ void k_zero_f32p(float* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.f;
}
__global__ void k_zero_f64p(double* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}
__global__ void k_gather_ranges(int32_t nh, const int32_t* __restrict__ rows,
                                const int32_t* __restrict__ ptr, int32_t* out) {
  for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += gridDim.x * blockDim.x) {
    out[2 * h] = ptr[rows[h]];
    out[2 * h + 1] = ptr[rows[h] + 1];
  }
}

}  // namespace


void free_part_plan(ditr_graph* g) {
  PartPlan& q = g->pp;
  for (void* p : {(void*)q.pid, (void*)q.loc_ptr, (void*)q.loc_idx, (void*)q.pw,
                  (void*)q.ext_ptr, (void*)q.ext_src, (void*)q.ext_row, (void*)q.heavy_rows,
                  (void*)q.part_heavy, (void*)q.heavy_src, (void*)q.item_row, (void*)q.part_items,
                  (void*)q.unit_src, (void*)q.unit_meta, (void*)q.item_word,
                  (void*)q.S, (void*)q.partials, (void*)q.counters, (void*)q.inv})
    g_free(g, p);
  q = PartPlan();
}

// device temporary bytes of the plan build's two radix sorts (n nodes, ni items)
size_t plan_sort_temp_bytes(int64_t n, int64_t ni) {
  size_t a = 0, b = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, (unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                           (int32_t*)nullptr, (int32_t*)nullptr, (int)std::max<int64_t>(n, 1), 0,
                                           64, nullptr);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (uint32_t*)nullptr, (uint32_t*)nullptr, (int32_t*)nullptr,
                                           (int32_t*)nullptr, (int)std::max<int64_t>(ni, 1), 0, 3, nullptr);
  return a + b;
}

// Build the partitioned-sweep tables for the current partition plan of g, all
// on the device (sorts and scans; the host reads back only sizes).
int build_part_plan(ditr_ctx* c, ditr_graph* g) {
  free_part_plan(g);
  PartPlan& q = g->pp;
  const int64_t n = g->n;
  const int K = (int)g->K;
  hipStream_t st = c->stream;
  std::vector<void*> temps;  // freed (or left in the workspace) at the end
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (void* p : temps) g_free(g, p);
    temps.clear();
  };
#define PP_TRY(expr)                                                                     \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      cleanup();                                                                         \
      return set_error(DITR_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e));        \
    }                                                                                    \
  } while (0)
#define PP_RC(expr)            \
  do {                         \
    const int _rc = (expr);    \
    if (_rc) {                 \
      cleanup();               \
      return _rc;              \
    }                          \
  } while (0)
  auto temp = [&](void** p, size_t bytes) -> hipError_t {
    const hipError_t e = g_alloc(g, p, bytes);
    if (e == hipSuccess) temps.push_back(*p);
    return e;
  };
  auto read_i32 = [&](const int32_t* d, int32_t* h) -> hipError_t {
    hipError_t e = hipMemcpyAsync(h, d, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    return e == hipSuccess ? hipStreamSynchronize(st) : e;
  };
  if (g->max_part > 65536) return set_error(DITR_EINVAL, "partitions above 65536 nodes");
  const int gb = grid_for(n, 256, 8192);
  const int gw = grid_for(n * 64, 256, 16384);  // one wave per row
  int32_t *cnt, *cnt2, *light_ptr, *heavy_ptr, *ord_in, *ord, *degp;
  unsigned long long *key_in, *key_out;
  PP_TRY(g_alloc(g, (void**)&q.pid, sizeof(int32_t) * n));
  PP_TRY(g_alloc(g, (void**)&q.inv, sizeof(uint16_t) * std::max<int64_t>(1, n)));
  PP_TRY(g_alloc(g, (void**)&q.loc_ptr, sizeof(int32_t) * (n + 1)));
  PP_TRY(temp((void**)&cnt, sizeof(int32_t) * (n + 1)));
  PP_TRY(temp((void**)&cnt2, sizeof(int32_t) * (n + 1)));
  PP_TRY(temp((void**)&light_ptr, sizeof(int32_t) * (n + 1)));
  PP_TRY(temp((void**)&heavy_ptr, sizeof(int32_t) * (n + 1)));
  PP_TRY(temp((void**)&degp, sizeof(int32_t) * (n + 1)));
  k_fill_pid<<<std::min(K, 8192), 256, 0, st>>>(K, g->part_ptr, q.pid);
  k_count_local<<<gb, 256, 0, st>>>(n, g->col_ptr, g->row_idx, q.pid, cnt);
  PP_TRY(hipGetLastError());

  // visiting order of each partition's nodes: falling local out-degree, ties in
  // node order (a stable radix sort of (partition, ~degree)), so that the 64
  // lanes of a wave push lists of about the same length; local id r of
  // partition k is node ord[lo_k + r], and inv maps a node to its local id
  {
    PP_TRY(temp((void**)&key_in, sizeof(unsigned long long) * std::max<int64_t>(1, n)));
    PP_TRY(temp((void**)&key_out, sizeof(unsigned long long) * std::max<int64_t>(1, n)));
    PP_TRY(temp((void**)&ord_in, sizeof(int32_t) * std::max<int64_t>(1, n)));
    PP_TRY(temp((void**)&ord, sizeof(int32_t) * std::max<int64_t>(1, n)));
    k_order_keys<<<gb, 256, 0, st>>>(n, q.pid, cnt, key_in, ord_in);
    int kbits = 1;
    while (kbits < 31 && (1LL << kbits) < (int64_t)K) ++kbits;
    size_t tb = 0;
    PP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key_in, key_out, ord_in, ord, (int)n, 0, 32 + kbits, st));
    void* tmp = nullptr;
    PP_TRY(temp(&tmp, tb));
    PP_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tb, key_in, key_out, ord_in, ord, (int)n, 0, 32 + kbits, st));
    k_inv<<<gb, 256, 0, st>>>(n, ord, q.pid, g->part_ptr, cnt, q.inv, degp);
    PP_TRY(hipGetLastError());
  }
  // local CSC in visiting order (pointer by local id, targets as local ids)
  PP_RC(scan_exclusive_i32(c, degp, n, q.loc_ptr, g));
  int32_t nloc = 0;
  PP_TRY(read_i32(q.loc_ptr + n, &nloc));
  PP_TRY(g_alloc(g, (void**)&q.loc_idx, sizeof(uint16_t) * (nloc + 4)));  // word copies may overrun by one
  k_fill_local<<<gb, 256, 0, st>>>(n, g->col_ptr, g->row_idx, q.pid, g->part_ptr, q.inv, q.loc_ptr, q.loc_idx);
  {
    int32_t* mx = nullptr;
    PP_TRY(temp((void**)&mx, sizeof(int32_t)));
    PP_TRY(hipMemsetAsync(mx, 0, sizeof(int32_t), st));
    k_part_max_edges<<<grid_for(K, 256, 1024), 256, 0, st>>>(K, g->part_ptr, q.loc_ptr, mx);
    PP_TRY(hipGetLastError());
    PP_TRY(read_i32(mx, &q.max_local_edges));
  }
  // external in-links per row: light rows stream them, heavy rows become items
  k_count_ext<<<gw, 256, 0, st>>>(n, g->row_ptr, g->csr_col, q.pid, cnt, cnt2);
  PP_TRY(hipGetLastError());
  PP_RC(scan_exclusive_i32(c, cnt, n, light_ptr, g));
  PP_RC(scan_exclusive_i32(c, cnt2, n, heavy_ptr, g));
  int32_t nlight = 0, nheavy_e = 0;
  PP_TRY(read_i32(light_ptr + n, &nlight));
  PP_TRY(read_i32(heavy_ptr + n, &nheavy_e));
  PP_TRY(g_alloc(g, (void**)&q.ext_src, sizeof(int32_t) * std::max(1, nlight)));
  PP_TRY(g_alloc(g, (void**)&q.ext_row, sizeof(uint16_t) * std::max(1, nlight)));
  PP_TRY(g_alloc(g, (void**)&q.heavy_src, sizeof(int32_t) * std::max(1, nheavy_e)));
  PP_TRY(g_alloc(g, (void**)&q.ext_ptr, sizeof(int32_t) * (K + 1)));
  k_fill_ext<<<gw, 256, 0, st>>>(n, g->row_ptr, g->csr_col, q.pid, q.inv, light_ptr, heavy_ptr,
                                 q.ext_src, q.ext_row, q.heavy_src);
  k_gather_ptr<<<grid_for(K + 1, 256, 1024), 256, 0, st>>>(K, g->part_ptr, light_ptr, q.ext_ptr);
  PP_TRY(hipGetLastError());

  // heavy rows, ascending (a scan of the heavy flags), and each partition's
  // range of them
  int32_t *hflag, *hpos;
  PP_TRY(temp((void**)&hflag, sizeof(int32_t) * (n + 1)));
  PP_TRY(temp((void**)&hpos, sizeof(int32_t) * (n + 1)));
  k_heavy_flag<<<gb, 256, 0, st>>>(n, heavy_ptr, hflag);
  PP_TRY(hipGetLastError());
  PP_RC(scan_exclusive_i32(c, hflag, n, hpos, g));
  int32_t nh = 0;
  PP_TRY(read_i32(hpos + n, &nh));
  PP_TRY(g_alloc(g, (void**)&q.heavy_rows, sizeof(int32_t) * std::max(1, nh)));
  PP_TRY(g_alloc(g, (void**)&q.part_heavy, sizeof(int32_t) * (K + 1)));
  k_heavy_rows<<<gb, 256, 0, st>>>(n, hflag, hpos, q.heavy_rows);
  k_gather_ptr<<<grid_for(K + 1, 256, 1024), 256, 0, st>>>(K, g->part_ptr, hpos, q.part_heavy);
  PP_TRY(hipGetLastError());

  // heavy items: the external in-links of each heavy row cut in pieces of
  // kItem, in heavy-row order (so grouped by partition)
  int32_t *icnt, *ioff;
  PP_TRY(temp((void**)&icnt, sizeof(int32_t) * (std::max(1, nh) + 1)));
  PP_TRY(temp((void**)&ioff, sizeof(int32_t) * (std::max(1, nh) + 1)));
  k_item_count<<<grid_for(std::max(1, nh), 256, 8192), 256, 0, st>>>(nh, q.heavy_rows, heavy_ptr, icnt);
  PP_TRY(hipGetLastError());
  PP_RC(scan_exclusive_i32(c, icnt, nh, ioff, g));
  int32_t ni = 0;
  PP_TRY(read_i32(ioff + nh, &ni));
  if (ni >= (1 << 27)) {
    cleanup();
    return set_error(DITR_EINVAL, "too many heavy items (%d)", ni);
  }
  q.n_items = ni;
  const int ni1 = std::max(1, ni);
  int32_t *ibeg, *iend, *by_in, *by;
  uint32_t *ikey_in, *ikey;
  PP_TRY(g_alloc(g, (void**)&q.item_row, sizeof(int32_t) * ni1));
  PP_TRY(g_alloc(g, (void**)&q.part_items, sizeof(int32_t) * (K + 1)));
  PP_TRY(temp((void**)&ibeg, sizeof(int32_t) * ni1));
  PP_TRY(temp((void**)&iend, sizeof(int32_t) * ni1));
  PP_TRY(temp((void**)&by_in, sizeof(int32_t) * ni1));
  PP_TRY(temp((void**)&by, sizeof(int32_t) * ni1));
  PP_TRY(temp((void**)&ikey_in, sizeof(uint32_t) * ni1));
  PP_TRY(temp((void**)&ikey, sizeof(uint32_t) * ni1));
  k_item_fill<<<grid_for(std::max(1, nh), 256, 8192), 256, 0, st>>>(nh, q.heavy_rows, heavy_ptr, ioff, q.inv,
                                                                   q.item_row, ibeg, iend, ikey_in, by_in);
  k_gather_ptr2<<<grid_for(K + 1, 256, 1024), 256, 0, st>>>(K, q.part_heavy, ioff, q.part_items);
  PP_TRY(hipGetLastError());

  // work units: an item takes a group of 2^l lanes, the fewest whose eight
  // slots hold its links. Groups are packed largest first (a stable sort by
  // size class), so each starts at a multiple of its size and a unit is full
  // before the next one starts: the lane of every group is a prefix sum.
  int32_t *gl, *loff;
  PP_TRY(temp((void**)&gl, sizeof(int32_t) * (ni1 + 1)));
  PP_TRY(temp((void**)&loff, sizeof(int32_t) * (ni1 + 1)));
  if (ni > 0) {
    size_t tb = 0;
    PP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, ikey_in, ikey, by_in, by, ni, 0, 3, st));
    void* tmp = nullptr;
    PP_TRY(temp(&tmp, tb));
    PP_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tb, ikey_in, ikey, by_in, by, ni, 0, 3, st));
    k_unit_lanes<<<grid_for(ni, 256, 8192), 256, 0, st>>>(ni, by, ibeg, iend, gl);
    PP_TRY(hipGetLastError());
  }
  PP_RC(scan_exclusive_i32(c, gl, ni, loff, g));
  int32_t lanes = 0;
  PP_TRY(read_i32(loff + ni, &lanes));
  const int64_t nu = ((int64_t)lanes + 63) / 64;
  q.n_units = (int32_t)nu;
  PP_TRY(g_alloc(g, (void**)&q.unit_src, sizeof(int32_t) * 512 * std::max<int64_t>(1, nu)));
  PP_TRY(g_alloc(g, (void**)&q.unit_meta, sizeof(int32_t) * 64 * std::max<int64_t>(1, nu)));
  k_fill_i32p<<<grid_for(512 * std::max<int64_t>(1, nu), 256, 8192), 256, 0, st>>>(q.unit_src, 512 * std::max<int64_t>(1, nu), -1);
  k_fill_i32p<<<grid_for(64 * std::max<int64_t>(1, nu), 256, 8192), 256, 0, st>>>(q.unit_meta, 64 * std::max<int64_t>(1, nu), 0);
  if (ni > 0)
    k_unit_fill<<<grid_for(ni, 256, 8192), 256, 0, st>>>(ni, by, loff, ibeg, iend, q.heavy_src, q.unit_src,
                                                         q.unit_meta);
  PP_TRY(hipGetLastError());
  PP_TRY(g_alloc(g, (void**)&q.item_word, sizeof(unsigned long long) * 2 * ni1));
  PP_TRY(hipMemsetAsync(q.item_word, 0, sizeof(unsigned long long) * 2 * ni1, st));
  q.n_heavy = nh;

  PP_TRY(g_alloc(g, (void**)&q.pw, sizeof(float) * n));
  k_weights<<<gb, 256, 0, st>>>(n, g->col_ptr, (float)g->d, q.pw);
  PP_TRY(hipGetLastError());
  PP_TRY(g_alloc(g, (void**)&q.S, sizeof(float) * 2 * n));
  PP_TRY(g_alloc(g, (void**)&q.counters, sizeof(int) * kCounters));
  PP_TRY(hipMemsetAsync(q.counters, 0, sizeof(int) * kCounters, st));
  PP_TRY(g_alloc(g, (void**)&q.partials, sizeof(double) * kStride * 2 * K));
  PP_TRY(hipStreamSynchronize(st));
  // the unit table replaces the per-row source list
  temps.push_back(q.heavy_src);
  q.heavy_src = nullptr;
  q.n_local = nloc;
  q.n_ext = nlight;
  q.n_heavy_edges = nheavy_e;
  cleanup();
  q.ready = true;
#undef PP_TRY
#undef PP_RC
  return DITR_OK;
}

__global__ void k_zero_u64p(unsigned long long* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

int launch_zero_u64(ditr_ctx* c, unsigned long long* p, int64_t n) {
  if (n <= 0) return DITR_OK;
  k_zero_u64p<<<(unsigned)std::min<int64_t>(1024, (n + 255) / 256), 256, 0, c->stream>>>(p, n);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

// sum over nodes of (#in_i + 1)(#out_i + 1) in FP64, one partial per block
__global__ void __launch_bounds__(256) k_prio_sum(int64_t n, const int32_t* __restrict__ col_ptr,
                                                  const int32_t* __restrict__ row_ptr, double* partial) {
  double s = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
    s += (double)(row_ptr[i + 1] - row_ptr[i] + 1) * (double)(col_ptr[i + 1] - col_ptr[i] + 1);
  s = wave_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Synchronizes.
int launch_prio_sum(ditr_ctx* c, const ditr_graph* g, double* h_sum) {
  const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (g->n + 255) / 256));
  if ((size_t)nb * 4 > c->partials_cap * 4) return set_error(DITR_EINVAL, "partials too small");
  k_prio_sum<<<nb, 256, 0, c->stream>>>(g->n, g->col_ptr, g->row_ptr, c->partials);
  HIP_TRY(hipGetLastError());
  std::vector<double> part(nb);
  HIP_TRY(hipMemcpyAsync(part.data(), c->partials, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double s = 0;
  for (double x : part) s += x;
  *h_sum = s;
  return DITR_OK;
}

SolveBufs graph_bufs(const ditr_graph* g) {
  ditr_graph* m = const_cast<ditr_graph*>(g);
  SolveBufs b;
  b.S = m->pp.S;
  b.item_word = m->pp.item_word;
  b.partials = m->pp.partials;
  b.counters = m->pp.counters;
  b.wh = m->wh;
  b.chunk_sum = m->chunk_sum;
  b.epoch = &m->pp.epoch;
  return b;
}

__global__ void k_zero_i32p(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Start of a stage of the partitioned sweep in one launch (each small launch
// costs microseconds of dispatch): the stage's control words, zero counters,
// zero shares.
__global__ void k_part_prepare(Ctrl* ctrl, double r0, double target, double T0, int* counters, float* S,
                               int64_t n2) {
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  if (i0 == 0) {
    ctrl->destroyed = 0;
    ctrl->r0 = r0;
    ctrl->target = target;
    ctrl->T = T0;
    ctrl->done = 0;
    ctrl->ticket = 0;
    ctrl->passed = 0;
  }
  if (i0 < kCounters) counters[i0] = 0;
  for (int64_t i = i0; i < n2; i += stride) S[i] = 0.f;
}

// Parameters of the next stage of a solve queued without host readbacks, from
// the device's own sums (one thread): the first stage reads the init pass
// (||B||_1, ||F_0||_1, max |F_0|), a later one the exact refresh before it
// (||F||_1, max |F|) and the threshold the previous stage ended at; the same
// rules as the host's stage loop. A stage whose start already meets the target,
// or that follows a non-finite input, a timed-out wait or an abort, is marked
// done, and its launch returns at once.
__global__ void k_part_stage(Ctrl* ctrl, const int* abort_flag, int first, int64_t n, double rel_tol,
                             double refresh_at, double alpha) {
  if (first) ctrl->b1 = ctrl->sum_abs;
  const double b1 = ctrl->b1;
  const double r = first ? ctrl->sum_abs_f32 : ctrl->sum_abs;
  const double mx = ctrl->max_abs;
  const double target = rel_tol * b1;
  double stage, T0;
  if (first) {
    stage = r > refresh_at * b1 ? fmax(target, refresh_at * b1) : 0.5 * target;
    T0 = fmin(mx / alpha, r / (double)(n > 1 ? n : 1));
  } else {
    stage = 0.5 * target;
    T0 = fmin(ctrl->T, mx / alpha);
  }
  T0 = fmax(T0, r * kPartTFloor);
  ctrl->destroyed = 0;
  ctrl->r0 = r;
  ctrl->target = stage;
  ctrl->T = T0;
  ctrl->ticket = 0;
  ctrl->passed = 0;
  // an abort raised during the previous stage skips this one too
  const int aborted = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
  ctrl->done = (ctrl->err != 0 || aborted || !(r > target)) ? 1 : 0;
}

// the zeroing part of k_part_prepare (counters, shares)
__global__ void k_part_clear(int* counters, float* S, int64_t n2) {
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  if (i0 < kCounters) counters[i0] = 0;
  for (int64_t i = i0; i < n2; i += stride) S[i] = 0.f;
}

int launch_part_stage(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, int first, double rel_tol,
                      double refresh_at, double alpha) {
  k_part_stage<<<1, 1, 0, c->stream>>>(c->ctrl, c->abort_dev, first, g->n, rel_tol, refresh_at, alpha);
  HIP_TRY(hipGetLastError());
  k_part_clear<<<std::min<int64_t>(4096, std::max<int64_t>(1, (2 * g->n + 255) / 256)), 256, 0, c->stream>>>(
      sb.counters, sb.S, 2 * g->n);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

int launch_part_prepare(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, double r0,
                        double target, double T0) {
  static_assert(kCounters <= 256, "the first block clears the counters");
  k_part_prepare<<<std::min<int64_t>(4096, std::max<int64_t>(1, (2 * g->n + 255) / 256)), 256, 0, c->stream>>>(
      c->ctrl, r0, target, T0, sb.counters, sb.S, 2 * g->n);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

// LDS of a partition workgroup: 20 bytes per node (+4) and 2 bytes per local
// target slot (two spare slots let the targets move as aligned 32-bit words)
size_t part_lds_bytes(int nodes, int local_edges, bool prio) {
  return (size_t)nodes * (prio ? 24 : 20) + 4 + (size_t)local_edges * 2 + 32;
}

// dynamic LDS both partition kernels may take (the larger static part counts)
int part_configure(ditr_ctx* c) {
  const void* fns[] = {reinterpret_cast<const void*>(&k_part_sweep<kPB, false>),
                       reinterpret_cast<const void*>(&k_part_resident<kPB, false, false>),
                       reinterpret_cast<const void*>(&k_part_resident<kPB, false, true>),
                       reinterpret_cast<const void*>(&k_part_sweep<kPB, true>),
                       reinterpret_cast<const void*>(&k_part_resident<kPB, true, false>),
                       reinterpret_cast<const void*>(&k_part_resident<kPB, true, true>),
                       reinterpret_cast<const void*>(&k_part_sweep<kPB / 2, false>),
                       reinterpret_cast<const void*>(&k_part_sweep<kPB / 2, true>),
                       reinterpret_cast<const void*>(&k_part_sweep<kPB / 4, false>),
                       reinterpret_cast<const void*>(&k_part_sweep<kPB / 4, true>)};
  size_t stat = 0;
  for (const void* fn : fns) {
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, fn) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(DITR_EHIP, "hipFuncGetAttributes failed");
    }
    stat = std::max(stat, at.sharedSizeBytes);
  }
  c->part_lds_static = stat;
  for (size_t total : {c->lds_per_cu, c->lds_per_block}) {
    if (total <= stat + 64) continue;
    const size_t dyn = total - stat;
    bool ok = true;
    for (const void* fn : fns)
      ok = ok && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) == hipSuccess;
    if (ok) {
      c->part_lds_dyn = dyn;
      return DITR_OK;
    }
    (void)hipGetLastError();
  }
  c->part_lds_dyn = c->lds_per_block > stat ? c->lds_per_block - stat : 0;
  return DITR_OK;
}

namespace {
int part_args(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, float* f, double* h, double alpha,
              int m, bool prio, PartArgs* out, size_t* lds) {
  const PartPlan& q = g->pp;
  PartArgs a;
  a.n = g->n;
  a.K = (int)g->K;
  a.m = m;
  a.part_ptr = g->part_ptr;
  a.col_ptr = g->col_ptr;
  a.loc_ptr = q.loc_ptr;
  a.loc_idx = q.loc_idx;
  a.inv = q.inv;
  a.ext_ptr = q.ext_ptr;
  a.ext_src = q.ext_src;
  a.ext_row = q.ext_row;
  a.part_items = q.part_items;
  a.item_row = q.item_row;
  a.unit_src = q.unit_src;
  a.unit_meta = q.unit_meta;
  a.item_word = sb.item_word;
  a.n_items = q.n_items;
  a.n_units = q.n_units;
  a.epoch0 = 0;
  a.F = f;
  a.H = h;
  a.S = sb.S;
  a.partials = sb.partials;
  a.counters = sb.counters;
  a.ctrl = c->ctrl;
  a.abort_flag = c->abort_dev;
  a.n_heavy = q.n_heavy;
  a.lds_nodes = std::max(1, g->max_part);
  a.prio = prio ? 1 : 0;
  a.row_ptr = g->row_ptr;
  a.max_levels = 0;
  a.alpha = (float)alpha;
  a.d = (float)g->d;
  a.dd = g->d;
  a.trace = c->trace;
  a.trace_cap = c->trace ? c->trace_cap : 0;
  a.tick_s = c->tick_s;
  if (part_lds_bytes(a.lds_nodes, 0, prio) > c->part_lds_dyn)
    return set_error(DITR_EINVAL, "partition of %d nodes needs %zu B of LDS (limit %zu)", a.lds_nodes,
                     part_lds_bytes(a.lds_nodes, 0, prio), c->part_lds_dyn);
  // local targets go to LDS when the largest partition's fit beside its nodes
  const int64_t room = ((int64_t)c->part_lds_dyn - (int64_t)part_lds_bytes(a.lds_nodes, 0, prio)) / 2;
  a.lds_edges = (int)std::max<int64_t>(0, std::min<int64_t>(room, (int64_t)q.max_local_edges + 2));
  *lds = part_lds_bytes(a.lds_nodes, a.lds_edges, prio);
  *out = a;
  return DITR_OK;
}
}  // namespace

int launch_part_sweeps(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, float* f, double* h,
                       double alpha, int m, int nlaunch, hipEvent_t* ev, bool prio) {
  PartArgs a;
  size_t lds = 0;
  int rc = part_args(c, g, sb, f, h, alpha, m, prio, &a, &lds);
  if (rc) return rc;
  const PartPlan& q = g->pp;
  // Every workgroup loads its partition, sweeps it in LDS and publishes it, one
  // after the other; a CU overlaps one workgroup's memory phases with another's
  // LDS sweeps only when several fit. Smaller partitions therefore run in
  // smaller workgroups: two of 512 threads per CU when the LDS of one fits in
  // half the CU's, four of 256 in a quarter.
  const size_t per_cu = c->lds_per_cu > c->part_lds_static ? c->lds_per_cu - c->part_lds_static : 0;
  const int block = lds * 4 <= per_cu ? kPB / 4 : lds * 2 <= per_cu ? kPB / 2 : kPB;
  for (int s = 0; s < nlaunch; ++s) {
    const int64_t units = q.n_units;
    if (units > 0)
      k_part_items<<<(unsigned)std::min<int64_t>((units + 3) / 4, 16384), 256, 0, c->stream>>>(a, s & 1);
    if (ev) HIP_TRY(hipEventRecord(ev[2 * s], c->stream));
    if (block == kPB) {
      if (prio) k_part_sweep<kPB, true><<<a.K, kPB, lds, c->stream>>>(a, s & 1);
      else k_part_sweep<kPB, false><<<a.K, kPB, lds, c->stream>>>(a, s & 1);
    } else if (block == kPB / 2) {
      if (prio) k_part_sweep<kPB / 2, true><<<a.K, kPB / 2, lds, c->stream>>>(a, s & 1);
      else k_part_sweep<kPB / 2, false><<<a.K, kPB / 2, lds, c->stream>>>(a, s & 1);
    } else {
      if (prio) k_part_sweep<kPB / 4, true><<<a.K, kPB / 4, lds, c->stream>>>(a, s & 1);
      else k_part_sweep<kPB / 4, false><<<a.K, kPB / 4, lds, c->stream>>>(a, s & 1);
    }
    if (ev) HIP_TRY(hipEventRecord(ev[2 * s + 1], c->stream));
  }
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

namespace {
// the resident sweep's instantiation for the node test and tracing
const void* resident_fn(bool prio, bool trace) {
  if (prio) return trace ? reinterpret_cast<const void*>(&k_part_resident<kPB, true, true>)
                         : reinterpret_cast<const void*>(&k_part_resident<kPB, true, false>);
  return trace ? reinterpret_cast<const void*>(&k_part_resident<kPB, false, true>)
               : reinterpret_cast<const void*>(&k_part_resident<kPB, false, false>);
}
}  // namespace

// Whether every partition workgroup of g can be resident at once (one
// cooperative launch of K workgroups).
int part_resident_fits(ditr_ctx* c, const ditr_graph* g, bool* fits, bool prio) {
  *fits = false;
  PartArgs a;
  size_t lds = 0;
  int rc = part_args(c, g, graph_bufs(g), nullptr, nullptr, 1.5, 1, prio, &a, &lds);
  if (rc) return rc;
  int per_cu = 0;
  const hipError_t oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, resident_fn(prio, c->trace != nullptr), kPB, lds);
  if (oe != hipSuccess) {
    (void)hipGetLastError();
    return DITR_OK;
  }
  *fits = (int64_t)per_cu * c->num_cus >= g->K;
  return DITR_OK;
}

int launch_part_resident(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, float* f, double* h,
                         double alpha, int m, int max_levels, bool prio) {
  PartArgs a;
  size_t lds = 0;
  int rc = part_args(c, g, sb, f, h, alpha, m, prio, &a, &lds);
  if (rc) return rc;
  a.max_levels = max_levels;
  // epochs of this launch's levels: above every flag an earlier launch stored
  const PartPlan& q = g->pp;
  if (*sb.epoch + max_levels + 1 >= (int64_t)1 << 30) {  // restart the epochs
    rc = launch_zero_u64(c, sb.item_word, 2 * (int64_t)std::max(1, q.n_items));
    if (rc) return rc;
    *sb.epoch = 0;
  }
  a.epoch0 = (int)(*sb.epoch + 1);
  *sb.epoch += max_levels + 1;
  // polls of about a microsecond: a stuck wait ends within seconds. The
  // environment variable DITR_SPIN_LIMIT lowers it (a test knob: 0 makes every
  // wait that is not already satisfied time out at its first poll, so the
  // error path runs with every wave leaving the kernel normally)
  int spin_limit = 1 << 24;
  if (const char* e = getenv("DITR_SPIN_LIMIT")) spin_limit = std::max(0, std::min(atoi(e), 1 << 24));
  // DITR_PLAIN_LAUNCH=1 dispatches the same grid with an ordinary launch.
  // part_resident_fits has checked that all K workgroups fit the device at
  // once, so on an otherwise idle device they are all resident; if some were
  // not, the bounded waits above end the launch with DITR_EHIP, never a hang.
  // It exists for profiler runs: rocprofv3 crashes at process exit after a
  // cooperative launch, once its results are written.
  const void* fn = resident_fn(prio, a.trace != nullptr);
  void* args[] = {&a, &spin_limit};
  const char* pe = getenv("DITR_PLAIN_LAUNCH");
  if (pe && atoi(pe) != 0) {
    HIP_TRY(hipLaunchKernel(fn, dim3(a.K), dim3(kPB), args, lds, c->stream));
    return DITR_OK;
  }
  HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(a.K), dim3(kPB), args, (unsigned)lds, c->stream));
  return DITR_OK;
}
