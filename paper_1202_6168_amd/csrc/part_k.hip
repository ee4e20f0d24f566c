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
#include <algorithm>
#include <vector>

#include "common.h"

namespace {

constexpr int kPB = 1024;     // threads per partition workgroup
constexpr int kStride = 4;    // doubles per block in the partials

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

__global__ void k_fill_local(int64_t n, const int32_t* __restrict__ col_ptr,
                             const int32_t* __restrict__ row_idx, const int32_t* __restrict__ pid,
                             const int32_t* __restrict__ part_ptr,
                             const int32_t* __restrict__ loc_ptr, uint16_t* loc_idx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t pi = pid[i], lo = part_ptr[pi];
    int32_t w = loc_ptr[i];
    for (int32_t e = col_ptr[i]; e < col_ptr[i + 1]; ++e) {
      const int32_t j = row_idx[e];
      if (pid[j] == pi) loc_idx[w++] = (uint16_t)(j - lo);
    }
  }
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
                           const int32_t* __restrict__ part_ptr,
                           const int32_t* __restrict__ light_ptr, const int32_t* __restrict__ heavy_ptr,
                           int32_t* ext_src, uint16_t* ext_row, int32_t* heavy_src) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t j = wid; j < n; j += nw) {
    const int32_t pj = pid[j];
    const bool heavy = heavy_ptr[j + 1] > heavy_ptr[j];
    int32_t w = heavy ? heavy_ptr[j] : light_ptr[j];
    const uint16_t jl = (uint16_t)(j - part_ptr[pj]);
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

__global__ void k_heavy_edge_rows(int32_t nh, const int32_t* __restrict__ rows,
                                  const int32_t* __restrict__ heavy_ptr, int32_t* hre) {
  for (int32_t h = blockIdx.x; h < nh; h += gridDim.x)
    for (int32_t e = heavy_ptr[rows[h]] + threadIdx.x; e < heavy_ptr[rows[h] + 1]; e += blockDim.x)
      hre[e] = h;
}

__global__ void k_heavy_list(int64_t n, const int32_t* __restrict__ heavy_ptr, int32_t* list,
                             int* count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += stride)
    if (heavy_ptr[j + 1] > heavy_ptr[j]) list[atomicAdd(count, 1)] = (int32_t)j;
}

__global__ void k_weights(int64_t n, const int32_t* __restrict__ col_ptr,
                          const int32_t* __restrict__ loc_ptr, float d, float* pw, int32_t* ext_deg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t k = col_ptr[i + 1] - col_ptr[i];
    pw[i] = k > 0 ? d / (float)k : 0.f;  // p_ji for every out-link of i
    ext_deg[i] = k - (loc_ptr[i + 1] - loc_ptr[i]);
  }
}

// ---------------------------------------------------------------- the sweep
struct PartArgs {
  int64_t n;
  int K;
  int m;  // local sweeps per launch
  const int32_t* __restrict__ part_ptr;
  const int32_t* __restrict__ col_ptr;
  const int32_t* __restrict__ loc_ptr;
  const uint16_t* __restrict__ loc_idx;
  const float* __restrict__ pw;
  const int32_t* __restrict__ ext_deg;
  const int32_t* __restrict__ ext_ptr;   // [K+1] light external in-links of each partition
  const int32_t* __restrict__ ext_src;
  const uint16_t* __restrict__ ext_row;
  const int32_t* __restrict__ heavy_rows;
  const int32_t* __restrict__ part_heavy;  // [K+1] heavy rows of each partition (ranges of heavy_rows)
  const int32_t* __restrict__ heavy_src;
  const int32_t* __restrict__ heavy_edge_row;  // heavy link -> index into heavy_rows
  int64_t n_heavy_edges;
  float* F;
  double* H;
  float* S;          // [2][n] published p_i dH_i
  double* heavy_in;  // [n_heavy] inflow of heavy rows in the current launch
  double* partials;
  int* counters;     // [1] finished workgroups (reset by the last)
  int n_chunks;
  Ctrl* ctrl;
  int n_heavy;
  int lds_nodes;   // node capacity of the LDS layout
  int lds_edges;   // local-target capacity (a larger partition reads its targets from memory)
  float alpha;
  float d;
  double dd;  // damping in FP64 for the published shares
};

// lane owning edge slot e: first lane whose inclusive prefix exceeds e
__device__ __forceinline__ int owner_of(int incl, int e) {
  int k = 0;
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    int v = __shfl(incl, k + s - 1, 64);
    if (v <= e) k += s;
  }
  return k;
}

// Inflow of the heavy rows, summed right before the partition launch that
// consumes it. The external in-links of all heavy rows form one list in row
// order; workgroup c sums the range [c kHeavyChunk, (c+1) kHeavyChunk) of it:
// each thread reduces a run of consecutive links per row, the runs meet in
// FP64 LDS slots (one per row of the range), and each slot goes to heavy_in
// with one device atomic. The partition owning the row clears it after use.
__global__ void __launch_bounds__(256) k_part_heavy(PartArgs a, int parity) {
  if (__hip_atomic_load(&a.ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const float* S_in = a.S + (size_t)(parity ^ 1) * a.n;
  __shared__ double acc[kHeavyChunk];
  const int tid = threadIdx.x;
  const int64_t beg = (int64_t)blockIdx.x * kHeavyChunk;
  const int64_t end = beg + kHeavyChunk < a.n_heavy_edges ? beg + kHeavyChunk : a.n_heavy_edges;
  const int h0 = a.heavy_edge_row[beg];
  const int nslot = a.heavy_edge_row[end - 1] - h0 + 1;
  for (int k = tid; k < nslot; k += 256) acc[k] = 0.0;
  __syncthreads();
  constexpr int R = kHeavyChunk / 256;  // consecutive links per thread
  const int64_t e0 = beg + (int64_t)tid * R;
  int hk[R];
  float v[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {  // all loads first
    const int64_t e = e0 + k;
    hk[k] = e < end ? a.heavy_edge_row[e] : -1;
    v[k] = e < end ? S_in[a.heavy_src[e]] : 0.f;
  }
  double run = 0;
  int hr = hk[0];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (hk[k] < 0) break;
    if (hk[k] != hr) {
      if (run != 0.0) atomicAdd(&acc[hr - h0], run);  // ds_add_f64
      run = 0;
      hr = hk[k];
    }
    run += (double)v[k];
  }
  if (hr >= 0 && run != 0.0) atomicAdd(&acc[hr - h0], run);
  __syncthreads();
  for (int k = tid; k < nslot; k += 256)
    if (acc[k] != 0.0) add_agent(&a.heavy_in[h0 + k], acc[k]);
}

// One launch of the partitioned sweep. Workgroup p:
//   1. loads Omega_p into LDS (fluid, history increment, local CSC);
//   2. adds the outside fluid: heavy rows take what k_part_heavy summed for
//      them, light rows pull S_in over their external in-links;
//   3. runs up to m threshold sweeps at the launch's T until none passes;
//   4. writes F and H back and publishes S_out = p_i dH_i;
//   5. the last workgroup to finish reduces the per-workgroup sums and sets
//      the next T and the stop flag (no separate step kernel).
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_part_sweep(PartArgs a, int parity) {
  if (__hip_atomic_load(&a.ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const float* S_in = a.S + (size_t)(parity ^ 1) * a.n;
  float* S_out = a.S + (size_t)parity * a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = BLOCK / 64;
  __shared__ double red[4][NW];
  __shared__ uint8_t s_mark[NW][2][64];  // per-wave scratch of the edge expansion
  __shared__ int s_off[NW][64];
  __shared__ float s_w[NW][64];
  __shared__ int s_last;

  // LDS: fluid, history increment, local CSC (offsets, out-degree, targets)
  extern __shared__ __align__(16) unsigned char smem[];
  const int cap = a.lds_nodes;
  double* dH = reinterpret_cast<double*>(smem);
  float* Fl = reinterpret_cast<float*>(smem + (size_t)cap * 8);
  int32_t* lptr = reinterpret_cast<int32_t*>(smem + (size_t)cap * 12);
  int32_t* odeg = reinterpret_cast<int32_t*>(smem + (size_t)cap * 16 + 4);
  uint32_t* lidx_words = reinterpret_cast<uint32_t*>(smem + (size_t)cap * 20 + 4);
  const int p = blockIdx.x;
  const int lo = a.part_ptr[p], np = a.part_ptr[p + 1] - lo;
  const int lbase = a.loc_ptr[lo];
  const int nl = a.loc_ptr[lo + np] - lbase;
  const bool lidx_in_lds = nl + 2 <= a.lds_edges;
  // the LDS copy keeps the parity of lbase so that it moves whole 32-bit words
  const uint16_t* lidx = lidx_in_lds ? reinterpret_cast<const uint16_t*>(lidx_words) + (lbase & 1)
                                     : a.loc_idx + lbase;

  // ---- 1. load the partition (several loads in flight per thread)
  {
    constexpr int U = 4;
    for (int i0 = tid; i0 < np; i0 += U * BLOCK) {
      float f[U];
      int32_t lp[U], c0[U], c1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * BLOCK;
        if (i < np) {
          f[u] = a.F[lo + i];
          lp[u] = a.loc_ptr[lo + i];
          c0[u] = a.col_ptr[lo + i];
          c1[u] = a.col_ptr[lo + i + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * BLOCK;
        if (i < np) {
          Fl[i] = f[u];
          dH[i] = 0.0;
          lptr[i] = lp[u] - lbase;
          odeg[i] = c1[u] - c0[u];
        }
      }
    }
  }
  if (tid == 0) lptr[np] = nl;
  if (lidx_in_lds) {
    constexpr int U = 8;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.loc_idx) + (lbase >> 1);
    const int words = ((lbase & 1) + nl + 1) >> 1;
    for (int w0 = tid; w0 < words; w0 += U * BLOCK) {
      uint32_t v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (w0 + u * BLOCK < words) v[u] = src[w0 + u * BLOCK];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (w0 + u * BLOCK < words) lidx_words[w0 + u * BLOCK] = v[u];
    }
  }
  __syncthreads();

  // ---- 2. outside fluid
  for (int h = a.part_heavy[p] + tid; h < a.part_heavy[p + 1]; h += BLOCK) {
    Fl[a.heavy_rows[h] - lo] += (float)a.heavy_in[h];  // summed by k_part_heavy just before
    a.heavy_in[h] = 0.0;
  }
  {
    const int e0 = a.ext_ptr[p], e1 = a.ext_ptr[p + 1];
    int e = e0 + tid;
    for (; e + 3 * BLOCK < e1; e += 4 * BLOCK) {  // four gathers in flight
      const int32_t s0 = a.ext_src[e], s1 = a.ext_src[e + BLOCK], s2 = a.ext_src[e + 2 * BLOCK],
                    s3 = a.ext_src[e + 3 * BLOCK];
      const uint16_t r0 = a.ext_row[e], r1 = a.ext_row[e + BLOCK], r2 = a.ext_row[e + 2 * BLOCK],
                     r3 = a.ext_row[e + 3 * BLOCK];
      const float v0 = S_in[s0], v1 = S_in[s1], v2 = S_in[s2], v3 = S_in[s3];
      if (v0 != 0.f) atomicAdd(&Fl[r0], v0);
      if (v1 != 0.f) atomicAdd(&Fl[r1], v1);
      if (v2 != 0.f) atomicAdd(&Fl[r2], v2);
      if (v3 != 0.f) atomicAdd(&Fl[r3], v3);
    }
    for (; e < e1; e += BLOCK) {
      const float v = S_in[a.ext_src[e]];
      if (v != 0.f) atomicAdd(&Fl[a.ext_row[e]], v);
    }
  }
  __syncthreads();

  // ---- 3. local threshold sweeps at one T until none passes (at most m)
  const float T = (float)a.ctrl->T;
  const float d = a.d;
  double edges = 0, diffs = 0;
  for (int s = 0; s < a.m; ++s) {
    int passed = 0;
    for (int base = wave * 64; base < np; base += NW * 64) {
      const int i = base + lane;
      float sent = 0.f;
      int ldeg = 0, src0 = 0;
      float w = 0.f;
      if (i < np && fabsf(Fl[i]) > T) {
        sent = atomicExch(&Fl[i], 0.f);
        dH[i] += (double)sent;
        src0 = lptr[i];
        ldeg = lptr[i + 1] - src0;
        const int od = odeg[i];
        w = od > 0 ? sent * (d / (float)od) : 0.f;
        edges += (double)od;
        diffs += 1.0;
        passed = 1;
      }
      // out-links of the passing nodes laid end to end; each lane takes every
      // 64th one. The owner of slot e is found by marking each segment's first
      // slot of the window in LDS and taking a running max across the lanes.
      // Two windows per step keep two dependency chains in flight.
      const int incl = wave_incl_scan_dpp(ldeg);
      const int total = __builtin_amdgcn_readlane(incl, 63);
      if (total == 0) continue;
      const int excl = incl - ldeg;
      s_off[wave][lane] = src0 - excl;
      s_w[wave][lane] = w;
      for (int e0 = 0; e0 < total; e0 += 128) {
        s_mark[wave][0][lane] = 0;
        s_mark[wave][1][lane] = 0;
        __builtin_amdgcn_wave_barrier();
        if (ldeg > 0 && incl > e0 && excl < e0 + 64)
          s_mark[wave][0][max(excl, e0) - e0] = (uint8_t)(lane + 1);
        if (ldeg > 0 && incl > e0 + 64 && excl < e0 + 128)
          s_mark[wave][1][max(excl, e0 + 64) - e0 - 64] = (uint8_t)(lane + 1);
        __builtin_amdgcn_wave_barrier();
        const int ownA = wave_incl_max_dpp((int)s_mark[wave][0][lane]) - 1;
        const int ownB = max(wave_incl_max_dpp((int)s_mark[wave][1][lane]) - 1, 0);
        const int eA = e0 + lane, eB = e0 + 64 + lane;
        const int tA = eA < total ? (int)lidx[s_off[wave][ownA] + eA] : -1;
        const int tB = eB < total ? (int)lidx[s_off[wave][ownB] + eB] : -1;
        const float wA = s_w[wave][ownA], wB = s_w[wave][ownB];
        if (tA >= 0) atomicAdd(&Fl[tA], wA);  // ds_add_f32
        if (tB >= 0) atomicAdd(&Fl[tB], wB);
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (!__syncthreads_or(passed)) break;  // barrier + "did any node pass"
  }

  // ---- 4. write back, publish p_i dH_i, partial sums
  double resid = 0, fmx = 0;
  {
    constexpr int U = 4;
    for (int i0 = tid; i0 < np; i0 += U * BLOCK) {
      double hv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * BLOCK;
        hv[u] = (i < np && dH[i] != 0.0) ? a.H[lo + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * BLOCK;
        if (i >= np) continue;
        const float f = Fl[i];
        const double dh = dH[i];
        a.F[lo + i] = f;
        float so = 0.f;
        if (dh != 0.0) {
          a.H[lo + i] = hv[u] + dh;
          const int od = odeg[i];
          if (od > 0) {
            so = (float)(a.dd * dh / (double)od);
            // in flight to the outside targets of i
            resid += fabs((double)so) * (double)(od - (lptr[i + 1] - lptr[i]));
          }
        }
        S_out[lo + i] = so;
        resid += fabs((double)f);
        fmx = fmax(fmx, fabs((double)f));
      }
    }
  }

  // ---- 5. per-workgroup sums; the last workgroup finishes the launch
  resid = wave_sum(resid);
  fmx = wave_maxd(fmx);
  edges = wave_sum(edges);
  diffs = wave_sum(diffs);
  if (lane == 0) {
    red[0][wave] = resid;
    red[1][wave] = fmx;
    red[2][wave] = edges;
    red[3][wave] = diffs;
  }
  __syncthreads();
  if (tid == 0) {
    double r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    for (int w = 0; w < NW; ++w) {
      r0 += red[0][w];
      r1 = fmax(r1, red[1][w]);
      r2 += red[2][w];
      r3 += red[3][w];
    }
    double* q = a.partials + (size_t)kStride * p;
    __hip_atomic_store(&q[0], r0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q[1], r1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q[2], r2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&q[3], r3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  D = wave_sum(D);
  E = wave_sum(E);
  P = wave_sum(P);
  M = wave_maxd(M);
  __syncthreads();
  if (lane == 0) {
    red[0][wave] = D;
    red[1][wave] = M;
    red[2][wave] = E;
    red[3][wave] = P;
  }
  __syncthreads();
  if (tid == 0) {
    D = 0, M = 0, E = 0, P = 0;
    for (int w = 0; w < NW; ++w) {
      D += red[0][w];
      M = fmax(M, red[1][w]);
      E += red[2][w];
      P += red[3][w];
    }
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
      ctrl->T = Tn;
    }
    a.counters[1] = 0;  // finish count of the next launch
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

// exclusive scan (graph_k.hip)
int scan_exclusive_i32(ditr_ctx* c, const int32_t* in, int64_t n, int32_t* out);

void free_part_plan(ditr_graph* g) {
  PartPlan& q = g->pp;
  for (void* p : {(void*)q.pid, (void*)q.loc_ptr, (void*)q.loc_idx, (void*)q.pw, (void*)q.ext_deg,
                  (void*)q.ext_ptr, (void*)q.ext_src, (void*)q.ext_row, (void*)q.heavy_rows,
                  (void*)q.part_heavy, (void*)q.heavy_src, (void*)q.heavy_edge_row, (void*)q.S,
                  (void*)q.heavy_in, (void*)q.partials, (void*)q.counters})
    (void)hipFree(p);
  q = PartPlan();
}

// Build the partitioned-sweep tables for the current partition plan of g.
int build_part_plan(ditr_ctx* c, ditr_graph* g) {
  free_part_plan(g);
  PartPlan& q = g->pp;
  const int64_t n = g->n;
  const int K = (int)g->K;
  hipStream_t st = c->stream;
  int32_t *cnt = nullptr, *cnt2 = nullptr, *light_ptr = nullptr, *heavy_ptr = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    (void)hipFree(cnt);
    (void)hipFree(cnt2);
    (void)hipFree(light_ptr);
    (void)hipFree(heavy_ptr);
  };
#define PP_TRY(expr)                                                                     \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      cleanup();                                                                         \
      return set_error(DITR_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e));        \
    }                                                                                    \
  } while (0)
  if (g->max_part > 65536) return set_error(DITR_EINVAL, "partitions above 65536 nodes");
  PP_TRY(hipMalloc((void**)&q.pid, sizeof(int32_t) * n));
  PP_TRY(hipMalloc((void**)&q.loc_ptr, sizeof(int32_t) * (n + 1)));
  PP_TRY(hipMalloc((void**)&cnt, sizeof(int32_t) * (n + 1)));
  PP_TRY(hipMalloc((void**)&cnt2, sizeof(int32_t) * (n + 1)));
  PP_TRY(hipMalloc((void**)&light_ptr, sizeof(int32_t) * (n + 1)));
  PP_TRY(hipMalloc((void**)&heavy_ptr, sizeof(int32_t) * (n + 1)));
  const int gb = grid_for(n, 256, 8192);
  const int gw = grid_for(n * 64, 256, 16384);  // one wave per row
  k_fill_pid<<<std::min(K, 8192), 256, 0, st>>>(K, g->part_ptr, q.pid);
  k_count_local<<<gb, 256, 0, st>>>(n, g->col_ptr, g->row_idx, q.pid, cnt);
  PP_TRY(hipGetLastError());
  int rc = scan_exclusive_i32(c, cnt, n, q.loc_ptr);
  if (rc) { cleanup(); return rc; }
  int32_t nloc = 0;
  PP_TRY(hipMemcpy(&nloc, q.loc_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost));
  PP_TRY(hipMalloc((void**)&q.loc_idx, sizeof(uint16_t) * (nloc + 4)));  // word copies may overrun by one
  k_fill_local<<<gb, 256, 0, st>>>(n, g->col_ptr, g->row_idx, q.pid, g->part_ptr, q.loc_ptr, q.loc_idx);
  k_count_ext<<<gw, 256, 0, st>>>(n, g->row_ptr, g->csr_col, q.pid, cnt, cnt2);
  PP_TRY(hipGetLastError());
  rc = scan_exclusive_i32(c, cnt, n, light_ptr);
  if (!rc) rc = scan_exclusive_i32(c, cnt2, n, heavy_ptr);
  if (rc) { cleanup(); return rc; }
  int32_t nlight = 0, nheavy_e = 0;
  PP_TRY(hipMemcpy(&nlight, light_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost));
  PP_TRY(hipMemcpy(&nheavy_e, heavy_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost));
  PP_TRY(hipMalloc((void**)&q.ext_src, sizeof(int32_t) * std::max(1, nlight)));
  PP_TRY(hipMalloc((void**)&q.ext_row, sizeof(uint16_t) * std::max(1, nlight)));
  PP_TRY(hipMalloc((void**)&q.heavy_src, sizeof(int32_t) * std::max(1, nheavy_e)));
  PP_TRY(hipMalloc((void**)&q.ext_ptr, sizeof(int32_t) * (K + 1)));
  k_fill_ext<<<gw, 256, 0, st>>>(n, g->row_ptr, g->csr_col, q.pid, g->part_ptr, light_ptr, heavy_ptr,
                                 q.ext_src, q.ext_row, q.heavy_src);
  k_gather_ptr<<<grid_for(K + 1, 256, 1024), 256, 0, st>>>(K, g->part_ptr, light_ptr, q.ext_ptr);
  PP_TRY(hipGetLastError());
  // heavy rows (sorted) and their chunks; per-partition ranges of the heavy list
  int* hcount = &c->ctrl->err;
  PP_TRY(hipMemsetAsync(hcount, 0, sizeof(int), st));
  PP_TRY(hipMalloc((void**)&q.heavy_rows, sizeof(int32_t) * std::max<int64_t>(1, n)));
  k_heavy_list<<<gb, 256, 0, st>>>(n, heavy_ptr, q.heavy_rows, hcount);
  int nh = 0;
  PP_TRY(hipMemcpyAsync(&nh, hcount, sizeof(int), hipMemcpyDeviceToHost, st));
  PP_TRY(hipStreamSynchronize(st));
  std::vector<int32_t> rows(nh);
  if (nh > 0) {
    PP_TRY(hipMemcpy(rows.data(), q.heavy_rows, sizeof(int32_t) * nh, hipMemcpyDeviceToHost));
    std::sort(rows.begin(), rows.end());
    PP_TRY(hipMemcpy(q.heavy_rows, rows.data(), sizeof(int32_t) * nh, hipMemcpyHostToDevice));
  }
  std::vector<int32_t> ph(K + 1);
  {
    size_t r = 0;
    for (int k = 0; k <= K; ++k) {
      const int64_t lo = g->part_ptr_host[k];
      while (r < rows.size() && rows[r] < lo) ++r;
      ph[k] = (int32_t)r;
    }
  }
  PP_TRY(hipMalloc((void**)&q.heavy_edge_row, sizeof(int32_t) * std::max(1, nheavy_e)));
  if (nh > 0)
    k_heavy_edge_rows<<<std::min(nh, 4096), 256, 0, st>>>(nh, q.heavy_rows, heavy_ptr, q.heavy_edge_row);
  PP_TRY(hipGetLastError());
  q.n_heavy = nh;
  q.n_chunks = (int32_t)(((int64_t)nheavy_e + kHeavyChunk - 1) / kHeavyChunk);
  PP_TRY(hipMalloc((void**)&q.part_heavy, sizeof(int32_t) * (K + 1)));
  PP_TRY(hipMemcpy(q.part_heavy, ph.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice));
  PP_TRY(hipMalloc((void**)&q.pw, sizeof(float) * n));
  PP_TRY(hipMalloc((void**)&q.ext_deg, sizeof(int32_t) * n));
  k_weights<<<gb, 256, 0, st>>>(n, g->col_ptr, q.loc_ptr, (float)g->d, q.pw, q.ext_deg);
  PP_TRY(hipGetLastError());
  PP_TRY(hipMalloc((void**)&q.S, sizeof(float) * 2 * n));
  PP_TRY(hipMalloc((void**)&q.heavy_in, sizeof(double) * std::max(1, nh)));
  PP_TRY(hipMalloc((void**)&q.counters, sizeof(int) * 2));
  PP_TRY(hipMemset(q.counters, 0, sizeof(int) * 2));
  PP_TRY(hipMalloc((void**)&q.partials, sizeof(double) * kStride * K));
  {
    std::vector<int32_t> lp(K + 1);
    int32_t* d_lp = nullptr;
    PP_TRY(hipMalloc((void**)&d_lp, sizeof(int32_t) * (K + 1)));
    k_gather_ptr<<<grid_for(K + 1, 256, 1024), 256, 0, st>>>(K, g->part_ptr, q.loc_ptr, d_lp);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(lp.data(), d_lp, sizeof(int32_t) * (K + 1), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_lp);
    PP_TRY(e);
    int32_t mx = 0;
    for (int k = 0; k < K; ++k) mx = std::max(mx, lp[k + 1] - lp[k]);
    q.max_local_edges = mx;
  }
  q.n_local = nloc;
  q.n_ext = nlight;
  q.n_heavy_edges = nheavy_e;
  cleanup();
  q.ready = true;
#undef PP_TRY
  return DITR_OK;
}

__global__ void k_zero_i32p(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

int launch_part_prepare(ditr_ctx* c, const ditr_graph* g) {
  const PartPlan& q = g->pp;
  k_zero_i32p<<<1, 64, 0, c->stream>>>(q.counters, 2);
  k_zero_f32p<<<std::min<int64_t>(4096, (2 * g->n + 255) / 256), 256, 0, c->stream>>>(q.S, 2 * g->n);
  if (q.n_heavy > 0)
    k_zero_f64p<<<std::min(1024, (q.n_heavy + 255) / 256), 256, 0, c->stream>>>(
        q.heavy_in, (int64_t)q.n_heavy);
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}

// LDS of a partition workgroup: 20 bytes per node (+4) and 2 bytes per local
// target slot (two spare slots let the targets move as aligned 32-bit words)
size_t part_lds_bytes(int nodes, int local_edges) {
  return (size_t)nodes * 20 + 4 + (size_t)local_edges * 2 + 16;
}

int part_configure(ditr_ctx* c) {
  hipFuncAttributes attr;
  if (hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_part_sweep<kPB>)) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(DITR_EHIP, "hipFuncGetAttributes failed");
  }
  for (size_t total : {c->lds_per_cu, c->lds_per_block}) {
    if (total <= attr.sharedSizeBytes + 64) continue;
    const size_t dyn = total - attr.sharedSizeBytes;
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_part_sweep<kPB>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) == hipSuccess) {
      c->part_lds_dyn = dyn;
      return DITR_OK;
    }
    (void)hipGetLastError();
  }
  c->part_lds_dyn = c->lds_per_block > attr.sharedSizeBytes ? c->lds_per_block - attr.sharedSizeBytes : 0;
  return DITR_OK;
}

int launch_part_sweeps(ditr_ctx* c, const ditr_graph* g, float* f, double* h, double alpha, int m,
                       int nlaunch, hipEvent_t* ev) {
  const PartPlan& q = g->pp;
  PartArgs a;
  a.n = g->n;
  a.K = (int)g->K;
  a.m = m;
  a.part_ptr = g->part_ptr;
  a.col_ptr = g->col_ptr;
  a.loc_ptr = q.loc_ptr;
  a.loc_idx = q.loc_idx;
  a.pw = q.pw;
  a.ext_deg = q.ext_deg;
  a.ext_ptr = q.ext_ptr;
  a.ext_src = q.ext_src;
  a.ext_row = q.ext_row;
  a.heavy_rows = q.heavy_rows;
  a.part_heavy = q.part_heavy;
  a.heavy_src = q.heavy_src;
  a.heavy_edge_row = q.heavy_edge_row;
  a.n_heavy_edges = q.n_heavy_edges;
  a.F = f;
  a.H = h;
  a.S = q.S;
  a.heavy_in = q.heavy_in;
  a.partials = q.partials;
  a.counters = q.counters;
  a.n_chunks = q.n_chunks;
  a.ctrl = c->ctrl;
  a.n_heavy = q.n_heavy;
  a.lds_nodes = std::max(1, g->max_part);
  a.alpha = (float)alpha;
  a.d = (float)g->d;
  a.dd = g->d;
  if (part_lds_bytes(a.lds_nodes, 0) > c->part_lds_dyn)
    return set_error(DITR_EINVAL, "partition of %d nodes needs %zu B of LDS (limit %zu)", a.lds_nodes,
                     part_lds_bytes(a.lds_nodes, 0), c->part_lds_dyn);
  // local targets go to LDS when the largest partition's fit beside its nodes
  const int64_t room = ((int64_t)c->part_lds_dyn - (int64_t)part_lds_bytes(a.lds_nodes, 0)) / 2;
  a.lds_edges = (int)std::max<int64_t>(0, std::min<int64_t>(room, (int64_t)q.max_local_edges + 2));
  const size_t lds = part_lds_bytes(a.lds_nodes, a.lds_edges);
  for (int s = 0; s < nlaunch; ++s) {
    if (q.n_chunks > 0) k_part_heavy<<<q.n_chunks, 256, 0, c->stream>>>(a, s & 1);
    if (ev) HIP_TRY(hipEventRecord(ev[2 * s], c->stream));
    k_part_sweep<kPB><<<a.K, kPB, lds, c->stream>>>(a, s & 1);
    if (ev) HIP_TRY(hipEventRecord(ev[2 * s + 1], c->stream));
  }
  HIP_TRY(hipGetLastError());
  return DITR_OK;
}
