// C-ABI of the ditr library: context, graph upload and partition plan,
// exact residual, and the host driver of the plain solve.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include "common.h"

int persistent_occupancy(ditr_ctx* c, int block, size_t lds, int* per_cu);

namespace {
thread_local char g_err[1024] = "";

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t lds_bytes_for(int nodes) {
  return (((size_t)nodes * 4 + 15) & ~(size_t)15) + (size_t)nodes * 8;
}

int read_ctrl(ditr_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return DITR_OK;
}

// Largest dynamic LDS (bytes) a persistent workgroup of `block` threads may take.
int max_dynamic_lds(ditr_ctx* c, int block, size_t* out) {
  const int slot = block == 256 ? 0 : block == 512 ? 1 : block == 1024 ? 2 : -1;
  if (slot < 0) return set_error(DITR_EINVAL, "block must be 256, 512 or 1024");
  *out = c->lds_dyn[slot];
  return DITR_OK;
}

}  // namespace

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

// the partition count a plan starts from (the plan loop only raises it):
// part_nodes per partition, or about 4096 nodes per partition and at least one
// partition per CU when n allows
int64_t initial_parts(const ditr_ctx* c, int64_t n, int32_t part_nodes) {
  int64_t K = part_nodes > 0 ? (n + part_nodes - 1) / part_nodes
                             : std::max<int64_t>((n + 4095) / 4096, std::min<int64_t>(c->num_cus, n / 256));
  return std::max<int64_t>(1, std::min<int64_t>(K, n));
}

extern "C" {

int ditr_version(void) { return DITR_ABI_VERSION; }

const char* ditr_last_error(void) { return g_err; }

int ditr_opts_default(ditr_opts* o) {
  if (!o) return set_error(DITR_EINVAL, "opts is NULL");
  memset(o, 0, sizeof(*o));
  o->alpha = 2.0;
  o->refresh_at = 0;  // the library's choice for the mode
  o->park_ratio = 0.5;
  o->rescale_cap = 4.0;
  o->mode = DITR_MODE_AUTO;
  o->part_type = DITR_PART_MINCUT;
  o->part_nodes = 0;
  o->block = 1024;
  o->wg_per_cu = 1;
  o->sweeps_per_claim = 0;
  o->max_rounds = 16;
  o->max_sweeps = 0;
  o->xcd_remap = 1;
  o->flags = 0;
  return DITR_OK;
}

int ditr_create(ditr_ctx** out, int device, void* hip_stream) {
  if (!out) return set_error(DITR_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error(DITR_EINVAL, "no device %d", device);
  HIP_TRY(hipSetDevice(device));
  ditr_ctx* c = new (std::nothrow) ditr_ctx();
  if (!c) return set_error(DITR_ENOMEM, "host allocation failed");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete c;
    return set_error(DITR_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  }
  c->num_cus = prop.multiProcessorCount;
  {
    int khz = 0;  // s_memrealtime runs at the device's wall-clock rate
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) {
      (void)hipGetLastError();
      khz = 100000;
    }
    c->tick_s = 1e-3 / (double)khz;
  }
  c->lds_per_block = prop.sharedMemPerBlock;
  c->lds_per_cu = std::max<size_t>(prop.maxSharedMemoryPerMultiProcessor, prop.sharedMemPerBlock);
  persistent_configure(c, c->lds_per_cu, c->lds_per_block);
  part_configure(c);
  c->partials_cap = 8192;
  bool ok = hipHostMalloc((void**)&c->abort_host, sizeof(int), hipHostMallocMapped) == hipSuccess &&
            hipHostGetDevicePointer((void**)&c->abort_dev, c->abort_host, 0) == hipSuccess &&
            hipMalloc((void**)&c->ctrl, sizeof(Ctrl)) == hipSuccess &&
            hipHostMalloc((void**)&c->ctrl_host, sizeof(Ctrl), hipHostMallocDefault) == hipSuccess &&
            hipMalloc((void**)&c->partials, sizeof(double) * 4 * c->partials_cap) == hipSuccess &&
            hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    ditr_destroy(c);
    return set_error(DITR_ENOMEM, "device or pinned allocation failed");
  }
  *c->abort_host = 0;
  const int nrc = noalloc_init(c);
  if (nrc) {
    ditr_destroy(c);
    return nrc;
  }
  if (hipMemset(c->ctrl, 0, sizeof(Ctrl)) != hipSuccess) {
    ditr_destroy(c);
    return set_error(DITR_EHIP, "hipMemset failed");
  }
  *out = c;
  return DITR_OK;
}

int ditr_destroy(ditr_ctx* c) {
  if (!c) return DITR_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->work) (void)hipStreamDestroy(c->work);
  if (c->abort_host) (void)hipHostFree(c->abort_host);
  if (c->ctrl) (void)hipFree(c->ctrl);
  if (c->ctrl_host) (void)hipHostFree(c->ctrl_host);
  if (c->partials) (void)hipFree(c->partials);
  delete c;
  return DITR_OK;
}

int ditr_abort(ditr_ctx* c) {
  if (!c || !c->abort_host) return set_error(DITR_EINVAL, "ctx is NULL");
  __atomic_store_n(c->abort_host, 1, __ATOMIC_SEQ_CST);
  return DITR_OK;
}

int ditr_set_trace(ditr_ctx* c, double* d_trace, int64_t capacity) {
  if (!c) return set_error(DITR_EINVAL, "ctx is NULL");
  if (capacity < 0) return set_error(DITR_EINVAL, "negative trace capacity");
  c->trace = capacity > 0 ? d_trace : nullptr;
  c->trace_cap = d_trace ? capacity : 0;
  return DITR_OK;
}

int ditr_partition(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* d_col_ptr,
                   const int32_t* d_row_idx, int part_type, int64_t K, int64_t* d_ptr) {
  if (!c || !d_col_ptr || !d_ptr) return set_error(DITR_EINVAL, "NULL argument");
  if (n < 1 || K < 1 || K > n) return set_error(DITR_EINVAL, "need 1 <= K <= n");
  if (part_type == DITR_PART_PMASS)
    return set_error(DITR_EINVAL, "the internal-mass partition needs the weights: use ditr_partition_pmass");
  if (part_type != DITR_PART_CB && part_type != DITR_PART_UNIFORM && part_type != DITR_PART_CB_INOUT &&
      part_type != DITR_PART_MINCUT)
    return set_error(DITR_EINVAL, "unknown partition type %d", part_type);
  if ((part_type == DITR_PART_CB_INOUT || part_type == DITR_PART_MINCUT) && nnz > 0 && !d_row_idx)
    return set_error(DITR_EINVAL, "this partition type needs the row indices");
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return set_error(DITR_EINVAL, "nnz out of range");
  HIP_TRY(hipSetDevice(c->device));
  if (part_type != DITR_PART_CB_INOUT && part_type != DITR_PART_MINCUT)
    return launch_partition(c, n, d_col_ptr, nullptr, part_type, K, d_ptr, nullptr);
  int32_t* in_prefix = nullptr;
  HIP_TRY(hipMalloc((void**)&in_prefix, sizeof(int32_t) * (n + 1)));
  int rc = launch_in_prefix(c, n, nnz, d_row_idx, in_prefix);
  if (!rc)
    rc = part_type == DITR_PART_MINCUT
             ? launch_partition_mincut(c, n, nnz, d_col_ptr, d_row_idx, in_prefix, K, d_ptr, nullptr)
             : launch_partition(c, n, d_col_ptr, in_prefix, part_type, K, d_ptr, nullptr);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(in_prefix);
  return rc;
}

int ditr_partition_pmass(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* d_col_ptr,
                         const int32_t* d_row_idx, const double* d_val, double damping, int64_t K,
                         int64_t* d_ptr) {
  if (!c || !d_col_ptr || !d_ptr || (nnz > 0 && !d_row_idx)) return set_error(DITR_EINVAL, "NULL argument");
  if (n < 1 || K < 1 || K > n) return set_error(DITR_EINVAL, "need 1 <= K <= n");
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return set_error(DITR_EINVAL, "nnz out of range");
  if (!d_val && !(damping > 0 && damping < 1)) return set_error(DITR_EINVAL, "damping must lie in (0, 1)");
  HIP_TRY(hipSetDevice(c->device));
  return launch_partition_pmass(c, n, nnz, d_col_ptr, d_row_idx, d_val, damping, K, d_ptr, nullptr);
}

int ditr_graph_destroy(ditr_graph* g) {
  if (!g) return DITR_OK;
  // the graph may outlive its context: use its own device id, and wait for the
  // whole device rather than the context's stream
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)g->row_ptr, (void*)g->csr_col, (void*)g->csr_val, (void*)g->colabs,
                  (void*)g->heavy_rows, (void*)g->chunk_h, (void*)g->chunk_beg, (void*)g->chunk_end,
                  (void*)g->chunk_sum, (void*)g->pull_s, (void*)g->pull_heavy, (void*)g->pull_partials,
                  (void*)g->wh, (void*)g->part_ptr, (void*)g->part_T, (void*)g->part_lock})
    g_free(g, p);
  delete[] g->part_ptr_host;
  free_part_plan(g);
  delete g;
  return DITR_OK;
}

// (re)build the partition plan with K parts; reads the boundaries back
static int make_plan(ditr_ctx* c, ditr_graph* g, int64_t K) {
  g_free(g, g->part_ptr);
  g_free(g, g->part_T);
  g_free(g, g->part_lock);
  g->part_ptr = nullptr;
  g->part_T = nullptr;
  g->part_lock = nullptr;
  delete[] g->part_ptr_host;
  g->part_ptr_host = new (std::nothrow) int64_t[K + 1];
  if (!g->part_ptr_host) return set_error(DITR_ENOMEM, "host allocation failed");
  g->K = K;
  HIP_TRY(g_alloc(g, (void**)&g->part_ptr, sizeof(int32_t) * (K + 1)));
  HIP_TRY(g_alloc(g, (void**)&g->part_T, sizeof(double) * K));
  HIP_TRY(g_alloc(g, (void**)&g->part_lock, sizeof(int) * K));
  HIP_TRY(hipMemsetAsync(g->part_lock, 0, sizeof(int) * K, c->stream));
  int64_t* tmp = nullptr;
  HIP_TRY(g_alloc(g, (void**)&tmp, sizeof(int64_t) * (K + 1)));
  int rc = g->part_type == DITR_PART_PMASS
               ? launch_partition_pmass(c, g->n, g->nnz, g->col_ptr, g->row_idx, g->val, g->d, K, tmp,
                                        g->part_ptr, g)
           : g->part_type == DITR_PART_MINCUT
               ? launch_partition_mincut(c, g->n, g->nnz, g->col_ptr, g->row_idx, g->row_ptr, K, tmp,
                                         g->part_ptr, g)
               : launch_partition(c, g->n, g->col_ptr, g->row_ptr, g->part_type, K, tmp, g->part_ptr);
  hipError_t e = rc ? hipSuccess
                    : hipMemcpyAsync(g->part_ptr_host, tmp, sizeof(int64_t) * (K + 1),
                                     hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  g_free(g, tmp);
  if (rc) return rc;
  HIP_TRY(e);
  int64_t mx = 0;
  for (int64_t k = 0; k < K; ++k) mx = std::max(mx, g->part_ptr_host[k + 1] - g->part_ptr_host[k]);
  g->max_part = (int32_t)mx;
  return DITR_OK;
}

}  // extern "C"

// Replace the partition boundaries of g by h_ptr (K + 1 nondecreasing values
// from 0 to n, no part above g->cap_nodes) and rebuild the partition tables.
int graph_set_plan(ditr_ctx* c, ditr_graph* g, const int64_t* h_ptr, int64_t K) {
  if (!c || !g || !h_ptr) return set_error(DITR_EINVAL, "NULL argument");
  if (g->arena.base)
    return set_error(DITR_EINVAL, "a graph in a caller workspace keeps the plan it was uploaded with");
  if (K < 1 || K > g->n) return set_error(DITR_EINVAL, "need 1 <= K <= n");
  if (h_ptr[0] != 0 || h_ptr[K] != g->n) return set_error(DITR_EINVAL, "boundaries must run from 0 to n");
  int64_t mx = 0;
  for (int64_t k = 0; k < K; ++k) {
    if (h_ptr[k + 1] < h_ptr[k]) return set_error(DITR_EINVAL, "boundaries must not decrease");
    mx = std::max(mx, h_ptr[k + 1] - h_ptr[k]);
  }
  if (mx > g->cap_nodes)
    return set_error(DITR_EINVAL, "a partition of %lld nodes exceeds the %lld one workgroup holds", (long long)mx,
                     (long long)g->cap_nodes);
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  free_part_plan(g);
  g_free(g, g->part_ptr);
  g_free(g, g->part_T);
  g_free(g, g->part_lock);
  g->part_ptr = nullptr;
  g->part_T = nullptr;
  g->part_lock = nullptr;
  delete[] g->part_ptr_host;
  g->part_ptr_host = new (std::nothrow) int64_t[K + 1];
  if (!g->part_ptr_host) return set_error(DITR_ENOMEM, "host allocation failed");
  memcpy(g->part_ptr_host, h_ptr, sizeof(int64_t) * (K + 1));
  g->K = K;
  g->max_part = (int32_t)mx;
  std::vector<int32_t> p32(K + 1);
  for (int64_t k = 0; k <= K; ++k) p32[k] = (int32_t)h_ptr[k];
  HIP_TRY(g_alloc(g, (void**)&g->part_ptr, sizeof(int32_t) * (K + 1)));
  HIP_TRY(g_alloc(g, (void**)&g->part_T, sizeof(double) * K));
  HIP_TRY(g_alloc(g, (void**)&g->part_lock, sizeof(int) * K));
  HIP_TRY(hipMemsetAsync(g->part_lock, 0, sizeof(int) * K, c->stream));
  HIP_TRY(hipMemcpy(g->part_ptr, p32.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice));
  return build_part_plan(c, g);
}

// Graph upload for the PageRank matrix (d_val == nullptr, p_ji = damping / #out_i)
// or a general matrix (one weight per CSC entry, Section 2).
static int graph_create_impl(ditr_ctx* c, ditr_graph** out, int64_t n, int64_t nnz,
                             const int32_t* d_col_ptr, const int32_t* d_row_idx, const double* d_val,
                             double damping, const ditr_opts* opts, void* d_workspace = nullptr,
                             size_t ws_bytes = 0) {
  if (!c || !out) return set_error(DITR_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 1 || n >= ((int64_t)1 << 31) - 1) return set_error(DITR_EINVAL, "n = %lld out of range", (long long)n);
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return set_error(DITR_EINVAL, "nnz = %lld out of range", (long long)nnz);
  if (!d_val && !(damping > 0 && damping < 1)) return set_error(DITR_EINVAL, "damping must lie in (0, 1)");
  if (!d_col_ptr || (nnz > 0 && !d_row_idx)) return set_error(DITR_EINVAL, "NULL CSC array");
  ditr_opts o;
  ditr_opts_default(&o);
  if (opts) o = *opts;
  if (o.part_type != DITR_PART_CB && o.part_type != DITR_PART_UNIFORM &&
      o.part_type != DITR_PART_CB_INOUT && o.part_type != DITR_PART_PMASS && o.part_type != DITR_PART_MINCUT)
    return set_error(DITR_EINVAL, "unknown partition type %d", o.part_type);
  if (o.block == 0) o.block = 1024;
  if (o.block != 256 && o.block != 512 && o.block != 1024)
    return set_error(DITR_EINVAL, "block must be 256, 512 or 1024");
  HIP_TRY(hipSetDevice(c->device));

  int rc = launch_validate_csc(c, n, nnz, d_col_ptr, d_row_idx);
  if (rc) return rc;
  rc = read_ctrl(c);
  if (rc) return rc;
  if (c->ctrl_host->err)
    return set_error(DITR_EGRAPH, "malformed CSC (flags %d: 1 = col_ptr ends, 2 = decreasing "
                     "col_ptr, 4 = row index out of range)", c->ctrl_host->err);

  ditr_graph* g = new (std::nothrow) ditr_graph();
  if (!g) return set_error(DITR_ENOMEM, "host allocation failed");
  g->ctx = c;
  g->device = c->device;
  g->n = n;
  g->nnz = nnz;
  g->d = damping;
  g->col_ptr = d_col_ptr;
  g->row_idx = d_row_idx;
  g->val = nnz > 0 ? d_val : nullptr;
  g->part_type = o.part_type;
  if (d_workspace) {
    g->arena.base = static_cast<unsigned char*>(d_workspace);
    g->arena.cap = ws_bytes;
  }
  bool ok = g_alloc(g, (void**)&g->row_ptr, sizeof(int32_t) * (n + 1)) == hipSuccess &&
            g_alloc(g, (void**)&g->csr_col, sizeof(int32_t) * std::max<int64_t>(nnz, 1)) == hipSuccess &&
            g_alloc(g, (void**)&g->heavy_rows, sizeof(int32_t) * n) == hipSuccess &&
            g_alloc(g, (void**)&g->wh, sizeof(double) * n) == hipSuccess;
  if (ok && g->val)
    ok = g_alloc(g, (void**)&g->csr_val, sizeof(double) * nnz) == hipSuccess &&
         g_alloc(g, (void**)&g->colabs, sizeof(double) * n) == hipSuccess;
  if (!ok) {
    ditr_graph_destroy(g);
    return set_error(DITR_ENOMEM, "device allocation failed (graph of n = %lld)", (long long)n);
  }
  if (g->val) {
    // a general matrix must be strictly contractive in the l1 column norm
    // (Section 1: the series sum P^n B converges; the bound of Section 2 then
    // holds with c = max_i sum_j |p_ji| in place of d)
    double cmax = 0;
    int bad = 0;
    rc = launch_col_abs(c, g, &cmax, &bad);
    if (rc) {
      ditr_graph_destroy(g);
      return rc;
    }
    if (bad || !(cmax < 1.0)) {
      ditr_graph_destroy(g);
      if (bad) return set_error(DITR_EINVAL, "a link weight is NaN or Inf");
      return set_error(DITR_EINVAL, "P is not strictly contractive: largest column l1 norm %.17g >= 1", cmax);
    }
    g->d = cmax;
  } else if (d_val) {
    g->d = 0.0;  // no links: P = 0
  }
  rc = launch_build_transpose(c, g);
  if (!rc) rc = build_heavy_chunks(c, g);
  if (rc) {
    ditr_graph_destroy(g);
    return rc;
  }

  // partition plan (Section 2.3): sized so that one partition fits in LDS
  size_t lds_max = 0;
  rc = max_dynamic_lds(c, o.block, &lds_max);
  if (rc) {
    ditr_graph_destroy(g);
    return rc;
  }
  // a partition's nodes must fit the LDS of both partitioned kernels
  // (12 bytes per node for the asynchronous one, 20 for the partitioned sweep)
  const int64_t cap_nodes = std::min<int64_t>(
      65536, std::min<int64_t>((int64_t)((lds_max - 16) / 12), (int64_t)((c->part_lds_dyn - 64) / 20)));
  g->cap_nodes = cap_nodes;
  int64_t K = initial_parts(c, n, o.part_nodes);
  const size_t plan_mark = g->arena.used;  // each plan attempt reuses the same workspace
  for (int attempt = 0;; ++attempt) {
    if (g->arena.base) {
      g->arena.used = plan_mark;
      g->part_ptr = nullptr;
      g->part_T = nullptr;
      g->part_lock = nullptr;
    }
    rc = make_plan(c, g, K);
    if (rc) {
      ditr_graph_destroy(g);
      return rc;
    }
    if (g->max_part <= cap_nodes) break;
    if (attempt > 20 || K == n) {
      ditr_graph_destroy(g);
      return set_error(DITR_EINVAL, "no partition plan fits %lld nodes per workgroup",
                       (long long)cap_nodes);
    }
    int64_t need = (n + (cap_nodes * 3 / 4) - 1) / std::max<int64_t>(1, cap_nodes * 3 / 4);
    K = std::min<int64_t>(n, std::max<int64_t>(2 * K, need));
  }
  rc = build_part_plan(c, g);
  if (rc) {
    ditr_graph_destroy(g);
    return rc;
  }
  *out = g;
  return DITR_OK;
}

extern "C" {

int ditr_graph_create(ditr_ctx* c, ditr_graph** out, int64_t n, int64_t nnz,
                      const int32_t* d_col_ptr, const int32_t* d_row_idx, double damping,
                      const ditr_opts* opts) {
  return graph_create_impl(c, out, n, nnz, d_col_ptr, d_row_idx, nullptr, damping, opts);
}

int ditr_graph_create_weighted(ditr_ctx* c, ditr_graph** out, int64_t n, int64_t nnz,
                               const int32_t* d_col_ptr, const int32_t* d_row_idx,
                               const double* d_val, const ditr_opts* opts) {
  if (nnz > 0 && !d_val) return set_error(DITR_EINVAL, "NULL weight array");
  static const double kNoLinks = 0.0;
  return graph_create_impl(c, out, n, nnz, d_col_ptr, d_row_idx, nnz > 0 ? d_val : &kNoLinks, 0.0, opts);
}

int ditr_workspace_bytes(ditr_ctx* c, int64_t n, int64_t nnz, int nrhs, const ditr_opts* opts,
                         size_t* bytes) {
  if (!c || !bytes) return set_error(DITR_EINVAL, "NULL argument");
  if (n < 1 || nnz < 0 || nnz >= ((int64_t)1 << 31)) return set_error(DITR_EINVAL, "sizes out of range");
  ditr_opts o;
  ditr_opts_default(&o);
  if (opts) o = *opts;
  if (nrhs == 0) {
    *bytes = graph_workspace_bound(c, n, nnz, o.part_type, initial_parts(c, n, o.part_nodes), n);
    return DITR_OK;
  }
  if (nrhs < 4 || nrhs > 256 || nrhs % 4)
    return set_error(DITR_EINVAL, "nrhs must be 0 (graph upload) or a multiple of 4 in [4, 256]");
  *bytes = batch_workspace_bytes(c, n, std::min<int64_t>(n, nnz / (kHeavyRow + 1) + 1), nrhs);
  return DITR_OK;
}

int ditr_graph_upload_csc(ditr_ctx* c, ditr_graph** out, int64_t n, int64_t nnz,
                          const int32_t* d_col_ptr, const int32_t* d_row_idx, double damping,
                          void* d_workspace, size_t ws_bytes, const ditr_opts* opts) {
  if (!d_workspace || ws_bytes == 0) return set_error(DITR_EINVAL, "NULL workspace");
  if (((uintptr_t)d_workspace) % 256) return set_error(DITR_EINVAL, "workspace must be 256-byte aligned");
  (void)workspace_overflow(true);
  const int rc = graph_create_impl(c, out, n, nnz, d_col_ptr, d_row_idx, nullptr, damping, opts, d_workspace,
                                   ws_bytes);
  if (rc != DITR_OK && workspace_overflow(true))
    return set_error(DITR_ENOMEM, "the workspace of %zu bytes is too small for this graph "
                     "(ditr_workspace_bytes gives an upper bound)", ws_bytes);
  return rc;
}

int ditr_graph_workspace_used(const ditr_graph* g, size_t* used) {
  if (!g || !used) return set_error(DITR_EINVAL, "NULL argument");
  *used = g->arena.base ? g->arena.peak : 0;
  return DITR_OK;
}

int ditr_graph_contraction(const ditr_graph* g, double* c_out) {
  if (!g || !c_out) return set_error(DITR_EINVAL, "NULL argument");
  *c_out = g->d;
  return DITR_OK;
}

int ditr_graph_partitions(const ditr_graph* g, int64_t* K_out, int64_t* h_ptr, int64_t cap) {
  if (!g || !K_out) return set_error(DITR_EINVAL, "NULL argument");
  *K_out = g->K;
  if (h_ptr) {
    if (cap < g->K + 1) return set_error(DITR_EINVAL, "cap < K + 1");
    memcpy(h_ptr, g->part_ptr_host, sizeof(int64_t) * (g->K + 1));
  }
  return DITR_OK;
}

int ditr_residual(ditr_ctx* c, const ditr_graph* g, const double* d_b, const double* d_h,
                  float* d_f, double* h_resid) {
  if (!c || !g || !d_b || !d_h || !d_f) return set_error(DITR_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(c->device));
  int rc = launch_refresh(c, g, d_b, d_h, d_f);
  if (rc) return rc;
  if (h_resid) {
    rc = read_ctrl(c);
    if (rc) return rc;
    *h_resid = c->ctrl_host->sum_abs;
  }
  return DITR_OK;
}

}  // extern "C"

// The plain solve (steps init, diffusion, transfer, residual, refresh) on the
// per-solve buffers sb. noalloc: the caller may not allocate, so only the
// partitioned sweep runs (its buffers are all in sb) and no timing events are
// created.
int solve_impl(ditr_ctx* c, const ditr_graph* g, const double* d_b, double* d_h, float* d_f, int warm,
               double rel_tol, const ditr_opts* opts, ditr_stats* stats, const SolveBufs& sb,
               bool noalloc) {
  const double t0 = now_s();
  ditr_stats st;
  memset(&st, 0, sizeof(st));
  auto finish = [&](int status) {
    st.status = status;
    st.seconds = now_s() - t0;
    if (stats) *stats = st;
    return status;
  };
  if (!c || !g || !d_b || !d_h || !d_f) return finish(set_error(DITR_EINVAL, "NULL argument"));
  if (!(rel_tol >= 0) || !std::isfinite(rel_tol)) return finish(set_error(DITR_EINVAL, "rel_tol must be >= 0"));
  if (warm < 0 || warm > 2) return finish(set_error(DITR_EINVAL, "warm must be 0, 1 or 2"));
  ditr_opts o;
  ditr_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.alpha > 1)) return finish(set_error(DITR_EINVAL, "alpha must be > 1"));
  if (!(o.refresh_at >= 0) || !std::isfinite(o.refresh_at))
    return finish(set_error(DITR_EINVAL, "refresh_at must be finite and >= 0"));
  if (o.block == 0) o.block = 1024;
  if (o.max_rounds <= 0) o.max_rounds = 16;
  HIP_TRY(hipSetDevice(c->device));
  __atomic_store_n(c->abort_host, 0, __ATOMIC_SEQ_CST);
  const int64_t n = g->n;

  int rc = launch_reset_ctrl(c);
  if (rc) return finish(rc);
  // A cold partitioned solve whose partitions are all resident queues its
  // usual two stages without host readbacks in between (init, stage, exact
  // refresh, stage, exact refresh): each stage's parameters come from the
  // device's own sums, and a stage made unnecessary returns at once. Further
  // stages, if any, go through the loop below. A start with the caller's F_0
  // (warm = 2) is queued the same way after its one pass over B, H_0 and F_0;
  // both stages end with an exact refresh, so the result is certified on an
  // exact residual whatever the given F_0 was.
  bool pipelined = false;
  if ((!warm || warm == 2) && (o.mode == DITR_MODE_AUTO || o.mode == DITR_MODE_PARTITION) && !g->val && !g->colabs &&
      !(o.flags & DITR_FLAG_NO_RESIDENT) && o.max_rounds >= 2 && g->part_ptr && g->pp.ready) {
    rc = part_resident_fits(c, g, &pipelined, (o.flags & DITR_FLAG_PRIORITY) != 0);
    if (rc) return finish(rc);
  }
  double b1 = 0, r = 0, fmax = 0;
  if (pipelined) {
    // read back after the stages
    rc = warm == 2 ? launch_given_start(c, n, d_b, d_h, d_f) : launch_init(c, n, d_b, d_h, d_f);
    if (rc) return finish(rc);
  } else if (!warm) {
    // F = B, H = 0; ||B||_1, ||F_0||_1 and max |F_0| in one pass
    rc = launch_init(c, n, d_b, d_h, d_f);
    if (!rc) rc = read_ctrl(c);
    if (rc) return finish(rc);
    if (c->ctrl_host->err) return finish(set_error(DITR_ENONFINITE, "B holds NaN or Inf"));
    b1 = c->ctrl_host->sum_abs;
    r = c->ctrl_host->sum_abs_f32;
    fmax = c->ctrl_host->max_abs;
  } else if (warm == 2) {
    // the caller's F holds B + P H_0 - H_0 already (rounded to FP32): one pass
    // for ||B||_1, ||F_0||_1 and max |F_0|; the first exact refresh below
    // replaces it, and the loop runs at least one stage so that the result is
    // certified on an exact residual whatever the given F was
    rc = launch_given_start(c, n, d_b, d_h, d_f);
    if (!rc) rc = read_ctrl(c);
    if (rc) return finish(rc);
    if (c->ctrl_host->err) return finish(set_error(DITR_ENONFINITE, "B, H_0 or F_0 holds NaN or Inf"));
    b1 = c->ctrl_host->sum_abs;
    r = c->ctrl_host->sum_abs_f32;
    fmax = c->ctrl_host->max_abs;
  } else {
    // warm start / resume: F_0 = B + P H_0 - H_0 (identity of equations defF and defH)
    rc = launch_norm_f64(c, n, d_b);
    if (!rc) rc = launch_check_finite(c, n, d_h);
    if (!rc) rc = read_ctrl(c);
    if (rc) return finish(rc);
    if (c->ctrl_host->err) return finish(set_error(DITR_ENONFINITE, "B or H_0 holds NaN or Inf"));
    b1 = c->ctrl_host->sum_abs;
    rc = launch_refresh_bufs(c, g, d_b, d_h, d_f, sb.wh, sb.chunk_sum);
    if (!rc) rc = read_ctrl(c);
    if (rc) return finish(rc);
    r = c->ctrl_host->sum_abs;
    fmax = c->ctrl_host->max_abs;
    st.refreshes += 1;
  }
  st.b_l1 = b1;
  double target = rel_tol * b1;
  // a warm start's FP32 fluid drifts like a cold one's: the same first stage applies
  bool refreshed = false;

  // persistent plan: static binding when every partition gets its own resident workgroup
  PersistentCfg cfg;
  memset(&cfg, 0, sizeof(cfg));
  int mode = o.mode;
  const bool general = g->val != nullptr || g->colabs != nullptr;
  if (mode == DITR_MODE_AUTO) mode = general ? DITR_MODE_SWEEP : DITR_MODE_PARTITION;
  if (general && mode != DITR_MODE_SWEEP)
    return finish(set_error(DITR_EINVAL, "a general matrix is solved by the pull sweep (DITR_MODE_SWEEP)"));
  if (mode != DITR_MODE_ASYNC && mode != DITR_MODE_SWEEP && mode != DITR_MODE_PARTITION)
    return finish(set_error(DITR_EINVAL, "unknown mode %d", mode));
  if (noalloc && mode != DITR_MODE_PARTITION)
    return finish(set_error(DITR_EINVAL, "the allocation-free solve runs the partitioned sweep only"));
  if (mode != DITR_MODE_SWEEP && (!g->part_ptr || !g->pp.ready))
    return finish(set_error(DITR_EINVAL, "the graph has no partition plan (a failed ditr_graph_set_partitions); "
                                         "set a valid one first"));
  const bool prio = (o.flags & DITR_FLAG_PRIORITY) != 0;
  if (prio && mode != DITR_MODE_PARTITION)
    return finish(set_error(DITR_EINVAL, "the normalized priority test runs in the partitioned sweep"));
  if (prio) {
    // The partitioned sweep keeps T >= 2^-28 of the total fluid D (its fixed
    // point). A level where no node passes has |F_i| <= T c_i for all i, so
    // D <= T sum_i c_i; with sum_i c_i < 2^28 some node always passes at the
    // lowest T, and the run cannot stall.
    double csum = 0;
    rc = launch_prio_sum(c, g, &csum);
    if (rc) return finish(rc);
    if (!(csum < 268435456.0))
      return finish(set_error(DITR_EINVAL, "the normalized priority test needs sum (#in+1)(#out+1) < 2^28 "
                              "(this graph: %.6g)", csum));
  }
  if (noalloc && (o.flags & DITR_FLAG_TIME_KERNELS))
    return finish(set_error(DITR_EINVAL, "the allocation-free solve creates no timing events"));
  if (mode == DITR_MODE_ASYNC) {
    cfg.block = o.block;
    cfg.lds_nodes = std::max<int>(1, g->max_part);
    cfg.lds_bytes = lds_bytes_for(cfg.lds_nodes);
    int per_cu = 0;
    rc = persistent_occupancy(c, cfg.block, cfg.lds_bytes, &per_cu);
    if (rc) return finish(rc);
    if (per_cu < 1)
      return finish(set_error(DITR_EINVAL, "persistent kernel does not fit a CU (block %d, LDS %zu)",
                              cfg.block, cfg.lds_bytes));
    const int wpc = o.wg_per_cu > 0 ? std::min(o.wg_per_cu, per_cu) : per_cu;
    const int64_t resident = (int64_t)c->num_cus * wpc;
    cfg.static_mode = g->K <= resident;
    cfg.grid = (int)(cfg.static_mode ? g->K : resident);
    cfg.max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 1 << 20;
    cfg.sweeps_per_claim = o.sweeps_per_claim > 0 ? o.sweeps_per_claim : 2;
    cfg.max_passes = (int)std::max<int64_t>(1, std::min<int64_t>(100000, ((int64_t)1 << 30) / g->K));
    cfg.xcd_remap = o.xcd_remap;
    cfg.alpha = o.alpha;
    cfg.park_ratio = o.park_ratio;
    cfg.rescale_cap = o.rescale_cap > 1 ? o.rescale_cap : 1.0;
  }

  // optional event timing of the diffusion launches (partitioned sweep: each
  // launch of its main kernel; other modes: each batch)
  const bool timed = (o.flags & DITR_FLAG_TIME_KERNELS) != 0;
  constexpr int kBatch = 8;
  hipEvent_t ev[2 * kBatch] = {};
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 2 * kBatch; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } ev_guard{ev};
  if (timed)
    for (int i = 0; i < 2 * kBatch; ++i) HIP_TRY(hipEventCreate(&ev[i]));
  // The interval ev[0]..ev[1] is read only once the stream has been
  // synchronized for another reason (the readback after the refresh) or before
  // the events are reused: waiting for it right after the launch would keep
  // the host from queueing the refresh behind the kernel.
  int64_t pending = 0;  // launches in the interval not yet added
  auto t_flush = [&]() -> int {
    if (!pending) return DITR_OK;
    HIP_TRY(hipEventSynchronize(ev[1]));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
    st.kernel_seconds += 1e-3 * ms;
    st.timed_launches += pending;
    pending = 0;
    return DITR_OK;
  };
  auto t_begin = [&]() -> int {
    if (!timed) return DITR_OK;
    const int rc2 = t_flush();
    if (rc2) return rc2;
    HIP_TRY(hipEventRecord(ev[0], c->stream));
    return DITR_OK;
  };
  auto t_end = [&](int64_t launches) -> int {
    if (!timed) return DITR_OK;
    HIP_TRY(hipEventRecord(ev[1], c->stream));
    pending = launches;
    return DITR_OK;
  };
  // sum the first `executed` launch intervals of a batch (later ones were no-ops)
  auto t_sum = [&](int64_t executed) -> int {
    if (!timed) return DITR_OK;
    for (int64_t i = 0; i < executed && i < kBatch; ++i) {
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      st.kernel_seconds += 1e-3 * ms;
      st.timed_launches += 1;
    }
    return DITR_OK;
  };

  // first exact refresh (0: the library's choice). The FP32 history
  // increments of the partitioned and pull sweeps round off about 2^-24 of the
  // history a stage adds, a few 1e-7 ||B||_1 at d = 0.85: a stage run below that
  // chases fluid the exact residual does not hold, one stopped far above it
  // restarts the threshold early. The asynchronous kernel keeps F itself in
  // FP32 and drifts more, so it refreshes earlier.
  const double refresh_at = o.refresh_at > 0 ? o.refresh_at : (mode == DITR_MODE_ASYNC ? 1e-5 : 1e-7);
  int status = DITR_OK;
  double t_carry = 0;
  bool resident_ran = false;
  bool must_refresh = warm == 2 && !pipelined;  // a given F_0 is trusted for one stage only
  if (pipelined) {
    for (int s = 0; s < 2; ++s) {
      rc = launch_part_stage(c, g, sb, s == 0, rel_tol, refresh_at, o.alpha);
      if (!rc && timed && hipEventRecord(ev[2 * s], c->stream) != hipSuccess)
        rc = set_error(DITR_EHIP, "hipEventRecord failed");
      if (!rc)
        rc = launch_part_resident(c, g, sb, d_f, d_h, o.alpha, o.sweeps_per_claim > 0 ? o.sweeps_per_claim : 3,
                                  o.max_sweeps > 0 ? (int)std::min<int64_t>(o.max_sweeps, 1 << 30) : 4096, prio);
      if (!rc && timed && hipEventRecord(ev[2 * s + 1], c->stream) != hipSuccess)
        rc = set_error(DITR_EHIP, "hipEventRecord failed");
      if (!rc) rc = launch_refresh_bufs(c, g, d_b, d_h, d_f, sb.wh, sb.chunk_sum);
      if (rc) return finish(rc);
    }
    rc = read_ctrl(c);
    if (rc) return finish(rc);
    const Ctrl& h = *c->ctrl_host;
    if (h.err == 2) return finish(set_error(DITR_EHIP, "a wait of the resident sweep timed out"));
    if (h.err)
      return finish(set_error(DITR_ENONFINITE, warm == 2 ? "B, H_0 or F_0 holds NaN or Inf" : "B holds NaN or Inf"));
    b1 = h.b1;
    st.b_l1 = b1;
    target = rel_tol * b1;
    st.rounds = h.stages;
    st.launches += h.stages;
    st.refreshes += 2;
    resident_ran = h.stages > 0;
    refreshed = true;
    t_carry = h.T;
    r = h.sum_abs;
    fmax = h.max_abs;
    if (timed)
      for (int s = 0; s < h.stages; ++s) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, ev[2 * s], ev[2 * s + 1]));
        st.kernel_seconds += 1e-3 * ms;
        st.timed_launches += 1;
      }
    if (!std::isfinite(r)) return finish(set_error(DITR_ENONFINITE, "residual became non-finite"));
  }
  while (r > target || must_refresh) {
    must_refresh = false;
    if (st.rounds >= o.max_rounds) {
      status = DITR_NOT_CONVERGED;
      break;
    }
    if (__atomic_load_n(c->abort_host, __ATOMIC_SEQ_CST)) {
      status = DITR_ABORTED;
      break;
    }
    // stage 1 stops at refresh_at ||B||_1, where the exact residual replaces the
    // FP32 fluid and its rounding drift; later stages aim below the target
    const double stage = (!refreshed && r > refresh_at * b1) ? std::max(target, refresh_at * b1)
                                                               : 0.5 * target;
    // the threshold continues from the previous round (never above max|F| / alpha);
    // the first one starts at max|F| / alpha or at the mean |F| if lower, so a
    // start whose fluid sits in a few large entries (a learned warm start)
    // does not spend its first levels on those alone
    double T0 = st.rounds > 0 ? std::min(t_carry, fmax / o.alpha)
                              : std::min(fmax / o.alpha, r / (double)std::max<int64_t>(1, g->n));
    if (mode == DITR_MODE_PARTITION) T0 = std::max(T0, r * kPartTFloor);
    // the partitioned sweep sets the launch target in its stage preparation
    rc = mode == DITR_MODE_PARTITION ? launch_part_prepare(c, g, sb, r, stage, T0)
                                     : launch_set_launch_target(c, r, stage, T0);
    if (rc) return finish(rc);
    if (mode == DITR_MODE_PARTITION) {
      const int m = o.sweeps_per_claim > 0 ? o.sweeps_per_claim : 3;
      const int batch = kBatch;
      const int64_t budget = o.max_sweeps > 0 ? o.max_sweeps : 4096;
      bool resident = false;
      if (!(o.flags & DITR_FLAG_NO_RESIDENT)) {
        rc = part_resident_fits(c, g, &resident, prio);
        if (rc) return finish(rc);
      }
      if (resident) {
        // every partition resident for the whole stage: one cooperative launch
        rc = t_begin();
        if (!rc) {
          rc = launch_part_resident(c, g, sb, d_f, d_h, o.alpha, m, (int)std::min<int64_t>(budget, 1 << 30),
                                    prio);
          if (rc == DITR_EHIP) {  // cooperative launch refused: relaunch per level instead
            (void)hipGetLastError();
            resident = false;
            rc = DITR_OK;
          }
        }
        // no readback here: the refresh below ends with one, which also
        // carries the wait-timeout flag of this launch
        if (!rc && resident) rc = t_end(1);
        if (rc) return finish(rc);
        if (resident) {
          st.launches += 1;
          resident_ran = true;
        }
      }
      // otherwise launches of m local sweeps in batches; the stop flag turns the
      // rest of a batch into no-ops
      for (int64_t done_l = 0; !resident && done_l < budget; done_l += batch) {
        const uint64_t before = c->ctrl_host->sweeps;
        rc = launch_part_sweeps(c, g, sb, d_f, d_h, o.alpha, m, batch, timed ? ev : nullptr, prio);
        if (!rc) rc = read_ctrl(c);
        if (!rc) rc = t_sum((int64_t)(c->ctrl_host->sweeps - before));
        if (rc) return finish(rc);
        st.launches += batch;
        if (c->ctrl_host->done || __atomic_load_n(c->abort_host, __ATOMIC_SEQ_CST)) break;
      }
    } else if (mode == DITR_MODE_ASYNC) {
      if (!cfg.static_mode) {
        rc = launch_fill_double(c, g->part_T, g->K, -1.0);
        if (rc) return finish(rc);
      }
      rc = t_begin();
      if (!rc) rc = launch_persistent(c, g, d_f, d_h, cfg);
      if (!rc) rc = t_end(1);
      if (rc) return finish(rc);
      st.launches += 1;
    } else {
      // pull sweeps in batches; the stop flag turns the rest of a batch into no-ops
      rc = launch_pull_prepare(c, g);
      if (rc) return finish(rc);
      const int batch = 16;
      const int64_t budget = o.max_sweeps > 0 ? o.max_sweeps : 4096;
      for (int64_t done_sweeps = 0; done_sweeps < budget; done_sweeps += batch) {
        rc = t_begin();
        if (!rc) rc = launch_pull_sweeps(c, g, d_f, d_h, o.alpha, 0, batch);
        if (!rc) rc = t_end(batch);
        if (!rc) rc = read_ctrl(c);
        if (rc) return finish(rc);
        st.launches += batch;
        if (c->ctrl_host->done || __atomic_load_n(c->abort_host, __ATOMIC_SEQ_CST)) break;
      }
    }
    rc = launch_refresh_bufs(c, g, d_b, d_h, d_f, sb.wh, sb.chunk_sum);
    if (!rc) rc = read_ctrl(c);
    if (!rc) rc = t_flush();
    if (rc) return finish(rc);
    if (resident_ran && c->ctrl_host->err == 2)
      return finish(set_error(DITR_EHIP, "a wait of the resident sweep timed out"));
    st.refreshes += 1;
    st.rounds += 1;
    refreshed = true;
    t_carry = c->ctrl_host->T;
    r = c->ctrl_host->sum_abs;
    fmax = c->ctrl_host->max_abs;
    if (!std::isfinite(r)) return finish(set_error(DITR_ENONFINITE, "residual became non-finite"));
  }
  if (status == DITR_OK && __atomic_load_n(c->abort_host, __ATOMIC_SEQ_CST) && r > target)
    status = DITR_ABORTED;
  st.edges = (int64_t)c->ctrl_host->edges;
  st.diffusions = (int64_t)c->ctrl_host->diffusions;
  st.sweeps = (int64_t)c->ctrl_host->sweeps;
  st.idle_polls = (int64_t)c->ctrl_host->idle_polls;
  st.resid_l1 = r;
  rc = t_flush();
  if (rc) return finish(rc);
  if (status == DITR_NOT_CONVERGED)
    set_error(status, "not converged after %d rounds (||F||_1 = %g, target %g)", st.rounds, r, target);
  return finish(status);
}

extern "C" {

int ditr_solve(ditr_ctx* c, const ditr_graph* g, const double* d_b, double* d_h, float* d_f,
               int warm, double rel_tol, const ditr_opts* opts, ditr_stats* stats) {
  if (!g) {
    if (stats) memset(stats, 0, sizeof(*stats));
    if (stats) stats->status = DITR_EINVAL;
    return set_error(DITR_EINVAL, "NULL argument");
  }
  return solve_impl(c, g, d_b, d_h, d_f, warm, rel_tol, opts, stats, graph_bufs(g), false);
}

int ditr_solve_batched(ditr_ctx* c, const ditr_graph* g, int nrhs, const double* d_b, double* d_h,
                       float* d_f, double rel_tol, const ditr_opts* opts, void* d_workspace,
                       size_t ws_bytes, ditr_stats* per_rhs, ditr_stats* total) {
  const double t0 = now_s();
  if (!c || !g || !d_b || !d_h || !d_f) return set_error(DITR_EINVAL, "NULL argument");
  if (!(rel_tol >= 0) || !std::isfinite(rel_tol)) return set_error(DITR_EINVAL, "rel_tol must be >= 0");
  ditr_opts o;
  ditr_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.alpha > 1)) return set_error(DITR_EINVAL, "alpha must be > 1");
  if (!(o.refresh_at >= 0) || !std::isfinite(o.refresh_at))
    return set_error(DITR_EINVAL, "refresh_at must be finite and >= 0");
  if (g->csr_val) return set_error(DITR_EINVAL, "the batched solve takes PageRank graphs (no link weights)");
  HIP_TRY(hipSetDevice(c->device));
  __atomic_store_n(c->abort_host, 0, __ATOMIC_SEQ_CST);
  int rc = launch_reset_ctrl(c);
  if (!rc) rc = launch_check_finite(c, g->n * (int64_t)nrhs, d_b);
  if (!rc) rc = read_ctrl(c);
  if (rc) return rc;
  if (c->ctrl_host->err) return set_error(DITR_ENONFINITE, "B holds NaN or Inf");
  ditr_stats tot;
  memset(&tot, 0, sizeof(tot));
  rc = batch_solve(c, g, nrhs, d_b, d_h, d_f, rel_tol, o, per_rhs, &tot, d_workspace, ws_bytes);
  tot.seconds = now_s() - t0;
  tot.status = rc;
  if (total) *total = tot;
  if (per_rhs && rc >= 0)
    for (int r = 0; r < nrhs; ++r) per_rhs[r].seconds = tot.seconds;
  return rc;
}

}  // extern "C"
