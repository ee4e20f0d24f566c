// Internal definitions of the ditr library (gfx950). Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ditr.h"

#define DITR_WAVE 64

// Device-resident control block of one solve. All cross-workgroup traffic on
// it uses agent-scope atomics: the L2 of one XCD is not coherent with the
// L2 of another, so plain loads of another workgroup's writes can be stale.
struct Ctrl {
  double destroyed;        // sum over diffusions of |sent| * (1 - d) (or |sent| if dangling)
  double r0;               // ||F||_1 when the current launch started
  double target;           // a launch stops once r0 - destroyed <= target
  double sum_abs;          // reduction output: sum |x| (FP64)
  double max_abs;          // reduction output: max |x|
  double sum_abs_f32;      // reduction output: sum |(float)x| (init only)
  double T;                // grid-wide threshold (sweep mode)
  unsigned long long edges, diffusions, sweeps, idle_polls;
  unsigned long long passed;   // nodes diffused by the current grid sweep (sweep mode)
  int done;
  int ticket;
  int err;                 // graph validation / non-finite input flag
  int stages;              // resident stages that ran (pipelined solve)
  double b1;               // ||B||_1 of the solve (pipelined solve)
};

struct ditr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t work = nullptr;  // private stream for graph-captured loops (default priority)
  int num_cus = 0;
  size_t lds_per_block = 0;    // default LDS limit of one workgroup
  size_t lds_per_cu = 0;       // LDS of one CU
  size_t lds_dyn[3] = {0, 0, 0};  // dynamic LDS the persistent kernel may take (block 256/512/1024)
  size_t part_lds_dyn = 0;        // dynamic LDS the partitioned sweep may take
  size_t part_lds_static = 0;     // largest static LDS of the partition kernels
  int* abort_host = nullptr;   // pinned, mapped
  int* abort_dev = nullptr;    // device view of abort_host
  Ctrl* ctrl = nullptr;        // device
  Ctrl* ctrl_host = nullptr;   // pinned mirror for readback
  double* partials = nullptr;  // reduction partials (2 doubles per block)
  size_t partials_cap = 0;     // in blocks
  unsigned char* scratch = nullptr;  // this device's static scratch (ditr_solve_noalloc)
  size_t scratch_bytes = 0;
  double* trace = nullptr;     // caller's per-partition trace (ditr_set_trace), or nullptr
  int64_t trace_cap = 0;       // records of DITR_TRACE_FIELDS doubles
  double tick_s = 0;           // seconds per tick of s_memrealtime
};

// Tables of the partitioned sweep (part_k.hip), built per partition plan.
struct PartPlan {
  bool ready = false;
  int32_t* pid = nullptr;        // [n] partition of each node
  int32_t* loc_ptr = nullptr;    // [n+1] local CSC: out-links that stay in the partition
  uint16_t* loc_idx = nullptr;   //   target - partition start
  uint16_t* inv = nullptr;       // [n] local id of each node: its rank in the partition's
                                 //   visiting order (falling local out-degree)
  float* pw = nullptr;           // [n] d / #out_i (0 for a dangling node)
  int32_t* ext_ptr = nullptr;    // [K+1] external in-links of each partition (light rows)
  int32_t* ext_src = nullptr;    //   source node
  uint16_t* ext_row = nullptr;   //   target - partition start
  int32_t* heavy_rows = nullptr; // rows with more than kPartHeavy external in-links, ascending
  int32_t* part_heavy = nullptr; // [K+1] range of heavy_rows inside each partition
  int32_t* heavy_src = nullptr;  // external in-links of heavy rows (CSR order; plan build only)
  int32_t* item_row = nullptr;   // heavy items (at most kItem links of one heavy row): local row
  int32_t* part_items = nullptr; // [K+1] items of each partition
  int32_t* unit_src = nullptr;   // [n_units][8][64] work units of the item sums: source of
                                 //   slot q of a lane (-1: none)
  int32_t* unit_meta = nullptr;  // [n_units][64] per lane: (item + 1 for the lane that leads
                                 //   its group, else 0) << 3 | log2(lanes of the group)
  unsigned long long* item_word = nullptr;  // [2][n_items] item inflow: FP32 bits | epoch << 32
  int32_t n_items = 0, n_units = 0;
  int64_t epoch = 0;             // epochs handed out to resident launches so far
  float* S = nullptr;            // [2][n] published p_i dH_i
  int* counters = nullptr;       // [8] finished workgroups at [1], level arrivals at [6..7]
  double* partials = nullptr;    // [2][K][4] per-workgroup sums
  int32_t n_heavy = 0;
  int32_t max_local_edges = 0;   // most local out-links in one partition
  int64_t n_local = 0, n_ext = 0, n_heavy_edges = 0;
};

// Device memory of a graph's tables: hipMalloc'd buffer by buffer
// (ditr_graph_create), or carved in order from a workspace the caller owns
// (ditr_graph_upload_csc), in which case nothing is freed before the caller
// releases the workspace.
struct DevArena {
  unsigned char* base = nullptr;  // caller workspace (nullptr: hipMalloc)
  size_t cap = 0;
  size_t used = 0;
  size_t peak = 0;
};

struct ditr_graph {
  ditr_ctx* ctx = nullptr;
  DevArena arena;
  int device = 0;                    // device of the context it was created on
  int64_t n = 0, nnz = 0;
  double d = 0.85;
  const int32_t* col_ptr = nullptr;  // borrowed
  const int32_t* row_idx = nullptr;  // borrowed
  const double* val = nullptr;       // borrowed: weight of each CSC entry (general matrix), or
                                     //   nullptr for the PageRank weights d / #out_i
  int32_t* row_ptr = nullptr;        // transpose (CSR): in-links of each node
  int32_t* csr_col = nullptr;
  double* csr_val = nullptr;         // general matrix: the weights in CSR order
  double* colabs = nullptr;          // general matrix: sum |p_ji| of each column
  int32_t* heavy_rows = nullptr;     // rows with in-degree > kHeavyRow, ascending
  int32_t n_heavy = 0;
  int32_t* chunk_h = nullptr;        // heavy chunk -> index into heavy_rows
  int32_t* chunk_beg = nullptr;      // heavy chunk -> first in-link (CSR position)
  int32_t* chunk_end = nullptr;      // heavy chunk -> one past its last in-link
  int32_t n_chunks = 0;
  double* chunk_sum = nullptr;       // [n_chunks] exact-residual sum of one heavy chunk
  float* pull_s = nullptr;           // [2][n] sent fluid times p_ji of the previous / current sweep
  double* pull_heavy = nullptr;      // [2][n_heavy] chunked inflow of heavy rows
  double* pull_partials = nullptr;   // per-workgroup sums of one pull sweep
  double* wh = nullptr;              // scratch [n]: d * H_i / #out_i
  int64_t K = 0;                     // partitions
  int32_t* part_ptr = nullptr;       // [K+1] device
  int64_t* part_ptr_host = nullptr;  // [K+1] host copy
  int32_t max_part = 0;              // nodes in the largest partition
  int64_t cap_nodes = 0;             // nodes one partition may hold (LDS of the partition kernels)
  int part_type = DITR_PART_CB;
  double* part_T = nullptr;          // [K] per-partition threshold carried between claims
  int* part_lock = nullptr;          // [K] claim locks (dynamic binding)
  PartPlan pp;                       // partitioned-sweep tables
};

constexpr int kHeavyRow = 64;     // in-degree above which a row's in-links are split in chunks
constexpr int kHeavyChunk = 2048; // in-links per chunk workgroup
constexpr int kPartHeavy = 4;     // external in-links above which a row's inflow is summed in items
constexpr int kItem = 512;        // links of a heavy row summed by one wave (8 per lane)
// lowest threshold of the partitioned sweep relative to the total fluid (its
// LDS fluid is fixed point in units of T 2^-32)
constexpr double kPartTFloor = 1.0 / 268435456.0;  // 2^-28

// Per-solve device buffers of the plain solve. ditr_solve takes them from the
// graph's tables; ditr_solve_noalloc carves them out of the static scratch.
struct SolveBufs {
  float* S = nullptr;                         // [2][n] published shares
  unsigned long long* item_word = nullptr;    // [2][n_items] heavy-item inflow words
  double* partials = nullptr;                 // [2][K][8] per-workgroup sums
  int* counters = nullptr;                    // [8] finish count, level arrivals
  double* wh = nullptr;                       // [n] p_ji H_i (exact residual)
  double* chunk_sum = nullptr;                // [n_chunks] heavy-chunk sums (exact residual)
  int64_t* epoch = nullptr;                   // host: item-word epochs handed out so far
};
SolveBufs graph_bufs(const ditr_graph* g);

// allocation of a graph's device tables (arena.hip): from its workspace when
// it has one (256-byte aligned, hipErrorOutOfMemory when it is full), else
// hipMalloc; g_free releases a hipMalloc'd buffer and ignores workspace ones
hipError_t g_alloc(ditr_graph* g, void** p, size_t bytes);
void g_free(ditr_graph* g, void* p);
bool workspace_overflow(bool reset);  // whether a workspace allocation failed on this thread
// upper bound of the workspace a graph upload needs (ditr_workspace_bytes)
size_t graph_workspace_bound(const ditr_ctx* c, int64_t n, int64_t nnz, int part_type, int64_t K_min,
                             int64_t K_max);
int64_t initial_parts(const ditr_ctx* c, int64_t n, int32_t part_nodes);
size_t batch_workspace_bytes(const ditr_ctx* c, int64_t n, int64_t n_heavy, int R);

// ---- error reporting (api.hip) ------------------------------------------
int set_error(int code, const char* fmt, ...);
#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return set_error(DITR_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                       __FILE__, __LINE__);                                             \
  } while (0)

// ---- device helpers -------------------------------------------------------
__device__ __forceinline__ float ld_agent(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float xchg_agent(float* p, float v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_agent(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_agent(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double fetch_add_agent(double* p, double v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_system(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// inclusive prefix sum over the 64 lanes of a wave (all lanes active)
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// DPP forms (all 64 lanes active): row shifts within rows of 16 lanes, then
// row broadcasts of lanes 15 and 31. Inclusive sum and max scans.
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_CTRL>
__device__ __forceinline__ int dpp_mov(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, BANK_MASK, BOUND_CTRL);
}
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
  v += dpp_mov<0x111, 0xf, 0xf, true>(0, v);   // row_shr:1
  v += dpp_mov<0x112, 0xf, 0xf, true>(0, v);   // row_shr:2
  v += dpp_mov<0x114, 0xf, 0xf, true>(0, v);   // row_shr:4
  v += dpp_mov<0x118, 0xf, 0xf, true>(0, v);   // row_shr:8
  v += dpp_mov<0x142, 0xa, 0xf, false>(0, v);  // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xc, 0xf, false>(0, v);  // row_bcast:31 into rows 2 and 3
  return v;
}
__device__ __forceinline__ int wave_incl_max_dpp(int v) {  // v >= 0
  v = max(v, dpp_mov<0x111, 0xf, 0xf, true>(0, v));
  v = max(v, dpp_mov<0x112, 0xf, 0xf, true>(0, v));
  v = max(v, dpp_mov<0x114, 0xf, 0xf, true>(0, v));
  v = max(v, dpp_mov<0x118, 0xf, 0xf, true>(0, v));
  v = max(v, dpp_mov<0x142, 0xa, 0xf, false>(0, v));
  v = max(v, dpp_mov<0x143, 0xc, 0xf, false>(0, v));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_maxd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---- launchers (graph_k.hip, solve_k.hip) -----------------------------------
int launch_validate_csc(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* col_ptr,
                        const int32_t* row_idx);
int launch_build_transpose(ditr_ctx* c, ditr_graph* g);
int launch_col_abs(ditr_ctx* c, ditr_graph* g, double* h_max, int* h_bad);
int launch_partition(ditr_ctx* c, int64_t n, const int32_t* col_ptr, const int32_t* row_ptr,
                     int part_type, int64_t K, int64_t* out64, int32_t* out32);
int launch_in_prefix(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* row_idx, int32_t* out);
int launch_partition_pmass(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* col_ptr,
                           const int32_t* row_idx, const double* val, double d, int64_t K,
                           int64_t* out64, int32_t* out32, ditr_graph* g = nullptr);
size_t pmass_temp_bytes(int64_t n, int64_t nnz);
int launch_partition_mincut(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* col_ptr, const int32_t* row_idx,
                            const int32_t* in_ptr, int64_t K, int64_t* out64, int32_t* out32,
                            ditr_graph* g = nullptr);
size_t mincut_temp_bytes(int64_t n, int64_t K_min, int64_t K_max);

int launch_init(ditr_ctx* c, int64_t n, const double* b, double* h, float* f);
int launch_check_finite(ditr_ctx* c, int64_t n, const double* x);
int launch_given_start(ditr_ctx* c, int64_t n, const double* b, const double* h, const float* f);
int launch_norm_f64(ditr_ctx* c, int64_t n, const double* x);
int launch_refresh(ditr_ctx* c, const ditr_graph* g, const double* b, const double* h, float* f);
int launch_refresh_bufs(ditr_ctx* c, const ditr_graph* g, const double* b, const double* h, float* f,
                       double* wh, double* chunk_sum);
int launch_reset_ctrl(ditr_ctx* c);
int launch_set_launch_target(ditr_ctx* c, double r0, double target, double T0);
int launch_fill_double(ditr_ctx* c, double* p, int64_t n, double v);
int launch_pull_prepare(ditr_ctx* c, const ditr_graph* g);
int launch_pull_sweeps(ditr_ctx* c, const ditr_graph* g, float* f, double* h, double alpha,
                       int first_parity, int nsweeps);
int build_heavy_chunks(ditr_ctx* c, ditr_graph* g);
int scan_exclusive_i32(ditr_ctx* c, const int32_t* in, int64_t n, int32_t* out, ditr_graph* g = nullptr);
int build_part_plan(ditr_ctx* c, ditr_graph* g);
void free_part_plan(ditr_graph* g);
int part_configure(ditr_ctx* c);
size_t part_lds_bytes(int nodes, int local_edges, bool prio = false);
size_t plan_sort_temp_bytes(int64_t n, int64_t ni);
int graph_set_plan(ditr_ctx* c, ditr_graph* g, const int64_t* h_ptr, int64_t K);
int launch_part_stage(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, int first, double rel_tol,
                      double refresh_at, double alpha);
int launch_part_prepare(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, double r0,
                        double target, double T0);
int launch_part_sweeps(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, float* f, double* h,
                       double alpha, int m, int nlaunch, hipEvent_t* ev, bool prio);
int part_resident_fits(ditr_ctx* c, const ditr_graph* g, bool* fits, bool prio);
int launch_part_resident(ditr_ctx* c, const ditr_graph* g, const SolveBufs& sb, float* f, double* h,
                         double alpha, int m, int max_levels, bool prio);
int launch_prio_sum(ditr_ctx* c, const ditr_graph* g, double* h_sum);
int launch_zero_u64(ditr_ctx* c, unsigned long long* p, int64_t n);
// static scratch of ditr_solve_noalloc (noalloc.hip): device address on the
// context's device, looked up once per device at context creation
int noalloc_init(ditr_ctx* c);
struct PersistentCfg {
  int block;
  int grid;
  int static_mode;
  int lds_nodes;
  size_t lds_bytes;
  int max_sweeps;
  int sweeps_per_claim;
  int max_passes;
  int xcd_remap;
  double alpha;
  double park_ratio;
  double rescale_cap;
};
int launch_persistent(ditr_ctx* c, const ditr_graph* g, float* f, double* h,
                      const PersistentCfg& cfg);
int persistent_occupancy(ditr_ctx* c, int block, size_t lds, int* per_cu);
int persistent_static_lds_impl(int block, size_t* bytes);
int persistent_configure(ditr_ctx* c, size_t cu_lds, size_t block_lds);

int batch_solve(ditr_ctx* c, const ditr_graph* g, int R, const double* d_b, double* d_h, float* d_f,
                double rel_tol, const ditr_opts& o, ditr_stats* per_rhs, ditr_stats* total,
                void* d_workspace, size_t ws_bytes);

// host driver of the plain solve (api.hip)
int solve_impl(ditr_ctx* c, const ditr_graph* g, const double* d_b, double* d_h, float* d_f, int warm,
               double rel_tol, const ditr_opts* opts, ditr_stats* stats, const SolveBufs& sb,
               bool noalloc);
