// Device memory of a graph's tables, and the workspace sizes the C-ABI
// reports. A graph created with ditr_graph_create allocates every table with
// hipMalloc; one uploaded with ditr_graph_upload_csc carves them, in order and
// 256-byte aligned, out of a workspace the caller owns. Temporaries of the
// plan build are carved as well and simply left in place, so the bound below
// counts them too.
#include <algorithm>

#include "common.h"

namespace {
constexpr size_t kAlign = 256;
thread_local bool g_overflow = false;  // a workspace allocation failed on this thread
size_t al(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
}  // namespace

hipError_t g_alloc(ditr_graph* g, void** p, size_t bytes) {
  *p = nullptr;
  DevArena& a = g->arena;
  if (!a.base) return hipMalloc(p, bytes);
  const size_t need = al(std::max<size_t>(bytes, 1));
  if (a.used + need > a.cap) {
    g_overflow = true;
    return hipErrorOutOfMemory;
  }
  *p = a.base + a.used;
  a.used += need;
  a.peak = std::max(a.peak, a.used);
  return hipSuccess;
}

bool workspace_overflow(bool reset) {
  const bool v = g_overflow;
  if (reset) g_overflow = false;
  return v;
}

void g_free(ditr_graph* g, void* p) {
  if (p && !g->arena.base) (void)hipFree(p);
}

// Upper bound of the device bytes ditr_graph_upload_csc takes for a PageRank
// graph of n nodes and nnz links whose plans have between K_min and K_max
// partitions (the plan loop starts at K_min and may raise K up to n). Per link: the transpose (4 B), local
// targets (2 B), external in-links (at most 6 B, light or heavy), heavy items
// (at most nnz / 5 of them, 20 B each with their words) and their work units
// (at most 0.45 nnz / 64 + 9 units of 2304 B). Per node: the transpose
// pointer, heavy-row list, exact-residual work array, pull-sweep shares, plan
// ids, local ids, weights, counts and their scans. Per partition: pointers,
// thresholds, locks, sums.
size_t graph_workspace_bound(const ditr_ctx* c, int64_t n, int64_t nnz, int part_type, int64_t K_min,
                             int64_t K_max) {
  const size_t N = (size_t)n, L = (size_t)std::max<int64_t>(nnz, 1), K = (size_t)std::max<int64_t>(K_max, 1);
  const size_t tiles = N / 4096 + 2;
  const size_t nh = std::min<size_t>(N, L / (kHeavyRow + 1) + 1);
  const size_t nc = L / kHeavyChunk + nh + 1;
  // a heavy row has more than kPartHeavy external in-links, and an item at
  // most kItem of them
  const size_t nhp = std::min<size_t>(N, L / (kPartHeavy + 1) + 1);
  const size_t ni = nhp + L / kItem + 1;
  const size_t nu = (L / 4 + ni) / 64 + 9;
  size_t b = 0;
  // graph tables and the transpose
  b += al(4 * (N + 1)) + al(4 * L) + al(4 * N) + al(8 * N);
  b += al(4 * (N + 1)) + al(4 * tiles);
  // heavy chunks and the pull-sweep buffers
  b += al(8 * nh) + 3 * al(4 * nc) + al(8 * nc) + al(8 * N) + al(16 * nh) +
       al(32 * ((size_t)c->num_cus * 8 + nc));
  // one partition plan (each retry reuses the same space)
  b += al(4 * (K + 1)) + al(8 * K) + al(4 * K) + al(8 * (K + 1));
  if (part_type == DITR_PART_PMASS) b += pmass_temp_bytes(n, nnz);
  if (part_type == DITR_PART_MINCUT) b += mincut_temp_bytes(n, K_min, (int64_t)K);
  // the partitioned-sweep tables and the temporaries of their build (left in
  // place in a workspace): ids, local CSC, external links, heavy rows, items
  // and their work units, the two sorts, six scans
  b += al(4 * N) + al(2 * N) + 6 * al(4 * (N + 1)) + 2 * al(8 * N) + 2 * al(4 * N) +
       al(plan_sort_temp_bytes(n, (int64_t)ni)) + 6 * al(4 * tiles) + al(4) + 2 * al(4 * (N + 1));
  b += al(2 * (L + 4)) + al(4 * L) + al(2 * L) + al(4 * L);
  b += 3 * al(4 * (K + 1)) + al(4 * nhp) + 2 * al(4 * (nhp + 1));
  b += al(4 * ni) + 6 * al(4 * ni) + 2 * al(4 * (ni + 1)) + al(2048 * nu) + al(256 * nu) + al(16 * ni);
  b += al(4 * N) + al(8 * N) + al(32) + al(128 * K);
  return b + 64 * kAlign;
}
