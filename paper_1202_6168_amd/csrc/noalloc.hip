// The plain solve for callers that cannot allocate device memory.
//
// ditr_solve takes its per-solve buffers (published shares, heavy-item words,
// per-workgroup sums, level counters, the exact residual's work arrays) from
// tables the library allocated when the graph was created. ditr_solve_noalloc
// takes them from one fixed array of device memory that is part of the
// library's code object, so the call itself performs no allocation of any kind.
//
// The array's address differs per device and cannot be taken from host code by
// its name (the host symbol is only a stand-in): each context looks it up with
// hipGetSymbolAddress when it is created, once per device, and every launch
// receives that device address as an ordinary kernel argument.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "common.h"

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device

// Every device that runs the library holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
unsigned char* g_addr[kMaxDevices] = {};  // device address of `scratch`, per device

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of the solve's buffers inside the scratch; returns the bytes needed.
size_t layout(const ditr_graph* g, unsigned char* base, SolveBufs* sb) {
  const int64_t n = g->n, K = g->K;
  const int64_t items = std::max<int64_t>(1, g->pp.n_items);
  const int64_t chunks = std::max<int64_t>(1, g->n_chunks);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  sb->S = reinterpret_cast<float*>(take(sizeof(float) * 2 * (size_t)n));
  sb->item_word = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * 2 * (size_t)items));
  sb->partials = reinterpret_cast<double*>(take(sizeof(double) * 8 * 2 * (size_t)K));
  sb->counters = reinterpret_cast<int*>(take(sizeof(int) * 8));
  sb->wh = reinterpret_cast<double*>(take(sizeof(double) * (size_t)n));
  sb->chunk_sum = reinterpret_cast<double*>(take(sizeof(double) * (size_t)chunks));
  return off;
}

}  // namespace

int noalloc_init(ditr_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return set_error(DITR_EINVAL, "device %d is beyond the library's device table", c->device);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[c->device]) {
    void* p = nullptr;  // the caller has made c->device current
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(DITR_EHIP, "hipGetSymbolAddress of the static scratch failed: %s",
                       hipGetErrorString(e));
    g_addr[c->device] = static_cast<unsigned char*>(p);
  }
  c->scratch = g_addr[c->device];
  c->scratch_bytes = kScratchBytes;
  return DITR_OK;
}

extern "C" {

size_t ditr_noalloc_scratch_bytes(void) { return kScratchBytes; }

int ditr_solve_noalloc(ditr_ctx* c, const ditr_graph* g, const double* d_b, double* d_h, float* d_f,
                       int warm, double rel_tol, const ditr_opts* opts, ditr_stats* stats) {
  if (stats) memset(stats, 0, sizeof(*stats));
  auto fail = [&](int rc) {
    if (stats) stats->status = rc;
    return rc;
  };
  if (!c || !g || !d_b || !d_h || !d_f) return fail(set_error(DITR_EINVAL, "NULL argument"));
  if (!c->scratch) return fail(set_error(DITR_EINVAL, "context has no static scratch"));
  if (g->device != c->device) return fail(set_error(DITR_EINVAL, "graph and context on different devices"));
  SolveBufs sb;
  const size_t need = layout(g, nullptr, &sb);
  if (need > c->scratch_bytes)
    return fail(set_error(DITR_EINVAL,
                          "graph of n = %lld needs %zu bytes of solve buffers; the static scratch "
                          "holds %zu",
                          (long long)g->n, need, c->scratch_bytes));
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return fail(set_error(DITR_EHIP, "hipSetDevice: %s", hipGetErrorString(e)));
  layout(g, c->scratch, &sb);
  // the scratch keeps whatever the previous call on this device left: the
  // heavy-item words must start below every epoch of this call (the stage
  // preparation clears the counters and shares itself)
  int rc = launch_zero_u64(c, sb.item_word, 2 * (int64_t)std::max<int32_t>(1, g->pp.n_items));
  if (rc) return fail(rc);
  int64_t epoch = 0;
  sb.epoch = &epoch;
  return solve_impl(c, g, d_b, d_h, d_f, warm, rel_tol, opts, stats, sb, true);
}

}  // extern "C"
