// Autotuner of the plain solve: partition plan (Section 2.3: type and size),
// threshold divisor alpha (Section 2.4), local sweeps per launch and the
// first exact-refresh point, searched by time to tolerance on the caller's
// problem and cached in a JSON file keyed by a fingerprint of that problem.
//
// The paper finds alpha uninfluential over [1.2, 2] (Section 2.4) and the
// partition balance decisive (Section 3.2). On the GPU each threshold level
// costs about the same whatever it diffuses, so a larger alpha (fewer levels)
// can pay once the plan keeps the levels from being bound by the exchange:
// the alpha grid reaches 3. The search is a short coordinate descent:
// partition first, then alpha, local sweeps and the refresh point, each
// candidate accepted only when it beats the incumbent by a margin larger
// than the timing noise.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "common.h"

namespace {

double wall_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---- problem fingerprint ---------------------------------------------------
// Sum over elements of a 64-bit mix of (stream, position, value): insensitive to
// the order in which threads add, sensitive to every value and its position.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_hash_words(const uint32_t* __restrict__ w, int64_t nw, uint64_t stream,
                             unsigned long long* out) {
  uint64_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += mix64(stream ^ mix64(((uint64_t)i << 32) ^ w[i]));
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, (unsigned long long)acc);
}

int hash_device_words(ditr_ctx* c, const void* p, int64_t nw, uint64_t stream,
                      unsigned long long* d_acc, uint64_t* out) {
  HIP_TRY(hipMemsetAsync(d_acc, 0, sizeof(unsigned long long), c->stream));
  if (nw > 0) {
    const int64_t blocks = std::min<int64_t>((nw + 255) / 256, 4096);
    hipLaunchKernelGGL(k_hash_words, dim3((unsigned)blocks), dim3(256), 0, c->stream,
                       (const uint32_t*)p, nw, stream, d_acc);
    HIP_TRY(hipGetLastError());
  }
  unsigned long long h = 0;
  HIP_TRY(hipMemcpyAsync(&h, d_acc, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *out = h;
  return DITR_OK;
}

uint64_t hash_bytes(const void* p, size_t n, uint64_t h) {
  const unsigned char* s = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = mix64(h ^ s[i]);
  return h;
}

// ---- a small JSON reader for the cache file -------------------------------
struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* k) const {
    if (kind != OBJ) return nullptr;
    for (auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* p;
  const char* end;
  int depth = 0;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool lit(const char* s) {
    size_t n = strlen(s);
    if ((size_t)(end - p) < n || strncmp(p, s, n) != 0) return false;
    p += n;
    return true;
  }
  bool string(std::string& out) {
    if (p >= end || *p != '"') return false;
    ++p;
    while (p < end && *p != '"') {
      char ch = *p++;
      if (ch == '\\') {
        if (p >= end) return false;
        char e = *p++;
        switch (e) {
          case '"': case '\\': case '/': out.push_back(e); break;
          case 'n': out.push_back('\n'); break;
          case 't': out.push_back('\t'); break;
          case 'r': out.push_back('\r'); break;
          case 'b': out.push_back('\b'); break;
          case 'f': out.push_back('\f'); break;
          case 'u':  // keys and values written here are ASCII; keep the escape as '?'
            if (end - p < 4) return false;
            p += 4;
            out.push_back('?');
            break;
          default: return false;
        }
      } else {
        if ((unsigned char)ch < 0x20) return false;
        out.push_back(ch);
      }
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool value(JVal& v) {
    if (++depth > 32) return false;
    ws();
    if (p >= end) return false;
    bool ok = false;
    if (*p == '{') {
      ++p;
      v.kind = JVal::OBJ;
      ws();
      if (p < end && *p == '}') {
        ++p;
        ok = true;
      } else {
        for (;;) {
          ws();
          std::pair<std::string, JVal> kv;
          if (!string(kv.first)) break;
          ws();
          if (p >= end || *p != ':') break;
          ++p;
          if (!value(kv.second)) break;
          v.obj.push_back(std::move(kv));
          ws();
          if (p < end && *p == ',') { ++p; continue; }
          if (p < end && *p == '}') { ++p; ok = true; }
          break;
        }
      }
    } else if (*p == '[') {
      ++p;
      v.kind = JVal::ARR;
      ws();
      if (p < end && *p == ']') {
        ++p;
        ok = true;
      } else {
        for (;;) {
          JVal e;
          if (!value(e)) break;
          v.arr.push_back(std::move(e));
          ws();
          if (p < end && *p == ',') { ++p; continue; }
          if (p < end && *p == ']') { ++p; ok = true; }
          break;
        }
      }
    } else if (*p == '"') {
      v.kind = JVal::STR;
      ok = string(v.str);
    } else if (lit("true")) {
      v.kind = JVal::BOOL;
      v.num = 1;
      ok = true;
    } else if (lit("false")) {
      v.kind = JVal::BOOL;
      ok = true;
    } else if (lit("null")) {
      ok = true;
    } else {
      std::string tok;
      while (p < end && (isdigit((unsigned char)*p) || *p == '-' || *p == '+' || *p == '.' ||
                         *p == 'e' || *p == 'E'))
        tok.push_back(*p++);
      char* q = nullptr;
      if (!tok.empty()) {
        v.kind = JVal::NUM;
        v.num = strtod(tok.c_str(), &q);
        ok = q && *q == '\0';
      }
    }
    --depth;
    return ok;
  }
};

// Cache file: {"format": "ditr-tune-cache", "version": 1, "entries": [entry...]}
// entry: {"key": "<16 hex digits>", "alpha": .., "refresh_at": .., "part_type": ..,
//         "part_nodes": .., "sweeps_per_claim": .., "seconds": .., "default_seconds": ..}
struct Entry {
  uint64_t key = 0;
  double alpha = 2.0, refresh_at = 0;
  int part_type = DITR_PART_MINCUT, part_nodes = 0, m = 0;
  double seconds = 0, default_seconds = 0;
};

// Entries of a cache file; false if it is missing or not a cache file.
bool read_cache(const char* path, std::vector<Entry>& out) {
  out.clear();
  FILE* fp = fopen(path, "rb");
  if (!fp) return false;
  std::string text;
  char buf[65536];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), fp)) > 0) {
    text.append(buf, got);
    if (text.size() > ((size_t)64 << 20)) break;
  }
  fclose(fp);
  JParser jp{text.data(), text.data() + text.size()};
  JVal root;
  if (!jp.value(root)) return false;
  const JVal* fmt = root.get("format");
  const JVal* ents = root.get("entries");
  if (!fmt || fmt->kind != JVal::STR || fmt->str != "ditr-tune-cache") return false;
  if (!ents || ents->kind != JVal::ARR) return false;
  for (const JVal& e : ents->arr) {
    const JVal* k = e.get("key");
    if (!k || k->kind != JVal::STR || k->str.size() != 16) continue;
    char* q = nullptr;
    Entry en;
    en.key = strtoull(k->str.c_str(), &q, 16);
    if (!q || *q) continue;
    auto num = [&](const char* name, double dflt) {
      const JVal* v = e.get(name);
      return v && v->kind == JVal::NUM ? v->num : dflt;
    };
    en.alpha = num("alpha", 2.0);
    en.refresh_at = num("refresh_at", 0);
    en.part_type = (int)num("part_type", DITR_PART_MINCUT);
    en.part_nodes = (int)num("part_nodes", 0);
    en.m = (int)num("sweeps_per_claim", 0);
    en.seconds = num("seconds", 0);
    en.default_seconds = num("default_seconds", 0);
    if (!(en.alpha > 1) || !(en.refresh_at >= 0) || en.part_nodes < 0 || en.m < 0 ||
        (en.part_type != DITR_PART_CB && en.part_type != DITR_PART_UNIFORM &&
         en.part_type != DITR_PART_CB_INOUT && en.part_type != DITR_PART_PMASS &&
         en.part_type != DITR_PART_MINCUT))
      continue;
    out.push_back(en);
  }
  return true;
}

// Rewrite the cache with `e` added (replacing an entry of the same key):
// written to a temporary file next to it, then renamed over it.
int write_cache(const char* path, const Entry& e) {
  std::vector<Entry> ents;
  read_cache(path, ents);
  ents.erase(std::remove_if(ents.begin(), ents.end(), [&](const Entry& x) { return x.key == e.key; }),
             ents.end());
  ents.push_back(e);
  std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
  FILE* fp = fopen(tmp.c_str(), "wb");
  if (!fp) return set_error(DITR_EINVAL, "cannot write tuning cache %s", tmp.c_str());
  fprintf(fp, "{\"format\": \"ditr-tune-cache\", \"version\": 1, \"entries\": [");
  for (size_t i = 0; i < ents.size(); ++i) {
    const Entry& x = ents[i];
    fprintf(fp,
            "%s\n  {\"key\": \"%016llx\", \"alpha\": %.17g, \"refresh_at\": %.17g, "
            "\"part_type\": %d, \"part_nodes\": %d, \"sweeps_per_claim\": %d, "
            "\"seconds\": %.9g, \"default_seconds\": %.9g}",
            i ? "," : "", (unsigned long long)x.key, x.alpha, x.refresh_at, x.part_type,
            x.part_nodes, x.m, x.seconds, x.default_seconds);
  }
  fprintf(fp, "\n]}\n");
  const bool ok = fflush(fp) == 0 && !ferror(fp);
  fclose(fp);
  if (!ok || rename(tmp.c_str(), path) != 0) {
    unlink(tmp.c_str());
    return set_error(DITR_EINVAL, "cannot write tuning cache %s", path);
  }
  return DITR_OK;
}

void apply(const Entry& e, ditr_opts* o) {
  o->alpha = e.alpha;
  o->refresh_at = e.refresh_at;
  o->part_type = e.part_type;
  o->part_nodes = e.part_nodes;
  o->sweeps_per_claim = e.m;
}

struct Problem {
  ditr_ctx* c;
  int64_t n, nnz;
  const int32_t *col_ptr, *row_idx;
  double d;
  const double* b;
  double* h;
  float* f;
  double tol;
};

// Best wall time to tolerance of `reps` solves with options `e`, after one
// untimed solve when `warm`. +inf if the plan does not fit or a solve fails.
int time_candidate(const Problem& P, const ditr_opts& base, const Entry& e, int reps, bool warm,
                   double* secs, int64_t* edges, bool may_skip = true) {
  *secs = INFINITY;
  *edges = 0;
  ditr_opts o = base;
  apply(e, &o);
  ditr_graph* g = nullptr;
  int rc = ditr_graph_create(P.c, &g, P.n, P.nnz, P.col_ptr, P.row_idx, P.d, &o);
  if (rc == DITR_EINVAL && may_skip) return DITR_OK;  // no plan of this size fits: skip it
  if (rc) return rc;
  for (int i = warm ? -1 : 0; i < reps; ++i) {
    ditr_stats st;
    const double t0 = wall_now();
    rc = ditr_solve(P.c, g, P.b, P.h, P.f, 0, P.tol, &o, &st);
    const double dt = wall_now() - t0;
    if (rc != DITR_OK) break;
    if (i >= 0 && dt < *secs) {
      *secs = dt;
      *edges = st.edges;
    }
  }
  ditr_graph_destroy(g);
  if (rc < 0) return rc;
  if (rc != DITR_OK) *secs = INFINITY;  // did not converge within its budget: rejected
  return DITR_OK;
}

}  // namespace

extern "C" {

int ditr_tune_cache_get(const char* path, uint64_t key, ditr_opts* out) {
  if (!path || !out) return set_error(DITR_EINVAL, "NULL argument");
  std::vector<Entry> ents;
  read_cache(path, ents);
  for (auto it = ents.rbegin(); it != ents.rend(); ++it)
    if (it->key == key) {
      apply(*it, out);
      return DITR_OK;
    }
  return DITR_NOT_FOUND;
}

int ditr_tune_cache_put(const char* path, uint64_t key, const ditr_opts* o, double seconds,
                        double default_seconds) {
  if (!path || !o) return set_error(DITR_EINVAL, "NULL argument");
  if (!(o->alpha > 1) || !(o->refresh_at >= 0) || o->part_nodes < 0 || o->sweeps_per_claim < 0 ||
      (o->part_type != DITR_PART_CB && o->part_type != DITR_PART_UNIFORM &&
       o->part_type != DITR_PART_CB_INOUT && o->part_type != DITR_PART_PMASS &&
       o->part_type != DITR_PART_MINCUT))
    return set_error(DITR_EINVAL, "options out of range");
  Entry e;
  e.key = key;
  e.alpha = o->alpha;
  e.refresh_at = o->refresh_at;
  e.part_type = o->part_type;
  e.part_nodes = o->part_nodes;
  e.m = o->sweeps_per_claim;
  e.seconds = seconds;
  e.default_seconds = default_seconds;
  return write_cache(path, e);
}

int ditr_tune_key(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* d_col_ptr,
                  const int32_t* d_row_idx, double damping, const double* d_b, double rel_tol,
                  uint64_t* key) {
  if (!c || !d_col_ptr || !d_b || !key || (nnz > 0 && !d_row_idx))
    return set_error(DITR_EINVAL, "NULL argument");
  if (n < 1 || nnz < 0) return set_error(DITR_EINVAL, "bad sizes");
  HIP_TRY(hipSetDevice(c->device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, c->device));
  unsigned long long* acc = nullptr;
  HIP_TRY(hipMalloc((void**)&acc, sizeof(*acc)));
  uint64_t hc = 0, hr = 0, hb = 0;
  int rc = hash_device_words(c, d_col_ptr, n + 1, 1, acc, &hc);
  if (!rc) rc = hash_device_words(c, d_row_idx, nnz, 2, acc, &hr);
  if (!rc) rc = hash_device_words(c, d_b, 2 * n, 3, acc, &hb);
  (void)hipFree(acc);
  if (rc) return rc;
  uint64_t k = mix64((uint64_t)n) ^ mix64((uint64_t)nnz + 1);
  k = hash_bytes(&damping, sizeof(damping), k);
  k = hash_bytes(&rel_tol, sizeof(rel_tol), k);
  k = hash_bytes(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)), k);
  k = hash_bytes(&prop.multiProcessorCount, sizeof(int), k);
  k = mix64(k ^ hc) ^ mix64(k + hr) ^ mix64(~k ^ hb);
  *key = k;
  return DITR_OK;
}

int ditr_tune(ditr_ctx* c, int64_t n, int64_t nnz, const int32_t* d_col_ptr,
              const int32_t* d_row_idx, double damping, const double* d_b, double* d_h, float* d_f,
              double rel_tol, int effort, const char* cache_path, ditr_opts* out,
              ditr_tune_info* info) {
  const double t_start = wall_now();
  if (!c || !d_col_ptr || !d_b || !d_h || !d_f || !out || (nnz > 0 && !d_row_idx))
    return set_error(DITR_EINVAL, "NULL argument");
  if (!(rel_tol > 0) || !std::isfinite(rel_tol)) return set_error(DITR_EINVAL, "rel_tol must be > 0");
  if (effort < 0 || effort > 2) return set_error(DITR_EINVAL, "effort must be 0, 1 or 2");
  ditr_tune_info inf;
  memset(&inf, 0, sizeof(inf));
  ditr_opts base;
  ditr_opts_default(&base);
  base.flags = 0;

  int rc = ditr_tune_key(c, n, nnz, d_col_ptr, d_row_idx, damping, d_b, rel_tol, &inf.key);
  if (rc) return rc;
  if (cache_path) {
    ditr_opts cached = base;
    if (ditr_tune_cache_get(cache_path, inf.key, &cached) == DITR_OK) {
      *out = cached;
      inf.from_cache = 1;
      inf.seconds = wall_now() - t_start;
      if (info) *info = inf;
      return DITR_OK;
    }
  }

  const Problem P{c, n, nnz, d_col_ptr, d_row_idx, damping, d_b, d_h, d_f, rel_tol};
  Entry def;  // the library defaults
  def.alpha = base.alpha;
  def.refresh_at = base.refresh_at;
  def.part_type = base.part_type;
  def.part_nodes = base.part_nodes;
  def.m = base.sweeps_per_claim;

  double t_def = 0;
  int64_t e_def = 0;
  rc = time_candidate(P, base, def, 1, true, &t_def, &e_def, false);
  if (rc) return rc;
  inf.candidates += 1;
  if (!std::isfinite(t_def)) return set_error(DITR_NOT_CONVERGED, "default options do not converge");
  // repetitions per candidate: fewer on large problems, where one solve is long
  const int reps = t_def > 0.25 ? 1 : t_def > 0.05 ? 2 : 3;
  const bool warm = t_def < 0.05;
  Entry best = def;
  double t_best = INFINITY;
  int64_t e_best = 0;
  rc = time_candidate(P, base, def, reps, false, &t_best, &e_best);
  if (rc) return rc;
  inf.candidates += 1;
  const double margin = 0.97;  // a candidate must be 3% faster to replace the incumbent

  auto consider = [&](const Entry& e) -> int {
    double t;
    int64_t ed;
    int r = time_candidate(P, base, e, reps, warm, &t, &ed);
    if (r) return r;
    inf.candidates += 1;
    if (t < margin * t_best) {
      best = e;
      t_best = t;
      e_best = ed;
    }
    return DITR_OK;
  };

  // stage 1: partition plan (type x nodes per partition; 0 = the library's choice)
  const int types_all[5] = {DITR_PART_MINCUT, DITR_PART_CB_INOUT, DITR_PART_CB, DITR_PART_UNIFORM,
                            DITR_PART_PMASS};
  const int ntypes = effort == 0 ? 1 : 5;
  const int sizes[6] = {0, 1024, 2048, 3072, 6144, 8192};
  for (int ti = 0; ti < ntypes; ++ti)
    for (int s : sizes) {
      Entry e = best;
      e.part_type = types_all[ti];
      e.part_nodes = s;
      if (e.part_type == best.part_type && e.part_nodes == best.part_nodes) continue;
      if ((rc = consider(e))) return rc;
    }
  const int passes = effort == 2 ? 2 : 1;
  for (int pass = 0; pass < passes; ++pass) {
    // stage 2: threshold divisor alpha (Section 2.4: [1.2, 2], and beyond)
    for (double a : {1.2, 1.5, 1.75, 2.0, 2.5, 3.0}) {
      Entry e = best;
      e.alpha = a;
      if (a == best.alpha) continue;
      if ((rc = consider(e))) return rc;
    }
    if (effort == 0) break;
    // stage 3: local sweeps per launch
    for (int m : {1, 2, 3, 4}) {
      Entry e = best;
      e.m = m;
      if (m == (best.m > 0 ? best.m : 3)) continue;
      if ((rc = consider(e))) return rc;
    }
    // stage 4: first exact refresh
    for (double ra : {1e-5, 1e-6, 1e-7, 1e-8}) {
      Entry e = best;
      e.refresh_at = ra;
      if (ra == best.refresh_at) continue;
      if ((rc = consider(e))) return rc;
    }
  }

  // re-time the winner against the defaults: the minimum that chose it is biased low
  double t_def2 = INFINITY, t_win = INFINITY;
  int64_t e_def2 = 0, e_win = 0;
  const int final_reps = std::max(reps, 2);
  rc = time_candidate(P, base, def, final_reps, warm, &t_def2, &e_def2);
  if (!rc) rc = time_candidate(P, base, best, final_reps, warm, &t_win, &e_win);
  if (rc) return rc;
  inf.candidates += 2;
  if (!(t_win < t_def2)) {
    best = def;
    t_win = t_def2;
    e_win = e_def2;
  }
  inf.default_seconds = t_def2;
  inf.default_edges = e_def2;
  inf.best_seconds = t_win;
  inf.best_edges = e_win;

  ditr_opts o = base;
  apply(best, &o);
  if (cache_path) {
    Entry ce = best;
    ce.key = inf.key;
    ce.seconds = t_win;
    ce.default_seconds = t_def2;
    rc = write_cache(cache_path, ce);
    if (rc) return rc;
  }
  *out = o;
  inf.seconds = wall_now() - t_start;
  if (info) *info = inf;
  return DITR_OK;
}

// Batched solve: the threshold schedule of every right-hand side (alpha) and
// the first exact-refresh point, by wall time to tolerance of the whole batch.
// The batched sweep has no partition plan, so these are its only schedule
// knobs; the graph and the workspace are the caller's.
int ditr_tune_batched(ditr_ctx* c, const ditr_graph* g, int nrhs, const double* d_b, double* d_h, float* d_f,
                      double rel_tol, void* d_workspace, size_t ws_bytes, int effort, ditr_opts* out,
                      ditr_tune_info* info) {
  const double t_start = wall_now();
  if (!c || !g || !d_b || !d_h || !d_f || !out) return set_error(DITR_EINVAL, "NULL argument");
  if (!(rel_tol > 0) || !std::isfinite(rel_tol)) return set_error(DITR_EINVAL, "rel_tol must be > 0");
  if (effort < 0 || effort > 2) return set_error(DITR_EINVAL, "effort must be 0, 1 or 2");
  ditr_tune_info inf;
  memset(&inf, 0, sizeof(inf));
  ditr_opts base;
  ditr_opts_default(&base);
  base.flags = 0;
  // best of reps timed batches with options o (+inf if a batch does not converge)
  auto timed = [&](const ditr_opts& o, int reps, double* secs, int64_t* edges) -> int {
    *secs = INFINITY;
    *edges = 0;
    for (int i = 0; i < reps; ++i) {
      ditr_stats tot;
      const double t0 = wall_now();
      const int rc = ditr_solve_batched(c, g, nrhs, d_b, d_h, d_f, rel_tol, &o, d_workspace, ws_bytes, nullptr, &tot);
      const double dt = wall_now() - t0;
      inf.candidates += 1;
      if (rc < 0) return rc;
      if (rc != DITR_OK) return DITR_OK;  // did not converge: rejected
      if (dt < *secs) {
        *secs = dt;
        *edges = tot.edges;
      }
    }
    return DITR_OK;
  };
  double t_def = 0;
  int64_t e_def = 0;
  int rc = timed(base, 1, &t_def, &e_def);  // also warms the workspace and the code
  if (rc) return rc;
  if (!std::isfinite(t_def)) return set_error(DITR_NOT_CONVERGED, "default options do not converge");
  const int reps = t_def > 0.25 ? 1 : 2;
  ditr_opts best = base;
  double t_best = INFINITY;
  int64_t e_best = 0;
  if ((rc = timed(base, reps, &t_best, &e_best))) return rc;
  const double margin = 0.97;
  auto consider = [&](const ditr_opts& o) -> int {
    double t;
    int64_t ed;
    const int r = timed(o, reps, &t, &ed);
    if (r) return r;
    if (t < margin * t_best) {
      best = o;
      t_best = t;
      e_best = ed;
    }
    return DITR_OK;
  };
  const int passes = effort == 2 ? 2 : 1;
  for (int pass = 0; pass < passes; ++pass) {
    for (double a : {1.25, 1.5, 2.0, 3.0, 4.0}) {
      if (a == best.alpha) continue;
      ditr_opts o = best;
      o.alpha = a;
      if ((rc = consider(o))) return rc;
    }
    if (effort == 0) break;
    for (double ra : {1e-5, 1e-6, 1e-7}) {
      if (ra == best.refresh_at) continue;
      ditr_opts o = best;
      o.refresh_at = ra;
      if ((rc = consider(o))) return rc;
    }
  }
  // re-time the winner against the defaults
  double t_def2, t_win;
  int64_t e_def2, e_win;
  const int final_reps = std::max(reps, 2);
  if ((rc = timed(base, final_reps, &t_def2, &e_def2))) return rc;
  if ((rc = timed(best, final_reps, &t_win, &e_win))) return rc;
  if (!(t_win < t_def2)) {
    best = base;
    t_win = t_def2;
    e_win = e_def2;
  }
  inf.default_seconds = t_def2;
  inf.default_edges = e_def2;
  inf.best_seconds = t_win;
  inf.best_edges = e_win;
  *out = best;
  inf.seconds = wall_now() - t_start;
  if (info) *info = inf;
  return DITR_OK;
}

}  // extern "C"
