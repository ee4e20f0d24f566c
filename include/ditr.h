/*
 * ditr.h — D-iteration fluid diffusion on AMD Instinct MI355X (gfx950).
 *
 * Solves X = P X + B for the PageRank-type matrix P with p_ji = d / #out_i on
 * every out-link i -> j (a dangling node has an all-zero column), by the
 * D-iteration of Hong, arXiv:1202.6168: a fluid vector F (F_0 = B) and a
 * history vector H (H_0 = 0) evolve by node diffusions
 *     sent = F_i;  H_i += sent;  F_i = 0;  F_j += sent * p_ji for each child j
 * (Section 2, equations defF and defH, and the Section 2.1 pseudo-code) until
 * ||F||_1 falls below a target. H then approximates X with
 * ||X - H||_1 <= ||F||_1 / (1 - d) (Section 2, the bound after defH).
 *
 * Conventions shared by every entry point:
 *   - Graphs are CSC with int32 indices: column i, entries
 *     col_ptr[i] .. col_ptr[i+1]-1 of row_idx, lists the out-neighbours of
 *     node i. Self-loops and repeated entries are legal; each entry carries
 *     d / #out_i. n < 2^31, nnz < 2^31.
 *   - "d_" pointers are DEVICE pointers on the context's device; the caller
 *     allocates and owns them (PyTorch tensors in the Python binding). The
 *     library keeps non-owning references: a graph borrows its CSC arrays,
 *     which must outlive the graph. "h_" pointers are host memory.
 *   - Every call is asynchronous on the context's stream unless it says it
 *     synchronizes. Calls that return host values synchronize the stream.
 *   - Every function returns a ditr_status. No exception or abort crosses
 *     the ABI; ditr_last_error() gives a message for the calling thread.
 *   - A context is used from one host thread at a time (ditr_abort excepted).
 *   - Graphs, tuning calls and networks use their context while they run; they
 *     may be destroyed after it (their destroy waits for the device).
 */
#ifndef DITR_H
#define DITR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DITR_ABI_VERSION 1

typedef enum {
  DITR_OK = 0,
  DITR_NOT_CONVERGED = 1, /* budget hit; H and F are valid (F = B + P H - H holds) */
  DITR_ABORTED = 2,       /* ditr_abort() was called; H and F are valid */
  DITR_NOT_FOUND = 3,     /* no tuning cache entry under the key */
  DITR_EINVAL = -1,       /* bad argument (null pointer, size, damping outside (0,1), ...) */
  DITR_EGRAPH = -2,       /* CSC is malformed (col_ptr not monotone, row out of range, ...) */
  DITR_ENOMEM = -3,       /* device or pinned host allocation failed */
  DITR_EHIP = -4,         /* a HIP runtime call failed, or a bounded wait inside the resident
                             partitioned sweep timed out (the kernel then exits normally) */
  DITR_ENONFINITE = -5    /* B or H_0 holds NaN or Inf */
} ditr_status;

typedef struct ditr_ctx ditr_ctx;     /* one device + one stream; opaque */
typedef struct ditr_graph ditr_graph; /* uploaded CSC + partition plan + transpose; opaque */

/* Node-set partition types (Section 2.3). */
enum { DITR_PART_CB = 0,       /* cost-balanced: contiguous ranges of ~L/K out-links */
       DITR_PART_UNIFORM = 1,  /* contiguous ranges of floor(N/K) ids, last one takes the rest */
       DITR_PART_CB_INOUT = 2, /* contiguous ranges of ~2L/K in+out links: a partition's whole
                                  link cost (a cheap proxy for the balance below) */
       DITR_PART_PMASS = 3,    /* the alternative balance the paper proposes after the CB rule:
                                  equal internal p mass sum_{n,m in Omega_k} |p_nm| per block
                                  (ditr_partition_pmass gives the exact rule) */
       DITR_PART_MINCUT = 4    /* cut-minimizing CB: CB targets on the node cost
                                  1 + #out + min(#in, h), each boundary then moved within a
                                  window, under a 10% balance slack, to where the least p mass
                                  of short links crosses (keeps more of the p mass inside the
                                  sets, the aim of the Section 2.3 alternative; exact rule at
                                  ditr_partition) */ };

/* Diffusion kernels. */
enum { DITR_MODE_AUTO = 0,       /* = DITR_MODE_PARTITION */
       DITR_MODE_ASYNC = 1,      /* persistent workgroups own partitions held in LDS and exchange
                                    fluid through atomic inboxes, no grid-wide barrier
                                    (Sections 2.3-2.6, asynchronous) */
       DITR_MODE_SWEEP = 2,      /* one grid-wide threshold sweep per launch, pulled over the
                                    transpose (Section 2.4 applied to a node set) */
       DITR_MODE_PARTITION = 3   /* per threshold level, m local threshold sweeps per partition
                                    in LDS, outside fluid pulled as p_ji times the H increment
                                    (Sections 2.3-2.5, synchronous exchange); partitions stay
                                    resident across levels when they all fit the device */ };

typedef struct {
  double alpha;        /* threshold divisor after each sweep (Section 2.4); > 1; default 2 */
  double refresh_at;   /* first exact FP64 residual refresh once ||F||_1 <= refresh_at ||B||_1
                          (cancels FP32 rounding drift); >= 0; default 0, the library's
                          choice: 1e-7 (partitioned and pull sweeps), 1e-5 (asynchronous
                          kernel), 1e-6 (batched solve) */
  double park_ratio;   /* a partition idles while its fluid is below park_ratio times its
                          node share of the remaining fluid (Section 2.4, r_k < T); default 0.5 */
  double rescale_cap;  /* max factor a reception may raise a partition threshold (Section 2.6) */
  int32_t mode;        /* DITR_MODE_* */
  int32_t part_type;   /* DITR_PART_*; default DITR_PART_MINCUT */
  int32_t part_nodes;  /* nodes per partition target; 0 = from LDS capacity */
  int32_t block;       /* threads per workgroup (64..1024, multiple of 64); 0 = auto */
  int32_t wg_per_cu;   /* resident workgroups per CU for the persistent kernel; 0 = auto */
  int32_t sweeps_per_claim; /* ASYNC: local sweeps per partition claim when partitions
                               outnumber workgroups; PARTITION: local sweeps per threshold
                               level (m); 0 = auto (2 for ASYNC, 3 for PARTITION) */
  int32_t max_rounds;  /* persistent launches (each followed by an exact residual) */
  int32_t max_sweeps;  /* PARTITION: threshold levels per stage; ASYNC: sweeps per workgroup
                          and launch; SWEEP: grid sweeps per stage (0 = auto) */
  int32_t xcd_remap;   /* 1: place neighbouring partitions on the same XCD */
  uint32_t flags;      /* DITR_FLAG_* bits */
} ditr_opts;

/* opts.flags: time every diffusion launch with HIP events on the context's
 * stream and report the sum in ditr_stats.kernel_seconds. */
#define DITR_FLAG_TIME_KERNELS 1u
/* opts.flags: in DITR_MODE_PARTITION, relaunch the sweep once per threshold
 * level even when every partition could stay resident in one cooperative
 * launch (the default whenever the partitions fit the device at once). */
#define DITR_FLAG_NO_RESIDENT 2u
/* opts.flags: in DITR_MODE_PARTITION, diffuse node i when its normalized
 * priority |F_i| / ((#in_i + 1)(#out_i + 1)) exceeds T, the quantity whose
 * argmax Section 2.4 names as the node choice, under the same cyclic threshold
 * schedule (T_0, T /= alpha, no-pass rule on that ratio). Needs
 * sum_i (#in_i + 1)(#out_i + 1) < 2^28 (DITR_EINVAL otherwise); other modes
 * return DITR_EINVAL. */
#define DITR_FLAG_PRIORITY 4u

typedef struct {
  int64_t edges;       /* elementary edge diffusions (Section 2.4: normalized iterations x L) */
  int64_t diffusions;  /* node diffusions */
  int64_t sweeps;      /* PARTITION: threshold levels; ASYNC: partition sweeps summed over
                          workgroups; SWEEP: grid sweeps */
  int64_t launches;    /* diffusion kernel launches */
  int64_t refreshes;   /* exact FP64 residual refreshes F = B + P H - H */
  int64_t idle_polls;  /* polls that found nothing yet (Section 3.3 idle time): ASYNC, an idle
                          workgroup on its inbox; PARTITION (resident), a partition waiting
                          for the others to finish the previous level */
  double resid_l1;     /* final exact ||F||_1 (FP64, from the last refresh) */
  double b_l1;         /* ||B||_1 */
  double seconds;      /* host wall time of the call */
  double kernel_seconds;  /* with DITR_FLAG_TIME_KERNELS: event-timed diffusion launches */
  int64_t timed_launches; /* kernel launches covered by kernel_seconds (a resident
                             partitioned stage is one launch of many levels) */
  int32_t rounds;      /* outer rounds used */
  int32_t status;      /* same as the return value */
} ditr_stats;

/* ---- library and context ---------------------------------------------- */
int ditr_version(void);
const char* ditr_last_error(void); /* thread-local; valid until the thread's next call */
int ditr_opts_default(ditr_opts* o);

/* Create a context on `device` that issues work on `hip_stream` (a hipStream_t;
 * NULL = the null stream). Allocates a pinned host abort word. */
int ditr_create(ditr_ctx** out, int device, void* hip_stream);
int ditr_destroy(ditr_ctx* ctx);
/* Ask a running ditr_solve on this context to stop (thread-safe). The solver
 * returns DITR_ABORTED with a consistent (H, F). Cleared by the next solve. */
int ditr_abort(ditr_ctx* ctx);

/* ---- graph (step: upload and partition plan) --------------------------- */
/* Validate the CSC on the device, build the transpose (CSR, used by the exact
 * residual) and the partition plan of Section 2.3 (type and size from opts;
 * NULL = defaults). Synchronizes. Errors: DITR_EGRAPH for a malformed CSC,
 * DITR_EINVAL for bad sizes or damping outside (0, 1). */
int ditr_graph_create(ditr_ctx* ctx, ditr_graph** out, int64_t n, int64_t nnz,
                      const int32_t* d_col_ptr, const int32_t* d_row_idx, double damping,
                      const ditr_opts* opts);
/* General matrix (Section 2: p_ij is the weight of the link j -> i, of either
 * sign; Section 1, equation affine, with any B): the same CSC plus d_val, one
 * FP64 weight per CSC entry (device, borrowed, must outlive the graph). P must
 * be strictly contractive in the l1 column norm, c = max_i sum_j |p_ji| < 1
 * (the series sum_n P^n B then converges, and the bound of Section 2 holds with
 * c in place of d); it is checked on the device, and DITR_EINVAL returned
 * otherwise or for a NaN or Inf weight. ditr_solve then runs the pull sweep
 * (DITR_MODE_AUTO or DITR_MODE_SWEEP); the other modes, the batched solve and
 * the warm-start network take PageRank graphs only and return DITR_EINVAL.
 * ditr_residual forms B + P H - H with these weights. Synchronizes. */
int ditr_graph_create_weighted(ditr_ctx* ctx, ditr_graph** out, int64_t n, int64_t nnz,
                               const int32_t* d_col_ptr, const int32_t* d_row_idx,
                               const double* d_val, const ditr_opts* opts);
/* Contraction factor of g's matrix: the damping d of a PageRank graph, c of a
 * general one (0 when it has no links). */
int ditr_graph_contraction(const ditr_graph* g, double* c_out);
int ditr_graph_destroy(ditr_graph* g);
/* ---- caller-owned workspaces ------------------------------------------- */
/* Device bytes a call needs from a caller-provided workspace (an upper bound
 * computed from the sizes alone):
 *   nrhs = 0:  ditr_graph_upload_csc of a PageRank graph of n nodes and nnz
 *              links with opts' partition type (NULL = defaults); the plan's
 *              every table and temporary (transpose, partition tables, work
 *              arrays of the solve and the exact residual) lies in it;
 *   nrhs = R:  ditr_solve_batched with R right-hand sides (multiple of 4,
 *              4..256): published shares, gathered inflow, activity flags,
 *              heavy-row sums, per-right-hand-side thresholds and partials.
 * Host-only (no device work). */
int ditr_workspace_bytes(ditr_ctx* ctx, int64_t n, int64_t nnz, int nrhs, const ditr_opts* opts,
                         size_t* bytes);
/* ditr_graph_create with every device table carved from d_workspace (device,
 * 256-byte aligned, ws_bytes long, owned by the caller, which must keep it
 * until ditr_graph_destroy): the library allocates no device memory for the
 * graph. DITR_ENOMEM if the workspace is too small (ditr_workspace_bytes with
 * nrhs = 0 always suffices; ditr_graph_workspace_used tells what a graph
 * took). PageRank matrices only. Synchronizes. */
int ditr_graph_upload_csc(ditr_ctx* ctx, ditr_graph** out, int64_t n, int64_t nnz,
                          const int32_t* d_col_ptr, const int32_t* d_row_idx, double damping,
                          void* d_workspace, size_t ws_bytes, const ditr_opts* opts);
/* Workspace bytes an uploaded graph actually used (0 for ditr_graph_create). */
int ditr_graph_workspace_used(const ditr_graph* g, size_t* used);

/* Replace the partition plan of g by the boundaries h_ptr[0..K] (host, 0 =
 * h_ptr[0] <= ... <= h_ptr[K] = n) and rebuild its tables (Section 2.3: any
 * node-set partition is valid). DITR_EINVAL if a part exceeds the nodes one
 * workgroup holds in LDS, or for a graph uploaded into a caller workspace
 * (which keeps its plan). Synchronizes. */
int ditr_graph_set_partitions(ditr_ctx* ctx, ditr_graph* g, const int64_t* h_ptr, int64_t K);

typedef struct {
  int32_t rounds;         /* adaptation rounds run */
  int32_t kept;           /* rounds whose plan was kept (the solve got faster) */
  double seconds_before;  /* best of 3 solves to tolerance with the plan on entry */
  double seconds_after;   /* the same with the plan on return (<= seconds_before) */
  double spread_before;   /* slowest partition's mean work per level over the mean, on entry */
  double spread_after;    /* the same on return */
  double seconds;         /* host wall time of the call */
} ditr_adapt_info;

/* Partition adaptation (Section 3.4, where the boundary between two PIDs moves
 * towards the one that does more work): time the partitioned solve of
 * (d_b, rel_tol) on g, trace each partition's work per level (ditr_set_trace),
 * move every boundary a fraction omega (0 < omega <= 1) of the way to the
 * points that split the measured work into K equal parts (a partition's nodes
 * share its work evenly), rebuild the plan and time again. A plan is kept only
 * if the solve is at least 0.5% faster; otherwise the previous one is restored
 * and the adaptation stops. At most `rounds` rounds (0..64). d_h and d_f are
 * work buffers (overwritten). DITR_EINVAL for a general matrix (solved by the
 * pull sweep, which has no partitions) or a graph in a caller workspace.
 * `info` may be NULL. Synchronizes. */
int ditr_graph_adapt(ditr_ctx* ctx, ditr_graph* g, const double* d_b, double* d_h, float* d_f,
                     double rel_tol, int rounds, double omega, ditr_adapt_info* info);

/* Number of partitions K of the plan and, if h_ptr != NULL and cap >= K+1,
 * the boundaries omega_0 = 0 < ... <= omega_K = n. Synchronizes. */
int ditr_graph_partitions(const ditr_graph* g, int64_t* K_out, int64_t* h_ptr, int64_t cap);
/* Standalone partition plan kernel (Section 2.3): writes K+1 boundaries to
 * d_ptr (device int64, 1 <= K <= n). CB: omega_k = min { j : K col_ptr[j] >= k nnz }.
 * CB_INOUT: the same with col_ptr[j] + in_prefix[j] against 2 nnz, where
 * in_prefix counts the entries of d_row_idx below j (d_row_idx may be NULL for
 * CB and UNIFORM). MINCUT (reads d_row_idx):
 *   - node cost c_i = 1 + #out_i + min(#in_i, h), h = max(1, floor(3 nnz / n)),
 *     prefix C; targets t_k = min { j : K C(j) >= k C(n) };
 *   - balance: every set costs at most cB + floor(cB/10) and holds at most
 *     sB + floor(sB/10) nodes, cB and sB the largest over the targets' sets;
 *   - a link i -> j, i != j, with |i - j| < 2 ceil(n/K) weighs
 *     floor(0.85 / #out_i * 2^32); cross(b) sums those with min < b <= max;
 *   - boundary k lies in [t_k - w_k, t_k + w_k], w_k = min(ceil(n/K)/2,
 *     (t_k - t_{k-1} - 1)/2, (t_{k+1} - t_k - 1)/2), at least 0;
 *   - when a plan exists that way, no boundary b has min < b <= max for a
 *     tight cycle: a directed 2- or 3-cycle of distinct nodes whose
 *     out-degrees multiply to at most 2, spanning fewer than 2 ceil(n/K) ids;
 *   - the plan minimizes sum_k cross(b_k); among equal sums b_{K-1} is the
 *     smallest possible, then b_{K-2}, and so on.
 * Takes device temporaries of about 40 bytes per node; EINVAL if no plan is
 * found (cannot happen for valid input: the targets are feasible).
 * Synchronizes for CB_INOUT and MINCUT (temporary in-link prefix). */
int ditr_partition(ditr_ctx* ctx, int64_t n, int64_t nnz, const int32_t* d_col_ptr,
                   const int32_t* d_row_idx, int part_type, int64_t K, int64_t* d_ptr);
/* Partition of equal internal p mass (Section 2.3, the balance the paper
 * proposes as possibly better than CB) into d_ptr (device int64, K+1
 * boundaries, 1 <= K <= n). A link i -> t weighs floor(|p_ti| 2^32) integer
 * units (p_ti = damping / #out_i, or d_val[e] for a general matrix: one weight
 * per CSC entry, NULL for PageRank), so block masses are exact; the result is
 * the contiguous K-block partition whose largest internal mass t* is smallest,
 * each block taking from the left as many nodes as keep its mass <= t*
 * (trailing boundaries n if fewer blocks cover the nodes). Also the plan of
 * DITR_PART_PMASS. Synchronizes. */
int ditr_partition_pmass(ditr_ctx* ctx, int64_t n, int64_t nnz, const int32_t* d_col_ptr,
                         const int32_t* d_row_idx, const double* d_val, double damping, int64_t K,
                         int64_t* d_ptr);

/* ---- plain solve (steps: init, diffusion, transfer, residual, refresh) -- */
/* Exact residual F = B + P H - H (identity of equations defF and defH):
 * FP64 arithmetic, FP32 store into d_f [n]. If h_resid != NULL the FP64
 * ||F||_1 before rounding is returned there (synchronizes). */
int ditr_residual(ditr_ctx* ctx, const ditr_graph* g, const double* d_b, const double* d_h,
                  float* d_f, double* h_resid);

/* Diffuse until ||F||_1 <= rel_tol * ||B||_1 (checked on the exact FP64
 * residual). d_b FP64 [n] (finite), d_h FP64 [n], d_f FP32 [n].
 *   warm = 0: start from H = 0, F = B (d_h is overwritten).
 *   warm = 1: start from the H_0 held in d_h; F_0 = B + P H_0 - H_0
 *             (warm start and resume).
 *   warm = 2: start from the H_0 in d_h and the F_0 in d_f that the caller
 *             formed already (ditr_gnn_predict_h0 leaves both): one pass for
 *             the norms instead of a residual; the first stage ends with the
 *             exact residual of H, so the stop is certified even if the given
 *             F_0 was inexact.
 * On return d_h = H and d_f = the exact residual of H rounded to FP32.
 * Synchronizes. Returns DITR_OK, DITR_NOT_CONVERGED, DITR_ABORTED or an error;
 * `stats` (may be NULL) is filled in every case. */
int ditr_solve(ditr_ctx* ctx, const ditr_graph* g, const double* d_b, double* d_h, float* d_f,
               int warm, double rel_tol, const ditr_opts* opts, ditr_stats* stats);

/* The plain solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, result and guarantees as ditr_solve, but its per-solve
 * buffers (published shares, heavy-item words, per-workgroup sums, level
 * counters, the exact residual's work arrays; about 16 n bytes) live in one
 * static device array of the library, 64 MiB on every device it runs on, held
 * until the process ends (ditr_noalloc_scratch_bytes() gives the size). The
 * call performs no device or host allocation. The caller still passes B, H and
 * F, and the context and graph are created beforehand as usual.
 *   - DITR_MODE_AUTO / DITR_MODE_PARTITION only, without
 *     DITR_FLAG_TIME_KERNELS; anything else returns DITR_EINVAL.
 *   - A graph whose buffers exceed the static array returns DITR_EINVAL with
 *     the sizes in the message (roughly n > 4e6).
 *   - Every call on one device shares that device's array and finds the
 *     previous call's contents there (the call clears what must start at
 *     zero): calls that overlap on one device, from several threads or
 *     contexts, race and must be serialized by the caller.
 * Synchronizes. */
int ditr_solve_noalloc(ditr_ctx* ctx, const ditr_graph* g, const double* d_b, double* d_h,
                       float* d_f, int warm, double rel_tol, const ditr_opts* opts,
                       ditr_stats* stats);
size_t ditr_noalloc_scratch_bytes(void);

/* Per-partition trace of the partitioned sweep: the fluid r_k each partition
 * (PID) still holds and the fluid s_k it has sent to the others but they have
 * not yet taken in (the quantities of Section 2.4's PID model and of the fluid
 * plots of Section 3.1), its work, and its idle time waiting for the others'
 * exchange (the idle proportion of Section 3.3). Registers d_trace, a device
 * buffer the caller owns and keeps alive while tracing is on, of `capacity`
 * records of DITR_TRACE_FIELDS doubles each. NULL or capacity 0 switches
 * tracing off (the default).
 *
 * Level l of a solve (counted over its stages; stats.sweeps is the number of
 * levels) writes partition k's record at index l * K + k, if it is below
 * `capacity`. Records past it are dropped. Fields, in order:
 *   0 r_k: sum of |F_i| over the partition once the level's sweeps end;
 *   1 s_k: the |shares| the level published for targets outside the partition
 *          (received at the next level);
 *   2 node diffusions of the level;
 *   3 edge diffusions of the level;
 *   4 seconds spent waiting for the other partitions before the level
 *     (resident sweep; 0 when every level is its own launch);
 *   5 seconds from the end of that wait to the partition's arrival (its work).
 * For PageRank (nonnegative fluid), sum_k (r_k + s_k) at the last level of a
 * stage equals the exact ||B + P H - H||_1 that follows it, up to the FP32 and
 * fixed-point rounding of the moved fluid. Applies to DITR_MODE_PARTITION (and
 * AUTO when it picks it); other modes write nothing. */
#define DITR_TRACE_FIELDS 6
int ditr_set_trace(ditr_ctx* ctx, double* d_trace, int64_t capacity);

/* ---- batched personalized PageRank (step: many right-hand sides) -------- */
/* Diffuse nrhs right-hand sides at once (multiple of 4, 4..256), each to its
 * own exact FP64 residual <= rel_tol * ||B_r||_1 (personalization vectors V of
 * Section 2.2 in X = d Q X + (1-d) V). Node-major layouts with row stride nrhs:
 * d_b FP64 [n][nrhs] (read), d_h FP64 [n][nrhs] (out: H, starts from 0),
 * d_f FP32 [n][nrhs] (out: exact residual rounded to FP32). Every right-hand
 * side has its own threshold T_r; all share each in-link read. d_workspace
 * (device, ws_bytes >= ditr_workspace_bytes(.., nrhs, ..), owned by the
 * caller) holds the solve's buffers, about 12 nrhs n bytes; NULL lets the call
 * allocate and free them itself. per_rhs (nullable, [nrhs]) gets each
 * right-hand side's residual, ||B_r||_1 and diffused edges; total (nullable)
 * the sums and timing. Synchronizes. */
int ditr_solve_batched(ditr_ctx* ctx, const ditr_graph* g, int nrhs, const double* d_b,
                       double* d_h, float* d_f, double rel_tol, const ditr_opts* opts,
                       void* d_workspace, size_t ws_bytes, ditr_stats* per_rhs, ditr_stats* total);

/* ---- autotuner (step: partition size and threshold schedule) ----------- */
typedef struct {
  uint64_t key;            /* fingerprint of (CSC, damping, B, rel_tol, device) */
  int32_t from_cache;      /* 1: options read from the cache, nothing timed */
  int32_t candidates;      /* option sets timed */
  double default_seconds;  /* time to tolerance with ditr_opts_default (re-timed at the end) */
  double best_seconds;     /* time to tolerance with the returned options (same re-timing) */
  int64_t default_edges;   /* diffused edges of those two solves */
  int64_t best_edges;
  double seconds;          /* host wall time of the tuning call */
} ditr_tune_info;

/* Pick the options of the plain solve that reach rel_tol ||B||_1 fastest on
 * this problem: partition type and nodes per partition (Section 2.3), the
 * threshold divisor alpha in [1.2, 3] (Section 2.4 finds [1.2, 2]
 * uninfluential; on the GPU a larger one can pay), local sweeps per level
 * and the first exact-refresh point, by coordinate descent over wall time to
 * tolerance (effort 0: partition size and alpha; 1: also local sweeps and the
 * refresh point; 2: a second pass). The returned options are never slower than
 * the defaults at the final re-timing, else they are the defaults.
 * The CSC arrays follow ditr_graph_create; d_b FP64 [n] is the right-hand side
 * to tune for; d_h FP64 [n] and d_f FP32 [n] are work buffers (overwritten).
 * If cache_path != NULL the result is looked up there first, under the key
 * ditr_tune_key computes, and stored there afterwards (a JSON file rewritten
 * through a temporary file and a rename; concurrent writers may lose entries
 * but never corrupt it; an unreadable file counts as empty). Builds and
 * destroys its own graphs. Synchronizes. */
int ditr_tune(ditr_ctx* ctx, int64_t n, int64_t nnz, const int32_t* d_col_ptr,
              const int32_t* d_row_idx, double damping, const double* d_b, double* d_h, float* d_f,
              double rel_tol, int effort, const char* cache_path, ditr_opts* out,
              ditr_tune_info* info);
/* Pick the options of the batched solve (ditr_solve_batched) that reach
 * rel_tol ||B_r||_1 for every right-hand side fastest on this graph and these
 * right-hand sides: the threshold divisor alpha of every right-hand side's
 * schedule (Section 2.4; candidates 1.25, 1.5, 2, 3, 4) and, with effort >= 1,
 * the first exact-refresh point (1e-5, 1e-6, 1e-7), by coordinate search over
 * wall time (effort 2: a second pass). The batched sweep has no partition plan,
 * so these are its schedule knobs. Arguments as ditr_solve_batched: d_b [n][nrhs]
 * is read, d_h and d_f are work buffers (overwritten), the workspace is the
 * caller's (NULL and 0: the library allocates per call). The returned options
 * are never slower than the defaults at the final re-timing, else they are the
 * defaults; info (may be NULL) gets the timings. No cache. Synchronizes. */
int ditr_tune_batched(ditr_ctx* ctx, const ditr_graph* g, int nrhs, const double* d_b, double* d_h,
                      float* d_f, double rel_tol, void* d_workspace, size_t ws_bytes, int effort,
                      ditr_opts* out, ditr_tune_info* info);
/* The cache key of a problem: a position-aware hash of col_ptr, row_idx and B
 * computed on the device, combined with n, nnz, damping, rel_tol and the
 * device's architecture name and CU count. Synchronizes. */
int ditr_tune_key(ditr_ctx* ctx, int64_t n, int64_t nnz, const int32_t* d_col_ptr,
                  const int32_t* d_row_idx, double damping, const double* d_b, double rel_tol,
                  uint64_t* key);
/* Host-only access to a tuning cache file. get: copies the tuned fields
 * (alpha, refresh_at, part_type, part_nodes, sweeps_per_claim) of the entry
 * under `key` into *out and leaves the others; DITR_NOT_FOUND if the file is
 * missing, not a cache, or has no such entry. put: adds or replaces that
 * entry; DITR_EINVAL for options out of range or a file that cannot be
 * written. */
int ditr_tune_cache_get(const char* path, uint64_t key, ditr_opts* out);
int ditr_tune_cache_put(const char* path, uint64_t key, const ditr_opts* o, double seconds,
                        double default_seconds);

/* ---- learned warm start (step: network, training, predicted H_0) ------- */
/* A two-layer message-passing network over P predicts y_i = log(N x_i / ||B||_1)
 * of the solution x of X = P X + B (Section 1) for uniform B; its prediction gives a
 * start H_0 whose exact fluid F_0 = B + P H_0 - H_0 (identity of equations
 * defF and defH) is all the D-iteration then diffuses (ditr_solve, warm = 1).
 *   features X_i = [log1p #in_i, log1p #out_i, [#out_i = 0], 1,
 *                   u_k = ((s >> 16k) & 0xffff) / 32768 - 1, k = 0..3],
 *                  s = SplitMix64 output for state i / block
 *   h1 = relu(X W1s + (P X) W1n + b1),  h2 = relu(h1 W2s + (P h1) W2n + b2)
 *   z = h2 w3 + b3, yhat = log(softplus(z));  training loss sum_i w_i (yhat_i - y_i)^2
 * BF16 weights and activations (round to nearest even), FP32 accumulation,
 * FP32 master weights, FP32 gradients, Adam (beta 0.9, 0.999, eps 1e-8).
 * Parameters are exchanged as one FP32 vector in this order, matrices
 * [input][output] row-major: W1s [8][64], W1n [8][64], b1 [64], W2s [64][64],
 * W2n [64][64], b2 [64], w3 [64], b3 [1]. The network holds device buffers
 * for the largest graph it has seen (about 900 bytes per node when training).
 * A network is used with graphs of the context it was created on. */
typedef struct ditr_gnn ditr_gnn;
#define DITR_GNN_PARAMS 9409
enum { DITR_GNN_ACT_X = 0,   /* features, BF16 [n][16] (8 used, 8 zero) */
       DITR_GNN_ACT_PX = 1,  /* P X, BF16 [n][16] */
       DITR_GNN_ACT_H1 = 2,  /* BF16 [n][64] */
       DITR_GNN_ACT_PH1 = 3, /* P h1, BF16 [n][64] */
       DITR_GNN_ACT_H2 = 4   /* BF16 [n][64] */ };

typedef struct {
  double b_l1;      /* ||B||_1 */
  double scale_c;   /* scale applied to xhat (0: cold start) */
  double f0_l1;     /* exact ||F_0||_1 of the returned H_0 (FP64) */
  int32_t fell_back;/* 1: H_0 = 0 (no scaled start leaves less L1 fluid than B) */
  int32_t pad;
  double seconds;   /* host wall time of the call */
} ditr_gnn_start;

/* hidden must be 64; block is the id-block size of the code features; seed
 * draws He-normal initial weights (SplitMix64, Box-Muller), zero biases, and a
 * head that starts near z = 1 (w3 scaled by 0.1, b3 = 1). */
int ditr_gnn_create(ditr_ctx* ctx, ditr_gnn** out, int hidden, int block, uint64_t seed);
int ditr_gnn_destroy(ditr_gnn* net);
/* h_theta: host FP32 [DITR_GNN_PARAMS]. set also clears the Adam state.
 * Synchronize. DITR_ENONFINITE for a NaN or Inf parameter. */
int ditr_gnn_get_params(ditr_gnn* net, float* h_theta);
int ditr_gnn_set_params(ditr_gnn* net, const float* h_theta);
/* yhat of every node of g into d_yhat (device FP32 [n], may be NULL). */
int ditr_gnn_forward(ditr_ctx* ctx, ditr_gnn* net, const ditr_graph* g, float* d_yhat);
/* Copy an activation of the last forward pass (DITR_GNN_ACT_*) for n nodes. */
int ditr_gnn_activation(ditr_ctx* ctx, const ditr_gnn* net, int which, int64_t n, uint16_t* d_out);
/* Training targets from a solved H (device FP64 [n]) of a right-hand side with
 * ||B||_1 = b_l1: y_i = log(N H_i / b_l1) and w_i = H_i / sum H (zero where
 * H_i <= 0). d_y, d_w: device FP32 [n].
 * Synchronizes. */
int ditr_gnn_targets(ditr_ctx* ctx, const ditr_graph* g, const double* d_h, double b_l1, float* d_y,
                     float* d_w);
/* Loss and its gradient at the current weights (forward + backward on g).
 * d_grad: device FP32 [DITR_GNN_PARAMS] (may be NULL); h_loss (may be NULL,
 * synchronizes). */
int ditr_gnn_grad(ditr_ctx* ctx, ditr_gnn* net, const ditr_graph* g, const float* d_y,
                  const float* d_w, float* d_grad, double* h_loss);
/* One Adam step with learning rate lr on the gradient of g's loss; h_loss gets
 * the loss before the step (may be NULL, synchronizes). */
int ditr_gnn_train_step(ditr_ctx* ctx, ditr_gnn* net, const ditr_graph* g, const float* d_y,
                        const float* d_w, double lr, double* h_loss);
/* Warm start for right-hand side d_b (device FP64 [n]): xhat = exp(yhat)
 * ||B||_1 / N, H_0 = c xhat into d_h0 (device FP64 [n]) with c the first of
 * {0, 0.50, 0.55, ..., 1.50} that minimizes the L1 fluid ||B + c (P - I) xhat||_1
 * of the start (evaluated from the FP32 residual); d_f0 (device FP32 [n]) gets
 * the start's fluid B + c (F - B), F = B + (P - I) xhat in FP64 rounded to FP32
 * (equal to B + P H_0 - H_0 up to that rounding). c = 0 is the cold start
 * H_0 = 0, F_0 = B (info->fell_back = 1), so the start never holds more fluid
 * than B. Then ditr_solve(..., warm = 2, ...) diffuses from (H_0, F_0), or
 * warm = 1 re-forms F_0 exactly. Synchronizes. */
int ditr_gnn_predict_h0(ditr_ctx* ctx, ditr_gnn* net, const ditr_graph* g, const double* d_b,
                        double* d_h0, float* d_f0, ditr_gnn_start* info);

#ifdef __cplusplus
}
#endif
#endif /* DITR_H */
