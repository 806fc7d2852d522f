/*
 * dt.h -- C ABI of the MI355X Delaunay triangulation library (libdt.so).
 *
 * The library computes DT(P), the Delaunay triangulation of a point set
 * P in R^D (D = 2 or 3), with the divide-and-conquer method of Funke,
 * Sanders and Winkler, "Load-Balancing for Parallel Delaunay
 * Triangulations": Algorithm 1 (partition, triangulate the partitions,
 * find the border simplices, triangulate their vertices, merge by hash
 * lookup) with the sample-based divide step of Algorithm 2 (triangulate a
 * random sample, partition its Delaunay graph into k blocks, give every
 * point the block of its nearest sample point).
 *
 * Result: the set of finite simplices of DT(P), each a row of D+1 input
 * indices (0-based, ascending within the row).  The paper defines DT(P) for
 * points in general position (Section "Delaunay Triangulations"); ties are
 * broken by a symbolic perturbation of the paraboloid lifting in which a
 * point with a smaller index has a larger height perturbation.  The result
 * therefore depends only on the points, never on k, the divide, the sample
 * or the execution order.
 *
 * Conventions shared by every entry point:
 *   - points are row-major n x D doubles; the caller owns them and the
 *     library never frees or modifies them.  `points_on_device` = 1 means a
 *     HIP device pointer, 0 a host pointer (then the call copies it).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     ordered on it; calls that return results synchronise it.
 *   - every call returns a status (DT_OK = 0, negative on error) and never
 *     aborts.  Results are opaque handles owning device memory until
 *     dt_result_free.
 *   - threads: calls on different results, streams or servers may run
 *     concurrently from several host threads.  One result must not be used
 *     by two calls at once.  The library keeps two process-wide caches,
 *     each behind its own lock:
 *       * device blocks of 16 MB and more that calls release (at most
 *         48 GB, see dt_release_cached_memory).  A block released during a
 *         call carries an event recorded on that call's stream; the next
 *         call that takes it makes its own stream wait for that event, so
 *         a release never waits for other streams.  Blocks of a result freed
 *         by dt_result_free are idle (every call that touches a result
 *         synchronises its stream before returning);
 *       * the launch tunables chosen by dt_batch_autotune, per size class.
 */
#ifndef DT_MI355X_H
#define DT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
  DT_OK = 0,
  DT_E_INVALID_ARG = -1, /* bad D, k, sample rate, sizes or pointers          */
  DT_E_NONFINITE = -2,   /* a coordinate is NaN or infinite                  */
  DT_E_DUPLICATE = -3,   /* two points are identical (P must be a set)       */
  DT_E_DEGENERATE = -4,  /* n < D+1, or all points in one hyperplane         */
  DT_E_NOMEM = -5,       /* device allocation failed / budget exceeded       */
  DT_E_DEVICE = -6,      /* a HIP runtime call failed                        */
  DT_E_INTERNAL = -7,    /* a device invariant failed (see dt_stats.fail)    */
  DT_E_NOT_READY = -8    /* serving: the job has not finished yet            */
};

/* ---------------------------------------------------------------- options */
/* DT_DIVIDE_AUTO draws the sample, then takes the kd divide when the
 * sample looks evenly spread (coefficient of variation of its counts over a
 * grid of about eta/4 cells at most DT_AUTO_CV) and k is a power of two,
 * else the sample divide; dt_stats.divide_used tells which. */
enum { DT_DIVIDE_SAMPLE = 0, DT_DIVIDE_KD = 1, DT_DIVIDE_AUTO = 2 };
#define DT_AUTO_CV 1.0
/* Edge weights of the sample graph, paper Table "weights":
 * d = |v-w| / d*, d* = length of the bounding-box diagonal. */
enum { DT_WEIGHT_LOG = 0, DT_WEIGHT_CONST = 1, DT_WEIGHT_INVERSE = 2, DT_WEIGHT_LINEAR = 3 };
/* Predicate precision: FP64 filter -> exact, or FP32 filter -> FP64 -> exact. */
enum { DT_PREC_FP64 = 0, DT_PREC_FP32 = 1 };
/* Border primitive (Algorithm 1, intersection test; Section "Geometric
 * Primitives"): the exact regions of the divide (sample Voronoi cells / kd
 * boxes); the paper's grid test (cells of edge grid_cell * (V/n)^(1/D)
 * occupied by another partition); the bounding-box test (the ball meets
 * another partition's bounding box); the exact test (a point of another
 * partition lies inside the circumsphere, decided with the exact perturbed
 * in-sphere predicate on the points of the grid cells the ball covers). */
enum { DT_BORDER_REGION = 0, DT_BORDER_GRID = 1, DT_BORDER_BBOX = 2, DT_BORDER_EXACT = 3,
       DT_BORDER_REFINED = 4 /* the region test, then the exact test on its hits */ };

typedef struct dt_options {
  int divide;        /* DT_DIVIDE_SAMPLE (Algorithm 2) or DT_DIVIDE_KD (cyclic median) */
  int weight;        /* DT_WEIGHT_*                                                   */
  int precision;     /* DT_PREC_*                                                     */
  int sort_output;   /* 1: rows in lexicographic order (canonical form)               */
  double eps;        /* partition imbalance: |V_i| <= (1+eps) ceil(|V|/k); default 0.05 */
  double grid_cell;  /* c_G of the grid-based border test; default 1                  */
  uint64_t seed;     /* sample seed; default 1                                        */
  int refine_iters;  /* label-propagation sweeps of the partitioner; default 16       */
  int keep_stages;   /* 1: keep per-stage arrays for dt_result_stage                  */
  int border;        /* DT_BORDER_*; default DT_BORDER_REGION                         */
  int profile;       /* 1: time the kernels below with HIP events (dt_stats.kern_*)   */
  /* Launch tunables of the parallel insertion (0 = default; dt_batch_autotune
   * picks them for a batch).  They change timing only, never the result. */
  int start_active;  /* points per set active in the first level; default 256       */
  int grow_div;      /* next level starts when pending < inserted/grow_div; default 64 */
  int cand_blocks;   /* cap on wavefronts of the cavity/insert launches; default 32768 */
  int grow_num;      /* growth of the threshold per level, in eighths (9..32, i.e.
                        x1.125..x4); default 10 for several sets, 12 for one set   */
  /* 1: recursive bisection (Section "Recursive Bisection"): log2 k levels of
   * 2-way division with the chosen divide (kd: cyclic median split; sample:
   * per block and level a new sample, its DT, a 2-way partition of its
   * graph and nearest-sample assignment), then k-1 merges bottom-up, whose
   * border test is the region test of the divide (DT_BORDER_GRID selects
   * the grid test); k must be a power of two.
   * 0 (default): one k-way division and one merge (Algorithm 1). */
  int recursive;
  /* Gift wrapping where it pays (timing only; the simplices are the same):
   * 0 (default) gift-wraps the sample of the sample divide when it has at
   * most 65,536 points, starts every single set of at least 65,536 points
   * (the border set, a direct triangulation) from the gift-wrapped
   * triangulation of its first 4096 or so points in insertion order, and
   * starts every set of at least 8192 points of a batched run (the blocks
   * of a divide, a batch) from a gift-wrapped seed of up to 1024 of its
   * first points; -1 inserts every point in parallel rounds.  A run in a
   * caller's workspace (dt_triangulate_noalloc) wraps nothing. */
  int gift_wrap;
  /* Pair exchanges in the partitioner's sweeps: 0 (default) lets a vertex
   * whose best block is full swap with a vertex of that block that wants
   * its block, when the exchange lowers the cut (block sizes unchanged);
   * -1 moves vertices into free room only.  The result does not depend on
   * it, the blocks and the border do. */
  int refine_swaps;
} dt_options;

/* Kernels timed when dt_options.profile = 1. */
enum { DT_KERN_K4_PICK = 0, DT_KERN_K4_CAVITY, DT_KERN_K4_INSERT, DT_KERN_ASSIGN,
       DT_KERN_BUCKET, DT_KERN_BORDER, DT_KERN_MERGE, DT_KERN_K4_SELECT, DT_NUM_KERN = 8 };

/* -------------------------------------------------------------- statistics */
enum {
  DT_STAGE_VALIDATE = 0, DT_STAGE_SAMPLE, DT_STAGE_SAMPLE_DT, DT_STAGE_PARTITION,
  DT_STAGE_ASSIGN, DT_STAGE_SCATTER, DT_STAGE_LOCAL_DT, DT_STAGE_BORDER,
  DT_STAGE_BORDER_DT, DT_STAGE_MERGE, DT_STAGE_OUTPUT, DT_STAGE_TOTAL, DT_NUM_STAGES
};

typedef struct dt_stats {
  int64_t n, eta, num_simplices;
  int64_t border_simplices;   /* |B|: flagged simplices of the T_i (finite)        */
  int64_t border_vertices;    /* |vertices(B)|, the border point set              */
  int64_t tb_simplices;       /* finite simplices of T_B                          */
  int64_t local_simplices;    /* finite simplices of all T_i                      */
  int32_t k, D;
  double cv;                  /* coefficient of variation of partition sizes      */
  double max_dev;             /* max_i p_i/(n/k) - 1                              */
  double o_dt;                /* (n + eta + |vertices(B)|) / n                     */
  double cut_weight;          /* weight of sample-graph edges between blocks      */
  int64_t max_part, min_part; /* largest / smallest partition                      */
  int64_t rounds;             /* insertion rounds of all local-DT launches         */
  int64_t pred[4][4];         /* [orient2D, orient3D, insphere2D, insphere3D] x
                                 [calls, decided by FP32, by FP64, by exact]      */
  uint32_t fail;              /* device failure bits when status is DT_E_INTERNAL */
  uint32_t pad;
  double stage_ms[DT_NUM_STAGES];
  int64_t probe_hist[16];     /* merge hash: lookups by probe count (last = 15+)  */
  double kern_ms[DT_NUM_KERN];        /* summed HIP-event time per kernel (profile)  */
  int64_t kern_launches[DT_NUM_KERN]; /* launches per kernel (profile)               */
  int64_t cavity_cells;       /* cells visited by winning and losing cavity searches */
  int64_t candidates;         /* cavity searches (winning and losing) over all rounds   */
  int64_t divide_used;        /* DT_DIVIDE_SAMPLE or DT_DIVIDE_KD                        */
  double divide_stat;         /* DT_DIVIDE_AUTO: the sample's grid-count variation       */
  int64_t large_cavities;     /* insertion rounds in which one cavity outgrew the
                                 per-candidate lists and used a pool-sized list   */
  int64_t wrap_levels;        /* facet levels of the gift-wrapped sample
                                 triangulation (0: parallel insertion)           */
  int64_t seeded_sets;        /* single sets started from a gift-wrapped seed     */
} dt_stats;

typedef struct dt_result dt_result;

/* Default options (sample divide, log weights, FP64+exact, eps 0.05, c_G 1,
 * seed 1, 16 refinement sweeps, unsorted output, no stage arrays). */
void dt_default_options(dt_options* opt);

/* Human-readable name of a status code. */
const char* dt_strerror(int status);

/*
 * dt_triangulate -- DT(P) by Algorithm 1 with the divide selected in opt.
 *   points      n x D doubles (see conventions)
 *   n, D        number of points (n >= D+1), dimension (2 or 3)
 *   k           number of partitions (1 <= k <= eta for the sample divide;
 *               a power of two for the kd divide); k = 1 triangulates
 *               the whole set directly
 *   sample_rate eta = round(sample_rate * n), at least D+2; 0 selects the
 *               paper's default sqrt(n) (Algorithm 2, Section "Sample Size")
 *   opt         NULL for defaults
 *   out         receives a result handle on DT_OK (else NULL)
 * Errors: DT_E_INVALID_ARG, DT_E_NONFINITE, DT_E_DUPLICATE,
 *         DT_E_DEGENERATE, DT_E_NOMEM, DT_E_DEVICE, DT_E_INTERNAL.
 */
int dt_triangulate(const double* points, int64_t n, int D, int k, double sample_rate,
                   const dt_options* opt, int points_on_device, void* stream,
                   dt_result** out);

/*
 * dt_release_cached_memory -- return to the driver the device blocks that
 * the library keeps between calls.  Large scratch and result buffers (16 MB
 * and more) are not freed when a call ends but kept, at most 48 GB per
 * process, and handed to later calls of about the same size.  This waits for
 * every device that holds such blocks and frees them.  Blocks in use by
 * results or by calls running on other threads are not affected; they join
 * the cache when released.  Returns DT_OK, or DT_E_DEVICE if a device call
 * fails (the remaining blocks are still freed).
 */
int dt_release_cached_memory(void);

/* Number of simplices in a result (all sets for batch results). */
int64_t dt_result_count(const dt_result* r);
/* Dimension D of a result. */
int dt_result_dim(const dt_result* r);
/* Copy the m x (D+1) int32 simplex rows to dst (device or host memory,
 * capacity `cap_rows` rows).  Returns DT_OK or DT_E_INVALID_ARG. */
int dt_result_copy(const dt_result* r, int32_t* dst, int64_t cap_rows, int dst_on_device,
                   void* stream);
/* Neighbours (Algorithm 1, neighbourhood update): m x (D+1) int32 to dst
 * (device or host memory, capacity cap_rows rows); entry (i, j) is the row
 * of the simplex that shares the facet of row i opposite its j-th vertex
 * (rows as dt_result_copy returns them), or -1 on the convex hull.  For a
 * batch result, rows of different sets are never neighbours.  Computed on
 * the device at the first call and kept with the result (not safe to call
 * concurrently on one result).  DT_OK, DT_E_INVALID_ARG, DT_E_NOMEM,
 * DT_E_DEVICE. */
int dt_result_neighbors(const dt_result* r, int32_t* dst, int64_t cap_rows, int dst_on_device,
                        void* stream);
/* Statistics of the run that produced r. */
int dt_result_stats(const dt_result* r, dt_stats* st);
void dt_result_free(dt_result* r);

/*
 * Per-stage arrays (only when opt.keep_stages = 1), copied to host memory:
 *   DT_ARR_SAMPLE    int64[eta]  sample point indices, ascending
 *   DT_ARR_SAMPLE_DT int32[m_s x (D+1)] finite simplices of DT(sample), as
 *                    input indices
 *   DT_ARR_PART      int32[eta]  block of every sample point
 *   DT_ARR_PID       int32[n]    partition of every point
 *   DT_ARR_ORDER     int32[n]    bucketed order: input index of each slot
 *   DT_ARR_BORDER_V  int32[|V_B|] border vertices, ascending
 *   DT_ARR_LOCAL     int32[m_l x (D+2)] finite simplices of all T_i as
 *                    input indices plus a last column: 1 if in B
 *   DT_ARR_BORDER_DT int32[m_b x (D+1)] finite simplices of T_B
 *   DT_ARR_NEAREST   int32[n]    nearest sample of every point (index into
 *                    DT_ARR_SAMPLE; sample divide only)
 *   DT_ARR_GRAPH     int32[e x 2] edges of the sample's Delaunay graph
 *                    (Algorithm 2), input indices u < v, rows ascending
 *                    (sample divide only)
 *   DT_ARR_WEIGHTS   double[e]   weight of each DT_ARR_GRAPH edge (Table
 *                    "weights", with the chosen dt_options.weight)
 * `count` receives the number of elements (rows x columns); pass dst = NULL
 * to query it.
 */
enum { DT_ARR_SAMPLE = 0, DT_ARR_SAMPLE_DT, DT_ARR_PART, DT_ARR_PID, DT_ARR_ORDER,
       DT_ARR_BORDER_V, DT_ARR_LOCAL, DT_ARR_BORDER_DT, DT_ARR_NEAREST, DT_ARR_GRAPH,
       DT_ARR_WEIGHTS, DT_NUM_ARR };
int dt_result_stage(const dt_result* r, int which, void* dst, int64_t cap, int64_t* count);

/*
 * dt_triangulate_noalloc -- dt_triangulate with k = 1 (the parallel
 * triangulation of the whole set, without a divide) for callers that
 * cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  The call allocates
 * nothing (no hipMalloc, hipFree, pinned host memory or library
 * allocation): its scratch memory is one static device array of
 * DT_NOALLOC_SCRATCH_BYTES per GPU, held by each GPU the library runs this
 * call on until the process ends.  The array keeps the contents of the
 * last call; the call clears what must start at zero.  Calls on one GPU
 * share the array: within a process they are serialised by a lock (one
 * call at a time per device), and the call synchronises `stream` before it
 * returns.
 *   points   device memory, n x D row-major doubles (caller-owned)
 *   n        D+1 <= n <= DT_NOALLOC_MAX_POINTS_2D / _3D
 *   opt      NULL for defaults; precision and the launch tunables apply,
 *            sort_output must be 0, the divide options are unused
 *   rows     device memory, cap_rows x (D+1) int32: the finite simplices
 *            of DT(P) as rows of input indices, ascending within a row
 *            (row order unspecified)
 *   count    receives the number of simplices m (also when cap_rows < m)
 * Errors: DT_E_INVALID_ARG (bad D or pointers, sort_output set, or
 * cap_rows < m: *count then says how many rows are needed),
 * DT_E_NOMEM (n above the maximum for D: the job does not fit the
 * scratch array), DT_E_NONFINITE, DT_E_DUPLICATE, DT_E_DEGENERATE,
 * DT_E_DEVICE, DT_E_INTERNAL.
 */
#define DT_NOALLOC_SCRATCH_BYTES (256u << 20)
#define DT_NOALLOC_MAX_POINTS_2D 131072
#define DT_NOALLOC_MAX_POINTS_3D 49152
int dt_triangulate_noalloc(const double* points, int64_t n, int D, const dt_options* opt,
                           int32_t* rows, int64_t cap_rows, int64_t* count, void* stream);

/*
 * dt_predicates -- the two geometric predicates that decide every
 * combinatorial step of the method (Section "Geometric Primitives"; the
 * triangulations rely on exact orientation and in-sphere tests), on a batch
 * of point tuples, evaluated on the device by the same chain of filters the
 * triangulation uses: with DT_PREC_FP32 an FP32 filter, then an FP64 filter,
 * then exact expansion arithmetic; with DT_PREC_FP64 the last two.  Each
 * filter certifies a sign only above its a-priori rounding bound, so the
 * answer is always the exact sign.
 *   kind   DT_PRED_ORIENT:   sign of Orient1(p_0..p_D) = det[p_i 1] (may be 0);
 *          DT_PRED_INSPHERE: sign of In(p_0..p_D, q) =
 *                            det[p_i |p_i|^2 1; q |q|^2 1] under the symbolic
 *                            perturbation of the lifting by `keys` (a
 *                            smaller key perturbs more); positive means q
 *                            is inside the circumsphere of a positively
 *                            oriented p_0..p_D.  Never 0 unless p_0..p_D
 *                            and q are all on one hyperplane.
 *   D      2 or 3
 *   pts    device memory, nq tuples of np = D+1 (orient) or D+2 (in-sphere,
 *          q last) points, row-major doubles: coordinate a of point i of
 *          tuple t at pts[(t*np + i)*D + a]; coordinates must be finite
 *   keys   device memory, nq x np int64 perturbation keys (in-sphere only;
 *          NULL = the position 0..np-1 inside the tuple); unused for orient
 *   sign   device memory, nq int8 results (-1, 0, 1)
 *   stage  device memory or NULL, nq int8: 0 decided by the FP32 filter,
 *          1 by the FP64 filter, 2 by the exact stage
 * The caller owns every buffer.  Synchronises `stream`.  DT_OK,
 * DT_E_INVALID_ARG (kind, D, precision, nq < 0, NULL pointers),
 * DT_E_INTERNAL (exact-stage capacity exceeded; results invalid),
 * DT_E_DEVICE, DT_E_NOMEM.
 */
enum { DT_PRED_ORIENT = 0, DT_PRED_INSPHERE = 1 };
int dt_predicates(int kind, int D, int precision, const double* pts, const int64_t* keys,
                  int64_t nq, int8_t* sign, int8_t* stage, void* stream);

/*
 * dt_batch_triangulate -- DT of many independent point sets in one batched
 * run (all sets share every kernel launch).  Set s holds rows
 * offsets[s] .. offsets[s+1]-1 of `points` (offsets: num_sets+1 int64,
 * host memory, offsets[0] = 0).  ids (nullable, n int64, host memory): the
 * label of every point, used both as output label and as the tie-break
 * order; NULL means the row index.  Output rows of set s follow those of
 * set s-1; dt_result_set_offsets gives the row ranges.  A set with fewer
 * than D+1 points or lying in one hyperplane yields no simplices and is
 * counted in dt_stats.fail-free field `min_part` = -1 (status stays DT_OK).
 */
int dt_batch_triangulate(const double* points, const int64_t* ids, const int64_t* offsets,
                         int64_t num_sets, int D, const dt_options* opt,
                         int points_on_device, void* stream, dt_result** out);
/* Row offsets (num_sets+1 int64, host) of the sets in a batch result. */
int dt_result_set_offsets(const dt_result* r, int64_t* dst, int64_t cap);

/*
 * dt_batch_autotune -- pick the launch tunables (dt_options.start_active,
 * grow_div, cand_blocks) for batches like this one.  Times batched runs on
 * every s-th set (about sample_points points in all; <= 0 means 4 Mi),
 * changing one tunable at a time from the defaults (a trial is the faster
 * of two runs; a change must gain 3 %); a result other than the defaults
 * is kept only if it is also 2 % faster on the whole batch.  Writes opt
 * (NULL = defaults) with the chosen tunables into *tuned.  The choice is cached
 * per (D, precision, log2 mean set size, log2 set count) for the life of
 * the process; a cached class returns at once.  points / offsets /
 * points_on_device / stream as for dt_batch_triangulate.  The tunables
 * never change a triangulation, only its time.
 */
int dt_batch_autotune(const double* points, const int64_t* offsets, int64_t num_sets, int D,
                      const dt_options* opt, int points_on_device, void* stream,
                      int64_t sample_points, dt_options* tuned);

/*
 * Serving (continuous batching; the paper's method applied to a stream of
 * independent requests).  A server owns a device-memory budget and two
 * worker threads, each with its own stream.  A job's points are copied to
 * device memory at submission and stay there until the job is done (the
 * queue lives on the device; these copies are outside the budget).  Jobs
 * are admitted in arrival order while their estimated footprint fits the
 * budget (a job alone may use the whole budget).  A worker takes the
 * admitted jobs that have not started: consecutive jobs of one dimension
 * with at most 2 Mi points each run together as one batched run of
 * independent sets (as dt_batch_triangulate, up to 32 Mi points; the k of
 * such a job is not used, since the result does not depend on it), a
 * larger job runs alone with its k-way divide-and-conquer; the workers'
 * runs overlap on the device.  Each job's result (rows labelled by row index, sorted
 * when opt.sort_output) is identical to dt_triangulate on its own; if a
 * batched run fails its jobs run again one by one, so each gets its own
 * status.  Statistics of a batched job are those of its batch (n, k,
 * num_simplices and part sizes are the job's own).
 *   dt_server_create:  hbm_budget_bytes > 0; opt NULL for defaults
 *                      (profile and keep_stages are ignored).
 *   dt_server_submit:  points (n x D row-major doubles, host or device
 *                      memory per points_on_device) are copied before it
 *                      returns; returns a ticket.  DT_E_INVALID_ARG for bad
 *                      arguments, DT_E_DEGENERATE when n < D+1, DT_E_NOMEM
 *                      when the job's estimate exceeds the whole budget.
 *   dt_server_poll:    DT_E_NOT_READY before the job is done; then its
 *                      status, with *out set (owned by the caller) on DT_OK.
 *                      A result is handed out once; later calls give DT_OK
 *                      with *out = NULL.  DT_E_INVALID_ARG: unknown ticket.
 *   dt_server_wait:    as poll, but blocks until the job is done.
 *   dt_server_destroy: finishes all submitted jobs, joins the workers,
 *                      frees every result not handed out and returns the
 *                      workers' cached scratch memory to the device.
 * A finished job keeps a small record (status, timestamps) until the
 * server is destroyed.  Submitted device points must be ready: the copy
 * runs on the default stream.
 */
typedef struct dt_server dt_server;
int dt_server_create(size_t hbm_budget_bytes, const dt_options* opt, dt_server** srv);
int dt_server_submit(dt_server* srv, const double* points, int64_t n, int D, int k,
                     double sample_rate, int points_on_device, uint64_t* ticket);
int dt_server_poll(dt_server* srv, uint64_t ticket, dt_result** out);
int dt_server_wait(dt_server* srv, uint64_t ticket, dt_result** out);
/* Timestamps (seconds on the server's monotonic clock) of a finished job:
 * t[0] submission, t[1] admission, t[2] completion. */
int dt_server_times(dt_server* srv, uint64_t ticket, double t[3]);
void dt_server_destroy(dt_server* srv);

#ifdef __cplusplus
}
#endif
#endif
