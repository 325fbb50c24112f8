/*
 * ccd.h - C ABI of the MI355X (gfx950) inclusion-based continuous collision
 * detection library.
 *
 * The library decides, for each vertex-face (VF) or edge-edge (EE) pair whose
 * vertices move linearly over t in [0, 1], whether and when the pair touches,
 * with the root finder of Wang, Ferguson, Schneider, Jiang, Attene and Panozzo,
 * "A Large Scale Benchmark and an Inclusion-Based Algorithm for Continuous
 * Collision Detection" (ACM TOG 40(5), 2021):
 *
 *   - the problem is a root of F_vf or F_ee on Omega (Sec. 3, eqs. F-vf, F-ee);
 *   - a box I of the (t, u, v) domain is tested with the axis-aligned box of F
 *     at the 8 corners of I (Sec. 5.2, eq. box) against the floating-point
 *     filter eps_c = K gamma_c^3 (Sec. 5.2, eq. ccd-error);
 *   - boxes are bisected breadth first, level by level, along the axis with
 *     the largest estimated co-domain extent (Alg. 2, SPLIT; eq. kappas) until
 *     the first colliding box of a level is smaller than delta or inside the
 *     filter cube, or until m_I boxes have been checked (Alg. 2);
 *   - with a minimum separation d > 0 the box is enlarged by d and the filter
 *     constants change (Sec. 6.1, eq. msccd-error); distances are L-infinity.
 *
 * All arithmetic is IEEE binary64 with no contraction; results are bit-for-bit
 * reproducible and independent of batch composition, launch shape and tuning.
 *
 * Conventions
 *   - Functions return CCD_OK (0) or a negative CCD_E* code; nothing throws.
 *   - Query coordinates: 8 points x 3 coordinates.  Points 0..3 are at t = 0,
 *     points 4..7 are the same vertices at t = 1.  VF: p, v1, v2, v3.
 *     EE: p1, p2 (edge A) and p3, p4 (edge B).
 *   - A query is invalid if a coordinate is not finite or exceeds 1e300 in
 *     magnitude, delta is not a positive finite number, max_iter < 1, min_sep is
 *     negative or not finite, min_sep is not below min_c gamma_c (Sec. 6.1
 *     assumes d < gamma).  A batch is rejected (CCD_EINVAL) when t_max is not
 *     in (0, 1].
 *   - Output convention (Alg. 2): hit = (toi <= 1); no collision is
 *     toi = +inf, t_width = 0.  toi is a conservative (never late) estimate of
 *     the earliest contact time; t_width is w(I_t) of the level it came from.
 *   - Shortened time interval (Sec. 7.2, line search: only the initial interval
 *     of Alg. 2 changes): with t_max < 1 the search covers t in [0, t_max].  The
 *     time axis is bisected in s = t / t_max and a box's time endpoints are
 *     fl(t_max * s); toi is such an endpoint and t_width = t_max * 2^-depth.
 *     kappa_t keeps eq. kappas (F at t = 0 and t = 1), and the split rule uses
 *     w(I_t) = t_max * 2^-depth.  t_max = 1 is the standard query.
 */
#ifndef CCD_H
#define CCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define CCD_OK 0
#define CCD_EINVAL (-1)     /* invalid argument or query; outputs untouched */
#define CCD_ENOMEM (-2)     /* device memory budget too small for the request */
#define CCD_EDEVICE (-3)    /* HIP runtime error or missing gfx950 device */
#define CCD_EAGAIN (-4)     /* serving: request does not fit right now */
#define CCD_ETIMEDOUT (-5)  /* serving: wait timed out */
#define CCD_ECANCELED (-6)  /* serving: request cancelled / server closed */

/* Query kinds. */
#define CCD_KIND_VF 0
#define CCD_KIND_EE 1

/* Per-query status bits. */
#define CCD_ST_CAP 0x01     /* returned because m_I checks were reached (Alg. 2) */
#define CCD_ST_CARRY 0x02   /* returned a remembered terminal box (see CCD_FLAG_LITERAL) */
#define CCD_ST_DEPTH 0x04   /* returned box was terminal only because a split would
                               go below 2^-52 on its axis */
#define CCD_ST_OVERFLOW 0x08 /* the next level of the query's frontier did not fit the
                               scratch the library could give it (the block engine's
                               arena, see ccd_tuning.block_capacity): the query returned
                               at the first colliding box of its current level, as Alg. 2
                               does at the m_I stop, so toi is still conservative (never
                               later than the first root) but may be earlier than a full
                               run's; n_checks counts the checks through that level */
#define CCD_ST_INVALID 0x80 /* device-side validation rejected the query
                               (toi = t_width = NaN, hit = 0, n_checks = 0) */

/* Parameter flags. */
#define CCD_FLAG_LITERAL 0x1u /* drop, as Alg. 2 is printed, a colliding box that meets
                                 the termination test but is not the first colliding box
                                 of its level.  Default (flag clear): remember the
                                 earliest such box and return it once no earlier
                                 candidate is left, which keeps toi conservative when
                                 the first box's region later turns out empty. */

/* Parameters of one query (Alg. 2 inputs; Sec. 6.1 adds min_sep). */
typedef struct ccd_params {
    double delta;      /* tolerance delta > 0 on the co-domain width; paper default 1e-6 */
    int64_t max_iter;  /* m_I >= 1: maximum number of box checks; paper default 1e6 */
    double min_sep;    /* d >= 0: minimum separation, L-infinity; 0 = standard CCD */
    double t_max;      /* 0 < t_max <= 1: search t in [0, t_max]; paper default 1 */
    uint32_t flags;    /* CCD_FLAG_* */
    uint32_t reserved; /* must be 0 */
} ccd_params;

/* Result of one query. */
typedef struct ccd_result {
    double toi;        /* earliest conservative time of impact, +inf if none */
    double t_width;    /* w(I_t) of the returned level, 0 if none */
    uint64_t n_checks; /* box checks of the sequential Alg. 2, saturated at m_I */
    uint8_t hit;       /* toi <= 1 */
    uint8_t status;    /* CCD_ST_* bits */
    uint8_t reserved[6];
} ccd_result;

/*
 * Single queries on the GPU of a library-owned default context (device 0),
 * run through the same kernels as ccd_batch.  x0: the 4 points at t = 0, x1:
 * the same points at t = 1 (host memory).  Blocking.  Returns CCD_EINVAL for
 * an invalid query or NULL pointer (out untouched), CCD_EDEVICE without a GPU.
 */
int ccd_vf(const double x0[4][3], const double x1[4][3], const ccd_params* params,
           ccd_result* out);
int ccd_ee(const double x0[4][3], const double x1[4][3], const ccd_params* params,
           ccd_result* out);

/* Fills *p with the paper's defaults: delta 1e-6, max_iter 1e6, min_sep 0, t_max 1. */
void ccd_params_default(ccd_params* p);

/* ------------------------------------------------------------------------- */
/* Contexts and batches. */

typedef struct ccd_context ccd_context;

/*
 * Creates a context on HIP device `device` whose scratch allocations (frontier
 * arenas, promotion records, queues) stay within mem_budget_bytes of device
 * memory (0 selects a default of 16 GiB).  The context owns its scratch; it is
 * not thread-safe (one host thread at a time per context).
 */
int ccd_context_create(int device, size_t mem_budget_bytes, ccd_context** out);
void ccd_context_destroy(ccd_context* ctx);

/* Engines selectable with ccd_context_set_engine. */
#define CCD_ENGINE_PERSISTENT 0 /* persistent kernels: lane per light query, group per
                                   wide query, block per huge query (default) */
#define CCD_ENGINE_PLAIN 1      /* one thread per query for every query up to its lane
                                   capacity, then the same group and block tiers */
int ccd_context_set_engine(ccd_context* ctx, int engine);

/* Launch and capacity knobs (what the autotuner searches); 0 keeps a field's
 * current value.  Values are clamped to supported ranges. */
typedef struct ccd_tuning {
    int32_t lane_waves_per_cu;    /* resident waves per CU of the lane-per-query kernel */
    int32_t lane_capacity;        /* boxes per level a lane may hold in LDS (8..32) */
    int64_t lane_budget;          /* checks a lane spends before it hands the query on */
    int32_t group_waves;          /* waves per group working on one wide query (1, 2, 4, 8) */
    int32_t group_count;          /* resident groups of the wide-query kernel */
    int64_t group_capacity;       /* boxes per level of a group's arena */
    int32_t block_count;          /* engines of the huge-query kernel (default 2 per CU); with
                                     at least 2 per CU each is a workgroup of 4 waves, else
                                     of 8 waves (the budget can lower the count) */
    int32_t group_occupancy;      /* single-wave groups: minimum waves per SIMD the register
                                     allocation must allow (1..4) */
    int64_t block_capacity;       /* words per level of a huge-query arena; 0 (default): 2 m_I + 2,
                                     enough for every query, clamped to a quarter of the
                                     budget.  Never below group_capacity.  A query whose
                                     level outgrows it returns with CCD_ST_OVERFLOW. */
    int64_t handoff_words;        /* largest pool (8-byte words) carrying a wide query's
                                     current level from the group to the block engine; the
                                     pool gets up to an eighth of the budget left after one
                                     arena of each engine, and after the engines' arenas
                                     whatever the budget still leaves.  When it is full the
                                     block engine restarts such a query at level 0 (same
                                     results, more work).  Default 2^33. */
    int32_t group_lds_words;      /* the first words of each level of a wide query stay in LDS
                                     (two buffers per group; the rest of a level spills to
                                     the HBM arena), for one-wave groups at occupancy 3 and
                                     eight-wave groups.  Default 0 (off); clamped to what a
                                     workgroup can hold beside the kernel's own LDS; rounded
                                     down to a multiple of 64 words per wave of the group. */
    int32_t block_lds_words;      /* the same for the huge-query engine.  Default 2048. */
} ccd_tuning;
int ccd_context_get_tuning(ccd_context* ctx, ccd_tuning* out);
int ccd_context_set_tuning(ccd_context* ctx, const ccd_tuning* t);

/*
 * The scratch a batch of n queries (largest m_I = max_iter) would be given on
 * a GPU of num_cu compute units under a memory budget (0: the 16 GiB
 * default) and a tuning (NULL: the defaults; zero fields keep the defaults).
 * Host-only: touches no device.  Sizes are computed with overflow-checked
 * arithmetic; the block engine's arena is 2 m_I + 2 words per buffer (enough
 * for every query, Alg. 2 stops a level below 2 m_I boxes) clamped to a
 * quarter of the budget and to the tuning's block_capacity.  Returns
 * CCD_ENOMEM when even one arena of each engine does not fit, CCD_EINVAL for
 * num_cu < 1, n < 0, max_iter < 1 or an unknown engine.
 */
typedef struct ccd_scratch_plan {
    uint64_t bytes;           /* device memory of the whole plan */
    uint64_t lane_lds_bytes;  /* LDS per lane-engine block (the lanes' frontiers) */
    int64_t lane_blocks;
    int64_t group_count;
    int64_t group_capacity;   /* words per level buffer */
    int64_t block_count;
    int64_t block_capacity;   /* words per level buffer */
    int64_t handoff_words;
} ccd_scratch_plan;
int ccd_plan_scratch(const ccd_tuning* tuning, int num_cu, size_t mem_budget_bytes, int64_t n,
                     int64_t max_iter, int engine, ccd_scratch_plan* out);


/* A batch of n queries in structure-of-arrays layout. */
typedef struct ccd_batch_desc {
    int64_t n;                 /* number of queries, >= 0 */
    const double* pos;         /* [24][n]: pos[(3k+c)*n + q] = coordinate c of point k */
    const uint8_t* kind;       /* [n] CCD_KIND_*; NULL: every query is default_kind */
    uint8_t default_kind;
    uint8_t reserved[7];
    const double* delta_q;     /* [n] per-query delta or NULL (params.delta) */
    const int64_t* max_iter_q; /* [n] per-query m_I or NULL (params.max_iter) */
    const double* min_sep_q;   /* [n] per-query d or NULL (params.min_sep) */
    ccd_params params;         /* batch parameters (flags and t_max always from here) */
    int32_t on_device;         /* 1: all pointers (inputs and outputs) are device memory */
    int32_t reserved2;
} ccd_batch_desc;

/* Outputs of a batch, one entry per query (caller-owned). */
typedef struct ccd_result_soa {
    double* toi;
    double* t_width;
    uint8_t* hit;
    uint64_t* n_checks;
    uint8_t* status;
} ccd_result_soa;

/*
 * Solves a batch.  `stream` is a hipStream_t (NULL: the legacy default stream).
 *   on_device = 1: inputs and outputs are device pointers; the call is
 *     asynchronous and completes on `stream`; inputs are validated on the
 *     device and invalid queries get status CCD_ST_INVALID.  Buffers must stay
 *     alive until the stream has passed the call.
 *   on_device = 0: host pointers; the whole batch is validated on the host
 *     first (CCD_EINVAL, outputs untouched, if any query is invalid), then
 *     copied, solved and copied back; the call returns when results are in the
 *     host arrays.
 * Results do not depend on batch composition, engine or tuning.  The context's
 * scratch is reused by the next call on it: calls on one context must not
 * overlap on different streams.
 */
int ccd_batch(ccd_context* ctx, const ccd_batch_desc* desc, const ccd_result_soa* out,
              void* stream);

/*
 * Allocation-free ccd_batch, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same inputs, outputs, results and tuning as ccd_batch with
 * on_device = 1 (device pointers only; CCD_EINVAL otherwise), asynchronous on
 * `stream`, kernels launched one by one (never a graph of the library's own).
 * It calls no hipMalloc, hipFree or other allocating routine: its scratch
 * (counters, hand-off records, frontier arenas) is one static device array of
 * 256 MiB per GPU, loaded with the library and held until the process ends.
 * A batch whose scratch plan (ccd_plan_scratch with a 256 MiB budget) does
 * not fit is rejected with CCD_ENOMEM before anything is launched; with the
 * default tuning that is a batch of more than about 960,000 queries.  With
 * per-query m_I (max_iter_q) the block engine's arena takes what the array
 * allows and a query needing more returns with CCD_ST_OVERFLOW.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (the counters are cleared by a kernel at the start of each call):
 * calls that overlap on one GPU, on any streams or contexts, race and must be
 * serialised by the caller.  ccd_context_last_stats does not describe these
 * calls.
 */
int ccd_batch_noalloc(ccd_context* ctx, const ccd_batch_desc* desc, const ccd_result_soa* out,
                      void* stream);

/*
 * Autotuner: coordinate descent over the ccd_tuning knobs (group occupancy and
 * count, lane budget, lane capacity, lane waves per CU, group width, group
 * LDS words), each
 * candidate timed (median of 3, after a warm-up) with events around whole
 * ccd_batch calls of the given device batch on `stream`; a candidate must be
 * 2% faster to be taken, and the winner is confirmed against the starting
 * tuning with 5 runs each.  Leaves the fastest tuning on the context and
 * returns it with its time.  `out` is overwritten by
 * every trial.  max_trials <= 0: no limit (about 20 trials).  Results of the
 * root finder do not depend on the tuning.  Synchronises the stream.
 */
int ccd_autotune(ccd_context* ctx, const ccd_batch_desc* desc, const ccd_result_soa* out,
                 void* stream, int max_trials, ccd_tuning* best, float* best_ms);

/*
 * Tuning cache in a text file, one line per (GPU architecture, CU count, HIP
 * runtime version, workload key).  store writes the context's current tuning
 * under `key` (no whitespace); load applies a matching line, or returns
 * CCD_EAGAIN when there is none.
 */
int ccd_tuning_cache_store(ccd_context* ctx, const char* path, const char* key);
int ccd_tuning_cache_load(ccd_context* ctx, const char* path, const char* key);

/*
 * The launch sequence of a batch is captured into a hipGraph and replayed while
 * its parameters (pointers, sizes, tuning) are unchanged; a change rebuilds it.
 * Enabled by default; disabling launches the kernels one by one, and so does
 * per-kernel timing (ccd_context_enable_timing).  Results are the same either way.  graph_counts reports how many graphs were built and
 * how many launches replayed an existing one.
 */
int ccd_context_enable_graphs(ccd_context* ctx, int enable);
int ccd_context_graph_counts(ccd_context* ctx, uint64_t* builds, uint64_t* replays);

/* Counters of the last ccd_batch on a context (host copy; synchronises). */
typedef struct ccd_stats {
    uint64_t checks[3][2];   /* box checks executed by tier [lane, group, block] x kind [VF, EE];
                                the lane tier includes the root pass */
    uint64_t promoted[2];    /* queries handed to the group tier, to the block tier */
    uint64_t lane_slots[3];  /* lane-iterations spent per tier; checks / lane_slots is the
                                fraction of SIMD lanes doing box checks */
    float kernel_ms[4];      /* device time of [root pass, lane, group, block] kernels
                                (only when timing is enabled, else 0) */
    uint32_t reserved;
    uint64_t overflowed;     /* queries returned with CCD_ST_OVERFLOW */
    uint64_t restarted;      /* group -> block hand-offs restarted at level 0 (pool full) */
    uint64_t deep;           /* lane -> group hand-offs because a level reached depth sum 64 */
    uint64_t handoff_words;  /* pool words the group -> block hand-offs asked for */
    uint64_t probes[2];      /* level probes of the wide engines: run, and decided the level
                                without checking it in full */
} ccd_stats;
int ccd_context_enable_timing(ccd_context* ctx, int enable);
int ccd_context_last_stats(ccd_context* ctx, ccd_stats* out);

/*
 * Smallest toi of a batch, for a line search: the step length is bounded by
 * the earliest time of impact over the candidate pairs (Sec. 7.2, Alg. 4: alpha
 * = min(t, alpha) over the MSCCD calls).  toi: n device doubles (a result's
 * toi array); out: one device double, 8-byte aligned.  Asynchronous on
 * `stream` (0 = default), ordered after the batch that wrote toi when issued
 * on the same stream.  NaN entries (invalid queries) are skipped; *out = +inf
 * when n = 0 or no entry is finite.  Returns CCD_EINVAL for a null pointer
 * with n > 0, n < 0 or a misaligned out, CCD_EDEVICE on a HIP error.
 */
int ccd_min_toi(ccd_context* ctx, const double* toi, int64_t n, double* out, void* stream);

/*
 * Candidate pairs over shared vertex arrays (Sec. 7: the active-set and line
 * search drivers run CCD on the pairs of a mesh's broad phase), with an
 * optional scene-wide filter.
 *
 * Query q is made of vertices ids[4q .. 4q+3] of v0 (positions at t = 0) and
 * v1 (at t = 1): VF (p, v1, v2, v3), EE (p1, p2, p3, p4).  An id outside
 * [0, n_vertices) makes the query invalid (status CCD_ST_INVALID).
 *
 * gamma: NULL, or 3 doubles, the scene-wide gamma per axis.  Sec. 7 computes
 * the tolerances of eq. ccd-error / msccd-error from the maximum over all the
 * vertices of the scene, so that they are the same for every query of a step;
 * eps_c = K gamma_c^3 then replaces the query's own.  A query whose own gamma
 * (max(1, max |x^c|) over its 8 points) exceeds gamma_c is invalid, as is one
 * with min_sep >= min_c gamma_c.  ccd_scene_gamma() computes gamma.
 *
 * Device memory only (on_device must be 1), asynchronous on `stream`; the
 * context's scratch holds the gathered coordinates (24 doubles per query) and
 * is reused by the next call: as for ccd_batch, calls on one context must not
 * overlap on different streams.
 */
typedef struct ccd_indexed_desc {
    int64_t n;                 /* number of queries (candidate pairs), >= 0 */
    int64_t n_vertices;        /* vertices in v0 / v1 */
    const double* v0;          /* [n_vertices][3] positions at t = 0 */
    const double* v1;          /* [n_vertices][3] positions at t = 1 */
    const int32_t* ids;        /* [n][4] vertex ids per query */
    const uint8_t* kind;       /* [n] CCD_KIND_*; NULL: every query is default_kind */
    const double* gamma;       /* [3] scene-wide gamma, or NULL for each query's own */
    uint8_t default_kind;
    uint8_t reserved[7];
    ccd_params params;         /* batch parameters */
    int32_t on_device;         /* must be 1 */
    int32_t reserved2;
} ccd_indexed_desc;
int ccd_batch_indexed(ccd_context* ctx, const ccd_indexed_desc* d, const ccd_result_soa* out,
                      void* stream);

/*
 * Scene-wide gamma per axis: gamma_c = max(1, max over the vertices of v0 and
 * v1 of |x^c|), non-finite coordinates skipped.  Device pointers; gamma: 3
 * device doubles, 8-byte aligned.  Asynchronous on `stream`.
 */
int ccd_scene_gamma(ccd_context* ctx, const double* v0, const double* v1, int64_t n_vertices,
                    double* gamma, void* stream);

/* ------------------------------------------------------------------------- */
/*
 * Serving: continuous batching of requests on one GPU.
 *
 * A request is a batch of queries in host memory (ccd_batch_desc with
 * on_device = 0 and no per-query parameter arrays; its params apply to all of
 * its queries).  A scheduler thread admits requests in arrival order while the
 * device pool has room for their inputs and outputs, and whenever a compute
 * stream is idle it launches one pass of the root finder over every admitted
 * request not yet started (their queries concatenated).  Requests arriving
 * meanwhile go into the next launch on another stream, overlapping the first.
 * Each request's results are bit-identical to ccd_batch on it alone.
 *
 * The caller's input and output arrays must stay valid until the ticket is
 * done.  Inputs in pinned host memory (hipHostMalloc) are copied
 * asynchronously; pageable inputs make the scheduler wait for their copy.
 * Results are staged in pinned memory owned by the server and copied into the
 * caller's arrays before the ticket completes.
 */
typedef struct ccd_server ccd_server;

typedef struct ccd_serve_config {
    int32_t device;
    int32_t streams;                /* compute streams (1..4), default 2 */
    int32_t max_requests;           /* requests per launch, default 1024 */
    int32_t launch_target_us;       /* latency bound: a launch takes at most as many queries as
                                       fill this much device time, from the device time per
                                       query measured on earlier launches (at least one
                                       request per launch); 0: off.  Default 5000 */
    int64_t max_queries_per_launch; /* default 4,000,000 (a larger single request still runs) */
    size_t pool_bytes;              /* device memory for resident requests, default 8 GiB */
    size_t scratch_bytes;           /* scratch budget per compute stream, default 12 GiB */
} ccd_serve_config;

typedef struct ccd_serve_info {
    int32_t state;     /* 0 queued, 1 admitted, 2 running, 3 done */
    int32_t rc;        /* CCD_OK or the request's error once done */
    int64_t n;
    double t_submit;   /* host steady-clock seconds */
    double t_admit;
    double t_launch;
    double t_done;     /* results are in the caller's arrays */
} ccd_serve_info;

typedef struct ccd_serve_stats {
    uint64_t submitted, admitted, completed, rejected, launches, queries_completed;
    uint64_t queued;       /* waiting for device memory */
    uint64_t pool_bytes, pool_in_use, pool_peak;
} ccd_serve_stats;

#define CCD_SERVE_NONBLOCKING 0x1 /* submit returns CCD_EAGAIN instead of queueing when the
                                     request cannot be admitted right away */

void ccd_serve_config_default(ccd_serve_config* cfg);
/* cfg NULL: defaults.  CCD_ENOMEM if the pools or scratch cannot be allocated. */
int ccd_serve_open(const ccd_serve_config* cfg, ccd_server** out);
/* Validates the request on the host (CCD_EINVAL), rejects one larger than the
 * pool (CCD_ENOMEM), then queues it and returns its ticket. */
int ccd_serve_submit(ccd_server* s, const ccd_batch_desc* desc, const ccd_result_soa* out,
                     int flags, int64_t* ticket);
/* 1 done (results in place), 0 pending, or the request's negative error code. */
int ccd_serve_poll(ccd_server* s, int64_t ticket);
/* Blocks until done (timeout_ms < 0: no limit); CCD_ETIMEDOUT otherwise. */
int ccd_serve_wait(ccd_server* s, int64_t ticket, int timeout_ms);
int ccd_serve_query(ccd_server* s, int64_t ticket, ccd_serve_info* info);
/* Forgets a finished ticket (CCD_EAGAIN while it is not done). */
int ccd_serve_release(ccd_server* s, int64_t ticket);
int ccd_serve_stats_get(ccd_server* s, ccd_serve_stats* out);
/* Finishes every submitted request, then frees the server. */
int ccd_serve_close(ccd_server* s);

/* Message for a return code. */
const char* ccd_strerror(int code);

/* Text of the last HIP failure or capacity error seen by the library on the
 * calling thread ("" if none); valid until the next library call. */
const char* ccd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CCD_H */
