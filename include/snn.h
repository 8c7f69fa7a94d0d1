/*
 * snn.h -- C ABI of the MI355X (gfx950) SNN library: exact fixed-radius
 * near-neighbour search by sorting (Chen & Guettel, "Fast and exact
 * fixed-radius neighbor search based on sorting").
 *
 * Result definition (normative for every entry point below).  For data
 * rows p_i and a query q, both promoted to double (exact),
 *
 *     N(q) = { i : S(p_i, q) <= fl(R*R) },
 *     S(p, q) = fl(... fl(fl(t_0*t_0) + fl(t_1*t_1)) ... + fl(t_{d-1}*t_{d-1})),
 *     t_k = fl(p_k - q_k),
 *
 * i.e. the direct squared distance of Section 4, eq. (ip1), summed left to
 * right as in the rounding analysis of Section 4, without fused
 * multiply-add, and compared inclusively with R^2 (Section 3.2).  The
 * returned distance is (float)sqrt(S).  Index sets are bit-identical to a
 * CPU float64 evaluation of this rule.
 *
 * Memory.  Every pointer named "device" is HIP device memory of the
 * device in snn_device.device; "host" pointers are ordinary host memory.
 * Inputs are borrowed for the duration of the call only.  Device memory
 * the library needs (the index, its workspace) comes from snn_device.alloc
 * (hipMalloc when NULL) and is returned through snn_device.free.
 *
 * Streams.  All device work of a call is enqueued on snn_device.stream
 * (NULL: the null stream).  snn_query / snn_query_self synchronise that
 * stream once, to learn the number of neighbours; they return with the CSR
 * arrays still being written by work enqueued on the stream.
 *
 * Errors.  Every entry point returns an snn_status; on failure
 * snn_last_error() describes it (thread-local, valid until the next call on
 * the thread).  No C++ exception crosses this interface.  Calls on one
 * index from several host threads must be serialised by the caller.
 *
 * Environment (read at every call).
 *   SNN_LOG=0..3      lines on stderr: 0 none (default), 1 every failing
 *                     call (status and message), 2 also one line per query
 *                     and per batch run (sizes, screen chosen, pairs, nnz,
 *                     device times when stats are asked for), 3 also
 *                     workspace growth, survivor-list retries and graph
 *                     capture.
 *   SNN_PROFILE=1     snn_stats.stage_ms holds the device time of each
 *                     stage of the query (SNN_STAGE_*); otherwise every
 *                     entry is -1.  Profiled single-instance calls launch
 *                     kernel by kernel (no replay of captured graphs, so
 *                     that events can sit between the stages); a batch
 *                     created with SNN_PROFILE=1 has clock stamps between
 *                     the stages inside its query graph.
 *   SNN_TUNE_CACHE=path  the batch autotuner's cache file when the batch
 *                     options name none.
 *   SNN_FAULT_INJECT=n  (tests) the n-th checked HIP result of each call
 *                     reads as a failure: the call returns SNN_EDEVICE after
 *                     freeing what it allocated, every kernel it launched
 *                     still runs to its end, and an index stays usable.
 */
#ifndef SNN_H_
#define SNN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Enumerations are int-sized.  Compiled as C++ they get int as their fixed
 * underlying type, so any int a C caller passes is a value of the type and
 * the library can reject it (without it, reading an out-of-range value of an
 * enumeration is undefined in C++). */
#ifdef __cplusplus
#define SNN_ENUM(tag) enum tag : int
#else
#define SNN_ENUM(tag) enum tag
#endif

typedef SNN_ENUM(snn_status_e) {
  SNN_OK = 0,
  SNN_EINVAL = -1,    /* bad argument, or NaN/Inf in the data or queries */
  SNN_ENOMEM = -2,    /* the allocator returned NULL */
  SNN_EDEVICE = -3,   /* a HIP call failed, or no usable gfx950 device */
  SNN_EOVERFLOW = -4, /* CSR capacity too small; csr.nnz holds the size needed */
  SNN_ENOTSUP = -5    /* valid but unsupported request */
} snn_status;

typedef SNN_ENUM(snn_dtype_e) { SNN_F32 = 0, SNN_F64 = 1 } snn_dtype;

/* How candidate distances are screened (all give the same exact result).
 * FP64:  every window pair is decided by the normative rule in float64.
 * MIXED: window pairs are screened on the matrix cores (bf16 operands,
 *        fp32 accumulation) against a rigorous rounding bound; only pairs
 *        the screen cannot reject are re-decided by the normative rule in
 *        float64 (the "precision form").
 * FP16:  the same screen with one fp16 operand per coordinate of the rows
 *        scaled by a power of two (d <= 128): a rounding band 8x narrower
 *        than one bf16 term at the same matrix-core rate.
 * FP32:  the same screen with fp32 operands on the matrix cores (d <= 16):
 *        a much narrower rounding band, for low dimensions with a radius
 *        that is small against the data's extent.
 * AUTO:  the library picks from the width of each screen's rounding band
 *        relative to R^2 and from d.
 * The 16-bit and fp32 screens need the centred rows within fp32 range (norms
 * below 2^60; fp16: below 2^75); beyond it they return SNN_ENOTSUP and AUTO
 * takes FP64. */
typedef SNN_ENUM(snn_precision_e) {
  SNN_PREC_FP64 = 0,
  SNN_PREC_MIXED = 1,
  SNN_PREC_AUTO = 2,
  SNN_PREC_FP32 = 3,
  SNN_PREC_FP16 = 4
} snn_precision;

/* Distance of a query (Section 2).
 * L2: the Euclidean rule above.
 * L1: Manhattan, N(q) = { i : M(p_i, q) <= R } with M the float64 sum, left
 *     to right, of |fl(p_k - q_k)|; dist = fl32(M).  Every such point lies in
 *     the Euclidean ball of radius R (the 2-norm never exceeds the 1-norm),
 *     so the Euclidean window and screen, run with R widened by the rounding
 *     of M, find a superset that the float64 recheck decides by M.
 * ANGULAR and COSINE: on unit vectors the angle is at most a iff
 *     ||u - v||^2 <= 2 - 2 cos(a), and the cosine distance is ||u - v||^2 / 2,
 *     so both are Euclidean searches of normalised rows (snn_normalize_rows;
 *     the rows are used as given) with the squared threshold
 *       ANGULAR: R = a in radians, 0 <= a <= pi:  T = fl(2 - 2 cos(a)),
 *                cos the host C library's double cosine;
 *       COSINE:  R = c >= 0:                       T = fl(2 c);
 *     N(q) = { i : S(p_i, q) <= T } with S the normative sum above, and
 *     dist = fl32(2 asin(min(1, sqrt(S) / 2))) (the angle, radians) or
 *     fl32(S / 2) (the cosine distance), evaluated in float64. */
typedef SNN_ENUM(snn_metric_e) { SNN_METRIC_L2 = 0, SNN_METRIC_L1 = 1, SNN_METRIC_ANGULAR = 2, SNN_METRIC_COSINE = 3 } snn_metric;

typedef struct {
  /* Device allocator; both NULL selects hipMalloc/hipFree.  alloc returns
   * 256-byte aligned device memory of at least `bytes`, or NULL. */
  void* (*alloc)(void* ctx, size_t bytes);
  void (*free)(void* ctx, void* ptr);
  void* ctx;
  void* stream; /* hipStream_t */
  int device;   /* HIP device ordinal */
} snn_device;

typedef struct {
  snn_precision precision;
  /* bf16 terms per coordinate in MIXED mode: 1 (one bf16 value) or 3
   * (hi/lo split: hi*hi + hi*lo + lo*hi, ~16 bits); 0 = automatic. */
  int mixed_terms;
  /* queries per tile / candidates per work unit; 0 = automatic. */
  int tile_q;
  int tile_c;
  /* snn_query_self only: 0 (default) scans each unordered pair once, from
   * the query that comes first in score order, and reports it in both rows
   * (the squared distance is exactly symmetric); 1 scans every (query,
   * candidate) pair.  Both give the same result. */
  int full_self_scan;
  /* snn_metric; 0 = L2 */
  int metric;
} snn_options;

typedef struct {
  int64_t* row_ptr; /* device, m+1 entries, always written */
  int32_t* col;     /* device, nnz_cap entries: original data row ids,
                       ascending within a row */
  float* dist;      /* device, nnz_cap entries: (float)sqrt(S) */
  int64_t nnz_cap;  /* in: capacity of col / dist */
  int64_t nnz;      /* out: number of neighbours (also on SNN_EOVERFLOW) */
} snn_csr;

/* Stages of a query (Algorithm 2) as timed under SNN_PROFILE=1. */
enum {
  SNN_STAGE_ORDER = 0,    /* steps 2-3: queries centred and projected, put
                             into score order; their screen operands */
  SNN_STAGE_WINDOW = 1,   /* step 4: candidate windows by eq. (lower), the
                             tile plan */
  SNN_STAGE_SCREEN = 2,   /* step 5: the candidate screen */
  SNN_STAGE_RECHECK = 3,  /* step 6: survivors re-decided by the normative rule */
  SNN_STAGE_ASSEMBLE = 4, /* row offsets, neighbours into rows, rows sorted by id */
  SNN_STAGES = 5
};

typedef struct {
  int64_t pairs_window;   /* sum over queries of |J_q| (Algorithm 2, step 4) */
  int64_t pairs_executed; /* (query, candidate) pairs the screen evaluated */
  int64_t pairs_recheck;  /* pairs re-decided in float64 by the normative rule */
  int64_t nnz;
  int32_t precision_used; /* snn_precision actually run */
  int32_t terms_used;     /* MIXED: bf16 terms per coordinate; FP16: 1 */
  double screen_ms;       /* device time of the candidate-screen kernel */
  double total_ms;        /* device time of the whole call */
  double flops_window;    /* algorithmic work of the window: sum over queries of
                             2 d |J_q| (the flop count of eq. (ip2) per candidate) */
  double stage_ms[SNN_STAGES]; /* with SNN_PROFILE=1: device time of each stage
                                  (SNN_STAGE_*), boundary to boundary on the
                                  stream; -1 when not profiled */
} snn_stats;

typedef struct snn_index_s* snn_index_t;

/* Algorithm 1 (Section 3.1): centre by the mean, first principal direction
 * (power iteration on the centred Gram matrix; any direction keeps the
 * result exact by eq. (lower)), sort rows by their score, keep the
 * sorted scores, squared norms and row copies the queries need.
 *   X: device, n x d row-major, dtype.  1 <= d <= 1024, 1 <= n < 2^31.
 * Errors: SNN_EINVAL (NULL/ranges/NaN/Inf in X), SNN_ENOMEM, SNN_EDEVICE. */
snn_status snn_index(const snn_device* dev, const void* X, int64_t n, int32_t d, snn_dtype dtype,
                     snn_index_t* out);

/* Algorithm 2 (Section 3.2) for m out-of-sample queries.
 *   Q: device, m x d row-major, same dtype as the index.  m >= 0.
 *   R: radius, finite and >= 0.  opts may be NULL (AUTO).
 *   out: caller-owned device CSR; rows follow the order of Q.
 *   st:  host, may be NULL.
 * If the neighbours do not fit, returns SNN_EOVERFLOW with out->nnz set to
 * the number needed and row_ptr written; col/dist are then unspecified. */
snn_status snn_query(snn_index_t idx, const void* Q, int64_t m, double R, const snn_options* opts,
                     snn_csr* out, snn_stats* st);

/* All-points self-query: every data row of the index is a query (rows of
 * the CSR follow the original data order).  Same contract as snn_query. */
snn_status snn_query_self(snn_index_t idx, double R, const snn_options* opts, snn_csr* out,
                          snn_stats* st);

/* Host-readable views of index internals, for checking and diagnostics.
 * Device pointers stay owned by the index. */
typedef struct {
  int64_t n;
  int32_t d;
  snn_dtype dtype;
  const double* mu;       /* device, d: column means */
  const double* v;        /* device, d: unit sorting direction */
  const double* key;      /* device, n: sorted scores, float32 values held in double */
  const int32_t* perm;    /* device, n: sorted position -> original row id */
  double max_norm;        /* host: max_i ||fl32(p_i - mu)|| */
  double key_eps;         /* host: bound on |key_i - v.(p_i - mu)| over all i */
  int32_t power_iters;    /* host: power iterations run */
} snn_index_view;

/* Streaming inserts (the online setting of Section 1): appends k rows of the
 * index's dtype and dimension, which get ids n .. n+k-1.  The centre mu and
 * the direction v stay those of the original build (eq. (lower) holds for
 * any fixed unit v and any common centre, so every later query stays exact;
 * only the window sizes depend on how well v fits the grown set).  The new
 * rows are centred, projected and sorted, then merged into the key order
 * (existing rows first among equal keys); the bounds over all rows are
 * updated and the screen operands rebuilt on the next query.
 *   X: device, k x d row-major.  Runs on the index's stream and returns when
 *   the index is updated.
 * Errors: SNN_EINVAL (NULL index or X, k < 0, n + k >= 2^31 - 1, NaN/Inf in
 * X -- the index is then unchanged), SNN_ENOMEM, SNN_EDEVICE. */
snn_status snn_index_insert(snn_index_t idx, const void* X, int64_t k);

snn_status snn_index_get_view(snn_index_t idx, snn_index_view* view);

void snn_index_free(snn_index_t idx);

/* ---- Batching form --------------------------------------------------------
 * Many independent instances, each a complete Algorithm 1 + Algorithm 2
 * (own data, queries, radius and dimension), run as one captured HIP graph of
 * batched kernels in which the candidate screen of every instance is one
 * persistent matrix-core launch (the MIXED screen with a float64 recheck, so
 * every result is exact).  A plan fixes the instance sizes and pointers to the
 * data; the data may change between runs, and the CSR structs are read again
 * at every run. */
typedef struct {
  const void* X;  /* device, n x d row-major, batch dtype; read at every index pass */
  const void* Q;  /* device, m x d row-major; NULL with m = n: all-points self-query;
                     NULL with m = 0: no queries */
  int64_t n;      /* 1 <= n < 2^31 */
  int64_t m;      /* 0 <= m < 2^31 */
  int32_t d;      /* 1 <= d <= 128 */
  double R;       /* finite, >= 0 */
  snn_csr* out;   /* host struct owned by the caller; it and its device arrays must
                     stay valid for the plan's lifetime (they may be replaced between
                     runs).  Rows follow the order of Q (of X for a self-query). */
} snn_instance;

typedef struct {
  int32_t mixed_terms;    /* 0: per instance from its rounding band; or 1 / 3 for all */
  int32_t tile_c;         /* candidates per work unit (multiple of 32); 0: tuned / 4096 */
  int32_t tile_g;         /* tiles per work group; 0: tuned / 8 */
  int32_t autotune;       /* 1: time candidate (tile_c, tile_g) on this batch at creation */
  const char* tune_cache; /* host path of a tuning cache file (read and appended), or NULL:
                             then SNN_TUNE_CACHE from the environment, if set */
} snn_batch_options;

typedef struct {
  int32_t tile_q;             /* query slots per tile */
  int32_t tile_c;             /* candidates per work unit */
  int32_t tile_g;             /* tiles per work group */
  int32_t operand_k;          /* bf16 operand row length of the screen */
  int32_t graph_timed_screen; /* 1 if the query graph times its screen kernel */
  float tuned_query_ms;       /* best query-pass time the autotuner measured (0: not tuned) */
  int32_t fp32_instances;     /* instances on the fp32 matrix-core screen (d <= 16, chosen
                                 when three bf16 terms would pass too many pairs) */
  int32_t fp32_k;             /* their padded operand length (0: none) */
} snn_batch_info_t;

typedef struct snn_batch_s* snn_batch_t;

enum { SNN_BATCH_INDEX = 1, SNN_BATCH_QUERY = 2 };

/* Validates the instances, allocates everything (dev->alloc), decides the
 * screen operands, captures the graphs and runs the index and query passes
 * once (so the outputs already hold a result).  opts may be NULL.
 * Errors: SNN_EINVAL (arguments, NaN/Inf in X), SNN_ENOTSUP, SNN_ENOMEM,
 * SNN_EDEVICE. */
snn_status snn_batch_create(const snn_device* dev, snn_dtype dtype, const snn_instance* instances,
                            int32_t count, const snn_batch_options* opts, snn_batch_t* out);

/* Runs the index pass, the query pass, or both (one graph launch) on
 * dev->stream and waits for it.  Every instance's out->nnz is set; if some
 * instance's neighbours exceed its nnz_cap the call returns SNN_EOVERFLOW
 * (that instance's col/dist unspecified, all others complete).  The query
 * pass uses the index of the latest index pass.  st (host, nullable) sums
 * over instances; screen_ms is -1 when the screen is not timed. */
snn_status snn_batch_run(snn_batch_t batch, int32_t what, snn_stats* st);

snn_status snn_batch_info(snn_batch_t batch, snn_batch_info_t* info);

void snn_batch_free(snn_batch_t batch);

/* One-shot form: create, run both passes once, free. */
snn_status snn_query_batch(const snn_device* dev, snn_dtype dtype, const snn_instance* instances,
                           int32_t count, const snn_batch_options* opts, snn_stats* st);

/* Rows scaled to unit Euclidean norm, for angular and cosine neighbours
 * (Section 2): y_i = x_i / ||x_i|| with ||x_i|| = sqrt of the float64 sum,
 * left to right, of the squared coordinates, the quotient rounded once to
 * the dtype (inputs promoted to float64 exactly).
 *   X, Y: device, n x d row-major, same dtype; Y may equal X.
 * Errors: SNN_EINVAL (NULL pointers, n < 0, d < 1, a row that is zero or
 * holds NaN/Inf -- Y is then unspecified), SNN_EDEVICE. */
snn_status snn_normalize_rows(const snn_device* dev, const void* X, int64_t n, int32_t d, snn_dtype dtype, void* Y);

/* ---- DBSCAN on self-query neighbour lists (Section 6.4) --------------------
 * Section 6.4 runs DBSCAN with SNN as its radius search (eps = R; its
 * experiments fix min_samples = 5).  Input: the CSR of an all-points
 * self-query, row i = { j : S(p_j, p_i) <= fl(eps*eps) } with i itself in
 * it and membership symmetric (j in row i iff i in row j), as
 * snn_query_self returns; only row_ptr and col are read.  Output:
 *   core[i]    = 1 iff row i has at least min_samples entries;
 *   labels[i]  = the cluster of a core point, where clusters are the
 *                connected components of the core points under "j in row
 *                i", numbered 0, 1, ... in order of their smallest core id;
 *                for a non-core point the smallest cluster number among the
 *                core points of its row; -1 (noise) if there is none.
 * These are the labels of the classic DBSCAN that visits the points in
 * index order (scikit-learn's).
 *   row_ptr:   device, n + 1 int64 (row_ptr[0] = 0, non-decreasing)
 *   col:       device, row_ptr[n] int32 ids in [0, n)
 *   labels:    device, n int32 (out)
 *   core:      device, n uint8 (out; NULL: not returned)
 *   nclusters: host (out; NULL: not returned)
 * Scratch comes from dev->alloc; the work runs on dev->stream and the call
 * returns when the labels are written.  Errors: SNN_EINVAL (NULL pointers,
 * n < 0, min_samples < 1, row_ptr not starting at 0 or decreasing, an id
 * outside [0, n) -- checked on the device before any other pass),
 * SNN_ENOMEM, SNN_EDEVICE. */
snn_status snn_dbscan(const snn_device* dev, int64_t n, const int64_t* row_ptr, const int32_t* col,
                      int32_t min_samples, int32_t* labels, uint8_t* core, int64_t* nclusters);

/* DBSCAN of the indexed points themselves: the all-points self-query with
 * radius eps (as snn_query_self) feeds the clustering directly, without
 * assembling neighbour lists or distances.  The labels, core flags and
 * cluster count are those snn_dbscan gives on snn_query_self's lists for
 * R = eps.  labels: device, n int32 (original point order); core: device, n
 * uint8 (nullable); nclusters: host (nullable); opts and st as for
 * snn_query_self (st->nnz = neighbour entries, self included).  Work runs on
 * the index's stream; the call returns when the labels are written.
 * Errors: SNN_EINVAL (NULL index or labels, min_samples < 1, eps < 0 or not
 * finite), SNN_ENOTSUP, SNN_ENOMEM, SNN_EDEVICE. */
snn_status snn_dbscan_index(snn_index_t index, double eps, int32_t min_samples, const snn_options* opts,
                            int32_t* labels, uint8_t* core, int64_t* nclusters, snn_stats* st);

/* Stable LSD radix sort of (key, value) pairs on bits [begin_bit, end_bit)
 * of the keys, in place (the building block of Algorithm 1, step 6).
 *   keys, vals: device, n entries each.  0 <= begin_bit < end_bit <= 32.
 * Scratch comes from dev->alloc.  Stable: equal keys keep their order. */
snn_status snn_sort_pairs_u32(const snn_device* dev, uint32_t* keys, uint32_t* vals, int64_t n,
                              int begin_bit, int end_bit);

/* The same sort without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the workspace is a static device array of the library
 * (18 MiB on every GPU it runs on, held until the process ends), so at most
 * 2^21 pairs.  dev->alloc / dev->free are not used; the work is enqueued on
 * dev->stream (kernel launches only: no allocation, copy, memset or
 * synchronisation) and the call returns without waiting for it.  All calls on
 * one GPU share that array: calls whose work overlaps on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * Errors: SNN_EINVAL (as snn_sort_pairs_u32, and n > 2^21), SNN_EDEVICE. */
snn_status snn_sort_pairs_u32_noalloc(const snn_device* dev, uint32_t* keys, uint32_t* vals, int64_t n,
                                      int begin_bit, int end_bit);

/* Message for the last failed call on this thread ("" if none). */
const char* snn_last_error(void);

/* Library version string. */
const char* snn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SNN_H_ */
