/*
 * tq.h -- C ABI of the ternary-quantised (EVP) embedding search library for
 * AMD MI355X (gfx950).
 *
 * The method is that of "Ultra-Quantisation: Efficient Embedding Search via
 * 1.58-bit Encodings" (Connor, Dearle, Claydon; arXiv 2506.00528):
 *
 *   - every float embedding u in R^d is replaced by its nearest {x,d}
 *     Equi-Voronoi-Polytope vertex v in {-1,0,+1}^d, the vector with exactly x
 *     non-zeros that carries the signs of the x largest-magnitude coordinates
 *     of u (Sec. 2.3 defines the polytope, Sec. 2.4 the nearest-vertex rule);
 *   - v is stored as two bit vectors, v+ (bit i set iff v_i = +1) and v-
 *     (bit i set iff v_i = -1) (Sec. 5.1.2, Table 3);
 *   - two codes are compared with Delta = b2sp(v,w), the scalar product of the
 *     ternary vectors computed from AND and popcount over the bit vectors
 *     (Sec. 5.1.2); larger Delta means nearer;
 *   - a query is answered by an exhaustive scan of the pre-encoded database
 *     followed by a per-query top-k (the kNN problem of Sec. 1.1 / Table 1).
 *
 * Conventions shared by every call
 *   - Every function returns an int status (TQ_OK or a negative TQ_ERR_*).
 *     Nothing throws across this boundary.  Arguments are validated before any
 *     GPU work is queued; on a validation failure nothing is written.
 *     tq_last_error() gives a human-readable reason for the last failing call
 *     made by the calling thread.
 *   - "Device pointer" means memory of the GPU that is current (hipSetDevice)
 *     when the call is made, e.g. the data_ptr() of a torch tensor on that GPU.
 *     "Host pointer" means ordinary CPU memory.  All memory passed in stays
 *     owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls that take a stream queue their GPU work on it and return without
 *     waiting, unless stated otherwise; the caller must keep the buffers alive
 *     until that work has completed (stream order).
 *   - Canonical code layout ("codes"): W = tq_code_words(d) = ceil(d/32)
 *     32-bit words per plane; a code row is the W words of v+ followed by the
 *     W words of v-, 2*W words in all; coordinate i is bit (i mod 32) of word
 *     (i / 32), least significant bit first (a little-endian byte view puts
 *     coordinate i at bit i of the row's byte string); bits for coordinates
 *     >= d are zero in both planes; no coordinate is set in both planes.
 *   - Results of a search are `ids` (int32, database row numbers) and
 *     `scores` (int32, Delta in [-x, x]), nq x k row-major, ordered nearest
 *     first: Delta descending, and on equal Delta the lower id first.  This is
 *     a total order, so the result is unique.
 */
#ifndef TQ_H
#define TQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------------- */
/* Status                                                                  */
/* ---------------------------------------------------------------------- */

enum tq_status {
  TQ_OK = 0,
  TQ_ERR_INVALID = -1,  /* bad argument, malformed code, or non-finite input */
  TQ_ERR_NOMEM = -2,    /* a device or host allocation failed (or the serving budget) */
  TQ_ERR_DEVICE = -3,   /* the HIP runtime reported an error */
  TQ_ERR_AGAIN = -4,    /* serving: the request is not finished yet */
  TQ_ERR_NOTFOUND = -5, /* serving: unknown, cancelled or already collected ticket */
  TQ_ERR_STATE = -6     /* the object is shutting down / the call is out of order */
};

/* Largest supported dimension d and number of neighbours k. */
#define TQ_MAX_D 1024
#define TQ_MAX_K 512

/* Static name of a status code ("TQ_OK", "TQ_ERR_INVALID", ...). */
const char *tq_status_str(int status);

/* Detail message of the last failing call on the calling thread ("" if none).
 * The pointer stays valid until the next tq_* call on the same thread. */
const char *tq_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int tq_version(void);

/* ---------------------------------------------------------------------- */
/* Layout                                                                  */
/* ---------------------------------------------------------------------- */

/* W = ceil(d/32), the number of 32-bit words of one bit plane (Sec. 5.1.2 /
 * Table 3 bit vectors, packed 32 coordinates per word).  Returns
 * TQ_ERR_INVALID if d < 1 or d > TQ_MAX_D. */
int tq_code_words(int d);

/* The x in 1..d with the most {x,d} vertices, C(d,x) * 2^x (Sec. 5.1.1: the
 * construction that maximises the number of Voronoi cells; Sec. 2.3 for the
 * count).  The count grows while 2(d - x) >= x + 1, so the maximum is at
 * ceil((2d - 1) / 3); when 3 divides 2d - 1 two neighbours tie and the
 * smaller is returned (which reproduces the paper's {333, 500}).  Returns
 * TQ_ERR_INVALID if d < 1 or d > TQ_MAX_D. */
int tq_default_x(int d);

/* ---------------------------------------------------------------------- */
/* Encode (Sec. 2.4, nearest {x,d} EVP vertex; Sec. 5.1.2 bit planes)      */
/* ---------------------------------------------------------------------- */

/* Encode n rows of d floats into their nearest {x,d} EVP vertices.
 *
 *   X      device pointer, n x d float32, row-major (row stride d).
 *   codes  device pointer, n x 2W uint32 in the canonical layout (written).
 *
 * For each row the x coordinates of largest |u_i| are chosen (equal
 * magnitudes: the lower index first; magnitudes are compared exactly, so
 * subnormals count), and get +1 if u_i is not negative (including +0.0 and
 * -0.0) and -1 if u_i < 0; the other coordinates are 0.  The rule is
 * invariant to positive scaling of a row, so rows need not be normalised.
 *
 * Requires n >= 0, 1 <= d <= TQ_MAX_D, 1 <= x <= d.  Asynchronous on
 * `stream`.  A NaN or infinite element makes its row's code all zero (which
 * tq_db_create rejects) and raises a sticky device flag that the next
 * tq_sync() reports as TQ_ERR_INVALID. */
int tq_encode(const float *X, int64_t n, int d, int x, uint32_t *codes, void *stream);

/* The b1.58 quantisation the paper compares against (Sec. 4.3), applied per
 * embedding: gamma = mean |u_i| of the row, v_i = max(-1, min(1, round(u_i /
 * gamma))) with round-half-to-even, in double precision (gamma summed in
 * double); an all-zero row gives the zero vector.  Same layout, limits and
 * NaN / infinity handling as tq_encode.  The number of non-zeros varies from
 * row to row, so such codes form a database with x = 0 (tq_db_create), where
 * Delta is the plain ternary scalar product. */
int tq_encode_b158(const float *X, int64_t n, int d, uint32_t *codes, void *stream);

/* ---------------------------------------------------------------------- */
/* Database (the pre-processed set S of Sec. 1.1)                          */
/* ---------------------------------------------------------------------- */

typedef struct tq_db tq_db;

/* Build a resident database from n canonical codes of an {x,d} EVP.
 *
 *   codes  device pointer, n x 2W uint32, canonical layout.
 *   x      the codes' number of non-zeros, or 0 for ternary codes with any
 *          number of them (e.g. tq_encode_b158).
 *
 * The library copies the codes into its own device memory (re-tiled for
 * streaming; the bits are unchanged; with 8x <= d also a second copy as
 * lists of the non-zero coordinates, see TQ_ENGINE_SPARSE, counted in
 * tq_db_info's device_bytes) and checks every row: exactly x
 * non-zeros (any number when x = 0), no coordinate in both planes, zero
 * padding bits.  A malformed row gives TQ_ERR_INVALID and no database.
 * Requires 1 <= n < 2^31, 0 <= x <= d.  The
 * call waits for its GPU work on `stream`, so `codes` may be freed when it
 * returns.  *out is owned by the caller; release it with tq_db_destroy().
 * A database is read-only after creation: any number of searches may use it
 * at once, on any streams of its device. */
int tq_db_create(const uint32_t *codes, int64_t n, int d, int x, void *stream, tq_db **out);

/* Write the database's codes back in the canonical layout (n x 2W uint32,
 * device pointer).  Asynchronous on `stream`. */
int tq_db_export(const tq_db *db, uint32_t *codes, void *stream);

/* Sizes of a database (any output pointer may be NULL). */
int tq_db_info(const tq_db *db, int64_t *n, int *d, int *x, size_t *device_bytes);

/* Free a database.  The caller must make sure no queued search still uses it
 * (e.g. tq_sync on the streams it was used on).  NULL is accepted. */
int tq_db_destroy(tq_db *db);

/* ---------------------------------------------------------------------- */
/* Search (exhaustive kNN over Delta; Sec. 1.1 / Table 1, Sec. 5.1.2)      */
/* ---------------------------------------------------------------------- */

enum tq_path {
  TQ_PATH_AUTO = 0,    /* pick per call from nq and the tuning cache */
  TQ_PATH_PLAIN = 1,   /* one full database pass per query (the baseline) */
  TQ_PATH_BATCHED = 2  /* all queries of the call share database passes */
};

typedef struct tq_search_opts {
  int path;          /* enum tq_path */
  int check_queries; /* non-zero: first verify every query code (exactly x
                        non-zeros, planes disjoint, zero padding); a malformed
                        one gives TQ_ERR_INVALID.  Costs a stream sync. */
  int grid;          /* 0 = auto; otherwise the number of workgroups of the
                        scan kernel (tuning / benchmarking) */
  int qtile;         /* 0 = auto; batched path: queries per workgroup tile:
                        2, 4, 8 or 16 on the popcount engine (at most 8 for
                        k > 128, 4 for k > 256), 64, 128 or 256 on the
                        matrix engine.  A tile of 64 or more with engine AUTO
                        selects the matrix engine. */
  int use_graph;     /* batched path: 1 = replay a captured hipGraph for the
                        batch-size bucket (default when the struct is NULL),
                        0 = launch the kernels directly */
  int engine;        /* TQ_ENGINE_AUTO, or on the batched path
                        TQ_ENGINE_POPCOUNT or TQ_ENGINE_MATRIX, or
                        TQ_ENGINE_SPARSE (plain path; AUTO path means plain);
                        results are identical */
  int metric;        /* enum tq_metric (0 = TQ_METRIC_DELTA) */
  int reserved[1];
} tq_search_opts;

/* What "nearest" means.  TQ_METRIC_DELTA: the largest Delta, the scalar
 * product of the ternary vectors (Sec. 5.1.2) -- a distance proxy when every
 * code has the same number of non-zeros, as {x,d} EVP codes do (Sec. 1.1:
 * for vectors of equal norm the scalar product orders them by l2 distance).
 * TQ_METRIC_L2: the smallest euclidean distance between the ternary vectors,
 * the proxy a database of codes with varying non-zero counts needs (b1.58,
 * Sec. 4.3; x = 0 databases); the reported score is
 * 2 Delta - nnz(v) = nnz(q) - |q - v|^2 (larger = nearer; the squared
 * distance is nnz(q) - score), same tie rule.  TQ_METRIC_L2 runs on the
 * bit planes (plain path, and the popcount engine of the batched path);
 * TQ_ENGINE_MATRIX or TQ_ENGINE_SPARSE with it is TQ_ERR_INVALID. */
enum tq_metric {
  TQ_METRIC_DELTA = 0,
  TQ_METRIC_L2 = 1
};

enum tq_engine {
  TQ_ENGINE_AUTO = 0,     /* the tuned / default choice */
  TQ_ENGINE_POPCOUNT = 1, /* Delta by AND / XOR / popcount on the vector ALUs */
  TQ_ENGINE_MATRIX = 2,   /* Delta as a ternary matrix product on the fp4 matrix
                             cores (exact; k <= 128) */
  TQ_ENGINE_SPARSE = 3    /* plain path: Delta gathered from the query at each
                             database code's listed non-zeros (a second,
                             index-list copy that tq_db_create keeps when
                             8x <= d: 2x bytes per vector instead of d/4;
                             Sec. 6 leaves small-x speed-ups open).  The plain
                             path with TQ_ENGINE_AUTO uses it when 16x <= d.
                             TQ_ERR_INVALID where there is no such copy. */
};

/* k nearest database codes of each of nq query codes.
 *
 *   qcodes  device pointer, nq x 2W uint32, canonical layout, encoded with the
 *           database's (d, x) (e.g. by tq_encode).
 *   ids     device pointer, nq x k int32 (written): database row numbers.
 *   scores  device pointer, nq x k int32 (written): Delta of each result.
 *   opts    may be NULL (automatic choices).
 *
 * Requires 1 <= nq, 1 <= k <= min(n, TQ_MAX_K).  Results are exact and
 * ordered as described at the top of this file, whatever path is used.
 * Asynchronous on `stream`. */
int tq_search_knn(const tq_db *db, const uint32_t *qcodes, int nq, int k, int32_t *ids,
                  int32_t *scores, const tq_search_opts *opts, void *stream);

/* tq_search_knn for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, hosts that forbid
 * it): the plain path only (opts->path AUTO or PLAIN; engine AUTO, POPCOUNT or
 * SPARSE; check_queries must be 0), with the same arguments, ownership and
 * results as tq_search_knn.  The scratch it needs (per query, grid x k 8-byte
 * keys plus a few rows) comes from a fixed 16 MiB device array inside the
 * library, one per GPU, held until the process ends; queries are processed in
 * rounds that fit it.  TQ_ERR_INVALID before anything is queued if one query
 * needs more than 16 MiB (only a grid above 4000 workgroups at k = 512, or
 * the like, can).  The call allocates nothing and times nothing; the first
 * call on a device looks up the array's device address.  Every such call on
 * one GPU shares the array: calls whose GPU work may overlap (other streams,
 * or other host threads on the same stream) race and must be serialised by
 * the caller. */
int tq_search_knn_noalloc(const tq_db *db, const uint32_t *qcodes, int nq, int k, int32_t *ids,
                          int32_t *scores, const tq_search_opts *opts, void *stream);

/* Time the candidate shapes of the batched path (query tile, workgroups) and
 * the plain path for every batch-size bucket (powers of two up to
 * min(nq_max, 1024)) and each of the nks values of k in `ks` (host array),
 * and remember the fastest per (d, k, bucket) for later TQ_PATH_AUTO and
 * TQ_PATH_BATCHED calls.  If the environment variable TQ_TUNE_CACHE names a
 * file, the results are also written there and read back by later processes.
 * Runs searches on `stream` and waits for them. */
int tq_autotune(const tq_db *db, int nq_max, const int *ks, int nks, void *stream);

/* ---------------------------------------------------------------------------
 * Masked addition (Sec. 5.1.2; the asymmetric variant of Sec. 6): k nearest
 * database codes of each of nq FLOAT queries, scored without encoding the
 * query: score(q, v) = sum of q_i where v+ is set - sum of q_i where v- is
 * set (the scalar product of q with the ternary v).  The two sums are taken
 * in double precision and rounded once to float; results are ordered by that
 * float score (larger first), the lower id on equal scores.  One database
 * pass per query, like TQ_PATH_PLAIN.
 *
 *   Q       device pointer, nq x d float32 (the database's d).
 *   ids     device pointer, nq x k int32 (written).
 *   scores  device pointer, nq x k float32 (written).
 *   opts    may be NULL; only opts->grid is used.
 *
 * Requires 1 <= nq, 1 <= k <= min(n, TQ_MAX_K).  Asynchronous on `stream`.
 * The summation order differs from a sequential one, so a score can differ
 * from the sequentially summed one in the last float bit when that sum lies
 * within ~1e-12 (relative) of a float rounding boundary. */
int tq_search_masked(const tq_db *db, const float *Q, int nq, int k, int32_t *ids, float *scores,
                     const tq_search_opts *opts, void *stream);

/* ---------------------------------------------------------------------------
 * Refinement of proxy candidates (the search behind the k@n recall of
 * Sec. 5.3): for each query, order its ncand candidate ids -- typically the
 * ids of tq_search_knn with k = n > the wanted k -- by the scalar product of
 * the original float vectors, and keep the best k.  For l2-normalised
 * embeddings (Sec. 1.1) that is the l2 order.  Products and sums are in
 * double precision; scores are written as doubles.  Order: larger score
 * first, the lower id on equal scores.
 *
 *   X       device pointer, n x d float32, row-major: the database vectors
 *           (the same floats that were encoded).
 *   Q       device pointer, nq x d float32: the queries.
 *   cand    device pointer, nq x ncand int32: candidate ids; an id outside
 *           [0, n) is ignored.  Ids of one query should be distinct.
 *   ids     device pointer, nq x k int32 (written); -1 where a query has
 *           fewer than k valid candidates.
 *   scores  device pointer, nq x k double (written); -infinity where ids
 *           holds -1.
 *
 * Requires n >= 1, 1 <= d <= TQ_MAX_D, nq >= 0, 1 <= ncand <= TQ_MAX_RERANK,
 * 1 <= k <= ncand; else TQ_ERR_INVALID before anything is queued.
 * Asynchronous on `stream`; reads each candidate row once (4d bytes). */
#define TQ_MAX_RERANK 1024
int tq_rerank(const float *X, int64_t n, int d, const float *Q, int nq, const int32_t *cand, int ncand, int k,
              int32_t *ids, double *scores, void *stream);

/* Debugging / parity aid: the full nq x n matrix of Delta(q_i, s_j)
 * (int32, row-major, device pointer), computed with the same device code as
 * the search.  Asynchronous on `stream`. */
int tq_delta_dump(const tq_db *db, const uint32_t *qcodes, int nq, int32_t *delta, void *stream);

/* Wait for `stream`, then report and clear the sticky device error flags of
 * the current device (TQ_ERR_INVALID after non-finite input to tq_encode). */
int tq_sync(void *stream);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching over a resident database                    */
/* ---------------------------------------------------------------------- */

typedef struct tq_server tq_server;

typedef struct tq_serve_cfg {
  uint64_t budget_bytes; /* device memory the in-flight requests may hold;
                            0 = 256 MiB */
  int max_slots;         /* most queries in flight at once; 0 = 4096 */
  int max_k;             /* largest k a request may ask for; 0 = 128 */
  int n_segments;        /* database segments per pass (a request needs one
                            tick per segment); 0 = one per 16M vectors */
  int max_request_nq;    /* largest nq of one request; 0 = 1024 */
  int tick_timeout_us;   /* watchdog: a tick whose GPU work has not finished
                            this many microseconds after it was queued stops
                            the server; its requests then report
                            TQ_ERR_DEVICE.  0 = no watchdog (the loop waits on
                            the GPU without polling) */
  int engine;            /* TQ_ENGINE_AUTO (the default choice per tick),
                            TQ_ENGINE_POPCOUNT or TQ_ENGINE_MATRIX (every tick
                            whose k allows it); results are identical */
  int reserved[2];
} tq_serve_cfg;

typedef struct tq_req_stats {
  uint64_t submit_ns;   /* CLOCK_MONOTONIC time stamps of the request's life */
  uint64_t admit_ns;
  uint64_t complete_ns; /* when the serve loop saw the results land on the host */
  int nq;
  int k;
  int ticks;            /* database segment passes the request took part in */
  int reserved;
} tq_req_stats;

/* Start a server over `db` (which must outlive the server).  The server owns a
 * host thread and a HIP stream of the database's device.  `cfg` may be NULL. */
int tq_serve_create(const tq_db *db, const tq_serve_cfg *cfg, tq_server **out);

/* Queue a request: nq query codes (host pointer, nq x 2W uint32, canonical
 * layout, copied before the call returns) and its k.  Thread-safe.  Returns
 * TQ_ERR_INVALID if nq, k or the request's memory need can never be served
 * under the server's configuration.  *ticket identifies the request. */
int tq_serve_submit(tq_server *srv, const uint32_t *qcodes_host, int nq, int k, uint64_t *ticket);

/* Collect a request.  TQ_OK: the results were copied to ids_host / scores_host
 * (host pointers, nq x k int32, same order as tq_search_knn), `st` (may be
 * NULL) filled, and the ticket retired.  TQ_ERR_AGAIN: not finished yet.
 * TQ_ERR_NOTFOUND: unknown or already collected ticket.  Thread-safe. */
int tq_serve_poll(tq_server *srv, uint64_t ticket, int32_t *ids_host, int32_t *scores_host,
                  tq_req_stats *st);

/* Like tq_serve_poll but blocks up to timeout_ms (< 0: no limit) for the
 * request to finish; TQ_ERR_AGAIN on time-out. */
int tq_serve_wait(tq_server *srv, uint64_t ticket, int timeout_ms, int32_t *ids_host,
                  int32_t *scores_host, tq_req_stats *st);

/* Cancel a request that has not been collected.  A pending request is dropped
 * at once; an admitted one finishes its current database pass and is then
 * discarded.  Afterwards the ticket is unknown (TQ_ERR_NOTFOUND). */
int tq_serve_cancel(tq_server *srv, uint64_t ticket);

/* Counters of a server (any pointer may be NULL). */
int tq_serve_stats(tq_server *srv, uint64_t *submitted, uint64_t *completed, uint64_t *ticks,
                   uint64_t *bytes_in_use);

/* Stop a server: stops admitting, lets admitted requests finish, cancels the
 * pending ones, joins the thread and frees everything.  NULL is accepted. */
int tq_serve_destroy(tq_server *srv);

/* ---------------------------------------------------------------------- */
/* Measurement                                                              */
/* ---------------------------------------------------------------------- */

/* The shader clock of the current device in MHz, measured while every compute
 * unit runs a chain of dependent vector instructions (the ratio of the
 * shader-clock and real-time counters read on the device).  Peaks quoted per
 * clock (vector ALU, matrix cores) scale with it.  Waits for `stream`. */
int tq_clock_mhz(double *mhz, void *stream);

/* Upper bound on the device memory the library holds at once -- resident
 * databases, search scratch, batched-path buffers and graphs' buffers,
 * servers -- in bytes; 0 (the default) means none.  An allocation that would
 * take the total past the bound fails as if the GPU were out of memory: the
 * call returns TQ_ERR_NOMEM (tq_db_create, tq_serve_create, searches that
 * need new scratch) and leaves nothing half-built.  Memory already held is
 * not released.  For processes that share a GPU, and for exercising the
 * out-of-memory paths in tests.  Process-wide, all devices together. */
int tq_set_device_limit(uint64_t bytes);

/* Device bytes the library holds at the moment (counted as for the limit). */
int tq_device_bytes(uint64_t *held);

/* Turn per-launch timing of the library's scan kernels on (1) or off (0).
 * When on, each scan launch is bracketed by HIP events on its own stream. */
int tq_timing_enable(int enable);

/* Sum of the timed scan-kernel durations since the last reset, and the number
 * of launches, for kernel family `which` (0 = plain scan, 1 = batched scan,
 * 2 = masked-addition scan, 3 = index-list scan).
 * Waits for the recorded events.  reset != 0 clears the counters. */
int tq_timing_read(int which, double *total_ms, int64_t *launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* TQ_H */
