/* ph0.h -- C ABI of the MI355X (gfx950) library for 0th persistent homology
 * (H0) barcodes of integer point clouds.
 *
 * The computation is the barcode algorithm of Section 2 of Rawson, "Linear
 * Run Time of Persistent Homology Computation with GPU Parallelization",
 * in the five GPU steps of Section 4:
 *   1. squared Euclidean distance of every pair i < j of the N points;
 *   2. sort the N(N-1)/2 edges by distance (ties: by larger endpoint j, then
 *      by i);
 *   3. remove duplicate distances to get D; an edge's grade is the 1-based
 *      index of its distance in D;
 *   4. column-reduce the N x N(N-1)/2 vertex-by-edge boundary matrix over F2,
 *      left to right, until every nonzero column has a distinct lowest entry
 *      (the low of a column is its largest row index);
 *   5. each surviving pivot of grade b is the interval (0, b); the vertex whose
 *      row never becomes a pivot (vertex 0) is the one infinite interval.
 *
 * All arithmetic is integer, so results are exact and deterministic: the same
 * input gives bit-identical output whatever the stream, batch or concurrency.
 *
 * Conventions for every entry point:
 *   - Return value: PH0_OK (0) or a negative ph0_status; on error the output
 *     buffers hold unspecified data and ph0_last_error() describes the cause.
 *   - Points are row-major N x d arrays of int8 (PH0_I8) or int16 (PH0_I16).
 *   - The caller owns every buffer it passes; the library keeps no pointer
 *     after a call returns.
 *   - Calls with host pointers block until their results are in host memory.
 *     Calls taking a `hip_stream` (a hipStream_t, NULL = the null stream)
 *     enqueue their work on that stream and also return only after it is
 *     complete (the reduction is steered from the host between rounds).
 */
#ifndef PH0_H
#define PH0_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PH0_INF 0xFFFFFFFFu /* death of the essential (never dying) class */

typedef enum { PH0_I8 = 1, PH0_I16 = 2 } ph0_dtype;

typedef enum {
  PH0_OK = 0,
  PH0_EINVAL = -1,  /* NULL pointer, n < 1, d < 1, bad dtype, small workspace */
  PH0_ERANGE = -2,  /* the packed 64-bit sort key cannot hold distance + edge id */
  PH0_ENOMEM = -3,  /* device or host allocation failed, or a budget is full */
  PH0_EDEVICE = -4, /* a HIP call failed or a kernel reported an inconsistency */
  PH0_EBUSY = -5    /* serving: the request was not admitted now; retry later */
} ph0_status;

/* One barcode interval (birth, death) in grade units: birth is always 0,
 * death is the grade b (1-based index in D) or PH0_INF. */
typedef struct {
  uint32_t birth;
  uint32_t death;
} ph0_bar;

/* Counters and stage timings of one call.  Times are GPU event times in ms
 * (0 when not measured). */
typedef struct {
  int64_t n;             /* points */
  int64_t E;             /* edges N(N-1)/2 */
  int64_t E_eff;         /* sorted position of the last pivot + 1 */
  int64_t distinct_eff;  /* |D| restricted to the first E_eff sorted edges */
  int64_t additions;     /* column additions of columns < E_eff (the sequential count) */
  int64_t additions_all; /* column additions performed, incl. columns >= E_eff */
  int64_t find_steps;    /* root look-ups made by the parallel commit rule */
  int64_t words_read;    /* pivot-table entries (4 bytes each) loaded by the reduction */
  int64_t rounds;        /* reduction rounds (walk, decide, commit), including rounds that
                            found nothing to do while the next distance range was sorted */
  int64_t window;        /* columns reduced side by side in one round */
  int32_t sort_passes;   /* LSD radix passes over the distance bits */
  int32_t delta_bits;    /* bits of the squared-distance bound */
  int32_t index_bits;    /* bits per vertex index in the packed key */
  int32_t keys_path;     /* 0 = vector ALU distances, 1 = int8 MFMA Gram */
  float ms_keys, ms_sort, ms_reduce, ms_rank, ms_emit, ms_total;
  /* Kernel-level event times (sum over launches) and launch counts. */
  float ms_walk_kernel;    /* reduction walk kernel (one launch per round) */
  float ms_radix_kernel;   /* LSD radix pass kernel (one launch per pass) */
  int32_t walk_launches;
  int32_t radix_launches;
  int32_t sort_chunks;     /* distance ranges sorted (1 = only the first) */
  int32_t reserved;
  int64_t sorted_keys;     /* keys put in sorted order: the sorted prefix length */
} ph0_stats;

/* Message for the last non-OK status returned on this thread. */
const char* ph0_last_error(void);

/* Device workspace needed by ph0_barcodes_device / ph0_pairs_device for a
 * cloud of n points in d dimensions.  Returns EINVAL / ERANGE like those
 * calls would.  The size is dominated by two 8-byte keys per edge. */
int ph0_workspace_bytes(int64_t n, int32_t d, ph0_dtype dt, size_t* bytes);

/* The whole barcode, host memory in and out.  `out` receives n bars sorted
 * by death ascending, PH0_INF last (the canonical barcode).  `st` may be NULL.
 * Allocates and frees its own device memory. */
int ph0_barcodes(const void* points, ph0_dtype dt, int64_t n, int32_t d, ph0_bar* out,
                 ph0_stats* st);

/* The whole barcode on device memory: d_points (n*d elements), d_out (n bars,
 * canonical order), d_workspace of at least ph0_workspace_bytes() bytes.  No
 * device allocation is made.  `st` may be NULL.  With st NULL, clouds with
 * n <= 256, n * d <= 8192 and d <= 64 run in one workgroup (the fused kernel
 * of the batched path); with st given they take the grid-wide passes, which
 * report the counters.  The barcode is the same either way. */
int ph0_barcodes_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d,
                        ph0_bar* d_out, void* d_workspace, size_t ws_bytes,
                        void* hip_stream, ph0_stats* st);

/* Real-valued points (the paper's workload, Section 4.1: points drawn
 * uniformly from the unit square).  The barcode is defined on exact integer
 * distances, so the coordinates are first put on the int16 grid
 * q = rint((x - lo) * 32767 / (hi - lo)), computed in double precision (one
 * subtraction, one multiplication by the host-computed factor
 * 32767 / (hi - lo), rounding half to even), and the grid cloud's barcode is
 * returned: the same as ph0_barcodes_device on those int16 points (its
 * grades are indices of the grid's distinct squared distances).  The order
 * of two real distances is kept except where they differ by less than the
 * grid's resolution.  d_points: n*d row-major floats in device memory;
 * every coordinate must lie in [lo, hi] (finite lo < hi), else EINVAL (the
 * call checks on the device and waits for that check).  d_workspace: at
 * least ph0_workspace_bytes_f32() bytes, not allocated by the call.  `st`
 * as in ph0_barcodes_device; EINVAL / ERANGE as ph0_barcodes_device on the
 * grid cloud. */
int ph0_workspace_bytes_f32(int64_t n, int32_t d, size_t* bytes);
int ph0_barcodes_f32_device(const float* d_points, int64_t n, int32_t d, double lo, double hi,
                            ph0_bar* d_out, void* d_workspace, size_t ws_bytes,
                            void* hip_stream, ph0_stats* st);

/* Per-vertex detail of the same computation (device pointers, any may be NULL):
 *   d_death_by_vertex[n] grade at which vertex r dies, PH0_INF for vertex 0
 *   d_killer_pos[n]      sorted position of the edge whose column became the
 *                        pivot of row r, -1 for vertex 0
 *   d_killer_edge[n]     that edge as (j << 32) | i, i < j; UINT64_MAX if none
 *   d_killer_sqdist[n]   its squared distance D[b]; -1 if none
 *   d_partner[n]         the other nonzero row of the reduced column stored
 *                        as the pivot of row r (it has exactly two), -1 if none
 * Vertex r != 0 dies when the component whose smallest vertex is r joins a
 * component with a smaller smallest vertex. */
int ph0_pairs_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d,
                     uint32_t* d_death_by_vertex, int64_t* d_killer_pos,
                     uint64_t* d_killer_edge, int64_t* d_killer_sqdist, int32_t* d_partner,
                     void* d_workspace, size_t ws_bytes, void* hip_stream, ph0_stats* st);

/* Step 1 alone: the packed keys (delta << 2b | j << b | i, b = index_bits) of
 * all edges i < j at colex position j(j-1)/2 + i.  d_keys holds E entries. */
int ph0_keys_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d,
                    uint64_t* d_keys, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* Steps 1-2: the packed keys in sorted (delta, j, i) order.  d_keys holds E. */
int ph0_sorted_keys_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d,
                           uint64_t* d_keys, void* d_workspace, size_t ws_bytes,
                           void* hip_stream);

/* Key layout the library would use: bits per vertex index (b) and bits of the
 * squared-distance bound.  Returns ERANGE when 2b + delta_bits > 64. */
int ph0_key_layout(int64_t n, int32_t d, ph0_dtype dt, int32_t* index_bits,
                   int32_t* delta_bits);

/* ---- Many clouds in one launch ---------------------------------------- */

/* Speed-only tuning of the batched path (never changes results).  A zero
 * field takes the built-in value; the built-in values (chunk_mult 6, 6, 8,
 * 48; two workgroups per CU; 8-bit digits; 8 waves per cloud) are those the
 * package's autotuner (paper_2203_02527_amd/autotune.py) measured best on
 * MI355X, which writes them to a table the Python binding passes by
 * default.  digit_bits outside 0..8 or waves_per_cloud other than 0, 8 or 16
 * is EINVAL. */
typedef struct {
  int32_t chunk_mult[4];    /* first sorted chunk holds about chunk_mult * n edges,
                               per cloud size bucket n <= 64, <= 128, <= 256, <= 512 */
  int32_t blocks_per_cu;    /* workgroups launched per compute unit (1 or 2) */
  int32_t digit_bits;       /* digit width of the chunk's radix passes (1..8) */
  int32_t waves_per_cloud;  /* waves of the workgroup that runs a cloud (8 or 16) */
} ph0_batch_tuning;

/* Device workspace for ph0_barcodes_batched_device on these clouds.
 * offsets: host array of nclouds + 1 row offsets into the concatenated
 * points (offsets[0] = 0, non-decreasing). */
int ph0_batched_workspace_bytes(const int64_t* offsets, int64_t nclouds, int32_t d,
                                ph0_dtype dt, const ph0_batch_tuning* tune, size_t* bytes);

/* Barcodes of nclouds clouds in one persistent launch.  d_points holds the
 * clouds' rows back to back (offsets[nclouds] x d, device); cloud c owns rows
 * offsets[c] .. offsets[c+1]-1 and gets its canonical barcode in the same
 * rows of d_out (offsets[nclouds] bars, device).  Each workgroup takes whole
 * clouds from a work queue, largest first, with its pivot table in LDS.
 * Clouds with n > 512 or n * d > 8192 run through the single-cloud path after
 * the launch.  Results are identical to ph0_barcodes_device on each cloud.
 * `tune` and `st` may be NULL. */
int ph0_barcodes_batched_device(const void* d_points, ph0_dtype dt, const int64_t* offsets,
                                int64_t nclouds, int32_t d, ph0_bar* d_out, void* d_workspace,
                                size_t ws_bytes, const ph0_batch_tuning* tune,
                                void* hip_stream, ph0_stats* st);

/* The same batched computation on host memory: points (offsets[nclouds] x d
 * rows, host), out (offsets[nclouds] bars, host; cloud c's canonical barcode
 * in rows offsets[c] .. offsets[c+1]-1).  The library allocates its device
 * buffers (points, bars, workspace) and a stream, copies in, runs
 * ph0_barcodes_batched_device, copies out and frees everything before it
 * returns.  tune_json (NULL = built-in table) is a JSON object with only the
 * members "chunk_mult" (up to four non-negative integers, per size bucket as
 * in ph0_batch_tuning), "blocks_per_cu", "digit_bits" and "waves_per_cloud"
 * (non-negative integers, ranges as in ph0_batch_tuning); zero means
 * built-in.  Any other member, or malformed text, is EINVAL before any
 * device call.  `st` may be NULL.  Errors as ph0_barcodes_batched_device, and
 * ENOMEM when the device allocation fails. */
int ph0_barcodes_batched(const void* points, ph0_dtype dt, const int64_t* offsets,
                         int64_t nclouds, int32_t d, ph0_bar* out, const char* tune_json,
                         ph0_stats* st);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same batched
 * computation as ph0_barcodes_batched_device, with no workspace argument.
 * Its workspace is a fixed 128 MiB device array inside the library (one per
 * device, held from the library's load until the process ends); the call
 * makes no device or pinned-host allocation and no hipFree.
 *   - Only clouds the fused kernel takes are accepted: every cloud needs
 *     n <= 512, n * d <= 8192 and d <= 64, otherwise EINVAL (nothing runs).
 *   - The workgroup count is lowered until 20 * emax bytes per workgroup
 *     (emax = n(n-1)/2 of the largest cloud) plus 16 bytes per cloud fit the
 *     array; when even one workgroup does not fit (more than about 8 million
 *     clouds), ENOMEM (nothing runs).
 *   - All calls on one device share the array: calls that overlap on one
 *     device (two host threads, or two streams without an ordering between
 *     them) race and give undefined results.  Each call clears what must
 *     start at zero, so sequential calls are independent.
 * Returns after the work is complete, like the other stream calls.  Results
 * are identical to ph0_barcodes_batched_device on the same clouds. */
int ph0_barcodes_batched_device_noalloc(const void* d_points, ph0_dtype dt,
                                        const int64_t* offsets, int64_t nclouds, int32_t d,
                                        ph0_bar* d_out, const ph0_batch_tuning* tune,
                                        void* hip_stream);

/* ---- Serving: continuous batching of independent requests -------------- */

/* A server owns one device memory pool of mem_budget_bytes and up to
 * max_slots request slots, each a host worker thread with its own HIP stream.
 * A request is admitted only when a slot is free and its device footprint
 * (points + bars + ph0_workspace_bytes) fits in the pool, so admission is by
 * memory; admitted requests run concurrently on their streams and overlap on
 * the device.  Results are bit-identical to ph0_barcodes on the same cloud. */
typedef struct ph0_server ph0_server;

int ph0_server_create(size_t mem_budget_bytes, int32_t max_slots, ph0_server** srv);

/* Device bytes a request of this shape reserves while it runs. */
int ph0_server_request_bytes(int64_t n, int32_t d, ph0_dtype dt, size_t* bytes);

/* Offer one cloud (host memory, copied before return).  Returns PH0_OK when
 * admitted, PH0_EBUSY when no slot or not enough pool memory is free now
 * (retry later), PH0_ENOMEM when it could never fit the pool, or EINVAL. */
int ph0_server_submit(ph0_server* srv, const void* points, ph0_dtype dt, int64_t n, int32_t d,
                      uint64_t tag);

/* Non-blocking.  Returns 1 and fills tag / status / n_out (and up to out_cap
 * bars of the canonical barcode into out) for one finished request, or 0 when
 * none is finished.  status is the request's ph0_status. */
int ph0_server_poll(ph0_server* srv, uint64_t* tag, int32_t* status, ph0_bar* out,
                    int64_t out_cap, int64_t* n_out);

/* Requests admitted and not yet polled. */
int64_t ph0_server_in_flight(ph0_server* srv);

/* Waits for running requests, then frees the server. */
void ph0_server_destroy(ph0_server* srv);

/* ---- H1: 1st persistent homology of the same filtration ----------------
 *
 * The higher-dimension repetition of the algorithm that Section 3 anticipates
 * (and the conclusion leaves to future work), on the 2-skeleton of the same
 * Vietoris-Rips filtration:
 *   - edges in the order and with the grades of the H0 computation;
 *   - a triangle enters with its latest edge (the last of its three edges in
 *     that order) and carries that edge's grade; triangles are ordered by
 *     (latest edge, third vertex);
 *   - the edge-by-triangle boundary matrix is column-reduced over F2 left to
 *     right (low = largest edge position); a reduced column with low e pairs
 *     edge e with the triangle, the interval [grade(e), grade(triangle)).
 * The complete 2-skeleton has no H1, so exactly E - n + 1 pairs exist and no
 * interval is infinite; pairs of length 0 are not bars.  n <= 512 (stored
 * columns are dense bitsets of E = n(n-1)/2 bits); larger n gives ERANGE. */
typedef struct {
  int64_t E;            /* edges n(n-1)/2 */
  int64_t T;            /* triangles n(n-1)(n-2)/6 */
  int64_t pivots;       /* pairs found: E - n + 1 */
  int64_t emergent;     /* pairs of a triangle with its own latest edge, stored unreduced */
  int64_t bars;         /* pairs of positive length */
  int64_t zero_length;  /* pairs of length 0 */
  int64_t additions;    /* column additions of the reduction (every column reduced) */
  int64_t rounds;       /* reduction rounds */
  int64_t walks;        /* column walks, counting repeats (each round's, and commits') */
  float ms_setup, ms_reduce, ms_total;  /* GPU event times when measured, else 0 */
  int32_t reserved;
} ph0_h1_stats;

/* Device workspace for ph0_h1_device (dominated by E x ceil(E/64) words of
 * stored columns, 20 bytes per triangle, and a store of up to 16 GB that
 * keeps survivors' partly reduced columns). */
int ph0_h1_workspace_bytes(int64_t n, int32_t d, ph0_dtype dt, size_t* bytes);

/* H1 barcode on device memory.  d_bars receives the bars (birth < death, in
 * grade units) sorted by (birth, death) and must hold E - n + 1 entries (the
 * most there can be); *n_bars (host) receives their number.  d_tri_of_edge
 * (E entries, may be NULL) receives, for the edge at each sorted position,
 * the index in triangle order of the triangle it pairs with, or -1.  `st` may
 * be NULL.  Blocks until done. */
int ph0_h1_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d, ph0_bar* d_bars,
                  int64_t* d_tri_of_edge, int64_t* n_bars, void* d_workspace, size_t ws_bytes,
                  void* hip_stream, ph0_h1_stats* st);

/* Base reduction window (columns reduced side by side per round, rounded up
 * to a power of two); 0 restores the built-in choice, max(65536, 4 n) capped
 * at E.  Values above 2^26 columns are taken as 2^26 (window positions are
 * kept as 32-bit offsets).  A round widens the window up to 16 times the base
 * while almost every column of the previous round became final, and narrows
 * it back when many stay.  Affects speed and workspace size only, never
 * results.  Process-wide. */
int ph0_set_window(int64_t columns);


#ifdef __cplusplus
}
#endif

#endif /* PH0_H */
