/*
 * acbm.h -- libacbm: block-matching motion estimation with the adaptive cost
 * block matching (ACBM) method on AMD Instinct MI355X (gfx950).
 *
 * Method: S. Lopez, G.M. Callico, J.F. Lopez, R. Sarmiento, "A High
 * Quality/Low Computational Cost Technique for Block Matching Motion
 * Estimation".  Every entry point below names the section it computes.
 *
 * Conventions shared by all calls
 *  - Frames are 8-bit luma (Section 2.1: luminance values), row-major, with a
 *    row pitch in bytes.  The current frame is cut into block_w x block_h
 *    blocks (N x M, Section 1); block (r, c) starts at x = c*N, y = r*M.
 *  - A candidate vector (u, v) with |u|, |v| <= p is evaluated only when the
 *    displaced block lies wholly inside the reference frame (Section 1: the
 *    search area is contained in the previous frame).  (0, 0) is always valid.
 *  - SAD (Section 2.1, SAD equation) pairs the horizontal index with mv_x:
 *    SAD(u,v) = sum_{j<M, i<N} |cur[y0+j][x0+i] - ref[y0+j+v][x0+i+u]|.
 *  - Cost (Section 2.1): J = SAD + lambda * R, R = se(u - px) + se(v - py),
 *    se(k) = bits of the signed Exp-Golomb codeword of k (1 for k = 0, else
 *    2*floor(log2|k|) + 3), (px, py) the component-wise median of the final
 *    vectors of the left, top and top-right blocks (left missing -> (0,0);
 *    first block row -> top and top-right take the left value; last column ->
 *    top-right is (0,0)).
 *  - Minimum: smallest J, then smallest |u|+|v|, then the earlier window
 *    position in raster order (v outer, top-left first).  Results are unique
 *    and every call is bit-exact and deterministic.
 *  - Device pointers are HIP device memory owned by the caller.  `stream` is
 *    a hipStream_t (NULL = the null stream).  Calls are asynchronous on that
 *    stream: argument errors return synchronously before anything is
 *    enqueued; device failures surface on a later call or synchronisation.
 *  - GPU layout requirements: frame pointers and pitch 4-byte aligned,
 *    block_w and block_h in {8, 16}, p <= 127, and for the searches at most
 *    1024 block rows (height / block_h).  Other shapes the method allows
 *    return ACBM_E_UNSUPPORTED.
 */
#ifndef ACBM_H
#define ACBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACBM_VERSION "0.1.0"

/* ---- status codes ------------------------------------------------------ */
#define ACBM_OK              0
#define ACBM_E_INVAL        -1  /* null pointer, zero size, pitch < width, gamma_den = 0, bad enum */
#define ACBM_E_SHAPE        -2  /* width % N, height % M, p > 127                       */
#define ACBM_E_RANGE        -3  /* a cost or threshold would not fit the integer types  */
#define ACBM_E_NOMEM        -4  /* workspace too small / request larger than the pool   */
#define ACBM_E_DEVICE       -5  /* HIP error; detail in acbm_last_error()               */
#define ACBM_E_BUSY         -6  /* server queue full                                    */
#define ACBM_E_UNSUPPORTED  -7  /* valid for the method but not for this library/GPU    */
#define ACBM_E_TIMEOUT      -8  /* a wait ended before its result was ready             */

/* ---- searches and per-block outcomes ----------------------------------- */
#define ACBM_ALGO_FSBM  0   /* full search over the (2p+1)^2 window (Section 2.3) */
#define ACBM_ALGO_PBM   1   /* predictive search (Section 2.2)                    */
#define ACBM_ALGO_ACBM  2   /* adaptive choice between the two (Section 3.2)      */

#define ACBM_MODE_FSBM      0  /* full search                                  */
#define ACBM_MODE_PBM_C1    1  /* ACBM kept PBM: Intra_SAD + SAD < alpha + beta*Qp^2 */
#define ACBM_MODE_PBM_C2    2  /* ACBM kept PBM: SAD < gamma * Intra_SAD        */
#define ACBM_MODE_CRITICAL  3  /* ACBM ran the full search                      */
#define ACBM_MODE_PBM       4  /* plain PBM run                                 */

/* workspace queries */
#define ACBM_OP_SAD_TABLE  0
#define ACBM_OP_FSBM       1
#define ACBM_OP_PBM        2
#define ACBM_OP_ACBM       3

typedef struct acbm_geom {
    uint32_t width, height;   /* pixels                                 */
    uint32_t pitch;           /* bytes between rows, >= width           */
    uint32_t block_w;         /* N: block width  (pairs with mv_x)      */
    uint32_t block_h;         /* M: block height (pairs with mv_y)      */
    uint32_t p;               /* maximum displacement per component     */
} acbm_geom;

/* lambda: Lagrange multiplier (Section 2.1); qp: quantisation step of the
 * first ACBM test; alpha, beta, gamma = gamma_num/gamma_den: ACBM thresholds
 * (Section 3.2; the paper's values for 16x16 blocks are 1000, 8, 1/4,
 * Section 4).
 * subpel: 0 integer-pel, 1 half-pel precision (Section 2.2's refinement on
 * the half-pixel grid; Table 1's full search counts the 8 half-pel
 * positions around the integer winner).  With 1, every vector (results,
 * predictors, the previous field) is in half-pel units, rates are counted
 * in those units, half-pel samples of the reference follow H.263's bilinear
 * interpolation with averages rounded half up, FSBM adds the valid half-pel
 * neighbours of its integer winner, and the PBM refinement ring is one
 * half-pel step.  Requires p <= 63 (vectors stay within +-126). */
typedef struct acbm_params {
    uint32_t lambda, qp;
    uint32_t alpha, beta;
    uint32_t gamma_num, gamma_den;
    uint32_t subpel;
} acbm_params;

typedef struct acbm_mv {
    int16_t x, y;
} acbm_mv;

/* 32 bytes per block, row-major [by][bx]. */
typedef struct acbm_block_result {
    acbm_mv  mv;         /* chosen vector                                   */
    uint32_t sad;        /* its SAD                                         */
    uint32_t j;          /* its J = SAD + lambda*R                          */
    uint32_t rate_bits;  /* its R                                           */
    uint32_t cands;      /* candidate positions evaluated for this block   */
    uint32_t mode;       /* ACBM_MODE_*                                     */
    uint64_t intra_x;    /* N*M*Intra_SAD (exact; Section 3.1)              */
} acbm_block_result;

/* Block statistics of Section 3.1, 32 bytes per block, row-major [by][bx]. */
typedef struct acbm_block_stats {
    uint32_t sad_min;        /* smallest SAD over the valid window            */
    uint32_t valid;          /* number of valid candidates (the window)       */
    uint64_t sad_deviation;  /* sum over the valid window of SAD - sad_min    */
    uint64_t intra_x;        /* N*M*Intra_SAD (exact)                         */
    uint64_t reserved;       /* written as 0                                  */
} acbm_block_stats;

/* ---- library ------------------------------------------------------------ */
/* The paper's ACBM thresholds for a block size (Section 4 gives alpha =
 * 1000, beta = 8, gamma = 1/4, tuned for 16x16 macroblocks).  The paper
 * gives no values for other sizes; because Intra_SAD and SAD both grow with
 * the pixel count, alpha and beta are scaled by block_w*block_h/256 (integer
 * division: 250 and 2 for 8x8 blocks); gamma is a ratio of the two and stays
 * 1/4.  lambda, qp and subpel are copied.  Pure host code: no device is
 * touched.  Errors: ACBM_E_INVAL for a NULL out or a zero block size. */
int acbm_default_params(uint32_t block_w, uint32_t block_h, uint32_t lambda, uint32_t qp,
                        uint32_t subpel, acbm_params* out);

const char* acbm_version(void);
const char* acbm_strerror(int status);
/* Detail of the last failing call on this thread ("" if none). */
const char* acbm_last_error(void);
/* Checks that the current HIP device is gfx950 (ACBM_E_UNSUPPORTED if not)
 * and creates the side streams acbm_batch uses on it.  Optional: without it
 * they are created at the first batch that needs them, which a stream capture
 * in hipStreamCaptureModeGlobal refuses, so call it once per device before
 * capturing acbm_batch in that mode. */
int acbm_init(void);

/* Bytes of device workspace an operation needs for `npairs` frame pairs of
 * this geometry (0 for ACBM_OP_SAD_TABLE).  Returns ACBM_E_* on bad geometry. */
int acbm_workspace_size(int op, const acbm_geom* g, uint32_t npairs, size_t* bytes);

/* Device-detected status of the last predictive (PBM/ACBM) run that used
 * this workspace: 0 when every block finished, ACBM_E_TIMEOUT when a
 * dependency wait gave up (the results are then incomplete).  Enqueues a
 * small copy on `stream` and waits for the stream. */
int acbm_workspace_status(const void* ws, size_t ws_bytes, void* stream, int* status);

/* SAD table (Section 2.1, SAD equation; the full set of Section 2.3):
 * table[r][c][v+p][u+p] (u32, [by][bx][2p+1][2p+1]) = SAD of block (r,c) at
 * (u,v), or 0xFFFFFFFF where (u,v) is not a valid candidate.  No workspace. */
int acbm_sad_table(const acbm_geom* g, const uint8_t* cur, const uint8_t* ref,
                   uint32_t* table, void* stream);

/* Block statistics of one frame pair (Section 3.1, Intra_SAD and
 * SAD_deviation equations): for every block, over its full valid window,
 * SAD_min, the number of valid positions, SAD_deviation = sum of
 * |SAD(u,v) - SAD_min| (every term is >= 0) and IntraX = N*M*Intra_SAD.
 * out is caller-owned device memory of by*bx records.  No workspace, no
 * allocation; asynchronous on `stream`.  Errors: as acbm_sad_table. */
int acbm_sad_stats(const acbm_geom* g, const uint8_t* cur, const uint8_t* ref,
                   acbm_block_stats* out, void* stream);

/* FSBM for one frame pair (Section 2.3 with the cost of Section 2.1):
 * out[r][c] = the minimum of J over the valid window; cands = number of valid
 * positions; mode = ACBM_MODE_FSBM. */
int acbm_fsbm_frame(const acbm_geom* g, const acbm_params* prm, const uint8_t* cur,
                    const uint8_t* ref, acbm_block_result* out, void* ws, size_t ws_bytes,
                    void* stream);

/* PBM for one frame pair (Section 2.2).  Predictors: (0,0); the final vectors
 * of the left, top-left, top, top-right blocks of this run; prev_field (the
 * previous pair's vectors, [by][bx], NULL = all zero) at the co-located block
 * and its 8 neighbours.  Predictors that are not valid candidates are dropped,
 * repeats count once; the cheapest predictor is refined once over its valid
 * integer 8-neighbours.  mode = ACBM_MODE_PBM. */
int acbm_pbm_frame(const acbm_geom* g, const acbm_params* prm, const uint8_t* cur,
                   const uint8_t* ref, const acbm_mv* prev_field, acbm_block_result* out,
                   void* ws, size_t ws_bytes, void* stream);

/* ACBM for one frame pair (Section 3.2): Intra_SAD, then PBM; PBM's vector is
 * kept when Intra_SAD + SAD_PBM < alpha + beta*Qp^2 (mode 1) or else when
 * SAD_PBM < gamma*Intra_SAD (mode 2); otherwise the block is critical and the
 * full search runs with the same predictor (mode 3, cands = PBM's + window).
 * Comparisons are exact (both sides scaled by N*M). */
int acbm_acbm_frame(const acbm_geom* g, const acbm_params* prm, const uint8_t* cur,
                    const uint8_t* ref, const acbm_mv* prev_field, acbm_block_result* out,
                    void* ws, size_t ws_bytes, void* stream);

/* ACBM for one frame pair that allocates nothing, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * hosts that forbid hipMalloc).  Same arguments and results as
 * acbm_acbm_frame, without a workspace: the scratch (a dependency-wait
 * header, the row order, the published vector words and the job tables) is
 * a fixed 2 MiB device array inside the library, one per GPU, held until the
 * process ends; frames of more than about 520,000 blocks need more and are
 * rejected with ACBM_E_NOMEM before anything is enqueued.  Every call on a
 * GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * No hipMalloc, hipFree or allocating library call is made (acbm_init looks
 * the array up ahead of time; otherwise the first call on a device does).
 * status (device memory, may be NULL) receives 0 when every block finished,
 * or 1 when a dependency wait gave up (the results are then incomplete), in
 * stream order after the results. */
int acbm_acbm_frame_noalloc(const acbm_geom* g, const acbm_params* prm, const uint8_t* cur,
                            const uint8_t* ref, const acbm_mv* prev_field,
                            acbm_block_result* out, uint32_t* status, void* stream);

/* ---- batches of sequences ----------------------------------------------- */
/* A job is one sequence: frame t-1 is the reference of frame t, so nframes
 * frames give nframes-1 pairs; PBM/ACBM take pair t-1's field as pair t's
 * temporal neighbourhood (Section 2.2), zero for the first pair.  frames is a
 * HOST array of nframes DEVICE pointers; out is device memory of
 * (nframes-1)*by*bx results. */
typedef struct acbm_job {
    acbm_geom geom;
    acbm_params params;
    uint32_t algo;                 /* ACBM_ALGO_*                     */
    uint32_t nframes;              /* >= 2                            */
    const uint8_t* const* frames;  /* host array of device pointers   */
    acbm_block_result* out;        /* device                          */
} acbm_job;

int acbm_batch_workspace_size(const acbm_job* jobs, size_t njobs, size_t* bytes);
/* Runs every job; all work is enqueued on `stream` and the call returns
 * without waiting.  Results are identical to running each pair through the
 * *_frame calls in order.  FSBM jobs (Section 2.3) are grouped by block size
 * and window-search plan; each group is one persistent full-search launch
 * over all (job, pair, block) items of its jobs plus one resolve launch
 * with a workgroup per pair, reading job tables that small kernels write
 * into `ws` first.  PBM/ACBM jobs (Sections 2.2, 3.2) are grouped by block
 * size and precision, at most 256 jobs a group; each group is one row-walker
 * launch whose walkers take the block rows of all its jobs in level order
 * (row r of pair t has level r + 2t), so the dependency chains of the jobs
 * run side by side.  A PBM/ACBM job of more than 4095 pairs runs alone.
 * When `stream` belongs to the current device, the walker launches go to up
 * to four side streams of that device (created by the library on first use
 * and kept until the process ends), forked off `stream` after the tables are
 * written and joined back into it before the call returns: the call stays
 * ordered on `stream`, and a capture of `stream` records them as parallel
 * branches.  ACBM_BATCH_STREAMS (0 to 4) caps the side streams; 0 keeps
 * every launch on `stream`.  Concurrent calls from several host threads are
 * serialised while they enqueue.
 * ws must hold acbm_batch_workspace_size bytes (per-job scratch plus the
 * tables) and must not be shared by overlapping calls. */
int acbm_batch(const acbm_job* jobs, size_t njobs, void* ws, size_t ws_bytes, void* stream);

/* Device-detected status of the last acbm_batch (or batch graph launch) of
 * these jobs on `ws`, as acbm_workspace_status reports it for one job: 0
 * when every PBM/ACBM block finished, ACBM_E_TIMEOUT when a dependency wait
 * of any walker gave up.  `jobs` must describe the same batch (the layout
 * of `ws` follows from it).  Enqueues small copies on `stream` and waits for
 * the stream. */
int acbm_batch_status(const acbm_job* jobs, size_t njobs, const void* ws, size_t ws_bytes,
                      void* stream, int* status);

/* A batch recorded once as a HIP graph and replayed with one launch.
 * create: validates like acbm_batch, then records exactly the sequence
 *   acbm_batch enqueues (job-table writes, the persistent FSBM groups, the
 *   PBM/ACBM walker groups) on a private stream and instantiates it.  Frame
 *   pointers, `out` arrays, parameters and `ws` are baked in: they must stay
 *   allocated at the same addresses for the graph's lifetime (their contents
 *   may change between launches).  The graph holds only kernel nodes (no
 *   memset or copy nodes).  create synchronises nothing but is not meant for
 *   a hot loop or for use while the calling thread captures another stream.
 *   Errors: as acbm_batch, ACBM_E_DEVICE if recording fails.
 * launch: enqueues the whole batch on `stream` (one hipGraphLaunch) and
 *   returns without waiting; results are identical to acbm_batch.  Launches
 *   of one graph must not overlap (they share `ws`).
 * destroy: call after the last launch has completed. */
typedef struct acbm_batch_graph acbm_batch_graph;
int acbm_batch_graph_create(const acbm_job* jobs, size_t njobs, void* ws, size_t ws_bytes,
                            acbm_batch_graph** out);
int acbm_batch_graph_launch(acbm_batch_graph* gr, void* stream);
int acbm_batch_graph_destroy(acbm_batch_graph* gr);

/* ---- autotuning --------------------------------------------------------- */
/* Times the full-search plans of one (block_w, block_h, p) on this device
 * (every candidate row blocking R that fits, on a synthetic frame pair of
 * g's size, after one warm-up) and makes the fastest the plan every later
 * search of that shape uses (process-wide; acbm_sad_table, acbm_fsbm_frame,
 * acbm_batch and graphs created afterwards).  The environment variable
 * ACBM_R still overrides.  Results never depend on the plan, only time does.
 * best_rows and best_ms (may be NULL) receive the chosen R and its time per
 * pair in milliseconds.  Allocates and frees scratch device memory and
 * synchronises `stream`.  Errors: as acbm_fsbm_frame's geometry checks,
 * ACBM_E_DEVICE. */
int acbm_autotune(const acbm_geom* g, uint32_t* best_rows, float* best_ms, void* stream);

/* ---- kernel timing ------------------------------------------------------ */
/* When enabled, every kernel the library launches is bracketed by HIP events
 * on the stream it runs on.  acbm_profile_read waits for the recorded events
 * and returns the summed device time and the launch count of one kernel
 * since the last reset.  Kernel names: "search" (window search, all block
 * sizes), "stats" (block statistics), "half" (half-pel SADs around single
 * possible winners), "resolve" (FSBM argmin), "predictive" (PBM/ACBM),
 * "setup" (predictive workspace set-up), "field" (served field extraction). */
int acbm_profile_enable(int on);
int acbm_profile_reset(void);
int acbm_profile_read(const char* kernel, double* total_ms, uint64_t* launches);

/* ---- serving ------------------------------------------------------------ */
/* Continuous batching of frame-pair requests over video streams whose
 * reference frame and motion field stay on the device.  A worker thread
 * gathers every queued request that can run now -- in submit order, one per
 * stream at a time (pair t needs pair t-1's frame and field), while the
 * requests on the GPU stay within max_inflight and the pass's results and
 * workspace fit in the largest free block of the pool -- into one pass on
 * one of `lanes` HIP streams: the frame uploads, the batched searches of
 * acbm_batch (one full-search launch per search class and one resolve for
 * the FSBM requests, one row-walker launch per block size for the PBM/ACBM
 * requests), the stored fields and one download of the results.  Requests
 * that arrive meanwhile join the next pass, and passes on different lanes
 * overlap on the device.  A request's result equals the *_frame call on
 * that pair, whatever it was batched with. */
typedef struct acbm_serve_cfg {
    size_t   pool_bytes;    /* device memory the server owns (frames, fields, results, workspace) */
    uint32_t max_streams;   /* video streams that can be open at once      */
    uint32_t max_inflight;  /* requests on the GPU at once, over all passes */
    uint32_t queue_depth;   /* requests waiting for admission              */
    uint32_t lanes;         /* passes in flight at once (HIP streams), 0 = 4, at most 16 */
    size_t   pinned_bytes;  /* pinned host staging for frames and results, 0 = 512 MiB; frames
                               take at most three quarters (beyond it they wait in host memory) */
} acbm_serve_cfg;

typedef struct acbm_serve_report {
    uint64_t completed, rejected;
    double   p50_us, p99_us, mean_us;   /* submit -> result ready on the host         */
    double   throughput_rps;            /* completed / (last done - first submit)     */
    double   device_busy_frac;          /* union of the passes' device intervals (HIP
                                           timing events around each pass) over the
                                           span from the first pass start to the last end */
    double   device_busy_ms;            /* that union in milliseconds                 */
    uint64_t passes;                    /* passes completed                           */
    double   mean_batch;                /* computed requests per pass                 */
} acbm_serve_report;

typedef struct acbm_server acbm_server;

int acbm_serve(const acbm_serve_cfg* cfg, acbm_server** out);
/* Submits the next frame of a video stream (host memory, copied before the
 * call returns).  The first frame of a stream only becomes its resident
 * reference (the ticket completes with no results); every later frame is
 * estimated against the stream's previous frame, which stays on the device.
 * Returns ACBM_E_BUSY when the queue is full, ACBM_E_NOMEM when the request
 * can never fit the pool. */
int acbm_serve_submit(acbm_server* s, uint32_t stream_id, const uint8_t* host_frame,
                      const acbm_geom* g, const acbm_params* prm, uint32_t algo,
                      uint64_t* ticket);
/* Waits for a ticket; copies by*bx results to host_out (may be NULL).
 * timeout_us < 0 waits forever; ACBM_E_TIMEOUT if not ready in time. */
int acbm_serve_wait(acbm_server* s, uint64_t ticket, acbm_block_result* host_out,
                    int64_t timeout_us);
/* Latency percentiles and throughput of every request completed so far. */
int acbm_serve_stats(acbm_server* s, acbm_serve_report* st);
/* The same as acbm_serve_stats (an older name, kept). */
int acbm_serve_stats_get(acbm_server* s, acbm_serve_report* st);
int acbm_serve_close(acbm_server* s);

#ifdef __cplusplus
}
#endif
#endif
