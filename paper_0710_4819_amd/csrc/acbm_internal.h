// acbm_internal.h -- host-side declarations shared by the libacbm sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/acbm.h"

namespace acbm {

// Geometry as the kernels see it.
struct KGeom {
  int width, height, pitch;
  int bw, bh, p;
  int bx, by, nb;
};

// Per-block record written by the full-search pass for the FSBM resolve:
// the block's SAD minimum, how many candidates can still win (their SAD is
// within lambda*(Rmax-2) of the minimum, see the pruning bound in the
// resolve kernel), IntraX, and, when at most kShort can win, those
// candidates packed as (SAD << 16 | window raster index).  When more can
// win, the record's list is unused and the block's overflow region holds
// all of them in the same packing, or, if even that does not fit, the
// block's whole row of SADs.
constexpr int kShort = 28;
struct BlockRec {
  uint32_t sad_min, count, intra_x, pad;
  uint32_t e[kShort];
};
static_assert(sizeof(BlockRec) == 128, "record is two cache lines of 64 B");

// Frame pointers of one launch: pair k uses f[k] as reference and f[k+1] as
// current frame.
constexpr int kMaxPairsPerLaunch = 64;
struct FramePtrs {
  const uint8_t* f[kMaxPairsPerLaunch + 1];
};

// Shape of a block's search window in LDS (see window_shape in
// acbm_device.h): rows y0-p .. of dws dwords starting at x0 + u_lo; the lane
// work unit is one quad of candidates x R candidate rows.
struct WindowShape {
  int p, u_lo;
  int quads;   // QX: quads per window row of candidates
  int groups;  // row groups of R candidate rows
  int rows;    // LDS rows (>= groups*R + M - 1)
  int dws;     // dwords per LDS row (>= quads + N/4)
  int stride;  // LDS row stride in dwords
  // ceil(2^32 / quads) and ceil(2^32 / dws): t / d == umulhi(t, magic)
  // exactly for every t < 2^16 and d < 2^8 (checked exhaustively); imagic the
  // same for the quads that hold no padding candidate (see task_of)
  uint32_t qmagic, dmagic, imagic;
};

// One FSBM job of a batch as the batch kernels read it (device memory).
// Search items are (pair, block) in pair-major order (with a tiled plan
// (pair, 2x2 tile of blocks), and `s` is the tile's 16x16 window shape),
// numbered from item0 within the job's search group; resolve workgroups, one per pair, are
// numbered from pair0 across all FSBM jobs of the batch.
struct BatchJob {
  KGeom g;
  WindowShape s;
  const uint8_t* const* frames;  // [npairs + 1] device pointers
  BlockRec* recs;                // [npairs][nb]
  uint16_t* ovf;                 // [npairs][nb][(2p+1)^2]
  acbm_block_result* out;        // [npairs][nb]
  uint32_t* mv_ws;               // [npairs][nb] resolve state if it does not fit in LDS, else null
  uint32_t slack, lam, npairs;
  uint32_t item0, pair0;
  uint32_t subpel;               // half-pel precision (vectors in half-pel units)
};

// Launch plan of the window search for one (N, M, p).  tile = 2: a
// workgroup searches a 2x2 tile of 8x8 blocks over the tile's 16x16 window
// (R, threads and lds_bytes are then those of the 16x16 window shape).
struct SearchPlan {
  int R;        // candidate rows per lane
  int threads;  // workgroup size (multiple of 64, >= tasks)
  int lds_bytes;
  int tile = 1;
};

// Workspace layout (all offsets 256-byte aligned).
struct WsHeader {
  uint32_t status;      // 0 ok, else a device-detected failure code
  uint32_t ticket;      // work counter of the dataflow kernel
  uint32_t pad[62];
};
static_assert(sizeof(WsHeader) == 256, "header is 256 bytes");

constexpr uint32_t kStatusSpinTimeout = 1;

size_t align256(size_t x);
int rate_max(int p);  // 2 * se_bits(2p)
uint32_t fsbm_slack(int p, const acbm_params& prm);
int lds_limit();      // dynamic LDS bytes a workgroup may use on this device

// Set the thread's error detail and return `code`.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// Validation shared by every entry point.
int check_geom(const acbm_geom* g, KGeom* k);
int check_params(const acbm_params* prm, const KGeom& k);
int check_frame_ptr(const void* p, const char* what);
int check_device();

// The window shape the search kernels use for (N, M, p, R).
WindowShape window_shape_host(int N, int M, int p, int R);
// Plan of the one-block-per-workgroup search (SAD tables, statistics, and
// FSBM where 2x2 tiles do not apply).
SearchPlan plan_search(int N, int M, int p, int max_threads = 1024);
// Whether the FSBM search of this geometry runs in 2x2 tiles of 8x8 blocks
// (8x8 blocks, an even number of block columns and rows; ACBM_SEARCH_TILES=0
// turns tiles off).
bool tiles_apply(const KGeom& g);
// The FSBM search plan of a geometry: tiled where tiles apply.
SearchPlan plan_fsbm_search(const KGeom& g);
// Plans by the cost model only (the candidates the autotuner times); tile 2
// plans a 2x2 tile of 8x8 blocks (N = M = 8).
SearchPlan plan_search_model(int N, int M, int p, int R, int tile = 1);
// Records a measured plan for (N, M, p, tile); the planners return it from
// then on.
void set_tuned_plan(int N, int M, int p, const SearchPlan& pl);
// The same, also appended to the tuning cache file (ACBM_TUNE_CACHE) with its
// measured time per pair, when that variable names one.
void save_tuned_plan(int N, int M, int p, const SearchPlan& pl, float ms);
// A plan for (N, M, p, tile) read from the tuning cache file, with its time.
bool cached_plan(int N, int M, int p, int tile, SearchPlan* pl, float* ms);

// Brackets one kernel launch with timing events when profiling is on
// (acbm_profile_enable); a no-op otherwise.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t st);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* name_;
  hipStream_t st_;
  void* a_ = nullptr;
};

// Launchers.  All enqueue on `s` and return ACBM_* codes.
int launch_sad_stats(const KGeom& g, const uint8_t* cur, const uint8_t* ref,
                     acbm_block_stats* out, hipStream_t st);
int launch_sad_table(const KGeom& g, const uint8_t* cur, const uint8_t* ref, uint32_t* table,
                     hipStream_t s);
size_t fsbm_ws_bytes(const KGeom& g, uint32_t npairs);
int launch_fsbm(const KGeom& g, const acbm_params& prm, const uint8_t* const* frames,
                uint32_t npairs, void* ws, size_t ws_bytes, acbm_block_result* out,
                hipStream_t s);
// Window search with an explicit plan, over `npairs` pairs of one job
// (kTable = false: BlockRec + overflow rows).
// Half-pel SADs around the possible winners of the blocks that have few
// (records and overflow regions of `npairs` pairs), before a half-pel
// resolve.
int launch_half_prep(const KGeom& g, const FramePtrs& fr, int npairs, BlockRec* recs,
                     uint16_t* ovf, hipStream_t st);
int launch_search_plan(const KGeom& g, const SearchPlan& pl, const uint8_t* const* frames,
                       int npairs, BlockRec* recs, uint16_t* ovf, uint32_t slack,
                       hipStream_t s);
size_t fsbm_recs_offset();                    // BlockRec array offset in an FSBM workspace
size_t fsbm_ovf_offset(const KGeom& g, uint32_t npairs);
size_t fsbm_ovf_entries(int p);  // u16 entries of one block's overflow region
size_t fsbm_mv_offset(const KGeom& g, uint32_t npairs);  // resolve state, if used
bool fsbm_mv_in_lds(const KGeom& g);
// Batch kernels: the full search of one group (at most 64 jobs with the
// same N, M and plan; one workgroup per item: a block, or a 2x2 tile of 8x8
// blocks with a tiled plan) and the resolve of every pair of a set of FSBM
// jobs (one workgroup per pair).
int launch_search_batch(int N, int M, const SearchPlan& pl, size_t lds, const BatchJob* jobs,
                        int njobs, uint32_t items, hipStream_t s);
// Creates the current device's side streams for batch walker launches.
int batch_side_streams_init();
// Looks up the current device's scratch array of the allocation-free entry
// point (once per device).
int noalloc_scratch_init();
// acbm_batch with a temporal field for the first pair of each PBM/ACBM job
// (prev0[i], may be null; prev0 itself may be null) and the choice of side
// streams; status_words (may be null) receives the device addresses of the
// status words of its walker launches (0 = every block finished).
int batch_enqueue(const acbm_job* jobs, size_t njobs, const acbm_mv* const* prev0, void* ws,
                  size_t ws_bytes, hipStream_t st, bool side_streams,
                  std::vector<const uint32_t*>* status_words);
// Resolves pairs pair_base .. pair_base + pairs - 1 (numbered by pair0) of
// the `njobs` jobs at `jobs`, which must hold every job with such a pair;
// max_by is the most block rows of those pairs' frames.  `sized`: the
// resolve runs beside other searches, and its workgroups are sized to the
// frames (see resolve_threads).
int launch_resolve_batch(const BatchJob* jobs, int njobs, uint32_t pair_base, uint32_t pairs,
                         size_t lds, int max_by, bool sized, hipStream_t s);
size_t predictive_ws_bytes(const KGeom& g, uint32_t npairs);
int launch_predictive(const KGeom& g, const acbm_params& prm, int algo,
                      const uint8_t* const* frames, uint32_t npairs, const acbm_mv* prev_field,
                      void* ws, size_t ws_bytes, acbm_block_result* out, hipStream_t s);

// Row walkers (PBM/ACBM) over several jobs in one launch.  Every job of a
// group has the same block size and precision; the walkers take the rows of
// all jobs from one ticket counter in level order (row r of pair t has level
// r + 2t), so the chains of the jobs run side by side.
//
// Circular window of the walkers: absolute dword column a lives at a & (cw-1),
// and columns 0 .. N/4+1 again at cw .. cw+N/4+1; rows are `stride` dwords
// apart (odd).
struct RingShape {
  WindowShape s;
  int cw;
  int stride;
};

// One job as the walkers read it (device memory).
struct PredArgs {
  KGeom g;
  RingShape w;
  int algo;
  uint32_t lam;
  uint64_t c1_rhs;        // N*M*(alpha + beta*qp^2), saturated
  uint32_t gamma_num, gamma_den;
  int npairs;
  int row_levels;         // (by-1) + 2(npairs-1) + 1
  const uint8_t* prev0;   // temporal field of pair 0 (acbm_mv at byte stride), or null
  int prev0_stride;
  WsHeader* hdr;          // ticket and status, shared by the jobs of a launch
  uint32_t* words;        // [npairs][nb] published vectors
  const uint8_t* const* frames;  // [npairs+1] frame pointers
  acbm_block_result* out;
};

// Row words of the merged ticket order: job (8 bits), pair (12), row (12).
constexpr int kPredMaxJobs = 256;
constexpr uint32_t kPredMaxPairs = 4095;

struct PredGroupPlan {
  int R = 0;        // row blocking of the critical search
  int threads = 0;  // threads per walker
  size_t lds = 0;   // dynamic LDS bytes (the largest ring of the group)
};
// Plans a group from its jobs' geometries (same block size) and its row count.
int plan_predictive_group(const KGeom* geoms, int n, bool hp, size_t total_rows,
                          PredGroupPlan* pl);
// The fields of a job that do not point into device memory.
PredArgs predictive_args(const KGeom& g, const acbm_params& prm, int algo, int R,
                         uint32_t npairs);
// Clears the jobs' vector words, writes the merged row order and resets the
// header (setup kernel), then runs the walkers over every row.
int launch_predictive_group(int bw, int bh, bool hp, const PredGroupPlan& pl,
                            const PredArgs* jobs, int njobs, uint32_t* order, WsHeader* hdr,
                            uint32_t total_rows, hipStream_t s);

}  // namespace acbm
