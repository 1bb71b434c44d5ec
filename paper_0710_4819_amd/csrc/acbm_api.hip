// acbm_api.hip -- C ABI of libacbm: argument checks, plans, workspace sizing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "acbm_device.h"
#include "acbm_internal.h"

namespace acbm {

static thread_local std::string t_last_error;

int fail(int code, const std::string& msg) {
  t_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  t_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return ACBM_E_DEVICE;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int se_bits_host(int k) {
  unsigned a = (unsigned)(k < 0 ? -k : k);
  if (a == 0) return 1;
  int fl = 31 - __builtin_clz(a);
  return 2 * fl + 3;
}

int rate_max(int p) { return 2 * se_bits_host(2 * p); }

int check_geom(const acbm_geom* g, KGeom* k) {
  if (!g) return fail(ACBM_E_INVAL, "geometry is NULL");
  if (!g->width || !g->height || !g->block_w || !g->block_h)
    return fail(ACBM_E_INVAL, "zero frame or block size");
  if (g->pitch < g->width) return fail(ACBM_E_INVAL, "pitch smaller than width");
  if (g->width % g->block_w || g->height % g->block_h)
    return fail(ACBM_E_SHAPE, "frame size is not a multiple of the block size");
  if (g->p > 127) return fail(ACBM_E_SHAPE, "p above 127");
  if ((g->block_w != 8 && g->block_w != 16) || (g->block_h != 8 && g->block_h != 16))
    return fail(ACBM_E_UNSUPPORTED, "block_w and block_h must be 8 or 16");
  if (g->pitch % 4) return fail(ACBM_E_UNSUPPORTED, "pitch must be a multiple of 4 bytes");
  if ((uint64_t)g->pitch * g->height > (1ull << 31))
    return fail(ACBM_E_UNSUPPORTED, "frame larger than 2 GiB");
  if (k) {
    k->width = (int)g->width;
    k->height = (int)g->height;
    k->pitch = (int)g->pitch;
    k->bw = (int)g->block_w;
    k->bh = (int)g->block_h;
    k->p = (int)g->p;
    k->bx = k->width / k->bw;
    k->by = k->height / k->bh;
    k->nb = k->bx * k->by;
  }
  return ACBM_OK;
}

int check_params(const acbm_params* prm, const KGeom& k) {
  if (!prm) return fail(ACBM_E_INVAL, "params is NULL");
  if (prm->gamma_den == 0) return fail(ACBM_E_INVAL, "gamma_den is zero");
  if (prm->subpel > 1) return fail(ACBM_E_INVAL, "subpel must be 0 or 1");
  if (prm->subpel && k.p > 63)
    return fail(ACBM_E_RANGE, "half-pel vectors need p <= 63");
  if (k.by > 1024)  // the FSBM resolve gives each block row of a step one thread
    return fail(ACBM_E_UNSUPPORTED, "at most 1024 block rows");
  const uint64_t jmax =
      255ull * k.bw * k.bh + (uint64_t)prm->lambda * rate_max(prm->subpel ? 2 * k.p : k.p);
  if (jmax >= (1ull << 32)) return fail(ACBM_E_RANGE, "lambda too large: J would not fit 32 bits");
  return ACBM_OK;
}

int check_frame_ptr(const void* p, const char* what) {
  if (!p) return fail(ACBM_E_INVAL, std::string(what) + " is NULL");
  if ((uintptr_t)p % 4) return fail(ACBM_E_UNSUPPORTED, std::string(what) + " is not 4-byte aligned");
  return ACBM_OK;
}

int check_device() {
  static std::mutex mu;
  static int known_dev = -1, known_rc = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(mu);
  if (dev == known_dev) return known_rc;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  known_dev = dev;
  known_rc = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0
                 ? ACBM_OK
                 : fail(ACBM_E_UNSUPPORTED, std::string("device is ") + prop.gcnArchName +
                                                ", this library is built for gfx950");
  return known_rc;
}

// Issue cost of one V_QSAD_PK_U16_U8 relative to a full-rate VALU op.  The
// instruction probe measures 3.9 on gfx950 (quarter rate: 16 absolute
// differences per lane every 4 clocks, the same byte rate as full-rate
// V_SAD_U8).  ACBM_QSAD_COST overrides it for tuning experiments.
static double qsad_cost() {
  static double c = [] {
    const char* e = std::getenv("ACBM_QSAD_COST");
    return e ? std::atof(e) : 4.0;
  }();
  return c;
}

// Dynamic LDS a workgroup may use on the current device (less a margin for
// the kernels' static LDS).
int lds_limit() {
  static int lim = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
      v = 64 * 1024;
    return v - 1024;
  }();
  return lim;
}

// Choose the candidate rows per lane R and the workgroup size.  Model per
// wave-task, in CU clocks: VALU = R*M*N/4 QSADs at their issue cost; LDS =
// (R+M-1) window rows of 2N bytes per lane at 128 B/clk; the slower of the
// two bounds the task, plus a fixed cost per wave.  With
// max_threads = 1024 every task gets its own thread (the full-search kernel
// keeps all SADs of a block in registers); otherwise tasks loop over a fixed
// group of max_threads.  R = 0 means no plan fits (window too large for LDS).
WindowShape window_shape_host(int N, int M, int p, int R) {
  if (N == 16 && M == 16) return window_shape<16, 16>(p, R);
  if (N == 16 && M == 8) return window_shape<16, 8>(p, R);
  if (N == 8 && M == 16) return window_shape<8, 16>(p, R);
  return window_shape<8, 8>(p, R);
}

static const int kPlanRs[] = {1, 2, 3, 4, 5, 6, 8, 11, 16};

// One workgroup of ceil(tasks/64) waves per block (or max_threads lanes in
// rounds); R = 0 when the window does not fit.
static SearchPlan plan_for(int N, int M, int p, int R, int max_threads, double* cost) {
  const WindowShape s = window_shape_host(N, M, p, R);
  const int tasks = s.quads * s.groups;
  const int lds = s.rows * s.stride * 4;
  int threads, rounds;
  if (max_threads >= 1024) {
    if (tasks > 1024) return SearchPlan{0, 0, 0};
    threads = (tasks + 63) / 64 * 64;
    rounds = 1;
  } else {
    threads = max_threads;
    rounds = (tasks + threads - 1) / threads;
  }
  if (lds > lds_limit()) return SearchPlan{0, 0, 0};
  if (threads < s.dws) return SearchPlan{0, 0, 0};  // the window load gives each dword column a thread
  const double valu = (double)R * M * (N / 4) * qsad_cost();
  const double ldsc = (double)(R + M - 1) * N;
  // kWaveFixed: per-wave cost of the window load, the scalar load of the
  // current block and the epilogue reductions, fitted to an R sweep of the
  // 1920x1088 p = 32 search on MI355X (R = 6 on 192 threads fastest at
  // 4.77 ms, then R = 5 at 5.15 ms and R = 11 at 5.42 ms; R = 8 5.94 ms and
  // R = 4 6.74 ms).
  constexpr double kWaveFixed = 400.0;
  *cost = (double)(threads / 64) * rounds * (std::max(valu, ldsc) + kWaveFixed);
  return SearchPlan{R, threads, lds};
}

// A 2x2 tile of 8x8 blocks is searched over the tile's 16x16 window with the
// 16x16 search's QSAD count; its four blocks keep four sets of R
// accumulators, so R stays at 6 or below (104 VGPRs at R = 6; R = 8 spills
// under the 1024-thread register budget of 128).
static bool tile_rows_ok(int R) { return R <= 6; }

SearchPlan plan_search_model(int N, int M, int p, int R, int tile) {
  double cost = 0;
  if (tile == 2) {
    if (N != 8 || M != 8 || !tile_rows_ok(R)) return SearchPlan{0, 0, 0};
    SearchPlan pl = plan_for(16, 16, p, R, 1024, &cost);
    pl.tile = 2;
    return pl;
  }
  return plan_for(N, M, p, R, 1024, &cost);
}

namespace {
std::mutex g_tuned_mu;
std::map<std::tuple<int, int, int, int>, SearchPlan> g_tuned;  // (N, M, p, tile)
// Plans read from the tuning cache, with the time per pair they were
// measured at (acbm_autotune returns these without timing again).
std::map<std::tuple<int, int, int, int>, float> g_cached_ms;
bool g_cache_loaded = false;

// Architecture name of the current device without its feature suffix
// ("gfx950" of "gfx950:sramecc+:xnack-").
std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "";
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));
}

// The tuning cache named by ACBM_TUNE_CACHE: one JSON object per line,
// {"arch": "gfx950", "N": 16, "M": 16, "p": 32, "R": 6, "ms_per_pair": 0.0887},
// with "tile": 2 at the end for a plan of 2x2 tiles of 8x8 blocks, appended
// by acbm_autotune; a later line for the same key wins.  Lines of
// another architecture or with a plan that no longer fits are ignored.
// g_tuned_mu is held.
void load_tune_cache_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = std::getenv("ACBM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  const std::string arch = device_arch();
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char a[64];
    int N = 0, M = 0, p = 0, R = 0;
    float ms = 0;
    if (std::sscanf(line, " { \"arch\" : \"%63[^\"]\" , \"N\" : %d , \"M\" : %d , \"p\" : %d , "
                          "\"R\" : %d , \"ms_per_pair\" : %f",
                    a, &N, &M, &p, &R, &ms) != 6 ||
        arch != a)
      continue;
    if ((N != 8 && N != 16) || (M != 8 && M != 16) || p < 0 || p > 127) continue;
    const int tile = std::strstr(line, "\"tile\": 2") ? 2 : 1;
    const SearchPlan pl = plan_search_model(N, M, p, R, tile);
    if (!pl.R) continue;
    g_tuned[std::make_tuple(N, M, p, tile)] = pl;
    g_cached_ms[std::make_tuple(N, M, p, tile)] = ms;
  }
  std::fclose(f);
}
}  // namespace

void set_tuned_plan(int N, int M, int p, const SearchPlan& pl) {
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  g_tuned[std::make_tuple(N, M, p, pl.tile)] = pl;
}

bool cached_plan(int N, int M, int p, int tile, SearchPlan* pl, float* ms) {
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  load_tune_cache_locked();
  auto it = g_cached_ms.find(std::make_tuple(N, M, p, tile));
  if (it == g_cached_ms.end()) return false;
  *pl = g_tuned[it->first];
  *ms = it->second;
  return true;
}

void save_tuned_plan(int N, int M, int p, const SearchPlan& pl, float ms) {
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  load_tune_cache_locked();
  const auto key = std::make_tuple(N, M, p, pl.tile);
  g_tuned[key] = pl;
  const char* path = std::getenv("ACBM_TUNE_CACHE");
  if (!path || !*path) return;
  g_cached_ms[key] = ms;
  FILE* f = std::fopen(path, "a");
  if (!f) return;  // an unwritable cache only costs the next process a re-tune
  std::fprintf(f, "{\"arch\": \"%s\", \"N\": %d, \"M\": %d, \"p\": %d, \"R\": %d, "
                  "\"ms_per_pair\": %.6f%s}\n",
               device_arch().c_str(), N, M, p, pl.R, ms, pl.tile == 2 ? ", \"tile\": 2" : "");
  std::fclose(f);
}

bool tiles_apply(const KGeom& g) {
  static const bool off = [] {
    const char* e = std::getenv("ACBM_SEARCH_TILES");
    return e && *e && std::atoi(e) == 0;
  }();
  return !off && g.bw == 8 && g.bh == 8 && g.bx % 2 == 0 && g.by % 2 == 0 && g.nb >= 4;
}

// The tiled plan: a measured one if there is, else the cost model's choice
// among the row blockings a tile can keep in registers (ACBM_R overrides).
static SearchPlan plan_search_tile(int p) {
  const char* force = std::getenv("ACBM_R");
  if (force && !*force) force = nullptr;
  if (!force) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    load_tune_cache_locked();
    auto it = g_tuned.find(std::make_tuple(8, 8, p, 2));
    if (it != g_tuned.end()) return it->second;
  }
  SearchPlan best{0, 0, 0};
  double best_cost = 1e300;
  for (int R : kPlanRs) {
    if (!tile_rows_ok(R) || (force && std::atoi(force) != R)) continue;
    double cost = 0;
    SearchPlan pl = plan_for(16, 16, p, R, 1024, &cost);
    if (pl.R && cost < best_cost) {
      best_cost = cost;
      best = pl;
      best.tile = 2;
    }
  }
  return best;
}

SearchPlan plan_fsbm_search(const KGeom& g) {
  if (tiles_apply(g)) {
    const SearchPlan t = plan_search_tile(g.p);
    if (t.R) return t;
  }
  return plan_search(g.bw, g.bh, g.p);
}

// Row blockings measured on MI355X where the cost model's choice is not the
// fastest: 16x16, p = 64: R = 6 1.38 ms per 3840x2160 pair against 1.74 for
// the model's R = 8 (0.37 against 0.45 ms at 1920x1088), though both run 7
// waves per SIMD.  A plan tuned in this process or read from the tuning
// cache still comes first.
static int measured_rows(int N, int M, int p) {
  if (N == 16 && M == 16 && p == 64) return 6;
  return 0;
}

SearchPlan plan_search(int N, int M, int p, int max_threads) {
  const char* force = std::getenv("ACBM_R");
  if (force && !*force) force = nullptr;  // set but empty: as if unset
  if (!force && max_threads >= 1024) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    load_tune_cache_locked();
    auto it = g_tuned.find(std::make_tuple(N, M, p, 1));
    if (it != g_tuned.end()) return it->second;
  }
  if (!force && max_threads >= 1024 && measured_rows(N, M, p)) {
    double cost = 0;
    const SearchPlan pl = plan_for(N, M, p, measured_rows(N, M, p), max_threads, &cost);
    if (pl.R) return pl;
  }
  SearchPlan best{0, 0, 0};
  double best_cost = 1e300;
  for (int R : kPlanRs) {
    if (force && std::atoi(force) != R) continue;
    double cost = 0;
    const SearchPlan pl = plan_for(N, M, p, R, max_threads, &cost);
    if (pl.R && cost < best_cost) {
      best_cost = cost;
      best = pl;
    }
  }
  return best;
}

}  // namespace acbm

using namespace acbm;

extern "C" {

const char* acbm_version(void) { return ACBM_VERSION; }

const char* acbm_strerror(int s) {
  switch (s) {
    case ACBM_OK: return "ok";
    case ACBM_E_INVAL: return "invalid argument";
    case ACBM_E_SHAPE: return "frame/block/search shape not allowed by the method";
    case ACBM_E_RANGE: return "value out of range for the integer cost";
    case ACBM_E_NOMEM: return "not enough workspace or pool memory";
    case ACBM_E_DEVICE: return "HIP device error";
    case ACBM_E_BUSY: return "queue full";
    case ACBM_E_UNSUPPORTED: return "not supported by this library or device";
    case ACBM_E_TIMEOUT: return "timed out";
    default: return "unknown status";
  }
}

const char* acbm_last_error(void) { return t_last_error.c_str(); }

int acbm_default_params(uint32_t block_w, uint32_t block_h, uint32_t lambda, uint32_t qp,
                        uint32_t subpel, acbm_params* out) {
  if (!out) return fail(ACBM_E_INVAL, "out is NULL");
  if (!block_w || !block_h) return fail(ACBM_E_INVAL, "zero block size");
  // Section 4's values for 16x16; alpha and beta scale with the pixel count
  const uint64_t nm = (uint64_t)block_w * block_h;
  const uint64_t alpha = 1000 * nm / 256, beta = 8 * nm / 256;
  if (alpha > 0xFFFFFFFFull || beta > 0xFFFFFFFFull)
    return fail(ACBM_E_RANGE, "block too large for the scaled thresholds");
  out->lambda = lambda;
  out->qp = qp;
  out->alpha = (uint32_t)alpha;
  out->beta = (uint32_t)beta;
  out->gamma_num = 1;
  out->gamma_den = 4;
  out->subpel = subpel;
  return ACBM_OK;
}

int acbm_init(void) {
  t_last_error.clear();
  int rc = check_device();
  if (!rc) rc = batch_side_streams_init();
  return rc ? rc : noalloc_scratch_init();
}

int acbm_workspace_size(int op, const acbm_geom* g, uint32_t npairs, size_t* bytes) {
  KGeom k;
  int rc = check_geom(g, &k);
  if (rc) return rc;
  if (!bytes) return fail(ACBM_E_INVAL, "bytes is NULL");
  if (npairs == 0) return fail(ACBM_E_INVAL, "npairs is zero");
  switch (op) {
    case ACBM_OP_SAD_TABLE: *bytes = 0; return ACBM_OK;
    case ACBM_OP_FSBM: *bytes = fsbm_ws_bytes(k, npairs); return ACBM_OK;
    case ACBM_OP_PBM:
    case ACBM_OP_ACBM: *bytes = predictive_ws_bytes(k, npairs); return ACBM_OK;
    default: return fail(ACBM_E_INVAL, "unknown operation");
  }
}

int acbm_workspace_status(const void* ws, size_t ws_bytes, void* stream, int* status) {
  if (!ws || !status) return fail(ACBM_E_INVAL, "workspace or status is NULL");
  if (ws_bytes < sizeof(WsHeader)) return fail(ACBM_E_NOMEM, "workspace too small");
  WsHeader h;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "reading the workspace header");
  *status = h.status == 0 ? ACBM_OK : ACBM_E_TIMEOUT;
  return ACBM_OK;
}

int acbm_sad_table(const acbm_geom* g, const uint8_t* cur, const uint8_t* ref, uint32_t* table,
                   void* stream) {
  KGeom k;
  int rc = check_geom(g, &k);
  if (rc) return rc;
  if ((rc = check_frame_ptr(cur, "cur")) || (rc = check_frame_ptr(ref, "ref"))) return rc;
  if (!table) return fail(ACBM_E_INVAL, "table is NULL");
  if ((rc = check_device())) return rc;
  return launch_sad_table(k, cur, ref, table, static_cast<hipStream_t>(stream));
}

int acbm_sad_stats(const acbm_geom* g, const uint8_t* cur, const uint8_t* ref,
                   acbm_block_stats* out, void* stream) {
  KGeom k;
  int rc = check_geom(g, &k);
  if (rc) return rc;
  if ((rc = check_frame_ptr(cur, "cur")) || (rc = check_frame_ptr(ref, "ref"))) return rc;
  if (!out) return fail(ACBM_E_INVAL, "out is NULL");
  if ((rc = check_device())) return rc;
  return launch_sad_stats(k, cur, ref, out, static_cast<hipStream_t>(stream));
}

int acbm_fsbm_frame(const acbm_geom* g, const acbm_params* prm, const uint8_t* cur,
                    const uint8_t* ref, acbm_block_result* out, void* ws, size_t ws_bytes,
                    void* stream) {
  KGeom k;
  int rc = check_geom(g, &k);
  if (rc) return rc;
  if ((rc = check_params(prm, k))) return rc;
  if ((rc = check_frame_ptr(cur, "cur")) || (rc = check_frame_ptr(ref, "ref"))) return rc;
  if (!out || !ws) return fail(ACBM_E_INVAL, "out or workspace is NULL");
  if ((rc = check_device())) return rc;
  const uint8_t* frames[2] = {ref, cur};
  return launch_fsbm(k, *prm, frames, 1, ws, ws_bytes, out, static_cast<hipStream_t>(stream));
}

static int predictive_frame(int algo, const acbm_geom* g, const acbm_params* prm,
                            const uint8_t* cur, const uint8_t* ref, const acbm_mv* prev,
                            acbm_block_result* out, void* ws, size_t ws_bytes, void* stream) {
  KGeom k;
  int rc = check_geom(g, &k);
  if (rc) return rc;
  if ((rc = check_params(prm, k))) return rc;
  if ((rc = check_frame_ptr(cur, "cur")) || (rc = check_frame_ptr(ref, "ref"))) return rc;
  if (!out || !ws) return fail(ACBM_E_INVAL, "out or workspace is NULL");
  if ((rc = check_device())) return rc;
  const uint8_t* frames[2] = {ref, cur};
  return launch_predictive(k, *prm, algo, frames, 1, prev, ws, ws_bytes, out,
                           static_cast<hipStream_t>(stream));
}

int acbm_pbm_frame(const acbm_geom* g, const acbm_params* prm, const uint8_t* cur,
                   const uint8_t* ref, const acbm_mv* prev_field, acbm_block_result* out,
                   void* ws, size_t ws_bytes, void* stream) {
  return predictive_frame(ACBM_ALGO_PBM, g, prm, cur, ref, prev_field, out, ws, ws_bytes,
                          stream);
}

int acbm_acbm_frame(const acbm_geom* g, const acbm_params* prm, const uint8_t* cur,
                    const uint8_t* ref, const acbm_mv* prev_field, acbm_block_result* out,
                    void* ws, size_t ws_bytes, void* stream) {
  return predictive_frame(ACBM_ALGO_ACBM, g, prm, cur, ref, prev_field, out, ws, ws_bytes,
                          stream);
}

}  // extern "C"
