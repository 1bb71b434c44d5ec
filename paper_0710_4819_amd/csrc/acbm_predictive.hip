// acbm_predictive.hip -- PBM (Section 2.2) and ACBM (Section 3.2) on gfx950.
//
// Both searches are sequential in the paper's raster order: a block's
// predictor set uses the final vectors of its left, top-left, top and
// top-right neighbours in this frame, and the previous frame's field around
// it.  The kernel below runs them as a dataflow over blocks instead of a
// raster loop, which gives identical results because every block only reads
// vectors of blocks that precede it:
//
//  * Tickets.  Block (r, c) of pair t gets level s + 4t with s = c + 2r.
//    Its spatial neighbours have levels s-3 .. s-1 and its temporal ones
//    (pair t-1, rows r-1..r+1, columns c-1..c+1) at most s + 3 + 4(t-1), so
//    every dependency has a smaller level.  Workgroups take tickets in level
//    order from one counter, so the smallest unfinished ticket always has its
//    dependencies done and the kernel cannot deadlock, however many
//    workgroups are resident.  Frames of a sequence overlap: pair t starts
//    while pair t-1 is still running.
//  * Publication.  A finished block stores its vector together with a ready
//    bit in one 32-bit word (relaxed, device scope); consumers poll that word
//    and need nothing else, so no fences are required.  Every wait is
//    bounded: on time-out the kernel records the failure in the workspace
//    header and all workgroups leave.
//  * Work per block.  The block's search window is staged in LDS while the
//    dependencies are awaited.  Predictor and ring SADs use one lane per
//    dword of the block (V_SAD_U8 on byte-aligned window dwords, wave
//    reduction); a critical block (ACBM) runs the same QSAD window search as
//    the full-search kernel, reduced to the J-minimum with this block's
//    predictor.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "acbm_device.h"
#include "acbm_internal.h"

namespace acbm {

constexpr uint32_t kReady = 0x80000000u;
constexpr int kMaxCands = 14 + 8;
constexpr int kPredThreads = 256;
constexpr uint32_t kSpinLimit = 1u << 22;

struct PredArgs {
  KGeom g;
  WindowShape s;
  int algo;
  uint32_t lam;
  uint64_t c1_rhs;       // N*M*(alpha + beta*qp^2), saturated
  uint32_t gamma_num, gamma_den;
  int npairs;
  int levels;            // number of ticket levels
  int spatial_steps;     // S = (bx-1) + 2(by-1) + 1
  const uint8_t* prev0;  // temporal field of pair 0 (acbm_mv at byte stride), or null
  int prev0_stride;
  WsHeader* hdr;
  uint32_t* level_start; // [levels+1]
  uint32_t* words;       // [npairs][nb] published vectors
  acbm_block_result* out;
};

// Blocks (r, c) with c + 2r = s: rows r_lo(s) .. r_hi(s).
__host__ __device__ inline int diag_rlo(int s, int bx) { return max(0, (s - (bx - 1) + 1) / 2); }
__host__ __device__ inline int diag_rhi(int s, int by) { return min(by - 1, s / 2); }
__host__ __device__ inline int diag_count(int s, int bx, int by, int S) {
  if (s < 0 || s >= S) return 0;
  return max(0, diag_rhi(s, by) - diag_rlo(s, bx) + 1);
}

// Prepares the workspace of one launch: level offsets, cleared vector words,
// ticket and status.  (A kernel rather than hipMemsetAsync so that the
// sequence can be captured in a graph.)
__global__ void k_pred_setup(PredArgs a) {
  const size_t nw = (size_t)a.npairs * a.g.nb;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (size_t)gridDim.x * blockDim.x)
    a.words[i] = 0;
  if (blockIdx.x == 0) {
    for (int lv = threadIdx.x; lv < a.levels; lv += blockDim.x) {
      int n = 0;
      for (int t = 0; t < a.npairs; ++t) n += diag_count(lv - 4 * t, a.g.bx, a.g.by, a.spatial_steps);
      a.level_start[lv + 1] = (uint32_t)n;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.level_start[0] = 0;
      for (int lv = 1; lv <= a.levels; ++lv) a.level_start[lv] += a.level_start[lv - 1];
      a.hdr->ticket = 0;
      a.hdr->status = 0;
    }
  }
}

__device__ __forceinline__ uint32_t load_word(const uint32_t* w) {
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_word(uint32_t* w, uint32_t v) {
  __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// SAD of candidates list[first..n) over the window in LDS; one lane per dword
// of the block, D = N*M/4 lanes per candidate.
template <int N, int M>
__device__ inline void list_sads(const uint32_t* __restrict__ win, const WindowShape& s,
                                 const uint32_t* __restrict__ curd, const int16_t* cu,
                                 const int16_t* cv, uint32_t* sads, int first, int n) {
  constexpr int D = M * N / 4;
  constexpr int CPW = 64 / D;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int slot = lane / D, l = lane % D;
  const int j = l / (N / 4), k = l % (N / 4);
  const uint32_t mine = curd[l];
  for (int base = first + wave * CPW; base < n; base += nwaves * CPW) {
    const int ci = base + slot;
    uint32_t part = 0;
    if (ci < n) {
      const int u = cu[ci], v = cv[ci];
      const int off = u - s.u_lo + 4 * k;
      const uint32_t* rowp = win + (v + s.p + j) * s.stride;
      const uint32_t lo = rowp[off >> 2], hi = rowp[(off >> 2) + 1];
      const uint32_t val = __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)(off & 3));
      part = __builtin_amdgcn_sad_u8(val, mine, 0u);
    }
#pragma unroll
    for (int o = D / 2; o >= 1; o >>= 1) part += (uint32_t)__shfl_xor((int)part, o, 64);
    if (ci < n && l == 0) sads[ci] = part;
  }
}

template <int N, int M, int R>
__global__ void __launch_bounds__(kPredThreads) k_predictive(const PredArgs a, const FramePtrs fr) {
  extern __shared__ uint32_t lds[];
  uint32_t* lstart = lds;                        // level table
  uint32_t* win = lds + ((a.levels + 1 + 3) & ~3);
  __shared__ uint64_t red[kPredThreads / 64];
  __shared__ uint32_t curd[M * N / 4];
  __shared__ int16_t cu[kMaxCands], cv[kMaxCands];
  __shared__ uint32_t csad[kMaxCands];
  __shared__ uint16_t dep[13];
  __shared__ int sh_ticket, sh_abort, sh_n, sh_np, sh_px, sh_py, sh_crit;
  __shared__ uint32_t sh_intra;

  const KGeom& g = a.g;
  const WindowShape& s = a.s;
  const int p = g.p, bx = g.bx, by = g.by, nb = g.nb;
  const uint32_t total = (uint32_t)a.npairs * nb;

  for (int i = threadIdx.x; i <= a.levels; i += blockDim.x) lstart[i] = a.level_start[i];
  __syncthreads();

  for (;;) {
    if (threadIdx.x == 0) {
      sh_ticket = (int)atomicAdd(&a.hdr->ticket, 1u);
      sh_abort = __hip_atomic_load(&a.hdr->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    __syncthreads();
    const uint32_t tk = (uint32_t)__builtin_amdgcn_readfirstlane(sh_ticket);
    if (tk >= total || sh_abort) return;

    // ---- ticket -> (t, r, c) -------------------------------------------
    int lo = 0, hi = a.levels - 1;
    while (lo < hi) {  // last level with lstart[level] <= tk
      const int mid = (lo + hi + 1) >> 1;
      if (lstart[mid] <= tk) lo = mid; else hi = mid - 1;
    }
    const int lv = lo;
    int idx = (int)(tk - lstart[lv]);
    int t = max(0, (lv - a.spatial_steps + 1 + 3) / 4), sd = 0;
    for (; t < a.npairs; ++t) {
      sd = lv - 4 * t;
      const int n = diag_count(sd, bx, by, a.spatial_steps);
      if (idx < n) break;
      idx -= n;
    }
    if (t >= a.npairs) {  // cannot happen for a consistent level table
      if (threadIdx.x == 0) atomicOr(&a.hdr->status, kStatusSpinTimeout);
      return;
    }
    t = __builtin_amdgcn_readfirstlane(t);
    const int r = __builtin_amdgcn_readfirstlane(diag_rlo(sd, bx) + idx);
    const int c = __builtin_amdgcn_readfirstlane(sd - 2 * r);
    const int b = r * bx + c;
    const int x0 = c * N, y0 = r * M;
    const uint8_t* __restrict__ ref = fr.f[t];
    const uint8_t* __restrict__ cur = fr.f[t + 1];

    // ---- independent work first: window, current block, IntraX ---------
    load_window<N, M>(win, s, ref, g.pitch, g.width, g.height, x0, y0);
    for (int l = threadIdx.x; l < M * N / 4; l += blockDim.x) {
      const int j = l / (N / 4), k = l % (N / 4);
      curd[l] = *reinterpret_cast<const uint32_t*>(cur + (size_t)(y0 + j) * g.pitch + x0 + 4 * k);
    }

    // ---- wait for the 4 spatial and 9 temporal neighbours ---------------
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      const uint32_t* w = nullptr;  // word to wait for
      uint16_t val = kMvUnset;      // kMvUnset = neighbour absent
      if (lane < 4) {
        const int dr = lane == 0 ? 0 : -1;
        const int dc = lane == 0 ? -1 : lane - 2;  // L, TL, T, TR
        const int rr = r + dr, cc = c + dc;
        if (rr >= 0 && cc >= 0 && cc < bx) w = a.words + (size_t)t * nb + rr * bx + cc;
      } else if (lane < 13) {
        const int dr = (lane - 4) / 3 - 1, dc = (lane - 4) % 3 - 1;
        const int rr = r + dr, cc = c + dc;
        if (rr >= 0 && rr < by && cc >= 0 && cc < bx) {
          if (t > 0) {
            w = a.words + (size_t)(t - 1) * nb + rr * bx + cc;
          } else if (a.prev0) {
            const acbm_mv m = *reinterpret_cast<const acbm_mv*>(
                a.prev0 + (size_t)(rr * bx + cc) * a.prev0_stride);
            val = pack_mv(m.x, m.y);
          } else {
            val = pack_mv(0, 0);
          }
        }
      }
      uint32_t word = 0;
      uint32_t spins = 0;
      bool failed = false;
      for (;;) {
        if (w && !(word & kReady)) word = load_word(w);
        const bool done = !w || (word & kReady);
        if (__all(done)) break;
        if (++spins > kSpinLimit) {
          failed = true;
          break;
        }
        if ((spins & 255) == 0 &&
            __hip_atomic_load(&a.hdr->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          failed = true;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (w) val = (uint16_t)(word & 0xFFFFu);
      if (lane < 13) dep[lane] = val;
      if (lane == 0) {
        sh_abort = failed;
        if (failed) atomicOr(&a.hdr->status, kStatusSpinTimeout);
      }
    }
    __syncthreads();
    if (sh_abort) return;

    // ---- predictor and predictor set (Section 2.2, step 1) --------------
    if (threadIdx.x == 0) {
      const uint16_t zero = pack_mv(0, 0);
      const uint16_t A = dep[0] != kMvUnset ? dep[0] : zero;
      uint16_t B, C;
      if (r == 0) {
        B = A;
        C = A;
      } else {
        B = dep[2];
        C = (c == bx - 1) ? zero : dep[3];
      }
      const int px = med3(mv_x(A), mv_x(B), mv_x(C));
      const int py = med3(mv_y(A), mv_y(B), mv_y(C));
      int n = 0;
      auto add = [&](int u, int v) {
        if (!cand_valid(u, v, p, x0, y0, N, M, g.width, g.height)) return;
        for (int k = 0; k < n; ++k)
          if (cu[k] == u && cv[k] == v) return;
        cu[n] = (int16_t)u;
        cv[n] = (int16_t)v;
        ++n;
      };
      add(0, 0);
      for (int k = 0; k < 13; ++k)
        if (dep[k] != kMvUnset) add(mv_x(dep[k]), mv_y(dep[k]));
      sh_np = n;
      sh_n = n;
      sh_px = px;
      sh_py = py;
    }
    // IntraX (Section 3.1) by wave 1 while thread 0 builds the set
    if (threadIdx.x >= 64 && threadIdx.x < 128) {
      const int lane = threadIdx.x - 64;
      constexpr int D = M * N / 4;
      const uint32_t d = lane < D ? curd[lane] : 0u;
      const uint32_t ssum = wave_sum_u32(__builtin_amdgcn_sad_u8(d, 0u, 0u));
      uint32_t acc = 0;
      if (lane < D) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = (int)(N * M) * (int)((d >> (8 * q)) & 0xFF) - (int)ssum;
          acc += (uint32_t)(e < 0 ? -e : e);
        }
      }
      acc = wave_sum_u32(acc);
      if (lane == 0) sh_intra = acc;
    }
    __syncthreads();
    const int px = sh_px, py = sh_py;

    // ---- step 2: SADs of the predictors, cheapest one --------------------
    list_sads<N, M>(win, s, curd, cu, cv, csad, 0, sh_np);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int n = sh_np;
      uint64_t best = ~0ull;
      int bi = 0;
      for (int k = 0; k < n; ++k) {
        const uint32_t j = csad[k] + a.lam * (se_bits(cu[k] - px) + se_bits(cv[k] - py));
        const uint64_t key = make_key(j, cu[k], cv[k], p);
        if (key < best) { best = key; bi = k; }
      }
      // step 3: one refinement ring on the integer grid
      const int bu = cu[bi], bv = cv[bi];
      int m = n;
      for (int dv = -1; dv <= 1; ++dv)
        for (int du = -1; du <= 1; ++du) {
          if (du == 0 && dv == 0) continue;
          const int u = bu + du, v = bv + dv;
          if (!cand_valid(u, v, p, x0, y0, N, M, g.width, g.height)) continue;
          bool seen = false;
          for (int k = 0; k < m; ++k) seen |= (cu[k] == u && cv[k] == v);
          if (seen) continue;
          cu[m] = (int16_t)u;
          cv[m] = (int16_t)v;
          ++m;
        }
      sh_n = m;
    }
    __syncthreads();
    list_sads<N, M>(win, s, curd, cu, cv, csad, sh_np, sh_n);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int n = sh_n;
      uint64_t best = ~0ull;
      int bi = 0;
      for (int k = 0; k < n; ++k) {
        const uint32_t j = csad[k] + a.lam * (se_bits(cu[k] - px) + se_bits(cv[k] - py));
        const uint64_t key = make_key(j, cu[k], cv[k], p);
        if (key < best) { best = key; bi = k; }
      }
      // ACBM decision (Section 3.2), both tests scaled by N*M
      int crit = 0, mode = ACBM_MODE_PBM;
      if (a.algo == ACBM_ALGO_ACBM) {
        const uint64_t nm = (uint64_t)(N * M);
        const uint64_t sadp = csad[bi], ix = sh_intra;
        if (ix + nm * sadp < a.c1_rhs) mode = ACBM_MODE_PBM_C1;
        else if ((uint64_t)a.gamma_den * nm * sadp < (uint64_t)a.gamma_num * ix) mode = ACBM_MODE_PBM_C2;
        else { mode = ACBM_MODE_CRITICAL; crit = 1; }
      }
      sh_crit = crit;
      if (!crit) {
        const int u = cu[bi], v = cv[bi];
        const uint32_t rate = se_bits(u - px) + se_bits(v - py);
        acbm_block_result res;
        res.mv.x = (int16_t)u;
        res.mv.y = (int16_t)v;
        res.sad = csad[bi];
        res.j = csad[bi] + a.lam * rate;
        res.rate_bits = rate;
        res.cands = (uint32_t)n;
        res.mode = (uint32_t)mode;
        res.intra_x = sh_intra;
        a.out[(size_t)t * nb + b] = res;
        store_word(a.words + (size_t)t * nb + b, kReady | pack_mv(u, v));
      }
    }
    __syncthreads();

    // ---- critical block: full search with the same predictor ------------
    if (sh_crit) {
      CurBlock<N, M> cb;
#pragma unroll
      for (int j = 0; j < M; ++j)
#pragma unroll
        for (int k = 0; k < N / 4; ++k) cb.d[j][k] = __builtin_amdgcn_readfirstlane(curd[j * (N / 4) + k]);
      uint64_t lbest = ~0ull;
      const int tasks = s.quads * s.groups;
      for (int task = threadIdx.x; task < tasks; task += blockDim.x) {
        const int q = task % s.quads, gi = task / s.quads;
        uint64_t acc[R];
        task_sads<N, M, R>(win, s.stride, q, gi, cb, acc);
        const int u0 = s.u_lo + 4 * q, v0 = -p + R * gi;
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int u = u0 + i, v = v0 + rr;
            if (!cand_valid(u, v, p, x0, y0, N, M, g.width, g.height)) continue;
            const uint32_t sad = (uint32_t)(acc[rr] >> (16 * i)) & 0xFFFFu;
            const uint32_t j = sad + a.lam * (se_bits(u - px) + se_bits(v - py));
            const uint64_t key = make_key(j, u, v, p);
            // carry the SAD in the low bits of a second key for the write-out
            lbest = key < lbest ? key : lbest;
          }
      }
      const uint64_t best = group_min_u64(lbest, red);
      if (threadIdx.x == 0) {
        const int W = 2 * p + 1;
        const int ras = (int)(best & 0xFFFFu);
        const int u = ras % W - p, v = ras / W - p;
        const uint32_t rate = se_bits(u - px) + se_bits(v - py);
        const uint32_t jv = (uint32_t)(best >> 32);
        acbm_block_result res;
        res.mv.x = (int16_t)u;
        res.mv.y = (int16_t)v;
        res.sad = jv - a.lam * rate;
        res.j = jv;
        res.rate_bits = rate;
        res.cands = (uint32_t)sh_n + valid_count(p, x0, y0, N, M, g.width, g.height);
        res.mode = ACBM_MODE_CRITICAL;
        res.intra_x = sh_intra;
        a.out[(size_t)t * nb + b] = res;
        store_word(a.words + (size_t)t * nb + b, kReady | pack_mv(u, v));
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int spatial_steps(const KGeom& g) { return (g.bx - 1) + 2 * (g.by - 1) + 1; }
static int num_levels(const KGeom& g, int npairs) { return spatial_steps(g) + 4 * (npairs - 1); }

size_t predictive_ws_bytes(const KGeom& g, uint32_t npairs) {
  const uint32_t per = std::min<uint32_t>(npairs, kMaxPairsPerLaunch);
  return align256(sizeof(WsHeader)) +
         align256(((size_t)num_levels(g, (int)per) + 1) * sizeof(uint32_t)) +
         align256((size_t)per * g.nb * sizeof(uint32_t));
}

#define ACBM_PRED_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(11) X(16)

template <int N, int M>
static int launch_pred_nm(const PredArgs& a, const FramePtrs& fr, int R, size_t lds, int grid,
                          hipStream_t st) {
  switch (R) {
#define ACBM_CASE(RR)                                                                    \
  case RR: {                                                                             \
    if (lds > 64 * 1024)                                                                 \
      (void)hipFuncSetAttribute((const void*)k_predictive<N, M, RR>,                     \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    ProfScope ps("predictive", st);                                                      \
    hipLaunchKernelGGL((k_predictive<N, M, RR>), dim3(grid), dim3(kPredThreads), lds, st, \
                       a, fr);                                                           \
    break;                                                                               \
  }
    ACBM_PRED_R_LIST(ACBM_CASE)
#undef ACBM_CASE
    default:
      return fail(ACBM_E_UNSUPPORTED, "no predictive kernel for this row blocking");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the predictive search");
}

static int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  return cus;
}

int launch_predictive(const KGeom& g, const acbm_params& prm, int algo,
                      const uint8_t* const* frames, uint32_t npairs, const acbm_mv* prev_field,
                      void* ws, size_t ws_bytes, acbm_block_result* out, hipStream_t st) {
  if (ws_bytes < predictive_ws_bytes(g, npairs)) return fail(ACBM_E_NOMEM, "workspace too small");
  const SearchPlan pl = plan_search(g.bw, g.bh, g.p, kPredThreads);
  if (!pl.R) return fail(ACBM_E_UNSUPPORTED, "search window does not fit in LDS");
  for (uint32_t p0 = 0; p0 < npairs; p0 += kMaxPairsPerLaunch) {
    const int n = (int)std::min<uint32_t>(kMaxPairsPerLaunch, npairs - p0);
    PredArgs a{};
    a.g = g;
    a.algo = algo;
    a.lam = prm.lambda;
    const unsigned __int128 t1 =
        ((unsigned __int128)prm.alpha + (unsigned __int128)prm.beta * prm.qp * prm.qp) *
        (unsigned __int128)(g.bw * g.bh);
    a.c1_rhs = t1 > (unsigned __int128)UINT64_MAX ? UINT64_MAX : (uint64_t)t1;
    a.gamma_num = prm.gamma_num;
    a.gamma_den = prm.gamma_den;
    a.npairs = n;
    a.spatial_steps = spatial_steps(g);
    a.levels = num_levels(g, n);
    if (p0 == 0) {
      a.prev0 = reinterpret_cast<const uint8_t*>(prev_field);
      a.prev0_stride = sizeof(acbm_mv);
    } else {
      a.prev0 = reinterpret_cast<const uint8_t*>(out + (size_t)(p0 - 1) * g.nb);
      a.prev0_stride = sizeof(acbm_block_result);
    }
    char* base = static_cast<char*>(ws);
    a.hdr = reinterpret_cast<WsHeader*>(base);
    a.level_start = reinterpret_cast<uint32_t*>(base + align256(sizeof(WsHeader)));
    a.words = reinterpret_cast<uint32_t*>(
        base + align256(sizeof(WsHeader)) +
        align256(((size_t)num_levels(g, (int)std::min<uint32_t>(npairs, kMaxPairsPerLaunch)) + 1) *
                 sizeof(uint32_t)));
    a.out = out + (size_t)p0 * g.nb;
    FramePtrs fr{};
    for (int k = 0; k <= n; ++k) fr.f[k] = frames[p0 + k];

    if (g.bw == 16 && g.bh == 16) a.s = window_shape<16, 16>(g.p, pl.R);
    else if (g.bw == 16 && g.bh == 8) a.s = window_shape<16, 8>(g.p, pl.R);
    else if (g.bw == 8 && g.bh == 16) a.s = window_shape<8, 16>(g.p, pl.R);
    else a.s = window_shape<8, 8>(g.p, pl.R);
    const size_t lds = (size_t)((a.levels + 1 + 3) & ~3) * 4 + (size_t)a.s.rows * a.s.stride * 4;
    if (lds > (size_t)lds_limit()) return fail(ACBM_E_UNSUPPORTED, "search window too large for LDS");

    const int setup_grid = (int)std::min<size_t>(1024, ((size_t)n * g.nb + 255) / 256 + 1);
    {
      ProfScope ps("setup", st);
      hipLaunchKernelGGL(k_pred_setup, dim3(setup_grid), dim3(256), 0, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "launching the predictive setup");

    const int per_cu = lds <= 32 * 1024 ? 4 : (lds <= 48 * 1024 ? 3 : 1);
    const int grid = (int)std::min<size_t>((size_t)device_cus() * per_cu, (size_t)n * g.nb);
    int rc;
    if (g.bw == 16 && g.bh == 16) rc = launch_pred_nm<16, 16>(a, fr, pl.R, lds, grid, st);
    else if (g.bw == 16 && g.bh == 8) rc = launch_pred_nm<16, 8>(a, fr, pl.R, lds, grid, st);
    else if (g.bw == 8 && g.bh == 16) rc = launch_pred_nm<8, 16>(a, fr, pl.R, lds, grid, st);
    else rc = launch_pred_nm<8, 8>(a, fr, pl.R, lds, grid, st);
    if (rc) return rc;
  }
  return ACBM_OK;
}

}  // namespace acbm
