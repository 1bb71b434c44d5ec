// acbm_predictive.hip -- PBM (Section 2.2) and ACBM (Section 3.2) on gfx950.
//
// Both searches are sequential in the paper's raster order: a block's
// predictor set uses the final vectors of its left, top-left, top and
// top-right neighbours in this frame, and the previous frame's field around
// it.  The kernel below runs them as a pipeline of block rows instead of one
// raster loop, which gives identical results because every block only reads
// vectors of blocks that precede it:
//
//  * Row tickets.  Row r of pair t gets level r + 2t.  The rows its blocks
//    read (r-1 of pair t; r-1, r, r+1 of pair t-1) have smaller levels.  A
//    workgroup (row walker) takes one row ticket at a time, in level order,
//    from one counter and walks the row left to right.  The smallest
//    unfinished ticket always has every row it reads finished, so the kernel
//    cannot deadlock however many workgroups are resident; rows of many
//    frames run at once (pair t starts while pair t-1 is still running).
//  * Publication.  A finished block stores its vector together with a ready
//    bit in one 32-bit word (relaxed, device scope); consumers poll exactly
//    the words they need, so no fences are required.  The words of the next
//    block are loaded one block ahead.  Every wait is bounded: on time-out
//    the kernel records the failure in the workspace header and all waves
//    leave.
//  * Window.  Consecutive blocks of a row share all but N/4 dword columns of
//    their search windows, so the window lives in a circular buffer of `cw`
//    columns (a power of two >= window + N/4) whose first N/4 + 2 columns are
//    mirrored after the last one: any N/4 + 2 consecutive columns can then be
//    read without wrapping.  The waves other than wave 0 fetch the N/4
//    columns the next block adds into registers while the block is worked
//    on, and park them in columns no longer needed.
//  * Work per block.  Wave 0 waits for the neighbours and builds the
//    predictor set while the other waves compute IntraX.  Then one QSAD pass
//    evaluates, for every predictor candidate (u, v), the 3 x 4 candidates
//    (u-1..u+2, v-1..v+1): one lane per candidate and block row, summed over
//    the rows with cross-lane adds.  That holds both the predictors' SADs and
//    the 8-neighbourhood of whichever predictor wins, so the two PBM steps
//    need a single pass.  A critical block (ACBM) then runs the full window
//    search over all lanes of the workgroup, pricing every candidate in the
//    same pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "acbm_device.h"
#include "acbm_internal.h"

namespace acbm {

constexpr uint32_t kReady = 0x80000000u;
constexpr int kMaxCands = 14;             // (0,0), left, 3 above, 9 of the previous field
constexpr int kFetch = 4;                 // new-column dwords each fetching lane holds
constexpr uint32_t kSpinLimit = 1u << 22;  // polls before a dependency wait gives up
#ifndef ACBM_PRED_WAVES
#define ACBM_PRED_WAVES 3  // waves per SIMD the register budget must allow
#endif

// Per-phase device time of the row walkers, in a build with
// ACBM_PHASE_PROFILE defined (libacbm_phases.so; never the product
// library): thread 0 of every walker stamps s_memrealtime (100 MHz) at the
// phase boundaries of each block and adds its totals here when it leaves.
// [0] blocks, [1] critical blocks, [2] dependency wait (wave 0), [3] phase A
// without the wait, [4] B, [5] C, [6] D (critical search), [7] row set-up.
#ifdef ACBM_PHASE_PROFILE
__device__ unsigned long long g_phase[8];
#define ACBM_PH(...) __VA_ARGS__
#else
#define ACBM_PH(...)
#endif

// Rows (t, r) with r + 2t = k.
__host__ __device__ inline int row_tlo(int k, int by) { return max(0, (k - (by - 1) + 1) / 2); }
__host__ __device__ inline int row_thi(int k, int npairs) { return min(npairs - 1, k / 2); }

__host__ __device__ inline uint32_t row_word(int job, int t, int r) {
  return ((uint32_t)job << 24) | ((uint32_t)t << 12) | (uint32_t)r;
}

// Rows of a job (by block rows, npairs pairs) with level below k.
__device__ inline uint32_t rows_below(int k, int by, int npairs) {
  uint32_t n = 0;
  for (int t = 0; t < npairs && 2 * t < k; ++t) n += (uint32_t)min(by, k - 2 * t);
  return n;
}

// Prepares one launch over `njobs` jobs: cleared vector words, the merged
// row order and the header.  The order lists the rows by level and, within
// a level, by job and pair, so every row comes after the rows it reads.
// Grid: y = job; x spans the job's words and rows.  (A kernel rather than
// hipMemsetAsync so that the sequence can be captured in a graph.)
__global__ void k_pred_setup(const PredArgs* __restrict__ jobs, int njobs,
                             uint32_t* __restrict__ order, WsHeader* __restrict__ hdr) {
  const int j = blockIdx.y;
  const PredArgs& a = jobs[j];
  const int by = a.g.by;
  const size_t nw = (size_t)a.npairs * a.g.nb;
  const size_t nrows = (size_t)a.npairs * by;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (size_t)gridDim.x * blockDim.x)
    st_global<uint32_t>(a.words + i, 0u);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
       i += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(i / by), r = (int)(i % by), k = r + 2 * t;
    uint32_t pos = (uint32_t)(t - row_tlo(k, by));
    for (int q = 0; q < njobs; ++q) {
      const int bq = jobs[q].g.by, nq = jobs[q].npairs;
      pos += rows_below(k, bq, nq);
      if (q < j) pos += (uint32_t)max(0, row_thi(k, nq) - row_tlo(k, bq) + 1);
    }
    order[pos] = row_word(j, t, r);
  }
  if (j == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->ticket = 0;
    hdr->status = 0;
  }
}

// The job table and frame pointers of a single-job launch, written on the
// stream from kernel arguments.
__global__ void k_pred_put_job(PredArgs a, FramePtrs fr, PredArgs* __restrict__ dst,
                               const uint8_t** __restrict__ frames) {
  if (threadIdx.x <= (unsigned)a.npairs) frames[threadIdx.x] = fr.f[threadIdx.x];
  if (threadIdx.x == 0) *dst = a;
}

// Published words and the header live in global memory (see ld_global).
typedef __attribute__((address_space(1))) uint32_t gu32;
__device__ __forceinline__ uint32_t load_word(const uint32_t* w) {
  return __hip_atomic_load((const gu32*)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_word(uint32_t* w, uint32_t v) {
  __hip_atomic_store((gu32*)w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t status_of(const WsHeader* h) {
  return __hip_atomic_load((const gu32*)&h->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Published word lane `lane` waits for at block (t, r, c), or null: lanes
// 2..4 read row r-1 of this pair (top-left, top, top-right), lanes 5..13 the
// previous pair's rows r-1..r+1, columns c-1..c+1 (pair 0 takes its previous
// field from the caller instead and waits for nothing).
__device__ __forceinline__ const uint32_t* dep_word(const PredArgs& a, const uint32_t* words,
                                                   int lane, int t, int r, int c) {
  const int bx = a.g.bx, by = a.g.by;
  if (lane >= 2 && lane < 5) {
    const int cc = c + lane - 3;
    if (r > 0 && cc >= 0 && cc < bx) return words + (r - 1) * bx + cc;
  } else if (lane >= 5 && lane < 14 && t > 0) {
    const int rr = r + (lane - 5) / 3 - 1, cc = c + (lane - 5) % 3 - 1;
    if (rr >= 0 && rr < by && cc >= 0 && cc < bx)
      return a.words + (size_t)(t - 1) * a.g.nb + rr * bx + cc;
  }
  return nullptr;
}

// ---------------------------------------------------------------------------
// Circular window.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ref_dword(const uint8_t* __restrict__ ref, const KGeom& g,
                                              int x, int y) {
  if (y >= 0 && y < g.height && x >= 0 && x + 3 < g.width)
    return ld_global<uint32_t>(ref + (size_t)y * g.pitch + x);
  return 0u;
}

template <int N>
__device__ __forceinline__ void ring_put(uint32_t* __restrict__ ring, const RingShape& w, int row,
                                         int a, uint32_t v) {
  const int c = a & (w.cw - 1);
  uint32_t* rp = ring + row * w.stride;
  rp[c] = v;
  if (c < N / 4 + 2) rp[w.cw + c] = v;
}

// Window columns [a0, a0 + ncol) of all rows straight into the ring (all
// threads); column a of the row strip covers x = u_lo + 4a.
template <int N>
__device__ __forceinline__ void load_columns(uint32_t* __restrict__ ring, const RingShape& w,
                                             const uint8_t* __restrict__ ref, const KGeom& g,
                                             int y0, int a0, int ncol) {
  const int total = w.s.rows * ncol;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int row = idx / ncol, a = a0 + idx % ncol;
    ring_put<N>(ring, w, row, a, ref_dword(ref, g, w.s.u_lo + 4 * a, y0 - w.s.p + row));
  }
}

// The N/4 columns block c+1 adds, fetched into registers by the waves other
// than wave 0 (`f` = lane index among them, `nf` = their count).
struct ColFetch {
  uint32_t v[kFetch];
};

template <int N>
__device__ __forceinline__ void fetch_columns(ColFetch& cf, const RingShape& w,
                                              const uint8_t* __restrict__ ref, const KGeom& g,
                                              int y0, int a0, int f, int nf) {
  constexpr int NC = N / 4;
  const int total = w.s.rows * NC;
#pragma unroll
  for (int k = 0; k < kFetch; ++k) {
    const int idx = f + k * nf;
    const int row = idx / NC, a = a0 + idx % NC;
    cf.v[k] = idx < total ? ref_dword(ref, g, w.s.u_lo + 4 * a, y0 - w.s.p + row) : 0u;
  }
}

template <int N>
__device__ __forceinline__ void park_columns(uint32_t* __restrict__ ring, const ColFetch& cf,
                                             const RingShape& w, const uint8_t* __restrict__ ref,
                                             const KGeom& g, int y0, int a0, int f, int nf) {
  constexpr int NC = N / 4;
  const int total = w.s.rows * NC;
#pragma unroll
  for (int k = 0; k < kFetch; ++k) {
    const int idx = f + k * nf;
    if (idx < total) ring_put<N>(ring, w, idx / NC, a0 + idx % NC, cf.v[k]);
  }
  for (int idx = f + kFetch * nf; idx < total; idx += nf) {
    const int row = idx / NC, a = a0 + idx % NC;
    ring_put<N>(ring, w, row, a, ref_dword(ref, g, w.s.u_lo + 4 * a, y0 - w.s.p + row));
  }
}

// ---------------------------------------------------------------------------
// PBM: SADs of the 3 x 4 neighbourhood (u-1..u+2) x (v-1..v+1) of every
// predictor candidate.  nbr[ci][dv] holds four u16 SADs, columns u-1+i in
// 16-bit lane i, for row v-1+dv.  One lane per (candidate, block row); the M
// lanes of a candidate are adjacent and M divides 64, so the row sum stays
// inside a wave.  Entries outside the window are garbage and belong to
// candidates that are invalid (|u| or |v| > p), which the caller drops.
// ---------------------------------------------------------------------------
template <int N, int M, int NT>
__device__ __forceinline__ void pbm_neighbourhoods(const uint32_t* __restrict__ ring,
                                                   const RingShape& w, int cb0,
                                                   const uint32_t* __restrict__ cd,
                                                   const int16_t* cu, const int16_t* cv, int np,
                                                   uint64_t (*nbr)[3]) {
  constexpr int NC = N / 4;
  constexpr int PER = NT / M;  // candidates per pass
  const int j = threadIdx.x % M;
  const int last_row = w.s.rows - 1;
  uint32_t c[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) c[k] = cd[j * NC + k];
  for (int base = 0; base < np; base += PER) {
    const int ci = base + (int)threadIdx.x / M;
    uint64_t acc[3] = {0, 0, 0};
    if (ci < np) {
      const int u = cu[ci], v = cv[ci];
      const int x = u - 1 - w.s.u_lo;  // byte of column u-1 in the window row (>= -1)
      const uint32_t sh = (uint32_t)(x & 3);
      const int col = (cb0 + (x >> 2)) & (w.cw - 1);
#pragma unroll
      for (int dv = 0; dv < 3; ++dv) {
        const int row = min(max(v + w.s.p - 1 + dv + j, 0), last_row);
        const uint32_t* rp = ring + row * w.stride + col;
        uint32_t d[NC + 2];
#pragma unroll
        for (int m = 0; m < NC + 2; ++m) d[m] = rp[m];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const uint32_t lo = __builtin_amdgcn_alignbyte(d[k + 1], d[k], sh);
          const uint32_t hi = __builtin_amdgcn_alignbyte(d[k + 2], d[k + 1], sh);
          acc[dv] = __builtin_amdgcn_qsad_pk_u16_u8(((uint64_t)hi << 32) | lo, c[k], acc[dv]);
        }
      }
    }
    // Sum over the block rows.  A 16-bit lane never carries (SAD <= 255*N*M),
    // so the two dwords add independently.
#pragma unroll
    for (int dv = 0; dv < 3; ++dv)
      acc[dv] = ((uint64_t)group_sum<M>((uint32_t)(acc[dv] >> 32)) << 32) |
                group_sum<M>((uint32_t)acc[dv]);
    if (ci < np && j == 0) {
#pragma unroll
      for (int dv = 0; dv < 3; ++dv) nbr[ci][dv] = acc[dv];
    }
  }
}

// ---------------------------------------------------------------------------
// Half-pel precision: SADs against H.263 half-pel samples, read from the
// ring.  Candidate (U, V) (half pixels) reads, for block row j, window row
// (V >> 1) + p + j (and the next one when V is odd) from byte
// (U >> 1) - u_lo of the block's first window column on (and the next byte
// when U is odd).  Valid candidates stay inside the window: |U|, |V| <= 2p.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ uint32_t ring_half_row(const uint32_t* __restrict__ ring,
                                                  const RingShape& w, int cb0,
                                                  const uint32_t* __restrict__ cd, int U, int V,
                                                  int j) {
  constexpr int NC = N / 4;
  const int xoff = (U >> 1) - w.s.u_lo;
  const int col = (cb0 + (xoff >> 2)) & (w.cw - 1);
  const int row0 = (V >> 1) + w.s.p + j;
  const uint32_t* r0 = ring + row0 * w.stride + col;
  const uint32_t* r1 = (V & 1) ? r0 + w.stride : r0;
  uint32_t d0[NC + 1], d1[NC + 1], c[NC];
#pragma unroll
  for (int q = 0; q <= NC; ++q) {
    d0[q] = r0[q];
    d1[q] = r1[q];
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) c[q] = cd[j * NC + q];
  return half_row_sad<NC>(d0, d1, (uint32_t)(xoff & 3), U & 1, V & 1, c, 0u);
}

// Half-pel SADs of the predictor candidates (cu, cv) into sadh: one lane
// per (candidate, block row), rows summed within groups of M lanes.
template <int N, int M, int NT>
__device__ __forceinline__ void pbm_half_sads(const uint32_t* __restrict__ ring,
                                              const RingShape& w, int cb0,
                                              const uint32_t* __restrict__ cd, const int16_t* cu,
                                              const int16_t* cv, int np, uint32_t* sadh) {
  constexpr int PER = NT / M;
  const int j = threadIdx.x % M;
  for (int base = 0; base < np; base += PER) {
    const int ci = base + (int)threadIdx.x / M;
    uint32_t acc = 0;
    if (ci < np) acc = ring_half_row<N>(ring, w, cb0, cd, cu[ci], cv[ci], j);
    acc = group_sum<M>(acc);
    if (ci < np && j == 0) sadh[ci] = acc;
  }
}

// Half-pel SADs of the ring neighbours k (bit k of `mask`) of (U0, V0) into
// sadr[k], by the first 8*M threads (whole waves).
template <int N, int M>
__device__ __forceinline__ void ring_half_sads(const uint32_t* __restrict__ ring,
                                               const RingShape& w, int cb0,
                                               const uint32_t* __restrict__ cd, int U0, int V0,
                                               uint32_t mask, uint32_t* sadr) {
  if ((int)threadIdx.x >= 8 * M) return;
  const int k = (int)threadIdx.x / M, j = (int)threadIdx.x % M;
  uint32_t acc = 0;
  if ((mask >> k) & 1u) {
    int du, dv;
    half_ring_offset(k, &du, &dv);
    acc = ring_half_row<N>(ring, w, cb0, cd, U0 + du, V0 + dv, j);
  }
  acc = group_sum<M>(acc);
  if (j == 0) sadr[k] = acc;
}

// Minimum over lanes 0..15 of a 64-bit key, left in each of those lanes
// (same DPP pattern as group_sum).
__device__ __forceinline__ uint64_t row_min_u64(uint64_t x) {
#define ACBM_ROW_MIN_STEP(CTRL)                                                       \
  {                                                                                   \
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)x, CTRL, 0xF, 0xF, false); \
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), CTRL, 0xF, 0xF, false); \
    const uint64_t y = ((uint64_t)hi << 32) | lo;                                     \
    x = y < x ? y : x;                                                                \
  }
  ACBM_ROW_MIN_STEP(0xB1)
  ACBM_ROW_MIN_STEP(0x4E)
  ACBM_ROW_MIN_STEP(0x141)
  ACBM_ROW_MIN_STEP(0x140)
#undef ACBM_ROW_MIN_STEP
  return x;
}

// Lane 0's value, in every lane (wave-uniform).
__device__ __forceinline__ uint64_t lane0_u64(uint64_t x) {
  return ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(x >> 32), 0) << 32) |
         __builtin_amdgcn_readlane((uint32_t)x, 0);
}

__device__ __forceinline__ uint32_t field16(uint64_t x, int i) {
  return (uint32_t)(x >> (16 * i)) & 0xFFFFu;
}

// ---------------------------------------------------------------------------
// Critical block: the full search.  Lane work unit = one quad of candidates
// (u_lo + 4q .. +3) times R candidate rows; the window row is the outer
// loop so that each window row is read once per task.  Every valid
// candidate is priced with this block's predictor in the same pass and the
// minimum key is reduced over the group.
// ---------------------------------------------------------------------------
template <int N, int M, int R>
__device__ __forceinline__ void task_sads_ring(const uint32_t* __restrict__ ring,
                                               const RingShape& w, int cb0, int q, int g,
                                               const uint32_t* __restrict__ cd,
                                               uint64_t (&acc)[R]) {
  constexpr int NC = N / 4;
  constexpr int WR = R + M - 1;  // window rows a task reads
#pragma unroll
  for (int rr = 0; rr < R; ++rr) acc[rr] = 0;
  const uint32_t* base = ring + (R * g) * w.stride + ((cb0 + q) & (w.cw - 1));
  // Block row j sits in cur[j % R] while window rows j .. j+R-1 pass.  The
  // outer loop over groups of R window rows stays rolled so that only one
  // group's loads are in registers at a time.
  uint32_t cur[R][NC];
#pragma unroll 1
  for (int w0 = 0; w0 < WR; w0 += R) {
    uint32_t wv[R][NC + 1];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int wr = w0 + i;
      if (wr < WR) {
        const uint32_t* rowp = base + wr * w.stride;
#pragma unroll
        for (int k = 0; k <= NC; ++k) wv[i][k] = rowp[k];
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int wr = w0 + i;
      // block row wr replaces row wr - R, whose last window row was wr - 1
      if (wr < M) {
#pragma unroll
        for (int k = 0; k < NC; ++k) cur[i][k] = cd[wr * NC + k];
      }
      if (wr < WR) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const uint64_t qw = (uint64_t)wv[i][k] | ((uint64_t)wv[i][k + 1] << 32);
#pragma unroll
          for (int rr = 0; rr < R; ++rr) {
            const int j = wr - rr;  // cur[j % R] = cur[(i - rr) mod R]
            if (j >= 0 && j < M)
              acc[rr] = __builtin_amdgcn_qsad_pk_u16_u8(qw, cur[(i - rr + R) % R][k], acc[rr]);
          }
        }
      }
    }
  }
}

// HP: the integer candidates are priced as half-pel vectors (2u, 2v) against
// the half-pel predictor, and keyed in the (4p+1)^2 half-pel window.
template <int N, int M, int R, bool HP>
__device__ __forceinline__ uint64_t critical_search(const uint32_t* __restrict__ ring,
                                                   const RingShape& w, int cb0,
                                                   const uint32_t* __restrict__ cd,
                                                   const ValidBox& vbox, int px, int py,
                                                   uint32_t lam, uint64_t* red) {
  constexpr int S = HP ? 2 : 1;
  const WindowShape& s = w.s;
  const int p = s.p, W = 2 * S * p + 1;
  // a block whose whole window is valid masks only the padding candidates
  const bool whole = vbox.u_min == -p && vbox.u_max == p && vbox.v_min == -p && vbox.v_max == p;
  const int tasks = s.quads * s.groups;
  uint64_t lbest = ~0ull;
#pragma unroll 1
  for (int task = threadIdx.x; task < tasks; task += blockDim.x) {
    const int gi = (int)__umulhi((uint32_t)task, s.qmagic);  // task / quads
    const int q = task - gi * s.quads;
    const int u0 = s.u_lo + 4 * q, v0 = -p + R * gi;
    uint64_t acc[R];
    task_sads_ring<N, M, R>(ring, w, cb0, q, gi, cd, acc);
    if (whole)
      mask_padding<R>(acc, p, u0, v0);
    else
      mask_invalid<R>(acc, vbox, u0, v0);
    uint32_t ru[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ru[i] = lam * se_bits(S * (u0 + i) - px);
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int v = v0 + rr;
      const uint32_t rv = lam * se_bits(S * v - py);
      const uint32_t rasb = (uint32_t)((S * v + S * p) * W + S * p);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t sad = field16(acc[rr], i);
        const int u = u0 + i;
        const uint64_t key =
            sad == 0xFFFFu ? ~0ull
                           : ((uint64_t)(sad + ru[i] + rv) << 32) |
                                 ((uint32_t)(S * (abs(u) + abs(v))) << 16) |
                                 (rasb + (uint32_t)(S * u));
        lbest = key < lbest ? key : lbest;
      }
    }
  }
  return group_min_u64(lbest, red);
}

__device__ __forceinline__ void write_result(acbm_block_result* out, uint32_t* word, int u, int v,
                                             uint32_t j, uint32_t rate, uint32_t lam,
                                             uint32_t cands, uint32_t mode, uint32_t intra) {
  put_result(out, u, v, j - lam * rate, j, rate, cands, mode, intra);
  store_word(word, kReady | pack_mv(u, v));
}

template <int N, int M, int R, int NT, bool HP>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(ACBM_PRED_WAVES)))
k_predictive(const PredArgs* __restrict__ jobs, const uint32_t* __restrict__ order,
             WsHeader* __restrict__ hdr, uint32_t total_rows, uint32_t spin_limit) {
  extern __shared__ uint32_t ring[];
  constexpr int D = M * N / 4;
  constexpr int NC = N / 4;
  static_assert(NT >= 128 && D <= NT - 64, "fetching waves must cover one current block");
  __shared__ uint64_t red[NT / 64];
  __shared__ uint32_t curd[2][D];
  __shared__ int16_t cu[kMaxCands], cv[kMaxCands];
  __shared__ uint64_t nbr[kMaxCands][3];
  __shared__ uint32_t sadh[kMaxCands], sadr[8];  // half-pel SADs: predictors, ring
  __shared__ uint32_t sh_row;
  __shared__ int sh_abort, sh_np, sh_px, sh_py;
  __shared__ uint32_t sh_intra;
  __shared__ uint16_t sh_left;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int f = (int)threadIdx.x - 64, nf = NT - 64;  // fetching lanes: waves 1..
  ACBM_PH(uint64_t ph[8] = {0, 0, 0, 0, 0, 0, 0, 0}; uint64_t ph_t0 = 0, ph_tw = 0;)

  for (;;) {
    ACBM_PH(const uint64_t ph_row = __builtin_amdgcn_s_memrealtime();)
    if (threadIdx.x == 0) {
      const uint32_t tk = atomicAdd(&hdr->ticket, 1u);
      sh_row = tk < total_rows ? order[tk] : 0xFFFFFFFFu;
      sh_abort = status_of(hdr) != 0;
    }
    __syncthreads();
    // LDS words are uniform; readfirstlane lets the compiler see that, so the
    // exits of this loop (which contains barriers) stay uniform branches
    const uint32_t rw = __builtin_amdgcn_readfirstlane(sh_row);
    if (rw == 0xFFFFFFFFu || __builtin_amdgcn_readfirstlane(sh_abort)) {
      ACBM_PH(if (threadIdx.x == 0) for (int k = 0; k < 8; ++k) atomicAdd(&g_phase[k], ph[k]);)
      return;
    }
    const PredArgs& a = jobs[rw >> 24];
    const int t = (int)((rw >> 12) & 0xFFFu);
    const int r = (int)(rw & 0xFFFu);
    const KGeom& g = a.g;
    const RingShape& w = a.w;
    const int p = g.p, bx = g.bx, by = g.by, nb = g.nb;
    const int W = 2 * (HP ? 2 : 1) * p + 1;  // key raster width (half-pel window with HP)
    const int y0 = r * M;
    const uint8_t* __restrict__ ref = ld_global<const uint8_t*>(a.frames + t);
    const uint8_t* __restrict__ cur = ld_global<const uint8_t*>(a.frames + t + 1);
    uint32_t* __restrict__ words = a.words + (size_t)t * nb;

    // first block of the row: its whole window and its current block
    load_columns<N>(ring, w, ref, g, y0, 0, w.s.dws);
    if (threadIdx.x < D) {
      const int j = threadIdx.x / NC, k = threadIdx.x % NC;
      curd[0][threadIdx.x] =
          ld_global<uint32_t>(cur + (size_t)(y0 + j) * g.pitch + 4 * k);
    }
    if (threadIdx.x == 0) sh_left = kMvUnset;
    uint32_t pre_word = 0;  // dependency word of this lane (wave 0), loaded one block ahead
    if (wave == 0) {
      const uint32_t* d0 = dep_word(a, words, lane, t, r, 0);
      pre_word = d0 ? load_word(d0) : 0u;
    }
    __syncthreads();
    ACBM_PH(if (threadIdx.x == 0) ph[7] += __builtin_amdgcn_s_memrealtime() - ph_row;)

    for (int c = 0; c < bx; ++c) {
      ACBM_PH(if (threadIdx.x == 0) ph_t0 = __builtin_amdgcn_s_memrealtime();)
      const int cb = c & 1;
      const uint32_t* cd = curd[cb];
      const int b = r * bx + c;
      const int x0 = c * N;
      const int cb0 = c * NC;  // first window column of this block
      const bool more = c + 1 < bx;

      // ---- A: neighbours, predictor and predictor set (wave 0); IntraX and
      //         the next block's columns (the other waves) ------------------
      ColFetch nxt;
      uint32_t nxt_cur = 0;
      if (wave == 0) {
        // lane 0: (0,0); 1: left (this row); 2..4: top-left, top, top-right;
        // 5..13: previous field at rows r-1..r+1, columns c-1..c+1
        const uint32_t* dw = dep_word(a, words, lane, t, r, c);
        uint16_t val = kMvUnset;  // kMvUnset = absent
        if (lane == 0) {
          val = pack_mv(0, 0);
        } else if (lane == 1) {
          if (c > 0) val = sh_left;
        } else if (lane >= 5 && lane < 14 && t == 0) {
          const int rr = r + (lane - 5) / 3 - 1, cc = c + (lane - 5) % 3 - 1;
          if (rr >= 0 && rr < by && cc >= 0 && cc < bx) {
            if (a.prev0) {
              // acbm_mv: x in the low, y in the high 16 bits.  A component
              // beyond +-127 would wrap in the packed byte; no such vector
              // is a valid candidate (p <= 127), so it is dropped here as
              // the validity test would drop it.
              const uint32_t m =
                  ld_global<uint32_t>(a.prev0 + (size_t)(rr * bx + cc) * a.prev0_stride);
              const int mx = (int16_t)(m & 0xFFFFu), my = (int16_t)(m >> 16);
              if (mx >= -127 && mx <= 127 && my >= -127 && my <= 127) val = pack_mv(mx, my);
            } else {
              val = pack_mv(0, 0);
            }
          }
        }
        uint32_t word = pre_word, spins = 0;
        bool failed = false;
        for (;;) {
          if (dw && !(word & kReady)) word = load_word(dw);
          if (__all(!dw || (word & kReady))) break;
          if (++spins > spin_limit || ((spins & 255) == 0 && status_of(hdr))) {
            failed = true;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        ACBM_PH(if (lane == 0) { ph_tw = __builtin_amdgcn_s_memrealtime(); ph[2] += ph_tw - ph_t0; })
        if (dw) val = (uint16_t)(word & 0xFFFFu);
        if (more) {
          const uint32_t* wn = dep_word(a, words, lane, t, r, c + 1);
          pre_word = wn ? load_word(wn) : 0u;
        }
        // predictor: median of left, top, top-right with the edge rules
        const uint32_t zero = pack_mv(0, 0);
        const uint32_t vl = __builtin_amdgcn_readlane((uint32_t)val, 1);
        const uint32_t vt = __builtin_amdgcn_readlane((uint32_t)val, 3);
        const uint32_t vtr = __builtin_amdgcn_readlane((uint32_t)val, 4);
        const uint16_t A = (uint16_t)(vl != kMvUnset ? vl : zero);
        const uint16_t B = r == 0 ? A : (uint16_t)vt;
        const uint16_t C = r == 0 ? A : (c == bx - 1 ? (uint16_t)zero : (uint16_t)vtr);
        const int px = med3(mv_x(A), mv_x(B), mv_x(C));
        const int py = med3(mv_y(A), mv_y(B), mv_y(C));
        // predictor set: valid candidates, first occurrence of each vector
        const int u = mv_x(val), v = mv_y(val);
        const bool ok = lane < 14 && val != kMvUnset &&
                        (HP ? cand_valid_half(u, v, p, x0, y0, N, M, g.width, g.height)
                            : cand_valid(u, v, p, x0, y0, N, M, g.width, g.height));
        const uint32_t tagged = ok ? (uint32_t)val : 0xFFFFFFFFu;
        bool dup = false;
#pragma unroll
        for (int q = 0; q < 13; ++q) dup |= (q < lane) & (__builtin_amdgcn_readlane(tagged, q) == tagged);
        const bool keep = ok && !dup;
        const uint64_t mask = __ballot(keep);
        if (keep) {
          const int pos = __builtin_popcountll(mask & ((1ull << lane) - 1));
          cu[pos] = (int16_t)u;
          cv[pos] = (int16_t)v;
        }
        if (lane == 0) {
          sh_np = __builtin_popcountll(mask);
          sh_px = px;
          sh_py = py;
          sh_abort = failed;
          if (failed) atomicOr(&hdr->status, kStatusSpinTimeout);
        }
      } else {
        if (more) {
          fetch_columns<N>(nxt, w, ref, g, y0, cb0 + w.s.dws, f, nf);
          if (f < D) {
            const int j = f / NC, k = f % NC;
            nxt_cur = ld_global<uint32_t>(cur + (size_t)(y0 + j) * g.pitch + x0 + N + 4 * k);
          }
        }
        if (wave == 1) {  // IntraX (Section 3.1) of the current block
          const uint32_t d = lane < D ? cd[lane] : 0u;
          const uint32_t ssum = wave_sum_u32(__builtin_amdgcn_sad_u8(d, 0u, 0u));
          uint32_t iacc = 0;
          if (lane < D) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int e = (int)(N * M) * (int)((d >> (8 * q)) & 0xFF) - (int)ssum;
              iacc += (uint32_t)(e < 0 ? -e : e);
            }
          }
          iacc = wave_sum_u32(iacc);
          if (lane == 0) sh_intra = iacc;
        }
      }
      __syncthreads();
      ACBM_PH(uint64_t ph_t1 = 0; if (threadIdx.x == 0) { ph_t1 = __builtin_amdgcn_s_memrealtime(); ph[3] += ph_t1 - ph_tw; })
      if (__builtin_amdgcn_readfirstlane(sh_abort)) return;
      const int px = __builtin_amdgcn_readfirstlane(sh_px);
      const int py = __builtin_amdgcn_readfirstlane(sh_py);
      const int np = __builtin_amdgcn_readfirstlane(sh_np);

      // ---- B: predictor neighbourhoods (all waves).  The predictor state is
      //         copied to registers before the barrier: once past it, wave 0
      //         may already rewrite it for the next block. ----------------
      const uint32_t intra = sh_intra;
      int cand_u = 0, cand_v = 0;
      if (lane < np) {
        cand_u = cu[lane];
        cand_v = cv[lane];
      }
      if constexpr (HP)
        pbm_half_sads<N, M, NT>(ring, w, cb0, cd, cu, cv, np, sadh);
      else
        pbm_neighbourhoods<N, M, NT>(ring, w, cb0, cd, cu, cv, np, nbr);
      __syncthreads();
      ACBM_PH(uint64_t ph_t2 = 0; if (threadIdx.x == 0) { ph_t2 = __builtin_amdgcn_s_memrealtime(); ph[4] += ph_t2 - ph_t1; })

      // ---- C: PBM steps 2 and 3, ACBM decision (every wave, redundantly, so
      //         that no barrier is needed to share it) -----------------------
      int crit_n = 0;  // candidates PBM evaluated, if the block is critical
      {
        const int u = cand_u, v = cand_v;
        constexpr int S = HP ? 2 : 1;  // key window of half-pel vectors with HP
        uint64_t key = ~0ull;
        if (lane < np) {
          const uint32_t sad = HP ? sadh[lane] : field16(nbr[lane][1], 1);
          key = make_key(sad + a.lam * (se_bits(u - px) + se_bits(v - py)), u, v, S * p);
        }
        // at most 14 predictors and 8 neighbours: minima over lanes 0..15
        const uint64_t k2 = lane0_u64(row_min_u64(key));
        const int bi = __builtin_ctzll(__ballot(lane < np && key == k2));
        const int bu = __builtin_amdgcn_readlane(u, bi), bv = __builtin_amdgcn_readlane(v, bi);
        // the valid 8-neighbours of the step-2 winner that are not predictors
        const int dd = lane < 4 ? lane : lane + 1;  // skip the centre
        const int du = dd % 3 - 1, dv = dd / 3 - 1;
        const int un = bu + du, vn = bv + dv;
        bool add = lane < 8 && (HP ? cand_valid_half(un, vn, p, x0, y0, N, M, g.width, g.height)
                                   : cand_valid(un, vn, p, x0, y0, N, M, g.width, g.height));
        const uint32_t mine = ((uint32_t)(u & 0xFFFF) << 16) | (uint32_t)(v & 0xFFFF);
        const uint32_t want = ((uint32_t)(un & 0xFFFF) << 16) | (uint32_t)(vn & 0xFFFF);
        for (int q = 0; q < np; ++q) add &= __builtin_amdgcn_readlane(mine, q) != want;
        if constexpr (HP) {
          // the ring's half-pel SADs: a second pass (every wave computed the
          // same ring, so the mask is uniform), shared through LDS
          ring_half_sads<N, M>(ring, w, cb0, cd, bu, bv, (uint32_t)__ballot(add), sadr);
          __syncthreads();
        }
        uint64_t key3 = ~0ull;
        if (add) {
          const uint32_t sad = HP ? sadr[lane] : field16(nbr[bi][dv + 1], du + 1);
          key3 = make_key(sad + a.lam * (se_bits(un - px) + se_bits(vn - py)), un, vn, S * p);
        }
        const uint64_t k3 = lane0_u64(row_min_u64(key3));
        const uint32_t n = (uint32_t)(np + __builtin_popcountll(__ballot(add)));
        int fu = bu, fv = bv;
        uint64_t best = k2;
        if (k3 < k2) {
          const int wl = __builtin_ctzll(__ballot(add && key3 == k3));
          fu = __builtin_amdgcn_readlane(un, wl);
          fv = __builtin_amdgcn_readlane(vn, wl);
          best = k3;
        }
        const uint32_t rate = se_bits(fu - px) + se_bits(fv - py);
        const uint32_t jv = (uint32_t)(best >> 32);
        const uint32_t sad = jv - a.lam * rate;
        int mode = ACBM_MODE_PBM;
        if (a.algo == ACBM_ALGO_ACBM) {
          const uint64_t nm = (uint64_t)(N * M), ix = intra;
          if (ix + nm * sad < a.c1_rhs) mode = ACBM_MODE_PBM_C1;
          else if ((uint64_t)a.gamma_den * nm * sad < (uint64_t)a.gamma_num * ix) mode = ACBM_MODE_PBM_C2;
          else mode = ACBM_MODE_CRITICAL;
        }
        if (mode == ACBM_MODE_CRITICAL) {
          crit_n = (int)n;
        } else if (threadIdx.x == 0) {
          write_result(a.out + (size_t)t * nb + b, words + b, fu, fv, jv, rate, a.lam, n,
                       (uint32_t)mode, intra);
          sh_left = pack_mv(fu, fv);
        }
      }

      ACBM_PH(uint64_t ph_t3 = 0; if (threadIdx.x == 0) { ph_t3 = __builtin_amdgcn_s_memrealtime(); ph[5] += ph_t3 - ph_t2; ph[0] += 1; })
      // ---- D: critical block: full search with the same predictor ---------
      if (crit_n) {  // uniform: every wave took the same decision
        const ValidBox vbox = valid_box(p, x0, y0, N, M, g.width, g.height);
        __builtin_amdgcn_s_setprio(3);  // the full search is on this row's critical path
        uint64_t best = critical_search<N, M, R, HP>(ring, w, cb0, cd, vbox, px, py, a.lam, red);
        uint32_t nh = 0;
        if constexpr (HP) {
          // the 8 half-pel positions around the integer winner
          const int hp = 2 * p, ras0 = (int)(best & 0xFFFFu);
          const int U0 = ras0 % W - hp, V0 = ras0 / W - hp;
          int du, dv;
          half_ring_offset(lane & 7, &du, &dv);
          const bool ok = lane < 8 && cand_valid_half(U0 + du, V0 + dv, p, x0, y0, N, M,
                                                      g.width, g.height);
          const uint64_t m = __ballot(ok);
          ring_half_sads<N, M>(ring, w, cb0, cd, U0, V0, (uint32_t)m, sadr);
          __syncthreads();
          uint64_t kk = ~0ull;
          if (ok)
            kk = make_key(sadr[lane] + a.lam * (se_bits(U0 + du - px) + se_bits(V0 + dv - py)),
                          U0 + du, V0 + dv, hp);
          kk = lane0_u64(row_min_u64(kk));
          best = kk < best ? kk : best;
          nh = (uint32_t)__builtin_popcountll(m);
        }
        __builtin_amdgcn_s_setprio(0);
        if (threadIdx.x == 0) {
          const int ras = (int)(best & 0xFFFFu);
          const int sp = (HP ? 2 : 1) * p;
          const int u = ras % W - sp, v = ras / W - sp;
          const uint32_t rate = se_bits(u - px) + se_bits(v - py);
          const uint32_t cands =
              (uint32_t)crit_n + valid_count(p, x0, y0, N, M, g.width, g.height) + nh;
          write_result(a.out + (size_t)t * nb + b, words + b, u, v, (uint32_t)(best >> 32), rate,
                       a.lam, cands, ACBM_MODE_CRITICAL, intra);
          sh_left = pack_mv(u, v);
          ACBM_PH(ph[6] += __builtin_amdgcn_s_memrealtime() - ph_t3; ph[1] += 1;)
        }
      }

      // ---- E: park what block c+1 adds.  No barrier: the next block's first
      //         barrier orders these writes before any read of them, and
      //         wave 0 meanwhile only touches the predictor state. -----------
      if (more && wave > 0) {
        park_columns<N>(ring, nxt, w, ref, g, y0, cb0 + w.s.dws, f, nf);
        if (f < D) curd[cb ^ 1][f] = nxt_cur;
      }
    }
    __syncthreads();  // the row's last block is done before the ring is refilled
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int row_levels(const KGeom& g, int npairs) { return (g.by - 1) + 2 * (npairs - 1) + 1; }

// Workspace of the single-job calls, reused by each launch of up to
// kMaxPairsPerLaunch pairs: header, row order, vector words, frame pointers
// and the one-entry job table.
size_t predictive_ws_bytes(const KGeom& g, uint32_t npairs) {
  const uint32_t per = std::min<uint32_t>(npairs, kMaxPairsPerLaunch);
  return align256(sizeof(WsHeader)) + align256((size_t)per * g.by * sizeof(uint32_t)) +
         align256((size_t)per * g.nb * sizeof(uint32_t)) +
         align256((size_t)(kMaxPairsPerLaunch + 1) * sizeof(void*)) + align256(sizeof(PredArgs));
}

template <int N, int M>
static RingShape ring_shape(int p, int R) {
  RingShape w;
  w.s = window_shape<N, M>(p, R);
  w.cw = 1;
  while (w.cw < w.s.dws + N / 4) w.cw <<= 1;
  w.stride = (w.cw + N / 4 + 2) | 1;
  return w;
}

static RingShape ring_for(const KGeom& g, int R) {
  if (g.bw == 16 && g.bh == 16) return ring_shape<16, 16>(g.p, R);
  if (g.bw == 16 && g.bh == 8) return ring_shape<16, 8>(g.p, R);
  if (g.bw == 8 && g.bh == 16) return ring_shape<8, 16>(g.p, R);
  return ring_shape<8, 8>(g.p, R);
}

static size_t ring_bytes(const RingShape& w) { return (size_t)w.s.rows * w.stride * 4; }

#define ACBM_PRED_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8)

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

// Row walkers per CU: as many as fit (the default), or fewer when
// ACBM_PRED_WALKERS_PER_CU says so; walkers on one CU share its SIMDs.
static int walkers_per_cu() {
  static int n = [] {
    const char* e = std::getenv("ACBM_PRED_WALKERS_PER_CU");
    const int v = e ? std::atoi(e) : 0;
    return v > 0 ? v : 1 << 20;
  }();
  return n;
}

struct PredLaunch {
  const PredArgs* jobs;
  const uint32_t* order;
  WsHeader* hdr;
  uint32_t total_rows;
  size_t lds;
  uint32_t spin_limit;
};

// Polls of a dependency wait before it gives up: kSpinLimit, or
// ACBM_PRED_SPIN_LIMIT (read at every launch), with which tests force the
// time-out path; the kernel then records the failure and every walker leaves.
static uint32_t spin_limit() {
  const char* e = std::getenv("ACBM_PRED_SPIN_LIMIT");
  const long v = e ? std::atol(e) : 0;
  return v > 0 ? (uint32_t)std::min<long>(v, (long)kSpinLimit) : kSpinLimit;
}

template <int N, int M, int NT, bool HP = false>
static int launch_pred_nmt(const PredLaunch& L, int R, hipStream_t st) {
  switch (R) {
#define ACBM_CASE(RR)                                                                        \
  case RR: {                                                                                 \
    const void* fn = (const void*)k_predictive<N, M, RR, NT, HP>;                            \
    if (L.lds > 64 * 1024)                                                                   \
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds); \
    int per_cu = 0;                                                                          \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, L.lds) != hipSuccess || \
        per_cu < 1)                                                                          \
      per_cu = 1;                                                                            \
    per_cu = std::min(per_cu, walkers_per_cu());                                             \
    /* about as many row walkers as can be resident, never more than rows */                \
    const int grid = (int)std::min<size_t>((size_t)device_cus() * per_cu, L.total_rows);    \
    ProfScope ps("predictive", st);                                                          \
    hipLaunchKernelGGL((k_predictive<N, M, RR, NT, HP>), dim3(grid), dim3(NT), L.lds, st,    \
                       L.jobs, L.order, L.hdr, L.total_rows, L.spin_limit);                  \
    break;                                                                                   \
  }
    ACBM_PRED_R_LIST(ACBM_CASE)
#undef ACBM_CASE
    default:
      return fail(ACBM_E_UNSUPPORTED, "no predictive kernel for this row blocking");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the predictive search");
}

// Half-pel precision runs with 256-thread walkers only.
template <int N, int M>
static int launch_pred_nm(const PredLaunch& L, int R, int nt, bool hp, hipStream_t st) {
  if (hp) return launch_pred_nmt<N, M, 256, true>(L, R, st);
  if (nt == 128) return launch_pred_nmt<N, M, 128>(L, R, st);
  if (nt == 512) return launch_pred_nmt<N, M, 512>(L, R, st);
  return launch_pred_nmt<N, M, 256>(L, R, st);
}

// Threads per row walker at integer precision (half-pel walkers always have
// 256).  A group of several sequences has rows to spare, so more, smaller
// walkers keep more rows in flight: on the 64-sequence batch its 8x8 group
// (28 sequences) took 9.6 ms with 128 threads against 11.8 with 256, its
// 16x16 group (36 sequences) 4.9 against 5.3.  One sequence is bound by its
// dependency chain instead, and its critical searches want the larger
// walkers (1920x1088 p = 32, 59 pairs: 10.8 ms with 128 threads against 6.9
// with 256).  Many jobs of one pair each (a served pass: up to 15 requests
// of 640x480 to 3840x2160 at p = 16-64) have only one pair's rows per job
// and are chain-bound like one sequence: 1,930 requests/s saturated with 256
// threads against 1,130 with 128.  So groups of at least four jobs with at
// least four pairs per job on average take 128 threads.
// ACBM_ROW_THREADS (128, 256 or 512) overrides.
static int row_threads(int njobs, double mean_pairs) {
  const char* e = std::getenv("ACBM_ROW_THREADS");
  if (e && *e) {
    const int v = std::atoi(e);
    return (v == 128 || v == 512) ? v : 256;
  }
  return njobs >= 4 && mean_pairs >= 4.0 ? 128 : 256;
}

// Row blocking R of the critical search.  When a launch has more block rows
// than the device has CUs, walkers share CUs and the launch is bound by the
// rows in flight times the per-block latency.  Measured there (16x16 and
// 8x8 walkers fit four per CU up to R = 3, 8x8 at R = 1 five):
//  * 1920x1088 16x16 p = 32 ACBM, 59 pairs: R = 3 6.4 ms, 1 6.9, 2 7.3;
//    with every block critical R = 3 10.6 ms, 1 11.3, 2 12.1;
//  * the same at half-pel precision: R = 1 7.7 ms, 3 7.8, 2 8.3;
//  * the 64-sequence batch's 8x8 group (28 sequences): R = 1 11.8 ms, 2 13.0,
//    3 14.6, 4 18.4, 5 20.2, 6 21.4; its 16x16 group: R = 1 5.0 ms, 3 5.2.
// So shared CUs take R = 3 for 16-wide blocks at integer precision and R = 1
// otherwise.  Alone on its CU, a walker's critical search latency matters:
// the least issue time per lane, rounds * (QSAD cycles of a task + its loads
// and pricing), among the R whose ring fits in LDS (a single HD pair: R = 5,
// 2.0 ms against 2.6 ms with R = 3).  ACBM_PRED_R overrides.
static int pick_rows(const KGeom& g, int nt, size_t total_rows, bool hp) {
  const bool shared_cus = total_rows > (size_t)device_cus();
  const char* force = std::getenv("ACBM_PRED_R");
  if (force && !*force) force = nullptr;  // set but empty: as if unset
  if (!force && shared_cus) {
    for (int R = (g.bw == 16 && !hp) ? 3 : 1; R >= 1; --R)
      if (ring_bytes(ring_for(g, R)) <= (size_t)lds_limit()) return R;
    return 0;
  }
  const int nc = g.bw / 4;
  int bestR = 0;
  long best = 0;
  for (int R : {1, 2, 3, 4, 5, 6, 8}) {
    const RingShape w = ring_for(g, R);
    if (ring_bytes(w) > (size_t)lds_limit()) continue;
    if (force && std::atoi(force) != R) continue;
    const long rounds = (w.s.quads * w.s.groups + nt - 1) / nt;
    const long cost = rounds * ((long)R * g.bh * nc * 16 + 8L * (R + g.bh - 1) + 160L * R);
    if (!bestR || cost < best) {
      bestR = R;
      best = cost;
    }
  }
  return bestR;
}

int plan_predictive_group(const KGeom* geoms, int n, bool hp, size_t total_rows,
                          PredGroupPlan* pl) {
  if (n < 1) return fail(ACBM_E_INVAL, "a predictive group needs a job");
  int imax = 0;  // the largest window decides which row blockings fit in LDS
  for (int i = 1; i < n; ++i)
    if (geoms[i].p > geoms[imax].p) imax = i;
  size_t rows_per_pair = 0;  // block rows of one pair of every job
  for (int i = 0; i < n; ++i) rows_per_pair += (size_t)geoms[i].by;
  const double mean_pairs = rows_per_pair ? (double)total_rows / (double)rows_per_pair : 0.0;
  pl->threads = hp ? 256 : row_threads(n, mean_pairs);
  pl->R = pick_rows(geoms[imax], pl->threads, total_rows, hp);
  if (!pl->R) return fail(ACBM_E_UNSUPPORTED, "search window too large for the predictive kernel");
  pl->lds = 0;
  for (int i = 0; i < n; ++i) pl->lds = std::max(pl->lds, ring_bytes(ring_for(geoms[i], pl->R)));
  return ACBM_OK;
}

PredArgs predictive_args(const KGeom& g, const acbm_params& prm, int algo, int R,
                         uint32_t npairs) {
  PredArgs a{};
  a.g = g;
  a.w = ring_for(g, R);
  a.algo = algo;
  a.lam = prm.lambda;
  const unsigned __int128 t1 =
      ((unsigned __int128)prm.alpha + (unsigned __int128)prm.beta * prm.qp * prm.qp) *
      (unsigned __int128)(g.bw * g.bh);
  a.c1_rhs = t1 > (unsigned __int128)UINT64_MAX ? UINT64_MAX : (uint64_t)t1;
  a.gamma_num = prm.gamma_num;
  a.gamma_den = prm.gamma_den;
  a.npairs = (int)npairs;
  a.row_levels = row_levels(g, (int)npairs);
  return a;
}

int launch_predictive_group(int bw, int bh, bool hp, const PredGroupPlan& pl,
                            const PredArgs* jobs, int njobs, uint32_t* order, WsHeader* hdr,
                            uint32_t total_rows, hipStream_t st) {
  if (njobs < 1 || njobs > kPredMaxJobs) return fail(ACBM_E_INVAL, "bad predictive group size");
  if (!total_rows) return ACBM_OK;
  {
    ProfScope ps("setup", st);
    hipLaunchKernelGGL(k_pred_setup, dim3(64, njobs), dim3(256), 0, st, jobs, njobs, order, hdr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "launching the predictive setup");
  const PredLaunch L{jobs, order, hdr, total_rows, pl.lds, spin_limit()};
  if (bw == 16 && bh == 16) return launch_pred_nm<16, 16>(L, pl.R, pl.threads, hp, st);
  if (bw == 16 && bh == 8) return launch_pred_nm<16, 8>(L, pl.R, pl.threads, hp, st);
  if (bw == 8 && bh == 16) return launch_pred_nm<8, 16>(L, pl.R, pl.threads, hp, st);
  return launch_pred_nm<8, 8>(L, pl.R, pl.threads, hp, st);
}

#ifdef ACBM_PHASE_PROFILE
// Reads (and with reset != 0 clears) the walkers' phase totals; exported by
// the profiling build only.
extern "C" int acbm_phase_profile_read(uint64_t* out8, int reset) {
  if (!out8) return fail(ACBM_E_INVAL, "out is NULL");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpyFromSymbol(out8, HIP_SYMBOL(g_phase), 8 * sizeof(uint64_t));
  if (e == hipSuccess && reset) {
    const uint64_t zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_phase), zero, sizeof(zero));
  }
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "reading the phase profile");
}
#endif

int launch_predictive(const KGeom& g, const acbm_params& prm, int algo,
                      const uint8_t* const* frames, uint32_t npairs, const acbm_mv* prev_field,
                      void* ws, size_t ws_bytes, acbm_block_result* out, hipStream_t st) {
  if (ws_bytes < predictive_ws_bytes(g, npairs)) return fail(ACBM_E_NOMEM, "workspace too small");
  const bool hp = prm.subpel != 0;
  const uint32_t per = std::min<uint32_t>(npairs, kMaxPairsPerLaunch);
  PredGroupPlan pl;
  int rc = plan_predictive_group(&g, 1, hp, (size_t)per * g.by, &pl);
  if (rc) return rc;
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  WsHeader* hdr = reinterpret_cast<WsHeader*>(base);
  off += align256(sizeof(WsHeader));
  uint32_t* order = reinterpret_cast<uint32_t*>(base + off);
  off += align256((size_t)per * g.by * sizeof(uint32_t));
  uint32_t* words = reinterpret_cast<uint32_t*>(base + off);
  off += align256((size_t)per * g.nb * sizeof(uint32_t));
  const uint8_t** fptr = reinterpret_cast<const uint8_t**>(base + off);
  off += align256((size_t)(kMaxPairsPerLaunch + 1) * sizeof(void*));
  PredArgs* table = reinterpret_cast<PredArgs*>(base + off);
  for (uint32_t p0 = 0; p0 < npairs; p0 += kMaxPairsPerLaunch) {
    const int n = (int)std::min<uint32_t>(kMaxPairsPerLaunch, npairs - p0);
    PredArgs a = predictive_args(g, prm, algo, pl.R, (uint32_t)n);
    if (p0 == 0) {
      a.prev0 = reinterpret_cast<const uint8_t*>(prev_field);
      a.prev0_stride = sizeof(acbm_mv);
    } else {  // the previous launch's last pair
      a.prev0 = reinterpret_cast<const uint8_t*>(out + (size_t)(p0 - 1) * g.nb);
      a.prev0_stride = sizeof(acbm_block_result);
    }
    a.hdr = hdr;
    a.words = words;
    a.frames = fptr;
    a.out = out + (size_t)p0 * g.nb;
    FramePtrs fr{};
    for (int k = 0; k <= n; ++k) fr.f[k] = frames[p0 + k];
    hipLaunchKernelGGL(k_pred_put_job, dim3(1), dim3(128), 0, st, a, fr, table, fptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "writing the predictive job");
    if ((rc = launch_predictive_group(g.bw, g.bh, hp, pl, table, 1, order, hdr,
                                      (uint32_t)n * g.by, st)))
      return rc;
  }
  return ACBM_OK;
}

}  // namespace acbm
