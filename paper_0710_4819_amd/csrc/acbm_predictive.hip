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
//    frames run at once (pair t starts while pair t-1 is still running).  A row walker has 128 threads
//    by default: on the 1920x1088 p = 32 sequence that measured faster than
//    64 (longer critical searches) and 256 (fewer rows in flight).
//  * Publication.  A finished block stores its vector together with a ready
//    bit in one 32-bit word (relaxed, device scope); consumers poll exactly
//    the words they need, so no fences are required.  The words of the next
//    block are loaded one block ahead.  Every wait is bounded: on time-out
//    the kernel records the failure in the workspace header and all waves
//    leave.
//  * Window.  Consecutive blocks of a row share all but N/4 dword columns of
//    their search windows, so the window lives in a circular buffer of `cw`
//    columns (a power of two >= window + N/4): each block fetches the N/4
//    columns its right neighbour adds, into registers while it works, and
//    parks them in columns it no longer needs.
//  * Work per block.  Predictor and ring SADs use one lane per dword of the
//    block (V_SAD_U8 on byte-aligned window dwords, DPP reduction); a
//    critical block (ACBM) runs the QSAD window search of the full-search
//    kernel, first for the SAD minimum, then pricing only the candidates
//    within lambda*(Rmax-2) of it (nothing else can win: R >= 2 everywhere
//    and R <= Rmax).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "acbm_device.h"
#include "acbm_internal.h"

namespace acbm {

constexpr uint32_t kReady = 0x80000000u;
constexpr int kMaxCands = 14 + 8;
constexpr int kFetch = 8;                 // new-column dwords each lane fetches ahead
constexpr int kMaxRounds = 16;            // task rounds of the pruned critical search
constexpr uint32_t kSpinLimit = 1u << 22;

// Circular window: absolute dword column a lives at a & (cw-1); rows are
// cw+1 dwords apart (odd, against bank conflicts).
struct RingShape {
  WindowShape s;
  int cw;
  int stride;
};

struct PredArgs {
  KGeom g;
  RingShape w;
  int algo;
  uint32_t lam;
  uint64_t c1_rhs;        // N*M*(alpha + beta*qp^2), saturated
  uint32_t gamma_num, gamma_den;
  uint32_t slack;         // lambda * (Rmax - 2): pruning bound of the full search
  int npairs;
  int row_levels;         // (by-1) + 2(npairs-1) + 1
  const uint8_t* prev0;   // temporal field of pair 0 (acbm_mv at byte stride), or null
  int prev0_stride;
  WsHeader* hdr;
  uint32_t* row_order;    // [npairs*by] ticket -> (t << 16) | r
  uint32_t* words;        // [npairs][nb] published vectors
  acbm_block_result* out;
};

// Rows (t, r) with r + 2t = k.
__host__ __device__ inline int row_tlo(int k, int by) { return max(0, (k - (by - 1) + 1) / 2); }
__host__ __device__ inline int row_thi(int k, int npairs) { return min(npairs - 1, k / 2); }

// Prepares the workspace of one launch: row order, cleared vector words,
// ticket and status.  (A kernel rather than hipMemsetAsync so that the
// sequence can be captured in a graph.)
__global__ void k_pred_setup(PredArgs a) {
  const size_t nw = (size_t)a.npairs * a.g.nb;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (size_t)gridDim.x * blockDim.x)
    a.words[i] = 0;
  if (blockIdx.x == 0) {
    const int by = a.g.by;
    for (int k = threadIdx.x; k < a.row_levels; k += blockDim.x) {
      int off = 0;  // rows in levels before k
      for (int q = 0; q < k; ++q) off += max(0, row_thi(q, a.npairs) - row_tlo(q, by) + 1);
      for (int t = row_tlo(k, by); t <= row_thi(k, a.npairs); ++t)
        a.row_order[off++] = ((uint32_t)t << 16) | (uint32_t)(k - 2 * t);
    }
    if (threadIdx.x == 0) {
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
__device__ __forceinline__ uint32_t status_of(const WsHeader* h) {
  return __hip_atomic_load(&h->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    return *reinterpret_cast<const uint32_t*>(ref + (size_t)y * g.pitch + x);
  return 0u;
}

// Window columns [a0, a0 + ncol) of all rows straight into the ring; column
// a of the row strip covers x = u_lo + 4a.
__device__ __forceinline__ void load_columns(uint32_t* __restrict__ ring, const RingShape& w,
                                             const uint8_t* __restrict__ ref, const KGeom& g,
                                             int y0, int a0, int ncol) {
  const int total = w.s.rows * ncol;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int row = idx / ncol, a = a0 + idx % ncol;
    ring[row * w.stride + (a & (w.cw - 1))] = ref_dword(ref, g, w.s.u_lo + 4 * a, y0 - w.s.p + row);
  }
}

// The N/4 columns block c+1 adds, fetched into registers.
struct ColFetch {
  uint32_t v[kFetch];
};

template <int N, int NT>
__device__ __forceinline__ void fetch_columns(ColFetch& f, const RingShape& w,
                                              const uint8_t* __restrict__ ref, const KGeom& g,
                                              int y0, int a0) {
  constexpr int NC = N / 4;
  const int total = w.s.rows * NC;
#pragma unroll
  for (int k = 0; k < kFetch; ++k) {
    const int idx = threadIdx.x + k * NT;
    const int row = idx / NC, a = a0 + idx % NC;
    f.v[k] = idx < total ? ref_dword(ref, g, w.s.u_lo + 4 * a, y0 - w.s.p + row) : 0u;
  }
}

template <int N, int NT>
__device__ __forceinline__ void park_columns(uint32_t* __restrict__ ring, const ColFetch& f,
                                             const RingShape& w, const uint8_t* __restrict__ ref,
                                             const KGeom& g, int y0, int a0) {
  constexpr int NC = N / 4;
  const int total = w.s.rows * NC;
#pragma unroll
  for (int k = 0; k < kFetch; ++k) {
    const int idx = threadIdx.x + k * NT;
    if (idx < total) ring[(idx / NC) * w.stride + ((a0 + idx % NC) & (w.cw - 1))] = f.v[k];
  }
  for (int idx = threadIdx.x + kFetch * NT; idx < total; idx += blockDim.x) {
    const int row = idx / NC, a = a0 + idx % NC;
    ring[row * w.stride + (a & (w.cw - 1))] = ref_dword(ref, g, w.s.u_lo + 4 * a, y0 - w.s.p + row);
  }
}

// SADs of candidates [first, n) of the list; one lane per dword of the
// block, D = N*M/4 lanes per candidate.  cb0 = first window column of the
// block (absolute).  Up to kBatch candidates per wave are loaded before any
// is reduced, so their LDS latencies overlap.
constexpr int kBatch = 8;

template <int N, int M>
__device__ inline void list_sads(const uint32_t* __restrict__ ring, const RingShape& w, int cb0,
                                 const uint32_t* __restrict__ curd, const int16_t* cu,
                                 const int16_t* cv, uint32_t* sads, int first, int n) {
  constexpr int D = M * N / 4;
  constexpr int CPW = 64 / D;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int slot = lane / D, l = lane % D;
  const int j = l / (N / 4), k = l % (N / 4);
  const uint32_t mine = curd[l];
  const int cmask = w.cw - 1;
  for (int base = first + wave * CPW * kBatch; base < n; base += nwaves * CPW * kBatch) {
    uint32_t part[kBatch];
#pragma unroll
    for (int e = 0; e < kBatch; ++e) {
      const int ci = base + e * CPW + slot;
      part[e] = 0;
      if (ci < n) {
        const int u = cu[ci], v = cv[ci];
        const int off = u - w.s.u_lo + 4 * k;
        const uint32_t* rowp = ring + (v + w.s.p + j) * w.stride;
        const int a = cb0 + (off >> 2);
        const uint32_t lo = rowp[a & cmask], hi = rowp[(a + 1) & cmask];
        part[e] = __builtin_amdgcn_sad_u8(__builtin_amdgcn_alignbyte(hi, lo, (uint32_t)(off & 3)),
                                          mine, 0u);
      }
    }
#pragma unroll
    for (int e = 0; e < kBatch; ++e) {
      if (base + e * CPW >= n) break;  // wave-uniform
      uint32_t sum;
      if constexpr (D == 64) {
        sum = wave_sum_u32(part[e]);
      } else {
        sum = part[e];
#pragma unroll
        for (int o = D / 2; o >= 1; o >>= 1) sum += (uint32_t)__shfl_xor((int)sum, o, 64);
      }
      const int ci = base + e * CPW + slot;
      if (ci < n && l == 0) sads[ci] = sum;
    }
  }
}

// SADs of one task of the window search over the circular window: acc[rr]
// holds candidates u_lo + 4q + i (i = 0..3) of row v = -p + R*g + rr.  The
// current-block row is the outer, rolled loop, so only N/4 of its dwords are
// live at a time; each iteration first loads every window dword it needs
// (R rows x N/4+1 columns) and only then issues its QSADs, so one LDS
// latency is paid per current-block row rather than per QSAD.
template <int N, int M, int R>
__device__ __forceinline__ void task_sads_ring(const uint32_t* __restrict__ ring,
                                               const RingShape& w, int cb0, int q, int g,
                                               const uint32_t* __restrict__ cd,
                                               uint64_t (&acc)[R]) {
  constexpr int NC = N / 4;
  int col[NC + 1];
#pragma unroll
  for (int k = 0; k <= NC; ++k) col[k] = (cb0 + q + k) & (w.cw - 1);
#pragma unroll
  for (int rr = 0; rr < R; ++rr) acc[rr] = 0;
  const uint32_t* base = ring + (R * g) * w.stride;
#pragma unroll 1
  for (int j = 0; j < M; ++j) {
    uint32_t c[NC];
    uint32_t wv[R][NC + 1];
#pragma unroll
    for (int k = 0; k < NC; ++k) c[k] = cd[j * NC + k];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const uint32_t* rowp = base + (rr + j) * w.stride;
#pragma unroll
      for (int k = 0; k <= NC; ++k) wv[rr][k] = rowp[col[k]];
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const uint64_t qw = (uint64_t)wv[rr][k] | ((uint64_t)wv[rr][k + 1] << 32);
        acc[rr] = __builtin_amdgcn_qsad_pk_u16_u8(qw, c[k], acc[rr]);
      }
  }
}

// Critical block: minimum key of J over the whole valid window with this
// block's predictor, reduced over the group.  Pass 1 finds the SAD minimum
// (remembering each round's lane minimum in `rmin`, kMaxRounds x group
// size); pass 2 recomputes only the rounds that hold a candidate within the
// pruning bound and prices those.
template <int N, int M, int R>
__device__ __forceinline__ uint64_t critical_search(const uint32_t* __restrict__ ring,
                                                   const RingShape& w, int cb0,
                                                   const uint32_t* cd, const ValidBox& vbox,
                                                   int px, int py, uint32_t lam, uint32_t slack,
                                                   uint64_t* red, uint16_t* rmin) {
  const WindowShape& s = w.s;
  const int p = s.p;
  const int tasks = s.quads * s.groups;
  const int rounds = (tasks + (int)blockDim.x - 1) / (int)blockDim.x;
  uint32_t lmin = 0xFFFFu;
#pragma unroll 1
  for (int k = 0; k < rounds; ++k) {
    const int task = threadIdx.x + k * blockDim.x;
    uint32_t m = 0xFFFFu;
    if (task < tasks) {
      const int q = task % s.quads, gi = task / s.quads;
      uint64_t acc[R];
      task_sads_ring<N, M, R>(ring, w, cb0, q, gi, cd, acc);
      mask_invalid<R>(acc, vbox, s.u_lo + 4 * q, -p + R * gi);
      m = min_u16_lanes<R>(acc);
    }
    rmin[k * blockDim.x + threadIdx.x] = (uint16_t)m;
    lmin = min(lmin, m);
  }
  const uint32_t smin = (uint32_t)group_min_u64(lmin, red);
  const uint32_t thr = (uint32_t)min<uint64_t>((uint64_t)smin + slack, 0xFFFEu);
  uint64_t lbest = ~0ull;
#pragma unroll 1
  for (int k = 0; k < rounds; ++k) {
    if (rmin[k * blockDim.x + threadIdx.x] > thr) continue;  // also rounds past the last task
    const int task = threadIdx.x + k * blockDim.x;
    const int q = task % s.quads, gi = task / s.quads;
    const int u0 = s.u_lo + 4 * q, v0 = -p + R * gi;
    uint64_t acc[R];
    task_sads_ring<N, M, R>(ring, w, cb0, q, gi, cd, acc);
    mask_invalid<R>(acc, vbox, u0, v0);
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t sad = (uint32_t)(acc[rr] >> (16 * i)) & 0xFFFFu;
        if (sad > thr) continue;
        const int u = u0 + i, v = v0 + rr;
        const uint32_t j = sad + lam * (se_bits(u - px) + se_bits(v - py));
        const uint64_t key = make_key(j, u, v, p);
        lbest = key < lbest ? key : lbest;
      }
  }
  return group_min_u64(lbest, red);
}

template <int N, int M, int R, int NT>
__global__ void __launch_bounds__(NT) k_predictive(const PredArgs a, const FramePtrs fr) {
  extern __shared__ uint32_t ring[];
  constexpr int D = M * N / 4;
  constexpr int NC = N / 4;
  __shared__ uint64_t red[NT / 64];
  __shared__ uint32_t curd[2][D];
  __shared__ int16_t cu[kMaxCands], cv[kMaxCands];
  __shared__ uint32_t csad[kMaxCands];
  __shared__ int sh_row, sh_abort, sh_n, sh_np, sh_px, sh_py, sh_crit;
  __shared__ uint32_t sh_intra;
  __shared__ uint16_t sh_left;
  __shared__ uint16_t rmin[kMaxRounds * NT];

  const KGeom& g = a.g;
  const RingShape& w = a.w;
  const int p = g.p, bx = g.bx, by = g.by, nb = g.nb;
  const uint32_t total_rows = (uint32_t)a.npairs * by;
  const int lane = threadIdx.x & 63;
  const bool w0 = threadIdx.x < 64;  // wave 0 does the per-block bookkeeping

  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t tk = atomicAdd(&a.hdr->ticket, 1u);
      sh_row = tk < total_rows ? (int)a.row_order[tk] : -1;
      sh_abort = status_of(a.hdr) != 0;
    }
    __syncthreads();
    if (sh_row < 0 || sh_abort) return;
    const int t = __builtin_amdgcn_readfirstlane(sh_row >> 16);
    const int r = __builtin_amdgcn_readfirstlane(sh_row & 0xFFFF);
    const int y0 = r * M;
    const uint8_t* __restrict__ ref = fr.f[t];
    const uint8_t* __restrict__ cur = fr.f[t + 1];
    uint32_t* __restrict__ words = a.words + (size_t)t * nb;

    // first block of the row: its whole window and its current block
    load_columns(ring, w, ref, g, y0, 0, w.s.dws);
    if (threadIdx.x < D) {
      const int j = threadIdx.x / NC, k = threadIdx.x % NC;
      curd[0][threadIdx.x] =
          *reinterpret_cast<const uint32_t*>(cur + (size_t)(y0 + j) * g.pitch + 4 * k);
    }
    if (threadIdx.x == 0) sh_left = kMvUnset;
    uint32_t pre_word = 0;  // dependency word of this lane (wave 0), loaded one block ahead
    if (w0) {
      const uint32_t* d0 = dep_word(a, words, lane, t, r, 0);
      pre_word = d0 ? load_word(d0) : 0u;
    }
    __syncthreads();

    for (int c = 0; c < bx; ++c) {
      const int cb = c & 1;
      const uint32_t* cd = curd[cb];
      const int b = r * bx + c;
      const int x0 = c * N;
      const int cb0 = c * NC;  // first window column of this block

      // ---- fetch what block c+1 adds (in flight while this block works) ---
      ColFetch nxt;
      uint32_t nxt_cur = 0;
      const bool more = c + 1 < bx;
      if (more) {
        fetch_columns<N, NT>(nxt, w, ref, g, y0, cb0 + w.s.dws);
        if (threadIdx.x < D) {
          const int j = threadIdx.x / NC, k = threadIdx.x % NC;
          nxt_cur = *reinterpret_cast<const uint32_t*>(cur + (size_t)(y0 + j) * g.pitch + x0 + N +
                                                       4 * k);
        }
      }

      // ---- wait for the neighbours, predictor, predictor set, IntraX ------
      if (w0) {
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
              const acbm_mv m = *reinterpret_cast<const acbm_mv*>(
                  a.prev0 + (size_t)(rr * bx + cc) * a.prev0_stride);
              val = pack_mv(m.x, m.y);
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
          if (++spins > kSpinLimit || ((spins & 255) == 0 && status_of(a.hdr))) {
            failed = true;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (dw) val = (uint16_t)(word & 0xFFFFu);
        if (more) {
          const uint32_t* wn = dep_word(a, words, lane, t, r, c + 1);
          pre_word = wn ? load_word(wn) : 0u;
        }
        // predictor: median of left, top, top-right with the edge rules
        const uint16_t zero = pack_mv(0, 0);
        const uint16_t vl = (uint16_t)__shfl((int)val, 1, 64);
        const uint16_t vt = (uint16_t)__shfl((int)val, 3, 64);
        const uint16_t vtr = (uint16_t)__shfl((int)val, 4, 64);
        const uint16_t A = vl != kMvUnset ? vl : zero;
        const uint16_t B = r == 0 ? A : vt;
        const uint16_t C = r == 0 ? A : (c == bx - 1 ? zero : vtr);
        const int px = med3(mv_x(A), mv_x(B), mv_x(C));
        const int py = med3(mv_y(A), mv_y(B), mv_y(C));
        // predictor set: valid candidates, first occurrence of each vector
        const int u = mv_x(val), v = mv_y(val);
        const bool ok = lane < 14 && val != kMvUnset &&
                        cand_valid(u, v, p, x0, y0, N, M, g.width, g.height);
        bool dup = false;
#pragma unroll
        for (int q = 0; q < 13; ++q) {
          const int oq = __shfl((int)ok, q, 64);
          const int vq = __shfl((int)val, q, 64);
          dup |= (q < lane) && oq && (uint16_t)vq == val;
        }
        const bool keep = ok && !dup;
        const uint64_t mask = __ballot(keep);
        if (keep) {
          const int pos = __builtin_popcountll(mask & ((1ull << lane) - 1));
          cu[pos] = (int16_t)u;
          cv[pos] = (int16_t)v;
        }
        // IntraX (Section 3.1) of the current block
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
        if (lane == 0) {
          sh_np = __builtin_popcountll(mask);
          sh_px = px;
          sh_py = py;
          sh_intra = iacc;
          sh_abort = failed;
          if (failed) atomicOr(&a.hdr->status, kStatusSpinTimeout);
        }
      }
      __syncthreads();
      if (sh_abort) return;
      const int px = sh_px, py = sh_py;

      // ---- step 2: SADs of the predictors and the cheapest one ------------
      list_sads<N, M>(ring, w, cb0, cd, cu, cv, csad, 0, sh_np);
      __syncthreads();
      if (w0) {
        const int np = sh_np;
        uint64_t key = ~0ull;
        if (lane < np) {
          const uint32_t j = csad[lane] + a.lam * (se_bits(cu[lane] - px) + se_bits(cv[lane] - py));
          key = make_key(j, cu[lane], cv[lane], p);
        }
        key = wave_min_u64(key);
        // step 3: the valid 8-neighbours of that predictor not yet evaluated
        const int W = 2 * p + 1;
        const int ras = (int)(key & 0xFFFFu);
        const int bu = ras % W - p, bv = ras / W - p;
        bool add = false;
        int u = 0, v = 0;
        if (lane < 8) {
          const int dd = lane < 4 ? lane : lane + 1;  // skip the centre
          u = bu + dd % 3 - 1;
          v = bv + dd / 3 - 1;
          add = cand_valid(u, v, p, x0, y0, N, M, g.width, g.height);
          for (int q = 0; q < np; ++q) add &= !(cu[q] == u && cv[q] == v);
        }
        const uint64_t mask = __ballot(add);
        if (add) {
          const int pos = np + __builtin_popcountll(mask & ((1ull << lane) - 1));
          cu[pos] = (int16_t)u;
          cv[pos] = (int16_t)v;
        }
        if (lane == 0) sh_n = np + __builtin_popcountll(mask);
      }
      __syncthreads();
      list_sads<N, M>(ring, w, cb0, cd, cu, cv, csad, sh_np, sh_n);
      __syncthreads();
      if (w0) {
        const int n = sh_n;
        uint64_t key = ~0ull;
        uint32_t sad = 0;
        if (lane < n) {
          sad = csad[lane];
          const uint32_t j = sad + a.lam * (se_bits(cu[lane] - px) + se_bits(cv[lane] - py));
          key = make_key(j, cu[lane], cv[lane], p);
        }
        const uint64_t best = wave_min_u64(key);
        if (key == best && lane < n) {  // the unique winner's lane decides
          int mode = ACBM_MODE_PBM;
          if (a.algo == ACBM_ALGO_ACBM) {
            const uint64_t nm = (uint64_t)(N * M), ix = sh_intra;
            if (ix + nm * sad < a.c1_rhs) mode = ACBM_MODE_PBM_C1;
            else if ((uint64_t)a.gamma_den * nm * sad < (uint64_t)a.gamma_num * ix) mode = ACBM_MODE_PBM_C2;
            else mode = ACBM_MODE_CRITICAL;
          }
          sh_crit = mode == ACBM_MODE_CRITICAL;
          if (mode != ACBM_MODE_CRITICAL) {
            const int u = cu[lane], v = cv[lane];
            const uint32_t rate = se_bits(u - px) + se_bits(v - py);
            acbm_block_result res;
            res.mv.x = (int16_t)u;
            res.mv.y = (int16_t)v;
            res.sad = sad;
            res.j = sad + a.lam * rate;
            res.rate_bits = rate;
            res.cands = (uint32_t)n;
            res.mode = (uint32_t)mode;
            res.intra_x = sh_intra;
            a.out[(size_t)t * nb + b] = res;
            store_word(words + b, kReady | pack_mv(u, v));
            sh_left = pack_mv(u, v);
          }
        }
      }
      __syncthreads();

      // ---- critical block: full search with the same predictor -----------
      if (sh_crit) {
        const ValidBox vbox = valid_box(p, x0, y0, N, M, g.width, g.height);
        const uint64_t best =
            critical_search<N, M, R>(ring, w, cb0, cd, vbox, px, py, a.lam, a.slack, red, rmin);
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
          store_word(words + b, kReady | pack_mv(u, v));
          sh_left = pack_mv(u, v);
        }
      }

      // ---- park what block c+1 adds ---------------------------------------
      if (more) {
        park_columns<N, NT>(ring, nxt, w, ref, g, y0, cb0 + w.s.dws);
        if (threadIdx.x < D) curd[cb ^ 1][threadIdx.x] = nxt_cur;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int row_levels(const KGeom& g, int npairs) { return (g.by - 1) + 2 * (npairs - 1) + 1; }

size_t predictive_ws_bytes(const KGeom& g, uint32_t npairs) {
  const uint32_t per = std::min<uint32_t>(npairs, kMaxPairsPerLaunch);
  return align256(sizeof(WsHeader)) + align256((size_t)per * g.by * sizeof(uint32_t)) +
         align256((size_t)per * g.nb * sizeof(uint32_t));
}

template <int N, int M>
static RingShape ring_shape(int p, int R) {
  RingShape w;
  w.s = window_shape<N, M>(p, R);
  w.cw = 1;
  while (w.cw < w.s.dws + N / 4) w.cw <<= 1;
  w.stride = w.cw + 1;
  return w;
}

static RingShape ring_for(const KGeom& g, int R) {
  if (g.bw == 16 && g.bh == 16) return ring_shape<16, 16>(g.p, R);
  if (g.bw == 16 && g.bh == 8) return ring_shape<16, 8>(g.p, R);
  if (g.bw == 8 && g.bh == 16) return ring_shape<8, 16>(g.p, R);
  return ring_shape<8, 8>(g.p, R);
}

#define ACBM_PRED_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(11) X(16)

template <int N, int M, int NT>
static int launch_pred_nmt(const PredArgs& a, const FramePtrs& fr, int R, size_t lds, int grid,
                           hipStream_t st) {
  switch (R) {
#define ACBM_CASE(RR)                                                                   \
  case RR: {                                                                            \
    if (lds > 64 * 1024)                                                                \
      (void)hipFuncSetAttribute((const void*)k_predictive<N, M, RR, NT>,                \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);  \
    ProfScope ps("predictive", st);                                                     \
    hipLaunchKernelGGL((k_predictive<N, M, RR, NT>), dim3(grid), dim3(NT), lds, st, a, fr); \
    break;                                                                              \
  }
    ACBM_PRED_R_LIST(ACBM_CASE)
#undef ACBM_CASE
    default:
      return fail(ACBM_E_UNSUPPORTED, "no predictive kernel for this row blocking");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the predictive search");
}

template <int N, int M>
static int launch_pred_nm(const PredArgs& a, const FramePtrs& fr, int R, int nt, size_t lds,
                          int grid, hipStream_t st) {
  if (nt == 64) return launch_pred_nmt<N, M, 64>(a, fr, R, lds, grid, st);
  if (nt == 128) return launch_pred_nmt<N, M, 128>(a, fr, R, lds, grid, st);
  return launch_pred_nmt<N, M, 256>(a, fr, R, lds, grid, st);
}

// Threads per row walker (64, 128 or 256); ACBM_ROW_THREADS overrides.
static int row_threads() {
  static int nt = [] {
    const char* e = std::getenv("ACBM_ROW_THREADS");
    const int v = e ? std::atoi(e) : 128;
    return (v == 64 || v == 256) ? v : 128;
  }();
  return nt;
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
  // Row blocking of the one-wave critical search: R <= 6 keeps the kernel at
  // about 160 VGPRs (three waves per SIMD); among those, the fewest lane
  // slots (rounds * R) with at most kMaxRounds rounds and a ring that fits.
  const int nt = row_threads();
  int bestR = 0;
  long best_slots = 0;
  for (int R : {6, 5, 4, 3, 2, 1}) {
    const RingShape w = ring_for(g, R);
    const int rounds = (w.s.quads * w.s.groups + nt - 1) / nt;
    const size_t lds = (size_t)w.s.rows * w.stride * 4;
    if (rounds > kMaxRounds || lds > (size_t)lds_limit()) continue;
    const long slots = (long)rounds * R;
    if (!bestR || slots < best_slots) {
      bestR = R;
      best_slots = slots;
    }
  }
  if (!bestR) return fail(ACBM_E_UNSUPPORTED, "search window too large for the predictive kernel");
  const SearchPlan pl{bestR, nt, 0};
  const uint32_t per = std::min<uint32_t>(npairs, kMaxPairsPerLaunch);
  char* base = static_cast<char*>(ws);
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
    const uint64_t slack64 = (uint64_t)prm.lambda * (uint64_t)(rate_max(g.p) - 2);
    a.slack = slack64 > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)slack64;
    a.npairs = n;
    a.row_levels = row_levels(g, n);
    if (p0 == 0) {
      a.prev0 = reinterpret_cast<const uint8_t*>(prev_field);
      a.prev0_stride = sizeof(acbm_mv);
    } else {
      a.prev0 = reinterpret_cast<const uint8_t*>(out + (size_t)(p0 - 1) * g.nb);
      a.prev0_stride = sizeof(acbm_block_result);
    }
    a.hdr = reinterpret_cast<WsHeader*>(base);
    a.row_order = reinterpret_cast<uint32_t*>(base + align256(sizeof(WsHeader)));
    a.words = reinterpret_cast<uint32_t*>(base + align256(sizeof(WsHeader)) +
                                          align256((size_t)per * g.by * sizeof(uint32_t)));
    a.out = out + (size_t)p0 * g.nb;
    FramePtrs fr{};
    for (int k = 0; k <= n; ++k) fr.f[k] = frames[p0 + k];

    a.w = ring_for(g, pl.R);
    const size_t lds = (size_t)a.w.s.rows * a.w.stride * 4;
    if (lds > (size_t)lds_limit())
      return fail(ACBM_E_UNSUPPORTED, "search window too large for LDS");

    const int setup_grid = (int)std::min<size_t>(1024, ((size_t)n * g.nb + 255) / 256 + 1);
    {
      ProfScope ps("setup", st);
      hipLaunchKernelGGL(k_pred_setup, dim3(setup_grid), dim3(256), 0, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "launching the predictive setup");

    // about as many row walkers as can be resident, never more than rows
    const int per_cu =
        std::max<int>(1, std::min<int>(16 * 64 / nt, (int)(150 * 1024 / (lds + 2048 + 32 * nt))));
    const int grid = (int)std::min<size_t>((size_t)device_cus() * per_cu, (size_t)n * g.by);
    int rc;
    if (g.bw == 16 && g.bh == 16) rc = launch_pred_nm<16, 16>(a, fr, pl.R, nt, lds, grid, st);
    else if (g.bw == 16 && g.bh == 8) rc = launch_pred_nm<16, 8>(a, fr, pl.R, nt, lds, grid, st);
    else if (g.bw == 8 && g.bh == 16) rc = launch_pred_nm<8, 16>(a, fr, pl.R, nt, lds, grid, st);
    else rc = launch_pred_nm<8, 8>(a, fr, pl.R, nt, lds, grid, st);
    if (rc) return rc;
  }
  return ACBM_OK;
}

}  // namespace acbm
