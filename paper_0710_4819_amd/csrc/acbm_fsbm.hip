// acbm_fsbm.hip -- SAD table and full search (FSBM) kernels for gfx950.
//
// Full search (Section 2.3) costs (2p+1)^2 SADs (Section 2.1, SAD equation)
// per block; that is where the time goes.  It is split in two kernels:
//
//  k_search  one workgroup per block.  The block's search window is staged
//            in LDS, the current block sits in scalar registers, and every
//            lane computes four horizontally adjacent candidates x R rows
//            with V_QSAD_PK_U16_U8.  Output: either the whole table
//            (acbm_sad_table) or, for FSBM, the block's SAD minimum and the
//            few candidates that can still win once the rate term is added.
//            8x8 blocks on an even grid search in 2x2 tiles instead
//            (k_search_tile: one workgroup, four blocks, the 16x16 window).
//  k_resolve one workgroup per frame pair.  The predictor of a block depends
//            on the final vectors of its left, top and top-right neighbours,
//            so the argmin of J is sequential in raster order; the kernel
//            resolves every block as soon as those three are known, either
//            in sweeps (blocks with a single possible winner need no
//            predictor at all) or, when many blocks have several, in
//            anti-diagonal steps with one block per lane.
// With half-pel precision k_half_prep first computes the half-pel SADs
// around the possible winners of few-winner blocks, and the resolve adds the
// 8 half-pel positions around each integer winner.
//
// Pruning bound (exact): R >= 2 for every candidate and R <= Rmax =
// 2*se(2p) (2*se(4p) in half-pel units), so the winner has
// J <= SAD_min + lambda*Rmax while any candidate has J >= SAD + 2*lambda;
// only candidates with SAD <= SAD_min + lambda*(Rmax - 2) can win (ties
// included).
#include <hip/hip_runtime.h>

#include "acbm_device.h"
#include "acbm_internal.h"

namespace acbm {

// Overflow rows hold (2p+1)^2 u16 SADs padded to a multiple of 8 entries,
// so that every row starts 16-byte aligned and can be read in uint4 pieces.
__host__ __device__ __forceinline__ size_t ovf_stride(int p) {
  const size_t ww = (size_t)(2 * p + 1) * (2 * p + 1);
  return (ww + 7) & ~(size_t)7;
}
// The same region holds, when a block has more than kShort but at most this
// many possible winners, their full list as u32 (SAD << 16 | raster index).
__host__ __device__ __forceinline__ uint32_t ovf_list_cap(int p) {
  return (uint32_t)(ovf_stride(p) / 2);
}

// With half-pel precision, blocks with at most this many possible winners
// get the 8 half-pel SADs around each winner prepared in their overflow
// region (8 entries per winner), which they do not otherwise use.
__host__ __device__ __forceinline__ uint32_t half_cap(int p) {
  const uint32_t c = (uint32_t)(ovf_stride(p) / 8);
  return c < (uint32_t)kShort ? c : (uint32_t)kShort;
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap so that each
// XCD gets one contiguous band of blocks: neighbouring blocks share most of
// their search windows, and a band then stays in one XCD's L2.
__device__ __forceinline__ int xcd_band(int wg, int n) {
  const int per = (n + 7) >> 3;
  return (wg & 7) * per + (wg >> 3);
}

// IntraX (Section 3.1, Intra_SAD scaled by N*M) of the block at (x0, y0),
// computed by one wave.  Every lane of the wave gets the value.
template <int N, int M>
__device__ __forceinline__ uint32_t wave_intra_x(const uint8_t* __restrict__ cur, int pitch,
                                                 int x0, int y0) {
  constexpr int D = M * N / 4;  // dwords in the block (<= 64)
  const int lane = threadIdx.x & 63;
  uint32_t d = 0;
  if (lane < D) {
    const int j = lane / (N / 4), k = lane % (N / 4);
    d = ld_global<uint32_t>(cur + (size_t)(y0 + j) * pitch + x0 + 4 * k);
  }
  const uint32_t s = wave_sum_u32(__builtin_amdgcn_sad_u8(d, 0u, 0u));
  uint32_t a = 0;
  if (lane < D) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int q = (int)(N * M) * (int)((d >> (8 * b)) & 0xFF) - (int)s;
      a += (uint32_t)(q < 0 ? -q : q);
    }
  }
  return wave_sum_u32(a);
}

// ---------------------------------------------------------------------------
// Window search of one block (all threads of the group).  What it writes
// depends on the kind K:
//  kKindTable  the block's u32 table `tab`;
//  kKindFsbm   its BlockRec `rec` (SAD minimum, the number of candidates that
//              can still win and, when at most kShort can, those candidates)
//              and, when more can win, its overflow region `row`: the list
//              of all of them while it fits (ovf_list_cap entries), else the
//              whole row of SADs;
//  kKindStats  its statistics `bst`: SAD minimum, valid count,
//              SAD_deviation and IntraX (Section 3.1).
// `win` is the window in LDS, `red` one slot per wave, `n_keep` a shared
// counter.
// ---------------------------------------------------------------------------
// The candidates of a task that can still win (SAD <= thr), as bits 4*rr + i.
template <int R>
__device__ __forceinline__ uint64_t keep_mask(const uint64_t (&acc)[R], uint32_t thr) {
  static_assert(4 * R <= 64, "a task's candidates fit the mask");
  uint64_t m = 0;
#pragma unroll
  for (int rr = 0; rr < R; ++rr)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      m |= (uint64_t)(((uint32_t)(acc[rr] >> (16 * i)) & 0xFFFFu) <= thr) << (4 * rr + i);
  return m;
}

// Stores the kept candidates of a task at dst[slot], dst[slot + 1], ... as
// (SAD << 16 | window raster index): one loop turn per kept candidate, the
// candidate's accumulator picked by a select chain (no dynamic register index).
// The stores are typed global: through a generic pointer (the batch kernels
// take theirs from the job table) they would be FLAT stores, which also hold
// up the next LDS wait.
template <int R>
__device__ __forceinline__ void write_kept(const uint64_t (&acc)[R], uint64_t keep, uint32_t slot,
                                           uint32_t* __restrict__ dst, int u0, int v0, int p,
                                           int W) {
  while (keep) {
    const int j = __builtin_ctzll(keep);
    keep &= keep - 1;
    const int rr = j >> 2, i = j & 3;
    uint64_t a = acc[0];
#pragma unroll
    for (int r = 1; r < R; ++r) a = rr == r ? acc[r] : a;
    const uint32_t sad = (uint32_t)(a >> (16 * i)) & 0xFFFFu;
    st_global<uint32_t>(dst + slot++, (sad << 16) | (uint32_t)((v0 + rr + p) * W + (u0 + i + p)));
  }
}

enum : int { kKindFsbm = 0, kKindTable = 1, kKindStats = 2 };

template <int N, int M, int R, int K>
__device__ __forceinline__ void search_block(const KGeom& g, const WindowShape& s,
                                             const uint8_t* __restrict__ ref,
                                             const uint8_t* __restrict__ cur, int b,
                                             uint32_t* __restrict__ tab, BlockRec* __restrict__ rec,
                                             uint16_t* __restrict__ row, uint32_t slack,
                                             uint32_t* win, uint64_t* red, uint32_t* n_keep,
                                             acbm_block_stats* __restrict__ bst = nullptr) {
  constexpr bool kTable = K == kKindTable;
  const int r = b / g.bx, c = b - r * g.bx;
  const int x0 = c * N, y0 = r * M;
  const int p = s.p, W = 2 * p + 1;

  load_window<N, M>(win, s, ref, g.pitch, g.width, g.height, x0, y0);
  CurBlock<N, M> cb;
  load_cur_uniform<N, M>(cb, cur, g.pitch, x0, y0);
  uint32_t intra = 0;
  if (!kTable && threadIdx.x < 64) intra = wave_intra_x<N, M>(cur, g.pitch, x0, y0);
  if (threadIdx.x == 0) *n_keep = 0;
  __syncthreads();

  const int tasks = s.quads * s.groups;
  const int t = threadIdx.x;
  const bool active = t < tasks;
  int q = 0, gi = 0;
  bool edge = false;
  if (active) task_of<R>(s, t, &q, &gi, &edge);
  uint64_t acc[R];
  if (active) task_sads<N, M, R>(win, s.stride, q, gi, cb, acc);

  const int u0 = s.u_lo + 4 * q, v0 = -p + R * gi;
  // invalid candidates (outside the frame, or the padding of the quads and
  // row groups beyond +-p) read as 0xFFFF from here on; a block whose whole
  // window is valid has them in its edge tasks only
  const ValidBox vbox = valid_box(p, x0, y0, N, M, g.width, g.height);
  const bool whole = vbox.u_min == -p && vbox.u_max == p && vbox.v_min == -p && vbox.v_max == p;
  if (active) {
    if (!whole)
      mask_invalid<R>(acc, vbox, u0, v0);
    else if (edge)
      mask_padding<R>(acc, p, u0, v0);
  }

  if (K == kKindStats) {
    // SAD_deviation = sum over the valid window of SAD - SAD_min.  Per lane
    // at most 4*R*65280 < 2^32; per wave at most 64 times that < 2^32 for
    // R <= 16, so u32 sums are exact and the group total is summed in u64.
    const uint32_t lmin = active ? min_u16_lanes<R>(acc) : 0xFFFFu;
    const uint32_t smin = group_min_u32(lmin, reinterpret_cast<uint32_t*>(red));
    uint32_t dev = 0, nvalid = 0;
    if (active) {
#pragma unroll
      for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t sad = (uint32_t)(acc[rr] >> (16 * i)) & 0xFFFFu;
          if (sad != 0xFFFFu) {
            dev += sad - smin;
            ++nvalid;
          }
        }
    }
    dev = wave_sum_u32(dev);
    nvalid = wave_sum_u32(nvalid);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = ((uint64_t)nvalid << 40) | dev;  // both fields stay below 2^40 and 2^24
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t d = 0, n = 0;
      for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) {
        d += red[w] & ((1ull << 40) - 1);
        n += red[w] >> 40;
      }
      bst->sad_min = smin;
      bst->valid = (uint32_t)n;
      bst->sad_deviation = d;
      bst->intra_x = intra;
      bst->reserved = 0;
    }
    return;
  }

  if (kTable) {
    if (!active) return;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int v = v0 + rr;
      if (v > p) break;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = u0 + i;
        if (u < -p || u > p) continue;
        const uint32_t sad = (uint32_t)(acc[rr] >> (16 * i)) & 0xFFFFu;
        tab[(v + p) * W + (u + p)] = sad == 0xFFFFu ? 0xFFFFFFFFu : sad;
      }
    }
    return;
  }

  // ---- FSBM: SAD minimum and the candidates that can still win ----------
  const uint32_t lmin = active ? min_u16_lanes<R>(acc) : 0xFFFFu;
  const uint32_t smin = group_min_u32(lmin, reinterpret_cast<uint32_t*>(red));
  const uint32_t thr = (uint32_t)min<uint64_t>((uint64_t)smin + slack, 0xFFFEu);

  // Count this lane's possible winners and reserve their slots; once the
  // block's total is known, write each entry once, where the resolve will
  // read it: the record (at most kShort), the overflow list (at most cap),
  // or, beyond that, the whole row of SADs.
  const bool any = active && lmin <= thr;
  uint64_t keep = 0;  // bit 4*rr + i: candidate (u0 + i, v0 + rr) can still win
  uint32_t slot = 0;
  if (any) {
    keep = keep_mask<R>(acc, thr);
    slot = atomicAdd(n_keep, (uint32_t)__popcll(keep));
  }
  __syncthreads();
  const uint32_t total = *n_keep;
  // (at small p the list holds fewer than kShort: the record takes up to kShort)
  if (total <= (uint32_t)kShort || total <= ovf_list_cap(p)) {
    if (keep)
      write_kept<R>(acc, keep, slot,
                    total <= (uint32_t)kShort ? rec->e : reinterpret_cast<uint32_t*>(row), u0,
                    v0, p, W);
  } else if (active) {
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int v = v0 + rr;
      if (v > p) break;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = u0 + i;
        if (u < -p || u > p) continue;
        st_global<uint16_t>(row + (v + p) * W + (u + p), (uint16_t)(acc[rr] >> (16 * i)));
      }
    }
  }
  if (threadIdx.x == 0) {
    st_global<uint32_t>(&rec->sad_min, smin);
    st_global<uint32_t>(&rec->count, total);
    st_global<uint32_t>(&rec->intra_x, intra);
  }
}

// One workgroup per (block, pair).
template <int N, int M, int R, bool kTable>
__global__ void __launch_bounds__(1024)
k_search(const KGeom g, const WindowShape s, const FramePtrs fr, uint32_t* __restrict__ table,
         BlockRec* __restrict__ recs, uint16_t* __restrict__ ovf, uint32_t slack) {
  extern __shared__ uint32_t win[];
  __shared__ uint64_t red[16];
  __shared__ uint32_t n_keep;
  const int b = xcd_band(blockIdx.x, g.nb);
  if (b >= g.nb) return;
  const int pair = blockIdx.y;
  const size_t WW = (size_t)(2 * s.p + 1) * (2 * s.p + 1);
  const size_t at = (size_t)pair * g.nb + b;
  search_block<N, M, R, kTable ? kKindTable : kKindFsbm>(g, s, fr.f[pair], fr.f[pair + 1], b,
                                kTable ? table + (size_t)b * WW : nullptr,
                                kTable ? nullptr : recs + at,
                                kTable ? nullptr : ovf + at * ovf_stride(s.p),
                                slack, win, red, &n_keep);
}

// Block statistics of one frame pair (Section 3.1): one workgroup per block,
// the same window search as k_search.
template <int N, int M, int R>
__global__ void __launch_bounds__(1024)
k_stats(const KGeom g, const WindowShape s, const uint8_t* __restrict__ ref,
        const uint8_t* __restrict__ cur, acbm_block_stats* __restrict__ out) {
  extern __shared__ uint32_t win[];
  __shared__ uint64_t red[16];
  __shared__ uint32_t n_keep;
  const int b = xcd_band(blockIdx.x, g.nb);
  if (b >= g.nb) return;
  search_block<N, M, R, kKindStats>(g, s, ref, cur, b, nullptr, nullptr, nullptr, 0, win, red,
                                    &n_keep, out + b);
}

// Full search over the jobs of one batch group: one workgroup per
// (job, pair, block) item, items numbered job by job (pair-major within a
// job) and handed out in one contiguous band per XCD like k_search.  The
// job of an item is found with one load per lane (lane k reads job k's
// first item) and a ballot, so a group of up to 64 jobs costs one memory
// round trip.
template <int N, int M, int R>
__global__ void __launch_bounds__(1024)
k_search_batch(const BatchJob* __restrict__ jobs, int njobs, uint32_t items) {
  extern __shared__ uint32_t win[];
  __shared__ uint64_t red[16];
  __shared__ uint32_t n_keep;
  const uint32_t it = (uint32_t)xcd_band(blockIdx.x, (int)items);
  if (it >= items) return;
  const int lane = threadIdx.x & 63;
  const uint32_t first = lane < njobs ? jobs[lane].item0 : 0xFFFFFFFFu;
  const int j = __builtin_amdgcn_readfirstlane(__popcll(__ballot(first <= it)) - 1);
  const BatchJob& J = jobs[j];
  const KGeom g = J.g;
  const uint32_t local = it - J.item0;
  const int pair = (int)(local / (uint32_t)g.nb), b = (int)(local % (uint32_t)g.nb);
  const size_t at = (size_t)pair * g.nb + b;
  // The window shape by value: read through a reference, it would be
  // reloaded after every LDS store that might alias it.  The frames are read
  // with global loads (load_window, load_cur_uniform), so the current block
  // lands in scalar registers as in k_search.
  const WindowShape s = J.s;
  const uint8_t* ref = ld_global<const uint8_t*>(J.frames + pair);
  const uint8_t* cur = ld_global<const uint8_t*>(J.frames + pair + 1);
  search_block<N, M, R, kKindFsbm>(g, s, ref, cur, b, nullptr,
                               J.recs + at, J.ovf + at * ovf_stride(g.p), J.slack, win, red,
                               &n_keep);
}

// ---------------------------------------------------------------------------
// Window search of a 2x2 tile of 8x8 blocks by one workgroup (FSBM records
// only).  The tile's 16x16 window holds every candidate of its four blocks;
// one pass of 16x16 tasks gives each block its SADs (task_sads_tile), and the
// epilogue of search_block runs once per block: border masks from the
// block's own position, SAD minimum, possible winners, record and overflow
// region.  Against four workgroups of one block each, the tile loads one
// 80x80 window instead of four 72x72 ones (p = 32), reads fewer LDS dwords
// per QSAD and pays the per-workgroup costs once.  `t` is the tile index in
// the frame's grid of (bx/2) x (by/2) tiles; `recs` and `ovf` are the pair's;
// `intra` is 4 words of LDS.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ void search_tile(const KGeom& g, const WindowShape& s,
                                            const uint8_t* __restrict__ ref,
                                            const uint8_t* __restrict__ cur, int t,
                                            BlockRec* __restrict__ recs,
                                            uint16_t* __restrict__ ovf, uint32_t slack,
                                            uint32_t* win, uint32_t* red, uint32_t* n_keep,
                                            uint32_t* intra) {
  const int tbx = g.bx >> 1;
  const int tr = t / tbx, tc = t - tr * tbx;
  const int x0 = tc * 16, y0 = tr * 16;
  const int p = s.p, W = 2 * p + 1;

  load_window<16, 16>(win, s, ref, g.pitch, g.width, g.height, x0, y0);
  CurBlock<16, 16> cb;
  load_cur_uniform<16, 16>(cb, cur, g.pitch, x0, y0);
  // IntraX of the four blocks in one pass of wave 0: lanes 16b .. 16b+15 hold
  // block b's 16 dwords (row k/2, dword k%2 for lane 16b + k), and both sums
  // are sums over those 16 lanes
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x, b = lane >> 4, k = lane & 15;
    const uint32_t d = ld_global<uint32_t>(
        cur + (size_t)(y0 + 8 * (b >> 1) + (k >> 1)) * g.pitch + x0 + 8 * (b & 1) + 4 * (k & 1));
    const uint32_t sum = group_sum<16>(__builtin_amdgcn_sad_u8(d, 0u, 0u));
    uint32_t a = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = 64 * (int)((d >> (8 * q)) & 0xFF) - (int)sum;
      a += (uint32_t)(e < 0 ? -e : e);
    }
    a = group_sum<16>(a);
    if (k == 0) intra[b] = a;
  }
  if (threadIdx.x < 4) n_keep[threadIdx.x] = 0;
  __syncthreads();

  const int tasks = s.quads * s.groups;
  const int th = threadIdx.x;
  const bool active = th < tasks;
  int q = 0, gi = 0;
  bool edge = false;
  if (active) task_of<R>(s, th, &q, &gi, &edge);
  uint64_t acc[4][R];
  if (active) task_sads_tile<R>(win, s.stride, q, gi, cb, acc);

  const int u0 = s.u_lo + 4 * q, v0 = -p + R * gi;
  uint32_t lmin[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const ValidBox vbox =
        valid_box(p, x0 + 8 * (b & 1), y0 + 8 * (b >> 1), 8, 8, g.width, g.height);
    const bool whole = vbox.u_min == -p && vbox.u_max == p && vbox.v_min == -p && vbox.v_max == p;
    if (active) {
      if (!whole)
        mask_invalid<R>(acc[b], vbox, u0, v0);
      else if (edge)
        mask_padding<R>(acc[b], p, u0, v0);
    }
    lmin[b] = active ? min_u16_lanes<R>(acc[b]) : 0xFFFFu;
  }
  // the four blocks' minima over the workgroup: one slot per (wave, block)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t m = wave_min_u32(lmin[b]);
    if (lane == 0) red[4 * wave + b] = m;
  }
  __syncthreads();
  uint32_t smin[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    uint32_t m = red[b];
    for (int w = 1; w < nw; ++w) m = min(m, red[4 * w + b]);
    smin[b] = m;
  }

  // per block as in search_block: count and reserve, then write each entry
  // once where the resolve reads it
  const uint32_t cap = ovf_list_cap(p);
  uint64_t keep[4];
  uint32_t slot[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t thr = (uint32_t)min<uint64_t>((uint64_t)smin[b] + slack, 0xFFFEu);
    keep[b] = 0;
    slot[b] = 0;
    if (active && lmin[b] <= thr) {
      keep[b] = keep_mask<R>(acc[b], thr);
      slot[b] = atomicAdd(&n_keep[b], (uint32_t)__popcll(keep[b]));
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t total = n_keep[b];
    const int blk = (2 * tr + (b >> 1)) * g.bx + 2 * tc + (b & 1);
    uint16_t* __restrict__ row = ovf + (size_t)blk * ovf_stride(p);
    if (total <= (uint32_t)kShort || total <= cap) {
      if (keep[b])
        write_kept<R>(acc[b], keep[b], slot[b],
                      total <= (uint32_t)kShort ? recs[blk].e : reinterpret_cast<uint32_t*>(row),
                      u0, v0, p, W);
    } else if (active) {
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int v = v0 + rr;
        if (v > p) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int u = u0 + i;
          if (u < -p || u > p) continue;
          st_global<uint16_t>(row + (v + p) * W + (u + p), (uint16_t)(acc[b][rr] >> (16 * i)));
        }
      }
    }
    if (threadIdx.x == 0) {
      BlockRec* __restrict__ rec = recs + blk;
      st_global<uint32_t>(&rec->sad_min, smin[b]);
      st_global<uint32_t>(&rec->count, total);
      st_global<uint32_t>(&rec->intra_x, intra[b]);
    }
  }
}

// One workgroup per (2x2 tile, pair).  A budget of six waves per SIMD: at
// R = 6 the four accumulator sets would take 90 VGPRs (five waves); with 80
// and a few epilogue values spilled the 8x8 p = 32 search is about 2 %
// faster.
template <int R>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6)))
k_search_tile(const KGeom g, const WindowShape s, const FramePtrs fr, BlockRec* __restrict__ recs,
              uint16_t* __restrict__ ovf, uint32_t slack) {
  extern __shared__ uint32_t win[];
  __shared__ uint32_t red[64];
  __shared__ uint32_t n_keep[4];
  __shared__ uint32_t intra[4];
  const int nt = g.nb >> 2;
  const int t = xcd_band(blockIdx.x, nt);
  if (t >= nt) return;
  const int pair = blockIdx.y;
  search_tile<R>(g, s, fr.f[pair], fr.f[pair + 1], t, recs + (size_t)pair * g.nb,
                 ovf + (size_t)pair * g.nb * ovf_stride(s.p), slack, win, red, n_keep, intra);
}

// The batch form: items are (job, pair, tile), numbered like k_search_batch
// (the same register budget).
template <int R>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6)))
k_search_batch_tile(const BatchJob* __restrict__ jobs, int njobs, uint32_t items) {
  extern __shared__ uint32_t win[];
  __shared__ uint32_t red[64];
  __shared__ uint32_t n_keep[4];
  __shared__ uint32_t intra[4];
  const uint32_t it = (uint32_t)xcd_band(blockIdx.x, (int)items);
  if (it >= items) return;
  const int lane = threadIdx.x & 63;
  const uint32_t first = lane < njobs ? jobs[lane].item0 : 0xFFFFFFFFu;
  const int j = __builtin_amdgcn_readfirstlane(__popcll(__ballot(first <= it)) - 1);
  const BatchJob& J = jobs[j];
  const KGeom g = J.g;
  const uint32_t nt = (uint32_t)g.nb >> 2;
  const uint32_t local = it - J.item0;
  const int pair = (int)(local / nt), t = (int)(local % nt);
  const WindowShape s = J.s;  // by value, as in k_search_batch
  const uint8_t* ref = ld_global<const uint8_t*>(J.frames + pair);
  const uint8_t* cur = ld_global<const uint8_t*>(J.frames + pair + 1);
  search_tile<R>(g, s, ref, cur, t, J.recs + (size_t)pair * g.nb,
                 J.ovf + (size_t)pair * g.nb * ovf_stride(g.p), J.slack, win, red, n_keep, intra);
}

// ---------------------------------------------------------------------------
// FSBM resolve: argmin of J = SAD + lambda*R per block, in dependency order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void window_uv(uint32_t ras, int p, int* u, int* v) {
  const int W = 2 * p + 1;
  *v = (int)(ras / (uint32_t)W) - p;
  *u = (int)(ras % (uint32_t)W) - p;
}

// Per-block state of the resolve: the decided vector packed in the low 16
// bits (kMvUnset while open) and its SAD in the high 16 bits.
__device__ __forceinline__ bool is_open(uint32_t w) { return (w & 0xFFFFu) == kMvUnset; }

// Predictor of block b from the decided vectors; false if one of the three
// neighbours it needs is still open.
__device__ __forceinline__ bool median_pred(const uint32_t* st, int b, int r, int c, int bx,
                                            int* px, int* py) {
  uint32_t A = pack_mv(0, 0), B, C;
  if (c > 0) {
    A = st[b - 1];
    if (is_open(A)) return false;
  }
  if (r == 0) {
    B = A;
    C = A;
  } else {
    B = st[b - bx];
    C = (c == bx - 1) ? (uint32_t)pack_mv(0, 0) : st[b - bx + 1];
    if (is_open(B) || is_open(C)) return false;
  }
  *px = med3(mv_x((uint16_t)A), mv_x((uint16_t)B), mv_x((uint16_t)C));
  *py = med3(mv_y((uint16_t)A), mv_y((uint16_t)B), mv_y((uint16_t)C));
  return true;
}

// Key of integer candidate (u, v) with SAD `sad`.  With half-pel precision
// (HP) the candidate is the half-pel vector (2u, 2v): its rate is taken
// against the half-pel predictor and it ranks by its half-pel |U|+|V| and
// its position in the (4p+1)^2 half-pel window, which orders the integer
// candidates exactly as the integer window does.
template <bool HP>
__device__ __forceinline__ uint64_t int_key(uint32_t sad, int u, int v, int p, int px, int py,
                                            uint32_t lam) {
  constexpr int s = HP ? 2 : 1;
  return make_key(sad + lam * (se_bits(s * u - px) + se_bits(s * v - py)), s * u, s * v, s * p);
}

// Cheapest candidate of one block, computed by a whole wave: the 128-byte
// record is read with one dword per lane, each listed candidate is priced by
// its own lane; an overflowed block's row is strided over the lanes.
template <bool HP>
__device__ __forceinline__ uint64_t wave_block_argmin(const BlockRec* __restrict__ rec,
                                                      const uint16_t* __restrict__ row, int p,
                                                      int px, int py, uint32_t lam) {
  const int lane = threadIdx.x & 63;
  const uint32_t w =
      lane < 32 ? ld_global<uint32_t>(reinterpret_cast<const uint32_t*>(rec) + lane) : 0u;
  const uint32_t n = (uint32_t)__shfl((int)w, 1, 64);  // rec->count
  uint64_t best = ~0ull;
  if (n > (uint32_t)kShort && n <= ovf_list_cap(p)) {
    // the full list of possible winners; v = ras / W by an exact
    // multiply-high with ceil(2^32 / W) (ras < 2^16, W < 2^8)
    const uint32_t W = 2u * (uint32_t)p + 1u;
    const uint32_t inv = (uint32_t)(((1ull << 32) + W - 1) / W);
    // up to kList entries per lane are loaded before any is used, so a long
    // list costs about one memory latency per 64 * kList entries
    const uint32_t* __restrict__ list = reinterpret_cast<const uint32_t*>(row);
    constexpr int kList = 8;
    for (uint32_t k0 = (uint32_t)lane; k0 < n; k0 += 64 * kList) {
      uint32_t e[kList];
#pragma unroll
      for (int t = 0; t < kList; ++t) {
        const uint32_t k = k0 + 64u * t;
        e[t] = k < n ? ld_global<uint32_t>(list + k) : 0u;
      }
#pragma unroll
      for (int t = 0; t < kList; ++t) {
        if (k0 + 64u * t < n) {
          const uint32_t ras = e[t] & 0xFFFFu;
          const uint32_t vq = __umulhi(ras, inv);
          const int v = (int)vq - p, u = (int)(ras - vq * W) - p;
          const uint64_t key = int_key<HP>(e[t] >> 16, u, v, p, px, py, lam);
          best = key < best ? key : best;
        }
      }
    }
  } else if (n <= (uint32_t)kShort) {
    const int k = lane - 4;  // e[k] is dword 4 + k of the record
    if (k >= 0 && k < (int)n) {
      int u, v;
      window_uv(w & 0xFFFFu, p, &u, &v);
      best = int_key<HP>(w >> 16, u, v, p, px, py, lam);
    }
  } else {
    // The whole row, read as uint4 pieces of 8 SADs: lane k takes pieces
    // k, k+64, ...; up to kPieces of them are loaded before any is used, so
    // the row costs about one memory latency.
    const int W = 2 * p + 1, WW = W * W;
    const int npieces = (WW + 7) / 8;
    const uint4* __restrict__ row4 = reinterpret_cast<const uint4*>(row);
    constexpr int kPieces = 9;  // 9 * 64 * 8 = 4608 >= (2*32+1)^2
    for (int c0 = lane; c0 < npieces; c0 += 64 * kPieces) {
      uint4 q[kPieces];
#pragma unroll
      for (int k = 0; k < kPieces; ++k) {
        const int c = c0 + 64 * k;
        q[k] = make_uint4(~0u, ~0u, ~0u, ~0u);
        if (c < npieces) {
          const u32x4 t = ld_global_x4(row4 + c);
          q[k] = make_uint4(t.x, t.y, t.z, t.w);
        }
      }
#pragma unroll
      for (int k = 0; k < kPieces; ++k) {
        // a guard, not a break: the loop stays unrolled and q[] in registers
        const int c = c0 + 64 * k;
        if (c < npieces) {
          const int pos = 8 * c;
          int u = pos % W - p, v = pos / W - p;
          const uint32_t w4[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const uint32_t sad = (w4[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
            if (sad != 0xFFFFu && pos + e < WW) {
              const uint64_t key = int_key<HP>(sad, u, v, p, px, py, lam);
              best = key < best ? key : best;
            }
            if (++u > p) {
              u = -p;
              ++v;
            }
          }
        }
      }
    }
  }
  return wave_min_u64(best);
}

// The nine-way choice of the half-pel step: the integer winner (U0, V0) with
// key `key`, and its 8 half-pel neighbours with SADs `sads` (0xFFFF: not a
// valid candidate), all priced with the predictor (px, py).  `writer`
// stores the block's result and its decision word.
__device__ __forceinline__ void half_finish(const KGeom& g, int b, int U0, int V0, uint64_t key,
                                            const uint32_t (&sads)[8], int px, int py,
                                            uint32_t lam, uint32_t intra_x, bool writer,
                                            acbm_block_result* __restrict__ out, uint32_t* st) {
  const int p = g.p;
  uint64_t best = key;
  uint32_t nh = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (sads[k] == 0xFFFFu) continue;
    int du, dv;
    half_ring_offset(k, &du, &dv);
    const int U = U0 + du, V = V0 + dv;
    const uint64_t kk = make_key(sads[k] + lam * (se_bits(U - px) + se_bits(V - py)), U, V, 2 * p);
    best = kk < best ? kk : best;
    ++nh;
  }
  int U = 0, V = 0;
  window_uv((uint32_t)(best & 0xFFFFu), 2 * p, &U, &V);
  const uint32_t rate = se_bits(U - px) + se_bits(V - py);
  const uint32_t j = (uint32_t)(best >> 32), sad = j - lam * rate;
  if (writer) {
    const int r = b / g.bx, c = b - r * g.bx;
    put_result(out, U, V, sad, j, rate,
               valid_count(p, c * g.bw, r * g.bh, g.bw, g.bh, g.width, g.height) + nh,
               ACBM_MODE_FSBM, intra_x);
    *st = (sad << 16) | pack_mv(U, V);
  }
}

// Half-pel step of block b (whole wave): `key` is the integer winner under
// the half-pel predictor (px, py); the 8 half-pel positions around it are
// priced with the same predictor and the cheapest of the nine is the block's
// result, written straight to `out` (the rate needs the predictor, which is
// known here).  Used for blocks with several possible winners; the 8 SADs
// are computed here from the frames.
__device__ __forceinline__ void half_decide(const KGeom& g, const BlockRec* __restrict__ rec,
                                            const uint8_t* __restrict__ cur,
                                            const uint8_t* __restrict__ ref, int b, int px,
                                            int py, uint32_t lam, uint64_t key,
                                            acbm_block_result* __restrict__ out, uint32_t* st) {
  const int p = g.p, lane = threadIdx.x & 63;
  int U0 = 0, V0 = 0;
  window_uv((uint32_t)(key & 0xFFFFu), 2 * p, &U0, &V0);
  const int r = b / g.bx, c = b - r * g.bx, x0 = c * g.bw, y0 = r * g.bh;
  uint32_t sads[8];
  if (g.bw == 16 && g.bh == 16) {
    wave_half_sads<16, 16>(g, cur, ref, x0, y0, U0, V0, sads);
  } else if (g.bw == 16) {
    wave_half_sads<16, 8>(g, cur, ref, x0, y0, U0, V0, sads);
  } else if (g.bh == 16) {
    wave_half_sads<8, 16>(g, cur, ref, x0, y0, U0, V0, sads);
  } else {
    wave_half_sads<8, 8>(g, cur, ref, x0, y0, U0, V0, sads);
  }
  half_finish(g, b, U0, V0, key, sads, px, py, lam, rec->intra_x, lane == 0, out, st);
}

// Same, for a block whose winners' half-pel SADs were prepared in its
// overflow region: lane s prices winner s and holds its 8 SADs.
__device__ __forceinline__ void half_decide_prepared(const KGeom& g,
                                                     const BlockRec* __restrict__ rec,
                                                     const uint16_t* __restrict__ row,
                                                     uint32_t count, int b, int px, int py,
                                                     uint32_t lam,
                                                     acbm_block_result* __restrict__ out,
                                                     uint32_t* st) {
  const int p = g.p, lane = threadIdx.x & 63;
  uint64_t key = ~0ull;
  uint4 hs = make_uint4(0u, 0u, 0u, 0u);
  if (lane < (int)count) {
    const uint32_t e = rec->e[lane];
    hs = reinterpret_cast<const uint4*>(row)[lane];
    int u = 0, v = 0;
    window_uv(e & 0xFFFFu, p, &u, &v);
    key = int_key<true>(e >> 16, u, v, p, px, py, lam);
  }
  const uint64_t k0 = wave_min_u64(key);
  const int w = __builtin_ctzll(__ballot(key == k0));  // keys are unique
  const uint32_t h4[4] = {(uint32_t)__builtin_amdgcn_readlane(hs.x, w),
                          (uint32_t)__builtin_amdgcn_readlane(hs.y, w),
                          (uint32_t)__builtin_amdgcn_readlane(hs.z, w),
                          (uint32_t)__builtin_amdgcn_readlane(hs.w, w)};
  uint32_t sads[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) sads[k] = (h4[k / 2] >> (16 * (k & 1))) & 0xFFFFu;
  int U0 = 0, V0 = 0;
  window_uv((uint32_t)(k0 & 0xFFFFu), 2 * p, &U0, &V0);
  half_finish(g, b, U0, V0, k0, sads, px, py, lam, rec->intra_x, lane == 0, out, st);
}

// What the half-pel resolve needs of one block's record, loaded a step
// ahead: the possible-winner count, the first entry and the 8 prepared
// half-pel SADs (e[1..4]), and IntraX.
struct HalfRec {
  uint32_t count;
  uint32_t e[5];
  uint32_t intra_x;
};

// The same decision for a block with a single possible winner, by one lane
// (its 8 half-pel SADs were prepared by k_half_prep).
__device__ __forceinline__ void half_decide_lane(const KGeom& g, const HalfRec& h, int b, int px,
                                                 int py, uint32_t lam,
                                                 acbm_block_result* __restrict__ out,
                                                 uint32_t* st) {
  const int p = g.p;
  int u = 0, v = 0;
  window_uv(h.e[0] & 0xFFFFu, p, &u, &v);
  const uint64_t key = int_key<true>(h.e[0] >> 16, u, v, p, px, py, lam);
  uint32_t sads[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) sads[k] = (h.e[1 + k / 2] >> (16 * (k & 1))) & 0xFFFFu;
  half_finish(g, b, 2 * u, 2 * v, key, sads, px, py, lam, h.intra_x, true, out, st);
}

// Half-pel resolve of one frame pair by the whole group.  Every block needs
// its predictor (the half-pel step is priced with it), so the blocks are
// decided in anti-diagonal order: step k holds the blocks (r, k - 2r), whose
// left, top and top-right neighbours all belong to earlier steps.  Thread i
// takes block i of every step (a step has at most `by` <= 1024 blocks, the
// group size), so a step's blocks fill the first waves and the rest skip the
// lane work.  A block with few possible winners is decided by its own lane;
// the others go to a list in LDS and, after a barrier, are decided by whole
// waves, one block per wave at a time.  Records do not depend on any
// decision, so each thread loads its block of the next step while the
// current step runs.
__device__ __forceinline__ int step_block(const KGeom& g, int k, int i) {
  const int r_lo = max(0, (k - (g.bx - 1) + 1) / 2), r_hi = min(g.by - 1, k / 2);
  const int r = r_lo + i;
  return r <= r_hi ? r * g.bx + (k - 2 * r) : -1;
}

// The blocks of the current step left to whole waves: block index and
// number of possible winners, and the list length of two consecutive steps
// (step k appends to cnt[k & 1] and clears cnt[(k + 1) & 1] for the next).
struct MultiList {
  uint32_t b[1024];
  uint32_t n[1024];
  int cnt[2];
};
__device__ __forceinline__ MultiList& multi_list() {
  __shared__ MultiList m;
  return m;
}

// Brings the record of this thread's block two steps ahead into the caches:
// the full prefetch of the next step then hits.  (The step loop waits for its
// prefetch at the end of each step, so that prefetch alone covers one step.)
// The word is only used one step later, after that wait, so the load adds
// no wait of its own.
__device__ __forceinline__ uint32_t touch_rec(const BlockRec* __restrict__ recs, int b) {
  return b >= 0 ? ld_global<uint32_t>(&recs[b].count) : 0u;
}
// Consumes the touched words so that the loads stay; emits no instruction.
__device__ __forceinline__ void keep(uint32_t v) { __asm__ volatile("" ::"v"(v)); }

__device__ __forceinline__ void load_half_rec(const BlockRec* __restrict__ recs, int b,
                                              HalfRec& h) {
  if (b < 0) return;  // global loads (see ld_global): only LDS waits follow
  const u32x4 a = ld_global_x4(recs + b);                          // sad_min, count, intra_x
  const u32x4 e = ld_global_x4(reinterpret_cast<const char*>(recs + b) + 16);  // e[0..3]
  h.count = a.y;
  h.intra_x = a.z;
  h.e[0] = e.x;
  h.e[1] = e.y;
  h.e[2] = e.z;
  h.e[3] = e.w;
  h.e[4] = ld_global<uint32_t>(&recs[b].e[4]);
}

__device__ __forceinline__ void resolve_pair_half(const KGeom& g,
                                                  const BlockRec* __restrict__ recs,
                                                  const uint16_t* __restrict__ ovf,
                                                  acbm_block_result* __restrict__ out,
                                                  uint32_t lam, uint32_t* st,
                                                  const uint8_t* __restrict__ cur,
                                                  const uint8_t* __restrict__ ref) {
  const int p = g.p, bx = g.bx, by = g.by;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int steps = (bx - 1) + 2 * (by - 1) + 1;
  const int i = threadIdx.x;  // this thread's place in every step
  MultiList& ml = multi_list();
  if (threadIdx.x < 2) ml.cnt[threadIdx.x] = 0;
  __syncthreads();
  HalfRec h{}, hn{};
  uint32_t sink = 0, touched = 0;
  int b = step_block(g, 0, i);
  load_half_rec(recs, b, h);
  for (int k = 0; k < steps; ++k) {
    const int bn = step_block(g, k + 1, i);
    load_half_rec(recs, bn, hn);  // in flight while this step is decided
    sink ^= touched;  // last step's word, waited for with the prefetch
    touched = touch_rec(recs, step_block(g, k + 2, i));
    // the next step's list: its last readers passed a barrier since
    if (threadIdx.x == 0) ml.cnt[(k + 1) & 1] = 0;
    if (b >= 0) {
      const int r = b / bx, c = b - r * bx;
      int px = 0, py = 0;
      median_pred(st, b, r, c, bx, &px, &py);  // its neighbours are decided
      if (h.count == 1) {
        half_decide_lane(g, h, b, px, py, lam, out + b, st + b);
      } else {
        const int q = atomicAdd(&ml.cnt[k & 1], 1);
        ml.b[q] = (uint32_t)b;
        ml.n[q] = h.count;
      }
    }
    __syncthreads();  // lane decisions and the list
    const int nm = __builtin_amdgcn_readfirstlane(ml.cnt[k & 1]);
    if (nm) {
      for (int j = wave; j < nm; j += nwaves) {
        const int bb = (int)ml.b[j];
        const uint32_t cnt = ml.n[j];
        const int r = bb / bx, c = bb - r * bx;
        int qx = 0, qy = 0;
        median_pred(st, bb, r, c, bx, &qx, &qy);
        const uint16_t* row = ovf + (size_t)bb * ovf_stride(p);
        if (cnt <= half_cap(p)) {
          half_decide_prepared(g, recs + bb, row, cnt, bb, qx, qy, lam, out + bb, st + bb);
        } else {
          const uint64_t key = wave_block_argmin<true>(recs + bb, row, p, qx, qy, lam);
          half_decide(g, recs + bb, cur, ref, bb, qx, qy, lam, key, out + bb, st + bb);
        }
      }
      __syncthreads();  // this step's decisions before the next step reads them
    }
    b = bn;
    h = hn;
  }
  keep(sink ^ touched);
}

// Lane 0's value to the four lanes of its quad (DPP quad_perm 0,0,0,0).
__device__ __forceinline__ uint32_t quad_bcast0(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x00, 0xF, 0xF, false);
}

// Minimum over the four lanes of a quad (quad_perm 1,0,3,2 then 2,3,0,1);
// every lane of the quad gets it.
__device__ __forceinline__ uint64_t quad_min_u64(uint64_t k) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)k, 0xB1, 0xF, 0xF, false);
  uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(k >> 32), 0xB1, 0xF, 0xF, false);
  uint64_t o = ((uint64_t)hi << 32) | lo;
  k = o < k ? o : k;
  lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)k, 0x4E, 0xF, 0xF, false);
  hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(k >> 32), 0x4E, 0xF, 0xF, false);
  o = ((uint64_t)hi << 32) | lo;
  return o < k ? o : k;
}

// Half-pel resolve with four lanes per block, for frames of at most 256
// block rows.  Each lane of a block's quad prefetches the record's header,
// e[0..4] and, as lane q, winner q's 8 prepared half-pel SADs (overflow
// entries 8q .. 8q+7).  A block with at most four possible winners (and
// prepared SADs) is decided by its quad: lane q prices winner q, a quad
// minimum gives the integer winner, and its lane finishes the half-pel step
// with its SADs (e[1..4] for a single winner).  Blocks with more winners go
// to the LDS list and whole waves, as in resolve_pair_half.
struct HalfPart {
  u32x4 hd;   // sad_min, count, intra_x, pad
  u32x4 e03;  // e[0..3]
  uint32_t e4;
  u32x4 hs;   // winner q's prepared SADs
};

__device__ __forceinline__ void load_half_part(const BlockRec* __restrict__ recs,
                                               const uint16_t* __restrict__ ovf, int p, int b,
                                               int q, HalfPart& r) {
  if (b < 0) return;
  const char* rb = reinterpret_cast<const char*>(recs + b);
  r.hd = ld_global_x4(rb);
  r.e03 = ld_global_x4(rb + 16);
  r.e4 = ld_global<uint32_t>(rb + 32);
  // only inside this block's overflow region (ovf_stride(p) entries)
  if (8 * q + 8 <= (int)ovf_stride(p)) r.hs = ld_global_x4(ovf + (size_t)b * ovf_stride(p) + 8 * q);
}

__device__ __forceinline__ void resolve_pair_half4(const KGeom& g,
                                                   const BlockRec* __restrict__ recs,
                                                   const uint16_t* __restrict__ ovf,
                                                   acbm_block_result* __restrict__ out,
                                                   uint32_t lam, uint32_t* st,
                                                   const uint8_t* __restrict__ cur,
                                                   const uint8_t* __restrict__ ref) {
  const int p = g.p, bx = g.bx, by = g.by;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int steps = (bx - 1) + 2 * (by - 1) + 1;
  const int i = (int)threadIdx.x >> 2, q = (int)threadIdx.x & 3;  // block slot, quad lane
  const uint32_t lim = min(4u, half_cap(p));  // winners a quad decides
  MultiList& ml = multi_list();
  if (threadIdx.x < 2) ml.cnt[threadIdx.x] = 0;
  __syncthreads();
  HalfPart h{}, hn{};
  uint32_t sink = 0, touched = 0;
  int b = step_block(g, 0, i);
  load_half_part(recs, ovf, p, b, q, h);
  for (int k = 0; k < steps; ++k) {
    const int bn = step_block(g, k + 1, i);
    load_half_part(recs, ovf, p, bn, q, hn);  // in flight while this step is decided
    sink ^= touched;                          // last step's word, waited for with the prefetch
    touched = q == 0 ? touch_rec(recs, step_block(g, k + 2, i)) : 0u;
    if (threadIdx.x == 0) ml.cnt[(k + 1) & 1] = 0;
    if (b >= 0) {  // the four lanes of a quad share b and its record
      const int r = b / bx, c = b - r * bx;
      int px = 0, py = 0;
      median_pred(st, b, r, c, bx, &px, &py);  // its neighbours are decided
      const uint32_t count = h.hd.y;
      if (count <= lim) {
        const bool has = (uint32_t)q < count;
        const uint32_t e = q == 0 ? h.e03.x : q == 1 ? h.e03.y : q == 2 ? h.e03.z : h.e03.w;
        int u = 0, v = 0;
        uint64_t key = ~0ull;
        if (has) {
          window_uv(e & 0xFFFFu, p, &u, &v);
          key = int_key<true>(e >> 16, u, v, p, px, py, lam);
        }
        const uint64_t k0 = quad_min_u64(key);
        if (has && key == k0) {  // the integer winner's lane (keys are unique)
          const uint32_t h4[4] = {count == 1 ? h.e03.y : h.hs.x, count == 1 ? h.e03.z : h.hs.y,
                                  count == 1 ? h.e03.w : h.hs.z, count == 1 ? h.e4 : h.hs.w};
          uint32_t sads[8];
#pragma unroll
          for (int s2 = 0; s2 < 8; ++s2) sads[s2] = (h4[s2 / 2] >> (16 * (s2 & 1))) & 0xFFFFu;
          half_finish(g, b, 2 * u, 2 * v, key, sads, px, py, lam, h.hd.z, true, out + b, st + b);
        }
      } else if (q == 0) {
        const int at = atomicAdd(&ml.cnt[k & 1], 1);
        ml.b[at] = (uint32_t)b;
        ml.n[at] = count;
      }
    }
    __syncthreads();  // quad decisions and the list
    const int nm = __builtin_amdgcn_readfirstlane(ml.cnt[k & 1]);
    if (nm) {
      for (int j = wave; j < nm; j += nwaves) {
        const int bb = (int)ml.b[j];
        const uint32_t cnt = ml.n[j];
        const int r = bb / bx, c = bb - r * bx;
        int qx = 0, qy = 0;
        median_pred(st, bb, r, c, bx, &qx, &qy);
        const uint16_t* row = ovf + (size_t)bb * ovf_stride(p);
        if (cnt <= half_cap(p)) {
          half_decide_prepared(g, recs + bb, row, cnt, bb, qx, qy, lam, out + bb, st + bb);
        } else {
          const uint64_t key = wave_block_argmin<true>(recs + bb, row, p, qx, qy, lam);
          half_decide(g, recs + bb, cur, ref, bb, qx, qy, lam, key, out + bb, st + bb);
        }
      }
      __syncthreads();  // this step's decisions before the next step reads them
    }
    b = bn;
    h = hn;
  }
  keep(sink ^ touched);
}

// Integer resolve: the same anti-diagonal order as the half-pel one.  Each
// thread prefetches the whole record of its block of the next step (header
// and the kShort listed winners, 8 x 16 bytes), so that a block with at most
// kShort possible winners is priced by its own lane with no memory access
// on the sequential path; a block with more (list or row formats) is priced
// by its whole wave.
struct IntRec {
  uint4 h;      // sad_min, count, intra_x, pad
  uint4 e[7];   // the kShort = 28 listed winners
};
static_assert(kShort == 28, "the record's list is 7 x 16 bytes");

__device__ __forceinline__ void load_int_rec(const BlockRec* __restrict__ recs, int b,
                                             IntRec& r) {
  if (b < 0) return;  // global loads (see ld_global): only LDS waits follow
  const char* q = reinterpret_cast<const char*>(recs + b);
  const u32x4 h = ld_global_x4(q);
  r.h = make_uint4(h.x, h.y, h.z, h.w);
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const u32x4 e = ld_global_x4(q + 16 * (1 + k));
    r.e[k] = make_uint4(e.x, e.y, e.z, e.w);
  }
}

// The decided block's result and decision word.
__device__ __forceinline__ void int_write(const KGeom& g, int b, int u, int v, uint32_t sad,
                                          int px, int py, uint32_t lam, uint32_t intra_x,
                                          acbm_block_result* __restrict__ out, uint32_t* st) {
  const int r = b / g.bx, c = b - r * g.bx;
  const uint32_t rate = se_bits(u - px) + se_bits(v - py);
  put_result(out, u, v, sad, sad + lam * rate,
             rate, valid_count(g.p, c * g.bw, r * g.bh, g.bw, g.bh, g.width, g.height),
             ACBM_MODE_FSBM, intra_x);
  *st = (sad << 16) | pack_mv(u, v);
}

__device__ __forceinline__ void int_decide_lane(const KGeom& g, const IntRec& rec, int b, int px,
                                                int py, uint32_t lam,
                                                acbm_block_result* __restrict__ out,
                                                uint32_t* st) {
  const int p = g.p;
  const uint32_t W = 2u * (uint32_t)p + 1u;
  const uint32_t inv = (uint32_t)(((1ull << 32) + W - 1) / W);  // ras / W = umulhi(ras, inv)
  const uint32_t count = rec.h.y;
  const uint32_t e[kShort] = {rec.e[0].x, rec.e[0].y, rec.e[0].z, rec.e[0].w, rec.e[1].x,
                              rec.e[1].y, rec.e[1].z, rec.e[1].w, rec.e[2].x, rec.e[2].y,
                              rec.e[2].z, rec.e[2].w, rec.e[3].x, rec.e[3].y, rec.e[3].z,
                              rec.e[3].w, rec.e[4].x, rec.e[4].y, rec.e[4].z, rec.e[4].w,
                              rec.e[5].x, rec.e[5].y, rec.e[5].z, rec.e[5].w, rec.e[6].x,
                              rec.e[6].y, rec.e[6].z, rec.e[6].w};
  uint64_t best = ~0ull;
#pragma unroll
  for (int s = 0; s < kShort; ++s) {
    if (s >= (int)count) break;
    const uint32_t ras = e[s] & 0xFFFFu;
    const uint32_t vq = __umulhi(ras, inv);
    const int v = (int)vq - p, u = (int)(ras - vq * W) - p;
    const uint64_t k = int_key<false>(e[s] >> 16, u, v, p, px, py, lam);
    best = k < best ? k : best;
  }
  const uint32_t ras = (uint32_t)(best & 0xFFFFu);
  const uint32_t vq = __umulhi(ras, inv);
  const int v = (int)vq - p, u = (int)(ras - vq * W) - p;
  const uint32_t sad = (uint32_t)(best >> 32) - lam * (se_bits(u - px) + se_bits(v - py));
  int_write(g, b, u, v, sad, px, py, lam, rec.h.z, out, st);
}

__device__ __forceinline__ void resolve_pair_int(const KGeom& g,
                                                 const BlockRec* __restrict__ recs,
                                                 const uint16_t* __restrict__ ovf,
                                                 acbm_block_result* __restrict__ out,
                                                 uint32_t lam, uint32_t* st) {
  const int p = g.p, bx = g.bx, by = g.by;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int steps = (bx - 1) + 2 * (by - 1) + 1;
  const int i = threadIdx.x;  // this thread's place in every step
  MultiList& ml = multi_list();
  if (threadIdx.x < 2) ml.cnt[threadIdx.x] = 0;
  __syncthreads();
  IntRec h{}, hn{};
  uint32_t sink = 0, touched = 0;
  int b = step_block(g, 0, i);
  load_int_rec(recs, b, h);
  for (int k = 0; k < steps; ++k) {
    const int bn = step_block(g, k + 1, i);
    load_int_rec(recs, bn, hn);  // in flight while this step is decided
    sink ^= touched;  // last step's word, waited for with the prefetch
    touched = touch_rec(recs, step_block(g, k + 2, i));
    // the next step's list: its last readers passed a barrier since
    if (threadIdx.x == 0) ml.cnt[(k + 1) & 1] = 0;
    if (b >= 0) {
      const int r = b / bx, c = b - r * bx;
      int px = 0, py = 0;
      median_pred(st, b, r, c, bx, &px, &py);  // its neighbours are decided
      if (h.h.y <= (uint32_t)kShort) {
        int_decide_lane(g, h, b, px, py, lam, out + b, st + b);
      } else {
        const int q = atomicAdd(&ml.cnt[k & 1], 1);
        ml.b[q] = (uint32_t)b;
        ml.n[q] = h.h.z;  // intra_x, for the result
      }
    }
    __syncthreads();  // lane decisions and the list
    const int nm = __builtin_amdgcn_readfirstlane(ml.cnt[k & 1]);
    if (nm) {
      for (int j = wave; j < nm; j += nwaves) {
        const int bb = (int)ml.b[j];
        const uint32_t ix = ml.n[j];
        const int r = bb / bx, c = bb - r * bx;
        int qx = 0, qy = 0;
        median_pred(st, bb, r, c, bx, &qx, &qy);
        const uint64_t key =
            wave_block_argmin<false>(recs + bb, ovf + (size_t)bb * ovf_stride(p), p, qx, qy, lam);
        int u = 0, v = 0;
        window_uv((uint32_t)(key & 0xFFFFu), p, &u, &v);
        const uint32_t sad = (uint32_t)(key >> 32) - lam * (se_bits(u - qx) + se_bits(v - qy));
        if (lane == 0) int_write(g, bb, u, v, sad, qx, qy, lam, ix, out + bb, st + bb);
      }
      __syncthreads();  // this step's decisions before the next step reads them
    }
    b = bn;
    h = hn;
  }
  keep(sink ^ touched);
}

// The same schedule with four lanes per block, for frames of at most 256
// block rows (a step then fits in a quarter of the group).  Lane q of a
// block's quad prefetches 32 bytes of its record for the next step: the
// header and e[0..3] for q = 0, e[8q-4 .. 8q+3] otherwise.  Each lane prices
// the listed winners it holds and a quad minimum gives the block's key, so
// the serial pricing of up to 28 winners becomes at most 8 per lane.
struct IntPart {
  u32x4 a, b;
};

__device__ __forceinline__ void load_int_part(const BlockRec* __restrict__ recs, int b, int q,
                                              IntPart& r) {
  if (b < 0) return;
  const char* base = reinterpret_cast<const char*>(recs + b) + 32 * q;
  r.a = ld_global_x4(base);
  r.b = ld_global_x4(base + 16);
}

__device__ __forceinline__ void resolve_pair_int4(const KGeom& g,
                                                  const BlockRec* __restrict__ recs,
                                                  const uint16_t* __restrict__ ovf,
                                                  acbm_block_result* __restrict__ out,
                                                  uint32_t lam, uint32_t* st) {
  const int p = g.p, bx = g.bx, by = g.by;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int steps = (bx - 1) + 2 * (by - 1) + 1;
  const int i = (int)threadIdx.x >> 2, q = (int)threadIdx.x & 3;  // block slot, quarter
  const uint32_t W = 2u * (uint32_t)p + 1u;
  const uint32_t inv = (uint32_t)(((1ull << 32) + W - 1) / W);  // ras / W = umulhi(ras, inv)
  const int s0 = q ? 8 * q - 4 : 0, nq = q ? 8 : 4;              // the entries this lane holds
  MultiList& ml = multi_list();
  if (threadIdx.x < 2) ml.cnt[threadIdx.x] = 0;
  __syncthreads();
  IntPart h0{}, h1{};
  uint32_t sink = 0, touched = 0;
  load_int_part(recs, step_block(g, 0, i), q, h0);
  // One step: decides the blocks of step k from h (prefetched one step
  // earlier) and prefetches step k + 1 into hn.
  auto step = [&](int k, const IntPart& h, IntPart& hn) {
    const int b = step_block(g, k, i);
    load_int_part(recs, step_block(g, k + 1, i), q, hn);  // in flight while this step is decided
    sink ^= touched;                 // last step's word, waited for with the prefetch
    touched = q == 0 ? touch_rec(recs, step_block(g, k + 2, i)) : 0u;
    if (threadIdx.x == 0) ml.cnt[(k + 1) & 1] = 0;
    const uint32_t count = quad_bcast0(h.a.y);  // the four lanes of a quad agree on b
    if (b >= 0) {
      const int r = b / bx, c = b - r * bx;
      int px = 0, py = 0;
      median_pred(st, b, r, c, bx, &px, &py);  // its neighbours are decided
      if (count <= (uint32_t)kShort) {
        const uint32_t e[8] = {q ? h.a.x : h.b.x, q ? h.a.y : h.b.y, q ? h.a.z : h.b.z,
                               q ? h.a.w : h.b.w, h.b.x, h.b.y, h.b.z, h.b.w};
        uint64_t best = ~0ull;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          if (s < nq && (uint32_t)(s0 + s) < count) {
            const uint32_t ras = e[s] & 0xFFFFu;
            const uint32_t vq = __umulhi(ras, inv);
            const int v = (int)vq - p, u = (int)(ras - vq * W) - p;
            const uint64_t kk = int_key<false>(e[s] >> 16, u, v, p, px, py, lam);
            best = kk < best ? kk : best;
          }
        }
        best = quad_min_u64(best);
        if (q == 0) {
          const uint32_t ras = (uint32_t)(best & 0xFFFFu);
          const uint32_t vq = __umulhi(ras, inv);
          const int v = (int)vq - p, u = (int)(ras - vq * W) - p;
          const uint32_t sad = (uint32_t)(best >> 32) - lam * (se_bits(u - px) + se_bits(v - py));
          int_write(g, b, u, v, sad, px, py, lam, h.a.z, out + b, st + b);
        }
      } else if (q == 0) {
        const int at = atomicAdd(&ml.cnt[k & 1], 1);
        ml.b[at] = (uint32_t)b;
        ml.n[at] = h.a.z;  // intra_x, for the result
      }
    }
    __syncthreads();  // lane decisions and the list
    const int nm = __builtin_amdgcn_readfirstlane(ml.cnt[k & 1]);
    if (nm) {
      for (int j = wave; j < nm; j += nwaves) {
        const int bb = (int)ml.b[j];
        const uint32_t ix = ml.n[j];
        const int r = bb / bx, c = bb - r * bx;
        int qx = 0, qy = 0;
        median_pred(st, bb, r, c, bx, &qx, &qy);
        const uint64_t key =
            wave_block_argmin<false>(recs + bb, ovf + (size_t)bb * ovf_stride(p), p, qx, qy, lam);
        int u = 0, v = 0;
        window_uv((uint32_t)(key & 0xFFFFu), p, &u, &v);
        const uint32_t sad = (uint32_t)(key >> 32) - lam * (se_bits(u - qx) + se_bits(v - qy));
        if (lane == 0) int_write(g, bb, u, v, sad, qx, qy, lam, ix, out + bb, st + bb);
      }
      __syncthreads();  // this step's decisions before the next step reads them
    }
  };
  // Two steps per iteration with the buffers swapped: no register copy, which
  // would wait for every memory operation of the step, stores included.
  for (int k = 0; k < steps; k += 2) {
    step(k, h0, h1);
    if (k + 1 < steps) step(k + 1, h1, h0);
  }
  keep(sink ^ touched);
}

// Integer resolve when few blocks have several possible winners: blocks
// with a single one are decided at once, in parallel, without a predictor;
// the rest are decided in sweeps as soon as their left, top and top-right
// neighbours are (each sweep decides at least the first open block in
// raster order, so nb sweeps always suffice); a wave prices each ready block
// of its 64-block chunk together.  Results are written in a final parallel
// pass.
constexpr uint32_t kOpen = 0xFFFF0000u | kMvUnset;

__device__ __forceinline__ void resolve_pair_sweeps(const KGeom& g,
                                                    const BlockRec* __restrict__ recs,
                                                    const uint16_t* __restrict__ ovf,
                                                    acbm_block_result* __restrict__ out,
                                                    uint32_t lam, uint32_t* st, int* pending_flag) {
  int& pending = *pending_flag;
  const int p = g.p, nb = g.nb, bx = g.bx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    uint32_t w = kOpen;
    if (recs[b].count == 1) {
      const uint32_t e = recs[b].e[0];
      int u, v;
      window_uv(e & 0xFFFFu, p, &u, &v);
      w = (e & 0xFFFF0000u) | pack_mv(u, v);
    }
    st[b] = w;
  }
  __syncthreads();
  for (int sweep = 0; sweep <= nb; ++sweep) {
    if (threadIdx.x == 0) pending = 0;
    __syncthreads();
    for (int base = wave * 64; base < nb; base += nwaves * 64) {
      const int b = base + lane;
      int px = 0, py = 0;
      bool ready = false;
      if (b < nb && is_open(st[b])) {
        const int r = b / bx, c = b - r * bx;
        ready = median_pred(st, b, r, c, bx, &px, &py);
        if (!ready) pending = 1;
      }
      uint64_t mask = __ballot(ready);
      while (mask) {
        const int k = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int bb = base + k;
        const int qx = __shfl(px, k, 64), qy = __shfl(py, k, 64);
        const uint64_t key =
            wave_block_argmin<false>(recs + bb, ovf + (size_t)bb * ovf_stride(p), p, qx, qy, lam);
        int u = 0, v = 0;
        window_uv((uint32_t)(key & 0xFFFFu), p, &u, &v);
        const uint32_t sad = (uint32_t)(key >> 32) - lam * (se_bits(u - qx) + se_bits(v - qy));
        if (lane == 0) st[bb] = (sad << 16) | pack_mv(u, v);
      }
    }
    __syncthreads();
    // one LDS word, uniform; readfirstlane keeps the break (the loop contains
    // barriers) a uniform branch for the compiler
    const int again = __builtin_amdgcn_readfirstlane(pending);
    __syncthreads();
    if (!again) break;
  }
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int r = b / bx, c = b - r * bx;
    int px = 0, py = 0;
    median_pred(st, b, r, c, bx, &px, &py);
    const uint32_t w = st[b];
    int_write(g, b, mv_x((uint16_t)w), mv_y((uint16_t)w), w >> 16, px, py, lam,
              recs[b].intra_x, out + b, st + b);
  }
}

// FSBM resolve of one frame pair by the whole group.  `st` is the pair's
// decision state (LDS or workspace); `shared` two words of LDS.  HP:
// half-pel precision (every block needs its predictor: anti-diagonal
// steps); cur and ref are then the pair's frames.  Integer precision picks
// sweeps when `sweeps` allows them and under a quarter of the blocks have
// several possible winners, and steps otherwise.  (A sweep scans the whole
// frame, so it wants every wave of a 1024-thread group; the steps need four
// lanes per block row.)  Both decide every block with its final predictor,
// so the results do not depend on the choice.
template <bool HP>
__device__ __forceinline__ void resolve_pair(const KGeom& g, const BlockRec* __restrict__ recs,
                                             const uint16_t* __restrict__ ovf,
                                             acbm_block_result* __restrict__ out, uint32_t lam,
                                             uint32_t* st, int* shared,
                                             const uint8_t* __restrict__ cur,
                                             const uint8_t* __restrict__ ref, bool sweeps) {
  if constexpr (HP) {
    if (4 * g.by <= (int)blockDim.x)
      resolve_pair_half4(g, recs, ovf, out, lam, st, cur, ref);
    else
      resolve_pair_half(g, recs, ovf, out, lam, st, cur, ref);
  } else {
    int nmulti = g.nb;
    if (sweeps) {
      if (threadIdx.x == 0) shared[1] = 0;
      __syncthreads();
      int multi = 0;
      for (int b = threadIdx.x; b < g.nb; b += blockDim.x) multi += recs[b].count > 1;
      multi = (int)wave_sum_u32((uint32_t)multi);
      if ((threadIdx.x & 63) == 0) atomicAdd(&shared[1], multi);
      __syncthreads();
      nmulti = __builtin_amdgcn_readfirstlane(shared[1]);
    }
    if (4 * nmulti < g.nb)
      resolve_pair_sweeps(g, recs, ovf, out, lam, st, shared);
    else if (4 * g.by <= (int)blockDim.x)
      resolve_pair_int4(g, recs, ovf, out, lam, st);
    else
      resolve_pair_int(g, recs, ovf, out, lam, st);
  }
}

// One workgroup per frame pair.  The state lives in LDS when it fits
// (st_global == nullptr), else in a workspace array; either way only this
// workgroup touches it.
template <bool HP>
__global__ void __launch_bounds__(1024)
k_resolve(const KGeom g, const BlockRec* __restrict__ recs, const uint16_t* __restrict__ ovf,
          acbm_block_result* __restrict__ out, uint32_t lam, uint32_t* st_global,
          const FramePtrs fr) {
  extern __shared__ uint32_t st_lds[];
  __shared__ int shared[2];
  const int pair = blockIdx.x;
  const BlockRec* r = recs + (size_t)pair * g.nb;
  const uint16_t* o = ovf + (size_t)pair * g.nb * ovf_stride(g.p);
  acbm_block_result* res = out + (size_t)pair * g.nb;
  const uint8_t* cur = HP ? fr.f[pair + 1] : nullptr;
  const uint8_t* ref = HP ? fr.f[pair] : nullptr;
  // two call sites, so that each sees one memory kind for the state (a
  // pointer that may be either compiles to FLAT accesses, whose waits also
  // cover the record prefetch)
  if (st_global)
    resolve_pair<HP>(g, r, o, res, lam, st_global + (size_t)pair * g.nb, shared, cur, ref, true);
  else
    resolve_pair<HP>(g, r, o, res, lam, st_lds, shared, cur, ref, true);
}

// Half-pel SADs prepared off the resolve's sequential path.  For every block
// with at most half_cap(p) possible winners, the 8 half-pel neighbours of
// each winner (they do not depend on the predictor): a single winner's go to
// the free record slots e[1..4], several winners' to the block's overflow
// region (winner s at entries 8s .. 8s+7), which only blocks with more than
// kShort winners use otherwise.  Ring order as half_ring_offset.
// One lane per block row: 64 / M blocks per wave.  A lane loads, for one
// winner (u, v), reference rows y0+j+v-1 .. y0+j+v+1 over the bytes
// x0+u-1 .. x0+u+N (two dword-aligned windows, for the left and the other
// columns) and its current row once, and computes its row of all 8
// neighbours from registers; the M rows of a neighbour are summed by DPP.
// Loads of invalid neighbours are clamped into the frame and their sums
// dropped.
template <int N, int M>
__global__ void __launch_bounds__(256)
k_half_prep(const KGeom g, const FramePtrs fr, int npairs, BlockRec* __restrict__ recs,
            uint16_t* __restrict__ ovf) {
  constexpr int NC = N / 4, PER = 64 / M;
  const int lane = threadIdx.x & 63, j = lane % M;
  const size_t item = ((size_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * PER + lane / M;
  const size_t items = (size_t)npairs * g.nb;
  const int p = g.p;
  const uint32_t cap = half_cap(p);
  int pair = 0, b = 0;
  uint32_t count = 0;
  if (item < items) {
    pair = (int)(item / (size_t)g.nb);
    b = (int)(item % (size_t)g.nb);
    count = recs[item].count;
  }
  const uint32_t ns = (count >= 1 && count <= cap) ? count : 0u;  // winners to prepare
  const uint32_t smax = __builtin_amdgcn_readfirstlane(__ockl_wfred_max_u32(ns));
  const int r = b / g.bx, c = b - r * g.bx;
  const int x0 = c * N, y0 = r * M;
  const uint8_t* __restrict__ cur = fr.f[pair + 1];
  const uint8_t* __restrict__ ref = fr.f[pair];
  const int last_dw = (g.pitch >> 2) - 1;
  uint32_t cw[NC];
  if (ns) {
    const uint32_t* cr = reinterpret_cast<const uint32_t*>(cur + (size_t)(y0 + j) * g.pitch + x0);
#pragma unroll
    for (int q = 0; q < NC; ++q) cw[q] = cr[q];
  }
  for (uint32_t s = 0; s < smax; ++s) {
    const bool act = s < ns;
    int u = 0, v = 0;
    if (act) window_uv(recs[item].e[s] & 0xFFFFu, p, &u, &v);
    // rows v-1, v, v+1 and the two column windows, clamped into the frame
    uint32_t wa[3][NC + 1], wb[3][NC + 1];
    const int xa = x0 + u - 1, xb = x0 + u;
    const int da = max(xa, 0) >> 2, db = xb >> 2;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int y = min(max(y0 + j + v - 1 + t, 0), g.height - 1);
      const uint32_t* row = reinterpret_cast<const uint32_t*>(ref + (size_t)y * g.pitch);
#pragma unroll
      for (int q = 0; q <= NC; ++q) {
        wa[t][q] = act ? row[min(da + q, last_dw)] : 0u;
        wb[t][q] = act ? row[min(max(db, 0) + q, last_dw)] : 0u;
      }
    }
    const uint32_t sha = (uint32_t)(xa & 3), shb = (uint32_t)(xb & 3);
    uint32_t sums[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int du, dv;
      half_ring_offset(k, &du, &dv);
      const int U = 2 * u + du, V = 2 * v + dv;
      const bool ok = act && cand_valid_half(U, V, p, x0, y0, N, M, g.width, g.height);
      // rows: dv = -1 reads v-1 and v; dv = 0 reads v; dv = +1 reads v and v+1
      const int t0 = dv < 0 ? 0 : 1, t1 = dv > 0 ? 2 : 1;
      const uint32_t(&w0)[NC + 1] = du < 0 ? wa[t0] : wb[t0];
      const uint32_t(&w1)[NC + 1] = du < 0 ? wa[t1] : wb[t1];
      const uint32_t acc = ok ? half_row_sad<NC>(w0, w1, du < 0 ? sha : shb, U & 1, V & 1, cw, 0u)
                              : 0u;
      const uint32_t sum = group_sum<M>(acc);
      sums[k] = ok ? sum : 0xFFFFu;
    }
    if (act && j == 0) {
      if (count == 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) recs[item].e[1 + q] = sums[2 * q] | (sums[2 * q + 1] << 16);
      } else {
        uint4* dst = reinterpret_cast<uint4*>(ovf + item * ovf_stride(p)) + s;
        *dst = make_uint4(sums[0] | (sums[1] << 16), sums[2] | (sums[3] << 16),
                          sums[4] | (sums[5] << 16), sums[6] | (sums[7] << 16));
      }
    }
  }
}

// The resolves of every pair of a set of FSBM jobs: one workgroup per pair,
// workgroup k resolving pair k + pair_base of the numbering by pair0.
__global__ void __launch_bounds__(1024)
k_resolve_batch(const BatchJob* __restrict__ jobs, int njobs, uint32_t pair_base, bool sweeps) {
  extern __shared__ uint32_t st_lds[];
  __shared__ int shared[2];
  const uint32_t wg = blockIdx.x + pair_base;
  int j = 0;
  for (int base = 0; base < njobs; base += 64) {  // jobs are sorted by pair0
    const int k = base + (int)(threadIdx.x & 63);
    const uint32_t first = k < njobs ? jobs[k].pair0 : 0xFFFFFFFFu;
    const int n = __popcll(__ballot(first <= wg));
    if (n == 0) break;
    j = base + n - 1;
  }
  j = __builtin_amdgcn_readfirstlane(j);  // uniform: the resolve loops contain barriers
  const BatchJob& J = jobs[j];
  const KGeom g = J.g;
  const int pair = (int)(wg - J.pair0);
  const BlockRec* recs = J.recs + (size_t)pair * g.nb;
  const uint16_t* ovf = J.ovf + (size_t)pair * g.nb * ovf_stride(g.p);
  acbm_block_result* out = J.out + (size_t)pair * g.nb;
  const bool hp = __builtin_amdgcn_readfirstlane(J.subpel) != 0;
  const uint8_t* cur = hp ? ld_global<const uint8_t*>(J.frames + pair + 1) : nullptr;
  const uint8_t* ref = hp ? ld_global<const uint8_t*>(J.frames + pair) : nullptr;
  // one call site per memory kind of the state (see k_resolve)
  if (__builtin_amdgcn_readfirstlane(J.mv_ws != nullptr)) {
    uint32_t* st = J.mv_ws + (size_t)pair * g.nb;
    if (hp)
      resolve_pair<true>(g, recs, ovf, out, J.lam, st, shared, cur, ref, sweeps);
    else
      resolve_pair<false>(g, recs, ovf, out, J.lam, st, shared, nullptr, nullptr, sweeps);
  } else {
    if (hp)
      resolve_pair<true>(g, recs, ovf, out, J.lam, st_lds, shared, cur, ref, sweeps);
    else
      resolve_pair<false>(g, recs, ovf, out, J.lam, st_lds, shared, nullptr, nullptr, sweeps);
  }
}

// ---------------------------------------------------------------------------
// Host side: plans and launches.
// ---------------------------------------------------------------------------
#define ACBM_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(11) X(16)

template <int N, int M, bool kTable>
static int launch_search_nm(const KGeom& g, const SearchPlan& pl, const FramePtrs& fr,
                            int npairs, uint32_t* table, BlockRec* recs, uint16_t* ovf,
                            uint32_t slack, hipStream_t st) {
  const WindowShape s = window_shape<N, M>(g.p, pl.R);
  const int grid_x = ((g.nb + 7) / 8) * 8;
  dim3 grid(grid_x, npairs), block(pl.threads);
  switch (pl.R) {
#define ACBM_CASE(RR)                                                                         \
  case RR: {                                                                                  \
    if (pl.lds_bytes > 64 * 1024)                                                             \
      (void)hipFuncSetAttribute((const void*)k_search<N, M, RR, kTable>,                      \
                                hipFuncAttributeMaxDynamicSharedMemorySize, pl.lds_bytes);    \
    ProfScope ps("search", st);                                                               \
    hipLaunchKernelGGL((k_search<N, M, RR, kTable>), grid, block, pl.lds_bytes, st, g, s, fr, \
                       table, recs, ovf, slack);                                              \
    break;                                                                                    \
  }
    ACBM_R_LIST(ACBM_CASE)
#undef ACBM_CASE
    default:
      return fail(ACBM_E_UNSUPPORTED, "no search kernel for this row blocking");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the window search");
}

// Rows of the tiled search (register budget of four blocks' accumulators).
#define ACBM_TILE_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6)

static int launch_search_tile(const KGeom& g, const SearchPlan& pl, const FramePtrs& fr,
                              int npairs, BlockRec* recs, uint16_t* ovf, uint32_t slack,
                              hipStream_t st) {
  if (g.bw != 8 || g.bh != 8 || (g.bx & 1) || (g.by & 1))
    return fail(ACBM_E_INVAL, "tiled search needs 8x8 blocks on an even grid");
  const WindowShape s = window_shape<16, 16>(g.p, pl.R);
  const int nt = g.nb >> 2;
  const int grid_x = ((nt + 7) / 8) * 8;
  dim3 grid(grid_x, npairs), block(pl.threads);
  switch (pl.R) {
#define ACBM_CASE(RR)                                                                      \
  case RR: {                                                                               \
    if (pl.lds_bytes > 64 * 1024)                                                          \
      (void)hipFuncSetAttribute((const void*)k_search_tile<RR>,                            \
                                hipFuncAttributeMaxDynamicSharedMemorySize, pl.lds_bytes); \
    ProfScope ps("search", st);                                                            \
    hipLaunchKernelGGL((k_search_tile<RR>), grid, block, pl.lds_bytes, st, g, s, fr, recs, \
                       ovf, slack);                                                        \
    break;                                                                                 \
  }
    ACBM_TILE_R_LIST(ACBM_CASE)
#undef ACBM_CASE
    default:
      return fail(ACBM_E_UNSUPPORTED, "no tiled search kernel for this row blocking");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the tiled window search");
}

template <bool kTable>
static int launch_search_with(const KGeom& g, const SearchPlan& pl, const FramePtrs& fr,
                              int npairs, uint32_t* table, BlockRec* recs, uint16_t* ovf,
                              uint32_t slack, hipStream_t st) {
  if (!pl.R) return fail(ACBM_E_UNSUPPORTED, "search window does not fit in LDS");
  if (pl.tile == 2) {
    if (kTable) return fail(ACBM_E_INVAL, "a SAD table is searched one block per workgroup");
    return launch_search_tile(g, pl, fr, npairs, recs, ovf, slack, st);
  }
  if (g.bw == 16 && g.bh == 16)
    return launch_search_nm<16, 16, kTable>(g, pl, fr, npairs, table, recs, ovf, slack, st);
  if (g.bw == 16 && g.bh == 8)
    return launch_search_nm<16, 8, kTable>(g, pl, fr, npairs, table, recs, ovf, slack, st);
  if (g.bw == 8 && g.bh == 16)
    return launch_search_nm<8, 16, kTable>(g, pl, fr, npairs, table, recs, ovf, slack, st);
  if (g.bw == 8 && g.bh == 8)
    return launch_search_nm<8, 8, kTable>(g, pl, fr, npairs, table, recs, ovf, slack, st);
  return fail(ACBM_E_UNSUPPORTED, "block size must be 8 or 16 in each direction");
}

template <bool kTable>
static int launch_search(const KGeom& g, const FramePtrs& fr, int npairs, uint32_t* table,
                         BlockRec* recs, uint16_t* ovf, uint32_t slack, hipStream_t st) {
  return launch_search_with<kTable>(g, kTable ? plan_search(g.bw, g.bh, g.p) : plan_fsbm_search(g),
                                    fr, npairs, table, recs, ovf, slack, st);
}

int launch_search_plan(const KGeom& g, const SearchPlan& pl, const uint8_t* const* frames,
                       int npairs, BlockRec* recs, uint16_t* ovf, uint32_t slack,
                       hipStream_t st) {
  if (npairs > kMaxPairsPerLaunch) return fail(ACBM_E_INVAL, "too many pairs for one search");
  FramePtrs fr{};
  for (int k = 0; k <= npairs; ++k) fr.f[k] = frames[k];
  return launch_search_with<false>(g, pl, fr, npairs, nullptr, recs, ovf, slack, st);
}

// Batch kernels ---------------------------------------------------------------
template <int N, int M>
static int launch_search_batch_nm(const SearchPlan& pl, size_t lds, const BatchJob* jobs,
                                  int njobs, uint32_t items, hipStream_t st) {
  const int grid = (int)(((uint64_t)items + 7) / 8 * 8);
  switch (pl.R) {
#define ACBM_CASE(RR)                                                                      \
  case RR: {                                                                               \
    if (lds > 64 * 1024)                                                                   \
      (void)hipFuncSetAttribute((const void*)k_search_batch<N, M, RR>,                     \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);     \
    ProfScope ps("search", st);                                                            \
    hipLaunchKernelGGL((k_search_batch<N, M, RR>), dim3(grid), dim3(pl.threads), lds, st,  \
                       jobs, njobs, items);                                                \
    break;                                                                                 \
  }
    ACBM_R_LIST(ACBM_CASE)
#undef ACBM_CASE
    default:
      return fail(ACBM_E_UNSUPPORTED, "no search kernel for this row blocking");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the batched window search");
}

static int launch_search_batch_tile(const SearchPlan& pl, size_t lds, const BatchJob* jobs,
                                    int njobs, uint32_t items, hipStream_t st) {
  const int grid = (int)(((uint64_t)items + 7) / 8 * 8);
  switch (pl.R) {
#define ACBM_CASE(RR)                                                                        \
  case RR: {                                                                                 \
    if (lds > 64 * 1024)                                                                     \
      (void)hipFuncSetAttribute((const void*)k_search_batch_tile<RR>,                        \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
    ProfScope ps("search", st);                                                              \
    hipLaunchKernelGGL((k_search_batch_tile<RR>), dim3(grid), dim3(pl.threads), lds, st,     \
                       jobs, njobs, items);                                                  \
    break;                                                                                   \
  }
    ACBM_TILE_R_LIST(ACBM_CASE)
#undef ACBM_CASE
    default:
      return fail(ACBM_E_UNSUPPORTED, "no tiled search kernel for this row blocking");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the batched tiled window search");
}

int launch_search_batch(int N, int M, const SearchPlan& pl, size_t lds, const BatchJob* jobs,
                        int njobs, uint32_t items, hipStream_t st) {
  if (!items) return ACBM_OK;
  if (njobs > 64) return fail(ACBM_E_INVAL, "more than 64 jobs in one search group");
  if (pl.tile == 2) {
    if (N != 8 || M != 8) return fail(ACBM_E_INVAL, "tiled search needs 8x8 blocks");
    return launch_search_batch_tile(pl, lds, jobs, njobs, items, st);
  }
  if (N == 16 && M == 16) return launch_search_batch_nm<16, 16>(pl, lds, jobs, njobs, items, st);
  if (N == 16 && M == 8) return launch_search_batch_nm<16, 8>(pl, lds, jobs, njobs, items, st);
  if (N == 8 && M == 16) return launch_search_batch_nm<8, 16>(pl, lds, jobs, njobs, items, st);
  if (N == 8 && M == 8) return launch_search_batch_nm<8, 8>(pl, lds, jobs, njobs, items, st);
  return fail(ACBM_E_UNSUPPORTED, "block size must be 8 or 16 in each direction");
}

// Threads of a batch resolve workgroup.  Alone on the device, 1024, so that
// pairs with few several-winner blocks can take sweeps.  Beside other
// searches (`sized`), four per block row of the tallest frame, so that every
// pair takes the four-lanes-per-block steps (resolve_pair_int4), and no
// more: each wave holds about a quarter of a SIMD's registers, and a
// 1024-thread group leaves its CU no room for search waves.  Such a group
// resolves by steps only.  Frames of more than 256 block rows take 1024
// threads (one per block row of a step).
static int resolve_threads(int max_by, bool sized) {
  if (!sized) return 1024;
  const int t = (4 * max_by + 63) / 64 * 64;
  return t > 1024 ? 1024 : (t < 256 ? 256 : t);
}

int launch_resolve_batch(const BatchJob* jobs, int njobs, uint32_t pair_base, uint32_t pairs,
                         size_t lds, int max_by, bool sized, hipStream_t st) {
  if (!pairs) return ACBM_OK;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_resolve_batch,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  ProfScope ps("resolve", st);
  const int threads = resolve_threads(max_by, sized);
  hipLaunchKernelGGL(k_resolve_batch, dim3(pairs), dim3(threads), lds, st, jobs, njobs, pair_base,
                     threads == 1024);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the batched resolve");
}


int launch_sad_table(const KGeom& g, const uint8_t* cur, const uint8_t* ref, uint32_t* table,
                     hipStream_t st) {
  FramePtrs fr{};
  fr.f[0] = ref;
  fr.f[1] = cur;
  return launch_search<true>(g, fr, 1, table, nullptr, nullptr, 0, st);
}

template <int N, int M>
static int launch_stats_nm(const KGeom& g, const uint8_t* cur, const uint8_t* ref,
                           acbm_block_stats* out, hipStream_t st) {
  const SearchPlan pl = plan_search(g.bw, g.bh, g.p);
  if (!pl.R) return fail(ACBM_E_UNSUPPORTED, "search window does not fit in LDS");
  const WindowShape s = window_shape<N, M>(g.p, pl.R);
  const int grid_x = ((g.nb + 7) / 8) * 8;
  switch (pl.R) {
#define ACBM_CASE(RR)                                                                       \
  case RR: {                                                                                \
    if (pl.lds_bytes > 64 * 1024)                                                           \
      (void)hipFuncSetAttribute((const void*)k_stats<N, M, RR>,                             \
                                hipFuncAttributeMaxDynamicSharedMemorySize, pl.lds_bytes);  \
    ProfScope ps("stats", st);                                                              \
    hipLaunchKernelGGL((k_stats<N, M, RR>), dim3(grid_x), dim3(pl.threads), pl.lds_bytes, st, \
                       g, s, ref, cur, out);                                                \
    break;                                                                                  \
  }
    ACBM_R_LIST(ACBM_CASE)
#undef ACBM_CASE
    default:
      return fail(ACBM_E_UNSUPPORTED, "no search kernel for this row blocking");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the block statistics");
}

int launch_sad_stats(const KGeom& g, const uint8_t* cur, const uint8_t* ref,
                     acbm_block_stats* out, hipStream_t st) {
  if (g.bw == 16 && g.bh == 16) return launch_stats_nm<16, 16>(g, cur, ref, out, st);
  if (g.bw == 16 && g.bh == 8) return launch_stats_nm<16, 8>(g, cur, ref, out, st);
  if (g.bw == 8 && g.bh == 16) return launch_stats_nm<8, 16>(g, cur, ref, out, st);
  if (g.bw == 8 && g.bh == 8) return launch_stats_nm<8, 8>(g, cur, ref, out, st);
  return fail(ACBM_E_UNSUPPORTED, "block size must be 8 or 16 in each direction");
}

static size_t ovf_row_bytes(const KGeom& g) { return ovf_stride(g.p) * sizeof(uint16_t); }

// State of the resolve kernel stays in LDS up to this many bytes (of the
// 160 KiB a workgroup can have on gfx950): up to 36864 blocks, e.g. 8x8
// blocks of 1920x1088 or 16x16 blocks of 3840x2160.
constexpr size_t kResolveLdsMax = 144 * 1024;

size_t fsbm_recs_offset() { return align256(sizeof(WsHeader)); }
size_t fsbm_ovf_entries(int p) { return ovf_stride(p); }

size_t fsbm_ovf_offset(const KGeom& g, uint32_t npairs) {
  return fsbm_recs_offset() + align256((size_t)npairs * g.nb * sizeof(BlockRec));
}
size_t fsbm_mv_offset(const KGeom& g, uint32_t npairs) {
  return fsbm_ovf_offset(g, npairs) + align256((size_t)npairs * g.nb * ovf_row_bytes(g));
}
bool fsbm_mv_in_lds(const KGeom& g) { return (size_t)g.nb * sizeof(uint32_t) <= kResolveLdsMax; }

size_t fsbm_ws_bytes(const KGeom& g, uint32_t npairs) {
  const size_t mv_bytes = (size_t)g.nb * sizeof(uint32_t) > kResolveLdsMax
                              ? align256((size_t)npairs * g.nb * sizeof(uint32_t))
                              : 0;
  return align256(sizeof(WsHeader)) + align256((size_t)npairs * g.nb * sizeof(BlockRec)) +
         align256((size_t)npairs * g.nb * ovf_row_bytes(g)) + mv_bytes;
}

// Pruning slack of the window search: with R >= 2 everywhere and R <= Rmax,
// a candidate can only win when SAD <= SAD_min + lambda*(Rmax - 2).  With
// half-pel precision the integer candidates are priced in half-pel units,
// so Rmax is that of |mvd| <= 4p.
uint32_t fsbm_slack(int p, const acbm_params& prm) {
  const int rmax = prm.subpel ? rate_max(2 * p) : rate_max(p);
  const uint64_t s = (uint64_t)prm.lambda * (uint64_t)(rmax - 2);
  return s > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)s;
}

int launch_half_prep(const KGeom& g, const FramePtrs& fr, int npairs, BlockRec* recs,
                     uint16_t* ovf, hipStream_t st) {
  const size_t items = (size_t)npairs * g.nb;
  const size_t per_group = 4 * (64 / (size_t)g.bh);  // 4 waves, 64 / M blocks per wave
  const dim3 grid((unsigned)((items + per_group - 1) / per_group)), block(256);
  ProfScope ps("half", st);
  if (g.bw == 16 && g.bh == 16)
    hipLaunchKernelGGL((k_half_prep<16, 16>), grid, block, 0, st, g, fr, npairs, recs, ovf);
  else if (g.bw == 16 && g.bh == 8)
    hipLaunchKernelGGL((k_half_prep<16, 8>), grid, block, 0, st, g, fr, npairs, recs, ovf);
  else if (g.bw == 8 && g.bh == 16)
    hipLaunchKernelGGL((k_half_prep<8, 16>), grid, block, 0, st, g, fr, npairs, recs, ovf);
  else if (g.bw == 8 && g.bh == 8)
    hipLaunchKernelGGL((k_half_prep<8, 8>), grid, block, 0, st, g, fr, npairs, recs, ovf);
  else
    return fail(ACBM_E_UNSUPPORTED, "block size must be 8 or 16 in each direction");
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the half-pel preparation");
}

int launch_fsbm(const KGeom& g, const acbm_params& prm, const uint8_t* const* frames,
                uint32_t npairs, void* ws, size_t ws_bytes, acbm_block_result* out,
                hipStream_t st) {
  if (ws_bytes < fsbm_ws_bytes(g, npairs)) return fail(ACBM_E_NOMEM, "workspace too small");
  char* base = static_cast<char*>(ws);
  BlockRec* recs = reinterpret_cast<BlockRec*>(base + align256(sizeof(WsHeader)));
  uint16_t* ovf = reinterpret_cast<uint16_t*>(
      base + align256(sizeof(WsHeader)) + align256((size_t)npairs * g.nb * sizeof(BlockRec)));
  const bool mv_in_lds = (size_t)g.nb * sizeof(uint32_t) <= kResolveLdsMax;
  uint32_t* mv_ws = mv_in_lds ? nullptr
                              : reinterpret_cast<uint32_t*>(
                                    base + align256(sizeof(WsHeader)) +
                                    align256((size_t)npairs * g.nb * sizeof(BlockRec)) +
                                    align256((size_t)npairs * g.nb * ovf_row_bytes(g)));
  const bool hp = prm.subpel != 0;
  const uint32_t slack = fsbm_slack(g.p, prm);
  for (uint32_t p0 = 0; p0 < npairs; p0 += kMaxPairsPerLaunch) {
    const int n = (int)std::min<uint32_t>(kMaxPairsPerLaunch, npairs - p0);
    FramePtrs fr{};
    for (int k = 0; k <= n; ++k) fr.f[k] = frames[p0 + k];
    BlockRec* r = recs + (size_t)p0 * g.nb;
    uint16_t* o = ovf + (size_t)p0 * g.nb * (ovf_row_bytes(g) / 2);
    int rc = launch_search<false>(g, fr, n, nullptr, r, o, slack, st);
    if (rc) return rc;
    if (hp && (rc = launch_half_prep(g, fr, n, r, o, st))) return rc;
    const size_t rlds = mv_in_lds ? (size_t)g.nb * sizeof(uint32_t) : 0;
    const void* fn = hp ? (const void*)k_resolve<true> : (const void*)k_resolve<false>;
    if (rlds > 64 * 1024)
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rlds);
    ProfScope ps("resolve", st);
    if (hp)
      hipLaunchKernelGGL(k_resolve<true>, dim3(n), dim3(1024), rlds, st, g, r, o,
                         out + (size_t)p0 * g.nb, prm.lambda,
                         mv_in_lds ? nullptr : mv_ws + (size_t)p0 * g.nb, fr);
    else
      hipLaunchKernelGGL(k_resolve<false>, dim3(n), dim3(1024), rlds, st, g, r, o,
                         out + (size_t)p0 * g.nb, prm.lambda,
                         mv_in_lds ? nullptr : mv_ws + (size_t)p0 * g.nb, fr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "launching the FSBM resolve");
  }
  return ACBM_OK;
}

}  // namespace acbm
