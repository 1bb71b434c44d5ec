// acbm_device.h -- device-side building blocks of libacbm (gfx950).
//
// Shared by the kernels: the rate term, the median predictor, the packed
// minimum key, wave/workgroup reductions and the window search core that
// evaluates SADs with V_QSAD_PK_U16_U8 (four horizontally adjacent candidates
// per instruction, 16 absolute differences).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "acbm_internal.h"

namespace acbm {

// Loads through pointers that were themselves read from memory (frame tables,
// job descriptors) compile to FLAT instructions, which also count against the
// LDS counter: every barrier would then wait for them.  Frames and results
// always live in global memory, so these accessors say so.
template <typename T>
__device__ __forceinline__ T ld_global(const void* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void st_global(void* p, const T& v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 ld_global_x4(const void* p) {
  return *(const __attribute__((address_space(1))) u32x4*)p;
}

// One block's result as two 16-byte global stores: mv (x in the low, y in
// the high half), sad, j, rate_bits | cands, mode, intra_x (u64 at byte 24).
static_assert(sizeof(acbm_block_result) == 32, "result layout");
static_assert(offsetof(acbm_block_result, intra_x) == 24, "result layout");
__device__ __forceinline__ void put_result(acbm_block_result* out, int u, int v, uint32_t sad,
                                           uint32_t j, uint32_t rate, uint32_t cands,
                                           uint32_t mode, uint32_t intra) {
  typedef __attribute__((address_space(1))) u32x4 gu32x4;
  gu32x4* o = (gu32x4*)out;
  o[0] = u32x4{((uint32_t)v << 16) | ((uint32_t)u & 0xFFFFu), sad, j, rate};
  o[1] = u32x4{cands, mode, intra, 0u};
}

// ---------------------------------------------------------------------------
// Rate term (Section 2.1, vectors sent differentially, Section 2.2): bits of
// the signed Exp-Golomb codeword of k: 1 for k = 0, 2*floor(log2|k|) + 3
// otherwise.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t se_bits(int k) {
  uint32_t a = (uint32_t)(k < 0 ? -k : k);
  return a == 0 ? 1u : 2u * (31u - (uint32_t)__builtin_clz(a)) + 3u;
}

__device__ __forceinline__ int med3(int a, int b, int c) {
  return max(min(a, b), min(max(a, b), c));
}

// Motion vectors travel between blocks packed in 16 bits (|mv| <= 127 fits a
// signed byte per component); 0x8080 (-128, -128) marks "not decided yet".
constexpr uint16_t kMvUnset = 0x8080u;
__device__ __forceinline__ uint16_t pack_mv(int x, int y) {
  return (uint16_t)((uint32_t)(x & 0xFF) | ((uint32_t)(y & 0xFF) << 8));
}
__device__ __forceinline__ int mv_x(uint16_t m) { return (int)(int8_t)(m & 0xFF); }
__device__ __forceinline__ int mv_y(uint16_t m) { return (int)(int8_t)(m >> 8); }

// Total order of candidates: J, then |u|+|v|, then window raster index.
// J < 2^32, |u|+|v| <= 254, raster < 2^16.
__device__ __forceinline__ uint64_t make_key(uint32_t j, int u, int v, int p) {
  uint32_t l1 = (uint32_t)(abs(u) + abs(v));
  uint32_t ras = (uint32_t)((v + p) * (2 * p + 1) + (u + p));
  return ((uint64_t)j << 32) | ((uint64_t)l1 << 16) | ras;
}

// ---------------------------------------------------------------------------
// Reductions over a wave64 (the ROCm device library's DPP reductions; every
// lane of the wave must be active) and over a workgroup.
// ---------------------------------------------------------------------------
}  // namespace acbm
extern "C" __device__ uint64_t __ockl_wfred_min_u64(uint64_t);
extern "C" __device__ uint32_t __ockl_wfred_min_u32(uint32_t);
extern "C" __device__ uint32_t __ockl_wfred_add_u32(uint32_t);
extern "C" __device__ uint32_t __ockl_wfred_max_u32(uint32_t);
namespace acbm {

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) { return __ockl_wfred_min_u64(x); }
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) { return __ockl_wfred_min_u32(x); }
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) { return __ockl_wfred_add_u32(x); }

// Minimum of the four 16-bit lanes of each of R accumulators.
typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));
template <int R>
__device__ __forceinline__ uint32_t min_u16_lanes(const uint64_t (&acc)[R]) {
  ushort2_t m = __builtin_bit_cast(ushort2_t, (uint32_t)acc[0]);
  m = __builtin_elementwise_min(m, __builtin_bit_cast(ushort2_t, (uint32_t)(acc[0] >> 32)));
#pragma unroll
  for (int rr = 1; rr < R; ++rr) {
    m = __builtin_elementwise_min(m, __builtin_bit_cast(ushort2_t, (uint32_t)acc[rr]));
    m = __builtin_elementwise_min(m, __builtin_bit_cast(ushort2_t, (uint32_t)(acc[rr] >> 32)));
  }
  return min((uint32_t)m.x, (uint32_t)m.y);
}

// Valid candidate range of a block: u in [u_min, u_max], v in [v_min, v_max]
// (|u|, |v| <= p and the displaced block inside the frame).
struct ValidBox {
  int u_min, u_max, v_min, v_max;
};
__device__ __forceinline__ ValidBox valid_box(int p, int x0, int y0, int N, int M, int width,
                                              int height) {
  ValidBox b;
  b.u_min = max(-p, -x0);
  b.u_max = min(p, width - N - x0);
  b.v_min = max(-p, -y0);
  b.v_max = min(p, height - M - y0);
  return b;
}

// Sets the 16-bit lane of every invalid candidate of a task to 0xFFFF (no
// valid SAD reaches it: 255 * 256 = 65280).  Lane i of acc[rr] is candidate
// (u0 + i, v0 + rr).
// For a block whose whole window is valid only the padding is invalid: the
// columns of the first and last quads outside [-p, p] (u_lo = -4*ceil(p/4)
// may lie below -p) and the last row group's rows beyond +p.
template <int R>
__device__ __forceinline__ void mask_padding(uint64_t (&acc)[R], int p, int u0, int v0) {
  uint64_t colmask = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (u0 + i < -p || u0 + i > p) colmask |= 0xFFFFull << (16 * i);
#pragma unroll
  for (int rr = 0; rr < R; ++rr) acc[rr] |= (v0 + rr > p) ? ~0ull : colmask;
}

template <int R>
__device__ __forceinline__ void mask_invalid(uint64_t (&acc)[R], const ValidBox& bx, int u0,
                                             int v0) {
  uint64_t colmask = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (u0 + i < bx.u_min || u0 + i > bx.u_max) colmask |= 0xFFFFull << (16 * i);
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    const int v = v0 + rr;
    acc[rr] |= (v < bx.v_min || v > bx.v_max) ? ~0ull : colmask;
  }
}

// Workgroup minimum of a 32-bit value (`scratch`: one slot per wave).
__device__ __forceinline__ uint32_t group_min_u32(uint32_t x, uint32_t* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  x = wave_min_u32(x);
  if (lane == 0) scratch[wave] = x;
  __syncthreads();
  uint32_t m = scratch[0];
  for (int w = 1; w < nw; ++w) m = scratch[w] < m ? scratch[w] : m;
  __syncthreads();
  return m;
}

// Workgroup minimum; `scratch` holds one slot per wave.  Every thread gets
// the result.  Contains barriers: all threads of the group must call it.
__device__ __forceinline__ uint64_t group_min_u64(uint64_t x, uint64_t* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  x = wave_min_u64(x);
  if (lane == 0) scratch[wave] = x;
  __syncthreads();
  uint64_t m = scratch[0];
  for (int w = 1; w < nw; ++w) m = scratch[w] < m ? scratch[w] : m;
  __syncthreads();
  return m;
}

// ---------------------------------------------------------------------------
// Search window staged in LDS.
//
// For block (r, c) at (x0, y0) the window holds reference rows
// y0 - p ... y0 - p + rows - 1 and reference columns starting at
// xs = x0 + u_lo, u_lo = -4*ceil(p/4) (so xs is dword aligned), `dws`
// dwords per row.  Lane work unit ("task") = one quad of candidates
// u = u_lo + 4q .. u_lo + 4q + 3 times R consecutive rows
// v = -p + R*g ... -p + R*g + R - 1.  Bytes outside the frame read as 0; the
// candidates that touch them are invalid and masked afterwards.
// ---------------------------------------------------------------------------
template <int N, int M>
__host__ __device__ inline WindowShape window_shape(int p, int R) {
  WindowShape s;
  s.p = p;
  s.u_lo = -4 * ((p + 3) / 4);
  s.quads = (p - s.u_lo + 1 + 3) / 4;
  s.groups = (2 * p + 1 + R - 1) / R;
  s.rows = s.groups * R + M - 1;
  s.dws = s.quads + N / 4;
  s.stride = s.dws | 1;  // odd stride spreads row starts over the LDS banks
  s.qmagic = (uint32_t)(((1ull << 32) + (uint64_t)s.quads - 1) / (uint64_t)s.quads);
  s.dmagic = (uint32_t)(((1ull << 32) + (uint64_t)s.dws - 1) / (uint64_t)s.dws);
  const int iq = s.quads - (s.u_lo < -p ? 1 : 0) - (s.u_lo + 4 * s.quads - 1 > p ? 1 : 0);
  s.imagic = iq > 1 ? (uint32_t)(((1ull << 32) + (uint64_t)iq - 1) / (uint64_t)iq) : 0u;
  return s;
}

// Lane t's task of a window search: quad q, row group gi.  The tasks that
// hold padding candidates (a first quad reaching below -p, a last quad
// beyond +p, a last row group beyond +p; `edge`) take the highest lane
// numbers, after the interior tasks in row-group-major order: for a block
// whose whole window is valid only the waves holding edge tasks mask
// anything.  Every interior candidate has |u|, |v| <= p.
template <int R>
__device__ __forceinline__ void task_of(const WindowShape& s, int t, int* q, int* gi,
                                        bool* edge) {
  const int p = s.p;
  const int q_lo = s.u_lo < -p ? 1 : 0;
  const int q_hi = s.u_lo + 4 * s.quads - 1 > p ? 1 : 0;
  const int g_hi = s.groups * R > 2 * p + 1 ? 1 : 0;
  const int iq = s.quads - q_lo - q_hi;
  const int interior = iq * (s.groups - g_hi);
  if (t < interior) {
    // t / iq (the magic of iq = 1 would be 2^32, which a u32 cannot hold)
    const int g = iq == 1 ? t : (int)__umulhi((uint32_t)t, s.imagic);
    *gi = g;
    *q = q_lo + (t - g * iq);
    *edge = false;
    return;
  }
  const int e = t - interior, ncol = q_lo + q_hi;
  *edge = true;
  if (e < ncol * s.groups) {  // the padding quads, over every row group
    const int c = ncol == 2 ? (e & 1) : 0;
    *gi = ncol == 2 ? (e >> 1) : e;
    *q = (c == 0 && q_lo) ? 0 : s.quads - 1;
  } else {  // the padding row group's interior quads
    *gi = s.groups - 1;
    *q = q_lo + (e - ncol * s.groups);
  }
}

// Cooperative load of the window into LDS (all threads of the group).  The
// group covers `per` = blockDim / dws whole rows at a time: each thread owns
// one dword column and walks down it `per` rows per step, so the addresses
// advance by constants; the threads beyond per * dws (fewer than dws) cover
// the rows left over.  A window inside the frame (the common case, decided
// once per block) skips the per-dword bounds test.
template <int N, int M>
__device__ inline void load_window(uint32_t* __restrict__ win, const WindowShape& s,
                                   const uint8_t* __restrict__ ref, int pitch, int width,
                                   int height, int x0, int y0) {
  const int xs = x0 + s.u_lo;  // multiple of 4
  const int ys = y0 - s.p;
  const int per = (int)blockDim.x / s.dws;  // >= 1: the plan gives every row a thread
  const int r0 = (int)__umulhi(threadIdx.x, s.dmagic);
  const int dw = (int)threadIdx.x - r0 * s.dws;
  const int main_rows = s.rows - s.rows % per;  // rows covered in whole steps
  const bool inside = xs >= 0 && xs + 4 * s.dws <= width && ys >= 0 && ys + s.rows <= height;
  if (inside) {
    const uint8_t* base = ref + (size_t)ys * pitch + xs + 4 * dw;
    if (r0 < per) {
#pragma unroll 4
      for (int row = r0; row < main_rows; row += per)
        win[row * s.stride + dw] = ld_global<uint32_t>(base + (size_t)row * pitch);
    }
    // the last rows % per rows: one per group of dws threads
    const int row = main_rows + r0;
    if (r0 < per && row < s.rows)
      win[row * s.stride + dw] = ld_global<uint32_t>(base + (size_t)row * pitch);
  } else {
    const int x = xs + 4 * dw;
    const bool xok = x >= 0 && x + 3 < width;
    for (int row = r0; r0 < per && row < s.rows; row += per) {
      const int y = ys + row;
      uint32_t val = 0;
      if (xok && y >= 0 && y < height)
        val = ld_global<uint32_t>(ref + (size_t)y * pitch + x);
      win[row * s.stride + dw] = val;
    }
  }
}

// The current block as M x N/4 little-endian dwords, loaded with a
// wave-uniform address so that it lands in scalar registers.
template <int N, int M>
struct CurBlock {
  uint32_t d[M][N / 4];
};

template <int N, int M>
__device__ __forceinline__ void load_cur_uniform(CurBlock<N, M>& cb,
                                                 const uint8_t* __restrict__ cur, int pitch,
                                                 int x0, int y0) {
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const uint32_t* rowp =
        reinterpret_cast<const uint32_t*>(cur + (size_t)(y0 + j) * pitch + x0);
#pragma unroll
    for (int k = 0; k < N / 4; ++k)
      cb.d[j][k] = __builtin_amdgcn_readfirstlane(ld_global<uint32_t>(rowp + k));
  }
}

// SADs of one task: acc[rr] holds four u16 SADs (candidates u_lo + 4q + i,
// i = 0..3, in 16-bit lanes) for candidate row v = -p + R*g + rr.  A u16
// cannot overflow: a SAD is at most 255 * N * M <= 65280.
template <int N, int M, int R>
__device__ __forceinline__ void task_sads(const uint32_t* __restrict__ win, int stride, int q,
                                          int g, const CurBlock<N, M>& cb, uint64_t (&acc)[R]) {
#pragma unroll
  for (int rr = 0; rr < R; ++rr) acc[rr] = 0;
  const uint32_t* base = win + (R * g) * stride + q;
#pragma unroll
  for (int w = 0; w < R + M - 1; ++w) {
    const uint32_t* rowp = base + w * stride;
    uint64_t qw[N / 4];
#pragma unroll
    for (int k = 0; k < N / 4; ++k)
      qw[k] = (uint64_t)rowp[k] | ((uint64_t)rowp[k + 1] << 32);
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int j = w - rr;
      if (j >= 0 && j < M) {
#pragma unroll
        for (int k = 0; k < N / 4; ++k)
          acc[rr] = __builtin_amdgcn_qsad_pk_u16_u8(qw[k], cb.d[j][k], acc[rr]);
      }
    }
  }
}

// The same task over a 16x16 tile of four 8x8 blocks: acc[b][rr] holds the
// SADs of block b (b = 2 * (row >= 8) + (column >= 8) within the tile).  A
// block's SAD at a displacement is one quadrant of the tile's, so the four
// blocks cost the QSADs of one 16x16 task.
template <int R>
__device__ __forceinline__ void task_sads_tile(const uint32_t* __restrict__ win, int stride,
                                               int q, int g, const CurBlock<16, 16>& cb,
                                               uint64_t (&acc)[4][R]) {
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int rr = 0; rr < R; ++rr) acc[b][rr] = 0;
  const uint32_t* base = win + (R * g) * stride + q;
#pragma unroll
  for (int w = 0; w < R + 15; ++w) {
    const uint32_t* rowp = base + w * stride;
    uint64_t qw[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) qw[k] = (uint64_t)rowp[k] | ((uint64_t)rowp[k + 1] << 32);
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int j = w - rr;
      if (j >= 0 && j < 16) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int b = 2 * (j >> 3) + (k >> 1);
          acc[b][rr] = __builtin_amdgcn_qsad_pk_u16_u8(qw[k], cb.d[j][k], acc[b][rr]);
        }
      }
    }
  }
}

// Validity of candidate (u, v) for the block at (x0, y0) (frame border and
// |u|, |v| <= p).
__device__ __forceinline__ bool cand_valid(int u, int v, int p, int x0, int y0, int N, int M,
                                           int width, int height) {
  return u >= -p && u <= p && v >= -p && v <= p && x0 + u >= 0 && x0 + u + N <= width &&
         y0 + v >= 0 && y0 + v + M <= height;
}

// ---------------------------------------------------------------------------
// Half-pel precision.  A half-pel vector (U, V) counts half pixels.  Pixel
// (i, j) of the block at (x0, y0) is compared with the reference's H.263
// bilinear sample at (2(x0+i) + U, 2(y0+j) + V): writing that position as
// (2x + fx, 2y + fy) and A, B, C, D for ref(x, y), ref(x+1, y), ref(x, y+1),
// ref(x+1, y+1), the sample is A, (A+B+1)/2, (A+C+1)/2 or (A+B+C+D+2)/4 for
// (fx, fy) = (0,0), (1,0), (0,1), (1,1).  All four cases are
// (A + B' + C' + D' + 2) / 4 with B' = fx ? B : A, C' = fy ? C : A and
// D' the pixel at (x + fx, y + fy), which the kernels use branch-free.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool cand_valid_half(int U, int V, int p, int x0, int y0, int N,
                                                int M, int width, int height) {
  const int xl = x0 + (U >> 1), yl = y0 + (V >> 1);  // arithmetic shifts: floor(U / 2)
  return U >= -2 * p && U <= 2 * p && V >= -2 * p && V <= 2 * p && xl >= 0 &&
         xl + N + (U & 1) <= width && yl >= 0 && yl + M + (V & 1) <= height;
}

// Per byte (a + b + c + d + 2) >> 2 of four packed u8 words, in two 16-bit
// lanes per half (4 * 255 + 2 < 2^16, so no lane carries into the next).
__device__ __forceinline__ uint32_t avg4_u8(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const uint32_t m = 0x00FF00FFu;
  const uint32_t lo = (a & m) + (b & m) + (c & m) + (d & m) + 0x00020002u;
  const uint32_t hi =
      ((a >> 8) & m) + ((b >> 8) & m) + ((c >> 8) & m) + ((d >> 8) & m) + 0x00020002u;
  return ((lo >> 2) & m) | (((hi >> 2) & m) << 8);
}

// Bytes sh .. sh+3 of the 8-byte value lo:hi (sh = 0..4).
__device__ __forceinline__ uint32_t bytes_at(uint32_t lo, uint32_t hi, uint32_t sh) {
  return sh >= 4 ? hi : __builtin_amdgcn_alignbyte(hi, lo, sh);
}

// SAD of one block row against half-pel samples.  d0 and d1 are NC+1 dwords
// of reference rows y and y+1 starting at the dword that holds byte x (sh =
// x & 3); c the NC dwords of the current row.
template <int NC>
__device__ __forceinline__ uint32_t half_row_sad(const uint32_t (&d0)[NC + 1],
                                                 const uint32_t (&d1)[NC + 1], uint32_t sh,
                                                 int fx, int fy, const uint32_t (&c)[NC],
                                                 uint32_t acc) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const uint32_t a = bytes_at(d0[k], d0[k + 1], sh);
    const uint32_t b = bytes_at(d0[k], d0[k + 1], sh + 1);
    const uint32_t cc = bytes_at(d1[k], d1[k + 1], sh);
    const uint32_t dd = bytes_at(d1[k], d1[k + 1], sh + 1);
    const uint32_t B = fx ? b : a, C = fy ? cc : a, D = fx ? (fy ? dd : b) : (fy ? cc : a);
    acc = __builtin_amdgcn_sad_u8(avg4_u8(a, B, C, D), c[k], acc);
  }
  return acc;
}

// Sum over aligned groups of G = 8 or 16 lanes, left in every lane of the
// group: swaps within quads, then the mirror within 8 lanes, then (G = 16)
// the mirror within 16 lanes.
template <int G>
__device__ __forceinline__ uint32_t group_sum(uint32_t x) {
  static_assert(G == 8 || G == 16, "row sums of 8 or 16 lanes");
  x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false);  // row_half_mirror
  if constexpr (G == 16)
    x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, false);  // row_mirror
  return x;
}

// The 8 half-pel neighbours of an integer vector, numbered k = 0..7 in
// raster order of the 3 x 3 ring without its centre.
__device__ __forceinline__ void half_ring_offset(int k, int* du, int* dv) {
  const int dd = k < 4 ? k : k + 1;
  *du = dd % 3 - 1;
  *dv = dd / 3 - 1;
}

// SADs of the 8 half-pel neighbours of (U0, V0) (even: an integer vector)
// for the block at (x0, y0), by one whole wave from the frames in global
// memory; 0xFFFF for a neighbour that is not a valid candidate.  Lane item
// (neighbour, block row); the M lanes of one neighbour are adjacent, so the
// row sum is a DPP group sum.  Every lane returns the same values.
template <int N, int M>
__device__ __forceinline__ void wave_half_sads(const KGeom& g, const uint8_t* __restrict__ cur,
                                               const uint8_t* __restrict__ ref, int x0, int y0,
                                               int U0, int V0, uint32_t (&sads)[8]) {
  constexpr int NC = N / 4;
  constexpr int PER = 64 / M;  // neighbours per pass
  const int lane = threadIdx.x & 63;
  const int j = lane % M;
  const int last_dw = (g.pitch >> 2) - 1;  // last dword of a row
#pragma unroll
  for (int pass = 0; pass < 8 / PER; ++pass) {
    const int k = pass * PER + lane / M;
    int du, dv;
    half_ring_offset(k, &du, &dv);
    const int U = U0 + du, V = V0 + dv;
    const bool ok = cand_valid_half(U, V, g.p, x0, y0, N, M, g.width, g.height);
    uint32_t acc = 0;
    if (ok) {
      const int x = x0 + (U >> 1), y = y0 + j + (V >> 1);
      const int fx = U & 1, fy = V & 1;
      const uint32_t* r0 = reinterpret_cast<const uint32_t*>(ref + (size_t)y * g.pitch);
      const uint32_t* r1 = fy ? r0 + (g.pitch >> 2) : r0;
      const uint32_t* cr = reinterpret_cast<const uint32_t*>(cur + (size_t)(y0 + j) * g.pitch + x0);
      uint32_t d0[NC + 1], d1[NC + 1], c[NC];
#pragma unroll
      for (int q = 0; q <= NC; ++q) {
        // dwords past the row's end only feed bytes beyond x + N, which no
        // sample uses; the index is clamped so that nothing is read there
        const int at = min((x >> 2) + q, last_dw);
        d0[q] = r0[at];
        d1[q] = r1[at];
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) c[q] = cr[q];
      acc = half_row_sad<NC>(d0, d1, (uint32_t)(x & 3), fx, fy, c, 0u);
    }
    acc = group_sum<M>(acc);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int kk = pass * PER + q;
      int eu, ev;
      half_ring_offset(kk, &eu, &ev);
      const bool okk = cand_valid_half(U0 + eu, V0 + ev, g.p, x0, y0, N, M, g.width, g.height);
      const uint32_t s = __builtin_amdgcn_readlane(acc, q * M);
      sads[kk] = okk ? s : 0xFFFFu;
    }
  }
}

// Number of valid candidates of a block: product of two interval lengths.
__device__ __forceinline__ uint32_t valid_count(int p, int x0, int y0, int N, int M, int width,
                                                int height) {
  int nu = min(p, width - N - x0) - max(-p, -x0) + 1;
  int nv = min(p, height - M - y0) - max(-p, -y0) + 1;
  return (uint32_t)(max(nu, 0) * max(nv, 0));
}

}  // namespace acbm
