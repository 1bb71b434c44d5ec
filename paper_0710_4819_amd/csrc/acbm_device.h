// acbm_device.h -- device-side building blocks of libacbm (gfx950).
//
// Shared by the kernels: the rate term, the median predictor, the packed
// minimum key, wave/workgroup reductions and the window search core that
// evaluates SADs with V_QSAD_PK_U16_U8 (four horizontally adjacent candidates
// per instruction, 16 absolute differences).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acbm {

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
// Reductions over a wave64 and over a workgroup.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    uint64_t y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, o, 64));
  return x;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += (uint32_t)__shfl_xor((int)x, o, 64);
  return x;
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
struct WindowShape {
  int p, u_lo;
  int quads;   // QX: quads per window row of candidates
  int groups;  // row groups of R candidate rows
  int rows;    // LDS rows (>= groups*R + M - 1)
  int dws;     // dwords per LDS row (>= quads + N/4)
  int stride;  // LDS row stride in dwords
};

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
  return s;
}

// Cooperative load of the window into LDS (all threads of the group).
template <int N, int M>
__device__ inline void load_window(uint32_t* __restrict__ win, const WindowShape& s,
                                   const uint8_t* __restrict__ ref, int pitch, int width,
                                   int height, int x0, int y0) {
  const int xs = x0 + s.u_lo;  // multiple of 4
  const int total = s.rows * s.dws;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int row = idx / s.dws, dw = idx - row * s.dws;
    const int y = y0 - s.p + row;
    const int x = xs + 4 * dw;
    uint32_t val = 0;
    if (y >= 0 && y < height && x >= 0 && x + 3 < width)
      val = *reinterpret_cast<const uint32_t*>(ref + (size_t)y * pitch + x);
    win[row * s.stride + dw] = val;
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
      cb.d[j][k] = __builtin_amdgcn_readfirstlane(rowp[k]);
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

// Validity of candidate (u, v) for the block at (x0, y0) (frame border and
// |u|, |v| <= p).
__device__ __forceinline__ bool cand_valid(int u, int v, int p, int x0, int y0, int N, int M,
                                           int width, int height) {
  return u >= -p && u <= p && v >= -p && v <= p && x0 + u >= 0 && x0 + u + N <= width &&
         y0 + v >= 0 && y0 + v + M <= height;
}

// Number of valid candidates of a block: product of two interval lengths.
__device__ __forceinline__ uint32_t valid_count(int p, int x0, int y0, int N, int M, int width,
                                                int height) {
  int nu = min(p, width - N - x0) - max(-p, -x0) + 1;
  int nv = min(p, height - M - y0) - max(-p, -y0) + 1;
  return (uint32_t)(max(nu, 0) * max(nv, 0));
}

}  // namespace acbm
