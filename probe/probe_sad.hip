// probe_sad.hip -- semantics and issue rate of the packed SAD instructions on
// the GPU this runs on.
//
// 1. Semantics: V_QSAD_PK_U16_U8, V_SAD_U8 and V_MSAD_U8 on random operands
//    against host models (which byte window each 16-bit lane sums, wrap or
//    clamp of the 16-bit accumulate, which operand V_MSAD_U8 masks).
// 2. Rate: long chains of independent instructions in every lane of a full
//    grid; the time per instruction is compared with V_ALIGNBYTE_B32 (a
//    full-rate op) run the same way, which gives the issue cost independent
//    of the clock.
// 3. Clock: the shader clock while a full grid runs a dependent full-rate
//    chain, from the cycle counter (s_memtime) against the constant-rate
//    wall clock (s_memrealtime), per workgroup, reported as min/median/max.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#define CHECK(x)                                                               \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      std::exit(1);                                                            \
    }                                                                          \
  } while (0)

__global__ void k_semantics(const uint64_t* a, const uint32_t* b, const uint64_t* c, int n,
                            uint64_t* qsad, uint32_t* sad, uint32_t* msad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  qsad[i] = __builtin_amdgcn_qsad_pk_u16_u8(a[i], b[i], c[i]);
  sad[i] = __builtin_amdgcn_sad_u8((uint32_t)a[i], b[i], (uint32_t)c[i]);
  msad[i] = __builtin_amdgcn_msad_u8((uint32_t)a[i], b[i], (uint32_t)c[i]);
}

constexpr int kIters = 2048;

__global__ void __launch_bounds__(256) k_rate_qsad(uint64_t* out, uint32_t seed) {
  uint64_t acc[8];
  uint64_t x = 0x0102030405060708ull * (threadIdx.x + seed);
  uint32_t y = 0x11223344u ^ (threadIdx.x * 7919u);
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = k;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_qsad_pk_u16_u8(x, y + k, acc[k]);
  }
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s ^= acc[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_rate_sad(uint32_t* out, uint32_t seed) {
  uint32_t acc[8];
  uint32_t x = 0x01020304u * (threadIdx.x + seed);
  uint32_t y = 0x11223344u ^ (threadIdx.x * 7919u);
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = k;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_sad_u8(x, y + k, acc[k]);
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s ^= acc[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_rate_add(uint32_t* out, uint32_t seed) {
  uint32_t acc[8];
  uint32_t y = 0x11223344u ^ (threadIdx.x * 7919u) ^ seed;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = k;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      // one V_ALIGNBYTE_B32 per step; the shift makes the chain impossible to fold
      acc[k] = __builtin_amdgcn_alignbyte(acc[k], y + k, 1u);
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s ^= acc[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Thread 0 of every workgroup stamps both counters around a dependent chain
// of full-rate ops; stamps[4*b .. 4*b+3] = cycles0, wall0, cycles1, wall1.
__global__ void __launch_bounds__(256) k_clock(uint64_t* stamps, uint32_t* sink, uint32_t seed) {
  __syncthreads();
  uint64_t c0 = 0, w0 = 0;
  if (threadIdx.x == 0) {
    c0 = clock64();
    w0 = wall_clock64();
  }
  uint32_t acc = threadIdx.x ^ seed;
  for (int it = 0; it < 64 * kIters; ++it) acc = __builtin_amdgcn_alignbyte(acc, acc + it, 1u);
  sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t c1 = clock64(), w1 = wall_clock64();
    stamps[4 * blockIdx.x + 0] = c0;
    stamps[4 * blockIdx.x + 1] = w0;
    stamps[4 * blockIdx.x + 2] = c1;
    stamps[4 * blockIdx.x + 3] = w1;
  }
}

static uint64_t model_qsad(uint64_t a, uint32_t b, uint64_t c, bool clamp) {
  uint64_t d = 0;
  for (int i = 0; i < 4; ++i) {
    uint32_t s = 0;
    for (int k = 0; k < 4; ++k) {
      int x = (int)((a >> (8 * (i + k))) & 0xFF), y = (int)((b >> (8 * k)) & 0xFF);
      s += (uint32_t)std::abs(x - y);
    }
    uint32_t acc = (uint32_t)((c >> (16 * i)) & 0xFFFF) + s;
    if (clamp && acc > 0xFFFF) acc = 0xFFFF;
    d |= (uint64_t)(acc & 0xFFFF) << (16 * i);
  }
  return d;
}

static uint32_t model_sad(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t s = c;
  for (int k = 0; k < 4; ++k)
    s += (uint32_t)std::abs((int)((a >> (8 * k)) & 0xFF) - (int)((b >> (8 * k)) & 0xFF));
  return s;
}

static uint32_t model_msad(uint32_t a, uint32_t b, uint32_t c, int masked_operand) {
  uint32_t s = c;
  for (int k = 0; k < 4; ++k) {
    int x = (int)((a >> (8 * k)) & 0xFF), y = (int)((b >> (8 * k)) & 0xFF);
    int m = masked_operand == 0 ? x : y;
    if (m != 0) s += (uint32_t)std::abs(x - y);
  }
  return s;
}

template <typename K, typename T>
static double time_kernel(K kern, T* out, int grid, int reps) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, 0, out, 1u);  // warm-up
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0, 0));
  for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, 0, out, (uint32_t)r);
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  return ms / reps;
}

int main() {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  std::printf("device %s, %d CUs, clock %d kHz\n", prop.gcnArchName, prop.multiProcessorCount,
              prop.clockRate);

  // ---- semantics ----
  const int n = 1 << 16;
  std::mt19937_64 rng(12345);
  std::vector<uint64_t> a(n), c(n), q(n);
  std::vector<uint32_t> b(n), s(n), m(n);
  for (int i = 0; i < n; ++i) {
    a[i] = rng();
    b[i] = (uint32_t)rng();
    c[i] = rng();
    if (i % 4 == 0) {  // zero bytes to exercise the mask of V_MSAD_U8
      a[i] &= 0xFFFFFFFF00FF00FFull;
      b[i] &= 0xFF00FF00u;
    }
    if (i % 8 == 1) c[i] |= 0xFFF0FFF0FFF0FFF0ull;  // accumulate near 0xFFFF
  }
  uint64_t *da, *dc, *dq;
  uint32_t *db, *ds, *dm;
  CHECK(hipMalloc(&da, n * 8));
  CHECK(hipMalloc(&dc, n * 8));
  CHECK(hipMalloc(&dq, n * 8));
  CHECK(hipMalloc(&db, n * 4));
  CHECK(hipMalloc(&ds, n * 4));
  CHECK(hipMalloc(&dm, n * 4));
  CHECK(hipMemcpy(da, a.data(), n * 8, hipMemcpyHostToDevice));
  CHECK(hipMemcpy(dc, c.data(), n * 8, hipMemcpyHostToDevice));
  CHECK(hipMemcpy(db, b.data(), n * 4, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_semantics, dim3(n / 256), dim3(256), 0, 0, da, db, dc, n, dq, ds, dm);
  CHECK(hipDeviceSynchronize());
  CHECK(hipMemcpy(q.data(), dq, n * 8, hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(s.data(), ds, n * 4, hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(m.data(), dm, n * 4, hipMemcpyDeviceToHost));
  int q_wrap = 0, q_clamp = 0, sad_ok = 0, msad0 = 0, msad1 = 0, msad_plain = 0;
  for (int i = 0; i < n; ++i) {
    q_wrap += q[i] == model_qsad(a[i], b[i], c[i], false);
    q_clamp += q[i] == model_qsad(a[i], b[i], c[i], true);
    sad_ok += s[i] == model_sad((uint32_t)a[i], b[i], (uint32_t)c[i]);
    msad0 += m[i] == model_msad((uint32_t)a[i], b[i], (uint32_t)c[i], 0);
    msad1 += m[i] == model_msad((uint32_t)a[i], b[i], (uint32_t)c[i], 1);
    msad_plain += m[i] == model_sad((uint32_t)a[i], b[i], (uint32_t)c[i]);
  }
  std::printf("semantics over %d operands:\n", n);
  std::printf("  qsad = sum_k |src0.byte[i+k] - src1.byte[k]| + src2.u16[i], 16-bit wrap : %d\n", q_wrap);
  std::printf("  qsad = same with the 16-bit accumulate clamped at 0xFFFF             : %d\n", q_clamp);
  std::printf("  sad_u8 = sum_k |src0.byte[k] - src1.byte[k]| + src2                 : %d\n", sad_ok);
  std::printf("  msad_u8 skipping bytes where src0 is 0 / src1 is 0 / never          : %d / %d / %d\n",
              msad0, msad1, msad_plain);

  // ---- rate ----
  const int grid = prop.multiProcessorCount * 32;  // 8 waves per SIMD
  const int reps = 20;
  void* out;
  CHECK(hipMalloc(&out, (size_t)grid * 256 * 8));
  double t_add = time_kernel(k_rate_add, (uint32_t*)out, grid, reps);
  double t_sad = time_kernel(k_rate_sad, (uint32_t*)out, grid, reps);
  double t_qsad = time_kernel(k_rate_qsad, (uint64_t*)out, grid, reps);
  const double ops = (double)grid * 256 * kIters * 8;  // lane-ops of the timed instruction
  std::printf("rate (%d workgroups x 256 lanes x %d x 8 ops):\n", grid, kIters);
  std::printf("  v_alignbyte_b32   %.3f ms  %.2f T lane-ops/s\n", t_add, ops / t_add / 1e9);
  std::printf("  v_sad_u8          %.3f ms  %.2f T lane-ops/s  %.1f T byte-diffs/s\n", t_sad,
              ops / t_sad / 1e9, 4 * ops / t_sad / 1e9);
  std::printf("  v_qsad_pk_u16_u8  %.3f ms  %.2f T lane-ops/s  %.1f T byte-diffs/s\n", t_qsad,
              ops / t_qsad / 1e9, 16 * ops / t_qsad / 1e9);
  std::printf("  issue cost relative to a full-rate op: sad_u8 %.2f, qsad %.2f\n",
              t_sad / t_add, t_qsad / t_add);

  // ---- clock ----
  int wall_khz = 0;
  CHECK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, 0));
  uint64_t* dstamps;
  CHECK(hipMalloc(&dstamps, (size_t)grid * 4 * 8));
  hipLaunchKernelGGL(k_clock, dim3(grid), dim3(256), 0, 0, dstamps, (uint32_t*)out, 1u);
  CHECK(hipDeviceSynchronize());
  hipLaunchKernelGGL(k_clock, dim3(grid), dim3(256), 0, 0, dstamps, (uint32_t*)out, 2u);
  CHECK(hipDeviceSynchronize());
  std::vector<uint64_t> st((size_t)grid * 4);
  CHECK(hipMemcpy(st.data(), dstamps, st.size() * 8, hipMemcpyDeviceToHost));
  std::vector<double> mhz;
  for (int b = 0; b < grid; ++b) {
    double cyc = (double)(st[4 * b + 2] - st[4 * b + 0]);
    double wall = (double)(st[4 * b + 3] - st[4 * b + 1]);
    if (wall > 0) mhz.push_back(cyc / wall * wall_khz / 1e3);
  }
  std::sort(mhz.begin(), mhz.end());
  if (!mhz.empty())
    std::printf("clock (cycle counter / %d kHz wall clock, %zu workgroups): min %.0f, median %.0f, "
                "max %.0f MHz\n", wall_khz, mhz.size(), mhz.front(), mhz[mhz.size() / 2],
                mhz.back());
  return 0;
}
