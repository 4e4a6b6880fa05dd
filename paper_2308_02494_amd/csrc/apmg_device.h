// Device-side building blocks of the APMGSRN kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace apmg {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef float f32x2a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32x2a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32x4a8 __attribute__((ext_vector_type(4), aligned(8)));

constexpr int kWave = 64;
constexpr int kBlock = 256;   // threads per workgroup in the tile kernels
// third dword of a raw buffer resource (untyped 32-bit accesses) on gfx950
constexpr int kBufferRsrcWord3 = 0x00020000;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr float kSMax = 87.0f;  // exp(-s) is taken as 0 above this (float32 range)

// ------------------------------------------------------------ bf16
// float -> bf16, round to nearest even (NaN stays NaN): gfx950's v_cvt_pk_bf16_f32, which
// converts two values per instruction.
typedef __bf16 bf16x2n __attribute__((ext_vector_type(2)));
typedef float f32x2n __attribute__((ext_vector_type(2)));
__device__ inline uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline uint32_t bf16_pack2(float a, float b) {
  const f32x2n x = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2n));   // a in the low half
}
__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// Eight floats as an MFMA bf16 operand (element e in bits 16(e%2).. of word e/2).
__device__ inline bf16x8 bf16_pack8(const float v[8]) {
  typedef uint32_t u32x4n __attribute__((ext_vector_type(4)));
  const u32x4n w = {bf16_pack2(v[0], v[1]), bf16_pack2(v[2], v[3]), bf16_pack2(v[4], v[5]), bf16_pack2(v[6], v[7])};
  return __builtin_bit_cast(bf16x8, w);
}

// ------------------------------------------------------------ MFMA wrappers
// v_mfma_f32_32x32x2_f32: A[i][k] in lane i + 32k, B[k][j] in lane j + 32k,
// D[i][j] in lane j + 32*((i/4)%2), register 4*(i/8) + i%4.
__device__ inline f32x16 mma_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
// v_mfma_f32_32x32x16_bf16: lane l holds A[l%32][8(l/32)+e] and B[8(l/32)+e][l%32].
__device__ inline f32x16 mma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Keeps the scheduler from hoisting loads across this point (bounds the number of
// operand loads kept in flight, and with it register pressure).
__device__ inline void sched_fence() { asm volatile("" ::: "memory"); }
// Machine-scheduler barrier: no instruction moves across it.
__device__ inline void sched_barrier() { __builtin_amdgcn_sched_barrier(0); }

// Row of a 32x32 accumulator block held in register r by lane half hf.
__host__ __device__ inline int acc_row(int r, int hf) { return 8 * (r >> 2) + 4 * hf + (r & 3); }

// ------------------------------------------------------------ cross-lane sums
// Sum over the 32 lanes of each wave half (lanes with equal lane/32).
__device__ inline float half_sum(float v) {
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double half_sum(double v) {
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------ Philox4x64-10
__device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  lo = a * b;
  hi = __umul64hi(a, b);
}
__device__ inline void philox4x64_10(uint64_t ctr[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, ctr[0], hi0, lo0);
    mulhilo64(M1, ctr[2], hi1, lo1);
    uint64_t n0 = hi1 ^ ctr[1] ^ k0, n2 = hi0 ^ ctr[3] ^ k1;
    ctr[0] = n0; ctr[1] = lo1; ctr[2] = n2; ctr[3] = lo0;
    k0 += W0; k1 += W1;
  }
}
constexpr uint64_t kPointKeyHi = 0x41504D47ull;
// Point j of the batch of (step, stream): 24-bit lattice coordinates in [-1, 1).
__device__ inline void uniform_point(uint64_t seed, uint64_t step, uint32_t stream, uint64_t j,
                                     float& x, float& y, float& z) {
  uint64_t c[4] = {j, step, (uint64_t)stream, 0};
  philox4x64_10(c, seed, kPointKeyHi);
  const float s = 1.0f / 8388608.0f;  // 2^-23
  x = (float)(uint32_t)(c[0] >> 40) * s - 1.0f;
  y = (float)(uint32_t)(c[1] >> 40) * s - 1.0f;
  z = (float)(uint32_t)(c[2] >> 40) * s - 1.0f;
}

// ------------------------------------------------------------ encoder pieces
// XCD-aware block order.  Workgroups are dispatched round-robin over the 8 XCDs (each with
// its own L2), so hardware block h runs on XCD h % 8.  xcd_logical deals logical blocks out
// so that XCD x runs the x-th contiguous eighth of the logical order: with spatially sorted
// work in logical order, each XCD works on one slab and its L2 holds that slab's data.
// A bijection for any total.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_logical(int64_t h, int64_t total) {
  const int64_t x = h % kXcds, k = h / kXcds;
  const int64_t q = total / kXcds, r = total % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Eq. (1) with a fixed fma order (the integer decisions depend on it).
__device__ inline void local_coords(const float* Gg, float x, float y, float z, float l[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    l[r] = __builtin_fmaf(Gg[4 * r + 2], z, __builtin_fmaf(Gg[4 * r + 1], y, __builtin_fmaf(Gg[4 * r + 0], x, Gg[4 * r + 3])));
}
// Eq. (2) mask and cell: inside = all(-1 <= l <= 1) (NaN -> outside);
// u = fma(l, h, h), h = (R-1)/2; i0 = clamp(floor(u), 0, R-2); w = u - i0.
__device__ inline bool cell_of(const float l[3], float h, int R, int i0[3], float w[3]) {
  bool in = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    in = in && (l[d] >= -1.0f) && (l[d] <= 1.0f);
    float u = __builtin_fmaf(l[d], h, h);
    float fl = fminf(fmaxf(floorf(u), 0.0f), (float)(R - 2));  // NaN -> 0 via fmaxf
    i0[d] = (int)fl;
    w[d] = u - fl;
  }
  return in;
}

// Load the 2*C values of an x-adjacent vertex pair (channel-last layout):
// out[0..C) = vertex x0, out[C..2C) = vertex x0+1.
template <int C, bool F16>
__device__ inline void load_pair(const void* base, uint32_t idx, float out[2 * C]) {
  if constexpr (!F16) {
    const float* p = (const float*)base + idx;
    if constexpr (C == 1) {
      f32x2a4 v = *(const f32x2a4*)p;
      out[0] = v.x; out[1] = v.y;
    } else if constexpr (C == 2) {
      f32x4a8 v = *(const f32x4a8*)p;
      out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
      f32x4 v0 = *(const f32x4*)p, v1 = *(const f32x4*)(p + 4);
      out[0] = v0.x; out[1] = v0.y; out[2] = v0.z; out[3] = v0.w;
      out[4] = v1.x; out[5] = v1.y; out[6] = v1.z; out[7] = v1.w;
    }
  } else {
    const __half* p = (const __half*)base + idx;
    if constexpr (C == 1) {
      const uint16_t* q = (const uint16_t*)p;
      out[0] = __half2float(__ushort_as_half(q[0])); out[1] = __half2float(__ushort_as_half(q[1]));
    } else if constexpr (C == 2) {
      u32x2a4 v = *(const u32x2a4*)p;
      const uint32_t wa = v.x, wb = v.y;
      float2 fa = __half22float2(*(const __half2*)&wa), fb = __half22float2(*(const __half2*)&wb);
      out[0] = fa.x; out[1] = fa.y; out[2] = fb.x; out[3] = fb.y;
    } else {
      u32x4a8 v = *(const u32x4a8*)p;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint32_t word = v[e];
        float2 fw = __half22float2(*(__half2*)&word);
        out[2 * e] = fw.x; out[2 * e + 1] = fw.y;
      }
    }
  }
}

// The 8 corner values (channel-last) of grid g's cell i0: val[q][c], q = a + 2b + 4c'.
// Element offsets fit 32 bits: a model's grids hold fewer than 2^31 values (checked on entry).
template <int C, bool F16>
__device__ inline void gather_cell(const void* F, int g, int R, const int i0[3], float val[8][C]) {
  const uint32_t RC = (uint32_t)R * C, RRC = (uint32_t)R * R * C;
  const uint32_t base = (((uint32_t)g * R + i0[2]) * R + i0[1]) * RC + (uint32_t)i0[0] * C;
#pragma unroll
  for (int q2 = 0; q2 < 4; ++q2) {  // q2 = b + 2c'
    float pr[2 * C];
    load_pair<C, F16>(F, base + (q2 & 1) * RC + (q2 >> 1) * RRC, pr);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      val[2 * q2][c] = pr[c];
      val[2 * q2 + 1][c] = pr[C + c];
    }
  }
}

// Trilinear interpolation of the 8 corner values with offsets w.
template <int C>
__device__ inline void trilerp(const float val[8][C], const float w[3], float e[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    float x00 = __builtin_fmaf(w[0], val[1][c] - val[0][c], val[0][c]);
    float x10 = __builtin_fmaf(w[0], val[3][c] - val[2][c], val[2][c]);
    float x01 = __builtin_fmaf(w[0], val[5][c] - val[4][c], val[4][c]);
    float x11 = __builtin_fmaf(w[0], val[7][c] - val[6][c], val[6][c]);
    float y0 = __builtin_fmaf(w[1], x10 - x00, x00);
    float y1 = __builtin_fmaf(w[1], x11 - x01, x01);
    e[c] = __builtin_fmaf(w[2], y1 - y0, y0);
  }
}

}  // namespace apmg
