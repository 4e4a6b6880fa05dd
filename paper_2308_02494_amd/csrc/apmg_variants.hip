// Adjoint of the two encoder variants of Sec. 9 (a hash grid inside each adaptive grid; 4-D
// grids with a time axis) with respect to their tables / grids and the transforms.
//
// The forward and the MLP adjoint are the tile kernels (k_forward, k_adjoint) instantiated
// with the variant's lookup (enc_tap); k_adjoint stores dL/dy per (feature grid, point) of the
// spatially sorted points.  The scatter below then adds w_q dL/dy_c into the corner entries
// with float atomics: a hash table entry collects the contributions of every vertex that maps
// to it, so the per-cell gather of the dense grids does not apply, and the 4-D grids share the
// scatter.  Neighbouring sorted points mostly share a cell, so each wave first sums the runs
// of lanes with the same cell and only the run's first lane issues the atomics.  The sums of
// float atomics are not in a fixed order (results reproducible to rounding).  The transform
// gradient through the interpolation weights is reduced per block in float64, in a fixed
// order.

namespace apmg {

struct EncScatterArgs {
  Shape s;
  EncArgs enc;
  const float* G;          // [M / L][12]
  const float* F;          // hash: tables [M][T][C]; time: channel-last [M][Rt][R^3][C]
  const float* pts; int64_t ld; int64_t n;
  const float* tau;        // time: [n] time of each point
  const float* dY;         // [M][n][C], dL/dy per feature grid (M feature grids)
  float* dF;               // same layout as F (channel-last for time), accumulated; NULL: no grid gradient
  double* dGpart;          // [M][nbx][12], or NULL for no transform gradient
  int nbx;                 // point blocks per feature grid
};

// dl_d = sum_c dy_c d(trilinear_c)/dw_d for corner values val and offsets w.
template <int C>
__device__ inline void trilerp_dw(const float val[8][C], const float w[3], const float dy[C], float dl[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) dl[d] = 0.f;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float wx = (q & 1) ? w[0] : 1.f - w[0], wy = (q & 2) ? w[1] : 1.f - w[1], wz = (q & 4) ? w[2] : 1.f - w[2];
    const float sx = (q & 1) ? 1.f : -1.f, sy = (q & 2) ? 1.f : -1.f, sz = (q & 4) ? 1.f : -1.f;
    float gq = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) gq = __builtin_fmaf(val[q][c], dy[c], gq);
    dl[0] = __builtin_fmaf(gq * sx, wy * wz, dl[0]);
    dl[1] = __builtin_fmaf(gq * sy, wx * wz, dl[1]);
    dl[2] = __builtin_fmaf(gq * sz, wx * wy, dl[2]);
  }
}

__device__ inline float tri_weight(int q, const float w[3]) {
  return ((q & 1) ? w[0] : 1.f - w[0]) * ((q & 2) ? w[1] : 1.f - w[1]) * ((q & 4) ? w[2] : 1.f - w[2]);
}

// Runs of consecutive lanes with the same key (the points are spatially sorted, so
// neighbouring lanes mostly share a cell): seg = the run's first lane; nxt[k] = lane
// + 2^k is in the same run.  A segmented suffix sum over the run then leaves each run's
// total in its first lane, which alone issues the atomics.
struct WaveRuns {
  bool head;
  bool nxt[6];
};
__device__ inline WaveRuns wave_runs(uint64_t key, int lane) {
  WaveRuns r;
  const uint32_t klo = (uint32_t)key, khi = (uint32_t)(key >> 32);
  const uint32_t plo = __shfl_up(klo, 1, 64), phi = __shfl_up(khi, 1, 64);
  r.head = lane == 0 || plo != klo || phi != khi;
  int seg = r.head ? lane : 0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(seg, o, 64);
    if (lane >= o) seg = max(seg, t);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int o = 1 << k;
    const int t = __shfl_down(seg, o, 64);
    r.nxt[k] = lane + o < 64 && t == seg;
  }
  return r;
}
__device__ inline float run_sum(float v, const WaveRuns& r) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float t = __shfl_down(v, 1 << k, 64);
    v += r.nxt[k] ? t : 0.f;
  }
  return v;
}

// One thread per (point, feature grid): blockIdx.y = feature grid g, 256 points per block.
template <int C, int ENC>
__global__ void __launch_bounds__(256) k_enc_scatter(EncScatterArgs a) {
  __shared__ float sG[12 * 256];
  __shared__ double sred[4][12];
  const Shape s = a.s;
  const int g = blockIdx.y, bx = blockIdx.x;
  const int mt = s.M / s.L;
  for (int i = threadIdx.x; i < 12 * mt; i += blockDim.x) sG[i] = a.G[i];
  __syncthreads();
  const int64_t p = (int64_t)bx * blockDim.x + threadIdx.x;
  const bool valid = p < a.n;
  float x = 0.f, y = 0.f, z = 0.f, tq = 0.f;
  if (valid) { x = a.pts[p]; y = a.pts[a.ld + p]; z = a.pts[2 * a.ld + p]; }
  if constexpr (ENC == kEncTime) tq = valid ? a.tau[p] : 0.f;
  float dy[C];
#pragma unroll
  for (int c = 0; c < C; ++c) dy[c] = valid ? a.dY[((size_t)g * a.n + p) * C + c] : 0.f;
  GridTap<C, ENC> t;
  const float hR = 0.5f * (float)(s.R - 1);
  enc_tap<C, false, ENC>(s, sG, a.F, a.enc, g, x, y, z, tq, valid, hR, t);
  float dl[3] = {0.f, 0.f, 0.f};
  const int lane = threadIdx.x & 63;
  if constexpr (ENC == kEncHash) {
    if (a.dF) {
      // the cell of this lane's point (the same float32 decision as the lookup)
      const int gt = g / s.L, k = g - gt * s.L;
      const int N = enc_level_res(a.enc, k);
      float l[3];
      local_coords(sG + 12 * gt, x, y, z, l);
      int i0[3];
      float w[3];
      cell_of(l, 0.5f * (float)N, N + 1, i0, w);
      (void)w;
      const uint64_t key = t.in ? ((uint64_t)i0[2] << 40 | (uint64_t)i0[1] << 20 | (uint64_t)i0[0]) : ~0ull - lane;
      const WaveRuns rn = wave_runs(key, lane);
      const uint32_t n1 = (uint32_t)N + 1u;
      const bool dense = (uint64_t)n1 * n1 * n1 <= (uint64_t)a.enc.tmask + 1u;
      float* base = a.dF + (size_t)g * ((size_t)a.enc.tmask + 1u) * C;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float wq = t.in ? tri_weight(q, t.w) : 0.f;
        float v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = run_sum(wq * dy[c], rn);
        if (t.in && rn.head) {
          const uint32_t ent = hash_entry((uint32_t)i0[0] + (q & 1), (uint32_t)i0[1] + ((q >> 1) & 1),
                                          (uint32_t)i0[2] + (q >> 2), n1, dense, a.enc.tmask);
#pragma unroll
          for (int c = 0; c < C; ++c) unsafeAtomicAdd(base + (size_t)ent * C + c, v[c]);
        }
      }
    }
  } else {
    if (a.dF) {
      float l[3];
      local_coords(sG + 12 * g, x, y, z, l);
      int i0[3];
      float w[3];
      cell_of(l, hR, s.R, i0, w);
      (void)w;
      const float ht = 0.5f * (float)(a.enc.Rt - 1);
      const float ut = __builtin_fmaf(tq, ht, ht);
      const int t0 = (int)fminf(fmaxf(floorf(ut), 0.0f), (float)(a.enc.Rt - 2));
      const uint32_t R = (uint32_t)s.R, RC = R * C, RRC = R * R * C;
      const uint64_t key = t.in ? ((((uint64_t)t0 * R + i0[2]) * R + i0[1]) * R + i0[0]) : ~0ull - lane;
      const WaveRuns rn = wave_runs(key, lane);
      const uint32_t cb = t.in ? ((uint32_t)i0[2] * R + i0[1]) * RC + (uint32_t)i0[0] * C : 0u;
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        const float ws = sl ? t.wt : 1.f - t.wt;
        float* base = a.dF + (((size_t)g * a.enc.Rt + (t.in ? t0 : 0) + sl) * R * R * R) * C;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float wq = t.in ? ws * tri_weight(q, t.w) : 0.f;
          const uint32_t o = cb + (q & 1) * C + ((q >> 1) & 1) * RC + (q >> 2) * RRC;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const float v = run_sum(wq * dy[c], rn);
            if (t.in && rn.head) unsafeAtomicAdd(base + o + c, v);
          }
        }
      }
    }
  }
  if (t.in) {
    if constexpr (ENC == kEncHash) {
      const int N = enc_level_res(a.enc, g - (g / s.L) * s.L);
      trilerp_dw<C>(t.val, t.w, dy, dl);
      const float sc = 0.5f * (float)N;
#pragma unroll
      for (int d = 0; d < 3; ++d) dl[d] *= sc;
    } else {
      float d0[3], d1[3];
      trilerp_dw<C>(t.va, t.w, dy, d0);
      trilerp_dw<C>(t.vb, t.w, dy, d1);
#pragma unroll
      for (int d = 0; d < 3; ++d) dl[d] = ((1.f - t.wt) * d0[d] + t.wt * d1[d]) * hR;
    }
  }
  if (a.dGpart) {
    const float xs[4] = {t.in ? x : 0.f, t.in ? y : 0.f, t.in ? z : 0.f, t.in ? 1.f : 0.f};
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = wave_sum((double)dl[r] * (double)xs[k]);
        if (lane == 0) sred[wave][4 * r + k] = v;
      }
    __syncthreads();
    if (threadIdx.x < 12) {
      const double v = sred[0][threadIdx.x] + sred[1][threadIdx.x] + sred[2][threadIdx.x] + sred[3][threadIdx.x];
      a.dGpart[((size_t)g * a.nbx + bx) * 12 + threadIdx.x] = v;
    }
  }
}

// dst[j] = src[perm[j]] (a per-point array in spatially sorted order).
__global__ void k_gather_f32(const float* __restrict__ src, const uint32_t* __restrict__ perm, int64_t n,
                             float* __restrict__ dst) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    dst[j] = src[perm[j]];
}

// 4-D grids: the time cell of each spatially sorted point (the float32 decision of the lookup;
// outside or NaN times -> 0) as a radix key, with the point's sorted position as its value.
__global__ void k_time_keys(const float* __restrict__ tau, const uint32_t* __restrict__ perm, int64_t n, int Rt,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const float ht = 0.5f * (float)(Rt - 1);
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const float t = tau[perm[j]];
    const float ft = fminf(fmaxf(floorf(__builtin_fmaf(t, ht, ht)), 0.0f), (float)(Rt - 2));
    keys[j] = (t >= -1.0f && t <= 1.0f) ? (uint32_t)ft : 0u;
    vals[j] = (uint32_t)j;
  }
}

// The points, dL/df and times in (time cell, spatial bin) order: position j takes spatially
// sorted position q = perm2[j] (original point perm[q]); also as (x, y, z, t) records.
__global__ void k_time_permute(const float* __restrict__ spts, const float* __restrict__ sf,
                               const float* __restrict__ tau, const uint32_t* __restrict__ perm,
                               const uint32_t* __restrict__ perm2, int64_t n, float* __restrict__ pts2,
                               float* __restrict__ f2, float* __restrict__ tau2, float4* __restrict__ rec) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t q = perm2[j];
    const float x = spts[q], y = spts[n + q], z = spts[2 * n + q], t = tau[perm[q]];
    pts2[j] = x;
    pts2[n + j] = y;
    pts2[2 * n + j] = z;
    f2[j] = sf[q];
    tau2[j] = t;
    rec[j] = make_float4(x, y, z, t);
  }
}

// start[k] for k in [0, (Rt - 1) NB^3]: the first position of the (time cell, bin) order whose
// combined key tc NB^3 + bin is >= k (as k_bin_starts over the combined keys: time keys
// tkey[j] of the sorted order, bin keys bkey[pos[j]] of the spatial order it was taken from).
__global__ void k_time_bin_starts(const uint32_t* __restrict__ tkey, const uint32_t* __restrict__ bkey,
                                  const uint32_t* __restrict__ pos, int64_t n, int Rt, uint32_t* __restrict__ start) {
  const uint32_t nb3 = (uint32_t)kBinsPerAxis * kBinsPerAxis * kBinsPerAxis;
  const uint32_t nkeys = (uint32_t)(Rt - 1) * nb3;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t lo = i == 0 ? 0u : tkey[i - 1] * nb3 + bkey[pos[i - 1]] + 1u;
    const uint32_t hi = i == n ? nkeys : tkey[i] * nb3 + bkey[pos[i]];
    for (uint32_t b = lo; b <= hi; ++b) start[b] = (uint32_t)i;
  }
}

// Channel-last [nm][V][C] -> the paper's order [nm][C][V], added into dst when accumulate.
template <int C>
__global__ void k_cl_to_paper(int64_t nm, int64_t V, const float* __restrict__ src, float* __restrict__ dst,
                              int accumulate) {
  const int64_t total = nm * V;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = i / V, v = i - g * V;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float* d = dst + (g * C + c) * V + v;
      *d = accumulate ? *d + src[i * C + c] : src[i * C + c];
    }
  }
}

hipError_t launch_enc_scatter(const EncScatterArgs& a, int enc, hipStream_t st) {
  const dim3 grid((unsigned)a.nbx, (unsigned)a.s.M);
  if (a.s.C != 2) return hipErrorInvalidValue;
  if (enc == kEncHash) hipLaunchKernelGGL((k_enc_scatter<2, kEncHash>), grid, dim3(256), 0, st, a);
  else if (enc == kEncTime) hipLaunchKernelGGL((k_enc_scatter<2, kEncTime>), grid, dim3(256), 0, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// The tile kernels of the variants (C = 2, H = 64): forward with the weights in LDS, and the
// tiled adjoint with the waves per block of the dense shapes.
hipError_t launch_enc_forward(const TileArgs& a, int enc, bool bf, dim3 grid, size_t shmem, hipStream_t st) {
  if (a.s.C != 2 || a.s.H != 64 || fwd_weight_bytes(a.s, bf) > kFwdWeightLdsMax) return hipErrorInvalidValue;
#define APMG_EF(E)                                                                                \
  if (bf) hipLaunchKernelGGL((k_forward<2, 64, false, true, true, E>), grid, dim3(kBlock), shmem, st, a); \
  else hipLaunchKernelGGL((k_forward<2, 64, false, false, true, E>), grid, dim3(kBlock), shmem, st, a);
  if (enc == kEncHash) { APMG_EF(kEncHash) }
  else if (enc == kEncTime) { APMG_EF(kEncTime) }
  else return hipErrorInvalidValue;
#undef APMG_EF
  return hipGetLastError();
}

hipError_t launch_enc_adjoint(const TileArgs& a, int enc, bool bf, dim3 grid, hipStream_t st) {
  if (a.s.C != 2 || !adjoint_applies(a.s)) return hipErrorInvalidValue;
  const int nw = adjoint_waves(0, bf);
  const size_t shmem = adjoint_lds_bytes(a.s, bf, nw);
  // 32 feature grids of 2 (64 features): the adjoint compiled for that shape
  const bool kf32 = a.s.M == 32;
#define APMG_EA(E, KF_)                                                                                     \
  if (bf) hipLaunchKernelGGL((k_adjoint<2, false, true, 4, E, KF_>), grid, dim3(4 * kWave), shmem, st, a);  \
  else hipLaunchKernelGGL((k_adjoint<2, false, false, 8, E, KF_>), grid, dim3(8 * kWave), shmem, st, a);
  if (enc == kEncHash) { if (kf32) { APMG_EA(kEncHash, 32) } else { APMG_EA(kEncHash, 0) } }
  else if (enc == kEncTime) { if (kf32) { APMG_EA(kEncTime, 32) } else { APMG_EA(kEncTime, 0) } }
  else return hipErrorInvalidValue;
#undef APMG_EA
  return hipGetLastError();
}

}  // namespace apmg
