// Feature-density loss (Sec. 4.2, Eqs. (7)-(9)), point generation and
// ground-truth sampling (Sec. 7 "Training", Sec. 4.3.1), brick assignment
// (Sec. 5.3), Adam (Sec. 7), layout conversion and fixed-order reductions.

namespace apmg {

// ------------------------------------------------------------------ fill / reduce
__global__ void k_fill_f32(float* p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double* p, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// out[model][e] (+)= sum_b part[(model*nblk + b)*len + off + e] for e < count, in float64.
// Element e lands at (e / cols) * ld_out + col0 + e % cols of the model's output.
// A block handles 32 elements; its 8 thread groups sum 8 contiguous ranges of b, which are
// then added in range order (a fixed order: bitwise reproducible).
constexpr int kRedElems = 32, kRedSplit = 8;
__global__ void __launch_bounds__(256) k_reduce_parts(const double* part, int nblk, int len, int off, int count,
                                                      int cols, int ld_out, int col0, float* outf, double* outd,
                                                      size_t out_stride, int accumulate, const int32_t* active) {
  __shared__ double sp[kRedSplit][kRedElems];
  const int model = blockIdx.y;
  if (active && !active[model]) return;
  const int el = threadIdx.x % kRedElems, sp_i = threadIdx.x / kRedElems;
  const int per = (nblk + kRedSplit - 1) / kRedSplit;
  const int b0 = sp_i * per, b1 = min(nblk, b0 + per);
  for (int base = blockIdx.x * kRedElems; base < count; base += gridDim.x * kRedElems) {
    const int e = base + el;
    double s = 0.0;
    if (e < count) {
      const double* p = part + (size_t)model * nblk * len + off + e;
#pragma unroll 8
      for (int b = b0; b < b1; ++b) s += p[(size_t)b * len];
    }
    sp[sp_i][el] = s;
    __syncthreads();
    if (sp_i == 0 && e < count) {
      double t = sp[0][el];
      for (int k = 1; k < kRedSplit; ++k) t += sp[k][el];
      const size_t oi = model * out_stride + (size_t)(e / cols) * ld_out + col0 + e % cols;
      if (outf) outf[oi] = accumulate ? outf[oi] + (float)t : (float)t;
      else outd[oi] = accumulate ? outd[oi] + t : t;
    }
    __syncthreads();
  }
}

__global__ void k_copy_f64(const double* src, int sstride, double* dst, int dstride, int n, double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[(size_t)i * dstride] = src[(size_t)i * sstride] * scale;
}

// ------------------------------------------------------------------ points / ground truth
__global__ void k_uniform_points(uint64_t seed, uint64_t step, uint32_t stream, int64_t start,
                                 int64_t n, float* pts, int64_t ld) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float x, y, z;
    uniform_point(seed, step, stream, (uint64_t)(start + i), x, y, z);
    pts[i] = x; pts[ld + i] = y; pts[2 * ld + i] = z;
  }
}

// Trilinear sample of a corner-aligned sub-volume: voxels [e0, e0+n) per axis of a
// [nz][ny][nx] volume; u = fma(x, (n-1)/2, (n-1)/2), lower voxel clamp(floor(u), 0, n-2).
__device__ inline float sample_volume(const float* vol, int vnx, int vny, const int e0[3],
                                      const int nn[3], float x, float y, float z) {
  const float p[3] = {x, y, z};
  int i0[3];
  float w[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float h = 0.5f * (float)(nn[d] - 1);
    const float u = __builtin_fmaf(p[d], h, h);
    const float fl = fminf(fmaxf(floorf(u), 0.f), (float)(nn[d] - 2));
    i0[d] = (int)fl;
    w[d] = u - fl;
  }
  const size_t sy = (size_t)vnx, sz = (size_t)vnx * vny;
  const float* b = vol + (size_t)(e0[2] + i0[2]) * sz + (size_t)(e0[1] + i0[1]) * sy + (e0[0] + i0[0]);
  const float v000 = b[0], v100 = b[1], v010 = b[sy], v110 = b[sy + 1];
  const float v001 = b[sz], v101 = b[sz + 1], v011 = b[sz + sy], v111 = b[sz + sy + 1];
  const float x00 = __builtin_fmaf(w[0], v100 - v000, v000), x10 = __builtin_fmaf(w[0], v110 - v010, v010);
  const float x01 = __builtin_fmaf(w[0], v101 - v001, v001), x11 = __builtin_fmaf(w[0], v111 - v011, v011);
  const float y0 = __builtin_fmaf(w[1], x10 - x00, x00), y1 = __builtin_fmaf(w[1], x11 - x01, x01);
  return __builtin_fmaf(w[2], y1 - y0, y0);
}

__global__ void k_gt_sample(const float* vol, int nx, int ny, int nz, const float* pts, int64_t ld,
                            int64_t n, float* v) {
  const int e0[3] = {0, 0, 0}, nn[3] = {nx, ny, nz};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = sample_volume(vol, nx, ny, e0, nn, pts[i], pts[ld + i], pts[2 * ld + i]);
}

// ------------------------------------------------------------------ cells / bricks
// G: [M][grows][4] (rows 0..2 read).
__global__ void k_cells(Shape s, const float* G, int grows, const float* pts, int64_t ld, int64_t n,
                        int32_t* cell, uint8_t* inside) {
  const float hR = 0.5f * (float)(s.R - 1);
  const int64_t total = n * s.M;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / s.M;
    const int g = (int)(i % s.M);
    float l[3];
    local_coords(G + 4 * grows * g, pts[p], pts[ld + p], pts[2 * ld + p], l);
    int i0[3];
    float w[3];
    const bool in = cell_of(l, hR, s.R, i0, w);
    if (cell) for (int d = 0; d < 3; ++d) cell[3 * i + d] = in ? i0[d] : -1;
    if (inside) inside[i] = in ? 1 : 0;
  }
}

__device__ inline int brick_of(const apmg_brick_table& t, const float p[3]);

__global__ void k_assign_bricks(apmg_brick_table t, const float* pts, int64_t ld, int64_t n, int32_t* brick) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float p[3] = {pts[i], pts[ld + i], pts[2 * ld + i]};
    brick[i] = brick_of(t, p);
  }
}

// ------------------------------------------------------------------ layout conversion
template <typename TS, typename TD>
__global__ void k_convert(int M, int C, int R, const TS* src, TD* dst, int to_cl) {
  const size_t R3 = (size_t)R * R * R, total = (size_t)M * C * R3;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    // i indexes the destination
    size_t si;
    if (to_cl) {  // dst [M][R3][C] from src [M][C][R3]
      const size_t c = i % C, v = (i / C) % R3, g = i / (C * R3);
      si = (g * C + c) * R3 + v;
    } else {      // dst [M][C][R3] from src [M][R3][C]
      const size_t v = i % R3, c = (i / R3) % C, g = i / (C * R3);
      si = (g * R3 + v) * C + c;
    }
    float val;
    if constexpr (sizeof(TS) == 2) val = __half2float(*(const __half*)&src[si]); else val = (float)src[si];
    if constexpr (sizeof(TD) == 2) { __half hv = __float2half_rn(val); dst[i] = *(TD*)&hv; } else dst[i] = (TD)val;
  }
}

// Gather mirror of nm grids (all models of a batch, one after another): dst is channel-last
// [nm][R^3][C] in TD; src is [nm][C][R^3] (SRC_PAPER) or [nm][R^3][C], in TS.  One thread per
// vertex: with the paper's order every channel plane is read coalesced and the C values of a
// vertex are stored together.  float -> half rounds to nearest even.
template <int C, typename TS, typename TD, bool SRC_PAPER>
__global__ void k_mirror_grids(int64_t nm, int64_t R3, const TS* __restrict__ src, TD* __restrict__ dst) {
  const int64_t total = nm * R3;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = i / R3, v = i - g * R3;
    float val[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const TS x = SRC_PAPER ? src[(g * C + c) * R3 + v] : src[i * C + c];
      if constexpr (sizeof(TS) == 2) val[c] = __half2float(*(const __half*)&x);
      else val[c] = (float)x;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if constexpr (sizeof(TD) == 2) { const __half h = __float2half_rn(val[c]); dst[i * C + c] = *(const TD*)&h; }
      else dst[i * C + c] = (TD)val[c];
    }
  }
}

// Rows 0..2 of ng transforms stored [ng][4][4] -> compact [ng][3][4].
__global__ void k_pack_G(int64_t ng, const float* __restrict__ src, float* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 12 * ng; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[(i / 12) * 16 + i % 12];
}

// ------------------------------------------------------------------ feature density
// det and cofactor of each transform's 3x3 block, float64: dc[g] = {det, cof[9]}.
__device__ inline void det_cof(const float* Gg, double out[10]) {
  double A[3][3];
  for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) A[r][c] = Gg[4 * r + c];
  out[1] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  out[2] = -(A[1][0] * A[2][2] - A[1][2] * A[2][0]);
  out[3] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  out[4] = -(A[0][1] * A[2][2] - A[0][2] * A[2][1]);
  out[5] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
  out[6] = -(A[0][0] * A[2][1] - A[0][1] * A[2][0]);
  out[7] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
  out[8] = -(A[0][0] * A[1][2] - A[0][2] * A[1][0]);
  out[9] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
  out[0] = A[0][0] * out[1] + A[0][1] * out[2] + A[0][2] * out[3];
}

// l^k by squaring, k >= 1
__device__ inline float powi(float l, int k) {
  float r = 1.f, b = l;
  while (k) { if (k & 1) r *= b; b *= b; k >>= 1; }
  return r;
}

// The flat-top exponent terms of Eq. (7): l^(2p), and l^(2p-1) for its derivative.  P > 0
// fixes p at compile time (P = 10, the paper's value, takes a short multiplication chain);
// P = 0 uses the runtime p.
template <int P>
__device__ inline float flat_pow(float l, int p) {
  if constexpr (P == 10) {
    const float l2 = l * l, l4 = l2 * l2, l8 = l4 * l4, l16 = l8 * l8;
    return l16 * l4;
  } else {
    return powi(l, 2 * p);
  }
}
template <int P>
__device__ inline void flat_pow2(float l, int p, float& e2p, float& e2pm1) {
  if constexpr (P == 10) {
    const float l2 = l * l, l4 = l2 * l2, l8 = l4 * l4, l16 = l8 * l8, l18 = l16 * l2;
    e2pm1 = l18 * l;
    e2p = l18 * l2;
  } else {
    e2p = powi(l, 2 * p);
    e2pm1 = powi(l, 2 * p - 1);
  }
}

// Pass A: rho per point (Eq. (7)) and block sums of rho and err.
// part: [model][block][2] = {sum rho, sum err}
// GEN: the training batch as it is drawn -- point i of model b regenerated from its counter
// (stream stream0 + b, the bits the sort and the ground truth use), rho kept at draw index i
// (pass B1 reads it through the sort's permutation), only part[..][0]; the error sums
// (part[..][1]) come from k_density_errsum once the adjoint has run.  This needs neither the
// sorted points nor the errors, so it runs beside the batch sort.
template <int PF, bool GEN = false>
__global__ void __launch_bounds__(256) k_density_a(Shape s, const float* Gall, size_t G_stride,
    const float* pts, int64_t ld, size_t pts_stride, int64_t n, const float* err, size_t err_stride,
    int p, int abs_det, float* rho, size_t rho_stride, double* part, const int32_t* active,
    uint64_t seed = 0, const uint64_t* step_ctr = nullptr, uint32_t stream0 = 0) {
  extern __shared__ float smem[];
  const int model = blockIdx.y;
  double* spart = (double*)smem;   // [wave][2]
  float* sG = (float*)(spart + 8);
  float* sdet = sG + 12 * s.M;
  const bool act = !active || active[model];
  const float* G = Gall + model * G_stride;
  for (int i = threadIdx.x; i < 12 * s.M; i += blockDim.x) sG[i] = G[i];
  __syncthreads();
  for (int g = threadIdx.x; g < s.M; g += blockDim.x) {
    double dc[10];
    det_cof(sG + 12 * g, dc);
    sdet[g] = (float)(abs_det ? fabs(dc[0]) : dc[0]);
  }
  __syncthreads();
  double srho = 0.0, serr = 0.0;
  const float* P = pts + model * pts_stride;
  const uint64_t step = GEN ? *step_ctr : 0;
  if (act) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      float x, y, z;
      if constexpr (GEN) uniform_point(seed, step, stream0 + (uint32_t)model, (uint64_t)i, x, y, z);
      else { x = P[i]; y = P[ld + i]; z = P[2 * ld + i]; }
      float r = 0.f;
      for (int g = 0; g < s.M; ++g) {
        float l[3];
        local_coords(sG + 12 * g, x, y, z, l);
        const float sv = flat_pow<PF>(l[0], p) + flat_pow<PF>(l[1], p) + flat_pow<PF>(l[2], p);
        if (sv <= kSMax) r = __builtin_fmaf(sdet[g], __expf(-sv), r);
      }
      if (rho) rho[model * rho_stride + i] = r;
      srho += r;
      if constexpr (!GEN) serr += err[model * err_stride + i];
    }
  }
  srho = wave_sum(srho);
  serr = wave_sum(serr);
  if ((threadIdx.x & 63) == 0) { spart[2 * (threadIdx.x >> 6)] = srho; spart[2 * (threadIdx.x >> 6) + 1] = serr; }
  __syncthreads();
  if (threadIdx.x < (GEN ? 1 : 2))
    part[((size_t)model * gridDim.x + blockIdx.x) * 2 + threadIdx.x] =
        ((spart[threadIdx.x] + spart[2 + threadIdx.x]) + spart[4 + threadIdx.x]) + spart[6 + threadIdx.x];
}

// The error half of pass A's partials (part[model][block][1] = block sum of err, the blocks and
// the order of k_density_a), for the training step's pass A over the drawn batch.
__global__ void __launch_bounds__(256) k_density_errsum(const float* err, size_t err_stride, int64_t n, double* part,
                                                        const int32_t* active) {
  __shared__ double spart[4];
  const int model = blockIdx.y;
  double serr = 0.0;
  if (!active || active[model])
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      serr += err[model * err_stride + i];
  serr = wave_sum(serr);
  if ((threadIdx.x & 63) == 0) spart[threadIdx.x >> 6] = serr;
  __syncthreads();
  if (threadIdx.x == 0)
    part[((size_t)model * gridDim.x + blockIdx.x) * 2 + 1] = ((spart[0] + spart[1]) + spart[2]) + spart[3];
}

// Fixed-order block sum of the K-tuples part[model][k][K], k < nblk: out[q] = sum_k [q].
// Thread t sums the contiguous range [t*per, (t+1)*per); the 256 range sums are then added
// by a fixed tree.  One block per model.
template <int K>
__device__ inline void tuple_sum(const double* part, int nblk, double out[K]) {
  __shared__ double sh[K][256];
  const int per = (nblk + 255) / 256;
  const int k0 = threadIdx.x * per, k1 = min(nblk, k0 + per);
  double x[K];
#pragma unroll
  for (int q = 0; q < K; ++q) x[q] = 0.0;
  for (int k = k0; k < k1; ++k)
#pragma unroll
    for (int q = 0; q < K; ++q) x[q] += part[K * (size_t)k + q];
#pragma unroll
  for (int q = 0; q < K; ++q) sh[q][threadIdx.x] = x[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < K; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < K; ++q) out[q] = sh[q][0];
}

// Reduce pass-A partials: sums[model] = {S, sum err}.
__global__ void __launch_bounds__(256) k_density_sums(const double* part, int nblk, double* sums, int nmodels) {
  const int model = blockIdx.x;
  double o[2];
  tuple_sum<2>(part + (size_t)model * nblk * 2, nblk, o);
  if (threadIdx.x == 0) { sums[2 * model] = o[0]; sums[2 * model + 1] = o[1]; }
}

// Target density and loss summand for one point, float64 (Eqs. (8), (9)): rho_s, the
// target rho* and, with it unnormalised, the loss summand and a = dL/drho_s.
__device__ inline void target_terms(double rho, double S, double hbar, double h, double eps, double N,
                                    double& term, double& a, double& rho_s, double& target) {
  rho_s = rho / S;
  const double lg = log(rho_s + eps);
  const double lt = hbar / (h + eps) * lg;
  const double rs = exp(lt);
  term = rs > 0.0 ? rs * (lt - lg) : 0.0;
  a = -rs / (N * (rho_s + eps));
  target = rs;
}

// Pass B1: per block, {sum of loss summands, Q = sum a rho_s, sum rho*} (a and the loss
// summands with the unnormalised target); a of every point is kept for the coefficient pass.
// part: [model][block][3]; a_out: [model][a_stride]
// rho_perm (or NULL): point i's rho is at rho_perm[model][i] (rho in the batch's draw order,
// the points and errors in sorted order).
__global__ void __launch_bounds__(256) k_density_b1(const float* rho, size_t rho_stride, const float* err,
    size_t err_stride, int64_t n, const double* sums, double eps, double* part, double* a_out, size_t a_stride,
    const int32_t* active, const uint32_t* rho_perm = nullptr) {
  __shared__ double spart[12];   // [wave][3]
  const int model = blockIdx.y;
  const bool act = (!active || active[model]) && sums[2 * model] != 0.0;
  double sl = 0.0, sq = 0.0, sz = 0.0;
  if (act) {
    const double S = sums[2 * model], hbar = sums[2 * model + 1] / (double)n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      double term, a, rs, tg;
      const int64_t ri = rho_perm ? (int64_t)rho_perm[model * n + i] : i;
      target_terms(rho[model * rho_stride + ri], S, hbar, err[model * err_stride + i], eps, (double)n, term, a, rs, tg);
      a_out[model * a_stride + i] = a;
      sl += term;
      sq += a * rs;
      sz += tg;
    }
  }
  sl = wave_sum(sl);
  sq = wave_sum(sq);
  sz = wave_sum(sz);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { spart[3 * w] = sl; spart[3 * w + 1] = sq; spart[3 * w + 2] = sz; }
  __syncthreads();
  if (threadIdx.x < 3)
    part[((size_t)model * gridDim.x + blockIdx.x) * 3 + threadIdx.x] =
        ((spart[threadIdx.x] + spart[3 + threadIdx.x]) + spart[6 + threadIdx.x]) + spart[9 + threadIdx.x];
}

// Reduce pass-B1 partials into lq[model] = {loss, Q, Z}: Z = 1 for the literal target, and
// Z = sum rho* for the renormalised one (target rho*/Z), for which
// loss = (sum of summands) / (n Z) - log(Z) / n and Q = Q_raw / Z.
__global__ void __launch_bounds__(256) k_density_lq(const double* part, int nblk, int64_t n, double* lq, int nmodels,
                                                    int norm_target) {
  const int model = blockIdx.x;
  double o[3];
  tuple_sum<3>(part + (size_t)model * nblk * 3, nblk, o);
  if (threadIdx.x == 0) {
    const double Z = (norm_target && o[2] > 0.0) ? o[2] : 1.0;
    double loss = n > 0 ? o[0] / ((double)n * Z) : 0.0;
    if (norm_target && n > 0) loss -= log(Z) / (double)n;
    lq[3 * model] = loss;
    lq[3 * model + 1] = o[1] / Z;
    lq[3 * model + 2] = Z;
  }
}

// Per-point coefficient c(x) = dL/drho(x) = (a(x)/Z - Q)/S (float64 arithmetic, stored float32).
__global__ void k_density_coef(const double* a_in, size_t a_stride, int64_t n, const double* sums, const double* lq,
                               float* coef, size_t coef_stride, const int32_t* active) {
  const int model = blockIdx.y;
  const bool act = (!active || active[model]) && sums[2 * model] != 0.0;
  const double S = sums[2 * model];
  const double Q = lq[3 * model + 1], Z = lq[3 * model + 2];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float c = 0.f;
    if (act) c = (float)((a_in[model * a_stride + i] / Z - Q) / S);
    coef[model * coef_stride + i] = c;
  }
}

// Pass B2: per grid i, U_i = {sum c phi_i, sum c phi_i q_d x_k (9), sum c phi_i q_d (3)}.
// Wave w of block (chunk, grid group, model) owns grid 4*blockIdx.y + w and streams the
// chunk's points; one wave reduction per (grid, chunk).  part: [model][M][chunk][13]
constexpr int kDensChunk = 4096;
template <int PF>
__global__ void __launch_bounds__(256) k_density_b2(Shape s, const float* Gall, size_t G_stride,
    const float* pts, int64_t ld, size_t pts_stride, int64_t n, const float* coef, size_t coef_stride, int p,
    double* part, const int32_t* active) {
  const int model = blockIdx.z, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = 4 * blockIdx.y + wave;
  const int nchunk = gridDim.x;
  if (g >= s.M) return;
  const bool act = !active || active[model];
  float Gg[12];
  for (int k = 0; k < 12; ++k) Gg[k] = Gall[model * G_stride + 12 * g + k];
  float u[13];
#pragma unroll
  for (int q = 0; q < 13; ++q) u[q] = 0.f;
  if (act) {
    const float* P = pts + model * pts_stride;
    const float* cf = coef + model * coef_stride;
    const int64_t i0 = (int64_t)blockIdx.x * kDensChunk, i1 = min(n, i0 + kDensChunk);
    for (int64_t i = i0 + lane; i < i1; i += 64) {
      const float c = cf[i];
      if (c == 0.f) continue;
      const float xs[3] = {P[i], P[ld + i], P[2 * ld + i]};
      float l[3];
      local_coords(Gg, xs[0], xs[1], xs[2], l);
      float e2p[3], e2pm1[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) flat_pow2<PF>(l[d], p, e2p[d], e2pm1[d]);
      const float sv = e2p[0] + e2p[1] + e2p[2];
      if (!(sv <= kSMax)) continue;
      const float cphi = c * __expf(-sv);
      u[0] += cphi;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float cq = cphi * e2pm1[d];
        u[1 + 3 * d] = __builtin_fmaf(cq, xs[0], u[1 + 3 * d]);
        u[2 + 3 * d] = __builtin_fmaf(cq, xs[1], u[2 + 3 * d]);
        u[3 + 3 * d] = __builtin_fmaf(cq, xs[2], u[3 + 3 * d]);
        u[10 + d] += cq;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 13; ++q) {
    const double t = wave_sum((double)u[q]);
    if (lane == 0) part[(((size_t)model * s.M + g) * nchunk + blockIdx.x) * 13 + q] = t;
  }
}

// U[model][g][q] = sum over chunks of part[model][g][chunk][q]: thread t sums a contiguous
// range of chunks, then a fixed tree adds the 256 range sums.  Grid (M, models).
__global__ void __launch_bounds__(256) k_density_b2_reduce(const double* part, int M, int nchunk, double* U,
                                                           const int32_t* active) {
  __shared__ double sh[256];
  const int model = blockIdx.y, g = blockIdx.x;
  if (active && !active[model]) return;
  const double* pp = part + ((size_t)model * M + g) * nchunk * 13;
  const int per = (nchunk + 255) / 256;
  const int k0 = threadIdx.x * per, k1 = min(nchunk, k0 + per);
  for (int q = 0; q < 13; ++q) {
    double x = 0.0;
    for (int k = k0; k < k1; ++k) x += pp[(size_t)k * 13 + q];
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) U[((size_t)model * M + g) * 13 + q] = sh[0];
    __syncthreads();
  }
}

// Assemble dG_i = cof_i U0 - 2p det_i [U1 | U2] from the reduced pass-B2 sums.
// Assemble dG_i = sgn_i cof_i U0 - 2p det_i [U1 | U2] from the reduced pass-B2 sums, where
// det_i and sgn_i are det(A_i) and 1 (signed reading) or |det(A_i)| and sign(det(A_i))
// (abs_det).  dG rows per transform: grows (3, or 4 with row 3 written as 0).
__global__ void k_density_grad(Shape s, const float* Gall, size_t G_stride, const double* U, int p, int abs_det,
                               double* dG, size_t dG_stride, int grows, int accumulate, const double* sums,
                               const int32_t* active) {
  const int model = blockIdx.y;
  if (active && !active[model]) return;
  const bool zero = sums[2 * model] == 0.0;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < s.M; g += gridDim.x * blockDim.x) {
    double dc[10];
    det_cof(Gall + model * G_stride + 12 * g, dc);
    const double sgn = abs_det ? (dc[0] > 0.0 ? 1.0 : (dc[0] < 0.0 ? -1.0 : 0.0)) : 1.0;
    const double det = abs_det ? fabs(dc[0]) : dc[0];
    const double* u = U + (size_t)model * 13 * s.M + 13 * g;
    double* o = dG + model * dG_stride + 4 * grows * g;
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) {
        const double v = zero ? 0.0 : sgn * dc[1 + 3 * r + k] * u[0] - 2.0 * p * det * u[1 + 3 * r + k];
        o[4 * r + k] = accumulate ? o[4 * r + k] + v : v;
      }
      const double v = zero ? 0.0 : -2.0 * p * det * u[10 + r];
      o[4 * r + 3] = accumulate ? o[4 * r + 3] + v : v;
    }
    if (grows == 4 && !accumulate)
      for (int k = 0; k < 4; ++k) o[12 + k] = 0.0;
  }
}

// ------------------------------------------------------------------ Adam
// theta -= lr * mhat / (sqrt(vhat) + eps), bias-corrected with step t+1 (t read from
// counters[model]).  gd (double) or gf (float) gradient.
// active: per model, skip when 0 (NULL = all); lr_scale: per model multiplier of lr (NULL = 1).
__global__ void k_adam(float* theta, float* m, float* v, const float* gf, const double* gd, size_t per_model,
                       const int32_t* counters, const int32_t* active, float lr, float b1, float b2,
                       float eps, const float* lr_scale) {
  const int model = blockIdx.y;
  if (active && !active[model]) return;
  // bias corrections in float64, once per block
  __shared__ float sc[2];
  if (threadIdx.x == 0) {
    const int t = counters[model] + 1;
    const float bc1 = (float)(1.0 - pow((double)b1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)b2, (double)t));
    const float lrm = lr_scale ? lr * lr_scale[model] : lr;
    sc[0] = lrm / bc1;
    sc[1] = 1.0f / sqrtf(bc2);
  }
  __syncthreads();
  const float step = sc[0], rb2 = sc[1];
  const size_t off = (size_t)model * per_model;
  auto one = [&](float g, float& mk, float& vk, float& th) {
    mk = __builtin_fmaf(b1, mk, (1.f - b1) * g);
    vk = __builtin_fmaf(b2, vk, (1.f - b2) * g * g);
    th = th - step * mk / (sqrtf(vk) * rb2 + eps);
  };
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i0 = 0;
  // four elements per thread with 16-byte accesses where every array allows it; the same
  // arithmetic per element as the scalar loop that finishes the rest
  if (gf && ((uintptr_t)(theta + off) | (uintptr_t)(m + off) | (uintptr_t)(v + off) |
                        (uintptr_t)(gf + off)) % 16 == 0) {
    const size_t n4 = per_model / 4;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += stride) {
      const size_t k = off + 4 * i;
      const float4 g4 = *(const float4*)(gf + k);
      float4 m4 = *(float4*)(m + k), v4 = *(float4*)(v + k), t4 = *(float4*)(theta + k);
      one(g4.x, m4.x, v4.x, t4.x);
      one(g4.y, m4.y, v4.y, t4.y);
      one(g4.z, m4.z, v4.z, t4.z);
      one(g4.w, m4.w, v4.w, t4.w);
      *(float4*)(m + k) = m4;
      *(float4*)(v + k) = v4;
      *(float4*)(theta + k) = t4;
    }
    i0 = 4 * n4;
  }
  for (size_t i = i0 + blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < per_model; i += stride) {
    const size_t k = off + i;
    float mk = m[k], vk = v[k], th = theta[k];
    one(gf ? gf[k] : (float)gd[k], mk, vk, th);
    m[k] = mk;
    v[k] = vk;
    theta[k] = th;
  }
}

// G is stored [M][3][4] float; its gradient is float64 of the same shape.
// live: models that trained this step; dlive: models whose transforms trained.
__global__ void k_step_counters(int32_t* t, int32_t* tG, const int32_t* live, const int32_t* dlive, uint64_t* step,
                                int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) {
    if (live[b]) t[b] += 1;
    if (dlive[b]) tG[b] += 1;
  }
  if (b == 0) *step += 1;
}

// live[b] = !frozen[b]; dlive[b] = live[b] && density_active[b].
__global__ void k_live_masks(const int32_t* frozen, const int32_t* density_active, int32_t* live, int32_t* dlive,
                             int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) {
    const int32_t l = frozen ? (frozen[b] ? 0 : 1) : 1;
    live[b] = l;
    dlive[b] = (l && density_active[b]) ? 1 : 0;
  }
}

// ------------------------------------------------------------------ training control
// One thread per model: the schedule of Sec. 4.3.2 (delayed start, transform early stop)
// and the plateau scheduler of Sec. 5.2, applied to the losses of the step just taken.
__global__ void k_train_control(apmg_control c, const double* losses) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= c.nb) return;
  if (c.frozen[b]) return;
  apmg_ctl_state st = c.state[b];
  const double lrec = losses[2 * b], lden = losses[2 * b + 1];
  const int it = st.iter + 1;
  // transform early stop over blocks of ma_window density iterations
  if (c.density_active[b]) {
    st.ma_sum += lden;
    st.ma_count += 1;
    if (st.ma_count == c.ma_window) {
      const double mean = st.ma_sum / (double)c.ma_window;
      if (st.have_prev && !(mean < st.ma_prev * (1.0 - c.ma_rel))) st.density_done = 1;
      st.ma_prev = mean;
      st.have_prev = 1;
      st.ma_sum = 0.0;
      st.ma_count = 0;
    }
  }
  const int limit = (int)(c.stop_frac * (float)c.total_iters);
  if (it + 1 > limit) st.density_done = 1;
  // plateau scheduler on L_rec
  if (it == 1 || lrec < st.best * (1.0 - c.plateau_rel)) {
    st.best = lrec;
    st.bad = 0;
  } else {
    st.bad += 1;
  }
  int frozen = 0;
  if (st.bad > c.patience) {
    c.lr_scale[b] = c.lr_scale[b] * c.plateau_factor;
    st.bad = 0;
    st.reductions += 1;
    if (st.reductions >= c.max_reductions) frozen = 1;
  }
  st.iter = it;
  c.state[b] = st;
  c.density_active[b] = (!frozen && it >= c.delay && !st.density_done) ? 1 : 0;
  c.frozen[b] = frozen;
}

}  // namespace apmg
