// Grid gradient dL/dF and the transform gradient through the trilinear
// weights (the adjoint of Eq. (2)), gathered per cell instead of scattered
// per point.  One thread owns one cell of one grid: it maps the cell's box
// back to global space (inverse of the transform of Eq. (1)), walks the points
// of the spatial bins that overlap it, keeps those whose float32 cell
// decision is this cell, and sums w_q * dL/dy_c for its 8 corners in
// registers.  A second kernel adds, for each vertex, the corner sums of its
// (up to 8) cells.  No atomics; every sum has a fixed order.

namespace apmg {

struct CellArgs {
  Shape s;
  const float* G; size_t G_stride;      // [M][12] per model
  const void* F; size_t F_stride;       // grids (corner values for the transform gradient)
  const float4* pts4; int64_t n;        // sorted points [model][n] as (x, y, z, 0)
  const uint32_t* start;                // [model][NB^3 + 1]
  const float* dY;                      // [model][M][n][C]
  float* CC;                            // [model][M][(R-1)^3][8][C]
  double* dGpart;                       // [model][M][nblk][12] (DG)
  const int32_t* active;
  int nblk;                             // blocks of 256 cells per grid; launch nmodels * M * nblk blocks
};

// XCD-aware block order.  Workgroups are dispatched round-robin over the 8 XCDs (each with
// its own L2), so hardware block h runs on XCD h % 8.  Logical blocks are dealt out so that
// XCD x runs the x-th contiguous eighth of the logical order; with the order (model, cell
// block, grid), an XCD works through a slab of cells for all grids at once and the points of
// that slab stay in its L2 while every grid reads them.  A bijection for any total.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_logical(int64_t h, int64_t total) {
  const int64_t x = h % kXcds, k = h / kXcds;
  const int64_t q = total / kXcds, r = total % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Candidates are taken U at a time (U = 2, 4 or 8, a launch-shape choice): their
// coordinates (and, for the accepted ones, dL/dy) are loaded together, and a rejected
// candidate adds exact zeros, so the sums keep the candidate order with no branch per point.
template <int C, bool GF16, bool DG, int U>
__global__ void __launch_bounds__(256) k_cell_pull(CellArgs a) {
  constexpr int kCellUnroll = U;
  __shared__ float sG[12];
  __shared__ float sInv[9];
  __shared__ int sBad;
  __shared__ double sred[4][12];
  const Shape s = a.s;
  const int64_t per_model = (int64_t)a.nblk * s.M;
  const int64_t L = xcd_logical(blockIdx.x, gridDim.x);
  const int model = (int)(L / per_model);
  const int blk = (int)((L % per_model) / s.M), g = (int)(L % s.M);
  const bool act = !a.active || a.active[model];
  const int R1 = s.R - 1;
  const int64_t ncell = (int64_t)R1 * R1 * R1;
  if (threadIdx.x < 12) sG[threadIdx.x] = a.G[model * a.G_stride + 12 * g + threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    // inverse of the 3x3 block, float64
    double A[3][3];
    for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) A[r][c] = sG[4 * r + c];
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1], c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    const double inv[9] = {c00, A[0][2] * A[2][1] - A[0][1] * A[2][2], A[0][1] * A[1][2] - A[0][2] * A[1][1],
                           c01, A[0][0] * A[2][2] - A[0][2] * A[2][0], A[0][2] * A[1][0] - A[0][0] * A[1][2],
                           c02, A[0][1] * A[2][0] - A[0][0] * A[2][1], A[0][0] * A[1][1] - A[0][1] * A[1][0]};
    int bad = !(fabs(det) > 1e-30);
    for (int k = 0; k < 9; ++k) {
      const double v = inv[k] / det;
      sInv[k] = (float)v;
      bad |= !isfinite((float)v);
    }
    sBad = bad;
  }
  __syncthreads();
  const int64_t cell = (int64_t)blk * blockDim.x + threadIdx.x;
  const bool valid = act && cell < ncell;
  float acc[8][C];
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[q][c] = 0.f;
  float gacc[DG ? 12 : 1];
#pragma unroll
  for (int k = 0; k < (DG ? 12 : 1); ++k) gacc[k] = 0.f;
  const float4* P4 = a.pts4 + (size_t)model * a.n;
  const float* dY = a.dY + ((size_t)model * s.M + g) * a.n * C;
  const uint32_t* start = a.start + (size_t)model * (kBinsPerAxis * kBinsPerAxis * kBinsPerAxis + 1);
  if (valid) {
    const int cx = (int)(cell % R1), cy = (int)((cell / R1) % R1), cz = (int)(cell / ((int64_t)R1 * R1));
    const float hR = 0.5f * (float)R1;
    // bins overlapping the cell's box in global space; the 1e-4 margin (world units) covers the
    // float32 rounding of the cell decision (~1e-6) and of this box
    int lo[3], hi[3];
    if (sBad) {
      for (int d = 0; d < 3; ++d) { lo[d] = 0; hi[d] = kBinsPerAxis - 1; }
    } else {
      const float lm[3] = {-1.f + (2.f * cx + 1.f) / R1 - sG[3], -1.f + (2.f * cy + 1.f) / R1 - sG[7],
                           -1.f + (2.f * cz + 1.f) / R1 - sG[11]};
      const float hl = 1.0f / R1;
      for (int d = 0; d < 3; ++d) {
        const float wc = sInv[3 * d] * lm[0] + sInv[3 * d + 1] * lm[1] + sInv[3 * d + 2] * lm[2];
        const float hw = (fabsf(sInv[3 * d]) + fabsf(sInv[3 * d + 1]) + fabsf(sInv[3 * d + 2])) * hl;
        const float b0 = floorf((wc - hw - 1e-4f + 1.f) * (0.5f * kBinsPerAxis));
        const float b1 = floorf((wc + hw + 1e-4f + 1.f) * (0.5f * kBinsPerAxis));
        lo[d] = (int)fminf(fmaxf(b0, 0.f), (float)(kBinsPerAxis - 1));
        hi[d] = (int)fminf(fmaxf(b1, 0.f), (float)(kBinsPerAxis - 1));
      }
    }
    float val[DG ? 8 : 1][C];
    if constexpr (DG) {
      const int me[3] = {cx, cy, cz};
      gather_cell<C, GF16>(GF16 ? (const void*)((const __half*)a.F + model * a.F_stride)
                                : (const void*)((const float*)a.F + model * a.F_stride),
                           g, s.R, me, val);
    }
    for (int bz = lo[2]; bz <= hi[2]; ++bz)
      for (int by = lo[1]; by <= hi[1]; ++by) {
        const int row = (bz * kBinsPerAxis + by) * kBinsPerAxis;
        const uint32_t p0 = start[row + lo[0]], p1 = start[row + hi[0] + 1];
        for (uint32_t p = p0; p < p1; p += kCellUnroll) {
          float4 q[kCellUnroll];
#pragma unroll
          for (int u = 0; u < kCellUnroll; ++u) q[u] = P4[min(p + u, p1 - 1)];
          bool ok[kCellUnroll];
          float w[kCellUnroll][3];
#pragma unroll
          for (int u = 0; u < kCellUnroll; ++u) {
            float l[3];
            local_coords(sG, q[u].x, q[u].y, q[u].z, l);
            int i0[3];
            const bool in = cell_of(l, hR, s.R, i0, w[u]);
            ok[u] = (p + u < p1) && in && i0[0] == cx && i0[1] == cy && i0[2] == cz;
#pragma unroll
            for (int d = 0; d < 3; ++d) w[u][d] = ok[u] ? w[u][d] : 0.f;
          }
          float dy[kCellUnroll][C];
#pragma unroll
          for (int u = 0; u < kCellUnroll; ++u)
#pragma unroll
            for (int c = 0; c < C; ++c) dy[u][c] = ok[u] ? dY[(size_t)(p + u) * C + c] : 0.f;
#pragma unroll
          for (int u = 0; u < kCellUnroll; ++u) {
#pragma unroll
            for (int qq = 0; qq < 8; ++qq) {
              const float wq = ((qq & 1) ? w[u][0] : 1.f - w[u][0]) * ((qq & 2) ? w[u][1] : 1.f - w[u][1]) *
                               ((qq & 4) ? w[u][2] : 1.f - w[u][2]);
#pragma unroll
              for (int c = 0; c < C; ++c) acc[qq][c] = __builtin_fmaf(wq, dy[u][c], acc[qq][c]);
            }
            if constexpr (DG) {
              const float* wu = w[u];
              float dl[3] = {0.f, 0.f, 0.f};
#pragma unroll
              for (int c = 0; c < C; ++c) {
                const float ax00 = val[1][c] - val[0][c], ax10 = val[3][c] - val[2][c];
                const float ax01 = val[5][c] - val[4][c], ax11 = val[7][c] - val[6][c];
                const float gx = (1.f - wu[2]) * ((1.f - wu[1]) * ax00 + wu[1] * ax10) +
                                 wu[2] * ((1.f - wu[1]) * ax01 + wu[1] * ax11);
                const float x00 = __builtin_fmaf(wu[0], ax00, val[0][c]);
                const float x10 = __builtin_fmaf(wu[0], ax10, val[2][c]);
                const float x01 = __builtin_fmaf(wu[0], ax01, val[4][c]);
                const float x11 = __builtin_fmaf(wu[0], ax11, val[6][c]);
                const float gy = (1.f - wu[2]) * (x10 - x00) + wu[2] * (x11 - x01);
                const float y0 = __builtin_fmaf(wu[1], x10 - x00, x00);
                const float y1 = __builtin_fmaf(wu[1], x11 - x01, x01);
                dl[0] = __builtin_fmaf(dy[u][c], gx, dl[0]);
                dl[1] = __builtin_fmaf(dy[u][c], gy, dl[1]);
                dl[2] = __builtin_fmaf(dy[u][c], y1 - y0, dl[2]);
              }
              // a rejected candidate may be a NaN point: its coordinates must not reach the sums
              const float xs[4] = {ok[u] ? q[u].x : 0.f, ok[u] ? q[u].y : 0.f, ok[u] ? q[u].z : 0.f, 1.f};
#pragma unroll
              for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 4; ++k) gacc[4 * r + k] = __builtin_fmaf(dl[r] * hR, xs[k], gacc[4 * r + k]);
            }
          }
        }
      }
    float* out = a.CC + (((size_t)model * s.M + g) * ncell + cell) * 8 * C;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c) out[q * C + c] = acc[q][c];
  }
  if constexpr (DG) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double t = wave_sum((double)gacc[k]);
      if (lane == 0) sred[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
      const double t = sred[0][threadIdx.x] + sred[1][threadIdx.x] + sred[2][threadIdx.x] + sred[3][threadIdx.x];
      a.dGpart[(((size_t)model * s.M + g) * a.nblk + blk) * 12 + threadIdx.x] = t;
    }
  }
}

// dF[model][g][v][c] (+)= sum over the cells adjacent to vertex v of their corner sums.
template <int C>
__global__ void k_cell_to_vertex(Shape s, const float* CC, float* dF, size_t dF_stride, int accumulate,
                                 const int32_t* active) {
  const int model = blockIdx.z, g = blockIdx.y;
  if (active && !active[model]) return;
  const int R = s.R, R1 = R - 1;
  const int64_t nv = (int64_t)R * R * R, ncell = (int64_t)R1 * R1 * R1;
  const float* cc = CC + ((size_t)model * s.M + g) * ncell * 8 * C;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    const int vx = (int)(v % R), vy = (int)((v / R) % R), vz = (int)(v / ((int64_t)R * R));
    float sum[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sum[c] = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int cx = vx - (q & 1), cy = vy - ((q >> 1) & 1), cz = vz - (q >> 2);
      if (cx < 0 || cy < 0 || cz < 0 || cx >= R1 || cy >= R1 || cz >= R1) continue;
      const float* src = cc + (((int64_t)cz * R1 + cy) * R1 + cx) * 8 * C + q * C;
#pragma unroll
      for (int c = 0; c < C; ++c) sum[c] += src[c];
    }
    float* dst = dF + model * dF_stride + ((size_t)g * nv + v) * C;
#pragma unroll
    for (int c = 0; c < C; ++c) dst[c] = accumulate ? dst[c] + sum[c] : sum[c];
  }
}

// dG[model][g][k] (+)= sum over the cell blocks of grid g of the per-block partials, in block order.
__global__ void k_reduce_cell_dG(const double* part, int M, int cb, double* dG, size_t dG_stride, int accumulate,
                                 const int32_t* active) {
  const int model = blockIdx.y;
  if (active && !active[model]) return;
  for (int e = threadIdx.x; e < 12 * M; e += blockDim.x) {
    const int g = e / 12, k = e % 12;
    double s = 0.0;
    for (int b = 0; b < cb; ++b) s += part[(((size_t)model * M + g) * cb + b) * 12 + k];
    double* o = dG + model * dG_stride + e;
    *o = accumulate ? *o + s : s;
  }
}

}  // namespace apmg
