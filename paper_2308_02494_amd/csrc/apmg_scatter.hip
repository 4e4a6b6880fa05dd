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
  float* CC;                            // [model][M][8][(R-1)^3][C] (corner-major)
  double* dGpart;                       // [model][M][nblk][12] (DG)
  const int32_t* active;
  int nblk;                             // blocks of 256 cells per grid; launch nmodels * M * nblk blocks
  int Rt;                               // 4-D grids (two time slices per cell): time vertices
};

// Corner weight q = a + 2b + 4c of the trilinear weights of offsets w.  Both gathers add
// round(w_q * dL/dy) to the corner sums (a product, then a sum: no fused multiply-add), so
// they produce the same bits.
__device__ inline float corner_weight(int qq, const float w[3]) {
  return ((qq & 1) ? w[0] : 1.f - w[0]) * ((qq & 2) ? w[1] : 1.f - w[1]) * ((qq & 4) ? w[2] : 1.f - w[2]);
}
__device__ inline float corner_product(float wq, float d) {
#pragma clang fp contract(off)
  return wq * d;
}
__device__ inline float add_rounded(float acc, float v) {
#pragma clang fp contract(off)
  return acc + v;
}

// The local box of the cells [c0, c0 + w) (per axis, clipped to the grid) minus the
// translation, widened by 1e-4 (covers the float32 rounding of the cell decision), in float64.
__device__ inline void local_box(const float* Gg, const int c0[3], int w, int R1, double blo[3], double bhi[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int e = min(c0[d] + w, R1);
    blo[d] = -1.0 + 2.0 * c0[d] / R1 - 1e-4 - (double)Gg[4 * d + 3];
    bhi[d] = -1.0 + 2.0 * e / R1 + 1e-4 - (double)Gg[4 * d + 3];
  }
}

// Tighter x-range [x0, x1] (bins, within [lo0, hi0]) of the bin row (yb, zb) for a local box:
// the x for which some (y, z) of the row satisfies each of the three slab constraints
// blo_d <= A_d . x <= bhi_d, taken one slab at a time (a superset of the exact range), in
// float64, with the row widened by 1e-5 (the float32 rounding of the binning) and the x-range
// by 1e-4.  The edge rows of the bin grid reach to infinity, because the binning clamps points
// outside the domain into them.  Returns false for an empty row.
// ra[d] = 1 / Gg[4 d] (0 where that coefficient is 0), from span_recips once per transform:
// the x-range's bounds are multiplied by it rather than divided (they are padded anyway).
__device__ inline void span_recips(const float* Gg, double ra[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) ra[d] = Gg[4 * d] != 0.f ? 1.0 / (double)Gg[4 * d] : 0.0;
}
__device__ inline bool row_x_span(const float* Gg, const double ra[3], const double blo[3], const double bhi[3],
                                  int lo0, int hi0, int yb, int zb, int& x0, int& x1) {
  constexpr double kInf = __builtin_inf(), kW = 2.0 / kBinsPerAxis;
  const double ylo = yb == 0 ? -kInf : -1.0 + yb * kW - 1e-5;
  const double yhi = yb == kBinsPerAxis - 1 ? kInf : -1.0 + (yb + 1) * kW + 1e-5;
  const double zlo = zb == 0 ? -kInf : -1.0 + zb * kW - 1e-5;
  const double zhi = zb == kBinsPerAxis - 1 ? kInf : -1.0 + (zb + 1) * kW + 1e-5;
  double xl = -kInf, xh = kInf;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double a0 = Gg[4 * d], a1 = Gg[4 * d + 1], a2 = Gg[4 * d + 2];
    // range of a1 y + a2 z over the row (a zero coefficient contributes exactly 0)
    const double m_lo = (a1 > 0 ? a1 * ylo : a1 < 0 ? a1 * yhi : 0.0) + (a2 > 0 ? a2 * zlo : a2 < 0 ? a2 * zhi : 0.0);
    const double m_hi = (a1 > 0 ? a1 * yhi : a1 < 0 ? a1 * ylo : 0.0) + (a2 > 0 ? a2 * zhi : a2 < 0 ? a2 * zlo : 0.0);
    const double P = blo[d] - m_hi, Q = bhi[d] - m_lo;      // P <= a0 x <= Q
    if (a0 > 0) { xl = fmax(xl, P * ra[d]); xh = fmin(xh, Q * ra[d]); }
    else if (a0 < 0) { xl = fmax(xl, Q * ra[d]); xh = fmin(xh, P * ra[d]); }
    else if (P > 0.0 || Q < 0.0) return false;
  }
  if (!(xl <= xh)) return false;
  const double f0 = floor((xl - 1e-4 + 1.0) * (0.5 * kBinsPerAxis));
  const double f1 = floor((xh + 1e-4 + 1.0) * (0.5 * kBinsPerAxis));
  x0 = (int)fmin(fmax(f0, (double)lo0), (double)hi0);
  x1 = (int)fmin(fmax(f1, (double)lo0), (double)hi0);
  return true;
}

// The adjoint of Eq. (2) with respect to the local coordinates for one point of a cell with
// corner values val and offsets w: dl_d = sum_c dL/dy_c d(trilerp_c)/du_d, then the transform
// gradient terms (dl h) x^T and (dl h) added to gacc (x masked to 0 for a rejected candidate,
// which may be a NaN point and has dL/dy = 0).
template <int C>
__device__ inline void add_transform_grad(const float val[8][C], const float wu[3], const float dyv[C], float hR,
                                          bool ok, float px, float py, float pz, float gacc[12]) {
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
    dl[0] = __builtin_fmaf(dyv[c], gx, dl[0]);
    dl[1] = __builtin_fmaf(dyv[c], gy, dl[1]);
    dl[2] = __builtin_fmaf(dyv[c], y1 - y0, dl[2]);
  }
  const float xs[4] = {ok ? px : 0.f, ok ? py : 0.f, ok ? pz : 0.f, 1.f};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) gacc[4 * r + k] = __builtin_fmaf(dl[r] * hR, xs[k], gacc[4 * r + k]);
}

// Block order: xcd_logical over (model, cell block, grid), so an XCD works through a slab of
// cells for all grids at once and the points of that slab stay in its L2.

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
    double blo[3], bhi[3], ra[3];
    const int me0[3] = {cx, cy, cz};
    local_box(sG, me0, 1, R1, blo, bhi);
    span_recips(sG, ra);
    for (int bz = lo[2]; bz <= hi[2]; ++bz)
      for (int by = lo[1]; by <= hi[1]; ++by) {
        int x0 = lo[0], x1 = hi[0];
        if (!sBad && !row_x_span(sG, ra, blo, bhi, lo[0], hi[0], by, bz, x0, x1)) continue;
        const int row = (bz * kBinsPerAxis + by) * kBinsPerAxis;
        const uint32_t p0 = start[row + x0], p1 = start[row + x1 + 1];
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
              const float wq = corner_weight(qq, w[u]);
#pragma unroll
              for (int c = 0; c < C; ++c) acc[qq][c] = add_rounded(acc[qq][c], corner_product(wq, dy[u][c]));
            }
            if constexpr (DG)
              add_transform_grad<C>(val, w[u], dy[u], hR, ok[u], q[u].x, q[u].y, q[u].z, gacc);
          }
        }
      }
    float* out = a.CC + ((size_t)model * s.M + g) * 8 * ncell * C + cell * C;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c) out[q * ncell * C + c] = acc[q][c];
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

// The grid gradient without the transform gradient, one wave per 4 x 4 x 4 block of cells
// of one grid.  The wave takes the rows of the bins that overlap the block's box (the union
// of its cells' candidates, each point read once) 128 rows at a time and splits each batch's
// points, as one flat sequence, into 64 / G contiguous runs of equal length, one per group
// of G lanes.  At a step each group tests the next G points of its run against the block
// (lane i of the group the i-th), so the points of a step come from all over the block's box
// and few of them share a cell, while each group still reads G consecutive records.  A
// matching point's (w, dL/dy) products are handed to the lane that owns its cell through
// LDS, and each owner adds the records addressed to it in lane order.  Each cell's sum has a
// fixed order (step, then lane) set by the candidate sequence and G: bitwise reproducible,
// but not the plain candidate order of k_cell_pull.
constexpr int kBlk = 4;                      // cells per block edge
constexpr int kLat = (kBlk + 1) * (kBlk + 1) * (kBlk + 1);   // vertices of a block
constexpr int kRowBatch = 128;               // bin rows per batch (two per lane)
// DG: also the transform gradient of L_rec through the trilinear weights: every lane adds
// the terms of the records it produces (in step order) to its own 12 sums, reduced per
// workgroup in a fixed order into dGpart[model][g][group][12].
// TS = 2: the 4-D grids of Sec. 9, one pass per time cell ("model" index = time cell tc over
// one shared point array sorted by (time cell, bin); start = [tc][NB^3] positions in it, the
// records (x, y, z, t), dL/dy [M][n][C]); a point of cell tc adds (1 - wt) w_q dL/dy to the
// cell's slice-0 corners and wt w_q dL/dy to its slice-1 corners (time weight wt, Eq. (2)
// extended by linear interpolation in time), written as CC[tc][g][slice][8][cells][C].
template <int C, bool GF16, int G, bool DG, int TS = 1>
__global__ void __launch_bounds__(256) k_cell_pull_wave(CellArgs a) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8, "lanes per run");
  static_assert(TS == 1 || (TS == 2 && !DG), "the 4-D pass has no transform gradient");
  constexpr int NR = 64 / G;                 // runs per batch
  constexpr int RW = 2 * C * TS;             // float4 words per record: the 8 TS C products w_q dL/dy_c
  __shared__ float4 sRec[4][64][RW];
  __shared__ float sG[4][12];
  __shared__ uint32_t sRow0[4][kRowBatch];   // first sorted position of each row of the batch
  __shared__ uint32_t sPre[4][kRowBatch + 1];  // exclusive prefix of the rows' lengths; [kRowBatch] = total
  __shared__ double sDG[DG ? 4 : 1][12];
  // TS = 1: the block's (kBlk + 1)^3 vertex lattice, C values per vertex
  __shared__ float sLat[TS == 1 ? 4 : 1][TS == 1 ? kLat * C : 1];
  const Shape s = a.s;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R1 = s.R - 1;
  const int nbx = (R1 + kBlk - 1) / kBlk;
  const int64_t nblk_grid = (int64_t)nbx * nbx * nbx;            // cell blocks per grid
  const int64_t groups = (nblk_grid + 3) / 4;                   // 4 waves per workgroup
  const int64_t per_model = groups * s.M;
  const int64_t L = xcd_logical(blockIdx.x, gridDim.x);
  const int model = (int)(L / per_model);
  const int64_t grp = (L % per_model) / s.M;
  const int g = (int)(L % s.M);
  const int64_t cb = grp * 4 + wave;                            // this wave's cell block
  const bool act = (TS == 2 || !a.active || a.active[model]) && cb < nblk_grid;
  if (lane < 12) sG[wave][lane] = a.G[model * a.G_stride + 12 * g + lane];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const float* Gg = sG[wave];
  const int bx = (int)(cb % nbx), by = (int)((cb / nbx) % nbx), bz = (int)(cb / ((int64_t)nbx * nbx));
  const int cx = bx * kBlk + (lane & 3), cy = by * kBlk + ((lane >> 2) & 3), cz = bz * kBlk + (lane >> 4);
  const bool own = act && cx < R1 && cy < R1 && cz < R1;
  float acc[8 * TS][C];
#pragma unroll
  for (int q = 0; q < 8 * TS; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[q][c] = 0.f;
  float gacc[DG ? 12 : 1];
#pragma unroll
  for (int k = 0; k < (DG ? 12 : 1); ++k) gacc[k] = 0.f;
  if (act) {
    // the block's box in global space (inverse of Eq. (1) applied to its local box)
    double A[3][3];
    for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) A[r][c] = Gg[4 * r + c];
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1], c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    const double inv[9] = {c00, A[0][2] * A[2][1] - A[0][1] * A[2][2], A[0][1] * A[1][2] - A[0][2] * A[1][1],
                           c01, A[0][0] * A[2][2] - A[0][2] * A[2][0], A[0][2] * A[1][0] - A[0][0] * A[1][2],
                           c02, A[0][1] * A[2][0] - A[0][0] * A[2][1], A[0][0] * A[1][1] - A[0][1] * A[1][0]};
    bool bad = !(fabs(det) > 1e-30);
    float Ai[9];
    const double rdet = 1.0 / det;
    for (int k = 0; k < 9; ++k) { Ai[k] = (float)(inv[k] * rdet); bad = bad || !isfinite(Ai[k]); }
    int lo[3], hi[3];
    const int b0[3] = {bx * kBlk, by * kBlk, bz * kBlk};
    if (bad) {
      for (int d = 0; d < 3; ++d) { lo[d] = 0; hi[d] = kBinsPerAxis - 1; }
    } else {
      float lm[3], hl[3];
      for (int d = 0; d < 3; ++d) {
        const int e = min(b0[d] + kBlk, R1);
        lm[d] = -1.f + (float)(b0[d] + e) / R1 - Gg[4 * d + 3];   // box centre minus the translation
        hl[d] = (float)(e - b0[d]) / R1;                           // box half-width (local units)
      }
      for (int d = 0; d < 3; ++d) {
        const float wc = Ai[3 * d] * lm[0] + Ai[3 * d + 1] * lm[1] + Ai[3 * d + 2] * lm[2];
        const float hw = fabsf(Ai[3 * d]) * hl[0] + fabsf(Ai[3 * d + 1]) * hl[1] + fabsf(Ai[3 * d + 2]) * hl[2];
        const float f0 = floorf((wc - hw - 1e-4f + 1.f) * (0.5f * kBinsPerAxis));
        const float f1 = floorf((wc + hw + 1e-4f + 1.f) * (0.5f * kBinsPerAxis));
        lo[d] = (int)fminf(fmaxf(f0, 0.f), (float)(kBinsPerAxis - 1));
        hi[d] = (int)fminf(fmaxf(f1, 0.f), (float)(kBinsPerAxis - 1));
      }
    }
    constexpr size_t kNB3 = (size_t)kBinsPerAxis * kBinsPerAxis * kBinsPerAxis;
    const float4* P4 = TS == 1 ? a.pts4 + (size_t)model * a.n : a.pts4;
    const float* dY = a.dY + ((size_t)(TS == 1 ? model : 0) * s.M + g) * a.n * C;
    const uint32_t* start = a.start + (size_t)model * (TS == 1 ? kNB3 + 1 : kNB3);
    const float ht = 0.5f * (float)(a.Rt - 1);
    const float hR = 0.5f * (float)R1;
    const int ny_r = hi[1] - lo[1] + 1, nz_r = hi[2] - lo[2] + 1;
    const int nrows = ny_r * nz_r;
    double blo[3], bhi[3], ra[3];
    local_box(Gg, b0, kBlk, R1, blo, bhi);
    span_recips(Gg, ra);
    // A candidate: its point and dL/dy, loaded for every lane (a lane past the end of its run
    // loads point 0), so the loads of the next step are in flight while this one is used.
    struct Cand { float4 q; float dy[C]; bool valid; };
    // the lane's place in its run: flat index f (< fend), row r, sorted position p, and the
    // points left in row r from p on
    uint32_t f = 0, fend = 0, p = 0, rem = 0;
    int r = 0;
    auto load = [&](Cand& cd) {
      cd.valid = f < fend;
      const uint32_t pp = cd.valid ? p : 0u;
      cd.q = P4[pp];
#pragma unroll
      for (int c = 0; c < C; ++c) cd.dy[c] = dY[(size_t)pp * C + c];
      if (cd.valid) {
        f += G;
        if (f < fend) {                      // move G points on, across rows (the one holding f exists)
          uint32_t k = G;
          while (k >= rem) {
            k -= rem;
            do { ++r; } while (sPre[wave][r + 1] == sPre[wave][r]);
            p = sRow0[wave][r];
            rem = sPre[wave][r + 1] - sPre[wave][r];
          }
          p += k;
          rem -= k;
        }
      }
    };
    const void* Fm = GF16 ? (const void*)((const __half*)a.F + model * a.F_stride)
                          : (const void*)((const float*)a.F + model * a.F_stride);
    auto consume = [&](const Cand& cd) {
      int t = -1;
      float w[3] = {0.f, 0.f, 0.f};
      int i0[3] = {0, 0, 0};
      float wt = 0.f;
      if (cd.valid) {
        float l[3];
        local_coords(Gg, cd.q.x, cd.q.y, cd.q.z, l);
        bool in = cell_of(l, hR, s.R, i0, w);
        if constexpr (TS == 2) {
          // the time cell and weight as the 4-D lookup takes them; times outside [-1, 1] add nothing
          const float tq = cd.q.w;
          const float ut = __builtin_fmaf(tq, ht, ht);
          const float ft = fminf(fmaxf(floorf(ut), 0.0f), (float)(a.Rt - 2));
          in = in && tq >= -1.0f && tq <= 1.0f && (int)ft == model;
          wt = ut - ft;
        }
        const int ox = i0[0] - b0[0], oy = i0[1] - b0[1], oz = i0[2] - b0[2];
        if (in && ox >= 0 && ox < kBlk && oy >= 0 && oy < kBlk && oz >= 0 && oz < kBlk)
          t = (oz * kBlk + oy) * kBlk + ox;
      }
      if (t >= 0) {
        float pr[8 * TS * C];
#pragma unroll
        for (int sl = 0; sl < TS; ++sl)
#pragma unroll
          for (int qq = 0; qq < 8; ++qq) {
            const float wq = TS == 1 ? corner_weight(qq, w) : (sl ? wt : 1.f - wt) * corner_weight(qq, w);
#pragma unroll
            for (int c = 0; c < C; ++c) pr[(8 * sl + qq) * C + c] = corner_product(wq, cd.dy[c]);
          }
#pragma unroll
        for (int k = 0; k < RW; ++k)
          sRec[wave][lane][k] = make_float4(pr[4 * k], pr[4 * k + 1], pr[4 * k + 2], pr[4 * k + 3]);
        if constexpr (DG) {
          float val[8][C];
          gather_cell<C, GF16>(Fm, g, s.R, i0, val);
          add_transform_grad<C>(val, w, cd.dy, hR, true, cd.q.x, cd.q.y, cd.q.z, gacc);
        }
      }
      // lanes whose point falls in my cell: agree on every bit of the target
      const bool has = t >= 0;
      uint64_t mask = __ballot(has);
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const uint64_t bb = __ballot(has && ((t >> b) & 1));
        mask &= ((lane >> b) & 1) ? bb : ~bb;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      while (mask) {
        const int k = __builtin_ctzll(mask);
        mask &= mask - 1;
#pragma unroll
        for (int j4 = 0; j4 < RW; ++j4) {
          const float4 v = sRec[wave][k][j4];
          const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int idx = 4 * j4 + e;
            acc[idx / C][idx % C] = add_rounded(acc[idx / C][idx % C], vv[e]);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // rows (z outer, y inner) kRowBatch at a time; each batch's points are one flat sequence
    for (int rb = 0; rb < nrows; rb += kRowBatch) {
      uint32_t s0[2] = {0, 0}, len[2] = {0, 0};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int rr = rb + 2 * lane + k;
        int x0 = lo[0], x1 = hi[0];
        if (rr < nrows) {
          const int yb = lo[1] + rr % ny_r, zb = lo[2] + rr / ny_r;
          if (bad || row_x_span(Gg, ra, blo, bhi, lo[0], hi[0], yb, zb, x0, x1)) {
            const int row = (zb * kBinsPerAxis + yb) * kBinsPerAxis;
            s0[k] = start[row + x0];
            len[k] = start[row + x1 + 1] - s0[k];
          }
        }
      }
      uint32_t x = len[0] + len[1];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      const uint32_t total = __shfl(x, 63, 64);
      const uint32_t ex = x - len[0] - len[1];
      sRow0[wave][2 * lane] = s0[0];
      sRow0[wave][2 * lane + 1] = s0[1];
      sPre[wave][2 * lane] = ex;
      sPre[wave][2 * lane + 1] = ex + len[0];
      if (lane == 0) sPre[wave][kRowBatch] = total;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // runs of S points (a multiple of G; the last runs may be shorter), S / G steps
      const uint32_t S = ((total + NR - 1) / NR + G - 1) / G * G;
      const uint32_t f0 = min((uint32_t)(lane / G) * S, total);
      fend = min(f0 + S, total);
      f = f0 + (uint32_t)(lane % G);
      if (f < fend) {
        // the row holding f: the last row whose exclusive prefix is <= f (it is non-empty)
        r = 0;
#pragma unroll
        for (int step = kRowBatch / 2; step >= 1; step >>= 1)
          if (sPre[wave][r + step] <= f) r += step;
        p = sRow0[wave][r] + (f - sPre[wave][r]);
        rem = sPre[wave][r + 1] - f;
      }
      const uint32_t nsteps = S / G;
      Cand ca, cbn;
      load(ca);
      for (uint32_t st = 0; st < nsteps; st += 2) {
        load(cbn);
        sched_barrier();
        consume(ca);
        load(ca);
        sched_barrier();
        if (st + 1 < nsteps) consume(cbn);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if constexpr (TS == 1) {
    // the block's cells fold their corner sums into its vertex lattice: in phase q every
    // owner adds its corner q to vertex cell + offset(q), which no other cell of the block
    // addresses in that phase (a fixed order, no atomics); the lattice is written whole, and
    // k_block_to_vertex adds the lattices of the (up to 8) blocks that share a vertex
    float* lat = sLat[wave];
    for (int i = lane; i < kLat * C; i += 64) lat[i] = 0.f;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (own) {
        const int v = ((lz + (q >> 2)) * (kBlk + 1) + ly + ((q >> 1) & 1)) * (kBlk + 1) + lx + (q & 1);
#pragma unroll
        for (int c = 0; c < C; ++c) lat[v * C + c] = add_rounded(lat[v * C + c], acc[q][c]);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (act) {
      float* out = a.CC + (((size_t)model * s.M + g) * nblk_grid + cb) * kLat * C;
      for (int i = lane; i < kLat * C; i += 64) out[i] = lat[i];
    }
  } else if (own) {
    const int64_t cell = ((int64_t)cz * R1 + cy) * R1 + cx;
    const int64_t ncell = (int64_t)R1 * R1 * R1;
    float* out = a.CC + ((size_t)model * s.M + g) * 8 * TS * ncell * C + cell * C;
#pragma unroll
    for (int q = 0; q < 8 * TS; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c) out[q * ncell * C + c] = acc[q][c];
  }
  if constexpr (DG) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double t = wave_sum((double)gacc[k]);
      if (lane == 0) sDG[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
      const double t = sDG[0][threadIdx.x] + sDG[1][threadIdx.x] + sDG[2][threadIdx.x] + sDG[3][threadIdx.x];
      a.dGpart[(((size_t)model * s.M + g) * groups + grp) * 12 + threadIdx.x] = t;
    }
  }
}

// dF[model][g][v][c] (+)= sum over the cells adjacent to vertex v of their corner sums.
template <int C>
// dF in the paper's order [M][C][R^3] when paper != 0, else channel-last [M][R^3][C].
__global__ void k_cell_to_vertex(Shape s, const float* CC, float* dF, size_t dF_stride, int paper, int accumulate,
                                 const int32_t* active) {
  const int model = blockIdx.z, g = blockIdx.y;
  if (active && !active[model]) return;
  const int R = s.R, R1 = R - 1;
  const int64_t nv = (int64_t)R * R * R, ncell = (int64_t)R1 * R1 * R1;
  const float* cc = CC + ((size_t)model * s.M + g) * 8 * ncell * C;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    const int vx = (int)(v % R), vy = (int)((v / R) % R), vz = (int)(v / ((int64_t)R * R));
    float sum[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sum[c] = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int cx = vx - (q & 1), cy = vy - ((q >> 1) & 1), cz = vz - (q >> 2);
      if (cx < 0 || cy < 0 || cz < 0 || cx >= R1 || cy >= R1 || cz >= R1) continue;
      const float* src = cc + ((q * ncell + ((int64_t)cz * R1 + cy) * R1 + cx)) * C;   // neighbours read neighbours
#pragma unroll
      for (int c = 0; c < C; ++c) sum[c] += src[c];
    }
    float* dst = dF + model * dF_stride + (paper ? (size_t)g * C * nv + v : ((size_t)g * nv + v) * C);
    const size_t cs = paper ? (size_t)nv : 1;
#pragma unroll
    for (int c = 0; c < C; ++c) dst[c * cs] = accumulate ? dst[c * cs] + sum[c] : sum[c];
  }
}

// dF[model][g][v][c] (+)= sum over the cell blocks that contain vertex v of their lattice
// values (the dense wave gather's output, [model][M][blocks][kLat][C]; along each axis a
// vertex at a block boundary belongs to two blocks), in a fixed order.  dF layout as for
// k_cell_to_vertex.
template <int C>
__global__ void k_block_to_vertex(Shape s, const float* BL, float* dF, size_t dF_stride, int paper, int accumulate,
                                  const int32_t* active) {
  const int model = blockIdx.z, g = blockIdx.y;
  if (active && !active[model]) return;
  const int R = s.R, R1 = R - 1;
  const int nbx = (R1 + kBlk - 1) / kBlk;
  const int64_t nv = (int64_t)R * R * R;
  const float* bl = BL + ((size_t)model * s.M + g) * ((size_t)nbx * nbx * nbx) * kLat * C;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    const int vc[3] = {(int)(v % R), (int)((v / R) % R), (int)(v / ((int64_t)R * R))};
    int b0[3], nb[3];
    for (int d = 0; d < 3; ++d) {
      // blocks b with 0 <= vc - kBlk b <= kBlk: the lower one (vc on its upper face) first
      const int hi = min(vc[d] / kBlk, nbx - 1);
      b0[d] = (vc[d] % kBlk == 0 && vc[d] > 0 && hi == vc[d] / kBlk) ? hi - 1 : hi;
      nb[d] = hi - b0[d] + 1;
    }
    float sum[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sum[c] = 0.f;
    for (int iz = 0; iz < nb[2]; ++iz)
      for (int iy = 0; iy < nb[1]; ++iy)
        for (int ix = 0; ix < nb[0]; ++ix) {
          const int bx = b0[0] + ix, by = b0[1] + iy, bz = b0[2] + iz;
          const int lx = vc[0] - kBlk * bx, ly = vc[1] - kBlk * by, lz = vc[2] - kBlk * bz;
          const float* src = bl + (((size_t)(bz * nbx + by) * nbx + bx) * kLat +
                                   (lz * (kBlk + 1) + ly) * (kBlk + 1) + lx) * C;
#pragma unroll
          for (int c = 0; c < C; ++c) sum[c] += src[c];
        }
    float* dst = dF + model * dF_stride + (paper ? (size_t)g * C * nv + v : ((size_t)g * nv + v) * C);
    const size_t cs = paper ? (size_t)nv : 1;
#pragma unroll
    for (int c = 0; c < C; ++c) dst[c * cs] = accumulate ? dst[c * cs] + sum[c] : sum[c];
  }
}

// 4-D grids: dF[g][t][v][c] += the slice-0 corner sums of time cell t and the slice-1 corner
// sums of time cell t - 1 over the cells adjacent to vertex v (CC of the TS = 2 gather,
// dF channel-last [M][Rt][R^3][C]); a fixed order.
template <int C>
__global__ void k_cell_to_vertex_time(Shape s, int Rt, const float* CC, float* dF) {
  const int g = blockIdx.y, tv = blockIdx.z;
  const int R = s.R, R1 = R - 1;
  const int64_t nv = (int64_t)R * R * R, ncell = (int64_t)R1 * R1 * R1;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    const int vx = (int)(v % R), vy = (int)((v / R) % R), vz = (int)(v / ((int64_t)R * R));
    float sum[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sum[c] = 0.f;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int tc = tv - sl;
      if (tc < 0 || tc > Rt - 2) continue;
      const float* cc = CC + (((size_t)tc * s.M + g) * 16 + 8 * sl) * ncell * C;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int cx = vx - (q & 1), cy = vy - ((q >> 1) & 1), cz = vz - (q >> 2);
        if (cx < 0 || cy < 0 || cz < 0 || cx >= R1 || cy >= R1 || cz >= R1) continue;
        const float* src = cc + ((q * ncell + ((int64_t)cz * R1 + cy) * R1 + cx)) * C;
#pragma unroll
        for (int c = 0; c < C; ++c) sum[c] += src[c];
      }
    }
    float* dst = dF + (((size_t)g * Rt + tv) * nv + v) * C;
#pragma unroll
    for (int c = 0; c < C; ++c) dst[c] += sum[c];
  }
}

// dG[model][g][k] (+)= sum over the cb per-block partials of grid g: one workgroup per (grid,
// model); thread t sums blocks t, t + 256, ... in order, then a fixed tree over the threads.
// dG rows per transform: grows (3, or 4 with row 3 written as 0).
__global__ void __launch_bounds__(256) k_reduce_cell_dG(const double* part, int M, int cb, double* dG,
                                                        size_t dG_stride, int grows, int accumulate,
                                                        const int32_t* active) {
  __shared__ double sp[256][13];
  const int g = blockIdx.x, model = blockIdx.y;
  if (active && !active[model]) return;
  const double* P = part + ((size_t)model * M + g) * cb * 12;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < cb; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] += P[(size_t)b * 12 + k];
#pragma unroll
  for (int k = 0; k < 12; ++k) sp[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 12; ++k) sp[threadIdx.x][k] += sp[threadIdx.x + w][k];
    __syncthreads();
  }
  if (threadIdx.x < 12) {
    double* o = dG + model * dG_stride + 4 * grows * g + threadIdx.x;
    *o = accumulate ? *o + sp[0][threadIdx.x] : sp[0][threadIdx.x];
  } else if (grows == 4 && threadIdx.x < 16 && !accumulate) {
    dG[model * dG_stride + 4 * grows * g + threadIdx.x] = 0.0;
  }
}

}  // namespace apmg
