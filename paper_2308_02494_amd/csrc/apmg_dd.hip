// Global-query inference over a domain decomposition (Sec. 5.3).  Each global
// point is hashed to its brick, mapped into that brick model's local frame, and
// the points are grouped by brick (a stable radix sort on the brick id) so that
// one launch of the forward tile kernel evaluates every brick's points with its
// own model (block row = brick, the points a contiguous segment); the outputs
// are scattered back to the input order.

namespace apmg {

// Brick of global point (x, y, z): the voxel coordinate u = fma(p, h, h),
// h = (n-1)/2, selects the base brick holding floor(u), clamped to the grid.
__device__ inline int brick_of(const apmg_brick_table& t, const float p[3]) {
  int idx[3];
  for (int d = 0; d < 3; ++d) {
    const float h = 0.5f * (float)(t.vol[d] - 1);
    float u = __builtin_fmaf(p[d], h, h);
    if (!(fabsf(u) <= 3.0e38f)) u = 0.f;  // a non-finite coordinate goes to brick 0 on that axis
    const float fl = fminf(fmaxf(floorf(u), 0.f), (float)t.vol[d]);
    const int k = (int)fl / t.B;
    idx[d] = k < t.dims[d] - 1 ? k : t.dims[d] - 1;
  }
  return idx[0] + t.dims[0] * (idx[1] + t.dims[1] * idx[2]);
}

// keys[i] = brick of point i, vals[i] = i.
__global__ void k_dd_keys(apmg_brick_table t, const float* pts, int64_t ld, int64_t n, uint32_t* keys,
                          uint32_t* vals) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float p[3] = {pts[i], pts[ld + i], pts[2 * ld + i]};
    keys[i] = (uint32_t)brick_of(t, p);
    vals[i] = (uint32_t)i;
  }
}

// Sorted point j (input point perm[j], brick keys[j]) in its brick model's local frame,
// the inverse of the training map u = e0 + (l + 1)/2 (e1 - e0):
//   l = fma(u - e0, 2 / (e1 - e0), -1), u = fma(p, h, h), each operation rounded once.
__global__ void k_dd_local(const float* pts, int64_t ld, int64_t n, const uint32_t* keys, const uint32_t* perm,
                           const apmg_brick* bricks, apmg_brick_table t, float* out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t i = perm[j];
    const apmg_brick br = bricks[keys[j]];
    for (int d = 0; d < 3; ++d) {
      const float h = 0.5f * (float)(t.vol[d] - 1);
      const float u = __builtin_fmaf(pts[d * ld + i], h, h);
      const int span = br.e1[d] - br.e0[d];
      const float sc = span > 0 ? __fdiv_rn(2.0f, (float)span) : 0.0f;
      out[d * n + j] = __builtin_fmaf(u - (float)br.e0[d], sc, -1.0f);
    }
  }
}

// start[b] = first sorted position with key >= b, b in [0, nseg]; binary search.
__global__ void k_seg_starts(const uint32_t* keys, int64_t n, int nseg, uint32_t* start) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nseg; b += gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < (uint32_t)b) lo = mid + 1; else hi = mid;
    }
    start[b] = (uint32_t)lo;
  }
}

// f[perm[j]] = fs[j].
__global__ void k_dd_scatter(const float* fs, const uint32_t* perm, int64_t n, float* f) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    f[perm[j]] = fs[j];
}

}  // namespace apmg
