// Spatial binning of a batch of points: a stable LSD radix sort of the points
// of every model by bin index (NB^3 bins over [-1, 1]^3, x fastest), then the
// first sorted position of every bin.  The order makes the per-point grid
// gathers of a wave hit neighbouring cells, and lets the grid-gradient pass
// visit, for each cell, only the points of the bins its footprint overlaps.
// Ties keep the generation order, so the sort and every sum taken over the
// sorted points are deterministic.

namespace apmg {

constexpr int kBinsPerAxis = 64;          // NB
constexpr int kBinBits = 18;              // 3 * log2(NB)
constexpr int kRadixBits = 9;
constexpr int kRadixDigits = 1 << kRadixBits;
constexpr int kSortTile = 4096;           // keys per block of the histogram / scatter kernels

// Bin index of a point; coordinates outside [-1, 1) clamp to the edge bins, NaN to 0.
__device__ inline uint32_t bin_of(float x, float y, float z) {
  const float p[3] = {x, y, z};
  uint32_t b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float u = floorf((p[d] + 1.0f) * (0.5f * kBinsPerAxis));
    b[d] = (uint32_t)fminf(fmaxf(u, 0.0f), (float)(kBinsPerAxis - 1));  // NaN -> 0
  }
  return (b[2] * kBinsPerAxis + b[1]) * kBinsPerAxis + b[0];
}

// keys[model][i] = bin of point i, vals = i.  pts SoA per model: [3][ld] at model * pts_stride.
__global__ void k_bin_keys(const float* pts, int64_t ld, size_t pts_stride, int64_t n, uint32_t* keys,
                           uint32_t* vals) {
  const int model = blockIdx.y;
  const float* P = pts + model * pts_stride;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    keys[model * n + i] = bin_of(P[i], P[ld + i], P[2 * ld + i]);
    vals[model * n + i] = (uint32_t)i;
  }
}

// Digit histogram per tile: hist[model][digit][tile].
__global__ void __launch_bounds__(256) k_radix_hist(const uint32_t* keys, int64_t n, int shift, uint32_t* hist,
                                                    int ntiles) {
  __shared__ uint32_t h[kRadixDigits];
  const int model = blockIdx.y, tile = blockIdx.x;
  for (int d = threadIdx.x; d < kRadixDigits; d += blockDim.x) h[d] = 0;
  __syncthreads();
  const uint32_t* K = keys + model * n;
  const int64_t base = (int64_t)tile * kSortTile;
  for (int k = threadIdx.x; k < kSortTile; k += blockDim.x) {
    const int64_t i = base + k;
    if (i < n) atomicAdd(&h[(K[i] >> shift) & (kRadixDigits - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadixDigits; d += blockDim.x)
    hist[((size_t)model * kRadixDigits + d) * ntiles + tile] = h[d];
}

// Exclusive scan of hist[model][*] (digit-major, tile-minor) in place; one block per model.
__global__ void __launch_bounds__(1024) k_radix_scan(uint32_t* hist, int len) {
  __shared__ uint32_t part[1024];
  uint32_t* H = hist + (size_t)blockIdx.x * len;
  const int per = (len + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per, hi = min(len, lo + per);
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) s += H[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {  // inclusive Hillis-Steele
    const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int i = lo; i < hi; ++i) {
    const uint32_t v = H[i];
    H[i] = run;
    run += v;
  }
}

// Stable scatter of one radix pass.  Each block walks its tile in rounds of 256
// keys in index order; within a round, lanes are ranked by wave (wave order) and
// by lane (lane order) among keys with the same digit.
__global__ void __launch_bounds__(256) k_radix_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                                                       uint32_t* vout, int64_t n, int shift, const uint32_t* offs,
                                                       int ntiles) {
  __shared__ uint32_t running[kRadixDigits];
  __shared__ uint32_t wcnt[4][kRadixDigits];
  const int model = blockIdx.y, tile = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t* Kin = kin + model * n;
  const uint32_t* Vin = vin + model * n;
  uint32_t* Kout = kout + model * n;
  uint32_t* Vout = vout + model * n;
  for (int d = threadIdx.x; d < kRadixDigits; d += blockDim.x)
    running[d] = offs[((size_t)model * kRadixDigits + d) * ntiles + tile];
  const int64_t base = (int64_t)tile * kSortTile;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kSortTile / 256; ++r) {
    for (int d = threadIdx.x; d < 4 * kRadixDigits; d += blockDim.x) (&wcnt[0][0])[d] = 0;
    __syncthreads();
    const int64_t i = base + r * 256 + threadIdx.x;
    const bool valid = i < n;
    uint32_t key = 0, val = 0, dig = 0;
    if (valid) { key = Kin[i]; val = Vin[i]; dig = (key >> shift) & (kRadixDigits - 1); }
    // lanes with the same digit (and valid)
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const uint64_t bal = __ballot(valid && ((dig >> b) & 1));
      same &= ((dig >> b) & 1) ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt_mask);
    if (valid && rank == 0) wcnt[wave][dig] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = running[dig] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dig];
      Kout[pos] = key;
      Vout[pos] = val;
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadixDigits; d += blockDim.x)
      running[d] += wcnt[0][d] + wcnt[1][d] + wcnt[2][d] + wcnt[3][d];
    __syncthreads();
  }
}

// start[model][b] = first sorted position with key >= b, for b in [0, NB^3]; binary search.
__global__ void k_bin_starts(const uint32_t* keys, int64_t n, uint32_t* start) {
  const int model = blockIdx.y;
  const uint32_t nbins = (uint32_t)kBinsPerAxis * kBinsPerAxis * kBinsPerAxis;
  const uint32_t* K = keys + model * n;
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b <= nbins; b += gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (K[mid] < b) lo = mid + 1; else hi = mid;
    }
    start[(size_t)model * (nbins + 1) + b] = (uint32_t)lo;
  }
}

// out[model][3][n] = points in sorted order (perm = sorted vals); optional per-point
// float arrays permuted alongside (src_f[perm[j]] -> dst_f[j]).
__global__ void k_permute_points(const float* pts, int64_t ld, size_t pts_stride, int64_t n, const uint32_t* perm,
                                 float* out, const float* src_f, float* dst_f) {
  const int model = blockIdx.y;
  const float* P = pts + model * pts_stride;
  float* O = out + (size_t)model * 3 * n;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t i = perm[model * n + j];
    O[j] = P[i]; O[n + j] = P[ld + i]; O[2 * n + j] = P[2 * ld + i];
    if (src_f) dst_f[model * n + j] = src_f[model * n + i];
  }
}

}  // namespace apmg
