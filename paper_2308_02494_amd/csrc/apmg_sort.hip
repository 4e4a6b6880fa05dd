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
constexpr int kSortThreads = 512;         // threads per block of the histogram / scatter kernels
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortRounds = kSortTile / kSortThreads;

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

// The input points of the sort: SoA [3][ld] at model * pts_stride, or, when pts4 is set,
// (x, y, z, _) records [model][n].
struct SortIn {
  const float* pts; int64_t ld; size_t pts_stride;
  const float4* pts4;
  __device__ inline void get(int model, int64_t n, int64_t i, float& x, float& y, float& z) const {
    if (pts4) {
      const float4 q = pts4[model * n + i];
      x = q.x; y = q.y; z = q.z;
    } else {
      const float* P = pts + model * pts_stride;
      x = P[i]; y = P[ld + i]; z = P[2 * ld + i];
    }
  }
};

// keys[model][i] = bin of point i, vals = i.
__global__ void k_bin_keys(SortIn in, int64_t n, uint32_t* keys, uint32_t* vals) {
  const int model = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float x, y, z;
    in.get(model, n, i, x, y, z);
    keys[model * n + i] = bin_of(x, y, z);
    vals[model * n + i] = (uint32_t)i;
  }
}

// Digit histogram per tile: hist[model][digit][tile].
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t* keys, int64_t n, int shift, uint32_t* hist,
                                                    int ntiles) {
  __shared__ uint32_t h[kRadixDigits];
  const int model = blockIdx.y, tile = blockIdx.x;
  for (int d = threadIdx.x; d < kRadixDigits; d += blockDim.x) h[d] = 0;
  __syncthreads();
  const uint32_t* K = keys + model * n;
  const int64_t base = (int64_t)tile * kSortTile;
  uint32_t kk[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    kk[r] = i < n ? K[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r)
    if (base + r * kSortThreads + threadIdx.x < n) atomicAdd(&h[(kk[r] >> shift) & (kRadixDigits - 1)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < kRadixDigits; d += blockDim.x)
    hist[((size_t)model * kRadixDigits + d) * ntiles + tile] = h[d];
}

// Exclusive scan of a 256-thread block's values; *total gets the block sum.
__device__ inline uint32_t block_excl_scan256(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint32_t pre = 0;
  for (int w = 0; w < wave; ++w) pre += wsum[w];
  *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  return pre + x - v;
}

// The digit-major, tile-minor exclusive scan of hist[model][digit][tile] in two steps:
// each row (digit) is scanned in place and its total kept, then the totals are scanned
// into dbase[model][digit]; the scatter adds the two.  Rows: grid (digits, models).
__global__ void __launch_bounds__(256) k_radix_rowscan(uint32_t* hist, int ntiles, uint32_t* rowtot) {
  const int model = blockIdx.y, d = blockIdx.x;
  uint32_t* H = hist + ((size_t)model * kRadixDigits + d) * ntiles;
  uint32_t carry = 0;
  for (int base = 0; base < ntiles; base += 256) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < ntiles ? H[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(v, &tot);
    if (i < ntiles) H[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) rowtot[(size_t)model * kRadixDigits + d] = carry;
}

__global__ void __launch_bounds__(256) k_radix_digitscan(const uint32_t* rowtot, uint32_t* dbase) {
  const int model = blockIdx.x;
  uint32_t carry = 0;
  for (int base = 0; base < kRadixDigits; base += 256) {
    const int d = base + threadIdx.x;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(rowtot[(size_t)model * kRadixDigits + d], &tot);
    dbase[(size_t)model * kRadixDigits + d] = carry + ex;
    carry += tot;
  }
}

// Stable scatter of one radix pass.  A block ranks its tile's keys among equal digits in
// index order (rounds of kSortThreads keys; within a round by wave, then lane), places them in LDS in
// digit order, and writes each digit's run of keys to consecutive output positions: stores
// of neighbouring threads land side by side instead of one word per digit bucket.
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                                                       uint32_t* vout, int64_t n, int shift, const uint32_t* offs,
                                                       const uint32_t* dbase, int ntiles) {
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];
  __shared__ uint32_t lcount[kRadixDigits];   // keys of each digit ranked so far, then the digit's first slot
  __shared__ uint32_t gbase[kRadixDigits];    // output position of the tile's first key of each digit
  __shared__ uint32_t wcnt[kSortWaves][kRadixDigits];  // keys of each digit in each wave of the current round
  __shared__ uint32_t wsum[kSortWaves];
  const int model = blockIdx.y, tile = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t* Kin = kin + model * n;
  const uint32_t* Vin = vin + model * n;
  uint32_t* Kout = kout + model * n;
  uint32_t* Vout = vout + model * n;
  for (int d = threadIdx.x; d < kRadixDigits; d += blockDim.x) {
    gbase[d] = offs[((size_t)model * kRadixDigits + d) * ntiles + tile] + dbase[(size_t)model * kRadixDigits + d];
    lcount[d] = 0;
  }
  for (int d = threadIdx.x; d < kSortWaves * kRadixDigits; d += blockDim.x) (&wcnt[0][0])[d] = 0;
  const int64_t base = (int64_t)tile * kSortTile;
  const int tn = (int)min((int64_t)kSortTile, n - base);   // keys in this tile
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t key[kSortRounds], val[kSortRounds], rk[kSortRounds];
  // every load of the tile is issued before the first barrier (one wait, not one per round)
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int e = r * kSortThreads + threadIdx.x;
    key[r] = e < tn ? Kin[base + e] : 0u;
    val[r] = e < tn ? Vin[base + e] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int e = r * kSortThreads + threadIdx.x;
    const bool valid = e < tn;
    const uint32_t dig = valid ? (key[r] >> shift) & (kRadixDigits - 1) : 0u;
    // lanes of this wave with the same digit (and valid)
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
      uint32_t q = lcount[dig] + rank;
      for (int w = 0; w < wave; ++w) q += wcnt[w][dig];
      rk[r] = q;
    }
    __syncthreads();
    // every rank is taken: the first lane of each (wave, digit) group adds its group to the
    // digit's count and clears the group's entry for the next round (only this wave writes it)
    if (valid && rank == 0) {
      atomicAdd(&lcount[dig], wcnt[wave][dig]);
      wcnt[wave][dig] = 0;
    }
  }
  __syncthreads();
  // exclusive scan of the digit counts: the first LDS slot of each digit (one digit a thread)
  static_assert(kSortThreads == kRadixDigits, "one digit per thread in the scan");
  {
    const uint32_t c0 = lcount[threadIdx.x];
    uint32_t x = c0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    lcount[threadIdx.x] = pre + x - c0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int e = r * kSortThreads + threadIdx.x;
    if (e < tn) {
      const uint32_t dig = (key[r] >> shift) & (kRadixDigits - 1);
      const uint32_t slot = lcount[dig] + rk[r];
      sk[slot] = key[r];
      sv[slot] = val[r];
    }
  }
  __syncthreads();
  // slot e holds the (e - first slot of its digit)-th key of that digit in index order
  for (int e = threadIdx.x; e < tn; e += kSortThreads) {
    const uint32_t k = sk[e];
    const uint32_t dig = (k >> shift) & (kRadixDigits - 1);
    const uint32_t pos = gbase[dig] + ((uint32_t)e - lcount[dig]);
    Kout[pos] = k;
    Vout[pos] = sv[e];
  }
}

// start[model][b] = first sorted position with key >= b, for b in [0, NB^3]: position i
// (0 < i < n) starts the bins (key[i-1], key[i]], position 0 the bins [0, key[0]] and the
// end n the bins (key[n-1], NB^3]; every bin is written exactly once.
__global__ void k_bin_starts(const uint32_t* keys, int64_t n, uint32_t* start) {
  const int model = blockIdx.y;
  const uint32_t nbins = (uint32_t)kBinsPerAxis * kBinsPerAxis * kBinsPerAxis;
  const uint32_t* K = keys + model * n;
  uint32_t* S = start + (size_t)model * (nbins + 1);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t lo = i == 0 ? 0u : K[i - 1] + 1u;       // first bin this position starts
    const uint32_t hi = i == n ? nbins : K[i];              // last bin this position starts
    for (uint32_t b = lo; b <= hi; ++b) S[b] = (uint32_t)i;
  }
}

// The same bin starts with one thread per bin: start[b] = the first position whose key is
// >= b (n if none), by binary search over the sorted keys.  Balanced where the points leave
// large runs of bins empty (the per-position kernel then has a few threads writing long
// gaps); used for large point sets.
__global__ void k_bin_starts_search(const uint32_t* keys, int64_t n, uint32_t* start) {
  const int model = blockIdx.y;
  const uint32_t nbins = (uint32_t)kBinsPerAxis * kBinsPerAxis * kBinsPerAxis;
  const uint32_t* K = keys + model * n;
  uint32_t* S = start + (size_t)model * (nbins + 1);
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b <= (int64_t)nbins;
       b += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;                 // first index in [lo, hi) with K >= b
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (K[mid] < (uint32_t)b) lo = mid + 1;
      else hi = mid;
    }
    S[b] = (uint32_t)lo;
  }
}

// The training batch's sort keys straight from the counter stream: point i of every model
// is generated and binned (the points themselves are not stored; they are regenerated in
// sorted order below).  Model b draws from stream stream0 + b.
__global__ void k_batch_keys(uint64_t seed, const uint64_t* step_ctr, uint32_t stream0, int64_t n, uint32_t* keys,
                             uint32_t* vals) {
  const int model = blockIdx.y;
  const uint64_t step = *step_ctr;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float x, y, z;
    uniform_point(seed, step, stream0 + (uint32_t)model, (uint64_t)i, x, y, z);
    keys[model * n + i] = bin_of(x, y, z);
    vals[model * n + i] = (uint32_t)i;
  }
}

// Sorted position j of every model gets point perm[j] regenerated from the counter stream
// (the same bits as at key time), written as [model][3][n] and (x, y, z, 0) records, and
// the ground truth there: a trilinear sample of the model's brick (extended extent e0..e1).
__global__ void k_batch_sorted(uint64_t seed, const uint64_t* step_ctr, uint32_t stream0, int64_t n, const uint32_t* perm, float* out,
                               float4* out4, const float* vol, int vnx, int vny, const apmg_brick* bricks, float* v) {
  const int model = blockIdx.y;
  const uint64_t step = *step_ctr;
  const apmg_brick br = bricks[model];
  const int e0[3] = {br.e0[0], br.e0[1], br.e0[2]};
  const int nn[3] = {br.e1[0] - br.e0[0] + 1, br.e1[1] - br.e0[1] + 1, br.e1[2] - br.e0[2] + 1};
  float* O = out + (size_t)model * 3 * n;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    float x, y, z;
    uniform_point(seed, step, stream0 + (uint32_t)model, (uint64_t)perm[model * n + j], x, y, z);
    O[j] = x; O[n + j] = y; O[2 * n + j] = z;
    out4[model * n + j] = make_float4(x, y, z, 0.f);
    v[(size_t)model * n + j] = sample_volume(vol, vnx, vny, e0, nn, x, y, z);
  }
}

// out[model][3][n] = points in sorted order (perm = sorted vals), also as (x, y, z, 0) records
// in out4[model][n]; optional per-point float arrays permuted alongside (src_f[perm[j]] -> dst_f[j]).
__global__ void k_permute_points(SortIn in, int64_t n, const uint32_t* perm, float* out, float4* out4,
                                 const float* src_f, float* dst_f) {
  const int model = blockIdx.y;
  float* O = out + (size_t)model * 3 * n;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t i = perm[model * n + j];
    float x, y, z;
    in.get(model, n, i, x, y, z);
    O[j] = x; O[n + j] = y; O[2 * n + j] = z;
    if (out4) out4[model * n + j] = make_float4(x, y, z, 0.f);
    if (src_f) dst_f[model * n + j] = src_f[model * n + i];
  }
}

}  // namespace apmg
