// Fused forward + adjoint tile kernel at two waves per SIMD (the shapes whose weight
// gradients fit in registers: hidden width 64, at most 64 input features).
//
// The MLP of Sec. 4.1.2 and its hand-derived backward pass, as in k_backward: a wave owns
// a tile of 32 points (lanes j and j+32 share point j and split the grids), recomputes the
// forward pass, back-propagates with the transposed weight swizzles and stores dL/dy per
// (grid, point) for the per-cell gather.  What differs is where the weight gradients
// dW2 = sum_p delta2_p h1_p^T and dW1 = sum_p delta1_p y_p^T accumulate.  Here a block has
// eight waves (two per SIMD, one block per compute unit), processes eight tiles per round,
// and every wave keeps a single 32 x 32 block of dW1 and of dW2 in registers (32
// accumulator registers instead of 128), summed over the points of other waves' tiles:
// each round the tiles' delta2 / h1 and then delta1 / y are published to LDS as
// [row][point] arrays, four tiles at a time, and each wave runs the matrix-core products
// of its blocks over its share of the published points.  The per-wave register budget
// (256 VGPR + AGPR) then allows two waves per SIMD, so one wave's gathers and vector work
// overlap the other's matrix products.

namespace apmg {

constexpr int kAdjPub = 4;                       // tiles published per sub-round
constexpr int kAdjPts = kAdjPub * 32;            // points per published set

// LDS arrays of published activations: [row][kAdjPts] with a padded pitch (float32: 130,
// so that 32 lanes reading 8 bytes of 32 consecutive rows hit 64 distinct banks; bf16: 136
// elements = 272 bytes, 16-byte aligned rows for 128-bit reads).
template <bool BF> struct AdjT {
  static constexpr int P = BF ? 136 : 130;
  typedef typename std::conditional<BF, uint16_t, float>::type T;
};

// Forward pass of one tile that also keeps the tile's features for the first-layer weight
// gradient: float32, yv[t] = feature hf * KH + t of this lane's point; bf16, the packed
// first-layer operands yb[st] (features 8 st .. 8 st + 7) and the packed second-layer
// operands hb[st] (h1 = relu(z1) in accumulator row order).  The grids of a half are
// unrolled at compile time (at most 32 features per half); gathers run PD - 1 grids ahead
// of the grid being interpolated.
template <int C, bool GF16, bool BF, int PD, int ENC = kEncDense>
__device__ inline void adj_fwd(const Shape& s, const float* sG, const void* F, const void* swz, const float* w3s,
                               float x, float y, float z, bool valid, int lane, f32x16 (&z1)[2], f32x16 (&z2)[2],
                               float& m, float (&yv)[32], bf16x8 (&yb)[4], bf16x8 (&hb)[4], const EncArgs& ea,
                               float tq) {
  constexpr int GMAX = 32 / C;
  constexpr int H = 64, NB = 2;
  const int hf = lane >> 5;
  const float hR = 0.5f * (float)(s.R - 1);
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) z1[b][r] = 0.f;
  if constexpr (!BF) {
#pragma unroll
    for (int t = 0; t < 32; ++t) yv[t] = 0.f;
  } else {
#pragma unroll
    for (int st = 0; st < 4; ++st) yb[st] = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  }
  GridTap<C, ENC> tp[PD];
  auto gidx = [&](int gi) { return gi < s.Mh ? hf * s.Mh + gi : s.M; };
#pragma unroll
  for (int q = 0; q < PD - 1; ++q) enc_tap<C, GF16, ENC>(s, sG, F, ea, gidx(q), x, y, z, tq, valid, hR, tp[q]);
  if constexpr (!BF) {
    const float* W1 = (const float*)swz;
#pragma unroll
    for (int gi = 0; gi < GMAX; ++gi) {
      if (gi < s.Mh) {
        if (gi + PD - 1 < GMAX) enc_tap<C, GF16, ENC>(s, sG, F, ea, gidx(gi + PD - 1), x, y, z, tq, valid, hR, tp[(gi + PD - 1) % PD]);
        sched_barrier();
        float e[C];
        enc_value<C, ENC>(tp[gi % PD], e);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int k = gi * C + c;
          yv[k] = e[c];
#pragma unroll
          for (int b = 0; b < NB; ++b) z1[b] = mma_f32(W1[(b * s.KHP + k) * 64 + lane], e[c], z1[b]);
        }
      }
    }
  } else {
    const bf16x8* W1 = (const bf16x8*)swz;
    constexpr int GPS = 8 / C;
    const int S1 = s.KHP / 8;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      if (st < S1) {
        float Bv[8];
#pragma unroll
        for (int u = 0; u < GPS; ++u) {
          const int gi = st * GPS + u;
          if (gi + PD - 1 < GMAX) enc_tap<C, GF16, ENC>(s, sG, F, ea, gidx(gi + PD - 1), x, y, z, tq, valid, hR, tp[(gi + PD - 1) % PD]);
          sched_barrier();
          float e[C];
          enc_value<C, ENC>(tp[gi % PD], e);
#pragma unroll
          for (int c = 0; c < C; ++c) Bv[u * C + c] = e[c];
        }
        const bf16x8 B = bf16_pack8(Bv);
        yb[st] = B;
#pragma unroll
        for (int b = 0; b < NB; ++b) z1[b] = mma_bf16(W1[(b * S1 + st) * 64 + lane], B, z1[b]);
      }
    }
  }
  // second layer
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) z2[b][r] = 0.f;
  if constexpr (!BF) {
    const float* W2 = (const float*)swz + (size_t)2 * H * s.KHP;
#pragma unroll
    for (int st = 0; st < H / 2; ++st) {
      const float hv = fmaxf(z1[st >> 4][st & 15], 0.f);
#pragma unroll
      for (int b = 0; b < NB; ++b) z2[b] = mma_f32(W2[((size_t)b * (H / 2) + st) * 64 + lane], hv, z2[b]);
      if ((st & 7) == 7) sched_fence();
    }
  } else {
    const bf16x8* W2 = (const bf16x8*)((const uint16_t*)swz + (size_t)2 * H * s.KHP);
#pragma unroll
    for (int st = 0; st < H / 16; ++st) {
      float Bv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) Bv[e] = fmaxf(z1[st >> 1][8 * (st & 1) + e], 0.f);
      const bf16x8 B = bf16_pack8(Bv);
      hb[st] = B;
#pragma unroll
      for (int b = 0; b < NB; ++b) z2[b] = mma_bf16(W2[((size_t)b * (H / 16) + st) * 64 + lane], B, z2[b]);
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc = __builtin_fmaf(w3s[hf * (H / 2) + 16 * b + r], fmaxf(z2[b][r], 0.f), acc);
  m = acc + __shfl_xor(acc, 32, 64);
}

// acc += A[arow .. arow+32) x B[brow .. brow+32)^T over the published points [p0, p0+len)
// (len a multiple of 16).  float32: each lane reads two consecutive points per row (the
// points of two matrix steps: step 2t takes point p0+4t+2h for k = h, step 2t+1 the next
// one -- the same assignment for A and B, so every point enters once).
template <bool BF>
__device__ inline f32x16 adj_dw(const typename AdjT<BF>::T* A, int arow, const typename AdjT<BF>::T* B, int brow,
                                int p0, int len, int lane, f32x16 acc) {
  constexpr int P = AdjT<BF>::P;
  const int li = lane & 31, h = lane >> 5;
  if constexpr (!BF) {
    const float* pa = A + (size_t)(arow + li) * P + p0 + 2 * h;
    const float* pb = B + (size_t)(brow + li) * P + p0 + 2 * h;
    for (int t = 0; t < len / 4; ++t) {
      const f32x2a4 av = *(const f32x2a4*)(pa + 4 * t), bv = *(const f32x2a4*)(pb + 4 * t);
      acc = mma_f32(av.x, bv.x, acc);
      acc = mma_f32(av.y, bv.y, acc);
    }
  } else {
    const uint16_t* pa = A + (size_t)(arow + li) * P + p0 + 8 * h;
    const uint16_t* pb = B + (size_t)(brow + li) * P + p0 + 8 * h;
    for (int t = 0; t < len / 16; ++t)
      acc = mma_bf16(*(const bf16x8*)(pa + 16 * t), *(const bf16x8*)(pb + 16 * t), acc);
  }
  return acc;
}

template <bool BF>
__device__ inline void adj_put(typename AdjT<BF>::T* T, int row, int col, float v) {
  if constexpr (BF) T[(size_t)row * AdjT<BF>::P + col] = bf16_bits(v);
  else T[(size_t)row * AdjT<BF>::P + col] = v;
}

// NW waves per block: 8 (one block per compute unit, two sub-rounds of four published
// tiles per round) or 4 (two blocks per compute unit when the LDS allows it -- bf16 --,
// one sub-round per round; the two blocks' barriers are independent, so the two waves of a
// SIMD drift into different phases).  The swizzled weights are staged in LDS.  (Measured
// at the headline workload: a deeper gather prefetch, PD = 3, changes nothing; float32
// weights read from global memory instead of LDS, to fit two four-wave blocks per CU,
// take twice as long.)
// KF > 0: an even number of feature grids and exactly KF features per half (KF = 16 or 32);
// the shape is then a compile-time constant (for the hash encoder all but its levels per
// grid) and the per-grid bounds tests of the unrolled loops fold away (otherwise their
// uniform outcomes are held in scalar registers).  KF = 0: the shape as given.
template <int C, bool GF16, bool BF, int NW, int ENC = kEncDense, int KF = 0>
__global__ void __launch_bounds__(NW * kWave, 8 / NW) k_adjoint(TileArgs a) {
  extern __shared__ float smem[];
  typedef typename AdjT<BF>::T TT_;
  constexpr int P = AdjT<BF>::P;
  constexpr int H = 64, NB = 2;
  constexpr int PD = 2;
  constexpr int kAdjWaves = NW;
  constexpr int NSUB = NW / kAdjPub;
  // logical block as in k_backward (partials indexed by it, in tile order)
  const int64_t lbl = xcd_logical(blockIdx.x + (int64_t)gridDim.x * blockIdx.y, (int64_t)gridDim.x * gridDim.y);
  const int model = (int)(lbl / gridDim.x), lb = (int)(lbl % gridDim.x);
  Shape s = a.s;
  if constexpr (KF > 0) {
    static_assert(KF == 16 || KF == 32, "fixed halves");
    s.C = C; s.H = H; s.M = 2 * KF / C; s.Mh = KF / C; s.KH = KF; s.KHP = KF; s.MC = 2 * KF;
    if constexpr (ENC != kEncHash) s.L = 1;
  }
  const PartLayout pl = part_layout(s, s.MC, H);
  double* part = a.part + ((size_t)model * gridDim.x + lb) * pl.len;
  const bool act = !a.active || a.active[model];

  // LDS: sG [12M] | sW3w [wave][H] | sLoss [wave] | swizzled weights | TD, TY [64][P]
  // (the cross-wave weight-gradient sums alias TD/TY at the end)
  const size_t esz = BF ? 2 : 4;
  const size_t wbytes = swz_sizes(s).total() * esz;
  char* lbase = (char*)smem;
  float* sG = smem;
  float* sW3w = sG + 12 * s.M;
  size_t off = (size_t)(12 * s.M + kAdjWaves * H) * 4;
  off = (off + 7) & ~(size_t)7;
  double* sLoss = (double*)(lbase + off);
  off = (off + 8 * kAdjWaves + 15) & ~(size_t)15;
  char* lw = lbase + off;
  TT_* TD = (TT_*)(lbase + off + wbytes);
  TT_* TY = TD + (size_t)64 * P;
  float* red = (float*)TD;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 31, hf = lane >> 5;
  const float* G = a.G + model * a.G_stride;
  for (int i = threadIdx.x; i < 12 * (s.M / s.L); i += blockDim.x) sG[i] = G[i];
  for (int i = threadIdx.x; i < kAdjWaves * H; i += blockDim.x) sW3w[i] = 0.f;
  const void* F = GF16 ? (const void*)((const __half*)a.F + model * a.F_stride)
                       : (const void*)((const float*)a.F + model * a.F_stride);
  block_copy16(lw, (const char*)a.swz + esz * model * a.swz_stride, wbytes);
  __syncthreads();
  const void* swz = lw;
  const float* w3s = a.w3s + (size_t)model * H;
  const float vs = a.bscale ? a.bscale[model] : a.vscale;
  const float vo = a.boff ? a.boff[model] : a.voff;
  const float* Pp = a.pts + model * a.pts_stride;
  float* dY = a.dY ? a.dY + (size_t)model * s.M * a.n * C : nullptr;
  const size_t o2t = (size_t)2 * H * s.KHP + (size_t)H * H, o1t = o2t + (size_t)H * H;
  // a model's dL/dy below 2 GiB is stored through a buffer resource (32-bit offsets)
  const size_t dy_bytes = (size_t)s.M * a.n * C * 4;
  const bool dy_buf = dY && dy_bytes < ((size_t)1 << 31);
  const __amdgpu_buffer_rsrc_t dy_rsrc =
      __builtin_amdgcn_make_buffer_rsrc(dY, (short)0, dy_buf ? (int)dy_bytes : 0, kBufferRsrcWord3);
  const int dy_grid = dy_buf ? (int)(a.n * C * 4) : 0;   // bytes per grid

  // this wave's weight-gradient blocks: dW2 block (ib2, kb2) over published points
  // [k2len part2, +k2len); dW1 block (ib1, kb1) over [k1len part1, +k1len)
  const int nkb1 = (s.MC + 31) / 32;
  const int B1 = 2 * nkb1, S1 = kAdjWaves / B1, k1len = kAdjPts / S1;
  const int b1 = wave % B1, part1 = wave / B1, ib1 = b1 / nkb1, kb1 = b1 % nkb1;
  constexpr int S2 = kAdjWaves / 4, k2len = kAdjPts / S2;
  const int b2 = wave & 3, part2 = wave >> 2, ib2 = b2 >> 1, kb2 = b2 & 1;
  f32x16 acc1, acc2;
#pragma unroll
  for (int r = 0; r < 16; ++r) { acc1[r] = 0.f; acc2[r] = 0.f; }
  double loss = 0.0;
  const int nblk = s.KHP / 16;

  const int64_t ntiles = act ? (a.n + 31) / 32 : 0;
  const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int64_t t_beg = lb * per, t_end = min(ntiles, (lb + 1) * per);
  for (int64_t rbase = t_beg; rbase < t_end; rbase += kAdjWaves) {
    const float* W2T = BF ? nullptr : (const float*)swz + o2t;
    const float* W1T = BF ? nullptr : (const float*)swz + o1t;
    const bf16x8* W2Tb = BF ? (const bf16x8*)((const uint16_t*)swz + o2t) : nullptr;
    const bf16x8* W1Tb = BF ? (const bf16x8*)((const uint16_t*)swz + o1t) : nullptr;
    const int64_t tile = rbase + wave;
    const int64_t p = tile * 32 + j;
    const bool valid = tile < t_end && p < a.n;
    const int dy_lane = dy_buf ? (int)(((int64_t)hf * s.Mh * a.n + p) * C * 4) : 0;
    float x = 0.f, y = 0.f, z = 0.f, tq = 0.f;
    if (valid) { x = Pp[p]; y = Pp[a.ld + p]; z = Pp[2 * a.ld + p]; }
    if constexpr (ENC == kEncTime) tq = valid ? a.tau[p] : 0.f;
    f32x16 z1[NB], z2[NB];
    float m;
    float yv[32];
    bf16x8 yb[4], hb[4];
    adj_fwd<C, GF16, BF, PD, ENC>(s, sG, F, swz, w3s, x, y, z, valid, lane, z1, z2, m, yv, yb, hb, a.enc, tq);

    float df = 0.f;
    if (valid) {
      if (a.df) {
        df = a.df[p];
      } else {
        const float fv = __builtin_fmaf(m, vs, vo);
        const float e = fv - a.v[model * a.v_stride + p];
        df = 2.0f * e / (float)a.n;
        if (lane < 32) {
          a.err[model * a.err_stride + p] = a.err_abs ? fabsf(e) : e * e;
          loss += (double)e * (double)e;
        }
      }
    }
    const float dm = df * vs;

    // output layer gradient (transposing butterfly over the half's 32 points, as in
    // k_backward; lanes 0..15 of each half own one row of the wave's LDS row)
    if (a.do_w3) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        float v[8];
        const bool up8 = (j & 8) != 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float lo = dm * fmaxf(z2[b][i], 0.f), hi = dm * fmaxf(z2[b][i + 8], 0.f);
          v[i] = (up8 ? hi : lo) + __shfl_xor(up8 ? lo : hi, 8, 64);
        }
#pragma unroll
        for (int mm = 8; mm > 1; mm >>= 1) {
          const int o = mm >> 1;
          const bool up = (j & o) != 0;
#pragma unroll
          for (int i = 0; i < mm / 2; ++i) {
            const float keep = up ? v[i + mm / 2] : v[i];
            const float send = up ? v[i] : v[i + mm / 2];
            v[i] = keep + __shfl_xor(send, o, 64);
          }
        }
        const float tot = v[0] + __shfl_xor(v[0], 16, 64);
        if (j < 16) sW3w[wave * H + 32 * b + acc_row(j, hf)] += tot;
      }
    }
    f32x16 d2[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) d2[b][r] = z2[b][r] > 0.f ? w3s[hf * (H / 2) + 16 * b + r] * dm : 0.f;
    // bf16: the packed operands stand in for delta2, h1, delta1 and y from here on (the
    // published values are bf16 as well); the ReLU pattern of z1 is kept as a bit mask
    bf16x8 d2b[4], d1b[4];
    uint32_t zmask = 0;
    if constexpr (BF) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        float Bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) Bv[e] = d2[st >> 1][8 * (st & 1) + e];
        d2b[st] = bf16_pack8(Bv);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) zmask |= (z1[b][r] > 0.f ? 1u : 0u) << (16 * b + r);
    }

    // delta1 = (W2^T delta2) * [z1 > 0]
    f32x16 d1[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) d1[b][r] = 0.f;
    if constexpr (!BF) {
#pragma unroll
      for (int st = 0; st < H / 2; ++st) {
        const float dv = d2[st >> 4][st & 15];
#pragma unroll
        for (int b = 0; b < NB; ++b) d1[b] = mma_f32(W2T[((size_t)b * (H / 2) + st) * 64 + lane], dv, d1[b]);
        if ((st & 7) == 7) sched_fence();
      }
    } else {
#pragma unroll
      for (int st = 0; st < H / 16; ++st) {
#pragma unroll
        for (int b = 0; b < NB; ++b) d1[b] = mma_bf16(W2Tb[((size_t)b * (H / 16) + st) * 64 + lane], d2b[st], d1[b]);
      }
    }
    if constexpr (!BF) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) d1[b][r] = z1[b][r] > 0.f ? d1[b][r] : 0.f;
    } else {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        float Bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int b = st >> 1, r = 8 * (st & 1) + e;
          Bv[e] = ((zmask >> (16 * b + r)) & 1u) ? d1[b][r] : 0.f;
        }
        d1b[st] = bf16_pack8(Bv);
      }
    }

    // dL/dy per block of 16 features of each half, stored per grid for the cell gather
    if (dY) {
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        if (blk < nblk) {
          f32x16 dy;
#pragma unroll
          for (int r = 0; r < 16; ++r) dy[r] = 0.f;
          if constexpr (!BF) {
#pragma unroll
            for (int st = 0; st < H / 2; ++st) {
              dy = mma_f32(W1T[((size_t)blk * (H / 2) + st) * 64 + lane], d1[st >> 4][st & 15], dy);
              if ((st & 7) == 7) sched_fence();
            }
          } else {
#pragma unroll
            for (int st = 0; st < H / 16; ++st) dy = mma_bf16(W1Tb[((size_t)blk * (H / 16) + st) * 64 + lane], d1b[st], dy);
          }
#pragma unroll
          for (int u = 0; u < 16 / C; ++u) {
            const int gi = 16 * blk / C + u;
            const int g = hf * s.Mh + gi;
            if (valid && gi < s.Mh && g < s.M) {
              if (dy_buf) {
                // byte offset = lane part (this half's first grid, this point) + a uniform
                // per-grid part: no 64-bit address per grid is held across the tile (the
                // builtin takes the value's bits as an unsigned integer)
#pragma unroll
                for (int c = 0; c < C; ++c)
                  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(dy[u * C + c]), dy_rsrc, dy_lane + 4 * c, gi * dy_grid, 0);
              } else {
                // (the grid index is opaque here, so its 64-bit offset is formed at the store
                // instead of being hoisted out of the tile loop and held, or spilled)
                int gl = g;
                asm volatile("" : "+v"(gl));
                float* dst = dY + ((size_t)gl * a.n + p) * C;
#pragma unroll
                for (int c = 0; c < C; ++c) dst[c] = dy[u * C + c];
              }
            }
          }
        }
      }
    }

    // weight gradients: NSUB sub-rounds, each publishing four tiles (waves 4 sub .. 4 sub + 3)
    const int slot = wave & 3;
#pragma unroll 1
    for (int sub = 0; sub < NSUB; ++sub) {
      const bool pub = (wave >> 2) == sub;
      if (pub) {
        if constexpr (!BF) {
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              adj_put<BF>(TD, 32 * b + acc_row(r, hf), 32 * slot + j, d2[b][r]);
              adj_put<BF>(TY, 32 * b + acc_row(r, hf), 32 * slot + j, fmaxf(z1[b][r], 0.f));
            }
        } else {
#pragma unroll
          for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int row = 32 * (st >> 1) + acc_row(8 * (st & 1) + e, hf);
              TD[(size_t)row * P + 32 * slot + j] = (uint16_t)d2b[st][e];
              TY[(size_t)row * P + 32 * slot + j] = (uint16_t)hb[st][e];
            }
        }
      }
      __syncthreads();
      acc2 = adj_dw<BF>(TD, 32 * ib2, TY, 32 * kb2, k2len * part2, k2len, lane, acc2);
      __syncthreads();
      if (pub) {
        if constexpr (!BF) {
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) adj_put<BF>(TD, 32 * b + acc_row(r, hf), 32 * slot + j, d1[b][r]);
#pragma unroll
          for (int t = 0; t < 32; ++t) {
            const int k = hf * s.KH + t;
            if (t < s.KH && k < s.MC) adj_put<BF>(TY, k, 32 * slot + j, yv[t]);
          }
        } else {
#pragma unroll
          for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int row = 32 * (st >> 1) + acc_row(8 * (st & 1) + e, hf);
              TD[(size_t)row * P + 32 * slot + j] = (uint16_t)d1b[st][e];
              const int t = 8 * st + e, k = hf * s.KH + t;
              if (t < s.KH && k < s.MC) TY[(size_t)k * P + 32 * slot + j] = (uint16_t)yb[st][e];
            }
        }
      }
      __syncthreads();
      acc1 = adj_dw<BF>(TD, 32 * ib1, TY, 32 * kb1, k1len * part1, k1len, lane, acc1);
      __syncthreads();
    }
  }

  // block partials: dW1 [H][MC] then dW2 [H][H] summed over the waves in a fixed order
  float* sW1 = red;
  float* sW2 = red + H * s.MC;
  for (int i = threadIdx.x; i < H * s.MC + H * H; i += blockDim.x) red[i] = 0.f;
  for (int w = 0; w < kAdjWaves; ++w) {
    __syncthreads();
    if (wave != w) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row2 = 32 * ib2 + acc_row(r, hf), col2 = 32 * kb2 + j;
      sW2[row2 * H + col2] += acc2[r];
      const int row1 = 32 * ib1 + acc_row(r, hf), col1 = 32 * kb1 + j;
      if (col1 < s.MC) sW1[row1 * s.MC + col1] += acc1[r];
    }
  }
  if (a.want_loss) {
    const double t = wave_sum(loss);
    if (lane == 0) sLoss[wave] = t;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < H * s.MC; i += blockDim.x) part[pl.o_w1 + i] = sW1[i];
  for (int i = threadIdx.x; i < H * H; i += blockDim.x) part[pl.o_w2 + i] = sW2[i];
  if (a.do_w3)
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
      double t = 0.0;
      for (int w = 0; w < kAdjWaves; ++w) t += (double)sW3w[w * H + i];
      part[pl.o_w3 + i] = t;
    }
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kAdjWaves; ++w) t += a.want_loss ? sLoss[w] : 0.0;
    part[pl.o_loss] = t;
  }
}

// LDS bytes of k_adjoint with nw waves per block.
size_t adjoint_lds_bytes(const Shape& s, bool bf, int nw) {
  size_t b = (size_t)(12 * s.M + nw * s.H) * 4;
  b = (b + 7) & ~(size_t)7;
  b += 8 * nw;
  b = (b + 15) & ~(size_t)15;
  const size_t esz = bf ? 2 : 4;
  b += swz_sizes(s).total() * esz;
  const size_t tbytes = (size_t)2 * 64 * (bf ? AdjT<true>::P : AdjT<false>::P) * esz;
  const size_t red = (size_t)(s.H * s.MC + s.H * s.H) * 4;
  b += std::max(tbytes, red);
  return b;
}

// The tiled adjoint applies to the register-resident shapes: hidden width 64 and at most
// 64 input features (two blocks of 16 per half).
bool adjoint_applies(const Shape& s) { return s.H == 64 && s.KHP <= 32; }

// waves per block of the tiled adjoint: variant 1 = eight, 2 = four, 0 = the faster one
// measured for the MLP dtype (eight for float32, whose 64 KB of staged weights leave room
// for one block per CU; four for bf16, two blocks per CU).
int adjoint_waves(int variant, bool bf) { return variant == 1 ? 8 : variant == 2 ? 4 : (bf ? 4 : 8); }

hipError_t launch_adjoint(const TileArgs& a, bool grid_f16, bool mlp_bf16, int variant, dim3 grid, hipStream_t st) {
  if (!adjoint_applies(a.s)) return hipErrorInvalidValue;
  const int nw = adjoint_waves(variant, mlp_bf16);
  const size_t shmem = adjoint_lds_bytes(a.s, mlp_bf16, nw);
  const int kf = (a.s.L == 1 && a.s.M % 2 == 0) ? (a.s.MC == 64 ? 32 : a.s.MC == 32 ? 16 : 0) : 0;
#define APMG_ADJ_K(CC, G16, B16, KF_)                                                                              \
  if (nw == 4) hipLaunchKernelGGL((k_adjoint<CC, G16, B16, 4, kEncDense, KF_>), grid, dim3(4 * kWave), shmem, st, a); \
  else hipLaunchKernelGGL((k_adjoint<CC, G16, B16, 8, kEncDense, KF_>), grid, dim3(8 * kWave), shmem, st, a);
#define APMG_ADJ_V(CC, G16, B16)                                                                                   \
  if (kf == 32) { APMG_ADJ_K(CC, G16, B16, 32) }                                                                  \
  else if (kf == 16) { APMG_ADJ_K(CC, G16, B16, 16) }                                                             \
  else { APMG_ADJ_K(CC, G16, B16, 0) }
#define APMG_ADJ(CC)                                                                                              \
  if (a.s.C == CC) {                                                                                              \
    if (!grid_f16 && !mlp_bf16) { APMG_ADJ_V(CC, false, false) }                                                  \
    else if (!grid_f16 && mlp_bf16) { APMG_ADJ_V(CC, false, true) }                                               \
    else if (grid_f16 && !mlp_bf16) { APMG_ADJ_V(CC, true, false) }                                               \
    else { APMG_ADJ_V(CC, true, true) }                                                                           \
    return hipGetLastError();                                                                                     \
  }
  APMG_ADJ(1)
  APMG_ADJ(2)
  APMG_ADJ(4)
#undef APMG_ADJ
#undef APMG_ADJ_V
#undef APMG_ADJ_K
  return hipErrorInvalidValue;
}

}  // namespace apmg
