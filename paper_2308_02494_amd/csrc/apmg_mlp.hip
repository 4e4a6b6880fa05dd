// Encoder + decoder forward and adjoint kernels (Sec. 4.1, Eqs. (1)-(3),
// the bias-free MLP of Sec. 4.1.2 and its hand-derived backward pass).
//
// Work decomposition: a wave processes a tile of 32 points.  Point j = lane%32
// is shared by lanes j and j+32 ("halves"); half hf encodes grids
// [hf*Mh, hf*Mh+Mh).  The per-grid features are produced in registers and fed
// straight into the first layer's matrix product as the B operand of
// v_mfma_f32_32x32x2_f32 (fp32) or v_mfma_f32_32x32x16_bf16 (bf16): the
// 32x32x2 B operand wants feature k of point j in lane j+32k, the bf16 one
// 8 consecutive features per lane half, which is exactly one point per lane
// pair with the two halves holding different features.  Every hidden layer's
// accumulator layout (rows 8(r/4)+4hf+r%4 of each 32-row block in register r)
// is reused as the next layer's B operand; the weights are pre-swizzled so
// the A operand row/k order matches.  Nothing but the transforms goes to LDS
// in the forward pass.
//
// The adjoint (k_backward here; the tiled k_adjoint in apmg_adjoint.hip for the
// register-resident shapes) recomputes the forward pass per tile,
// back-propagates through the MLP with the transposed swizzles, stores dL/dy
// per (grid, point) for the per-cell gather of the grid gradient, and forms
// the weight gradients as matrix products over the tile's points after an LDS
// transpose (or stores the activations for k_dw_gemm).

namespace apmg {

// ------------------------------------------------------------------ swizzle
// Source weights per model: W1 [H][MC], W2 [H][H], W3 [H] at W + model*wstride.
// Output per model at swz + model*swz_stride elements: [w1 | w2 | w2t | w1t]
// (float or bf16 bits) and w3s + model*H (float, [hf][H/2] row order).
__device__ inline int feat_of_half(const Shape& s, int hf, int t) {
  if (t >= s.KH) return -1;
  int k = hf * s.KH + t;
  return k < s.MC ? k : -1;
}

template <bool BF>
__global__ void k_swizzle(Shape s, const float* __restrict__ W1all, const float* __restrict__ W2all,
                          const float* __restrict__ W3all, size_t wstride, void* swz,
                          size_t swz_stride, float* w3s) {
  const int model = blockIdx.y;
  const float* W1 = W1all + model * wstride;
  const float* W2 = W2all + model * wstride;
  const float* W3 = W3all + model * wstride;
  const SwzSizes z = swz_sizes(s);
  const size_t total = z.total() + (size_t)s.H;
  const int H = s.H;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    size_t o = idx;
    if (o < z.w1) {
      int l, e = 0, b, st;
      if (!BF) { l = o % 64; size_t q = o / 64; st = q % s.KHP; b = q / s.KHP; }
      else { e = o % 8; l = (o / 8) % 64; size_t q = o / 512; st = q % (s.KHP / 8); b = q / (s.KHP / 8); }
      int t = BF ? 8 * st + e : st;
      int k = feat_of_half(s, l >> 5, t);
      v = k >= 0 ? W1[(size_t)(32 * b + (l & 31)) * s.MC + k] : 0.f;
    } else if ((o -= z.w1) < z.w2 + z.w2t) {
      bool tr = o >= z.w2;
      if (tr) o -= z.w2;
      int l, e = 0, b, st, row;
      if (!BF) { l = o % 64; size_t q = o / 64; st = q % (H / 2); b = q / (H / 2);
                 row = 32 * (st >> 4) + acc_row(st & 15, l >> 5); }
      else { e = o % 8; l = (o / 8) % 64; size_t q = o / 512; st = q % (H / 16); b = q / (H / 16);
             row = 32 * (st >> 1) + acc_row(8 * (st & 1) + e, l >> 5); }
      int col = 32 * b + (l & 31);
      v = tr ? W2[(size_t)row * H + col] : W2[(size_t)col * H + row];
    } else if ((o -= z.w2 + z.w2t) < z.w1t) {
      int l, e = 0, b, st, row;
      if (!BF) { l = o % 64; size_t q = o / 64; st = q % (H / 2); b = q / (H / 2);
                 row = 32 * (st >> 4) + acc_row(st & 15, l >> 5); }
      else { e = o % 8; l = (o / 8) % 64; size_t q = o / 512; st = q % (H / 16); b = q / (H / 16);
             row = 32 * (st >> 1) + acc_row(8 * (st & 1) + e, l >> 5); }
      int p = l & 31, hfp = (p >> 2) & 1, rp = 4 * (p >> 3) + (p & 3);
      int k = feat_of_half(s, hfp, 16 * b + rp);
      v = k >= 0 ? W1[(size_t)row * s.MC + k] : 0.f;
    } else {
      o -= z.w1t;  // w3s: [hf][bb*16 + r] = W3[32bb + acc_row(r, hf)]
      int hf = o / (H / 2), rr = o % (H / 2);
      w3s[(size_t)model * H + o] = W3[32 * (rr >> 4) + acc_row(rr & 15, hf)];
      continue;
    }
    if (BF) ((uint16_t*)swz)[model * swz_stride + idx] = bf16_bits(v);
    else ((float*)swz)[model * swz_stride + idx] = v;
  }
}

// ------------------------------------------------------------------ tile pieces
// LDS transpose tiles: [row][32 points], row stride LDT elements.
template <bool BF> struct TT {
  static constexpr int LDT = BF ? 40 : 33;
  typedef typename std::conditional<BF, uint16_t, float>::type T;
};

// One 32-point tile's block of stored activations (rows x 32 points, float32 or bf16) behind
// a buffer resource based at the block's row row0: a store's row offset is then a constant or
// uniform operand of the instruction, not a 64-bit address per row held in registers across
// the tile.  Row row0 + vrow + srow of point j: vrow may differ per lane, srow is uniform.
template <bool BF>
struct ActTile {
  static constexpr int kEsz = BF ? 2 : 4, kRowBytes = 32 * kEsz;
  __amdgpu_buffer_rsrc_t rsrc;
  int lane_off;   // j * element size
  __device__ inline ActTile(void* block, int row0, int rows, int j)
      : rsrc(__builtin_amdgcn_make_buffer_rsrc((char*)block + (size_t)row0 * kRowBytes, (short)0,
                                               (rows - row0) * kRowBytes, kBufferRsrcWord3)),
        lane_off(j * kEsz) {}
  __device__ inline void put(int vrow, int srow, float v) const {
    // (the builtins take the value's bits as an unsigned integer)
    if constexpr (BF)
      __builtin_amdgcn_raw_buffer_store_b16(bf16_bits(v), rsrc, lane_off + vrow * kRowBytes, srow * kRowBytes, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rsrc, lane_off + vrow * kRowBytes,
                                            srow * kRowBytes, 0);
  }
};

template <bool BF>
__device__ inline void tt_put(typename TT<BF>::T* t, int row, int j, float v) {
  if constexpr (BF) t[row * TT<BF>::LDT + j] = bf16_bits(v);
  else t[row * TT<BF>::LDT + j] = v;
}

// One grid's contribution split in two so the gathers of the next grid can be in flight
// while this one is consumed: grid_tap issues the 8 corner loads (always from a valid
// address: cell 0 of grid 0 when the point is outside, invalid or past the last grid),
// grid_tap_value interpolates and applies the Eq. (2) mask.
template <int C, int ENC = kEncDense> struct GridTap {
  float w[3];
  float val[8][C];
  bool in;
};
// 4-D grids: the corners of the two time slices and the time offset
template <int C> struct GridTap<C, kEncTime> {
  float w[3];
  float wt;
  float va[8][C], vb[8][C];
  bool in;
};

template <int C, bool GF16>
__device__ inline void grid_tap(const Shape& s, const float* sG, const void* F, int g, float x, float y, float z,
                                bool valid, float hR, GridTap<C>& t) {
  const bool gok = valid && g < s.M;
  const int gg = gok ? g : 0;
  float l[3];
  local_coords(sG + 12 * gg, x, y, z, l);
  int i0[3];
  t.in = cell_of(l, hR, s.R, i0, t.w) && gok;
#pragma unroll
  for (int d = 0; d < 3; ++d) i0[d] = t.in ? i0[d] : 0;
  gather_cell<C, GF16>(F, gg, s.R, i0, t.val);
}

template <int C>
__device__ inline void grid_tap_value(const GridTap<C>& t, float e[C]) {
  trilerp<C>(t.val, t.w, e);
#pragma unroll
  for (int c = 0; c < C; ++c) e[c] = t.in ? e[c] : 0.f;
}

// Entry of vertex (vx, vy, vz) of a hash level with n1 = N + 1 vertices per axis: one entry
// per vertex while the level's n1^3 vertices fit the table (x fastest), else the spatial hash
// of Mueller et al. 2022 (coordinates times 1, 2654435761 and 805459861, XOR, mod 2^32),
// masked to the table size.
__device__ inline uint32_t hash_entry(uint32_t vx, uint32_t vy, uint32_t vz, uint32_t n1, bool dense, uint32_t tmask) {
  return dense ? vx + n1 * (vy + n1 * vz) : ((vx ^ (vy * 2654435761u) ^ (vz * 805459861u)) & tmask);
}

// The lookup of feature grid g for the encoder variants.  Hash (Sec. 9 (1)): the local point of
// transform g / L (Eq. (1)), the mask of Eq. (2), the cell of level k = g % L at N_k cells per
// axis (u = fma(l, N_k/2, N_k/2), as a dense grid with R - 1 = N_k), and the C features of its 8
// corner entries in table g.  Time (Sec. 9 (2)): the spatial cell of Eq. (2), the time cell
// u_t = fma(t, (Rt-1)/2, (Rt-1)/2) (lower vertex clamped to [0, Rt-2]; a time outside [-1, 1]
// masks the grid), and the corners of the two time slices.  Every load reads a valid address.
template <int C, bool GF16, int ENC>
__device__ inline void enc_tap(const Shape& s, const float* sG, const void* F, const EncArgs& ea, int g, float x,
                               float y, float z, float tq, bool valid, float hR, GridTap<C, ENC>& t) {
  if constexpr (ENC == kEncDense) {
    grid_tap<C, GF16>(s, sG, F, g, x, y, z, valid, hR, t);
  } else if constexpr (ENC == kEncHash) {
    const bool gok = valid && g < s.M;
    const int gg = gok ? g : 0;
    const int gt = gg / s.L, k = gg - gt * s.L;
    const int N = enc_level_res(ea, k);
    float l[3];
    local_coords(sG + 12 * gt, x, y, z, l);
    int i0[3];
    t.in = cell_of(l, 0.5f * (float)N, N + 1, i0, t.w) && gok;
#pragma unroll
    for (int d = 0; d < 3; ++d) i0[d] = t.in ? i0[d] : 0;
    const uint32_t n1 = (uint32_t)N + 1u;
    const bool dense = (uint64_t)n1 * n1 * n1 <= (uint64_t)ea.tmask + 1u;
    const float* base = (const float*)F + (size_t)gg * ((size_t)ea.tmask + 1u) * C;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint32_t ent = hash_entry((uint32_t)i0[0] + (q & 1), (uint32_t)i0[1] + ((q >> 1) & 1),
                                      (uint32_t)i0[2] + (q >> 2), n1, dense, ea.tmask);
      const float* p = base + (size_t)ent * C;
      if constexpr (C == 1) {
        t.val[q][0] = p[0];
      } else if constexpr (C == 2) {
        const f32x2a4 v = *(const f32x2a4*)p;
        t.val[q][0] = v.x; t.val[q][1] = v.y;
      } else {
        const f32x4 v = *(const f32x4*)p;
        t.val[q][0] = v.x; t.val[q][1] = v.y; t.val[q][2] = v.z; t.val[q][3] = v.w;
      }
    }
  } else {
    const bool gok = valid && g < s.M;
    const int gg = gok ? g : 0;
    float l[3];
    local_coords(sG + 12 * gg, x, y, z, l);
    int i0[3];
    bool in = cell_of(l, hR, s.R, i0, t.w);
    const float ht = 0.5f * (float)(ea.Rt - 1);
    const float ut = __builtin_fmaf(tq, ht, ht);
    const float ft = fminf(fmaxf(floorf(ut), 0.0f), (float)(ea.Rt - 2));   // NaN -> 0 via fmaxf
    t.in = in && (tq >= -1.0f) && (tq <= 1.0f) && gok;
    t.wt = ut - ft;
    const int t0 = t.in ? (int)ft : 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) i0[d] = t.in ? i0[d] : 0;
    gather_cell<C, false>(F, gg * ea.Rt + t0, s.R, i0, t.va);
    gather_cell<C, false>(F, gg * ea.Rt + t0 + 1, s.R, i0, t.vb);
  }
}

template <int C, int ENC>
__device__ inline void enc_value(const GridTap<C, ENC>& t, float e[C]) {
  if constexpr (ENC != kEncTime) {
    trilerp<C>(t.val, t.w, e);
  } else {
    float e0[C], e1[C];
    trilerp<C>(t.va, t.w, e0);
    trilerp<C>(t.vb, t.w, e1);
#pragma unroll
    for (int c = 0; c < C; ++c) e[c] = __builtin_fmaf(t.wt, e1[c] - e0[c], e0[c]);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) e[c] = t.in ? e[c] : 0.f;
}

// Forward pass of one 32-point tile.  With STY, the features are also written to the
// LDS tile Ty in dy-block order: feature t of half hf goes to row 32 (t/16) + 16 hf + t%16.
template <int C, int H, bool GF16, bool BF, bool STY = false, int ENC = kEncDense>
__device__ inline void tile_fwd(const Shape& s, const float* sG, const void* F, const void* swz,
                                const float* w3s, float x, float y, float z, bool valid, int lane,
                                f32x16 (&z1)[H / 32], f32x16 (&z2)[H / 32], float& m,
                                typename TT<BF>::T* Ty = nullptr, const ActTile<BF>* yact = nullptr,
                                EncArgs ea = {}, float tq = 0.f) {
  constexpr int NB = H / 32;
  const int hf = lane >> 5;
  const float hR = 0.5f * (float)(s.R - 1);
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) z1[b][r] = 0.f;
  // grid gi of this half is g = hf * Mh + gi.  Its gathers are issued one grid ahead into
  // two alternating taps (no register copies); every tap load is unconditional (a zero tap
  // past the last grid), so the loads stay in straight-line code and each grid waits only
  // for its own.
  GridTap<C, ENC> ta, tb;
  auto gidx = [&](int gi) { return gi < s.Mh ? hf * s.Mh + gi : s.M; };
  enc_tap<C, GF16, ENC>(s, sG, F, ea, gidx(0), x, y, z, tq, valid, hR, ta);
  if constexpr (!BF) {
    const float* W1 = (const float*)swz;
    auto consume = [&](const GridTap<C, ENC>& t, int gi) {
      float e[C];
      enc_value<C, ENC>(t, e);
      if (yact && hf * s.Mh + gi < s.M) {
#pragma unroll
        for (int c = 0; c < C; ++c) yact->put(hf * s.Mh * C, gi * C + c, e[c]);
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int k = gi * C + c;
        if constexpr (STY) tt_put<BF>(Ty, 32 * (k >> 4) + 16 * hf + (k & 15), lane & 31, e[c]);
#pragma unroll
        for (int b = 0; b < NB; ++b) z1[b] = mma_f32(W1[(b * s.KHP + k) * 64 + lane], e[c], z1[b]);
      }
    };
    for (int gi = 0; gi < s.Mh; gi += 2) {
      enc_tap<C, GF16, ENC>(s, sG, F, ea, gidx(gi + 1), x, y, z, tq, valid, hR, tb);
      sched_barrier();   // keep the loads ahead of the consumer (no sinking under register pressure)
      consume(ta, gi);
      enc_tap<C, GF16, ENC>(s, sG, F, ea, gidx(gi + 2), x, y, z, tq, valid, hR, ta);
      sched_barrier();
      if (gi + 1 < s.Mh) consume(tb, gi + 1);
    }
  } else {
    const bf16x8* W1 = (const bf16x8*)swz;
    constexpr int GPS = 8 / C;   // grids per 8-feature operand step (even for C = 1, 2, 4)
    const int S1 = s.KHP / 8;
    for (int st = 0; st < S1; ++st) {
      float Bv[8];
#pragma unroll
      for (int u = 0; u < GPS; ++u) {
        const int gi = st * GPS + u;
        GridTap<C, ENC>& cur = (u & 1) ? tb : ta;
        GridTap<C, ENC>& nxt = (u & 1) ? ta : tb;
        enc_tap<C, GF16, ENC>(s, sG, F, ea, gidx(gi + 1), x, y, z, tq, valid, hR, nxt);
        sched_barrier();
        float e[C];
        enc_value<C, ENC>(cur, e);
        if (yact && gi < s.Mh && hf * s.Mh + gi < s.M) {
#pragma unroll
          for (int c = 0; c < C; ++c) yact->put(hf * s.Mh * C, gi * C + c, e[c]);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
          Bv[u * C + c] = e[c];
          const int t = 8 * st + u * C + c;
          if constexpr (STY) tt_put<BF>(Ty, 32 * (t >> 4) + 16 * hf + (t & 15), lane & 31, e[c]);
        }
      }
      const bf16x8 B = bf16_pack8(Bv);
#pragma unroll
      for (int b = 0; b < NB; ++b) z1[b] = mma_bf16(W1[(b * S1 + st) * 64 + lane], B, z1[b]);
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
#pragma unroll
      for (int b = 0; b < NB; ++b) z2[b] = mma_bf16(W2[((size_t)b * (H / 16) + st) * 64 + lane], B, z2[b]);
    }
  }
  // output layer (H -> 1) on the vector ALUs
  float acc = 0.f;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc = __builtin_fmaf(w3s[hf * (H / 2) + 16 * b + r], fmaxf(z2[b][r], 0.f), acc);
  m = acc + __shfl_xor(acc, 32, 64);
}

// ------------------------------------------------------------------ forward
// Copies `bytes` (a multiple of 16) from global memory to LDS with the whole block.
__device__ inline void block_copy16(void* dst, const void* src, size_t bytes) {
  const u32x4a8* s = (const u32x4a8*)src;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4* d = (u32x4*)dst;
  for (size_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

// Bytes of the swizzled first and second layer (the forward pass's operands).
__host__ __device__ inline size_t fwd_weight_bytes(const Shape& s, bool bf) {
  const SwzSizes z = swz_sizes(s);
  return (z.w1 + z.w2) * (bf ? 2 : 4);
}

// WL: the swizzled weights are staged in LDS (after the transforms).
// NWF waves per block: 4, or 8 where the staged weights are so large that one block fills a
// CU's LDS (then eight waves share them, two per SIMD, instead of one; measured on the 64-grid
// 256-128-128-1 BF16 model: 8.06 -> 6.14 ms per 16.6 M-point frame; twelve waves, three per
// SIMD, 6.26 ms).
template <int C, int H, bool GF16, bool BF, bool WL, int ENC = kEncDense, int NWF = kWavesPerBlock>
__global__ void __launch_bounds__(NWF * kWave) k_forward(TileArgs a) {
  extern __shared__ float smem[];
  // logical block: models in order, each model's blocks over contiguous runs of its
  // (spatially sorted) tiles, dealt to the XCDs in slabs
  const int64_t lbl = xcd_logical(blockIdx.x + (int64_t)gridDim.x * blockIdx.y, (int64_t)gridDim.x * gridDim.y);
  const int model = (int)(lbl / gridDim.x), lb = (int)(lbl % gridDim.x);
  if (a.active && !a.active[model]) return;
  const Shape s = a.s;
  float* sG = smem;
  const float* G = a.G + model * a.G_stride;
  for (int i = threadIdx.x; i < 12 * (s.M / s.L); i += blockDim.x) sG[i] = G[i];
  const void* F = GF16 ? (const void*)((const __half*)a.F + model * a.F_stride)
                       : (const void*)((const float*)a.F + model * a.F_stride);
  const size_t esz = BF ? 2 : 4;
  const void* swz = (const char*)a.swz + esz * model * a.swz_stride;
  if constexpr (WL) {
    // byte offsets from the LDS base keep the pointer in the LDS address space
    char* lw = (char*)smem + ((12 * s.M * 4 + 15) & ~15);
    block_copy16(lw, swz, fwd_weight_bytes(s, BF));
    swz = lw;
  }
  __syncthreads();
  const float* w3s = a.w3s + (size_t)model * H;
  const float vs = a.bscale ? a.bscale[model] : a.vscale;
  const float vo = a.boff ? a.boff[model] : a.voff;
  // points of this model: [model * pts_stride, + n) of its own arrays, or, with segments,
  // [seg[model], seg[model + 1]) of one shared array (outputs at the same positions)
  const int64_t base = a.seg ? (int64_t)a.seg[model] : 0;
  const int64_t cnt = a.seg ? (int64_t)a.seg[model + 1] - base : a.n;
  const float* P = a.seg ? a.pts + base : a.pts + model * a.pts_stride;
  float* fo = a.seg ? a.f + base : a.f + (size_t)model * a.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 31;
  const int64_t ntiles = (cnt + 31) / 32;
  const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int64_t t_end = min(ntiles, (lb + 1) * per);
  for (int64_t tile = lb * per + wave; tile < t_end; tile += NWF) {
    const int64_t p = tile * 32 + j;
    const bool valid = p < cnt;
    // the point at the tile's position p, or, in a spatial order, at position perm[p]
    const int64_t q = (a.perm && valid) ? (int64_t)a.perm[p] : p;
    float x = 0.f, y = 0.f, z = 0.f, tq = 0.f;
    if (valid) { x = P[q]; y = P[a.ld + q]; z = P[2 * a.ld + q]; }
    if constexpr (ENC == kEncTime) tq = valid ? a.tau[q] : 0.f;
    f32x16 z1[H / 32], z2[H / 32];
    float m;
    tile_fwd<C, H, GF16, BF, false, ENC>(s, sG, F, swz, w3s, x, y, z, valid, lane, z1, z2, m, nullptr, nullptr,
                                          a.enc, tq);
    if (valid && lane < 32) fo[q] = __builtin_fmaf(m, vs, vo);
  }
}

// ------------------------------------------------------------------ adjoint
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc += A_rows[ia..ia+32) x B_rows[ib..ib+32)^T over the 32 points of the tile
template <bool BF>
__device__ inline f32x16 tt_mma(const typename TT<BF>::T* Ta, int ia, const typename TT<BF>::T* Tb,
                                int ib, int lane, f32x16 acc) {
  constexpr int LDT = TT<BF>::LDT;
  const int li = lane & 31, hk = lane >> 5;
  if constexpr (!BF) {
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      acc = mma_f32(Ta[(ia + li) * LDT + 2 * st + hk], Tb[(ib + li) * LDT + 2 * st + hk], acc);
      if ((st & 7) == 7) sched_fence();
    }
  } else {
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      bf16x8 A = *(const bf16x8*)&Ta[(ia + li) * LDT + 16 * st + 8 * hk];
      bf16x8 B = *(const bf16x8*)&Tb[(ib + li) * LDT + 16 * st + 8 * hk];
      acc = mma_bf16(A, B, acc);
    }
  }
  return acc;
}

// KB > 0: register-resident weight-gradient accumulators (H = 64, KB = KHP/16 dy blocks,
// every column and row in one launch).  KB == 0: per-tile LDS accumulation, any shape,
// gradient rows/columns split across launches.
// ACT (KB == 0 only): the activation path, the per-point activations are stored (a.act) and
// no weight gradient is accumulated in the kernel.
template <int C, int H, bool GF16, bool BF, int KB, bool ACT>
__global__ void __launch_bounds__(kBlock) k_backward(TileArgs a) {
  static_assert(!ACT || KB == 0, "the activation path has no register accumulators");
  extern __shared__ float smem[];
  typedef typename TT<BF>::T TTy;
  constexpr int NB = H / 32;
  constexpr int LDT = TT<BF>::LDT;
  constexpr bool REG = KB > 0;
  // logical block as in k_forward (the partial sums are indexed by it, so their fixed
  // reduction order follows the tiles)
  const int64_t lbl = xcd_logical(blockIdx.x + (int64_t)gridDim.x * blockIdx.y, (int64_t)gridDim.x * gridDim.y);
  const int model = (int)(lbl / gridDim.x), lb = (int)(lbl % gridDim.x);
  const Shape s = a.s;
  const int ncols = a.c1_hi - a.c1_lo;
  const int nrows2 = a.w2_hi - a.w2_lo;
  const PartLayout pl = part_layout(s, ncols, nrows2);
  double* part = a.part + ((size_t)model * gridDim.x + lb) * pl.len;
  const bool act = !a.active || a.active[model];

  // LDS: sG [12M] | sW3w [wave][H] | sLoss (double) | (REG) swizzled weights | per-wave
  // transpose tiles Ta [H rows] (a delta), Tb [32 rows] (an activation block) and (REG)
  // Ty [32 KB rows] (the features) | sW1 [H*ncols], sW2 [nrows2*H] (after the tiles, or,
  // with REG, aliased onto them once the tile loop is done)
  const size_t esz = BF ? 2 : 4;
  const size_t wbytes = REG ? swz_sizes(s).total() * esz : 0;
  // carve by byte offsets from the LDS base (keeps every pointer in the LDS address space)
  char* lbase = (char*)smem;
  size_t off = (size_t)(12 * s.M + kWavesPerBlock * H) * 4;
  float* sG = smem;
  float* sW3w = sG + 12 * s.M;
  off = (off + 7) & ~(size_t)7;
  double* sLoss = (double*)(lbase + off);   // [wave]
  off = (off + 8 * kWavesPerBlock + 15) & ~(size_t)15;
  char* lw = lbase + off;
  TTy* tiles = (TTy*)(lbase + off + wbytes);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 31, hf = lane >> 5;
  const int wrows = H + 32 + (REG ? 32 * KB : 0);
  TTy* Ta = tiles + (size_t)wave * wrows * LDT;
  TTy* Tb = Ta + (size_t)H * LDT;
  TTy* Ty = Tb + (size_t)32 * LDT;
  float* sW1 = REG ? (float*)tiles : (float*)(tiles + (size_t)kWavesPerBlock * wrows * LDT);
  float* sW2 = sW1 + H * ncols;

  const float* G = a.G + model * a.G_stride;
  for (int i = threadIdx.x; i < 12 * s.M; i += blockDim.x) sG[i] = G[i];
  for (int i = threadIdx.x; i < kWavesPerBlock * H; i += blockDim.x) sW3w[i] = 0.f;
  if (!REG)
    for (int i = threadIdx.x; i < H * ncols + nrows2 * H; i += blockDim.x) sW1[i] = 0.f;

  const void* F = GF16 ? (const void*)((const __half*)a.F + model * a.F_stride)
                       : (const void*)((const float*)a.F + model * a.F_stride);
  const void* swz = (const char*)a.swz + esz * model * a.swz_stride;
  if constexpr (REG) {
    block_copy16(lw, swz, wbytes);
    swz = lw;
  }
  __syncthreads();
  const float* w3s = a.w3s + (size_t)model * H;
  const float vs = a.bscale ? a.bscale[model] : a.vscale;
  const float vo = a.boff ? a.boff[model] : a.voff;
  const float* P = a.pts + model * a.pts_stride;
  float* dY = a.dY ? a.dY + (size_t)model * s.M * a.n * C : nullptr;
  const float hR = 0.5f * (float)(s.R - 1);
  const float* W2T = nullptr; const bf16x8* W2Tb = nullptr;
  const float* W1T = nullptr; const bf16x8* W1Tb = nullptr;
  {
    const size_t o2t = (size_t)2 * H * s.KHP + (size_t)H * H, o1t = o2t + (size_t)H * H;
    if (BF) { W2Tb = (const bf16x8*)((const uint16_t*)swz + o2t); W1Tb = (const bf16x8*)((const uint16_t*)swz + o1t); }
    else { W2T = (const float*)swz + o2t; W1T = (const float*)swz + o1t; }
  }
  f32x16 aw2[REG ? NB : 1][REG ? NB : 1];
  f32x16 aw1[REG ? NB : 1][REG ? KB : 1];
  if constexpr (REG) {
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
#pragma unroll
      for (int kb = 0; kb < NB; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) aw2[ib][kb][r] = 0.f;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) aw1[ib][kb][r] = 0.f;
    }
  }
  double loss = 0.0;
  const int nblk = REG ? KB : s.KHP / 16;

  const int64_t ntiles = act ? (a.n + 31) / 32 : 0;
  const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int64_t t_end = min(ntiles, (lb + 1) * per);
  for (int64_t tile = lb * per + wave; tile < t_end; tile += kWavesPerBlock) {
    const int64_t p = tile * 32 + j;
    const bool valid = p < a.n;
    float x = 0.f, y = 0.f, z = 0.f;
    if (valid) { x = P[p]; y = P[a.ld + p]; z = P[2 * a.ld + p]; }
    f32x16 z1[NB], z2[NB];
    float m;
    // stored activations: every lane of the tile writes (points past n write zeros), the
    // features y through ya (rows from 0), h1, delta1 and delta2 through ha (rows from MC)
    void* ablk = (char*)a.act + ((size_t)model * a.act_stride + (size_t)tile * a.act_rows * 32) * (BF ? 2 : 4);
    const ActTile<BF> ya(ablk, 0, s.MC, j), ha(ablk, s.MC, a.act_rows, j);
    tile_fwd<C, H, GF16, BF, REG>(s, sG, F, swz, w3s, x, y, z, valid, lane, z1, z2, m, Ty,
                                  ACT ? &ya : nullptr);
    if constexpr (ACT) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          ha.put(4 * hf, 32 * b + 8 * (r >> 2) + (r & 3), fmaxf(z1[b][r], 0.f));
    }

    // dL/df for this point
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

    // output layer: dW3 (reduced over the tile's points into this wave's row) and delta2
    if (a.do_w3) {
      // dm * relu(z2) summed over the half's 32 points, one row block at a time, by a
      // transposing butterfly: each step halves the values a lane holds and adds the other
      // half from the lane whose index differs in one bit, so after offsets 8, 4, 2, 1 lane
      // j holds value j % 16 summed over its 16-lane group, and one more shuffle adds the
      // other group: 16 shuffles per block instead of 5 per value.  Lanes 0..15 of each half
      // own one row each of the wave's LDS row and add the tiles in order.
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
        for (int m = 8; m > 1; m >>= 1) {
          const int o = m >> 1;
          const bool up = (j & o) != 0;
#pragma unroll
          for (int i = 0; i < m / 2; ++i) {
            const float keep = up ? v[i + m / 2] : v[i];
            const float send = up ? v[i] : v[i + m / 2];
            v[i] = keep + __shfl_xor(send, o, 64);
          }
        }
        const float tot = v[0] + __shfl_xor(v[0], 16, 64);
        if (j < 16) sW3w[wave * H + 32 * b + acc_row(j, hf)] += tot;   // one row per lane: no conflicts
      }
    }
    f32x16 d2[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) d2[b][r] = z2[b][r] > 0.f ? w3s[hf * (H / 2) + 16 * b + r] * dm : 0.f;

    if constexpr (ACT) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          ha.put(4 * hf, 2 * H + 32 * b + 8 * (r >> 2) + (r & 3), d2[b][r]);
    }

    // dW2 rows [w2_lo, w2_hi) = sum_j delta2_j h1_j^T, one 32-row block of h1 at a time
    // (the register path only: other shapes take the activation path or want no dW)
    if (REG && nrows2 > 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) tt_put<BF>(Ta, 32 * b + acc_row(r, hf), j, d2[b][r]);
#pragma unroll
      for (int kb = 0; kb < NB; ++kb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) tt_put<BF>(Tb, acc_row(r, hf), j, fmaxf(z1[kb][r], 0.f));
        wave_lds_sync();
        if constexpr (REG) {
#pragma unroll
          for (int ib = 0; ib < NB; ++ib) aw2[ib][kb] = tt_mma<BF>(Ta, 32 * ib, Tb, 0, lane, aw2[ib][kb]);
        }
        wave_lds_sync();
      }
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
        float Bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) Bv[e] = d2[st >> 1][8 * (st & 1) + e];
        const bf16x8 B = bf16_pack8(Bv);
#pragma unroll
        for (int b = 0; b < NB; ++b) d1[b] = mma_bf16(W2Tb[((size_t)b * (H / 16) + st) * 64 + lane], B, d1[b]);
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) d1[b][r] = z1[b][r] > 0.f ? d1[b][r] : 0.f;
    if constexpr (ACT) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          ha.put(4 * hf, H + 32 * b + 8 * (r >> 2) + (r & 3), d1[b][r]);
    }

    const bool any_w1 = REG && ncols > 0;
    if (any_w1) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) tt_put<BF>(Ta, 32 * b + acc_row(r, hf), j, d1[b][r]);
    }

    // dL/dy per block of 16 features of each half: stored per grid for the cell pass,
    // and (with the features regathered) the first-layer gradient
#pragma unroll(REG ? KB : 1)
    for (int blk = 0; blk < nblk; ++blk) {
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
        for (int st = 0; st < H / 16; ++st) {
          float Bv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) Bv[e] = d1[st >> 1][8 * (st & 1) + e];
          const bf16x8 B = bf16_pack8(Bv);
          dy = mma_bf16(W1Tb[((size_t)blk * (H / 16) + st) * 64 + lane], B, dy);
        }
      }
      const bool need_y = any_w1;
#pragma unroll
      for (int u = 0; u < 16 / C; ++u) {
        const int gi = 16 * blk / C + u;
        const int g = hf * s.Mh + gi;
        const bool gvalid = gi < s.Mh && g < s.M && valid;
        if (dY && gvalid) {
          float* dst = dY + ((size_t)g * a.n + p) * C;
#pragma unroll
          for (int c = 0; c < C; ++c) dst[c] = dy[u * C + c];
        }
      }
      if (need_y) {
        wave_lds_sync();
        if constexpr (REG) {
#pragma unroll
          for (int ib = 0; ib < NB; ++ib)
            aw1[ib][blk] = tt_mma<BF>(Ta, 32 * ib, Ty + (size_t)32 * blk * LDT, 0, lane, aw1[ib][blk]);
        }
        wave_lds_sync();
      }
    }
  }

  // block-level reductions, waves added in a fixed order (bitwise reproducible)
  if constexpr (REG) {
    __syncthreads();  // the tiles are dead: reuse them for the cross-wave sums
    for (int i = threadIdx.x; i < H * ncols + nrows2 * H; i += blockDim.x) sW1[i] = 0.f;
    for (int w = 0; w < kWavesPerBlock; ++w) {
      __syncthreads();
      if (wave != w) continue;
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
#pragma unroll
        for (int kb = 0; kb < NB; ++kb)
#pragma unroll
          for (int r = 0; r < 16; ++r) sW2[(32 * ib + acc_row(r, hf)) * H + 32 * kb + j] += aw2[ib][kb][r];
#pragma unroll
        for (int blk = 0; blk < KB; ++blk) {
          const int col = (j >> 4) * s.KH + 16 * blk + (j & 15);
          if ((16 * blk + (j & 15)) < s.KH && col < s.MC) {
#pragma unroll
            for (int r = 0; r < 16; ++r) sW1[(32 * ib + acc_row(r, hf)) * ncols + col] += aw1[ib][blk][r];
          }
        }
      }
    }
  }

  if (a.want_loss) {
    const double t = wave_sum(loss);
    if (lane == 0) sLoss[wave] = t;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < H * ncols; i += blockDim.x) part[pl.o_w1 + i] = sW1[i];
  for (int i = threadIdx.x; i < nrows2 * H; i += blockDim.x) part[pl.o_w2 + i] = sW2[i];
  if (a.do_w3)
    for (int i = threadIdx.x; i < H; i += blockDim.x)
      part[pl.o_w3 + i] = (double)sW3w[i] + (double)sW3w[H + i] + (double)sW3w[2 * H + i] + (double)sW3w[3 * H + i];
  if (threadIdx.x == 0) part[pl.o_loss] = a.want_loss ? ((sLoss[0] + sLoss[1]) + sLoss[2]) + sLoss[3] : 0.0;
}

// Weight-gradient products from stored activations: part[chunk][off + i * cols + j] = sum over
// the chunk's points p of A[i][p] B[j][p], where A is rows a_row0.. and B rows b_row0.. of the
// activation blocks (act_rows x 32 points per tile, float32 or bf16 as the MLP, zeros past the
// last point).  A wave owns one 32-row block and up to four 32-column blocks; the matrix-core
// k dimension runs over points (lane half kh takes 16 (float32) or 8 (bf16) consecutive points
// of each step).  Partials are float64, reduced over the chunks afterwards in a fixed order.
constexpr int kGemmChunk = 2048;   // points per chunk (a multiple of 32)
template <bool BF>
__global__ void __launch_bounds__(256) k_dw_gemm(const void* act, int act_rows, int a_row0, int b_row0,
                                                 int64_t npad, int rows, int cols, double* part, int part_len,
                                                 int part_off) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 31, kh = lane >> 5;
  const int rb = blockIdx.y * 4 + wave;
  if (32 * rb >= rows) return;
  const int64_t p0 = (int64_t)blockIdx.x * kGemmChunk, p1 = min(npad, p0 + kGemmChunk);
  const int row = 32 * rb + i;
  int col[4];
  bool cok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) { col[c] = 32 * (blockIdx.z * 4 + c) + i; cok[c] = col[c] < cols; }
  f32x16 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;
  for (int64_t base = p0; base < p1; base += 32) {
    const size_t tb = (size_t)(base / 32) * act_rows * 32;   // this tile's block
    if constexpr (!BF) {
      const f32x4* ar = (const f32x4*)((const float*)act + tb + (size_t)(a_row0 + row) * 32 + 16 * kh);
      f32x4 av[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) av[q] = ar[q];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        f32x4 bv[4];
        if (cok[c]) {
          const f32x4* br = (const f32x4*)((const float*)act + tb + (size_t)(b_row0 + col[c]) * 32 + 16 * kh);
#pragma unroll
          for (int q = 0; q < 4; ++q) bv[q] = br[q];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) bv[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int st = 0; st < 16; ++st) acc[c] = mma_f32(av[st >> 2][st & 3], bv[st >> 2][st & 3], acc[c]);
      }
    } else {
      const bf16x8* ar = (const bf16x8*)((const uint16_t*)act + tb + (size_t)(a_row0 + row) * 32 + 8 * kh);
      const bf16x8 a0 = ar[0], a1 = ar[2];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        bf16x8 b0 = bf16x8{0, 0, 0, 0, 0, 0, 0, 0}, b1 = b0;
        if (cok[c]) {
          const bf16x8* br = (const bf16x8*)((const uint16_t*)act + tb + (size_t)(b_row0 + col[c]) * 32 + 8 * kh);
          b0 = br[0];
          b1 = br[2];
        }
        acc[c] = mma_bf16(a0, b0, acc[c]);
        acc[c] = mma_bf16(a1, b1, acc[c]);
      }
    }
  }
  double* out = part + (size_t)blockIdx.x * part_len + part_off;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (cok[c]) {
#pragma unroll
      for (int r = 0; r < 16; ++r) out[(size_t)(32 * rb + acc_row(r, kh)) * cols + col[c]] = (double)acc[c][r];
    }
}

// ------------------------------------------------------------------ instantiation
constexpr size_t kFwdWeightLdsMax = 120 * 1024;
// above this much LDS per block only one forward block fits a compute unit: eight-wave blocks
constexpr size_t kFwdWideLds = 80 * 1024;

template <int C, int H, bool GF16, bool BF>
hipError_t launch_tile_kernels(bool backward, int kb, const TileArgs& a, dim3 grid, size_t shmem,
                               hipStream_t st) {
  if (!backward) {
    if (fwd_weight_bytes(a.s, BF) > kFwdWeightLdsMax)
      hipLaunchKernelGGL((k_forward<C, H, GF16, BF, false>), grid, dim3(kBlock), shmem, st, a);
    else if (shmem > kFwdWideLds)
      hipLaunchKernelGGL((k_forward<C, H, GF16, BF, true, kEncDense, 8>), grid, dim3(8 * kWave), shmem, st, a);
    else
      hipLaunchKernelGGL((k_forward<C, H, GF16, BF, true>), grid, dim3(kBlock), shmem, st, a);
  } else if (a.act) {
    hipLaunchKernelGGL((k_backward<C, H, GF16, BF, 0, true>), grid, dim3(kBlock), shmem, st, a);
  } else if constexpr (H == 64) {
    if (kb == 1) hipLaunchKernelGGL((k_backward<C, H, GF16, BF, 1, false>), grid, dim3(kBlock), shmem, st, a);
    else if (kb == 2) hipLaunchKernelGGL((k_backward<C, H, GF16, BF, 2, false>), grid, dim3(kBlock), shmem, st, a);
    else hipLaunchKernelGGL((k_backward<C, H, GF16, BF, 0, false>), grid, dim3(kBlock), shmem, st, a);
  } else {
    hipLaunchKernelGGL((k_backward<C, H, GF16, BF, 0, false>), grid, dim3(kBlock), shmem, st, a);
  }
  return hipGetLastError();
}

// Register-accumulated adjoint applies when H = 64 and at most 2 dy blocks per half.
int register_kb(const Shape& s) { return (s.H == 64 && s.KHP <= 32) ? s.KHP / 16 : 0; }

size_t backward_lds_bytes(const Shape& s, int ncols, int nrows2, bool bf, int kb) {
  const int ldt = bf ? 40 : 33;
  const size_t esz = bf ? 2 : 4;
  size_t b = (size_t)(12 * s.M + kWavesPerBlock * s.H) * 4;
  b = (b + 7) & ~(size_t)7;
  b += 8 * kWavesPerBlock;
  b = (b + 15) & ~(size_t)15;
  if (kb) b += swz_sizes(s).total() * esz;
  const size_t tiles = (size_t)kWavesPerBlock * (s.H + 32 + 32 * kb) * ldt * esz;
  const size_t red = (size_t)(s.H * ncols + nrows2 * s.H) * 4;
  b += kb ? std::max(tiles, red) : tiles + red;
  return b;
}

size_t forward_lds_bytes(const Shape& s, bool bf) {
  size_t b = (size_t)12 * s.M * 4;
  b = (b + 15) & ~(size_t)15;
  if (fwd_weight_bytes(s, bf) <= kFwdWeightLdsMax) b += fwd_weight_bytes(s, bf);
  return b;
}

hipError_t launch_tile(bool backward, int kb, const TileArgs& a, bool grid_f16, bool mlp_bf16, dim3 grid,
                       size_t shmem, hipStream_t st) {
  const int C = a.s.C, H = a.s.H;
  // only the register-resident adjoint accumulates weight gradients in the kernel
  if (backward && kb == 0 && (a.c1_hi > a.c1_lo || a.w2_hi > a.w2_lo)) return hipErrorInvalidValue;
#define APMG_DISPATCH(CC, HH)                                                                  \
  if (C == CC && H == HH) {                                                                    \
    if (!grid_f16 && !mlp_bf16) return launch_tile_kernels<CC, HH, false, false>(backward, kb, a, grid, shmem, st); \
    if (!grid_f16 && mlp_bf16) return launch_tile_kernels<CC, HH, false, true>(backward, kb, a, grid, shmem, st);   \
    if (grid_f16 && !mlp_bf16) return launch_tile_kernels<CC, HH, true, false>(backward, kb, a, grid, shmem, st);   \
    return launch_tile_kernels<CC, HH, true, true>(backward, kb, a, grid, shmem, st);              \
  }
  APMG_DISPATCH(1, 64)
  APMG_DISPATCH(2, 64)
  APMG_DISPATCH(4, 64)
  APMG_DISPATCH(1, 128)
  APMG_DISPATCH(2, 128)
  APMG_DISPATCH(4, 128)
#undef APMG_DISPATCH
  return hipErrorInvalidValue;
}

hipError_t launch_swizzle(const Shape& s, bool bf, const float* W1, const float* W2, const float* W3,
                          size_t wstride, void* swz, size_t swz_stride, float* w3s, int nmodels,
                          hipStream_t st) {
  const size_t total = swz_sizes(s).total() + s.H;
  dim3 grid((unsigned)((total + 255) / 256 > 4096 ? 4096 : (total + 255) / 256), nmodels);
  if (bf) hipLaunchKernelGGL(k_swizzle<true>, grid, dim3(256), 0, st, s, W1, W2, W3, wstride, swz, swz_stride, w3s);
  else hipLaunchKernelGGL(k_swizzle<false>, grid, dim3(256), 0, st, s, W1, W2, W3, wstride, swz, swz_stride, w3s);
  return hipGetLastError();
}

}  // namespace apmg
