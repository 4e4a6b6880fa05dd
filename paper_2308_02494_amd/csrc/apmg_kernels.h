// Kernel argument blocks and launcher declarations shared by the HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apmg {

// Shape of one model as the tile kernels see it.
struct Shape {
  int M, C, R, H;   // grids, channels, vertices per axis, hidden width
  int Mh;           // grids per lane half: ceil(M/2); half hf owns grids [hf*Mh, hf*Mh+Mh)
  int KH;           // features per half = Mh*C
  int KHP;          // KH rounded up to a multiple of 16
  int MC;           // M*C (= width[0])
  int L;            // feature grids per transform: 1, or the hash levels of the hash-grid encoder
                    // (grid g then reads transform g / L); transforms = M / L
};

// Encoder variants of Sec. 9 (the dense trilinear grids of Eq. (2) are encoder 0).
// 1: a hash grid inside each adaptive grid: feature grid g = (grid g / L, level g % L), level k
//    with res(k) cells per axis, a table of T = tmask + 1 entries of C features per (grid,
//    level), tables [M][L][T][C]; 2: 4-D grids with Rt time vertices, gathered from the
//    channel-last copy [M][Rt][R^3][C] (time slice t of grid g is grid g * Rt + t there),
//    the time coordinate in a fourth row of the points.
constexpr int kEncDense = 0, kEncHash = 1, kEncTime = 2;
constexpr int kMaxLevels = 8;
struct EncArgs {
  uint32_t res2[kMaxLevels / 2];   // hash: cells per axis of level k in bits 16 (k % 2) of word k / 2
  uint32_t tmask;                  // hash: T - 1
  int Rt;                          // time: vertices along the time axis
};
__host__ __device__ inline int enc_level_res(const EncArgs& e, int k) {
  const uint32_t w = k < 2 ? e.res2[0] : k < 4 ? e.res2[1] : k < 6 ? e.res2[2] : e.res2[3];
  return (int)((w >> (16 * (k & 1))) & 0xffffu);
}

// Element counts of the swizzled weight operands of one model: the first
// layer (A operand order), the second layer and its transpose, the first
// layer's transpose (for dL/dy), and the output layer in accumulator row order.
struct SwzSizes {
  size_t w1, w2, w3, w2t, w1t;
  __host__ __device__ size_t total() const { return w1 + w2 + w2t + w1t; }  // w3 is stored separately (float)
};
__host__ __device__ inline SwzSizes swz_sizes(const Shape& s) {
  SwzSizes z;
  z.w1 = (size_t)2 * s.H * s.KHP;
  z.w2 = (size_t)s.H * s.H;
  z.w2t = z.w2;
  z.w1t = (size_t)2 * s.KHP * s.H;
  z.w3 = (size_t)s.H;
  return z;
}

// Arguments of the tile kernels (forward and adjoint).  Model b of a batch
// (blockIdx.y) adds b * stride to every per-model pointer.
struct TileArgs {
  Shape s;
  const float* G; size_t G_stride;        // [M][12] per model (floats)
  const void* F; size_t F_stride;         // grids per model (elements)
  const void* swz; size_t swz_stride;     // swizzled weights per model (elements)
  const float* w3s;                       // [model][H]
  float vscale, voff;                     // output scaling when bscale == NULL
  const float* bscale;                    // per model (vmax - vmin) or NULL
  const float* boff;                      // per model vmin or NULL
  const float* pts; int64_t ld; size_t pts_stride; int64_t n;
  const uint32_t* seg;                    // forward only: [models + 1] segment starts in one shared array, or NULL
  const uint32_t* perm;                   // forward only, model 0, no segments: the tile's point p is input and
                                          // output position perm[p] (a spatial order of the points), or NULL
  // forward
  float* f;
  // adjoint
  const float* df;                        // [n] dL/df, or NULL: MSE against v
  const float* v; size_t v_stride;        // ground truth (training)
  float* err; size_t err_stride;          // h(x) out (training)
  int err_abs;
  float* dY;                              // [model][M][n][C] dL/dy per grid (sorted points) or NULL
  int c1_lo, c1_hi;                       // first-layer gradient columns accumulated by this launch
  int w2_lo, w2_hi;                       // second-layer gradient rows (multiples of 32)
  int do_w3;                              // accumulate the output layer gradient
  int want_loss;                          // accumulate sum (f - v)^2
  double* part; int part_len;             // per-block partials [model][block][part_len]
  const int32_t* active;                  // per model: skip the model when 0 (or NULL)
  // activation path: when non-NULL, the per-point activations of the weight-gradient
  // products are stored instead of accumulated (float32, or bf16 with the bf16 MLP), one block
  // per 32-point tile of act_rows rows x 32 points, rows y [MC] | h1 [H] | delta1 [H] | delta2 [H]
  void* act; int act_rows; size_t act_stride;   // act_stride: elements per model
  EncArgs enc;                            // encoder variants (zero for the dense grids)
  const float* tau;                       // 4-D grids: [n] time of each point (model 0 only)
};

// Per-block partial sums of the adjoint, float64: [dW1 slice H x ncols]
// [dW2 rows nrows2 x H] [dW3 H] [dG M x 12] [loss 1].
struct PartLayout {
  int o_w1, o_w2, o_w3, o_g, o_loss, len;
};
__host__ __device__ inline PartLayout part_layout(const Shape& s, int ncols, int nrows2) {
  PartLayout p;
  p.o_w1 = 0;
  p.o_w2 = s.H * ncols;
  p.o_w3 = p.o_w2 + nrows2 * s.H;
  p.o_g = p.o_w3 + s.H;
  p.o_loss = p.o_g + 12 * s.M;
  p.len = p.o_loss + 1;
  return p;
}

}  // namespace apmg
