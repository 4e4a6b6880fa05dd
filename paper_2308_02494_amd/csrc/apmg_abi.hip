// Host side of the C ABI declared in include/apmg.h: argument validation,
// workspace layout and the launch sequence of every entry point.
#include <mutex>
#include <vector>

using namespace apmg;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Bump allocator over the caller's workspace (or a size counter when base == NULL).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T> T* take(size_t count) {
    T* p = base ? (T*)(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

constexpr int kMaxTileBlocks = 512;
constexpr int kDensBlocks = 1024;
constexpr size_t kLdsLimit = 160 * 1024;

apmg_status check_model(const apmg_model* m, bool need_params, Shape* out) {
  if (!m) return APMG_EINVAL;
  if (m->M < 1 || m->C < 1 || m->R < 2 || m->n_layers < 1 || m->n_layers > APMG_MAX_LAYERS) return APMG_EINVAL;
  if (m->width[0] != m->M * m->C || m->width[m->n_layers] != 1) return APMG_EINVAL;
  for (int k = 0; k <= m->n_layers; ++k) if (m->width[k] < 1) return APMG_EINVAL;
  if (need_params) {
    if (!m->G || !m->F) return APMG_EINVAL;
    for (int k = 0; k < m->n_layers; ++k) if (!m->W[k]) return APMG_EINVAL;
  }
  if (m->grid_layout != APMG_GRIDS_MCRRR && m->grid_layout != APMG_GRIDS_MRRRC) return APMG_EINVAL;
  if (!(m->G_rows == 0 || m->G_rows == 3 || m->G_rows == 4)) return APMG_EINVAL;
  if (m->grid_dtype != APMG_F32 && m->grid_dtype != APMG_F16) return APMG_EUNSUPPORTED;
  if (m->mlp_dtype != APMG_F32 && m->mlp_dtype != APMG_BF16) return APMG_EUNSUPPORTED;
  if (!(m->C == 1 || m->C == 2 || m->C == 4)) return APMG_EUNSUPPORTED;
  if (m->M * m->C > 256) return APMG_EUNSUPPORTED;
  if (m->n_layers != 3 || m->width[1] != m->width[2] || !(m->width[1] == 64 || m->width[1] == 128))
    return APMG_EUNSUPPORTED;
  if ((double)m->R * m->R * m->R * m->M * m->C > 2e9) return APMG_EUNSUPPORTED;
  Shape s;
  s.M = m->M; s.C = m->C; s.R = m->R; s.H = m->width[1];
  s.Mh = (m->M + 1) / 2;
  s.KH = s.Mh * s.C;
  s.KHP = (s.KH + 15) / 16 * 16;
  s.MC = m->M * m->C;
  s.L = 1;
  if (out) *out = s;
  return APMG_OK;
}

inline int g_rows(const apmg_model* m) { return m->G_rows == 4 ? 4 : 3; }
inline bool paper_grids(const apmg_model* m) { return m->grid_layout == APMG_GRIDS_MCRRR; }
size_t f_elems(const Shape& s) { return (size_t)s.M * s.R * s.R * s.R * s.C; }

apmg_status check_points(const float* pts, int64_t ld, int64_t n) {
  if (n < 0 || ld < n) return APMG_EINVAL;
  if (n > 0 && !pts) return APMG_EINVAL;
  return APMG_OK;
}

apmg_status hip_status(hipError_t e) { return e == hipSuccess ? APMG_OK : APMG_EHIP; }

inline unsigned red_blocks(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 31) / 32, 2048));
}

inline unsigned grid1(int64_t n, int64_t cap = 4096) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return (unsigned)std::min<int64_t>(g, cap);
}

int tile_blocks(int64_t n) {
  const int64_t tiles = (n + 31) / 32;
  int64_t b = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxTileBlocks));
}

// Training-step launch shapes (apmg_tuning): tile-kernel blocks per model, default one
// per CU over all models when nb divides the CUs evenly, else about two per CU, at most 4x the default,
// 1024, and the number of 4-tile groups; gather batch of 2, 4 or 8 candidates; lanes per
// candidate run of the wave gather, 1, 2, 4 or 8.
constexpr int kDefaultCellGroup = 4;
// adjoint: 0 = tiled adjoint, waves per block by dtype; 1 = eight waves; 2 = four waves;
// 3 = the one-wave-per-SIMD register kernel.
struct Tune { int tile_blocks; int cell_unroll; int cell_kernel; int cell_group; int adjoint; };
int step_groups(int64_t n) {
  const int64_t tiles = (std::max<int64_t>(n, 1) + 31) / 32;
  return (int)std::max<int64_t>(1, (tiles + kWavesPerBlock - 1) / kWavesPerBlock);
}
// The register-resident adjoint kernel runs one block per compute unit: one round of
// blocks (one per CU) when the models share the CUs evenly, else about two per CU.
int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return kMaxTileBlocks / 2;
  return cus;
}
// apmg_backward: one round of the adjoint kernel's blocks (one per CU), at most one per 4 tiles.
// (two rounds when the tiled adjoint runs four-wave blocks, two per CU)
int bwd_blocks(int64_t n, bool bf) {
  const int cap = adjoint_waves(0, bf) == 4 ? 2 * device_cus() : device_cus();
  return std::max(1, std::min(tile_blocks(n), cap));
}
int step_default_blocks(int64_t n, int nb) {
  const int cus = device_cus();
  const int one = (cus + nb - 1) / nb;
  const int b = one * nb <= cus ? one : (2 * cus + nb - 1) / nb;
  return std::max(1, std::min(b, step_groups(n)));
}
int step_max_blocks(int64_t n, int nb) {
  return std::max(1, std::min(std::min(4 * step_default_blocks(n, nb), 1024), step_groups(n)));
}
bool resolve_tune(const apmg_tuning* t, int64_t n, int nb, bool bf, Tune* out) {
  out->tile_blocks = step_default_blocks(n, nb);
  out->cell_unroll = 4;
  out->cell_kernel = 0;
  out->cell_group = kDefaultCellGroup;
  out->adjoint = 0;
  // four-wave tiled adjoint blocks run two per compute unit
  const auto two_per_cu = [&]() {
    if (out->adjoint < 3 && adjoint_waves(out->adjoint, bf) == 4)
      out->tile_blocks = std::min(2 * out->tile_blocks, step_max_blocks(n, nb));
  };
  if (!t) {
    two_per_cu();
    return true;
  }
  if (t->tile_blocks < 0 || t->tile_blocks > step_max_blocks(n, nb)) return false;
  if (t->cell_unroll != 0 && t->cell_unroll != 2 && t->cell_unroll != 4 && t->cell_unroll != 8) return false;
  if (t->cell_kernel < 0 || t->cell_kernel > 2) return false;
  if (t->cell_group != 0 && t->cell_group != 1 && t->cell_group != 2 && t->cell_group != 4 && t->cell_group != 8)
    return false;
  if (t->tile_blocks > 0) out->tile_blocks = t->tile_blocks;
  if (t->cell_unroll > 0) out->cell_unroll = t->cell_unroll;
  if (t->cell_kernel > 0) out->cell_kernel = t->cell_kernel - 1;
  if (t->cell_group > 0) out->cell_group = t->cell_group;
  if (t->adjoint_kernel < 0 || t->adjoint_kernel > 3) return false;
  out->adjoint = t->adjoint_kernel;
  if (t->tile_blocks == 0) two_per_cu();
  return true;
}

// Adjoint passes: each accumulates a block of second-layer gradient rows and a slice of
// first-layer gradient columns in LDS; the first pass also scatters dF, reduces dG and
// the output-layer gradient.  Chosen so that every pass fits the LDS.
struct Pass { int c1_lo, c1_hi, w2_lo, w2_hi; bool first; };
std::vector<Pass> plan_passes(const Shape& s, bool bf, bool want_w) {
  std::vector<Pass> out;
  if (!want_w) { out.push_back({0, 0, 0, 0, true}); return out; }
  int r0 = 0, c0 = 0;
  while (r0 < s.H || c0 < s.MC) {
    int r = 0;
    while (r0 + r + 32 <= s.H && backward_lds_bytes(s, 0, r + 32, bf, 0) <= kLdsLimit) r += 32;
    int c = 0;
    if (r0 + r >= s.H) {  // rows done in this pass: give the rest of the budget to columns
      int lo = 0, hi = s.MC - c0;
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (backward_lds_bytes(s, mid, r, bf, 0) <= kLdsLimit) lo = mid; else hi = mid - 1;
      }
      c = lo;
    }
    if (r == 0 && c == 0) return {};
    out.push_back({c0, c0 + c, r0, r0 + r, out.empty()});
    r0 += r;
    c0 += c;
  }
  return out;
}
int max_part_len(const Shape& s, bool bf) {
  int len = part_layout(s, 0, 0).len;
  for (const Pass& p : plan_passes(s, bf, true))
    len = std::max(len, part_layout(s, p.c1_hi - p.c1_lo, p.w2_hi - p.w2_lo).len);
  return len;
}

// ---------------------------------------------------------------- model operands
// What the kernels read: transforms as [model][M][3][4] and grids as a channel-last mirror
// [model][M][R^3][C] in the dtype the encoder gathers.  Where the caller's arrays are not in
// that form already (4-row transforms, paper-order grids, F16 gathers of float32 masters)
// the copies live in the workspace and are rebuilt by every call.
struct OpsWs { float* G; void* F; };
void take_ops(Carver& cv, const Shape& s, int nb, bool pack_G, bool mirror, bool f16, OpsWs* o) {
  o->G = pack_G ? cv.take<float>((size_t)nb * 12 * s.M) : nullptr;
  o->F = mirror ? cv.take<char>((size_t)nb * f_elems(s) * (f16 ? 2 : 4)) : nullptr;
}
template <int C>
void mirror_c(const Shape& s, int nb, const void* src, bool sf16, bool spaper, void* dst, bool df16, hipStream_t st) {
  const int64_t nm = (int64_t)nb * s.M, R3 = (int64_t)s.R * s.R * s.R;
  const dim3 g(grid1(nm * R3, 8192)), b(256);
  if (!sf16 && !df16) {
    if (spaper) hipLaunchKernelGGL((k_mirror_grids<C, float, float, true>), g, b, 0, st, nm, R3, (const float*)src, (float*)dst);
    else hipLaunchKernelGGL((k_mirror_grids<C, float, float, false>), g, b, 0, st, nm, R3, (const float*)src, (float*)dst);
  } else if (!sf16 && df16) {
    if (spaper) hipLaunchKernelGGL((k_mirror_grids<C, float, uint16_t, true>), g, b, 0, st, nm, R3, (const float*)src, (uint16_t*)dst);
    else hipLaunchKernelGGL((k_mirror_grids<C, float, uint16_t, false>), g, b, 0, st, nm, R3, (const float*)src, (uint16_t*)dst);
  } else {   // F16 grids gathered as F16: only the order changes
    hipLaunchKernelGGL((k_mirror_grids<C, uint16_t, uint16_t, true>), g, b, 0, st, nm, R3, (const uint16_t*)src, (uint16_t*)dst);
  }
}
// Builds the copies of take_ops from the caller's G ([nb][M][grows][4]) and F (layout and
// dtype as given) and returns the pointers the kernels take.
hipError_t launch_ops(const Shape& s, int nb, const float* G, int grows, const void* F, bool sf16, bool spaper,
                      const OpsWs& w, bool df16, hipStream_t st, const float** Gc, const void** Fc) {
  *Gc = G;
  if (Fc) *Fc = F;
  if (w.G) {
    hipLaunchKernelGGL(k_pack_G, dim3(grid1((int64_t)nb * 12 * s.M)), dim3(256), 0, st, (int64_t)nb * s.M, G, w.G);
    *Gc = w.G;
  }
  if (w.F && Fc) {
    if (s.C == 1) mirror_c<1>(s, nb, F, sf16, spaper, w.F, df16, st);
    else if (s.C == 2) mirror_c<2>(s, nb, F, sf16, spaper, w.F, df16, st);
    else mirror_c<4>(s, nb, F, sf16, spaper, w.F, df16, st);
    *Fc = w.F;
  }
  (void)grows;
  return hipGetLastError();
}

// ---------------------------------------------------------------- workspace layouts
// Spatial sort of nb models' points: keys/values ping-pong, digit histograms, bin starts,
// sorted points and an optional permuted per-point array.
struct SortWs { uint32_t *k0, *v0, *k1, *v1, *hist, *rowtot, *dbase, *start; float *spts, *sf; float4* spts4; };
inline int sort_tiles(int64_t n) { return (int)std::max<int64_t>(1, (n + kSortTile - 1) / kSortTile); }
void take_sort(Carver& cv, int64_t n, int nb, bool with_f, SortWs* o, bool keys_only = false);

// Forward operands; from kFwdSortMin points on, the points are first sorted into spatial
// bins (neighbouring points of a wave then share grid cells in cache) and the tiles read
// their points and write their outputs through the sort's permutation.
constexpr int64_t kFwdSortMin = (int64_t)1 << 15;
struct FwdWs { void* swz; float* w3s; bool sorted; SortWs srt; OpsWs ops; };
// sortable = false: the direct tile path for every n (the sort only orders the work; each
// output is bitwise the same either way)
size_t fwd_ws(const Shape& s, const apmg_model* m, int64_t n, void* ws, FwdWs* o, bool sortable = true) {
  Carver cv(ws);
  const bool bf = m->mlp_dtype == APMG_BF16;
  const size_t esz = bf ? 2 : 4;
  FwdWs w;
  take_ops(cv, s, 1, g_rows(m) == 4, paper_grids(m), m->grid_dtype == APMG_F16, &w.ops);
  w.swz = cv.take<char>(swz_sizes(s).total() * esz);
  w.w3s = cv.take<float>(s.H);
  w.sorted = sortable && n >= kFwdSortMin;
  if (w.sorted) take_sort(cv, n, 1, false, &w.srt, true);
  if (o) *o = w;
  return cv.off;
}

// keys_only: the radix passes' buffers alone (a forward pass reads through the permutation)
void take_sort(Carver& cv, int64_t n, int nb, bool with_f, SortWs* o, bool keys_only) {
  const int64_t nn = std::max<int64_t>(n, 1);
  o->k0 = cv.take<uint32_t>((size_t)nb * nn);
  o->v0 = cv.take<uint32_t>((size_t)nb * nn);
  o->k1 = cv.take<uint32_t>((size_t)nb * nn);
  o->v1 = cv.take<uint32_t>((size_t)nb * nn);
  o->hist = cv.take<uint32_t>((size_t)nb * kRadixDigits * sort_tiles(n));
  o->rowtot = cv.take<uint32_t>((size_t)nb * kRadixDigits);
  o->dbase = cv.take<uint32_t>((size_t)nb * kRadixDigits);
  if (keys_only) {
    o->start = nullptr; o->spts = nullptr; o->sf = nullptr; o->spts4 = nullptr;
    return;
  }
  o->start = cv.take<uint32_t>((size_t)nb * (kBinsPerAxis * kBinsPerAxis * kBinsPerAxis + 1));
  o->spts = cv.take<float>((size_t)nb * 3 * nn);
  o->sf = with_f ? cv.take<float>((size_t)nb * nn) : nullptr;
  o->spts4 = cv.take<float4>((size_t)nb * nn);
}

// LSD radix passes over the keys/values in k0/v0; after an even number of passes the sorted
// keys/values are back in k0/v0.
void radix_passes(int64_t n, int nb, int nt, const SortWs& w, hipStream_t st) {
  uint32_t *ki = w.k0, *vi = w.v0, *ko = w.k1, *vo = w.v1;
  static_assert((kBinBits + kRadixBits - 1) / kRadixBits % 2 == 0, "an even number of passes");
  for (int shift = 0; shift < kBinBits; shift += kRadixBits) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nt, nb), dim3(kSortThreads), 0, st, ki, n, shift, w.hist, nt);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(kRadixDigits, nb), dim3(256), 0, st, w.hist, nt, w.rowtot);
    hipLaunchKernelGGL(k_radix_digitscan, dim3(nb), dim3(256), 0, st, w.rowtot, w.dbase);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nt, nb), dim3(kSortThreads), 0, st, ki, vi, ko, vo, n, shift, w.hist, w.dbase,
                       nt);
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
}

// with_starts: also the points in sorted order, the 16-byte point records and the bin starts
// (the per-cell gather's candidate lists); a forward pass, which sorts only to order its
// work, reads its points through the permutation (v0) and needs none of them
hipError_t launch_sort(const float* pts, int64_t ld, size_t pts_stride, const float4* pts4, int64_t n, int nb,
                       const SortWs& w, const float* src_f, hipStream_t st, bool with_starts = true) {
  const int nt = sort_tiles(n);
  SortIn in;
  in.pts = pts; in.ld = ld; in.pts_stride = pts_stride; in.pts4 = pts4;
  hipLaunchKernelGGL(k_bin_keys, dim3(grid1(n), nb), dim3(256), 0, st, in, n, w.k0, w.v0);
  radix_passes(n, nb, nt, w, st);
  if (!with_starts) return hipGetLastError();
  hipLaunchKernelGGL(k_permute_points, dim3(grid1(n), nb), dim3(256), 0, st, in, n, w.v0, w.spts, w.spts4, src_f,
                     w.sf);
  // bin starts: one thread per position (gaps between neighbouring keys are short when the
  // points are few per bin), or one per bin (binary search) for large point sets, whose empty
  // regions would leave a few position threads writing long gaps
  constexpr int64_t kBins = (int64_t)kBinsPerAxis * kBinsPerAxis * kBinsPerAxis;
  if (n > 8 * kBins)
    hipLaunchKernelGGL(k_bin_starts_search, dim3(grid1(kBins + 1), nb), dim3(256), 0, st, w.k0, n, w.start);
  else
    hipLaunchKernelGGL(k_bin_starts, dim3(grid1(n + 1), nb), dim3(256), 0, st, w.k0, n, w.start);
  return hipGetLastError();
}

// The training batch: keys from the counter stream, the radix passes, then the points
// regenerated in sorted order together with their ground truth (no gather of stored points).
hipError_t launch_step_sort(uint64_t seed, const uint64_t* step_ctr, uint32_t stream0, int64_t n, int nb,
                            const SortWs& w, const float* vol, int vnx, int vny, const apmg_brick* bricks, float* v,
                            hipStream_t st) {
  const int nt = sort_tiles(n);
  hipLaunchKernelGGL(k_batch_keys, dim3(grid1(n, 2048), nb), dim3(256), 0, st, seed, step_ctr, stream0, n, w.k0,
                     w.v0);
  radix_passes(n, nb, nt, w, st);
  hipLaunchKernelGGL(k_batch_sorted, dim3(grid1(n, 2048), nb), dim3(256), 0, st, seed, step_ctr, stream0, n, w.v0,
                     w.spts,
                     w.spts4, vol, vnx, vny, bricks, v);
  hipLaunchKernelGGL(k_bin_starts, dim3(grid1(n + 1), nb), dim3(256), 0, st, w.k0, n, w.start);
  return hipGetLastError();
}

// Per-cell pass buffers: dL/dy per grid, corner sums per cell, transform-gradient partials.
struct CellWs { float *dY, *CC; double* dGpart; };
inline int64_t n_cells(const Shape& s) { return (int64_t)(s.R - 1) * (s.R - 1) * (s.R - 1); }
inline int cell_blocks(const Shape& s) { return (int)((n_cells(s) + 255) / 256); }
// workgroups per grid of the wave gather (4 waves, each a 4x4x4 block of cells)
inline int wave_groups(const Shape& s) {
  const int64_t nbx = (s.R - 1 + kBlk - 1) / kBlk;
  return (int)((nbx * nbx * nbx + 3) / 4);
}
// transform-gradient partials per grid written by the gather cell_kernel selects
inline int dg_parts(const Shape& s, int cell_kernel) { return cell_kernel != 1 ? wave_groups(s) : cell_blocks(s); }
void take_cell(Carver& cv, const Shape& s, int64_t n, int nb, CellWs* o) {
  o->dY = cv.take<float>((size_t)nb * s.M * std::max<int64_t>(n, 1) * s.C);
  // corner sums per cell (the per-cell gather) or vertex lattices per cell block (the wave gather)
  const int64_t nbx = (s.R - 1 + kBlk - 1) / kBlk;
  o->CC = cv.take<float>((size_t)nb * s.M * std::max<int64_t>(n_cells(s) * 8, nbx * nbx * nbx * kLat) * s.C);
  o->dGpart = cv.take<double>((size_t)nb * s.M * std::max(cell_blocks(s), wave_groups(s)) * 12);
}

// timing hooks: [0] the adjoint tile kernel, [1] the grid-gradient gather
hipEvent_t g_prof_start[2] = {nullptr, nullptr}, g_prof_stop[2] = {nullptr, nullptr};
void prof_begin(hipStream_t st, int k) { if (g_prof_start[k]) hipEventRecord(g_prof_start[k], st); }
void prof_end(hipStream_t st, int k) {
  if (g_prof_stop[k]) hipEventRecord(g_prof_stop[k], st);
  g_prof_start[k] = g_prof_stop[k] = nullptr;
}

// Grid gradient (into dF when non-NULL) and, when want_dG, the per-block transform-gradient
// partials (reduced into dG when non-NULL; otherwise left for a later k_reduce_cell_dG).
hipError_t launch_cells(const Shape& s, bool gf16, const float* G, size_t G_stride, const void* F, size_t F_stride,
                        const SortWs& sw, int64_t n, const CellWs& cw, float* dF, size_t dF_stride, int dF_paper,
                        int accumulate, bool want_dG, double* dG, size_t dG_stride, int dG_rows, int dG_accumulate, int nb,
                        const int32_t* active, hipStream_t st, int unroll = 4, const int32_t* dG_active = nullptr,
                        int cell_kernel = 0, int cell_group = kDefaultCellGroup) {
  CellArgs c;
  memset(&c, 0, sizeof(c));
  c.s = s; c.G = G; c.G_stride = G_stride; c.F = F; c.F_stride = F_stride;
  c.pts4 = sw.spts4; c.n = n; c.start = sw.start; c.dY = cw.dY; c.CC = cw.CC;
  c.dGpart = cw.dGpart; c.active = active; c.nblk = cell_blocks(s);
  const int64_t nblocks = (int64_t)cell_blocks(s) * s.M * nb;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblocks);
#define APMG_PULL(CC_, F16_, DG_)                                                                   \
  {                                                                                                 \
    if (unroll == 2) hipLaunchKernelGGL((k_cell_pull<CC_, F16_, DG_, 2>), grid, dim3(256), 0, st, c); \
    else if (unroll == 8) hipLaunchKernelGGL((k_cell_pull<CC_, F16_, DG_, 8>), grid, dim3(256), 0, st, c); \
    else hipLaunchKernelGGL((k_cell_pull<CC_, F16_, DG_, 4>), grid, dim3(256), 0, st, c);           \
  }
  const int64_t wgroups = (int64_t)wave_groups(s) * s.M * nb;
  if (wgroups > 0x7fffffff) return hipErrorInvalidValue;
  const bool wave_kernel = cell_kernel != 1;
#define APMG_WAVE(CC_, F16_, DG_)                                                                   \
  {                                                                                                 \
    const dim3 wg((unsigned)wgroups);                                                               \
    if (cell_group == 1) hipLaunchKernelGGL((k_cell_pull_wave<CC_, F16_, 1, DG_>), wg, dim3(256), 0, st, c); \
    else if (cell_group == 2) hipLaunchKernelGGL((k_cell_pull_wave<CC_, F16_, 2, DG_>), wg, dim3(256), 0, st, c); \
    else if (cell_group == 8) hipLaunchKernelGGL((k_cell_pull_wave<CC_, F16_, 8, DG_>), wg, dim3(256), 0, st, c); \
    else hipLaunchKernelGGL((k_cell_pull_wave<CC_, F16_, 4, DG_>), wg, dim3(256), 0, st, c);         \
  }
#define APMG_CELL(CC_, F16_)                                                                        \
  if (s.C == CC_ && gf16 == F16_) {                                                                 \
    prof_begin(st, 1);                                                                              \
    if (wave_kernel) {                                                                              \
      if (want_dG) APMG_WAVE(CC_, F16_, true) else APMG_WAVE(CC_, F16_, false)                      \
    } else if (want_dG) APMG_PULL(CC_, F16_, true)                                                   \
    else APMG_PULL(CC_, F16_, false)                                                                 \
    prof_end(st, 1);                                                                                \
    if (dF && wave_kernel)                                                                          \
      hipLaunchKernelGGL((k_block_to_vertex<CC_>), dim3(grid1((int64_t)s.R * s.R * s.R, 1024), s.M, nb),   \
                         dim3(256), 0, st, s, cw.CC, dF, dF_stride, dF_paper, accumulate, active);    \
    else if (dF) hipLaunchKernelGGL((k_cell_to_vertex<CC_>), dim3(grid1((int64_t)s.R * s.R * s.R, 1024), s.M, nb), \
                                    dim3(256), 0, st, s, cw.CC, dF, dF_stride, dF_paper, accumulate, active); \
  }
  APMG_CELL(1, false) APMG_CELL(2, false) APMG_CELL(4, false)
  APMG_CELL(1, true) APMG_CELL(2, true) APMG_CELL(4, true)
#undef APMG_CELL
#undef APMG_WAVE
#undef APMG_PULL
  if (dG)
    hipLaunchKernelGGL(k_reduce_cell_dG, dim3(s.M, nb), dim3(256), 0, st, cw.dGpart, s.M, dg_parts(s, cell_kernel), dG,
                       dG_stride, dG_rows, dG_accumulate, dG_active ? dG_active : active);
  return hipGetLastError();
}

// Shapes outside the register-resident adjoint (H != 64 or more than 64 input features) take
// their weight gradients from stored per-point activations and k_dw_gemm, in one adjoint pass
// with no LDS accumulators (deterministic, no multi-pass recomputation of the forward).
bool act_path(const Shape& s, bool bf) { return !(plan_passes(s, bf, true).size() == 1 && register_kb(s) > 0); }
inline int64_t act_ld(int64_t n) { return (std::max<int64_t>(n, 1) + 31) / 32 * 32; }
inline int gemm_chunks(int64_t n) { return (int)((act_ld(n) + kGemmChunk - 1) / kGemmChunk); }
inline int gemm_part_len(const Shape& s) { return s.H * s.MC + s.H * s.H; }

struct BwdWs { FwdWs f; double* part; SortWs srt; CellWs cell; void* act; double* gpart; OpsWs ops; };
size_t bwd_ws(const Shape& s, const apmg_model* m, int64_t n, void* ws, BwdWs* o) {
  Carver cv(ws);
  BwdWs w;
  const bool bf = m->mlp_dtype == APMG_BF16;
  const size_t esz = bf ? 2 : 4;
  take_ops(cv, s, 1, g_rows(m) == 4, paper_grids(m), m->grid_dtype == APMG_F16, &w.ops);
  w.f.swz = cv.take<char>(swz_sizes(s).total() * esz);
  w.f.w3s = cv.take<float>(s.H);
  w.part = cv.take<double>((size_t)bwd_blocks(n, bf) * max_part_len(s, bf));
  take_sort(cv, n, 1, true, &w.srt);
  take_cell(cv, s, n, 1, &w.cell);
  w.act = nullptr;
  w.gpart = nullptr;
  if (act_path(s, bf)) {
    w.act = cv.take<char>((size_t)(s.MC + 3 * s.H) * act_ld(n) * esz);
    w.gpart = cv.take<double>((size_t)gemm_chunks(n) * gemm_part_len(s));
  }
  if (o) *o = w;
  return cv.off;
}

int dens_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, kDensBlocks)); }
int dens_chunks(int64_t n) { return (int)std::max<int64_t>(1, (n + kDensChunk - 1) / kDensChunk); }

struct DenWs { float *rho, *coef; double *pa, *sums, *pb1, *lq, *pb2, *U, *a; };
size_t den_ws(const Shape& s, int64_t n, int nb, void* ws, DenWs* o) {
  Carver cv(ws);
  DenWs d;
  d.rho = cv.take<float>((size_t)nb * std::max<int64_t>(n, 1));
  d.coef = cv.take<float>((size_t)nb * std::max<int64_t>(n, 1));
  d.pa = cv.take<double>((size_t)nb * kDensBlocks * 2);
  d.sums = cv.take<double>((size_t)nb * 2);
  d.pb1 = cv.take<double>((size_t)nb * kDensBlocks * 3);
  d.lq = cv.take<double>((size_t)nb * 3);
  d.pb2 = cv.take<double>((size_t)nb * dens_chunks(n) * 13 * s.M);
  d.U = cv.take<double>((size_t)nb * 13 * s.M);
  d.a = cv.take<double>((size_t)nb * std::max<int64_t>(n, 1));
  if (o) *o = d;
  return cv.off;
}

// apmg_density_loss: the packed transforms (4-row input) and the density buffers.
size_t den_model_ws(const Shape& s, const apmg_model* m, int64_t n, void* ws, OpsWs* ops, DenWs* o) {
  Carver cv(ws);
  OpsWs w;
  take_ops(cv, s, 1, g_rows(m) == 4, false, false, &w);
  const size_t off = cv.off;
  const size_t dsz = den_ws(s, n, 1, ws ? (char*)ws + off : nullptr, o);
  if (ops) *ops = w;
  return off + dsz;
}

// Density loss launch sequence for nb models sharing one shape.  pts/err/rho are per
// model with the given strides; outputs loss (stride lstride) and dG (stride dG_stride).
// flags: APMG_DENSITY_ABS_DET, APMG_DENSITY_NORM_TARGET; dG has dG_rows rows per transform.
// Pass A of the training step over the batch as drawn (counter stream), before the sort has
// finished: rho in draw order into w.rho and the rho half of the pass-A partials.
void launch_density_a_gen(const Shape& s, const float* G, size_t G_stride, uint64_t seed, const uint64_t* step_ctr,
                          uint32_t stream0, int64_t n, int p, uint32_t flags, const DenWs& w, int nb,
                          const int32_t* active, hipStream_t st) {
  const int abs_det = (flags & APMG_DENSITY_ABS_DET) ? 1 : 0;
  const size_t rho_stride = (size_t)std::max<int64_t>(n, 1);
  const int ba = dens_blocks(n);
  const size_t shA = 64 + (size_t)13 * s.M * 4;
  if (p == 10)
    hipLaunchKernelGGL((k_density_a<10, true>), dim3(ba, nb), dim3(256), shA, st, s, G, G_stride, (const float*)nullptr,
                       (int64_t)0, (size_t)0, n, (const float*)nullptr, (size_t)0, p, abs_det, w.rho, rho_stride, w.pa,
                       active, seed, step_ctr, stream0);
  else
    hipLaunchKernelGGL((k_density_a<0, true>), dim3(ba, nb), dim3(256), shA, st, s, G, G_stride, (const float*)nullptr,
                       (int64_t)0, (size_t)0, n, (const float*)nullptr, (size_t)0, p, abs_det, w.rho, rho_stride, w.pa,
                       active, seed, step_ctr, stream0);
}

// rho_perm (the training step): pass A already ran over the drawn batch (launch_density_a_gen,
// rho in draw order); only its error sums are formed here and B1 reads rho through rho_perm.
hipError_t launch_density(const Shape& s, const float* G, size_t G_stride, const float* pts, int64_t ld,
                          size_t pts_stride, int64_t n, const float* err, size_t err_stride, double eps,
                          int p, uint32_t flags, double* loss, int lstride, double* dG, size_t dG_stride, int dG_rows,
                          int accumulate, float* rho_user, const DenWs& w, int nb, const int32_t* active,
                          hipStream_t st, const uint32_t* rho_perm = nullptr) {
  const int abs_det = (flags & APMG_DENSITY_ABS_DET) ? 1 : 0, norm = (flags & APMG_DENSITY_NORM_TARGET) ? 1 : 0;
  float* rho = rho_user ? rho_user : w.rho;
  const size_t rho_stride = rho_user ? (size_t)n : (size_t)std::max<int64_t>(n, 1);
  const int ba = dens_blocks(n), nch = dens_chunks(n);
  const size_t shA = 64 + (size_t)13 * s.M * 4;
  if (rho_perm)
    hipLaunchKernelGGL(k_density_errsum, dim3(ba, nb), dim3(256), 0, st, err, err_stride, n, w.pa, active);
  else if (p == 10)
    hipLaunchKernelGGL(k_density_a<10>, dim3(ba, nb), dim3(256), shA, st, s, G, G_stride, pts, ld, pts_stride, n,
                       err, err_stride, p, abs_det, rho, rho_stride, w.pa, active, 0, nullptr, 0);
  else
    hipLaunchKernelGGL(k_density_a<0>, dim3(ba, nb), dim3(256), shA, st, s, G, G_stride, pts, ld, pts_stride, n,
                       err, err_stride, p, abs_det, rho, rho_stride, w.pa, active, 0, nullptr, 0);
  hipLaunchKernelGGL(k_density_sums, dim3(nb), dim3(256), 0, st, w.pa, ba, w.sums, nb);
  const size_t astride = (size_t)std::max<int64_t>(n, 1);
  hipLaunchKernelGGL(k_density_b1, dim3(ba, nb), dim3(256), 0, st, rho, rho_stride, err, err_stride, n,
                     w.sums, eps, w.pb1, w.a, astride, active, rho_perm);
  hipLaunchKernelGGL(k_density_lq, dim3(nb), dim3(256), 0, st, w.pb1, ba, n, w.lq, nb, norm);
  if (dG) {
    const size_t cstride = (size_t)std::max<int64_t>(n, 1);
    hipLaunchKernelGGL(k_density_coef, dim3(grid1(n, 2048), nb), dim3(256), 0, st, w.a, astride, n, w.sums, w.lq,
                       w.coef, cstride, active);
    if (p == 10)
      hipLaunchKernelGGL(k_density_b2<10>, dim3(nch, (s.M + 3) / 4, nb), dim3(256), 0, st, s, G, G_stride, pts,
                         ld, pts_stride, n, w.coef, cstride, p, w.pb2, active);
    else
      hipLaunchKernelGGL(k_density_b2<0>, dim3(nch, (s.M + 3) / 4, nb), dim3(256), 0, st, s, G, G_stride, pts,
                         ld, pts_stride, n, w.coef, cstride, p, w.pb2, active);
    hipLaunchKernelGGL(k_density_b2_reduce, dim3(s.M, nb), dim3(256), 0, st, w.pb2, s.M, nch, w.U,
                       active);
    hipLaunchKernelGGL(k_density_grad, dim3(1, nb), dim3(64), 0, st, s, G, G_stride, w.U, p, abs_det, dG, dG_stride,
                       dG_rows, accumulate, w.sums, active);
  }
  if (loss) hipLaunchKernelGGL(k_copy_f64, dim3((nb + 63) / 64), dim3(64), 0, st, w.lq, 3, loss, lstride, nb, 1.0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- training step
struct StepWs {
  float* v;       // [nb][n] ground truth at the sorted points
  float* err;     // [nb][n]
  void* swz;      // [nb][swizzled weights]
  float* w3s;     // [nb][H]
  float* scale;   // [2][nb]: vmax - vmin, then vmin
  float* dF;      // [nb][F]
  float* dW;      // [nb][W]
  double* dG;     // [nb][12 M]  transform gradient used by Adam
  double* lrec;   // [nb] sum (f - v)^2
  double* part;   // adjoint partials
  int32_t* live;  // [nb] models that train this step (not frozen)
  int32_t* dlive; // [nb] models whose transforms train this step
  SortWs srt;
  CellWs cell;
  DenWs den;
  void* act;      // activation path: [nb][tiles][MC + 3H][32] (float32 or bf16)
  double* gpart;  // [nb][chunks][H*MC + H*H]
  OpsWs ops;      // gather mirror of the grids (paper order or F16 gathers), else unused
};

size_t w_elems(const Shape& s) { return (size_t)s.H * s.MC + (size_t)s.H * s.H + s.H; }

size_t step_ws(const apmg_batch* b, const Shape& s, void* ws, StepWs* o) {
  Carver cv(ws);
  const bool bf = b->shape.mlp_dtype == APMG_BF16;
  const int nb = b->nb;
  const int64_t n = std::max<int64_t>(b->n, 1);
  StepWs w;
  take_ops(cv, s, nb, false, paper_grids(&b->shape) || b->shape.grid_dtype == APMG_F16,
           b->shape.grid_dtype == APMG_F16, &w.ops);
  w.v = cv.take<float>((size_t)nb * n);
  w.err = cv.take<float>((size_t)nb * n);
  w.swz = cv.take<char>((size_t)nb * swz_sizes(s).total() * (bf ? 2 : 4));
  w.w3s = cv.take<float>((size_t)nb * s.H);
  w.scale = cv.take<float>((size_t)nb * 2);
  w.dF = cv.take<float>((size_t)nb * f_elems(s));
  w.dW = cv.take<float>((size_t)nb * w_elems(s));
  w.dG = cv.take<double>((size_t)nb * 12 * s.M);
  w.lrec = cv.take<double>((size_t)nb);
  w.part = cv.take<double>((size_t)nb * step_max_blocks(b->n, nb) * max_part_len(s, bf));
  w.live = cv.take<int32_t>((size_t)nb);
  w.dlive = cv.take<int32_t>((size_t)nb);
  take_sort(cv, b->n, nb, false, &w.srt);
  take_cell(cv, s, b->n, nb, &w.cell);
  w.act = nullptr;
  w.gpart = nullptr;
  if (act_path(s, bf)) {
    w.act = cv.take<char>((size_t)nb * (s.MC + 3 * s.H) * act_ld(b->n) * (bf ? 2 : 4));
    w.gpart = cv.take<double>((size_t)nb * gemm_chunks(b->n) * gemm_part_len(s));
  }
  size_t off = cv.off;
  DenWs d;
  size_t dsz = den_ws(s, b->n, nb, ws ? (char*)ws + off : nullptr, &d);
  w.den = d;
  if (o) *o = w;
  return off + dsz;
}

__global__ void k_brick_scale(const apmg_brick* bricks, float* scale, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) { scale[b] = bricks[b].vmax - bricks[b].vmin; scale[nb + b] = bricks[b].vmin; }
}

// A side stream per device (default priority, non-blocking) and its fork/join events,
// created on the first training step that runs on that device outside graph capture; a
// step captured before that runs all its phases on the caller's stream.
struct SideStream { hipStream_t s = nullptr; hipEvent_t fork = nullptr, join = nullptr; bool ok = false; };
constexpr int kMaxDevices = 64;
std::mutex g_side_mu;
SideStream g_side[kMaxDevices];
SideStream* side_stream(hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  SideStream& ss = g_side[dev];
  if (!ss.ok) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    if (!ss.s && hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking) != hipSuccess) { ss.s = nullptr; return nullptr; }
    if (!ss.fork && hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) != hipSuccess) { ss.fork = nullptr; return nullptr; }
    if (!ss.join && hipEventCreateWithFlags(&ss.join, hipEventDisableTiming) != hipSuccess) { ss.join = nullptr; return nullptr; }
    ss.ok = true;
  }
  return &ss;
}

}  // namespace


// ======================================================================== ABI
// domain-decomposition inference workspace (defined with its entry point below)
struct DdWs;
size_t dd_ws(const Shape& s, const apmg_model* shape, int nb, int64_t n, void* ws, DdWs* o);

extern "C" {

apmg_status apmg_profile_kernel_events(int32_t kernel, hipEvent_t start, hipEvent_t stop) {
  if ((start == nullptr) != (stop == nullptr) || kernel < 0 || kernel > 1) return APMG_EINVAL;
  g_prof_start[kernel] = start;
  g_prof_stop[kernel] = stop;
  return APMG_OK;
}

apmg_status apmg_profile_events(hipEvent_t start, hipEvent_t stop) {
  return apmg_profile_kernel_events(APMG_PROF_ADJOINT, start, stop);
}

const char* apmg_status_string(apmg_status s) {
  switch (s) {
    case APMG_OK: return "ok";
    case APMG_EINVAL: return "invalid argument";
    case APMG_EUNSUPPORTED: return "unsupported shape or dtype";
    case APMG_EWORKSPACE: return "workspace too small";
    case APMG_EHIP: return "HIP launch error";
  }
  return "unknown status";
}

size_t apmg_workspace_bytes(int op, const void* mb, int64_t n) {
  if (!mb || n < 0) return 0;
  if (op == APMG_OP_BATCHED_STEP) {
    const apmg_batch* b = (const apmg_batch*)mb;
    Shape s;
    if (b->nb < 1 || b->n < 0 || check_model(&b->shape, false, &s) != APMG_OK) return 0;
    return step_ws(b, s, nullptr, nullptr);
  }
  if (op == APMG_OP_DD_FORWARD) {
    const apmg_dd_models* d = (const apmg_dd_models*)mb;
    Shape s;
    if (d->nb < 1 || check_model(&d->shape, false, &s) != APMG_OK) return 0;
    return dd_ws(s, &d->shape, d->nb, n, nullptr, nullptr);
  }
  Shape s;
  const apmg_model* m = (const apmg_model*)mb;
  if (check_model(m, false, &s) != APMG_OK) return 0;
  switch (op) {
    case APMG_OP_FORWARD: return fwd_ws(s, m, n, nullptr, nullptr);
    case APMG_OP_BACKWARD: return bwd_ws(s, m, n, nullptr, nullptr);
    case APMG_OP_DENSITY: return den_model_ws(s, m, n, nullptr, nullptr, nullptr);
  }
  return 0;
}

}  // extern "C"

// The forward pass's scratch for callers that cannot allocate: one array per device, held
// until the process ends.  In host code `scratch` names a host-side stand-in; the device
// address comes from hipGetSymbolAddress, once per device with that device current, and
// only that address is passed on.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
// apmg_forward on a given workspace; sortable = false keeps to the direct tile path.
apmg_status forward_impl(const apmg_model* m, const float* pts, int64_t ld, int64_t n, float* f, void* ws,
                         size_t ws_bytes, hipStream_t st, bool sortable) {
  Shape s;
  apmg_status rc = check_model(m, true, &s);
  if (rc != APMG_OK) return rc;
  if ((rc = check_points(pts, ld, n)) != APMG_OK) return rc;
  if (n > 0 && !f) return APMG_EINVAL;
  const bool bf = m->mlp_dtype == APMG_BF16, gf16 = m->grid_dtype == APMG_F16;
  if (ws_bytes < fwd_ws(s, m, n, nullptr, nullptr, sortable) || !ws) return APMG_EWORKSPACE;
  if (n == 0) return APMG_OK;
  FwdWs w;
  fwd_ws(s, m, n, ws, &w, sortable);
  const float* Gc;
  const void* Fc;
  hipError_t e = launch_ops(s, 1, m->G, g_rows(m), m->F, gf16, paper_grids(m), w.ops, gf16, st, &Gc, &Fc);
  if (e != hipSuccess) return APMG_EHIP;
  e = launch_swizzle(s, bf, m->W[0], m->W[1], m->W[2], 0, w.swz, 0, w.w3s, 1, st);
  if (e != hipSuccess) return APMG_EHIP;
  if (w.sorted && (e = launch_sort(pts, ld, 0, nullptr, n, 1, w.srt, nullptr, st, false)) != hipSuccess)
    return APMG_EHIP;
  TileArgs a;
  memset(&a, 0, sizeof(a));
  a.s = s;
  a.G = Gc; a.F = Fc; a.swz = w.swz; a.w3s = w.w3s;
  a.vscale = m->vmax - m->vmin; a.voff = m->vmin;
  a.pts = pts; a.ld = ld; a.f = f;
  if (w.sorted) a.perm = w.srt.v0;   // tiles walk the spatial order, inputs and outputs in place
  a.n = n;
  const int64_t tiles = (n + 31) / 32;
  dim3 grid((unsigned)std::min<int64_t>((tiles + kWavesPerBlock - 1) / kWavesPerBlock, 8192), 1);
  e = launch_tile(false, 0, a, gf16, bf, grid, forward_lds_bytes(s, bf), st);
  if (e != hipSuccess) return APMG_EHIP;
  return hip_status(hipGetLastError());
}

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
void* device_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

apmg_status apmg_forward(const apmg_model* m, const float* pts, int64_t ld, int64_t n, float* f, void* ws,
                         size_t ws_bytes, hipStream_t st) {
  return forward_impl(m, pts, ld, n, f, ws, ws_bytes, st, true);
}

apmg_status apmg_forward_noalloc(const apmg_model* m, const float* pts, int64_t ld, int64_t n, float* f,
                                 hipStream_t st) {
  Shape s;
  apmg_status rc = check_model(m, true, &s);
  if (rc != APMG_OK) return rc;
  if ((rc = check_points(pts, ld, n)) != APMG_OK) return rc;    // before sizing: n >= 0
  if (fwd_ws(s, m, n, nullptr, nullptr, false) > kScratchBytes) return APMG_EWORKSPACE;
  void* ws = device_scratch();
  if (!ws) return APMG_EHIP;
  return forward_impl(m, pts, ld, n, f, ws, kScratchBytes, st, false);
}

size_t apmg_forward_noalloc_scratch_bytes(void) { return kScratchBytes; }

apmg_status apmg_backward(const apmg_model* m, const float* pts, int64_t ld, int64_t n, const float* df,
                          float* dF, double* dG, float* const* dW, uint32_t flags, void* ws, size_t ws_bytes,
                          hipStream_t st) {
  Shape s;
  apmg_status rc = check_model(m, true, &s);
  if (rc != APMG_OK) return rc;
  if ((rc = check_points(pts, ld, n)) != APMG_OK) return rc;
  if (n > 0 && !df) return APMG_EINVAL;
  if (dW) for (int k = 0; k < m->n_layers; ++k) if (!dW[k]) return APMG_EINVAL;
  const bool bf = m->mlp_dtype == APMG_BF16, gf16 = m->grid_dtype == APMG_F16;
  if (ws_bytes < bwd_ws(s, m, n, nullptr, nullptr) || !ws) return APMG_EWORKSPACE;
  const int grows = g_rows(m);
  const bool use_act = dW != nullptr && act_path(s, bf);
  const std::vector<Pass> passes = use_act ? std::vector<Pass>{{0, 0, 0, 0, true}} : plan_passes(s, bf, dW != nullptr);
  if (passes.empty()) return APMG_EUNSUPPORTED;
  const bool acc = flags & APMG_ACCUMULATE;
  const size_t nF = (size_t)s.M * s.R * s.R * s.R * s.C;
  if (!acc) {
    if (dW) {
      hipLaunchKernelGGL(k_fill_f32, dim3(grid1((int64_t)s.H * s.MC)), dim3(256), 0, st, dW[0], (size_t)s.H * s.MC, 0.f);
      hipLaunchKernelGGL(k_fill_f32, dim3(grid1((int64_t)s.H * s.H)), dim3(256), 0, st, dW[1], (size_t)s.H * s.H, 0.f);
      hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(256), 0, st, dW[2], (size_t)s.H, 0.f);
    }
    if (n == 0) {
      if (dF) hipLaunchKernelGGL(k_fill_f32, dim3(grid1(nF)), dim3(256), 0, st, dF, nF, 0.f);
      if (dG) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, st, dG, (size_t)4 * grows * s.M, 0.0);
    }
  }
  if (n == 0) return hip_status(hipGetLastError());
  BwdWs w;
  bwd_ws(s, m, n, ws, &w);
  const float* Gc;
  const void* Fc;
  hipError_t e = launch_ops(s, 1, m->G, grows, m->F, gf16, paper_grids(m), w.ops, gf16, st, &Gc, &Fc);
  if (e != hipSuccess) return APMG_EHIP;
  // points (and dL/df) in spatial-bin order
  e = launch_sort(pts, ld, 0, nullptr, n, 1, w.srt, df, st);
  if (e != hipSuccess) return APMG_EHIP;
  e = launch_swizzle(s, bf, m->W[0], m->W[1], m->W[2], 0, w.f.swz, 0, w.f.w3s, 1, st);
  if (e != hipSuccess) return APMG_EHIP;
  const int nblk = bwd_blocks(n, bf);
  const bool want_cells = dF || dG;
  const int kb = (!use_act && passes.size() == 1) ? register_kb(s) : 0;
  for (const Pass& ps : passes) {
    TileArgs a;
    memset(&a, 0, sizeof(a));
    a.s = s;
    a.G = Gc; a.F = Fc; a.swz = w.f.swz; a.w3s = w.f.w3s;
    a.act = use_act ? w.act : nullptr;
    a.act_rows = s.MC + 3 * s.H;
    a.vscale = m->vmax - m->vmin; a.voff = m->vmin;
    a.pts = w.srt.spts; a.ld = n; a.n = n;
    a.df = w.srt.sf;
    a.dY = (ps.first && want_cells) ? w.cell.dY : nullptr;
    a.c1_lo = ps.c1_lo; a.c1_hi = ps.c1_hi;
    a.w2_lo = ps.w2_lo; a.w2_hi = ps.w2_hi;
    a.do_w3 = (ps.first && dW) ? 1 : 0;
    a.part = w.part;
    const int ncols = ps.c1_hi - ps.c1_lo, nrows = ps.w2_hi - ps.w2_lo;
    const PartLayout pl = part_layout(s, ncols, nrows);
    a.part_len = pl.len;
    if (ps.first) prof_begin(st, 0);
    e = kb > 0 ? launch_adjoint(a, gf16, bf, 0, dim3(nblk, 1), st)
               : launch_tile(true, kb, a, gf16, bf, dim3(nblk, 1), backward_lds_bytes(s, ncols, nrows, bf, kb), st);
    if (e != hipSuccess) return APMG_EHIP;
    if (&ps == &passes.back()) prof_end(st, 0);
    if (ncols > 0)
      hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * ncols), 1), dim3(256), 0, st, w.part,
                         nblk, pl.len, pl.o_w1, s.H * ncols, ncols, s.MC, ps.c1_lo, dW[0], (double*)nullptr,
                         (size_t)0, 1, (const int32_t*)nullptr);
    if (nrows > 0)
      hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * nrows), 1), dim3(256), 0, st, w.part, nblk,
                         pl.len, pl.o_w2, s.H * nrows, s.H * nrows, 0, ps.w2_lo * s.H, dW[1], (double*)nullptr,
                         (size_t)0, 1, (const int32_t*)nullptr);
    if (a.do_w3)
      hipLaunchKernelGGL(k_reduce_parts, dim3(1, 1), dim3(256), 0, st, w.part, nblk, pl.len, pl.o_w3, s.H, s.H, 0,
                         0, dW[2], (double*)nullptr, (size_t)0, 1, (const int32_t*)nullptr);
  }
  // the weight-gradient products (activation path) and the grid-gradient gather both read
  // what the adjoint kernel wrote and write disjoint outputs: the products run on the
  // device's side stream, overlapping the gather
  std::unique_lock<std::mutex> lk(g_side_mu, std::defer_lock);
  hipStream_t pst = st;
  SideStream* side = nullptr;
  if (use_act && want_cells) {
    lk.lock();
    side = side_stream(st);
    if (side && hipEventRecord(side->fork, st) == hipSuccess && hipStreamWaitEvent(side->s, side->fork, 0) == hipSuccess)
      pst = side->s;
  }
  if (use_act) {
    // dW1 = sum_p delta1_p y_p^T and dW2 = sum_p delta2_p h1_p^T from the stored activations
    // (rows of each tile's block: y [0, MC), h1 [MC, MC+H), delta1 [MC+H, ..), delta2 [MC+2H, ..))
    const int64_t np = act_ld(n);
    const int rows_tot = s.MC + 3 * s.H;
    const int nch = gemm_chunks(n), plen = gemm_part_len(s);
    const dim3 g1(nch, (s.H + 127) / 128, (s.MC + 127) / 128), g2(nch, (s.H + 127) / 128, (s.H + 127) / 128);
    if (bf) {
      hipLaunchKernelGGL(k_dw_gemm<true>, g1, dim3(256), 0, pst, w.act, rows_tot, s.MC + s.H, 0, np, s.H, s.MC,
                         w.gpart, plen, 0);
      hipLaunchKernelGGL(k_dw_gemm<true>, g2, dim3(256), 0, pst, w.act, rows_tot, s.MC + 2 * s.H, s.MC, np, s.H, s.H,
                         w.gpart, plen, s.H * s.MC);
    } else {
      hipLaunchKernelGGL(k_dw_gemm<false>, g1, dim3(256), 0, pst, w.act, rows_tot, s.MC + s.H, 0, np, s.H, s.MC,
                         w.gpart, plen, 0);
      hipLaunchKernelGGL(k_dw_gemm<false>, g2, dim3(256), 0, pst, w.act, rows_tot, s.MC + 2 * s.H, s.MC, np, s.H,
                         s.H, w.gpart, plen, s.H * s.MC);
    }
    hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * s.MC), 1), dim3(256), 0, pst, w.gpart, nch,
                       plen, 0, s.H * s.MC, s.MC, s.MC, 0, dW[0], (double*)nullptr, (size_t)0, 1,
                       (const int32_t*)nullptr);
    hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * s.H), 1), dim3(256), 0, pst, w.gpart, nch,
                       plen, s.H * s.MC, s.H * s.H, s.H, s.H, 0, dW[1], (double*)nullptr, (size_t)0, 1,
                       (const int32_t*)nullptr);
  }
  hipError_t ec = hipSuccess;
  if (want_cells)
    ec = launch_cells(s, gf16, Gc, 0, Fc, 0, w.srt, n, w.cell, dF, 0, paper_grids(m) ? 1 : 0, acc ? 1 : 0,
                      dG != nullptr, dG, 0, grows, acc ? 1 : 0, 1, nullptr, st);
  hipError_t ej = hipSuccess;
  if (pst != st) {
    ej = hipEventRecord(side->join, pst);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(st, side->join, 0);
  }
  if (ec != hipSuccess || ej != hipSuccess) return APMG_EHIP;
  return hip_status(hipGetLastError());
}

apmg_status apmg_density_loss(const apmg_model* m, const float* pts, int64_t ld, int64_t n, const float* err,
                              double eps, int32_t p, double* loss, double* dG, float* rho, uint32_t flags,
                              void* ws, size_t ws_bytes, hipStream_t st) {
  Shape s;
  if (!m || !m->G) return APMG_EINVAL;
  apmg_status rc = check_model(m, false, &s);
  if (rc != APMG_OK) return rc;
  if ((rc = check_points(pts, ld, n)) != APMG_OK) return rc;
  if (!loss || (n > 0 && !err) || p < 1 || !(eps >= 0.0)) return APMG_EINVAL;
  if (ws_bytes < den_model_ws(s, m, n, nullptr, nullptr, nullptr) || !ws) return APMG_EWORKSPACE;
  const bool acc = flags & APMG_ACCUMULATE;
  const int grows = g_rows(m);
  if (n == 0) {
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, st, loss, (size_t)1, 0.0);
    if (dG && !acc) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, st, dG, (size_t)4 * grows * s.M, 0.0);
    return hip_status(hipGetLastError());
  }
  DenWs w;
  OpsWs ops;
  den_model_ws(s, m, n, ws, &ops, &w);
  const float* Gc;
  if (launch_ops(s, 1, m->G, grows, nullptr, false, false, ops, false, st, &Gc, nullptr) != hipSuccess)
    return APMG_EHIP;
  return hip_status(launch_density(s, Gc, 0, pts, ld, 0, n, err, 0, eps, p, flags, loss, 1, dG, 0, grows,
                                   acc ? 1 : 0, rho, w, 1, nullptr, st));
}

apmg_status apmg_cells(const apmg_model* m, const float* pts, int64_t ld, int64_t n, int32_t* cell,
                       uint8_t* inside, hipStream_t st) {
  Shape s;
  if (!m || !m->G) return APMG_EINVAL;
  if (m->M < 1 || m->R < 2) return APMG_EINVAL;
  apmg_status rc = check_points(pts, ld, n);
  if (rc != APMG_OK) return rc;
  if (n == 0) return APMG_OK;
  if (!cell && !inside) return APMG_EINVAL;
  if (!(m->G_rows == 0 || m->G_rows == 3 || m->G_rows == 4)) return APMG_EINVAL;
  s.M = m->M; s.C = m->C; s.R = m->R;
  hipLaunchKernelGGL(k_cells, dim3(grid1(n * m->M)), dim3(256), 0, st, s, m->G, g_rows(m), pts, ld, n, cell, inside);
  return hip_status(hipGetLastError());
}

apmg_status apmg_uniform_points(uint64_t seed, uint64_t step, uint32_t stream_id, int64_t start, int64_t n,
                                float* pts, int64_t ld, hipStream_t st) {
  if (n < 0 || start < 0 || ld < n || (n > 0 && !pts)) return APMG_EINVAL;
  if (n == 0) return APMG_OK;
  hipLaunchKernelGGL(k_uniform_points, dim3(grid1(n)), dim3(256), 0, st, seed, step, stream_id, start, n, pts, ld);
  return hip_status(hipGetLastError());
}

apmg_status apmg_gt_sample(const float* volume, int32_t nx, int32_t ny, int32_t nz, const float* pts, int64_t ld,
                           int64_t n, float* v, hipStream_t st) {
  if (!volume || nx < 2 || ny < 2 || nz < 2) return APMG_EINVAL;
  apmg_status rc = check_points(pts, ld, n);
  if (rc != APMG_OK) return rc;
  if (n == 0) return APMG_OK;
  if (!v) return APMG_EINVAL;
  hipLaunchKernelGGL(k_gt_sample, dim3(grid1(n)), dim3(256), 0, st, volume, nx, ny, nz, pts, ld, n, v);
  return hip_status(hipGetLastError());
}

apmg_status apmg_make_bricks(int32_t nx, int32_t ny, int32_t nz, int32_t B, int32_t ghost,
                             apmg_brick_table* t, apmg_brick* bricks, int32_t cap) {
  if (!t || nx < 2 || ny < 2 || nz < 2 || B < 1 || ghost < 0) return APMG_EINVAL;
  const int32_t n3[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d) { t->vol[d] = n3[d]; t->dims[d] = (n3[d] + B - 1) / B; }
  t->B = B;
  t->ghost = ghost;
  const int64_t nb = (int64_t)t->dims[0] * t->dims[1] * t->dims[2];
  if (!bricks) return APMG_OK;
  if (cap < nb) return APMG_EINVAL;
  int64_t id = 0;
  for (int k = 0; k < t->dims[2]; ++k)
    for (int j = 0; j < t->dims[1]; ++j)
      for (int i = 0; i < t->dims[0]; ++i, ++id) {
        apmg_brick& b = bricks[id];
        const int ijk[3] = {i, j, k};
        for (int d = 0; d < 3; ++d) {
          b.ijk[d] = ijk[d];
          b.e0[d] = std::max(ijk[d] * B - ghost, 0);
          b.e1[d] = std::min((ijk[d] + 1) * B - 1 + ghost, n3[d] - 1);
        }
        b.vmin = 0.f;
        b.vmax = 1.f;
      }
  return APMG_OK;
}

apmg_status apmg_assign_bricks(const apmg_brick_table* t, const float* pts, int64_t ld, int64_t n, int32_t* brick,
                               hipStream_t st) {
  if (!t || t->B < 1) return APMG_EINVAL;
  for (int d = 0; d < 3; ++d) if (t->dims[d] < 1 || t->vol[d] < 2) return APMG_EINVAL;
  apmg_status rc = check_points(pts, ld, n);
  if (rc != APMG_OK) return rc;
  if (n == 0) return APMG_OK;
  if (!brick) return APMG_EINVAL;
  hipLaunchKernelGGL(k_assign_bricks, dim3(grid1(n)), dim3(256), 0, st, *t, pts, ld, n, brick);
  return hip_status(hipGetLastError());
}

apmg_status apmg_convert_grids(int32_t M, int32_t C, int32_t R, const void* src, int32_t sd, void* dst, int32_t dd,
                               int32_t to_cl, hipStream_t st) {
  if (M < 1 || C < 1 || R < 2 || !src || !dst) return APMG_EINVAL;
  if (!((sd == APMG_F32 || sd == APMG_F16) && (dd == APMG_F32 || dd == APMG_F16))) return APMG_EUNSUPPORTED;
  const size_t total = (size_t)M * C * R * R * R;
  const unsigned g = grid1((int64_t)total);
  if (sd == APMG_F32 && dd == APMG_F32)
    hipLaunchKernelGGL((k_convert<float, float>), dim3(g), dim3(256), 0, st, M, C, R, (const float*)src, (float*)dst, to_cl);
  else if (sd == APMG_F32 && dd == APMG_F16)
    hipLaunchKernelGGL((k_convert<float, uint16_t>), dim3(g), dim3(256), 0, st, M, C, R, (const float*)src, (uint16_t*)dst, to_cl);
  else if (sd == APMG_F16 && dd == APMG_F32)
    hipLaunchKernelGGL((k_convert<uint16_t, float>), dim3(g), dim3(256), 0, st, M, C, R, (const uint16_t*)src, (float*)dst, to_cl);
  else
    hipLaunchKernelGGL((k_convert<uint16_t, uint16_t>), dim3(g), dim3(256), 0, st, M, C, R, (const uint16_t*)src, (uint16_t*)dst, to_cl);
  return hip_status(hipGetLastError());
}

}  // extern "C"

namespace {

apmg_status check_batch(const apmg_batch* b, Shape* s) {
  if (!b || b->nb < 1 || b->n < 0) return APMG_EINVAL;
  apmg_status rc = check_model(&b->shape, false, s);
  if (rc != APMG_OK) return rc;
  if (!b->G || !b->F || !b->W || !b->mG || !b->vG || !b->mF || !b->vF || !b->mW || !b->vW || !b->t ||
      !b->tG || !b->density_active || !b->volume || !b->bricks || !b->step || !b->losses)
    return APMG_EINVAL;
  if (b->shape.G_rows == 4) return APMG_EUNSUPPORTED;
  for (int d = 0; d < 3; ++d) if (b->vol[d] < 2) return APMG_EINVAL;
  if (b->p < 1 || !(b->eps_density >= 0.0)) return APMG_EINVAL;
  // Adam: 1 - beta^t is the bias correction's divisor, so each beta lies in [0, 1)
  if (!(b->beta1 >= 0.f && b->beta1 < 1.f && b->beta2 >= 0.f && b->beta2 < 1.f && b->adam_eps >= 0.f &&
        b->lr >= 0.f && b->lr_G >= 0.f))
    return APMG_EINVAL;
  return APMG_OK;
}

// The phases of one training step; `update` adds the Adam updates and counter increments.
apmg_status run_step(const apmg_batch* b, const Shape& s, void* ws, const Tune& tu, bool update, hipStream_t st) {
  const bool bf = b->shape.mlp_dtype == APMG_BF16, gf16 = b->shape.grid_dtype == APMG_F16;
  const int nb = b->nb;
  const int64_t n = b->n;
  StepWs w;
  step_ws(b, s, ws, &w);
  const size_t nF = f_elems(s), nW = w_elems(s), nG = (size_t)12 * s.M;
  const size_t swz_stride = swz_sizes(s).total();
  hipLaunchKernelGGL(k_live_masks, dim3((nb + 63) / 64), dim3(64), 0, st, b->frozen, b->density_active, w.live,
                     w.dlive, nb);
  const bool paper = paper_grids(&b->shape);
  const void* Fg = nullptr;
  hipError_t e = hipSuccess;
  {
    // The gather copy of the grids, the weights' operands, the output scaling and the zeroed
    // gradients do not depend on the batch points: they run on the device's side stream while
    // the points are generated, sorted and sampled.
    std::lock_guard<std::mutex> lk(g_side_mu);     // one fork..join at a time per process
    SideStream* side = n > 0 ? side_stream(st) : nullptr;
    hipStream_t pst = st;
    if (side && hipEventRecord(side->fork, st) == hipSuccess && hipStreamWaitEvent(side->s, side->fork, 0) == hipSuccess)
      pst = side->s;
    // the grids the encoder gathers: the masters themselves (channel-last float32) or their
    // mirror (paper order, or F16 gathers); the step's transforms are [nb][M][3][4] already
    const float* Gc;
    if (launch_ops(s, nb, b->G, 3, b->F, false, paper, w.ops, gf16, pst, &Gc, &Fg) != hipSuccess) return APMG_EHIP;
    (void)Gc;
    // 2. operands of this step's weights, output scaling, zeroed gradients
    e = launch_swizzle(s, bf, b->W, b->W + (size_t)s.H * s.MC, b->W + (size_t)s.H * s.MC + (size_t)s.H * s.H, nW,
                       w.swz, swz_stride, w.w3s, nb, pst);
    if (e != hipSuccess) return APMG_EHIP;
    hipLaunchKernelGGL(k_brick_scale, dim3((nb + 63) / 64), dim3(64), 0, pst, b->bricks, w.scale, nb);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid1((int64_t)(nb * nW))), dim3(256), 0, pst, w.dW, nb * nW, 0.f);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, pst, w.lrec, (size_t)nb, 0.0);
    // an empty batch: every gradient of the (empty) losses is zero, the transforms' included
    // (the density chain that writes dG runs only for a non-empty batch)
    if (n == 0) {
      hipLaunchKernelGGL(k_fill_f32, dim3(grid1((int64_t)(nb * nF))), dim3(256), 0, pst, w.dF, nb * nF, 0.f);
      hipLaunchKernelGGL(k_fill_f64, dim3(grid1((int64_t)(nb * nG))), dim3(256), 0, pst, w.dG, nb * nG, 0.0);
    }
    // pass A of the density loss needs the drawn points and the transforms only: beside the sort
    if (n > 0)
      launch_density_a_gen(s, b->G, nG, b->seed, b->step, b->stream0, n, b->p, b->flags, w.den, nb, w.dlive, pst);
    // 1. batch points, sorted by spatial bin, and the ground truth at the sorted points
    if (n > 0) {
      hipError_t e0 = launch_step_sort(b->seed, b->step, b->stream0, n, nb, w.srt, b->volume, b->vol[0], b->vol[1],
                                       b->bricks, w.v, st);
      if (e0 != hipSuccess) return APMG_EHIP;
    }
    if (pst != st) {
      if (hipEventRecord(side->join, pst) != hipSuccess || hipStreamWaitEvent(st, side->join, 0) != hipSuccess)
        return APMG_EHIP;
    }
  }

  // 3. forward + adjoint of L_rec (part 1 of the step)
  const int nblk = tu.tile_blocks;
  const bool use_act = act_path(s, bf);
  const std::vector<Pass> passes = use_act ? std::vector<Pass>{{0, 0, 0, 0, true}} : plan_passes(s, bf, true);
  if (passes.empty()) return APMG_EUNSUPPORTED;
  const int kb = (!use_act && passes.size() == 1) ? register_kb(s) : 0;
  const bool rec_dG = b->flags & APMG_ADD_REC_DG;
  const size_t act_stride = (size_t)(s.MC + 3 * s.H) * act_ld(n);
  // activation path: dW1 and dW2 of every model from its stored activations
  auto act_products = [&](hipStream_t rs) {
    const int64_t np = act_ld(n);
    const int rows_tot = s.MC + 3 * s.H, nch = gemm_chunks(n), plen = gemm_part_len(s);
    const size_t esz = bf ? 2 : 4;
    const dim3 g1(nch, (s.H + 127) / 128, (s.MC + 127) / 128), g2(nch, (s.H + 127) / 128, (s.H + 127) / 128);
    for (int mb = 0; mb < nb; ++mb) {
      const void* act = (const char*)w.act + (size_t)mb * act_stride * esz;
      double* gp = w.gpart + (size_t)mb * nch * plen;
      if (bf) {
        hipLaunchKernelGGL(k_dw_gemm<true>, g1, dim3(256), 0, rs, act, rows_tot, s.MC + s.H, 0, np, s.H, s.MC, gp,
                           plen, 0);
        hipLaunchKernelGGL(k_dw_gemm<true>, g2, dim3(256), 0, rs, act, rows_tot, s.MC + 2 * s.H, s.MC, np, s.H, s.H,
                           gp, plen, s.H * s.MC);
      } else {
        hipLaunchKernelGGL(k_dw_gemm<false>, g1, dim3(256), 0, rs, act, rows_tot, s.MC + s.H, 0, np, s.H, s.MC, gp,
                           plen, 0);
        hipLaunchKernelGGL(k_dw_gemm<false>, g2, dim3(256), 0, rs, act, rows_tot, s.MC + 2 * s.H, s.MC, np, s.H, s.H,
                           gp, plen, s.H * s.MC);
      }
    }
    hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * s.MC), nb), dim3(256), 0, rs, w.gpart, nch,
                       plen, 0, s.H * s.MC, s.MC, s.MC, 0, w.dW, (double*)nullptr, nW, 0, (const int32_t*)w.live);
    hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * s.H), nb), dim3(256), 0, rs, w.gpart, nch,
                       plen, s.H * s.MC, s.H * s.H, s.H, s.H, s.H * s.MC, w.dW, (double*)nullptr, nW, 0,
                       (const int32_t*)w.live);
  };
  // block partials of one pass -> dW (and, for the first pass, dW3 and the L_rec sum)
  auto reduce_pass = [&](const Pass& ps, hipStream_t rs) {
    const int ncols = ps.c1_hi - ps.c1_lo, nrows = ps.w2_hi - ps.w2_lo;
    const PartLayout pl = part_layout(s, ncols, nrows);
    if (ncols > 0)
      hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * ncols), nb), dim3(256), 0, rs, w.part, nblk,
                         pl.len, pl.o_w1, s.H * ncols, ncols, s.MC, ps.c1_lo, w.dW, (double*)nullptr, nW, 0,
                         (const int32_t*)w.live);
    if (nrows > 0)
      hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * nrows), nb), dim3(256), 0, rs, w.part, nblk,
                         pl.len, pl.o_w2, s.H * nrows, s.H * nrows, 0, s.H * s.MC + ps.w2_lo * s.H, w.dW,
                         (double*)nullptr, nW, 0, (const int32_t*)w.live);
    if (ps.first) {
      hipLaunchKernelGGL(k_reduce_parts, dim3(1, nb), dim3(256), 0, rs, w.part, nblk, pl.len, pl.o_w3, s.H, s.H, 0,
                         s.H * s.MC + s.H * s.H, w.dW, (double*)nullptr, nW, 0, (const int32_t*)w.live);
      hipLaunchKernelGGL(k_reduce_parts, dim3(1, nb), dim3(256), 0, rs, w.part, nblk, pl.len, pl.o_loss, 1, 1, 0, 0,
                         (float*)nullptr, w.lrec, (size_t)1, 0, (const int32_t*)w.live);
    }
  };
  for (size_t pi = 0; pi < passes.size() && n > 0; ++pi) {
    const Pass& ps = passes[pi];
    TileArgs a;
    memset(&a, 0, sizeof(a));
    a.s = s;
    a.G = b->G; a.G_stride = nG;
    a.F = Fg; a.F_stride = nF;
    a.swz = w.swz; a.swz_stride = swz_stride; a.w3s = w.w3s;
    a.bscale = w.scale; a.boff = w.scale + nb;
    a.pts = w.srt.spts; a.ld = n; a.pts_stride = (size_t)3 * n; a.n = n;
    a.df = nullptr; a.v = w.v; a.v_stride = n; a.err = w.err; a.err_stride = n;
    a.err_abs = (b->flags & APMG_ERR_ABS) ? 1 : 0;
    a.dY = ps.first ? w.cell.dY : nullptr;
    a.c1_lo = ps.c1_lo; a.c1_hi = ps.c1_hi;
    a.w2_lo = ps.w2_lo; a.w2_hi = ps.w2_hi;
    a.do_w3 = ps.first;
    a.want_loss = ps.first;
    a.part = w.part;
    a.active = w.live;
    a.act = use_act ? w.act : nullptr;
    a.act_rows = s.MC + 3 * s.H;
    a.act_stride = act_stride;
    const int ncols = ps.c1_hi - ps.c1_lo, nrows = ps.w2_hi - ps.w2_lo;
    const PartLayout pl = part_layout(s, ncols, nrows);
    a.part_len = pl.len;
    if (pi == 0) prof_begin(st, 0);
    e = (kb > 0 && tu.adjoint < 3)
            ? launch_adjoint(a, gf16, bf, tu.adjoint, dim3(nblk, nb), st)
            : launch_tile(true, kb, a, gf16, bf, dim3(nblk, nb), backward_lds_bytes(s, ncols, nrows, bf, kb), st);
    if (e != hipSuccess) return APMG_EHIP;
    if (pi + 1 == passes.size()) prof_end(st, 0);
    // the last pass's reductions wait for the fork below (they overlap the gather)
    if (pi + 1 < passes.size()) reduce_pass(ps, st);
  }
  if (n == 0) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, st, b->losses, (size_t)2 * nb, 0.0);

  // 4. grid gradient from the per-cell pass (L_rec's transform gradient only under
  // APMG_ADD_REC_DG) and 5. the density loss and its transform gradient (part 2) for models
  // whose transforms train.  The gather needs dL/dy only; the last pass's weight-gradient
  // reductions, L_rec and the density passes need the adjoint's partials and errors and
  // write buffers the gather does not touch, so they run on the device's side stream,
  // overlapping the gather.
  if (n > 0) {
    std::lock_guard<std::mutex> lk(g_side_mu);     // one fork..join at a time per process
    SideStream* side = side_stream(st);
    hipStream_t dst = st;
    if (side && hipEventRecord(side->fork, st) == hipSuccess && hipStreamWaitEvent(side->s, side->fork, 0) == hipSuccess)
      dst = side->s;
    // the density chain first: it is the longer of the two streams' work, and the
    // weight-gradient reductions are needed only by Adam
    const hipError_t ed = launch_density(s, b->G, nG, w.srt.spts, n, (size_t)3 * n, n, w.err, n, b->eps_density,
                                         b->p, b->flags, b->losses + 1, 2, w.dG, nG, 3, 0, nullptr, w.den, nb,
                                         w.dlive, dst, w.srt.v0);
    reduce_pass(passes.back(), dst);
    if (use_act) act_products(dst);
    hipLaunchKernelGGL(k_copy_f64, dim3((nb + 63) / 64), dim3(64), 0, dst, w.lrec, 1, b->losses, 2, nb,
                       1.0 / (double)n);
    const hipError_t ec = launch_cells(s, gf16, b->G, nG, Fg, nF, w.srt, n, w.cell, w.dF, nF, paper ? 1 : 0, 0,
                                       rec_dG, nullptr, 0, 3, 0, nb, w.live, st, tu.cell_unroll, nullptr,
                                       tu.cell_kernel, tu.cell_group);
    hipError_t ej = hipSuccess;
    if (dst != st) {
      ej = hipEventRecord(side->join, dst);
      if (ej == hipSuccess) ej = hipStreamWaitEvent(st, side->join, 0);
    }
    if (ed != hipSuccess || ec != hipSuccess || ej != hipSuccess) return APMG_EHIP;
    if (rec_dG)
      hipLaunchKernelGGL(k_reduce_cell_dG, dim3(s.M, nb), dim3(256), 0, st, w.cell.dGpart, s.M,
                         dg_parts(s, tu.cell_kernel), w.dG, nG, 3, 1, w.dlive);
  }
  if (!update) return hip_status(hipGetLastError());

  // 6. Adam: grids and MLP every step, transforms while the density phase is active
  hipLaunchKernelGGL(k_adam, dim3(grid1(((int64_t)nF + 3) / 4), nb), dim3(256), 0, st, b->F, b->mF, b->vF, (const float*)w.dF,
                     (const double*)nullptr, nF, (const int32_t*)b->t, (const int32_t*)w.live, b->lr, b->beta1,
                     b->beta2, b->adam_eps, b->lr_scale);
  hipLaunchKernelGGL(k_adam, dim3(grid1(((int64_t)nW + 3) / 4), nb), dim3(256), 0, st, b->W, b->mW, b->vW, (const float*)w.dW,
                     (const double*)nullptr, nW, (const int32_t*)b->t, (const int32_t*)w.live, b->lr, b->beta1,
                     b->beta2, b->adam_eps, b->lr_scale);
  hipLaunchKernelGGL(k_adam, dim3(1, nb), dim3(256), 0, st, b->G, b->mG, b->vG, (const float*)nullptr,
                     (const double*)w.dG, nG, (const int32_t*)b->tG, (const int32_t*)w.dlive, b->lr_G, b->beta1,
                     b->beta2, b->adam_eps, b->lr_scale);
  hipLaunchKernelGGL(k_step_counters, dim3((nb + 63) / 64), dim3(64), 0, st, b->t, b->tG, (const int32_t*)w.live,
                     (const int32_t*)w.dlive, b->step, nb);
  return hip_status(hipGetLastError());
}

}  // namespace

extern "C" apmg_status apmg_batched_step(const apmg_batch* b, void* ws, size_t ws_bytes, hipStream_t st) {
  Shape s;
  apmg_status rc = check_batch(b, &s);
  if (rc != APMG_OK) return rc;
  Tune tu;
  if (!resolve_tune(b->tuning, b->n, b->nb, b->shape.mlp_dtype == APMG_BF16, &tu)) return APMG_EINVAL;
  if (!ws || ws_bytes < step_ws(b, s, nullptr, nullptr)) return APMG_EWORKSPACE;
  return run_step(b, s, ws, tu, true, st);
}

extern "C" apmg_status apmg_autotune_batched_step(const apmg_batch* b, void* ws, size_t ws_bytes, hipStream_t st,
                                                  apmg_tuning* best, float* best_ms) {
  Shape s;
  apmg_status rc = check_batch(b, &s);
  if (rc != APMG_OK) return rc;
  if (!best) return APMG_EINVAL;
  if (!ws || ws_bytes < step_ws(b, s, nullptr, nullptr)) return APMG_EWORKSPACE;
  const int d = step_default_blocks(b->n, b->nb), mx = step_max_blocks(b->n, b->nb);
  std::vector<int> blocks;
  for (int c : {d / 2, d, 2 * d, 4 * d}) {
    const int v = std::max(1, std::min(c, mx));
    if (std::find(blocks.begin(), blocks.end(), v) == blocks.end()) blocks.push_back(v);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return APMG_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return APMG_EHIP; }
  float best_t = -1.f;
  Tune best_tu = {d, 4, 0, kDefaultCellGroup, 0};
  apmg_status out = APMG_OK;
  // one warm-up step, then the mean of three (no parameter update)
  const auto time_tune = [&](const Tune& tu) -> apmg_status {
    apmg_status r = run_step(b, s, ws, tu, false, st);
    if (r != APMG_OK) return r;
    if (hipEventRecord(e0, st) != hipSuccess) return APMG_EHIP;
    for (int k = 0; k < 3 && r == APMG_OK; ++k) r = run_step(b, s, ws, tu, false, st);
    if (r != APMG_OK) return r;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return APMG_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return APMG_EHIP;
    ms /= 3.f;
    if (best_t < 0.f || ms < best_t) { best_t = ms; best_tu = tu; }
    return APMG_OK;
  };
  // 1. tile-kernel blocks per model x waves per adjoint block (eight, or four with two blocks
  // per CU) for the register-resident shapes, with the default gather
  std::vector<int> adjs = {0};
  if (adjoint_applies(s)) adjs = {1, 2};
  for (int tb : blocks) {
    for (int adj : adjs) {
      if ((out = time_tune({tb, 4, 0, kDefaultCellGroup, adj})) != APMG_OK) break;
    }
    if (out != APMG_OK) break;
  }
  // 2. with those: the wave-cooperative gather with 2, 4 or 8 lanes per candidate run, and
  // one thread per cell with 2, 4 or 8 candidates per batch
  struct Gather { int kernel, unroll, group; };
  const Gather gathers[] = {{0, 4, 2}, {0, 4, 8}, {1, 2, kDefaultCellGroup}, {1, 4, kDefaultCellGroup},
                            {1, 8, kDefaultCellGroup}};
  const Tune stage1 = best_tu;
  for (const Gather& ga : gathers) {
    if (out != APMG_OK) break;
    out = time_tune({stage1.tile_blocks, ga.unroll, ga.kernel, ga.group, stage1.adjoint});
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (out != APMG_OK) return out;
  memset(best, 0, sizeof(*best));
  best->tile_blocks = best_tu.tile_blocks;
  best->cell_unroll = best_tu.cell_unroll;
  best->cell_kernel = best_tu.cell_kernel + 1;
  best->cell_group = best_tu.cell_group;
  best->adjoint_kernel = best_tu.adjoint;
  if (best_ms) *best_ms = best_t;
  return APMG_OK;
}

extern "C" apmg_status apmg_train_control(const apmg_control* c, const double* losses, hipStream_t st) {
  if (!c || !losses || c->nb < 1 || !c->state || !c->density_active || !c->frozen || !c->lr_scale) return APMG_EINVAL;
  if (c->delay < 0 || c->ma_window < 1 || c->patience < 0 || c->max_reductions < 1 || c->total_iters < 0)
    return APMG_EINVAL;
  hipLaunchKernelGGL(k_train_control, dim3((c->nb + 63) / 64), dim3(64), 0, st, *c, losses);
  return hip_status(hipGetLastError());
}

// ---------------------------------------------------------------- domain-decomposition inference
struct DdWs {
  uint32_t *k0, *v0, *k1, *v1, *hist, *rowtot, *dbase, *seg;
  float *lpts, *fs, *w3s, *scale;
  void* swz;
  OpsWs ops;
};
int key_bits(int nseg) { int b = 1; while ((1 << b) < nseg) ++b; return b; }
size_t dd_ws(const Shape& s, const apmg_model* shape, int nb, int64_t n, void* ws, DdWs* o) {
  Carver cv(ws);
  const bool bf = shape->mlp_dtype == APMG_BF16;
  const int64_t nn = std::max<int64_t>(n, 1);
  DdWs w;
  take_ops(cv, s, nb, g_rows(shape) == 4, paper_grids(shape), shape->grid_dtype == APMG_F16, &w.ops);
  w.k0 = cv.take<uint32_t>(nn); w.v0 = cv.take<uint32_t>(nn);
  w.k1 = cv.take<uint32_t>(nn); w.v1 = cv.take<uint32_t>(nn);
  w.hist = cv.take<uint32_t>((size_t)kRadixDigits * sort_tiles(n));
  w.rowtot = cv.take<uint32_t>(kRadixDigits);
  w.dbase = cv.take<uint32_t>(kRadixDigits);
  w.seg = cv.take<uint32_t>((size_t)nb + 1);
  w.lpts = cv.take<float>((size_t)3 * nn);
  w.fs = cv.take<float>(nn);
  w.swz = cv.take<char>((size_t)nb * swz_sizes(s).total() * (bf ? 2 : 4));
  w.w3s = cv.take<float>((size_t)nb * s.H);
  w.scale = cv.take<float>((size_t)2 * nb);
  if (o) *o = w;
  return cv.off;
}

extern "C" apmg_status apmg_dd_forward(const apmg_dd_models* d, const apmg_brick_table* t, const float* pts,
                                       int64_t ld, int64_t n, float* f, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!d || !t || d->nb < 1 || !d->G || !d->F || !d->W || !d->bricks) return APMG_EINVAL;
  Shape s;
  apmg_status rc = check_model(&d->shape, false, &s);
  if (rc != APMG_OK) return rc;
  if ((rc = check_points(pts, ld, n)) != APMG_OK) return rc;
  if (n > 0 && !f) return APMG_EINVAL;
  if (t->B < 1 || (int64_t)t->dims[0] * t->dims[1] * t->dims[2] != d->nb) return APMG_EINVAL;
  for (int k = 0; k < 3; ++k) if (t->dims[k] < 1 || t->vol[k] < 2) return APMG_EINVAL;
  if (n > 0xffffffffLL) return APMG_EUNSUPPORTED;
  const bool bf = d->shape.mlp_dtype == APMG_BF16, gf16 = d->shape.grid_dtype == APMG_F16;
  if (!ws || ws_bytes < dd_ws(s, &d->shape, d->nb, n, nullptr, nullptr)) return APMG_EWORKSPACE;
  if (n == 0) return APMG_OK;
  DdWs w;
  dd_ws(s, &d->shape, d->nb, n, ws, &w);
  const int nb = d->nb;
  const size_t nF = f_elems(s), nW = w_elems(s), nG = (size_t)12 * s.M;
  const float* Gc;
  const void* Fc;
  if (launch_ops(s, nb, d->G, g_rows(&d->shape), d->F, gf16, paper_grids(&d->shape), w.ops, gf16, st, &Gc, &Fc) !=
      hipSuccess)
    return APMG_EHIP;
  // brick ids, then a stable radix sort of the points by brick
  hipLaunchKernelGGL(k_dd_keys, dim3(grid1(n)), dim3(256), 0, st, *t, pts, ld, n, w.k0, w.v0);
  const int nt = sort_tiles(n);
  uint32_t *ki = w.k0, *vi = w.v0, *ko = w.k1, *vo = w.v1;
  for (int shift = 0; shift < key_bits(nb); shift += kRadixBits) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nt, 1), dim3(kSortThreads), 0, st, ki, n, shift, w.hist, nt);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(kRadixDigits, 1), dim3(256), 0, st, w.hist, nt, w.rowtot);
    hipLaunchKernelGGL(k_radix_digitscan, dim3(1), dim3(256), 0, st, w.rowtot, w.dbase);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nt, 1), dim3(kSortThreads), 0, st, ki, vi, ko, vo, n, shift, w.hist, w.dbase, nt);
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  hipLaunchKernelGGL(k_seg_starts, dim3(grid1((int64_t)nb + 1)), dim3(256), 0, st, ki, n, nb, w.seg);
  hipLaunchKernelGGL(k_dd_local, dim3(grid1(n)), dim3(256), 0, st, pts, ld, n, ki, vi, d->bricks, *t, w.lpts);
  // every brick's model over its segment, one launch
  hipError_t e = launch_swizzle(s, bf, d->W, d->W + (size_t)s.H * s.MC, d->W + (size_t)s.H * s.MC + (size_t)s.H * s.H,
                                nW, w.swz, swz_sizes(s).total(), w.w3s, nb, st);
  if (e != hipSuccess) return APMG_EHIP;
  hipLaunchKernelGGL(k_brick_scale, dim3((nb + 63) / 64), dim3(64), 0, st, d->bricks, w.scale, nb);
  TileArgs a;
  memset(&a, 0, sizeof(a));
  a.s = s;
  a.G = Gc; a.G_stride = nG;
  a.F = Fc; a.F_stride = nF;
  a.swz = w.swz; a.swz_stride = swz_sizes(s).total(); a.w3s = w.w3s;
  a.bscale = w.scale; a.boff = w.scale + nb;
  a.pts = w.lpts; a.ld = n; a.pts_stride = 0; a.n = n;
  a.seg = w.seg;
  a.f = w.fs;
  // blocks per brick: twice the even share of the tiles, at least one
  const int64_t per = (n + nb - 1) / nb;
  const int nblk = std::max(1, std::min(2 * tile_blocks(per), kMaxTileBlocks));
  e = launch_tile(false, 0, a, gf16, bf, dim3(nblk, nb), forward_lds_bytes(s, bf), st);
  if (e != hipSuccess) return APMG_EHIP;
  hipLaunchKernelGGL(k_dd_scatter, dim3(grid1(n)), dim3(256), 0, st, w.fs, vi, n, f);
  return hip_status(hipGetLastError());
}


// ---------------------------------------------------------------- encoder variants (Sec. 9)
namespace {

// The variant's shape as the tile kernels see it: feature grids M' = M * levels (hash; grid g
// reads transform g / levels) or M (time), C = 2, H = 64, at most 64 features.
apmg_status check_variant(const apmg_model* m, const apmg_encoder* e, bool need_params, Shape* out,
                          EncArgs* ea) {
  if (!m || !e) return APMG_EINVAL;
  if (m->M < 1 || m->C < 1 || m->n_layers != 3) return m->n_layers == 3 ? APMG_EINVAL : APMG_EUNSUPPORTED;
  if (m->width[3] != 1 || m->width[1] < 1 || m->width[2] < 1) return APMG_EINVAL;
  if (need_params) {
    if (!m->G || !m->F) return APMG_EINVAL;
    for (int k = 0; k < 3; ++k) if (!m->W[k]) return APMG_EINVAL;
  }
  if (!(m->G_rows == 0 || m->G_rows == 3 || m->G_rows == 4)) return APMG_EINVAL;
  if (m->grid_layout != APMG_GRIDS_MCRRR && m->grid_layout != APMG_GRIDS_MRRRC) return APMG_EINVAL;
  EncArgs a;
  memset(&a, 0, sizeof(a));
  Shape s;
  memset(&s, 0, sizeof(s));
  if (e->kind == APMG_ENC_HASH) {
    if (e->levels < 1 || e->levels > kMaxLevels || e->table_log2 < 1 || e->table_log2 > 24) return APMG_EINVAL;
    for (int k = 0; k < e->levels; ++k) {
      if (e->level_res[k] < 1 || e->level_res[k] > 65534) return APMG_EINVAL;
      a.res2[k / 2] |= (uint32_t)e->level_res[k] << (16 * (k & 1));
    }
    a.tmask = (1u << e->table_log2) - 1u;
    if (m->width[0] != m->M * e->levels * m->C) return APMG_EINVAL;
    if ((double)m->M * e->levels * ((double)a.tmask + 1.0) * m->C > 2e9) return APMG_EUNSUPPORTED;
    s.M = m->M * e->levels;
    s.L = e->levels;
    s.R = 2;
  } else if (e->kind == APMG_ENC_TIME) {
    if (e->Rt < 2 || m->R < 2) return APMG_EINVAL;
    if (m->width[0] != m->M * m->C) return APMG_EINVAL;
    if ((double)m->M * e->Rt * (double)m->R * m->R * m->R * m->C > 2e9) return APMG_EUNSUPPORTED;
    a.Rt = e->Rt;
    s.M = m->M;
    s.L = 1;
    s.R = m->R;
  } else {
    return APMG_EINVAL;
  }
  if (m->C != 2 || m->grid_dtype != APMG_F32) return APMG_EUNSUPPORTED;
  if (m->mlp_dtype != APMG_F32 && m->mlp_dtype != APMG_BF16) return APMG_EUNSUPPORTED;
  if (m->width[1] != 64 || m->width[2] != 64 || m->width[0] > 64) return APMG_EUNSUPPORTED;
  s.C = m->C;
  s.H = 64;
  s.Mh = (s.M + 1) / 2;
  s.KH = s.Mh * s.C;
  s.KHP = (s.KH + 15) / 16 * 16;
  s.MC = s.M * s.C;
  if (!adjoint_applies(s)) return APMG_EUNSUPPORTED;
  if (out) *out = s;
  if (ea) *ea = a;
  return APMG_OK;
}

// grid values of the model: hash tables M' T C, time grids M Rt R^3 C
size_t variant_f_elems(const Shape& s, const EncArgs& ea, int kind) {
  return kind == APMG_ENC_HASH ? (size_t)s.M * ((size_t)ea.tmask + 1u) * s.C
                               : (size_t)s.M * ea.Rt * s.R * s.R * s.R * s.C;
}
inline int variant_nbx(int64_t n) { return (int)std::max<int64_t>(1, (n + 255) / 256); }
// 4-D grids with at most one radix digit of time cells are sorted by time cell as well
inline bool time_sorted(const EncArgs& ea) { return ea.Rt >= 3 && ea.Rt - 1 <= kRadixDigits; }

struct VarWs {
  float* G;        // packed 3-row transforms (4-row input)
  float* F;        // channel-last copy of paper-order time grids
  void* swz; float* w3s;
  double* part;    // adjoint partials (backward)
  float* dY;       // [M'][n][C] (backward)
  double* dGpart;  // [M'][nbx][12] (backward)
  float* dFcl;     // channel-last time-grid gradient (backward, paper-order grids)
  SortWs srt;      // the points (and dL/df) in spatial-bin order (backward)
  float* tau;      // their times (backward, time grids)
  // time grids: a further stable pass by time cell -> (time cell, spatial bin) order
  uint32_t *tk0, *tv0, *tk1, *tv1;
  float *tpts, *tdf;
  // and the atomic-free per-cell gather of the 4-D grid gradient: (x, y, z, t) records, the
  // starts of every (time cell, bin) and the per-time-cell corner sums
  float4* trec; uint32_t* tstart; float* tcc;
  bool fsorted;    // forward from kFwdSortMin points on: the tiles walk a spatial order (srt keys only)
};
size_t var_ws(const Shape& s, const EncArgs& ea, const apmg_model* m, const apmg_encoder* e, int64_t n,
              bool backward, void* ws, VarWs* o) {
  Carver cv(ws);
  VarWs w;
  memset(&w, 0, sizeof(w));
  const bool bf = m->mlp_dtype == APMG_BF16;
  const bool time_paper = e->kind == APMG_ENC_TIME && paper_grids(m);
  if (g_rows(m) == 4) w.G = cv.take<float>((size_t)12 * (s.M / s.L));
  if (time_paper) w.F = cv.take<float>(variant_f_elems(s, ea, e->kind));
  w.swz = cv.take<char>(swz_sizes(s).total() * (bf ? 2 : 4));
  w.w3s = cv.take<float>(s.H);
  if (!backward && n >= kFwdSortMin) {
    take_sort(cv, n, 1, false, &w.srt, true);
    w.fsorted = true;
  }
  if (backward) {
    w.part = cv.take<double>((size_t)bwd_blocks(n, bf) * part_layout(s, s.MC, s.H).len);
    w.dY = cv.take<float>((size_t)s.M * std::max<int64_t>(n, 1) * s.C);
    w.dGpart = cv.take<double>((size_t)s.M * variant_nbx(n) * 12);
    if (time_paper) w.dFcl = cv.take<float>(variant_f_elems(s, ea, e->kind));
    take_sort(cv, n, 1, true, &w.srt);
    if (e->kind == APMG_ENC_TIME) {
      const size_t nn = (size_t)std::max<int64_t>(n, 1);
      w.tau = cv.take<float>(nn);
      if (time_sorted(ea)) {
        w.tk0 = cv.take<uint32_t>(nn); w.tv0 = cv.take<uint32_t>(nn);
        w.tk1 = cv.take<uint32_t>(nn); w.tv1 = cv.take<uint32_t>(nn);
        w.tpts = cv.take<float>(3 * nn); w.tdf = cv.take<float>(nn);
        w.trec = cv.take<float4>(nn);
        w.tstart = cv.take<uint32_t>((size_t)(ea.Rt - 1) * kBinsPerAxis * kBinsPerAxis * kBinsPerAxis + 1);
        w.tcc = cv.take<float>((size_t)(ea.Rt - 1) * s.M * 16 * n_cells(s) * s.C);
      }
    }
  }
  if (o) *o = w;
  return cv.off;
}

// transforms and grids as the kernels read them
hipError_t variant_ops(const Shape& s, const EncArgs& ea, const apmg_model* m, const apmg_encoder* e,
                       const VarWs& w, hipStream_t st, const float** Gc, const float** Fc) {
  *Gc = m->G;
  *Fc = (const float*)m->F;
  if (w.G) {
    hipLaunchKernelGGL(k_pack_G, dim3(grid1((int64_t)12 * (s.M / s.L))), dim3(256), 0, st, (int64_t)(s.M / s.L), m->G,
                       w.G);
    *Gc = w.G;
  }
  if (w.F) {
    const int64_t V = (int64_t)ea.Rt * s.R * s.R * s.R;
    hipLaunchKernelGGL((k_mirror_grids<2, float, float, true>), dim3(grid1(s.M * V, 8192)), dim3(256), 0, st,
                       (int64_t)s.M, V, (const float*)m->F, w.F);
    *Fc = w.F;
  }
  (void)e;
  return hipGetLastError();
}

}  // namespace

extern "C" {

size_t apmg_variant_workspace_bytes(int op, const apmg_model* m, const apmg_encoder* e, int64_t n) {
  Shape s;
  EncArgs ea;
  if (n < 0 || check_variant(m, e, false, &s, &ea) != APMG_OK) return 0;
  if (op == APMG_OP_FORWARD) return var_ws(s, ea, m, e, n, false, nullptr, nullptr);
  if (op == APMG_OP_BACKWARD) return var_ws(s, ea, m, e, n, true, nullptr, nullptr);
  return 0;
}

apmg_status apmg_variant_forward(const apmg_model* m, const apmg_encoder* e, const float* pts, int64_t ld,
                                 int64_t n, float* f, void* ws, size_t ws_bytes, hipStream_t st) {
  Shape s;
  EncArgs ea;
  apmg_status rc = check_variant(m, e, true, &s, &ea);
  if (rc != APMG_OK) return rc;
  if ((rc = check_points(pts, ld, n)) != APMG_OK) return rc;
  if (n > 0 && !f) return APMG_EINVAL;
  if (!ws || ws_bytes < var_ws(s, ea, m, e, n, false, nullptr, nullptr)) return APMG_EWORKSPACE;
  if (n == 0) return APMG_OK;
  const bool bf = m->mlp_dtype == APMG_BF16;
  VarWs w;
  var_ws(s, ea, m, e, n, false, ws, &w);
  const float *Gc, *Fc;
  if (variant_ops(s, ea, m, e, w, st, &Gc, &Fc) != hipSuccess) return APMG_EHIP;
  if (launch_swizzle(s, bf, m->W[0], m->W[1], m->W[2], 0, w.swz, 0, w.w3s, 1, st) != hipSuccess) return APMG_EHIP;
  TileArgs a;
  memset(&a, 0, sizeof(a));
  a.s = s;
  a.enc = ea;
  a.G = Gc; a.F = Fc; a.swz = w.swz; a.w3s = w.w3s;
  a.vscale = m->vmax - m->vmin; a.voff = m->vmin;
  a.pts = pts; a.ld = ld; a.f = f; a.n = n;
  a.tau = pts + 3 * ld;
  // as apmg_forward: the tiles walk the points' spatial order (each value is unchanged)
  if (w.fsorted) {
    if (launch_sort(pts, ld, 0, nullptr, n, 1, w.srt, nullptr, st, false) != hipSuccess) return APMG_EHIP;
    a.perm = w.srt.v0;
  }
  const int64_t tiles = (n + 31) / 32;
  const dim3 grid((unsigned)std::min<int64_t>((tiles + kWavesPerBlock - 1) / kWavesPerBlock, 8192), 1);
  if (launch_enc_forward(a, e->kind, bf, grid, forward_lds_bytes(s, bf), st) != hipSuccess) return APMG_EHIP;
  return APMG_OK;
}

apmg_status apmg_variant_backward(const apmg_model* m, const apmg_encoder* e, const float* pts, int64_t ld,
                                  int64_t n, const float* df, float* dF, double* dG, float* const* dW,
                                  uint32_t flags, void* ws, size_t ws_bytes, hipStream_t st) {
  Shape s;
  EncArgs ea;
  apmg_status rc = check_variant(m, e, true, &s, &ea);
  if (rc != APMG_OK) return rc;
  if ((rc = check_points(pts, ld, n)) != APMG_OK) return rc;
  if (n > 0 && !df) return APMG_EINVAL;
  if (dW) for (int k = 0; k < 3; ++k) if (!dW[k]) return APMG_EINVAL;
  if (!ws || ws_bytes < var_ws(s, ea, m, e, n, true, nullptr, nullptr)) return APMG_EWORKSPACE;
  const bool bf = m->mlp_dtype == APMG_BF16, acc = flags & APMG_ACCUMULATE;
  const int grows = g_rows(m), mt = s.M / s.L;
  const size_t nF = variant_f_elems(s, ea, e->kind);
  VarWs w;
  var_ws(s, ea, m, e, n, true, ws, &w);
  if (!acc) {
    if (dW) {
      hipLaunchKernelGGL(k_fill_f32, dim3(grid1((int64_t)s.H * s.MC)), dim3(256), 0, st, dW[0], (size_t)s.H * s.MC, 0.f);
      hipLaunchKernelGGL(k_fill_f32, dim3(grid1((int64_t)s.H * s.H)), dim3(256), 0, st, dW[1], (size_t)s.H * s.H, 0.f);
      hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(256), 0, st, dW[2], (size_t)s.H, 0.f);
    }
    if (dF) hipLaunchKernelGGL(k_fill_f32, dim3(grid1(nF)), dim3(256), 0, st, dF, nF, 0.f);
    if (dG) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, st, dG, (size_t)4 * grows * mt, 0.0);
  }
  if (n == 0) return hip_status(hipGetLastError());
  const float *Gc, *Fc;
  if (variant_ops(s, ea, m, e, w, st, &Gc, &Fc) != hipSuccess) return APMG_EHIP;
  if (launch_swizzle(s, bf, m->W[0], m->W[1], m->W[2], 0, w.swz, 0, w.w3s, 1, st) != hipSuccess) return APMG_EHIP;
  // the points, dL/df (and times) in spatial-bin order: neighbouring lanes of the adjoint and
  // of the scatter then share cells, and the scatter adds each run of equal cells once
  if (launch_sort(pts, ld, 0, nullptr, n, 1, w.srt, df, st) != hipSuccess) return APMG_EHIP;
  const float* bpts = w.srt.spts;
  const float* bdf = w.srt.sf;
  if (w.tpts) {
    // then a stable pass by time cell: neighbouring points share the time slices too
    const int nt = sort_tiles(n);
    hipLaunchKernelGGL(k_time_keys, dim3(grid1(n)), dim3(256), 0, st, pts + 3 * ld, w.srt.v0, n, ea.Rt, w.tk0, w.tv0);
    hipLaunchKernelGGL(k_radix_hist, dim3(nt, 1), dim3(kSortThreads), 0, st, w.tk0, n, 0, w.srt.hist, nt);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(kRadixDigits, 1), dim3(256), 0, st, w.srt.hist, nt, w.srt.rowtot);
    hipLaunchKernelGGL(k_radix_digitscan, dim3(1), dim3(256), 0, st, w.srt.rowtot, w.srt.dbase);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nt, 1), dim3(kSortThreads), 0, st, w.tk0, w.tv0, w.tk1, w.tv1, n, 0, w.srt.hist,
                       w.srt.dbase, nt);
    hipLaunchKernelGGL(k_time_permute, dim3(grid1(n)), dim3(256), 0, st, w.srt.spts, w.srt.sf, pts + 3 * ld,
                       w.srt.v0, w.tv1, n, w.tpts, w.tdf, w.tau, w.trec);
    hipLaunchKernelGGL(k_time_bin_starts, dim3(grid1(n + 1)), dim3(256), 0, st, w.tk1, w.srt.k0, w.tv1, n, ea.Rt,
                       w.tstart);
    bpts = w.tpts;
    bdf = w.tdf;
  } else if (w.tau) {
    hipLaunchKernelGGL(k_gather_f32, dim3(grid1(n)), dim3(256), 0, st, pts + 3 * ld, w.srt.v0, n, w.tau);
  }
  const bool want_enc = dF || dG;
  const int nblk = bwd_blocks(n, bf);
  const PartLayout pl = part_layout(s, s.MC, s.H);
  TileArgs a;
  memset(&a, 0, sizeof(a));
  a.s = s;
  a.enc = ea;
  a.G = Gc; a.F = Fc; a.swz = w.swz; a.w3s = w.w3s;
  a.vscale = m->vmax - m->vmin; a.voff = m->vmin;
  a.pts = bpts; a.ld = n; a.n = n;
  a.tau = w.tau;
  a.df = bdf;
  a.dY = want_enc ? w.dY : nullptr;
  a.c1_lo = 0; a.c1_hi = s.MC;
  a.w2_lo = 0; a.w2_hi = s.H;
  a.do_w3 = dW ? 1 : 0;
  a.part = w.part;
  a.part_len = pl.len;
  if (launch_enc_adjoint(a, e->kind, bf, dim3(nblk, 1), st) != hipSuccess) return APMG_EHIP;
  if (dW) {
    hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * s.MC), 1), dim3(256), 0, st, w.part, nblk,
                       pl.len, pl.o_w1, s.H * s.MC, s.MC, s.MC, 0, dW[0], (double*)nullptr, (size_t)0, 1,
                       (const int32_t*)nullptr);
    hipLaunchKernelGGL(k_reduce_parts, dim3(red_blocks((int64_t)s.H * s.H), 1), dim3(256), 0, st, w.part, nblk,
                       pl.len, pl.o_w2, s.H * s.H, s.H * s.H, 0, 0, dW[1], (double*)nullptr, (size_t)0, 1,
                       (const int32_t*)nullptr);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1, 1), dim3(256), 0, st, w.part, nblk, pl.len, pl.o_w3, s.H, s.H, 0, 0,
                       dW[2], (double*)nullptr, (size_t)0, 1, (const int32_t*)nullptr);
  }
  if (!want_enc) return hip_status(hipGetLastError());
  // grid / table gradient by the scatter (into the caller's dF, or a channel-last buffer that
  // is then laid out in the paper's order), transform gradient per block in float64
  float* dst = dF ? (w.dFcl ? w.dFcl : dF) : nullptr;
  if (dst && w.dFcl) hipLaunchKernelGGL(k_fill_f32, dim3(grid1(nF)), dim3(256), 0, st, w.dFcl, nF, 0.f);
  // 4-D grids in (time cell, bin) order: the grid gradient by the per-cell gather (one pass per
  // time cell, no atomics, a fixed order), then the vertex sums over both time neighbours
  const bool pull = dst && w.tcc;
  if (pull) {
    CellArgs c;
    memset(&c, 0, sizeof(c));
    c.s = s; c.G = Gc; c.F = Fc;
    c.pts4 = w.trec; c.n = n; c.start = w.tstart; c.dY = w.dY; c.CC = w.tcc; c.Rt = ea.Rt;
    const int64_t wgroups = (int64_t)wave_groups(s) * s.M * (ea.Rt - 1);
    if (wgroups > 0x7fffffff) return APMG_EUNSUPPORTED;
    hipLaunchKernelGGL((k_cell_pull_wave<2, false, kDefaultCellGroup, false, 2>), dim3((unsigned)wgroups), dim3(256),
                       0, st, c);
    hipLaunchKernelGGL(k_cell_to_vertex_time<2>, dim3(grid1((int64_t)s.R * s.R * s.R, 1024), s.M, ea.Rt), dim3(256),
                       0, st, s, ea.Rt, w.tcc, dst);
  }
  if (!dG && pull) {
    if (w.dFcl && dF) {
      const int64_t V = (int64_t)ea.Rt * s.R * s.R * s.R;
      hipLaunchKernelGGL(k_cl_to_paper<2>, dim3(grid1(s.M * V, 8192)), dim3(256), 0, st, (int64_t)s.M, V, w.dFcl, dF,
                         acc ? 1 : 0);
    }
    return hip_status(hipGetLastError());
  }
  EncScatterArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.s = s; sa.enc = ea; sa.G = Gc; sa.F = Fc;
  sa.pts = bpts; sa.ld = n; sa.n = n;
  sa.tau = w.tau;
  sa.dY = w.dY;
  sa.dF = pull ? nullptr : dst;   // with the gather done, the scatter forms the transform gradient only
  sa.dGpart = dG ? w.dGpart : nullptr;
  sa.nbx = variant_nbx(n);
  if (launch_enc_scatter(sa, e->kind, st) != hipSuccess) return APMG_EHIP;
  if (w.dFcl && dF) {
    const int64_t V = (int64_t)ea.Rt * s.R * s.R * s.R;
    hipLaunchKernelGGL(k_cl_to_paper<2>, dim3(grid1(s.M * V, 8192)), dim3(256), 0, st, (int64_t)s.M, V, w.dFcl, dF,
                       acc ? 1 : 0);
  }
  if (dG)
    hipLaunchKernelGGL(k_reduce_cell_dG, dim3(mt, 1), dim3(256), 0, st, w.dGpart, mt, s.L * sa.nbx, dG,
                       (size_t)0, grows, acc ? 1 : 0, (const int32_t*)nullptr);
  return hip_status(hipGetLastError());
}

}  // extern "C"
