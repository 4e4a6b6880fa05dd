/*
 * apmg.h -- C ABI of the MI355X (gfx950) library for the hot path of the
 * adaptively placed multi-grid scene representation network (APMGSRN) of
 * Wurster et al., "Adaptively Placed Multi-Grid Scene Representation
 * Networks for Large-Scale Data Visualization".
 *
 * Model (Sec. 4.1): f(x) = d(e(x)) for x in [-1,1]^3.
 *   Encoder (Sec. 4.1.1): M feature grids of C channels at R^3 vertices.
 *     Eq. (1): grid i maps a global point to its local frame,
 *              l = G_i[0:3,0:3] x + G_i[0:3,3].
 *     Eq. (2): e_i = trilinear interpolation of grid i at l, with vertices
 *              corner-aligned at -1 and +1, when -1 <= l_d <= 1 on every
 *              axis (inclusive; a NaN coordinate is outside); otherwise the
 *              C features are exactly 0.
 *     Eq. (3): y = e_0 (+) e_1 (+) ... (+) e_{M-1}, feature index i*C + c.
 *   Decoder (Sec. 4.1.2): a bias-free MLP, ReLU after every layer but the
 *     last, then d(y) = m(y) (vmax - vmin) + vmin.
 * Feature density (Sec. 4.2): Eq. (7) flat-top density, Eq. (8) target
 * density, Eq. (9) KL loss.  Training (Sec. 4.3.2, Sec. 7): L_rec updates F
 * and the MLP, L_density updates the transforms, Adam.
 * Domain decomposition (Sec. 5.1, 5.3): bricks with ghost cells and a
 * spatial hash from global points to bricks.
 *
 * Conventions shared by every call
 * --------------------------------
 * - All array pointers are DEVICE pointers unless stated otherwise, owned
 *   by the caller.  The library allocates nothing per call: scratch memory
 *   is the caller's workspace (size from apmg_workspace_bytes()).
 * - Every call is asynchronous on `stream` (0 = the null stream) and may be
 *   captured in a HIP graph; no call reads device data back to the host or
 *   synchronises, and no call records a memset (buffers are cleared with
 *   kernels).
 * - Points are structure-of-arrays: x at pts[0..n), y at pts[ld..ld+n),
 *   z at pts[2*ld..2*ld+n), with ld >= n.
 * - Grids are the paper's encoder tensor [M, C, D, H, W] (Sec. 4.1.1) with
 *   D = H = W = R, axes (z, y, x), x fastest: F[i, c, z, y, x] is at
 *   (((i*C + c)*R + z)*R + y)*R + x (model.grid_layout = APMG_GRIDS_MCRRR,
 *   the default).  Grid gradients are returned in the same order.  The
 *   kernels gather from a channel-last mirror [M][R][R][R][C] (an x-adjacent
 *   vertex pair is 2C contiguous values); with the default layout every call
 *   builds that mirror in its workspace.  A caller that keeps its grids
 *   channel-last already may say so with APMG_GRIDS_MRRRC (then F, and dF,
 *   are [M][R][R][R][C]) and skip the copy; apmg_convert_grids() converts
 *   between the two orders.
 * - Transforms are the matrices of Eq. (1), float32 row-major: [M][3][4]
 *   (rows 0..2, model.G_rows = 3, the default) or the full [M][4][4]
 *   (model.G_rows = 4; row 3 is (0,0,0,1) by Eq. (1) and is never read).
 *   Transform gradients are returned in the same shape (row 3 written as 0).
 * - MLP weights W_k are [width[k+1]][width[k]] row-major float32 (the
 *   master copy); mlp_dtype selects the arithmetic of the matrix products.
 * - Status: APMG_EINVAL for a NULL required pointer, n < 0, ld < n, or an
 *   inconsistent shape; APMG_EUNSUPPORTED for a shape or dtype outside the
 *   built kernels (there is no slow fallback); APMG_EWORKSPACE when ws_bytes
 *   is below apmg_workspace_bytes(); APMG_EHIP when a launch fails (faults
 *   inside kernels surface at the caller's next synchronisation).
 *   Nothing is launched when a call returns an error.
 * - Values are not validated (that would need a device read): non-finite
 *   points fall outside every grid and give f = vmin.
 * - n = 0 is valid: outputs are written as for an empty batch (zeros).
 * - Calls are reentrant given distinct workspaces and outputs.
 */
#ifndef APMG_H
#define APMG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  APMG_OK = 0,
  APMG_EINVAL = -1,
  APMG_EUNSUPPORTED = -2,
  APMG_EWORKSPACE = -3,
  APMG_EHIP = -4
} apmg_status;

typedef enum { APMG_F32 = 0, APMG_F16 = 1, APMG_BF16 = 2 } apmg_dtype;

/* flags */
#define APMG_ACCUMULATE     0x1u  /* add into the outputs instead of overwriting them */
#define APMG_DETERMINISTIC  0x2u  /* reserved: accepted and ignored, since every reduction of
                                     the library already runs in a fixed order (bitwise
                                     reproducible results for a given launch shape) */
#define APMG_ADD_REC_DG     0x4u  /* training step: add L_rec's transform gradient to L_density's */
#define APMG_ERR_ABS        0x8u  /* training step: h(x) = |f - v| instead of (f - v)^2 */
/* Readings of the feature density other than the literal one (apmg_density_loss and the
 * training step).  Eq. (7) as printed weights grid i by its signed det(A_i); Sec. 4.2
 * describes that factor as the grid's density, which grows as the grid shrinks and does
 * not depend on its handedness:
 *   APMG_DENSITY_ABS_DET: rho_i = |det(A_i)| exp(-sum_d l_d^{2p}).
 * Eq. (9) compares an unnormalised target with the normalised rho_scaled:
 *   APMG_DENSITY_NORM_TARGET: the target is rho* / sum_X rho*, so that both arguments
 *   of the divergence sum to one over the batch. */
#define APMG_DENSITY_ABS_DET     0x10u
#define APMG_DENSITY_NORM_TARGET 0x20u

/* grid layouts (apmg_model.grid_layout) */
#define APMG_GRIDS_MCRRR 0   /* [M][C][R][R][R], the paper's order (default) */
#define APMG_GRIDS_MRRRC 1   /* [M][R][R][R][C], channel-last */

#define APMG_MAX_LAYERS 8

/* One APMGSRN.  Supported by the built kernels: C in {1, 2, 4}; M*C <= 256;
 * n_layers == 3 with width = {M*C, H, H, 1} and H in {64, 128};
 * grid_dtype F32 or F16; mlp_dtype F32 or BF16.  A zero-initialised struct
 * has the default layouts (paper-order grids, [M][3][4] transforms). */
typedef struct apmg_model {
  int32_t M;                        /* number of feature grids (>= 1) */
  int32_t C;                        /* feature channels per grid (>= 1) */
  int32_t R;                        /* vertices per axis (>= 2) */
  int32_t n_layers;                 /* number of weight matrices */
  int32_t width[APMG_MAX_LAYERS + 1]; /* width[0] = M*C, width[n_layers] = 1 */
  int32_t grid_dtype;               /* apmg_dtype of F */
  int32_t mlp_dtype;                /* apmg_dtype of the MLP products (F32 or BF16, fp32 accumulate) */
  const float* G;                   /* [M][G_rows][4] transforms, global -> local (Eq. (1)) */
  const void* F;                    /* grids in grid_layout order, grid_dtype */
  const float* W[APMG_MAX_LAYERS];  /* W_k: [width[k+1]][width[k]], no biases */
  float vmin, vmax;                 /* output scaling, Sec. 4.1.2 "Scaling" */
  int32_t grid_layout;              /* APMG_GRIDS_MCRRR (0, default) or APMG_GRIDS_MRRRC */
  int32_t G_rows;                   /* rows stored per transform: 3 (0 = 3, default) or 4 */
} apmg_model;

/* ---------------------------------------------------------------- forward
 * f[n] = d(e(x_n)) for n points (Sec. 4.1, Eqs. (1)-(3) and the decoder).
 * f: [n] float32 output.  From 2^15 points on, the points are first sorted
 * into spatial bins (the workspace then grows with n) and the tiles walk that
 * order, reading each point and writing its output in the caller's order; each
 * value is the same either way. */
apmg_status apmg_forward(const apmg_model* model, const float* pts, int64_t ld, int64_t n,
                         float* f, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- forward without a workspace
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): apmg_forward with no workspace
 * argument.  Its scratch (swizzled MLP operands, and for paper-order grids or 4x4
 * transforms their gather copies) lives in one static device array per GPU of
 * apmg_forward_noalloc_scratch_bytes() = 16 MiB, held until the process ends; the call
 * allocates nothing.  It takes the direct tile path for every n (no spatial sort), so
 * each output is bitwise the value apmg_forward gives.  APMG_EWORKSPACE when the model's
 * scratch exceeds the array (for example paper-order grids of more than about 15 MiB:
 * pass them channel-last, APMG_GRIDS_MRRRC, which needs no copy); APMG_EHIP when the
 * array's device address cannot be had.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (two streams, two host threads) race and must be
 * serialised by the caller.  Other arguments and errors as apmg_forward. */
apmg_status apmg_forward_noalloc(const apmg_model* model, const float* pts, int64_t ld, int64_t n,
                                 float* f, hipStream_t stream);
size_t apmg_forward_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------- adjoint
 * Gradients of L = sum_n df[n] * f(x_n), computed by recomputing the
 * forward pass for each tile of points and back-propagating by hand
 * (ReLU'(0) = 0; the mask of Eq. (2) contributes no gradient; at a vertex
 * the one-sided derivative of the selected cell).
 *   df: [n] float32, dL/df.
 *   dF: float32 grids in model.grid_layout order (also when grids are F16),
 *       or NULL.
 *   dG: [M][G_rows][4] float64 or NULL (gradient through the trilinear
 *       weights).
 *   dW: host array of n_layers device pointers, each [width[k+1]][width[k]]
 *       float32, or NULL for no MLP gradient.
 * Outputs are overwritten unless APMG_ACCUMULATE.  The points are first
 * sorted (stably) into spatial bins; dF is then gathered per grid cell from
 * the points of the bins the cell overlaps, with no atomics, and every
 * reduction (dF, dG in float64, dW in float64 over per-block partials) runs
 * in a fixed order: results are bitwise reproducible, and
 * APMG_DETERMINISTIC is accepted but changes nothing.  MLP shapes outside
 * the register-resident adjoint (H != 64, or more than 64 input features)
 * store the per-point activations in the workspace and form dW1 and dW2 as
 * matrix products over the points. */
apmg_status apmg_backward(const apmg_model* model, const float* pts, int64_t ld, int64_t n,
                          const float* df, float* dF, double* dG, float* const* dW,
                          uint32_t flags, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- encoder variants
 * The two extensions of the encoder named in Sec. 9 ("Conclusion and future work"); the
 * transforms (Eq. (1)), the mask of Eq. (2), the concatenation of Eq. (3) and the decoder
 * are those of the dense model.
 *  APMG_ENC_HASH -- a hash grid inside each adaptive grid (the multiresolution hash
 *   encoding of Mueller et al., "Instant neural graphics primitives", 2022): grid i has
 *   `levels` levels; level k has level_res[k] = N_k cells per axis across the local cube,
 *   vertex coordinate u = fma(l, N_k/2, N_k/2), lower vertex clamp(floor(u), 0, N_k - 1)
 *   (float32, as the dense grids with R - 1 = N_k), and a table of T = 2^table_log2
 *   entries of C features.  Vertex v of level k reads entry v_x + (N_k+1)(v_y + (N_k+1) v_z)
 *   when (N_k+1)^3 <= T, else (v_x XOR 2654435761 v_y XOR 805459861 v_z) mod 2^32 mod T.
 *   The level's C features are the trilinear interpolation of its 8 corner entries; grid i
 *   emits levels*C features, index (i*levels + k)*C + c, so width[0] = M*levels*C.
 *   F: tables [M][levels][T][C] float32 (grid_layout ignored); R is not used.
 *  APMG_ENC_TIME -- 4-D grids: F is [M][C][Rt][R][R][R] (APMG_GRIDS_MCRRR) or
 *   [M][Rt][R][R][R][C] (APMG_GRIDS_MRRRC), float32; the points carry a fourth row, the
 *   normalised time tau in [-1, 1] at pts[3*ld + n].  Time vertex k sits at
 *   -1 + 2k/(Rt-1); u_t = fma(tau, (Rt-1)/2, (Rt-1)/2), lower vertex clamp(floor(u_t), 0,
 *   Rt-2).  The features are the linear interpolation in time of the trilinear
 *   interpolations (Eq. (2)) of the two time slices; a point with tau outside [-1, 1]
 *   (or NaN) gets zero features from every grid.  width[0] = M*C.
 * Built for C = 2, grid_dtype F32, MLP {width[0], 64, 64, 1} with width[0] <= 64, mlp_dtype
 * F32 or BF16 (APMG_EUNSUPPORTED otherwise).  From 2^15 points on the forward sorts the
 * points into spatial bins first and its tiles walk that order, as apmg_forward does (each
 * value is the same either way).  The backward first sorts the points into spatial bins (as
 * apmg_backward does).  Hash grids: the table gradient is added with float atomics (every
 * entry a vertex maps to, colliding vertices included; a run of sorted points in one cell
 * is summed in registers and added once), so dF is reproducible to rounding only.  4-D grids
 * with Rt >= 3: a further stable sort by time cell, then the grid gradient is gathered per
 * (time cell, grid cell) as apmg_backward gathers dF, in a fixed order (bitwise
 * reproducible); with Rt = 2 it is added with atomics as for the hash grids.  dW and dG
 * (float64 per block, fixed order) are as in apmg_backward.
 * Workspace: apmg_variant_workspace_bytes(APMG_OP_FORWARD or APMG_OP_BACKWARD, ...).
 * Arguments, outputs, flags and errors otherwise as apmg_forward / apmg_backward; dF has
 * F's layout. */
#define APMG_ENC_HASH 1
#define APMG_ENC_TIME 2
typedef struct apmg_encoder {
  int32_t kind;             /* APMG_ENC_HASH or APMG_ENC_TIME */
  int32_t levels;           /* hash: levels per grid, 1..8 */
  int32_t table_log2;       /* hash: T = 2^table_log2 entries per (grid, level), 1..24 */
  int32_t level_res[8];     /* hash: cells per axis of level k, 1..65534 */
  int32_t Rt;               /* time: vertices along the time axis, >= 2 */
} apmg_encoder;

size_t apmg_variant_workspace_bytes(int op, const apmg_model* model, const apmg_encoder* enc, int64_t n);
apmg_status apmg_variant_forward(const apmg_model* model, const apmg_encoder* enc, const float* pts, int64_t ld,
                                 int64_t n, float* f, void* ws, size_t ws_bytes, hipStream_t stream);
apmg_status apmg_variant_backward(const apmg_model* model, const apmg_encoder* enc, const float* pts, int64_t ld,
                                  int64_t n, const float* df, float* dF, double* dG, float* const* dW,
                                  uint32_t flags, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- density
 * Sec. 4.2.  rho(x) = sum_i det(G_i[0:3,0:3]) exp(-sum_d l_d^{2p})  (Eq. (7),
 * signed determinant, exp(-s) taken as 0 for s > 87 or NaN);
 * rho_s = rho / sum_X rho; h_bar = mean(err);
 * rho* = exp(h_bar/(err+eps) log(rho_s + eps))                  (Eq. (8));
 * loss = (1/n) sum rho* (log rho* - log(rho_s + eps)), 0 log 0 = 0 (Eq. (9)).
 * dG = d loss / dG with rho* held constant.  If sum_X rho == 0 the loss and
 * gradient are 0.
 *   err: [n] float32, the per-point error h(x).
 *   loss: [1] float64 output.  dG: [M][G_rows][4] float64 or NULL.
 *   rho: [n] float32 output of Eq. (7), or NULL.
 * flags: APMG_ACCUMULATE adds into dG (loss is always overwritten);
 * APMG_DENSITY_ABS_DET and APMG_DENSITY_NORM_TARGET select the alternative
 * readings defined with the flags (the gradient of |det| is sign(det) times
 * the cofactor matrix; the renormalised target is held constant too).
 * Per-point arithmetic is float32; all sums over points are float64. */
apmg_status apmg_density_loss(const apmg_model* model, const float* pts, int64_t ld, int64_t n,
                              const float* err, double eps, int32_t p,
                              double* loss, double* dG, float* rho, uint32_t flags,
                              void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- bricks
 * Sec. 5.1: a volume of nx*ny*nz voxels split into bricks of edge B voxels,
 * I = ceil(nx/B) (etc.) bricks per axis, listed in x, y, z order
 * (id = i + I j + I J k, Sec. 5.3).  Brick i's base extent is voxels
 * [iB, min((i+1)B, n)); its extended extent adds `ghost` voxels on each side,
 * clipped to the volume: [max(iB-g, 0), min((i+1)B-1+g, n-1)] inclusive.
 * A brick model's local coordinate l in [-1,1] maps corner-aligned onto the
 * extended extent. */
typedef struct apmg_brick {
  int32_t ijk[3];
  int32_t e0[3];            /* first voxel of the extended extent (x, y, z) */
  int32_t e1[3];            /* last voxel of the extended extent (inclusive) */
  float vmin, vmax;         /* the brick model's output scaling */
} apmg_brick;

typedef struct apmg_brick_table {
  int32_t dims[3];          /* I, J, K */
  int32_t vol[3];           /* nx, ny, nz */
  int32_t B, ghost;
} apmg_brick_table;

/* Host-only: fills *table and, if bricks != NULL, up to cap bricks (host
 * memory; vmin/vmax set to 0/1).  Returns EINVAL for non-positive sizes,
 * ghost < 0, or cap < I*J*K when bricks != NULL. */
apmg_status apmg_make_bricks(int32_t nx, int32_t ny, int32_t nz, int32_t B, int32_t ghost,
                             apmg_brick_table* table, apmg_brick* bricks, int32_t cap);

/* Sec. 5.3 spatial hash for uneven bricks: the voxel coordinate
 * u_d = fma(p_d, (n_d-1)/2, (n_d-1)/2) (float32) picks the base brick holding
 * floor(u_d): i = clamp(floor(u) div B, 0, I-1).  brick: [n] int32 output. */
apmg_status apmg_assign_bricks(const apmg_brick_table* table, const float* pts, int64_t ld,
                               int64_t n, int32_t* brick, hipStream_t stream);

/* ---------------------------------------------------------------- domain-decomposition inference
 * Global-query inference across all brick models (Sec. 5.3): every global
 * point p in [-1,1]^3 of the whole volume goes to its brick b by the hash of
 * apmg_assign_bricks (table), is mapped into brick b's local frame, the
 * inverse of the training map u = e0 + (l + 1)/2 (e1 - e0) over b's extended
 * extent:
 *   u_d = fma(p_d, (n_d-1)/2, (n_d-1)/2),
 *   l_d = fma(u_d - e0_d, 2/(e1_d - e0_d), -1)   (float32, each operation
 *                                                 rounded once),
 * and evaluated by model b (f = m (vmax_b - vmin_b) + vmin_b with brick b's
 * vmin/vmax).  f[i] is written in the input order.  One call evaluates every
 * brick in one launch of the forward kernel.
 * EINVAL also when nb != I*J*K of the table. */
typedef struct apmg_dd_models {
  int32_t nb;                 /* models, one per brick, in brick-id order */
  apmg_model shape;           /* M, C, R, n_layers, width, dtypes, layouts; pointers ignored */
  const float* G;             /* [nb][M][G_rows][4] */
  const void* F;              /* [nb] grids in shape.grid_layout order, shape.grid_dtype */
  const float* W;             /* [nb][layers concatenated] float32 */
  const apmg_brick* bricks;   /* [nb] device: extended extents, vmin, vmax */
} apmg_dd_models;

apmg_status apmg_dd_forward(const apmg_dd_models* models, const apmg_brick_table* table, const float* pts,
                            int64_t ld, int64_t n, float* f, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- training step
 * One training iteration (Sec. 4.3.2, Sec. 7) for nb independent models of
 * one shape, each trained on its own brick of one volume (nb = 1 with one
 * brick spanning the volume is the single-model step).  For every model b:
 *   1. n uniform points in [-1,1)^3 from Philox4x64-10 (counter
 *      (j, step, stream0 + b, 0), key (seed, 0x41504D47); coordinate =
 *      (w >> 40) 2^-23 - 1);
 *   2. v = trilinear sample of brick b's extended sub-volume;
 *   3. forward, L_rec = mean (f - v)^2, h = (f - v)^2 (or |f - v|);
 *   4. adjoint of L_rec into F and W;
 *   5. if density_active[b]: L_density and its transform gradient (+ L_rec's
 *      transform gradient under APMG_ADD_REC_DG);
 *   6. Adam (bias-corrected, float32 master weights): F and W with lr, every
 *      step; G with lr_G, only when density_active[b].
 *   7. *step += 1 (device counter; a captured graph replays fresh batches).
 * Grids F (and the moments mF, vF) are float32 master copies in
 * shape.grid_layout order.  With grid_dtype F16 the encoder gathers from an
 * F16 copy of the masters (round to nearest) that the step builds in its
 * workspace at its start, while gradients and Adam stay float32; the same
 * copy holds the channel-last mirror of paper-order grids.  Transforms are
 * [nb][M][3][4] (shape.G_rows must be 3 or 0).
 * flags: APMG_ADD_REC_DG, APMG_ERR_ABS, APMG_DENSITY_ABS_DET,
 * APMG_DENSITY_NORM_TARGET.
 * All per-model arrays are contiguous arenas indexed by model: model b's
 * block starts at b * (block size).  Adam moments and counters are device
 * memory the caller zero-initialises.
 * The density passes (5) and the last weight-gradient reductions run on a
 * side stream the library keeps per device (default priority), forked from
 * and joined back into `stream` within the call, so the call stays ordered
 * on `stream` and can be captured in a graph; concurrent calls take turns
 * for the fork and join.  A step captured before any eager step on that
 * device runs entirely on `stream`. */
/* Launch shapes of the training step (fields of 0 take the defaults).
 *   tile_blocks: blocks of the fused forward+adjoint tile kernel per model
 *     (each block = 8 or 4 waves of 32-point tiles); default CUs / nb when nb divides
 *     the device's compute units (one round of blocks), else ceil(2 CUs / nb); at
 *     most 4 times the default and at most the number of 4-tile groups.
 *   cell_kernel: grid-gradient gather, 1 = one wave per 4x4x4 block of cells
 *     (the default; the wave reads each candidate point once), 2 = one thread
 *     per cell.  Either also produces L_rec's transform gradient when it is
 *     requested.
 *   cell_unroll: candidates per batch of the one-thread-per-cell gather, 2, 4
 *     or 8 (default 4).
 *   cell_group: lanes per candidate run of the wave gather, 1, 2, 4 or 8
 *     (default 4): the wave splits its candidates into 64 / cell_group runs
 *     and each group of lanes reads cell_group consecutive points per step.
 *   adjoint_kernel: the fused forward + adjoint tile kernel for shapes with hidden
 *     width 64 and at most 64 input features.  The tiled kernels (each wave keeps
 *     one 32x32 block of dW1 and of dW2 and accumulates it over the tiles of its
 *     whole block, two waves per SIMD): 1 = eight waves per block, one block per
 *     CU; 2 = four waves per block, two blocks per CU (bf16: its LDS allows it);
 *     0 (default) = 1 for a float32 MLP, 2 for bf16.  3 = four waves per block,
 *     one per SIMD, each wave accumulating all of dW1 and dW2 over its own tiles.
 * The two gathers add each cell's terms in different fixed orders (the
 * per-cell thread in point order, the wave in its own step-then-lane order),
 * so the grid gradients agree to float32 rounding; cell_unroll does not
 * change the order, cell_group does.  Results also depend on tile_blocks and
 * adjoint_kernel through the order of the weight-gradient sums.  Each setting is
 * bitwise reproducible run to run. */
typedef struct apmg_tuning {
  int32_t tile_blocks;
  int32_t cell_unroll;
  int32_t cell_kernel;
  int32_t cell_group;
  int32_t adjoint_kernel;
  int32_t reserved[3];
} apmg_tuning;

typedef struct apmg_batch {
  int32_t nb;                 /* number of models */
  apmg_model shape;           /* M, C, R, n_layers, width, dtypes; pointers ignored */
  float* G;                   /* [nb][M][3][4] */
  float* F;                   /* [nb] float32 master grids in shape.grid_layout order */
  float* W;                   /* [nb][sum_k width[k+1]*width[k]], layers concatenated */
  float* mG; float* vG;       /* Adam moments, shapes of G */
  float* mF; float* vF;       /* shapes of F */
  float* mW; float* vW;       /* shapes of W */
  int32_t* t;                 /* [nb] Adam step of F and W */
  int32_t* tG;                /* [nb] Adam step of G (counts density steps only) */
  const int32_t* density_active; /* [nb] 0/1 */
  const float* volume;        /* [nz][ny][nx] float32 */
  const apmg_brick* bricks;   /* [nb] device brick descriptors (extents, vmin, vmax) */
  int32_t vol[3];             /* nx, ny, nz */
  int64_t n;                  /* points per model per step; n = 0 is an empty batch: both losses
                                 0, every gradient zero, so Adam still steps from its moments */
  uint64_t seed;
  uint64_t* step;             /* device step counter */
  float lr, lr_G, beta1, beta2, adam_eps;  /* lr, lr_G, adam_eps >= 0; beta1, beta2 in [0, 1), else
                                             APMG_EINVAL */
  double eps_density;
  int32_t p;                  /* flat-top strength (10) */
  uint32_t flags;
  double* losses;             /* [nb][2] output: L_rec, L_density */
  const apmg_tuning* tuning;  /* HOST pointer, read when the call is made; NULL = defaults */
  const int32_t* frozen;      /* [nb] or NULL: 1 = model retired, nothing of it changes */
  const float* lr_scale;      /* [nb] or NULL: multiplies lr and lr_G of each model */
  uint32_t stream0;           /* model b draws its points from counter stream stream0 + b: a
                                 subset of bricks stepped on its own (say one of several
                                 devices) draws the same points as in the whole batch */
} apmg_batch;

apmg_status apmg_batched_step(const apmg_batch* batch, void* ws, size_t ws_bytes,
                              hipStream_t stream);

/* Autotuner: times the training step's phases (points, sort, ground truth,
 * tile kernel, grid-gradient gather, density passes; no Adam update, no
 * counter change -- parameters, moments and the step counter are left as they
 * are, the losses array is written) for candidate launch shapes around the
 * defaults -- first tile-kernel blocks per model (1/2x to 4x the default) times the
 * adjoint's waves per block (eight, or four with two blocks per CU) with the default
 * gather, then the gathers (wave-cooperative with 2/4/8 lanes per run, one thread per
 * cell with 2/4/8 candidates per batch) at the best of those -- and returns the
 * fastest in *best (HOST) with its time in *best_ms.
 * Needs the workspace of APMG_OP_BATCHED_STEP for this batch.  Synchronises
 * `stream` (hipEvent timing), so it must not be called during graph capture.
 * The caller keeps the result and passes it as batch->tuning. */
apmg_status apmg_autotune_batched_step(const apmg_batch* batch, void* ws, size_t ws_bytes,
                                       hipStream_t stream, apmg_tuning* best, float* best_ms);

/* ---------------------------------------------------------------- training control
 * On-device schedule of a training run (Sec. 4.3.2 "Delayed start" and
 * "Early stopping"; Sec. 5.2 early stopping of brick models), applied after
 * each training step to that step's losses, per model:
 *   - delayed start: transforms are not trained during the first `delay`
 *     iterations (500 in the paper);
 *   - transform early stop: the mean of L_density over each block of
 *     `ma_window` density iterations (1000) is compared with the previous
 *     block's mean; when it is not lower by the relative amount `ma_rel`
 *     (1e-4, "0.01%"), transform training stops for good; it also stops once
 *     the next iteration would exceed stop_frac * total_iters (80%);
 *   - plateau scheduler on L_rec: an iteration whose L_rec is below
 *     best * (1 - plateau_rel) (1e-4) becomes the best and resets the count of
 *     bad iterations; after more than `patience` (500) bad iterations in a
 *     row the model's learning rates are multiplied by plateau_factor (0.1)
 *     and the count restarts; the max_reductions-th (3rd) reduction retires
 *     the model (frozen = 1).
 * State per model is apmg_ctl_state (device, zero-initialised by the caller);
 * density_active, frozen and lr_scale are the batch's arrays for the next
 * step (initialise them to (delay == 0), 0 and 1).  A frozen model's state no
 * longer changes.  Asynchronous and graph-capturable like the step. */
typedef struct apmg_ctl_state {
  int32_t iter;               /* iterations completed */
  int32_t density_done;       /* transform training stopped */
  int32_t ma_count;           /* density iterations in the current block */
  int32_t have_prev;          /* a previous block mean exists */
  int32_t bad;                /* plateau: bad iterations in a row */
  int32_t reductions;         /* plateau: learning-rate reductions so far */
  double ma_sum;              /* sum of L_density over the current block */
  double ma_prev;             /* mean of the previous block */
  double best;                /* plateau: best L_rec */
} apmg_ctl_state;

typedef struct apmg_control {
  int32_t nb;
  int32_t delay;              /* 500 */
  int32_t total_iters;        /* length of the run */
  int32_t ma_window;          /* 1000 */
  int32_t patience;           /* 500 */
  int32_t max_reductions;     /* 3 */
  float stop_frac;            /* 0.8 */
  float plateau_factor;       /* 0.1 */
  double ma_rel;              /* 1e-4 */
  double plateau_rel;         /* 1e-4 */
  apmg_ctl_state* state;      /* [nb] */
  int32_t* density_active;    /* [nb] written */
  int32_t* frozen;            /* [nb] written */
  float* lr_scale;            /* [nb] written */
} apmg_control;

/* losses: [nb][2] (L_rec, L_density) of the step just taken (the batch's
 * losses array).  EINVAL for a NULL pointer, nb < 1, delay < 0, ma_window < 1,
 * patience < 0, max_reductions < 1. */
apmg_status apmg_train_control(const apmg_control* control, const double* losses, hipStream_t stream);

/* ---------------------------------------------------------------- workspace
 * Bytes of workspace for `op` (one of the values below) on a model (or, for
 * APMG_OP_BATCHED_STEP, a batch) with n points.  0 for an invalid request. */
#define APMG_OP_FORWARD 0
#define APMG_OP_BACKWARD 1
#define APMG_OP_DENSITY 2
#define APMG_OP_BATCHED_STEP 3
#define APMG_OP_DD_FORWARD 4     /* model_or_batch: an apmg_dd_models */
size_t apmg_workspace_bytes(int op, const void* model_or_batch, int64_t n);

const char* apmg_status_string(apmg_status status);

/* ---------------------------------------------------------------- layout
 * Converts grids between the paper's [M][C][R][R][R] order (to_channel_last
 * = 1: src is paper order) and the library's [M][R][R][R][C] order, in the
 * same float32 or F16 dtype, optionally converting float32 -> F16 when
 * dst_dtype is F16 and src_dtype F32.  src and dst must not overlap. */
apmg_status apmg_convert_grids(int32_t M, int32_t C, int32_t R, const void* src, int32_t src_dtype,
                               void* dst, int32_t dst_dtype, int32_t to_channel_last,
                               hipStream_t stream);

/* ---------------------------------------------------------------- test exports
 * The integer decisions of Eq. (2), in the library's float32 arithmetic:
 * l_r = fma(G[r,2], x_z, fma(G[r,1], x_y, fma(G[r,0], x_x, G[r,3]))),
 * inside = all(-1 <= l_d <= 1), u = fma(l, (R-1)/2, (R-1)/2),
 * cell = clamp(floor(u), 0, R-2).
 *   cell: [n][M][3] int32 (x, y, z), -1 on every axis where outside.
 *   inside: [n][M] uint8. */
apmg_status apmg_cells(const apmg_model* model, const float* pts, int64_t ld, int64_t n,
                       int32_t* cell, uint8_t* inside, hipStream_t stream);

/* The training step's point generator (step 1 above) for model `stream_id`:
 * points start .. start+n-1 written SoA to pts [3][ld]. */
apmg_status apmg_uniform_points(uint64_t seed, uint64_t step, uint32_t stream_id, int64_t start,
                                int64_t n, float* pts, int64_t ld, hipStream_t stream);

/* Trilinear ground-truth sampling of a [nz][ny][nx] float32 volume at global
 * points (Sec. 4.3.1): voxel k of an axis of n voxels sits at -1 + 2k/(n-1);
 * u = fma(x, (n-1)/2, (n-1)/2), lower voxel clamp(floor(u), 0, n-2).
 *   v: [n] float32 output. */
apmg_status apmg_gt_sample(const float* volume, int32_t nx, int32_t ny, int32_t nz,
                           const float* pts, int64_t ld, int64_t n, float* v, hipStream_t stream);

/* ---------------------------------------------------------------- tracing
 * Timing hook for the dominant kernel: once set, the next apmg_backward or
 * apmg_batched_step call records `start` on its stream just before the first
 * launch of the adjoint tile kernel and `stop` just after its last launch,
 * then clears the hook.  The events are the caller's (hipEventCreate);
 * NULL, NULL clears the hook.  One hook per process; not thread-safe. */
apmg_status apmg_profile_events(hipEvent_t start, hipEvent_t stop);

/* The same hook for a chosen kernel: APMG_PROF_ADJOINT (as apmg_profile_events) or
 * APMG_PROF_GATHER, the per-cell grid-gradient gather of the next call that computes dF
 * (events around its launch, before the vertex sums).  One hook per kernel kind. */
#define APMG_PROF_ADJOINT 0
#define APMG_PROF_GATHER 1
apmg_status apmg_profile_kernel_events(int32_t kernel, hipEvent_t start, hipEvent_t stop);

#ifdef __cplusplus
}
#endif
#endif /* APMG_H */
