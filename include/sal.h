/*
 * sal.h -- C ABI of the MI355X (gfx950) seismic saliency library.
 *
 * The library computes the saliency map of Shafiq, Long, Alshawi and AlRegib, "Saliency
 * detection for seismic applications using multi-dimensional spectral projections and
 * directional comparisons" (ICIP 2017), Sec. 2:
 *   step 1  local 3D DFT of a sliding cube of side L around every voxel (DFT definition
 *           after Eq. (2), including the 1/L^3 factor);
 *   step 2  projection of each local spectrum along f_t, f_x, f_y (Eqs. (1)-(4)), with
 *           the DC bin excluded (paragraph after Fig. 2);
 *   step 3  spectral energies E_t, E_x, E_y: mean magnitude of each projected spectrum;
 *   step 4  directional center-surround comparison (Eq. (5)) with Gaussian weights;
 *   step 5  weighted combination S = a S_t + b S_x + c S_y (Eq. (6)).
 *
 * Conventions shared by every entry point:
 *   - Volumes are contiguous C-order arrays [n0][n1][n2]; axis 0 is t (time/depth),
 *     axis 1 is x, axis 2 is y (fastest).  Sec. 2 calls the volume "T x X x Y".
 *   - Every pointer named V, E, S, spectra or workspace is DEVICE memory on the context's
 *     device, owned by the caller; the library never frees or retains it beyond the call.
 *     Pointers must be 16-byte aligned.
 *   - Per-component maps are stored as [3][n0][n1][n2] in the order t, x, y.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the default
 *     stream).  Nothing synchronises unless stated.  A device fault of an earlier call is
 *     reported as SAL_E_DEVICE by a later call.
 *   - Every call returns a sal_status; no exception or abort crosses the ABI.  On an error
 *     nothing is enqueued and sal_last_error() describes it.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Window boundaries: samples outside the volume are reflected without repeating the
 *     edge sample (-1 -> 1, n -> n-2).  Every dimension must exceed max(floor(L/2), r).
 */
#ifndef SAL_H
#define SAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sal_ctx sal_ctx;

typedef enum {
    SAL_OK = 0,
    SAL_E_INVAL = 1,        /* bad argument: null/misaligned pointer, bad size or parameter */
    SAL_E_UNSUPPORTED = 2,  /* valid method parameters this GPU build does not implement */
    SAL_E_DEVICE = 3,       /* HIP runtime or device error */
    SAL_E_WORKSPACE = 4     /* workspace smaller than sal_workspace_size() */
} sal_status;

/* Arithmetic of the DFT contractions (steps 1-3).  Everything after step 3 is FP32 with
 * FP64 normalisation statistics and combination in every mode. */
typedef enum {
    SAL_FP32 = 0,         /* FP32 operands, FP32 accumulation (MFMA f32) */
    SAL_BF16 = 1,         /* BF16 data and DFT matrix, FP32 accumulation */
    SAL_BF16_SPLIT = 2,   /* DFT matrix and data each split into BF16 hi + lo parts; the
                             products W_hi d_hi, W_lo d_hi, W_hi d_lo (and W_lo d_lo where
                             it costs nothing) are accumulated in FP32 */
    SAL_FP16 = 3,         /* FP16 data and DFT matrix, FP32 accumulation */
    SAL_FP16_SPLIT = 4,   /* as SAL_BF16_SPLIT with FP16 parts */
    SAL_BF16_SPLITW = 5,  /* BF16 data times the DFT matrix split hi + lo (two products) */
    SAL_FP16_SPLITW = 6   /* FP16 data times the DFT matrix split hi + lo */
} sal_precision;
/* In every 16-bit form each contraction stage rounds its input to the 16-bit type; the FP16
 * forms scale each stage's FP32 output by 1/L (exact) to stay in range and need
 * |V| < 65504. */

/* Rays of the directional comparison of Eq. (5), one bit each.  Bits 0-5: the axis rays
 * +t, -t, +x, -x, +y, -y.  Oriented rays (Fig. 3 shows a t-x diagonal comparison): bits
 * 6-9 the t-x diagonals with step (t, x) = (+1,+1), (-1,-1), (+1,-1), (-1,+1); bits 10-13
 * the t-y and bits 14-17 the x-y diagonals in the same sign order; bits 18-25 the body
 * diagonals, bit 18 + k stepping -1 along t, x, y where bit 0, 1, 2 of k is set, else +1.
 * The s-th sample of a ray with step e is v + s e, weighted by
 * exp(-|s e|^2 / (2 sigma^2)). */
enum {
    SAL_RAY_PT = 1, SAL_RAY_MT = 2, SAL_RAY_PX = 4,
    SAL_RAY_MX = 8, SAL_RAY_PY = 16, SAL_RAY_MY = 32,
    SAL_RAY_DIAG_TX = 0xF << 6, SAL_RAY_DIAG_TY = 0xF << 10, SAL_RAY_DIAG_XY = 0xF << 14,
    SAL_RAY_BODY = 0xFF << 18, SAL_RAY_ALL = (1 << 26) - 1
};

/* Length of the statistics vector written by sal_saliency:
 * {lo_t, hi_t, lo_x, hi_x, lo_y, hi_y, max|V|}. */
#define SAL_STATS_LEN 7

typedef struct {
    int32_t L;          /* cube side of the local DFT (Sec. 2 step 1; the paper uses 5; the
                           last paragraph sets the resolution by the cube size).  GPU build:
                           2..20; the 16-bit forms at 8 and 16 only. */
    int32_t d;          /* length of the d x 1 comparison line (after Fig. 3), default L;
                           the line is r = floor(d/2) neighbours on each enabled ray. */
    double sigma;       /* width of the Gaussian neighbour weight w(s) = exp(-s^2/(2 sigma^2))
                           of Eq. (5); the paper gives none, default d/4. */
    uint32_t rays[3];   /* SAL_RAY_* masks used by S_t, S_x, S_y; default {+-t, +-x, +-y}:
                           each map compares along its own axis (Sec. 2, after Fig. 3). */
    double a, b, c;     /* weights of Eq. (6); default 1/3 each (equal shares, Sec. 2). */
    int32_t normalize;  /* 1: map each S_m to [0,1] by its volume-wide min and max before
                           Eq. (6) (default); 0: combine the raw maps. */
    double zero_range;  /* a component whose range is <= zero_range * max|V| has no
                           contrast and contributes 0 (default 1e-6). */
    int32_t precision;  /* sal_precision, default SAL_FP32 */
    int32_t stride;     /* window stride s: 1 (default) = one window per voxel; 2 <= s < L/2
                           (Sec. 2 step 1 asks for more than 50% overlap) or s = L (the
                           non-overlapping cubes of the predecessor method, Sec. 1) = windows
                           on the lattice of multiples of s, energies interpolated trilinearly
                           to every voxel, the last lattice value held at the far faces;
                           Eq. (5) and Eq. (6) on the full grid.  Strides above 2 run in FP32. */
    int32_t t_direct;   /* cube 8 or 16, FP32, stride 1 or 2: 0 (default) = each window's
                           spectrum is the previous window's along t plus the 2-D DFT of the
                           entering minus the leaving t-plane (the same DFT, a different
                           rounding; volumes of at least 2L x (L/2 + 1) x (L/2 + 1)); 1 = every
                           window's t contraction computed on its own.  Ignored elsewhere. */
} sal_params;

/* Fill *p with the defaults above for cube side L. */
void sal_default_params(sal_params *p, int32_t L);

/* Validate *p (copied) and create a context on HIP device `device`.  Builds the DFT
 * matrices and projection weight tables on that device.  Errors: SAL_E_INVAL (null out,
 * L < 2, d outside [2, 64], sigma <= 0, an empty ray mask or one with bits above 25, bad
 * precision, stride < 1, a stride of at least L/2 other than L), SAL_E_UNSUPPORTED (L above
 * 20, a 16-bit precision with L other than 8 and 16, a 16-bit precision with stride above 2),
 * SAL_E_DEVICE. */
sal_status sal_create(const sal_params *p, int device, sal_ctx **out);

/* Free the context and its device tables (waits for nothing; the caller must ensure no
 * enqueued work still uses the context). NULL is ignored. */
void sal_destroy(sal_ctx *ctx);

/* Text of the last error of this context (or of sal_create when ctx is NULL). */
const char *sal_last_error(const sal_ctx *ctx);

/* Bytes of device workspace sal_saliency needs for an n0 x n1 x n2 volume. */
sal_status sal_workspace_size(sal_ctx *ctx, int64_t n0, int64_t n1, int64_t n2, size_t *bytes);

/*
 * Local spectra of the voxels of the box [lo, lo + bn) of V (Sec. 2 step 1, DFT definition
 * after Eq. (2)).  spectra: device complex64 (re, im float pairs)
 * [bn0][bn1][bn2][L][L][L] in unshifted order mu, nu, om = 0..L-1 along (t, x, y),
 * including the 1/L^3 factor.  The box must lie inside the volume.  Meant for checks on
 * small boxes: the output is L^3 complex values per voxel.
 */
sal_status sal_local_spectra(sal_ctx *ctx, const float *V, int64_t n0, int64_t n1, int64_t n2,
                             const int64_t lo[3], const int64_t bn[3], void *spectra,
                             void *stream);

/*
 * Spectral energies from given spectra (Sec. 2 steps 2-3, Eqs. (1)-(4)):
 *   E_m = (1/(L^3-1)) sum over the bins other than DC of w_m(i,j,k) |F[mu,nu,om]|,
 *   w_t = sqrt(j^2+k^2)/rho, w_x = sqrt(i^2+k^2)/rho, w_y = sqrt(i^2+j^2)/rho,
 *   rho = sqrt(i^2+j^2+k^2), (i,j,k) the signed frequencies of (mu,nu,om).
 * spectra: device complex64 [nvox][L][L][L] (layout of sal_local_spectra);
 * E: device float [3][nvox].
 */
sal_status sal_project(sal_ctx *ctx, const void *spectra, int64_t nvox, float *E, void *stream);

/*
 * Directional center-surround comparison (Eq. (5)) on given energies:
 *   S_m[v] = (1/Q_m) sum over enabled rays e of m, s = 1..r, of |E_m[v] - w(s) E_m[v + s e]|,
 *   Q_m = (enabled rays of m) * r, w(s) = exp(-s^2 / (2 sigma^2)), reflected at the edges.
 * E, S_raw: device float [3][n0][n1][n2]; they must not overlap.
 */
sal_status sal_directional_compare(sal_ctx *ctx, const float *E, int64_t n0, int64_t n1,
                                   int64_t n2, float *S_raw, void *stream);

/*
 * The whole method, steps 1-5, on a device-resident volume.
 *   V          device float [n0][n1][n2], input
 *   S          device float [n0][n1][n2], output saliency map (Eq. (6))
 *   E_out      optional device float [3][n0][n1][n2]: energies (NULL: not written)
 *   S_raw_out  optional device float [3][n0][n1][n2]: maps of Eq. (5) before
 *              normalisation (NULL: not written)
 *   stats_out  optional DEVICE double [SAL_STATS_LEN]: {lo_t, hi_t, lo_x, hi_x, lo_y, hi_y,
 *              max|V|}, the volume-wide FP64 statistics used by the normalisation
 *   workspace  device scratch of at least sal_workspace_size() bytes, ws_bytes its size
 * The normalisation statistics are reduced in FP64 and Eq. (6) is evaluated in FP64 per
 * voxel, then stored as FP32.  Errors: SAL_E_INVAL, SAL_E_WORKSPACE, SAL_E_DEVICE.
 */
sal_status sal_saliency(sal_ctx *ctx, const float *V, int64_t n0, int64_t n1, int64_t n2,
                        float *S, float *E_out, float *S_raw_out, double *stats_out,
                        void *workspace, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sal_saliency without a workspace.  The
 * energies and raw maps are required outputs (E_out, S_raw_out, DEVICE float
 * [3][n0][n1][n2]); the per-block partial reductions and, when stats_out is NULL, the
 * statistics go to a 16 MiB device scratch array that the library holds on each GPU for the
 * life of the process.  Nothing is allocated or freed.  Every call on one GPU shares that
 * GPU's scratch and leaves its last contents there: calls that overlap on one GPU (several
 * streams, threads or contexts) race and must be serialised by the caller.  Stride 1 only.
 * Results equal those of sal_saliency bit for bit.  Errors: SAL_E_INVAL (null or misaligned
 * pointers, bad dimensions, a volume whose partials need more than the 16 MiB scratch),
 * SAL_E_UNSUPPORTED (stride > 1), SAL_E_DEVICE.
 */
sal_status sal_saliency_noalloc(sal_ctx *ctx, const float *V, int64_t n0, int64_t n1, int64_t n2,
                                float *S, float *E_out, float *S_raw_out, double *stats_out,
                                void *stream);

/*
 * Per-kernel timing of sal_saliency.  While enabled (on != 0), every sal_saliency call
 * records HIP events on its stream around each of its kernels: [0] the fused steps 1-3
 * kernel, [1] the comparison of Eq. (5), [2] the FP64 statistics, [3] the FP64
 * combination.  sal_profile_read waits for the recorded events, returns the summed
 * durations in milliseconds in ms[4] and the number of timed calls in *calls, and forgets
 * them when reset != 0.  Disabling also forgets them.  Timing adds four event records
 * per call and no synchronisation until read.
 */
sal_status sal_profile_enable(sal_ctx *ctx, int on);
sal_status sal_profile_read(sal_ctx *ctx, double ms[4], int64_t *calls, int reset);

/*
 * Steps 1-4 for one box of the volume (Sec. 2, Eqs. (1)-(5)): the raw maps S_t, S_x, S_y of
 * the positions box_lo + [0, box_dims), written box-local to S_raw_box (DEVICE float
 * [3][b0][b1][b2]), equal to the same positions of the whole-volume maps of sal_saliency.
 * The energies are computed on the box grown by r = floor(d/2) (clipped to the volume) and
 * windows reflect at the volume faces only, so V may be the whole volume or any crop whose
 * faces inside the volume lie at least floor(L/2) + r from the box.  With stride s > 1 the
 * energies of the grown box are interpolated from the lattice windows around it, the lattice
 * starting at the first sample of V (a crop must start on a multiple of s, and lie at least
 * floor(L/2) + r + s from the box, for the whole volume's values).  Equal means bit for bit,
 * except where the windows slide along t (cube 8 or 16, FP32, stride 1 or 2, t_direct = 0):
 * their running spectra restart at fixed rows of the volume given, so a box of that volume
 * equals its whole-volume maps bit for bit and a crop equals them to rounding.  workspace: at least
 * sal_raw_box_workspace_size(box_dims) bytes, DEVICE, 16-byte aligned.
 */
sal_status sal_raw_box_workspace_size(sal_ctx *ctx, const int64_t box_dims[3], size_t *bytes);
sal_status sal_raw_box(sal_ctx *ctx, const float *V, int64_t n0, int64_t n1, int64_t n2,
                       const int64_t box_lo[3], const int64_t box_dims[3], float *S_raw_box,
                       void *workspace, size_t ws_bytes, void *stream);

/*
 * Largest magnitude of a device array, the scale of the zero-contrast rule of
 * sal_normalize_combine when the volume is not resident (e.g. reduced slab by slab while a
 * host volume streams through HBM).  V: DEVICE float [n] (may be NULL when n = 0);
 * vmax_out: DEVICE float, set to
 * max |V[i]| (accumulate == 0) or to max(*vmax_out, max |V[i]|) (accumulate != 0, *vmax_out
 * >= 0 before the call).  NaN elements are ignored.  Errors: SAL_E_INVAL, SAL_E_DEVICE.
 */
sal_status sal_absmax(sal_ctx *ctx, const float *V, int64_t n, float *vmax_out, int accumulate, void *stream);

/*
 * Steps 4b-5 on given raw maps S_raw float [3][n0][n1][n2]: the FP64 volume-wide statistics
 * and the normalised combination of Eq. (6) (same arithmetic as sal_saliency).  The scale of
 * the zero-contrast rule is max|V| over V (float [n0][n1][n2]) when V is given, else the
 * caller's vmax (> 0; e.g. reduced slab by slab when V is not resident).  stats_out:
 * optional DEVICE double [SAL_STATS_LEN].  workspace: at least sal_workspace_size() bytes.
 */
sal_status sal_normalize_combine(sal_ctx *ctx, const float *V, double vmax, const float *S_raw,
                                 int64_t n0, int64_t n1, int64_t n2, float *S, double *stats_out,
                                 void *workspace, size_t ws_bytes, void *stream);

/*
 * Tile check of a predicted raw map against the plain method: over the tile
 * [tile_lo, tile_lo + tile_dims) of S_raw (float [3][n0][n1][n2]) and the same voxels of
 * `exact` (float [3][c0][c1][c2], the plain method's raw maps on the crop starting at
 * crop_lo), err = max over voxels and components m of |pred - exact| / (hi_m - lo_m) with
 * the range from `stats` (DEVICE double [SAL_STATS_LEN], e.g. of the predicted map).  Writes
 * err to *err_out (DEVICE float) and, when err > bound, overwrites the tile of S_raw with
 * the exact values.  The tile must lie inside both the volume and the crop.
 */
/* A difference that is not finite (a NaN or infinite prediction) counts as an infinite error,
 * so such a tile is always replaced. */
sal_status sal_tile_merge(sal_ctx *ctx, float *S_raw, int64_t n0, int64_t n1, int64_t n2,
                          const float *exact, const int64_t crop_lo[3], const int64_t crop_dims[3],
                          const int64_t tile_lo[3], const int64_t tile_dims[3],
                          const double *stats, double bound, float *err_out, void *stream);

/*
 * Batched tile check (the surrogate's fallback): for nbox tiles of equal size tile_dims,
 * steps 1-4 (Sec. 2, Eqs. (1)-(5)) on each tile as sal_raw_box computes them, then the check
 * and replacement of sal_tile_merge, in one pass over all tiles.
 *   V, n0..n2   DEVICE float volumes, each n0 x n1 x n2; volume b starts at V + b * vol_stride
 *               (vol_stride = 0: every tile lies in the same volume, else a multiple of 4 of
 *               at least n0 n1 n2 floats).  A volume may be a crop of a larger one: windows
 *               reflect at its faces, so a face inside the larger volume must lie at least
 *               floor(L/2) + r from the tile (with windows sliding along t the crop's maps
 *               then equal the larger volume's to rounding, as for sal_raw_box).
 *   box_lo      HOST int64 [nbox][3]: origin of tile b in volume b
 *   S_raw, m0..m2  DEVICE float [3][m0][m1][m2]: the predicted raw maps
 *   tile_lo     HOST int64 [nbox][3]: origin of tile b in S_raw
 *   stats       DEVICE double [SAL_STATS_LEN] giving the ranges hi_m - lo_m of the error
 *   err_out     DEVICE float [nbox]: err of each tile as in sal_tile_merge; tiles with
 *               err > bound are overwritten in S_raw with the exact maps
 *   exact_out   optional DEVICE float [nbox][3][d0][d1][d2]: the exact maps (NULL: kept in
 *               the workspace)
 *   workspace   DEVICE, at least sal_check_tiles_workspace_size() bytes for the same
 *               n0..n2, nbox and tile_dims
 * Tiles must not overlap (the replacement of one would otherwise race with the check of
 * another).  The tile tables are copied from host memory into the workspace at call time
 * (through a pinned staging buffer of the context, reused only after the previous copy from
 * it has completed, which may wait for that copy); the call therefore cannot be captured
 * into a HIP graph and is refused on a capturing stream.  With stride s > 1 each tile's
 * energies come from the lattice windows around its grown box, as in sal_raw_box.
 * Errors: SAL_E_INVAL (a tile outside its volume or the map, nbox outside [1, 2^20], tile
 * sides outside [1, 1024], or a batch whose energy boxes hold more than 2^31 - 1 voxels:
 * split it over several calls), SAL_E_UNSUPPORTED (a capturing stream),
 * SAL_E_WORKSPACE, SAL_E_DEVICE.
 */
sal_status sal_check_tiles_workspace_size(sal_ctx *ctx, int64_t n0, int64_t n1, int64_t n2, int64_t nbox,
                                          const int64_t tile_dims[3], size_t *bytes);
sal_status sal_check_tiles(sal_ctx *ctx, const float *V, int64_t n0, int64_t n1, int64_t n2,
                           int64_t vol_stride, const int64_t *box_lo, float *S_raw, int64_t m0, int64_t m1,
                           int64_t m2, const int64_t *tile_lo, int64_t nbox, const int64_t tile_dims[3],
                           const double *stats, double bound, float *err_out, float *exact_out,
                           void *workspace, size_t ws_bytes, void *stream);

/*
 * Per-tile extremes of raw maps S_raw (float [3][n0][n1][n2]) over the tiles of side `tile`
 * (the last tile along an axis may be shorter), tiles numbered (t, x, y) with y fastest:
 * out (DEVICE float [ntiles][6]) = {min_t, max_t, min_x, max_x, min_y, max_y} per tile,
 * ntiles = ceil(n0/tile) ceil(n1/tile) ceil(n2/tile).  Used to find every tile whose
 * predicted values could set the volume-wide statistics of Eq. (6).
 */
sal_status sal_tile_minmax(sal_ctx *ctx, const float *S_raw, int64_t n0, int64_t n1, int64_t n2,
                           int32_t tile, float *out, void *stream);

/* ------------------------------------------------------------------------------------
 * Learned surrogate (not part of the paper's method): five 3x3x3 convolutions, channels
 * 1 -> 24 -> 24 -> 24 -> 24 -> 3 with GELU between them, predicting the raw maps
 * S_t, S_x, S_y of Eq. (5) from the volume; BF16 weights/activations, FP32 accumulation,
 * FP32 master weights trained with Adam.  The normalisation and Eq. (6) stay exact
 * (sal_normalize_combine).  Activations are channel-last over nb blocks of n0 x n1 x n2
 * voxels; convolution taps are reflected inside each block.  Parameters are one flat FP32
 * vector: for each layer, W[co][27][ci] (tap k = (dt*3+du)*3+dw reads (t+dt-1, u+du-1,
 * w+dw-1)) then the bias[co].  A sal_net owns its device buffers; not thread-safe.
 */
typedef struct sal_net sal_net;

int64_t sal_net_num_params(void);
const char *sal_net_last_error(const sal_net *net);
/* Kaiming-uniform weights from `seed`, zero biases. */
sal_status sal_net_create(int device, uint64_t seed, sal_net **out);
void sal_net_destroy(sal_net *net);
/* Copy the FP32 master parameters to (write = 0) or from (write = 1) host memory. */
sal_status sal_net_params(sal_net *net, float *host, int64_t count, int write);
/* Copy the accumulated FP32 gradient to host memory; zero it when zero != 0 (synchronises). */
sal_status sal_net_grads(sal_net *net, float *host, int64_t count, int zero);
/* Inference output = network output * scale[c] (the training targets are divided by it). */
sal_status sal_net_set_output_scale(sal_net *net, const float scale[3]);
/* Device workspace of sal_net_forward/backward/train_step (train != 0) or sal_net_infer. */
sal_status sal_net_workspace_size(sal_net *net, int64_t nb, int64_t n0, int64_t n1, int64_t n2,
                                  int train, size_t *bytes);
/* Forward pass: X float [nb][n0][n1][n2] -> Y float [nb][n0][n1][n2][3]; keeps the
 * activations in the workspace for sal_net_backward. */
sal_status sal_net_forward(sal_net *net, const float *X, int64_t nb, int64_t n0, int64_t n1,
                           int64_t n2, float *Y, void *workspace, size_t ws_bytes, void *stream);
/* Backward pass after sal_net_forward on the same X and workspace: adds the gradient of
 * sum(dY * Y) to the net's gradient.  Exact only when dY vanishes within 5 voxels of every
 * block face (the input gradient uses zero padding). */
sal_status sal_net_backward(sal_net *net, const float *X, const float *dY, int64_t nb, int64_t n0,
                            int64_t n1, int64_t n2, void *workspace, size_t ws_bytes,
                            void *stream);
/* Arithmetic of the network's convolutions: SAL_BF16 (default; BF16 weights and activations,
 * FP32 accumulation) or SAL_FP32 (the same kernels with FP32 weights and activations, for
 * element-wise checks against an FP64 reference).  Applies to every later call; workspace
 * sizes depend on it.  Errors: SAL_E_INVAL. */
sal_status sal_net_set_precision(sal_net *net, int32_t precision);
/* One Adam step (betas 0.9/0.999, eps 1e-8, bias-corrected with the net's step count) of
 * learning rate lr >= 0 on the FP32 master parameters from the gradient accumulated by
 * sal_net_backward, which it then clears; rebuilds the operand tables.  Asynchronous on
 * `stream`.  Errors: SAL_E_INVAL, SAL_E_DEVICE. */
sal_status sal_net_adam(sal_net *net, float lr, void *stream);
/* One training step: forward, the gradient of the mean squared error between the
 * network output and T float [nb][S][S][S][3] over the voxels at least `margin` (>= 5)
 * from every face of their S^3 block, then sal_net_adam(lr).  loss_out: optional DEVICE
 * float. */
sal_status sal_net_train_step(sal_net *net, const float *X, const float *T, int64_t nb, int64_t S,
                              int32_t margin, float lr, float *loss_out, void *workspace,
                              size_t ws_bytes, void *stream);
/* Whole-volume inference: V float [n0][n1][n2] -> S_raw float [3][n0][n1][n2]. */
sal_status sal_net_infer(sal_net *net, const float *V, int64_t n0, int64_t n1, int64_t n2,
                         float *S_raw, void *workspace, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SAL_H */
