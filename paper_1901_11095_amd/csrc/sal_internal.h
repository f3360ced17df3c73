// Internal declarations shared by the C-ABI front end and the gfx950 kernels of libsal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sal.h"
#include "sal_device.h"

// Device tables built once per context from FP64 values rounded to the kernel's type.
struct sal_tables {
    float *w_c;      // [2L][2L] real form of the L-point DFT matrix: row (freq, re|im),
                     // column (tap, re|im); the y contraction's A operand (and the x one's at
                     // cube 8).  At cube 16 the rows are in the folded order (M tile 0 pairs
                     // om with L - om in each lane group)
    float *w_a;      // [16*MTA][L] real-input DFT along t: row (mu, re|im) for mu <= L/2,
                     // zero rows above
    float *w_bin;    // per weight group (mu, k <= L/2), M tile, lane group: 8 floats holding
                     // the projection weights (t, x, y) of the two bins a lane owns (one set
                     // for a folded tile, whose two bins share it), times the Hermitian
                     // multiplicity and 1/(L^3 (L^3-1)) (and L^2 for the FP16 forms, whose
                     // stage outputs are scaled by 1/L); DC has weight 0
    float *twiddle;  // [L][2] exp(-2 pi i k / L), for the per-voxel spectra kernel
    float *w_proj;   // [L^3][4] projection weights / (L^3 - 1) of bin (mu,nu,om), DC = 0
    uint32_t *w_c16;  // 16-bit forms: per M tile, operand and lane, the eight 16-bit A-operand
                      // values of the y contraction (and the x one's at cube 8), in the K
                      // orders of sal_energy16.hip (three products at cube 16 with the data
                      // split: operands W_hi, W_lo; else J = L/8 operands of W_hi | W_lo)
    uint32_t *w_a16;  // likewise for the t contraction (one or two words per tap)
    uint32_t *w_c16b;  // cube 16: the x contraction's operands, in the stage-B halves' row
                       // order with the data split (rows nu = k and L - k of a weight group in
                       // the same half), in frequency order without
    float *w_cb;       // cube 16, FP32 kernel: the stage-B matrix of the two halves, rows in
                       // the halves' order, as per-lane A operands [half][K step][lane]
    float *w_gen;     // vector-ALU kernel (L < 8): [mu <= L/2][nu][om][3] projection weights
                      // times the conjugate multiplicity of mu, / (L^3 (L^3 - 1)), DC = 0
    float *w_s1;      // cube 8 or 16, FP32 with windows sliding along t: stage-1 (packed real
                      // DFT along x) A operands [K step][lane]
    float *w_s2;      // its stage-2 (complex DFT along y) A operands [M tile][K step][lane],
                      // rows ky and -ky in one lane group
    float *w_sp;      // its projection weights [column][lane group][slide_weights_per_group(L)]
};

// Windows sliding along t (cube L = 8 or 16, FP32, stride 1): the running spectra restart
// from zero at the windows t0 = 0, r = L/2 and every multiple of SLIDE_SEG from SLIDE_SEG on;
// segment k covers the windows [slide_seg_start(k, r), slide_seg_start(k + 1, r)).
constexpr int SLIDE_SEG = 512;
__host__ __device__ inline int slide_seg_id(int t, int r) { return t < r ? 0 : (t < SLIDE_SEG ? 1 : t / SLIDE_SEG + 1); }
__host__ __device__ inline int slide_seg_start(int k, int r) { return k == 0 ? 0 : (k == 1 ? r : (k - 1) * SLIDE_SEG); }
// Projection weights per (column, lane group) of that kernel: column 0 holds two sets per
// slot of M tile 0 (A and B, 6 (L/2 + 1)) and one per slot of the others (3 (L/2 + 1) each)
__host__ __device__ constexpr int slide_weights_per_group(int L)
{
    return ((12 * (L / 2 + 1) + (L / 8 - 1) * 6 * (L / 2 + 1)) + 7) / 8 * 8;
}

struct sal_ctx {
    sal_params p;
    int device;
    int L, H, h, r, nrows;
    float g[96];       // Gaussian neighbour weights w(s |e|), s = 1..r (index 32 (|e|^2 - 1) + s - 1)
    float Q[3];        // number of terms of Eq. (5) per component
    float tw_host[64]; // e^{-2 pi i k / L} (re, im), k < L
    sal_tables t;
    std::string err;
    // per-kernel timing of sal_saliency (sal_profile_enable / sal_profile_read)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;  // 5 events per timed call
    size_t ev_used = 0;
    // pinned staging of the box tables of sal_check_tiles, reused once the event recorded
    // after the last upload from it has completed
    int *tab_host = nullptr;
    size_t tab_cap = 0;
    hipEvent_t tab_done = nullptr;
    void *scratch = nullptr;  // device address of this device's sal_saliency_noalloc scratch
};

// Bytes of the device scratch of sal_saliency_noalloc (one static array per GPU).
#define SAL_NOALLOC_SCRATCH_BYTES (16u << 20)

// Arguments of the directional comparison kernel.
struct dcs_args {
    int r;
    uint32_t rays[3];
    float Q[3];
    float g[96];  // w(s |e|) at index 32 (|e|^2 - 1) + s - 1
};

// Ray bits with a step along t, x, y (axis rays, the diagonals of the planes holding the
// axis, the body diagonals)
constexpr uint32_t RAYS_T = 0x3u | (0xFu << 6) | (0xFu << 10) | (0xFFu << 18);
constexpr uint32_t RAYS_X = 0xCu | (0xFu << 6) | (0xFu << 14) | (0xFFu << 18);
constexpr uint32_t RAYS_Y = 0x30u | (0xFu << 10) | (0xFu << 14) | (0xFFu << 18);

// Step (t, x, y) of ray bit b of a comparison mask (axis rays, face and body diagonals;
// the bit layout of SAL_RAY_*).
__host__ __device__ inline void ray_step(int b, int &dt, int &dx, int &dy)
{
    dt = dx = dy = 0;
    if (b < 6) {
        const int d = (b & 1) ? -1 : 1;
        if (b < 2) dt = d;
        else if (b < 4) dx = d;
        else dy = d;
    } else if (b < 18) {
        const int pl = (b - 6) >> 2, k = (b - 6) & 3;
        const int s0 = (k == 0 || k == 2) ? 1 : -1, s1 = (k == 0 || k == 3) ? 1 : -1;
        if (pl == 0) { dt = s0; dx = s1; }
        else if (pl == 1) { dt = s0; dy = s1; }
        else { dx = s0; dy = s1; }
    } else {
        const int k = b - 18;
        dt = (k & 1) ? -1 : 1;
        dx = (k & 2) ? -1 : 1;
        dy = (k & 4) ? -1 : 1;
    }
}

// Output box of the fused kernels: E is computed for the volume positions o + [0, d) (the
// positions o + S k, k < ceil(d / S), with stride S) and stored in a frame: as
// [3][fk0][fk1][fk2] with position p at index (p - fo) / S.  For one box the frame is the
// box itself; windows still read the whole volume (reflected at its faces).
// Batched boxes (tile checks): when `table` is set, workgroup w serves table entry
// e = w / per_box (after the XCD-aware renumbering), whose ENERGY_TABLE ints hold
// {o, d, fo, fk, v}: the box, its frame, and the index v of its volume (which starts
// v * vstride floats into V) and of its E (v * estride floats into E).  The grid of one
// entry is sized for the largest box; workgroups past a smaller box exit at once.
struct ebox {
    int o0, o1, o2, d0, d1, d2;
    int fo0 = 0, fo1 = 0, fo2 = 0, fk0 = 0, fk1 = 0, fk2 = 0;
    const int *table = nullptr;
    int per_box = 0;
    int64_t vstride = 0, estride = 0;
};
constexpr int ENERGY_TABLE = 16;
// ints per tile in the table of the comparison and merge kernels of a batch: grown box
// {o0, o1, o2, d0, d1, d2} in volume b, the tile origin in volume b, the tile origin in the
// predicted map
constexpr int BOX_TABLE = 12;

// A box that is its own frame.
inline ebox framed_box(int o0, int o1, int o2, int d0, int d1, int d2, int S)
{
    ebox b{o0, o1, o2, d0, d1, d2};
    b.fo0 = o0;
    b.fo1 = o1;
    b.fo2 = o2;
    b.fk0 = (d0 + S - 1) / S;
    b.fk1 = (d1 + S - 1) / S;
    b.fk2 = (d2 + S - 1) / S;
    return b;
}

// Workgroup -> tile of its box; for a batch it also loads the geometry of its table entry
// and returns in *v the index of the entry's volume and E (the caller moves its pointers).
__device__ __forceinline__ int box_tile(ebox &bx, int *v)
{
    const int t = sal_dev::xcd_tile(blockIdx.x, gridDim.x);
    *v = 0;
    if (!bx.table) return t;
    const int e = t / bx.per_box;
    const int *q = bx.table + ENERGY_TABLE * e;
    bx.o0 = q[0];
    bx.o1 = q[1];
    bx.o2 = q[2];
    bx.d0 = q[3];
    bx.d1 = q[4];
    bx.d2 = q[5];
    bx.fo0 = q[6];
    bx.fo1 = q[7];
    bx.fo2 = q[8];
    bx.fk0 = q[9];
    bx.fk1 = q[10];
    bx.fk2 = q[11];
    *v = q[12];
    return t - e * bx.per_box;
}

// ------------------------------------------------------------------ launchers
// All return hipSuccess or the launch error.
// box: NULL for the whole volume, else {o0, o1, o2, d0, d1, d2}: E of the positions o + [0, d)
// stored box-local as [3][d0][d1][d2]
hipError_t launch_energy(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                         const int64_t *box, float *E, float *vmax_part, int *nparts,
                         hipStream_t s);
int64_t energy_num_blocks(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2);
hipError_t launch_energy16(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                           const ebox &bx, float *E, float *vmax_part, int nby, int nbx, int tt,
                           int64_t nb, hipStream_t s);
// nbox table entries (ENERGY_TABLE ints each, device) of boxes of at most maxd voxels per
// axis; returns the number of vmax partials written in *nparts
hipError_t launch_energy_boxes(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                               int64_t vstride, const int *table, int nbox, const int64_t maxd[3], float *E,
                               int64_t estride, float *vmax_part, int *nparts, hipStream_t s);
// Eq. (5) on the tiles of a batch (tile origin in volume b from the table), each from the E
// of its grown box; S_box[b][3][d0][d1][d2] written sstride floats apart
hipError_t launch_dcs_boxes(const sal_ctx *c, const float *Eb, int64_t estride, const int *table, int nbox,
                            const int64_t n[3], const int64_t bd[3], float *S_box, hipStream_t s);
// error and replacement of the tiles of a batch in the predicted map (origin from the table)
hipError_t launch_tile_merge_boxes(float *S_raw, int64_t n0, int64_t n1, int64_t n2, const float *exact,
                                   const int *table, int nbox, const int64_t td[3], const double *stats,
                                   double bound, float *err, hipStream_t s);

int64_t energy_gen_num_blocks(int L, int64_t d0, int64_t d1, int64_t d2, int64_t nbox = 1);
// Window-by-window energies (strides >= 3, the non-overlapping stride L, cube sides without a
// fused kernel): bx as for the fused kernels, windows at o + stride k.
hipError_t launch_energy_win(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, const ebox &bx,
                             float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox = 1);
int64_t energy_win_num_blocks(const sal_ctx *c, int64_t k0, int64_t k1, int64_t k2);
// Whether the energies of this context come from the window-by-window kernel.
inline bool uses_window_kernel(const sal_ctx *c)
{
    const int L = c->L, S = c->p.stride;
    if (S >= 3 || (S > 1 && S == L)) return true;
    return !(L <= 8 || L == 16);
}
// Whether the energies of a volume n0 x n1 x n2 come from the kernel whose windows slide
// along t: cube 8 or 16, FP32, stride 1 or any overlapping stride below L/2, unless the
// context asks for the direct t contraction; the t walk needs 2L rows, the reflected window
// rows L/2 + 1 samples per axis.  Checked before the window-by-window kernel.
inline bool uses_slide_kernel(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2)
{
    const int L = c->L;
    return (L == 8 || L == 16) && c->p.precision == SAL_FP32 && 2 * c->p.stride < L && !c->p.t_direct &&
           n0 >= 2 * L && n1 >= L / 2 + 1 && n2 >= L / 2 + 1;
}
hipError_t launch_energy_slide(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, ebox bx,
                               float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox = 1);
int64_t energy_slide_num_blocks(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2);
// bx.table set: nbox boxes of at most bx.d voxels per axis (the grid is nbox times that of one)
hipError_t launch_energy_gen(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, const ebox &bx,
                             float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox = 1);

hipError_t launch_dcs(const sal_ctx *c, const float *E, int64_t n0, int64_t n1, int64_t n2,
                      float *S_raw, float *minmax_part, hipStream_t s);
int64_t dcs_num_blocks(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2);
hipError_t launch_upsample(const float *El, int64_t K0, int64_t K1, int64_t K2, int S, int64_t n0, int64_t n1,
                           int64_t n2, float *E, hipStream_t s);
// ints per box of the batched interpolation: {kd, klo, K, eo, ed} (three each)
constexpr int LAT_TABLE = 15;
// nbox boxes, table entries of LAT_TABLE ints (device), maxed the largest box
hipError_t launch_upsample_boxes(const float *El, int64_t lstride, const int *table, int nbox, const int64_t maxed[3],
                                 int S, float *E, int64_t estride, hipStream_t s);
// El: the lattice points klo + [0, kd) of a volume with lattice dims K; E: the voxels
// eo + [0, ed), box-local
hipError_t launch_upsample_box(const float *El, const int64_t kd[3], const int64_t klo[3], const int64_t K[3], int S,
                               const int64_t eo[3], const int64_t ed[3], float *E, hipStream_t s);
hipError_t launch_dcs_box(const sal_ctx *c, const float *Eb, const int64_t eo[3], const int64_t ed[3],
                          const int64_t n[3], const int64_t bo[3], const int64_t bd[3], float *S,
                          hipStream_t s);

hipError_t launch_stats(const float *vmax_part, int64_t nv, const float *minmax_part,
                        int64_t nm, double *stats, hipStream_t s);

hipError_t launch_combine(const float *S_raw, int64_t nvox, const double *stats, double a,
                          double b, double c, int normalize, double zero_range, float *S,
                          hipStream_t s);

int64_t merge_red_blocks(int64_t N);
// out[0] = max(out[0], max |V[0..N)|) (accumulate != 0) or max |V[0..N)| (accumulate == 0)
hipError_t launch_absmax_acc(const float *V, int64_t N, float *out, int accumulate, hipStream_t s);
hipError_t launch_minmax_absmax(const float *V, float vmax, const float *S_raw, int64_t N,
                                float *mm_part, float *vmax_part, hipStream_t s);
hipError_t launch_tile_merge(float *S_raw, int64_t n0, int64_t n1, int64_t n2, const float *exact,
                             const int64_t crop_lo[3], const int64_t crop_dims[3],
                             const int64_t tile_lo[3], const int64_t tile_dims[3],
                             const double *stats, double bound, float *err, hipStream_t s);

hipError_t launch_tile_minmax(const float *S_raw, int64_t n0, int64_t n1, int64_t n2, int tile,
                              float *out, hipStream_t s);

hipError_t launch_local_spectra(const sal_ctx *c, const float *V, int64_t n0, int64_t n1,
                                int64_t n2, const int64_t lo[3], const int64_t bn[3],
                                float *out, hipStream_t s);

hipError_t launch_project(const sal_ctx *c, const float *spectra, int64_t nvox, float *E,
                          hipStream_t s);
