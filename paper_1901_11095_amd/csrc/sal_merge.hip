// Reductions and tile merging used when raw maps come from elsewhere than the fused path
// (the learned surrogate): per-block min/max of the three raw maps, per-block max|V|, and
// the check/merge of a predicted tile against the plain method's values.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "sal_device.h"
#include "sal_internal.h"

namespace {
constexpr int RED_BLOCKS = 4096;
}

// partial {min_t, max_t, min_x, max_x, min_y, max_y} of S_raw [3][N] per workgroup
__global__ __launch_bounds__(256) void k_minmax3(const float *__restrict__ S, int64_t N, float *__restrict__ part)
{
    float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < N; v += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const float x = S[m * N + v];
            mn[m] = fminf(mn[m], x);
            mx[m] = fmaxf(mx[m], x);
        }
    __shared__ float red[4][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            mn[m] = fminf(mn[m], __shfl_xor(mn[m], o));
            mx[m] = fmaxf(mx[m], __shfl_xor(mx[m], o));
        }
        if (lane == 0) {
            red[wave][2 * m] = mn[m];
            red[wave][2 * m + 1] = mx[m];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float r = red[0][k];
        for (int w = 1; w < 4; ++w) r = (k & 1) ? fmaxf(r, red[w][k]) : fminf(r, red[w][k]);
        part[(int64_t)blockIdx.x * 6 + k] = r;
    }
}

// partial max|V| per workgroup (the given value when V is absent)
__global__ __launch_bounds__(256) void k_absmax(const float *__restrict__ V, int64_t N, float vmax,
                                                float *__restrict__ part)
{
    float m = V ? 0.f : vmax;
    if (V)
        for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < N; v += (int64_t)gridDim.x * 256)
            m = fmaxf(m, fabsf(V[v]));
    __shared__ float red[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ void k_fill_f32(float *p, float v) { *p = v; }

// out[0] = max(out[0], max |V|): block maxima joined by an atomic max on the bit pattern (the
// values are non-negative, so float order equals unsigned order)
__global__ __launch_bounds__(256) void k_absmax_acc(const float *__restrict__ V, int64_t N, float *__restrict__ out)
{
    float m = 0.f;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < N; v += (int64_t)gridDim.x * 256)
        m = fmaxf(m, fabsf(V[v]));
    __shared__ float red[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned int *>(out),
                  __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
}

// |pred - exact| * inv for the tile check; a non-finite difference (a NaN or infinite
// prediction) counts as +inf, so its tile is always over the bound and replaced
__device__ __forceinline__ float tile_diff(float pred, float exact, float inv)
{
    const float d = fabsf(pred - exact) * inv;
    return d <= FLT_MAX ? d : __int_as_float(0x7f800000);
}

struct box3 {
    int64_t lo[3], d[3];
};

// err = max |pred - exact| / range_m over the tile; max combined with atomicMax on the bit
// pattern (errors are non-negative, so float order equals unsigned order)
__global__ __launch_bounds__(256) void k_tile_err(const float *__restrict__ S, int n0, int n1, int n2,
                                                  const float *__restrict__ X, box3 crop, box3 tile,
                                                  const double *__restrict__ stats, float *__restrict__ err)
{
    const int64_t nt = tile.d[0] * tile.d[1] * tile.d[2];
    const int64_t N = (int64_t)n0 * n1 * n2, NC = crop.d[0] * crop.d[1] * crop.d[2];
    float inv[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double r = stats[2 * m + 1] - stats[2 * m];
        inv[m] = r > 0.0 ? (float)(1.0 / r) : 0.f;
    }
    float e = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nt; i += (int64_t)gridDim.x * 256) {
        const int64_t a = i / (tile.d[1] * tile.d[2]), b = (i / tile.d[2]) % tile.d[1], c = i % tile.d[2];
        const int64_t t = tile.lo[0] + a, x = tile.lo[1] + b, y = tile.lo[2] + c;
        const int64_t vo = (t * n1 + x) * n2 + y;
        const int64_t co = ((t - crop.lo[0]) * crop.d[1] + (x - crop.lo[1])) * crop.d[2] + (y - crop.lo[2]);
#pragma unroll
        for (int m = 0; m < 3; ++m) e = fmaxf(e, tile_diff(S[m * N + vo], X[m * NC + co], inv[m]));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) e = fmaxf(e, __shfl_xor(e, o));
    if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned int *>(err), __float_as_uint(e));
}

__global__ __launch_bounds__(256) void k_tile_copy(float *__restrict__ S, int n0, int n1, int n2,
                                                   const float *__restrict__ X, box3 crop, box3 tile,
                                                   const float *__restrict__ err, float bound)
{
    if (!(*err > bound)) return;
    const int64_t nt = tile.d[0] * tile.d[1] * tile.d[2];
    const int64_t N = (int64_t)n0 * n1 * n2, NC = crop.d[0] * crop.d[1] * crop.d[2];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nt; i += (int64_t)gridDim.x * 256) {
        const int64_t a = i / (tile.d[1] * tile.d[2]), b = (i / tile.d[2]) % tile.d[1], c = i % tile.d[2];
        const int64_t t = tile.lo[0] + a, x = tile.lo[1] + b, y = tile.lo[2] + c;
        const int64_t vo = (t * n1 + x) * n2 + y;
        const int64_t co = ((t - crop.lo[0]) * crop.d[1] + (x - crop.lo[1])) * crop.d[2] + (y - crop.lo[2]);
#pragma unroll
        for (int m = 0; m < 3; ++m) S[m * N + vo] = X[m * NC + co];
    }
}

__global__ __launch_bounds__(256) void k_fill_n(float *__restrict__ p, int n, float v)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// The tile check of k_tile_err / k_tile_copy for the tiles of a batch: workgroups
// [b * per_box, (b + 1) * per_box) serve tile b, at the origin in the predicted map given by
// its table entry; its exact maps are X[b][3][td].
__global__ __launch_bounds__(256) void k_tile_err_boxes(const float *__restrict__ S, int n0, int n1, int n2,
                                                        const float *__restrict__ X, const int *__restrict__ table,
                                                        int per_box, int3 td, const double *__restrict__ stats,
                                                        float *__restrict__ err)
{
    const int b = blockIdx.x / per_box, blk = blockIdx.x - b * per_box;
    const int *q = table + BOX_TABLE * b;
    const int nt = td.x * td.y * td.z;
    const int64_t N = (int64_t)n0 * n1 * n2;
    X += (int64_t)b * 3 * nt;
    float inv[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double r = stats[2 * m + 1] - stats[2 * m];
        inv[m] = r > 0.0 ? (float)(1.0 / r) : 0.f;
    }
    float e = 0.f;
    for (int i = blk * 256 + threadIdx.x; i < nt; i += per_box * 256) {
        const int t = q[9] + i / (td.y * td.z), x = q[10] + (i / td.z) % td.y, y = q[11] + i % td.z;
        const int64_t vo = ((int64_t)t * n1 + x) * n2 + y;
#pragma unroll
        for (int m = 0; m < 3; ++m) e = fmaxf(e, tile_diff(S[m * N + vo], X[m * nt + i], inv[m]));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) e = fmaxf(e, __shfl_xor(e, o));
    if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned int *>(err + b), __float_as_uint(e));
}

__global__ __launch_bounds__(256) void k_tile_copy_boxes(float *__restrict__ S, int n0, int n1, int n2,
                                                         const float *__restrict__ X, const int *__restrict__ table,
                                                         int per_box, int3 td, const float *__restrict__ err,
                                                         float bound)
{
    const int b = blockIdx.x / per_box, blk = blockIdx.x - b * per_box;
    if (!(err[b] > bound)) return;
    const int *q = table + BOX_TABLE * b;
    const int nt = td.x * td.y * td.z;
    const int64_t N = (int64_t)n0 * n1 * n2;
    X += (int64_t)b * 3 * nt;
    for (int i = blk * 256 + threadIdx.x; i < nt; i += per_box * 256) {
        const int t = q[9] + i / (td.y * td.z), x = q[10] + (i / td.z) % td.y, y = q[11] + i % td.z;
        const int64_t vo = ((int64_t)t * n1 + x) * n2 + y;
#pragma unroll
        for (int m = 0; m < 3; ++m) S[m * N + vo] = X[m * nt + i];
    }
}

// {min, max} of each raw map over one tile per workgroup; tiles numbered (t, x, y), y fastest.
// A NaN in a tile makes its extremes -inf and +inf, so the check of the tiles that pass the
// checked tiles' extremes always takes it.
__global__ __launch_bounds__(256) void k_tile_minmax(const float *__restrict__ S, int n0, int n1, int n2, int tile,
                                                     int ntx, int nty, float *__restrict__ out)
{
    const int ti = blockIdx.x;
    const int c = ti % nty, b = (ti / nty) % ntx, a = ti / (nty * ntx);
    const int t0 = a * tile, x0 = b * tile, y0 = c * tile;
    const int dt = min(tile, n0 - t0), dx = min(tile, n1 - x0), dy = min(tile, n2 - y0);
    const int cnt = dt * dx * dy;
    const int64_t N = (int64_t)n0 * n1 * n2;
    float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int i = threadIdx.x; i < cnt; i += 256) {
        const int y = i % dy, r = i / dy;
        const int x = r % dx, t = r / dx;
        const int64_t v = ((int64_t)(t0 + t) * n1 + (x0 + x)) * n2 + (y0 + y);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const float s = S[m * N + v];
            const bool nan = !(s == s);
            mn[m] = nan ? -__int_as_float(0x7f800000) : fminf(mn[m], s);
            mx[m] = nan ? __int_as_float(0x7f800000) : fmaxf(mx[m], s);
        }
    }
    __shared__ float red[4][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            mn[m] = fminf(mn[m], __shfl_xor(mn[m], o));
            mx[m] = fmaxf(mx[m], __shfl_xor(mx[m], o));
        }
        if (lane == 0) {
            red[wave][2 * m] = mn[m];
            red[wave][2 * m + 1] = mx[m];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float r = red[0][k];
        for (int w = 1; w < 4; ++w) r = (k & 1) ? fmaxf(r, red[w][k]) : fminf(r, red[w][k]);
        out[(int64_t)ti * 6 + k] = r;
    }
}

int64_t merge_red_blocks(int64_t N)
{
    const int64_t nb = (N + 255) / 256;
    return nb < RED_BLOCKS ? nb : RED_BLOCKS;
}

hipError_t launch_absmax_acc(const float *V, int64_t N, float *out, int accumulate, hipStream_t s)
{
    if (!accumulate) hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(1), 0, s, out, 0.f);
    if (N > 0) hipLaunchKernelGGL(k_absmax_acc, dim3((unsigned)merge_red_blocks(N)), dim3(256), 0, s, V, N, out);
    return hipGetLastError();
}

hipError_t launch_minmax_absmax(const float *V, float vmax, const float *S_raw, int64_t N,
                                float *mm_part, float *vmax_part, hipStream_t s)
{
    const unsigned nb = (unsigned)merge_red_blocks(N);
    hipLaunchKernelGGL(k_minmax3, dim3(nb), dim3(256), 0, s, S_raw, N, mm_part);
    hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(256), 0, s, V, N, vmax, vmax_part);
    return hipGetLastError();
}

hipError_t launch_tile_merge(float *S_raw, int64_t n0, int64_t n1, int64_t n2, const float *exact,
                             const int64_t crop_lo[3], const int64_t crop_dims[3], const int64_t tile_lo[3],
                             const int64_t tile_dims[3], const double *stats, double bound, float *err,
                             hipStream_t s)
{
    box3 c, t;
    for (int a = 0; a < 3; ++a) {
        c.lo[a] = crop_lo[a];
        c.d[a] = crop_dims[a];
        t.lo[a] = tile_lo[a];
        t.d[a] = tile_dims[a];
    }
    const int64_t nt = tile_dims[0] * tile_dims[1] * tile_dims[2];
    const unsigned nb = (unsigned)((nt + 255) / 256 < 1024 ? (nt + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(1), 0, s, err, 0.f);
    hipLaunchKernelGGL(k_tile_err, dim3(nb), dim3(256), 0, s, S_raw, (int)n0, (int)n1, (int)n2, exact, c, t,
                       stats, err);
    hipLaunchKernelGGL(k_tile_copy, dim3(nb), dim3(256), 0, s, S_raw, (int)n0, (int)n1, (int)n2, exact, c, t,
                       err, (float)bound);
    return hipGetLastError();
}

hipError_t launch_tile_merge_boxes(float *S_raw, int64_t n0, int64_t n1, int64_t n2, const float *exact,
                                   const int *table, int nbox, const int64_t td[3], const double *stats,
                                   double bound, float *err, hipStream_t s)
{
    const int64_t nt = td[0] * td[1] * td[2];
    const int per_box = (int)((nt + 255) / 256 < 32 ? (nt + 255) / 256 : 32);
    const int3 t3 = make_int3((int)td[0], (int)td[1], (int)td[2]);
    hipLaunchKernelGGL(k_fill_n, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, s, err, nbox, 0.f);
    hipLaunchKernelGGL(k_tile_err_boxes, dim3((unsigned)(per_box * nbox)), dim3(256), 0, s, S_raw, (int)n0, (int)n1,
                       (int)n2, exact, table, per_box, t3, stats, err);
    hipLaunchKernelGGL(k_tile_copy_boxes, dim3((unsigned)(per_box * nbox)), dim3(256), 0, s, S_raw, (int)n0,
                       (int)n1, (int)n2, exact, table, per_box, t3, err, (float)bound);
    return hipGetLastError();
}

hipError_t launch_tile_minmax(const float *S_raw, int64_t n0, int64_t n1, int64_t n2, int tile, float *out,
                              hipStream_t s)
{
    const int nt0 = (int)((n0 + tile - 1) / tile), nt1 = (int)((n1 + tile - 1) / tile),
              nt2 = (int)((n2 + tile - 1) / tile);
    hipLaunchKernelGGL(k_tile_minmax, dim3((unsigned)nt0 * nt1 * nt2), dim3(256), 0, s, S_raw, (int)n0, (int)n1,
                       (int)n2, tile, nt1, nt2, out);
    return hipGetLastError();
}
