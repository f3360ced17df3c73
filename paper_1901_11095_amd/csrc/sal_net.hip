// Learned surrogate of the saliency method: five 3x3x3 convolutions, channels
// 1 -> 24 -> 24 -> 24 -> 24 -> 3, GELU after the first four, predicting the three raw
// directional-comparison maps (S_t, S_x, S_y) of the plain method from the volume.  BF16
// weights and activations, FP32 accumulation on MFMA, FP32 master weights and Adam.
//
// Tensors are channel-last, act[b][t][u][w][c], over nb blocks of n0 x n1 x n2 voxels (a
// batch of training crops, or one whole volume).  Weights W[co][k][ci], tap k = (dt*3+du)*3+dw
// reading the input at (t+dt-1, u+du-1, w+dw-1), reflected inside the block (-1 -> 1).
//
// Training: the loss covers only voxels at least `margin` (>= 5) from every block face, so
// every nonzero gradient of a layer's output stays one voxel further inside than the
// previous one and the backward pass never meets the reflected taps: the input gradient is
// a zero-padded convolution with the flipped, transposed kernel, run by the same kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "sal_device.h"
#include "sal_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NL = 5;
constexpr int CH[NL + 1] = {1, 24, 24, 24, 24, 3};
constexpr int TT = 4, TU = 4, TW = 16;                  // output tile of a weight-gradient workgroup
constexpr int PT = TT + 2, PU = TU + 2, PW = TW + 2;    // input tile with the 1-voxel halo
constexpr int NPOS = PT * PU * PW;
// Output tile of a convolution workgroup: FT x FU x FW voxels, one wave per 4 rows of FW.
// Layers with 24 output channels take 4 x 8 x 16 (eight waves; the 6 x 10 x 18 input tile
// is 2.1 times the output instead of 2.5 times for 4 x 4 x 16), the 3-channel output layer
// keeps 4 x 4 x 16 (four waves), which measured faster there.
constexpr int FT = 4, FW = 16, FPT = FT + 2, FPW = FW + 2;
__host__ __device__ constexpr int conv_fu(int co) { return co >= 16 ? 8 : 4; }
__host__ __device__ constexpr int conv_threads(int co) { return 64 * FT * conv_fu(co) / 4; }
constexpr int WG_BLOCKS = 512;                          // workgroups of the weight-gradient pass
constexpr unsigned CONV_BLOCKS = 2048;                  // persistent workgroups of a convolution

enum { MODE_REFLECT = 0, MODE_ZERO = 1 };
enum { EPI_GELU = 0, EPI_LINEAR = 1, EPI_DGELU = 2 };

__host__ __device__ constexpr int pad8(int c) { return (c + 7) / 8 * 8; }
// K of a conv with ci input channels: taps x channels padded to 8; a single channel packs
// 27 taps into one 32-wide step
__host__ __device__ constexpr int kgroups(int ci) { return ci == 1 ? 4 : 27 * pad8(ci) / 8; }
__host__ __device__ constexpr int ksteps(int ci) { return (kgroups(ci) + 3) / 4; }

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f)
{
    const __bf16 h = (__bf16)f;
    return __builtin_bit_cast(uint16_t, h);
}

// erf by Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7), GELU(z) = z/2 (1 + erf(z/sqrt2)).
__device__ __forceinline__ void erf_as(float x, float &erfv, float &gauss)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    const float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f),
                                         -0.284496736f), 0.254829592f);
    gauss = __expf(-ax * ax);
    erfv = copysignf(1.0f - poly * gauss, x);
}
__device__ __forceinline__ float gelu_f(float z)
{
    float e, gs;
    erf_as(z * 0.70710678118654752f, e, gs);
    return 0.5f * z * (1.0f + e);
}
__device__ __forceinline__ float gelu_grad_f(float z)
{
    float e, gs;
    erf_as(z * 0.70710678118654752f, e, gs);  // gs = exp(-z^2/2)
    return 0.5f * (1.0f + e) + z * gs * 0.39894228040143268f;
}

// Storage type of activations and gradients: BF16 (the network's arithmetic) or FP32 (the
// FP32-operand mode, which runs the same kernels with FP32 operands for element-wise checks)
template <bool F32>
struct ActT {
    using type = uint16_t;
};
template <>
struct ActT<true> {
    using type = float;
};
template <bool F32>
__device__ __forceinline__ typename ActT<F32>::type to_act(float f)
{
    if constexpr (F32)
        return f;
    else
        return f2bf(f);
}
template <bool F32>
__device__ __forceinline__ float from_act(typename ActT<F32>::type a)
{
    if constexpr (F32)
        return a;
    else
        return bf2f(a);
}

// 16 bytes from global memory straight into LDS at the row base `dst` + 16 * lane
__device__ __forceinline__ void load16_to_lds(const uint16_t *src, uint16_t *dst)
{
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
}

// four consecutive channels of one voxel (16-byte aligned in FP32, 8-byte in BF16)
template <bool F32>
__device__ __forceinline__ void store4(typename ActT<F32>::type *p, const typename ActT<F32>::type r[4])
{
    if constexpr (F32)
        *reinterpret_cast<float4 *>(p) = make_float4(r[0], r[1], r[2], r[3]);
    else
        *reinterpret_cast<uint2 *>(p) = make_uint2(r[0] | ((uint32_t)r[1] << 16), r[2] | ((uint32_t)r[3] << 16));
}
// two consecutive channels of one voxel (8-byte aligned in FP32, 4-byte in BF16)
template <bool F32>
__device__ __forceinline__ void store2(typename ActT<F32>::type *p, const typename ActT<F32>::type r[2])
{
    if constexpr (F32)
        *reinterpret_cast<float2 *>(p) = make_float2(r[0], r[1]);
    else
        *reinterpret_cast<uint32_t *>(p) = r[0] | ((uint32_t)r[1] << 16);
}
template <bool F32>
__device__ __forceinline__ void load4(const typename ActT<F32>::type *p, typename ActT<F32>::type r[4])
{
    if constexpr (F32) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        r[0] = v.x;
        r[1] = v.y;
        r[2] = v.z;
        r[3] = v.w;
    } else {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        r[0] = (uint16_t)(v.x & 0xffff);
        r[1] = (uint16_t)(v.x >> 16);
        r[2] = (uint16_t)(v.y & 0xffff);
        r[3] = (uint16_t)(v.y >> 16);
    }
}

__device__ __forceinline__ int map_idx(int u, int n, int mode)
{
    if (mode == MODE_ZERO) return (u < 0 || u >= n) ? -1 : u;
    return refl_idx(u, n);
}

}  // namespace

// ------------------------------------------------------------------------------------
// 3x3x3 convolution as an implicit GEMM on 16x16x32 BF16 MFMA: D[co][voxel] =
// sum_K A[co][K] B[K][voxel], K = (tap, input channel).  A (the weights) stays in registers
// for the whole workgroup; B is read from the LDS input tile, 8 channels of one tap = 16
// bytes per lane.  Each wave computes 4 rows of 16 voxels.
//   in:   CI == 1: float [nb][n0][n1][n2]; else Act [nb][...][CI]
//   wtab: Act [MT*16][ksteps*32] (rows >= CO and K past the taps are zero)
//   EPI_GELU:   z = acc + bias -> out0 (Act, optional), GELU(z) -> out1 (Act)
//   EPI_LINEAR: (acc + bias) * oscale[c] -> out0 (float), element (v, c) at v*vstride + c*cstride
//   EPI_DGELU:  acc * GELU'(zprev) -> out0 (Act)
// Act is BF16, or FP32 with F32: the same tiles, K order and epilogues, each 16x16x32 step
// done as eight 16x16x4 FP32 MFMAs over the eight K elements a lane holds (a lane of group g
// holds K = 8g + e, e < 8, in both forms), the weights read from the table at each step,
// the tiles loaded synchronously (two FP32 buffers would not fit the LDS).
template <int CI, int CO, int MODE, int EPI, bool F32>
__global__ __launch_bounds__(conv_threads(CO)) void k_conv3(const void *__restrict__ in, int nb, int n0, int n1,
                                               int n2, const void *__restrict__ wtab,
                                               const float *__restrict__ bias,
                                               const void *__restrict__ zprev, void *out0,
                                               void *out1, int64_t vstride, int64_t cstride,
                                               float3 oscale)
{
    using Act = typename ActT<F32>::type;
    constexpr int CIP = CI == 1 ? 1 : pad8(CI);
    constexpr int KS = ksteps(CI), MT = (CO + 15) / 16;
    constexpr int FU = conv_fu(CO), FPU = FU + 2, FNPOS = FPT * FPU * FPW;
    constexpr int FWAVES = FT * FU / 4, FTHREADS = conv_threads(CO);
    // multi-channel BF16 layers with reflected borders (the forward pass) stream the next
    // tile into a second LDS buffer by direct global-to-LDS loads while the current one
    // computes
    constexpr bool ASYNC = !F32 && CI > 1 && CI % 8 == 0 && MODE == MODE_REFLECT;
    // forward BF16 layers with 24 input channels: two output rows share their input reads
    // (the weight table of these layers is laid out in the matching K order)
    constexpr bool PAIR = !F32 && CI == 24 && MODE == MODE_REFLECT;
    static_assert(!PAIR || ksteps(CI) == 21, "paired rows expect 27 taps x 3 chunks in 7 x 3 K steps");
    // two separate LDS objects, so the compiler can tell reads of one from the loads landing
    // in the other (a read of the same object would wait for them)
    __shared__ __attribute__((aligned(16))) Act tileA[FNPOS * CIP];
    __shared__ __attribute__((aligned(16))) Act tileB[ASYNC ? FNPOS * CIP : 8];
    // biases in LDS: a global load in the epilogue would wait for the tile in flight
    __shared__ float bias_s[MT * 16];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int ntw = (n2 + FW - 1) / FW, ntu = (n1 + FU - 1) / FU, ntt = (n0 + FT - 1) / FT;
    const int ntiles = nb * ntt * ntu * ntw;
    const int64_t vol = (int64_t)n0 * n1 * n2;
    const Act *act_in = reinterpret_cast<const Act *>(in);

    // asynchronous load of tile `id` into buffer `bf`: each wave takes whole rows of FPW
    // positions; lane j < FPW * CIP / 8 brings 16 bytes (8 channels) and the hardware puts
    // them at row base + 16 j, which is the row's layout in LDS
    auto issue = [&](int id, Act *dst) {
        if constexpr (ASYNC) {
            constexpr int CHK = CIP / 8, ROWLEN = FPW * CHK;
            int bi = id;
            const int tw2 = bi % ntw;
            bi /= ntw;
            const int tu2 = bi % ntu;
            bi /= ntu;
            const int tt2 = bi % ntt;
            const int b2 = bi / ntt;
            const Act *src = act_in + b2 * vol * CI;
            const int pw = lane / CHK, ch = lane - (lane / CHK) * CHK;
            const int gw = refl_idx(tw2 * FW - 1 + pw, n2);
            const int wv = __builtin_amdgcn_readfirstlane(wave);
#pragma unroll
            for (int it = 0; it < (FPT * FPU + FWAVES - 1) / FWAVES; ++it) {
                const int row = FWAVES * it + wv;
                if (row < FPT * FPU) {
                    const int pt = row / FPU, pu = row - pt * FPU;
                    const int gt = refl_idx(tt2 * FT - 1 + pt, n0), gu = refl_idx(tu2 * FU - 1 + pu, n1);
                    if (lane < ROWLEN)
                        load16_to_lds(src + (((int64_t)gt * n1 + gu) * n2 + gw) * CI + 8 * ch, &dst[row * FPW * CIP]);
                }
            }
        }
    };
    for (int i = threadIdx.x; i < MT * 16; i += FTHREADS) bias_s[i] = (bias && i < CO) ? bias[i] : 0.f;
    __syncthreads();
    if (ASYNC && (int)blockIdx.x < ntiles) issue(blockIdx.x, tileA);

    // BF16: the weights stay in registers while the workgroup walks its tiles
    u32x4 A[MT][F32 ? 1 : KS];
    if constexpr (!F32) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int s = 0; s < KS; ++s)
                A[mt][s] = reinterpret_cast<const u32x4 *>(wtab)[((mt * 16 + n) * KS * 32 + s * 32 + 8 * g) / 8];
    }

    // one tile: wait for its input, start the next tile's loads into the other buffer,
    // convolve, write the epilogue
    auto process = [&](int tile_id, Act *tile, Act *other) __attribute__((always_inline)) {
    int bid = tile_id;
    const int tw_ = bid % ntw;
    bid /= ntw;
    const int tu_ = bid % ntu;
    bid /= ntu;
    const int tt_ = bid % ntt;
    const int b = bid / ntt;
    const int t0 = tt_ * FT, u0 = tu_ * FU, w0 = tw_ * FW;
    if (ASYNC) {
        // this tile's loads have landed (every wave waits for its own, then the barrier);
        // the other buffer is free again, so the next tile's loads can start
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tile_id + (int)gridDim.x < ntiles) issue(tile_id + gridDim.x, other);
    } else {
        __syncthreads();  // the previous tile is no longer read
    }

    // input tile with halo: one row of FPW positions per (pt, pu).  Each wave loads whole
    // rows, so the row's (t, u) source index is wave-uniform and a lane's position along
    // w is fixed for the tile.
    if (CI == 1) {
        // three rows of FPW floats per wave and step
        const float *src = reinterpret_cast<const float *>(in) + b * vol;
        const int r3 = lane / FPW, pw = lane - r3 * FPW;
        const bool act = r3 < 3;
        const int gw = map_idx(w0 - 1 + pw, n2, MODE);
#pragma unroll
        for (int it = 0; it < (FPT * FPU + 3 * FWAVES - 1) / (3 * FWAVES); ++it) {
            const int row = 3 * FWAVES * it + 3 * wave + r3;
            if (act && row < FPT * FPU) {
                const int pt = row / FPU, pu = row - pt * FPU;
                const int gt = map_idx(t0 - 1 + pt, n0, MODE), gu = map_idx(u0 - 1 + pu, n1, MODE);
                const float v = (gt < 0 || gu < 0 || gw < 0) ? 0.f : src[((int64_t)gt * n1 + gu) * n2 + gw];
                tile[row * FPW + pw] = to_act<F32>(v);
            }
        }
    } else if (ASYNC) {
        // loaded by issue()
    } else if (CI % 8 == 0) {
        // chunks of 8 channels (16 bytes in BF16, two 16-byte halves in FP32); a row of FPW
        // positions is ROWLEN <= 64 chunks
        constexpr int CHK = CIP / 8, ROWLEN = FPW * CHK, NQ = F32 ? 2 : 1;
        static_assert(ROWLEN <= 64, "one wave loads a whole row");
        const Act *src = act_in + b * vol * CI;
        const bool act = lane < ROWLEN;
        const int pw = lane / CHK, ch = lane - (lane / CHK) * CHK;
        const int gw = map_idx(w0 - 1 + pw, n2, MODE);
        const int wv = __builtin_amdgcn_readfirstlane(wave);
#pragma unroll
        for (int it = 0; it < (FPT * FPU + FWAVES - 1) / FWAVES; ++it) {
            const int row = FWAVES * it + wv;
            if (row < FPT * FPU) {
                const int pt = row / FPU, pu = row - pt * FPU;
                const int gt = map_idx(t0 - 1 + pt, n0, MODE), gu = map_idx(u0 - 1 + pu, n1, MODE);
                u32x4 val[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) val[q] = u32x4{0u, 0u, 0u, 0u};
                if (act && gt >= 0 && gu >= 0 && gw >= 0) {
                    const u32x4 *p = reinterpret_cast<const u32x4 *>(src + (((int64_t)gt * n1 + gu) * n2 + gw) * CI + 8 * ch);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) val[q] = p[q];
                }
                if (act) {
                    u32x4 *d = reinterpret_cast<u32x4 *>(&tile[(row * FPW + pw) * CIP + 8 * ch]);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) d[q] = val[q];
                }
            }
        }
    } else {
        const Act *src = act_in + b * vol * CI;
        for (int i = threadIdx.x; i < FNPOS * CIP; i += FTHREADS) {
            const int p = i / CIP, c = i - p * CIP;
            const int row = p / FPW, pw = p - row * FPW;
            const int pt = row / FPU, pu = row - pt * FPU;
            const int gt = map_idx(t0 - 1 + pt, n0, MODE), gu = map_idx(u0 - 1 + pu, n1, MODE),
                      gw = map_idx(w0 - 1 + pw, n2, MODE);
            tile[i] = (c >= CI || gt < 0 || gu < 0 || gw < 0) ? (Act)0 : src[(((int64_t)gt * n1 + gu) * n2 + gw) * CI + c];
        }
    }
    // (asynchronous tiles were complete at the barrier above; a barrier here would wait for
    // the next tile's loads)
    if (!ASYNC) __syncthreads();

    // epilogue of one row of 16 output voxels (lt, lu, n) of the tile
    auto epilogue = [&](f4(&acc)[MT], int lt, int lu) __attribute__((always_inline)) {
        // epilogue: lane (g, n) holds channels 16mt + 4g + j of voxel n.  With 24 output
        // channels the last M tile holds 8, all in lane groups 0 and 1: its channels +2 and +3
        // move to lane groups 2 and 3 (one lane swap per pair, done by every lane), so each lane
        // evaluates two GELUs there instead of half the lanes evaluating four.
        constexpr bool SPREAD = EPI == EPI_GELU && CO % 16 == 8;
        float sp[2] = {0.f, 0.f};
        if constexpr (SPREAD) {
            const auto s0 = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[MT - 1][0]),
                                                             __float_as_uint(acc[MT - 1][2]), false, false);
            const auto s1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[MT - 1][1]),
                                                             __float_as_uint(acc[MT - 1][3]), false, false);
            sp[0] = __uint_as_float(s0[0]);
            sp[1] = __uint_as_float(s1[0]);
        }
        const int gt = t0 + lt, gu = u0 + lu, gw = w0 + n;
        if (gt < n0 && gu < n1 && gw < n2) {
            const int64_t v = b * vol + ((int64_t)gt * n1 + gu) * n2 + gw;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int cb = 16 * mt + 4 * g;
                if (SPREAD && mt == MT - 1) {
                    // channels c2, c2 + 1 of this voxel
                    const int c2 = 16 * mt + 4 * (g & 1) + 2 * (g >> 1);
                    Act zz[2], r[2];
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        zz[j] = to_act<F32>(sp[j] + bias_s[c2 + j]);
                        r[j] = to_act<F32>(gelu_f(from_act<F32>(zz[j])));
                    }
                    if (out0) store2<F32>(reinterpret_cast<Act *>(out0) + v * CO + c2, zz);
                    store2<F32>(reinterpret_cast<Act *>(out1) + v * CO + c2, r);
                } else if (EPI == EPI_LINEAR) {
                    float *o = reinterpret_cast<float *>(out0);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (cb + j < CO) {
                            const float sc = cb + j == 0 ? oscale.x : (cb + j == 1 ? oscale.y : oscale.z);
                            o[v * vstride + (cb + j) * cstride] = (acc[mt][j] + bias_s[cb + j]) * sc;
                        }
                } else if (cb < CO) {  // CO is a multiple of 4 here
                    Act r[4];
                    if (EPI == EPI_GELU) {
                        Act zz[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float z = acc[mt][j] + bias_s[cb + j];
                            zz[j] = to_act<F32>(z);
                            r[j] = to_act<F32>(gelu_f(from_act<F32>(zz[j])));
                        }
                        if (out0) store4<F32>(reinterpret_cast<Act *>(out0) + v * CO + cb, zz);
                        store4<F32>(reinterpret_cast<Act *>(out1) + v * CO + cb, r);
                    } else {
                        Act zv[4];
                        load4<F32>(reinterpret_cast<const Act *>(zprev) + v * CO + cb, zv);
#pragma unroll
                        for (int j = 0; j < 4; ++j) r[j] = to_act<F32>(acc[mt][j] * gelu_grad_f(from_act<F32>(zv[j])));
                        store4<F32>(reinterpret_cast<Act *>(out0) + v * CO + cb, r);
                    }
                }
            }
        }
    };

    if constexpr (PAIR) {
        // Two rows (lu, lu + 1) at a time: for each (dt, dw, channel chunk) a lane reads the
        // four input rows lu .. lu + 3 once, and the three K steps du = 0, 1, 2 use rows du and
        // du + 1 for the two output rows (4 LDS reads for 12 MFMAs instead of 6; four
        // independent accumulator chains).  K slot (3 sg + du, g) of the weight table holds
        // tap (dt, du, dw) and chunk ch of tc = 4 sg + g = (dt * 3 + dw) * 3 + ch.
#pragma unroll 1
        for (int rp = 0; rp < 2; ++rp) {
            const int lt = wave % FT, lu = (wave / FT) * 4 + 2 * rp;
            f4 acc0[MT], acc1[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc0[mt] = acc1[mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int sg = 0; sg < KS / 3; ++sg) {
                const int tc = 4 * sg + g;
                u32x4 P[4];
                if (tc < 27) {
                    const int dt = tc / 9, dw = (tc / 3) % 3, ch = tc % 3;
                    const Act *src = &tile[(((lt + dt) * FPU + lu) * FPW + n + dw) * CIP + 8 * ch];
#pragma unroll
                    for (int i = 0; i < 4; ++i) P[i] = *reinterpret_cast<const u32x4 *>(src + i * FPW * CIP);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) P[i] = u32x4{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (int du = 0; du < 3; ++du) {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        acc0[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A[mt][3 * sg + du]),
                                                                           __builtin_bit_cast(bf16x8, P[du]), acc0[mt], 0, 0, 0);
                        acc1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A[mt][3 * sg + du]),
                                                                           __builtin_bit_cast(bf16x8, P[du + 1]), acc1[mt], 0, 0, 0);
                    }
                }
            }
            epilogue(acc0, lt, lu);
            epilogue(acc1, lt, lu + 1);
        }
    } else {
#pragma unroll 1
    for (int row = 0; row < 4; ++row) {
        const int lt = wave % FT, lu = (wave / FT) * 4 + row;  // output voxel (lt, lu, n) of the tile
        f4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if constexpr (F32) {
                // the eight K elements of this lane, K = 32 s + 8 g + e, as FP32
                float bk[8];
                if (CI == 1) {
                    // K element e of group g is tap 8g + e
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int k = 8 * g + e;
                        bk[e] = 0.f;
                        if (k < 27) bk[e] = tile[((lt + k / 9) * FPU + (lu + (k / 3) % 3)) * FPW + n + k % 3];
                    }
                } else {
                    const int q = 4 * s + g;  // K group: tap q / (CIP/8), channels 8*(q % (CIP/8))
#pragma unroll
                    for (int e = 0; e < 8; ++e) bk[e] = 0.f;
                    if (q < kgroups(CI)) {
                        const int k = q / (CIP / 8), c0 = 8 * (q % (CIP / 8));
                        const int p = ((lt + k / 9) * FPU + (lu + (k / 3) % 3)) * FPW + n + k % 3;
                        const float4 *src4 = reinterpret_cast<const float4 *>(&tile[p * CIP + c0]);
                        const float4 lo = src4[0], hi = src4[1];
                        bk[0] = lo.x; bk[1] = lo.y; bk[2] = lo.z; bk[3] = lo.w;
                        bk[4] = hi.x; bk[5] = hi.y; bk[6] = hi.z; bk[7] = hi.w;
                    }
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const float *wr = reinterpret_cast<const float *>(wtab) + (mt * 16 + n) * KS * 32 + s * 32 + 8 * g;
#pragma unroll
                    for (int e = 0; e < 8; ++e) acc[mt] = mfma4(wr[e], bk[e], acc[mt]);
                }
            } else {
                u32x4 bv;
                if (CI == 1) {
                    // K element e of group g is tap 8g + e
#pragma unroll
                    for (int e2 = 0; e2 < 4; ++e2) {
                        uint32_t pr = 0;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int k = 8 * g + 2 * e2 + h;
                            uint32_t val = 0;
                            if (k < 27) {
                                const int p = ((lt + k / 9) * FPU + (lu + (k / 3) % 3)) * FPW + n + k % 3;
                                val = tile[p];
                            }
                            pr |= val << (16 * h);
                        }
                        bv[e2] = pr;
                    }
                } else {
                    const int q = 4 * s + g;  // K group: tap q / (CIP/8), channels 8*(q % (CIP/8))
                    if (q < kgroups(CI)) {
                        const int k = q / (CIP / 8), c0 = 8 * (q % (CIP / 8));
                        const int p = ((lt + k / 9) * FPU + (lu + (k / 3) % 3)) * FPW + n + k % 3;
                        bv = *reinterpret_cast<const u32x4 *>(&tile[p * CIP + c0]);
                    } else {
                        bv = u32x4{0u, 0u, 0u, 0u};
                    }
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A[mt][s]),
                                                                      __builtin_bit_cast(bf16x8, bv), acc[mt], 0,
                                                                      0, 0);
            }
        }
        epilogue(acc, lt, lu);
    }
    }
    };

    if constexpr (ASYNC) {
        // even steps read tileA and fill tileB, odd steps the other way round
        for (int tile_id = blockIdx.x; tile_id < ntiles;) {
            process(tile_id, tileA, tileB);
            tile_id += gridDim.x;
            if (tile_id >= ntiles) break;
            process(tile_id, tileB, tileA);
            tile_id += gridDim.x;
        }
    } else {
#pragma unroll 1
        for (int tile_id = blockIdx.x; tile_id < ntiles; tile_id += gridDim.x) process(tile_id, tileA, tileB);
    }

}

// ------------------------------------------------------------------------------------
// Weight and bias gradient of one layer: dW[co][k][ci] = sum_v dz[v][co] in[refl(v+k-1)][ci],
// db[co] = sum_v dz[v][co].  FP32 16x16x4 MFMA with M = co, N = ci, K = 4 voxels; wave w
// owns taps w, w+8, w+16, w+24.  Each workgroup walks a fixed stride of tiles and writes
// its own partial sums (summed afterwards in a fixed order: deterministic).
template <int CI, int CO, bool F32>
__global__ __launch_bounds__(512) void k_conv3_wgrad(const void *__restrict__ in,
                                                     const void *__restrict__ dz_, int nb, int n0,
                                                     int n1, int n2, float *__restrict__ part)
{
    using Act = typename ActT<F32>::type;
    const Act *dz = reinterpret_cast<const Act *>(dz_);
    constexpr int MT = (CO + 15) / 16, NT = (CI + 15) / 16, NKW = 4;
    constexpr int NPAR = CO * 27 * CI + CO;
    __shared__ float tin[NPOS * CI];
    __shared__ float tdz[TT * TU * TW * CO];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int ntw = (n2 + TW - 1) / TW, ntu = (n1 + TU - 1) / TU, ntt = (n0 + TT - 1) / TT;
    const int ntiles = nb * ntt * ntu * ntw;
    const int64_t vol = (int64_t)n0 * n1 * n2;

    f4 acc[NKW][MT][NT];
#pragma unroll
    for (int a = 0; a < NKW; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[a][mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int bid = tile;
        const int tw_ = bid % ntw;
        bid /= ntw;
        const int tu_ = bid % ntu;
        bid /= ntu;
        const int tt_ = bid % ntt;
        const int b = bid / ntt;
        const int t0 = tt_ * TT, u0 = tu_ * TU, w0 = tw_ * TW;
        __syncthreads();
        for (int i = threadIdx.x; i < NPOS * CI; i += 512) {
            const int p = i / CI, c = i - p * CI;
            const int pt = p / (PU * PW), pu = (p / PW) % PU, pw = p % PW;
            const int64_t gi = b * vol + ((int64_t)refl_idx(t0 - 1 + pt, n0) * n1 + refl_idx(u0 - 1 + pu, n1)) * n2 +
                               refl_idx(w0 - 1 + pw, n2);
            tin[i] = CI == 1 ? reinterpret_cast<const float *>(in)[gi]
                             : from_act<F32>(reinterpret_cast<const Act *>(in)[gi * CI + c]);
        }
        for (int i = threadIdx.x; i < TT * TU * TW * CO; i += 512) {
            const int vv = i / CO, c = i - vv * CO;
            const int gt = t0 + vv / (TU * TW), gu = u0 + (vv / TW) % TU, gw = w0 + vv % TW;
            tdz[i] = (gt < n0 && gu < n1 && gw < n2)
                         ? from_act<F32>(dz[(b * vol + ((int64_t)gt * n1 + gu) * n2 + gw) * CO + c])
                         : 0.f;
        }
        __syncthreads();
        if (threadIdx.x < CO)
            for (int vv = 0; vv < TT * TU * TW; ++vv) dbias += tdz[vv * CO + threadIdx.x];
#pragma unroll 1
        for (int v4 = 0; v4 < TT * TU * TW; v4 += 4) {
            const int vv = v4 + g;  // this lane group's voxel
            const int lt = vv / (TU * TW), lu = (vv / TW) % TU, lw = vv % TW;
            float av[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) av[mt] = (16 * mt + n < CO) ? tdz[vv * CO + 16 * mt + n] : 0.f;
#pragma unroll
            for (int a = 0; a < NKW; ++a) {
                const int k = wave + 8 * a;
                if (k < 27) {
                    const int p = ((lt + k / 9) * PU + (lu + (k / 3) % 3)) * PW + lw + k % 3;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const float bv = (16 * nt + n < CI) ? tin[p * CI + 16 * nt + n] : 0.f;
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
                            acc[a][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt], bv, acc[a][mt][nt], 0, 0, 0);
                    }
                }
            }
        }
    }
    float *pp = part + (int64_t)blockIdx.x * NPAR;
#pragma unroll
    for (int a = 0; a < NKW; ++a) {
        const int k = wave + 8 * a;
        if (k >= 27) continue;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int co = 16 * mt + 4 * g + j, ci = 16 * nt + n;
                    if (co < CO && ci < CI) pp[(co * 27 + k) * CI + ci] = acc[a][mt][nt][j];
                }
    }
    if (threadIdx.x < CO) pp[CO * 27 * CI + threadIdx.x] = dbias;
}

// grad[j] += sum over partials (fixed order)
__global__ __launch_bounds__(256) void k_sum_partials(const float *__restrict__ part, int nparts,
                                                      int npar, float *__restrict__ grad)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= npar) return;
    float s = 0.f;
    for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * npar + j];
    grad[j] += s;
}

// Masked mean squared error: dY = 2 (Y - T) / count on voxels at least `margin` from every
// face of their block (0 elsewhere), as bf16 [..][3]; loss partial sums per workgroup.
template <bool F32>
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ Y, const float *__restrict__ T,
                                             int nb, int S, int margin, float inv_count,
                                             typename ActT<F32>::type *__restrict__ dY, float *__restrict__ loss_part)
{
    const int64_t tot = (int64_t)nb * S * S * S;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (i < tot) {
        const int w = (int)(i % S), u = (int)((i / S) % S), t = (int)((i / ((int64_t)S * S)) % S);
        const bool in = t >= margin && t < S - margin && u >= margin && u < S - margin && w >= margin &&
                        w < S - margin;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = in ? Y[i * 3 + c] - T[i * 3 + c] : 0.f;
            l += d * d;
            dY[i * 3 + c] = to_act<F32>(2.f * d * inv_count);
        }
    }
    __shared__ float red[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * inv_count;
}

__global__ __launch_bounds__(256) void k_sum_loss(const float *__restrict__ part, int n, float *__restrict__ loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0];
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// Adam on the FP32 master parameters (bias-corrected), then clear the gradient.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, float *__restrict__ gr,
                                              float *__restrict__ m, float *__restrict__ v, int n,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gg = gr[i];
    const float mm = b1 * m[i] + (1.f - b1) * gg;
    const float vv = b2 * v[i] + (1.f - b2) * gg * gg;
    m[i] = mm;
    v[i] = vv;
    p[i] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    gr[i] = 0.f;
}

// Operand tables of one layer from the FP32 master, in BF16 and in FP32 (the FP32-operand
// mode): forward [rows][ksteps*32] and the flipped/transposed kernel of the input-gradient
// conv.
__global__ __launch_bounds__(256) void k_prep_tables(const float *__restrict__ W, int ci, int co,
                                                     uint16_t *__restrict__ fwd, float *__restrict__ fwd32,
                                                     int fwd_rows, int fwd_k, uint16_t *__restrict__ bwd,
                                                     float *__restrict__ bwd32, int bwd_rows, int bwd_k)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    // forward: row co, K index = tap * pad8(ci) + c (ci > 1) or tap (ci == 1).  The BF16 table
    // of the 24-channel layers is in the paired-row order of k_conv3: K index 32 s + 8 g + e
    // holds tap (dt, du, dw) and channel 8 ch + e, with s = 3 sg + du and 4 sg + g =
    // (dt * 3 + dw) * 3 + ch (zero past the 27 taps x 3 chunks).
    if (i < fwd_rows * fwd_k) {
        const int r = i / fwd_k, kk = i % fwd_k;
        float w = 0.f, wp = 0.f;
        if (r < co) {
            if (ci == 1) {
                if (kk < 27) w = W[(r * 27 + kk) * ci];
                wp = w;
            } else {
                const int cp = pad8(ci), k = kk / cp, c = kk % cp;
                if (k < 27 && c < ci) w = W[(r * 27 + k) * ci + c];
                wp = w;
                if (ci == 24) {
                    const int st = kk / 32, gg = (kk / 8) % 4, e = kk % 8;
                    const int tc = 4 * (st / 3) + gg, du = st % 3;
                    wp = 0.f;
                    if (tc < 27) {
                        const int dt = tc / 9, dw = (tc / 3) % 3, ch = tc % 3;
                        wp = W[(r * 27 + (dt * 3 + du) * 3 + dw) * ci + 8 * ch + e];
                    }
                }
            }
        }
        fwd[i] = f2bf(wp);
        fwd32[i] = w;
    }
    // backward (input gradient): row = input channel c, K = tap' * pad8(co) + o, weight
    // W[o][26 - tap'][c]
    if (bwd && i < bwd_rows * bwd_k) {
        const int r = i / bwd_k, kk = i % bwd_k;
        const int cp = pad8(co), k = kk / cp, o = kk % cp;
        float w = 0.f;
        if (r < ci && k < 27 && o < co) w = W[(o * 27 + (26 - k)) * ci + r];
        bwd[i] = f2bf(w);
        bwd32[i] = w;
    }
}

// ====================================================================== host side

struct sal_net {
    int device;
    std::vector<int64_t> woff, boff;  // offsets of W and bias of each layer in the flat vector
    int64_t npar;
    float *p, *gr, *m, *v;            // FP32 master, gradient, Adam moments
    uint16_t *fwd[NL], *bwd[NL];      // BF16 operand tables
    float *fwd32[NL], *bwd32[NL];     // FP32 operand tables (FP32-operand mode)
    bool f32 = false;                 // operands and activations in FP32 instead of BF16
    int64_t step;
    float out_scale[3];               // inference output = network output * out_scale
    std::string err;
};

namespace {

thread_local std::string g_net_err;

sal_status nfail(sal_net *n, sal_status s, const std::string &m)
{
    if (n)
        n->err = m;
    else
        g_net_err = m;
    return s;
}

int fwd_rows(int l) { return (CH[l + 1] + 15) / 16 * 16; }
int fwd_k(int l) { return ksteps(CH[l]) * 32; }
int bwd_rows(int l) { return (CH[l] + 15) / 16 * 16; }
int bwd_k(int l) { return ksteps(CH[l + 1]) * 32; }

hipError_t prep_tables(sal_net *n, hipStream_t s)
{
    for (int l = 0; l < NL; ++l) {
        const int nf = fwd_rows(l) * fwd_k(l), nbk = l > 0 ? bwd_rows(l) * bwd_k(l) : 0;
        const int tot = nf > nbk ? nf : nbk;
        hipLaunchKernelGGL(k_prep_tables, dim3((tot + 255) / 256), dim3(256), 0, s, n->p + n->woff[l],
                           CH[l], CH[l + 1], n->fwd[l], n->fwd32[l], fwd_rows(l), fwd_k(l),
                           l > 0 ? n->bwd[l] : nullptr, l > 0 ? n->bwd32[l] : nullptr, bwd_rows(l), bwd_k(l));
    }
    return hipGetLastError();
}

int64_t nvox_of(int64_t nb, int64_t n0, int64_t n1, int64_t n2) { return nb * n0 * n1 * n2; }
unsigned conv_grid(int64_t nb, int64_t n0, int64_t n1, int64_t n2)
{
    return (unsigned)(nb * ((n0 + TT - 1) / TT) * ((n1 + TU - 1) / TU) * ((n2 + TW - 1) / TW));
}
unsigned conv_tiles_fwd(int co, int64_t nb, int64_t n0, int64_t n1, int64_t n2)
{
    const int fu = conv_fu(co);
    return (unsigned)(nb * ((n0 + FT - 1) / FT) * ((n1 + fu - 1) / fu) * ((n2 + FW - 1) / FW));
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Training workspace: z1..z4, a1..a4 (24 ch), Y (f32, 3 ch), dY (3 ch), two gradient buffers
// (24 ch), weight-gradient partials, loss partials; activations and gradients take `es`
// bytes per value (2: BF16, 4: the FP32-operand mode).
struct TrainWs {
    size_t z[4], a[4], y, dy, g0, g1, part, lossp, total;
};
TrainWs train_ws(int64_t nv, size_t es)
{
    TrainWs w;
    size_t o = 0;
    for (int l = 0; l < 4; ++l) {
        w.z[l] = o;
        o += al(nv * 24 * es);
        w.a[l] = o;
        o += al(nv * 24 * es);
    }
    w.y = o;
    o += al(nv * 3 * 4);
    w.dy = o;
    o += al(nv * 3 * es);
    w.g0 = o;
    o += al(nv * 24 * es);
    w.g1 = o;
    o += al(nv * 24 * es);
    w.part = o;
    o += al((size_t)WG_BLOCKS * (24 * 27 * 24 + 24) * 4);
    w.lossp = o;
    o += al(((nv + 255) / 256) * 4);
    w.total = o;
    return w;
}
size_t act_bytes(const sal_net *n) { return n->f32 ? 4 : 2; }
// inference workspace: two ping-pong activation buffers of 24 channels
size_t infer_ws(const sal_net *n, int64_t nv) { return 2 * al(nv * 24 * act_bytes(n)); }

template <int CI, int CO, int MODE, int EPI, bool F32>
void conv(const void *in, int64_t nb, int64_t n0, int64_t n1, int64_t n2, const void *w,
          const float *bias, const void *zprev, void *o0, void *o1, int64_t vs, int64_t cs,
          hipStream_t s, float3 oscale = make_float3(1.f, 1.f, 1.f))
{
    // persistent workgroups: a few per CU, each walking tiles with its weights in registers
    const unsigned tiles = conv_tiles_fwd(CO, nb, n0, n1, n2);
    const unsigned grid = tiles < CONV_BLOCKS ? tiles : CONV_BLOCKS;
    hipLaunchKernelGGL((k_conv3<CI, CO, MODE, EPI, F32>), dim3(grid), dim3(conv_threads(CO)), 0, s,
                       in, (int)nb, (int)n0, (int)n1, (int)n2, w, bias, zprev, o0, o1, vs, cs, oscale);
}

// forward through all layers; stores z/a (training) or ping-pongs (inference)
template <bool F32>
hipError_t net_forward_t(sal_net *n, const float *X, int64_t nb, int64_t n0, int64_t n1, int64_t n2,
                         char *ws, const TrainWs *tw, float *Y, int64_t vs, int64_t cs, float3 oscale,
                         hipStream_t s)
{
    using Act = typename ActT<F32>::type;
    const float *b[NL];
    const void *w[NL];
    for (int l = 0; l < NL; ++l) {
        b[l] = n->p + n->boff[l];
        w[l] = F32 ? (const void *)n->fwd32[l] : (const void *)n->fwd[l];
    }
    Act *z[4], *a[4];
    for (int l = 0; l < 4; ++l) {
        z[l] = tw ? (Act *)(ws + tw->z[l]) : nullptr;
        a[l] = (Act *)(ws + (tw ? tw->a[l] : (l % 2) * al(nvox_of(nb, n0, n1, n2) * 24 * sizeof(Act))));
    }
    conv<1, 24, MODE_REFLECT, EPI_GELU, F32>(X, nb, n0, n1, n2, w[0], b[0], nullptr, z[0], a[0], 0, 0, s);
    for (int l = 1; l < 4; ++l)
        conv<24, 24, MODE_REFLECT, EPI_GELU, F32>(a[l - 1], nb, n0, n1, n2, w[l], b[l], nullptr, z[l], a[l], 0, 0, s);
    conv<24, 3, MODE_REFLECT, EPI_LINEAR, F32>(a[3], nb, n0, n1, n2, w[4], b[4], nullptr, Y, nullptr, vs, cs, s,
                                               oscale);
    return hipGetLastError();
}
hipError_t net_forward(sal_net *n, const float *X, int64_t nb, int64_t n0, int64_t n1, int64_t n2, char *ws,
                       const TrainWs *tw, float *Y, int64_t vs, int64_t cs, float3 oscale, hipStream_t s)
{
    return n->f32 ? net_forward_t<true>(n, X, nb, n0, n1, n2, ws, tw, Y, vs, cs, oscale, s)
                  : net_forward_t<false>(n, X, nb, n0, n1, n2, ws, tw, Y, vs, cs, oscale, s);
}

template <int CI, int CO, bool F32>
void wgrad(sal_net *n, int l, const void *in, const void *dz, int64_t nb, int64_t n0, int64_t n1, int64_t n2,
           float *part, hipStream_t s)
{
    const int64_t tiles = conv_grid(nb, n0, n1, n2);
    const int grid = (int)(tiles < WG_BLOCKS ? tiles : WG_BLOCKS);
    hipLaunchKernelGGL((k_conv3_wgrad<CI, CO, F32>), dim3(grid), dim3(512), 0, s, in, dz, (int)nb, (int)n0,
                       (int)n1, (int)n2, part);
    const int npar = CO * 27 * CI + CO;
    hipLaunchKernelGGL(k_sum_partials, dim3((npar + 255) / 256), dim3(256), 0, s, part, grid, npar,
                       n->gr + n->woff[l]);
}

// backward from dY ([..][3] in the activation type) through all layers, accumulating the
// gradient
template <bool F32>
hipError_t net_backward_t(sal_net *n, const float *X, const void *dY, int64_t nb, int64_t n0, int64_t n1,
                          int64_t n2, char *ws, const TrainWs &tw, hipStream_t s)
{
    using Act = typename ActT<F32>::type;
    Act *z[4], *a[4];
    for (int l = 0; l < 4; ++l) {
        z[l] = (Act *)(ws + tw.z[l]);
        a[l] = (Act *)(ws + tw.a[l]);
    }
    const void *wb[NL];
    for (int l = 1; l < NL; ++l) wb[l] = F32 ? (const void *)n->bwd32[l] : (const void *)n->bwd[l];
    Act *gbuf[2] = {(Act *)(ws + tw.g0), (Act *)(ws + tw.g1)};
    float *part = (float *)(ws + tw.part);
    // layer 5 (index 4): dW from a4 and dY; input gradient -> dz4 = (W5^T * dY) . GELU'(z4)
    wgrad<24, 3, F32>(n, 4, a[3], dY, nb, n0, n1, n2, part, s);
    conv<3, 24, MODE_ZERO, EPI_DGELU, F32>(dY, nb, n0, n1, n2, wb[4], nullptr, z[3], gbuf[0], nullptr, 0, 0, s);
    const Act *dz = gbuf[0];
    for (int l = 3; l >= 1; --l) {
        wgrad<24, 24, F32>(n, l, a[l - 1], dz, nb, n0, n1, n2, part, s);
        Act *dst = gbuf[(4 - l) % 2];
        conv<24, 24, MODE_ZERO, EPI_DGELU, F32>(dz, nb, n0, n1, n2, wb[l], nullptr, z[l - 1], dst, nullptr, 0, 0, s);
        dz = dst;
    }
    wgrad<1, 24, F32>(n, 0, X, dz, nb, n0, n1, n2, part, s);
    return hipGetLastError();
}
hipError_t net_backward(sal_net *n, const float *X, const void *dY, int64_t nb, int64_t n0, int64_t n1,
                        int64_t n2, char *ws, const TrainWs &tw, hipStream_t s)
{
    return n->f32 ? net_backward_t<true>(n, X, dY, nb, n0, n1, n2, ws, tw, s)
                  : net_backward_t<false>(n, X, dY, nb, n0, n1, n2, ws, tw, s);
}

// One Adam step on the accumulated gradient (which it clears), then the operand tables.
hipError_t adam_step(sal_net *n, float lr, hipStream_t s)
{
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f / (1.0f - std::pow(b1, (float)n->step)), c2 = 1.0f / (1.0f - std::pow(b2, (float)n->step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n->npar + 255) / 256)), dim3(256), 0, s, n->p, n->gr, n->m, n->v,
                       (int)n->npar, lr, b1, b2, 1e-8f, c1, c2);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = prep_tables(n, s);
    return e;
}

struct NetDev {
    int prev = -1;
    explicit NetDev(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(d);
    }
    ~NetDev()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

int64_t sal_net_num_params(void)
{
    int64_t t = 0;
    for (int l = 0; l < NL; ++l) t += (int64_t)CH[l + 1] * 27 * CH[l] + CH[l + 1];
    return t;
}

const char *sal_net_last_error(const sal_net *n) { return n ? n->err.c_str() : g_net_err.c_str(); }

sal_status sal_net_create(int device, uint64_t seed, sal_net **out)
{
    if (!out) return nfail(nullptr, SAL_E_INVAL, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return nfail(nullptr, SAL_E_DEVICE, "no such HIP device");
    NetDev nd(device);
    sal_net *n = new (std::nothrow) sal_net();
    if (!n) return nfail(nullptr, SAL_E_DEVICE, "out of host memory");
    n->device = device;
    n->step = 0;
    n->out_scale[0] = n->out_scale[1] = n->out_scale[2] = 1.f;
    n->p = n->gr = n->m = n->v = nullptr;
    for (int l = 0; l < NL; ++l) {
        n->fwd[l] = n->bwd[l] = nullptr;
        n->fwd32[l] = n->bwd32[l] = nullptr;
    }
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        n->woff.push_back(o);
        o += (int64_t)CH[l + 1] * 27 * CH[l];
        n->boff.push_back(o);
        o += CH[l + 1];
    }
    n->npar = o;
    // Kaiming-uniform weights (bound sqrt(6 / fan_in)), zero biases, from a seeded PCG-free
    // 64-bit Mersenne twister so the initial state depends only on the seed
    std::vector<float> h((size_t)o, 0.f);
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> uni(-1.0, 1.0);
    for (int l = 0; l < NL; ++l) {
        const double bound = std::sqrt(6.0 / (27.0 * CH[l])) * (l == NL - 1 ? 0.5 : 1.0);
        for (int64_t i = 0; i < (int64_t)CH[l + 1] * 27 * CH[l]; ++i) h[n->woff[l] + i] = (float)(bound * uni(rng));
    }
    hipError_t e = hipSuccess;
    float **bufs[4] = {&n->p, &n->gr, &n->m, &n->v};
    for (float **b : bufs) {
        if (e == hipSuccess) e = hipMalloc((void **)b, sizeof(float) * o);
        if (e == hipSuccess) e = hipMemset(*b, 0, sizeof(float) * o);
    }
    if (e == hipSuccess) e = hipMemcpy(n->p, h.data(), sizeof(float) * o, hipMemcpyHostToDevice);
    for (int l = 0; l < NL && e == hipSuccess; ++l) {
        e = hipMalloc((void **)&n->fwd[l], 2 * (size_t)fwd_rows(l) * fwd_k(l));
        if (e == hipSuccess) e = hipMalloc((void **)&n->fwd32[l], 4 * (size_t)fwd_rows(l) * fwd_k(l));
        if (e == hipSuccess && l > 0) e = hipMalloc((void **)&n->bwd[l], 2 * (size_t)bwd_rows(l) * bwd_k(l));
        if (e == hipSuccess && l > 0) e = hipMalloc((void **)&n->bwd32[l], 4 * (size_t)bwd_rows(l) * bwd_k(l));
    }
    if (e == hipSuccess) e = prep_tables(n, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        sal_net_destroy(n);
        return nfail(nullptr, SAL_E_DEVICE, std::string("net create: ") + hipGetErrorString(e));
    }
    *out = n;
    return SAL_OK;
}

void sal_net_destroy(sal_net *n)
{
    if (!n) return;
    NetDev nd(n->device);
    float *fb[] = {n->p, n->gr, n->m, n->v};
    for (float *b : fb)
        if (b) (void)hipFree(b);
    for (int l = 0; l < NL; ++l) {
        if (n->fwd[l]) (void)hipFree(n->fwd[l]);
        if (n->bwd[l]) (void)hipFree(n->bwd[l]);
        if (n->fwd32[l]) (void)hipFree(n->fwd32[l]);
        if (n->bwd32[l]) (void)hipFree(n->bwd32[l]);
    }
    delete n;
}

sal_status sal_net_set_precision(sal_net *n, int32_t precision)
{
    if (!n) return nfail(n, SAL_E_INVAL, "null argument");
    if (precision != SAL_BF16 && precision != SAL_FP32)
        return nfail(n, SAL_E_INVAL, "the network runs in SAL_BF16 or SAL_FP32");
    n->f32 = precision == SAL_FP32;
    return SAL_OK;
}

sal_status sal_net_params(sal_net *n, float *host, int64_t count, int write)
{
    if (!n || !host) return nfail(n, SAL_E_INVAL, "null argument");
    if (count != n->npar) return nfail(n, SAL_E_INVAL, "parameter count mismatch");
    NetDev nd(n->device);
    hipError_t e;
    if (write) {
        e = hipMemcpy(n->p, host, sizeof(float) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = prep_tables(n, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
    } else {
        e = hipMemcpy(host, n->p, sizeof(float) * count, hipMemcpyDeviceToHost);
    }
    return e == hipSuccess ? SAL_OK : nfail(n, SAL_E_DEVICE, hipGetErrorString(e));
}

sal_status sal_net_grads(sal_net *n, float *host, int64_t count, int zero)
{
    if (!n || !host) return nfail(n, SAL_E_INVAL, "null argument");
    if (count != n->npar) return nfail(n, SAL_E_INVAL, "parameter count mismatch");
    NetDev nd(n->device);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host, n->gr, sizeof(float) * count, hipMemcpyDeviceToHost);
    if (e == hipSuccess && zero) e = hipMemset(n->gr, 0, sizeof(float) * count);
    return e == hipSuccess ? SAL_OK : nfail(n, SAL_E_DEVICE, hipGetErrorString(e));
}

sal_status sal_net_set_output_scale(sal_net *n, const float scale[3])
{
    if (!n || !scale) return nfail(n, SAL_E_INVAL, "null argument");
    for (int c = 0; c < 3; ++c) n->out_scale[c] = scale[c];
    return SAL_OK;
}

sal_status sal_net_workspace_size(sal_net *n, int64_t nb, int64_t n0, int64_t n1, int64_t n2, int train,
                                  size_t *bytes)
{
    if (!n || !bytes || nb < 1 || n0 < 2 || n1 < 2 || n2 < 2) return nfail(n, SAL_E_INVAL, "bad argument");
    const int64_t nv = nvox_of(nb, n0, n1, n2);
    *bytes = train ? train_ws(nv, act_bytes(n)).total : infer_ws(n, nv);
    return SAL_OK;
}

static sal_status check_blocks(sal_net *n, int64_t nb, int64_t n0, int64_t n1, int64_t n2)
{
    if (nb < 1 || n0 < 2 || n1 < 2 || n2 < 2) return nfail(n, SAL_E_INVAL, "every block dimension must be >= 2");
    if (nvox_of(nb, n0, n1, n2) * 24 > ((int64_t)1 << 40)) return nfail(n, SAL_E_INVAL, "too large");
    if (conv_grid(nb, n0, n1, n2) > 0x7fffffffu) return nfail(n, SAL_E_INVAL, "too many tiles");
    return SAL_OK;
}

sal_status sal_net_forward(sal_net *n, const float *X, int64_t nb, int64_t n0, int64_t n1, int64_t n2, float *Y,
                           void *ws, size_t ws_bytes, void *stream)
{
    if (!n || !X || !Y || !ws) return nfail(n, SAL_E_INVAL, "null argument");
    sal_status st = check_blocks(n, nb, n0, n1, n2);
    if (st != SAL_OK) return st;
    const TrainWs tw = train_ws(nvox_of(nb, n0, n1, n2), act_bytes(n));
    if (ws_bytes < tw.total) return nfail(n, SAL_E_WORKSPACE, "workspace too small");
    NetDev nd(n->device);
    hipError_t e = net_forward(n, X, nb, n0, n1, n2, (char *)ws, &tw, Y, 3, 1, make_float3(1.f, 1.f, 1.f),
                               (hipStream_t)stream);
    return e == hipSuccess ? SAL_OK : nfail(n, SAL_E_DEVICE, hipGetErrorString(e));
}

sal_status sal_net_backward(sal_net *n, const float *X, const float *dY, int64_t nb, int64_t n0, int64_t n1,
                            int64_t n2, void *ws, size_t ws_bytes, void *stream)
{
    if (!n || !X || !dY || !ws) return nfail(n, SAL_E_INVAL, "null argument");
    sal_status st = check_blocks(n, nb, n0, n1, n2);
    if (st != SAL_OK) return st;
    const int64_t nv = nvox_of(nb, n0, n1, n2);
    const TrainWs tw = train_ws(nv, act_bytes(n));
    if (ws_bytes < tw.total) return nfail(n, SAL_E_WORKSPACE, "workspace too small");
    NetDev nd(n->device);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    const void *dYa = dY;  // the FP32-operand mode reads the caller's FP32 gradient directly
    if (!n->f32) {
        hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((nv * 3 + 255) / 256)), dim3(256), 0, s, dY, nv * 3,
                           (uint16_t *)(w + tw.dy));
        dYa = w + tw.dy;
    }
    hipError_t e = net_backward(n, X, dYa, nb, n0, n1, n2, w, tw, s);
    return e == hipSuccess ? SAL_OK : nfail(n, SAL_E_DEVICE, hipGetErrorString(e));
}

sal_status sal_net_adam(sal_net *n, float lr, void *stream)
{
    if (!n) return nfail(n, SAL_E_INVAL, "null argument");
    if (!(lr >= 0.f)) return nfail(n, SAL_E_INVAL, "lr must be >= 0");
    NetDev nd(n->device);
    hipError_t e = adam_step(n, lr, (hipStream_t)stream);
    return e == hipSuccess ? SAL_OK : nfail(n, SAL_E_DEVICE, hipGetErrorString(e));
}

sal_status sal_net_train_step(sal_net *n, const float *X, const float *T, int64_t nb, int64_t S, int32_t margin,
                              float lr, float *loss_out, void *ws, size_t ws_bytes, void *stream)
{
    if (!n || !X || !T || !ws) return nfail(n, SAL_E_INVAL, "null argument");
    if (margin < NL || 2 * margin >= S) return nfail(n, SAL_E_INVAL, "margin must be >= 5 and < S/2");
    if (!(lr >= 0.f)) return nfail(n, SAL_E_INVAL, "lr must be >= 0");
    sal_status st = check_blocks(n, nb, S, S, S);
    if (st != SAL_OK) return st;
    const int64_t nv = nvox_of(nb, S, S, S);
    const TrainWs tw = train_ws(nv, act_bytes(n));
    if (ws_bytes < tw.total) return nfail(n, SAL_E_WORKSPACE, "workspace too small");
    NetDev nd(n->device);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    float *Y = (float *)(w + tw.y);
    hipError_t e = net_forward(n, X, nb, S, S, S, w, &tw, Y, 3, 1, make_float3(1.f, 1.f, 1.f), s);
    const int64_t inner = S - 2 * margin;
    const float inv = 1.0f / (float)(nb * inner * inner * inner * 3);
    const unsigned nblk = (unsigned)((nv + 255) / 256);
    if (n->f32)
        hipLaunchKernelGGL(k_mse<true>, dim3(nblk), dim3(256), 0, s, Y, T, (int)nb, (int)S, margin, inv,
                           (float *)(w + tw.dy), (float *)(w + tw.lossp));
    else
        hipLaunchKernelGGL(k_mse<false>, dim3(nblk), dim3(256), 0, s, Y, T, (int)nb, (int)S, margin, inv,
                           (uint16_t *)(w + tw.dy), (float *)(w + tw.lossp));
    if (loss_out)
        hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, s, (const float *)(w + tw.lossp), (int)nblk, loss_out);
    if (e == hipSuccess) e = net_backward(n, X, w + tw.dy, nb, S, S, S, w, tw, s);
    if (e == hipSuccess) e = adam_step(n, lr, s);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? SAL_OK : nfail(n, SAL_E_DEVICE, hipGetErrorString(e));
}

// Inference over a whole volume: raw maps [3][n0][n1][n2] in the units of the training
// targets times out_scale.
sal_status sal_net_infer(sal_net *n, const float *V, int64_t n0, int64_t n1, int64_t n2, float *S_raw, void *ws,
                         size_t ws_bytes, void *stream)
{
    if (!n || !V || !S_raw || !ws) return nfail(n, SAL_E_INVAL, "null argument");
    sal_status st = check_blocks(n, 1, n0, n1, n2);
    if (st != SAL_OK) return st;
    const int64_t nv = nvox_of(1, n0, n1, n2);
    if (ws_bytes < infer_ws(n, nv)) return nfail(n, SAL_E_WORKSPACE, "workspace too small");
    NetDev nd(n->device);
    hipError_t e = net_forward(n, V, 1, n0, n1, n2, (char *)ws, nullptr, S_raw, 1, nv,
                               make_float3(n->out_scale[0], n->out_scale[1], n->out_scale[2]), (hipStream_t)stream);
    return e == hipSuccess ? SAL_OK : nfail(n, SAL_E_DEVICE, hipGetErrorString(e));
}

}  // extern "C"
