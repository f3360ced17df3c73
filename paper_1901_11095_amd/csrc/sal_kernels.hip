// gfx950 kernels of the seismic saliency method (Shafiq et al., ICIP 2017, Sec. 2).
//
// k_energy     steps 1-3: per-voxel local DFT of the L^3 window as three separable
//              contractions on MFMA (t: real -> half spectrum, then x, then y), the plane
//              projections of Eqs. (1)-(4) with DC excluded, and the absolute means E_m.
// k_dcs        step 4: directional center-surround comparison, Eq. (5), plus per-block
//              min/max of every raw map.
// k_stats      FP64 reduction of the per-block partials into the volume-wide statistics.
// k_combine    step 5: per-component min-max normalisation and Eq. (6), in FP64.
// k_local_spectra / k_project   un-fused steps 1 and 2-3 for checks on small boxes.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "sal_internal.h"

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Reflect u into [0, n) without repeating the edge sample; exact for -(n-1) <= u <= 2(n-1).
// The final clamp only matters for padding positions of edge tiles, whose results are
// never stored.
__device__ __forceinline__ int refl_idx(int u, int n)
{
    u = u < 0 ? -u : u;
    u = u >= n ? 2 * (n - 1) - u : u;
    return u < 0 ? 0 : (u >= n ? n - 1 : u);
}

// Workgroup -> tile order that keeps neighbouring tiles on one XCD: workgroups are
// dispatched round-robin over the 8 XCDs, so workgroup b runs on XCD b % 8; giving each XCD
// a contiguous range of tiles lets halo re-reads hit that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblk)
{
    const int q = nblk >> 3;
    if (bid >= (q << 3)) return bid;
    return (bid & 7) * q + (bid >> 3);
}

template <int L>
struct Geo {
    static constexpr int H = L / 2;                         // window start = v - H
    static constexpr int h = L / 2 + 1;                     // t frequencies kept (Hermitian half)
    static constexpr int KS = (2 * L) / 4;                  // 16x16x4 steps of a complex contraction
    static constexpr int MT = (2 * L) / 16;                 // 16-row tiles of (freq, re|im)
    static constexpr int KSA = L / 4;                       // steps of the real t contraction
    static constexpr int MTA = (2 * h + 15) / 16;           // row tiles of the t contraction
    static constexpr int NR = (h - 2) * L + 2 * (L / 2 + 1);  // (mu, nu) rows kept
};

template <int L>
struct TileCfg;
template <>
struct TileCfg<8> {
    static constexpr int NW = 4, TY = 32;
    static constexpr bool W_LDS = true;
};
template <>
struct TileCfg<16> {
    static constexpr int NW = 4, TY = 16;
    static constexpr bool W_LDS = false;
};

}  // namespace

// ------------------------------------------------------------------------------------
// Steps 1-3, FP32.  One workgroup = NW waves owns a tile of NW x-rows by TY y-columns and
// walks t over [t_begin, t_end).  For every t0:
//   stage A (all waves): A[x', y', mu] = sum_p W[mu, p] V[t0 - H + p, x', y'] for the whole
//            (NW + L - 1) x (TY + L - 1) patch, mu <= L/2, MFMA with N = 16 positions;
//   stage B (wave w, x-row x0 = w): per mu, B[nu, y'] = sum_q W[nu, q] A[x0 + q, y', mu];
//   stage C (wave w): per kept (mu, nu) row, F[om, y0] = sum_r W[om, r] B[nu, y0 + r], the
//            window sum of 16 consecutive voxels as one 16x16 tile (y0 on N, (om, re|im)
//            on M), never leaving the accumulators; each lane turns its two complex bins
//            into magnitudes and folds them with the projection weights into E_t, E_x, E_y.
// Rows (mu, nu) with mu in {0, L/2} keep nu <= L/2 only: the remaining bins are complex
// conjugates of kept ones, and the weights carry the multiplicity.
template <int L>
__global__ __launch_bounds__(64 * TileCfg<L>::NW) void k_energy_f32(
    const float *__restrict__ V, int n0, int n1, int n2, int tt_len, int nby, int nbx,
    const float *__restrict__ w_c, const float *__restrict__ w_a,
    const float *__restrict__ w_bin, float *__restrict__ E, float *__restrict__ vmax_part)
{
    using G = Geo<L>;
    using C = TileCfg<L>;
    constexpr int H = G::H, h = G::h, KS = G::KS, MT = G::MT, KSA = G::KSA, MTA = G::MTA;
    constexpr int NW = C::NW, TY = C::TY;
    constexpr int PX = NW + L - 1, PY = TY + L - 1;
    constexpr int NTB = (PY + 15) / 16, PYB = NTB * 16, NTC = TY / 16;
    constexpr int NPOS = PX * PY, NTA = (NPOS + 15) / 16, NJ = (NTA + NW - 1) / NW;
    constexpr int NWB = C::W_LDS ? G::NR * MT * 32 : 1;

    __shared__ float2 A_s[NPOS * h];
    __shared__ float2 B_s[NW][L * PYB];
    __shared__ float wb_s[NWB];
    __shared__ float red_s[NW];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int ty = tile % nby, tx = (tile / nby) % nbx, tb = tile / (nby * nbx);
    const int y_base = ty * TY, x_base = tx * NW;
    const int t_begin = tb * tt_len;
    const int t_end = min(n0, t_begin + tt_len);

    // constant MFMA A-operands: lane (g, n) holds row n of each M tile at K = KS*g + kk
    float wc[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) wc[mt][kk] = w_c[(16 * mt + n) * (2 * L) + KS * g + kk];
    float wa[MTA][KSA];
#pragma unroll
    for (int mt = 0; mt < MTA; ++mt)
#pragma unroll
        for (int kk = 0; kk < KSA; ++kk) wa[mt][kk] = w_a[(16 * mt + n) * L + KSA * g + kk];
    if (C::W_LDS)
        for (int i = threadIdx.x; i < NWB; i += 64 * NW) wb_s[i] = w_bin[i];

    // stage-A positions of this wave (fixed for the whole t walk)
    int off_xy[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        int pos = min((wave + NW * jj) * 16 + n, NPOS - 1);
        int xp = pos / PY, yp = pos - xp * PY;
        int gx = refl_idx(x_base - H + xp, n1), gy = refl_idx(y_base - H + yp, n2);
        off_xy[jj] = gx * n2 + gy;
    }
    const int64_t plane = (int64_t)n1 * n2;
    const int64_t nvox = plane * n0;
    float vmax = 0.0f;
    float2 *Bw = B_s[wave];

    for (int t0 = t_begin; t0 < t_end; ++t0) {
        __syncthreads();  // previous t0 is done with A_s
        // ---------------- stage A: real DFT along t -------------------------------------
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int tl = wave + NW * jj;
            if (tl < NTA) {
                f4 acc[MTA];
#pragma unroll
                for (int mt = 0; mt < MTA; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < KSA; ++kk) {
                    const int tr = refl_idx(t0 - H + KSA * g + kk, n0);
                    const float v = V[tr * plane + off_xy[jj]];
                    vmax = fmaxf(vmax, fabsf(v));
#pragma unroll
                    for (int mt = 0; mt < MTA; ++mt) acc[mt] = mfma4(wa[mt][kk], v, acc[mt]);
                }
                const int pos = tl * 16 + n;
                if (pos < NPOS) {
#pragma unroll
                    for (int mt = 0; mt < MTA; ++mt) {
                        const int mu0 = 8 * mt + 2 * g;
                        if (mu0 < h) A_s[pos * h + mu0] = make_float2(acc[mt][0], acc[mt][1]);
                        if (mu0 + 1 < h) A_s[pos * h + mu0 + 1] = make_float2(acc[mt][2], acc[mt][3]);
                    }
                }
            }
        }
        __syncthreads();

        float e[NTC][3];
#pragma unroll
        for (int c = 0; c < NTC; ++c) e[c][0] = e[c][1] = e[c][2] = 0.f;
        int row = 0;
#pragma unroll 1
        for (int mu = 0; mu < h; ++mu) {
            // ---------------- stage B: complex DFT along x for this mu ------------------
#pragma unroll
            for (int nb = 0; nb < NTB; ++nb) {
                const int yp = min(nb * 16 + n, PY - 1);
                f4 acc[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < KS; kk += 2) {
                    const int q = (KS * g + kk) >> 1;
                    const float2 a = A_s[((wave + q) * PY + yp) * h + mu];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        acc[mt] = mfma4(wc[mt][kk], a.x, acc[mt]);
                        acc[mt] = mfma4(wc[mt][kk + 1], a.y, acc[mt]);
                    }
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int nu0 = 8 * mt + 2 * g;
                    Bw[nu0 * PYB + nb * 16 + n] = make_float2(acc[mt][0], acc[mt][1]);
                    Bw[(nu0 + 1) * PYB + nb * 16 + n] = make_float2(acc[mt][2], acc[mt][3]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // ---------------- stage C: complex DFT along y, projections, energies -------
            const int nuc = (mu == 0 || mu == L / 2) ? L / 2 + 1 : L;
#pragma unroll 1
            for (int nu = 0; nu < nuc; ++nu, ++row) {
                float wv[MT][6];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int wo = ((row * MT + mt) * 4 + g) * 8;
#pragma unroll
                    for (int k = 0; k < 6; ++k) wv[mt][k] = C::W_LDS ? wb_s[wo + k] : w_bin[wo + k];
                }
#pragma unroll
                for (int c = 0; c < NTC; ++c) {
                    const int y0 = c * 16 + n;
                    f4 acc[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kk = 0; kk < KS; kk += 2) {
                        const int rr = (KS * g + kk) >> 1;
                        const float2 b = Bw[nu * PYB + y0 + rr];
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            acc[mt] = mfma4(wc[mt][kk], b.x, acc[mt]);
                            acc[mt] = mfma4(wc[mt][kk + 1], b.y, acc[mt]);
                        }
                    }
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const float m0 = __builtin_amdgcn_sqrtf(
                            fmaf(acc[mt][0], acc[mt][0], acc[mt][1] * acc[mt][1]));
                        const float m1 = __builtin_amdgcn_sqrtf(
                            fmaf(acc[mt][2], acc[mt][2], acc[mt][3] * acc[mt][3]));
#pragma unroll
                        for (int m = 0; m < 3; ++m)
                            e[c][m] = fmaf(wv[mt][3 + m], m1, fmaf(wv[mt][m], m0, e[c][m]));
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // reduce the four lane groups (lanes n, n+16, n+32, n+48 hold the same voxel)
        const int x = x_base + wave;
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                float s = e[c][m];
                s += __shfl_xor(s, 16);
                s += __shfl_xor(s, 32);
                e[c][m] = s;
            }
            const int y = y_base + c * 16 + n;
            if (g == 0 && x < n1 && y < n2) {
                const int64_t o = ((int64_t)t0 * n1 + x) * n2 + y;
                E[o] = e[c][0];
                E[nvox + o] = e[c][1];
                E[2 * nvox + o] = e[c][2];
            }
        }
    }
    // max |V| of everything this workgroup read (all of it lies in the volume)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    if (lane == 0) red_s[wave] = vmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = red_s[0];
        for (int w = 1; w < NW; ++w) m = fmaxf(m, red_s[w]);
        vmax_part[blockIdx.x] = m;
    }
}

// ------------------------------------------------------------------------------------
// Step 4, Eq. (5): one thread per voxel; neighbours are read through the caches.
__global__ __launch_bounds__(256) void k_dcs(const float *__restrict__ E, int n0, int n1, int n2,
                                             dcs_args a, float *__restrict__ S,
                                             float *__restrict__ mm_part)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    if (v < N) {
        const int y = (int)(v % n2);
        const int64_t rest = v / n2;
        const int x = (int)(rest % n1);
        const int t = (int)(rest / n1);
        const int pos[3] = {t, x, y};
        const int dims[3] = {n0, n1, n2};
        const int64_t stride[3] = {(int64_t)n1 * n2, n2, 1};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const float *Em = E + m * N;
            const float c = Em[v];
            float sum = 0.f;
            for (int b = 0; b < 6; ++b) {
                if (!((a.rays[m] >> b) & 1u)) continue;
                const int ax = b >> 1;
                const int dir = (b & 1) ? -1 : 1;
                const int64_t base = v - (int64_t)pos[ax] * stride[ax];
                for (int s = 1; s <= a.r; ++s) {
                    const int u = refl_idx(pos[ax] + dir * s, dims[ax]);
                    sum += fabsf(c - a.g[s - 1] * Em[base + (int64_t)u * stride[ax]]);
                }
            }
            const float sv = a.Q[m] > 0.f ? sum / a.Q[m] : 0.f;
            S[m * N + v] = sv;
            mn[m] = sv;
            mx[m] = sv;
        }
    }
    if (mm_part == nullptr) return;
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
        mm_part[(int64_t)blockIdx.x * 6 + k] = r;
    }
}

// ------------------------------------------------------------------------------------
// FP64 volume-wide statistics {lo_t, hi_t, lo_x, hi_x, lo_y, hi_y, max|V|} from partials.
__global__ __launch_bounds__(256) void k_stats(const float *__restrict__ vmax_part, int64_t nv,
                                               const float *__restrict__ mm, int64_t nm,
                                               double *__restrict__ stats)
{
    __shared__ double red[7][256];
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    double vm = 0.0;
    for (int64_t i = threadIdx.x; i < nv; i += 256) vm = fmax(vm, (double)vmax_part[i]);
    for (int64_t i = threadIdx.x; i < nm; i += 256)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            lo[m] = fmin(lo[m], (double)mm[i * 6 + 2 * m]);
            hi[m] = fmax(hi[m], (double)mm[i * 6 + 2 * m + 1]);
        }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        red[2 * m][threadIdx.x] = lo[m];
        red[2 * m + 1][threadIdx.x] = hi[m];
    }
    red[6][threadIdx.x] = vm;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                const double o = red[k][threadIdx.x + w];
                double &me = red[k][threadIdx.x];
                me = (k < 6 && !(k & 1)) ? fmin(me, o) : fmax(me, o);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) stats[threadIdx.x] = red[threadIdx.x][0];
}

// ------------------------------------------------------------------------------------
// Step 5, Eq. (6) after per-component min-max normalisation, evaluated in FP64.
__global__ __launch_bounds__(256) void k_combine(const float *__restrict__ S_raw, int64_t N,
                                                 const double *__restrict__ stats, double wa,
                                                 double wb, double wc, int normalize,
                                                 double zero_range, float *__restrict__ S)
{
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= N) return;
    const double w[3] = {wa, wb, wc};
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double x = (double)S_raw[m * N + v];
        if (normalize) {
            const double lo = stats[2 * m], range = stats[2 * m + 1] - lo;
            const double sc = range > zero_range * stats[6] ? 1.0 / range : 0.0;
            acc += w[m] * ((x - lo) * sc);
        } else {
            acc += w[m] * x;
        }
    }
    S[v] = (float)acc;
}

// ------------------------------------------------------------------------------------
// Step 1 for the voxels of a box: the full L^3 spectrum of every window, three separable
// passes in LDS with FP32 complex arithmetic, scaled by 1/L^3 (exact for L a power of 2).
template <int L>
__global__ __launch_bounds__(256) void k_local_spectra(const float *__restrict__ V, int n0, int n1,
                                                       int n2, int lo0, int lo1, int lo2, int b1,
                                                       int b2, const float2 *__restrict__ tw_g,
                                                       float2 *__restrict__ out)
{
    constexpr int L3 = L * L * L, H = L / 2;
    __shared__ float2 buf0[L3], buf1[L3];
    __shared__ float2 tw[L];
    const int vox = blockIdx.x;
    const int c = vox % b2, b = (vox / b2) % b1, a = vox / (b1 * b2);
    const int t = lo0 + a, x = lo1 + b, y = lo2 + c;
    for (int i = threadIdx.x; i < L3; i += 256) {
        const int p = i / (L * L), q = (i / L) % L, r = i % L;
        const int gt = refl_idx(t - H + p, n0), gx = refl_idx(x - H + q, n1), gy = refl_idx(y - H + r, n2);
        buf0[i] = make_float2(V[((int64_t)gt * n1 + gx) * n2 + gy], 0.f);
    }
    if (threadIdx.x < L) tw[threadIdx.x] = tw_g[threadIdx.x];
    __syncthreads();
    // r -> om
    for (int i = threadIdx.x; i < L3; i += 256) {
        const int pq = i / L, om = i % L;
        float re = 0.f, im = 0.f;
        for (int r = 0; r < L; ++r) {
            const float2 f = buf0[pq * L + r], w = tw[(r * om) % L];
            re = fmaf(f.x, w.x, fmaf(-f.y, w.y, re));
            im = fmaf(f.x, w.y, fmaf(f.y, w.x, im));
        }
        buf1[i] = make_float2(re, im);
    }
    __syncthreads();
    // q -> nu
    for (int i = threadIdx.x; i < L3; i += 256) {
        const int p = i / (L * L), nu = (i / L) % L, om = i % L;
        float re = 0.f, im = 0.f;
        for (int q = 0; q < L; ++q) {
            const float2 f = buf1[(p * L + q) * L + om], w = tw[(q * nu) % L];
            re = fmaf(f.x, w.x, fmaf(-f.y, w.y, re));
            im = fmaf(f.x, w.y, fmaf(f.y, w.x, im));
        }
        buf0[i] = make_float2(re, im);
    }
    __syncthreads();
    // p -> mu, times 1/L^3
    const float sc = 1.0f / (float)L3;
    for (int i = threadIdx.x; i < L3; i += 256) {
        const int mu = i / (L * L), nuom = i % (L * L);
        float re = 0.f, im = 0.f;
        for (int p = 0; p < L; ++p) {
            const float2 f = buf0[p * L * L + nuom], w = tw[(p * mu) % L];
            re = fmaf(f.x, w.x, fmaf(-f.y, w.y, re));
            im = fmaf(f.x, w.y, fmaf(f.y, w.x, im));
        }
        out[(int64_t)vox * L3 + i] = make_float2(re * sc, im * sc);
    }
}

// Steps 2-3 on given spectra: one wave per voxel.
template <int L>
__global__ __launch_bounds__(64) void k_project(const float2 *__restrict__ F, int64_t nvox,
                                                const float4 *__restrict__ w_proj,
                                                float *__restrict__ E)
{
    constexpr int L3 = L * L * L;
    const int64_t v = blockIdx.x;
    const float2 *f = F + v * L3;
    float e0 = 0.f, e1 = 0.f, e2 = 0.f;
    for (int b = threadIdx.x; b < L3; b += 64) {
        const float2 z = f[b];
        const float m = sqrtf(fmaf(z.x, z.x, z.y * z.y));
        const float4 w = w_proj[b];
        e0 = fmaf(w.x, m, e0);
        e1 = fmaf(w.y, m, e1);
        e2 = fmaf(w.z, m, e2);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        e0 += __shfl_xor(e0, o);
        e1 += __shfl_xor(e1, o);
        e2 += __shfl_xor(e2, o);
    }
    if (threadIdx.x == 0) {
        E[v] = e0;
        E[nvox + v] = e1;
        E[2 * nvox + v] = e2;
    }
}

// ====================================================================== launchers

static int tt_len_for(int64_t n0, int64_t tiles_xy)
{
    // enough workgroups to fill 256 CUs several times over; long t walks otherwise
    int64_t tt = 32;
    while (tt > 2 && tiles_xy * ((n0 + tt - 1) / tt) < 2048) tt >>= 1;
    return (int)tt;
}

template <int L>
static void energy_grid(int64_t n0, int64_t n1, int64_t n2, int *nby, int *nbx, int *tt, int64_t *nblk)
{
    using C = TileCfg<L>;
    *nby = (int)((n2 + C::TY - 1) / C::TY);
    *nbx = (int)((n1 + C::NW - 1) / C::NW);
    *tt = tt_len_for(n0, (int64_t)(*nby) * (*nbx));
    *nblk = (int64_t)(*nby) * (*nbx) * ((n0 + *tt - 1) / *tt);
}

int64_t energy_num_blocks(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2)
{
    int nby, nbx, tt;
    int64_t nb;
    if (c->L == 8)
        energy_grid<8>(n0, n1, n2, &nby, &nbx, &tt, &nb);
    else
        energy_grid<16>(n0, n1, n2, &nby, &nbx, &tt, &nb);
    return nb;
}

template <int L>
static hipError_t launch_energy_L(const sal_ctx *c, const float *V, int64_t n0, int64_t n1,
                                  int64_t n2, float *E, float *vmax_part, int *nparts,
                                  hipStream_t s)
{
    int nby, nbx, tt;
    int64_t nb;
    energy_grid<L>(n0, n1, n2, &nby, &nbx, &tt, &nb);
    if (nparts) *nparts = (int)nb;
    hipLaunchKernelGGL(k_energy_f32<L>, dim3((unsigned)nb), dim3(64 * TileCfg<L>::NW), 0, s, V,
                       (int)n0, (int)n1, (int)n2, tt, nby, nbx, c->t.w_c, c->t.w_a, c->t.w_bin,
                       E, vmax_part);
    return hipGetLastError();
}

hipError_t launch_energy(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                         float *E, float *vmax_part, int *nparts, hipStream_t s)
{
    if (c->L == 8) return launch_energy_L<8>(c, V, n0, n1, n2, E, vmax_part, nparts, s);
    return launch_energy_L<16>(c, V, n0, n1, n2, E, vmax_part, nparts, s);
}

int64_t dcs_num_blocks(int64_t n0, int64_t n1, int64_t n2) { return (n0 * n1 * n2 + 255) / 256; }

hipError_t launch_dcs(const sal_ctx *c, const float *E, int64_t n0, int64_t n1, int64_t n2,
                      float *S_raw, float *minmax_part, hipStream_t s)
{
    dcs_args a;
    a.r = c->r;
    for (int m = 0; m < 3; ++m) {
        a.rays[m] = c->p.rays[m];
        a.Q[m] = c->Q[m];
    }
    for (int i = 0; i < 32; ++i) a.g[i] = c->g[i];
    hipLaunchKernelGGL(k_dcs, dim3((unsigned)dcs_num_blocks(n0, n1, n2)), dim3(256), 0, s, E,
                       (int)n0, (int)n1, (int)n2, a, S_raw, minmax_part);
    return hipGetLastError();
}

hipError_t launch_stats(const float *vmax_part, int64_t nv, const float *minmax_part, int64_t nm,
                        double *stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(256), 0, s, vmax_part, nv, minmax_part, nm, stats);
    return hipGetLastError();
}

hipError_t launch_combine(const float *S_raw, int64_t nvox, const double *stats, double a,
                          double b, double c, int normalize, double zero_range, float *S,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((nvox + 255) / 256)), dim3(256), 0, s, S_raw,
                       nvox, stats, a, b, c, normalize, zero_range, S);
    return hipGetLastError();
}

hipError_t launch_local_spectra(const sal_ctx *c, const float *V, int64_t n0, int64_t n1,
                                int64_t n2, const int64_t lo[3], const int64_t bn[3], float *out,
                                hipStream_t s)
{
    const unsigned nb = (unsigned)(bn[0] * bn[1] * bn[2]);
    if (nb == 0) return hipSuccess;
    const float2 *tw = reinterpret_cast<const float2 *>(c->t.twiddle);
    float2 *o = reinterpret_cast<float2 *>(out);
    if (c->L == 8)
        hipLaunchKernelGGL(k_local_spectra<8>, dim3(nb), dim3(256), 0, s, V, (int)n0, (int)n1,
                           (int)n2, (int)lo[0], (int)lo[1], (int)lo[2], (int)bn[1], (int)bn[2], tw, o);
    else
        hipLaunchKernelGGL(k_local_spectra<16>, dim3(nb), dim3(256), 0, s, V, (int)n0, (int)n1,
                           (int)n2, (int)lo[0], (int)lo[1], (int)lo[2], (int)bn[1], (int)bn[2], tw, o);
    return hipGetLastError();
}

hipError_t launch_project(const sal_ctx *c, const float *spectra, int64_t nvox, float *E,
                          hipStream_t s)
{
    if (nvox == 0) return hipSuccess;
    const float2 *F = reinterpret_cast<const float2 *>(spectra);
    const float4 *w = reinterpret_cast<const float4 *>(c->t.w_proj);
    if (c->L == 8)
        hipLaunchKernelGGL(k_project<8>, dim3((unsigned)nvox), dim3(64), 0, s, F, nvox, w, E);
    else
        hipLaunchKernelGGL(k_project<16>, dim3((unsigned)nvox), dim3(64), 0, s, F, nvox, w, E);
    return hipGetLastError();
}
