// Steps 1-3 at cube L = 8 and 16 in FP32 with the window sliding along t (Sec. 2 steps 1-3),
// for windows at every voxel (stride S = 1) or on the lattice of a stride S below L/2.
//
// The L^3 DFT of the window centred on (t0, x0, y0) factors into a 2-D DFT of each of its
// L t-planes (x then y) followed by the DFT along t of those plane spectra.  With the
// t-phase taken from the absolute row index v (a unit-modulus factor per window and
// frequency, which the magnitudes of Eqs. (1)-(4) do not see),
//     D_t0[kt, kx, ky] = sum_{v = t0-L/2}^{t0+L/2-1} P_v[kx, ky] e^{-2 pi i kt v / L},
// and since e^{-2 pi i kt (v + L) / L} = e^{-2 pi i kt v / L}, the next window's spectrum
// is this one's plus (P_{v_in} - P_{v_out}) e^{-2 pi i kt v_in / L}, where the plane
// leaving (v_out = v_in - L) and the plane entering share the twiddle.  By linearity
// P_{v_in} - P_{v_out} is the 2-D DFT of the plane difference V[v_in] - V[v_out], so each
// window costs one 2-D plane DFT (matrix cores) and one complex multiply-add per bin (vector
// ALUs) instead of a full DFT along t.  Rows are reflected at the t faces exactly as the
// window's own rows are.
//
// Each product is rounded before it is added, so a plane that enters and later leaves
// cancels exactly (a unit spike leaves exact zeros behind).  The running sums restart from
// zero at fixed absolute rows (window t0 = 0, L/2, 512, 1024, ...; restarting at t0 = L/2
// keeps the rows reflected at the t = 0 face out of every later window's history), so a
// window's result does not depend on the box or batch it is computed in, and the rounding
// drift of the sums stays within 527 steps.
//
// Workgroup: one x0, 16 y0 S apart, one t segment; L/2 waves, wave c owning column c of
// the 2-D plane spectrum (c = 1..L/2-1: the x frequency kx = c; c = 0: kx = 0 and kx = L/2
// packed as one complex column Z = X_0 + i X_{L/2} of two real sequences).  Per t-step:
//   stage 1 (waves 1 .. L/2 - 1, 16 positions at a time): X[comp, y] =
//     sum_tau M1[comp, tau] dV[x0 - L/2 + tau, y] for the PY = 15 S + L positions y of the
//     tile, the real DFT along x packed into L real components;
//   stage 2 (wave c): P[ky, y0] = sum_tau W[ky, tau] X_c[y0 - L/2 + tau], complex, L ky on
//     L/8 M tiles whose lane groups hold ky and -ky, the 16 windows on N;
//   stage 3 (wave c): the lane's 4L bins (M tiles x two ky x L kt) of its window take their
//     update; at output steps (every S-th window along t) their magnitudes are weighted into
//     E_t, E_x, E_y.
// With S > 1 every row still enters and leaves (the sums slide one row per step), while the
// workgroups, the y positions and the magnitudes are those of the lattice windows only.
// In wave 0 the bins (kt, ky) and (-kt, -ky) of the packed column sit in one lane; its
// update is applied to U = Z[k] + conj Z[-k] = 2 D_{kx=0}[k] and V = Z[k] - conj Z[-k] =
// 2i D_{kx=L/2}[k] instead (the plane spectra transformed the same way), so every slot is one
// bin's magnitude.  On the self-conjugate rows ky in {0, L/2} the slots kt and L - kt hold U
// and conj V, and kt in {0, L/2} hold Z itself, whose real and imaginary parts are two
// self-conjugate bins.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sal_device.h"
#include "sal_internal.h"

namespace {

constexpr int STY = 16;  // windows along y per workgroup

template <int L, int S>
struct SlideGeo {
    static constexpr int H = L / 2;            // window start = centre - H
    static constexpr int PY = S * (STY - 1) + L;  // stage-1 positions along y
    static constexpr int PLS = (PY + 15) / 32 * 32 + 16;  // plane row stride: tau rows 16 banks apart
    static constexpr int NW = L / 2;           // waves = packed columns of the x spectrum
    static constexpr int MT = L / 8;           // M tiles of the y contraction
    static constexpr int S1S = L + 2;          // stage-1 output row stride (floats)
    static constexpr int KS1 = L / 4;          // K steps of the x contraction
    static constexpr int KS2 = L / 2;          // K steps of the y contraction
    static constexpr int NP = L / 2 + 1;       // |kt| values
    static constexpr int SWP = slide_weights_per_group(L);
    static constexpr int NS1 = (PY + 15) / 16;  // stage-1 blocks of 16 positions
    static constexpr int NLD = (L * PY + 64 * NW - 1) / (64 * NW);  // plane samples per thread
    static constexpr int RW = NS1 + 1 < NW ? NS1 + 1 : NW - 1;       // the wave storing E
    static_assert(16 * NS1 <= PLS && 2 * S < L, "tile geometry");
};

__device__ __forceinline__ float mag(float re, float im) { return __builtin_amdgcn_sqrtf(fmaf(re, re, im * im)); }

}  // namespace

template <int L, int S>
__global__ __attribute__((amdgpu_waves_per_eu(2))) __launch_bounds__(64 * (L / 2)) void k_energy_slide(
    const float *__restrict__ V, int n0, int n1, int n2, ebox bx, int nseg, int nbx, int nby,
    const float *__restrict__ w_s1, const float *__restrict__ w_s2, const float *__restrict__ w_sp,
    const float2 *__restrict__ tw, float *__restrict__ E, float *__restrict__ vmax_part)
{
    using G = SlideGeo<L, S>;
    constexpr int SL = L, SH = G::H, SPY = G::PY, SNW = G::NW, MT = G::MT, S1S = G::S1S;
    constexpr int KS1 = G::KS1, KS2 = G::KS2, NP = G::NP, SWP = G::SWP, NS1 = G::NS1, NLD = G::NLD;
    constexpr int RW = G::RW, PLS = G::PLS;
    __shared__ float plane_s[2][SL * PLS];
    __shared__ float s1_s[2][SPY * S1S + 2];
    __shared__ float wt_s[SNW * 4 * SWP];
    __shared__ float red_s[2][SNW][3][STY];
    __shared__ float vred_s[SNW];
    // constant A operands, per lane: stage 1 [lane][K step], stage 2 [K step / 4][lane][4]
    __shared__ float4 a1_s[64];
    __shared__ float4 a2_s[MT * KS2 / 4][64];
    __shared__ float2 tw_s[SL];

    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, n = lane & 15;

    int box;
    const int tile = box_tile(bx, &box);
    V += box * bx.vstride;
    E += box * bx.estride;
    // x0 fastest: the workgroups of neighbouring x0 (L - 1 of their L plane rows shared) run
    // together on one XCD and meet the rows in its L2.  The t segment next: each XCD takes a
    // contiguous range of tiles, which must hold the short first segments and the long ones
    // in the same mix on every XCD.
    const int xr = tile % nbx, kr = (tile / nbx) % nseg, ty = tile / (nbx * nseg);
    const int y_base = bx.o2 + S * STY * ty, x0 = bx.o1 + S * xr;
    const int k = slide_seg_id(bx.o0, SH) + kr;
    const int s_start = slide_seg_start(k, SH);
    const int t_lo = max(s_start, bx.o0), t_hi = min(slide_seg_start(k + 1, SH), min(n0, bx.o0 + bx.d0));
    if (kr >= nseg || t_lo >= t_hi || x0 >= bx.o1 + bx.d1 || y_base >= bx.o2 + bx.d2) {
        if (threadIdx.x == 0 && vmax_part) vmax_part[blockIdx.x] = 0.f;
        return;
    }
    const int K1 = bx.fk1, K2 = bx.fk2;
    const int64_t nbox = (int64_t)bx.fk0 * K1 * K2;
    const int y_end = bx.o2 + bx.d2;

    for (int i = threadIdx.x; i < SNW * 4 * SWP; i += 64 * SNW) wt_s[i] = w_sp[i];
    if (threadIdx.x < SL) tw_s[threadIdx.x] = tw[threadIdx.x];
    // (at cube 16 the 16 stage-2 operands would not fit the registers beside the 128 of the
    // spectra)
    if (threadIdx.x < 64) {
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
        a.x = w_s1[lane];
        a.y = w_s1[64 + lane];
        if (KS1 > 2) {
            a.z = w_s1[128 + lane];
            a.w = w_s1[192 + lane];
        }
        a1_s[lane] = a;
    }
    for (int i = threadIdx.x; i < MT * KS2 * 16; i += 64 * SNW) {
        const int r = i >> 6, ln = i & 63;  // operands 4 r .. 4 r + 3 in the order (mt, kk)
        float4 a;
        a.x = w_s2[(4 * r) * 64 + ln];
        a.y = w_s2[(4 * r + 1) * 64 + ln];
        a.z = w_s2[(4 * r + 2) * 64 + ln];
        a.w = w_s2[(4 * r + 3) * 64 + ln];
        a2_s[r][ln] = a;
    }

    // plane samples: sample i = threadIdx.x + 64 NW l < L PY (slot l of the thread) is
    // (tau, yy) = (i / PY, i % PY)
    const int n12 = n1 * n2;  // the volume holds at most 2^31 - 1 samples
    bool loader[NLD];
    int off[NLD], pidx[NLD];
#pragma unroll
    for (int l = 0; l < NLD; ++l) {
        const int i = threadIdx.x + 64 * SNW * l;
        loader[l] = i < SL * SPY;
        off[l] = pidx[l] = 0;
        if (loader[l]) {
            const int tau = i / SPY, yy = i - tau * SPY;
            off[l] = refl_idx(x0 - SH + tau, n1) * n2 + refl_idx(y_base - SH + yy, n2);
            pidx[l] = tau * PLS + yy;
        }
    }
    // step j brings row v_in = s_start - L/2 + j in and, from j = L on, takes v_in - L out;
    // the window t0 = s_start + j - (L - 1) is complete after step j
    const int nsteps = t_hi - s_start + SL - 1;
    float vmax = 0.f;
    // the samples of step j are loaded two steps ahead and only read when the plane is
    // written to LDS, so the loads' latency overlaps a whole step
    float ra[NLD], rb[NLD];
#pragma unroll
    for (int l = 0; l < NLD; ++l) ra[l] = rb[l] = 0.f;
    auto load_plane = [&](int j) {
        const int vin = s_start - SH + j;
        const int r_in = refl_idx(vin, n0) * n12, r_out = refl_idx(vin - SL, n0) * n12;
#pragma unroll
        for (int l = 0; l < NLD; ++l)
            if (loader[l]) {
                ra[l] = V[(uint32_t)(r_in + off[l])];
                rb[l] = V[(uint32_t)(r_out + off[l])];  // in the volume; unused before j = L
            }
    };
    // the plane difference of step j into LDS buffer buf
    auto store_plane = [&](int j, int buf) {
#pragma unroll
        for (int l = 0; l < NLD; ++l)
            if (loader[l]) {
                vmax = fmaxf(vmax, fmaxf(fabsf(ra[l]), fabsf(rb[l])));
                plane_s[buf][pidx[l]] = j >= SL ? ra[l] - rb[l] : ra[l];
            }
    };
    auto stage1 = [&](int buf) {
        // waves 1 .. L/2 - 1: positions 16 jt + n for jt = wave - 1, wave - 1 + L/2 - 1, ...
        const float4 a1 = a1_s[lane];
        for (int jt = wave - 1; jt < NS1; jt += SNW - 1) {
            f4 acc = f4{0.f, 0.f, 0.f, 0.f};
            const float *pl = plane_s[buf] + 16 * jt + n;
            acc = mfma4(a1.x, pl[g * PLS], acc);
            acc = mfma4(a1.y, pl[(4 + g) * PLS], acc);
            if (KS1 > 2) {
                acc = mfma4(a1.z, pl[(8 + g) * PLS], acc);
                acc = mfma4(a1.w, pl[(12 + g) * PLS], acc);
            }
            const int yy = 16 * jt + n;
            if (yy < SPY && 4 * g < SL) {
                float *o = s1_s[buf] + yy * S1S + 4 * g;
                *reinterpret_cast<float2 *>(o) = make_float2(acc[0], acc[1]);
                *reinterpret_cast<float2 *>(o + 2) = make_float2(acc[2], acc[3]);
            }
        }
    };

    // E of the window completed at step jo (red_s[buf]), summed over the waves in a fixed
    // order, at the lattice windows of the box
    auto store_energies = [&](int jo, int buf) {
        const int t0 = s_start + jo - (SL - 1);
        if (t0 < t_lo || (t0 - bx.o0) % S != 0 || lane >= 3 * STY) return;
        const int m = lane >> 4, yy = lane & 15;
        float e = red_s[buf][0][m][yy];
#pragma unroll
        for (int w = 1; w < SNW; ++w) e += red_s[buf][w][m][yy];
        const int y = y_base + S * yy;
        if (y < y_end) {
            const int64_t o = ((int64_t)((t0 - bx.fo0) / S) * K1 + (x0 - bx.fo1) / S) * K2 + (y - bx.fo2) / S;
            E[m * nbox + o] = e;
        }
    };

    load_plane(0);
    store_plane(0, 0);
    __syncthreads();
    if (wave >= 1) stage1(0);
    if (nsteps > 1) load_plane(1);

    // spectrum state: [M tile][ky slot][kt]
    float Dr[MT][2][SL], Di[MT][2][SL];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int kt = 0; kt < SL; ++kt) Dr[mt][q][kt] = Di[mt][q][kt] = 0.f;

    const float *wl = wt_s + (wave * 4 + g) * SWP;
    const bool sp_lane = g == 0;  // wave 0: lane group holding the self-conjugate rows 0, L/2

#pragma unroll 1
    for (int j = 0; j < nsteps; ++j) {
        const int b = j & 1;
        if (j + 1 < nsteps) store_plane(j + 1, b ^ 1);
        __syncthreads();
        if (j + 2 < nsteps) load_plane(j + 2);
        if (wave >= 1 && j + 1 < nsteps) stage1(b ^ 1);
        // the previous step's energies: sum over the waves in a fixed order
        if (wave == RW && j >= SL) store_energies(j - 1, b ^ 1);

        // ---------------- stage 2: DFT along y of column c = wave -----------------------
        f4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
        {
            const float *src = s1_s[b] + (S * n + g) * S1S + 2 * wave;
#pragma unroll
            for (int kh = 0; kh < KS2 / 4; ++kh) {
                // operands (mt, kk) for kk = 4 kh .. 4 kh + 3
                float4 wm[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) wm[mt] = a2_s[mt * (KS2 / 4) + kh][lane];
                const float2 x0 = *reinterpret_cast<const float2 *>(src + 8 * kh * S1S);
                const float2 x1 = *reinterpret_cast<const float2 *>(src + (8 * kh + 4) * S1S);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma4(wm[mt].x, x0.x, acc[mt]);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma4(wm[mt].y, x0.y, acc[mt]);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma4(wm[mt].z, x1.x, acc[mt]);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma4(wm[mt].w, x1.y, acc[mt]);
            }
        }

        // ---------------- stage 3: the t update -----------------------------------------
        const int v = (s_start - SH + j) & (SL - 1);
        const float sh = (v & 1) ? -1.f : 1.f;  // the twiddle of kt = L/2
        // (from LDS: a scalar load in flight would make every LDS wait of the step wait for it)
        float2 w[SH];
#pragma unroll
        for (int kt = 1; kt < SH; ++kt) w[kt] = tw_s[(kt * v) & (SL - 1)];
        // D[kt] += lo w(kt), D[L - kt] += hi conj(w(kt)), D[0] += self, D[L/2] += self sh; each
        // product rounded before it is added
        auto update = [&](int mt, int q, float2 lo, float2 hi, float2 self) __attribute__((always_inline)) {
            Dr[mt][q][0] += self.x;
            Di[mt][q][0] += self.y;
            Dr[mt][q][SH] = fmaf(sh, self.x, Dr[mt][q][SH]);
            Di[mt][q][SH] = fmaf(sh, self.y, Di[mt][q][SH]);
#pragma unroll
            for (int kt = 1; kt < SH; ++kt) {
                const float wr = w[kt].x, wi = w[kt].y;
                const float b1 = lo.y * wi, d1 = lo.y * wr;
                Dr[mt][q][kt] += fmaf(lo.x, wr, -b1);
                Di[mt][q][kt] += fmaf(lo.x, wi, d1);
                const float b2 = hi.y * wi, d2 = hi.y * wr;
                Dr[mt][q][SL - kt] += fmaf(hi.x, wr, b2);
                Di[mt][q][SL - kt] += fmaf(-hi.x, wi, d2);
            }
        };
        const int t0 = s_start + j - (SL - 1);
        const bool out = j >= SL - 1 && t0 >= t_lo && (t0 - bx.o0) % S == 0;
        // Slot inputs.  Columns 1..L/2-1: the plane spectrum itself.  Column 0: U = P_a +
        // conj P_b and V = P_a - conj P_b for the rows (a, b = -a); on the self-conjugate rows
        // (lane group 0 of M tile 0) Z itself at kt in {0, L/2}, 2 Re Z at kt = 1..L/2-1 (U)
        // and -2i Im Z at kt = L/2+1..L-1 (conj V).  One update code for all waves keeps the
        // spectrum registers in place.
        {
            const bool w0 = wave == 0;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const float2 pa = make_float2(acc[mt][0], acc[mt][1]), pb = make_float2(acc[mt][2], acc[mt][3]);
                const float2 u = make_float2(pa.x + pb.x, pa.y - pb.y), vv = make_float2(pa.x - pb.x, pa.y + pb.y);
                if (mt >= 1) {
                    const float2 p0 = w0 ? u : pa, p1 = w0 ? vv : pb;
                    update(mt, 0, p0, p0, p0);
                    update(mt, 1, p1, p1, p1);
                } else if (w0) {
                    const float2 se0 = sp_lane ? pa : u, se1 = sp_lane ? pb : vv;
                    const float2 lo0 = sp_lane ? make_float2(2.f * pa.x, 0.f) : se0;
                    const float2 hi0 = sp_lane ? make_float2(0.f, -2.f * pa.y) : se0;
                    const float2 lo1 = sp_lane ? make_float2(2.f * pb.x, 0.f) : se1;
                    const float2 hi1 = sp_lane ? make_float2(0.f, -2.f * pb.y) : se1;
                    update(0, 0, lo0, hi0, se0);
                    update(0, 1, lo1, hi1, se1);
                } else {
                    update(0, 0, pa, pa, pa);
                    update(0, 1, pb, pb, pb);
                }
            }
        }
        float e[3] = {0.f, 0.f, 0.f};
        if (out && wave != 0) {
            // M tile 0: the ky of the two slots differ in lane group 0 (0 and L/2): a weight
            // set per slot; M tile 1: ky and -ky, one set.  kt and L - kt share weights.
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                float m0[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    m0[q] = mag(Dr[0][q][p], Di[0][q][p]);
                    if (p > 0 && p < SH) m0[q] += mag(Dr[0][q][SL - p], Di[0][q][SL - p]);
                }
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    e[m] = fmaf(wl[3 * NP + 3 * p + m], m0[1], fmaf(wl[3 * p + m], m0[0], e[m]));
#pragma unroll
                for (int mt = 1; mt < MT; ++mt) {
                    float m1 = mag(Dr[mt][0][p], Di[mt][0][p]) + mag(Dr[mt][1][p], Di[mt][1][p]);
                    if (p > 0 && p < SH)
                        m1 += mag(Dr[mt][0][SL - p], Di[mt][0][SL - p]) + mag(Dr[mt][1][SL - p], Di[mt][1][SL - p]);
#pragma unroll
                    for (int m = 0; m < 3; ++m) e[m] = fmaf(wl[6 * NP + 3 * p + m], m1, e[m]);
                }
            }
        } else if (out) {
            // M tile 0: weights A (slot kt) and B (slot L - kt) per ky slot; at kt in {0, L/2}
            // A weighs |Re Z| and B |Im Z| on the self-conjugate rows, A the magnitude
            // elsewhere.  M tile 1: one set per ky slot.
            const float sel = sp_lane ? 0.f : 1.f;
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    float ma, mb;
                    if (p == 0 || p == SH) {
                        const float re = Dr[0][q][p], im = Di[0][q][p];
                        ma = __builtin_amdgcn_sqrtf(fmaf(re, re, sel * im * im));
                        mb = fabsf(im);
                    } else {
                        ma = mag(Dr[0][q][p], Di[0][q][p]);
                        mb = mag(Dr[0][q][SL - p], Di[0][q][SL - p]);
                    }
                    const float *wa = wl + (q * NP + p) * 6;
#pragma unroll
                    for (int m = 0; m < 3; ++m) e[m] = fmaf(wa[3 + m], mb, fmaf(wa[m], ma, e[m]));
#pragma unroll
                    for (int mt = 1; mt < MT; ++mt) {
                        float m1 = mag(Dr[mt][q][p], Di[mt][q][p]);
                        if (p > 0 && p < SH) m1 += mag(Dr[mt][q][SL - p], Di[mt][q][SL - p]);
                        const float *wm = wl + 12 * NP + (q * NP + p) * 3;
#pragma unroll
                        for (int m = 0; m < 3; ++m) e[m] = fmaf(wm[m], m1, e[m]);
                    }
                }
        }
        if (out) {
            // lanes n, n + 16, n + 32, n + 48 hold the same window
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                float s = e[m];
                s += __shfl_xor(s, 16);
                s += __shfl_xor(s, 32);
                if (g == 0) red_s[b][wave][m][n] = s;
            }
        }
    }
    __syncthreads();
    if (wave == RW) store_energies(nsteps - 1, (nsteps - 1) & 1);
    // max |V| of everything this workgroup read (all of it lies in the volume)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    if (lane == 0) vred_s[wave] = vmax;
    __syncthreads();
    if (threadIdx.x == 0 && vmax_part) {
        float m = vred_s[0];
        for (int w = 1; w < SNW; ++w) m = fmaxf(m, vred_s[w]);
        vmax_part[blockIdx.x] = m;
    }
}

// ====================================================================== launcher

// Segments of the t walk (window rows [slide_seg_start(k), slide_seg_start(k + 1)))
// touched by the box rows [o0, o0 + d0); the grid covers the most any box of the batch needs.
static int slide_nseg(int o0, int d0, int r) { return slide_seg_id(o0 + d0 - 1, r) - slide_seg_id(o0, r) + 1; }

int64_t energy_slide_num_blocks(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2)
{
    const int64_t S = c->p.stride, k1 = (n1 + S - 1) / S, k2 = (n2 + S - 1) / S;
    return (int64_t)slide_nseg(0, (int)n0, c->L / 2) * k1 * ((k2 + STY - 1) / STY);
}

template <int L, int S>
static hipError_t launch_slide_L(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, ebox bx,
                                 float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox)
{
    int nseg;
    if (bx.table)
        nseg = (bx.d0 + SLIDE_SEG - 1) / SLIDE_SEG + 2;  // any o0
    else
        nseg = slide_nseg(bx.o0, bx.d0, L / 2);
    // lattice windows of the box along x, groups of 16 along y
    const int nbx = (bx.d1 + S - 1) / S, nby = ((bx.d2 + S - 1) / S + STY - 1) / STY;
    int64_t nb = (int64_t)nseg * nbx * nby;
    if (bx.table) {
        bx.per_box = (int)nb;
        nb *= nbox;
    }
    if (nparts) *nparts = (int)nb;
    hipLaunchKernelGGL((k_energy_slide<L, S>), dim3((unsigned)nb), dim3(64 * (L / 2)), 0, s, V, (int)n0, (int)n1,
                       (int)n2, bx, nseg, nbx, nby, c->t.w_s1, c->t.w_s2, c->t.w_sp,
                       (const float2 *)c->t.twiddle, E, vmax_part);
    return hipGetLastError();
}

hipError_t launch_energy_slide(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, ebox bx,
                               float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox)
{
#define SAL_SLIDE(LL, SS) \
    if (c->L == LL && c->p.stride == SS) return launch_slide_L<LL, SS>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox)
    SAL_SLIDE(8, 1);
    SAL_SLIDE(8, 2);
    SAL_SLIDE(8, 3);
    SAL_SLIDE(16, 1);
    SAL_SLIDE(16, 2);
    SAL_SLIDE(16, 3);
    SAL_SLIDE(16, 4);
    SAL_SLIDE(16, 5);
    SAL_SLIDE(16, 6);
    SAL_SLIDE(16, 7);
#undef SAL_SLIDE
    return hipErrorInvalidValue;
}
