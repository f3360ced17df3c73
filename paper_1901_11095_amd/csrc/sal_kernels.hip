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
#include <climits>
#include <cstdint>

#include "sal_device.h"
#include "sal_internal.h"

// ------------------------------------------------------------------------------------
// Steps 1-3, FP32.  One workgroup = NW waves owns a tile of NW x-rows by TY y-columns and
// walks t over [t_begin, t_end).  For every t0:
//   stage A (all waves): A[x', y', mu] = sum_p W[mu, p] V[t0 - H + p, x', y'] for the whole
//            (NW + L - 1) x (TY + L - 1) patch, mu <= L/2, MFMA with N = 16 positions (the
//            volume samples of the next t0 are already in flight while this one computes);
//   stage B (wave w, x-row x0 = w): per mu, B[nu, y'] = sum_q W[nu, q] A[x0 + q, y', mu];
//            for mu in {0, L/2} the input is real and the imaginary K steps are skipped;
//   stage C (wave w): per kept (mu, nu) row, F[om, y0] = sum_r W[om, r] B[nu, y0 + r], the
//            window sums of 16 consecutive voxels as one 16x16 tile (y0 on N, (om, re|im)
//            on M) that never leaves the accumulators; each lane turns its two complex bins
//            into magnitudes and folds them with the projection weights into E_t, E_x, E_y.
// Rows (mu, nu) with mu in {0, L/2} keep nu <= L/2 only: the other bins are complex
// conjugates of kept ones; the weights carry the multiplicity.  For other mu, rows nu and
// L - nu have identical projection weights (they depend on squared frequencies), so their
// magnitudes are summed before weighting: one "group" per (mu, k), k = 0..L/2.
// Floating-point MFMA and VALU work serialise on a SIMD on this chip, so the per-bin VALU
// count (|F|^2, sqrt, three weighted sums) is kept minimal.
template <int L, int S>
__global__ __attribute__((amdgpu_waves_per_eu(S == 1 ? TileCfg<L>::WPE : 2))) __launch_bounds__(64 * TileCfg<L>::NW) void k_energy_f32(
    const float *__restrict__ V, int n0, int n1, int n2, ebox bx, int tt_len, int nby, int nbx,
    const float *__restrict__ w_c, const float *__restrict__ w_a, const float *__restrict__ w_cb,
    const float *__restrict__ w_grp, float *__restrict__ E, float *__restrict__ vmax_part)
{
    using G = Geo<L>;
    using C = TileCfg<L>;
    constexpr int H = G::H, h = G::h, KS = G::KS, MT = G::MT, KSA = G::KSA, MTA = G::MTA;
    constexpr int NW = C::NW, TY = C::TY;
    // windows of the x-rows and y-columns S apart (S = 1: every voxel, S = 2: the
    // half-resolution lattice) cover this patch
    constexpr int PX = S * (NW - 1) + L, PY = S * (TY - 1) + L;
    constexpr int NTB = (PY + 15) / 16, PYB = NTB * 16, NTC = TY / 16;
    constexpr int NPOS = PX * PY, NTA = (NPOS + 15) / 16, NJ = (NTA + NW - 1) / NW;
    constexpr int NGK = L / 2 + 1;  // groups per mu
    // cube 16: the stage-C matrix rows are ordered so that lane group g of M tile 0 holds the
    // bins om and L - om (equal weights); stage B has its own matrix (the halves' table)
    constexpr bool FOLD = L == 16;
    constexpr int NWB = C::W_LDS ? h * NGK * MT * 32 : 1;

    // At cube 16, stage B runs in two halves of eight frequency rows, each followed by the
    // stage C of the weight groups whose rows it holds, so B_s keeps eight rows at a time
    // and two workgroups fit a CU.  The stage-B matrix of the halves (rows in the halves'
    // order) is read from LDS when used.
    constexpr int NH = L == 16 ? 2 : 1, NROW = NH > 1 ? 8 : L;
    __shared__ float2 A_s[NPOS * h];
    __shared__ float2 B_s[NW][NROW * PYB];
    __shared__ float wcb_s[NH > 1 ? NH * KS * 64 : 1];
    __shared__ float wb_s[NWB];
    __shared__ float wa_s[16 * MTA * L];
    __shared__ float red_s[NW];

    // the wave index is uniform: kept in a scalar register, so per-wave offsets are scalar
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, n = lane & 15;

    int box;
    const int tile = box_tile(bx, &box);
    V += box * bx.vstride;
    E += box * bx.estride;
    const int ty = tile % nby, tx = (tile / nby) % nbx, tb = tile / (nby * nbx);
    const int y_base = bx.o2 + S * ty * TY, x_base = bx.o1 + S * tx * NW;
    const int t_begin = bx.o0 + S * tb * tt_len;
    const int t_end = min(bx.o0 + bx.d0, t_begin + S * tt_len);
    if (t_begin >= t_end || x_base >= bx.o1 + bx.d1 || y_base >= bx.o2 + bx.d2) {
        // past a box smaller than the grid's (batched boxes): nothing to compute
        if (threadIdx.x == 0 && vmax_part) vmax_part[blockIdx.x] = 0.f;
        return;
    }
    // E frame (the box itself unless a batch entry says otherwise)
    const int K1 = bx.fk1, K2 = bx.fk2;

    // constant MFMA A-operands: lane (g, n) holds row n of each M tile at K = KS*g + kk
    float wc[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) wc[mt][kk] = w_c[(16 * mt + n) * (2 * L) + KS * g + kk];
    // the stage-A matrix is read from LDS when used (it is needed once per t0 only)
    for (int i = threadIdx.x; i < 16 * MTA * L; i += 64 * NW) wa_s[i] = w_a[i];
    if (NH > 1)
        for (int i = threadIdx.x; i < NH * KS * 64; i += 64 * NW) wcb_s[i] = w_cb[i];
    if (C::W_LDS)
        for (int i = threadIdx.x; i < NWB; i += 64 * NW) wb_s[i] = w_grp[i];

    const int n12 = n1 * n2;  // the volume holds at most 2^31 - 1 samples
    const int64_t nbox = (int64_t)bx.fk0 * K1 * K2;
    float vmax = 0.0f;
    float2 *Bw = B_s[wave];

    // Volume samples of the stage-A positions of this wave for one t0.  The loads for the
    // next t0 are issued after stage C, so they hold no registers through stages B and C.
    // The 32-bit position offsets are kept; the row offsets of the lane's taps are formed
    // once per t0 and each load adds the two.
    int off_xy[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int pos = min((wave + NW * jj) * 16 + n, NPOS - 1);
        const int xp = pos / PY, yp = pos - xp * PY;
        off_xy[jj] = refl_idx(x_base - H + xp, n1) * n2 + refl_idx(y_base - H + yp, n2);
    }
    float vnext[NJ][KSA];
    auto load_a = [&](int t0) {
        int rowo[KSA];
#pragma unroll
        for (int kk = 0; kk < KSA; ++kk) rowo[kk] = refl_idx(t0 - H + KSA * g + kk, n0) * n12;
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int off = opaque(off_xy[jj]);
#pragma unroll
            for (int kk = 0; kk < KSA; ++kk)
                vnext[jj][kk] = (wave + NW * jj < NTA) ? V[(uint32_t)(rowo[kk] + off)] : 0.f;
        }
    };
    load_a(t_begin);

    for (int t0 = t_begin; t0 < t_end; t0 += S) {
        __syncthreads();  // previous t0 is done with A_s
        float vcur[NJ][KSA];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
            for (int kk = 0; kk < KSA; ++kk) vcur[jj][kk] = vnext[jj][kk];
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
                    const float v = vcur[jj][kk];
                    vmax = fmaxf(vmax, fabsf(v));
#pragma unroll
                    for (int mt = 0; mt < MTA; ++mt)
                        acc[mt] = mfma4(wa_s[(16 * mt + n) * L + KSA * g + kk], v, acc[mt]);
                }
                const int pos = tl * 16 + opaque(n);
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
#pragma unroll 1
        for (int mu = 0; mu < h; ++mu) {
            const bool self = (mu == 0 || mu == L / 2);  // real stage-A output
#pragma unroll 1
            for (int hp = 0; hp < NH; ++hp) {
                // ---------- stage B: complex DFT along x for this mu (rows of half hp) ------
                // one pass: row nu at position nu; halves: position i holds the i-th frequency
                // of the half's list (the matrix rows of w_cb are ordered the same way)
                constexpr int BT = NH > 1 ? 1 : MT;  // M tiles per pass
#pragma unroll
                for (int nb = 0; nb < NTB; ++nb) {
                    const int yp = min(nb * 16 + n, PY - 1);
                    f4 acc[BT];
#pragma unroll
                    for (int mt = 0; mt < BT; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
                    auto wstage = [&](int mt, int kk) -> float {
                        return NH > 1 ? wcb_s[(hp * KS + kk) * 64 + lane] : wc[mt][kk];
                    };
                    if (self) {
#pragma unroll
                        for (int kk = 0; kk < KS; kk += 2) {
                            const float a = A_s[((S * wave + ((KS * g + kk) >> 1)) * PY + yp) * h + mu].x;
#pragma unroll
                            for (int mt = 0; mt < BT; ++mt) acc[mt] = mfma4(wstage(mt, kk), a, acc[mt]);
                        }
                    } else {
#pragma unroll
                        for (int kk = 0; kk < KS; kk += 2) {
                            const float2 a = A_s[((S * wave + ((KS * g + kk) >> 1)) * PY + yp) * h + mu];
#pragma unroll
                            for (int mt = 0; mt < BT; ++mt) {
                                acc[mt] = mfma4(wstage(mt, kk), a.x, acc[mt]);
                                acc[mt] = mfma4(wstage(mt, kk + 1), a.y, acc[mt]);
                            }
                        }
                    }
#pragma unroll
                    for (int mt = 0; mt < BT; ++mt) {
                        const int nu0 = 8 * mt + 2 * g;
                        Bw[nu0 * PYB + nb * 16 + n] = make_float2(acc[mt][0], acc[mt][1]);
                        Bw[(nu0 + 1) * PYB + nb * 16 + n] = make_float2(acc[mt][2], acc[mt][3]);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // ---------- stage C: complex DFT along y, projections, energies -------------
                // weight group (mu, k) of entry ei of the pass: rows nu = k at position pa and,
                // unless mu is 0 or L/2 or k is 0 or L/2, nu = L - k at position pb.  The NTC
                // voxel tiles of a row run as independent MFMA chains, interleaved, so each
                // tile's dependent steps and result latency overlap the other tiles'.
                const int nent = NH == 1 ? NGK : (hp == 0 ? 5 : 4);
#pragma unroll 1
                for (int ei = 0; ei < nent; ++ei) {
                    int k, pa, pb;
                    if (NH == 1) {
                        k = ei;
                        pa = ei;
                        pb = L - ei;
                    } else if (hp == 0) {
                        k = ei < 4 ? ei : 8;
                        pa = ei == 0 ? 0 : (ei < 4 ? 2 * ei - 1 : 7);
                        pb = 2 * ei;
                    } else {
                        k = 4 + ei;
                        pa = 2 * ei;
                        pb = 2 * ei + 1;
                    }
                    const int grp = mu * NGK + k;
                    const bool pair = !self && k > 0 && k < L / 2;
                    // for mu, nu in {0, L/2} the stage-B row is real (the quarter-turn twiddles
                    // are exact, so its imaginary part is an exact zero): skip those K steps
                    const bool real_row = self && (k == 0 || k == L / 2);
                    // weights of the group: a uniform base (scalar register) plus the
                    // lane's fixed offset; a folded tile needs three per lane
                    float wv[MT][6];
                    const float *wgp = C::W_LDS ? wb_s + grp * (MT * 32) : w_grp + grp * (MT * 32);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int q = 0; q < 6; ++q)
                            wv[mt][q] = (FOLD && mt == 0 && q >= 3) ? 0.f : wgp[(mt * 4 + g) * 8 + q];
                    f4 acc[NTC][MT];
                    auto row_dft = [&](int pos, bool real) {
#pragma unroll
                        for (int c = 0; c < NTC; ++c)
#pragma unroll
                            for (int mt = 0; mt < MT; ++mt) acc[c][mt] = f4{0.f, 0.f, 0.f, 0.f};
                        const float2 *Brow = Bw + pos * PYB + S * n + ((KS * g) >> 1);
                        if (real) {
#pragma unroll
                            for (int kk = 0; kk < KS; kk += 2)
#pragma unroll
                                for (int c = 0; c < NTC; ++c) {
                                    const float b = Brow[S * c * 16 + (kk >> 1)].x;
#pragma unroll
                                    for (int mt = 0; mt < MT; ++mt) acc[c][mt] = mfma4(wc[mt][kk], b, acc[c][mt]);
                                }
                        } else {
#pragma unroll
                            for (int kk = 0; kk < KS; kk += 2) {
                                float2 b[NTC];
#pragma unroll
                                for (int c = 0; c < NTC; ++c) b[c] = Brow[S * c * 16 + (kk >> 1)];
#pragma unroll
                                for (int c = 0; c < NTC; ++c)
#pragma unroll
                                    for (int mt = 0; mt < MT; ++mt) acc[c][mt] = mfma4(wc[mt][kk], b[c].x, acc[c][mt]);
#pragma unroll
                                for (int c = 0; c < NTC; ++c)
#pragma unroll
                                    for (int mt = 0; mt < MT; ++mt)
                                        acc[c][mt] = mfma4(wc[mt][kk + 1], b[c].y, acc[c][mt]);
                            }
                        }
                    };
                    float m0[NTC][MT], m1[NTC][MT];
                    row_dft(pa, real_row);
#pragma unroll
                    for (int c = 0; c < NTC; ++c)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            const f4 a = acc[c][mt];
                            m0[c][mt] = __builtin_amdgcn_sqrtf(fmaf(a[0], a[0], a[1] * a[1]));
                            m1[c][mt] = __builtin_amdgcn_sqrtf(fmaf(a[2], a[2], a[3] * a[3]));
                        }
                    if (pair) {
                        row_dft(pb, false);
#pragma unroll
                        for (int c = 0; c < NTC; ++c)
#pragma unroll
                            for (int mt = 0; mt < MT; ++mt) {
                                const f4 a = acc[c][mt];
                                m0[c][mt] += __builtin_amdgcn_sqrtf(fmaf(a[0], a[0], a[1] * a[1]));
                                m1[c][mt] += __builtin_amdgcn_sqrtf(fmaf(a[2], a[2], a[3] * a[3]));
                            }
                    }
#pragma unroll
                    for (int c = 0; c < NTC; ++c)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            if (FOLD && mt == 0) {
                                // the lane's two bins are om and L - om: one set of weights
                                const float sm = m0[c][mt] + m1[c][mt];
#pragma unroll
                                for (int m = 0; m < 3; ++m) e[c][m] = fmaf(wv[mt][m], sm, e[c][m]);
                            } else {
#pragma unroll
                                for (int m = 0; m < 3; ++m)
                                    e[c][m] = fmaf(wv[mt][3 + m], m1[c][mt], fmaf(wv[mt][m], m0[c][mt], e[c][m]));
                            }
                        }
                }
                // the next pass's stage B overwrites B_s
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        if (t0 + S < t_end) load_a(t0 + S);
        // reduce the four lane groups (lanes n, n+16, n+32, n+48 hold the same voxel)
        const int x = x_base + S * wave;
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                float s = e[c][m];
                s += __shfl_xor(s, 16);
                s += __shfl_xor(s, 32);
                e[c][m] = s;
            }
            const int y = y_base + S * (c * 16 + opaque(n));
            if (g == 0 && x < bx.o1 + bx.d1 && y < bx.o2 + bx.d2) {
                const int64_t o = ((int64_t)((t0 - bx.fo0) / S) * K1 + (x - bx.fo1) / S) * K2 + (y - bx.fo2) / S;
                E[o] = e[c][0];
                E[nbox + o] = e[c][1];
                E[2 * nbox + o] = e[c][2];
            }
        }
    }
    // max |V| of everything this workgroup read (all of it lies in the volume)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    if (lane == 0) red_s[wave] = vmax;
    __syncthreads();
    if (threadIdx.x == 0 && vmax_part) {
        float m = red_s[0];
        for (int w = 1; w < NW; ++w) m = fmaxf(m, red_s[w]);
        vmax_part[blockIdx.x] = m;
    }
}

// ------------------------------------------------------------------------------------
// Step 4, Eq. (5): grid-stride over voxels, one voxel per thread and trip; neighbours are
// read through the caches.  The bounded grid keeps the min/max partials few.  Handles every
// ray of the 26-neighbourhood (the oriented comparisons of Fig. 3): each coordinate of a
// neighbour is reflected at the volume faces, and the weight is the Gaussian of its
// Euclidean distance s |e|.  Sums run over the ray bits in order, then the steps.
__global__ __launch_bounds__(256) void k_dcs(const float *__restrict__ E, int n0, int n1, int n2,
                                             dcs_args a, float *__restrict__ S,
                                             float *__restrict__ mm_part)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < N; v += (int64_t)gridDim.x * 256) {
        const int y = (int)(v % n2);
        const int64_t rest = v / n2;
        const int x = (int)(rest % n1);
        const int t = (int)(rest / n1);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const float *Em = E + m * N;
            const float c = Em[v];
            float sum = 0.f;
            for (int b = 0; b < 26; ++b) {
                if (!((a.rays[m] >> b) & 1u)) continue;
                int dt, dx, dy;
                ray_step(b, dt, dx, dy);
                const float *gw = a.g + 32 * (dt * dt + dx * dx + dy * dy - 1);
                for (int s = 1; s <= a.r; ++s) {
                    const int ut = refl_idx(t + dt * s, n0), ux = refl_idx(x + dx * s, n1),
                              uy = refl_idx(y + dy * s, n2);
                    sum += fabsf(c - gw[s - 1] * Em[((int64_t)ut * n1 + ux) * n2 + uy]);
                }
            }
            const float sv = a.Q[m] > 0.f ? sum / a.Q[m] : 0.f;
            S[m * N + v] = sv;
            mn[m] = fminf(mn[m], sv);
            mx[m] = fmaxf(mx[m], sv);
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
// Strided windows: energies on the lattice of stride S (El [3][K0][K1][K2], positions k S)
// interpolated trilinearly onto every voxel; beyond the last lattice point of an axis the
// last value is held.  Corners are summed in the order (t, x, y) = 000, 001, ..., 111.
// Lattice energies to voxel energies (windows on the stride-S lattice): E at voxel u is the
// trilinear interpolation of the lattice values at floor(u/S) and the next lattice point
// along each axis (the last one held past the last lattice point, K = ceil(n/S) of the
// volume), the weights (u - kS)/S being exact.  El holds the lattice points klo + [0, kd)
// of the volume; E receives the voxels eo + [0, ed) box-local, [3][ed0][ed1][ed2].
struct lat_box {
    int kd0, kd1, kd2, klo0, klo1, klo2, K0, K1, K2, eo0, eo1, eo2, ed0, ed1, ed2;
};
static_assert(sizeof(lat_box) == LAT_TABLE * sizeof(int), "lat_box is one table entry");

// voxel (t, x, y) of the volume, box-local index v of the box b, from the lattice energies
// El of b
__device__ __forceinline__ void upsample_voxel(const float *__restrict__ El, const lat_box &b, int S, float inv,
                                               int t, int x, int y, int64_t v, int64_t N, int64_t NK,
                                               float *__restrict__ E)
{
    const int kt = t / S, kx = x / S, ky = y / S;
    const int kt1 = min(kt + 1, b.K0 - 1), kx1 = min(kx + 1, b.K1 - 1), ky1 = min(ky + 1, b.K2 - 1);
    const float ft = kt1 == kt ? 0.f : (float)(t - kt * S) * inv;
    const float fx = kx1 == kx ? 0.f : (float)(x - kx * S) * inv;
    const float fy = ky1 == ky ? 0.f : (float)(y - ky * S) * inv;
    const int at = kt - b.klo0, ax = kx - b.klo1, ay = ky - b.klo2;
    const int at1 = kt1 - b.klo0, ax1 = kx1 - b.klo1, ay1 = ky1 - b.klo2;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const float *P = El + m * NK;
        float acc = 0.f;
#pragma unroll
        for (int corner = 0; corner < 8; ++corner) {
            const int ht = (corner >> 2) & 1, hx = (corner >> 1) & 1, hy = corner & 1;
            const float w = (ht ? ft : 1.f - ft) * (hx ? fx : 1.f - fx) * (hy ? fy : 1.f - fy);
            acc = fmaf(w, P[((int64_t)(ht ? at1 : at) * b.kd1 + (hx ? ax1 : ax)) * b.kd2 + (hy ? ay1 : ay)], acc);
        }
        E[m * N + v] = acc;
    }
}

// voxel v (box-local index) of the box b
__device__ __forceinline__ void upsample_at(const float *__restrict__ El, const lat_box &b, int S, float inv,
                                            int64_t v, int64_t N, int64_t NK, float *__restrict__ E)
{
    const int y = b.eo2 + (int)(v % b.ed2);
    const int64_t rest = v / b.ed2;
    const int x = b.eo1 + (int)(rest % b.ed1), t = b.eo0 + (int)(rest / b.ed1);
    upsample_voxel(El, b, S, inv, t, x, y, v, N, NK, E);
}

// One box (the whole volume): a workgroup takes rows (t, x) of the box, its threads the
// voxels along y, so no voxel index is divided (the same arithmetic per voxel as
// upsample_at).  (Giving each workgroup a run of consecutive rows instead measured slower.)
__global__ __launch_bounds__(256) void k_upsample(const float *__restrict__ El, lat_box b, int S,
                                                  float *__restrict__ E)
{
    const int64_t N = (int64_t)b.ed0 * b.ed1 * b.ed2, NK = (int64_t)b.kd0 * b.kd1 * b.kd2;
    const float inv = 1.0f / (float)S;
    const int nrows = b.ed0 * b.ed1;
    for (int row = blockIdx.x; row < nrows; row += gridDim.x) {
        const int tl = row / b.ed1, xl = row - tl * b.ed1;
        for (int yl = threadIdx.x; yl < b.ed2; yl += 256)
            upsample_voxel(El, b, S, inv, b.eo0 + tl, b.eo1 + xl, b.eo2 + yl, (int64_t)row * b.ed2 + yl, N, NK, E);
    }
}

// The same for the tiles of a batch: workgroups [i * per_box, (i + 1) * per_box) serve box
// i, whose lat_box is entry i of the table (LAT_TABLE ints), its lattice energies at
// El + i * lstride and its voxel energies at E + i * estride.
__global__ __launch_bounds__(256) void k_upsample_boxes(const float *__restrict__ El, int64_t lstride,
                                                        const int *__restrict__ table, int per_box, int S,
                                                        float *__restrict__ E, int64_t estride)
{
    const int i = blockIdx.x / per_box, blk = blockIdx.x - i * per_box;
    const int *q = table + LAT_TABLE * i;
    const lat_box b{q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], q[8], q[9], q[10], q[11], q[12], q[13], q[14]};
    const int64_t N = (int64_t)b.ed0 * b.ed1 * b.ed2, NK = (int64_t)b.kd0 * b.kd1 * b.kd2;
    const float inv = 1.0f / (float)S;
    El += i * lstride;
    E += i * estride;
    for (int64_t v = (int64_t)blk * 256 + threadIdx.x; v < N; v += (int64_t)per_box * 256)
        upsample_at(El, b, S, inv, v, N, NK, E);
}

// ------------------------------------------------------------------------------------
// Step 4, Eq. (5) on a box of the volume: E is given on the box grown by r (clipped to the
// volume), Eb [3][ed0][ed1][ed2] at origin eo; S_raw of the box positions bo + [0, bd) is
// written box-local [3][bd0][bd1][bd2].  Neighbours are reflected at the volume faces and
// then read from the grown box, which holds every such position.  Same order of the sums as
// k_dcs.
// Eq. (5) at position pos of a box: energies Eb of the grown box (origin org, size ed),
// output element i of the box-local maps S[3][nb]
__device__ __forceinline__ void dcs_box_at(const float *__restrict__ Eb, const int org[3], const int ed[3],
                                           const int dims[3], const int pos[3], const dcs_args &a,
                                           float *__restrict__ S, int nb, int i)
{
    const int64_t NE = (int64_t)ed[0] * ed[1] * ed[2];
    const int64_t stride[3] = {(int64_t)ed[1] * ed[2], ed[2], 1};
    const int64_t v = (pos[0] - org[0]) * stride[0] + (pos[1] - org[1]) * stride[1] + (pos[2] - org[2]);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const float *Em = Eb + m * NE;
        const float c = Em[v];
        float sum = 0.f;
        for (int b = 0; b < 26; ++b) {
            if (!((a.rays[m] >> b) & 1u)) continue;
            int st[3];
            ray_step(b, st[0], st[1], st[2]);
            const float *gw = a.g + 32 * (st[0] * st[0] + st[1] * st[1] + st[2] * st[2] - 1);
            for (int s = 1; s <= a.r; ++s) {
                int u[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) u[k] = refl_idx(pos[k] + st[k] * s, dims[k]) - org[k];
                sum += fabsf(c - gw[s - 1] * Em[u[0] * stride[0] + u[1] * stride[1] + u[2]]);
            }
        }
        S[(int64_t)m * nb + i] = a.Q[m] > 0.f ? sum / a.Q[m] : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_dcs_box(const float *__restrict__ Eb, int3 eo, int3 ed, int3 nv,
                                                 int3 bo, int3 bd, dcs_args a, float *__restrict__ S)
{
    const int nb = bd.x * bd.y * bd.z;
    const int dims[3] = {nv.x, nv.y, nv.z}, org[3] = {eo.x, eo.y, eo.z}, edim[3] = {ed.x, ed.y, ed.z};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < nb; i += gridDim.x * 256) {
        const int pos[3] = {bo.x + i / (bd.y * bd.z), bo.y + (i / bd.z) % bd.y, bo.z + i % bd.z};
        dcs_box_at(Eb, org, edim, dims, pos, a, S, nb, i);
    }
}

// The same for the tiles of a batch: workgroups [b * per_box, (b + 1) * per_box) serve box
// b, whose grown box and tile origin come from its table entry; E of box b starts estride
// floats after that of box b - 1, its maps 3 * |bd| floats after.
__global__ __launch_bounds__(256) void k_dcs_boxes(const float *__restrict__ Eb, int64_t estride,
                                                   const int *__restrict__ table, int per_box, int3 nv,
                                                   int3 bd, dcs_args a, float *__restrict__ S)
{
    const int b = blockIdx.x / per_box, blk = blockIdx.x - b * per_box;
    const int *q = table + BOX_TABLE * b;
    const int org[3] = {q[0], q[1], q[2]}, edim[3] = {q[3], q[4], q[5]}, bo[3] = {q[6], q[7], q[8]};
    const int dims[3] = {nv.x, nv.y, nv.z};
    const int nb = bd.x * bd.y * bd.z;
    Eb += b * estride;
    S += (int64_t)b * 3 * nb;
    for (int i = blk * 256 + threadIdx.x; i < nb; i += per_box * 256) {
        const int pos[3] = {bo[0] + i / (bd.y * bd.z), bo[1] + (i / bd.z) % bd.y, bo[2] + i % bd.z};
        dcs_box_at(Eb, org, edim, dims, pos, a, S, nb, i);
    }
}

// ------------------------------------------------------------------------------------
// Step 4, Eq. (5), tiled: a workgroup owns DTX x DTY voxels in (x, y) and walks DTT values
// of t.  For every component m it keeps in LDS a ring of 2*ht+1 planes of E_m (ht = r if
// m has rays along t, else 0), each plane DTX x DTY plus a halo of r along x (y) when m has
// rays along x (y).  Planes are stored at logical coordinates with the reflection applied
// when they are loaded, so every neighbour of Eq. (5) is a plain LDS read.  With the
// default rays each E value is read from memory about 1.4 times instead of 2r+1 times.
constexpr int DTX = 8, DTY = 32, DTT = 32, DMAXE = 4;

// R = r at compile time (unrolled neighbour loops), or 0 for any r.
template <int R>
__global__ __launch_bounds__(256) void k_dcs_tiled(const float *__restrict__ E, int n0, int n1,
                                                   int n2, dcs_args a, int nbx, int nby,
                                                   float *__restrict__ S,
                                                   float *__restrict__ mm_part)
{
    extern __shared__ float lds[];
    const int64_t plane = (int64_t)n1 * n2, N = plane * n0;
    const int bid = blockIdx.x;
    const int ty = bid % nby, tx = (bid / nby) % nbx, tb = bid / (nby * nbx);
    const int x_base = tx * DTX, y_base = ty * DTY;
    const int t_begin = tb * DTT, t_end = min(n0, t_begin + DTT);
    const int tid = threadIdx.x, lx = tid / DTY, ly = tid % DTY;
    const int x = x_base + lx, y = y_base + ly;
    const bool valid = x < n1 && y < n2;
    const int r = R > 0 ? R : a.r;
    float g[R > 0 ? R : 32];
#pragma unroll
    for (int s = 0; s < (R > 0 ? R : 32); ++s) g[s] = a.g[s];
    const bool diag = ((a.rays[0] | a.rays[1] | a.rays[2]) & ~63u) != 0;

    int ht[3], hx[3], hy[3], W[3], HW[3], depth[3], off[3];
    int o = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        ht[m] = (a.rays[m] & RAYS_T) ? r : 0;
        hx[m] = (a.rays[m] & RAYS_X) ? r : 0;
        hy[m] = (a.rays[m] & RAYS_Y) ? r : 0;
        W[m] = DTY + 2 * hy[m];
        HW[m] = (DTX + 2 * hx[m]) * W[m];
        depth[m] = 2 * ht[m] + 1;
        off[m] = o;
        o += depth[m] * HW[m];
    }
    // this thread's share of every plane: LDS offset and (reflected) volume offset
    int gofs[3][DMAXE];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int e = 0; e < DMAXE; ++e) {
            const int i = tid + 256 * e;
            const int ix = i / W[m], iy = i - ix * W[m];
            gofs[m][e] = i < HW[m] ? refl_idx(x_base - hx[m] + ix, n1) * n2 + refl_idx(y_base - hy[m] + iy, n2) : -1;
        }
    float pv[3][DMAXE];
    auto fetch = [&](int m, int tl) {
        const float *src = E + m * N + (int64_t)refl_idx(tl, n0) * plane;
#pragma unroll
        for (int e = 0; e < DMAXE; ++e) pv[m][e] = gofs[m][e] >= 0 ? src[gofs[m][e]] : 0.f;
    };
    auto store = [&](int m, int tl) {
        float *pl = lds + off[m] + (tl % depth[m]) * HW[m];
#pragma unroll
        for (int e = 0; e < DMAXE; ++e)
            if (gofs[m][e] >= 0) pl[tid + 256 * e] = pv[m][e];
    };
    // planes t_begin - ht .. t_begin + ht - 1 (logical t >= -r; shift by a multiple of
    // depth keeps the slot index non-negative)
#pragma unroll
    for (int m = 0; m < 3; ++m)
        for (int tl = t_begin - ht[m]; tl < t_begin + ht[m]; ++tl) {
            fetch(m, tl);
            store(m, tl + 2 * depth[m]);
        }
#pragma unroll
    for (int m = 0; m < 3; ++m) fetch(m, t_begin + ht[m]);

    float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int t = t_begin; t < t_end; ++t) {
#pragma unroll
        for (int m = 0; m < 3; ++m) store(m, t + ht[m]);
        if (t + 1 < t_end) {
#pragma unroll
            for (int m = 0; m < 3; ++m) fetch(m, t + 1 + ht[m]);
        }
        __syncthreads();
        if (valid) {
            const int64_t ov = ((int64_t)t * n1 + x) * n2 + y;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const uint32_t rm = a.rays[m];
                const float *ring = lds + off[m];
                const int idx = (lx + hx[m]) * W[m] + ly + hy[m];
                const int s0 = t % depth[m];  // slot of plane t; plane t+d sits in s0+d (mod depth)
                const float *cpl = ring + s0 * HW[m] + idx;
                const float c = cpl[0];
                float sum = 0.f;
                if (rm & 1u) {
#pragma unroll
                    for (int s = 1; s <= (R > 0 ? R : 32); ++s) {
                        if (R == 0 && s > r) break;
                        const int sl = s0 + s - (s0 + s >= depth[m] ? depth[m] : 0);
                        sum += fabsf(c - g[s - 1] * ring[sl * HW[m] + idx]);
                    }
                }
                if (rm & 2u) {
#pragma unroll
                    for (int s = 1; s <= (R > 0 ? R : 32); ++s) {
                        if (R == 0 && s > r) break;
                        const int sl = s0 - s + (s0 - s < 0 ? depth[m] : 0);
                        sum += fabsf(c - g[s - 1] * ring[sl * HW[m] + idx]);
                    }
                }
#pragma unroll
                for (int ax = 1; ax < 3; ++ax) {
                    const int step = ax == 1 ? W[m] : 1;
                    if (rm & (4u << (2 * (ax - 1)))) {
#pragma unroll
                        for (int s = 1; s <= (R > 0 ? R : 32); ++s) {
                            if (R == 0 && s > r) break;
                            sum += fabsf(c - g[s - 1] * cpl[s * step]);
                        }
                    }
                    if (rm & (8u << (2 * (ax - 1)))) {
#pragma unroll
                        for (int s = 1; s <= (R > 0 ? R : 32); ++s) {
                            if (R == 0 && s > r) break;
                            sum += fabsf(c - g[s - 1] * cpl[-s * step]);
                        }
                    }
                }
                // oriented rays (face and body diagonals): plane t + s dt of the ring,
                // offset s (dx W + dy) inside it
                if (diag && (rm & ~63u)) {
#pragma unroll 1
                    for (int b = 6; b < 26; ++b) {
                        if (!((rm >> b) & 1u)) continue;
                        int dt, dx, dy;
                        ray_step(b, dt, dx, dy);
                        const float *gw = a.g + 32 * (dt * dt + dx * dx + dy * dy - 1);
                        const int dxy = dx * W[m] + dy;
                        for (int s = 1; s <= r; ++s) {
                            int sl = s0 + dt * s;
                            sl += sl < 0 ? depth[m] : (sl >= depth[m] ? -depth[m] : 0);
                            sum += fabsf(c - gw[s - 1] * ring[sl * HW[m] + idx + s * dxy]);
                        }
                    }
                }
                const float sv = a.Q[m] > 0.f ? sum / a.Q[m] : 0.f;
                S[m * N + ov] = sv;
                mn[m] = fminf(mn[m], sv);
                mx[m] = fmaxf(mx[m], sv);
            }
        }
        __syncthreads();
    }
    if (mm_part == nullptr) return;
    const int lane = tid & 63, wave = tid >> 6;
    float *red = lds;  // reuse: the walk is over
#pragma unroll
    for (int m = 0; m < 3; ++m) {
#pragma unroll
        for (int q = 32; q >= 1; q >>= 1) {
            mn[m] = fminf(mn[m], __shfl_xor(mn[m], q));
            mx[m] = fmaxf(mx[m], __shfl_xor(mx[m], q));
        }
        if (lane == 0) {
            red[wave * 6 + 2 * m] = mn[m];
            red[wave * 6 + 2 * m + 1] = mx[m];
        }
    }
    __syncthreads();
    if (tid < 6) {
        float v = red[tid];
        for (int w = 1; w < 4; ++w) v = (tid & 1) ? fmaxf(v, red[w * 6 + tid]) : fminf(v, red[w * 6 + tid]);
        mm_part[(int64_t)bid * 6 + tid] = v;
    }
}

// Step 4, Eq. (5), for the default rays (map m compared along its own axis, both ways) at a
// compile-time r, on the tiles and t walk of k_dcs_tiled.  Map t compares a voxel with its
// own column along t only: each thread keeps the 2r + 1 values of its column in registers
// and shifts them by one per step.  Maps x and y keep one plane each in LDS with its halo,
// read at constant offsets.  The sums run in the order of k_dcs_tiled and dcs_box_at (the
// + ray before the - ray, s = 1..r), so all three give the same bits.
template <int R>
__global__ __launch_bounds__(256) void k_dcs_axis(const float *__restrict__ E, int n0, int n1, int n2,
                                                  dcs_args a, int nbx, int nby, float *__restrict__ S,
                                                  float *__restrict__ mm_part)
{
    constexpr int D = 2 * R + 1;
    constexpr int W1 = DTY, HW1 = (DTX + 2 * R) * W1;     // map x: halo along x
    constexpr int W2 = DTY + 2 * R, HW2 = DTX * W2;       // map y: halo along y
    constexpr int N1 = (HW1 + 255) / 256, N2 = (HW2 + 255) / 256;
    __shared__ float pl1[HW1];
    __shared__ float pl2[HW2];
    __shared__ float red[4 * 6];

    const int64_t plane = (int64_t)n1 * n2, N = plane * n0;
    const int bid = blockIdx.x;
    const int ty = bid % nby, tx = (bid / nby) % nbx, tb = bid / (nby * nbx);
    const int x_base = tx * DTX, y_base = ty * DTY;
    const int t_begin = tb * DTT, t_end = min(n0, t_begin + DTT);
    const int tid = threadIdx.x, lx = tid / DTY, ly = tid % DTY;
    const int x = x_base + lx, y = y_base + ly;
    const bool valid = x < n1 && y < n2;
    float g[R];
#pragma unroll
    for (int s = 0; s < R; ++s) g[s] = a.g[s];

    // this thread's samples of the x and y planes: volume offset (reflected), or -1
    int o1[N1], o2[N2];
#pragma unroll
    for (int e = 0; e < N1; ++e) {
        const int i = tid + 256 * e, ix = i / W1, iy = i % W1;
        o1[e] = i < HW1 ? refl_idx(x_base - R + ix, n1) * n2 + refl_idx(y_base + iy, n2) : -1;
    }
#pragma unroll
    for (int e = 0; e < N2; ++e) {
        const int i = tid + 256 * e, ix = i / W2, iy = i % W2;
        o2[e] = i < HW2 ? refl_idx(x_base + ix, n1) * n2 + refl_idx(y_base - R + iy, n2) : -1;
    }
    const int o0 = valid ? x * n2 + y : 0;
    float col[D], nxt = 0.f, p1[N1], p2[N2];
    auto at0 = [&](int tl) { return E[(int64_t)refl_idx(tl, n0) * plane + o0]; };
    auto fetch12 = [&](int tl) {
        const float *src1 = E + N + (int64_t)refl_idx(tl, n0) * plane, *src2 = src1 + N;
#pragma unroll
        for (int e = 0; e < N1; ++e) p1[e] = o1[e] >= 0 ? src1[o1[e]] : 0.f;
#pragma unroll
        for (int e = 0; e < N2; ++e) p2[e] = o2[e] >= 0 ? src2[o2[e]] : 0.f;
    };
    // column values t_begin - R .. t_begin + R - 1, then the next one in flight
#pragma unroll
    for (int i = 0; i < D - 1; ++i) col[i] = valid ? at0(t_begin - R + i) : 0.f;
    if (valid) nxt = at0(t_begin + R);
    fetch12(t_begin);

    float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int t = t_begin; t < t_end; ++t) {
        col[D - 1] = nxt;  // plane t + R
#pragma unroll
        for (int e = 0; e < N1; ++e)
            if (o1[e] >= 0) pl1[tid + 256 * e] = p1[e];
#pragma unroll
        for (int e = 0; e < N2; ++e)
            if (o2[e] >= 0) pl2[tid + 256 * e] = p2[e];
        if (t + 1 < t_end) {
            if (valid) nxt = at0(t + 1 + R);
            fetch12(t + 1);
        }
        __syncthreads();
        if (valid) {
            const int64_t ov = ((int64_t)t * n1 + x) * n2 + y;
            float sum[3];
            {   // map t: plane t + d in col[R + d]
                const float c = col[R];
                float su = 0.f;
#pragma unroll
                for (int s = 1; s <= R; ++s) su += fabsf(c - g[s - 1] * col[R + s]);
#pragma unroll
                for (int s = 1; s <= R; ++s) su += fabsf(c - g[s - 1] * col[R - s]);
                sum[0] = su;
            }
            {   // map x
                const float *b = pl1 + (lx + R) * W1 + ly;
                const float c = b[0];
                float su = 0.f;
#pragma unroll
                for (int s = 1; s <= R; ++s) su += fabsf(c - g[s - 1] * b[s * W1]);
#pragma unroll
                for (int s = 1; s <= R; ++s) su += fabsf(c - g[s - 1] * b[-s * W1]);
                sum[1] = su;
            }
            {   // map y
                const float *b = pl2 + lx * W2 + ly + R;
                const float c = b[0];
                float su = 0.f;
#pragma unroll
                for (int s = 1; s <= R; ++s) su += fabsf(c - g[s - 1] * b[s]);
#pragma unroll
                for (int s = 1; s <= R; ++s) su += fabsf(c - g[s - 1] * b[-s]);
                sum[2] = su;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const float sv = a.Q[m] > 0.f ? sum[m] / a.Q[m] : 0.f;
                S[m * N + ov] = sv;
                mn[m] = fminf(mn[m], sv);
                mx[m] = fmaxf(mx[m], sv);
            }
        }
#pragma unroll
        for (int i = 0; i < D - 1; ++i) col[i] = col[i + 1];
        __syncthreads();
    }
    if (mm_part == nullptr) return;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
#pragma unroll
        for (int q = 32; q >= 1; q >>= 1) {
            mn[m] = fminf(mn[m], __shfl_xor(mn[m], q));
            mx[m] = fmaxf(mx[m], __shfl_xor(mx[m], q));
        }
        if (lane == 0) {
            red[wave * 6 + 2 * m] = mn[m];
            red[wave * 6 + 2 * m + 1] = mx[m];
        }
    }
    __syncthreads();
    if (tid < 6) {
        float v = red[tid];
        for (int w = 1; w < 4; ++w) v = (tid & 1) ? fmaxf(v, red[w * 6 + tid]) : fminf(v, red[w * 6 + tid]);
        mm_part[(int64_t)bid * 6 + tid] = v;
    }
}

// LDS floats the tiled comparison needs for these rays and r, or a huge value when a
// plane does not fit the per-thread element budget.
static int64_t dcs_tiled_lds_floats(const uint32_t rays[3], int r)
{
    int64_t tot = 0;
    for (int m = 0; m < 3; ++m) {
        const int ht = (rays[m] & RAYS_T) ? r : 0, hx = (rays[m] & RAYS_X) ? r : 0, hy = (rays[m] & RAYS_Y) ? r : 0;
        const int64_t hw = (int64_t)(DTX + 2 * hx) * (DTY + 2 * hy);
        if (hw > 256 * DMAXE) return INT64_MAX / 2;
        tot += (2 * ht + 1) * hw;
    }
    return tot;
}
// up to 144 KiB of the 160 KiB a gfx950 workgroup may use
static const int64_t DCS_LDS_MAX_FLOATS = 144 * 1024 / 4;

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

// Same, four consecutive voxels per thread (N divisible by 4, 16-byte aligned maps).
__global__ __launch_bounds__(256) void k_combine4(const float4 *__restrict__ S_raw, int64_t N4,
                                                  const double *__restrict__ stats, double wa,
                                                  double wb, double wc, int normalize,
                                                  double zero_range, float4 *__restrict__ S)
{
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= N4) return;
    const double w[3] = {wa, wb, wc};
    double lo[3], sc[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        lo[m] = normalize ? stats[2 * m] : 0.0;
        const double range = stats[2 * m + 1] - stats[2 * m];
        sc[m] = normalize ? (range > zero_range * stats[6] ? 1.0 / range : 0.0) : 1.0;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const float4 x = S_raw[m * N4 + v];
        acc[0] += w[m] * (((double)x.x - lo[m]) * sc[m]);
        acc[1] += w[m] * (((double)x.y - lo[m]) * sc[m]);
        acc[2] += w[m] * (((double)x.z - lo[m]) * sc[m]);
        acc[3] += w[m] * (((double)x.w - lo[m]) * sc[m]);
    }
    S[v] = make_float4((float)acc[0], (float)acc[1], (float)acc[2], (float)acc[3]);
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

// grid of one box (nbox > 1: the t walk is sized for that many boxes in one launch)
template <int L>
static void energy_grid(int64_t n0, int64_t n1, int64_t n2, int *nby, int *nbx, int *tt, int64_t *nblk,
                        int64_t nbox = 1)
{
    using C = TileCfg<L>;
    *nby = (int)((n2 + C::TY - 1) / C::TY);
    *nbx = (int)((n1 + C::NW - 1) / C::NW);
    *tt = tt_len_for(n0, (int64_t)(*nby) * (*nbx) * nbox);
    *nblk = (int64_t)(*nby) * (*nbx) * ((n0 + *tt - 1) / *tt);
}

int64_t energy_num_blocks(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2)
{
    // the grid covers the window positions: every voxel, or the stride-S lattice
    const int S = c->p.stride;
    const int64_t k0 = (n0 + S - 1) / S, k1 = (n1 + S - 1) / S, k2 = (n2 + S - 1) / S;
    int nby, nbx, tt;
    int64_t nb;
    if (uses_slide_kernel(c, n0, n1, n2)) return energy_slide_num_blocks(c, n0, n1, n2);
    if (uses_window_kernel(c)) return energy_win_num_blocks(c, k0, k1, k2);
    if (c->L == 8)
        energy_grid<8>(k0, k1, k2, &nby, &nbx, &tt, &nb);
    else if (c->L == 16)
        energy_grid<16>(k0, k1, k2, &nby, &nbx, &tt, &nb);
    else
        nb = energy_gen_num_blocks(c->L, k0, k1, k2);
    return nb;
}

template <int L>
static hipError_t launch_energy_L(const sal_ctx *c, const float *V, int64_t n0, int64_t n1,
                                  int64_t n2, ebox bx, float *E, float *vmax_part,
                                  int *nparts, hipStream_t s, int nbox = 1)
{
    const int S = c->p.stride;
    int nby, nbx, tt;
    int64_t nb;
    energy_grid<L>((bx.d0 + S - 1) / S, (bx.d1 + S - 1) / S, (bx.d2 + S - 1) / S, &nby, &nbx, &tt, &nb, nbox);
    if (bx.table) {
        bx.per_box = (int)nb;
        nb *= nbox;
    }
    if (nparts) *nparts = (int)nb;
    if (c->p.precision != SAL_FP32)
        return launch_energy16(c, V, n0, n1, n2, bx, E, vmax_part, nby, nbx, tt, nb, s);
    if (S == 2)
        hipLaunchKernelGGL((k_energy_f32<L, 2>), dim3((unsigned)nb), dim3(64 * TileCfg<L>::NW), 0, s, V,
                           (int)n0, (int)n1, (int)n2, bx, tt, nby, nbx, c->t.w_c, c->t.w_a, c->t.w_cb, c->t.w_bin, E,
                           vmax_part);
    else
        hipLaunchKernelGGL((k_energy_f32<L, 1>), dim3((unsigned)nb), dim3(64 * TileCfg<L>::NW), 0, s, V,
                           (int)n0, (int)n1, (int)n2, bx, tt, nby, nbx, c->t.w_c, c->t.w_a, c->t.w_cb, c->t.w_bin, E,
                           vmax_part);
    return hipGetLastError();
}

hipError_t launch_energy(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                         const int64_t *box, float *E, float *vmax_part, int *nparts,
                         hipStream_t s)
{
    const int S = c->p.stride;
    ebox bx = box ? framed_box((int)box[0], (int)box[1], (int)box[2], (int)box[3], (int)box[4], (int)box[5], S)
                  : framed_box(0, 0, 0, (int)n0, (int)n1, (int)n2, S);
    if (uses_slide_kernel(c, n0, n1, n2)) return launch_energy_slide(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s);
    if (uses_window_kernel(c)) return launch_energy_win(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s);
    if (c->L == 8) return launch_energy_L<8>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s);
    if (c->L == 16) return launch_energy_L<16>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s);
    return launch_energy_gen(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s);
}

hipError_t launch_energy_boxes(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                               int64_t vstride, const int *table, int nbox, const int64_t maxd[3], float *E,
                               int64_t estride, float *vmax_part, int *nparts, hipStream_t s)
{
    ebox bx{0, 0, 0, (int)maxd[0], (int)maxd[1], (int)maxd[2]};
    bx.table = table;
    bx.vstride = vstride;
    bx.estride = estride;
    if (uses_slide_kernel(c, n0, n1, n2))
        return launch_energy_slide(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    if (uses_window_kernel(c)) return launch_energy_win(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    if (c->L == 8) return launch_energy_L<8>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    if (c->L == 16) return launch_energy_L<16>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    return launch_energy_gen(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
}

int64_t dcs_num_blocks(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2)
{
    if (dcs_tiled_lds_floats(c->p.rays, c->r) <= DCS_LDS_MAX_FLOATS)
        return ((n1 + DTX - 1) / DTX) * ((n2 + DTY - 1) / DTY) * ((n0 + DTT - 1) / DTT);
    const int64_t nb = (n0 * n1 * n2 + 255) / 256;
    return nb < 8192 ? nb : 8192;
}

hipError_t launch_dcs(const sal_ctx *c, const float *E, int64_t n0, int64_t n1, int64_t n2,
                      float *S_raw, float *minmax_part, hipStream_t s)
{
    dcs_args a;
    a.r = c->r;
    for (int m = 0; m < 3; ++m) {
        a.rays[m] = c->p.rays[m];
        a.Q[m] = c->Q[m];
    }
    for (int i = 0; i < 96; ++i) a.g[i] = c->g[i];
    const int64_t nf = dcs_tiled_lds_floats(c->p.rays, c->r);
    const unsigned nb = (unsigned)dcs_num_blocks(c, n0, n1, n2);
    if (nf <= DCS_LDS_MAX_FLOATS) {
        const size_t lds = (size_t)(nf > 24 ? nf : 24) * sizeof(float);
        const int nbx = (int)((n1 + DTX - 1) / DTX), nby = (int)((n2 + DTY - 1) / DTY);
        // the default rays at a compile-time r: constant LDS offsets
        const bool axis = a.rays[0] == (SAL_RAY_PT | SAL_RAY_MT) && a.rays[1] == (SAL_RAY_PX | SAL_RAY_MX) &&
                          a.rays[2] == (SAL_RAY_PY | SAL_RAY_MY);
#define SAL_DCS_A(RR)                                                                                            \
    case RR:                                                                                                      \
        hipLaunchKernelGGL(k_dcs_axis<RR>, dim3(nb), dim3(256), 0, s, E, (int)n0, (int)n1, (int)n2, a, nbx, nby,  \
                           S_raw, minmax_part);                                                                   \
        return hipGetLastError();
        if (axis) {
            switch (c->r) {
                SAL_DCS_A(1)
                SAL_DCS_A(2)
                SAL_DCS_A(3)
                SAL_DCS_A(4)
                SAL_DCS_A(8)
            default: break;
            }
        }
#undef SAL_DCS_A
#define SAL_DCS_T(RR)                                                                                            \
    do {                                                                                                          \
        if (lds > 65536)                                                                                          \
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_dcs_tiled<RR>),                           \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                      \
        hipLaunchKernelGGL(k_dcs_tiled<RR>, dim3(nb), dim3(256), lds, s, E, (int)n0, (int)n1, (int)n2, a, nbx, nby, \
                           S_raw, minmax_part);                                                                   \
    } while (0)
        // r known at compile time for the default d = L of every supported cube side
        switch (c->r) {
        case 1: SAL_DCS_T(1); break;
        case 2: SAL_DCS_T(2); break;
        case 3: SAL_DCS_T(3); break;
        case 4: SAL_DCS_T(4); break;
        case 8: SAL_DCS_T(8); break;
        default: SAL_DCS_T(0); break;
        }
#undef SAL_DCS_T
    } else {
        hipLaunchKernelGGL(k_dcs, dim3(nb), dim3(256), 0, s, E, (int)n0, (int)n1, (int)n2, a,
                           S_raw, minmax_part);
    }
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
    if (nvox % 4 == 0) {
        const int64_t n4 = nvox / 4;
        hipLaunchKernelGGL(k_combine4, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const float4 *>(S_raw), n4, stats, a, b, c, normalize,
                           zero_range, reinterpret_cast<float4 *>(S));
        return hipGetLastError();
    }
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
#define SAL_SPECTRA(LL)                                                                                        \
    hipLaunchKernelGGL(k_local_spectra<LL>, dim3(nb), dim3(256), 0, s, V, (int)n0, (int)n1, (int)n2, (int)lo[0], \
                       (int)lo[1], (int)lo[2], (int)bn[1], (int)bn[2], tw, o)
    switch (c->L) {
    case 2: SAL_SPECTRA(2); break;
    case 3: SAL_SPECTRA(3); break;
    case 4: SAL_SPECTRA(4); break;
    case 5: SAL_SPECTRA(5); break;
    case 6: SAL_SPECTRA(6); break;
    case 7: SAL_SPECTRA(7); break;
    case 8: SAL_SPECTRA(8); break;
    case 9: SAL_SPECTRA(9); break;
    case 10: SAL_SPECTRA(10); break;
    case 11: SAL_SPECTRA(11); break;
    case 12: SAL_SPECTRA(12); break;
    case 13: SAL_SPECTRA(13); break;
    case 14: SAL_SPECTRA(14); break;
    case 15: SAL_SPECTRA(15); break;
    case 16: SAL_SPECTRA(16); break;
    case 17: SAL_SPECTRA(17); break;
    case 18: SAL_SPECTRA(18); break;
    case 19: SAL_SPECTRA(19); break;
    case 20: SAL_SPECTRA(20); break;
    default: return hipErrorInvalidValue;
    }
#undef SAL_SPECTRA
    return hipGetLastError();
}

hipError_t launch_project(const sal_ctx *c, const float *spectra, int64_t nvox, float *E,
                          hipStream_t s)
{
    if (nvox == 0) return hipSuccess;
    const float2 *F = reinterpret_cast<const float2 *>(spectra);
    const float4 *w = reinterpret_cast<const float4 *>(c->t.w_proj);
#define SAL_PROJECT(LL) hipLaunchKernelGGL(k_project<LL>, dim3((unsigned)nvox), dim3(64), 0, s, F, nvox, w, E)
    switch (c->L) {
    case 2: SAL_PROJECT(2); break;
    case 3: SAL_PROJECT(3); break;
    case 4: SAL_PROJECT(4); break;
    case 5: SAL_PROJECT(5); break;
    case 6: SAL_PROJECT(6); break;
    case 7: SAL_PROJECT(7); break;
    case 8: SAL_PROJECT(8); break;
    case 9: SAL_PROJECT(9); break;
    case 10: SAL_PROJECT(10); break;
    case 11: SAL_PROJECT(11); break;
    case 12: SAL_PROJECT(12); break;
    case 13: SAL_PROJECT(13); break;
    case 14: SAL_PROJECT(14); break;
    case 15: SAL_PROJECT(15); break;
    case 16: SAL_PROJECT(16); break;
    case 17: SAL_PROJECT(17); break;
    case 18: SAL_PROJECT(18); break;
    case 19: SAL_PROJECT(19); break;
    case 20: SAL_PROJECT(20); break;
    default: return hipErrorInvalidValue;
    }
#undef SAL_PROJECT
    return hipGetLastError();
}

hipError_t launch_dcs_box(const sal_ctx *c, const float *Eb, const int64_t eo[3], const int64_t ed[3],
                          const int64_t n[3], const int64_t bo[3], const int64_t bd[3], float *S,
                          hipStream_t s)
{
    dcs_args a;
    a.r = c->r;
    for (int m = 0; m < 3; ++m) {
        a.rays[m] = c->p.rays[m];
        a.Q[m] = c->Q[m];
    }
    for (int i = 0; i < 96; ++i) a.g[i] = c->g[i];
    const int64_t nb = bd[0] * bd[1] * bd[2];
    const unsigned blocks = (unsigned)((nb + 255) / 256 < 4096 ? (nb + 255) / 256 : 4096);
    auto i3 = [](const int64_t *v) { return make_int3((int)v[0], (int)v[1], (int)v[2]); };
    hipLaunchKernelGGL(k_dcs_box, dim3(blocks), dim3(256), 0, s, Eb, i3(eo), i3(ed), i3(n), i3(bo), i3(bd), a,
                       S);
    return hipGetLastError();
}

hipError_t launch_dcs_boxes(const sal_ctx *c, const float *Eb, int64_t estride, const int *table, int nbox,
                            const int64_t n[3], const int64_t bd[3], float *S_box, hipStream_t s)
{
    dcs_args a;
    a.r = c->r;
    for (int m = 0; m < 3; ++m) {
        a.rays[m] = c->p.rays[m];
        a.Q[m] = c->Q[m];
    }
    for (int i = 0; i < 96; ++i) a.g[i] = c->g[i];
    const int64_t nb = bd[0] * bd[1] * bd[2];
    const int per_box = (int)((nb + 255) / 256 < 64 ? (nb + 255) / 256 : 64);
    hipLaunchKernelGGL(k_dcs_boxes, dim3((unsigned)(per_box * nbox)), dim3(256), 0, s, Eb, estride, table,
                       per_box, make_int3((int)n[0], (int)n[1], (int)n[2]),
                       make_int3((int)bd[0], (int)bd[1], (int)bd[2]), a, S_box);
    return hipGetLastError();
}

hipError_t launch_upsample(const float *El, int64_t K0, int64_t K1, int64_t K2, int S, int64_t n0, int64_t n1,
                           int64_t n2, float *E, hipStream_t s)
{
    const int64_t z[3] = {0, 0, 0}, K[3] = {K0, K1, K2}, n[3] = {n0, n1, n2};
    return launch_upsample_box(El, K, z, K, S, z, n, E, s);
}

hipError_t launch_upsample_boxes(const float *El, int64_t lstride, const int *table, int nbox, const int64_t maxed[3],
                                 int S, float *E, int64_t estride, hipStream_t s)
{
    const int64_t N = maxed[0] * maxed[1] * maxed[2];
    const int per_box = (int)((N + 255) / 256 < 64 ? (N + 255) / 256 : 64);
    hipLaunchKernelGGL(k_upsample_boxes, dim3((unsigned)(per_box * nbox)), dim3(256), 0, s, El, lstride, table, per_box,
                       S, E, estride);
    return hipGetLastError();
}

hipError_t launch_upsample_box(const float *El, const int64_t kd[3], const int64_t klo[3], const int64_t K[3], int S,
                               const int64_t eo[3], const int64_t ed[3], float *E, hipStream_t s)
{
    const lat_box b{(int)kd[0], (int)kd[1], (int)kd[2], (int)klo[0], (int)klo[1], (int)klo[2], (int)K[0], (int)K[1],
                    (int)K[2], (int)eo[0], (int)eo[1], (int)eo[2], (int)ed[0], (int)ed[1], (int)ed[2]};
    const int64_t N = ed[0] * ed[1] * ed[2], rows = ed[0] * ed[1];
    const unsigned nb = (unsigned)(rows < 32768 ? rows : 32768);
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_upsample, dim3(nb), dim3(256), 0, s, El, b, S, E);
    return hipGetLastError();
}
