// Steps 1-3 of the saliency method (Shafiq et al., ICIP 2017, Sec. 2) window by window:
// the local 3D DFT of each window (DFT definition after Eq. (2)), its plane projections
// with DC excluded (Eqs. (1)-(4)) and the mean magnitudes E_t, E_x, E_y, with nothing
// shared between windows.  Used where the fused kernels' sharing of the first two axes
// between neighbouring windows does not apply or does not fit:
//   * windows on a lattice of stride s >= 3 (Sec. 2 asks only for more than 50 % overlap,
//     s < L/2) where the sliding kernel of cube 8 and 16 does not take them, and the
//     non-overlapping s = L of the predecessor method (Sec. 1): the work falls by s^3 while
//     unshared windows cost 2.5 times the shared contraction per window;
//   * cube sides without a fused kernel (9..15, 17..20).
// FP32; cube 16 on the matrix cores (k_energy_win_mfma below), the other sides on the vector
// ALUs.  A workgroup walks windows (grid-stride over the windows of its box); per window:
//   load    the L^3 samples, reflected at the volume faces, into LDS;
//   stage A per column (q, r): A[mu][q][r] = sum_p W[mu, p] win[p][q][r], mu <= L/2;
//   stage B per (mu, r): B[mu][nu][r] = sum_q W[nu, q] A[mu][q][r], every nu;
//   stage C per row (mu, nu): F[om] = sum_r W[om, r] B[mu][nu][r], |F| weighted by the
//           projections (times the conjugate multiplicity of mu and 1/(L^3 (L^3 - 1))),
//           summed over the workgroup into E_t, E_x, E_y.
// On the vector ALUs every stage takes its L-point DFTs with the terms and outputs in
// conjugate pairs (sal_dft.h).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sal_device.h"
#include "sal_dft.h"
#include "sal_internal.h"

namespace {

template <int L>
struct WinCfg {
    static constexpr int h = L / 2 + 1;
    static constexpr int NT = 64 * ((h * L + 63) / 64);  // one thread per (mu, r) / (mu, nu)
    static constexpr int LP = L + 1;                      // padded row of B (LDS banks)
};

template <int L>
struct WinTw {
    float2 w[L];  // e^{-2 pi i k / L}, k = 0..L-1
};

}  // namespace

// bx: the windows of the volume positions o + S k, k < ceil(d / S), E stored in the frame
// (fo, fk) at index (p - fo) / S; with a table, workgroups [e * per_box, (e+1) * per_box)
// serve entry e.
template <int L>
__global__ __launch_bounds__(WinCfg<L>::NT) void k_energy_win(const float *__restrict__ V, int n0, int n1, int n2,
                                                              ebox bx, int S, WinTw<L> tw,
                                                              const float *__restrict__ wgen, float *__restrict__ E,
                                                              float *__restrict__ vmax_part)
{
    using C = WinCfg<L>;
    constexpr int H = L / 2, h = C::h, NT = C::NT, LP = C::LP, L2 = L * L, L3 = L * L * L;
    constexpr int NWV = NT / 64;
    __shared__ float win[L3];            // [p][q][r]
    __shared__ float2 A_s[h * L2];       // [mu][q][r]
    __shared__ float2 B_s[h * L * LP];   // [mu][nu][r], rows padded
    __shared__ float red_s[NWV][4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int box;
    const int blk = box_tile(bx, &box);
    V += box * bx.vstride;
    E += box * bx.estride;
    const int nblk = bx.table ? bx.per_box : (int)gridDim.x;
    const int kd0 = (bx.d0 + S - 1) / S, kd1 = (bx.d1 + S - 1) / S, kd2 = (bx.d2 + S - 1) / S;
    const int nwin = kd0 * kd1 * kd2;
    const int K1 = bx.fk1, K2 = bx.fk2;
    const int64_t nfr = (int64_t)bx.fk0 * K1 * K2;
    const int64_t plane = (int64_t)n1 * n2;
    float vmax = 0.f;

    // The samples of the next window are loaded into registers while the current one
    // computes, so their latency is hidden; every thread holds NLD of them.
    constexpr int NLD = (L3 + NT - 1) / NT;
    float pre[NLD];
    auto load_win = [&](int w) {
        const int k2 = w % kd2, k1 = (w / kd2) % kd1, k0 = w / (kd2 * kd1);
        const int q0 = bx.o0 + S * k0 - H, q1 = bx.o1 + S * k1 - H, q2 = bx.o2 + S * k2 - H;
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = tid + NT * j;
            if (i < L3) {
                const int r = i % L, q = (i / L) % L, p = i / L2;
                pre[j] = V[(int64_t)refl_idx(q0 + p, n0) * plane + (int64_t)refl_idx(q1 + q, n1) * n2 +
                           refl_idx(q2 + r, n2)];
            }
        }
    };
    if (blk < nwin) load_win(blk);

    for (int w = blk; w < nwin; w += nblk) {
        const int k2 = w % kd2, k1 = (w / kd2) % kd1, k0 = w / (kd2 * kd1);
        const int p0 = bx.o0 + S * k0, p1 = bx.o1 + S * k1, p2 = bx.o2 + S * k2;
        __syncthreads();  // the previous window is done with win, A_s, B_s and red_s
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = tid + NT * j;
            if (i < L3) {
                vmax = fmaxf(vmax, fabsf(pre[j]));
                win[i] = pre[j];
            }
        }
        __syncthreads();
        if (w + nblk < nwin) load_win(w + nblk);
        // ---------------- stage A: real DFT along t, mu <= L/2 ---------------------------
        for (int c = tid; c < L2; c += NT) {
            float v[L];
            float2 x[h];
#pragma unroll
            for (int p = 0; p < L; ++p) v[p] = win[p * L2 + c];
            sal_dft::rdft_half<L>(v, tw.w, x);
#pragma unroll
            for (int mu = 0; mu < h; ++mu) A_s[mu * L2 + c] = x[mu];
        }
        __syncthreads();
        // ---------------- stage B: DFT along x per (mu, r), every nu ---------------------
        if (tid < h * L) {
            const int mu = tid / L, r = tid - (tid / L) * L;
            float2 a[L], f[L];
#pragma unroll
            for (int q = 0; q < L; ++q) a[q] = A_s[(mu * L + q) * L + r];
            sal_dft::cdft<L>(a, tw.w, f);
#pragma unroll
            for (int nu = 0; nu < L; ++nu) B_s[(mu * L + nu) * LP + r] = f[nu];
        }
        __syncthreads();
        // ---------------- stage C: DFT along y per row (mu, nu), projections -------------
        float e0 = 0.f, e1 = 0.f, e2 = 0.f;
        if (tid < h * L) {
            const int mu = tid / L, nu = tid - (tid / L) * L;
            float2 b[L], f[L];
#pragma unroll
            for (int r = 0; r < L; ++r) b[r] = B_s[(mu * L + nu) * LP + r];
            sal_dft::cdft<L>(b, tw.w, f);
            const float *wr = wgen + (int64_t)(mu * L + nu) * L * 3;
#pragma unroll
            for (int om = 0; om < L; ++om) {
                const float m = __builtin_amdgcn_sqrtf(fmaf(f[om].x, f[om].x, f[om].y * f[om].y));
                e0 = fmaf(wr[3 * om], m, e0);
                e1 = fmaf(wr[3 * om + 1], m, e1);
                e2 = fmaf(wr[3 * om + 2], m, e2);
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            e0 += __shfl_xor(e0, o);
            e1 += __shfl_xor(e1, o);
            e2 += __shfl_xor(e2, o);
        }
        if (lane == 0) {
            red_s[wave][0] = e0;
            red_s[wave][1] = e1;
            red_s[wave][2] = e2;
        }
        __syncthreads();
        if (tid == 0) {
            float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
            for (int v = 0; v < NWV; ++v) {
                s0 += red_s[v][0];
                s1 += red_s[v][1];
                s2 += red_s[v][2];
            }
            const int64_t o = ((int64_t)((p0 - bx.fo0) / S) * K1 + (p1 - bx.fo1) / S) * K2 + (p2 - bx.fo2) / S;
            E[o] = s0;
            E[nfr + o] = s1;
            E[2 * nfr + o] = s2;
        }
    }
    // max |V| of everything this workgroup read (all of it lies in the volume)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    __syncthreads();
    if (lane == 0) red_s[wave][3] = vmax;
    __syncthreads();
    if (tid == 0 && vmax_part) {
        float m = red_s[0][3];
        for (int v = 1; v < NWV; ++v) m = fmaxf(m, red_s[v][3]);
        vmax_part[blockIdx.x] = m;
    }
}

// ------------------------------------------------------------------------------------
// Cube 16 on the matrix cores (FP32 16x16x4 MFMA), one window at a time per group of three
// waves (WM_GROUPS groups per workgroup would share the weight table; one group per workgroup,
// three workgroups per CU, measured fastest: 90 ms against 119 ms with two on a stride-4
// lattice of the 512 x 1024 x 1024 volume), the three contractions as small matrix products:
//   stage A (t, real -> half spectrum): rows (x, y) of the window, 16 per M tile (tile = x),
//           K = t, 16 columns (mu, re|im) for mu <= 8: the imaginary parts of mu = 0 and 8
//           are zero for a real input, so column 1 carries the real part of mu = 8; the
//           samples are the A operand straight from global memory (the next window's are
//           in flight during stages B and C);
//   stage B (x): rows y for one mu (tile = mu), K = (x, re|im), columns (re|im, nu);
//   stage C (y): rows nu for one mu (tile = mu), K = (y, re|im), columns (re|im, om): a lane
//           holds re and im of its bins in its two accumulators, so |F|, the projection
//           weights and the sums into E_t, E_x, E_y follow in registers.
// Stage outputs live in one LDS buffer per group [mu][row][re|im][17 columns] (B in place of
// A, plane by plane), the per-lane projection weights of stage C in another.  The wave that
// computes plane mu in stage B also reads it in stage C, so only stage A's output needs a
// barrier.  352 MFMAs per window (721 kflop; the separable transform counted with complex
// mu = 0 and 8 is 737 kflop).
namespace {
constexpr int WM_WAVES = 3, WM_GROUPS = 1;
constexpr int WM_L = 16, WM_H = 8, WM_h = 9, WM_RS = 17;  // row stride of the LDS planes
constexpr int WM_PLANE = WM_L * 2 * WM_RS;                // floats per mu plane
}  // namespace

__global__ __launch_bounds__(64 * WM_WAVES * WM_GROUPS) void k_energy_win_mfma(
    const float *__restrict__ V, int n0, int n1, int n2, ebox bx, int S, WinTw<16> tw,
    const float *__restrict__ wgen, float *__restrict__ E, float *__restrict__ vmax_part)
{
    constexpr int L = WM_L, H = WM_H, h = WM_h, RS = WM_RS, PL = WM_PLANE, G = WM_GROUPS;
    constexpr int NWV = WM_WAVES * G;
    constexpr int MTA = (L + WM_WAVES - 1) / WM_WAVES;  // stage-A M tiles per wave (at most)
    constexpr int MTB = (h + WM_WAVES - 1) / WM_WAVES;  // stage-B/C M tiles per wave
    __shared__ float P[G][h * PL];               // per group [mu][row][re|im][col], see above
    __shared__ float wl[h * 4 * 3 * 64];         // [mu][j][m][lane] projection weights
    __shared__ float red_s[NWV][4];

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int grp = wave / WM_WAVES, wv = wave - grp * WM_WAVES;  // group, wave in group
    const int g = lane >> 4, n = lane & 15;
    int box;
    const int blk = box_tile(bx, &box);
    V += box * bx.vstride;
    E += box * bx.estride;
    const int nblk = bx.table ? bx.per_box : (int)gridDim.x;
    const int kd0 = (bx.d0 + S - 1) / S, kd1 = (bx.d1 + S - 1) / S, kd2 = (bx.d2 + S - 1) / S;
    const int nwin = kd0 * kd1 * kd2;
    const int K1 = bx.fk1, K2 = bx.fk2;
    const int64_t nfr = (int64_t)bx.fk0 * K1 * K2;
    const int n12 = n1 * n2;  // the volume holds at most 2^31 - 1 samples
    float vmax = 0.f;
    float *Pg = P[grp];

    // weights of the bins (mu, nu = 4g + j, om = n) of this lane, with the conjugate
    // multiplicity of mu and 1/(L^3 (L^3 - 1)) (DC has weight 0)
    for (int i = tid; i < h * 4 * 3 * 64; i += 64 * NWV) {
        const int ln = i & 63, m = (i >> 6) % 3, j = (i / 192) & 3, mu = i / 768;
        wl[i] = wgen[((mu * L + 4 * (ln >> 4) + j) * L + (ln & 15)) * 3 + m];
    }
    // constant B operands: lane (g, n) at K step ks holds K = 4 ks + g, column n
    // stage A column n: (mu, re|im) = (n / 2, n % 2), except column 1 = (8, re)
    const int amu = n == 1 ? L / 2 : n >> 1, aim = n == 1 ? 0 : n & 1;
    float wa[4], wb[8][2];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const float2 w = tw.w[(amu * (4 * ks + g)) % L];
        wa[ks] = aim ? w.y : w.x;
    }
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            // K = (tap, re|im of the input), column (re|im of the output = nt, frequency n);
            // out = in * e^{-2 pi i tap f / L}, w = (cos, -sin)
            const int k = 4 * ks + g, tap = k >> 1, ci = k & 1;
            const float2 w = tw.w[(tap * n) % L];
            wb[ks][nt] = nt == 0 ? (ci == 0 ? w.x : -w.y) : (ci == 0 ? w.y : w.x);
        }

    // samples of this wave's stage-A tiles (x = wv + 3 i) for one window: lane (g, n)
    // holds V[t = 4 ks + g][x][y = n]
    float smp[MTA][4];
    auto load_win = [&](int w) {
        const int k2 = w % kd2, k1 = (w / kd2) % kd1, k0 = w / (kd2 * kd1);
        const int q0 = bx.o0 + S * k0 - H, q1 = bx.o1 + S * k1 - H, q2 = bx.o2 + S * k2 - H;
        const int yo = refl_idx(q2 + n, n2);
        int rowo[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) rowo[ks] = refl_idx(q0 + 4 * ks + g, n0) * n12 + yo;
#pragma unroll
        for (int i = 0; i < MTA; ++i) {
            const int x = wv + WM_WAVES * i;
            if (x < L) {
                const int xo = refl_idx(q1 + x, n1) * n2;
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) smp[i][ks] = V[(uint32_t)(rowo[ks] + xo)];
            }
        }
    };
    if (G * blk + grp < nwin) load_win(G * blk + grp);
    __syncthreads();  // wl complete

    // every wave of the workgroup takes the same number of steps (the barriers need it); a
    // group past the last window idles through its step
    for (int wb0 = G * blk; wb0 < nwin; wb0 += G * nblk) {
        const int w = wb0 + grp;
        const bool act = w < nwin;
        const int k2 = w % kd2, k1 = (w / kd2) % kd1, k0 = w / (kd2 * kd1);
        const int p0 = bx.o0 + S * k0, p1 = bx.o1 + S * k1, p2 = bx.o2 + S * k2;
        // ---------------- stage A: real DFT along t --------------------------------------
        if (act) {
#pragma unroll
            for (int i = 0; i < MTA; ++i) {
                const int x = wv + WM_WAVES * i;
                if (x < L) {
                    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        vmax = fmaxf(vmax, fabsf(smp[i][ks]));
                        acc = mfma4(smp[i][ks], wa[ks], acc);
                    }
                    // lane (g, n): rows y = 4g + j, column n = (amu, aim); lanes 0 and 1 also
                    // write the zero imaginary parts of mu = 0 and 8
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        Pg[amu * PL + (x * 2 + aim) * RS + 4 * g + j] = acc[j];
                        if (n < 2) Pg[amu * PL + (x * 2 + 1) * RS + 4 * g + j] = 0.f;
                    }
                }
            }
            if (w + G * nblk < nwin) load_win(w + G * nblk);
        }
        __syncthreads();
        float e0 = 0.f, e1 = 0.f, e2 = 0.f;
        if (act) {
#pragma unroll
            for (int i = 0; i < MTB; ++i) {
                const int mu = wv + WM_WAVES * i;
                if (mu < h) {
                    float *pl = Pg + mu * PL;
                    // ------------ stage B: DFT along x, plane mu in place ------------------
                    f4 acc[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
                    for (int ks = 0; ks < 8; ++ks) {
                        const int k = 4 * ks + g;  // (x, re|im) = (k / 2, k % 2), row y = n
                        const float a = pl[k * RS + n];
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt) acc[nt] = mfma4(a, wb[ks][nt], acc[nt]);
                    }
                    // rows y = 4g + j, column nu = n: (re, im) = (acc[0][j], acc[1][j]); every
                    // read of the plane is issued before these writes
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        pl[(n * 2) * RS + 4 * g + j] = acc[0][j];
                        pl[(n * 2 + 1) * RS + 4 * g + j] = acc[1][j];
                    }
                    // ------------ stage C: DFT along y, projections, energies -------------
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 8; ++ks) {
                        const int k = 4 * ks + g;  // (y, re|im) = (k / 2, k % 2), row nu = n
                        const float a = pl[(n * 2 + (k & 1)) * RS + (k >> 1)];
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt) acc[nt] = mfma4(a, wb[ks][nt], acc[nt]);
                    }
                    const float *wr = wl + mu * 768 + lane;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float m = __builtin_amdgcn_sqrtf(fmaf(acc[0][j], acc[0][j], acc[1][j] * acc[1][j]));
                        e0 = fmaf(wr[(j * 3 + 0) * 64], m, e0);
                        e1 = fmaf(wr[(j * 3 + 1) * 64], m, e1);
                        e2 = fmaf(wr[(j * 3 + 2) * 64], m, e2);
                    }
                }
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            e0 += __shfl_xor(e0, o);
            e1 += __shfl_xor(e1, o);
            e2 += __shfl_xor(e2, o);
        }
        if (lane == 0) {
            red_s[wave][0] = e0;
            red_s[wave][1] = e1;
            red_s[wave][2] = e2;
        }
        __syncthreads();  // red_s complete; every wave is done with its group's P
        if (act && wv == 0 && lane == 0) {
            float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
            for (int v = 0; v < WM_WAVES; ++v) {
                s0 += red_s[wave + v][0];
                s1 += red_s[wave + v][1];
                s2 += red_s[wave + v][2];
            }
            const int64_t o = ((int64_t)((p0 - bx.fo0) / S) * K1 + (p1 - bx.fo1) / S) * K2 + (p2 - bx.fo2) / S;
            E[o] = s0;
            E[nfr + o] = s1;
            E[2 * nfr + o] = s2;
        }
        // (the next step's stage A may write P now; red_s is rewritten one barrier later)
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    __syncthreads();
    if (lane == 0) red_s[wave][3] = vmax;
    __syncthreads();
    if (tid == 0 && vmax_part) {
        float m = red_s[0][3];
        for (int v = 1; v < NWV; ++v) m = fmaxf(m, red_s[v][3]);
        vmax_part[blockIdx.x] = m;
    }
}

// ====================================================================== launchers

namespace {

constexpr int64_t WIN_BLOCKS = 4096;   // workgroups of a whole-volume launch
constexpr int64_t WIN_PER_BOX = 64;    // workgroups per box of a batch

int64_t win_blocks(int64_t nwin, int64_t nbox)
{
    if (nbox > 1) return (nwin < WIN_PER_BOX ? (nwin > 0 ? nwin : 1) : WIN_PER_BOX) * nbox;
    return nwin < WIN_BLOCKS ? (nwin > 0 ? nwin : 1) : WIN_BLOCKS;
}

template <int L>
hipError_t launch_win_L(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, ebox bx, int S,
                        float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox)
{
    const int64_t nwin = ((bx.d0 + S - 1) / S) * ((bx.d1 + S - 1) / S) * ((bx.d2 + S - 1) / S);
    const int64_t nb = win_blocks(nwin, bx.table ? nbox : 1);
    if (bx.table) bx.per_box = (int)(nb / nbox);
    if (nparts) *nparts = (int)nb;
    WinTw<L> tw;
    for (int k = 0; k < L; ++k) tw.w[k] = make_float2(c->tw_host[2 * k], c->tw_host[2 * k + 1]);
    if constexpr (L == 16)
        hipLaunchKernelGGL(k_energy_win_mfma, dim3((unsigned)nb), dim3(64 * WM_WAVES * WM_GROUPS), 0, s, V, (int)n0, (int)n1,
                           (int)n2, bx, S, tw, c->t.w_gen, E, vmax_part);
    else
        hipLaunchKernelGGL(k_energy_win<L>, dim3((unsigned)nb), dim3(WinCfg<L>::NT), 0, s, V, (int)n0, (int)n1,
                           (int)n2, bx, S, tw, c->t.w_gen, E, vmax_part);
    return hipGetLastError();
}

}  // namespace

int64_t energy_win_num_blocks(const sal_ctx *c, int64_t k0, int64_t k1, int64_t k2)
{
    (void)c;
    return win_blocks(k0 * k1 * k2, 1);
}

hipError_t launch_energy_win(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, const ebox &bx,
                             float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox)
{
    const int S = c->p.stride;
#define SAL_WIN(LL) \
    case LL: return launch_win_L<LL>(c, V, n0, n1, n2, bx, S, E, vmax_part, nparts, s, nbox)
    switch (c->L) {
        SAL_WIN(2); SAL_WIN(3); SAL_WIN(4); SAL_WIN(5); SAL_WIN(6); SAL_WIN(7); SAL_WIN(8);
        SAL_WIN(9); SAL_WIN(10); SAL_WIN(11); SAL_WIN(12); SAL_WIN(13); SAL_WIN(14); SAL_WIN(15);
        SAL_WIN(16); SAL_WIN(17); SAL_WIN(18); SAL_WIN(19); SAL_WIN(20);
    default: return hipErrorInvalidValue;
    }
#undef SAL_WIN
}
