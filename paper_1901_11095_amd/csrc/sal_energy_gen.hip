// Steps 1-3 of the saliency method (Shafiq et al., ICIP 2017, Sec. 2) for cube sides that
// do not fill 16-wide matrix tiles: L = 2..7, among them the paper's own 5 x 5 x 5 cube.
// The contractions have 2L <= 14 real rows and columns, so a 16 x 16 matrix-core tile would
// be mostly padding; at these sizes the work per voxel is a few thousand flops and the
// vector ALUs carry it in FP32.
//
// The decomposition is the one of the matrix-core kernels: the window DFT (with 1/L^3
// folded into the weights) as three separable contractions that share the first two axes
// between overlapping windows, t real -> half spectrum mu <= L/2, then x, then y per
// voxel, followed by the plane projections of Eqs. (1)-(4) with DC excluded and the mean
// magnitudes E_m.  A workgroup owns NX x-rows by NY y-columns and walks t:
//   ring    the L t-planes of the (NX + L - 1) x (NY + L - 1) patch the windows cover, one
//           new plane per t (reflected at the volume faces when loaded);
//   stage A A[pos][mu] = sum_p W[mu, p] V[t0 - H + p, pos] for every patch position;
//   stage B per mu: B[x0][y'][nu] = sum_q W[nu, q] A[x0 + q, y'][mu], one thread per
//           patch position for all nu;
//   stage C per mu and nu, one thread per voxel (x0, y0): F[om] = sum_r W[om, r]
//           B[x0][y0 + r][nu], |F| weighted by the projections into E_t, E_x, E_y.
// Every stage takes its L-point DFTs with the terms and outputs in conjugate pairs.
// Bins with mu and L - mu have equal magnitudes and weights (conjugates); the weight table
// carries that multiplicity, so only mu <= L/2 is computed.  Stage C likewise takes the
// conjugate rows of the real t frequencies mu = 0 (and L/2) once, twice weighted.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sal_device.h"
#include "sal_dft.h"
#include "sal_internal.h"

namespace {

template <int L>
struct GenCfg {
    static constexpr int NX = L <= 5 ? 16 : 8;  // x-rows per workgroup
    static constexpr int NY = 256 / NX;         // y-columns per workgroup
};

template <int L>
struct GenTw {
    float2 w[L];  // e^{-2 pi i k / L}, k = 0..L-1
};

}  // namespace

template <int L, int S>
__global__ __launch_bounds__(256) void k_energy_gen(const float *__restrict__ V, int n0, int n1, int n2, ebox bx,
                                                    int tt_len, int nby, int nbx, GenTw<L> tw,
                                                    const float *__restrict__ wgen, float *__restrict__ E,
                                                    float *__restrict__ vmax_part)
{
    constexpr int H = L / 2, h = L / 2 + 1;
    constexpr int NX = GenCfg<L>::NX, NY = GenCfg<L>::NY;
    // windows of x-rows and y-columns S apart (S = 2: the half-resolution lattice)
    constexpr int PX = S * (NX - 1) + L, PY = S * (NY - 1) + L, NP = PX * PY;
    constexpr int NW3 = h * L * L * 3;
    __shared__ float ring[L][NP];
    __shared__ float2 A_s[NP * h];
    __shared__ float2 B_s[NX * PY * L];
    __shared__ float wg_s[NW3];
    __shared__ float red_s[4];

    const int tid = threadIdx.x;
    int box;
    const int tile = box_tile(bx, &box);
    V += box * bx.vstride;
    E += box * bx.estride;
    const int ty = tile % nby, tx = (tile / nby) % nbx, tb = tile / (nby * nbx);
    const int y_base = bx.o2 + S * ty * NY, x_base = bx.o1 + S * tx * NX;
    const int t_begin = bx.o0 + S * tb * tt_len;
    const int t_end = min(bx.o0 + bx.d0, t_begin + S * tt_len);
    if (t_begin >= t_end || x_base >= bx.o1 + bx.d1 || y_base >= bx.o2 + bx.d2) {
        // past a box smaller than the grid's (batched boxes): nothing to compute
        if (tid == 0 && vmax_part) vmax_part[blockIdx.x] = 0.f;
        return;
    }
    const int64_t plane = (int64_t)n1 * n2;
    // E frame (the box itself unless a batch entry says otherwise)
    const int K1 = bx.fk1, K2 = bx.fk2;
    const int64_t nbox = (int64_t)bx.fk0 * K1 * K2;

    for (int i = tid; i < NW3; i += 256) wg_s[i] = wgen[i];

    float vmax = 0.f;
    auto load_plane = [&](int tv) {
        const int slot = ((tv % L) + L) % L;
        const int64_t gt = refl_idx(tv, n0);
        for (int p = tid; p < NP; p += 256) {
            const int xp = p / PY, yp = p - xp * PY;
            const int gx = refl_idx(x_base - H + xp, n1), gy = refl_idx(y_base - H + yp, n2);
            const float v = V[gt * plane + (int64_t)gx * n2 + gy];
            vmax = fmaxf(vmax, fabsf(v));
            ring[slot][p] = v;
        }
    };
    for (int k = 0; k < L - S; ++k) load_plane(t_begin - H + k);

    const int x0 = tid / NY, y0 = tid - (tid / NY) * NY;
    for (int t0 = t_begin; t0 < t_end; t0 += S) {
        // the S planes that enter the windows of t0 (the ring slots of the S that left)
        for (int k = L - S; k < L; ++k) load_plane(t0 - H + k);
        __syncthreads();
        // ---------------- stage A: real DFT along t, mu <= L/2 ---------------------------
        for (int p = tid; p < NP; p += 256) {
            float v[L];
            float2 a[h];
#pragma unroll
            for (int k = 0; k < L; ++k) v[k] = ring[(((t0 - H + k) % L) + L) % L][p];
            sal_dft::rdft_half<L>(v, tw.w, a);
#pragma unroll
            for (int mu = 0; mu < h; ++mu) A_s[p * h + mu] = a[mu];
        }
        __syncthreads();
        float e0 = 0.f, e1 = 0.f, e2 = 0.f;
#pragma unroll 1
        for (int mu = 0; mu < h; ++mu) {
            // ---------------- stage B: DFT along x for this mu, all nu of a position ----
            for (int j = tid; j < NX * PY; j += 256) {
                const int yp = j % PY, xr = j / PY;
                float2 a[L], f[L];
#pragma unroll
                for (int q = 0; q < L; ++q) a[q] = A_s[((S * xr + q) * PY + yp) * h + mu];
                sal_dft::cdft<L>(a, tw.w, f);
#pragma unroll
                for (int nu = 0; nu < L; ++nu) B_s[(xr * PY + yp) * L + nu] = f[nu];
            }
            __syncthreads();
            // ---------------- stage C: DFT along y per voxel, projections, energies ------
            // The weights depend on the squares of the signed frequencies, so the bins om and
            // L - om of a row share theirs, and so do the conjugate bins (mu, nu, om) and
            // (mu, L - nu, L - om).  On the rows mu = 0 (and L/2 for even L) the t spectrum is
            // real, the row L - nu is the conjugate of the row nu bin for bin, and the rows
            // past L/2 count as twice the rows 1 .. (L - 1)/2.
            const bool real_mu = mu == 0 || 2 * mu == L;
            const int nu_end = real_mu ? L / 2 + 1 : L;
#pragma unroll 1
            for (int nu = 0; nu < nu_end; ++nu) {
                float2 b[L], f[L];
#pragma unroll
                for (int r = 0; r < L; ++r) b[r] = B_s[(x0 * PY + S * y0 + r) * L + nu];
                sal_dft::cdft<L>(b, tw.w, f);
                const float *w = &wg_s[(mu * L + nu) * L * 3];
                float m[L];
#pragma unroll
                for (int om = 0; om < L; ++om) m[om] = __builtin_amdgcn_sqrtf(fmaf(f[om].x, f[om].x, f[om].y * f[om].y));
                float q0 = 0.f, q1 = 0.f, q2 = 0.f;
#pragma unroll
                for (int om = 0; om <= L / 2; ++om) {
                    const float mm = (om == 0 || 2 * om == L) ? m[om] : m[om] + m[L - om];
                    q0 = fmaf(w[3 * om], mm, q0);
                    q1 = fmaf(w[3 * om + 1], mm, q1);
                    q2 = fmaf(w[3 * om + 2], mm, q2);
                }
                const float k2 = (real_mu && nu != 0 && 2 * nu != L) ? 2.f : 1.f;
                e0 = fmaf(k2, q0, e0);
                e1 = fmaf(k2, q1, e1);
                e2 = fmaf(k2, q2, e2);
            }
            __syncthreads();
        }
        const int x = x_base + S * x0, y = y_base + S * y0;
        if (x < bx.o1 + bx.d1 && y < bx.o2 + bx.d2) {
            const int64_t o = ((int64_t)((t0 - bx.fo0) / S) * K1 + (x - bx.fo1) / S) * K2 + (y - bx.fo2) / S;
            E[o] = e0;
            E[nbox + o] = e1;
            E[2 * nbox + o] = e2;
        }
    }
    // max |V| of everything this workgroup read (all of it lies in the volume)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    if ((tid & 63) == 0) red_s[tid >> 6] = vmax;
    __syncthreads();
    if (tid == 0 && vmax_part) vmax_part[blockIdx.x] = fmaxf(fmaxf(red_s[0], red_s[1]), fmaxf(red_s[2], red_s[3]));
}

// ====================================================================== launchers

namespace {

int gen_tt_len(int64_t n0, int64_t tiles_xy)
{
    // enough workgroups to fill 256 CUs several times over; long t walks otherwise
    int64_t tt = 32;
    while (tt > 2 && tiles_xy * ((n0 + tt - 1) / tt) < 2048) tt >>= 1;
    return (int)tt;
}

// grid of one box (nbox > 1: the t walk is sized for that many boxes in one launch)
template <int L>
void gen_grid(int64_t d0, int64_t d1, int64_t d2, int *nby, int *nbx, int *tt, int64_t *nb, int64_t nbox = 1)
{
    *nby = (int)((d2 + GenCfg<L>::NY - 1) / GenCfg<L>::NY);
    *nbx = (int)((d1 + GenCfg<L>::NX - 1) / GenCfg<L>::NX);
    *tt = gen_tt_len(d0, (int64_t)(*nby) * (*nbx) * nbox);
    *nb = (int64_t)(*nby) * (*nbx) * ((d0 + *tt - 1) / *tt);
}

template <int L>
hipError_t launch_gen_L(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, ebox bx,
                        float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox)
{
    const int S = c->p.stride;
    int nby, nbx, tt;
    int64_t nb;
    gen_grid<L>((bx.d0 + S - 1) / S, (bx.d1 + S - 1) / S, (bx.d2 + S - 1) / S, &nby, &nbx, &tt, &nb, nbox);
    if (bx.table) {
        bx.per_box = (int)nb;
        nb *= nbox;
    }
    if (nparts) *nparts = (int)nb;
    if (nb == 0) return hipSuccess;
    GenTw<L> tw;
    for (int k = 0; k < L; ++k) tw.w[k] = make_float2(c->tw_host[2 * k], c->tw_host[2 * k + 1]);
    if (S == 2 && L > 2)
        hipLaunchKernelGGL((k_energy_gen<L, (L > 2 ? 2 : 1)>), dim3((unsigned)nb), dim3(256), 0, s, V, (int)n0,
                           (int)n1, (int)n2, bx, tt, nby, nbx, tw, c->t.w_gen, E, vmax_part);
    else
        hipLaunchKernelGGL((k_energy_gen<L, 1>), dim3((unsigned)nb), dim3(256), 0, s, V, (int)n0, (int)n1,
                           (int)n2, bx, tt, nby, nbx, tw, c->t.w_gen, E, vmax_part);
    return hipGetLastError();
}

}  // namespace

int64_t energy_gen_num_blocks(int L, int64_t d0, int64_t d1, int64_t d2, int64_t nbox)
{
    int nby, nbx, tt;
    int64_t nb = 0;
    switch (L) {
    case 2: gen_grid<2>(d0, d1, d2, &nby, &nbx, &tt, &nb, nbox); break;
    case 3: gen_grid<3>(d0, d1, d2, &nby, &nbx, &tt, &nb, nbox); break;
    case 4: gen_grid<4>(d0, d1, d2, &nby, &nbx, &tt, &nb, nbox); break;
    case 5: gen_grid<5>(d0, d1, d2, &nby, &nbx, &tt, &nb, nbox); break;
    case 6: gen_grid<6>(d0, d1, d2, &nby, &nbx, &tt, &nb, nbox); break;
    case 7: gen_grid<7>(d0, d1, d2, &nby, &nbx, &tt, &nb, nbox); break;
    default: break;
    }
    return nb;
}

hipError_t launch_energy_gen(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, const ebox &bx,
                             float *E, float *vmax_part, int *nparts, hipStream_t s, int nbox)
{
    switch (c->L) {
    case 2: return launch_gen_L<2>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    case 3: return launch_gen_L<3>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    case 4: return launch_gen_L<4>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    case 5: return launch_gen_L<5>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    case 6: return launch_gen_L<6>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    case 7: return launch_gen_L<7>(c, V, n0, n1, n2, bx, E, vmax_part, nparts, s, nbox);
    default: return hipErrorInvalidValue;
    }
}
