// Steps 1-3 of the saliency method (Shafiq et al., ICIP 2017, Sec. 2) with 16-bit MFMA
// operands: BF16 or FP16 data, and the DFT matrix either rounded once or split into a
// high and a low 16-bit part (W = W_hi + W_lo) whose products are summed by the same MFMAs
// in FP32.  With DS (data split) every stage input is also split, d = d_hi + d_lo: about
// 16 significant bits per operand.  Everything else matches the FP32 kernel: three separable
// contractions (t real -> half spectrum, x, y), the spectrum of each voxel kept in the
// accumulators, projections and energies in FP32.
//
// Every stage rounds its input to 16 bits, so the data passed between stages lives in LDS
// as packed 16-bit complex values (re in the low half), hi and lo parts in separate planes.
// FP16 stage outputs are scaled by 1/L (exact, L a power of two) before rounding so FP16
// keeps the input's range, and the projection weights carry the matching L^2; BF16 has the
// FP32 exponent range and is not scaled.
//
// K order of the t contraction (real input): lane group g holds the taps TPL g .. TPL g +
// TPL - 1 (TPL = L / 4) of its position.  With DS each tap is one 32-bit word d_hi | d_lo
// (lo in the high half) used twice, against (W_hi, W_hi) and (W_lo, W_lo): all four
// products W_{hi,lo} d_{hi,lo}.  Without it each tap is d | d against (W_hi, W_lo).
// K order of a complex contraction (x and y): each 32-bit word is one complex tap (re, im).
//   cube 16 with DS: three MFMAs per 16 rows, (W_hi, d_hi), (W_lo, d_hi) and (W_hi, d_lo)
//     (W_lo d_lo is below the rounding of the others), lane group g holding taps 4g .. 4g+3;
//   otherwise: MFMA j covers taps 8j .. 8j+7, lane group g the part g >> 1 (W_hi, W_lo) of
//     taps 8j + 4(g & 1) .. +3, once with d_hi and (DS) once more with d_lo.
// So each lane's data operand is four consecutive complex taps, 16 contiguous bytes of LDS
// along y, or four words PY apart along x.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "sal_device.h"
#include "sal_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

// A constant in a scalar register, opaque to the compiler (so it is not folded into an
// instruction constant, whose expansion for packed 16-bit operands is not the value's bits).
__device__ __forceinline__ uint32_t sreg(uint32_t v)
{
    asm volatile("" : "+s"(v));
    return v;
}

template <typename T>
struct Half16;
template <>
struct Half16<__bf16> {
    static constexpr bool SCALE = false;  // stage outputs are rounded unscaled
    static __device__ __forceinline__ f4 mma(u32x4 a, u32x4 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
    // round-to-nearest-even of both values, lo in bits 0..15
    static __device__ __forceinline__ uint32_t pack(float lo, float hi)
    {
        const bf16x2 v = {(__bf16)lo, (__bf16)hi};
        return __builtin_bit_cast(uint32_t, v);
    }
    // c - (value in bits 0..15 of p), resp. bits 16..31: exact (the difference of a float
    // and its rounding to 8 significant bits is a float), one dot-product instruction.  The
    // mask (-1, 0) or (0, -1) is passed in a scalar register with its exact bits, not as an
    // instruction constant.
    static __device__ __forceinline__ float sub_lo(uint32_t p, float c)
    {
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, p), __builtin_bit_cast(bf16x2, sreg(0x0000bf80u)), c,
                                               false);
    }
    static __device__ __forceinline__ float sub_hi(uint32_t p, float c)
    {
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, p), __builtin_bit_cast(bf16x2, sreg(0xbf800000u)), c,
                                               false);
    }
};
template <>
struct Half16<_Float16> {
    static constexpr bool SCALE = true;
    static __device__ __forceinline__ f4 mma(u32x4 a, u32x4 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ uint32_t pack(float lo, float hi)
    {
        const f16x2 v = {(_Float16)lo, (_Float16)hi};
        return __builtin_bit_cast(uint32_t, v);
    }
    static __device__ __forceinline__ float sub_lo(uint32_t p, float c)
    {
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2, p), __builtin_bit_cast(f16x2, sreg(0x0000bc00u)), c, false);
    }
    static __device__ __forceinline__ float sub_hi(uint32_t p, float c)
    {
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2, p), __builtin_bit_cast(f16x2, sreg(0xbc000000u)), c, false);
    }
};

// Store the complex value (re, im) as packed 16-bit parts: hi = round(v) at hi_arr[0], and
// with DS also lo = round(v - hi) at hi_arr[lo_off].
template <bool DS, typename T>
__device__ __forceinline__ void store_c(uint32_t *p, int lo_off, float re, float im)
{
    const uint32_t hi = Half16<T>::pack(re, im);
    p[0] = hi;
    if (DS) p[lo_off] = Half16<T>::pack(Half16<T>::sub_lo(hi, re), Half16<T>::sub_hi(hi, im));
}

// One volume sample as the data word of the t contraction: d_hi | d_lo with DS, else d | d.
template <bool DS, typename T>
__device__ __forceinline__ uint32_t sample_word(float v)
{
    if (!DS) return Half16<T>::pack(v, v);
    const uint32_t hi = Half16<T>::pack(v, 0.0f);
    return Half16<T>::pack(v, Half16<T>::sub_lo(hi, v));
}

__device__ __forceinline__ u32x4 lds4(const uint32_t *p) { return u32x4{p[0], p[1], p[2], p[3]}; }
template <int ST>
__device__ __forceinline__ u32x4 lds4s(const uint32_t *p)
{
    return u32x4{p[0], p[ST], p[2 * ST], p[3 * ST]};
}

}  // namespace

// Waves per SIMD the register allocation must allow, as measured best: six at cube 8 (the
// LDS of a workgroup admits three per CU), four at cube 16.  Strided tiles are LDS-bound.
#ifndef SAL_HWPE8D
#define SAL_HWPE8D 6
#endif
#ifndef SAL_HWPE8
#define SAL_HWPE8 6
#endif
#ifndef SAL_HWPE16D
#define SAL_HWPE16D 4
#endif
#ifndef SAL_HWPE16
#define SAL_HWPE16 4
#endif
template <int L, bool DS, int S>
struct HWpe {
    static constexpr int v = S != 1 ? 2 : L == 8 ? (DS ? SAL_HWPE8D : SAL_HWPE8) : (DS ? SAL_HWPE16D : SAL_HWPE16);
};

// Operand counts shared by the kernel and the host tables.
template <int L, bool DS>
struct H16Lay {
    static constexpr int TPL = L / 4;                   // t taps per lane group
    static constexpr int NWA = DS ? 2 * TPL : TPL;       // data words of the t contraction
    static constexpr int JA = (NWA + 3) / 4;             // its MFMAs per M tile
    static constexpr bool THREE = L == 16 && DS;         // three-product complex contractions
    static constexpr int J = L / 8;                      // otherwise: MFMAs per data part
    static constexpr int NA = THREE ? 2 : J;             // A operands per M tile (complex)
};

template <int L, typename T, bool DS, int S>
__global__ __attribute__((amdgpu_waves_per_eu(HWpe<L, DS, S>::v))) __launch_bounds__(64 * TileCfg<L>::NW) void k_energy_h(
    const float *__restrict__ V, int n0, int n1, int n2, ebox bx, int tt_len, int nby, int nbx,
    const uint32_t *__restrict__ w_c16, const uint32_t *__restrict__ w_a16,
    const uint32_t *__restrict__ w_c16b, const float *__restrict__ w_grp, float *__restrict__ E,
    float *__restrict__ vmax_part)
{
    using G = Geo<L>;
    using C = TileCfg<L>;
    using HT = Half16<T>;
    using Y = H16Lay<L, DS>;
    constexpr int H = G::H, h = G::h, MT = G::MT, MTA = G::MTA;
    constexpr int TPL = Y::TPL, NWA = Y::NWA, JA = Y::JA, J = Y::J, NA = Y::NA;
    constexpr bool THREE = Y::THREE;
    constexpr int NW = C::NW, TY = C::TY;
    // windows of x-rows and y-columns S apart (S = 2: the half-resolution lattice)
    constexpr int PX = S * (NW - 1) + L, PY = S * (TY - 1) + L;
    constexpr int NTB = (PY + 15) / 16, PYB = NTB * 16, NTC = TY / 16;
    constexpr int NPOS = PX * PY, NTA = (NPOS + 15) / 16, NJ = (NTA + NW - 1) / NW;
    constexpr int NGK = L / 2 + 1;
    // cube 16: the stage-C matrix rows are ordered so that lane group g of M tile 0 holds the
    // bins om and L - om (equal weights), and stage B reads its own matrix from LDS
    constexpr bool FOLD = L == 16;
    constexpr int NWB = C::W_LDS ? h * NGK * MT * 32 : 1;
    constexpr float oscale = HT::SCALE ? 1.0f / (float)L : 1.0f;
    static_assert(3 * PY <= 255, "stage-B operand offsets must fit a paired LDS read");

    constexpr int NP = DS ? 2 : 1;  // 16-bit parts stored per value
    // stage-A output, position-major: [mu][part][x'][y'] (position x' PY + y')
    __shared__ uint32_t A_s[h * NP * NPOS];
    // With the data split at cube 16, stage B runs in two halves of eight frequency rows,
    // each followed by the stage C of the weight groups whose rows it holds, so B_s keeps
    // eight rows at a time and two workgroups fit a CU.  Otherwise one pass over all rows.
    constexpr int NH = (L == 16 && DS) ? 2 : 1, NROW = NH > 1 ? 8 : L;
    __shared__ uint32_t B_s[NW][NROW * NP * PYB];  // per wave [row][part][y']
    // cube 16, stage-B matrix: with the data split per half (rows in the halves' order) NA
    // operands, else per M tile (rows in frequency order) J operands
    constexpr int NWCB = L == 16 ? (NH > 1 ? NH * NA : MT * NA) : 0;
    __shared__ u32x4 wcb_s[NWCB > 0 ? NWCB * 64 : 1];
    __shared__ float wb_s[NWB];
    __shared__ u32x4 wa_s[MTA * JA * 64];
    __shared__ float red_s[NW];

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

    u32x4 wc[MT][NA];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < NA; ++j) wc[mt][j] = reinterpret_cast<const u32x4 *>(w_c16)[(mt * NA + j) * 64 + lane];
    for (int i = threadIdx.x; i < MTA * JA * 64; i += 64 * NW) wa_s[i] = reinterpret_cast<const u32x4 *>(w_a16)[i];
    if (NWCB > 0)
        for (int i = threadIdx.x; i < NWCB * 64; i += 64 * NW) wcb_s[i] = reinterpret_cast<const u32x4 *>(w_c16b)[i];
    if (C::W_LDS)
        for (int i = threadIdx.x; i < NWB; i += 64 * NW) wb_s[i] = w_grp[i];

    const int n12 = n1 * n2;  // the volume holds at most 2^31 - 1 samples
    const int64_t nbox = (int64_t)bx.fk0 * K1 * K2;
    float vmax = 0.0f;
    uint32_t *Bw = B_s[wave];
    // first complex tap of this lane's data operand in MFMA j (see the K order above)
    auto ctap = [&](int j) { return THREE ? 4 * g : 8 * j + 4 * (g & 1); };

    // samples of this wave's stage-A positions for one t0; the next t0's loads are issued
    // after stage C so they hold no registers through B and C.  The row offsets are formed
    // once per t0, each load adds the kept 32-bit position offset.
    int off_xy[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int pos = min((wave + NW * jj) * 16 + n, NPOS - 1);
        const int xp = pos / PY, yp = pos - xp * PY;
        off_xy[jj] = refl_idx(x_base - H + xp, n1) * n2 + refl_idx(y_base - H + yp, n2);
    }
    float vnext[NJ][TPL];
    auto load_a = [&](int t0) {
        int rowo[TPL];
#pragma unroll
        for (int i = 0; i < TPL; ++i) rowo[i] = refl_idx(t0 - H + TPL * g + i, n0) * n12;
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int off = opaque(off_xy[jj]);
#pragma unroll
            for (int i = 0; i < TPL; ++i)
                vnext[jj][i] = (wave + NW * jj < NTA) ? V[(uint32_t)(rowo[i] + off)] : 0.f;
        }
    };
    load_a(t_begin);

    for (int t0 = t_begin; t0 < t_end; t0 += S) {
        __syncthreads();
        float vcur[NJ][TPL];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
            for (int i = 0; i < TPL; ++i) vcur[jj][i] = vnext[jj][i];
        // ---------------- stage A: real DFT along t -------------------------------------
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int tl = wave + NW * jj;
            if (tl < NTA) {
                uint32_t sw[TPL];
#pragma unroll
                for (int i = 0; i < TPL; ++i) {
                    vmax = fmaxf(vmax, fabsf(vcur[jj][i]));
                    sw[i] = sample_word<DS, T>(vcur[jj][i]);
                }
                u32x4 b[JA];
#pragma unroll
                for (int ja = 0; ja < JA; ++ja)
#pragma unroll
                    for (int wd = 0; wd < 4; ++wd) {
                        const int q = 4 * ja + wd;
                        b[ja][wd] = DS ? sw[q >> 1] : (q < TPL ? sw[q] : 0u);
                    }
                f4 acc[MTA];
#pragma unroll
                for (int mt = 0; mt < MTA; ++mt) {
                    acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ja = 0; ja < JA; ++ja) acc[mt] = HT::mma(wa_s[(mt * JA + ja) * 64 + lane], b[ja], acc[mt]);
                }
                const int pos = tl * 16 + opaque(n);
                if (pos < NPOS) {
#pragma unroll
                    for (int mt = 0; mt < MTA; ++mt) {
                        const int mu0 = 8 * mt + 2 * g;
                        if (mu0 < h)
                            store_c<DS, T>(&A_s[mu0 * NP * NPOS + pos], NPOS, acc[mt][0] * oscale, acc[mt][1] * oscale);
                        if (mu0 + 1 < h)
                            store_c<DS, T>(&A_s[(mu0 + 1) * NP * NPOS + pos], NPOS, acc[mt][2] * oscale,
                                           acc[mt][3] * oscale);
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
            const bool self = (mu == 0 || mu == L / 2);
#pragma unroll 1
            for (int hp = 0; hp < NH; ++hp) {
                // ---------- stage B: complex DFT along x for this mu (rows of half hp) ----------
                // one pass: row nu at position nu; halves: position i holds the i-th frequency
                // of the half's list (the matrix rows of w_c16b are ordered the same way)
                constexpr int BT = NH > 1 ? 1 : MT;  // M tiles per pass
#pragma unroll
                for (int nb = 0; nb < NTB; ++nb) {
                    const int yp = min(nb * 16 + n, PY - 1);
                    const uint32_t *Ab = &A_s[mu * NP * NPOS + S * wave * PY + yp];
                    f4 acc[BT];
#pragma unroll
                    for (int mt = 0; mt < BT; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
                    auto wB = [&](int mt, int j) -> u32x4 {
                        return NWCB > 0 ? wcb_s[((NH > 1 ? hp : mt) * NA + j) * 64 + lane] : wc[mt][j];
                    };
                    if (THREE) {
                        const u32x4 bh = lds4s<PY>(Ab + ctap(0) * PY);
                        const u32x4 bl = lds4s<PY>(Ab + NPOS + ctap(0) * PY);
#pragma unroll
                        for (int mt = 0; mt < BT; ++mt) {
                            acc[mt] = HT::mma(wB(mt, 0), bh, acc[mt]);
                            acc[mt] = HT::mma(wB(mt, 1), bh, acc[mt]);
                            acc[mt] = HT::mma(wB(mt, 0), bl, acc[mt]);
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < J; ++j) {
                            const u32x4 b = lds4s<PY>(Ab + ctap(j) * PY);
                            u32x4 bl;
                            if (DS) bl = lds4s<PY>(Ab + NPOS + ctap(j) * PY);
#pragma unroll
                            for (int mt = 0; mt < BT; ++mt) {
                                acc[mt] = HT::mma(wB(mt, j), b, acc[mt]);
                                if (DS) acc[mt] = HT::mma(wB(mt, j), bl, acc[mt]);
                            }
                        }
                    }
#pragma unroll
                    for (int mt = 0; mt < BT; ++mt) {
                        const int i0 = 8 * mt + 2 * g;
                        store_c<DS, T>(&Bw[i0 * NP * PYB + nb * 16 + n], PYB, acc[mt][0] * oscale, acc[mt][1] * oscale);
                        store_c<DS, T>(&Bw[(i0 + 1) * NP * PYB + nb * 16 + n], PYB, acc[mt][2] * oscale,
                                       acc[mt][3] * oscale);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // ---------- stage C: complex DFT along y, projections, energies ----------------
                // weight group (mu, k) of entry ei of the half: rows nu = k at position pa and,
                // unless mu is 0 or L/2 or k is 0 or L/2, nu = L - k at position pb; the NTC
                // voxel tiles of a row run as independent, interleaved MFMA chains
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
                    const bool pair = !self && k > 0 && k < L / 2;
                    const int grp = mu * NGK + k;
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
                    auto row_dft = [&](int pos) {
#pragma unroll
                        for (int c = 0; c < NTC; ++c)
#pragma unroll
                            for (int mt = 0; mt < MT; ++mt) acc[c][mt] = f4{0.f, 0.f, 0.f, 0.f};
                        if (THREE) {
                            u32x4 bh[NTC], bl[NTC];
#pragma unroll
                            for (int c = 0; c < NTC; ++c) {
                                const int bo = pos * NP * PYB + S * (c * 16 + n) + ctap(0);
                                bh[c] = lds4(&Bw[bo]);
                                bl[c] = lds4(&Bw[bo + PYB]);
                            }
#pragma unroll
                            for (int c = 0; c < NTC; ++c)
#pragma unroll
                                for (int mt = 0; mt < MT; ++mt) acc[c][mt] = HT::mma(wc[mt][0], bh[c], acc[c][mt]);
#pragma unroll
                            for (int c = 0; c < NTC; ++c)
#pragma unroll
                                for (int mt = 0; mt < MT; ++mt) acc[c][mt] = HT::mma(wc[mt][1], bh[c], acc[c][mt]);
#pragma unroll
                            for (int c = 0; c < NTC; ++c)
#pragma unroll
                                for (int mt = 0; mt < MT; ++mt) acc[c][mt] = HT::mma(wc[mt][0], bl[c], acc[c][mt]);
                        } else {
#pragma unroll
                            for (int j = 0; j < J; ++j) {
                                u32x4 b[NTC], bl[NTC];
#pragma unroll
                                for (int c = 0; c < NTC; ++c) {
                                    const int bo = pos * NP * PYB + S * (c * 16 + n) + ctap(j);
                                    b[c] = lds4(&Bw[bo]);
                                    if (DS) bl[c] = lds4(&Bw[bo + PYB]);
                                }
#pragma unroll
                                for (int c = 0; c < NTC; ++c)
#pragma unroll
                                    for (int mt = 0; mt < MT; ++mt) acc[c][mt] = HT::mma(wc[mt][j], b[c], acc[c][mt]);
                                if (DS) {
#pragma unroll
                                    for (int c = 0; c < NTC; ++c)
#pragma unroll
                                        for (int mt = 0; mt < MT; ++mt)
                                            acc[c][mt] = HT::mma(wc[mt][j], bl[c], acc[c][mt]);
                                }
                            }
                        }
                    };
                    float m0[NTC][MT], m1[NTC][MT];
                    row_dft(pa);
#pragma unroll
                    for (int c = 0; c < NTC; ++c)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            const f4 a = acc[c][mt];
                            m0[c][mt] = __builtin_amdgcn_sqrtf(fmaf(a[0], a[0], a[1] * a[1]));
                            m1[c][mt] = __builtin_amdgcn_sqrtf(fmaf(a[2], a[2], a[3] * a[3]));
                        }
                    if (pair) {
                        row_dft(pb);
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
                // the next half's stage B overwrites B_s
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        if (t0 + S < t_end) load_a(t0 + S);
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

template <int L, typename T, bool DS>
static hipError_t launch_h(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                           const ebox &bx, float *E, float *vmax_part, int nby, int nbx, int tt,
                           int64_t nb, hipStream_t s)
{
    if (c->p.stride == 2)
        hipLaunchKernelGGL((k_energy_h<L, T, DS, 2>), dim3((unsigned)nb), dim3(64 * TileCfg<L>::NW), 0, s,
                           V, (int)n0, (int)n1, (int)n2, bx, tt, nby, nbx, c->t.w_c16, c->t.w_a16,
                           c->t.w_c16b, c->t.w_bin, E, vmax_part);
    else
        hipLaunchKernelGGL((k_energy_h<L, T, DS, 1>), dim3((unsigned)nb), dim3(64 * TileCfg<L>::NW), 0, s,
                           V, (int)n0, (int)n1, (int)n2, bx, tt, nby, nbx, c->t.w_c16, c->t.w_a16,
                           c->t.w_c16b, c->t.w_bin, E, vmax_part);
    return hipGetLastError();
}

hipError_t launch_energy16(const sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                           const ebox &bx, float *E, float *vmax_part, int nby, int nbx, int tt,
                           int64_t nb, hipStream_t s)
{
    const int p = c->p.precision;
    const bool bf = p == SAL_BF16 || p == SAL_BF16_SPLIT || p == SAL_BF16_SPLITW;
    const bool ds = p == SAL_BF16_SPLIT || p == SAL_FP16_SPLIT;
#define SAL_LAUNCH_H(LL, TT, DD) launch_h<LL, TT, DD>(c, V, n0, n1, n2, bx, E, vmax_part, nby, nbx, tt, nb, s)
    if (c->L == 8) {
        if (bf) return ds ? SAL_LAUNCH_H(8, __bf16, true) : SAL_LAUNCH_H(8, __bf16, false);
        return ds ? SAL_LAUNCH_H(8, _Float16, true) : SAL_LAUNCH_H(8, _Float16, false);
    }
    if (bf) return ds ? SAL_LAUNCH_H(16, __bf16, true) : SAL_LAUNCH_H(16, __bf16, false);
    return ds ? SAL_LAUNCH_H(16, _Float16, true) : SAL_LAUNCH_H(16, _Float16, false);
#undef SAL_LAUNCH_H
}
