// C-ABI front end of libsal: argument checks, per-context device tables, workspace
// layout and the launch sequence of the method (Shafiq et al., ICIP 2017, Sec. 2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sal_internal.h"

namespace {

thread_local std::string g_create_err;

// exp(-2 pi i k / L) in FP64 with the quarter-turn values exact (0, +-1).
void twiddle(long k, long L, double *c, double *s)
{
    k %= L;
    if (k < 0) k += L;
    if ((4 * k) % L == 0) {
        static const double C4[4] = {1.0, 0.0, -1.0, 0.0}, S4[4] = {0.0, -1.0, 0.0, 1.0};
        const long q = 4 * k / L;
        *c = C4[q];
        *s = S4[q];
        return;
    }
    const double a = 2.0 * M_PI * (double)k / (double)L;
    *c = std::cos(a);
    *s = -std::sin(a);
}

long sfreq(long u, long L) { return u <= L / 2 ? u : u - L; }

// projection weights (t, x, y) of bin with signed frequencies (i, j, k); DC -> 0
void proj_w(long i, long j, long k, double w[3])
{
    const double rho = std::sqrt((double)(i * i + j * j + k * k));
    if (rho == 0.0) {
        w[0] = w[1] = w[2] = 0.0;
        return;
    }
    w[0] = std::sqrt((double)(j * j + k * k)) / rho;
    w[1] = std::sqrt((double)(i * i + k * k)) / rho;
    w[2] = std::sqrt((double)(i * i + j * j)) / rho;
}

uint16_t to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;  // round to nearest even (inputs are finite)
    return (uint16_t)(u >> 16);
}
float from_bf16(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
uint16_t to_f16(float f)
{
    _Float16 h = (_Float16)f;  // RNE
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}
float from_f16(uint16_t b)
{
    _Float16 h;
    std::memcpy(&h, &b, 2);
    return (float)h;
}

struct DevScope {
    int prev = -1;
    bool ok = false;
    explicit DevScope(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DevScope()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

sal_status fail(sal_ctx *c, sal_status s, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_create_err = msg;
    return s;
}

sal_status dev_fail(sal_ctx *c, hipError_t e, const char *where)
{
    return fail(c, SAL_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src)
{
    hipError_t e = hipMalloc((void **)dst, sizeof(T) * src.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

hipError_t build_tables(sal_ctx *c)
{
    const long L = c->L, h = c->h;
    const long L3 = L * L * L;
    const long MT = 2 * L / 16, MTA = (2 * h + 15) / 16;
    // w_c[(f, co)][(tap, ci)]: F = sum_tap e^{-2 pi i f tap / L} a_tap in real form
    std::vector<double> wc((size_t)(2 * L) * (2 * L));
    for (long f = 0; f < L; ++f)
        for (long tp = 0; tp < L; ++tp) {
            double cs, sn;
            twiddle(f * tp, L, &cs, &sn);
            wc[(2 * f) * 2 * L + 2 * tp] = cs;
            wc[(2 * f) * 2 * L + 2 * tp + 1] = -sn;
            wc[(2 * f + 1) * 2 * L + 2 * tp] = sn;
            wc[(2 * f + 1) * 2 * L + 2 * tp + 1] = cs;
        }
    std::vector<double> wa((size_t)16 * MTA * L, 0.0);
    for (long mu = 0; mu < h; ++mu)
        for (long p = 0; p < L; ++p) {
            double cs, sn;
            twiddle(mu * p, L, &cs, &sn);
            wa[(2 * mu) * L + p] = cs;
            wa[(2 * mu + 1) * L + p] = sn;
        }
    // Stage-C output order: slot s (M rows 2s, 2s+1, lane group (s mod 8) / 2 of M tile s / 8)
    // holds frequency ordc[s].  At cube 16 tile 0 pairs om with L - om in every lane (the
    // projection weights depend on squared frequencies, so both bins share them); the
    // x-stage matrices keep frequency order.
    std::vector<long> ordc(L);
    static const long ord16[16] = {1, 15, 2, 14, 3, 13, 4, 12, 5, 11, 6, 10, 7, 9, 0, 8};
    for (long s = 0; s < L; ++s) ordc[s] = L == 16 ? ord16[s] : s;
    auto crow = [&](long r) { return 2 * ordc[r / 2] + (r & 1); };  // stage-C M row -> w_c row
    // Weights of the two bins lane group g owns in M tile mt, for every group (mu, k),
    // k = 0..L/2: the row nu = k, joined by its mirror row nu = L - k when mu is not 0 or
    // L/2 (same squared frequencies, so same weights).  The multiplicity counts the
    // conjugate bins (-mu, -nu, -om) that the half spectrum leaves out; 1/L^3 of the DFT and
    // 1/(L^3 - 1) of the mean are folded in.
    std::vector<float> wb;
    // the FP16 forms scale the t and x stage outputs by 1/L each (range of FP16)
    const int pr = c->p.precision;
    const bool fp16_form = pr == SAL_FP16 || pr == SAL_FP16_SPLIT || pr == SAL_FP16_SPLITW;
    const double stage_gain = fp16_form ? (double)(L * L) : 1.0;
    const double scale = stage_gain / ((double)L3 * (double)(L3 - 1));
    for (long mu = 0; mu < h; ++mu) {
        const bool self = (mu == 0 || mu == L / 2);
        for (long nu = 0; nu <= L / 2; ++nu) {
            const double mult = (self && (nu == 0 || nu == L / 2)) ? 1.0 : 2.0;
            for (long mt = 0; mt < MT; ++mt)
                for (long g = 0; g < 4; ++g) {
                    float ent[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    for (long bb = 0; bb < 2; ++bb) {
                        const long om = ordc[8 * mt + 2 * g + bb];
                        double w[3];
                        proj_w(sfreq(mu, L), sfreq(nu, L), sfreq(om, L), w);
                        for (int m = 0; m < 3; ++m) ent[3 * bb + m] = (float)(w[m] * mult * scale);
                    }
                    wb.insert(wb.end(), ent, ent + 8);
                }
        }
    }
    std::vector<float> tw(2 * L);
    for (long k = 0; k < L; ++k) {
        double cs, sn;
        twiddle(k, L, &cs, &sn);
        tw[2 * k] = (float)cs;
        tw[2 * k + 1] = (float)sn;
        c->tw_host[2 * k] = (float)cs;
        c->tw_host[2 * k + 1] = (float)sn;
    }
    // vector-ALU kernels (L < 8, and the window-by-window kernel of every L): weights of
    // every bin (mu <= L/2, nu, om) with the multiplicity of the conjugate bin (-mu, -nu, -om)
    // the half spectrum leaves out, and 1/L^3 of the DFT and 1/(L^3 - 1) of the mean
    std::vector<float> wg;
    for (long mu = 0; mu < h; ++mu) {
        const double mult = (mu == 0 || 2 * mu == L) ? 1.0 : 2.0;
        for (long nu = 0; nu < L; ++nu)
            for (long om = 0; om < L; ++om) {
                double w[3];
                proj_w(sfreq(mu, L), sfreq(nu, L), sfreq(om, L), w);
                for (int m = 0; m < 3; ++m)
                    wg.push_back((float)(w[m] * mult / ((double)L3 * (double)(L3 - 1))));
            }
    }
    std::vector<float> wp((size_t)4 * L3, 0.f);
    for (long mu = 0; mu < L; ++mu)
        for (long nu = 0; nu < L; ++nu)
            for (long om = 0; om < L; ++om) {
                double w[3];
                proj_w(sfreq(mu, L), sfreq(nu, L), sfreq(om, L), w);
                const long b = (mu * L + nu) * L + om;
                for (int m = 0; m < 3; ++m) wp[4 * b + m] = (float)(w[m] / (double)(L3 - 1));
            }
    std::vector<float> wcf(wc.size()), waf(wa.size());
    for (long r = 0; r < 2 * L; ++r)
        for (long q = 0; q < 2 * L; ++q) wcf[r * 2 * L + q] = (float)wc[crow(r) * 2 * L + q];
    for (size_t i = 0; i < wa.size(); ++i) waf[i] = (float)wa[i];
    // 16-bit forms: hi = RNE(w), lo = RNE(w - hi) (lo = 0 when the matrix is not split),
    // laid out as the per-lane A operands of the 16x16x32 MFMAs in the K orders of
    // sal_energy16.hip
    const int prec = c->p.precision;
    const bool bf = prec == SAL_BF16 || prec == SAL_BF16_SPLIT || prec == SAL_BF16_SPLITW;
    const bool split = prec != SAL_BF16 && prec != SAL_FP16;
    const bool dsplit = prec == SAL_BF16_SPLIT || prec == SAL_FP16_SPLIT;
    auto r16 = [&](double v) -> uint16_t { return bf ? to_bf16((float)v) : to_f16((float)v); };
    auto f16v = [&](uint16_t b) -> double { return bf ? (double)from_bf16(b) : (double)from_f16(b); };
    auto part = [&](double v, int s) -> uint16_t {
        const uint16_t hi = r16(v);
        if (s == 0) return hi;
        return split ? r16(v - f16v(hi)) : (uint16_t)0;
    };
    auto word = [](uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); };
    // complex contractions: three products at cube 16 with the data split (A operands W_hi,
    // W_lo over taps 4g..4g+3), else J = L/8 MFMAs, lane group g holding part g >> 1 of taps
    // 8j + 4(g & 1)..+3; t contraction: TPL = L/4 taps per lane group, one word per tap
    // (two with the data split)
    const bool three = L == 16 && dsplit;
    const long J = L / 8, NA = three ? 2 : J, TPL = L / 4;
    const long NWA = dsplit ? 2 * TPL : TPL, JA = (NWA + 3) / 4;
    std::vector<uint32_t> c16((size_t)MT * NA * 64 * 4, 0u), a16((size_t)MTA * JA * 64 * 4, 0u);
    // cube 16, stage B in two halves of eight rows: half p holds the frequencies nu below,
    // so that the rows nu = k and 16 - k of every weight group lie in the same half
    static const long half_nu[2][8] = {{0, 1, 15, 2, 14, 3, 13, 8}, {4, 12, 5, 11, 6, 10, 7, 9}};
    // cube 16: stage-B operands of their own (halves' row order with the data split, else
    // frequency order per M tile)
    std::vector<uint32_t> c16b(L == 16 ? (size_t)2 * NA * 64 * 4 : 4, 0u);
    if (prec != SAL_FP32) {
        // A operand of M row `row` (freq, re|im) for lane group g, operand a, word w
        auto cword = [&](long row, long g, long a, long w) -> uint32_t {
            long q, prt;
            if (three) {
                q = 4 * g + w;
                prt = a;
            } else {
                q = 8 * a + 4 * (g & 1) + w;
                prt = g >> 1;
            }
            return word(part(wc[row * 2 * L + 2 * q], (int)prt), part(wc[row * 2 * L + 2 * q + 1], (int)prt));
        };
        for (long mt = 0; mt < MT; ++mt)
            for (long a = 0; a < NA; ++a)
                for (long lane = 0; lane < 64; ++lane)
                    for (long w = 0; w < 4; ++w)
                        c16[((mt * NA + a) * 64 + lane) * 4 + w] = cword(crow(16 * mt + lane % 16), lane / 16, a, w);
        if (L == 16 && !three)
            for (long mt = 0; mt < MT; ++mt)
                for (long a = 0; a < NA; ++a)
                    for (long lane = 0; lane < 64; ++lane)
                        for (long w = 0; w < 4; ++w)
                            c16b[((mt * NA + a) * 64 + lane) * 4 + w] = cword(16 * mt + lane % 16, lane / 16, a, w);
        if (three)
            for (long hp = 0; hp < 2; ++hp)
                for (long a = 0; a < NA; ++a)
                    for (long lane = 0; lane < 64; ++lane) {
                        const long i = lane % 16, row = 2 * half_nu[hp][i / 2] + (i & 1);
                        for (long w = 0; w < 4; ++w) c16b[((hp * NA + a) * 64 + lane) * 4 + w] = cword(row, lane / 16, a, w);
                    }
        for (long mt = 0; mt < MTA; ++mt)
            for (long ja = 0; ja < JA; ++ja)
                for (long lane = 0; lane < 64; ++lane) {
                    const long g = lane / 16, i = lane % 16;
                    for (long w = 0; w < 4; ++w) {
                        const long q = 4 * ja + w;
                        uint32_t v = 0u;
                        if (dsplit) {
                            // data word d_hi | d_lo against (W_part, W_part)
                            const long p = TPL * g + q / 2;
                            const uint16_t x = part(wa[(16 * mt + i) * L + p], (int)(q & 1));
                            v = word(x, x);
                        } else if (q < TPL) {
                            // data word d | d against (W_hi, W_lo)
                            const double x = wa[(16 * mt + i) * L + TPL * g + q];
                            v = word(part(x, 0), part(x, 1));
                        }
                        a16[((mt * JA + ja) * 64 + lane) * 4 + w] = v;
                    }
                }
    }
    // the FP32 kernel's stage-B halves at cube 16: lane (g, n) of K step kk holds row n of
    // the half's tile at K = KS g + kk, the tile's rows being (nu, re|im) of the half's list
    const long KSF = 2 * L / 4;
    std::vector<float> wcb(L == 16 ? (size_t)2 * KSF * 64 : 1, 0.f);
    if (L == 16)
        for (long hp = 0; hp < 2; ++hp)
            for (long kk = 0; kk < KSF; ++kk)
                for (long lane = 0; lane < 64; ++lane) {
                    const long g = lane / 16, i = lane % 16;
                    const long row = 2 * half_nu[hp][i / 2] + (i & 1);
                    wcb[(hp * KSF + kk) * 64 + lane] = (float)wc[row * 2 * L + KSF * g + kk];
                }
    // cube 8 and 16, FP32, windows sliding along t (sal_energy_slide.hip).  Stage 1 (real DFT
    // along x, packed): row 2c + part of column c: c = 0 holds X_0 (part 0) and X_{L/2}
    // (part 1), c >= 1 Re and Im of X_c; rows from L on are zero; A operand of lane (g, n) at
    // K step kk is row n, tap 4 kk + g.
    const bool slide = L == 8 || L == 16;
    const long SH = L / 2, NP = L / 2 + 1, SMT = L / 8, SWP = slide_weights_per_group((int)L);
    std::vector<float> ws1(slide ? (size_t)(L / 4) * 64 : 1, 0.f), ws2(slide ? (size_t)SMT * SH * 64 : 1, 0.f);
    std::vector<float> wsp(slide ? (size_t)SH * 4 * SWP : 1, 0.f);
    if (slide) {
        for (long kk = 0; kk < L / 4; ++kk)
            for (long lane = 0; lane < 64; ++lane) {
                const long g = lane / 16, row = lane % 16, tap = 4 * kk + g, col = row / 2, part = row % 2;
                if (row >= L) continue;
                double cs, sn;
                twiddle(col == 0 ? SH * part * tap : col * tap, L, &cs, &sn);
                ws1[kk * 64 + lane] = (float)(col == 0 ? cs : (part == 0 ? cs : sn));
            }
        // Stage 2 (complex DFT along y): M tile mt, lane group g' of the tile holds rows
        // (ky_a re, ky_a im, ky_b re, ky_b im) with (ky_a, ky_b) = (0, L/2) for mt = g' = 0,
        // else (4 mt + g', L - 4 mt - g'); K step kk of lane group g is tap 4 (kk / 2) + g,
        // input part kk mod 2.
        auto kyslot = [L, SH](long mt, long gg, long q) {
            return q == 0 ? 4 * mt + gg : (mt == 0 && gg == 0 ? SH : L - (4 * mt + gg));
        };
        for (long mt = 0; mt < SMT; ++mt)
            for (long kk = 0; kk < SH; ++kk)
                for (long lane = 0; lane < 64; ++lane) {
                    const long g = lane / 16, row = lane % 16;
                    const long ky = kyslot(mt, row / 4, (row % 4) / 2), po = row % 2;
                    const long tap = 4 * (kk / 2) + g, pi = kk % 2;
                    double cs, sn;  // W = cs + i sn = e^{-2 pi i ky tap / L}
                    twiddle(ky * tap, L, &cs, &sn);
                    const double v = po == 0 ? (pi == 0 ? cs : -sn) : (pi == 0 ? sn : cs);
                    ws2[(mt * SH + kk) * 64 + lane] = (float)v;
                }
        // Projection weights per (column c, lane group g), with 1/L^3 of the DFT and
        // 1/(L^3 - 1) of the mean; p = |kt| = 0..L/2, the slots kt and L - kt summed.  Columns
        // 1..L/2-1 (kx = c): each bin stands for itself and its conjugate (kx = L - c),
        // factor 2; M tile 0 per ky slot [q][p][m] (6 NP floats, NP = L/2 + 1), the other
        // M tiles [p][m] at 6 NP (the two slots are ky and -ky).  Column 0 (U = 2 D_{kx=0} and
        // V = 2i D_{kx=L/2} slots, each standing for a bin and its conjugate, factor 1):
        // M tile 0 [q][p][A|B][m] at 0 (12 NP floats), A weighing slot kt = p and B slot
        // L - p; on the self-conjugate rows (lane group 0: ky = 0, L/2) the slot L - p holds
        // conj V, and at p in {0, L/2} A weighs |Re Z| (kx = 0) and B |Im Z| (kx = L/2); the
        // other M tiles [q][p][m] at 12 NP.
        const double nrm = 1.0 / ((double)L3 * (double)(L3 - 1));
        for (long cc = 0; cc < SH; ++cc)
            for (long g = 0; g < 4; ++g) {
                float *o = wsp.data() + (cc * 4 + g) * SWP;
                double w[3];
                for (long p = 0; p < NP; ++p) {
                    if (cc > 0) {
                        for (long q = 0; q < 2; ++q) {
                            proj_w(p, cc, sfreq(kyslot(0, g, q), L), w);
                            for (int m = 0; m < 3; ++m) o[q * 3 * NP + 3 * p + m] = (float)(2.0 * w[m] * nrm);
                        }
                        if (SMT > 1) {
                            proj_w(p, cc, sfreq(kyslot(1, g, 0), L), w);
                            for (int m = 0; m < 3; ++m) o[6 * NP + 3 * p + m] = (float)(2.0 * w[m] * nrm);
                        }
                        continue;
                    }
                    for (long q = 0; q < 2; ++q) {
                        double wa[3], wbv[3];
                        if (g == 0) {
                            const long ky = SH * q;
                            proj_w(p, 0, ky, wa);
                            proj_w(p, SH, ky, wbv);
                        } else {
                            proj_w(p, SH * q, g, wa);
                            for (int m = 0; m < 3; ++m) wbv[m] = (p == 0 || p == SH) ? 0.0 : wa[m];
                        }
                        for (int m = 0; m < 3; ++m) {
                            o[(q * NP + p) * 6 + m] = (float)(wa[m] * nrm);
                            o[(q * NP + p) * 6 + 3 + m] = (float)(wbv[m] * nrm);
                        }
                        if (SMT > 1) {
                            proj_w(p, SH * q, sfreq(kyslot(1, g, 0), L), w);
                            for (int m = 0; m < 3; ++m) o[12 * NP + (q * NP + p) * 3 + m] = (float)(w[m] * nrm);
                        }
                    }
                }
            }
    }
    hipError_t e;
    if ((e = upload(&c->t.w_c, wcf)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_cb, wcb)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_s1, ws1)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_s2, ws2)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_sp, wsp)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_a, waf)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_bin, wb)) != hipSuccess) return e;
    if ((e = upload(&c->t.twiddle, tw)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_proj, wp)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_c16, c16)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_a16, a16)) != hipSuccess) return e;
    if ((e = upload(&c->t.w_c16b, c16b)) != hipSuccess) return e;
    if (!wg.empty() && (e = upload(&c->t.w_gen, wg)) != hipSuccess) return e;
    return hipSuccess;
}

void free_tables(sal_tables *t)
{
    float **fp[] = {&t->w_c, &t->w_a, &t->w_bin, &t->twiddle, &t->w_proj, &t->w_gen, &t->w_cb,
                    &t->w_s1, &t->w_s2, &t->w_sp};
    for (float **p : fp)
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    if (t->w_c16) (void)hipFree(t->w_c16);
    if (t->w_a16) (void)hipFree(t->w_a16);
    if (t->w_c16b) (void)hipFree(t->w_c16b);
    t->w_c16 = t->w_a16 = t->w_c16b = nullptr;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
    size_t e, s_raw, vmax, mm, stats, e_lat, total;
};

// lattice sizes K = ceil(n / stride) of the window positions
void lattice_dims(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2, int64_t K[3])
{
    const int S = c->p.stride;
    K[0] = (n0 + S - 1) / S;
    K[1] = (n1 + S - 1) / S;
    K[2] = (n2 + S - 1) / S;
}

WsLayout ws_layout(const sal_ctx *c, int64_t n0, int64_t n1, int64_t n2)
{
    const size_t N = (size_t)n0 * n1 * n2;
    int64_t K[3];
    lattice_dims(c, n0, n1, n2, K);
    WsLayout w;
    w.e = 0;
    w.s_raw = w.e + align256(3 * N * sizeof(float));
    w.vmax = w.s_raw + align256(3 * N * sizeof(float));
    w.mm = w.vmax + align256((size_t)energy_num_blocks(c, n0, n1, n2) * sizeof(float));
    w.stats = w.mm + align256((size_t)dcs_num_blocks(c, n0, n1, n2) * 6 * sizeof(float));
    w.e_lat = w.stats + align256(8 * sizeof(double));
    w.total = w.e_lat + (c->p.stride > 1 ? align256((size_t)3 * K[0] * K[1] * K[2] * sizeof(float)) : 0);
    return w;
}

sal_status check_dims(sal_ctx *c, int64_t n0, int64_t n1, int64_t n2)
{
    const int64_t need = (c->H > c->r ? c->H : c->r);
    if (n0 <= need || n1 <= need || n2 <= need)
        return fail(c, SAL_E_INVAL, "every dimension must exceed max(floor(L/2), r) = " +
                                        std::to_string(need));
    if (n0 > (1 << 30) || n1 > (1 << 30) || n2 > (1 << 30) ||
        n0 * n1 * n2 > ((int64_t)1 << 31) - 1 || n1 * n2 > ((int64_t)1 << 31) - 1)
        return fail(c, SAL_E_INVAL, "volume too large (at most 2^31-1 voxels)");
    return SAL_OK;
}

void release_events(sal_ctx *c)
{
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    c->ev_pool.clear();
    c->ev_used = 0;
}

// Events for one timed call (5 marks), or nullptr if profiling is off or creation fails.
hipEvent_t *take_events(sal_ctx *c)
{
    if (!c->profiling) return nullptr;
    while (c->ev_pool.size() < c->ev_used + 5) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    hipEvent_t *ev = &c->ev_pool[c->ev_used];
    c->ev_used += 5;
    return ev;
}

sal_status sticky(sal_ctx *c)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dev_fail(c, e, "earlier device error");
    return SAL_OK;
}

}  // namespace

// Device scratch of sal_saliency_noalloc (per-block partials and statistics), one copy per
// GPU for the life of the process.  Host code never uses this name as an address: the
// device address of each GPU's copy is looked up once per device (with that device current)
// and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[SAL_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch;  // device address of `scratch` per device, NULL until looked up

// With `dev` current: the address of this device's scratch (looked up on first use).
hipError_t scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

void sal_default_params(sal_params *p, int32_t L)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->L = L;
    p->d = L;
    p->sigma = (double)L / 4.0;
    p->rays[0] = SAL_RAY_PT | SAL_RAY_MT;
    p->rays[1] = SAL_RAY_PX | SAL_RAY_MX;
    p->rays[2] = SAL_RAY_PY | SAL_RAY_MY;
    p->a = p->b = p->c = 1.0 / 3.0;
    p->normalize = 1;
    p->zero_range = 1e-6;
    p->precision = SAL_FP32;
    p->stride = 1;
}

sal_status sal_create(const sal_params *p, int device, sal_ctx **out)
{
    if (!p || !out) return fail(nullptr, SAL_E_INVAL, "null params or output pointer");
    *out = nullptr;
    if (p->L < 2) return fail(nullptr, SAL_E_INVAL, "L must be >= 2");
    if (p->d < 2 || p->d > 64) return fail(nullptr, SAL_E_INVAL, "d must be in [2, 64]");
    if (!(p->sigma > 0.0)) return fail(nullptr, SAL_E_INVAL, "sigma must be > 0 (may be inf)");
    for (int m = 0; m < 3; ++m)
        if (p->rays[m] == 0 || p->rays[m] > (uint32_t)SAL_RAY_ALL)
            return fail(nullptr, SAL_E_INVAL, "each ray mask must be a nonempty subset of the 26 rays");
    if (p->precision < SAL_FP32 || p->precision > SAL_FP16_SPLITW)
        return fail(nullptr, SAL_E_INVAL, "unknown precision");
    if (!(p->zero_range >= 0.0)) return fail(nullptr, SAL_E_INVAL, "zero_range must be >= 0");
    if (p->L > 20) return fail(nullptr, SAL_E_UNSUPPORTED, "the GPU build implements L = 2..20");
    if (p->stride < 1) return fail(nullptr, SAL_E_INVAL, "stride must be >= 1");
    if (p->stride > 1 && 2 * p->stride >= p->L && p->stride != p->L)
        return fail(nullptr, SAL_E_INVAL,
                    "stride must be below L/2 (windows overlap by more than half) or equal L (no overlap)");
    if (p->precision != SAL_FP32 && (p->L != 8 && p->L != 16))
        return fail(nullptr, SAL_E_UNSUPPORTED, "16-bit forms exist for L = 8 and 16 only");
    if (p->precision != SAL_FP32 && p->stride > 2)
        return fail(nullptr, SAL_E_UNSUPPORTED, "strides above 2 run in FP32 only");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(nullptr, SAL_E_DEVICE, "no such HIP device");
    DevScope ds(device);
    if (!ds.ok) return fail(nullptr, SAL_E_DEVICE, "hipSetDevice failed");
    sal_ctx *c = new (std::nothrow) sal_ctx();
    if (!c) return fail(nullptr, SAL_E_DEVICE, "out of host memory");
    c->p = *p;
    c->device = device;
    c->L = p->L;
    c->H = p->L / 2;
    c->h = p->L / 2 + 1;
    c->r = p->d / 2;
    c->nrows = (c->h - 2) * c->L + 2 * (c->L / 2 + 1);
    // neighbour weights at distance s |e| for the three step lengths |e|^2 = 1, 2, 3
    for (int k = 1; k <= 3; ++k)
        for (int s = 0; s < 32; ++s)
            c->g[32 * (k - 1) + s] = (s < c->r) ? (float)std::exp(-(double)((s + 1) * (s + 1) * k) /
                                                                  (2.0 * p->sigma * p->sigma))
                                                : 0.f;
    for (int m = 0; m < 3; ++m) {
        int nr = 0;
        for (int b = 0; b < 26; ++b) nr += (p->rays[m] >> b) & 1;
        c->Q[m] = (float)(nr * c->r);
    }
    hipError_t e = build_tables(c);
    if (e != hipSuccess) {
        free_tables(&c->t);
        delete c;
        return fail(nullptr, SAL_E_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
    }
    if ((e = scratch_address(device, &c->scratch)) != hipSuccess) {
        free_tables(&c->t);
        delete c;
        return fail(nullptr, SAL_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    }
    *out = c;
    return SAL_OK;
}

void sal_destroy(sal_ctx *c)
{
    if (!c) return;
    DevScope ds(c->device);
    release_events(c);
    free_tables(&c->t);
    if (c->tab_done) {
        (void)hipEventSynchronize(c->tab_done);
        (void)hipEventDestroy(c->tab_done);
    }
    if (c->tab_host) (void)hipHostFree(c->tab_host);
    delete c;
}

const char *sal_last_error(const sal_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

sal_status sal_workspace_size(sal_ctx *c, int64_t n0, int64_t n1, int64_t n2, size_t *bytes)
{
    if (!c || !bytes) return fail(c, SAL_E_INVAL, "null argument");
    sal_status st = check_dims(c, n0, n1, n2);
    if (st != SAL_OK) return st;
    *bytes = ws_layout(c, n0, n1, n2).total;
    return SAL_OK;
}

sal_status sal_local_spectra(sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2,
                             const int64_t lo[3], const int64_t bn[3], void *spectra, void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!V || !lo || !bn || !spectra) return fail(c, SAL_E_INVAL, "null pointer");
    if (!aligned16(V) || !aligned16(spectra)) return fail(c, SAL_E_INVAL, "pointers must be 16-byte aligned");
    sal_status st = check_dims(c, n0, n1, n2);
    if (st != SAL_OK) return st;
    const int64_t n[3] = {n0, n1, n2};
    for (int a = 0; a < 3; ++a)
        if (lo[a] < 0 || bn[a] < 0 || lo[a] + bn[a] > n[a])
            return fail(c, SAL_E_INVAL, "box outside the volume");
    if (bn[0] * bn[1] * bn[2] > (int64_t)1 << 24) return fail(c, SAL_E_INVAL, "box too large");
    DevScope ds(c->device);
    if ((st = sticky(c)) != SAL_OK) return st;
    hipError_t e = launch_local_spectra(c, V, n0, n1, n2, lo, bn, (float *)spectra, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(c, e, "local spectra launch");
    return SAL_OK;
}

sal_status sal_project(sal_ctx *c, const void *spectra, int64_t nvox, float *E, void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!spectra || !E) return fail(c, SAL_E_INVAL, "null pointer");
    if (!aligned16(spectra) || !aligned16(E)) return fail(c, SAL_E_INVAL, "pointers must be 16-byte aligned");
    if (nvox < 0 || nvox > ((int64_t)1 << 31) - 1) return fail(c, SAL_E_INVAL, "bad voxel count");
    DevScope ds(c->device);
    sal_status st;
    if ((st = sticky(c)) != SAL_OK) return st;
    hipError_t e = launch_project(c, (const float *)spectra, nvox, E, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(c, e, "project launch");
    return SAL_OK;
}

sal_status sal_directional_compare(sal_ctx *c, const float *E, int64_t n0, int64_t n1, int64_t n2,
                                   float *S_raw, void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!E || !S_raw) return fail(c, SAL_E_INVAL, "null pointer");
    if (!aligned16(E) || !aligned16(S_raw)) return fail(c, SAL_E_INVAL, "pointers must be 16-byte aligned");
    sal_status st = check_dims(c, n0, n1, n2);
    if (st != SAL_OK) return st;
    const size_t bytes = (size_t)3 * n0 * n1 * n2 * sizeof(float);
    const char *a = (const char *)E, *b = (const char *)S_raw;
    if (a < b + bytes && b < a + bytes) return fail(c, SAL_E_INVAL, "E and S_raw overlap");
    DevScope ds(c->device);
    if ((st = sticky(c)) != SAL_OK) return st;
    hipError_t e = launch_dcs(c, E, n0, n1, n2, S_raw, nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(c, e, "dcs launch");
    return SAL_OK;
}

// The launch sequence of the whole method (steps 1-5) on caller-placed buffers: E and Sr
// the maps, vmax and mm the per-block partials of the energy and comparison kernels, stats
// the FP64 statistics, El the lattice energies (stride > 1); ev (optional) five events.
static sal_status run_saliency(sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, float *S, float *E,
                               float *Sr, float *vmax, float *mm, double *stats, float *El, hipStream_t s,
                               hipEvent_t *ev)
{
    const int64_t N = n0 * n1 * n2;
    int nv = 0;
    if (ev) (void)hipEventRecord(ev[0], s);
    hipError_t e;
    if (c->p.stride > 1) {
        // windows on the lattice, energies interpolated onto every voxel
        int64_t K[3];
        lattice_dims(c, n0, n1, n2, K);
        e = launch_energy(c, V, n0, n1, n2, nullptr, El, vmax, &nv, s);
        if (e != hipSuccess) return dev_fail(c, e, "energy launch");
        e = launch_upsample(El, K[0], K[1], K[2], c->p.stride, n0, n1, n2, E, s);
    } else {
        e = launch_energy(c, V, n0, n1, n2, nullptr, E, vmax, &nv, s);
    }
    if (e != hipSuccess) return dev_fail(c, e, "energy launch");
    if (ev) (void)hipEventRecord(ev[1], s);
    e = launch_dcs(c, E, n0, n1, n2, Sr, mm, s);
    if (e != hipSuccess) return dev_fail(c, e, "dcs launch");
    if (ev) (void)hipEventRecord(ev[2], s);
    e = launch_stats(vmax, nv, mm, dcs_num_blocks(c, n0, n1, n2), stats, s);
    if (e != hipSuccess) return dev_fail(c, e, "stats launch");
    if (ev) (void)hipEventRecord(ev[3], s);
    e = launch_combine(Sr, N, stats, c->p.a, c->p.b, c->p.c, c->p.normalize, c->p.zero_range, S, s);
    if (e != hipSuccess) return dev_fail(c, e, "combine launch");
    if (ev) (void)hipEventRecord(ev[4], s);
    return SAL_OK;
}

sal_status sal_saliency(sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, float *S,
                        float *E_out, float *S_raw_out, double *stats_out, void *workspace,
                        size_t ws_bytes, void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!V || !S || !workspace) return fail(c, SAL_E_INVAL, "null pointer");
    if (!aligned16(V) || !aligned16(S) || !aligned16(workspace) || (E_out && !aligned16(E_out)) ||
        (S_raw_out && !aligned16(S_raw_out)) || (stats_out && !aligned16(stats_out)))
        return fail(c, SAL_E_INVAL, "pointers must be 16-byte aligned");
    sal_status st = check_dims(c, n0, n1, n2);
    if (st != SAL_OK) return st;
    const WsLayout w = ws_layout(c, n0, n1, n2);
    if (ws_bytes < w.total)
        return fail(c, SAL_E_WORKSPACE, "workspace too small: need " + std::to_string(w.total) + " bytes");
    DevScope ds(c->device);
    if ((st = sticky(c)) != SAL_OK) return st;
    char *ws = (char *)workspace;
    float *E = E_out ? E_out : (float *)(ws + w.e);
    float *Sr = S_raw_out ? S_raw_out : (float *)(ws + w.s_raw);
    double *stats = stats_out ? stats_out : (double *)(ws + w.stats);
    return run_saliency(c, V, n0, n1, n2, S, E, Sr, (float *)(ws + w.vmax), (float *)(ws + w.mm), stats,
                        (float *)(ws + w.e_lat), (hipStream_t)stream, take_events(c));
}

sal_status sal_saliency_noalloc(sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, float *S,
                                float *E_out, float *S_raw_out, double *stats_out, void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!V || !S || !E_out || !S_raw_out) return fail(c, SAL_E_INVAL, "null pointer (V, S, E_out and S_raw_out are required)");
    if (!aligned16(V) || !aligned16(S) || !aligned16(E_out) || !aligned16(S_raw_out) ||
        (stats_out && !aligned16(stats_out)))
        return fail(c, SAL_E_INVAL, "pointers must be 16-byte aligned");
    if (c->p.stride != 1) return fail(c, SAL_E_UNSUPPORTED, "sal_saliency_noalloc computes stride 1 only");
    sal_status st = check_dims(c, n0, n1, n2);
    if (st != SAL_OK) return st;
    // the per-block partials and the statistics live in the library's device scratch
    const size_t o_mm = align256((size_t)energy_num_blocks(c, n0, n1, n2) * sizeof(float));
    const size_t o_st = o_mm + align256((size_t)dcs_num_blocks(c, n0, n1, n2) * 6 * sizeof(float));
    const size_t need = o_st + align256(8 * sizeof(double));
    if (need > SAL_NOALLOC_SCRATCH_BYTES)
        return fail(c, SAL_E_INVAL, "volume needs " + std::to_string(need) + " bytes of scratch; the limit is " +
                                        std::to_string((size_t)SAL_NOALLOC_SCRATCH_BYTES));
    DevScope ds(c->device);
    if ((st = sticky(c)) != SAL_OK) return st;
    char *ws = (char *)c->scratch;
    double *stats = stats_out ? stats_out : (double *)(ws + o_st);
    return run_saliency(c, V, n0, n1, n2, S, E_out, S_raw_out, (float *)ws, (float *)(ws + o_mm), stats, nullptr,
                        (hipStream_t)stream, nullptr);
}

// The box grown by r along every axis, clipped to the volume: E of these positions holds
// every neighbour Eq. (5) reads for the box.
static void grow_box(const sal_ctx *c, const int64_t n[3], const int64_t lo[3], const int64_t bd[3], int64_t eo[3],
              int64_t ed[3])
{
    for (int a = 0; a < 3; ++a) {
        eo[a] = lo[a] - c->r > 0 ? lo[a] - c->r : 0;
        const int64_t hi = lo[a] + bd[a] + c->r < n[a] ? lo[a] + bd[a] + c->r : n[a];
        ed[a] = hi - eo[a];
    }
}

// Windows on the stride-S lattice: the lattice points whose interpolation reaches the
// voxels eo + [0, ed) (floor(u/S) and the next one, held at the last point K - 1), as the
// lattice index range klo + [0, kd) and the voxel box {o, d} whose lattice they are.
static void lattice_box(const sal_ctx *c, const int64_t n[3], const int64_t eo[3], const int64_t ed[3], int64_t klo[3],
                        int64_t kd[3], int64_t K[3], int64_t vbox[6])
{
    const int64_t S = c->p.stride;
    for (int a = 0; a < 3; ++a) {
        K[a] = (n[a] + S - 1) / S;
        klo[a] = eo[a] / S;
        int64_t khi = (eo[a] + ed[a] - 1) / S + 1;
        if (khi > K[a] - 1) khi = K[a] - 1;
        kd[a] = khi - klo[a] + 1;
        vbox[a] = klo[a] * S;
        vbox[3 + a] = (kd[a] - 1) * S + 1;
    }
}

// An upper bound of the energy kernels' workgroups for a box of k window positions per axis
// that grows with the box: every fused tile holds at least 8 x 16 positions and walks at
// least 2 of them along t; a sliding one holds one x position and 16 y positions for every
// t segment its k[0] stride rows touch; the window-by-window kernel launches at most 4096.
static int64_t energy_blocks_bound(const sal_ctx *c, const int64_t k[3])
{
    const int64_t slide = ((k[0] * c->p.stride + SLIDE_SEG - 1) / SLIDE_SEG + 2) * k[1] * ((k[2] + 15) / 16);
    const int64_t other = uses_window_kernel(c) ? 4096 : ((k[1] + 7) / 8) * ((k[2] + 15) / 16) * ((k[0] + 1) / 2);
    return other > slide ? other : slide;
}

// workspace of sal_raw_box: E of the grown box, then (stride > 1) the lattice energies it
// interpolates, then the energy kernel's partials; kd bounds the lattice box
static size_t raw_box_ws(const sal_ctx *c, const int64_t ed[3], const int64_t kd[3])
{
    const int64_t S = c->p.stride;
    size_t w = align256((size_t)3 * ed[0] * ed[1] * ed[2] * sizeof(float));
    if (S > 1) w += align256((size_t)3 * kd[0] * kd[1] * kd[2] * sizeof(float));
    const int64_t nb = energy_blocks_bound(c, S > 1 ? kd : ed);
    return w + align256((size_t)nb * sizeof(float));
}

sal_status sal_raw_box_workspace_size(sal_ctx *c, const int64_t box_dims[3], size_t *bytes)
{
    if (!c || !box_dims || !bytes) return fail(c, SAL_E_INVAL, "null argument");
    int64_t ed[3], kd[3];
    for (int a = 0; a < 3; ++a) {
        if (box_dims[a] < 1 || box_dims[a] > (1 << 20)) return fail(c, SAL_E_INVAL, "bad box size");
        ed[a] = box_dims[a] + 2 * c->r;
        kd[a] = (ed[a] - 1) / c->p.stride + 3;  // at most this many lattice points reach a box of ed
    }
    *bytes = raw_box_ws(c, ed, kd);
    return SAL_OK;
}

sal_status sal_raw_box(sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, const int64_t box_lo[3],
                       const int64_t box_dims[3], float *S_raw_box, void *workspace, size_t ws_bytes, void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!V || !box_lo || !box_dims || !S_raw_box || !workspace) return fail(c, SAL_E_INVAL, "null pointer");
    if (!aligned16(V) || !aligned16(S_raw_box) || !aligned16(workspace))
        return fail(c, SAL_E_INVAL, "pointers must be 16-byte aligned");
    sal_status st = check_dims(c, n0, n1, n2);
    if (st != SAL_OK) return st;
    const int64_t n[3] = {n0, n1, n2};
    for (int a = 0; a < 3; ++a)
        if (box_lo[a] < 0 || box_dims[a] < 1 || box_lo[a] + box_dims[a] > n[a])
            return fail(c, SAL_E_INVAL, "box outside the volume");
    int64_t eo[3], ed[3], klo[3], kd[3], K[3], vbox[6];
    grow_box(c, n, box_lo, box_dims, eo, ed);
    lattice_box(c, n, eo, ed, klo, kd, K, vbox);
    const size_t need = raw_box_ws(c, ed, kd);
    if (ws_bytes < need) return fail(c, SAL_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    DevScope ds(c->device);
    if ((st = sticky(c)) != SAL_OK) return st;
    char *ws = (char *)workspace;
    float *Eb = (float *)ws;
    size_t off = align256((size_t)3 * ed[0] * ed[1] * ed[2] * sizeof(float));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (c->p.stride > 1) {
        // the lattice energies around the grown box, interpolated onto it
        float *El = (float *)(ws + off);
        off += align256((size_t)3 * kd[0] * kd[1] * kd[2] * sizeof(float));
        e = launch_energy(c, V, n0, n1, n2, vbox, El, (float *)(ws + off), nullptr, s);
        if (e != hipSuccess) return dev_fail(c, e, "energy launch");
        e = launch_upsample_box(El, kd, klo, K, c->p.stride, eo, ed, Eb, s);
        if (e != hipSuccess) return dev_fail(c, e, "upsample launch");
    } else {
        const int64_t box[6] = {eo[0], eo[1], eo[2], ed[0], ed[1], ed[2]};
        e = launch_energy(c, V, n0, n1, n2, box, Eb, (float *)(ws + off), nullptr, s);
        if (e != hipSuccess) return dev_fail(c, e, "energy launch");
    }
    e = launch_dcs_box(c, Eb, eo, ed, n, box_lo, box_dims, S_raw_box, s);
    if (e != hipSuccess) return dev_fail(c, e, "dcs launch");
    return SAL_OK;
}

// Energy boxes one tile's check needs, inside the tile's grown box (eo, ed).  Eq. (5) reads
// E_m only along the rays of map m: with axis rays only, that is the tile grown by r along y
// (when some ray runs along y) plus slabs of r beyond its faces along t and along x (when
// some ray runs along them); reflected neighbours stay inside the same ranges.  With a
// diagonal ray, the whole grown box.  Returns the boxes as {o[3], d[3]}.
static int check_boxes(const sal_ctx *c, const int64_t lo[3], const int64_t td[3], const int64_t eo[3],
                       const int64_t ed[3], int64_t out[5][6])
{
    uint32_t any = 0;
    for (int m = 0; m < 3; ++m) any |= c->p.rays[m];
    auto put = [&](int k, const int64_t o[3], const int64_t d[3]) {
        for (int a = 0; a < 3; ++a) {
            out[k][a] = o[a];
            out[k][3 + a] = d[a];
        }
    };
    if (any >> 6) {
        put(0, eo, ed);
        return 1;
    }
    const bool along[3] = {(any & 3u) != 0, (any & 12u) != 0, (any & 48u) != 0};
    int k = 0;
    {
        int64_t o[3] = {lo[0], lo[1], lo[2]}, d[3] = {td[0], td[1], td[2]};
        if (along[2]) {
            o[2] = eo[2];
            d[2] = ed[2];
        }
        put(k++, o, d);
    }
    for (int a = 0; a < 2; ++a) {
        if (!along[a]) continue;
        int64_t o[3] = {lo[0], lo[1], lo[2]}, d[3] = {td[0], td[1], td[2]};
        o[a] = eo[a];
        d[a] = lo[a] - eo[a];
        if (d[a] > 0) put(k++, o, d);
        o[a] = lo[a] + td[a];
        d[a] = eo[a] + ed[a] - o[a];
        if (d[a] > 0) put(k++, o, d);
    }
    return k;
}

// workspace of sal_check_tiles: E of every grown box, the exact tile maps, and the tables
// (at most five energy boxes per tile)
// With windows on a lattice (stride > 1), one energy box per tile: its lattice box, whose
// energies (lstride floats apart) are interpolated onto the grown box (LAT_TABLE ints each).
struct CheckWs {
    size_t e, exact, lat, table, total;
    int64_t maxg[3], estride, maxkd[3], lstride;
};
static CheckWs check_ws(const sal_ctx *c, const int64_t n[3], int64_t nbox, const int64_t td[3])
{
    CheckWs w;
    const int64_t S = c->p.stride;
    for (int a = 0; a < 3; ++a) {
        w.maxg[a] = td[a] + 2 * c->r < n[a] ? td[a] + 2 * c->r : n[a];
        w.maxkd[a] = S > 1 ? (w.maxg[a] - 1) / S + 3 : 0;
    }
    w.estride = 3 * w.maxg[0] * w.maxg[1] * w.maxg[2];
    w.lstride = 3 * w.maxkd[0] * w.maxkd[1] * w.maxkd[2];
    w.e = 0;
    w.exact = w.e + align256((size_t)nbox * w.estride * sizeof(float));
    w.lat = w.exact + align256((size_t)nbox * 3 * td[0] * td[1] * td[2] * sizeof(float));
    w.table = w.lat + (S > 1 ? align256((size_t)nbox * w.lstride * sizeof(float)) : 0);
    w.total = w.table + align256((size_t)nbox * (5 * ENERGY_TABLE + BOX_TABLE + (S > 1 ? LAT_TABLE : 0)) * sizeof(int));
    return w;
}

static sal_status check_tile_args(sal_ctx *c, int64_t n0, int64_t n1, int64_t n2, int64_t nbox,
                                  const int64_t td[3])
{
    sal_status st = check_dims(c, n0, n1, n2);
    if (st != SAL_OK) return st;
    if (nbox < 1 || nbox > (1 << 20)) return fail(c, SAL_E_INVAL, "nbox must be in [1, 2^20]");
    for (int a = 0; a < 3; ++a)
        if (td[a] < 1 || td[a] > 1024) return fail(c, SAL_E_INVAL, "tile sides must be in [1, 1024]");
    return SAL_OK;
}

sal_status sal_check_tiles_workspace_size(sal_ctx *c, int64_t n0, int64_t n1, int64_t n2, int64_t nbox,
                                          const int64_t tile_dims[3], size_t *bytes)
{
    if (!c || !tile_dims || !bytes) return fail(c, SAL_E_INVAL, "null argument");
    sal_status st = check_tile_args(c, n0, n1, n2, nbox, tile_dims);
    if (st != SAL_OK) return st;
    const int64_t n[3] = {n0, n1, n2};
    *bytes = check_ws(c, n, nbox, tile_dims).total;
    return SAL_OK;
}

sal_status sal_check_tiles(sal_ctx *c, const float *V, int64_t n0, int64_t n1, int64_t n2, int64_t vol_stride,
                           const int64_t *box_lo, float *S_raw, int64_t m0, int64_t m1, int64_t m2,
                           const int64_t *tile_lo, int64_t nbox, const int64_t tile_dims[3], const double *stats,
                           double bound, float *err_out, float *exact_out, void *workspace, size_t ws_bytes,
                           void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!V || !box_lo || !S_raw || !tile_lo || !tile_dims || !stats || !err_out || !workspace)
        return fail(c, SAL_E_INVAL, "null pointer");
    if (!aligned16(V) || !aligned16(S_raw) || !aligned16(workspace) || (exact_out && !aligned16(exact_out)))
        return fail(c, SAL_E_INVAL, "pointers must be 16-byte aligned");
    sal_status st = check_tile_args(c, n0, n1, n2, nbox, tile_dims);
    if (st != SAL_OK) return st;
    if (m0 < 1 || m1 < 1 || m2 < 1 || m0 * m1 * m2 > ((int64_t)1 << 31) - 1)
        return fail(c, SAL_E_INVAL, "map dimensions out of range");
    const int64_t N = n0 * n1 * n2;
    if (vol_stride != 0 && (vol_stride < N || (vol_stride & 3) != 0))
        return fail(c, SAL_E_INVAL, "vol_stride must be 0 or a multiple of 4 of at least n0 n1 n2");
    if (!(bound >= 0.0)) return fail(c, SAL_E_INVAL, "bound must be >= 0");
    const int64_t n[3] = {n0, n1, n2}, m[3] = {m0, m1, m2};
    // energy boxes (ENERGY_TABLE ints each) first, then one BOX_TABLE entry per tile
    std::vector<int> etab, ttab((size_t)nbox * BOX_TABLE, 0), ltab;
    etab.reserve((size_t)nbox * 5 * ENERGY_TABLE);
    int64_t maxd[3] = {1, 1, 1};
    for (int64_t b = 0; b < nbox; ++b) {
        const int64_t *lo = box_lo + 3 * b, *to = tile_lo + 3 * b;
        for (int a = 0; a < 3; ++a) {
            if (lo[a] < 0 || lo[a] + tile_dims[a] > n[a])
                return fail(c, SAL_E_INVAL, "box " + std::to_string(b) + " outside its volume");
            if (to[a] < 0 || to[a] + tile_dims[a] > m[a])
                return fail(c, SAL_E_INVAL, "tile " + std::to_string(b) + " outside the map");
        }
        int64_t eo[3], ed[3], sub[5][6];
        grow_box(c, n, lo, tile_dims, eo, ed);
        int *q = &ttab[(size_t)b * BOX_TABLE];
        for (int a = 0; a < 3; ++a) {
            q[a] = (int)eo[a];
            q[3 + a] = (int)ed[a];
            q[6 + a] = (int)lo[a];
            q[9 + a] = (int)to[a];
        }
        if (c->p.stride > 1) {
            // the lattice box around the grown box, framed by itself; then its interpolation
            int64_t klo[3], kd[3], K[3], vbox[6];
            lattice_box(c, n, eo, ed, klo, kd, K, vbox);
            const int e[ENERGY_TABLE] = {(int)vbox[0], (int)vbox[1], (int)vbox[2], (int)vbox[3], (int)vbox[4],
                                         (int)vbox[5], (int)vbox[0], (int)vbox[1], (int)vbox[2], (int)kd[0],
                                         (int)kd[1], (int)kd[2], (int)b, 0, 0, 0};
            etab.insert(etab.end(), e, e + ENERGY_TABLE);
            const int l[LAT_TABLE] = {(int)kd[0], (int)kd[1], (int)kd[2], (int)klo[0], (int)klo[1], (int)klo[2],
                                      (int)K[0], (int)K[1], (int)K[2], (int)eo[0], (int)eo[1], (int)eo[2],
                                      (int)ed[0], (int)ed[1], (int)ed[2]};
            ltab.insert(ltab.end(), l, l + LAT_TABLE);
            for (int a = 0; a < 3; ++a) maxd[a] = vbox[3 + a] > maxd[a] ? vbox[3 + a] : maxd[a];
            continue;
        }
        const int k = check_boxes(c, lo, tile_dims, eo, ed, sub);
        for (int i = 0; i < k; ++i) {
            const int e[ENERGY_TABLE] = {(int)sub[i][0], (int)sub[i][1], (int)sub[i][2], (int)sub[i][3],
                                         (int)sub[i][4], (int)sub[i][5], (int)eo[0], (int)eo[1], (int)eo[2],
                                         (int)ed[0], (int)ed[1], (int)ed[2], (int)b, 0, 0, 0};
            etab.insert(etab.end(), e, e + ENERGY_TABLE);
            for (int a = 0; a < 3; ++a) maxd[a] = sub[i][3 + a] > maxd[a] ? sub[i][3 + a] : maxd[a];
        }
    }
    const int nent = (int)(etab.size() / ENERGY_TABLE);
    const CheckWs w = check_ws(c, n, nbox, tile_dims);
    // every workgroup of the energy grid covers at least one voxel of an entry's largest box
    if ((double)nent * maxd[0] * maxd[1] * maxd[2] > 2147483647.0)
        return fail(c, SAL_E_INVAL, "batch too large: split the tiles over several calls");
    if (ws_bytes < w.total) return fail(c, SAL_E_WORKSPACE, "workspace too small: need " + std::to_string(w.total) + " bytes");
    DevScope ds(c->device);
    if ((st = sticky(c)) != SAL_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // The box tables come from host memory at call time, so a captured graph would replay
    // the upload of whatever the staging buffer holds then: refuse capture.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return dev_fail(c, e, "stream capture query");
    if (cap != hipStreamCaptureStatusNone)
        return fail(c, SAL_E_UNSUPPORTED, "sal_check_tiles cannot be captured into a graph");
    char *ws = (char *)workspace;
    float *Eb = (float *)(ws + w.e);
    float *X = exact_out ? exact_out : (float *)(ws + w.exact);
    int *etab_d = (int *)(ws + w.table), *ttab_d = etab_d + etab.size(), *ltab_d = ttab_d + ttab.size();
    etab.insert(etab.end(), ttab.begin(), ttab.end());
    etab.insert(etab.end(), ltab.begin(), ltab.end());
    // stage the tables in the context's pinned buffer, once the previous upload from it is done
    if (!c->tab_done && (e = hipEventCreateWithFlags(&c->tab_done, hipEventDisableTiming)) != hipSuccess)
        return dev_fail(c, e, "event create");
    if ((e = hipEventSynchronize(c->tab_done)) != hipSuccess) return dev_fail(c, e, "staging wait");
    if (c->tab_cap < etab.size()) {
        if (c->tab_host) (void)hipHostFree(c->tab_host);
        c->tab_host = nullptr;
        c->tab_cap = 0;
        if ((e = hipHostMalloc((void **)&c->tab_host, etab.size() * sizeof(int), hipHostMallocDefault)) != hipSuccess)
            return dev_fail(c, e, "pinned staging");
        c->tab_cap = etab.size();
    }
    std::memcpy(c->tab_host, etab.data(), etab.size() * sizeof(int));
    e = hipMemcpyAsync(etab_d, c->tab_host, etab.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return dev_fail(c, e, "box table upload");
    if ((e = hipEventRecord(c->tab_done, s)) != hipSuccess) return dev_fail(c, e, "event record");
    if (c->p.stride > 1) {
        float *El = (float *)(ws + w.lat);
        e = launch_energy_boxes(c, V, n0, n1, n2, vol_stride, etab_d, nent, maxd, El, w.lstride, nullptr, nullptr, s);
        if (e != hipSuccess) return dev_fail(c, e, "energy launch");
        e = launch_upsample_boxes(El, w.lstride, ltab_d, (int)nbox, w.maxg, (int)c->p.stride, Eb, w.estride, s);
        if (e != hipSuccess) return dev_fail(c, e, "upsample launch");
    } else {
        e = launch_energy_boxes(c, V, n0, n1, n2, vol_stride, etab_d, nent, maxd, Eb, w.estride, nullptr, nullptr, s);
        if (e != hipSuccess) return dev_fail(c, e, "energy launch");
    }
    e = launch_dcs_boxes(c, Eb, w.estride, ttab_d, (int)nbox, n, tile_dims, X, s);
    if (e != hipSuccess) return dev_fail(c, e, "dcs launch");
    e = launch_tile_merge_boxes(S_raw, m0, m1, m2, X, ttab_d, (int)nbox, tile_dims, stats, bound, err_out, s);
    if (e != hipSuccess) return dev_fail(c, e, "tile merge launch");
    return SAL_OK;
}

sal_status sal_absmax(sal_ctx *c, const float *V, int64_t n, float *vmax_out, int accumulate, void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if ((!V && n > 0) || !vmax_out) return fail(c, SAL_E_INVAL, "null pointer");
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(c, SAL_E_INVAL, "bad count");
    DevScope ds(c->device);
    sal_status st;
    if ((st = sticky(c)) != SAL_OK) return st;
    hipError_t e = launch_absmax_acc(V, n, vmax_out, accumulate, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(c, e, "absmax launch");
    return SAL_OK;
}

sal_status sal_normalize_combine(sal_ctx *c, const float *V, double vmax_in, const float *S_raw, int64_t n0,
                                 int64_t n1, int64_t n2, float *S, double *stats_out, void *workspace,
                                 size_t ws_bytes, void *stream)
{
    if (!V && !(vmax_in > 0.0)) return fail(c, SAL_E_INVAL, "vmax must be > 0 when V is NULL");
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!S_raw || !S || !workspace) return fail(c, SAL_E_INVAL, "null pointer");
    if (!aligned16(S_raw) || !aligned16(S) || !aligned16(workspace) || (V && !aligned16(V)) ||
        (stats_out && !aligned16(stats_out)))
        return fail(c, SAL_E_INVAL, "pointers must be 16-byte aligned");
    sal_status st = check_dims(c, n0, n1, n2);
    if (st != SAL_OK) return st;
    const WsLayout w = ws_layout(c, n0, n1, n2);
    if (ws_bytes < w.total) return fail(c, SAL_E_WORKSPACE, "workspace too small");
    DevScope ds(c->device);
    if ((st = sticky(c)) != SAL_OK) return st;
    const int64_t N = n0 * n1 * n2, nb = merge_red_blocks(N);
    char *ws = (char *)workspace;
    float *mm = (float *)(ws + w.e);
    float *vmax = (float *)(ws + w.e + align256((size_t)nb * 6 * sizeof(float)));
    double *stats = stats_out ? stats_out : (double *)(ws + w.stats);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_minmax_absmax(V, (float)vmax_in, S_raw, N, mm, vmax, s);
    if (e == hipSuccess) e = launch_stats(vmax, nb, mm, nb, stats, s);
    if (e == hipSuccess)
        e = launch_combine(S_raw, N, stats, c->p.a, c->p.b, c->p.c, c->p.normalize, c->p.zero_range, S, s);
    if (e != hipSuccess) return dev_fail(c, e, "normalize/combine launch");
    return SAL_OK;
}

sal_status sal_tile_merge(sal_ctx *c, float *S_raw, int64_t n0, int64_t n1, int64_t n2, const float *exact,
                          const int64_t crop_lo[3], const int64_t crop_dims[3], const int64_t tile_lo[3],
                          const int64_t tile_dims[3], const double *stats, double bound, float *err_out,
                          void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!S_raw || !exact || !crop_lo || !crop_dims || !tile_lo || !tile_dims || !stats || !err_out)
        return fail(c, SAL_E_INVAL, "null pointer");
    const int64_t n[3] = {n0, n1, n2};
    for (int a = 0; a < 3; ++a) {
        if (tile_dims[a] < 1 || tile_lo[a] < 0 || tile_lo[a] + tile_dims[a] > n[a])
            return fail(c, SAL_E_INVAL, "tile outside the volume");
        if (crop_dims[a] < 1 || crop_lo[a] < 0 || tile_lo[a] < crop_lo[a] ||
            tile_lo[a] + tile_dims[a] > crop_lo[a] + crop_dims[a])
            return fail(c, SAL_E_INVAL, "tile outside the crop");
    }
    if (!(bound >= 0.0)) return fail(c, SAL_E_INVAL, "bound must be >= 0");
    DevScope ds(c->device);
    sal_status st;
    if ((st = sticky(c)) != SAL_OK) return st;
    hipError_t e = launch_tile_merge(S_raw, n0, n1, n2, exact, crop_lo, crop_dims, tile_lo, tile_dims, stats,
                                     bound, err_out, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(c, e, "tile merge launch");
    return SAL_OK;
}

sal_status sal_tile_minmax(sal_ctx *c, const float *S_raw, int64_t n0, int64_t n1, int64_t n2, int32_t tile,
                           float *out, void *stream)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    if (!S_raw || !out) return fail(c, SAL_E_INVAL, "null pointer");
    if (n0 < 1 || n1 < 1 || n2 < 1 || n0 * n1 * n2 > ((int64_t)1 << 31) - 1)
        return fail(c, SAL_E_INVAL, "volume dimensions out of range");
    if (tile < 1 || tile > 1024) return fail(c, SAL_E_INVAL, "tile must be in [1, 1024]");
    const int64_t nt = ((n0 + tile - 1) / tile) * ((n1 + tile - 1) / tile) * ((n2 + tile - 1) / tile);
    if (nt > ((int64_t)1 << 31) - 1) return fail(c, SAL_E_INVAL, "too many tiles");
    DevScope ds(c->device);
    sal_status st;
    if ((st = sticky(c)) != SAL_OK) return st;
    if (hipError_t e = launch_tile_minmax(S_raw, n0, n1, n2, tile, out, (hipStream_t)stream); e != hipSuccess)
        return dev_fail(c, e, "tile min/max launch");
    return SAL_OK;
}

sal_status sal_profile_enable(sal_ctx *c, int on)
{
    if (!c) return fail(c, SAL_E_INVAL, "null context");
    DevScope ds(c->device);
    c->profiling = on != 0;
    if (!c->profiling) release_events(c);
    return SAL_OK;
}

sal_status sal_profile_read(sal_ctx *c, double ms[4], int64_t *calls, int reset)
{
    if (!c || !ms || !calls) return fail(c, SAL_E_INVAL, "null argument");
    DevScope ds(c->device);
    for (int k = 0; k < 4; ++k) ms[k] = 0.0;
    const size_t n = c->ev_used / 5;
    for (size_t i = 0; i < n; ++i) {
        hipEvent_t *ev = &c->ev_pool[5 * i];
        hipError_t e = hipEventSynchronize(ev[4]);
        if (e != hipSuccess) return dev_fail(c, e, "event synchronize");
        for (int k = 0; k < 4; ++k) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            if (e != hipSuccess) return dev_fail(c, e, "event elapsed time");
            ms[k] += (double)t;
        }
    }
    *calls = (int64_t)n;
    if (reset) c->ev_used = 0;
    return SAL_OK;
}

}  // extern "C"
