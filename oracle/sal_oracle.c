/*
 * sal_oracle.c -- plain, slow FP64 CPU oracle for the seismic saliency method of
 * Shafiq, Long, Alshawi, AlRegib, "Saliency detection for seismic applications using
 * multi-dimensional spectral projections and directional comparisons", ICIP 2017.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library.  It shares no code, header, table or constant
 * with the GPU path; neither includes or links the other.
 *
 * Everything is computed in double precision from FP32 inputs.  Each function names the
 * passage of the paper it follows.  Readings of points the paper leaves open are marked
 * "reading:" and listed in the design notes of the repository.
 *
 * Conventions (all arrays C-order, axis 0 = t slowest, axis 2 = y fastest):
 *   V      : float  [n0][n1][n2]               input volume (Sec. 2, "V of size T x X x Y")
 *   F      : double [L][L][L][2]               one local spectrum, (re, im) interleaved
 *   E      : double [3][n0][n1][n2]            spectral energies E_t, E_x, E_y
 *   S_raw  : double [3][n0][n1][n2]            DCS maps S_t, S_x, S_y before normalisation
 *   S      : double [n0][n1][n2]               combined saliency map
 * Parity status of every function: pinned by the CPU tests (brute-force sums, library
 * FFT, Parseval, closed forms and invariants) except where a header says otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Reflect an index into [0, n) without repeating the edge sample (reading: the paper is
 * silent on boundaries; the reflect rule "...,2,1,0,1,2,..." is the declared one).
 * Valid for -(n-1) <= u <= 2(n-1). */
static long refl_index(long u, long n)
{
    if (u < 0) return -u;
    if (u >= n) return 2 * (n - 1) - u;
    return u;
}

/* Signed frequency of DFT index u in [0, L): u for u <= L/2, u - L above (Sec. 2: the
 * spectral cube is centred on DC, so the projection formulas use signed coordinates). */
static long signed_freq(long u, long L)
{
    return (u <= L / 2) ? u : u - L;
}

/*
 * Local spectrum of the window of voxel (t, x, y) -- Sec. 2, first step, and the DFT
 * definition that follows Eq. (2):
 *     F[mu,nu,om] = L^-3 sum_{p,q,r} f[p,q,r] exp(-2 pi i (p mu + q nu + r om) / L).
 * reading: one window per voxel (stride 1, which is "more than 50% overlap"); the window
 * starts at v - floor(L/2) along every axis, samples outside the volume are reflected.
 * The triple sum is evaluated as three one-dimensional sums (it factorises exactly).
 */
void oracle_window_spectrum(const float *V, long n0, long n1, long n2,
                            long t, long x, long y, long L, double *F)
{
    const long h = L / 2;
    const long L3 = L * L * L;
    double *f = (double *)malloc(sizeof(double) * 2 * L3);
    double *g = (double *)malloc(sizeof(double) * 2 * L3);
    /* exp(-2 pi i k / L) for k in [0, L); every exponent p*mu is reduced mod L first */
    double *cw = (double *)malloc(sizeof(double) * L);
    double *sw = (double *)malloc(sizeof(double) * L);
    for (long k = 0; k < L; ++k) {
        cw[k] = cos(2.0 * M_PI * (double)k / (double)L);
        sw[k] = -sin(2.0 * M_PI * (double)k / (double)L);
    }
    /* gather the window f[p][q][r] (real) */
    for (long p = 0; p < L; ++p)
        for (long q = 0; q < L; ++q)
            for (long r = 0; r < L; ++r) {
                long a = refl_index(t - h + p, n0);
                long b = refl_index(x - h + q, n1);
                long c = refl_index(y - h + r, n2);
                long o = (p * L + q) * L + r;
                f[2 * o] = (double)V[(a * n1 + b) * n2 + c];
                f[2 * o + 1] = 0.0;
            }
    /* sum over r -> om : g[p][q][om] */
    for (long p = 0; p < L; ++p)
        for (long q = 0; q < L; ++q)
            for (long om = 0; om < L; ++om) {
                double re = 0.0, im = 0.0;
                for (long r = 0; r < L; ++r) {
                    double c = cw[r * om % L], s = sw[r * om % L];
                    long o = (p * L + q) * L + r;
                    re += f[2 * o] * c - f[2 * o + 1] * s;
                    im += f[2 * o] * s + f[2 * o + 1] * c;
                }
                long o = (p * L + q) * L + om;
                g[2 * o] = re;
                g[2 * o + 1] = im;
            }
    /* sum over q -> nu : f[p][nu][om] */
    for (long p = 0; p < L; ++p)
        for (long nu = 0; nu < L; ++nu)
            for (long om = 0; om < L; ++om) {
                double re = 0.0, im = 0.0;
                for (long q = 0; q < L; ++q) {
                    double c = cw[q * nu % L], s = sw[q * nu % L];
                    long o = (p * L + q) * L + om;
                    re += g[2 * o] * c - g[2 * o + 1] * s;
                    im += g[2 * o] * s + g[2 * o + 1] * c;
                }
                long o = (p * L + nu) * L + om;
                f[2 * o] = re;
                f[2 * o + 1] = im;
            }
    /* sum over p -> mu, times 1/L^3 : F[mu][nu][om] */
    for (long mu = 0; mu < L; ++mu)
        for (long nu = 0; nu < L; ++nu)
            for (long om = 0; om < L; ++om) {
                double re = 0.0, im = 0.0;
                for (long p = 0; p < L; ++p) {
                    double c = cw[p * mu % L], s = sw[p * mu % L];
                    long o = (p * L + nu) * L + om;
                    re += f[2 * o] * c - f[2 * o + 1] * s;
                    im += f[2 * o] * s + f[2 * o + 1] * c;
                }
                long o = (mu * L + nu) * L + om;
                F[2 * o] = re / (double)L3;
                F[2 * o + 1] = im / (double)L3;
            }
    free(f);
    free(g);
    free(cw);
    free(sw);
}

/*
 * Plane projections and spectral energies of one local spectrum -- Eqs. (1)-(4), the DC
 * rule that follows Fig. 2, and the third step of Sec. 2:
 *     F_t = F * sqrt(j^2+k^2)/sqrt(i^2+j^2+k^2)   (projection along f_t)
 *     F_x = F * sqrt(i^2+k^2)/sqrt(i^2+j^2+k^2)
 *     F_y = F * sqrt(i^2+j^2)/sqrt(i^2+j^2+k^2)
 *     E_m = mean of |F_m| over the cube, DC bin excluded.
 * reading: (i, j, k) are the signed frequencies of (mu, nu, om) on axes (t, x, y); the
 * mean runs over the L^3 - 1 bins that remain once DC is dropped.
 */
void oracle_project(const double *F, long L, double E[3])
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (long mu = 0; mu < L; ++mu)
        for (long nu = 0; nu < L; ++nu)
            for (long om = 0; om < L; ++om) {
                if (mu == 0 && nu == 0 && om == 0) continue; /* DC excluded */
                double i = (double)signed_freq(mu, L);
                double j = (double)signed_freq(nu, L);
                double k = (double)signed_freq(om, L);
                double rho = sqrt(i * i + j * j + k * k);
                long o = (mu * L + nu) * L + om;
                double mag = sqrt(F[2 * o] * F[2 * o] + F[2 * o + 1] * F[2 * o + 1]);
                acc[0] += mag * sqrt(j * j + k * k) / rho; /* |F_t| */
                acc[1] += mag * sqrt(i * i + k * k) / rho; /* |F_x| */
                acc[2] += mag * sqrt(i * i + j * j) / rho; /* |F_y| */
            }
    double nbins = (double)(L * L * L - 1);
    E[0] = acc[0] / nbins;
    E[1] = acc[1] / nbins;
    E[2] = acc[2] / nbins;
}

/* Local spectra of every voxel of the box [lo, lo+bn) -- Sec. 2, first step.
 * out: double [bn0][bn1][bn2][L][L][L][2]. */
void oracle_local_spectra(const float *V, long n0, long n1, long n2, long L,
                          const long lo[3], const long bn[3], double *out)
{
    const long per = 2 * L * L * L;
    const long nb = bn[0] * bn[1] * bn[2];
#pragma omp parallel for schedule(dynamic, 16)
    for (long v = 0; v < nb; ++v) {
        long a = v / (bn[1] * bn[2]);
        long b = (v / bn[2]) % bn[1];
        long c = v % bn[2];
        oracle_window_spectrum(V, n0, n1, n2, lo[0] + a, lo[1] + b, lo[2] + c, L, out + v * per);
    }
}

/* Spectral energies of every voxel of the box [lo, lo+bn) -- Sec. 2, steps one to three.
 * E: double [3][bn0][bn1][bn2]. */
void oracle_energy_box(const float *V, long n0, long n1, long n2, long L,
                       const long lo[3], const long bn[3], double *E)
{
    const long nb = bn[0] * bn[1] * bn[2];
#pragma omp parallel
    {
        double *F = (double *)malloc(sizeof(double) * 2 * L * L * L);
#pragma omp for schedule(dynamic, 16)
        for (long v = 0; v < nb; ++v) {
            long a = v / (bn[1] * bn[2]);
            long b = (v / bn[2]) % bn[1];
            long c = v % bn[2];
            double e[3];
            oracle_window_spectrum(V, n0, n1, n2, lo[0] + a, lo[1] + b, lo[2] + c, L, F);
            oracle_project(F, L, e);
            E[v] = e[0];
            E[nb + v] = e[1];
            E[2 * nb + v] = e[2];
        }
        free(F);
    }
}

/* Spectral energies of the whole volume. */
void oracle_energy(const float *V, long n0, long n1, long n2, long L, double *E)
{
    long lo[3] = {0, 0, 0};
    long bn[3] = {n0, n1, n2};
    oracle_energy_box(V, n0, n1, n2, L, lo, bn, E);
}

/* Step vector (t, x, y) of ray bit b of the comparison masks. */
static void ray_step(int b, long e[3])
{
    e[0] = e[1] = e[2] = 0;
    if (b < 6) {
        e[b / 2] = (b % 2 == 0) ? 1 : -1;
    } else if (b < 18) {
        /* planes (t,x), (t,y), (x,y); signs (+,+), (-,-), (+,-), (-,+) */
        static const int ax[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        static const int sg[4][2] = {{1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
        int pl = (b - 6) / 4, k = (b - 6) % 4;
        e[ax[pl][0]] = sg[k][0];
        e[ax[pl][1]] = sg[k][1];
    } else {
        int k = b - 18;
        e[0] = (k & 1) ? -1 : 1;
        e[1] = (k & 2) ? -1 : 1;
        e[2] = (k & 4) ? -1 : 1;
    }
}

/*
 * Directional center-surround comparison -- Eq. (5), the paragraph after it and Fig. 3
 * (comparisons along t, along x and along the t-x diagonal; the orientation is a tunable
 * choice of the method):
 *     S_m[v] = (1/Q) sum_{neighbours u} | E_m[v] - w(u) E_m[u] |.
 * reading: the d x 1 window centred on v is taken as rays of r = floor(d/2) steps from v;
 * a ray has a step vector e of the 26-neighbourhood and its s-th sample is v + s e;
 * w = exp(-|s e|^2 / (2 sigma^2)) (Gaussian in the Euclidean distance from the centre);
 * Q = (number of enabled rays) * r; each coordinate of a neighbour beyond the volume is
 * reflected.  Bits of rays[m] (see ray_step): 0-5 the axis rays +t, -t, +x, -x, +y, -y;
 * 6-17 the face diagonals of the t-x, t-y and x-y planes; 18-25 the body diagonals.
 * E is given on the box [elo, elo+ebn) of a volume of dims n; S_raw is produced for the box
 * [lo, lo+bn), which must lie inside the E box together with every neighbour it reads.
 */
int oracle_dcs_box(const double *E, const long elo[3], const long ebn[3],
                   long n0, long n1, long n2, long r, double sigma,
                   const uint32_t rays[3], const long lo[3], const long bn[3], double *S)
{
    const long n[3] = {n0, n1, n2};
    const long ne = ebn[0] * ebn[1] * ebn[2];
    const long nb = bn[0] * bn[1] * bn[2];
    int bad = 0;
    for (int m = 0; m < 3; ++m) {
        long nrays = 0;
        for (int b = 0; b < 26; ++b) nrays += (rays[m] >> b) & 1u;
        double Q = (double)(nrays * r);
        for (long v = 0; v < nb; ++v) {
            long pos[3] = {lo[0] + v / (bn[1] * bn[2]), lo[1] + (v / bn[2]) % bn[1], lo[2] + v % bn[2]};
            long ec = ((pos[0] - elo[0]) * ebn[1] + (pos[1] - elo[1])) * ebn[2] + (pos[2] - elo[2]);
            double centre = E[m * ne + ec];
            double sum = 0.0;
            for (int b = 0; b < 26; ++b) {
                if (!((rays[m] >> b) & 1u)) continue;
                long e[3];
                ray_step(b, e);
                long len2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                for (long s = 1; s <= r; ++s) {
                    long rel[3];
                    for (int a = 0; a < 3; ++a) rel[a] = refl_index(pos[a] + e[a] * s, n[a]) - elo[a];
                    if (rel[0] < 0 || rel[0] >= ebn[0] || rel[1] < 0 || rel[1] >= ebn[1] ||
                        rel[2] < 0 || rel[2] >= ebn[2]) {
                        bad = 1;
                        continue;
                    }
                    double w = exp(-(double)(s * s * len2) / (2.0 * sigma * sigma));
                    double nbv = E[m * ne + (rel[0] * ebn[1] + rel[1]) * ebn[2] + rel[2]];
                    sum += fabs(centre - w * nbv);
                }
            }
            S[m * nb + v] = (Q > 0.0) ? sum / Q : 0.0;
        }
    }
    return bad;
}

/* Eq. (5) on a whole volume. */
int oracle_dcs(const double *E, long n0, long n1, long n2, long r, double sigma,
               const uint32_t rays[3], double *S)
{
    long lo[3] = {0, 0, 0};
    long bn[3] = {n0, n1, n2};
    return oracle_dcs_box(E, lo, bn, n0, n1, n2, r, sigma, rays, lo, bn, S);
}

/* Sigma = infinity variant used by exactness checks: every neighbour has weight one. */
int oracle_dcs_unweighted(const double *E, long n0, long n1, long n2, long r,
                          const uint32_t rays[3], double *S)
{
    return oracle_dcs(E, n0, n1, n2, r, INFINITY, rays, S);
}

/*
 * Volume-wide normalisation and the combination of Eq. (6):  S = a S_t + b S_x + c S_y.
 * reading: each component is mapped to [0,1] by its own volume-wide min and max before it
 * is weighted (so that equal weights give each direction an equal share); a component whose
 * range is at most zero_range * vmax is treated as having no contrast and contributes 0.
 * With normalize = 0 the raw components are combined.  stats[6] receives
 * {lo_t, hi_t, lo_x, hi_x, lo_y, hi_y}.
 */
void oracle_combine(const double *S_raw, long nvox, const double abc[3], int normalize,
                    double zero_range, double vmax, double *S, double *stats)
{
    double lo[3], hi[3], scale[3];
    for (int m = 0; m < 3; ++m) {
        lo[m] = INFINITY;
        hi[m] = -INFINITY;
        for (long v = 0; v < nvox; ++v) {
            double s = S_raw[m * nvox + v];
            if (s < lo[m]) lo[m] = s;
            if (s > hi[m]) hi[m] = s;
        }
        if (stats) {
            stats[2 * m] = lo[m];
            stats[2 * m + 1] = hi[m];
        }
        scale[m] = (hi[m] - lo[m] > zero_range * vmax) ? 1.0 / (hi[m] - lo[m]) : 0.0;
    }
    for (long v = 0; v < nvox; ++v) {
        double s = 0.0;
        for (int m = 0; m < 3; ++m) {
            double x = S_raw[m * nvox + v];
            s += abc[m] * (normalize ? (x - lo[m]) * scale[m] : x);
        }
        S[v] = s;
    }
}

/* Combination of given raw maps with caller-given stats (used to check a sub-block of a
 * large volume against the volume-wide statistics).  Same formula as oracle_combine. */
void oracle_combine_with_stats(const double *S_raw, long nvox, const double abc[3],
                               int normalize, double zero_range, double vmax,
                               const double *stats, double *S)
{
    double scale[3];
    for (int m = 0; m < 3; ++m) {
        double range = stats[2 * m + 1] - stats[2 * m];
        scale[m] = (range > zero_range * vmax) ? 1.0 / range : 0.0;
    }
    for (long v = 0; v < nvox; ++v) {
        double s = 0.0;
        for (int m = 0; m < 3; ++m) {
            double x = S_raw[m * nvox + v];
            s += abc[m] * (normalize ? (x - stats[2 * m]) * scale[m] : x);
        }
        S[v] = s;
    }
}

/* max |V| over the volume (scale of the zero-contrast rule in oracle_combine). */
double oracle_absmax(const float *V, long n)
{
    double m = 0.0;
    for (long i = 0; i < n; ++i) {
        double a = fabs((double)V[i]);
        if (a > m) m = a;
    }
    return m;
}

/*
 * The whole method on a volume -- Sec. 2, steps one to five.  E, S_raw may be NULL.
 * rays[3] as in oracle_dcs_box; abc = (a, b, c) of Eq. (6).
 */
void oracle_saliency(const float *V, long n0, long n1, long n2, long L, long r, double sigma,
                     const uint32_t rays[3], const double abc[3], int normalize,
                     double zero_range, double *S, double *E_out, double *S_raw_out,
                     double *stats)
{
    const long nvox = n0 * n1 * n2;
    double *E = E_out ? E_out : (double *)malloc(sizeof(double) * 3 * nvox);
    double *Sr = S_raw_out ? S_raw_out : (double *)malloc(sizeof(double) * 3 * nvox);
    oracle_energy(V, n0, n1, n2, L, E);
    oracle_dcs(E, n0, n1, n2, r, sigma, rays, Sr);
    oracle_combine(Sr, nvox, abc, normalize, zero_range, oracle_absmax(V, nvox), S, stats);
    if (!E_out) free(E);
    if (!S_raw_out) free(Sr);
}

/*
 * Strided windows -- Sec. 2, first step: the sliding cube only has to overlap its
 * neighbours by more than half, so windows may sit on a lattice of stride s < L/2 while
 * the map keeps the size of V.
 * reading: the lattice holds the positions k s, k = 0 .. ceil(n/s) - 1, along every axis;
 * the energies of Sec. 2 (third step) are computed there, and every voxel takes the
 * trilinear interpolation of the lattice points around it (beyond the last lattice point
 * of an axis the last value is held).  Eq. (5) and Eq. (6) then run on the full grid.
 * E_lat: double [3][K0][K1][K2] with K_a = ceil(n_a / s).
 */
void oracle_energy_lattice(const float *V, long n0, long n1, long n2, long L, long s, double *E_lat)
{
    const long K0 = (n0 + s - 1) / s, K1 = (n1 + s - 1) / s, K2 = (n2 + s - 1) / s;
    const long nk = K0 * K1 * K2;
#pragma omp parallel
    {
        double *F = (double *)malloc(sizeof(double) * 2 * L * L * L);
#pragma omp for schedule(dynamic, 16)
        for (long v = 0; v < nk; ++v) {
            long a = v / (K1 * K2), b = (v / K2) % K1, c = v % K2;
            double e[3];
            oracle_window_spectrum(V, n0, n1, n2, a * s, b * s, c * s, L, F);
            oracle_project(F, L, e);
            for (int m = 0; m < 3; ++m) E_lat[m * nk + v] = e[m];
        }
        free(F);
    }
}

/* Trilinear interpolation of lattice values (stride s) onto the full grid n0 x n1 x n2. */
void oracle_upsample(const double *E_lat, long s, long n0, long n1, long n2, double *E)
{
    const long K[3] = {(n0 + s - 1) / s, (n1 + s - 1) / s, (n2 + s - 1) / s};
    const long nk = K[0] * K[1] * K[2], nv = n0 * n1 * n2;
    for (long v = 0; v < nv; ++v) {
        const long pos[3] = {v / (n1 * n2), (v / n2) % n1, v % n2};
        long k0[3], k1[3];
        double f[3];
        for (int a = 0; a < 3; ++a) {
            k0[a] = pos[a] / s;
            k1[a] = k0[a] + 1 < K[a] ? k0[a] + 1 : k0[a];
            f[a] = k1[a] == k0[a] ? 0.0 : (double)(pos[a] - k0[a] * s) / (double)s;
        }
        for (int m = 0; m < 3; ++m) {
            double acc = 0.0;
            for (int corner = 0; corner < 8; ++corner) {
                long idx[3];
                double w = 1.0;
                for (int a = 0; a < 3; ++a) {
                    int hi = (corner >> (2 - a)) & 1;
                    idx[a] = hi ? k1[a] : k0[a];
                    w *= hi ? f[a] : 1.0 - f[a];
                }
                acc += w * E_lat[m * nk + (idx[0] * K[1] + idx[1]) * K[2] + idx[2]];
            }
            E[m * nv + v] = acc;
        }
    }
}

/* The whole method with windows on the stride-s lattice (s = 1 is oracle_saliency). */
void oracle_saliency_strided(const float *V, long n0, long n1, long n2, long L, long s, long r,
                             double sigma, const uint32_t rays[3], const double abc[3], int normalize,
                             double zero_range, double *S, double *E_out, double *S_raw_out, double *stats)
{
    const long nvox = n0 * n1 * n2;
    const long nk = ((n0 + s - 1) / s) * ((n1 + s - 1) / s) * ((n2 + s - 1) / s);
    double *E_lat = (double *)malloc(sizeof(double) * 3 * nk);
    double *E = E_out ? E_out : (double *)malloc(sizeof(double) * 3 * nvox);
    double *Sr = S_raw_out ? S_raw_out : (double *)malloc(sizeof(double) * 3 * nvox);
    oracle_energy_lattice(V, n0, n1, n2, L, s, E_lat);
    oracle_upsample(E_lat, s, n0, n1, n2, E);
    oracle_dcs(E, n0, n1, n2, r, sigma, rays, Sr);
    oracle_combine(Sr, nvox, abc, normalize, zero_range, oracle_absmax(V, nvox), S, stats);
    free(E_lat);
    if (!E_out) free(E);
    if (!S_raw_out) free(Sr);
}

/*
 * Raw maps (E and S_raw) of the box [lo, lo+bn) of a large volume, without computing the
 * whole volume: energies are evaluated on the box grown by r on every side (clipped to
 * the volume), which holds every neighbour Eq. (5) reads, reflected ones included.
 * E_box: double [3][bn...], S_box: double [3][bn...].  Returns nonzero on a range error.
 */
int oracle_raw_box(const float *V, long n0, long n1, long n2, long L, long r, double sigma,
                   const uint32_t rays[3], const long lo[3], const long bn[3],
                   double *E_box, double *S_box)
{
    const long n[3] = {n0, n1, n2};
    long elo[3], ebn[3];
    for (int a = 0; a < 3; ++a) {
        long b = lo[a] - r < 0 ? 0 : lo[a] - r;
        long e = lo[a] + bn[a] + r > n[a] ? n[a] : lo[a] + bn[a] + r;
        elo[a] = b;
        ebn[a] = e - b;
    }
    const long ne = ebn[0] * ebn[1] * ebn[2];
    const long nb = bn[0] * bn[1] * bn[2];
    double *E = (double *)malloc(sizeof(double) * 3 * ne);
    oracle_energy_box(V, n0, n1, n2, L, elo, ebn, E);
    int bad = oracle_dcs_box(E, elo, ebn, n0, n1, n2, r, sigma, rays, lo, bn, S_box);
    for (int m = 0; m < 3; ++m)
        for (long v = 0; v < nb; ++v) {
            long a = lo[0] + v / (bn[1] * bn[2]) - elo[0];
            long b = lo[1] + (v / bn[2]) % bn[1] - elo[1];
            long c = lo[2] + v % bn[2] - elo[2];
            E_box[m * nb + v] = E[m * ne + (a * ebn[1] + b) * ebn[2] + c];
        }
    free(E);
    return bad;
}
