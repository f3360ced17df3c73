/*
 * A C program using the saliency library through its C ABI only (no Python, no PyTorch):
 * device buffers from the HIP runtime, the map of a small synthetic volume by
 * sal_saliency, compared with the FP64 oracle linked beside it; every other entry point
 * against a result it must reproduce; then the error paths.
 * Test infrastructure: built next to the library, run by tests/test_gpu_c_abi.py.
 * Exit status 0 when every check passes.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "sal.h"

/* the FP64 oracle (liboracle.so) */
void oracle_saliency(const float *V, long n0, long n1, long n2, long L, long r, double sigma,
                     const uint32_t rays[3], const double abc[3], int normalize, double zero_range,
                     double *S, double *E_out, double *S_raw_out, double *stats);

#define CHECK_HIP(x)                                                         \
    do {                                                                     \
        hipError_t e_ = (x);                                                 \
        if (e_ != hipSuccess) {                                              \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
            return 2;                                                        \
        }                                                                    \
    } while (0)

static int run_case(int L, int32_t precision, double tol, long n0, int32_t t_direct)
{
    const long n1 = 24, n2 = 29, N = n0 * n1 * n2;
    float *V = (float *)malloc(sizeof(float) * N);
    float *S = (float *)malloc(sizeof(float) * N);
    double *S_ref = (double *)malloc(sizeof(double) * N);
    /* layered signal with a tilted interface and a deterministic perturbation */
    for (long i = 0; i < N; ++i) {
        const long t = i / (n1 * n2), x = (i / n2) % n1, y = i % n2;
        V[i] = (float)(sin(0.7 * t + 0.05 * x) + (t > 9 + x / 6 ? 0.5 : -0.3) * cos(0.3 * y) +
                       0.01 * (double)((i * 2654435761u) % 97));
    }
    sal_params p;
    sal_default_params(&p, L);
    p.precision = precision;
    p.t_direct = t_direct;
    sal_ctx *ctx = NULL;
    if (sal_create(&p, 0, &ctx) != SAL_OK) {
        fprintf(stderr, "sal_create: %s\n", sal_last_error(NULL));
        return 1;
    }
    size_t ws_bytes = 0;
    if (sal_workspace_size(ctx, n0, n1, n2, &ws_bytes) != SAL_OK) return 1;
    float *dV, *dS;
    void *dws;
    CHECK_HIP(hipMalloc((void **)&dV, sizeof(float) * N));
    CHECK_HIP(hipMalloc((void **)&dS, sizeof(float) * N));
    CHECK_HIP(hipMalloc(&dws, ws_bytes));
    CHECK_HIP(hipMemcpy(dV, V, sizeof(float) * N, hipMemcpyHostToDevice));
    if (sal_saliency(ctx, dV, n0, n1, n2, dS, NULL, NULL, NULL, dws, ws_bytes, NULL) != SAL_OK) {
        fprintf(stderr, "sal_saliency: %s\n", sal_last_error(ctx));
        return 1;
    }
    CHECK_HIP(hipDeviceSynchronize());
    CHECK_HIP(hipMemcpy(S, dS, sizeof(float) * N, hipMemcpyDeviceToHost));

    const double abc[3] = {p.a, p.b, p.c};
    oracle_saliency(V, n0, n1, n2, L, p.d / 2, p.sigma, p.rays, abc, p.normalize, p.zero_range, S_ref,
                    NULL, NULL, NULL);
    double err = 0.0, ref = 0.0;
    for (long i = 0; i < N; ++i) {
        err = fmax(err, fabs((double)S[i] - S_ref[i]));
        ref = fmax(ref, fabs(S_ref[i]));
    }
    const double rel = err / ref;
    printf("L=%d precision=%d rows=%ld t_direct=%d max rel err %.3e (bound %.0e)\n", L, (int)precision, n0,
           (int)t_direct, rel, tol);

    /* a workspace one byte short is refused before anything is enqueued */
    const int ws_ok = sal_saliency(ctx, dV, n0, n1, n2, dS, NULL, NULL, NULL, dws, ws_bytes - 1, NULL) ==
                      SAL_E_WORKSPACE;
    (void)hipFree(dV);
    (void)hipFree(dS);
    (void)hipFree(dws);
    sal_destroy(ctx);
    free(V);
    free(S);
    free(S_ref);
    if (!ws_ok) {
        fprintf(stderr, "short workspace not refused\n");
        return 1;
    }
    return rel <= tol ? 0 : 1;
}

/* Batched tile check against the one-box path: the exact maps of two tiles from
 * sal_check_tiles equal sal_raw_box and the whole-volume raw maps bit for bit, and with the
 * predicted maps equal to the exact ones every error is 0 and nothing is replaced. */
static int check_tiles_case(void)
{
    const long n0 = 19, n1 = 24, n2 = 29, N = n0 * n1 * n2;
    const int64_t td[3] = {8, 8, 8};
    const int64_t lo[2][3] = {{0, 0, 0}, {11, 9, 21}};  /* a corner tile and one at the far faces */
    const long nt = td[0] * td[1] * td[2];
    float *V = (float *)malloc(sizeof(float) * N);
    for (long i = 0; i < N; ++i) V[i] = (float)(cos(0.37 * (double)(i % 97)) + 0.002 * (double)(i % 13));
    sal_params p;
    sal_default_params(&p, 8);
    sal_ctx *ctx = NULL;
    if (sal_create(&p, 0, &ctx) != SAL_OK) return 1;
    size_t ws_bytes = 0, wsc_bytes = 0, wsb_bytes = 0;
    if (sal_workspace_size(ctx, n0, n1, n2, &ws_bytes) != SAL_OK ||
        sal_check_tiles_workspace_size(ctx, n0, n1, n2, 2, td, &wsc_bytes) != SAL_OK ||
        sal_raw_box_workspace_size(ctx, td, &wsb_bytes) != SAL_OK)
        return 1;
    float *dV, *dS, *dSr, *dX, *dB, *derr;
    double *dstats;
    void *dws, *dwsc, *dwsb;
    CHECK_HIP(hipMalloc((void **)&dV, sizeof(float) * N));
    CHECK_HIP(hipMalloc((void **)&dS, sizeof(float) * N));
    CHECK_HIP(hipMalloc((void **)&dSr, sizeof(float) * 3 * N));
    CHECK_HIP(hipMalloc((void **)&dX, sizeof(float) * 2 * 3 * nt));
    CHECK_HIP(hipMalloc((void **)&dB, sizeof(float) * 3 * nt));
    CHECK_HIP(hipMalloc((void **)&derr, sizeof(float) * 2));
    CHECK_HIP(hipMalloc((void **)&dstats, sizeof(double) * 8));
    CHECK_HIP(hipMalloc(&dws, ws_bytes));
    CHECK_HIP(hipMalloc(&dwsc, wsc_bytes));
    CHECK_HIP(hipMalloc(&dwsb, wsb_bytes));
    CHECK_HIP(hipMemcpy(dV, V, sizeof(float) * N, hipMemcpyHostToDevice));
    int bad = sal_saliency(ctx, dV, n0, n1, n2, dS, NULL, dSr, dstats, dws, ws_bytes, NULL) != SAL_OK;
    bad |= sal_check_tiles(ctx, dV, n0, n1, n2, 0, &lo[0][0], dSr, n0, n1, n2, &lo[0][0], 2, td, dstats, 0.0,
                           derr, dX, dwsc, wsc_bytes, NULL) != SAL_OK;
    CHECK_HIP(hipDeviceSynchronize());
    float *X = (float *)malloc(sizeof(float) * 2 * 3 * nt), *B = (float *)malloc(sizeof(float) * 3 * nt);
    float *Sr = (float *)malloc(sizeof(float) * 3 * N), err[2];
    CHECK_HIP(hipMemcpy(X, dX, sizeof(float) * 2 * 3 * nt, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(Sr, dSr, sizeof(float) * 3 * N, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(err, derr, sizeof(err), hipMemcpyDeviceToHost));
    long mism = 0;
    for (int b = 0; b < 2; ++b) {
        bad |= sal_raw_box(ctx, dV, n0, n1, n2, lo[b], td, dB, dwsb, wsb_bytes, NULL) != SAL_OK;
        CHECK_HIP(hipMemcpy(B, dB, sizeof(float) * 3 * nt, hipMemcpyDeviceToHost));
        for (long m = 0; m < 3; ++m)
            for (long i = 0; i < nt; ++i) {
                const long t = lo[b][0] + i / 64, x = lo[b][1] + (i / 8) % 8, y = lo[b][2] + i % 8;
                const float xv = X[(b * 3 + m) * nt + i];
                mism += xv != B[m * nt + i];
                mism += xv != Sr[m * N + (t * n1 + x) * n2 + y];
            }
        bad |= err[b] != 0.0f;
    }
    printf("check_tiles: %ld mismatches, err %g %g\n", mism, err[0], err[1]);
    bad |= mism != 0;
    (void)hipFree(dV); (void)hipFree(dS); (void)hipFree(dSr); (void)hipFree(dX); (void)hipFree(dB);
    (void)hipFree(derr); (void)hipFree(dstats); (void)hipFree(dws); (void)hipFree(dwsc); (void)hipFree(dwsb);
    sal_destroy(ctx);
    free(V); free(X); free(B); free(Sr);
    return bad;
}

static double relmax_f(const float *a, const float *b, long n)
{
    double e = 0.0, r = 0.0;
    for (long i = 0; i < n; ++i) {
        e = fmax(e, fabs((double)a[i] - (double)b[i]));
        r = fmax(r, fabs((double)b[i]));
    }
    return r > 0.0 ? e / r : e;
}

/* Every other entry point of the ABI, each against a result it must reproduce: the un-fused
 * steps against the fused path, the normalisation of given raw maps against sal_saliency,
 * the reductions against host reductions, the profile counters, and the network calls. */
static int other_entry_points(void)
{
    const long n0 = 18, n1 = 20, n2 = 22, N = n0 * n1 * n2, L = 8;
    float *V = (float *)malloc(sizeof(float) * N);
    for (long i = 0; i < N; ++i) V[i] = (float)(sin(0.31 * (double)(i % 101)) + 0.01 * (double)(i % 7));
    sal_params p;
    sal_default_params(&p, (int32_t)L);
    sal_ctx *ctx = NULL;
    if (sal_create(&p, 0, &ctx) != SAL_OK) return 1;
    size_t ws_bytes = 0;
    if (sal_workspace_size(ctx, n0, n1, n2, &ws_bytes) != SAL_OK) return 1;
    const int64_t lo[3] = {3, 0, 17}, bn[3] = {2, 3, 4};
    const long nb = bn[0] * bn[1] * bn[2];
    float *dV, *dS, *dS2, *dE, *dSr, *dSr2, *dF, *dEb, *dmm, *dvmax, *derr;
    double *dst;
    void *dws;
    CHECK_HIP(hipMalloc((void **)&dV, sizeof(float) * N));
    CHECK_HIP(hipMalloc((void **)&dS, sizeof(float) * N));
    CHECK_HIP(hipMalloc((void **)&dS2, sizeof(float) * N));
    CHECK_HIP(hipMalloc((void **)&dE, sizeof(float) * 3 * N));
    CHECK_HIP(hipMalloc((void **)&dSr, sizeof(float) * 3 * N));
    CHECK_HIP(hipMalloc((void **)&dSr2, sizeof(float) * 3 * N));
    CHECK_HIP(hipMalloc((void **)&dF, sizeof(float) * 2 * nb * L * L * L));
    CHECK_HIP(hipMalloc((void **)&dEb, sizeof(float) * 3 * nb));
    CHECK_HIP(hipMalloc((void **)&dmm, sizeof(float) * 6 * 8));
    CHECK_HIP(hipMalloc((void **)&dvmax, sizeof(float)));
    CHECK_HIP(hipMalloc((void **)&derr, sizeof(float)));
    CHECK_HIP(hipMalloc((void **)&dst, sizeof(double) * 8));
    CHECK_HIP(hipMalloc(&dws, ws_bytes));
    CHECK_HIP(hipMemcpy(dV, V, sizeof(float) * N, hipMemcpyHostToDevice));
    int bad = 0;
    double ms[4];
    int64_t calls = -1;
    bad |= sal_profile_enable(ctx, 1) != SAL_OK;
    bad |= sal_saliency(ctx, dV, n0, n1, n2, dS, dE, dSr, dst, dws, ws_bytes, NULL) != SAL_OK;
    bad |= sal_profile_read(ctx, ms, &calls, 1) != SAL_OK;
    bad |= calls != 1 || !(ms[0] > 0.0 && ms[1] > 0.0 && ms[2] > 0.0 && ms[3] > 0.0);
    bad |= sal_profile_enable(ctx, 0) != SAL_OK;
    /* un-fused steps 1-3 on a box against the fused energies */
    bad |= sal_local_spectra(ctx, dV, n0, n1, n2, lo, bn, dF, NULL) != SAL_OK;
    bad |= sal_project(ctx, dF, nb, dEb, NULL) != SAL_OK;
    /* Eq. (5) on the fused energies against the fused raw maps */
    bad |= sal_directional_compare(ctx, dE, n0, n1, n2, dSr2, NULL) != SAL_OK;
    /* the normalisation of given raw maps against sal_saliency */
    bad |= sal_normalize_combine(ctx, dV, 0.0, dSr, n0, n1, n2, dS2, NULL, dws, ws_bytes, NULL) != SAL_OK;
    bad |= sal_absmax(ctx, dV, N, dvmax, 0, NULL) != SAL_OK;
    bad |= sal_tile_minmax(ctx, dSr, n0, n1, n2, 16, dmm, NULL) != SAL_OK;
    const int64_t crop_lo[3] = {0, 0, 0}, crop_d[3] = {n0, n1, n2}, tlo[3] = {2, 4, 6}, tdim[3] = {5, 6, 7};
    bad |= sal_tile_merge(ctx, dSr2, n0, n1, n2, dSr, crop_lo, crop_d, tlo, tdim, dst, 0.0, derr, NULL) != SAL_OK;
    CHECK_HIP(hipDeviceSynchronize());
    float *E = (float *)malloc(sizeof(float) * 3 * N), *Eb = (float *)malloc(sizeof(float) * 3 * nb);
    float *Sr = (float *)malloc(sizeof(float) * 3 * N), *Sr2 = (float *)malloc(sizeof(float) * 3 * N);
    float *S = (float *)malloc(sizeof(float) * N), *S2 = (float *)malloc(sizeof(float) * N);
    float mm[48], vmax, err;
    CHECK_HIP(hipMemcpy(E, dE, sizeof(float) * 3 * N, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(Eb, dEb, sizeof(float) * 3 * nb, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(Sr, dSr, sizeof(float) * 3 * N, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(Sr2, dSr2, sizeof(float) * 3 * N, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(S, dS, sizeof(float) * N, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(S2, dS2, sizeof(float) * N, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(mm, dmm, sizeof(mm), hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(&vmax, dvmax, sizeof(float), hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(&err, derr, sizeof(float), hipMemcpyDeviceToHost));
    /* box energies of the un-fused steps, gathered from the fused map */
    double e_box = 0.0, r_box = 0.0;
    for (long m = 0; m < 3; ++m)
        for (long i = 0; i < nb; ++i) {
            const long t = lo[0] + i / (bn[1] * bn[2]), x = lo[1] + (i / bn[2]) % bn[1], y = lo[2] + i % bn[2];
            const double ref = E[m * N + (t * n1 + x) * n2 + y];
            e_box = fmax(e_box, fabs(Eb[m * nb + i] - ref));
            r_box = fmax(r_box, fabs(ref));
        }
    const double rel_box = e_box / r_box, rel_dcs = relmax_f(Sr2, Sr, 3 * N);
    long s_mism = 0;
    for (long i = 0; i < N; ++i) s_mism += S2[i] != S[i];
    float hv = 0.f, hmm[6] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (long i = 0; i < N; ++i) hv = fmaxf(hv, fabsf(V[i]));
    for (long m = 0; m < 3; ++m)
        for (long t = 0; t < 16; ++t)
            for (long x = 0; x < 16; ++x)
                for (long y = 0; y < 16; ++y) {
                    const float v = Sr[m * N + (t * n1 + x) * n2 + y];
                    hmm[2 * m] = fminf(hmm[2 * m], v);
                    hmm[2 * m + 1] = fmaxf(hmm[2 * m + 1], v);
                }
    int mm_bad = 0;
    for (int k = 0; k < 6; ++k) mm_bad |= mm[k] != hmm[k];
    printf("entry points: project %.2e, compare %.2e, combine %ld mismatches, absmax %d, minmax %d, merge err %g\n",
           rel_box, rel_dcs, s_mism, vmax == hv, !mm_bad, err);
    bad |= !(rel_box <= 1e-5) || !(rel_dcs <= 1e-5) || s_mism != 0 || vmax != hv || mm_bad;
    bad |= !(err <= 1e-5);
    (void)hipFree(dV); (void)hipFree(dS); (void)hipFree(dS2); (void)hipFree(dE); (void)hipFree(dSr);
    (void)hipFree(dSr2); (void)hipFree(dF); (void)hipFree(dEb); (void)hipFree(dmm); (void)hipFree(dvmax);
    (void)hipFree(derr); (void)hipFree(dst); (void)hipFree(dws);
    sal_destroy(ctx);
    free(V); free(E); free(Eb); free(Sr); free(Sr2); free(S); free(S2);

    /* the network: inference equals the forward pass (channels moved to planes), one
     * training step and one Adam step, parameters and gradients through host memory */
    const int64_t np = sal_net_num_params();
    sal_net *net = NULL;
    if (np <= 0 || sal_net_create(0, 3, &net) != SAL_OK) {
        fprintf(stderr, "sal_net_create: %s\n", sal_net_last_error(NULL));
        return 1;
    }
    const long S0 = 12, NV = S0 * S0 * S0;
    size_t wt = 0, wi = 0;
    bad |= sal_net_set_precision(net, SAL_BF16) != SAL_OK;
    bad |= sal_net_set_precision(net, SAL_FP16) != SAL_E_INVAL;
    bad |= sal_net_workspace_size(net, 1, S0, S0, S0, 1, &wt) != SAL_OK;
    bad |= sal_net_workspace_size(net, 1, S0, S0, S0, 0, &wi) != SAL_OK;
    float *X = (float *)malloc(sizeof(float) * NV), *Y = (float *)malloc(sizeof(float) * 3 * NV);
    float *Z = (float *)malloc(sizeof(float) * 3 * NV), *T = (float *)malloc(sizeof(float) * 3 * NV);
    float *par = (float *)malloc(sizeof(float) * np), *gr = (float *)malloc(sizeof(float) * np);
    for (long i = 0; i < NV; ++i) X[i] = (float)sin(0.1 * (double)i);
    for (long i = 0; i < 3 * NV; ++i) T[i] = 0.5f * (float)cos(0.05 * (double)i);
    float *dX, *dY, *dZ, *dT, *dloss;
    void *dwt, *dwi;
    CHECK_HIP(hipMalloc((void **)&dX, sizeof(float) * NV));
    CHECK_HIP(hipMalloc((void **)&dY, sizeof(float) * 3 * NV));
    CHECK_HIP(hipMalloc((void **)&dZ, sizeof(float) * 3 * NV));
    CHECK_HIP(hipMalloc((void **)&dT, sizeof(float) * 3 * NV));
    CHECK_HIP(hipMalloc((void **)&dloss, sizeof(float)));
    CHECK_HIP(hipMalloc(&dwt, wt));
    CHECK_HIP(hipMalloc(&dwi, wi));
    CHECK_HIP(hipMemcpy(dX, X, sizeof(float) * NV, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dT, T, sizeof(float) * 3 * NV, hipMemcpyHostToDevice));
    const float one[3] = {1.f, 1.f, 1.f};
    bad |= sal_net_set_output_scale(net, one) != SAL_OK;
    bad |= sal_net_forward(net, dX, 1, S0, S0, S0, dY, dwt, wt, NULL) != SAL_OK;
    bad |= sal_net_infer(net, dX, S0, S0, S0, dZ, dwi, wi, NULL) != SAL_OK;
    bad |= sal_net_backward(net, dX, dT, 1, S0, S0, S0, dwt, wt, NULL) != SAL_OK;
    bad |= sal_net_grads(net, gr, np, 0) != SAL_OK;
    bad |= sal_net_params(net, par, np, 0) != SAL_OK;
    bad |= sal_net_adam(net, 1e-3f, NULL) != SAL_OK;
    bad |= sal_net_train_step(net, dX, dT, 1, S0, 5, 1e-3f, dloss, dwt, wt, NULL) != SAL_OK;
    CHECK_HIP(hipDeviceSynchronize());
    float *par2 = (float *)malloc(sizeof(float) * np), loss = 0.f;
    bad |= sal_net_params(net, par2, np, 0) != SAL_OK;
    bad |= sal_net_params(net, par, np, 1) != SAL_OK; /* write back the initial parameters */
    CHECK_HIP(hipMemcpy(Y, dY, sizeof(float) * 3 * NV, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(Z, dZ, sizeof(float) * 3 * NV, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(&loss, dloss, sizeof(float), hipMemcpyDeviceToHost));
    long y_mism = 0, moved = 0, gnz = 0;
    for (long v = 0; v < NV; ++v)
        for (long c = 0; c < 3; ++c) y_mism += Y[v * 3 + c] != Z[c * NV + v];
    for (long i = 0; i < np; ++i) {
        moved += par2[i] != par[i];
        gnz += gr[i] != 0.f;
    }
    printf("net: infer/forward %ld mismatches, %ld of %ld gradients nonzero, %ld parameters moved, loss %g\n",
           y_mism, gnz, (long)np, moved, loss);
    bad |= y_mism != 0 || gnz == 0 || moved == 0 || !(loss > 0.f && loss < 1e30f);
    (void)hipFree(dX); (void)hipFree(dY); (void)hipFree(dZ); (void)hipFree(dT); (void)hipFree(dloss);
    (void)hipFree(dwt); (void)hipFree(dwi);
    sal_net_destroy(net);
    free(X); free(Y); free(Z); free(T); free(par); free(par2); free(gr);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run_case(8, SAL_FP32, 1e-5, 19, 0);
    bad |= run_case(5, SAL_FP32, 1e-5, 19, 0);
    bad |= run_case(16, SAL_BF16_SPLIT, 1e-3, 19, 0);
    bad |= run_case(16, SAL_FP32, 1e-5, 40, 0);  /* windows sliding along t */
    bad |= run_case(16, SAL_FP32, 1e-5, 40, 1);  /* every window contracted along t */
    bad |= check_tiles_case();
    bad |= other_entry_points();

    /* parameters the build does not implement, and invalid ones */
    sal_params p;
    sal_ctx *ctx = NULL;
    sal_default_params(&p, 21);
    if (sal_create(&p, 0, &ctx) != SAL_E_UNSUPPORTED || ctx != NULL || strlen(sal_last_error(NULL)) == 0) {
        fprintf(stderr, "L = 21 not refused as unsupported\n");
        bad = 1;
    }
    sal_default_params(&p, 8);
    p.rays[1] = 0;
    if (sal_create(&p, 0, &ctx) != SAL_E_INVAL) {
        fprintf(stderr, "empty ray mask not refused\n");
        bad = 1;
    }
    printf(bad ? "c abi client: FAILED\n" : "c abi client: ok\n");
    return bad;
}
