/*
 * A C program using the saliency library through its C ABI only (no Python, no PyTorch):
 * device buffers from the HIP runtime, the map of a small synthetic volume by
 * sal_saliency, compared with the FP64 oracle linked beside it; then the error paths.
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

static int run_case(int L, int32_t precision, double tol)
{
    const long n0 = 19, n1 = 24, n2 = 29, N = n0 * n1 * n2;
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
    printf("L=%d precision=%d max rel err %.3e (bound %.0e)\n", L, (int)precision, rel, tol);

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

int main(void)
{
    int bad = 0;
    bad |= run_case(8, SAL_FP32, 1e-5);
    bad |= run_case(5, SAL_FP32, 1e-5);
    bad |= run_case(16, SAL_BF16_SPLIT, 1e-3);
    bad |= check_tiles_case();

    /* parameters the build does not implement, and invalid ones */
    sal_params p;
    sal_ctx *ctx = NULL;
    sal_default_params(&p, 9);
    if (sal_create(&p, 0, &ctx) != SAL_E_UNSUPPORTED || ctx != NULL || strlen(sal_last_error(NULL)) == 0) {
        fprintf(stderr, "L = 9 not refused as unsupported\n");
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
