/*
 * net_oracle.c -- plain FP64 CPU oracle of the learned surrogate: a stack of 3x3x3
 * convolutions with GELU, its forward pass and its exact gradient.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  Shares nothing with the
 * GPU path.  The paper has no learned part; the network shape is the one the surrogate is
 * specified with (five 3x3x3 convolutions, GELU between them).
 *
 * Conventions: activations are channel-last, x[b][t][u][w][c] over a crop of S^3 voxels;
 * weights W[co][k][ci] with tap k = (dt*3 + du)*3 + dw, dt, du, dw in {0,1,2}; the tap reads
 * the input at (t+dt-1, u+du-1, w+dw-1), reflected inside the crop (-1 -> 1, S -> S-2).
 * GELU(z) = z/2 (1 + erf(z / sqrt 2)).
 * Parity status: pinned by the CPU tests (shift kernels, linearity, GELU identities and
 * central finite differences of the gradient).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static long nrefl(long u, long n)
{
    if (u < 0) return -u;
    if (u >= n) return 2 * (n - 1) - u;
    return u;
}

double oracle_gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }

double oracle_gelu_grad(double z)
{
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
}

/* y = conv(x) + b over nb crops of S^3 (reflect padding inside each crop). */
void oracle_conv3d(const double *x, long nb, long S, long ci_n, const double *W,
                   const double *bias, long co_n, double *y)
{
    const long S3 = S * S * S;
    for (long b = 0; b < nb; ++b)
        for (long t = 0; t < S; ++t)
            for (long u = 0; u < S; ++u)
                for (long w = 0; w < S; ++w) {
                    const long v = (t * S + u) * S + w;
                    for (long co = 0; co < co_n; ++co) {
                        double acc = bias ? bias[co] : 0.0;
                        for (long k = 0; k < 27; ++k) {
                            const long tt = nrefl(t + k / 9 - 1, S), uu = nrefl(u + (k / 3) % 3 - 1, S),
                                       ww = nrefl(w + k % 3 - 1, S);
                            const double *xp = x + ((b * S3) + (tt * S + uu) * S + ww) * ci_n;
                            const double *wp = W + (co * 27 + k) * ci_n;
                            for (long ci = 0; ci < ci_n; ++ci) acc += wp[ci] * xp[ci];
                        }
                        y[(b * S3 + v) * co_n + co] = acc;
                    }
                }
}

/* Exact adjoint of oracle_conv3d: given dy, accumulate dW, dbias and write dx (reflected
 * taps scatter their gradient back to the sample they read). */
void oracle_conv3d_backward(const double *x, long nb, long S, long ci_n, const double *W,
                            long co_n, const double *dy, double *dx, double *dW, double *db)
{
    const long S3 = S * S * S;
    if (dx) memset(dx, 0, sizeof(double) * nb * S3 * ci_n);
    for (long b = 0; b < nb; ++b)
        for (long t = 0; t < S; ++t)
            for (long u = 0; u < S; ++u)
                for (long w = 0; w < S; ++w) {
                    const long v = (t * S + u) * S + w;
                    for (long co = 0; co < co_n; ++co) {
                        const double g = dy[(b * S3 + v) * co_n + co];
                        if (db) db[co] += g;
                        for (long k = 0; k < 27; ++k) {
                            const long tt = nrefl(t + k / 9 - 1, S), uu = nrefl(u + (k / 3) % 3 - 1, S),
                                       ww = nrefl(w + k % 3 - 1, S);
                            const long xo = ((b * S3) + (tt * S + uu) * S + ww) * ci_n;
                            for (long ci = 0; ci < ci_n; ++ci) {
                                if (dW) dW[(co * 27 + k) * ci_n + ci] += g * x[xo + ci];
                                if (dx) dx[xo + ci] += g * W[(co * 27 + k) * ci_n + ci];
                            }
                        }
                    }
                }
}

/*
 * Forward pass of the stack: nl layers, channels ch[0] -> ch[1] -> ... -> ch[nl]; GELU after
 * every layer but the last.  params: for each layer W (ch[l+1]*27*ch[l]) then bias
 * (ch[l+1]).  z_out (optional): pre-activations of every layer, concatenated.  y: output.
 */
static long layer_offset(const long *ch, long l)
{
    long o = 0;
    for (long i = 0; i < l; ++i) o += ch[i + 1] * 27 * ch[i] + ch[i + 1];
    return o;
}

void oracle_net_forward(const double *x, long nb, long S, long nl, const long *ch,
                        const double *params, double *y, double *z_out)
{
    const long S3 = S * S * S;
    double *a = (double *)malloc(sizeof(double) * nb * S3 * ch[0]);
    memcpy(a, x, sizeof(double) * nb * S3 * ch[0]);
    long zo = 0;
    for (long l = 0; l < nl; ++l) {
        const long o = layer_offset(ch, l);
        double *z = (double *)malloc(sizeof(double) * nb * S3 * ch[l + 1]);
        oracle_conv3d(a, nb, S, ch[l], params + o, params + o + ch[l + 1] * 27 * ch[l], ch[l + 1], z);
        if (z_out) memcpy(z_out + zo, z, sizeof(double) * nb * S3 * ch[l + 1]);
        zo += nb * S3 * ch[l + 1];
        free(a);
        a = z;
        if (l + 1 < nl)
            for (long i = 0; i < nb * S3 * ch[l + 1]; ++i) a[i] = oracle_gelu(a[i]);
    }
    memcpy(y, a, sizeof(double) * nb * S3 * ch[nl]);
    free(a);
}

/*
 * The same network in the arithmetic it is specified with (BF16 weights and activations,
 * wider accumulation): every value that the specification keeps in BF16 is rounded to BF16
 * (8 significant bits, round to nearest, ties to even) where it is formed -- the input, each
 * layer's weights, each pre-activation z = conv + bias and each activation GELU(z) -- and
 * everything else stays FP64 (sums, biases, the output of the last layer).
 */
double oracle_round_bf16(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    const double m = frexp(v, &e); /* v = m 2^e, 0.5 <= |m| < 1 */
    return ldexp(nearbyint(ldexp(m, 8)), e - 8);
}

void oracle_net_forward_bf16(const double *x, long nb, long S, long nl, const long *ch,
                             const double *params, double *y)
{
    const long S3 = S * S * S;
    double *a = (double *)malloc(sizeof(double) * nb * S3 * ch[0]);
    for (long i = 0; i < nb * S3 * ch[0]; ++i) a[i] = oracle_round_bf16(x[i]);
    for (long l = 0; l < nl; ++l) {
        const long o = layer_offset(ch, l), nw = ch[l + 1] * 27 * ch[l];
        double *W = (double *)malloc(sizeof(double) * nw);
        for (long i = 0; i < nw; ++i) W[i] = oracle_round_bf16(params[o + i]);
        double *z = (double *)malloc(sizeof(double) * nb * S3 * ch[l + 1]);
        oracle_conv3d(a, nb, S, ch[l], W, params + o + nw, ch[l + 1], z);
        free(W);
        free(a);
        a = z;
        if (l + 1 < nl)
            for (long i = 0; i < nb * S3 * ch[l + 1]; ++i)
                a[i] = oracle_round_bf16(oracle_gelu(oracle_round_bf16(a[i])));
    }
    memcpy(y, a, sizeof(double) * nb * S3 * ch[nl]);
    free(a);
}

/* Gradient of sum(dy * y) w.r.t. every parameter (backpropagation of the forward above). */
void oracle_net_backward(const double *x, long nb, long S, long nl, const long *ch,
                         const double *params, const double *dy, double *grads)
{
    const long S3 = S * S * S;
    long ztot = 0;
    for (long l = 0; l < nl; ++l) ztot += nb * S3 * ch[l + 1];
    double *z = (double *)malloc(sizeof(double) * ztot);
    double *y = (double *)malloc(sizeof(double) * nb * S3 * ch[nl]);
    oracle_net_forward(x, nb, S, nl, ch, params, y, z);
    memset(grads, 0, sizeof(double) * layer_offset(ch, nl));
    double *g = (double *)malloc(sizeof(double) * nb * S3 * ch[nl]);
    memcpy(g, dy, sizeof(double) * nb * S3 * ch[nl]);
    long zo = ztot;
    for (long l = nl - 1; l >= 0; --l) {
        zo -= nb * S3 * ch[l + 1];
        /* input of layer l: x, or GELU of the previous pre-activation */
        double *in = (double *)malloc(sizeof(double) * nb * S3 * ch[l]);
        if (l == 0)
            memcpy(in, x, sizeof(double) * nb * S3 * ch[0]);
        else
            for (long i = 0; i < nb * S3 * ch[l]; ++i) in[i] = oracle_gelu(z[zo - nb * S3 * ch[l] + i]);
        const long o = layer_offset(ch, l);
        double *gin = (double *)malloc(sizeof(double) * nb * S3 * ch[l]);
        oracle_conv3d_backward(in, nb, S, ch[l], params + o, ch[l + 1], g, gin, grads + o,
                               grads + o + ch[l + 1] * 27 * ch[l]);
        if (l > 0)
            for (long i = 0; i < nb * S3 * ch[l]; ++i)
                gin[i] *= oracle_gelu_grad(z[zo - nb * S3 * ch[l] + i]);
        free(g);
        free(in);
        g = gin;
    }
    free(g);
    free(y);
    free(z);
}
