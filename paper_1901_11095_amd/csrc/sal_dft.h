// Small DFTs for the vector-ALU energy kernels (cube sides that do not fill a matrix-core
// tile, and the window-by-window kernel).  Since w^(om (L - r)) = conj w^(om r) for the
// twiddles w^k = e^{-2 pi i k / L}, the terms r and L - r enter through their sum and
// difference, and each pass over the pairs yields the outputs om and L - om together: about
// a quarter of the flops of the plain sum over all terms.  w[k] holds w^k; the conjugates are
// formed, not read.
#pragma once

#include <hip/hip_runtime.h>

namespace sal_dft {

// F[om] = sum_r b[r] w^(om r), om = 0..L-1.  With P = b_0 + sum_r u_r Re w^(om r)
// (+ b_(L/2) (-1)^om for even L) and Q = sum_r d_r Im w^(om r), u_r = b_r + b_(L-r),
// d_r = b_r - b_(L-r): F[om] = P + iQ and F[L - om] = P - iQ (P, Q complex).
template <int L>
__device__ __forceinline__ void cdft(const float2 (&b)[L], const float2 (&w)[L], float2 (&F)[L])
{
    constexpr int M = (L - 1) / 2;  // pairs (r, L - r), r = 1..M
    constexpr bool EV = L % 2 == 0;
    float2 u[M + 1], d[M + 1];
    float2 f0 = b[0];
#pragma unroll
    for (int r = 1; r <= M; ++r) {
        u[r] = make_float2(b[r].x + b[L - r].x, b[r].y + b[L - r].y);
        d[r] = make_float2(b[r].x - b[L - r].x, b[r].y - b[L - r].y);
        f0.x += u[r].x;
        f0.y += u[r].y;
    }
    if (EV) {
        f0.x += b[L / 2].x;
        f0.y += b[L / 2].y;
    }
    F[0] = f0;
#pragma unroll
    for (int om = 1; om <= M; ++om) {
        float2 P = b[0], Q = make_float2(0.f, 0.f);
#pragma unroll
        for (int r = 1; r <= M; ++r) {
            const float2 t = w[(om * r) % L];
            P.x = fmaf(u[r].x, t.x, P.x);
            P.y = fmaf(u[r].y, t.x, P.y);
            Q.x = fmaf(d[r].x, t.y, Q.x);
            Q.y = fmaf(d[r].y, t.y, Q.y);
        }
        if (EV) {
            const float sg = (om & 1) ? -1.f : 1.f;
            P.x = fmaf(sg, b[L / 2].x, P.x);
            P.y = fmaf(sg, b[L / 2].y, P.y);
        }
        F[om] = make_float2(P.x - Q.y, P.y + Q.x);
        F[L - om] = make_float2(P.x + Q.y, P.y - Q.x);
    }
    if (EV) {
        float2 fh = b[0];
#pragma unroll
        for (int r = 1; r <= M; ++r) {
            const float sg = (r & 1) ? -1.f : 1.f;
            fh.x = fmaf(sg, u[r].x, fh.x);
            fh.y = fmaf(sg, u[r].y, fh.y);
        }
        const float sg = ((L / 2) & 1) ? -1.f : 1.f;
        F[L / 2] = make_float2(fmaf(sg, b[L / 2].x, fh.x), fmaf(sg, b[L / 2].y, fh.y));
    }
}

// X[mu] = sum_p v[p] w^(mu p) of real v, mu = 0..L/2: Re X[mu] = v_0 + sum_p u_p Re w^(mu p)
// (+ v_(L/2) (-1)^mu for even L), Im X[mu] = sum_p d_p Im w^(mu p); X[L/2] of even L is real.
template <int L>
__device__ __forceinline__ void rdft_half(const float (&v)[L], const float2 (&w)[L], float2 (&X)[L / 2 + 1])
{
    constexpr int M = (L - 1) / 2;
    constexpr bool EV = L % 2 == 0;
    float u[M + 1], d[M + 1];
    float x0 = v[0];
#pragma unroll
    for (int p = 1; p <= M; ++p) {
        u[p] = v[p] + v[L - p];
        d[p] = v[p] - v[L - p];
        x0 += u[p];
    }
    if (EV) x0 += v[L / 2];
    X[0] = make_float2(x0, 0.f);
#pragma unroll
    for (int mu = 1; mu <= M; ++mu) {
        float re = v[0], im = 0.f;
#pragma unroll
        for (int p = 1; p <= M; ++p) {
            const float2 t = w[(mu * p) % L];
            re = fmaf(u[p], t.x, re);
            im = fmaf(d[p], t.y, im);
        }
        if (EV) re = fmaf((mu & 1) ? -1.f : 1.f, v[L / 2], re);
        X[mu] = make_float2(re, im);
    }
    if (EV) {
        float xh = v[0];
#pragma unroll
        for (int p = 1; p <= M; ++p) xh = fmaf((p & 1) ? -1.f : 1.f, u[p], xh);
        X[L / 2] = make_float2(fmaf(((L / 2) & 1) ? -1.f : 1.f, v[L / 2], xh), 0.f);
    }
}

}  // namespace sal_dft
