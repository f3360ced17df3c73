// Device helpers shared by the gfx950 kernels of libsal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

typedef float f4 __attribute__((ext_vector_type(4)));

namespace sal_dev {

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Reflect u into [0, n) without repeating the edge sample; exact for -(n-1) <= u <= 2(n-1).
// The final clamp only matters for padding positions of edge tiles, whose results are
// never stored.
__device__ __forceinline__ int refl_idx(int u, int n)
{
    u = u < 0 ? -u : u;
    u = u >= n ? 2 * (n - 1) - u : u;
    return u < 0 ? 0 : (u >= n ? n - 1 : u);
}

// Workgroup -> tile order that keeps neighbouring tiles on one XCD: workgroups are
// dispatched round-robin over the 8 XCDs, so workgroup b runs on XCD b % 8; giving each XCD
// a contiguous range of tiles lets halo re-reads hit that XCD's L2.
// The value unchanged, but opaque to the optimiser: an index derived from it inside a loop
// is recomputed there instead of being hoisted and held in registers across the loop.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ int xcd_tile(int bid, int nblk)
{
    const int q = nblk >> 3;
    if (bid >= (q << 3)) return bid;
    return (bid & 7) * q + (bid >> 3);
}

template <int L>
struct Geo {
    static constexpr int H = L / 2;                         // window start = v - H
    static constexpr int h = L / 2 + 1;                     // t frequencies kept (Hermitian half)
    static constexpr int KS = (2 * L) / 4;                  // 16x16x4 steps of a complex contraction
    static constexpr int MT = (2 * L) / 16;                 // 16-row tiles of (freq, re|im)
    static constexpr int KSA = L / 4;                       // steps of the real t contraction
    static constexpr int MTA = (2 * h + 15) / 16;           // row tiles of the t contraction
    static constexpr int NR = (h - 2) * L + 2 * (L / 2 + 1);  // (mu, nu) rows kept
};

// Tile shapes: NW waves (= x-rows) per workgroup, TY voxels along y.
#ifndef SAL_NW8
#define SAL_NW8 8
#endif
#ifndef SAL_TY8
#define SAL_TY8 32
#endif
#ifndef SAL_NW16
#define SAL_NW16 8
#endif
#ifndef SAL_TY16
#define SAL_TY16 16
#endif
// WPE: waves per SIMD the register allocation must allow (unit-stride tiles; strided ones
// are LDS-bound at two).  At L = 8 the LDS of a workgroup admits three per CU, i.e. six
// waves per SIMD; at L = 16 (stage B in two halves) two per CU, i.e. four waves per SIMD.
// The registers are capped to match.
#ifndef SAL_WPE8
#define SAL_WPE8 6
#endif
#ifndef SAL_WPE16
#define SAL_WPE16 4
#endif
template <int L>
struct TileCfg;
template <>
struct TileCfg<8> {
    static constexpr int NW = SAL_NW8, TY = SAL_TY8, WPE = SAL_WPE8;
    static constexpr bool W_LDS = true;
};
template <>
struct TileCfg<16> {
    static constexpr int NW = SAL_NW16, TY = SAL_TY16, WPE = SAL_WPE16;
    static constexpr bool W_LDS = false;
};

}  // namespace sal_dev
using namespace sal_dev;

