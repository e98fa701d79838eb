// d3q19.hpp -- lattice constants and per-node arithmetic of the WDLB step
// on gfx950.  Device code only; included by wdlb.hip.
//
// Storage encoding of the populations.  After the collision at node s the
// library keeps the node's density and post-collision velocity
// u*_s = (j + F)/rho and the deviation h_a(s) = f*_a(s) - feq_a(rho_s, u*_s),
// which carries no mass and no momentum.  A population streamed to node r is
//     f_a(r) = w_a rho_s  +  w_a rho_s P_a(u*_s)  +  h_a(s),
//     P_a(u) = 3 c_a.u + 9/2 (c_a.u)^2 - 3/2 u.u,
// and the three parts are never added into one number before the moments
// are formed from differences of mirror-image sources.  The flow therefore
// lives in u* (full FP32 relative precision) instead of in differences of
// populations of size w rho: plain FP32 populations lose about four digits
// of the momentum, and an encoding against the collision velocity u leaves
// half the force in h, where the large wall-normal mean-field force of the
// layers next to a wall swamps the small driving force in FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wdlb {

constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// the populations with c = +1 along an axis, and their mirror images across it
constexpr int PX[5] = {1, 7, 9, 11, 13}, MXP[5] = {2, 10, 8, 14, 12};
constexpr int PY[5] = {3, 7, 10, 15, 17}, MYP[5] = {4, 9, 8, 18, 16};
constexpr int PZ[5] = {5, 11, 14, 15, 18}, MZP[5] = {6, 13, 12, 17, 16};

template <typename R>
__host__ __device__ constexpr R wgt(int a)
{
    return a == 0 ? R(1) / R(3) : (a <= 6 ? R(1) / R(18) : R(1) / R(36));
}

template <typename R>
struct alignas(4 * sizeof(R)) V4 {
    R x, y, z, w;
};

// h storage type: R itself for FP32/FP64; 16-bit brain float for BF16.
struct bf16 {
    uint16_t bits;
};

// BF16 mode: h carries no mass and no momentum, but its BF16 roundings do.
// Four populations (rest, +x, +y, +z) are therefore stored in FP32 and set
// from the rounded others so that the stored h closes mass and momentum:
// the FP32 value is split into its high half (in the population's own
// plane) and its low half (in plane 19 + closure slot).
__host__ __device__ constexpr int closure_slot(int a) { return a == 0 ? 0 : (a == 1 ? 1 : (a == 3 ? 2 : (a == 5 ? 3 : -1))); }
template <typename HS>
__host__ __device__ constexpr int hplanes() { return 19; }
template <>
__host__ __device__ constexpr int hplanes<bf16>() { return 23; }

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    // round to nearest even; NaN stays NaN
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

// Stochastic rounding to BF16: the FP32 bit pattern of |v| plus a uniform
// 16-bit integer, truncated to its upper half, is v rounded up or down with
// probabilities given by the distance to the two neighbours (unbiased).
__device__ __forceinline__ uint16_t f32_to_bf16_sr(float f, uint32_t r16)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return f32_to_bf16(f);
    const uint32_t mag = u & 0x7fffffffu;
    const uint32_t up = mag + (r16 & 0xffffu);
    if ((up & 0x7f800000u) == 0x7f800000u) return f32_to_bf16(f);  // would round to infinity
    return uint16_t(((u & 0x80000000u) | up) >> 16);
}

// SplitMix64 output function (Steele, Lea and Flood, 2014): a counter-based
// source of 64 random bits per input
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// P_a(u) for the velocity a (compile-time after unrolling)
template <typename R>
__device__ __forceinline__ R pterm(int a, R ux, R uy, R uz)
{
    R cu = R(CX[a]) * ux + R(CY[a]) * uy + R(CZ[a]) * uz;
    R uu = ux * ux + uy * uy + uz * uz;
    return R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
}

// One z-plane of a lattice of stacked slits (the serving lattice): fluid or
// a solid gap between two slits; fluid planes carry their slit's body force
// and relaxation (omega = 1/tau, ksrc = 1 - 1/(2 tau)).
struct ZPlane {
    double gx, gy, gz, omega, ksrc;
    int fluid, pad0, pad1, pad2, pad3, pad4;
};

struct Geom {
    int nx, ny, nz, walls;
    long long N;
    int tiny;              // 1 when an axis is shorter than the stencil reach: wrap by modulo
    const ZPlane *zp;      // per-plane table of a stacked lattice, or null (one slit)
};

// the plane z (in range when periodic) holds fluid: between the walls, and
// not a gap of a stacked lattice
__device__ __forceinline__ bool zfluid(const Geom &g, int z)
{
    if (g.walls && (z < 0 || z >= g.nz)) return false;
    return g.zp == nullptr || g.zp[z].fluid != 0;
}

__device__ __forceinline__ int wrap1(int v, int n)
{
    // v in [-n, 2n)
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

__device__ __forceinline__ int wrapm(int v, int n)
{
    int m = v % n;
    return m < 0 ? m + n : m;
}

}  // namespace wdlb
