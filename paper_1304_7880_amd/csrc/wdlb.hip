// wdlb.hip -- MI355X (gfx950) implementation of the WDLB time step behind
// the C ABI of include/wdlb.h.
//
// One step (Sec. 5 of the paper, steps 2-4; the step-1 initialisation is
// k_init) is five kernels on the caller's stream:
//   k_moments    pull-stream the stored populations, density and momentum
//   k_ball       Fischer-Methfessel smoothed density nbar (ball of diameter sigma)
//   k_gamma      Carnahan-Starling contact value at the 8 half-lattice
//                midpoints of every node, gamma_h(r) = g_CS(nbar(r + h/2))
//   k_meanfield  contact-shell sum of the mean-field force F^mf; the velocity
//                u1 = j/rho + (g + F^mf)/2 with which F^v and A_ij are formed
//   k_collide    contact-shell sums of the viscous force F^v and the SMDB
//                field A_ij, forced BGK collision with the A-source, and the
//                write of the post-collision populations (streaming happens
//                in the next pull, with half-way bounce-back at the walls)
//
// The shell sums visit the contact shell in groups of four mirror images
// (+-a, +-b, c): the x- and y-odd parts of every sum are formed as
// differences of mirror images before they are accumulated, so a state that
// does not depend on x or y gives exactly zero x and y forces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wdlb.h"
#include "d3q19.hpp"

using namespace wdlb;

namespace {

constexpr double KT = 1.0 / 3.0;
constexpr int MAX_QUADS = 8192;
constexpr int MAX_BALL = 32768;
constexpr int FLAG_ETA = 1, FLAG_RHO = 2;

// one group of contact-shell offsets (+-a, +-b, c); p = weight*alpha,
// q = weight*alpha_i alpha_j with alpha = (a, b, c)/|e|; weight 1, 1/2 or
// 1/4 undoes the repeated members when a or b is zero
template <typename R>
struct Quad {
    int a, b, c, hidx;
    R px, py, pz, qxx, qyy, qzz, qxy, qxz, qyz, pad0, pad1, pad2;
};

template <typename R, typename HS>
__device__ __forceinline__ R ldh(const HS *p);
template <>
__device__ __forceinline__ float ldh<float, float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ double ldh<double, double>(const double *p) { return *p; }
template <>
__device__ __forceinline__ float ldh<float, bf16>(const bf16 *p) { return bf16_to_f32(p->bits); }

template <typename R, typename HS>
__device__ __forceinline__ void sth(HS *p, R v);
template <>
__device__ __forceinline__ void sth<float, float>(float *p, float v) { *p = v; }
template <>
__device__ __forceinline__ void sth<double, double>(double *p, double v) { *p = v; }
template <>
__device__ __forceinline__ void sth<float, bf16>(bf16 *p, float v) { p->bits = f32_to_bf16(v); }

__device__ __forceinline__ void raise_flag(int *flag, int bit)
{
    __hip_atomic_fetch_or(flag, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// pull: the population arriving at (x, y, z) with velocity c_a,
//   f_a = w_a rho_s (1 + P_a(u*_s)) + h_a(s),
// from the source s = r - c_a, or by half-way bounce-back from r itself.
// The pull, the moments and the collision run in FP64 arithmetic: near a
// wall u* has a large wall-normal part (half the mean-field force per unit
// mass) next to a tiny flow part, and FP32 products c.u* and sums of
// populations of size w rho lose the flow to rounding.  FP64 sums of the
// stored parts are exact enough that no special summation order is needed.
// On gfx950 an FP64 FMA issues at the rate of an unpacked FP32 FMA, and this
// part is a few percent of the step's arithmetic; storage keeps the
// precision of the mode.
// ---------------------------------------------------------------------------
typedef double D;

template <typename R, typename HS>
__device__ __forceinline__ D fpull(const Geom &g, const V4<R> *__restrict__ ru, const HS *__restrict__ h, int x,
                                   int y, int z, int r, int a)
{
    int sz = z - CZ[a];
    bool bb = false;
    if (CZ[a] != 0) {
        if (g.walls) bb = (sz < 0 || sz >= g.nz);
        else sz = wrap1(sz, g.nz);
    }
    int s, ha;
    if (bb) {
        s = r;
        ha = OPP[a];
    } else {
        int sx = CX[a] ? wrap1(x - CX[a], g.nx) : x;
        int sy = CY[a] ? wrap1(y - CY[a], g.ny) : y;
        s = (sz * g.ny + sy) * g.nx + sx;
        ha = a;
    }
    const V4<R> q = ru[s];
    const D ux = q.y, uy = q.z, uz = q.w;
    D cu = D(CX[a]) * ux + D(CY[a]) * uy + D(CZ[a]) * uz;
    if (bb) cu = -cu;
    const D P = D(3) * cu + D(4.5) * cu * cu - D(1.5) * (ux * ux + uy * uy + uz * uz);
    return wgt<D>(a) * D(q.x) * (D(1) + P) + D(ldh<R, HS>(h + (long long)ha * g.N + s));
}

template <typename R, typename HS>
__device__ __forceinline__ void pull_moments(const Geom &g, const V4<R> *__restrict__ ru, const HS *__restrict__ h,
                                             int x, int y, int z, D &rho, D &jx, D &jy, D &jz)
{
    const int r = (z * g.ny + y) * g.nx + x;
    rho = jx = jy = jz = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const D f = fpull<R, HS>(g, ru, h, x, y, z, r, a);
        rho += f;
        if (CX[a]) jx += D(CX[a]) * f;
        if (CY[a]) jy += D(CY[a]) * f;
        if (CZ[a]) jz += D(CZ[a]) * f;
    }
}

__device__ __forceinline__ bool node_of(const Geom &g, long long i, int &x, int &y, int &z)
{
    if (i >= g.N) return false;
    int ii = (int)i;
    x = ii % g.nx;
    int t = ii / g.nx;
    y = t % g.ny;
    z = t / g.ny;
    return true;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_fill(Geom g, V4<R> *ru, R n0, R ux, R uy, R uz)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < g.N) ru[i] = V4<R>{n0, ux, uy, uz};
}

// Sec. 5, step 1: the populations at every node r are feq(n(r), u(r)).  The
// library stores pre-stream populations, so node s keeps for direction a the
// value that the next pull delivers to t = s + c_a, feq_a(n(t), u(t)), or,
// when t lies in a wall, the value that bounces back into s itself,
// feq_abar(n(s), u(s)); h is that minus feq_a(n(s), u(s)) in difference form.
template <typename R, typename HS>
__global__ __launch_bounds__(256) void k_init(Geom g, const V4<R> *__restrict__ ru, HS *__restrict__ h)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const V4<R> q = ru[i];
    const R uu = q.y * q.y + q.z * q.z + q.w * q.w;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const R w = wgt<R>(a);
        R cu = R(CX[a]) * q.y + R(CY[a]) * q.z + R(CZ[a]) * q.w;
        R Ps = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
        int tz = z + CZ[a];
        bool bb = false;
        if (CZ[a] != 0) {
            if (g.walls) bb = (tz < 0 || tz >= g.nz);
            else tz = wrap1(tz, g.nz);
        }
        R val;
        if (bb) {
            val = -R(6) * w * q.x * cu;  // feq_abar(s) - feq_a(s)
        } else {
            int tx = CX[a] ? wrap1(x + CX[a], g.nx) : x;
            int ty = CY[a] ? wrap1(y + CY[a], g.ny) : y;
            V4<R> t = ru[(tz * g.ny + ty) * g.nx + tx];
            R ct = R(CX[a]) * t.y + R(CY[a]) * t.z + R(CZ[a]) * t.w;
            R Pt = R(3) * ct + R(4.5) * ct * ct - R(1.5) * (t.y * t.y + t.z * t.z + t.w * t.w);
            val = w * ((t.x - q.x) + (t.x * Pt - q.x * Ps));
        }
        sth<R, HS>(h + (long long)a * g.N + i, val);
    }
}

template <typename R, typename HS>
__global__ __launch_bounds__(256) void k_moments(Geom g, const V4<R> *__restrict__ ru, const HS *__restrict__ h, R *__restrict__ rho,
                          R *__restrict__ jx, R *__restrict__ jy, R *__restrict__ jz, int *flag)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    D r, a, b, c;
    pull_moments<R, HS>(g, ru, h, x, y, z, r, a, b, c);
    if (!(r > D(0)) || !(r < D(INFINITY))) raise_flag(flag, FLAG_RHO);
    rho[i] = R(r);
    jx[i] = R(a);
    jy[i] = R(b);
    jz[i] = R(c);
}

template <typename R>
__global__ __launch_bounds__(256) void k_ball(Geom g, const R *__restrict__ rho, const int4 *__restrict__ ball, int nball, R inv_nball,
                       R *__restrict__ nbar)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    R s = 0;
    for (int q = 0; q < nball; ++q) {
        int4 e = ball[q];
        int zz = z + e.z;
        if (g.walls) {
            if (zz < 0 || zz >= g.nz) continue;
        } else {
            zz = g.tiny ? wrapm(zz, g.nz) : wrap1(zz, g.nz);
        }
        int xx = g.tiny ? wrapm(x + e.x, g.nx) : wrap1(x + e.x, g.nx);
        int yy = g.tiny ? wrapm(y + e.y, g.ny) : wrap1(y + e.y, g.ny);
        s += rho[(zz * g.ny + yy) * g.nx + xx];
    }
    nbar[i] = s * inv_nball;
}

template <typename R>
__global__ __launch_bounds__(256) void k_gamma(Geom g, const R *__restrict__ nbar, R eta_per_n, R wS, R *__restrict__ gam, int *flag)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    int xs[2] = {x, wrap1(x + 1, g.nx)}, ys[2] = {y, wrap1(y + 1, g.ny)};
    int z1 = z + 1;
    bool zin = true;
    if (g.walls) zin = z1 < g.nz;
    else z1 = wrap1(z1, g.nz);
    int zs[2] = {z, zin ? z1 : z};
    for (int hi = 0; hi < 8; ++hi) {
        int hx = hi & 1, hy = (hi >> 1) & 1, hz = (hi >> 2) & 1;
        R s = 0;
        int cnt = 0;
        bool inside = true;
        for (int cz = 0; cz <= hz; ++cz)
            for (int cy = 0; cy <= hy; ++cy)
                for (int cx = 0; cx <= hx; ++cx) {
                    bool ok = !(cz == 1 && !zin);
                    inside = inside && ok;
                    if (ok) s += nbar[(zs[cz] * g.ny + ys[cy]) * g.nx + xs[cx]];
                    ++cnt;
                }
        R eta = eta_per_n * (s / R(cnt));
        R val;
        if (eta < R(1)) {
            R om = R(1) - eta;
            val = wS * (R(1) - R(0.5) * eta) / (om * om * om);
        } else {
            if (inside) raise_flag(flag, FLAG_ETA);
            val = R(0);
        }
        gam[(long long)hi * g.N + i] = val;
    }
}

// member m of quad (a, b, c): e = (sx a, sy b, c), (sx, sy) = (+,+), (-,+), (+,-), (-,-)
struct Member {
    int s;       // node index of r + e (clamped)
    int mid;     // node index of r + floor(e/2) (clamped)
    bool in;     // r + e inside the slit
};

__device__ __forceinline__ Member member(const Geom &g, int x, int y, int z, int ex, int ey, int ez)
{
    Member m;
    int zz = z + ez, zm = z + (ez >> 1);
    m.in = true;
    if (g.walls) {
        m.in = (zz >= 0 && zz < g.nz);
        zz = min(max(zz, 0), g.nz - 1);
        zm = min(max(zm, 0), g.nz - 1);
    } else {
        zz = g.tiny ? wrapm(zz, g.nz) : wrap1(zz, g.nz);
        zm = g.tiny ? wrapm(zm, g.nz) : wrap1(zm, g.nz);
    }
    int xx = g.tiny ? wrapm(x + ex, g.nx) : wrap1(x + ex, g.nx);
    int yy = g.tiny ? wrapm(y + ey, g.ny) : wrap1(y + ey, g.ny);
    int xm = g.tiny ? wrapm(x + (ex >> 1), g.nx) : wrap1(x + (ex >> 1), g.nx);
    int ym = g.tiny ? wrapm(y + (ey >> 1), g.ny) : wrap1(y + (ey >> 1), g.ny);
    m.s = (zz * g.ny + yy) * g.nx + xx;
    m.mid = (zm * g.ny + ym) * g.nx + xm;
    return m;
}

template <typename R>
__global__ __launch_bounds__(256) void k_meanfield(Geom g, const R *__restrict__ rho, const R *__restrict__ jx, const R *__restrict__ jy,
                            const R *__restrict__ jz, const R *__restrict__ gam,
                            const Quad<R> *__restrict__ quads, int nq, R cmf, R gx, R gy, R gz,
                            V4<R> *__restrict__ ru1, V4<R> *__restrict__ fmf)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    R fx = 0, fy = 0, fz = 0;
    for (int q = 0; q < nq; ++q) {
        const Quad<R> &Qd = quads[q];
        const R *gh = gam + (long long)Qd.hidx * g.N;
        R G[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int ex = (m & 1) ? -Qd.a : Qd.a, ey = (m & 2) ? -Qd.b : Qd.b;
            Member M = member(g, x, y, z, ex, ey, Qd.c);
            G[m] = M.in ? gh[M.mid] * rho[M.s] : R(0);
        }
        R P1 = G[0] + G[1], M1 = G[0] - G[1], P2 = G[2] + G[3], M2 = G[2] - G[3];
        fx += Qd.px * (M1 + M2);
        fy += Qd.py * (P1 - P2);
        fz += Qd.pz * (P1 + P2);
    }
    R Fx = cmf * fx, Fy = cmf * fy, Fz = cmf * fz;
    R r = rho[i];
    R inv = R(1) / r;
    ru1[i] = V4<R>{r, jx[i] * inv + R(0.5) * (gx + Fx), jy[i] * inv + R(0.5) * (gy + Fy),
                   jz[i] * inv + R(0.5) * (gz + Fz)};
    fmf[i] = V4<R>{Fx, Fy, Fz, R(0)};
}

template <typename R, typename HS, bool READ>
__global__ __launch_bounds__(256) void k_collide(Geom g, const V4<R> *__restrict__ ru1, const V4<R> *__restrict__ fmf,
                          const R *__restrict__ gam, const Quad<R> *__restrict__ quads, int nq, R cv, R cA,
                          R omega, R ksrc, R gx, R gy, R gz, int smdb, const V4<R> *__restrict__ ru_in,
                          const HS *__restrict__ h_in, V4<R> *__restrict__ ru_out, HS *__restrict__ h_out,
                          R *__restrict__ u_rd, R *__restrict__ F_rd, R *__restrict__ A_rd)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    V4<R> c0 = ru1[i];
    R vx = 0, vy = 0, vz = 0;                         // F^v sums
    R axx = 0, ayy = 0, azz = 0, axy = 0, axz = 0, ayz = 0;  // A sums
    for (int q = 0; q < nq; ++q) {
        const Quad<R> &Qd = quads[q];
        const R *gh = gam + (long long)Qd.hidx * g.N;
        R Wx[4], Wy[4], Wz[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int ex = (m & 1) ? -Qd.a : Qd.a, ey = (m & 2) ? -Qd.b : Qd.b;
            Member M = member(g, x, y, z, ex, ey, Qd.c);
            V4<R> s = ru1[M.s];
            R G = M.in ? gh[M.mid] * s.x : R(0);
            Wx[m] = G * (s.y - c0.y);
            Wy[m] = G * (s.z - c0.z);
            Wz[m] = G * (s.w - c0.w);
        }
        // Hadamard transform over the mirror signs (sx, sy)
        R xP1 = Wx[0] + Wx[1], xM1 = Wx[0] - Wx[1], xP2 = Wx[2] + Wx[3], xM2 = Wx[2] - Wx[3];
        R yP1 = Wy[0] + Wy[1], yM1 = Wy[0] - Wy[1], yP2 = Wy[2] + Wy[3], yM2 = Wy[2] - Wy[3];
        R zP1 = Wz[0] + Wz[1], zM1 = Wz[0] - Wz[1], zP2 = Wz[2] + Wz[3], zM2 = Wz[2] - Wz[3];
        R x0 = xP1 + xP2, xX = xM1 + xM2, xY = xP1 - xP2, xXY = xM1 - xM2;
        R y0 = yP1 + yP2, yX = yM1 + yM2, yY = yP1 - yP2, yXY = yM1 - yM2;
        R z0 = zP1 + zP2, zX = zM1 + zM2, zY = zP1 - zP2;
        vx += Qd.qxx * x0 + Qd.qxy * yXY + Qd.qxz * zX;
        vy += Qd.qxy * xXY + Qd.qyy * y0 + Qd.qyz * zY;
        vz += Qd.qxz * xX + Qd.qyz * yY + Qd.qzz * z0;
        axx += Qd.px * xX;
        ayy += Qd.py * yY;
        azz += Qd.pz * z0;
        axy += Qd.py * xY + Qd.px * yX;
        axz += Qd.pz * x0 + Qd.px * zX;
        ayz += Qd.pz * y0 + Qd.py * zY;
    }
    // forces and the traceless SMDB field
    const R r0 = c0.x;
    V4<R> fm = fmf[i];
    R Fx = r0 * (gx + fm.x + cv * vx), Fy = r0 * (gy + fm.y + cv * vy), Fz = r0 * (gz + fm.z + cv * vz);
    R ca = cA * r0;
    R Axx = ca * R(2) * axx, Ayy = ca * R(2) * ayy, Azz = ca * R(2) * azz;
    R Axy = ca * axy, Axz = ca * axz, Ayz = ca * ayz;
    R tr = (Axx + Ayy + Azz) / R(3);
    Axx -= tr;
    Ayy -= tr;
    Azz -= tr;
    if (!smdb) Axx = Ayy = Azz = Axy = Axz = Ayz = R(0);

    D rho, jx, jy, jz;
    pull_moments<R, HS>(g, ru_in, h_in, x, y, z, rho, jx, jy, jz);
    const D inv = D(1) / rho;
    const D Fxd = Fx, Fyd = Fy, Fzd = Fz;
    const D ux = (jx + D(0.5) * Fxd) * inv, uy = (jy + D(0.5) * Fyd) * inv, uz = (jz + D(0.5) * Fzd) * inv;
    if (READ) {
        const long long N = g.N;
        u_rd[i] = R(ux);
        u_rd[N + i] = R(uy);
        u_rd[2 * N + i] = R(uz);
        F_rd[i] = Fx;
        F_rd[N + i] = Fy;
        F_rd[2 * N + i] = Fz;
        A_rd[i] = Axx;
        A_rd[N + i] = Ayy;
        A_rd[2 * N + i] = Azz;
        A_rd[3 * N + i] = Axy;
        A_rd[4 * N + i] = Axz;
        A_rd[5 * N + i] = Ayz;
        return;
    }
    // Forced BGK with the SMDB source (trapezoidal weighting ksrc = 1 - 1/(2 tau)),
    // stored against the post-collision velocity u* = u + F/(2 rho):
    //   h*_a = (1 - omega)(f_a - feq_a(u)) + [feq_a(u) - feq_a(u*)] + ksrc (guo_a + sa_a)
    // so the deviation carries no momentum and the flow lives in u* alone.
    const D uu = ux * ux + uy * uy + uz * uz;
    const D uF = ux * Fxd + uy * Fyd + uz * Fzd;
    const D keep = D(1) - D(omega), ks = D(ksrc);
    const D dx = D(0.5) * Fxd * inv, dy = D(0.5) * Fyd * inv, dz = D(0.5) * Fzd * inv;  // u* - u
    const D sx = D(2) * ux + dx, sy = D(2) * uy + dy, sz = D(2) * uz + dz;                // u + u*
    const D dsum = dx * sx + dy * sy + dz * sz;
    const D Axxd = Axx, Ayyd = Ayy, Azzd = Azz, Axyd = Axy, Axzd = Axz, Ayzd = Ayz;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const D w = wgt<D>(a);
        const D cu = D(CX[a]) * ux + D(CY[a]) * uy + D(CZ[a]) * uz;
        const D P = D(3) * cu + D(4.5) * cu * cu - D(1.5) * uu;
        const D fneq = fpull<R, HS>(g, ru_in, h_in, x, y, z, (z * g.ny + y) * g.nx + x, a) - w * rho * (D(1) + P);
        const D cF = D(CX[a]) * Fxd + D(CY[a]) * Fyd + D(CZ[a]) * Fzd;
        const D guo = w * (D(3) * (cF - uF) + D(9) * cu * cF);
        const D cAc = D(CX[a] * CX[a]) * Axxd + D(CY[a] * CY[a]) * Ayyd + D(CZ[a] * CZ[a]) * Azzd +
                      D(2 * CX[a] * CY[a]) * Axyd + D(2 * CX[a] * CZ[a]) * Axzd + D(2 * CY[a] * CZ[a]) * Ayzd;
        const D sa = D(4.5) * w * cAc;
        const D cd = D(CX[a]) * dx + D(CY[a]) * dy + D(CZ[a]) * dz;
        const D cs = D(CX[a]) * sx + D(CY[a]) * sy + D(CZ[a]) * sz;
        const D deq = w * rho * (-D(3) * cd - D(4.5) * cd * cs + D(1.5) * dsum);
        sth<R, HS>(h_out + (long long)a * g.N + i, R(keep * fneq + deq + ks * (guo + sa)));
    }
    ru_out[i] = V4<R>{R(rho), R(ux + dx), R(uy + dy), R(uz + dz)};
}

template <typename R, typename HS>
__global__ __launch_bounds__(256) void k_populations(Geom g, const V4<R> *__restrict__ ru, const HS *__restrict__ h, R *__restrict__ f)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const int r = (z * g.ny + y) * g.nx + x;
#pragma unroll
    for (int a = 0; a < Q; ++a) f[(long long)a * g.N + i] = R(fpull<R, HS>(g, ru, h, x, y, z, r, a));
}

// FP64 plane sums of rho, u_x and rho*u_x; one block per z-plane, fixed
// reduction order (deterministic)
template <typename R>
__global__ __launch_bounds__(256) void k_planes(Geom g, const R *__restrict__ rho, const R *__restrict__ ux, double *__restrict__ out)
{
    __shared__ double sh[3][256];
    const int z = blockIdx.x;
    const int plane = g.nx * g.ny;
    double a = 0, b = 0, c = 0;
    for (int k = threadIdx.x; k < plane; k += blockDim.x) {
        int i = z * plane + k;
        double r = (double)rho[i], u = (double)ux[i];
        a += r;
        b += u;
        c += r * u;
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    sh[2][threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[z] = sh[0][0];
        out[g.nz + z] = sh[1][0];
        out[2 * g.nz + z] = sh[2][0];
    }
}

}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct wdlb_ctx {
    wdlb_lattice_desc desc;
    wdlb_params prm;
    hipStream_t stream;
    Geom g;
    int prec;
    size_t rsize;      // bytes of one real (compute type)
    size_t hsize;      // bytes of one stored h
    char *ws;
    size_t ws_bytes;
    // carved device arrays
    void *ru[2], *h[2];
    void *rho, *jx, *jy, *jz, *nbar, *gam, *ru1, *fmf, *u_rd, *F_rd, *A_rd;
    double *planes;
    int *flag;
    void *quads;
    int4 *ball;
    int nq, nball;
    double wS;         // 4 pi / |S|
    int cur;
    int64_t step;
    bool inited;
    std::string err;
    // event timing of the step kernels
    bool prof = false;
    std::vector<hipEvent_t> ev_free;
    struct Pending {
        int k;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    double prof_ms[WDLB_NKERNELS] = {0};
    int64_t prof_n[WDLB_NKERNELS] = {0};
};

namespace {

wdlb_status fail(wdlb_ctx *c, wdlb_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

#define HIPCHK(ctx, call)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(ctx, WDLB_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool desc_ok(const wdlb_lattice_desc *d)
{
    if (!d || d->nx < 1 || d->ny < 1 || d->nz < 1) return false;
    long long N = (long long)d->nx * d->ny * d->nz;
    if (N * 19 >= (1LL << 31)) return false;
    return d->precision == WDLB_FP32 || d->precision == WDLB_FP64 || d->precision == WDLB_BF16_NEQ;
}

bool params_ok(const wdlb_params *p)
{
    if (!p) return false;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return false;
    if (p->nonlocal && !(p->sigma >= 1.0 && p->sigma <= 24.0)) return false;
    if (!(p->eta > 0.0 && p->eta < 1.0)) return false;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->g[i])) return false;
    return true;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t off_ru[2], off_h[2], off_rho, off_j[3], off_nbar, off_gam, off_ru1, off_fmf, off_urd, off_Frd, off_Ard,
        off_planes, off_flag, off_quads, off_ball, total;
};

Layout layout(const wdlb_lattice_desc *d)
{
    Layout L;
    size_t N = (size_t)d->nx * d->ny * d->nz;
    size_t r = d->precision == WDLB_FP64 ? 8 : 4;
    size_t hs = d->precision == WDLB_FP64 ? 8 : (d->precision == WDLB_BF16_NEQ ? 2 : 4);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    for (int b = 0; b < 2; ++b) {
        L.off_ru[b] = take(4 * r * N);
        L.off_h[b] = take(19 * hs * N);
    }
    L.off_rho = take(r * N);
    for (int c = 0; c < 3; ++c) L.off_j[c] = take(r * N);
    L.off_nbar = take(r * N);
    L.off_gam = take(8 * r * N);
    L.off_ru1 = take(4 * r * N);
    L.off_fmf = take(4 * r * N);
    L.off_urd = take(3 * r * N);
    L.off_Frd = take(3 * r * N);
    L.off_Ard = take(6 * r * N);
    L.off_planes = take(3 * sizeof(double) * (size_t)d->nz);
    L.off_flag = take(256);
    L.off_quads = take(MAX_QUADS * sizeof(Quad<double>));
    L.off_ball = take(MAX_BALL * sizeof(int4));
    L.total = o;
    return L;
}

// stencil tables (Sec. 3): ball |e|^2 <= sigma^2/4; shell (sigma-1/2)^2 <= |e|^2 < (sigma+1/2)^2
std::vector<int4> build_ball(double sigma)
{
    std::vector<int4> b;
    int R = (int)std::ceil(sigma / 2.0) + 1;
    for (int z = -R; z <= R; ++z)
        for (int y = -R; y <= R; ++y)
            for (int x = -R; x <= R; ++x)
                if (4.0 * (x * x + y * y + z * z) <= sigma * sigma) b.push_back(make_int4(x, y, z, 0));
    return b;
}

template <typename R>
std::vector<Quad<R>> build_quads(double sigma, int &nshell)
{
    std::vector<Quad<R>> v;
    int R_ = (int)std::ceil(sigma + 0.5) + 1;
    double lo = (sigma - 0.5) * (sigma - 0.5), hi = (sigma + 0.5) * (sigma + 0.5);
    nshell = 0;
    for (int c = -R_; c <= R_; ++c)
        for (int b = -R_; b <= R_; ++b)
            for (int a = -R_; a <= R_; ++a) {
                double r2 = double(a * a + b * b + c * c);
                if (r2 >= lo && r2 < hi) ++nshell;
            }
    for (int c = -R_; c <= R_; ++c)
        for (int b = 0; b <= R_; ++b)
            for (int a = 0; a <= R_; ++a) {
                double r2 = double(a * a + b * b + c * c);
                if (!(r2 >= lo && r2 < hi)) continue;
                double len = std::sqrt(r2);
                double ax = a / len, ay = b / len, az = c / len;
                double w = (a > 0 ? 1.0 : 0.5) * (b > 0 ? 1.0 : 0.5);
                Quad<R> q;
                q.a = a;
                q.b = b;
                q.c = c;
                q.hidx = (a & 1) | ((b & 1) << 1) | ((c & 1) << 2);
                q.px = R(w * ax);
                q.py = R(w * ay);
                q.pz = R(w * az);
                q.qxx = R(w * ax * ax);
                q.qyy = R(w * ay * ay);
                q.qzz = R(w * az * az);
                q.qxy = R(w * ax * ay);
                q.qxz = R(w * ax * az);
                q.qyz = R(w * ay * az);
                q.pad0 = q.pad1 = q.pad2 = R(0);
                v.push_back(q);
            }
    return v;
}

template <typename R>
wdlb_status upload_tables(wdlb_ctx *c)
{
    if (!c->prm.nonlocal) {
        c->nq = 0;
        c->nball = 0;
        return WDLB_OK;
    }
    int nshell = 0;
    auto q = build_quads<R>(c->prm.sigma, nshell);
    auto b = build_ball(c->prm.sigma);
    if ((int)q.size() > MAX_QUADS || (int)b.size() > MAX_BALL) return fail(c, WDLB_E_INVAL, "stencil too large");
    HIPCHK(c, hipMemcpyAsync(c->quads, q.data(), q.size() * sizeof(Quad<R>), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ball, b.data(), b.size() * sizeof(int4), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->nq = (int)q.size();
    c->nball = (int)b.size();
    c->wS = 4.0 * M_PI / nshell;
    c->g.tiny = 0;
    int reach = (int)std::ceil(c->prm.sigma + 0.5) + 1;
    if (c->g.nx <= reach || c->g.ny <= reach || (!c->g.walls && c->g.nz <= reach)) c->g.tiny = 1;
    return WDLB_OK;
}

wdlb_status tables(wdlb_ctx *c)
{
    if (c->prec == WDLB_FP64) return upload_tables<double>(c);
    return upload_tables<float>(c);
}

inline dim3 grid1(long long N, int bs) { return dim3((unsigned)((N + bs - 1) / bs)); }

enum { K_MOMENTS = 0, K_BALL, K_GAMMA, K_MEANFIELD, K_COLLIDE };
const char *const KNAMES[WDLB_NKERNELS] = {"k_moments", "k_ball", "k_gamma", "k_meanfield", "k_collide"};

hipEvent_t take_event(wdlb_ctx *c)
{
    if (c->ev_free.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
}

wdlb_status prof_flush(wdlb_ctx *c)
{
    if (c->pending.empty()) return WDLB_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof_ms[p.k] += ms;
            c->prof_n[p.k] += 1;
        }
        c->ev_free.push_back(p.a);
        c->ev_free.push_back(p.b);
    }
    c->pending.clear();
    return WDLB_OK;
}

// launch through this wrapper so that profiling can bracket the kernel
template <typename L>
wdlb_status launch(wdlb_ctx *c, int k, L &&fn)
{
    if (!c->prof) {
        fn();
        return WDLB_OK;
    }
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return fail(c, WDLB_E_HIP, "hipEventCreate failed");
    HIPCHK(c, hipEventRecord(a, c->stream));
    fn();
    HIPCHK(c, hipEventRecord(b, c->stream));
    c->pending.push_back({k, a, b});
    if (c->pending.size() >= 4096) return prof_flush(c);
    return WDLB_OK;
}

// one pass of fields (and collision unless READ) on the current buffers
template <typename R, typename HS, bool READ>
wdlb_status run_pass(wdlb_ctx *c)
{
    const Geom g = c->g;
    const int bs = 256;
    dim3 grid = grid1(g.N, bs);
    const int cur = c->cur, nxt = cur ^ 1;
    auto *ru_in = (const V4<R> *)c->ru[cur];
    auto *h_in = (const HS *)c->h[cur];
    const wdlb_params &p = c->prm;
    const double s = p.sigma;
    wdlb_status st;
    st = launch(c, K_MOMENTS, [&] {
        hipLaunchKernelGGL((k_moments<R, HS>), grid, dim3(bs), 0, c->stream, g, ru_in, h_in, (R *)c->rho,
                           (R *)c->jx, (R *)c->jy, (R *)c->jz, c->flag);
    });
    if (st != WDLB_OK) return st;
    if (p.nonlocal) {
        st = launch(c, K_BALL, [&] {
            hipLaunchKernelGGL((k_ball<R>), grid, dim3(bs), 0, c->stream, g, (const R *)c->rho,
                               (const int4 *)c->ball, c->nball, R(1.0 / c->nball), (R *)c->nbar);
        });
        if (st != WDLB_OK) return st;
        st = launch(c, K_GAMMA, [&] {
            hipLaunchKernelGGL((k_gamma<R>), grid, dim3(bs), 0, c->stream, g, (const R *)c->nbar,
                               R(M_PI * s * s * s / 6.0), R(c->wS), (R *)c->gam, c->flag);
        });
        if (st != WDLB_OK) return st;
    }
    st = launch(c, K_MEANFIELD, [&] {
        hipLaunchKernelGGL((k_meanfield<R>), grid, dim3(bs), 0, c->stream, g, (const R *)c->rho, (const R *)c->jx,
                           (const R *)c->jy, (const R *)c->jz, (const R *)c->gam, (const Quad<R> *)c->quads, c->nq,
                           R(-KT * s * s), R(p.g[0]), R(p.g[1]), R(p.g[2]), (V4<R> *)c->ru1, (V4<R> *)c->fmf);
    });
    if (st != WDLB_OK) return st;
    st = launch(c, K_COLLIDE, [&] {
        hipLaunchKernelGGL((k_collide<R, HS, READ>), grid, dim3(bs), 0, c->stream, g, (const V4<R> *)c->ru1,
                           (const V4<R> *)c->fmf, (const R *)c->gam, (const Quad<R> *)c->quads, c->nq,
                           R(2.0 * s * s * std::sqrt(KT / M_PI)), R(-(KT / 5.0) * s * s), R(1.0 / p.tau),
                           R(1.0 - 0.5 / p.tau), R(p.g[0]), R(p.g[1]), R(p.g[2]), p.smdb, ru_in, h_in,
                           (V4<R> *)c->ru[nxt], (HS *)c->h[nxt], (R *)c->u_rd, (R *)c->F_rd, (R *)c->A_rd);
    });
    if (st != WDLB_OK) return st;
    HIPCHK(c, hipGetLastError());
    return WDLB_OK;
}

template <bool READ>
wdlb_status pass(wdlb_ctx *c)
{
    switch (c->prec) {
    case WDLB_FP64: return run_pass<double, double, READ>(c);
    case WDLB_FP32: return run_pass<float, float, READ>(c);
    default: return run_pass<float, bf16, READ>(c);
    }
}

wdlb_status check_flag(wdlb_ctx *c)
{
    int f = 0;
    HIPCHK(c, hipMemcpyAsync(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (f & FLAG_RHO) return fail(c, WDLB_E_UNSTABLE, "non-finite or non-positive density");
    if (f & FLAG_ETA) return fail(c, WDLB_E_UNSTABLE, "midpoint packing fraction reached 1");
    return WDLB_OK;
}

template <typename R>
void to_double(const std::vector<R> &src, double *dst, size_t n)
{
    for (size_t i = 0; i < n; ++i) dst[i] = (double)src[i];
}

template <typename R>
wdlb_status copy_out(wdlb_ctx *c, const void *dev, size_t n, double *host)
{
    if (!host) return WDLB_OK;
    std::vector<R> tmp(n);
    HIPCHK(c, hipMemcpyAsync(tmp.data(), dev, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    to_double(tmp, host, n);
    return WDLB_OK;
}

wdlb_status copy_out_r(wdlb_ctx *c, const void *dev, size_t n, double *host)
{
    return c->prec == WDLB_FP64 ? copy_out<double>(c, dev, n, host) : copy_out<float>(c, dev, n, host);
}

wdlb_status read_pass(wdlb_ctx *c)
{
    if (!c->inited) return fail(c, WDLB_E_STATE, "context not initialised");
    bool prof = c->prof;
    c->prof = false;  // only the stepping kernels are timed
    wdlb_status st = pass<true>(c);
    c->prof = prof;
    if (st != WDLB_OK) return st;
    return check_flag(c);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

wdlb_status wdlb_workspace_size(const wdlb_lattice_desc *desc, const wdlb_params *params, size_t *bytes)
{
    if (!desc_ok(desc) || !params_ok(params) || !bytes) return WDLB_E_INVAL;
    *bytes = layout(desc).total;
    return WDLB_OK;
}

wdlb_status wdlb_create(const wdlb_lattice_desc *desc, const wdlb_params *params, void *d_workspace, size_t bytes,
                        wdlb_ctx **out)
{
    if (!out) return WDLB_E_INVAL;
    *out = nullptr;
    if (!desc_ok(desc) || !params_ok(params) || !d_workspace) return WDLB_E_INVAL;
    if (((uintptr_t)d_workspace & 255) != 0) return WDLB_E_INVAL;
    Layout L = layout(desc);
    if (bytes < L.total) return WDLB_E_NOMEM;
    wdlb_ctx *c = new (std::nothrow) wdlb_ctx();
    if (!c) return WDLB_E_NOMEM;
    c->desc = *desc;
    c->prm = *params;
    c->stream = (hipStream_t)desc->stream;
    c->prec = desc->precision;
    c->rsize = c->prec == WDLB_FP64 ? 8 : 4;
    c->hsize = c->prec == WDLB_FP64 ? 8 : (c->prec == WDLB_BF16_NEQ ? 2 : 4);
    c->g.nx = desc->nx;
    c->g.ny = desc->ny;
    c->g.nz = desc->nz;
    c->g.walls = desc->walls_z ? 1 : 0;
    c->g.N = (long long)desc->nx * desc->ny * desc->nz;
    c->g.tiny = 0;
    c->ws = (char *)d_workspace;
    c->ws_bytes = bytes;
    for (int b = 0; b < 2; ++b) {
        c->ru[b] = c->ws + L.off_ru[b];
        c->h[b] = c->ws + L.off_h[b];
    }
    c->rho = c->ws + L.off_rho;
    c->jx = c->ws + L.off_j[0];
    c->jy = c->ws + L.off_j[1];
    c->jz = c->ws + L.off_j[2];
    c->nbar = c->ws + L.off_nbar;
    c->gam = c->ws + L.off_gam;
    c->ru1 = c->ws + L.off_ru1;
    c->fmf = c->ws + L.off_fmf;
    c->u_rd = c->ws + L.off_urd;
    c->F_rd = c->ws + L.off_Frd;
    c->A_rd = c->ws + L.off_Ard;
    c->planes = (double *)(c->ws + L.off_planes);
    c->flag = (int *)(c->ws + L.off_flag);
    c->quads = c->ws + L.off_quads;
    c->ball = (int4 *)(c->ws + L.off_ball);
    c->cur = 0;
    c->step = 0;
    c->inited = false;
    wdlb_status st = tables(c);
    if (st != WDLB_OK) {
        delete c;
        return st;
    }
    *out = c;
    return WDLB_OK;
}

wdlb_status wdlb_set_params(wdlb_ctx *c, const wdlb_params *params)
{
    if (!c) return WDLB_E_INVAL;
    if (!params_ok(params)) return fail(c, WDLB_E_INVAL, "invalid parameters");
    c->prm = *params;
    return tables(c);
}

static wdlb_status do_init(wdlb_ctx *c, int uniform, const double u0[3], const double *h_n, const double *h_u)
{
    const Geom g = c->g;
    const size_t N = (size_t)g.N;
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    double n0 = 6.0 * c->prm.eta / (M_PI * c->prm.sigma * c->prm.sigma * c->prm.sigma);
    c->cur = 0;
    if (!uniform) {
        if (c->prec == WDLB_FP64) {
            std::vector<V4<double>> v(N);
            for (size_t i = 0; i < N; ++i) v[i] = V4<double>{h_n[i], h_u[i], h_u[N + i], h_u[2 * N + i]};
            HIPCHK(c, hipMemcpyAsync(c->ru[0], v.data(), N * sizeof(V4<double>), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        } else {
            std::vector<V4<float>> v(N);
            for (size_t i = 0; i < N; ++i)
                v[i] = V4<float>{(float)h_n[i], (float)h_u[i], (float)h_u[N + i], (float)h_u[2 * N + i]};
            HIPCHK(c, hipMemcpyAsync(c->ru[0], v.data(), N * sizeof(V4<float>), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    dim3 grid = grid1(g.N, 256);
    double ux = u0 ? u0[0] : 0, uy = u0 ? u0[1] : 0, uz = u0 ? u0[2] : 0;
    switch (c->prec) {
    case WDLB_FP64:
        if (uniform)
            hipLaunchKernelGGL((k_fill<double>), grid, dim3(256), 0, c->stream, g, (V4<double> *)c->ru[0], n0, ux,
                               uy, uz);
        hipLaunchKernelGGL((k_init<double, double>), grid, dim3(256), 0, c->stream, g,
                           (const V4<double> *)c->ru[0], (double *)c->h[0]);
        break;
    case WDLB_FP32:
        if (uniform)
            hipLaunchKernelGGL((k_fill<float>), grid, dim3(256), 0, c->stream, g, (V4<float> *)c->ru[0],
                               (float)n0, (float)ux, (float)uy, (float)uz);
        hipLaunchKernelGGL((k_init<float, float>), grid, dim3(256), 0, c->stream, g, (const V4<float> *)c->ru[0],
                           (float *)c->h[0]);
        break;
    default:
        if (uniform)
            hipLaunchKernelGGL((k_fill<float>), grid, dim3(256), 0, c->stream, g, (V4<float> *)c->ru[0],
                               (float)n0, (float)ux, (float)uy, (float)uz);
        hipLaunchKernelGGL((k_init<float, bf16>), grid, dim3(256), 0, c->stream, g, (const V4<float> *)c->ru[0],
                           (bf16 *)c->h[0]);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->step = 0;
    c->inited = true;
    return WDLB_OK;
}

wdlb_status wdlb_init_uniform(wdlb_ctx *c, const double u0[3])
{
    if (!c) return WDLB_E_INVAL;
    return do_init(c, 1, u0, nullptr, nullptr);
}

wdlb_status wdlb_init_fields(wdlb_ctx *c, const double *h_n, const double *h_u)
{
    if (!c) return WDLB_E_INVAL;
    if (!h_n || !h_u) return fail(c, WDLB_E_INVAL, "null field");
    return do_init(c, 0, nullptr, h_n, h_u);
}

wdlb_status wdlb_step(wdlb_ctx *c, int64_t nsteps)
{
    if (!c) return WDLB_E_INVAL;
    if (nsteps < 0) return fail(c, WDLB_E_INVAL, "negative step count");
    if (!c->inited) return fail(c, WDLB_E_STATE, "context not initialised");
    for (int64_t t = 0; t < nsteps; ++t) {
        wdlb_status st = pass<false>(c);
        if (st != WDLB_OK) return st;
        c->cur ^= 1;
        c->step++;
    }
    return WDLB_OK;
}

wdlb_status wdlb_sync(wdlb_ctx *c)
{
    if (!c) return WDLB_E_INVAL;
    return check_flag(c);
}

wdlb_status wdlb_read_fields_ex(wdlb_ctx *c, double *h_n, double *h_u, double *h_F, double *h_A0)
{
    if (!c) return WDLB_E_INVAL;
    wdlb_status st = read_pass(c);
    if (st != WDLB_OK) return st;
    const size_t N = (size_t)c->g.N;
    if ((st = copy_out_r(c, c->rho, N, h_n)) != WDLB_OK) return st;
    if ((st = copy_out_r(c, c->u_rd, 3 * N, h_u)) != WDLB_OK) return st;
    if ((st = copy_out_r(c, c->F_rd, 3 * N, h_F)) != WDLB_OK) return st;
    if (h_A0) {
        std::vector<double> a6(6 * N);
        if ((st = copy_out_r(c, c->A_rd, 6 * N, a6.data())) != WDLB_OK) return st;
        // stored order xx, yy, zz, xy, xz, yz -> row-major 3x3
        const int map[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
        for (int k = 0; k < 9; ++k)
            for (size_t i = 0; i < N; ++i) h_A0[k * N + i] = a6[map[k] * N + i];
    }
    return WDLB_OK;
}

wdlb_status wdlb_read_fields(wdlb_ctx *c, double *h_n, double *h_u)
{
    return wdlb_read_fields_ex(c, h_n, h_u, nullptr, nullptr);
}

static wdlb_status planes(wdlb_ctx *c, std::vector<double> &out)
{
    wdlb_status st = read_pass(c);
    if (st != WDLB_OK) return st;
    const Geom g = c->g;
    if (c->prec == WDLB_FP64)
        hipLaunchKernelGGL((k_planes<double>), dim3(g.nz), dim3(256), 0, c->stream, g, (const double *)c->rho,
                           (const double *)c->u_rd, c->planes);
    else
        hipLaunchKernelGGL((k_planes<float>), dim3(g.nz), dim3(256), 0, c->stream, g, (const float *)c->rho,
                           (const float *)c->u_rd, c->planes);
    HIPCHK(c, hipGetLastError());
    out.assign(3 * g.nz, 0.0);
    HIPCHK(c, hipMemcpyAsync(out.data(), c->planes, out.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return WDLB_OK;
}

wdlb_status wdlb_read_profiles(wdlb_ctx *c, double *h_n_z, double *h_ux_z)
{
    if (!c) return WDLB_E_INVAL;
    std::vector<double> p;
    wdlb_status st = planes(c, p);
    if (st != WDLB_OK) return st;
    const int nz = c->g.nz;
    const double plane = (double)c->g.nx * c->g.ny;
    for (int z = 0; z < nz; ++z) {
        if (h_n_z) h_n_z[z] = p[z] / plane;
        if (h_ux_z) h_ux_z[z] = p[nz + z] / plane;
    }
    return WDLB_OK;
}

wdlb_status wdlb_read_flux(wdlb_ctx *c, double *j_pore, double *u_pore, double *mass)
{
    if (!c) return WDLB_E_INVAL;
    std::vector<double> p;
    wdlb_status st = planes(c, p);
    if (st != WDLB_OK) return st;
    const int nz = c->g.nz;
    const double plane = (double)c->g.nx * c->g.ny;
    double M = 0, U = 0, J = 0;
    for (int z = 0; z < nz; ++z) {
        M += p[z];
        U += p[nz + z] / plane;
        J += p[2 * nz + z];
    }
    if (j_pore) *j_pore = J / (double)c->g.N;
    if (u_pore) *u_pore = U / nz;
    if (mass) *mass = M;
    return WDLB_OK;
}

wdlb_status wdlb_read_populations(wdlb_ctx *c, double *h_f)
{
    if (!c || !h_f) return WDLB_E_INVAL;
    if (!c->inited) return fail(c, WDLB_E_STATE, "context not initialised");
    const Geom g = c->g;
    dim3 grid = grid1(g.N, 256);
    const int cur = c->cur;
    // the per-step scratch arrays (gamma .. A_rd, >= 28 N reals, contiguous)
    // are free between steps and hold the 19 N reconstructed populations
    void *scratch = c->gam;
    switch (c->prec) {
    case WDLB_FP64:
        hipLaunchKernelGGL((k_populations<double, double>), grid, dim3(256), 0, c->stream, g,
                           (const V4<double> *)c->ru[cur], (const double *)c->h[cur], (double *)scratch);
        break;
    case WDLB_FP32:
        hipLaunchKernelGGL((k_populations<float, float>), grid, dim3(256), 0, c->stream, g,
                           (const V4<float> *)c->ru[cur], (const float *)c->h[cur], (float *)scratch);
        break;
    default:
        hipLaunchKernelGGL((k_populations<float, bf16>), grid, dim3(256), 0, c->stream, g,
                           (const V4<float> *)c->ru[cur], (const bf16 *)c->h[cur], (float *)scratch);
    }
    HIPCHK(c, hipGetLastError());
    return copy_out_r(c, scratch, 19 * (size_t)g.N, h_f);
}

namespace {
struct StateHeader {
    char magic[8];
    int32_t nx, ny, nz, walls, precision, pad;
    int64_t step;
};
size_t state_bytes(const wdlb_ctx *c)
{
    const size_t N = (size_t)c->g.N;
    return sizeof(StateHeader) + 4 * c->rsize * N + 19 * c->hsize * N;
}
}  // namespace

wdlb_status wdlb_state_size(const wdlb_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return WDLB_E_INVAL;
    *bytes = state_bytes(c);
    return WDLB_OK;
}

wdlb_status wdlb_save_state(wdlb_ctx *c, void *h_buf, size_t bytes)
{
    if (!c || !h_buf) return WDLB_E_INVAL;
    if (!c->inited) return fail(c, WDLB_E_STATE, "context not initialised");
    if (bytes < state_bytes(c)) return fail(c, WDLB_E_INVAL, "state buffer too small");
    StateHeader hd;
    memcpy(hd.magic, "WDLBST01", 8);
    hd.nx = c->g.nx;
    hd.ny = c->g.ny;
    hd.nz = c->g.nz;
    hd.walls = c->g.walls;
    hd.precision = c->prec;
    hd.pad = 0;
    hd.step = c->step;
    char *p = (char *)h_buf;
    memcpy(p, &hd, sizeof(hd));
    const size_t N = (size_t)c->g.N;
    HIPCHK(c, hipMemcpyAsync(p + sizeof(hd), c->ru[c->cur], 4 * c->rsize * N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(p + sizeof(hd) + 4 * c->rsize * N, c->h[c->cur], 19 * c->hsize * N,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return WDLB_OK;
}

wdlb_status wdlb_load_state(wdlb_ctx *c, const void *h_buf, size_t bytes)
{
    if (!c || !h_buf) return WDLB_E_INVAL;
    if (bytes < state_bytes(c)) return fail(c, WDLB_E_STATE, "state buffer too small");
    StateHeader hd;
    memcpy(&hd, h_buf, sizeof(hd));
    if (memcmp(hd.magic, "WDLBST01", 8) != 0 || hd.nx != c->g.nx || hd.ny != c->g.ny || hd.nz != c->g.nz ||
        hd.walls != c->g.walls || hd.precision != c->prec)
        return fail(c, WDLB_E_STATE, "state does not match this context");
    const char *p = (const char *)h_buf;
    const size_t N = (size_t)c->g.N;
    c->cur = 0;
    HIPCHK(c, hipMemcpyAsync(c->ru[0], p + sizeof(hd), 4 * c->rsize * N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h[0], p + sizeof(hd) + 4 * c->rsize * N, 19 * c->hsize * N, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->step = hd.step;
    c->inited = true;
    return WDLB_OK;
}

wdlb_status wdlb_get_step(const wdlb_ctx *c, int64_t *step)
{
    if (!c || !step) return WDLB_E_INVAL;
    *step = c->step;
    return WDLB_OK;
}

wdlb_status wdlb_profile(wdlb_ctx *c, int32_t enable)
{
    if (!c) return WDLB_E_INVAL;
    wdlb_status st = prof_flush(c);
    if (st != WDLB_OK) return st;
    if (enable)
        for (int k = 0; k < WDLB_NKERNELS; ++k) {
            c->prof_ms[k] = 0;
            c->prof_n[k] = 0;
        }
    c->prof = enable != 0;
    return WDLB_OK;
}

wdlb_status wdlb_profile_read(wdlb_ctx *c, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!c || kernel < 0 || kernel >= WDLB_NKERNELS) return WDLB_E_INVAL;
    wdlb_status st = prof_flush(c);
    if (st != WDLB_OK) return st;
    if (total_ms) *total_ms = c->prof_ms[kernel];
    if (launches) *launches = c->prof_n[kernel];
    return WDLB_OK;
}

const char *wdlb_kernel_name(int32_t kernel) { return (kernel >= 0 && kernel < WDLB_NKERNELS) ? KNAMES[kernel] : ""; }

const char *wdlb_last_error(const wdlb_ctx *c) { return c ? c->err.c_str() : "null context"; }

void wdlb_destroy(wdlb_ctx *c)
{
    if (!c) return;
    prof_flush(c);
    for (auto e : c->ev_free) hipEventDestroy(e);
    delete c;
}

}  // extern "C"
