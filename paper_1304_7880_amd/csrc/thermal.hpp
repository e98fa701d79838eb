// thermal.hpp -- contact-shell sums of the thermal fields of Sec. 3 at given
// density, velocity and temperature.  Device code only; included by
// wdlb.hip after kernels.hpp.
//
// With k = e/|e|, dT = T(r+e) - T(r), dv = u(r+e) - u(r) and the shell weight
// G = w_S gamma_mid rho(r+e) of the step's contact-shell sums (k_B = m = 1):
//   Q(r)     = n(r) sigma^2 sum_e G [ -T(r) (k.dv)/2 + sqrt(T(r)/pi) dT ]   (eq. campob1)
//   B_i(r)   = -2 T(r) n(r) sigma^2 sum_e k_i G dT                         (eq. campos)
//   F^T_i(r) = -(sigma^2/2) sum_e k_i G dT                                 (eq. thermalforce)
// The factor k_B T of eq. campob1 cancels the 1/T of its temperature term.
// The isothermal step never needs these fields (B, Q and F^T vanish at
// uniform T); they are evaluated on request, between steps, in the per-step
// padded arrays: (rho, u) in the (rho, u1) array, T in the density array,
// and the contact values from the density kernel.
#pragma once

namespace wdlb {

// a field given at the nodes into a padded array, with its periodic images
template <typename R>
__global__ __launch_bounds__(256) void k_pad(Geom g, Pad p, const R *__restrict__ src, R *__restrict__ dst)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const R v = src[i];
    for_images(g, p, x, y, z, [&](int k) { dst[k] = v; });
}

// (rho, u) from n[N] and u[3N] (component-major) into the padded V4 array
template <typename R>
__global__ __launch_bounds__(256) void k_pad_ru(Geom g, Pad p, const R *__restrict__ n, const R *__restrict__ u,
                                                V4<R> *__restrict__ dst)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const V4<R> v = {n[i], u[i], u[g.N + i], u[2 * g.N + i]};
    for_images(g, p, x, y, z, [&](int k) { dst[k] = v; });
}

// One lane per node on 32 x 8 tiles of a plane; the shell from the quad
// table (mirror groups (+-a, +-b, c)), the images' rho, u, T and contact
// values read through the caches.  Per group: the four image terms
// D_m = G_m dT_m and V_m = G_m dv_m (products unfused, as in the step's
// shell sums), their Hadamard transform over the mirror signs, and one FMA
// per weight.  A state that does not depend on x (or y) gives exactly zero
// x (y) components.  The contact values of the density kernel carry the
// shell weight w_S; s2 = sigma^2.
template <typename R>
__global__ __launch_bounds__(256) void k_thermal(Geom g, Pad p, const V4<R> *__restrict__ ru_p,
                                                 const R *__restrict__ T_p, const R *__restrict__ gam_p,
                                                 const Quad<R> *__restrict__ quads, int nq, R s2, int tiles_x,
                                                 int tiles_y, R *__restrict__ Qo, R *__restrict__ Bo,
                                                 R *__restrict__ FTo)
{
    const TileCoord tc = tile_coord<32, 8, 1>(tiles_x, tiles_y, g.nz);
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0;
    if (x >= g.nx || y >= g.ny) return;
    const int gbase = pidx(p, x, y, z);
    const V4<R> c0 = ru_p[gbase];
    const R T0 = T_p[gbase];
    R ax = 0, ay = 0, az = 0, aT = 0, aV = 0;
    for (int q = 0; q < nq; ++q) {
        const Quad<R> Qd = quads[q];
        int so[4], mo[4];
        quad_offsets(Qd.a, Qd.b, Qd.c, p.PX, p.PXY, so, mo);
        const R *gb = gam_p + (long long)Qd.hidx * p.NP + gbase;
        // the plain weight of the group: 1, 1/2 or 1/4 for a or b zero (its
        // images repeat); px, py, pz carry it times k
        const R w = R(Qd.a > 0 ? 1.0 : 0.5) * R(Qd.b > 0 ? 1.0 : 0.5);
        R hx, hy, h0, vx, vy, vz;
        {
#pragma clang fp contract(off)
            R D[4], Vx[4], Vy[4], Vz[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const V4<R> s = ru_p[gbase + so[m]];
                const R G = gb[mo[m]] * s.x;
                D[m] = G * (T_p[gbase + so[m]] - T0);
                Vx[m] = G * (s.y - c0.y);
                Vy[m] = G * (s.z - c0.z);
                Vz[m] = G * (s.w - c0.w);
            }
            const R P1 = D[0] + D[1], M1 = D[0] - D[1], P2 = D[2] + D[3], M2 = D[2] - D[3];
            hx = M1 + M2;
            hy = P1 - P2;
            h0 = P1 + P2;
            vx = (Vx[0] - Vx[1]) + (Vx[2] - Vx[3]);
            vy = (Vy[0] + Vy[1]) - (Vy[2] + Vy[3]);
            vz = (Vz[0] + Vz[1]) + (Vz[2] + Vz[3]);
        }
        ax += Qd.px * hx;
        ay += Qd.py * hy;
        az += Qd.pz * h0;
        aT += w * h0;
        aV += Qd.px * vx;
        aV += Qd.py * vy;
        aV += Qd.pz * vz;
    }
    const long long N = g.N;
    const int i = (z * g.ny + y) * g.nx + x;
    const R n0 = c0.x, kq = n0 * s2, kb = R(-2) * T0 * n0 * s2, kf = R(-0.5) * s2;
    Qo[i] = kq * (R(-0.5) * T0 * aV + sqrt(T0 / R(M_PI)) * aT);
    Bo[i] = kb * ax;
    Bo[N + i] = kb * ay;
    Bo[2 * N + i] = kb * az;
    FTo[i] = kf * ax;
    FTo[N + i] = kf * ay;
    FTo[2 * N + i] = kf * az;
}

}  // namespace wdlb
