// thermal_flow.hpp -- the kernels that the coupled thermal flow adds to the
// isothermal step (a hybrid reading: the paper's lattice scheme is
// isothermal).  Device code only; included by wdlb.hip after thermal.hpp.
// R is the storage real (FP64 or FP32); the viscous force is recovered from
// the step's total force, to the rounding of that total.
//
// With theta = T / kT at every node: the mean-field force carries theta,
// the viscous force sqrt(theta), A theta (Sec. 3: F^mf ~ k_B T,
// F^v ~ sqrt(k_B T), A_ij ~ k_B T), the thermal force F^T is added (and u1
// of the viscous and thermal sums carries it with the other forces), the
// populations relax towards the equilibrium with its temperature term
// w_a rho (3/2)(theta - 1)(|c_a|^2 - 1), and T follows the energy balance
// with flow (Sec. 2 eq. energyequation; the heat flux of eq. qexplicit, the
// pressure tensor of eqs. pexplicit and extrapressure), with its kinetic
// conduction sub-cycled.
#pragma once

namespace wdlb {

constexpr int FLAG_T = 4;  // a non-positive or non-finite temperature

template <typename D>
__device__ __forceinline__ D theta_term(int a, D rho, D theta)
{
    const D c2 = D(CX[a] * CX[a] + CY[a] * CY[a] + CZ[a] * CZ[a]);
    return wgt<D>(a) * rho * D(1.5) * (theta - D(1)) * (c2 - D(1));
}

// the temperature term added to the stored populations: after the next pull
// node t holds feq(n(t), u(t)) plus the term at n(t), theta(t); a direction
// that bounces back at a wall returns to the node itself
template <typename R>
__global__ __launch_bounds__(256) void k_th_init(Geom g, const V4<R> *__restrict__ ru, const R *__restrict__ T, double kT,
                                                 R *__restrict__ h)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        int tz = z + CZ[a];
        bool bb = false;
        if (CZ[a] != 0) {
            if (g.walls) bb = !zfluid(g, tz);
            else tz = wrap1(tz, g.nz);
        }
        long long t = i;
        if (!bb) {
            const int tx = CX[a] ? wrap1(x + CX[a], g.nx) : x;
            const int ty = CY[a] ? wrap1(y + CY[a], g.ny) : y;
            t = ((long long)tz * g.ny + ty) * g.nx + tx;
        }
        // once per run: FP64 arithmetic, one rounding to the storage
        h[a * g.N + i] = R(double(h[a * g.N + i]) + theta_term<double>(a, double(ru[t].x), double(T[t]) / kT));
    }
}

// after the mean-field kernel and the thermal kernel at u = 0: F^mf <- theta F^mf and
// u1 = j/rho + (g + theta F^mf + F^T)/2 (every force known before the
// viscous sums) into the padded (rho, u1) array with its images; a
// temperature that is not positive and finite raises FLAG_T
template <typename R>
__global__ __launch_bounds__(256) void k_th_u1(Geom g, Pad p, const R *__restrict__ T, R kT, const R *__restrict__ jx,
                                               const R *__restrict__ jy, const R *__restrict__ jz,
                                               const R *__restrict__ FT, R gx, R gy, R gz, V4<R> *__restrict__ fmf,
                                               V4<R> *__restrict__ ru1_p, int *flag)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const R Ti = T[i];
    if (!(Ti > R(0)) || !(Ti < R(INFINITY))) raise_flag(flag, FLAG_T);
    const R th = Ti / kT, rr = ru1_p[pidx(p, x, y, z)].x;
    V4<R> f = fmf[i];
    f.x = th * f.x;
    f.y = th * f.y;
    f.z = th * f.z;
    fmf[i] = f;
    const long long N = g.N;
    const V4<R> v = {rr, jx[i] / rr + R(0.5) * (gx + f.x + FT[i]), jy[i] / rr + R(0.5) * (gy + f.y + FT[N + i]),
                     jz[i] / rr + R(0.5) * (gz + f.z + FT[2 * N + i])};
    for_images(g, p, x, y, z, [&](int k) { ru1_p[k] = v; });
}

// after the viscous/SMDB kernel (whose F holds rho (g + theta F^mf + F^v(kT))
// and whose trace sums S = sum_e k.W are in S):
// F = rho (g + theta F^mf + sqrt(theta) F^v(kT) + F^T), A <- theta A, and Q
// (its conduction part from the thermal kernel at u = 0) gains its
// compression part -(n sigma^2 T / 2) S (eq. campob1)
template <typename R>
__global__ __launch_bounds__(256) void k_th_force(Geom g, Pad p, const V4<R> *__restrict__ ru1_p,
                                                  const R *__restrict__ T, R kT, const V4<R> *__restrict__ fmf,
                                                  const R *__restrict__ FT, const R *__restrict__ S, R s2, R gx, R gy,
                                                  R gz, R *__restrict__ F, R *__restrict__ A, R *__restrict__ Q)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const long long N = g.N;
    const R r = ru1_p[pidx(p, x, y, z)].x, Ti = T[i], th = Ti / kT, sq = sqrt(th);
    const V4<R> fm = fmf[i];
    const R gg[3] = {gx, gy, gz}, fmc[3] = {fm.x, fm.y, fm.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const R fv = F[d * N + i] / r - gg[d] - fmc[d];
        F[d * N + i] = r * (gg[d] + fmc[d] + sq * fv + FT[d * N + i]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) A[k * N + i] = th * A[k * N + i];
    Q[i] += r * s2 * (R(-0.5) * Ti * S[i]);
}

// velocity u = (j + F/2)/rho of node (x, y, z) (unpadded index q, padded density)
template <typename R>
__device__ __forceinline__ void th_vel(const Geom &g, const Pad &p, const V4<R> *__restrict__ ru1_p,
                                       const R *__restrict__ jx, const R *__restrict__ jy, const R *__restrict__ jz,
                                       const R *__restrict__ F, int x, int y, int z, R (&u)[3])
{
    const long long q = ((long long)z * g.ny + y) * g.nx + x, N = g.N;
    const R r = ru1_p[pidx(p, x, y, z)].x;
    u[0] = (jx[q] + R(0.5) * F[q]) / r;
    u[1] = (jy[q] + R(0.5) * F[N + q]) / r;
    u[2] = (jz[q] + R(0.5) * F[2 * N + q]) / r;
}

// The two energy kernels march along z: a thread owns the column (x, y) of a
// 64 x 4 tile over zc planes (blockIdx.z: the chunk of planes), carrying
// the fields of the planes z - 1, z, z + 1 of its own column in registers,
// so that each plane of an array is read from memory about once; the x and
// y neighbours come from the same plane, through the caches.
__host__ __device__ constexpr int ENERGY_TX = 64, ENERGY_TY = 4;

// the column's plane zz, or false beyond a wall (periodic: wrapped)
__device__ __forceinline__ bool energy_plane(const Geom &g, int zz, int &zw)
{
    if (g.walls) {
        zw = zz;
        return zz >= 0 && zz < g.nz;
    }
    zw = zz < 0 ? zz + g.nz : (zz >= g.nz ? zz - g.nz : zz);
    return true;
}

// the part of dT/dt held fixed over the step's sub-steps:
//   -u.grad T + (2/(3n)) (-div delta q - P:grad u + Q)
// central differences (beyond a wall u is mirrored to -u, T to T), delta q =
// B/(2 omega0) through the faces (none through a wall); P of eqs. pexplicit
// and extrapressure with the step's A (stored xx, yy, zz, xy, xz, yz)
template <typename R>
__global__ __launch_bounds__(256) void k_energy_fixed(Geom g, Pad p, int zc, const V4<R> *__restrict__ ru1_p,
                                                      const R *__restrict__ T_p, const R *__restrict__ jx,
                                                      const R *__restrict__ jy, const R *__restrict__ jz,
                                                      const R *__restrict__ F, const R *__restrict__ A,
                                                      const R *__restrict__ Q, const R *__restrict__ B, R omega0,
                                                      R *__restrict__ Rfix)
{
    const int x = blockIdx.x * ENERGY_TX + (threadIdx.x & (ENERGY_TX - 1));
    const int y = blockIdx.y * ENERGY_TY + (threadIdx.x / ENERGY_TX);
    if (x >= g.nx || y >= g.ny) return;
    const int z0 = blockIdx.z * zc, z1 = min(z0 + zc, g.nz);
    const long long N = g.N;
    const int xp = x + 1 == g.nx ? 0 : x + 1, xm = x == 0 ? g.nx - 1 : x - 1;
    const int yp = y + 1 == g.ny ? 0 : y + 1, ym = y == 0 ? g.ny - 1 : y - 1;
    auto node = [&](int zz) { return ((long long)zz * g.ny + y) * g.nx + x; };
    const R h2w = R(2) * omega0;
    // the column's planes z - 1 (m), z (0), z + 1 (p): u, T, B_z
    R um[3] = {0, 0, 0}, u0[3], up[3] = {0, 0, 0}, Tm = 0, T0, Tp = 0, Bm = 0, B0, Bp = 0;
    int zw;
    bool hm = energy_plane(g, z0 - 1, zw);
    if (hm) {
        th_vel<R>(g, p, ru1_p, jx, jy, jz, F, x, y, zw, um);
        Tm = T_p[pidx(p, x, y, zw)];
        Bm = B[2 * N + node(zw)];
    }
    th_vel<R>(g, p, ru1_p, jx, jy, jz, F, x, y, z0, u0);
    T0 = T_p[pidx(p, x, y, z0)];
    B0 = B[2 * N + node(z0)];
    for (int z = z0; z < z1; ++z) {
        const bool hp = energy_plane(g, z + 1, zw);
        if (hp) {
            th_vel<R>(g, p, ru1_p, jx, jy, jz, F, x, y, zw, up);
            Tp = T_p[pidx(p, x, y, zw)];
            Bp = B[2 * N + node(zw)];
        }
        const long long i = node(z);
        const R n = ru1_p[pidx(p, x, y, z)].x, Tr = T0;
        R gu[3][3], gT[3], divdq = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R vp[3], vm[3], Tpa, Tma, Bpa = 0, Bma = 0;
            bool okp = true, okm = true;
            if (a == 0) {
                th_vel<R>(g, p, ru1_p, jx, jy, jz, F, xp, y, z, vp);
                th_vel<R>(g, p, ru1_p, jx, jy, jz, F, xm, y, z, vm);
                Tpa = T_p[pidx(p, xp, y, z)];
                Tma = T_p[pidx(p, xm, y, z)];
                Bpa = B[((long long)z * g.ny + y) * g.nx + xp];
                Bma = B[((long long)z * g.ny + y) * g.nx + xm];
            } else if (a == 1) {
                th_vel<R>(g, p, ru1_p, jx, jy, jz, F, x, yp, z, vp);
                th_vel<R>(g, p, ru1_p, jx, jy, jz, F, x, ym, z, vm);
                Tpa = T_p[pidx(p, x, yp, z)];
                Tma = T_p[pidx(p, x, ym, z)];
                Bpa = B[N + ((long long)z * g.ny + yp) * g.nx + x];
                Bma = B[N + ((long long)z * g.ny + ym) * g.nx + x];
            } else {
                okp = hp;
                okm = hm;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    vp[b] = okp ? up[b] : -u0[b];
                    vm[b] = okm ? um[b] : -u0[b];
                }
                Tpa = okp ? Tp : Tr;
                Tma = okm ? Tm : Tr;
                Bpa = Bp;
                Bma = Bm;
            }
#pragma unroll
            for (int b = 0; b < 3; ++b) gu[a][b] = R(0.5) * (vp[b] - vm[b]);
            gT[a] = R(0.5) * (Tpa - Tma);
            const R q0 = (a == 2 ? B0 : B[a * N + i]) / h2w;
            const R fp = okp ? R(0.5) * (q0 + Bpa / h2w) : R(0);
            const R fm = okm ? R(0.5) * (Bma / h2w + q0) : R(0);
            divdq += fp - fm;
        }
        // A0 (row-major) from the stored xx, yy, zz, xy, xz, yz
        const R A0[3][3] = {{A[i], A[3 * N + i], A[4 * N + i]},
                            {A[3 * N + i], A[N + i], A[5 * N + i]},
                            {A[4 * N + i], A[5 * N + i], A[2 * N + i]}};
        const R divu = gu[0][0] + gu[1][1] + gu[2][2];
        R work = 0, adv = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            adv += u0[a] * gT[a];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const R P = (a == b ? n * Tr : R(0)) -
                            n * Tr / omega0 * (gu[a][b] + gu[b][a] - (a == b ? R(2) / R(3) * divu : R(0))) +
                            R(2) / omega0 * A0[a][b];
                work += P * gu[a][b];
            }
        }
        Rfix[i] = -adv + R(2) / (R(3) * n) * (-divdq - work + Q[i]);
        // advance the column: plane z becomes z - 1, z + 1 becomes z
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            um[b] = u0[b];
            u0[b] = up[b];
        }
        Tm = T0;
        T0 = Tp;
        Bm = B0;
        B0 = Bp;
        hm = true;
    }
}

// one sub-step: T_out = T + (Rfix + (2/(3n)) (-div q_kin)) / nsub, the
// kinetic flux through the six faces (none through a wall); the column's
// T and n of the planes z - 1, z, z + 1 carried (padded arrays: the plane
// beyond a wall is there, zero, and not used)
template <typename R>
__global__ __launch_bounds__(256) void k_energy_sub(Geom g, Pad p, int zc, const R *__restrict__ T_p,
                                                    const V4<R> *__restrict__ ru1_p, const R *__restrict__ Rfix,
                                                    R omega0, int nsub, R *__restrict__ T_out)
{
    const int x = blockIdx.x * ENERGY_TX + (threadIdx.x & (ENERGY_TX - 1));
    const int y = blockIdx.y * ENERGY_TY + (threadIdx.x / ENERGY_TX);
    if (x >= g.nx || y >= g.ny) return;
    const int z0 = blockIdx.z * zc, z1 = min(z0 + zc, g.nz);
    int gb = pidx(p, x, y, z0);
    R Tm = T_p[gb - p.PXY], nm = ru1_p[gb - p.PXY].x, T0 = T_p[gb], n0 = ru1_p[gb].x;
    const R ck = -R(2.5) / omega0 * R(0.5);
    for (int z = z0; z < z1; ++z, gb += p.PXY) {
        const R Tp = T_p[gb + p.PXY], np_ = ru1_p[gb + p.PXY].x;
        const R n = n0, Tr = T0;
        R div = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R fp = 0, fm = 0;
            const bool okp = !(a == 2 && g.walls && z == g.nz - 1), okm = !(a == 2 && g.walls && z == 0);
            R Tpa, npa, Tma, nma;
            if (a == 2) {
                Tpa = Tp, npa = np_, Tma = Tm, nma = nm;
            } else {
                const int d = a == 0 ? 1 : p.PX;
                Tpa = T_p[gb + d], npa = ru1_p[gb + d].x, Tma = T_p[gb - d], nma = ru1_p[gb - d].x;
            }
            if (okp) fp = ck * (n * Tr + npa * Tpa) * (Tpa - Tr);
            if (okm) fm = ck * (nma * Tma + n * Tr) * (Tr - Tma);
            div += fp - fm;
        }
        const long long i = ((long long)z * g.ny + y) * g.nx + x;
        T_out[i] = Tr + (Rfix[i] + R(2) / (R(3) * n) * (-div)) / R(nsub);
        Tm = T0, nm = n0, T0 = Tp, n0 = np_;
    }
}

// after the collision: the stored post-collision populations gain the
// temperature term relaxed at 1/tau, at the pre-collision rho and theta
// (arithmetic D, one rounding to the storage)
template <typename R, typename D>
__global__ __launch_bounds__(256) void k_th_post(Geom g, Pad p, const V4<R> *__restrict__ ru1_p,
                                                 const R *__restrict__ T, D kT, D inv_tau, R *__restrict__ h)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const D r = ru1_p[pidx(p, x, y, z)].x, th = D(T[i]) / kT;
#pragma unroll
    for (int a = 0; a < Q; ++a) h[a * g.N + i] = R(D(h[a * g.N + i]) + theta_term<D>(a, r, th) * inv_tau);
}

}  // namespace wdlb
