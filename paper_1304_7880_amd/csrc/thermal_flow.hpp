// thermal_flow.hpp -- the kernels that the coupled thermal flow adds to the
// isothermal step (a hybrid reading: the paper's lattice scheme is
// isothermal).  Device code only; included by wdlb.hip after thermal.hpp.
// R is the storage real (FP64 or FP32); the viscous force is recovered from
// the step's total force, to the rounding of that total.
//
// With theta = T / kT at every node: the mean-field force and u1 carry
// theta, the viscous force sqrt(theta), A theta (Sec. 3: F^mf ~ k_B T,
// F^v ~ sqrt(k_B T), A_ij ~ k_B T), the thermal force F^T is added, the
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

// after the mean-field kernel: F^mf <- theta F^mf and u1 = j/rho + (g + theta F^mf)/2
// into the padded (rho, u1) array with its images; a temperature that is not
// positive and finite raises FLAG_T
template <typename R>
__global__ __launch_bounds__(256) void k_th_u1(Geom g, Pad p, const R *__restrict__ T, R kT, const R *__restrict__ jx,
                                               const R *__restrict__ jy, const R *__restrict__ jz, R gx, R gy, R gz,
                                               V4<R> *__restrict__ fmf, V4<R> *__restrict__ ru1_p, int *flag)
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
    const V4<R> v = {rr, jx[i] / rr + R(0.5) * (gx + f.x), jy[i] / rr + R(0.5) * (gy + f.y),
                     jz[i] / rr + R(0.5) * (gz + f.z)};
    for_images(g, p, x, y, z, [&](int k) { ru1_p[k] = v; });
}

// after the viscous/SMDB kernel (whose F holds rho (g + theta F^mf + F^v(kT))):
// F = rho (g + theta F^mf + sqrt(theta) F^v(kT) + F^T) and A <- theta A
template <typename R>
__global__ __launch_bounds__(256) void k_th_force(Geom g, Pad p, const V4<R> *__restrict__ ru1_p,
                                                  const R *__restrict__ T, R kT, const V4<R> *__restrict__ fmf,
                                                  const R *__restrict__ FT, R gx, R gy, R gz, R *__restrict__ F,
                                                  R *__restrict__ A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const long long N = g.N;
    const R r = ru1_p[pidx(p, x, y, z)].x, th = T[i] / kT, sq = sqrt(th);
    const V4<R> fm = fmf[i];
    const R gg[3] = {gx, gy, gz}, fmc[3] = {fm.x, fm.y, fm.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const R fv = F[d * N + i] / r - gg[d] - fmc[d];
        F[d * N + i] = r * (gg[d] + fmc[d] + sq * fv + FT[d * N + i]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) A[k * N + i] = th * A[k * N + i];
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

// the part of dT/dt held fixed over the step's sub-steps:
//   -u.grad T + (2/(3n)) (-div delta q - P:grad u + Q)
// central differences (beyond a wall u is mirrored to -u, T to T), delta q =
// B/(2 omega0) through the faces (none through a wall); P of eqs. pexplicit
// and extrapressure with the step's A (stored xx, yy, zz, xy, xz, yz)
template <typename R>
__global__ __launch_bounds__(256) void k_energy_fixed(Geom g, Pad p, const V4<R> *__restrict__ ru1_p,
                                                      const R *__restrict__ T_p, const R *__restrict__ jx,
                                                      const R *__restrict__ jy, const R *__restrict__ jz,
                                                      const R *__restrict__ F, const R *__restrict__ A,
                                                      const R *__restrict__ Q, const R *__restrict__ B, R omega0,
                                                      R *__restrict__ Rfix)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const long long N = g.N;
    const int gb = pidx(p, x, y, z);
    const R n = ru1_p[gb].x, Tr = T_p[gb];
    R u0[3];
    th_vel<R>(g, p, ru1_p, jx, jy, jz, F, x, y, z, u0);
    R gu[3][3], gT[3], divdq = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int dx = a == 0, dy = a == 1, dz = a == 2;
        int xp = x + dx, yp = y + dy, zp = z + dz, xm = x - dx, ym = y - dy, zm = z - dz;
        xp = xp == g.nx ? 0 : xp;
        xm = xm < 0 ? g.nx - 1 : xm;
        yp = yp == g.ny ? 0 : yp;
        ym = ym < 0 ? g.ny - 1 : ym;
        bool okp = true, okm = true;
        if (g.walls) {
            okp = zp < g.nz;
            okm = zm >= 0;
        } else {
            zp = zp == g.nz ? 0 : zp;
            zm = zm < 0 ? g.nz - 1 : zm;
        }
        R up[3], um[3];
        if (okp) th_vel<R>(g, p, ru1_p, jx, jy, jz, F, xp, yp, zp, up);
        else up[0] = -u0[0], up[1] = -u0[1], up[2] = -u0[2];
        if (okm) th_vel<R>(g, p, ru1_p, jx, jy, jz, F, xm, ym, zm, um);
        else um[0] = -u0[0], um[1] = -u0[1], um[2] = -u0[2];
#pragma unroll
        for (int b = 0; b < 3; ++b) gu[a][b] = R(0.5) * (up[b] - um[b]);
        const R Tp = okp ? T_p[pidx(p, xp, yp, zp)] : Tr, Tm = okm ? T_p[pidx(p, xm, ym, zm)] : Tr;
        gT[a] = R(0.5) * (Tp - Tm);
        const long long ip = ((long long)zp * g.ny + yp) * g.nx + xp, im = ((long long)zm * g.ny + ym) * g.nx + xm;
        const R q0 = B[a * N + i] / (R(2) * omega0);
        const R fp = okp ? R(0.5) * (q0 + B[a * N + ip] / (R(2) * omega0)) : R(0);
        const R fm = okm ? R(0.5) * (B[a * N + im] / (R(2) * omega0) + q0) : R(0);
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
}

// one sub-step: T_out = T + (Rfix + (2/(3n)) (-div q_kin)) / nsub, the
// kinetic flux through the six faces (none through a wall)
template <typename R>
__global__ __launch_bounds__(256) void k_energy_sub(Geom g, Pad p, const R *__restrict__ T_p,
                                                    const V4<R> *__restrict__ ru1_p, const R *__restrict__ Rfix,
                                                    R omega0, int nsub, R *__restrict__ T_out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const int gb = pidx(p, x, y, z);
    const R n = ru1_p[gb].x, Tr = T_p[gb];
    const int dp[3] = {1, p.PX, p.PXY};
    R div = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R fp = 0, fm = 0;
        const bool okp = !(a == 2 && g.walls && z == g.nz - 1), okm = !(a == 2 && g.walls && z == 0);
        if (okp) {
            const R Tp = T_p[gb + dp[a]], np_ = ru1_p[gb + dp[a]].x;
            fp = -R(2.5) / omega0 * R(0.5) * (n * Tr + np_ * Tp) * (Tp - Tr);
        }
        if (okm) {
            const R Tm = T_p[gb - dp[a]], nm = ru1_p[gb - dp[a]].x;
            fm = -R(2.5) / omega0 * R(0.5) * (nm * Tm + n * Tr) * (Tr - Tm);
        }
        div += fp - fm;
    }
    T_out[i] = Tr + (Rfix[i] + R(2) / (R(3) * n) * (-div)) / R(nsub);
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
