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

// (rho, u) from n[N] and u[3N] (component-major; null: at rest) into the
// padded V4 array
template <typename R>
__global__ __launch_bounds__(256) void k_pad_ru(Geom g, Pad p, const R *__restrict__ n, const R *__restrict__ u,
                                                V4<R> *__restrict__ dst)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const V4<R> v = u ? V4<R>{n[i], u[i], u[g.N + i], u[2 * g.N + i]} : V4<R>{n[i], R(0), R(0), R(0)};
    for_images(g, p, x, y, z, [&](int k) { dst[k] = v; });
}

// One mirror group of the thermal sums from its four images: s (rho, u), tm
// (T) and gm (contact value with w_S).  D_m = G_m dT_m and V_m = G_m dv_m,
// products unfused as in the step's shell sums, then the Hadamard transform
// over the mirror signs and one FMA per weight.  w is the group's plain
// weight: 1, or 1/2 (1/4) when a (and b) is zero and its images repeat;
// px, py, pz carry it times k.
template <typename R>
__device__ __forceinline__ void th_quad(const Quad<R> &Qd, const R (&gm)[4], const V4<R> (&sm)[4], const R (&tm)[4],
                                        const V4<R> &c0, R T0, R &ax, R &ay, R &az, R &aT, R &aV)
{
    const R w = R(Qd.a > 0 ? 1.0 : 0.5) * R(Qd.b > 0 ? 1.0 : 0.5);
    R hx, hy, h0, vx, vy, vz;
    {
#pragma clang fp contract(off)
        R D[4], Vx[4], Vy[4], Vz[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const R G = gm[m] * sm[m].x;
            D[m] = G * (tm[m] - T0);
            Vx[m] = G * (sm[m].y - c0.y);
            Vy[m] = G * (sm[m].z - c0.z);
            Vz[m] = G * (sm[m].w - c0.w);
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

// Q, B and F^T of the node from the five sums
template <typename R>
__device__ __forceinline__ void th_finish(const Geom &g, int x, int y, int z, R n0, R T0, R s2, R ax, R ay, R az,
                                          R aT, R aV, R *__restrict__ Qo, R *__restrict__ Bo, R *__restrict__ FTo)
{
    const long long N = g.N;
    const int i = (z * g.ny + y) * g.nx + x;
    const R kq = n0 * s2, kb = R(-2) * T0 * n0 * s2, kf = R(-0.5) * s2;
    Qo[i] = kq * (R(-0.5) * T0 * aV + sqrt(T0 / R(M_PI)) * aT);
    Bo[i] = kb * ax;
    Bo[N + i] = kb * ay;
    Bo[2 * N + i] = kb * az;
    FTo[i] = kf * ax;
    FTo[N + i] = kf * ay;
    FTo[2 * N + i] = kf * az;
}

// NoU (all three thermal kernels): the fields at u = 0 -- the velocity is not
// used and Q keeps its conduction part only (the coupled thermal flow forms
// its compression part from the viscous kernel's trace sums).
//
// k_thermal: one lane per node on 32 x 8 tiles of a plane; the shell from
// the quad table (mirror groups (+-a, +-b, c), in the table's order), the
// images' rho, u, T and contact values read through the caches.  A state
// that does not depend on x (or y) gives exactly zero x (y) components.  The
// contact values of the density kernel carry the shell weight w_S;
// s2 = sigma^2.  Used where the LDS rings of k_thermal_r do not fit.
template <typename R, bool NoU = false>
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
        R gm[4], tm[4];
        V4<R> sm[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            gm[m] = gb[mo[m]];
            sm[m] = ru_p[gbase + so[m]];
            tm[m] = T_p[gbase + so[m]];
        }
        th_quad<R>(Qd, gm, sm, tm, c0, T0, ax, ay, az, aT, aV);
    }
    th_finish<R>(g, x, y, z, c0.x, T0, s2, ax, ay, az, aT, NoU ? R(0) : aV, Qo, Bo, FTo);
}

// k_thermal_r: the same sums on TX x TY x TZ tiles with (rho, u) and T
// staged in two LDS rings of planes that advance along e_z (the plane ring
// of the step's shell kernels, one for V4 (rho, u) and one for T; see
// ShellRings), the contact values read through the caches.  The groups are
// visited in the same order as by k_thermal, with the same arithmetic, so
// the two kernels give the same bits.
template <typename R, int TX, int TY, int TZ, int NR, bool NoU = false>
__global__ __launch_bounds__(TX *TY *TZ) void k_thermal_r(Geom g, Pad p, int Rr, const V4<R> *__restrict__ ru_p,
                                                          const R *__restrict__ T_p, const R *__restrict__ gam_p,
                                                          const Quad<R> *__restrict__ quads,
                                                          const int *__restrict__ qstart, R s2, int tiles_x,
                                                          int tiles_y, int tiles_z, R *__restrict__ Qo,
                                                          R *__restrict__ Bo, R *__restrict__ FTo)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ>(tiles_x, tiles_y, tiles_z);
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    ShellRings<R, V4<R>, TX, TY, TZ, NR, 0> rg;   // (rho, u) ring; fill ends with a barrier
    rg.init(lds_raw, p, Rr, tc, ru_p, gam_p);
    constexpr int NT = TX * TY * TZ, NS = TZ + 1;
    PlaneRing<R, R, NT, NR> tr;                    // T ring after the (rho, u) ring
    tr.setup(p, Rr, TX, TY, tc.x0, tc.y0);
    R *twin = reinterpret_cast<R *>(lds_raw + (size_t)NS * rg.pr.LP * sizeof(V4<R>));
    {
        R tst[TZ][1][NR];
#pragma unroll
        for (int k = 0; k < TZ; ++k) tr.fetch_to(tst[k], T_p, p, tc.z0 - Rr + k);
#pragma unroll
        for (int k = 0; k < TZ; ++k) tr.store_all(tst[k], twin, k);
    }
    __syncthreads();
    const int gbase = pidx(p, min(x, g.nx - 1), min(y, g.ny - 1), min(z, g.nz - 1));
    const V4<R> c0 = ru_p[gbase];
    const R T0 = T_p[gbase];
    const int LX = rg.pr.LX;
    constexpr int QB = 8;
    R ax = 0, ay = 0, az = 0, aT = 0, aV = 0;
    for (int c = -Rr; c <= Rr; ++c) {
        rg.template begin<0>(c, p, ru_p, gam_p);
        if (c < Rr) tr.template fetch<0, true>(T_p, p, tc.z0 + c + TZ);
        const V4<R> *pl = rg.plane(c);
        const R *tl = twin + ((tc.lz + c + Rr) % NS) * tr.LP + rg.lbase;
        const int qb = qstart[c + Rr], qe = qstart[c + Rr + 1];
        // contact values of QB groups at a time, all loads issued before the
        // first is used (one cache latency per batch rather than per group)
        for (int q0 = qb; q0 < qe; q0 += QB) {
            R gb[QB][4];
#pragma unroll
            for (int k = 0; k < QB; ++k)
                if (q0 + k < qe) {
                    const Quad<R> Qd = quads[q0 + k];
                    gamma_quad<R, false>(nullptr, 0, 0, gam_p, p, gbase, Qd.a, Qd.b, Qd.c, Qd.hidx, gb[k]);
                }
#pragma unroll
            for (int k = 0; k < QB; ++k)
                if (q0 + k < qe) {
                    const Quad<R> Qd = quads[q0 + k];
                    const int a = Qd.a, b = Qd.b;
                    R tm[4];
                    V4<R> sm[4];
                    sm[0] = pl[a + b * LX];
                    sm[1] = pl[-a + b * LX];
                    sm[2] = pl[a - b * LX];
                    sm[3] = pl[-a - b * LX];
                    tm[0] = tl[a + b * LX];
                    tm[1] = tl[-a + b * LX];
                    tm[2] = tl[a - b * LX];
                    tm[3] = tl[-a - b * LX];
                    th_quad<R>(Qd, gb[k], sm, tm, c0, T0, ax, ay, az, aT, aV);
                }
        }
        if (c < Rr) tr.template store<0>(twin, (c + TZ + Rr) % NS);
        rg.template end<0>(c);   // stores the next (rho, u) plane, then the barrier
    }
    if (!valid) return;
    th_finish<R>(g, x, y, z, c0.x, T0, s2, ax, ay, az, aT, NoU ? R(0) : aV, Qo, Bo, FTo);
}

// k_thermal_s: the same sums compiled for the shell of 2 sigma = S2:
// the e_z steps and the groups unrolled, every LDS offset an immediate,
// every weight a literal; the contact values by buffer loads whose image
// offset is a scalar (see gamma_img).  Groups with a or b zero sum their
// distinct images once with doubled (quadrupled) weights, which is exact, so
// the result is bit-identical to k_thermal_r and k_thermal.
template <typename R, int S2, int TX, int TY, int TZ, int NR, bool NoU = false>
__global__ __launch_bounds__(TX *TY *TZ) void k_thermal_s(Geom g, Pad p, const V4<R> *__restrict__ ru_p,
                                                          const R *__restrict__ T_p, const R *__restrict__ gam_p,
                                                          R s2, int tiles_x, int tiles_y, int tiles_z,
                                                          R *__restrict__ Qo, R *__restrict__ Bo, R *__restrict__ FTo)
{
    using SH = Shell<S2>;
    constexpr int RC = SH::R, LX = TX + 2 * RC, O = (RC + 1) >> 1, NT = TX * TY * TZ, NS = TZ + 1;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ, TZ == 1>(tiles_x, tiles_y, tiles_z);
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    ShellRings<R, V4<R>, TX, TY, TZ, NR, 0> rg;
    rg.init(lds_raw, p, RC, tc, ru_p, gam_p);
    PlaneRing<R, R, NT, NR> tr;
    tr.setup(p, RC, TX, TY, tc.x0, tc.y0);
    R *twin = reinterpret_cast<R *>(lds_raw + (size_t)NS * rg.pr.LP * sizeof(V4<R>));
    {
        R tst[TZ][1][NR];
#pragma unroll
        for (int k = 0; k < TZ; ++k) tr.fetch_to(tst[k], T_p, p, tc.z0 - RC + k);
#pragma unroll
        for (int k = 0; k < TZ; ++k) tr.store_all(tst[k], twin, k);
    }
    __syncthreads();
    const int gbase = pidx(p, min(x, g.nx - 1), min(y, g.ny - 1), min(z, g.nz - 1));
    const unsigned gvo = (unsigned)gbase * (unsigned)sizeof(R);
    const V4<R> c0 = ru_p[gbase];
    const R T0 = T_p[gbase];
    R ax = 0, ay = 0, az = 0, aT = 0, aV = 0;
    static_for<-RC, RC + 1>([&](auto ci) __attribute__((always_inline)) {
        constexpr int c = decltype(ci)::value;
        rg.template begin<0>(c, p, ru_p, gam_p);
        if constexpr (c < RC) tr.template fetch<0, true>(T_p, p, tc.z0 + c + TZ);
        const V4<R> *pc = rg.plane(c) - (RC + RC * LX);
        const R *tcp = twin + ((tc.lz + c + RC) % NS) * tr.LP + rg.lbase - (RC + RC * LX);
        __amdgpu_buffer_rsrc_t gr[4];
        gamma_rsrc<R>(gam_p, p, c, O, gr);
        static_for<SH::T.qs[c + RC], SH::T.qs[c + RC + 1]>([&](auto qi) __attribute__((always_inline)) {
            constexpr CQuad Q = SH::T.q[decltype(qi)::value];
            constexpr int a = Q.a, b = Q.b;
#define WDLB_TGAM(SA, SB) gamma_img<R, false, O, 1, 1, a, b, Q.h, SA, SB>(nullptr, gr, p.PX, gvo)
            if constexpr (a == 0 && b == 0) {
                R D, Vz;
                {
#pragma clang fp contract(off)
                    const V4<R> sv = pc[RC + RC * LX];
                    const R G = WDLB_TGAM(1, 1) * sv.x;
                    D = G * (tcp[RC + RC * LX] - T0);
                    Vz = G * (sv.w - c0.w);
                }
                az += R(4 * Q.pz) * D;
                aT += D;
                aV += R(4 * Q.pz) * Vz;
            } else if constexpr (a == 0) {  // images (0, b), (0, -b)
                R dp, dm, vy, vz;
                {
#pragma clang fp contract(off)
                    const V4<R> s0 = pc[RC + (RC + b) * LX], s2_ = pc[RC + (RC - b) * LX];
                    const R G0 = WDLB_TGAM(1, 1) * s0.x, G2 = WDLB_TGAM(1, -1) * s2_.x;
                    const R D0 = G0 * (tcp[RC + (RC + b) * LX] - T0), D2 = G2 * (tcp[RC + (RC - b) * LX] - T0);
                    dp = D0 + D2;
                    dm = D0 - D2;
                    vy = G0 * (s0.z - c0.z) - G2 * (s2_.z - c0.z);
                    vz = G0 * (s0.w - c0.w) + G2 * (s2_.w - c0.w);
                }
                ay += R(2 * Q.py) * dm;
                az += R(2 * Q.pz) * dp;
                aT += dp;
                aV += R(2 * Q.py) * vy;
                aV += R(2 * Q.pz) * vz;
            } else if constexpr (b == 0) {  // images (a, 0), (-a, 0)
                R dp, dm, vx, vz;
                {
#pragma clang fp contract(off)
                    const V4<R> s0 = pc[(RC + a) + RC * LX], s1 = pc[(RC - a) + RC * LX];
                    const R G0 = WDLB_TGAM(1, 1) * s0.x, G1 = WDLB_TGAM(-1, 1) * s1.x;
                    const R D0 = G0 * (tcp[(RC + a) + RC * LX] - T0), D1 = G1 * (tcp[(RC - a) + RC * LX] - T0);
                    dp = D0 + D1;
                    dm = D0 - D1;
                    vx = G0 * (s0.y - c0.y) - G1 * (s1.y - c0.y);
                    vz = G0 * (s0.w - c0.w) + G1 * (s1.w - c0.w);
                }
                ax += R(2 * Q.px) * dm;
                az += R(2 * Q.pz) * dp;
                aT += dp;
                aV += R(2 * Q.px) * vx;
                aV += R(2 * Q.pz) * vz;
            } else {
                const R gm[4] = {WDLB_TGAM(1, 1), WDLB_TGAM(-1, 1), WDLB_TGAM(1, -1), WDLB_TGAM(-1, -1)};
                const V4<R> sm[4] = {pc[(RC + a) + (RC + b) * LX], pc[(RC - a) + (RC + b) * LX],
                                     pc[(RC + a) + (RC - b) * LX], pc[(RC - a) + (RC - b) * LX]};
                const R tm[4] = {tcp[(RC + a) + (RC + b) * LX], tcp[(RC - a) + (RC + b) * LX],
                                 tcp[(RC + a) + (RC - b) * LX], tcp[(RC - a) + (RC - b) * LX]};
                R hx, hy, h0, vx, vy, vz;
                {
#pragma clang fp contract(off)
                    R D[4], Vx[4], Vy[4], Vz[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const R G = gm[m] * sm[m].x;
                        D[m] = G * (tm[m] - T0);
                        Vx[m] = G * (sm[m].y - c0.y);
                        Vy[m] = G * (sm[m].z - c0.z);
                        Vz[m] = G * (sm[m].w - c0.w);
                    }
                    const R P1 = D[0] + D[1], M1 = D[0] - D[1], P2 = D[2] + D[3], M2 = D[2] - D[3];
                    hx = M1 + M2;
                    hy = P1 - P2;
                    h0 = P1 + P2;
                    vx = (Vx[0] - Vx[1]) + (Vx[2] - Vx[3]);
                    vy = (Vy[0] + Vy[1]) - (Vy[2] + Vy[3]);
                    vz = (Vz[0] + Vz[1]) + (Vz[2] + Vz[3]);
                }
                ax += R(Q.px) * hx;
                ay += R(Q.py) * hy;
                az += R(Q.pz) * h0;
                aT += h0;
                aV += R(Q.px) * vx;
                aV += R(Q.py) * vy;
                aV += R(Q.pz) * vz;
            }
#undef WDLB_TGAM
        });
        pin(ax);
        pin(ay);
        pin(az);
        pin(aT);
        if constexpr (!NoU) pin(aV);
        if constexpr (c < RC) tr.template store<0>(twin, (c + TZ + RC) % NS);
        rg.template end<0>(c);
    });
    if (!valid) return;
    th_finish<R>(g, x, y, z, c0.x, T0, s2, ax, ay, az, aT, NoU ? R(0) : aV, Qo, Bo, FTo);
}

// ring of density planes filled from the (rho, u) array's first component:
// the plane ring of PlaneRing<R, R> (same window, same element order) with
// 4-byte LDS entries
template <typename R, int NT, int NR>
struct RhoRing {
    int LX, LP;
    int off[NR];
    R st[2][NR];  // two staging sets: one in flight while the other is stored

    __device__ __forceinline__ void setup(const Pad &p, int Rr, int TX, int TY, int x0, int y0)
    {
        LX = TX + 2 * Rr;
        LP = LX * (TY + 2 * Rr);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int e = min((int)threadIdx.x + k * NT, LP - 1);
            const int X = min(max(x0 - Rr + e % LX + p.P, 0), p.PX - 1);
            const int Y = min(max(y0 - Rr + e / LX + p.P, 0), p.PY - 1);
            off[k] = Y * p.PX + X;
        }
    }
    __device__ __forceinline__ void fetch_to(R (&d)[NR], const V4<R> *__restrict__ src, const Pad &p, int pz)
    {
        const long long zb = (long long)min(max(pz + p.P, 0), p.PZ - 1) * p.PXY;
#pragma unroll
        for (int k = 0; k < NR; ++k) d[k] = src[zb + off[k]].x;
    }
    template <int S>
    __device__ __forceinline__ void fetch(const V4<R> *__restrict__ src, const Pad &p, int pz)
    {
        fetch_to(st[S], src, p, pz);
    }
    __device__ __forceinline__ void store_all(const R (&d)[NR], R *win, int slot)
    {
#pragma unroll
        for (int k = 0; k < NR; ++k) win[slot * LP + min((int)threadIdx.x + k * NT, LP - 1)] = d[k];
    }
    template <int S>
    __device__ __forceinline__ void store(R *win, int slot)
    {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int e = (int)threadIdx.x + k * NT;
            if (e < LP) win[slot * LP + e] = st[S][k];
        }
    }
};

// LDS of k_thermal_s0 on TX x TY x TZ tiles: the density and T rings (TZ + 1
// planes each), then the contact-value ring (2 TZ slices of four sub-lattices)
__host__ __device__ constexpr size_t thermal0_lds_bytes(int TX, int TY, int TZ, int Rr, size_t rbytes)
{
    return (size_t)(TZ + 1) * (TX + 2 * Rr) * (TY + 2 * Rr) * 2 * rbytes +
           (size_t)2 * TZ * 4 * (TX + Rr) * (TY + Rr) * rbytes;
}
template <int TX, int TY, int TZ, int RC>
struct Thermal0Tile {
    static constexpr int NT = TX * TY * TZ;
    static constexpr int NR = ((TX + 2 * RC) * (TY + 2 * RC) + NT - 1) / NT;
    static constexpr int NG = (4 * (TX + RC) * (TY + RC) + NT - 1) / NT;
};

// The thermal sums at u = 0 compiled for the shell of 2 sigma = S2 on
// TX x TY x TZ tiles: F^T, B and the conduction part of Q, the velocity not
// read.  The density, T and the contact values all come from LDS rings
// that advance along e_z (the contact values as in the mean-field kernel,
// and with its prefetch depth 2: each step loads what the next one stores),
// so the texture path carries only the ring fills; the arithmetic repeats
// k_thermal_s's term for term (the same bits).
template <typename R, int S2, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_thermal_s0(Geom g, Pad p, const V4<R> *__restrict__ ru_p,
                                                       const R *__restrict__ T_p, const R *__restrict__ gam_p, R s2,
                                                       int tiles_x, int tiles_y, int tiles_z, R *__restrict__ Qo,
                                                       R *__restrict__ Bo, R *__restrict__ FTo)
{
    using SH = Shell<S2>;
    constexpr int RC = SH::R, LX = TX + 2 * RC, O = (RC + 1) >> 1, LXg = TX + RC, LG = LXg * (TY + RC);
    constexpr int NT = TX * TY * TZ, NS = TZ + 1, NSG = 2 * TZ;
    constexpr int NR = Thermal0Tile<TX, TY, TZ, RC>::NR, NG = Thermal0Tile<TX, TY, TZ, RC>::NG;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ, TZ == 1>(tiles_x, tiles_y, tiles_z);
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    RhoRing<R, NT, NR> rr;
    rr.setup(p, RC, TX, TY, tc.x0, tc.y0);
    PlaneRing<R, R, NT, NR> tr;
    tr.setup(p, RC, TX, TY, tc.x0, tc.y0);
    GammaRing<R, NT, NG> gr;
    gr.setup(p, RC, TX, TY, tc.x0, tc.y0);
    R *rwin = reinterpret_cast<R *>(lds_raw);
    R *twin = rwin + NS * rr.LP;
    R *gwin = twin + NS * rr.LP;
    {
        // the first TZ planes and 2 TZ - 1 slices, all fetched before any is stored
        R rst[TZ][NR], tst[TZ][1][NR], gst[2 * TZ - 1][NG];
#pragma unroll
        for (int k = 0; k < TZ; ++k) {
            rr.fetch_to(rst[k], ru_p, p, tc.z0 - RC + k);
            tr.fetch_to(tst[k], T_p, p, tc.z0 - RC + k);
        }
#pragma unroll
        for (int j = 0; j < 2 * TZ - 1; ++j) gr.fetch_to(gst[j], gam_p, p, tc.z0, j - RC);
        // what step -RC stores at its end (prefetch depth 2, as the mean-field kernel)
        rr.template fetch<0>(ru_p, p, tc.z0 + TZ - RC);
        tr.template fetch<0, false>(T_p, p, tc.z0 + TZ - RC);
        gr.template fetch<0, false>(gam_p, p, tc.z0, 2 * TZ - 1 - RC);
#pragma unroll
        for (int k = 0; k < TZ; ++k) {
            rr.store_all(rst[k], rwin, k);
            tr.store_all(tst[k], twin, k);
        }
#pragma unroll
        for (int j = 0; j < 2 * TZ - 1; ++j) gr.store_all(gst[j], gwin, (j - RC + 64) % NSG);
    }
    __syncthreads();
    const int lbase = (tc.ly + RC) * LX + (tc.lx + RC), gcen = (tc.ly + O) * LXg + (tc.lx + O);
    const int gbase = pidx(p, min(x, g.nx - 1), min(y, g.ny - 1), min(z, g.nz - 1));
    const R n0 = ru_p[gbase].x, T0 = T_p[gbase];
    R ax = 0, ay = 0, az = 0, aT = 0;
    static_for<-RC, RC + 1>([&](auto ci) __attribute__((always_inline)) {
        constexpr int c = decltype(ci)::value;
        constexpr int S = (c + RC) & 1;
        if constexpr (c + 1 < RC) {  // for the store at the end of step c + 1
            rr.template fetch<S ^ 1>(ru_p, p, tc.z0 + c + 1 + TZ);
            tr.template fetch<S ^ 1, false>(T_p, p, tc.z0 + c + 1 + TZ);
            gr.template fetch<S ^ 1, false>(gam_p, p, tc.z0, c + 2 * TZ);
        }
        const R *pc = rwin + ((tc.lz + c + RC) % NS) * rr.LP + lbase - (RC + RC * LX);
        const R *tcp = twin + ((tc.lz + c + RC) % NS) * rr.LP + lbase - (RC + RC * LX);
        const R *gc = gwin + ((c + 2 * tc.lz + 64) % NSG) * gr.LS + gcen - (O + O * LXg);
        __amdgpu_buffer_rsrc_t gnone[4];  // unused: the contact values come from LDS
        static_for<SH::T.qs[c + RC], SH::T.qs[c + RC + 1]>([&](auto qi) __attribute__((always_inline)) {
            constexpr CQuad Q = SH::T.q[decltype(qi)::value];
            constexpr int a = Q.a, b = Q.b;
#define WDLB_TGAM(SA, SB) gamma_img<R, true, O, LXg, LG, a, b, Q.h, SA, SB>(gc, gnone, p.PX, 0u)
            if constexpr (a == 0 && b == 0) {
                R D;
                {
#pragma clang fp contract(off)
                    const R G = WDLB_TGAM(1, 1) * pc[RC + RC * LX];
                    D = G * (tcp[RC + RC * LX] - T0);
                }
                az += R(4 * Q.pz) * D;
                aT += D;
            } else if constexpr (a == 0) {  // images (0, b), (0, -b)
                R dp, dm;
                {
#pragma clang fp contract(off)
                    const R G0 = WDLB_TGAM(1, 1) * pc[RC + (RC + b) * LX];
                    const R G2 = WDLB_TGAM(1, -1) * pc[RC + (RC - b) * LX];
                    const R D0 = G0 * (tcp[RC + (RC + b) * LX] - T0), D2 = G2 * (tcp[RC + (RC - b) * LX] - T0);
                    dp = D0 + D2;
                    dm = D0 - D2;
                }
                ay += R(2 * Q.py) * dm;
                az += R(2 * Q.pz) * dp;
                aT += dp;
            } else if constexpr (b == 0) {  // images (a, 0), (-a, 0)
                R dp, dm;
                {
#pragma clang fp contract(off)
                    const R G0 = WDLB_TGAM(1, 1) * pc[(RC + a) + RC * LX];
                    const R G1 = WDLB_TGAM(-1, 1) * pc[(RC - a) + RC * LX];
                    const R D0 = G0 * (tcp[(RC + a) + RC * LX] - T0), D1 = G1 * (tcp[(RC - a) + RC * LX] - T0);
                    dp = D0 + D1;
                    dm = D0 - D1;
                }
                ax += R(2 * Q.px) * dm;
                az += R(2 * Q.pz) * dp;
                aT += dp;
            } else {
                const R gm[4] = {WDLB_TGAM(1, 1), WDLB_TGAM(-1, 1), WDLB_TGAM(1, -1), WDLB_TGAM(-1, -1)};
                const R rm[4] = {pc[(RC + a) + (RC + b) * LX], pc[(RC - a) + (RC + b) * LX],
                                 pc[(RC + a) + (RC - b) * LX], pc[(RC - a) + (RC - b) * LX]};
                const R tm[4] = {tcp[(RC + a) + (RC + b) * LX], tcp[(RC - a) + (RC + b) * LX],
                                 tcp[(RC + a) + (RC - b) * LX], tcp[(RC - a) + (RC - b) * LX]};
                R hx, hy, h0;
                {
#pragma clang fp contract(off)
                    R D[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) D[m] = (gm[m] * rm[m]) * (tm[m] - T0);
                    const R P1 = D[0] + D[1], M1 = D[0] - D[1], P2 = D[2] + D[3], M2 = D[2] - D[3];
                    hx = M1 + M2;
                    hy = P1 - P2;
                    h0 = P1 + P2;
                }
                ax += R(Q.px) * hx;
                ay += R(Q.py) * hy;
                az += R(Q.pz) * h0;
                aT += h0;
            }
#undef WDLB_TGAM
        });
        pin(ax);
        pin(ay);
        pin(az);
        pin(aT);
        if constexpr (c < RC) {
            rr.template store<S>(rwin, (c + TZ + RC) % NS);
            tr.template store<S>(twin, (c + TZ + RC) % NS);
            gr.template store<S>(gwin, (c + 2 * TZ - 1 + 64) % NSG);
        }
        __syncthreads();
    });
    if (!valid) return;
    th_finish<R>(g, x, y, z, n0, T0, s2, ax, ay, az, aT, R(0), Qo, Bo, FTo);
}

// LDS bytes of k_thermal_r: the (rho, u) ring, then the T ring
__host__ __device__ constexpr size_t thermal_lds_bytes(int TX, int TY, int TZ, int Rr, size_t rbytes)
{
    return (size_t)(TZ + 1) * (TX + 2 * Rr) * (TY + 2 * Rr) * 5 * rbytes;
}

// ---------------------------------------------------------------------------
// k_conduct: one forward-Euler step of the energy balance at rest (u = 0,
// fixed n; Sec. 2 eq. energyequation in the setting of Sec. 4's
// conductivity), T_new = T + dt (-div q + Q) / ((3/2) n), with the heat flux
// of eq. qexplicit through the six faces of the node: kinetic
// -kin * mean(n T) * (T(r + e) - T(r)), kin = 5 / (2 omega0), plus the mean
// of delta q = cq B, cq = 1 / (2 omega0), at the two nodes; no flux through a
// wall.  T and n come padded (periodic images in place), B unpadded.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_conduct(Geom g, Pad p, const R *__restrict__ T_p,
                                                 const V4<R> *__restrict__ ru_p, const R *__restrict__ Q,
                                                 const R *__restrict__ B, R kin, R cq, R dt, R *__restrict__ T_out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const long long N = g.N;
    const int gb = pidx(p, x, y, z);
    const R T0 = T_p[gb], n0 = ru_p[gb].x, nT0 = n0 * T0;
    const int dp[3] = {1, p.PX, p.PXY};
    // unpadded neighbour indices (periodic wrap; at a wall the face is closed)
    const int xp = x + 1 == g.nx ? 0 : x + 1, xm = x == 0 ? g.nx - 1 : x - 1;
    const int yp = y + 1 == g.ny ? 0 : y + 1, ym = y == 0 ? g.ny - 1 : y - 1;
    const int zp = z + 1 == g.nz ? 0 : z + 1, zm = z == 0 ? g.nz - 1 : z - 1;
    const long long row = (long long)(z * g.ny + y) * g.nx;
    const long long ip[3] = {row + xp, (long long)(z * g.ny + yp) * g.nx + x, (long long)(zp * g.ny + y) * g.nx + x};
    const long long im[3] = {row + xm, (long long)(z * g.ny + ym) * g.nx + x, (long long)(zm * g.ny + y) * g.nx + x};
    R div = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R Tp = T_p[gb + dp[a]], Tm = T_p[gb - dp[a]];
        const R nTp = ru_p[gb + dp[a]].x * Tp, nTm = ru_p[gb - dp[a]].x * Tm;
        const R q0 = cq * B[a * N + i];
        R fp = -kin * (R(0.5) * (nT0 + nTp)) * (Tp - T0) + R(0.5) * (q0 + cq * B[a * N + ip[a]]);
        R fm = -kin * (R(0.5) * (nTm + nT0)) * (T0 - Tm) + R(0.5) * (cq * B[a * N + im[a]] + q0);
        if (a == 2 && g.walls) {
            if (z == g.nz - 1) fp = R(0);
            if (z == 0) fm = R(0);
        }
        div += fp - fm;
    }
    T_out[i] = T0 + dt * ((-div + Q[i]) / (R(1.5) * n0));
}

}  // namespace wdlb
