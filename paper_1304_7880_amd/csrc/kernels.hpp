// kernels.hpp -- the gfx950 kernels of one WDLB step.  Device code only;
// included by wdlb.hip.
//
// One step (Sec. 5 of the paper, steps 2-4) is six kernels:
//   k_moments    pull-stream the stored populations; density (padded array,
//                with periodic images) and momentum
//   k_ball       Fischer-Methfessel smoothed density nbar, ball |e| <= sigma/2
//   k_gamma      Carnahan-Starling contact value at the 8 half-lattice
//                midpoints of every node, gamma_h(r) = g_CS(nbar(r + h/2))
//   k_meanfield  contact-shell sum of the mean-field force F^mf, and the
//                velocity u1 = j/rho + (g + F^mf)/2 with which F^v and A_ij
//                are formed
//   k_shell      contact-shell sums of the viscous force F^v and the SMDB
//                field A_ij (the dominant kernel: LDS window of (rho, u1)
//                planes rolled along e_z)
//   k_collide    forced BGK collision with the SMDB source; the
//                post-collision populations are streamed by the next pull,
//                with half-way bounce-back at the walls
//
// Padded arrays.  rho, nbar, gamma and (rho, u1) live in arrays padded by P
// (the contact-shell reach) on every side.  The kernel that writes a node
// also writes its periodic images into the padding; beyond a wall the
// padding stays zero, so rho = u = 0 outside the slit needs no test.  Every
// stencil access is then the node's padded index plus a uniform offset.
//
// Contact-shell sums visit the shell in groups of four mirror images
// (+-a, +-b, c).  The x- and y-odd parts of every sum are formed as
// differences of mirror images before they are accumulated, so a state that
// does not depend on x or y gives exactly zero x and y forces.
#pragma once
#include "d3q19.hpp"

namespace wdlb {

constexpr int FLAG_ETA = 1, FLAG_RHO = 2;

// one group of contact-shell offsets (+-a, +-b, c), sorted by c; p = weight
// * alpha, q = weight * alpha_i alpha_j with alpha = (a, b, c)/|e|; the
// weight 1, 1/2 or 1/4 undoes the repeated members when a or b is zero
template <typename R>
struct Quad {
    int a, b, c, hidx;
    R px, py, pz, qxx, qyy, qzz, qxy, qxz, qyz, pad0, pad1, pad2;
};

struct Pad {
    int P;             // halo width (contact-shell reach)
    int PX, PY, PZ;    // padded extents
    int PXY;           // PX * PY
    long long NP;      // PX * PY * PZ
    int kx, ky, kz;    // periodic image ranges
};

__device__ __forceinline__ int pidx(const Pad &p, int x, int y, int z)
{
    return ((z + p.P) * p.PY + (y + p.P)) * p.PX + (x + p.P);
}

// call f(padded index) for the node and each of its periodic images inside
// the padded box (no images across walls)
template <typename Fn>
__device__ __forceinline__ void for_images(const Geom &g, const Pad &p, int x, int y, int z, Fn &&f)
{
    for (int kz = -p.kz; kz <= p.kz; ++kz) {
        int zz = z + kz * g.nz;
        if (zz < -p.P || zz >= g.nz + p.P) continue;
        for (int ky = -p.ky; ky <= p.ky; ++ky) {
            int yy = y + ky * g.ny;
            if (yy < -p.P || yy >= g.ny + p.P) continue;
            for (int kx = -p.kx; kx <= p.kx; ++kx) {
                int xx = x + kx * g.nx;
                if (xx < -p.P || xx >= g.nx + p.P) continue;
                f(pidx(p, xx, yy, zz));
            }
        }
    }
}

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

// ---------------------------------------------------------------------------
// step 1 (initialisation)
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_fill(Geom g, V4<R> *ru, R n0, R ux, R uy, R uz)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < g.N) ru[i] = V4<R>{n0, ux, uy, uz};
}

// The populations at every node r are feq(n(r), u(r)).  The library stores
// pre-stream populations, so node s keeps for direction a the value that the
// next pull delivers to t = s + c_a, feq_a(n(t), u(t)), or, when t lies in a
// wall, the value that bounces back into s itself, feq_abar(n(s), u(s)); h
// is that minus feq_a(n(s), u(s)).
template <typename R, typename HS>
__global__ __launch_bounds__(256) void k_init(Geom g, const V4<R> *__restrict__ ru, HS *__restrict__ h)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const V4<R> q = ru[i];
    const D qx = q.x, qy = q.y, qz = q.z, qw = q.w;
    const D uu = qy * qy + qz * qz + qw * qw;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const D w = wgt<D>(a);
        D cu = D(CX[a]) * qy + D(CY[a]) * qz + D(CZ[a]) * qw;
        D Ps = D(3) * cu + D(4.5) * cu * cu - D(1.5) * uu;
        int tz = z + CZ[a];
        bool bb = false;
        if (CZ[a] != 0) {
            if (g.walls) bb = (tz < 0 || tz >= g.nz);
            else tz = wrap1(tz, g.nz);
        }
        D val;
        if (bb) {
            val = -D(6) * w * qx * cu;  // feq_abar(s) - feq_a(s)
        } else {
            int tx = CX[a] ? wrap1(x + CX[a], g.nx) : x;
            int ty = CY[a] ? wrap1(y + CY[a], g.ny) : y;
            V4<R> t = ru[(tz * g.ny + ty) * g.nx + tx];
            const D ty_ = t.y, tz_ = t.z, tw = t.w;
            D ct = D(CX[a]) * ty_ + D(CY[a]) * tz_ + D(CZ[a]) * tw;
            D Pt = D(3) * ct + D(4.5) * ct * ct - D(1.5) * (ty_ * ty_ + tz_ * tz_ + tw * tw);
            val = w * ((D(t.x) - qx) + (D(t.x) * Pt - qx * Ps));
        }
        sth<R, HS>(h + (long long)a * g.N + i, R(val));
    }
}

// ---------------------------------------------------------------------------
// steps 2-4
// ---------------------------------------------------------------------------
template <typename R, typename HS>
__global__ __launch_bounds__(256) void k_moments(Geom g, Pad p, const V4<R> *__restrict__ ru,
                                                 const HS *__restrict__ h, R *__restrict__ rho_p,
                                                 R *__restrict__ jx, R *__restrict__ jy, R *__restrict__ jz,
                                                 int *flag)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    D r, a, b, c;
    pull_moments<R, HS>(g, ru, h, x, y, z, r, a, b, c);
    if (!(r > D(0)) || !(r < D(INFINITY))) raise_flag(flag, FLAG_RHO);
    const R rr = R(r);
    for_images(g, p, x, y, z, [&](int k) { rho_p[k] = rr; });
    jx[i] = R(a);
    jy[i] = R(b);
    jz[i] = R(c);
}

// nbar(r) = (1/|B|) sum over the ball of rho; boff[] = padded offsets
template <typename R>
__global__ __launch_bounds__(256) void k_ball(Geom g, Pad p, const R *__restrict__ rho_p,
                                              const int *__restrict__ boff, int nball, R inv_nball,
                                              R *__restrict__ nbar_p)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const R *base = rho_p + pidx(p, x, y, z);
    R s = 0;
    for (int q = 0; q < nball; ++q) s += base[boff[q]];
    const R v = s * inv_nball;
    for_images(g, p, x, y, z, [&](int k) { nbar_p[k] = v; });
}

// gamma_h(r) = (4 pi/|S|) g_CS(pi sigma^3 nbar_mid / 6), nbar_mid the mean of
// nbar over the 2^|h| lattice nodes of r + h/2 (outside the slit nbar = 0)
template <typename R>
__global__ __launch_bounds__(256) void k_gamma(Geom g, Pad p, const R *__restrict__ nbar_p, R eta_per_n, R wS,
                                               R *__restrict__ gam_p, int *flag)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const int b = pidx(p, x, y, z);
    const R n000 = nbar_p[b], n100 = nbar_p[b + 1], n010 = nbar_p[b + p.PX], n110 = nbar_p[b + p.PX + 1];
    const R n001 = nbar_p[b + p.PXY], n101 = nbar_p[b + p.PXY + 1], n011 = nbar_p[b + p.PXY + p.PX],
            n111 = nbar_p[b + p.PXY + p.PX + 1];
    const bool zin = !g.walls || z + 1 < g.nz;  // the upper corners lie in the slit
    R m[8];
    m[0] = n000;
    m[1] = (n000 + n100) * R(0.5);
    m[2] = (n000 + n010) * R(0.5);
    m[3] = ((n000 + n100) + (n010 + n110)) * R(0.25);
    m[4] = (n000 + n001) * R(0.5);
    m[5] = ((n000 + n100) + (n001 + n101)) * R(0.25);
    m[6] = ((n000 + n010) + (n001 + n011)) * R(0.25);
    m[7] = (((n000 + n100) + (n010 + n110)) + ((n001 + n101) + (n011 + n111))) * R(0.125);
#pragma unroll
    for (int hi = 0; hi < 8; ++hi) {
        const R eta = eta_per_n * m[hi];
        R val;
        if (eta < R(1)) {
            const R om = R(1) - eta;
            val = wS * (R(1) - R(0.5) * eta) / (om * om * om);
        } else {
            if (hi < 4 || zin) raise_flag(flag, FLAG_ETA);
            val = R(0);
        }
        R *dst = gam_p + (long long)hi * p.NP;
        for_images(g, p, x, y, z, [&](int k) { dst[k] = val; });
    }
}

// uniform offsets of the four members (+-a, +-b, c) of a quad: source node
// (so) and midpoint node (mo) in a padded array with row pitch PX and plane
// pitch PXY
__device__ __forceinline__ void quad_offsets(int a, int b, int c, int PX, int PXY, int so[4], int mo[4])
{
    const int sa[4] = {a, -a, a, -a}, sb[4] = {b, b, -b, -b};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        so[m] = sa[m] + sb[m] * PX + c * PXY;
        mo[m] = (sa[m] >> 1) + (sb[m] >> 1) * PX + (c >> 1) * PXY;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_meanfield(Geom g, Pad p, const R *__restrict__ rho_p,
                                                   const R *__restrict__ jx, const R *__restrict__ jy,
                                                   const R *__restrict__ jz, const R *__restrict__ gam_p,
                                                   const Quad<R> *__restrict__ quads, int nq, R cmf, R gx, R gy,
                                                   R gz, V4<R> *__restrict__ ru1_p, V4<R> *__restrict__ fmf)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const int b = pidx(p, x, y, z);
    const R *rb = rho_p + b;
    R fx = 0, fy = 0, fz = 0;
    for (int q = 0; q < nq; ++q) {
        const Quad<R> Qd = quads[q];
        int so[4], mo[4];
        quad_offsets(Qd.a, Qd.b, Qd.c, p.PX, p.PXY, so, mo);
        const R *gb = gam_p + (long long)Qd.hidx * p.NP + b;
        R hx, hy, h0;
        {
            // the mirror products and their Hadamard must not be fused into
            // FMAs: fma(G0a, G0b, -G1) of identical mirror images is the
            // rounding error of G1, not zero
#pragma clang fp contract(off)
            R G[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) G[m] = gb[mo[m]] * rb[so[m]];
            const R P1 = G[0] + G[1], M1 = G[0] - G[1], P2 = G[2] + G[3], M2 = G[2] - G[3];
            hx = M1 + M2;
            hy = P1 - P2;
            h0 = P1 + P2;
        }
        fx += Qd.px * hx;
        fy += Qd.py * hy;
        fz += Qd.pz * h0;
    }
    const R Fx = cmf * fx, Fy = cmf * fy, Fz = cmf * fz;
    const R r = rb[0];
    const R inv = R(1) / r;
    const V4<R> v = {r, jx[i] * inv + R(0.5) * (gx + Fx), jy[i] * inv + R(0.5) * (gy + Fy),
                     jz[i] * inv + R(0.5) * (gz + Fz)};
    for_images(g, p, x, y, z, [&](int k) { ru1_p[k] = v; });
    fmf[i] = V4<R>{Fx, Fy, Fz, R(0)};
}

// ---------------------------------------------------------------------------
// k_shell: F^v = c_v sum_e k (k.W), A_ij = cA rho sum_e (k_j W_i + k_i W_j),
// W = gamma_mid rho(r+e) (u1(r+e) - u1(r)).
// A block owns a TX x TY x TZ tile.  The loop over the shell runs e_z = c
// from -R to R; for each c the (rho, u1) planes z0+c .. z0+c+TZ-1 of the
// tile plus an R-wide halo sit in an LDS ring of TZ+1 slots, the next plane
// is fetched while the current c is summed, and one barrier separates the
// c-steps.  gamma comes through L1/L2 from the padded array.  Blocks are
// ordered so that each XCD receives a contiguous run of tiles (shared halos
// stay in that XCD's L2).
// ---------------------------------------------------------------------------
template <typename R, int TX, int TY, int TZ, int NREG>
__global__ __launch_bounds__(TX *TY *TZ) void k_shell(Geom g, Pad p, int Rr, const V4<R> *__restrict__ ru1_p,
                                                      const R *__restrict__ gam_p, const V4<R> *__restrict__ fmf,
                                                      const Quad<R> *__restrict__ quads,
                                                      const int *__restrict__ qstart, R cv, R cA, R gx, R gy, R gz,
                                                      int smdb, int tiles_x, int tiles_y, int tiles_z,
                                                      R *__restrict__ Fo, R *__restrict__ Ao)
{
    constexpr int NT = TX * TY * TZ, NS = TZ + 1;
    extern __shared__ unsigned char lds_raw[];
    V4<R> *win = reinterpret_cast<V4<R> *>(lds_raw);
    const int LX = TX + 2 * Rr, LY = TY + 2 * Rr, LP = LX * LY;

    // XCD-aware tile order: hardware block id -> contiguous run per XCD
    const int nb = tiles_x * tiles_y * tiles_z;
    const int id = blockIdx.x, xcd = id & 7, qq = nb >> 3, rem = nb & 7;
    const int lid = (xcd < rem ? xcd * (qq + 1) : rem * (qq + 1) + (xcd - rem) * qq) + (id >> 3);
    const int x0 = (lid % tiles_x) * TX;
    const int t1 = lid / tiles_x;
    const int y0 = (t1 % tiles_y) * TY, z0 = (t1 / tiles_y) * TZ;

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    const bool valid = x < g.nx && y < g.ny && z < g.nz;

    // staging of one (rho, u1) plane of the tile plus halo, NREG float4 per
    // thread: element e of the plane is (ii, jj) = (e % LX, e / LX); the
    // offsets are fixed per thread, the plane moves
    int soff[NREG];
#pragma unroll
    for (int k = 0; k < NREG; ++k) {
        const int e = min(tid + k * NT, LP - 1);
        const int X = min(max(x0 - Rr + e % LX + p.P, 0), p.PX - 1);
        const int Y = min(max(y0 - Rr + e / LX + p.P, 0), p.PY - 1);
        soff[k] = Y * p.PX + X;
    }
#define WDLB_FETCH(pz)                                                                  \
    {                                                                                   \
        const long long zb_ = (long long)min(max((pz) + p.P, 0), p.PZ - 1) * p.PXY;    \
        _Pragma("unroll") for (int k_ = 0; k_ < NREG; ++k_) {                           \
            const V4<R> v_ = ru1_p[zb_ + soff[k_]];                                     \
            rx[k_] = v_.x;                                                              \
            ry[k_] = v_.y;                                                              \
            rz[k_] = v_.z;                                                              \
            rw[k_] = v_.w;                                                              \
        }                                                                               \
    }
#define WDLB_STORE(sl)                                                                  \
    {                                                                                   \
        const int sl_ = (sl);                                                           \
        _Pragma("unroll") for (int k_ = 0; k_ < NREG; ++k_) {                           \
            const int e_ = tid + k_ * NT;                                               \
            if (e_ < LP) win[sl_ * LP + e_] = V4<R>{rx[k_], ry[k_], rz[k_], rw[k_]};    \
        }                                                                               \
    }
    R rx[NREG], ry[NREG], rz[NREG], rw[NREG];
#pragma unroll
    for (int pk = 0; pk < TZ; ++pk) {
        WDLB_FETCH(z0 - Rr + pk);
        WDLB_STORE(pk);
    }
    __syncthreads();

    const int zc = min(z, g.nz - 1), yc = min(y, g.ny - 1), xc = min(x, g.nx - 1);
    const int gbase = pidx(p, xc, yc, zc);
    const V4<R> c0 = ru1_p[gbase];
    const int lbase = (ly + Rr) * LX + (lx + Rr);

    R vx = 0, vy = 0, vz = 0;
    R axx = 0, ayy = 0, azz = 0, axy = 0, axz = 0, ayz = 0;
    for (int c = -Rr; c <= Rr; ++c) {
        const bool more = c < Rr;
        if (more) WDLB_FETCH(z0 + c + TZ);
        const V4<R> *pl = win + ((lz + c + Rr) % NS) * LP + lbase;
        const int qb = qstart[c + Rr], qe = qstart[c + Rr + 1];
        for (int q = qb; q < qe; ++q) {
            const Quad<R> Qd = quads[q];
            const int a = Qd.a, bb = Qd.b;
            int so[4], mo[4];
            quad_offsets(a, bb, Qd.c, p.PX, p.PXY, so, mo);
            const int lo[4] = {a + bb * LX, -a + bb * LX, a - bb * LX, -a - bb * LX};
            const R *gb = gam_p + (long long)Qd.hidx * p.NP + gbase;
            R x0_, xX, xY, xXY, y0_, yX, yY, yXY, z0_, zX, zY;
            {
                // mirror products and Hadamard without FMA fusion (exact
                // zeros for identical mirror images)
#pragma clang fp contract(off)
                R Wx[4], Wy[4], Wz[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const V4<R> s = pl[lo[m]];
                    const R G = gb[mo[m]] * s.x;
                    Wx[m] = G * (s.y - c0.y);
                    Wy[m] = G * (s.z - c0.z);
                    Wz[m] = G * (s.w - c0.w);
                }
                // Hadamard transform over the mirror signs (sx, sy)
                const R xP1 = Wx[0] + Wx[1], xM1 = Wx[0] - Wx[1], xP2 = Wx[2] + Wx[3], xM2 = Wx[2] - Wx[3];
                const R yP1 = Wy[0] + Wy[1], yM1 = Wy[0] - Wy[1], yP2 = Wy[2] + Wy[3], yM2 = Wy[2] - Wy[3];
                const R zP1 = Wz[0] + Wz[1], zM1 = Wz[0] - Wz[1], zP2 = Wz[2] + Wz[3], zM2 = Wz[2] - Wz[3];
                x0_ = xP1 + xP2;
                xX = xM1 + xM2;
                xY = xP1 - xP2;
                xXY = xM1 - xM2;
                y0_ = yP1 + yP2;
                yX = yM1 + yM2;
                yY = yP1 - yP2;
                yXY = yM1 - yM2;
                z0_ = zP1 + zP2;
                zX = zM1 + zM2;
                zY = zP1 - zP2;
            }
            vx += Qd.qxx * x0_ + Qd.qxy * yXY + Qd.qxz * zX;
            vy += Qd.qxy * xXY + Qd.qyy * y0_ + Qd.qyz * zY;
            vz += Qd.qxz * xX + Qd.qyz * yY + Qd.qzz * z0_;
            axx += Qd.px * xX;
            ayy += Qd.py * yY;
            azz += Qd.pz * z0_;
            axy += Qd.py * xY + Qd.px * yX;
            axz += Qd.pz * x0_ + Qd.px * zX;
            ayz += Qd.pz * y0_ + Qd.py * zY;
        }
        if (more) WDLB_STORE((c + TZ + Rr) % NS);
        __syncthreads();
    }
#undef WDLB_FETCH
#undef WDLB_STORE
    if (!valid) return;
    const long long N = g.N;
    const int i = (z * g.ny + y) * g.nx + x;
    const R r0 = c0.x;
    const V4<R> fm = fmf[i];
    Fo[i] = r0 * (gx + fm.x + cv * vx);
    Fo[N + i] = r0 * (gy + fm.y + cv * vy);
    Fo[2 * N + i] = r0 * (gz + fm.z + cv * vz);
    R Axx = 0, Ayy = 0, Azz = 0, Axy = 0, Axz = 0, Ayz = 0;
    if (smdb) {
        const R ca = cA * r0;
        Axx = ca * R(2) * axx;
        Ayy = ca * R(2) * ayy;
        Azz = ca * R(2) * azz;
        Axy = ca * axy;
        Axz = ca * axz;
        Ayz = ca * ayz;
        const R tr = (Axx + Ayy + Azz) / R(3);
        Axx -= tr;
        Ayy -= tr;
        Azz -= tr;
    }
    Ao[i] = Axx;
    Ao[N + i] = Ayy;
    Ao[2 * N + i] = Azz;
    Ao[3 * N + i] = Axy;
    Ao[4 * N + i] = Axz;
    Ao[5 * N + i] = Ayz;
}

// F (3N) and A (xx, yy, zz, xy, xz, yz; 6N) for nonlocal = 0: F = rho g
template <typename R>
__global__ __launch_bounds__(256) void k_plainforce(Geom g, Pad p, const R *__restrict__ rho_p, R gx, R gy, R gz,
                                                    R *__restrict__ Fo, R *__restrict__ Ao)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const R r = rho_p[pidx(p, x, y, z)];
    const long long N = g.N;
    Fo[i] = r * gx;
    Fo[N + i] = r * gy;
    Fo[2 * N + i] = r * gz;
    for (int k = 0; k < 6; ++k) Ao[k * N + i] = R(0);
}

// Forced BGK with the SMDB source (trapezoidal weighting ksrc = 1 - 1/(2 tau)),
// stored against the post-collision velocity u* = u + F/(2 rho):
//   h*_a = (1 - omega)(f_a - feq_a(u)) + [feq_a(u) - feq_a(u*)] + ksrc (guo_a + sa_a)
// so the deviation carries no momentum and the flow lives in u* alone.
// READ: only u = (j + F/2)/rho is written (the fields of the current state).
template <typename R, typename HS, bool READ>
__global__ __launch_bounds__(256) void k_collide(Geom g, const R *__restrict__ Fi, const R *__restrict__ Ai,
                                                 R omega, R ksrc, const V4<R> *__restrict__ ru_in,
                                                 const HS *__restrict__ h_in, V4<R> *__restrict__ ru_out,
                                                 HS *__restrict__ h_out, R *__restrict__ u_rd)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const long long N = g.N;
    D rho, jx, jy, jz;
    pull_moments<R, HS>(g, ru_in, h_in, x, y, z, rho, jx, jy, jz);
    const D inv = D(1) / rho;
    const D Fx = Fi[i], Fy = Fi[N + i], Fz = Fi[2 * N + i];
    const D ux = (jx + D(0.5) * Fx) * inv, uy = (jy + D(0.5) * Fy) * inv, uz = (jz + D(0.5) * Fz) * inv;
    if (READ) {
        u_rd[i] = R(ux);
        u_rd[N + i] = R(uy);
        u_rd[2 * N + i] = R(uz);
        return;
    }
    const D Axx = Ai[i], Ayy = Ai[N + i], Azz = Ai[2 * N + i], Axy = Ai[3 * N + i], Axz = Ai[4 * N + i],
            Ayz = Ai[5 * N + i];
    const D uu = ux * ux + uy * uy + uz * uz;
    const D uF = ux * Fx + uy * Fy + uz * Fz;
    const D keep = D(1) - D(omega), ks = D(ksrc);
    const D dx = D(0.5) * Fx * inv, dy = D(0.5) * Fy * inv, dz = D(0.5) * Fz * inv;  // u* - u
    const D sx = D(2) * ux + dx, sy = D(2) * uy + dy, sz = D(2) * uz + dz;          // u + u*
    const D dsum = dx * sx + dy * sy + dz * sz;
    const int r = (z * g.ny + y) * g.nx + x;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const D w = wgt<D>(a);
        const D cu = D(CX[a]) * ux + D(CY[a]) * uy + D(CZ[a]) * uz;
        const D P = D(3) * cu + D(4.5) * cu * cu - D(1.5) * uu;
        const D fneq = fpull<R, HS>(g, ru_in, h_in, x, y, z, r, a) - w * rho * (D(1) + P);
        const D cF = D(CX[a]) * Fx + D(CY[a]) * Fy + D(CZ[a]) * Fz;
        const D guo = w * (D(3) * (cF - uF) + D(9) * cu * cF);
        const D cAc = D(CX[a] * CX[a]) * Axx + D(CY[a] * CY[a]) * Ayy + D(CZ[a] * CZ[a]) * Azz +
                      D(2 * CX[a] * CY[a]) * Axy + D(2 * CX[a] * CZ[a]) * Axz + D(2 * CY[a] * CZ[a]) * Ayz;
        const D sa = D(4.5) * w * cAc;
        const D cd = D(CX[a]) * dx + D(CY[a]) * dy + D(CZ[a]) * dz;
        const D cs = D(CX[a]) * sx + D(CY[a]) * sy + D(CZ[a]) * sz;
        const D deq = w * rho * (-D(3) * cd - D(4.5) * cd * cs + D(1.5) * dsum);
        sth<R, HS>(h_out + (long long)a * N + i, R(keep * fneq + deq + ks * (guo + sa)));
    }
    ru_out[i] = V4<R>{R(rho), R(ux + dx), R(uy + dy), R(uz + dz)};
}

// the post-stream populations a0 .. a0+7 (those below Q) into f[(a - a0) N + i]
template <typename R, typename HS>
__global__ __launch_bounds__(256) void k_populations(Geom g, const V4<R> *__restrict__ ru, const HS *__restrict__ h,
                                                     int a0, R *__restrict__ f)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    const int r = (z * g.ny + y) * g.nx + x;
#pragma unroll
    for (int a = 0; a < Q; ++a)
        if (a >= a0 && a < a0 + 8) f[(long long)(a - a0) * g.N + i] = R(fpull<R, HS>(g, ru, h, x, y, z, r, a));
}

// FP64 plane sums of rho, u_x and rho*u_x; one block per z-plane, fixed
// reduction order (deterministic)
template <typename R>
__global__ __launch_bounds__(256) void k_planes(Geom g, Pad p, const R *__restrict__ rho_p,
                                                const R *__restrict__ ux, double *__restrict__ out)
{
    __shared__ double sh[3][256];
    const int z = blockIdx.x;
    const int plane = g.nx * g.ny;
    double a = 0, b = 0, c = 0;
    for (int k = threadIdx.x; k < plane; k += blockDim.x) {
        const int x = k % g.nx, y = k / g.nx;
        const double r = (double)rho_p[pidx(p, x, y, z)], u = (double)ux[z * plane + k];
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

// copy the density out of the padded array (reads)
template <typename R>
__global__ __launch_bounds__(256) void k_unpad(Geom g, Pad p, const R *__restrict__ src, R *__restrict__ dst)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    dst[i] = src[pidx(p, x, y, z)];
}

}  // namespace wdlb
