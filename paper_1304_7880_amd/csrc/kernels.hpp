// kernels.hpp -- the gfx950 kernels of one WDLB step.  Device code only;
// included by wdlb.hip.
//
// One step (Sec. 5 of the paper, steps 2-4) is six kernels:
//   k_moments    pull-stream the stored populations; density (padded array,
//                with periodic images) and momentum
//   k_density    Fischer-Methfessel smoothed density nbar (ball
//                |e| <= sigma/2) and the Carnahan-Starling contact value at
//                the 8 half-lattice midpoints of every node,
//                gamma_h(r) = g_CS(nbar(r + h/2)); nbar stays in LDS
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
// Padded arrays.  rho, gamma and (rho, u1) live in arrays padded by P
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
#include <type_traits>
#include <utility>

#include "d3q19.hpp"
#include "shell.hpp"

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

// h_a of node s (plane a of N); see closure_slot for the BF16 planes
template <typename R, typename HS>
__device__ __forceinline__ R ldh(const HS *h, int a, long long N, long long s)
{
    return h[a * N + s];
}
template <>
__device__ __forceinline__ float ldh<float, bf16>(const bf16 *h, int a, long long N, long long s)
{
    const uint16_t hi = h[a * N + s].bits;
    const int k = closure_slot(a);
    if (k < 0) return bf16_to_f32(hi);
    const uint16_t lo = h[(19 + k) * N + s].bits;
    return __uint_as_float((uint32_t(hi) << 16) | uint32_t(lo));
}

// store h_a of node i: FP32/FP64 as is; BF16 rounded, except the closure
// populations, which keep their FP32 value exactly
template <typename R, typename HS>
__device__ __forceinline__ void sth(HS *h, int a, long long N, long long i, R v)
{
    h[a * N + i] = v;
}
template <>
__device__ __forceinline__ void sth<float, bf16>(bf16 *h, int a, long long N, long long i, float v)
{
    const int k = closure_slot(a);
    if (k < 0) {
        h[a * N + i].bits = f32_to_bf16(v);
    } else {
        const uint32_t u = __float_as_uint(v);
        h[a * N + i].bits = uint16_t(u >> 16);
        h[(19 + k) * N + i].bits = uint16_t(u & 0xffffu);
    }
}

__device__ __forceinline__ void raise_flag(int *flag, int bit)
{
    __hip_atomic_fetch_or(flag, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// flag[0] for the lattice and, in a stacked lattice, flag[1 + z] for plane z
// (which slit went bad)
__device__ __forceinline__ void raise_flag_at(const Geom &g, int *flag, int z, int bit)
{
    raise_flag(flag, bit);
    if (g.zp != nullptr) raise_flag(flag + 1 + z, bit);
}

// the body force of plane z: the slit's own in a stacked lattice, else the
// lattice's (passed in)
template <typename R>
__device__ __forceinline__ void plane_force(const Geom &g, int z, R &gx, R &gy, R &gz)
{
    if (g.zp != nullptr) {
        gx = R(g.zp[z].gx);
        gy = R(g.zp[z].gy);
        gz = R(g.zp[z].gz);
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

// XCD-aware tile order: consecutive hardware block ids go to different XCDs
// (round robin), so block id -> tile index gives each XCD a contiguous run of
// tiles and the halos they share stay in that XCD's L2
__device__ __forceinline__ int xcd_tile(int id, int nb)
{
    const int xcd = id & 7, qq = nb >> 3, rem = nb & 7;
    return (xcd < rem ? xcd * (qq + 1) : rem * (qq + 1) + (xcd - rem) * qq) + (id >> 3);
}

struct TileCoord {
    int x0, y0, z0, lx, ly, lz;
};

// Within an XCD's run, tiles go x fastest, so that the tiles in flight read
// the same planes at the same time.  With ZF (kernels whose tiles are one
// plane deep) they go z fastest once a plane of tiles is large (128 tiles or
// more): the tiles in flight are then z-neighbours whose stencil windows
// share all but one plane, and that column of windows fits in an XCD's L2.
template <int TX, int TY, int TZ, bool ZF = false>
__device__ __forceinline__ TileCoord tile_coord(int tiles_x, int tiles_y, int tiles_z)
{
    TileCoord t;
    const int lid = xcd_tile(blockIdx.x, tiles_x * tiles_y * tiles_z);
    if (ZF && tiles_x * tiles_y >= 128) {
        const int t1 = lid / tiles_z;
        t.z0 = (lid % tiles_z) * TZ;
        t.x0 = (t1 % tiles_x) * TX;
        t.y0 = (t1 / tiles_x) * TY;
    } else {
        const int t1 = lid / tiles_x;
        t.x0 = (lid % tiles_x) * TX;
        t.y0 = (t1 % tiles_y) * TY;
        t.z0 = (t1 / tiles_y) * TZ;
    }
    t.lx = threadIdx.x % TX;
    t.ly = (threadIdx.x / TX) % TY;
    t.lz = threadIdx.x / (TX * TY);
    return t;
}

// The node of a thread in the per-node kernels (moments, collide): blocks of
// 256 threads cover (1 << lgx) x (256 >> lgx) tiles in x, y of one plane,
// and the blocks of one XCD (consecutive in xcd_tile order) take the planes
// of one tile in turn, so the planes z -+ 1 that a pull reads were fetched
// into that XCD's L2 by its previous blocks.
struct NodeTiles {
    int tx, ty, nzr, lgx;  // tiles in x and y, planes, log2 of the tile width
};

__device__ __forceinline__ bool node_tiled(const Geom &g, const NodeTiles &t, int &x, int &y, int &z, long long &i)
{
    const int lid = xcd_tile(blockIdx.x, t.tx * t.ty * t.nzr);
    z = lid % t.nzr;
    const int tt = lid / t.nzr;
    x = ((tt % t.tx) << t.lgx) + ((int)threadIdx.x & ((1 << t.lgx) - 1));
    y = (tt / t.tx) * (256 >> t.lgx) + ((int)threadIdx.x >> t.lgx);
    if (x >= g.nx || y >= g.ny) return false;
    i = ((long long)z * g.ny + y) * g.nx + x;
    return true;
}

// ---------------------------------------------------------------------------
// pull: the population arriving at (x, y, z) with velocity c_a,
//   f_a = w_a rho_s (1 + P_a(u*_s)) + h_a(s),
// from the source s = r - c_a, or by half-way bounce-back from r itself.
// The local kernels (moments, collision) work with
//   phi_a = f_a - w_a rho_r = w_a (rho_s - rho_r) + [w_a rho_s P_a(u*_s) + h_a(s)],
// rho_r the node's own stored density: every term is small, so sums of phi
// keep their absolute accuracy in FP32 (the large w_a rho parts cancel
// exactly in the difference rho_s - rho_r instead of in a sum of 19
// populations of size w rho, which would lose the flow to rounding).  Then
//   rho = rho_r + sum_a phi_a,  j = sum_a c_a phi_a,
//   f_a - feq_a(rho, u) = phi_a - w_a (delta + rho P_a(u)),  delta = rho - rho_r.
// D is the arithmetic type of these kernels: the storage type, or FP64 with
// FP32 storage in the modes that keep FP64 local arithmetic.
// ---------------------------------------------------------------------------

// The neighbours a node pulls from, found once per node: the wrapped
// coordinates x -+ 1, y -+ 1, z -+ 1 and whether the planes z - 1 and z + 1
// are fluid (bbm, bbp: a population arriving from a non-fluid plane is
// bounced back at the node itself).  With them every pull is straight-line
// code, so the compiler can issue all 19 pairs of loads before it waits.
struct PullNbr {
    int xm, xp, ym, yp, zm, zp;
    bool bbm, bbp;
};

__device__ __forceinline__ PullNbr pull_nbr(const Geom &g, int x, int y, int z)
{
    PullNbr n;
    n.xm = wrap1(x - 1, g.nx);
    n.xp = wrap1(x + 1, g.nx);
    n.ym = wrap1(y - 1, g.ny);
    n.yp = wrap1(y + 1, g.ny);
    if (g.walls) {
        n.zm = z - 1;
        n.zp = z + 1;
        n.bbm = !zfluid(g, z - 1);
        n.bbp = !zfluid(g, z + 1);
    } else {
        n.zm = wrap1(z - 1, g.nz);
        n.zp = wrap1(z + 1, g.nz);
        n.bbm = n.bbp = false;
    }
    return n;
}

// phi_a of the node r (see above); rho_r is the node's stored density
template <typename R, typename HS, typename D>
__device__ __forceinline__ D fpull_phi(const Geom &g, const V4<R> *__restrict__ ru, const HS *__restrict__ h,
                                       const PullNbr &n, int x, int y, int z, int r, int a, R rho_r)
{
    // source s = r - c_a
    const int sx = CX[a] > 0 ? n.xm : (CX[a] < 0 ? n.xp : x);
    const int sy = CY[a] > 0 ? n.ym : (CY[a] < 0 ? n.yp : y);
    const int sz = CZ[a] > 0 ? n.zm : (CZ[a] < 0 ? n.zp : z);
    const bool bb = CZ[a] > 0 ? n.bbm : (CZ[a] < 0 ? n.bbp : false);
    const int s = bb ? r : (sz * g.ny + sy) * g.nx + sx;
    const int ha = bb ? OPP[a] : a;
    const V4<R> q = ru[s];
    const D ux = q.y, uy = q.z, uz = q.w;
    D cu = D(CX[a]) * ux + D(CY[a]) * uy + D(CZ[a]) * uz;
    if (bb) cu = -cu;
    const D P = D(3) * cu + D(4.5) * cu * cu - D(1.5) * (ux * ux + uy * uy + uz * uz);
    const D w = wgt<D>(a);
    return w * (D(q.x) - D(rho_r)) + (w * D(q.x) * P + D(ldh<R, HS>(h, ha, g.N, s)));
}

// delta = rho - rho_r and j of the node from its 19 pulled populations
template <typename R, typename HS, typename D>
__device__ __forceinline__ void pull_moments(const Geom &g, const V4<R> *__restrict__ ru, const HS *__restrict__ h,
                                             int x, int y, int z, R &rho_r, D &delta, D &jx, D &jy, D &jz)
{
    const int r = (z * g.ny + y) * g.nx + x;
    const PullNbr n = pull_nbr(g, x, y, z);
    rho_r = ru[r].x;
    delta = jx = jy = jz = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const D f = fpull_phi<R, HS, D>(g, ru, h, n, x, y, z, r, a, rho_r);
        delta += f;
        if (CX[a]) jx += D(CX[a]) * f;
        if (CY[a]) jy += D(CY[a]) * f;
        if (CZ[a]) jz += D(CZ[a]) * f;
    }
}

// ---------------------------------------------------------------------------
// step 1 (initialisation)
// ---------------------------------------------------------------------------
// nodes i0 .. i0 + cnt - 1 (a whole lattice, or the planes of one slit of a
// stacked lattice)
template <typename R>
__global__ __launch_bounds__(256) void k_fill(Geom g, V4<R> *ru, R n0, R ux, R uy, R uz, long long i0, long long cnt)
{
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) ru[i0 + t] = V4<R>{n0, ux, uy, uz};
}

// The populations at every node r are feq(n(r), u(r)).  The library stores
// pre-stream populations, so node s keeps for direction a the value that the
// next pull delivers to t = s + c_a, feq_a(n(t), u(t)), or, when t lies in a
// wall, the value that bounces back into s itself, feq_abar(n(s), u(s)); h
// is that minus feq_a(n(s), u(s)).
template <typename R, typename HS>
__global__ __launch_bounds__(256) void k_init(Geom g, const V4<R> *__restrict__ ru, HS *__restrict__ h, long long i0,
                                              long long cnt)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const long long i = i0 + t;
    int x, y, z;
    if (!node_of(g, i, x, y, z)) return;
    using D = double;  // once per run: FP64 in every mode
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
            if (g.walls) bb = !zfluid(g, tz);
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
        sth<R, HS>(h, a, g.N, i, R(val));
    }
}

// ---------------------------------------------------------------------------
// steps 2-4
// ---------------------------------------------------------------------------
template <typename R, typename HS, typename D>
__global__ __launch_bounds__(256) void k_moments(Geom g, NodeTiles nt, Pad p, const V4<R> *__restrict__ ru,
                                                 const HS *__restrict__ h, R *__restrict__ rho_p,
                                                 R *__restrict__ jx, R *__restrict__ jy, R *__restrict__ jz,
                                                 int *flag)
{
    long long i;
    int x, y, z;
    if (!node_tiled(g, nt, x, y, z, i)) return;
    if (!zfluid(g, z)) {  // a gap plane of a stacked lattice: rho = 0 for every stencil
        for_images(g, p, x, y, z, [&](int k) { rho_p[k] = R(0); });
        jx[i] = jy[i] = jz[i] = R(0);
        return;
    }
    R r0;
    D dl, a, b, c;
    pull_moments<R, HS, D>(g, ru, h, x, y, z, r0, dl, a, b, c);
    const D r = D(r0) + dl;
    if (!(r > D(0)) || !(r < D(INFINITY))) raise_flag_at(g, flag, z, FLAG_RHO);
    const R rr = R(r);
    for_images(g, p, x, y, z, [&](int k) { rho_p[k] = rr; });
    jx[i] = R(a);
    jy[i] = R(b);
    jz[i] = R(c);
}

// The sums of a c-step are finished before its barrier: an empty asm that
// reads and writes the accumulator keeps the compiler from sinking the
// arithmetic of every c-step to the end of the kernel (which would keep all
// loaded operands of the whole shell live at once).  It emits no code.
__device__ __forceinline__ void pin(float &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }

template <int B, typename F, int... I>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, B + I>{}), ...);
}
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (E > B) static_for_seq<B>(f, std::make_integer_sequence<int, E - B>{});
}

// ---------------------------------------------------------------------------
// k_density: the smoothed density and the contact values in one pass over
// TX x TY x TZ tiles.  LDS holds rho over the tile plus the ball reach rb on
// every side and one more node on the high side of each axis; nbar is formed
// there for the tile plus that extra layer (the 2^3 corners of every
// half-lattice point), then gamma_h for the tile's nodes.  nbar never goes
// to memory.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr size_t density_lds_bytes(int TX, int TY, int TZ, int rb, size_t rbytes)
{
    return ((size_t)(TX + 2 * rb + 1) * (TY + 2 * rb + 1) * (TZ + 2 * rb + 1) + (size_t)(TX + 1) * (TY + 1) * (TZ + 1)) *
               rbytes +
           (size_t)(TZ + 1) * sizeof(int);  // fluid flags of the nbar planes
}

// rho over the tile, the ball reach and one extra node (from the padded
// array: images and zeros beyond the walls are in place), and the fluid flag
// of each of the TZ + 1 nbar planes (zfl).  The window is fetched in rounds
// of 8 elements per lane, all 8 loads issued before the first is stored; a
// load and its store take the same branch, so that the compiler does not
// sink the load next to the store (one load latency per round).
template <typename R, int NT, int TZ>
__device__ __forceinline__ void density_fill(const Geom &g, const TileCoord &tc, const Pad &p, int rb, int LX, int LY,
                                             int LZ, const R *__restrict__ rho_p, R *win, int *zfl)
{
    const int NE = LX * LY * LZ;
    const int t0 = threadIdx.x;
    // NE > NT (the window holds the tile and more), so every lane runs the first round
    for (int e0 = t0; e0 < NE; e0 += 8 * NT) {
        R v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * NT;
            if (e < NE) {
                const int ix = e % LX, t = e / LX, iy = t % LY, iz = t / LY;
                const int X = min(max(tc.x0 - rb + ix + p.P, 0), p.PX - 1);
                const int Y = min(max(tc.y0 - rb + iy + p.P, 0), p.PY - 1);
                const int Z = min(max(tc.z0 - rb + iz + p.P, 0), p.PZ - 1);
                v[u] = rho_p[(long long)Z * p.PXY + (long long)Y * p.PX + X];
            }
        }
        // in the first round, behind the window loads: the plane flags
        if (e0 == t0 && t0 <= TZ) zfl[t0] = !g.walls || zfluid(g, tc.z0 + t0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * NT;
            if (e < NE) win[e] = v[u];
        }
    }
}

// gamma_h of the lane's node from nbar at the 8 corners of its half-lattice
// points (m0: nbar of the node in the (TX+1)(TY+1)(TZ+1) block), written
// with the node's periodic images
template <typename R, int TX, int TY>
__device__ __forceinline__ void density_gamma(const Geom &g, const Pad &p, int x, int y, int z, const R *m0,
                                              R eta_per_n, R wS, R *__restrict__ gam_p, int *flag)
{
    constexpr int DX = 1, DY = TX + 1, DZ = (TX + 1) * (TY + 1);
    const R n000 = m0[0], n100 = m0[DX], n010 = m0[DY], n110 = m0[DX + DY];
    const R n001 = m0[DZ], n101 = m0[DZ + DX], n011 = m0[DZ + DY], n111 = m0[DZ + DY + DX];
    const bool zin = !g.walls || zfluid(g, z + 1);  // the upper corners lie in the slit
    R m[8];
    m[0] = n000;
    m[1] = (n000 + n100) * R(0.5);
    m[2] = (n000 + n010) * R(0.5);
    m[3] = ((n000 + n100) + (n010 + n110)) * R(0.25);
    m[4] = (n000 + n001) * R(0.5);
    m[5] = ((n000 + n100) + (n001 + n101)) * R(0.25);
    m[6] = ((n000 + n010) + (n001 + n011)) * R(0.25);
    m[7] = (((n000 + n100) + (n010 + n110)) + ((n001 + n101) + (n011 + n111))) * R(0.125);
    R val[8];
    bool bad = false;
#pragma unroll
    for (int hi = 0; hi < 8; ++hi) {
        const R eta = eta_per_n * m[hi];
        if (eta < R(1)) {
            const R om = R(1) - eta;
            val[hi] = wS * (R(1) - R(0.5) * eta) / (om * om * om);
        } else {
            bad = bad || hi < 4 || zin;
            val[hi] = R(0);
        }
    }
    if (bad) raise_flag_at(g, flag, z, FLAG_ETA);
    for_images(g, p, x, y, z, [&](int k) {
#pragma unroll
        for (int hi = 0; hi < 8; ++hi) gam_p[(long long)hi * p.NP + k] = val[hi];
    });
}

// nbar over the (TX+1)(TY+1)(TZ+1) block: first the tile's TX columns (lanes
// of a half-wave on one row of the window: no LDS bank conflicts), then the
// extra column mx = TX
template <int TX, int TY, int TZ, typename F>
__device__ __forceinline__ void density_nbar_sweep(F &&nbar_at)
{
    constexpr int NT = TX * TY * TZ, MY = TY + 1, MZ = TZ + 1;
    for (int e = threadIdx.x; e < TX * MY * MZ; e += NT) {
        const int t = e / TX;
        nbar_at(e % TX, t % MY, t / MY);
    }
    for (int e = threadIdx.x; e < MY * MZ; e += NT) nbar_at(TX, e % MY, e / MY);
}

// generic: the ball from its table of window offsets (relative to the
// corner of a node's ball window; order z, then y, then x), summed into 8
// interleaved partial sums, point k into sum k mod 8 (the order of the
// specialised kernel, so both give the same bits)
template <typename R, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_density(Geom g, Pad p, int rb, const R *__restrict__ rho_p,
                                                        const int *__restrict__ boff, int nball, R inv_nball,
                                                        R eta_per_n, R wS, int tiles_x, int tiles_y, int tiles_z,
                                                        R *__restrict__ gam_p, int *flag)
{
    constexpr int NT = TX * TY * TZ;
    constexpr int MX = TX + 1, MY = TY + 1, MZ = TZ + 1, MN = MX * MY * MZ;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ>(tiles_x, tiles_y, tiles_z);
    const int LX = TX + 2 * rb + 1, LY = TY + 2 * rb + 1, LZ = TZ + 2 * rb + 1, LXY = LX * LY;
    R *win = reinterpret_cast<R *>(lds_raw);
    R *nb = win + (size_t)LX * LY * LZ;
    int *zfl = reinterpret_cast<int *>(nb + MN);
    density_fill<R, NT, TZ>(g, tc, p, rb, LX, LY, LZ, rho_p, win, zfl);
    __syncthreads();
    auto nbar_at = [&](int mx, int my, int mz) {
        R v = 0;
        if (zfl[mz]) {
            const R *c = win + mz * LXY + my * LX + mx;
            R s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int k = 0;
            for (; k + 8 <= nball; k += 8) {
#pragma unroll
                for (int m = 0; m < 8; ++m) s[m] += c[boff[k + m]];
            }
#pragma unroll
            for (int m = 0; m < 7; ++m)
                if (k + m < nball) s[m] += c[boff[k + m]];
            v = (((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]))) * inv_nball;
        }
        nb[(mz * MY + my) * MX + mx] = v;
    };
    density_nbar_sweep<TX, TY, TZ>(nbar_at);
    __syncthreads();
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    density_gamma<R, TX, TY>(g, p, x, y, z, nb + (tc.lz * MY + tc.ly) * MX + tc.lx, eta_per_n, wS, gam_p, flag);
}

// the union table of the ball's column of MZ points, as a constant
template <int S2, int MZ>
struct Column {
    static constexpr BallColumn<S2, MZ> T{};
};

// specialised for the ball of 2 sigma = S2: offsets are LDS immediates, the
// sum runs in 8 interleaved partial sums
template <typename R, int S2, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX *TY *TZ) void k_density_s(Geom g, Pad p, const R *__restrict__ rho_p, R inv_nball,
                                                          R eta_per_n, R wS, int tiles_x, int tiles_y, int tiles_z,
                                                          R *__restrict__ gam_p, int *flag)
{
    using B = Ball<S2>;
    constexpr int rb = B::RB, NT = TX * TY * TZ;
    constexpr int MX = TX + 1, MY = TY + 1, MZ = TZ + 1, MN = MX * MY * MZ;
    constexpr int LX = TX + 2 * rb + 1, LY = TY + 2 * rb + 1, LZ = TZ + 2 * rb + 1, LXY = LX * LY;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ>(tiles_x, tiles_y, tiles_z);
    R *win = reinterpret_cast<R *>(lds_raw);
    R *nb = win + (size_t)LX * LY * LZ;
    int *zfl = reinterpret_cast<int *>(nb + MN);
    density_fill<R, NT, TZ>(g, tc, p, rb, LX, LY, LZ, rho_p, win, zfl);
    __syncthreads();
    // a lane forms nbar for the column (mx, my) of all MZ planes: the union
    // of the MZ stacked balls is read once, each value added into the
    // partial sums of every point whose ball holds it; a point's terms
    // arrive in its ball order, into sum k mod 8, as in the one-point sum
    using BC = BallColumn<S2, MZ>;
    static_assert(BC::NU > 0, "ball column table");
    auto nbar_col = [&](int mx, int my) __attribute__((always_inline)) {
        const R *c = win + my * LX + mx;  // corner of the ball window of the column's lowest point
        R s[MZ][8];
#pragma unroll
        for (int j = 0; j < MZ; ++j)
#pragma unroll
            for (int m = 0; m < 8; ++m) s[j][m] = R(0);
        static_for<0, BC::NU>([&](auto ui) __attribute__((always_inline)) {
            constexpr int u = decltype(ui)::value;
            using CT = Column<S2, MZ>;
            // one window row (z, y) at a time: the sums of a row are finished
            // and no load is hoisted above the start of its row, which bounds
            // the values in flight
            if constexpr (u > 0 && (CT::T.z[u] != CT::T.z[u - 1] || CT::T.y[u] != CT::T.y[u - 1])) {
#pragma unroll
                for (int j = 0; j < MZ; ++j)
#pragma unroll
                    for (int m = 0; m < 8; ++m) pin(s[j][m]);
                asm volatile("" ::: "memory");
            }
            const R v = c[(CT::T.z[u] + rb) * LXY + (CT::T.y[u] + rb) * LX + (CT::T.x[u] + rb)];
            static_for<0, MZ>([&](auto ji) __attribute__((always_inline)) {
                constexpr int j = decltype(ji)::value;
                constexpr int k = CT::T.k[u][j];
                if constexpr (k >= 0) s[j][k & 7] += v;
            });
        });
#pragma unroll
        for (int j = 0; j < MZ; ++j) {
            const R v = zfl[j] ? (((s[j][0] + s[j][1]) + (s[j][2] + s[j][3])) +
                                  ((s[j][4] + s[j][5]) + (s[j][6] + s[j][7]))) * inv_nball
                               : R(0);
            nb[(j * MY + my) * MX + mx] = v;
        }
    };
    // the tile's TX columns first (lanes of a half-wave on one window row:
    // no bank conflicts), then the extra column mx = TX
    for (int e = threadIdx.x; e < TX * MY + MY; e += NT) {
        if (e < TX * MY) nbar_col(e % TX, e / TX);
        else nbar_col(TX, e - TX * MY);
    }
    __syncthreads();
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    density_gamma<R, TX, TY>(g, p, x, y, z, nb + (tc.lz * MY + tc.ly) * MX + tc.lx, eta_per_n, wS, gam_p, flag);
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

// ---------------------------------------------------------------------------
// Contact-shell tiles (k_meanfield, k_shell).  A block owns a TX x TY x TZ
// tile and runs over the shell as e_z = c from -R to R.  Two LDS rings
// advance by one entry per c-step:
//  - planes z0+c .. z0+c+TZ-1 of rho (k_meanfield) or of (rho, u1)
//    (k_shell) over the tile plus an R-wide halo: TZ + 1 slots;
//  - slices of the contact value.  Slice t = 2j + hz holds, for the padded
//    z-plane z0 + j and z-parity hz, the four (x, y)-parity sub-lattices
//    gamma_h over the tile plus the half-reach halo.  The half-lattice point
//    r + e/2 of a node in tile plane lz lies in slice c + 2 lz, so step c
//    reads slices c .. c + 2(TZ-1): 2 TZ slots with the one being fetched.
// The next plane and slice are fetched into registers while the current c
// is summed and stored after it; one barrier separates the c-steps.  With
// NG = 0 gamma is read through L1/L2 from the padded arrays instead (tiles
// whose rings do not fit in LDS).  Blocks are ordered so that each XCD gets
// a contiguous run of tiles (shared halos stay in that XCD's L2).
// ---------------------------------------------------------------------------
// the gamma ring of one block: element e of a slice is sub-lattice
// e / LG, row (e % LG) / LXg, column (e % LG) % LXg of the window whose
// origin is the tile origin shifted by floor(-R/2) in x and y
template <typename R, int NT, int NG>
struct GammaRing {
    int LXg, LG, LS;
    int gh[NG], goff[NG];
    R st[2][NG];  // two staging sets: one in flight while the other is stored

    __device__ __forceinline__ void setup(const Pad &p, int Rr, int TX, int TY, int x0, int y0)
    {
        const int o = -((Rr + 1) >> 1);
        LXg = TX + Rr;
        LG = LXg * (TY + Rr);
        LS = 4 * LG;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int e = min((int)threadIdx.x + k * NT, LS - 1);
            gh[k] = e / LG;
            const int rem = e - gh[k] * LG;
            const int X = min(max(x0 + o + rem % LXg + p.P, 0), p.PX - 1);
            const int Y = min(max(y0 + o + rem / LXg + p.P, 0), p.PY - 1);
            goff[k] = Y * p.PX + X;
        }
    }
    // slice t (plane z0 + floor(t/2), z-parity t & 1) into registers d
    __device__ __forceinline__ void fetch_to(R (&d)[NG], const R *__restrict__ gam_p, const Pad &p, int z0, int t)
    {
        const int hz = t & 1;
        const long long zb = (long long)min(max(z0 + (t >> 1) + p.P, 0), p.PZ - 1) * p.PXY;
#pragma unroll
        for (int k = 0; k < NG; ++k) d[k] = gam_p[(long long)(gh[k] + 4 * hz) * p.NP + zb + goff[k]];
    }
    // With GUARD the fetch takes the store's branch per element: unguarded,
    // the compiler may sink a fetch into that branch, to the end of the step
    // (where store() runs), and expose its whole latency there.  That costs
    // a step with one step of prefetch (PD = 1); with PD = 2 it does not.
    template <int S, bool GUARD>
    __device__ __forceinline__ void fetch(const R *__restrict__ gam_p, const Pad &p, int z0, int t)
    {
        if constexpr (!GUARD) {
            fetch_to(st[S], gam_p, p, z0, t);
        } else {
            const int hz = t & 1;
            const long long zb = (long long)min(max(z0 + (t >> 1) + p.P, 0), p.PZ - 1) * p.PXY;
#pragma unroll
            for (int k = 0; k < NG; ++k)
                if ((int)threadIdx.x + k * NT < LS)
                    st[S][k] = gam_p[(long long)(gh[k] + 4 * hz) * p.NP + zb + goff[k]];
        }
    }
    // Store without a branch: a lane past the end of the slice holds the
    // slice's last element (its fetch offset was clamped) and writes it where
    // the lane that owns it does.  Used once, before the step loop, where the
    // branch of store() would let the compiler sink each fetch next to its
    // store and serialise the loads of the whole fill.
    __device__ __forceinline__ void store_all(const R (&d)[NG], R *win, int slot)
    {
#pragma unroll
        for (int k = 0; k < NG; ++k) win[slot * LS + min((int)threadIdx.x + k * NT, LS - 1)] = d[k];
    }
    template <int S>
    __device__ __forceinline__ void store(R *win, int slot)
    {
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int e = (int)threadIdx.x + k * NT;
            if (e < LS) win[slot * LS + e] = st[S][k];
        }
    }
};

// ring of rho (V = R) or (rho, u1) (V = V4<R>) planes: element e of a plane
// is row e / LX, column e % LX of the window whose origin is the tile origin
// shifted by -R in x and y.  A staged float4 is kept as four scalars (an
// array of vector structs would be placed in scratch memory).
template <typename R>
struct Comp {
    static constexpr int n = 1;
    __device__ static R get(const R &v, int) { return v; }
    __device__ static void set(R &v, int, R x) { v = x; }
};
template <typename R>
struct Comp<V4<R>> {
    static constexpr int n = 4;
    __device__ static R get(const V4<R> &v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w)); }
    __device__ static void set(V4<R> &v, int k, R x)
    {
        if (k == 0) v.x = x;
        else if (k == 1) v.y = x;
        else if (k == 2) v.z = x;
        else v.w = x;
    }
};

template <typename R, typename V, int NT, int NR>
struct PlaneRing {
    static constexpr int NC = Comp<V>::n;
    int LX, LP;
    int off[NR];
    R st[2][NC][NR];  // two staging sets: one in flight while the other is stored

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
    __device__ __forceinline__ void fetch_to(R (&d)[NC][NR], const V *__restrict__ src, const Pad &p, int pz)
    {
        const long long zb = (long long)min(max(pz + p.P, 0), p.PZ - 1) * p.PXY;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const V v = src[zb + off[k]];
#pragma unroll
            for (int m = 0; m < NC; ++m) d[m][k] = Comp<V>::get(v, m);
        }
    }
    // GUARD as in GammaRing::fetch
    template <int S, bool GUARD>
    __device__ __forceinline__ void fetch(const V *__restrict__ src, const Pad &p, int pz)
    {
        if constexpr (!GUARD) {
            fetch_to(st[S], src, p, pz);
        } else {
            const long long zb = (long long)min(max(pz + p.P, 0), p.PZ - 1) * p.PXY;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                if ((int)threadIdx.x + k * NT < LP) {
                    const V v = src[zb + off[k]];
#pragma unroll
                    for (int m = 0; m < NC; ++m) st[S][m][k] = Comp<V>::get(v, m);
                }
            }
        }
    }
    // branch-free store of a whole plane, as GammaRing::store_all
    __device__ __forceinline__ void store_all(const R (&d)[NC][NR], V *win, int slot)
    {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            V v;
#pragma unroll
            for (int m = 0; m < NC; ++m) Comp<V>::set(v, m, d[m][k]);
            win[slot * LP + min((int)threadIdx.x + k * NT, LP - 1)] = v;
        }
    }
    template <int S>
    __device__ __forceinline__ void store(V *win, int slot)
    {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int e = (int)threadIdx.x + k * NT;
            if (e < LP) {
                V v;
#pragma unroll
                for (int m = 0; m < NC; ++m) Comp<V>::set(v, m, st[S][m][k]);
                win[slot * LP + e] = v;
            }
        }
    }
};

// LDS bytes of the two rings (host and device agree on this layout: the
// plane ring first, then the gamma ring)
__host__ __device__ constexpr size_t shell_lds_bytes(int TX, int TY, int TZ, int Rr, size_t vbytes, size_t rbytes,
                                                     bool gamma_lds)
{
    return (size_t)(TZ + 1) * (TX + 2 * Rr) * (TY + 2 * Rr) * vbytes +
           (gamma_lds ? (size_t)(2 * TZ) * 4 * (TX + Rr) * (TY + Rr) * rbytes : 0);
}

// Both rings of one block and the per-lane pointers into them.  With
// prefetch depth PD = 1 a c-step is
//   begin<S>(c)  fetch the plane and slice that step c + 1 will read,
//   ...          sum the quads of e_z = c from plane(c) and gamma(c),
//   end<S>(c)    store them into the free slots (those of the plane and
//                slice last read at step c - 1), barrier.
// With PD = 2 the fetches run one step earlier, into two register sets that
// alternate with the parity S = (c + R) & 1 of the step: begin<S>(c)
// fetches for step c + 2 into set S ^ 1 while set S holds what end<S>(c)
// stores.  PD = 2 hides more load latency at the cost of registers (the
// mean-field kernel, light on arithmetic per step, uses it).
template <typename R, typename V, int TX, int TY, int TZ, int NR, int NG, int PD = 1>
struct ShellRings {
    static_assert(PD == 1 || PD == 2, "prefetch depth 1 or 2");
    static constexpr int NT = TX * TY * TZ, NS = TZ + 1, NSG = 2 * TZ;
    static constexpr bool GL = NG > 0;
    PlaneRing<R, V, NT, NR> pr;
    GammaRing<R, NT, GL ? NG : 1> gr;
    V *win;
    R *gwin;
    int Rr, z0, lz, lbase, gcen;

    __device__ __forceinline__ void init(unsigned char *lds, const Pad &p, int Rr_, const TileCoord &tc,
                                         const V *__restrict__ src, const R *__restrict__ gam_p)
    {
        Rr = Rr_;
        z0 = tc.z0;
        lz = tc.lz;
        pr.setup(p, Rr, TX, TY, tc.x0, tc.y0);
        win = reinterpret_cast<V *>(lds);
        gwin = reinterpret_cast<R *>(lds + (size_t)NS * pr.LP * sizeof(V));
        lbase = (tc.ly + Rr) * pr.LX + (tc.lx + Rr);
        const int o = (Rr + 1) >> 1;
        gcen = 0;
        if constexpr (GL) {
            gr.setup(p, Rr, TX, TY, tc.x0, tc.y0);
            gcen = (tc.ly + o) * gr.LXg + (tc.lx + o);
        }
        // the fill: the first TZ planes and 2 TZ - 1 slices, all fetched
        // before any is stored (one load latency for the whole fill)
        R pst[TZ][PlaneRing<R, V, NT, NR>::NC][NR];
        R gst[GL ? 2 * TZ - 1 : 1][GL ? NG : 1];
#pragma unroll
        for (int k = 0; k < TZ; ++k) pr.fetch_to(pst[k], src, p, z0 - Rr + k);
        if constexpr (GL) {
#pragma unroll
            for (int j = 0; j < 2 * TZ - 1; ++j) gr.fetch_to(gst[j], gam_p, p, z0, j - Rr);
        }
        if constexpr (PD == 2) {  // what step -R stores at its end
            pr.template fetch<0, false>(src, p, z0 + TZ - Rr);
            if constexpr (GL) gr.template fetch<0, false>(gam_p, p, z0, 2 * TZ - 1 - Rr);
        }
#pragma unroll
        for (int k = 0; k < TZ; ++k) pr.store_all(pst[k], win, k);
        if constexpr (GL) {
#pragma unroll
            for (int j = 0; j < 2 * TZ - 1; ++j) gr.store_all(gst[j], gwin, (j - Rr + 64) % NSG);
        }
        __syncthreads();
    }
    template <int S>
    __device__ __forceinline__ void begin(int c, const Pad &p, const V *__restrict__ src, const R *__restrict__ gam_p)
    {
        if constexpr (PD == 2) {
            if (c + 1 < Rr) {
                pr.template fetch<S ^ 1, false>(src, p, z0 + c + 1 + TZ);
                if constexpr (GL) gr.template fetch<S ^ 1, false>(gam_p, p, z0, c + 2 * TZ);
            }
        } else if (c < Rr) {
            pr.template fetch<0, true>(src, p, z0 + c + TZ);
            if constexpr (GL) gr.template fetch<0, true>(gam_p, p, z0, c + 2 * TZ - 1);
        }
    }
    template <int S>
    __device__ __forceinline__ void end(int c)
    {
        constexpr int SS = PD == 2 ? S : 0;
        if (c < Rr) {
            pr.template store<SS>(win, (c + TZ + Rr) % NS);
            if constexpr (GL) gr.template store<SS>(gwin, (c + 2 * TZ - 1 + 64) % NSG);
        }
        __syncthreads();
    }
    // the lane's node in the plane window of e_z = c, and its half-lattice
    // point in the gamma slice of e_z = c (both at in-plane offset 0)
    __device__ __forceinline__ const V *plane(int c) const { return win + ((lz + c + Rr) % NS) * pr.LP + lbase; }
    __device__ __forceinline__ const R *gamma(int c) const
    {
        return gwin + ((c + 2 * lz + 64) % NSG) * gr.LS + gcen;
    }
};

// One quad of the mean-field sum: G_m = gamma_m rho_m for the four mirror
// images and their Hadamard transform, accumulated with the quad's weights.
// The mirror products and the transform must not be fused into FMAs:
// fma(gamma_0, rho_0, -G_1) of identical mirror images is the rounding error
// of G_1, not zero.
template <typename R>
__device__ __forceinline__ void mf_quad(const R (&gm)[4], const R (&rm)[4], R px, R py, R pz, R &fx, R &fy, R &fz)
{
    R hx, hy, h0;
    {
#pragma clang fp contract(off)
        R G[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) G[m] = gm[m] * rm[m];
        const R P1 = G[0] + G[1], M1 = G[0] - G[1], P2 = G[2] + G[3], M2 = G[2] - G[3];
        hx = M1 + M2;
        hy = P1 - P2;
        h0 = P1 + P2;
    }
    fx += px * hx;
    fy += py * hy;
    fz += pz * h0;
}

// One quad of the viscous / SMDB sums: W_m = gamma_m rho_m (u1_m - u1_0),
// the Hadamard transform over the mirror signs, accumulated with the quad's
// weights (same no-fusion rule as mf_quad for the products and transform).
template <typename R>
__device__ __forceinline__ void sh_quad(const R (&gm)[4], const V4<R> (&sm)[4], const V4<R> &c0, R px, R py, R pz,
                                        R qxx, R qyy, R qzz, R qxy, R qxz, R qyz, R (&acc)[9])
{
    R x0_, xX, xY, xXY, y0_, yX, yY, yXY, z0_, zX, zY;
    {
#pragma clang fp contract(off)
        R Wx[4], Wy[4], Wz[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const R G = gm[m] * sm[m].x;
            Wx[m] = G * (sm[m].y - c0.y);
            Wy[m] = G * (sm[m].z - c0.z);
            Wz[m] = G * (sm[m].w - c0.w);
        }
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
    // one FMA per term, in a fixed order
    acc[0] += qxx * x0_;
    acc[0] += qxy * yXY;
    acc[0] += qxz * zX;
    acc[1] += qxy * xXY;
    acc[1] += qyy * y0_;
    acc[1] += qyz * zY;
    acc[2] += qxz * xX;
    acc[2] += qyz * yY;
    acc[2] += qzz * z0_;
    acc[3] += px * xX;
    acc[4] += py * yY;
    acc[5] += pz * z0_;
    acc[6] += py * xY;
    acc[6] += px * yX;
    acc[7] += pz * x0_;
    acc[7] += px * zX;
    acc[8] += pz * y0_;
    acc[8] += py * zY;
}

// u1 = j/rho + (g + F^mf)/2 into the padded (rho, u1) array with its images,
// and F^mf
template <typename R>
__device__ __forceinline__ void mf_finish_v(const Geom &g, const Pad &p, int x, int y, int z, R rr, R Fx, R Fy,
                                            R Fz, R jxi, R jyi, R jzi, R gx, R gy, R gz, V4<R> *__restrict__ ru1_p,
                                            V4<R> *__restrict__ fmf)
{
    const int i = (z * g.ny + y) * g.nx + x;
    V4<R> v = {R(0), R(0), R(0), R(0)};
    if (zfluid(g, z)) {
        plane_force(g, z, gx, gy, gz);
        const R inv = R(1) / rr;
        v = V4<R>{rr, jxi * inv + R(0.5) * (gx + Fx), jyi * inv + R(0.5) * (gy + Fy), jzi * inv + R(0.5) * (gz + Fz)};
    }
    for_images(g, p, x, y, z, [&](int k) { ru1_p[k] = v; });
    fmf[i] = V4<R>{Fx, Fy, Fz, R(0)};
}
template <typename R>
__device__ __forceinline__ void mf_finish(const Geom &g, const Pad &p, int x, int y, int z, R rr, R Fx, R Fy, R Fz,
                                          const R *__restrict__ jx, const R *__restrict__ jy,
                                          const R *__restrict__ jz, R gx, R gy, R gz, V4<R> *__restrict__ ru1_p,
                                          V4<R> *__restrict__ fmf)
{
    const int i = (z * g.ny + y) * g.nx + x;
    mf_finish_v<R>(g, p, x, y, z, rr, Fx, Fy, Fz, jx[i], jy[i], jz[i], gx, gy, gz, ru1_p, fmf);
}

// F = rho (g + F^mf + c_v sum k (k.W)) and the traceless SMDB field
// A = cA rho (sum_e (k_j W_i + k_i W_j)) minus its trace / 3
template <typename R>
__device__ __forceinline__ void sh_finish_v(const Geom &g, int x, int y, int z, R r0, const R (&acc)[9], R cv, R cA,
                                            R gx, R gy, R gz, int smdb, const V4<R> &fm, R *__restrict__ Fo,
                                            R *__restrict__ Ao, R *__restrict__ So);
template <typename R>
__device__ __forceinline__ void sh_finish(const Geom &g, int x, int y, int z, R r0, const R (&acc)[9], R cv, R cA,
                                          R gx, R gy, R gz, int smdb, const V4<R> *__restrict__ fmf,
                                          R *__restrict__ Fo, R *__restrict__ Ao, R *__restrict__ So)
{
    sh_finish_v<R>(g, x, y, z, r0, acc, cv, cA, gx, gy, gz, smdb, fmf[(z * g.ny + y) * g.nx + x], Fo, Ao, So);
}
// So (optional, null in the isothermal step): the trace sum sum_e k.W of the
// shell, from which the coupled thermal flow forms the compression term of Q
template <typename R>
__device__ __forceinline__ void sh_finish_v(const Geom &g, int x, int y, int z, R r0, const R (&acc)[9], R cv, R cA,
                                            R gx, R gy, R gz, int smdb, const V4<R> &fm, R *__restrict__ Fo,
                                            R *__restrict__ Ao, R *__restrict__ So)
{
    const long long N = g.N;
    const int i = (z * g.ny + y) * g.nx + x;
    plane_force(g, z, gx, gy, gz);
    Fo[i] = r0 * (gx + fm.x + cv * acc[0]);
    Fo[N + i] = r0 * (gy + fm.y + cv * acc[1]);
    Fo[2 * N + i] = r0 * (gz + fm.z + cv * acc[2]);
    R Axx = 0, Ayy = 0, Azz = 0, Axy = 0, Axz = 0, Ayz = 0;
    if (smdb) {
        const R ca = cA * r0;
        Axx = ca * R(2) * acc[3];
        Ayy = ca * R(2) * acc[4];
        Azz = ca * R(2) * acc[5];
        Axy = ca * acc[6];
        Axz = ca * acc[7];
        Ayz = ca * acc[8];
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
    if (So) So[i] = acc[3] + acc[4] + acc[5];
}

// gamma of the four mirror images of quad (a, b, c) for the generic kernels:
// from the gamma ring (GL) or through the caches from the padded arrays
template <typename R, bool GL>
__device__ __forceinline__ void gamma_quad(const R *gl, int LG, int LXg, const R *__restrict__ gam_p, const Pad &p,
                                           int gbase, int a, int b, int c, int hidx, R (&gm)[4])
{
    if constexpr (GL) {
        const int hb = (hidx & 3) * LG, ha = a >> 1, hna = (-a) >> 1;
        const int hbb = (b >> 1) * LXg, hnb = ((-b) >> 1) * LXg;
        gm[0] = gl[hb + ha + hbb];
        gm[1] = gl[hb + hna + hbb];
        gm[2] = gl[hb + ha + hnb];
        gm[3] = gl[hb + hna + hnb];
    } else {
        int so[4], mo[4];
        quad_offsets(a, b, c, p.PX, p.PXY, so, mo);
        const R *gb = gam_p + (long long)hidx * p.NP + gbase;
#pragma unroll
        for (int m = 0; m < 4; ++m) gm[m] = gb[mo[m]];
    }
}

// ---------------------------------------------------------------------------
// k_meanfield: F^mf = -kT sigma^2 sum_e k G, G = gamma_mid rho(r+e); then
// u1 = j/rho + (g + F^mf)/2.  Generic: the shell comes from the quad table.
// ---------------------------------------------------------------------------
template <typename R, int TX, int TY, int TZ, int NR, int NG>
__global__ __launch_bounds__(TX *TY *TZ) void k_meanfield(Geom g, Pad p, int Rr, const R *__restrict__ rho_p,
                                                          const R *__restrict__ jx, const R *__restrict__ jy,
                                                          const R *__restrict__ jz, const R *__restrict__ gam_p,
                                                          const Quad<R> *__restrict__ quads,
                                                          const int *__restrict__ qstart, R cmf, R gx, R gy, R gz,
                                                          int tiles_x, int tiles_y, int tiles_z,
                                                          V4<R> *__restrict__ ru1_p, V4<R> *__restrict__ fmf)
{
    constexpr bool GL = NG > 0;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ>(tiles_x, tiles_y, tiles_z);
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    ShellRings<R, R, TX, TY, TZ, NR, NG, 2> rg;
    rg.init(lds_raw, p, Rr, tc, rho_p, gam_p);
    const int gbase = pidx(p, min(x, g.nx - 1), min(y, g.ny - 1), min(z, g.nz - 1));
    const int LX = rg.pr.LX;
    R fx = 0, fy = 0, fz = 0;
    auto cstep = [&](auto si, int c) __attribute__((always_inline)) {
        constexpr int S = decltype(si)::value;
        rg.template begin<S>(c, p, rho_p, gam_p);
        const R *pl = rg.plane(c);
        const R *gl = GL ? rg.gamma(c) : nullptr;
        const int qb = qstart[c + Rr], qe = qstart[c + Rr + 1];
        for (int q = qb; q < qe; ++q) {
            const Quad<R> Qd = quads[q];
            const int a = Qd.a, b = Qd.b;
            R gm[4], rm[4];
            gamma_quad<R, GL>(gl, rg.gr.LG, rg.gr.LXg, gam_p, p, gbase, a, b, Qd.c, Qd.hidx, gm);
            rm[0] = pl[a + b * LX];
            rm[1] = pl[-a + b * LX];
            rm[2] = pl[a - b * LX];
            rm[3] = pl[-a - b * LX];
            mf_quad<R>(gm, rm, Qd.px, Qd.py, Qd.pz, fx, fy, fz);
        }
        rg.template end<S>(c);
    };
    for (int c = -Rr; c <= Rr; c += 2) {
        cstep(std::integral_constant<int, 0>{}, c);
        if (c + 1 <= Rr) cstep(std::integral_constant<int, 1>{}, c + 1);
    }
    if (!valid) return;
    mf_finish<R>(g, p, x, y, z, rho_p[gbase], cmf * fx, cmf * fy, cmf * fz, jx, jy, jz, gx, gy, gz, ru1_p, fmf);
}

// ---------------------------------------------------------------------------
// k_shell: F^v = c_v sum_e k (k.W), A_ij = cA rho sum_e (k_j W_i + k_i W_j),
// W = gamma_mid rho(r+e) (u1(r+e) - u1(r)); the dominant kernel.  Generic:
// the shell comes from the quad table.
// ---------------------------------------------------------------------------
template <typename R, int TX, int TY, int TZ, int NR, int NG>
__global__ __launch_bounds__(TX *TY *TZ) void k_shell(Geom g, Pad p, int Rr, const V4<R> *__restrict__ ru1_p,
                                                      const R *__restrict__ gam_p, const V4<R> *__restrict__ fmf,
                                                      const Quad<R> *__restrict__ quads,
                                                      const int *__restrict__ qstart, R cv, R cA, R gx, R gy, R gz,
                                                      int smdb, int tiles_x, int tiles_y, int tiles_z,
                                                      R *__restrict__ Fo, R *__restrict__ Ao, R *__restrict__ So)
{
    constexpr bool GL = NG > 0;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ>(tiles_x, tiles_y, tiles_z);
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    ShellRings<R, V4<R>, TX, TY, TZ, NR, NG> rg;
    rg.init(lds_raw, p, Rr, tc, ru1_p, gam_p);
    const int gbase = pidx(p, min(x, g.nx - 1), min(y, g.ny - 1), min(z, g.nz - 1));
    const V4<R> c0 = ru1_p[gbase];
    const int LX = rg.pr.LX;
    R acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    auto cstep = [&](auto si, int c) __attribute__((always_inline)) {
        constexpr int S = decltype(si)::value;
        rg.template begin<S>(c, p, ru1_p, gam_p);
        const V4<R> *pl = rg.plane(c);
        const R *gl = GL ? rg.gamma(c) : nullptr;
        const int qb = qstart[c + Rr], qe = qstart[c + Rr + 1];
        for (int q = qb; q < qe; ++q) {
            const Quad<R> Qd = quads[q];
            const int a = Qd.a, b = Qd.b;
            R gm[4];
            V4<R> sm[4];
            gamma_quad<R, GL>(gl, rg.gr.LG, rg.gr.LXg, gam_p, p, gbase, a, b, Qd.c, Qd.hidx, gm);
            sm[0] = pl[a + b * LX];
            sm[1] = pl[-a + b * LX];
            sm[2] = pl[a - b * LX];
            sm[3] = pl[-a - b * LX];
            sh_quad<R>(gm, sm, c0, Qd.px, Qd.py, Qd.pz, Qd.qxx, Qd.qyy, Qd.qzz, Qd.qxy, Qd.qxz, Qd.qyz, acc);
        }
        rg.template end<S>(c);
    };
    for (int c = -Rr; c <= Rr; c += 2) {
        cstep(std::integral_constant<int, 0>{}, c);
        if (c + 1 <= Rr) cstep(std::integral_constant<int, 1>{}, c + 1);
    }
    if (!valid) return;
    sh_finish<R>(g, x, y, z, c0.x, acc, cv, cA, gx, gy, gz, smdb, fmf, Fo, Ao, So);
}

// ---------------------------------------------------------------------------
// The same two kernels specialised for the shell of 2 sigma = S2 (rings in
// LDS only): the e_z steps and the quads are unrolled at compile time, so
// every LDS offset is an immediate and every weight a literal.  Offsets are
// taken from the corner of each lane's stencil window (non-negative).
// ---------------------------------------------------------------------------
// Quads with a = 0 or b = 0 have only two distinct mirror images (one when
// both are 0), and their x- or y-odd Hadamard outputs are exact zeros whose
// weights are zero as well.  The compiled kernels sum the distinct images
// once, with the weights scaled by 2 (or 4): doubling is exact, so the
// result is bit-identical to the four-image path of the table-driven
// kernels, which repeats each image (weight 1/2 or 1/4).
template <typename R>
__device__ __forceinline__ void mf_quad_pair(R g0, R r0, R g1, R r1, R p_odd, R pz, R &f_odd, R &fz)
{
    R d, s;
    {
#pragma clang fp contract(off)
        const R G0 = g0 * r0, G1 = g1 * r1;
        d = G0 - G1;
        s = G0 + G1;
    }
    f_odd += p_odd * d;
    fz += pz * s;
}

template <typename R>
__device__ __forceinline__ void sh_w(R g, const V4<R> &sv, const V4<R> &c0, R &wx, R &wy, R &wz)
{
#pragma clang fp contract(off)
    const R G = g * sv.x;
    wx = G * (sv.y - c0.y);
    wy = G * (sv.z - c0.z);
    wz = G * (sv.w - c0.w);
}

// Buffer descriptors of the four (x, y)-parity sub-lattices of the contact
// value in the plane z + floor(c/2) (z-parity c & 1), each based at the
// corner (-O, -O) of the half-reach window, so that every image offset is
// non-negative.  A raw buffer (stride 0) of num_records bytes; reads past it
// return 0 (the lattices that use these kernels stay well inside).
template <typename R>
__device__ __forceinline__ void gamma_rsrc(const R *__restrict__ gam_p, const Pad &p, int c, int O,
                                           __amdgpu_buffer_rsrc_t (&gr)[4])
{
    const long long zoff = (long long)(c >> 1) * p.PXY - (long long)O * p.PX - O;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const R *b = gam_p + (long long)(k + 4 * (c & 1)) * p.NP + zoff;
        gr[k] = __builtin_amdgcn_make_buffer_rsrc(const_cast<R *>(b), (short)0, 0x7fffffff, 0x00020000);
    }
}

// gamma of the image (sa a, sb b, c) of a compiled quad Q (sa, sb = +-1): from
// the LDS gamma ring (GL; gc is the ring slice of e_z = c shifted to the
// corner of the lane's window), or through the vector caches from the padded
// arrays by a buffer load whose image offset is a scalar (the same for the
// whole wave) and whose lane offset gvo is the lane's padded index in bytes.
// Either way no vector instruction forms the address.
template <typename R, bool GL, int O, int LXg, int LG, int A, int B, int H, int SA, int SB>
__device__ __forceinline__ R gamma_img(const R *gc, const __amdgpu_buffer_rsrc_t (&gr)[4], int PX, unsigned gvo)
{
    constexpr int ox = (SA * A) >> 1, oy = (SB * B) >> 1;
    if constexpr (GL) {
        return gc[(H & 3) * LG + (O + ox) + (O + oy) * LXg];
    } else if constexpr (sizeof(R) == 4) {
        return __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(gr[H & 3], (int)gvo, ((oy + O) * PX + (ox + O)) * 4, 0));
    } else {
        static_assert(sizeof(R) == 8, "contact values through buffer loads are FP32 or FP64");
        return __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(gr[H & 3], (int)gvo, ((oy + O) * PX + (ox + O)) * 8, 0));
    }
}

template <typename R, int S2, int TX, int TY, int TZ, int NR, int NG>
__global__ __launch_bounds__(TX *TY *TZ) void k_meanfield_s(Geom g, Pad p, const R *__restrict__ rho_p,
                                                            const R *__restrict__ jx, const R *__restrict__ jy,
                                                            const R *__restrict__ jz, const R *__restrict__ gam_p,
                                                            R cmf, R gx, R gy, R gz, int tiles_x, int tiles_y,
                                                            int tiles_z, V4<R> *__restrict__ ru1_p,
                                                            V4<R> *__restrict__ fmf)
{
    constexpr bool GL = NG > 0;
    using SH = Shell<S2>;
    constexpr int RC = SH::R, LX = TX + 2 * RC, O = (RC + 1) >> 1, LXg = TX + RC, LG = LXg * (TY + RC);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ>(tiles_x, tiles_y, tiles_z);
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    ShellRings<R, R, TX, TY, TZ, NR, NG, 2> rg;
    rg.init(lds_raw, p, RC, tc, rho_p, gam_p);
    // the node's own inputs of mf_finish, fetched now and pinned after the
    // first c-step so that their latency hides behind it
    const int xc = min(x, g.nx - 1), yc = min(y, g.ny - 1), zc = min(z, g.nz - 1), ic = (zc * g.ny + yc) * g.nx + xc;
    const int gbase = pidx(p, xc, yc, zc);
    const unsigned gvo = (unsigned)gbase * (unsigned)sizeof(R);
    R rr = rho_p[gbase], jxi = jx[ic], jyi = jy[ic], jzi = jz[ic];
    R fx = 0, fy = 0, fz = 0;
    static_for<-RC, RC + 1>([&](auto ci) __attribute__((always_inline)) {
        constexpr int c = decltype(ci)::value;
        constexpr int S = (c + RC) & 1;
        if constexpr (c == -RC + 1) {
            pin(rr);
            pin(jxi);
            pin(jyi);
            pin(jzi);
        }
        rg.template begin<S>(c, p, rho_p, gam_p);
        const R *pc = rg.plane(c) - (RC + RC * LX);
        const R *gc = GL ? rg.gamma(c) - (O + O * LXg) : nullptr;
        __amdgpu_buffer_rsrc_t gr[4];
        if constexpr (!GL) gamma_rsrc<R>(gam_p, p, c, O, gr);
        static_for<SH::T.qs[c + RC], SH::T.qs[c + RC + 1]>([&](auto qi) __attribute__((always_inline)) {
            constexpr CQuad Q = SH::T.q[decltype(qi)::value];
            constexpr int a = Q.a, b = Q.b;
#define WDLB_GAM(SA, SB) gamma_img<R, GL, O, LXg, LG, a, b, Q.h, SA, SB>(gc, gr, p.PX, gvo)
            if constexpr (a == 0 && b == 0) {
                R G;
                {
#pragma clang fp contract(off)
                    G = WDLB_GAM(1, 1) * pc[RC + RC * LX];
                }
                fz += R(4 * Q.pz) * G;
            } else if constexpr (a == 0) {  // images (0, b) and (0, -b)
                mf_quad_pair<R>(WDLB_GAM(1, 1), pc[RC + (RC + b) * LX], WDLB_GAM(1, -1), pc[RC + (RC - b) * LX],
                                R(2 * Q.py), R(2 * Q.pz), fy, fz);
            } else if constexpr (b == 0) {  // images (a, 0) and (-a, 0)
                mf_quad_pair<R>(WDLB_GAM(1, 1), pc[(RC + a) + RC * LX], WDLB_GAM(-1, 1), pc[(RC - a) + RC * LX],
                                R(2 * Q.px), R(2 * Q.pz), fx, fz);
            } else {
                const R gm[4] = {WDLB_GAM(1, 1), WDLB_GAM(-1, 1), WDLB_GAM(1, -1), WDLB_GAM(-1, -1)};
                const R rm[4] = {pc[(RC + a) + (RC + b) * LX], pc[(RC - a) + (RC + b) * LX],
                                 pc[(RC + a) + (RC - b) * LX], pc[(RC - a) + (RC - b) * LX]};
                mf_quad<R>(gm, rm, R(Q.px), R(Q.py), R(Q.pz), fx, fy, fz);
            }
        });
        pin(fx);
        pin(fy);
        pin(fz);
        rg.template end<S>(c);
    });
    if (!valid) return;
    mf_finish_v<R>(g, p, x, y, z, rr, cmf * fx, cmf * fy, cmf * fz, jxi, jyi, jzi, gx, gy, gz, ru1_p, fmf);
}

template <typename R, int S2, int TX, int TY, int TZ, int NR, int NG>
__global__ __launch_bounds__(TX *TY *TZ) void k_shell_s(Geom g, Pad p, const V4<R> *__restrict__ ru1_p,
                                                        const R *__restrict__ gam_p, const V4<R> *__restrict__ fmf,
                                                        R cv, R cA, R gx, R gy, R gz, int smdb, int tiles_x,
                                                        int tiles_y, int tiles_z, R *__restrict__ Fo,
                                                        R *__restrict__ Ao, R *__restrict__ So)
{
    constexpr bool GL = NG > 0;
    using SH = Shell<S2>;
    constexpr int RC = SH::R, LX = TX + 2 * RC, O = (RC + 1) >> 1, LXg = TX + RC, LG = LXg * (TY + RC);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const TileCoord tc = tile_coord<TX, TY, TZ>(tiles_x, tiles_y, tiles_z);
    const int x = tc.x0 + tc.lx, y = tc.y0 + tc.ly, z = tc.z0 + tc.lz;
    const bool valid = x < g.nx && y < g.ny && z < g.nz;
    ShellRings<R, V4<R>, TX, TY, TZ, NR, NG> rg;
    rg.init(lds_raw, p, RC, tc, ru1_p, gam_p);
    const int gbase = pidx(p, min(x, g.nx - 1), min(y, g.ny - 1), min(z, g.nz - 1));
    const unsigned gvo = (unsigned)gbase * (unsigned)sizeof(R);
    const V4<R> c0 = ru1_p[gbase];
    // F^mf of the node for sh_finish, fetched now, pinned after the first c-step
    V4<R> fm = fmf[(min(z, g.nz - 1) * g.ny + min(y, g.ny - 1)) * g.nx + min(x, g.nx - 1)];
    R acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static_for<-RC, RC + 1>([&](auto ci) __attribute__((always_inline)) {
        constexpr int c = decltype(ci)::value;
        constexpr int S = (c + RC) & 1;
        if constexpr (c == -RC + 1) {
            pin(fm.x);
            pin(fm.y);
            pin(fm.z);
        }
        rg.template begin<S>(c, p, ru1_p, gam_p);
        const V4<R> *pc = rg.plane(c) - (RC + RC * LX);
        const R *gc = GL ? rg.gamma(c) - (O + O * LXg) : nullptr;
        __amdgpu_buffer_rsrc_t gr[4];
        if constexpr (!GL) gamma_rsrc<R>(gam_p, p, c, O, gr);
        static_for<SH::T.qs[c + RC], SH::T.qs[c + RC + 1]>([&](auto qi) __attribute__((always_inline)) {
            constexpr CQuad Q = SH::T.q[decltype(qi)::value];
            constexpr int a = Q.a, b = Q.b;
            if constexpr (a == 0 && b == 0) {
                // one image: only the z-even outputs, 4 W, remain
                R wx, wy, wz;
                sh_w<R>(WDLB_GAM(1, 1), pc[RC + RC * LX], c0, wx, wy, wz);
                acc[2] += R(4 * Q.qzz) * wz;
                acc[5] += R(4 * Q.pz) * wz;
                acc[7] += R(4 * Q.pz) * wx;
                acc[8] += R(4 * Q.pz) * wy;
            } else if constexpr (a == 0) {
                // images (0, b), (0, -b): the x-odd outputs vanish, the others
                // are twice the sum (even) or difference (y-odd) of the two
                R w0x, w0y, w0z, w2x, w2y, w2z, x0h, xYh, y0h, yYh, z0h, zYh;
                sh_w<R>(WDLB_GAM(1, 1), pc[RC + (RC + b) * LX], c0, w0x, w0y, w0z);
                sh_w<R>(WDLB_GAM(1, -1), pc[RC + (RC - b) * LX], c0, w2x, w2y, w2z);
                {
#pragma clang fp contract(off)
                    x0h = w0x + w2x;
                    xYh = w0x - w2x;
                    y0h = w0y + w2y;
                    yYh = w0y - w2y;
                    z0h = w0z + w2z;
                    zYh = w0z - w2z;
                }
                acc[1] += R(2 * Q.qyy) * y0h;
                acc[1] += R(2 * Q.qyz) * zYh;
                acc[2] += R(2 * Q.qyz) * yYh;
                acc[2] += R(2 * Q.qzz) * z0h;
                acc[4] += R(2 * Q.py) * yYh;
                acc[5] += R(2 * Q.pz) * z0h;
                acc[6] += R(2 * Q.py) * xYh;
                acc[7] += R(2 * Q.pz) * x0h;
                acc[8] += R(2 * Q.pz) * y0h;
                acc[8] += R(2 * Q.py) * zYh;
            } else if constexpr (b == 0) {
                // images (a, 0), (-a, 0): the y-odd outputs vanish
                R w0x, w0y, w0z, w1x, w1y, w1z, x0h, xXh, y0h, yXh, z0h, zXh;
                sh_w<R>(WDLB_GAM(1, 1), pc[(RC + a) + RC * LX], c0, w0x, w0y, w0z);
                sh_w<R>(WDLB_GAM(-1, 1), pc[(RC - a) + RC * LX], c0, w1x, w1y, w1z);
                {
#pragma clang fp contract(off)
                    x0h = w0x + w1x;
                    xXh = w0x - w1x;
                    y0h = w0y + w1y;
                    yXh = w0y - w1y;
                    z0h = w0z + w1z;
                    zXh = w0z - w1z;
                }
                acc[0] += R(2 * Q.qxx) * x0h;
                acc[0] += R(2 * Q.qxz) * zXh;
                acc[2] += R(2 * Q.qxz) * xXh;
                acc[2] += R(2 * Q.qzz) * z0h;
                acc[3] += R(2 * Q.px) * xXh;
                acc[5] += R(2 * Q.pz) * z0h;
                acc[6] += R(2 * Q.px) * yXh;
                acc[7] += R(2 * Q.pz) * x0h;
                acc[7] += R(2 * Q.px) * zXh;
                acc[8] += R(2 * Q.pz) * y0h;
            } else {
                const R gm[4] = {WDLB_GAM(1, 1), WDLB_GAM(-1, 1), WDLB_GAM(1, -1), WDLB_GAM(-1, -1)};
                const V4<R> sm[4] = {pc[(RC + a) + (RC + b) * LX], pc[(RC - a) + (RC + b) * LX],
                                     pc[(RC + a) + (RC - b) * LX], pc[(RC - a) + (RC - b) * LX]};
                sh_quad<R>(gm, sm, c0, R(Q.px), R(Q.py), R(Q.pz), R(Q.qxx), R(Q.qyy), R(Q.qzz), R(Q.qxy),
                           R(Q.qxz), R(Q.qyz), acc);
            }
        });
#pragma unroll
        for (int k = 0; k < 9; ++k) pin(acc[k]);
        rg.template end<S>(c);
    });
    if (!valid) return;
    sh_finish_v<R>(g, x, y, z, c0.x, acc, cv, cA, gx, gy, gz, smdb, fm, Fo, Ao, So);
}
#undef WDLB_GAM

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
    plane_force(g, z, gx, gy, gz);
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
template <typename R, typename HS, typename D, bool READ>
__global__ __launch_bounds__(256) void k_collide(Geom g, NodeTiles nt, const R *__restrict__ Fi,
                                                 const R *__restrict__ Ai, R omega, R ksrc,
                                                 const V4<R> *__restrict__ ru_in, const HS *__restrict__ h_in,
                                                 V4<R> *__restrict__ ru_out, HS *__restrict__ h_out,
                                                 R *__restrict__ u_rd, uint64_t step)
{
    long long i;
    int x, y, z;
    if (!node_tiled(g, nt, x, y, z, i)) return;
    const long long N = g.N;
    if (!zfluid(g, z)) {  // gap plane of a stacked lattice: no state
        if (READ) u_rd[i] = u_rd[N + i] = u_rd[2 * N + i] = R(0);
        return;
    }
    if (g.zp != nullptr) {
        omega = R(g.zp[z].omega);
        ksrc = R(g.zp[z].ksrc);
    }
    const int r = (z * g.ny + y) * g.nx + x;
    // the 19 pulled populations as phi_a = f_a - w_a rho_r, kept for the
    // collision (moments summed in the order of pull_moments)
    D f[Q];
    D delta = 0, jx = 0, jy = 0, jz = 0;
    const PullNbr nbr = pull_nbr(g, x, y, z);
    const R rho_r = ru_in[r].x;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        f[a] = fpull_phi<R, HS, D>(g, ru_in, h_in, nbr, x, y, z, r, a, rho_r);
        delta += f[a];
        if (CX[a]) jx += D(CX[a]) * f[a];
        if (CY[a]) jy += D(CY[a]) * f[a];
        if (CZ[a]) jz += D(CZ[a]) * f[a];
    }
    const D rho = D(rho_r) + delta;
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
    R hv[Q];  // BF16 mode: h* kept for the closure
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const D w = wgt<D>(a);
        const D cu = D(CX[a]) * ux + D(CY[a]) * uy + D(CZ[a]) * uz;
        const D P = D(3) * cu + D(4.5) * cu * cu - D(1.5) * uu;
        const D fneq = f[a] - w * (delta + rho * P);
        const D cF = D(CX[a]) * Fx + D(CY[a]) * Fy + D(CZ[a]) * Fz;
        const D guo = w * (D(3) * (cF - uF) + D(9) * cu * cF);
        const D cAc = D(CX[a] * CX[a]) * Axx + D(CY[a] * CY[a]) * Ayy + D(CZ[a] * CZ[a]) * Azz +
                      D(2 * CX[a] * CY[a]) * Axy + D(2 * CX[a] * CZ[a]) * Axz + D(2 * CY[a] * CZ[a]) * Ayz;
        const D sa = D(4.5) * w * cAc;
        const D cd = D(CX[a]) * dx + D(CY[a]) * dy + D(CZ[a]) * dz;
        const D cs = D(CX[a]) * sx + D(CY[a]) * sy + D(CZ[a]) * sz;
        const D deq = w * rho * (-D(3) * cd - D(4.5) * cd * cs + D(1.5) * dsum);
        const R hva = R(keep * fneq + deq + ks * (guo + sa));
        if constexpr (std::is_same<HS, bf16>::value) hv[a] = hva;  // rounded and closed below
        else sth<R, HS>(h_out, a, N, i, hva);
    }
    if constexpr (std::is_same<HS, bf16>::value) {
        // round the others stochastically (dither from a counter-based
        // generator keyed by step, node and population), then close mass
        // and momentum with the FP32 four
        uint64_t rnd[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) rnd[k] = splitmix64((step << 34) ^ ((uint64_t)i << 2) ^ (uint64_t)k);
        D m = 0, mx = 0, my = 0, mz = 0;
        int nb = 0;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            if (closure_slot(a) >= 0) continue;
            const uint32_t r16 = uint32_t(rnd[nb >> 2] >> (16 * (nb & 3))) & 0xffffu;
            ++nb;
            const uint16_t b = f32_to_bf16_sr(float(hv[a]), r16);
            h_out[a * N + i].bits = b;
            const D r = bf16_to_f32(b);
            m += r;
            if (CX[a]) mx += D(CX[a]) * r;
            if (CY[a]) my += D(CY[a]) * r;
            if (CZ[a]) mz += D(CZ[a]) * r;
        }
        const D h1 = -mx, h3 = -my, h5 = -mz;
        sth<R, HS>(h_out, 1, N, i, R(h1));
        sth<R, HS>(h_out, 3, N, i, R(h3));
        sth<R, HS>(h_out, 5, N, i, R(h5));
        sth<R, HS>(h_out, 0, N, i, R(-(m + h1 + h3 + h5)));
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
    const PullNbr n = pull_nbr(g, x, y, z);
    const R rho_r = ru[r].x;
#pragma unroll
    for (int a = 0; a < Q; ++a)
        if (a >= a0 && a < a0 + 8)
            f[(long long)(a - a0) * g.N + i] =
                R(wgt<double>(a) * double(rho_r) + fpull_phi<R, HS, double>(g, ru, h, n, x, y, z, r, a, rho_r));
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
