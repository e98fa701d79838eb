// wdlb.hip -- host side of the MI355X (gfx950) WDLB library behind the C
// ABI of include/wdlb.h: workspace layout, stencil tables, kernel launches
// (kernels.hpp), reads, checkpoints and event timing.
#include "context.hpp"
#include "thermal.hpp"
#include "thermal_flow.hpp"

namespace {

using wdlb_lib::launch_thermal;

bool desc_ok(const wdlb_lattice_desc *d)
{
    if (!d || d->nx < 1 || d->ny < 1 || d->nz < 1) return false;
    long long N = (long long)d->nx * d->ny * d->nz;
    long long NP = (long long)(d->nx + 2 * MAX_REACH) * (d->ny + 2 * MAX_REACH) * (d->nz + 2 * MAX_REACH);
    if (N * 19 >= (1LL << 31) || NP >= (1LL << 31)) return false;
    return d->precision >= WDLB_FP64 && d->precision <= WDLB_BF16_NEQ_LOCAL64;
}

// the storage of a precision mode (the LOCAL64 modes store like their base)
int storage_of(int prec)
{
    return prec == WDLB_FP32_LOCAL64 ? WDLB_FP32 : (prec == WDLB_BF16_NEQ_LOCAL64 ? WDLB_BF16_NEQ : prec);
}

bool params_ok(const wdlb_params *p)
{
    if (!p) return false;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return false;
    if (!(p->sigma >= 1.0 && p->sigma <= MAX_SIGMA)) return false;
    if (!(p->eta > 0.0 && p->eta < 1.0)) return false;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->g[i])) return false;
    return true;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// contact-shell reach: the largest offset component of the shell
int shell_reach(double sigma)
{
    int R = 0, lim = (int)std::ceil(sigma + 0.5) + 1;
    double lo = (sigma - 0.5) * (sigma - 0.5), hi = (sigma + 0.5) * (sigma + 0.5);
    for (int z = -lim; z <= lim; ++z)
        for (int y = -lim; y <= lim; ++y)
            for (int x = -lim; x <= lim; ++x) {
                double r2 = double(x * x + y * y + z * z);
                if (r2 >= lo && r2 < hi) R = std::max(R, std::abs(x));
            }
    return std::max(R, 1);
}

Pad make_pad(const wdlb_lattice_desc *d, int P)
{
    Pad p;
    p.P = P;
    p.PX = d->nx + 2 * P;
    p.PY = d->ny + 2 * P;
    p.PZ = d->nz + 2 * P;
    p.PXY = p.PX * p.PY;
    p.NP = (long long)p.PXY * p.PZ;
    p.kx = (P + d->nx - 1) / d->nx;
    p.ky = (P + d->ny - 1) / d->ny;
    p.kz = d->walls_z ? 0 : (P + d->nz - 1) / d->nz;
    return p;
}

struct Layout {
    size_t off_ru[2], off_h[2], off_rho_p, off_gam_p, off_ru1_p, off_j[3], off_fmf, off_F, off_A, off_urd,
        off_rhord, off_planes, off_flag, off_quads, off_qstart, off_ball, off_zp, total;
};

// the layout does not depend on sigma: padded arrays are sized for the
// largest supported reach
Layout layout(const wdlb_lattice_desc *d)
{
    Layout L;
    size_t N = (size_t)d->nx * d->ny * d->nz;
    Pad pm = make_pad(d, MAX_REACH);
    size_t NP = (size_t)pm.NP;
    const int st = storage_of(d->precision);
    size_t r = st == WDLB_FP64 ? 8 : 4;
    size_t hs = st == WDLB_FP64 ? 8 : (st == WDLB_BF16_NEQ ? 2 : 4);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    for (int b = 0; b < 2; ++b) {
        L.off_ru[b] = take(4 * r * N);
        L.off_h[b] = take((size_t)(st == WDLB_BF16_NEQ ? hplanes<bf16>() : 19) * hs * N);
    }
    L.off_rho_p = take(r * NP);
    L.off_gam_p = take(8 * r * NP);
    L.off_ru1_p = take(4 * r * NP);
    for (int c = 0; c < 3; ++c) L.off_j[c] = take(r * N);
    L.off_fmf = take(4 * r * N);
    L.off_F = take(3 * r * N);
    L.off_A = take(6 * r * N);
    L.off_urd = take(3 * r * N);
    L.off_rhord = take(r * N);
    L.off_planes = take(3 * sizeof(double) * (size_t)d->nz);
    L.off_flag = take(sizeof(int) * (1 + (size_t)d->nz));  // lattice flag, then one per plane
    L.off_quads = take(MAX_QUADS * sizeof(Quad<double>));
    L.off_qstart = take((2 * MAX_REACH + 2) * sizeof(int));
    L.off_ball = take(MAX_BALL * sizeof(int));
    L.off_zp = take((size_t)d->nz * sizeof(ZPlane));
    L.total = o;
    return L;
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
    for (int c = -R_; c <= R_; ++c)  // sorted by c
        for (int b = 0; b <= R_; ++b)
            for (int a = 0; a <= R_; ++a) {
                double r2 = double(a * a + b * b + c * c);
                if (!(r2 >= lo && r2 < hi)) continue;
                const CQuad cq = make_cquad(a, b, c);
                Quad<R> q;
                q.a = cq.a;
                q.b = cq.b;
                q.c = cq.c;
                q.hidx = cq.h;
                q.px = R(cq.px);
                q.py = R(cq.py);
                q.pz = R(cq.pz);
                q.qxx = R(cq.qxx);
                q.qyy = R(cq.qyy);
                q.qzz = R(cq.qzz);
                q.qxy = R(cq.qxy);
                q.qxz = R(cq.qxz);
                q.qyz = R(cq.qyz);
                q.pad0 = q.pad1 = q.pad2 = R(0);
                v.push_back(q);
            }
    return v;
}

// Contact-shell tile variants (k_meanfield and k_shell use the same one).
// Wide lattices try, in this order, 32 x 8 x 2 tiles with both LDS rings for
// growing reach, a 32 x 16 x 1 tile, and a 16 x 16 x 1 tile that reads gamma
// through L1/L2 (NG = 0).  Lattices at most 16 nodes wide in x (the stacked
// serving lattice) take the 16 x 16 x 2 tile when it fits, so no lane of a
// 32-wide row idles.  NR / NG are the plane / gamma-slice elements each
// thread stages.
struct ShellTile {
    int TX, TY, TZ, NR, NG;
};
constexpr ShellTile SHELL_TILES[] = {{32, 8, 2, 2, 5},   {32, 8, 2, 3, 6},  {32, 8, 2, 4, 8}, {32, 16, 1, 7, 13},
                                     {16, 16, 1, 10, 0}, {16, 16, 2, 2, 5}, {32, 8, 2, 4, 0}};
constexpr int NARROW_TILE = 5;  // the 16 x 16 x 2 variant
// 32 x 8 x 2 with only the (rho, u1) ring in LDS, gamma read through the
// vector caches: the LDS then serves the images alone, and a block needs
// half the LDS (more blocks per CU).  The automatic choice of the viscous /
// SMDB kernel for wide FP32 lattices with a compiled shell of 2 sigma >=
// L1G_MIN_S2 (the mean-field kernel, whose quads read four times fewer
// bytes of images, keeps its gamma ring: through the caches it is slower).
constexpr int L1G_TILE = 6;
constexpr int L1G_MIN_S2 = 16;
constexpr int NTILES = (int)(sizeof(SHELL_TILES) / sizeof(SHELL_TILES[0]));
static_assert(NTILES == WDLB_NTILES, "the header's variant count");

// k_density tiles: 32 x 8 x 2 while its LDS stays within 96 KB (one block
// per CU at the FP64 ball of sigma = 10, still faster than the smaller tile
// and its larger halo per node), else 16 x 8 x 1; lattices at most 16 wide
// take 16 x 16 x 2
struct DensityTile {
    int TX, TY, TZ;
    size_t lds_cap;
};
constexpr DensityTile DENSITY_TILES[3] = {{32, 8, 2, 96 * 1024}, {16, 8, 1, 160 * 1024}, {16, 16, 2, 64 * 1024}};
constexpr int NARROW_DENSITY_TILE = 2;
constexpr bool density_fits(const DensityTile &t, int rb, size_t rbytes)
{
    return density_lds_bytes(t.TX, t.TY, t.TZ, rb, rbytes) <= t.lds_cap;
}
constexpr int pick_density_tile(int rb, size_t rbytes, int nx)
{
    if (nx <= 16 && density_fits(DENSITY_TILES[NARROW_DENSITY_TILE], rb, rbytes)) return NARROW_DENSITY_TILE;
    return density_fits(DENSITY_TILES[0], rb, rbytes) ? 0 : (density_fits(DENSITY_TILES[1], rb, rbytes) ? 1 : -1);
}

constexpr bool tile_fits(const ShellTile &t, int reach, size_t rbytes)
{
    const int NT = t.TX * t.TY * t.TZ;
    const int LP = (t.TX + 2 * reach) * (t.TY + 2 * reach), LS = 4 * (t.TX + reach) * (t.TY + reach);
    if ((LP + NT - 1) / NT > t.NR) return false;
    if (t.NG > 0 && (LS + NT - 1) / NT > t.NG) return false;
    return shell_lds_bytes(t.TX, t.TY, t.TZ, reach, 4 * rbytes, rbytes, t.NG > 0) <= LDS_MAX;
}

// the automatic choice for wide lattices
constexpr int pick_tile_wide(int reach, size_t rbytes)
{
    for (int k = 0; k < NARROW_TILE; ++k)
        if (tile_fits(SHELL_TILES[k], reach, rbytes)) return k;
    return -1;
}

// the first of the variants 0..3 whose rings hold those of the mean-field
// kernel alone (its plane ring holds rho, not (rho, u1)), or -1
constexpr int pick_tile_mf(int reach, size_t rbytes)
{
    for (int k = 0; k < 4; ++k) {
        const ShellTile &t = SHELL_TILES[k];
        const int NT = t.TX * t.TY * t.TZ;
        const int LP = (t.TX + 2 * reach) * (t.TY + 2 * reach), LS = 4 * (t.TX + reach) * (t.TY + reach);
        if ((LP + NT - 1) / NT <= t.NR && (LS + NT - 1) / NT <= t.NG &&
            shell_lds_bytes(t.TX, t.TY, t.TZ, reach, rbytes, rbytes, true) <= LDS_MAX)
            return k;
    }
    return -1;
}

constexpr int pick_tile(int reach, size_t rbytes, int nx)
{
    if (nx <= 16 && tile_fits(SHELL_TILES[NARROW_TILE], reach, rbytes)) return NARROW_TILE;
    return pick_tile_wide(reach, rbytes);
}


// compiled kernels exist for the wide automatic tiles of every compiled
// shell (when gamma is staged in LDS), and for the narrow tiles at sigma = 4
// in FP32 (the serving configuration)
template <typename R>
bool compiled_shell(int s2, int tile, int reach)
{
    if (s2 == 0) return false;
    if (tile == NARROW_TILE) return std::is_same<R, float>::value && s2 == 8;
    if (tile == L1G_TILE) return std::is_same<R, float>::value && s2 >= L1G_MIN_S2;
    return tile == pick_tile_wide(reach, sizeof(R)) && SHELL_TILES[tile].NG > 0;
}
template <typename R>
bool compiled_density(int s2, int dtile, int rb)
{
    if (s2 == 0) return false;
    if (dtile == NARROW_DENSITY_TILE) return std::is_same<R, float>::value && s2 == 8;
    return dtile == pick_density_tile(rb, sizeof(R), 1 << 30);
}

template <typename R>
wdlb_status upload_tables(wdlb_ctx *c)
{
    int nshell = 0;
    auto q = build_quads<R>(c->prm.sigma, nshell);
    int reach = shell_reach(c->prm.sigma);
    if ((int)q.size() > MAX_QUADS || reach > MAX_REACH) return fail(c, WDLB_E_INVAL, "stencil too large");
    c->pad = make_pad(&c->desc, reach);
    std::vector<int> qs(2 * reach + 2, 0);
    for (auto &e : q) qs[e.c + reach + 1]++;
    for (int k = 1; k < (int)qs.size(); ++k) qs[k] += qs[k - 1];
    // the ball |e|^2 <= sigma^2/4 (order z, then y, then x), its reach and
    // the density tile
    std::vector<int> bx, by, bz;
    int rb = 0;
    const double s2 = c->prm.sigma * c->prm.sigma;
    const int RB = (int)std::ceil(c->prm.sigma / 2.0) + 1;
    for (int z = -RB; z <= RB; ++z)
        for (int y = -RB; y <= RB; ++y)
            for (int x = -RB; x <= RB; ++x)
                if (4.0 * (x * x + y * y + z * z) <= s2) {
                    bx.push_back(x);
                    by.push_back(y);
                    bz.push_back(z);
                    rb = std::max(rb, std::abs(x));
                }
    if ((int)bx.size() > MAX_BALL) return fail(c, WDLB_E_INVAL, "stencil too large");
    if (rb + 1 > c->pad.P) return fail(c, WDLB_E_INVAL, "sigma too small for the padded arrays");
    const int dtile = pick_density_tile(rb, sizeof(R), c->g.nx);
    if (dtile < 0) return fail(c, WDLB_E_INVAL, "sigma too large for the density tiles");
    // window offsets of the ball from the corner of a node's window
    const int LX = DENSITY_TILES[dtile].TX + 2 * rb + 1, LY = DENSITY_TILES[dtile].TY + 2 * rb + 1;
    std::vector<int> b(bx.size());
    for (size_t k = 0; k < bx.size(); ++k) b[k] = (bz[k] + rb) * LX * LY + (by[k] + rb) * LX + (bx[k] + rb);
    c->spec_s2 = 0;
    c->spec_b2 = 0;
    const int s2c = specialised_s2(c->prm.sigma);
    if (c->tile_req >= 0) {
        if (!tile_fits(SHELL_TILES[c->tile_req], reach, sizeof(R)))
            return fail(c, WDLB_E_INVAL, "the requested shell tile does not fit this sigma");
        c->tile = c->tile_mf = c->tile_req;
    } else {
        c->tile = c->tile_mf = pick_tile(reach, sizeof(R), c->g.nx);
        // the cache-gamma tile for the viscous/SMDB kernel: its buffer loads
        // take a lane offset below 2^31 bytes into one padded sub-lattice
        if (std::is_same<R, float>::value && s2c >= L1G_MIN_S2 && c->tile >= 0 && c->tile != NARROW_TILE &&
            compiled_shell<R>(s2c, c->tile, reach) && tile_fits(SHELL_TILES[L1G_TILE], reach, sizeof(R)) &&
            (double)sizeof(R) * (double)c->pad.NP < 2.0e9)
            c->tile = L1G_TILE;
        if (c->tile >= 0 && compiled_shell<R>(s2c, c->tile_mf, reach) && compiled_shell<R>(s2c, c->tile, reach))
            c->spec_s2 = s2c;
        // the FP64 shell for which no tile holds both LDS rings of the
        // viscous/SMDB kernel (2 sigma = 20, the largest compiled shell): it
        // runs compiled on the cache-gamma tile, the compiled mean-field
        // kernel on the first tile that holds its own two rings (same buffer
        // offset bound as above)
        if (std::is_same<R, double>::value && c->spec_s2 == 0 && s2c == 20 && c->tile >= 0 &&
            c->tile != NARROW_TILE && tile_fits(SHELL_TILES[L1G_TILE], reach, sizeof(R)) &&
            pick_tile_mf(reach, sizeof(R)) >= 0 && (double)sizeof(R) * (double)c->pad.NP < 2.0e9) {
            c->tile = L1G_TILE;
            c->tile_mf = pick_tile_mf(reach, sizeof(R));
            c->spec_s2 = s2c;
        }
        if (compiled_density<R>(s2c, dtile, rb)) c->spec_b2 = s2c;
    }
    if (c->tile < 0) return fail(c, WDLB_E_INVAL, "sigma too large for the shell tiles");
    HIPCHK(c, hipMemcpyAsync(c->quads, q.data(), q.size() * sizeof(Quad<R>), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->qstart, qs.data(), qs.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ball, b.data(), b.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    // padded arrays start at zero: beyond a wall they stay zero
    HIPCHK(c, hipMemsetAsync(c->rho_p, 0, c->padded_bytes, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->nq = (int)q.size();
    c->nball = (int)b.size();
    c->rb = rb;
    c->dtile = dtile;
    c->reach = reach;
    c->wS = 4.0 * M_PI / nshell;
    return WDLB_OK;
}

void drop_graphs(wdlb_ctx *c)
{
    for (auto &e : c->gexec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    for (auto &e : c->tgexec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    c->tg_T = nullptr;
}

wdlb_status tables(wdlb_ctx *c)
{
    drop_graphs(c);  // launch parameters may change
    if (c->store == WDLB_FP64) return upload_tables<double>(c);
    return upload_tables<float>(c);
}


const char *const KNAMES[WDLB_NKERNELS] = {"k_moments", "k_density", "k_meanfield", "k_shell", "k_collide",
                                           "k_thermal"};


template <typename R, int TX, int TY, int TZ, int NR, int NG>
wdlb_status launch_shell_pair(wdlb_ctx *c)
{
    const Geom g = c->g;
    const wdlb_params &p = c->prm;
    const double s = p.sigma;
    const int tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY, tz = (c->nz_run + TZ - 1) / TZ;
    const dim3 grid(tx * ty * tz), block(TX * TY * TZ);
    const size_t lmf = shell_lds_bytes(TX, TY, TZ, c->reach, sizeof(R), sizeof(R), NG > 0);
    const size_t lsh = shell_lds_bytes(TX, TY, TZ, c->reach, sizeof(V4<R>), sizeof(R), NG > 0);
    auto kmf = k_meanfield<R, TX, TY, TZ, NR, NG>;
    auto ksh = k_shell<R, TX, TY, TZ, NR, NG>;
    HIPCHK(c, hipFuncSetAttribute((const void *)kmf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lmf));
    HIPCHK(c, hipFuncSetAttribute((const void *)ksh, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lsh));
    wdlb_status st = WDLB_OK;
    if (c->shell_part & 1)
        st = launch(c, K_MEANFIELD, [&] {
            hipLaunchKernelGGL(kmf, grid, block, lmf, c->stream, g, c->pad, c->reach, (const R *)c->rho_p,
                               (const R *)c->jx, (const R *)c->jy, (const R *)c->jz, (const R *)c->gam_p,
                               (const Quad<R> *)c->quads, (const int *)c->qstart, R(-KT * s * s), R(p.g[0]),
                               R(p.g[1]), R(p.g[2]), tx, ty, tz, (V4<R> *)c->ru1_p, (V4<R> *)c->fmf);
        });
    if (st != WDLB_OK || !(c->shell_part & 2)) return st;
    return launch(c, K_SHELL, [&] {
        hipLaunchKernelGGL(ksh, grid, block, lsh, c->stream, g, c->pad, c->reach, (const V4<R> *)c->ru1_p,
                           (const R *)c->gam_p, (const V4<R> *)c->fmf, (const Quad<R> *)c->quads,
                           (const int *)c->qstart, R(2.0 * s * s * std::sqrt(KT / M_PI)), R(-(KT / 5.0) * s * s),
                           R(p.g[0]), R(p.g[1]), R(p.g[2]), p.smdb, tx, ty, tz, (R *)c->F, (R *)c->A,
                           (R *)c->shell_trace);
    });
}

// the viscous/SMDB kernel compiled for the shell 2 sigma = S2 on tile TIS
template <typename R, int S2, int TIS>
wdlb_status launch_visc_s(wdlb_ctx *c)
{
    constexpr int RC = Shell<S2>::R;
    constexpr ShellTile T = SHELL_TILES[TIS];
    const Geom g = c->g;
    const wdlb_params &p = c->prm;
    const double s = p.sigma;
    const int tx = (g.nx + T.TX - 1) / T.TX, ty = (g.ny + T.TY - 1) / T.TY, tz = (c->nz_run + T.TZ - 1) / T.TZ;
    const size_t lsh = shell_lds_bytes(T.TX, T.TY, T.TZ, RC, sizeof(V4<R>), sizeof(R), T.NG > 0);
    auto ksh = k_shell_s<R, S2, T.TX, T.TY, T.TZ, T.NR, T.NG>;
    HIPCHK(c, hipFuncSetAttribute((const void *)ksh, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lsh));
    return launch(c, K_SHELL, [&] {
        hipLaunchKernelGGL(ksh, dim3(tx * ty * tz), dim3(T.TX * T.TY * T.TZ), lsh, c->stream, g, c->pad,
                           (const V4<R> *)c->ru1_p, (const R *)c->gam_p, (const V4<R> *)c->fmf,
                           R(2.0 * s * s * std::sqrt(KT / M_PI)), R(-(KT / 5.0) * s * s), R(p.g[0]), R(p.g[1]),
                           R(p.g[2]), p.smdb, tx, ty, tz, (R *)c->F, (R *)c->A, (R *)c->shell_trace);
    });
}

// the pair specialised for the shell 2 sigma = S2: the mean-field kernel on
// tile TIM, the viscous/SMDB kernel on tile TIS
template <typename R, int S2, int TIM, int TIS>
wdlb_status launch_shell_pair_s(wdlb_ctx *c)
{
    constexpr int RC = Shell<S2>::R;
    static_assert(TIM >= 0 && TIS >= 0, "no tile for this shell");
    if (c->tile_mf != TIM || c->tile != TIS) return fail(c, WDLB_E_STATE, "compiled shell kernels are for other tiles");
    if (c->reach != RC) return fail(c, WDLB_E_STATE, "compiled shell does not match the shell of sigma");
    if constexpr (SHELL_TILES[TIM].NG == 0 || (TIM != TIS && TIS != L1G_TILE)) {
        // no compiled kernels on these tiles (the automatic choice never asks)
        return fail(c, WDLB_E_STATE, "no compiled shell kernels for these tiles");
    } else {
        const Geom g = c->g;
        const wdlb_params &p = c->prm;
        const double s = p.sigma;
        wdlb_status st = WDLB_OK;
        if (c->shell_part & 1) {
            constexpr ShellTile T = SHELL_TILES[TIM];
            const int tx = (g.nx + T.TX - 1) / T.TX, ty = (g.ny + T.TY - 1) / T.TY, tz = (c->nz_run + T.TZ - 1) / T.TZ;
            const size_t lmf = shell_lds_bytes(T.TX, T.TY, T.TZ, RC, sizeof(R), sizeof(R), T.NG > 0);
            auto kmf = k_meanfield_s<R, S2, T.TX, T.TY, T.TZ, T.NR, T.NG>;
            HIPCHK(c, hipFuncSetAttribute((const void *)kmf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lmf));
            st = launch(c, K_MEANFIELD, [&] {
                hipLaunchKernelGGL(kmf, dim3(tx * ty * tz), dim3(T.TX * T.TY * T.TZ), lmf, c->stream, g, c->pad,
                                   (const R *)c->rho_p, (const R *)c->jx, (const R *)c->jy, (const R *)c->jz,
                                   (const R *)c->gam_p, R(-KT * s * s), R(p.g[0]), R(p.g[1]), R(p.g[2]), tx, ty, tz,
                                   (V4<R> *)c->ru1_p, (V4<R> *)c->fmf);
            });
        }
        if (st != WDLB_OK || !(c->shell_part & 2)) return st;
        return launch_visc_s<R, S2, TIS>(c);
    }
}

// the table-driven pair on one tile
template <typename R>
wdlb_status launch_shell_table(wdlb_ctx *c, int tile)
{
    static_assert(NTILES == 7, "one case per entry of SHELL_TILES");
    switch (tile) {
    case 0: return launch_shell_pair<R, 32, 8, 2, 2, 5>(c);
    case 1: return launch_shell_pair<R, 32, 8, 2, 3, 6>(c);
    case 2: return launch_shell_pair<R, 32, 8, 2, 4, 8>(c);
    case 3: return launch_shell_pair<R, 32, 16, 1, 7, 13>(c);
    case 4: return launch_shell_pair<R, 16, 16, 1, 10, 0>(c);
    case 5: return launch_shell_pair<R, 16, 16, 2, 2, 5>(c);
    default: return launch_shell_pair<R, 32, 8, 2, 4, 0>(c);
    }
}

template <typename R>
wdlb_status launch_shells(wdlb_ctx *c)
{
#define WDLB_TW(S2) pick_tile_wide(Shell<S2>::R, sizeof(R))
#define WDLB_WIDE(S2) launch_shell_pair_s<R, S2, WDLB_TW(S2), WDLB_TW(S2)>(c)
    if (c->spec_s2 > 0) {
        if constexpr (std::is_same<R, double>::value) {
            if (c->tile == L1G_TILE && c->spec_s2 == 20)
                return launch_shell_pair_s<R, 20, pick_tile_mf(Shell<20>::R, sizeof(R)), L1G_TILE>(c);
        }
        if constexpr (std::is_same<R, float>::value) {
            if (c->tile == NARROW_TILE && c->spec_s2 == 8)
                return launch_shell_pair_s<R, 8, NARROW_TILE, NARROW_TILE>(c);
            if (c->tile == L1G_TILE) {
                static_assert(L1G_MIN_S2 == 16, "one case per shell that uses the cache-gamma tile");
                switch (c->spec_s2) {
                case 16: return launch_shell_pair_s<R, 16, WDLB_TW(16), L1G_TILE>(c);
                case 20: return launch_shell_pair_s<R, 20, WDLB_TW(20), L1G_TILE>(c);
                default: break;
                }
            }
        }
        switch (c->spec_s2) {
        case 6: return WDLB_WIDE(6);
        case 8: return WDLB_WIDE(8);
        case 12: return WDLB_WIDE(12);
        case 16: return WDLB_WIDE(16);
        case 20: return WDLB_WIDE(20);
        default: break;
        }
    }
#undef WDLB_WIDE
#undef WDLB_TW
    return launch_shell_table<R>(c, c->tile);
}

template <typename R, int TX, int TY, int TZ>
wdlb_status launch_density_g(wdlb_ctx *c)
{
    const Geom g = c->g;
    const double s = c->prm.sigma;
    const int tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY, tz = (c->nz_run + TZ - 1) / TZ;
    const size_t lds = density_lds_bytes(TX, TY, TZ, c->rb, sizeof(R));
    auto kern = k_density<R, TX, TY, TZ>;
    HIPCHK(c, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return launch(c, K_DENSITY, [&] {
        hipLaunchKernelGGL(kern, dim3(tx * ty * tz), dim3(TX * TY * TZ), lds, c->stream, g, c->pad, c->rb,
                           (const R *)c->rho_p, (const int *)c->ball, c->nball, R(1.0 / c->nball),
                           R(M_PI * s * s * s / 6.0), R(c->wS), tx, ty, tz, (R *)c->gam_p, c->flag);
    });
}

// specialised for the ball of 2 sigma = S2 on density tile DT
template <typename R, int S2, int DT>
wdlb_status launch_density_s(wdlb_ctx *c)
{
    constexpr int RB = Ball<S2>::RB;
    static_assert(DT >= 0, "no density tile for this ball");
    constexpr int TX = DENSITY_TILES[DT].TX, TY = DENSITY_TILES[DT].TY, TZ = DENSITY_TILES[DT].TZ;
    if (c->rb != RB || c->nball != Ball<S2>::NB || c->dtile != DT)
        return fail(c, WDLB_E_STATE, "compiled ball does not match the ball of sigma");
    const Geom g = c->g;
    const double s = c->prm.sigma;
    const int tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY, tz = (c->nz_run + TZ - 1) / TZ;
    const size_t lds = density_lds_bytes(TX, TY, TZ, RB, sizeof(R));
    auto kern = k_density_s<R, S2, TX, TY, TZ>;
    HIPCHK(c, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return launch(c, K_DENSITY, [&] {
        hipLaunchKernelGGL(kern, dim3(tx * ty * tz), dim3(TX * TY * TZ), lds, c->stream, g, c->pad,
                           (const R *)c->rho_p, R(1.0 / c->nball), R(M_PI * s * s * s / 6.0), R(c->wS), tx, ty, tz,
                           (R *)c->gam_p, c->flag);
    });
}

template <typename R>
wdlb_status launch_density(wdlb_ctx *c)
{
#define WDLB_WIDE(S2) launch_density_s<R, S2, pick_density_tile(Ball<S2>::RB, sizeof(R), 1 << 30)>(c)
    if constexpr (std::is_same<R, float>::value)
        if (c->spec_b2 == 8 && c->dtile == NARROW_DENSITY_TILE)
            return launch_density_s<R, 8, NARROW_DENSITY_TILE>(c);
    switch (c->spec_b2) {
    case 6: return WDLB_WIDE(6);
    case 8: return WDLB_WIDE(8);
    case 12: return WDLB_WIDE(12);
    case 16: return WDLB_WIDE(16);
    case 20: return WDLB_WIDE(20);
    default: break;
    }
#undef WDLB_WIDE
    switch (c->dtile) {
    case 0: return launch_density_g<R, 32, 8, 2>(c);
    case 1: return launch_density_g<R, 16, 8, 1>(c);
    default: return launch_density_g<R, 16, 16, 2>(c);
    }
}

// one pass of the step kernels on the current buffers; READ stops after the
// fields (u = (j + F/2)/rho into u_rd) and leaves the state untouched
template <typename R, typename HS, typename D, bool READ>
wdlb_status run_pass(wdlb_ctx *c)
{
    const Geom g = c->g;
    const Pad pd = c->pad;
    const int bs = 256;
    dim3 grid = grid1((long long)g.nx * g.ny * c->nz_run, bs);  // planes 0 .. nz_run - 1
    // per-node kernels with pulls: tiles of 64 x 4 (16 x 16 for narrow lattices), planes swept per XCD
    const int lgx = g.nx >= 64 ? 6 : (g.nx >= 32 ? 5 : 4);
    const NodeTiles nt{(g.nx + (1 << lgx) - 1) >> lgx, (g.ny + (256 >> lgx) - 1) / (256 >> lgx), c->nz_run, lgx};
    const dim3 gridt((unsigned)nt.tx * nt.ty * nt.nzr);
    const int cur = c->cur, nxt = cur ^ 1;
    auto *ru_in = (const V4<R> *)c->ru[cur];
    auto *h_in = (const HS *)c->h[cur];
    const wdlb_params &p = c->prm;
    const double s = p.sigma;
    wdlb_status st;
    st = launch(c, K_MOMENTS, [&] {
        hipLaunchKernelGGL((k_moments<R, HS, D>), gridt, dim3(bs), 0, c->stream, g, nt, pd, ru_in, h_in, (R *)c->rho_p,
                           (R *)c->jx, (R *)c->jy, (R *)c->jz, c->flag);
    });
    if (st != WDLB_OK) return st;
    if (p.nonlocal) {
        st = launch_density<R>(c);
        if (st != WDLB_OK) return st;
        st = launch_shells<R>(c);
        if (st != WDLB_OK) return st;
    } else {
        st = launch(c, K_SHELL, [&] {
            hipLaunchKernelGGL((k_plainforce<R>), grid, dim3(bs), 0, c->stream, g, pd, (const R *)c->rho_p,
                               R(p.g[0]), R(p.g[1]), R(p.g[2]), (R *)c->F, (R *)c->A);
        });
        if (st != WDLB_OK) return st;
    }
    st = launch(c, K_COLLIDE, [&] {
        hipLaunchKernelGGL((k_collide<R, HS, D, READ>), gridt, dim3(bs), 0, c->stream, g, nt, (const R *)c->F,
                           (const R *)c->A, R(1.0 / p.tau), R(1.0 - 0.5 / p.tau), ru_in, h_in, (V4<R> *)c->ru[nxt],
                           (HS *)c->h[nxt], (R *)c->u_rd, (uint64_t)c->step);
    });
    if (st != WDLB_OK) return st;
    if (READ)
        hipLaunchKernelGGL((k_unpad<R>), grid, dim3(bs), 0, c->stream, g, pd, (const R *)c->rho_p,
                           (R *)c->rho_rd);
    HIPCHK(c, hipGetLastError());
    return WDLB_OK;
}

template <bool READ>
wdlb_status pass(wdlb_ctx *c)
{
    switch (c->prec) {
    case WDLB_FP64: return run_pass<double, double, double, READ>(c);
    case WDLB_FP32: return run_pass<float, float, float, READ>(c);
    case WDLB_BF16_NEQ: return run_pass<float, bf16, float, READ>(c);
    case WDLB_FP32_LOCAL64: return run_pass<float, float, double, READ>(c);
    default: return run_pass<float, bf16, double, READ>(c);
    }
}

wdlb_status check_flag(wdlb_ctx *c)
{
    int f = 0;
    HIPCHK(c, hipMemcpyAsync(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (f & FLAG_RHO) return fail(c, WDLB_E_UNSTABLE, "non-finite or non-positive density");
    if (f & FLAG_ETA) return fail(c, WDLB_E_UNSTABLE, "midpoint packing fraction reached 1");
    if (f & FLAG_T) return fail(c, WDLB_E_UNSTABLE, "non-finite or non-positive temperature");
    return WDLB_OK;
}

template <typename R>
wdlb_status copy_out(wdlb_ctx *c, const void *dev, size_t n, double *host)
{
    if (!host) return WDLB_OK;
    std::vector<R> tmp(n);
    HIPCHK(c, hipMemcpyAsync(tmp.data(), dev, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < n; ++i) host[i] = (double)tmp[i];
    return WDLB_OK;
}

wdlb_status copy_out_r(wdlb_ctx *c, const void *dev, size_t n, double *host)
{
    return c->store == WDLB_FP64 ? copy_out<double>(c, dev, n, host) : copy_out<float>(c, dev, n, host);
}

wdlb_status read_pass(wdlb_ctx *c)
{
    if (!c->inited) return fail(c, WDLB_E_STATE, "context not initialised");
    const int prof = c->prof;
    c->prof = 0;  // only the stepping kernels are timed
    wdlb_status st = pass<true>(c);
    c->prof = prof;
    if (st != WDLB_OK) return st;
    return check_flag(c);
}

struct StateHeader {
    char magic[8];
    int32_t nx, ny, nz, walls, precision, pad;
    int64_t step;
};

size_t state_bytes(const wdlb_ctx *c)
{
    const size_t N = (size_t)c->g.N;
    return sizeof(StateHeader) + 4 * c->rsize * N + (size_t)c->hplanes * c->hsize * N;
}

// Thermal fields at given n, u, T.  The device part (thermal_launch) reads
// n[N], u[3N], T[N] and writes Q[N], B[3N], F^T[3N] (arrays of the storage
// real) through the per-step arrays that the next step rewrites before it
// reads them: n is padded into the density array, the step's density kernel
// forms the contact values from it, (n, u) is padded into the (rho, u1)
// array and T over the density array.  The state is untouched.
template <typename R>
wdlb_status thermal_launch(wdlb_ctx *c, const R *n, const R *u, const R *T, R *Q, R *B, R *FT)
{
    const Geom g = c->g;
    const Pad pd = c->pad;
    const dim3 grid = grid1(g.N, 256);
    hipLaunchKernelGGL((k_pad<R>), grid, dim3(256), 0, c->stream, g, pd, n, (R *)c->rho_p);
    HIPCHK(c, hipGetLastError());
    const int prof = c->prof;
    c->prof = prof & (1 << K_THERMAL);  // only k_thermal is timed here
    wdlb_status st = launch_density<R>(c);
    c->prof = prof;
    if (st != WDLB_OK) return st;
    hipLaunchKernelGGL((k_pad_ru<R>), grid, dim3(256), 0, c->stream, g, pd, n, u, (V4<R> *)c->ru1_p);
    hipLaunchKernelGGL((k_pad<R>), grid, dim3(256), 0, c->stream, g, pd, T, (R *)c->rho_p);
    HIPCHK(c, hipGetLastError());
    st = launch_thermal<R>(c, Q, B, FT);
    if (st != WDLB_OK) return st;
    HIPCHK(c, hipGetLastError());
    return WDLB_OK;
}

// host fields: n to jx, T to jy, u to u_rd (FP64 -> storage real), Q to
// rho_rd, B to F and F^T to the first three planes of A, then back
template <typename R>
wdlb_status thermal_fields(wdlb_ctx *c, const double *h_n, const double *h_u, const double *h_T, double *h_Q,
                           double *h_B, double *h_FT)
{
    const size_t N = (size_t)c->g.N;
    {
        std::vector<R> v(N);
        for (size_t i = 0; i < N; ++i) v[i] = (R)h_n[i];
        HIPCHK(c, hipMemcpyAsync(c->jx, v.data(), N * sizeof(R), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < N; ++i) v[i] = (R)h_T[i];
        HIPCHK(c, hipMemcpyAsync(c->jy, v.data(), N * sizeof(R), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        std::vector<R> w(3 * N);
        for (size_t i = 0; i < 3 * N; ++i) w[i] = (R)h_u[i];
        HIPCHK(c, hipMemcpyAsync(c->u_rd, w.data(), 3 * N * sizeof(R), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    // the call raises and reads its own flag word (the first per-plane word,
    // which only stacked lattices use), so that a step's instability not yet
    // reported by a synchronising call survives it
    struct FlagSwap {
        wdlb_ctx *c;
        int *saved;
        ~FlagSwap() { c->flag = saved; }
    } swap{c, c->flag};
    c->flag = swap.saved + 1;
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    wdlb_status st = thermal_launch<R>(c, (const R *)c->jx, (const R *)c->u_rd, (const R *)c->jy, (R *)c->rho_rd,
                                       (R *)c->F, (R *)c->A);
    if (st != WDLB_OK) return st;
    if ((st = check_flag(c)) != WDLB_OK) return st;
    if ((st = copy_out_r(c, c->rho_rd, N, h_Q)) != WDLB_OK) return st;
    if ((st = copy_out_r(c, c->F, 3 * N, h_B)) != WDLB_OK) return st;
    return copy_out_r(c, c->A, 3 * N, h_FT);
}

// The energy balance at rest (wdlb_conduction_at_rest): n to jx, T to jy;
// the contact values of n once; then per step T is padded over the density
// array, the thermal fields at u = 0 go to rho_rd (Q), F (B) and A (F^T,
// unused), and k_conduct writes the new T into jy.  The state is untouched.
template <typename R>
wdlb_status conduction_steps(wdlb_ctx *c, const double *h_n, double *h_T, double omega0, double dt, int64_t nsteps)
{
    const Geom g = c->g;
    const Pad pd = c->pad;
    const size_t N = (size_t)g.N;
    {
        std::vector<R> v(N);
        for (size_t i = 0; i < N; ++i) v[i] = (R)h_n[i];
        HIPCHK(c, hipMemcpyAsync(c->jx, v.data(), N * sizeof(R), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < N; ++i) v[i] = (R)h_T[i];
        HIPCHK(c, hipMemcpyAsync(c->jy, v.data(), N * sizeof(R), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    struct FlagSwap {  // the call's own flag word, as in thermal_fields
        wdlb_ctx *c;
        int *saved;
        ~FlagSwap() { c->flag = saved; }
    } swap{c, c->flag};
    c->flag = swap.saved + 1;
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    const dim3 grid = grid1(g.N, 256);
    hipLaunchKernelGGL((k_pad<R>), grid, dim3(256), 0, c->stream, g, pd, (const R *)c->jx, (R *)c->rho_p);
    HIPCHK(c, hipGetLastError());
    const int prof = c->prof;
    c->prof = prof & (1 << K_THERMAL);
    wdlb_status st = launch_density<R>(c);
    c->prof = prof;
    if (st != WDLB_OK) return st;
    hipLaunchKernelGGL((k_pad_ru<R>), grid, dim3(256), 0, c->stream, g, pd, (const R *)c->jx, (const R *)nullptr,
                       (V4<R> *)c->ru1_p);
    HIPCHK(c, hipGetLastError());
    for (int64_t t = 0; t < nsteps; ++t) {
        hipLaunchKernelGGL((k_pad<R>), grid, dim3(256), 0, c->stream, g, pd, (const R *)c->jy, (R *)c->rho_p);
        st = launch_thermal<R>(c, (R *)c->rho_rd, (R *)c->F, (R *)c->A);
        if (st != WDLB_OK) return st;
        hipLaunchKernelGGL((k_conduct<R>), grid, dim3(256), 0, c->stream, g, pd, (const R *)c->rho_p,
                           (const V4<R> *)c->ru1_p, (const R *)c->rho_rd, (const R *)c->F, R(2.5 / omega0),
                           R(0.5 / omega0), R(dt), (R *)c->jy);
        HIPCHK(c, hipGetLastError());
    }
    if ((st = check_flag(c)) != WDLB_OK) return st;
    return copy_out_r(c, c->jy, N, h_T);
}

// One step of the coupled thermal flow (storage R, FP64 or FP32; the local
// kernels in D) on the current buffers, T (N values of R on the device)
// updated in place.  The step's kernels
// with the mean-field and viscous/SMDB kernels launched apart:
//   k_moments, k_density, k_meanfield;
//   k_pad         T over the density array (no longer needed);
//   k_thermal     F^T, B and the conduction part of Q (the variant at u = 0:
//                 they depend on n and T alone) into the next parity's h
//                 array (rewritten by the collision only after they are read);
//   k_th_u1       F^mf <- theta F^mf, u1 = j/rho + (g + theta F^mf + F^T)/2
//                 (into the (rho, u1) array);
//   k_shell       F^v and A from that u1, and the trace sums sum_e k.W;
//   k_th_force    F = rho (g + theta F^mf + sqrt(theta) F^v + F^T), A <- theta A,
//                 Q += its compression part -(n sigma^2 T / 2) sum_e k.W;
//   k_energy_fixed  the advection, work, delta q and Q part of dT/dt (rho_rd),
//                 marching along z like k_energy_sub;
//   k_collide, then k_th_post  the temperature term relaxed at 1/tau;
//   nsub sub-steps of k_energy_sub (u_rd between them, the last into T).
template <typename R, typename D>
wdlb_status thermal_flow_pass(wdlb_ctx *c, R *T, int nsub)
{
    const Geom g = c->g;
    const Pad pd = c->pad;
    const int bs = 256;
    const dim3 grid = grid1(g.N, bs);
    const int lgx = g.nx >= 64 ? 6 : (g.nx >= 32 ? 5 : 4);
    const NodeTiles nt{(g.nx + (1 << lgx) - 1) >> lgx, (g.ny + (256 >> lgx) - 1) / (256 >> lgx), c->nz_run, lgx};
    const dim3 gridt((unsigned)nt.tx * nt.ty * nt.nzr);
    const int cur = c->cur, nxt = cur ^ 1;
    auto *ru_in = (const V4<R> *)c->ru[cur];
    auto *h_in = (const R *)c->h[cur];
    const wdlb_params &p = c->prm;
    const R kT = R(KT), omega0 = R(1.0 / p.tau);
    const long long N = g.N;
    R *Qf = (R *)c->h[nxt], *Bf = Qf + N, *FT = Qf + 4 * N, *Sk = Qf + 7 * N;
    R *Rfix = (R *)c->rho_rd, *Tmid = (R *)c->u_rd;
    wdlb_status st = launch(c, K_MOMENTS, [&] {
        hipLaunchKernelGGL((k_moments<R, R, D>), gridt, dim3(bs), 0, c->stream, g, nt, pd, ru_in, h_in, (R *)c->rho_p,
                           (R *)c->jx, (R *)c->jy, (R *)c->jz, c->flag);
    });
    if (st != WDLB_OK) return st;
    if ((st = launch_density<R>(c)) != WDLB_OK) return st;
    struct PartReset {
        wdlb_ctx *c;
        ~PartReset()
        {
            c->shell_part = 3;
            c->shell_trace = nullptr;
        }
    } reset{c};
    c->shell_part = 1;
    if ((st = launch_shells<R>(c)) != WDLB_OK) return st;
    hipLaunchKernelGGL((k_pad<R>), grid, dim3(bs), 0, c->stream, g, pd, (const R *)T, (R *)c->rho_p);
    HIPCHK(c, hipGetLastError());
    if ((st = launch_thermal<R, true>(c, Qf, Bf, FT)) != WDLB_OK) return st;
    hipLaunchKernelGGL((k_th_u1<R>), grid, dim3(bs), 0, c->stream, g, pd, (const R *)T, kT, (const R *)c->jx,
                       (const R *)c->jy, (const R *)c->jz, (const R *)FT, R(p.g[0]), R(p.g[1]), R(p.g[2]),
                       (V4<R> *)c->fmf, (V4<R> *)c->ru1_p, c->flag);
    HIPCHK(c, hipGetLastError());
    c->shell_part = 2;
    c->shell_trace = Sk;
    if ((st = launch_shells<R>(c)) != WDLB_OK) return st;
    c->shell_part = 3;
    c->shell_trace = nullptr;
    hipLaunchKernelGGL((k_th_force<R>), grid, dim3(bs), 0, c->stream, g, pd, (const V4<R> *)c->ru1_p, (const R *)T,
                       kT, (const V4<R> *)c->fmf, (const R *)FT, (const R *)Sk, R(p.sigma * p.sigma), R(p.g[0]),
                       R(p.g[1]), R(p.g[2]), (R *)c->F, (R *)c->A, Qf);
    // the energy kernels march along z in chunks of zc planes (a quarter of
    // the lattice's, at most 4, or 16 on lattices of 2^21 nodes and more)
    const int zc = std::max(1, std::min(g.nz / 4, g.N >= (1LL << 21) ? 16 : 4));
    const dim3 egrid((g.nx + ENERGY_TX - 1) / ENERGY_TX, (g.ny + ENERGY_TY - 1) / ENERGY_TY, (g.nz + zc - 1) / zc);
    hipLaunchKernelGGL((k_energy_fixed<R>), egrid, dim3(ENERGY_TX * ENERGY_TY), 0, c->stream, g, pd, zc,
                       (const V4<R> *)c->ru1_p, (const R *)c->rho_p, (const R *)c->jx, (const R *)c->jy,
                       (const R *)c->jz, (const R *)c->F, (const R *)c->A, (const R *)Qf, (const R *)Bf, omega0, Rfix);
    HIPCHK(c, hipGetLastError());
    st = launch(c, K_COLLIDE, [&] {
        hipLaunchKernelGGL((k_collide<R, R, D, false>), gridt, dim3(bs), 0, c->stream, g, nt, (const R *)c->F,
                           (const R *)c->A, R(1.0 / p.tau), R(1.0 - 0.5 / p.tau), ru_in, h_in, (V4<R> *)c->ru[nxt],
                           (R *)c->h[nxt], (R *)c->u_rd, (uint64_t)c->step);
    });
    if (st != WDLB_OK) return st;
    hipLaunchKernelGGL((k_th_post<R, D>), grid, dim3(bs), 0, c->stream, g, pd, (const V4<R> *)c->ru1_p, (const R *)T,
                       D(KT), D(1.0 / p.tau), (R *)c->h[nxt]);
    for (int s = 0; s < nsub; ++s) {
        const bool last = s == nsub - 1;
        hipLaunchKernelGGL((k_energy_sub<R>), egrid, dim3(ENERGY_TX * ENERGY_TY), 0, c->stream, g, pd, zc,
                           (const R *)c->rho_p, (const V4<R> *)c->ru1_p, (const R *)Rfix, omega0, nsub,
                           last ? T : Tmid);
        if (!last)
            hipLaunchKernelGGL((k_pad<R>), grid, dim3(bs), 0, c->stream, g, pd, (const R *)Tmid, (R *)c->rho_p);
    }
    HIPCHK(c, hipGetLastError());
    return WDLB_OK;
}

// the coupled thermal flow runs on FP64 or FP32 storage (not the BF16
// deviations, whose rounding and closure the added term would bypass), the
// nonlocal fields, one slit (not a stacked lattice)
wdlb_status thermal_flow_ok(wdlb_ctx *c)
{
    if (c->store == WDLB_BF16_NEQ) return fail(c, WDLB_E_INVAL, "the coupled thermal flow needs FP64 or FP32 storage");
    if (!c->prm.nonlocal) return fail(c, WDLB_E_INVAL, "the coupled thermal flow needs the nonlocal fields");
    if (c->g.zp != nullptr) return fail(c, WDLB_E_STATE, "coupled thermal flow on a stacked lattice");
    return WDLB_OK;
}

template <typename R>
wdlb_status init_thermal(wdlb_ctx *c, const double *h_T, R *d_T)
{
    const Geom g = c->g;
    std::vector<R> v((size_t)g.N);
    for (long long i = 0; i < g.N; ++i) v[i] = (R)h_T[i];
    HIPCHK(c, hipMemcpyAsync(d_T, v.data(), (size_t)g.N * sizeof(R), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL((k_th_init<R>), grid1(g.N, 256), dim3(256), 0, c->stream, g, (const V4<R> *)c->ru[0],
                       (const R *)d_T, KT, (R *)c->h[0]);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return WDLB_OK;
}

wdlb_status thermal_flow_step(wdlb_ctx *c, void *d_T, int nsub)
{
    switch (c->prec) {
    case WDLB_FP64: return thermal_flow_pass<double, double>(c, (double *)d_T, nsub);
    case WDLB_FP32: return thermal_flow_pass<float, float>(c, (float *)d_T, nsub);
    default: return thermal_flow_pass<float, double>(c, (float *)d_T, nsub);  // FP32 storage, FP64 local
    }
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
    c->store = storage_of(c->prec);
    c->rsize = c->store == WDLB_FP64 ? 8 : 4;
    c->hsize = c->store == WDLB_FP64 ? 8 : (c->store == WDLB_BF16_NEQ ? 2 : 4);
    c->hplanes = c->store == WDLB_BF16_NEQ ? hplanes<bf16>() : 19;
    c->g.nx = desc->nx;
    c->g.ny = desc->ny;
    c->g.nz = desc->nz;
    c->g.walls = desc->walls_z ? 1 : 0;
    c->g.N = (long long)desc->nx * desc->ny * desc->nz;
    c->g.tiny = 0;
    c->g.zp = nullptr;
    c->nz_run = desc->nz;
    c->ws = (char *)d_workspace;
    c->ws_bytes = bytes;
    for (int b = 0; b < 2; ++b) {
        c->ru[b] = c->ws + L.off_ru[b];
        c->h[b] = c->ws + L.off_h[b];
    }
    c->rho_p = c->ws + L.off_rho_p;
    c->gam_p = c->ws + L.off_gam_p;
    c->ru1_p = c->ws + L.off_ru1_p;
    c->padded_bytes = L.off_j[0] - L.off_rho_p;
    c->scratch = c->gam_p;  // 8 NP >= 8 N reals, free between steps
    c->jx = c->ws + L.off_j[0];
    c->jy = c->ws + L.off_j[1];
    c->jz = c->ws + L.off_j[2];
    c->fmf = c->ws + L.off_fmf;
    c->F = c->ws + L.off_F;
    c->A = c->ws + L.off_A;
    c->u_rd = c->ws + L.off_urd;
    c->rho_rd = c->ws + L.off_rhord;
    c->planes = (double *)(c->ws + L.off_planes);
    c->flag = (int *)(c->ws + L.off_flag);
    c->quads = c->ws + L.off_quads;
    c->qstart = (int *)(c->ws + L.off_qstart);
    c->ball = (int *)(c->ws + L.off_ball);
    c->zp_dev = (ZPlane *)(c->ws + L.off_zp);
    c->cur = 0;
    c->step = 0;
    c->inited = false;
    c->tile_req = -1;
    // no instability is pending before the first step (a sync or an
    // asynchronous thermal-field call before init reads these words)
    if (hipMemsetAsync(c->flag, 0, sizeof(int) * (1 + (size_t)desc->nz), c->stream) != hipSuccess) {
        delete c;
        return WDLB_E_HIP;
    }
    wdlb_status st = tables(c);
    if (st != WDLB_OK) {
        delete c;
        return st;
    }
    *out = c;
    return WDLB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The static workspace of wdlb_create_static: one array per device in the
// library's code object, so a context can be made without any device
// allocation.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// used.  At most one context per device holds it at a time.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t STATIC_WS_BYTES = WDLB_STATIC_WORKSPACE_BYTES;
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[STATIC_MAX_DEVICES] = {};
bool g_static_busy[STATIC_MAX_DEVICES] = {};
}  // namespace
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

extern "C" {

wdlb_status wdlb_create_static(const wdlb_lattice_desc *desc, const wdlb_params *params, wdlb_ctx **out)
{
    if (!out) return WDLB_E_INVAL;
    *out = nullptr;
    if (!desc_ok(desc) || !params_ok(params)) return WDLB_E_INVAL;
    if (layout(desc).total > STATIC_WS_BYTES) return WDLB_E_NOMEM;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES) return WDLB_E_HIP;
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_busy[dev]) return WDLB_E_STATE;
        if (!g_static_ptr[dev]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
                (void)hipGetLastError();
                return WDLB_E_HIP;
            }
            g_static_ptr[dev] = p;
        }
        ws = g_static_ptr[dev];
        g_static_busy[dev] = true;
    }
    // the same context as wdlb_create on a caller workspace; create clears
    // the padded arrays and uploads the tables, init writes the state
    wdlb_status st = wdlb_create(desc, params, ws, STATIC_WS_BYTES, out);
    if (st != WDLB_OK) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[dev] = false;
        return st;
    }
    (*out)->static_dev = dev;
    (*out)->graphs = false;  // graph capture and instantiation allocate
    return WDLB_OK;
}

wdlb_status wdlb_set_params(wdlb_ctx *c, const wdlb_params *params)
{
    if (!c) return WDLB_E_INVAL;
    if (!params_ok(params)) return fail(c, WDLB_E_INVAL, "invalid parameters");
    c->prm = *params;
    return tables(c);
}

// the two-step graph for the current parity, captured on first use (on the
// private stream: the caller's may be the null stream, which cannot be
// captured).  *ex stays null if capture is not possible; the caller then
// steps eagerly.
static wdlb_status step_graph(wdlb_ctx *c, hipGraphExec_t *ex)
{
    if (c->graph_nz_run != c->nz_run) {
        drop_graphs(c);
        c->graph_nz_run = c->nz_run;
    }
    const int par = c->cur;
    if (!c->gexec[par]) {
        if (!c->cap && hipStreamCreate(&c->cap) != hipSuccess) {
            c->graphs = false;
            return WDLB_OK;
        }
        hipStream_t keep = c->stream;
        c->stream = c->cap;
        hipGraph_t graph = nullptr;
        bool ok = hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed) == hipSuccess;
        wdlb_status st = WDLB_OK;
        if (ok) {
            st = pass<false>(c);
            c->cur ^= 1;
            if (st == WDLB_OK) st = pass<false>(c);
            c->cur ^= 1;
            ok = hipStreamEndCapture(c->cap, &graph) == hipSuccess && st == WDLB_OK && graph != nullptr;
        }
        c->stream = keep;
        hipGraphExec_t e = nullptr;
        if (ok) ok = hipGraphInstantiate(&e, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        if (!ok) {
            c->graphs = false;  // step eagerly from now on
            return WDLB_OK;
        }
        c->gexec[par] = e;
    }
    *ex = c->gexec[par];
    return WDLB_OK;
}

// a graph of two coupled thermal-flow steps from the current parity, for
// the T array d_T and nsub sub-steps (captured as step_graph captures the
// isothermal pair; a new T array or nsub drops the pair)
static wdlb_status thermal_graph(wdlb_ctx *c, void *d_T, int nsub, hipGraphExec_t *ex)
{
    if (c->graph_nz_run != c->nz_run) {
        drop_graphs(c);
        c->graph_nz_run = c->nz_run;
    }
    if (c->tg_T != d_T || c->tg_nsub != nsub) {
        for (auto &e : c->tgexec)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
        c->tg_T = d_T;
        c->tg_nsub = nsub;
    }
    const int par = c->cur;
    if (!c->tgexec[par]) {
        if (!c->cap && hipStreamCreate(&c->cap) != hipSuccess) {
            c->graphs = false;
            return WDLB_OK;
        }
        hipStream_t keep = c->stream;
        c->stream = c->cap;
        hipGraph_t graph = nullptr;
        bool ok = hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed) == hipSuccess;
        wdlb_status st = WDLB_OK;
        if (ok) {
            st = thermal_flow_step(c, d_T, nsub);
            c->cur ^= 1;
            if (st == WDLB_OK) st = thermal_flow_step(c, d_T, nsub);
            c->cur ^= 1;
            ok = hipStreamEndCapture(c->cap, &graph) == hipSuccess && st == WDLB_OK && graph != nullptr;
        }
        c->stream = keep;
        hipGraphExec_t e = nullptr;
        if (ok) ok = hipGraphInstantiate(&e, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        if (!ok) {
            c->graphs = false;  // step eagerly from now on
            return WDLB_OK;
        }
        c->tgexec[par] = e;
    }
    *ex = c->tgexec[par];
    return WDLB_OK;
}

static wdlb_status do_init(wdlb_ctx *c, int uniform, const double u0[3], const double *h_n, const double *h_u)
{
    const Geom g = c->g;
    const size_t N = (size_t)g.N;
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    double n0 = 6.0 * c->prm.eta / (M_PI * c->prm.sigma * c->prm.sigma * c->prm.sigma);
    c->cur = 0;
    if (!uniform) {
        if (c->store == WDLB_FP64) {
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
    switch (c->store) {
    case WDLB_FP64:
        if (uniform)
            hipLaunchKernelGGL((k_fill<double>), grid, dim3(256), 0, c->stream, g, (V4<double> *)c->ru[0], n0, ux,
                               uy, uz, 0LL, g.N);
        hipLaunchKernelGGL((k_init<double, double>), grid, dim3(256), 0, c->stream, g,
                           (const V4<double> *)c->ru[0], (double *)c->h[0], 0LL, g.N);
        break;
    case WDLB_FP32:
        if (uniform)
            hipLaunchKernelGGL((k_fill<float>), grid, dim3(256), 0, c->stream, g, (V4<float> *)c->ru[0],
                               (float)n0, (float)ux, (float)uy, (float)uz, 0LL, g.N);
        hipLaunchKernelGGL((k_init<float, float>), grid, dim3(256), 0, c->stream, g, (const V4<float> *)c->ru[0],
                           (float *)c->h[0], 0LL, g.N);
        break;
    default:
        if (uniform)
            hipLaunchKernelGGL((k_fill<float>), grid, dim3(256), 0, c->stream, g, (V4<float> *)c->ru[0],
                               (float)n0, (float)ux, (float)uy, (float)uz, 0LL, g.N);
        hipLaunchKernelGGL((k_init<float, bf16>), grid, dim3(256), 0, c->stream, g, (const V4<float> *)c->ru[0],
                           (bf16 *)c->h[0], 0LL, g.N);
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
    // pairs of steps by graph replay (not while kernels are timed, and not
    // in the BF16 mode, whose rounding dither is keyed by the step number)
    if (c->graphs && c->prof == 0 && c->store != WDLB_BF16_NEQ) {
        while (nsteps >= 2) {
            hipGraphExec_t ex = nullptr;
            wdlb_status st = step_graph(c, &ex);
            if (st != WDLB_OK) return st;
            if (!ex) break;  // capture not available: step eagerly
            HIPCHK(c, hipGraphLaunch(ex, c->stream));
            c->step += 2;
            nsteps -= 2;
        }
    }
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
    if ((st = copy_out_r(c, c->rho_rd, N, h_n)) != WDLB_OK) return st;
    if ((st = copy_out_r(c, c->u_rd, 3 * N, h_u)) != WDLB_OK) return st;
    if ((st = copy_out_r(c, c->F, 3 * N, h_F)) != WDLB_OK) return st;
    if (h_A0) {
        std::vector<double> a6(6 * N);
        if ((st = copy_out_r(c, c->A, 6 * N, a6.data())) != WDLB_OK) return st;
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

wdlb_status wdlb_thermal_fields(wdlb_ctx *c, const double *h_n, const double *h_u, const double *h_T, double *h_Q,
                                double *h_B, double *h_FT)
{
    if (!c) return WDLB_E_INVAL;
    if (!h_n || !h_u || !h_T) return fail(c, WDLB_E_INVAL, "null field");
    if (c->g.zp != nullptr) return fail(c, WDLB_E_STATE, "thermal fields of a stacked lattice");
    const size_t N = (size_t)c->g.N;
    for (size_t i = 0; i < N; ++i) {
        if (!(std::isfinite(h_n[i]) && h_n[i] >= 0.0)) return fail(c, WDLB_E_INVAL, "density negative or not finite");
        if (!(std::isfinite(h_T[i]) && h_T[i] > 0.0)) return fail(c, WDLB_E_INVAL, "temperature not positive");
    }
    for (size_t i = 0; i < 3 * N; ++i)
        if (!std::isfinite(h_u[i])) return fail(c, WDLB_E_INVAL, "velocity not finite");
    if (c->store == WDLB_FP64) return thermal_fields<double>(c, h_n, h_u, h_T, h_Q, h_B, h_FT);
    return thermal_fields<float>(c, h_n, h_u, h_T, h_Q, h_B, h_FT);
}

wdlb_status wdlb_conduction_at_rest(wdlb_ctx *c, const double *h_n, double *h_T, double omega0, double dt,
                                    int64_t nsteps)
{
    if (!c) return WDLB_E_INVAL;
    if (!h_n || !h_T) return fail(c, WDLB_E_INVAL, "null field");
    if (!(omega0 > 0.0) || !(dt >= 0.0) || !std::isfinite(dt) || nsteps < 0)
        return fail(c, WDLB_E_INVAL, "omega0 must be positive, dt finite and non-negative, nsteps non-negative");
    if (c->g.zp != nullptr) return fail(c, WDLB_E_STATE, "conduction on a stacked lattice");
    const size_t N = (size_t)c->g.N;
    for (size_t i = 0; i < N; ++i) {
        if (!(std::isfinite(h_n[i]) && h_n[i] > 0.0)) return fail(c, WDLB_E_INVAL, "density not positive");
        if (!(std::isfinite(h_T[i]) && h_T[i] > 0.0)) return fail(c, WDLB_E_INVAL, "temperature not positive");
    }
    if (c->store == WDLB_FP64) return conduction_steps<double>(c, h_n, h_T, omega0, dt, nsteps);
    return conduction_steps<float>(c, h_n, h_T, omega0, dt, nsteps);
}

wdlb_status wdlb_thermal_fields_device(wdlb_ctx *c, const void *d_n, const void *d_u, const void *d_T, void *d_Q,
                                       void *d_B, void *d_FT)
{
    if (!c) return WDLB_E_INVAL;
    if (!d_n || !d_u || !d_T || !d_Q || !d_B || !d_FT) return fail(c, WDLB_E_INVAL, "null device array");
    if (c->g.zp != nullptr) return fail(c, WDLB_E_STATE, "thermal fields of a stacked lattice");
    if (c->store == WDLB_FP64)
        return thermal_launch<double>(c, (const double *)d_n, (const double *)d_u, (const double *)d_T,
                                      (double *)d_Q, (double *)d_B, (double *)d_FT);
    return thermal_launch<float>(c, (const float *)d_n, (const float *)d_u, (const float *)d_T, (float *)d_Q,
                                 (float *)d_B, (float *)d_FT);
}

wdlb_status wdlb_init_thermal(wdlb_ctx *c, const double *h_n, const double *h_u, const double *h_T, void *d_T)
{
    if (!c) return WDLB_E_INVAL;
    if (!h_n || !h_u || !h_T || !d_T) return fail(c, WDLB_E_INVAL, "null field");
    wdlb_status st = thermal_flow_ok(c);
    if (st != WDLB_OK) return st;
    for (long long i = 0; i < c->g.N; ++i)
        if (!(h_T[i] > 0.0) || !std::isfinite(h_T[i])) return fail(c, WDLB_E_INVAL, "temperature not positive");
    if ((st = do_init(c, 0, nullptr, h_n, h_u)) != WDLB_OK) return st;
    if (c->store == WDLB_FP64) return init_thermal<double>(c, h_T, (double *)d_T);
    return init_thermal<float>(c, h_T, (float *)d_T);
}

wdlb_status wdlb_step_thermal(wdlb_ctx *c, void *d_T, int64_t nsteps, int32_t nsub)
{
    if (!c) return WDLB_E_INVAL;
    if (!d_T) return fail(c, WDLB_E_INVAL, "null temperature");
    if (nsteps < 0 || nsub < 1) return fail(c, WDLB_E_INVAL, "negative step count or sub-step count below 1");
    wdlb_status st = thermal_flow_ok(c);
    if (st != WDLB_OK) return st;
    if (!c->inited) return fail(c, WDLB_E_STATE, "context not initialised");
    // pairs of steps by graph replay (not while kernels are timed), as wdlb_step
    if (c->graphs && c->prof == 0) {
        while (nsteps >= 2) {
            hipGraphExec_t ex = nullptr;
            if ((st = thermal_graph(c, d_T, nsub, &ex)) != WDLB_OK) return st;
            if (!ex) break;  // capture not available: step eagerly
            HIPCHK(c, hipGraphLaunch(ex, c->stream));
            c->step += 2;
            nsteps -= 2;
        }
    }
    for (int64_t t = 0; t < nsteps; ++t) {
        if ((st = thermal_flow_step(c, d_T, nsub)) != WDLB_OK) return st;
        c->cur ^= 1;
        c->step++;
    }
    return WDLB_OK;
}

static wdlb_status planes(wdlb_ctx *c, std::vector<double> &out)
{
    wdlb_status st = read_pass(c);
    if (st != WDLB_OK) return st;
    const Geom g = c->g;
    if (c->store == WDLB_FP64)
        hipLaunchKernelGGL((k_planes<double>), dim3(g.nz), dim3(256), 0, c->stream, g, c->pad,
                           (const double *)c->rho_p, (const double *)c->u_rd, c->planes);
    else
        hipLaunchKernelGGL((k_planes<float>), dim3(g.nz), dim3(256), 0, c->stream, g, c->pad,
                           (const float *)c->rho_p, (const float *)c->u_rd, c->planes);
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
    // 8 populations at a time through the gamma array (8 NP >= 8 N reals)
    for (int a0 = 0; a0 < 19; a0 += 8) {
        const int na = std::min(8, 19 - a0);
        switch (c->store) {
        case WDLB_FP64:
            hipLaunchKernelGGL((k_populations<double, double>), grid, dim3(256), 0, c->stream, g,
                               (const V4<double> *)c->ru[cur], (const double *)c->h[cur], a0, (double *)c->scratch);
            break;
        case WDLB_FP32:
            hipLaunchKernelGGL((k_populations<float, float>), grid, dim3(256), 0, c->stream, g,
                               (const V4<float> *)c->ru[cur], (const float *)c->h[cur], a0, (float *)c->scratch);
            break;
        default:
            hipLaunchKernelGGL((k_populations<float, bf16>), grid, dim3(256), 0, c->stream, g,
                               (const V4<float> *)c->ru[cur], (const bf16 *)c->h[cur], a0, (float *)c->scratch);
        }
        HIPCHK(c, hipGetLastError());
        wdlb_status st = copy_out_r(c, c->scratch, na * (size_t)g.N, h_f + (size_t)a0 * g.N);
        if (st != WDLB_OK) return st;
    }
    // the gamma array was overwritten: its padding (zero beyond walls) is rebuilt
    HIPCHK(c, hipMemsetAsync(c->gam_p, 0, 8 * c->rsize * (size_t)c->pad.NP, c->stream));
    return WDLB_OK;
}

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
    memcpy(hd.magic, "WDLBST02", 8);
    hd.nx = c->g.nx;
    hd.ny = c->g.ny;
    hd.nz = c->g.nz;
    hd.walls = c->g.walls;
    hd.precision = c->store;
    hd.pad = 0;
    hd.step = c->step;
    char *p = (char *)h_buf;
    memcpy(p, &hd, sizeof(hd));
    const size_t N = (size_t)c->g.N;
    HIPCHK(c, hipMemcpyAsync(p + sizeof(hd), c->ru[c->cur], 4 * c->rsize * N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(p + sizeof(hd) + 4 * c->rsize * N, c->h[c->cur], (size_t)c->hplanes * c->hsize * N,
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
    if (memcmp(hd.magic, "WDLBST02", 8) != 0 || hd.nx != c->g.nx || hd.ny != c->g.ny || hd.nz != c->g.nz ||
        hd.walls != c->g.walls || hd.precision != c->store)
        return fail(c, WDLB_E_STATE, "state does not match this context");
    const char *p = (const char *)h_buf;
    const size_t N = (size_t)c->g.N;
    c->cur = 0;
    HIPCHK(c, hipMemcpyAsync(c->ru[0], p + sizeof(hd), 4 * c->rsize * N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h[0], p + sizeof(hd) + 4 * c->rsize * N, (size_t)c->hplanes * c->hsize * N, hipMemcpyHostToDevice,
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

wdlb_status wdlb_profile(wdlb_ctx *c, int32_t mask)
{
    if (!c) return WDLB_E_INVAL;
    wdlb_status st = prof_flush(c);
    if (st != WDLB_OK) return st;
    if (mask)
        for (int k = 0; k < WDLB_NKERNELS; ++k) {
            c->prof_ms[k] = 0;
            c->prof_n[k] = 0;
        }
    c->prof = mask & ((1 << WDLB_NKERNELS) - 1);
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

wdlb_status wdlb_set_tile(wdlb_ctx *c, int32_t variant)
{
    if (!c) return WDLB_E_INVAL;
    if (variant < -1 || variant >= WDLB_NTILES) return fail(c, WDLB_E_INVAL, "tile variant out of range");
    const int old = c->tile_req;
    c->tile_req = variant;
    wdlb_status st = tables(c);
    if (st != WDLB_OK) {
        c->tile_req = old;
        tables(c);
        return fail(c, st, "the requested shell tile does not fit this sigma");
    }
    return WDLB_OK;
}

wdlb_status wdlb_get_tile(wdlb_ctx *c, int32_t *variant, int32_t *specialised)
{
    if (!c || !variant) return WDLB_E_INVAL;
    *variant = c->tile;
    if (specialised) *specialised = c->spec_s2 > 0 ? 1 : 0;
    return WDLB_OK;
}

const char *wdlb_kernel_name(int32_t kernel) { return (kernel >= 0 && kernel < WDLB_NKERNELS) ? KNAMES[kernel] : ""; }

const char *wdlb_last_error(const wdlb_ctx *c) { return c ? c->err.c_str() : "null context"; }

wdlb_status wdlb_set_graphs(wdlb_ctx *c, int32_t enable)
{
    if (!c) return WDLB_E_INVAL;
    c->graphs = enable != 0;
    if (!c->graphs) drop_graphs(c);
    return WDLB_OK;
}

void wdlb_destroy(wdlb_ctx *c)
{
    if (!c) return;
    prof_flush(c);
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    for (auto e : c->ev_free) (void)hipEventDestroy(e);
    if (c->static_dev >= 0) {  // the stream has drained: the static workspace is free
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[c->static_dev] = false;
    }
    delete c;
}

}  // extern "C"

// the serving loop (uses the context internals above)
#include "server.hpp"
