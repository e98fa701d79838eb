// thermal_launch.hip -- the launches of the thermal-field kernels
// (thermal.hpp), a translation unit of its own so that the library's device
// code compiles in two parts side by side.
#include "context.hpp"
#include "thermal.hpp"

namespace wdlb_lib {

// The thermal-field kernels: compiled for the shell (FP32, compiled sigma),
// else table-driven on LDS-ring tiles (32 x 8 x 2 in FP32, 32 x 8 x 1 in
// FP64) where the two rings fit, else the cache kernel.
template <typename R, int TZ, int NR, bool NoU>
wdlb_status launch_thermal_r(wdlb_ctx *c, R *Q, R *B, R *FT)
{
    const Geom g = c->g;
    const double s = c->prm.sigma;
    const int tx = (g.nx + 31) / 32, ty = (g.ny + 7) / 8, tz = (g.nz + TZ - 1) / TZ;
    const size_t lds = thermal_lds_bytes(32, 8, TZ, c->reach, sizeof(R));
    auto kern = k_thermal_r<R, 32, 8, TZ, NR, NoU>;
    HIPCHK(c, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return launch(c, K_THERMAL, [&] {
        hipLaunchKernelGGL(kern, dim3((unsigned)(tx * ty * tz)), dim3(32 * 8 * TZ), lds, c->stream, g, c->pad,
                           c->reach, (const V4<R> *)c->ru1_p, (const R *)c->rho_p, (const R *)c->gam_p,
                           (const Quad<R> *)c->quads, (const int *)c->qstart, R(s * s), tx, ty, tz, Q, B, FT);
    });
}

// compiled for the shell of 2 sigma = S2 (FP32) on 32 x 16 x 1 tiles: at
// sigma = 10 their two rings (75 KB) leave room for two blocks per CU
template <typename R, int S2, bool NoU>
wdlb_status launch_thermal_s(wdlb_ctx *c, R *Q, R *B, R *FT)
{
    // At u = 0 k_thermal_s0 (density, T and contact values in LDS rings): in
    // FP32 on two-plane tiles, its three rings (123 KB at sigma = 10) for one
    // 1024-lane block per CU, half the barriers and ring fills per node of
    // one-plane tiles; in FP64 on one-plane tiles (127 KB at sigma = 10).
    // Otherwise k_thermal_s on one-plane tiles, the contact values through
    // the caches (in FP64 its two rings take 146 KB at sigma = 10).
    constexpr bool F32 = std::is_same<R, float>::value;
    constexpr int RC = Shell<S2>::R;
    constexpr bool S0 = NoU && thermal0_lds_bytes(32, 16, F32 ? 2 : 1, RC, sizeof(R)) <= LDS_MAX;
    constexpr int TX = 32, TY = 16, TZ = S0 && F32 ? 2 : 1, NT = TX * TY * TZ;
    constexpr int NR = ((TX + 2 * RC) * (TY + 2 * RC) + NT - 1) / NT;
    constexpr size_t LDS = S0 ? thermal0_lds_bytes(TX, TY, TZ, RC, sizeof(R)) : thermal_lds_bytes(TX, TY, TZ, RC, sizeof(R));
    static_assert(LDS <= LDS_MAX, "rings fit in LDS");
    if (c->reach != RC) return fail(c, WDLB_E_STATE, "compiled shell does not match the shell of sigma");
    const Geom g = c->g;
    const double s = c->prm.sigma;
    const int tx = (g.nx + TX - 1) / TX, ty = (g.ny + TY - 1) / TY, tz = (g.nz + TZ - 1) / TZ;
    auto kern = [] {
        if constexpr (S0) return k_thermal_s0<R, S2, TX, TY, TZ>;
        else return k_thermal_s<R, S2, TX, TY, TZ, NR, NoU>;
    }();
    HIPCHK(c, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS));
    return launch(c, K_THERMAL, [&] {
        hipLaunchKernelGGL(kern, dim3((unsigned)(tx * ty * tz)), dim3(NT), LDS, c->stream, g, c->pad,
                           (const V4<R> *)c->ru1_p, (const R *)c->rho_p, (const R *)c->gam_p, R(s * s), tx, ty,
                           tz, Q, B, FT);
    });
}

template <typename R, bool NoU>
wdlb_status launch_thermal(wdlb_ctx *c, R *Q, R *B, R *FT)
{
    // the buffer loads of the contact values take a lane offset below 2^31
    // bytes into one padded sub-lattice; a forced shell tile (wdlb_set_tile
    // >= 0) selects the table-driven kernels here too
    if (c->tile_req < 0 && (double)sizeof(R) * (double)c->pad.NP < 2.0e9) {
        if constexpr (std::is_same<R, float>::value) {
            switch (specialised_s2(c->prm.sigma)) {
            case 6: return launch_thermal_s<R, 6, NoU>(c, Q, B, FT);
            case 8: return launch_thermal_s<R, 8, NoU>(c, Q, B, FT);
            case 12: return launch_thermal_s<R, 12, NoU>(c, Q, B, FT);
            case 16: return launch_thermal_s<R, 16, NoU>(c, Q, B, FT);
            case 20: return launch_thermal_s<R, 20, NoU>(c, Q, B, FT);
            default: break;
            }
        } else {
            // FP64: the shell of sigma = 10 only, where the table-driven
            // kernels are slowest
            if (specialised_s2(c->prm.sigma) == 20) return launch_thermal_s<R, 20, NoU>(c, Q, B, FT);
        }
    }
    constexpr int TZ = std::is_same<R, float>::value ? 2 : 1;
    const int Rr = c->reach, LP = (32 + 2 * Rr) * (8 + 2 * Rr), nr = (LP + 32 * 8 * TZ - 1) / (32 * 8 * TZ);
    if (thermal_lds_bytes(32, 8, TZ, Rr, sizeof(R)) <= LDS_MAX) {
        if constexpr (TZ == 2) {
            switch (nr) {
            case 1: return launch_thermal_r<R, TZ, 1, NoU>(c, Q, B, FT);
            case 2: return launch_thermal_r<R, TZ, 2, NoU>(c, Q, B, FT);
            case 3: return launch_thermal_r<R, TZ, 3, NoU>(c, Q, B, FT);
            case 4: return launch_thermal_r<R, TZ, 4, NoU>(c, Q, B, FT);
            case 5: return launch_thermal_r<R, TZ, 5, NoU>(c, Q, B, FT);
            default: break;
            }
        } else {
            switch (nr) {
            case 1: return launch_thermal_r<R, TZ, 1, NoU>(c, Q, B, FT);
            case 2: return launch_thermal_r<R, TZ, 2, NoU>(c, Q, B, FT);
            case 3: return launch_thermal_r<R, TZ, 3, NoU>(c, Q, B, FT);
            case 4: return launch_thermal_r<R, TZ, 4, NoU>(c, Q, B, FT);
            case 5: return launch_thermal_r<R, TZ, 5, NoU>(c, Q, B, FT);
            case 6: return launch_thermal_r<R, TZ, 6, NoU>(c, Q, B, FT);
            case 7: return launch_thermal_r<R, TZ, 7, NoU>(c, Q, B, FT);
            case 8: return launch_thermal_r<R, TZ, 8, NoU>(c, Q, B, FT);
            default: break;
            }
        }
    }
    const Geom g = c->g;
    const double s = c->prm.sigma;
    const int tx = (g.nx + 31) / 32, ty = (g.ny + 7) / 8;
    return launch(c, K_THERMAL, [&] {
        hipLaunchKernelGGL((k_thermal<R, NoU>), dim3((unsigned)(tx * ty * g.nz)), dim3(256), 0, c->stream, g, c->pad,
                           (const V4<R> *)c->ru1_p, (const R *)c->rho_p, (const R *)c->gam_p,
                           (const Quad<R> *)c->quads, c->nq, R(s * s), tx, ty, Q, B, FT);
    });
}

template wdlb_status launch_thermal<float, false>(wdlb_ctx *, float *, float *, float *);
template wdlb_status launch_thermal<float, true>(wdlb_ctx *, float *, float *, float *);
template wdlb_status launch_thermal<double, false>(wdlb_ctx *, double *, double *, double *);
template wdlb_status launch_thermal<double, true>(wdlb_ctx *, double *, double *, double *);

}  // namespace wdlb_lib
