// context.hpp -- the context of the WDLB library (struct wdlb_ctx) and the
// host helpers that its translation units share: error reporting, launch
// timing, grid sizes.  Included by wdlb.hip and thermal_launch.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/wdlb.h"
#include "kernels.hpp"

using namespace wdlb;

namespace {
constexpr double KT = 1.0 / 3.0;
constexpr int MAX_QUADS = 4096;
constexpr int MAX_BALL = 8192;
constexpr int MAX_REACH = 17;
constexpr double MAX_SIGMA = 16.0;
}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct wdlb_ctx {
    wdlb_lattice_desc desc;
    wdlb_params prm;
    hipStream_t stream;
    Geom g;
    Pad pad;
    int prec;          // wdlb_precision requested (storage and local arithmetic)
    int store;         // its storage: WDLB_FP64, WDLB_FP32 or WDLB_BF16_NEQ
    size_t rsize;      // bytes of one real (compute type)
    size_t hsize;      // bytes of one stored h
    int hplanes;       // planes of h per node (19; 23 in the BF16 mode)
    char *ws;
    size_t ws_bytes;
    // carved device arrays
    void *ru[2], *h[2];                  // state: (rho, u*) and deviations, two parities
    void *rho_p, *gam_p, *ru1_p;  // padded per-step arrays
    void *jx, *jy, *jz, *fmf, *F, *A, *u_rd, *rho_rd;
    void *scratch;                        // >= 8 N reals, free between steps
    size_t padded_bytes;                  // bytes from rho_p to the end of ru1_p
    double *planes;
    int *flag;
    void *quads;
    int *qstart;
    int *ball;
    ZPlane *zp_dev;                       // per-plane table (used by stacked lattices)
    int nq, nball, rb, reach;  // quad count; ball size and reach; shell reach
    int dtile;                 // k_density tile (index into DENSITY_TILES)
    double wS;         // 4 pi / |S|
    int tile;          // contact-shell tile variant of the viscous/SMDB kernel (index into SHELL_TILES)
    int tile_mf;       // and of the mean-field kernel
    int tile_req;      // requested variant, -1 = automatic
    int spec_s2;       // 2 sigma of the specialised shell kernels in use, 0 = generic
    int spec_b2;       // 2 sigma of the specialised density kernel in use, 0 = generic
    int cur;
    // HIP graphs of two steps (one per starting parity), replayed by
    // wdlb_step; captured on a private stream, launched on the caller's
    bool graphs = true;
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int graph_nz_run = -1;
    // the same for pairs of coupled thermal-flow steps, for one T array and nsub
    hipGraphExec_t tgexec[2] = {nullptr, nullptr};
    void *tg_T = nullptr;
    int tg_nsub = 0;
    int nz_run;        // planes the step kernels process (nz; fewer in a partly filled stacked lattice)
    int64_t step;
    bool inited;
    int static_dev = -1;  // device whose static workspace this context holds (wdlb_create_static), else -1
    int shell_part = 3;   // bit 0: launch the mean-field kernel, bit 1: the viscous/SMDB kernel (the thermal step runs them apart)
    void *shell_trace = nullptr;  // the viscous/SMDB kernel's trace sums go here when set (the thermal step)
    std::string err;
    // event timing of the step kernels
    int prof = 0;  // bit k: time kernel k
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

#define HIPCHK(ctx, call)                                                                                  \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess) return fail(ctx, WDLB_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t LDS_MAX = 160 * 1024;

// 2 sigma of the shells and balls compiled into the library, else 0
int specialised_s2(double sigma)
{
    static const int S2[] = {6, 8, 12, 16, 20};
    for (int s2 : S2)
        if (sigma == 0.5 * s2) return s2;
    return 0;
}

inline dim3 grid1(long long N, int bs) { return dim3((unsigned)((N + bs - 1) / bs)); }

enum { K_MOMENTS = 0, K_DENSITY, K_MEANFIELD, K_SHELL, K_COLLIDE, K_THERMAL };

// Timing events are created without the system-scope fence: a default event
// writes back and invalidates the caches when it is recorded, which slows
// the timed kernel's successor and inflates the measured times.  prof_flush
// synchronises the stream before it reads them, so no fence is needed.
hipEvent_t take_event(wdlb_ctx *c)
{
    if (c->ev_free.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
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
    if (!(c->prof >> k & 1)) {
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

}  // namespace

// the thermal-field kernels (thermal_launch.hip): compiled for the shell
// (FP32, compiled sigma), else table-driven on LDS-ring tiles, else through
// the caches; NoU: their variant at u = 0
namespace wdlb_lib {
template <typename R, bool NoU = false>
wdlb_status launch_thermal(wdlb_ctx *c, R *Q, R *B, R *FT);
}  // namespace wdlb_lib

