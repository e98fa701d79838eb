// server.hpp -- the serving loop of the WDLB library: batched solves over
// resident requests.  Part of the host translation unit wdlb.hip (included at
// its end; it uses the context internals defined there).
//
// Requests are stacked along z in one lattice of nx x ny x Z planes.  A
// resident request owns H fluid planes followed by R gap planes (R = shell
// reach), so no stencil of one slit reaches another: gap planes hold rho = 0
// and pulls from them bounce back (the per-plane table ZPlane, which also
// carries each slit's body force and relaxation).  A worker thread
//   - admits queued requests, in arrival order, into the first free run of
//     H + R planes (those that do not fit yet wait; later ones may pass),
//   - initialises their planes, steps every resident slit together, one
//     launch chain per step, check_every steps at a time,
//   - takes FP64 plane sums, and retires a slit when its pore flux changed by
//     less than tol (relative) over the last check_every steps, or after
//     max_steps; its planes become gap planes again.
// A slit's arithmetic reads only its own planes and its gaps, in an order
// that does not depend on its position, so its result is the same alone and
// in a mix.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

struct wdlb_server {
    wdlb_lattice_desc desc;
    wdlb_server_params sp;
    wdlb_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    int gap = 0, Z = 0;
    double plane = 0;  // nodes per plane

    // worker-only state
    std::vector<ZPlane> zp;  // host copy of the per-plane table
    std::vector<int> used;   // plane taken by a resident slit (its fluid or gap planes)
    struct Slot {
        uint64_t id;
        int z0, H;
        double n0;
        int64_t steps;
        double Jprev;
        bool have_prev;
    };
    std::vector<Slot> active;
    std::vector<std::pair<int, int>> to_clear;  // planes (first, count) of retired slits

    // shared state (under mu)
    struct Job {
        uint64_t id;
        wdlb_request req;
    };
    std::deque<Job> queue;
    struct Entry {
        wdlb_result res;
        std::vector<double> ux;
    };
    std::map<uint64_t, Entry> entries;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    bool dead = false;
    uint64_t next_id = 1;
    int64_t pending = 0;  // submitted and not finished
    wdlb_server_stats stats{};
    std::string err;
    std::chrono::steady_clock::time_point t0;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

wdlb_params server_lattice_params(const wdlb_server_params *sp)
{
    wdlb_params p{};
    p.sigma = sp->sigma;
    p.eta = 0.1;  // per request (initial density only)
    p.tau = 1.0;  // per plane
    p.nonlocal = 1;
    p.smdb = 1;
    return p;
}

bool server_params_ok(const wdlb_lattice_desc *d, const wdlb_server_params *sp)
{
    if (!d || !sp) return false;
    if (!d->walls_z || (d->precision != WDLB_FP32 && d->precision != WDLB_FP32_LOCAL64)) return false;
    if (!(sp->tol > 0) || sp->check_every < 1 || sp->max_steps < sp->check_every) return false;
    wdlb_params p = server_lattice_params(sp);
    return desc_ok(d) && params_ok(&p);
}

// first run of n free planes, or -1
int find_run(const wdlb_server *S, int n)
{
    int run = 0;
    for (int z = 0; z < S->Z; ++z) {
        run = S->used[z] ? 0 : run + 1;
        if (run == n) return z - n + 1;
    }
    return -1;
}

// finish a request (worker, under the lock)
void finish(wdlb_server *S, uint64_t id, wdlb_status st, int64_t steps, double J, double U, std::vector<double> ux)
{
    auto &e = S->entries[id];
    e.res.state = 2;
    e.res.status = st;
    e.res.steps = steps;
    e.res.j_pore = J;
    e.res.u_pore = U;
    e.res.t_done = S->now();
    e.ux = std::move(ux);
    S->pending--;
    S->stats.finished++;
}

// fail everything after a device error (worker, under the lock)
void fail_all(wdlb_server *S, wdlb_status st, const std::string &msg)
{
    S->err = msg;
    for (auto &s : S->active) finish(S, s.id, st, s.steps, 0, 0, {});
    S->active.clear();
    for (auto &j : S->queue) finish(S, j.id, st, 0, 0, 0, {});
    S->queue.clear();
    S->dead = true;
    S->cv_done.notify_all();
}

// GPU part of one round (worker, without the lock): upload the plane table,
// initialise the fresh slits, step, and take plane sums and the flag
wdlb_status server_round(wdlb_server *S, const std::vector<wdlb_server::Slot> &fresh, std::vector<double> &sums,
                         std::vector<int> &flags)
{
    wdlb_ctx *c = S->ctx;
    const Geom g = c->g;
    // the padded fields of retired slits back to zero: planes above the run
    // extent are not rewritten by the step, and a slit admitted next to them
    // must see rho = 0 (and finite values) there
    const Pad &pd = c->pad;
    for (const auto &r : S->to_clear) {
        const size_t at = (size_t)(r.first + pd.P) * pd.PXY, n = (size_t)r.second * pd.PXY;
        HIPCHK(c, hipMemsetAsync((float *)c->rho_p + at, 0, n * sizeof(float), c->stream));
        HIPCHK(c, hipMemsetAsync((V4<float> *)c->ru1_p + at, 0, n * sizeof(V4<float>), c->stream));
        for (int h = 0; h < 8; ++h)
            HIPCHK(c, hipMemsetAsync((float *)c->gam_p + (size_t)h * pd.NP + at, 0, n * sizeof(float), c->stream));
    }
    S->to_clear.clear();
    HIPCHK(c, hipMemcpyAsync(c->zp_dev, S->zp.data(), S->zp.size() * sizeof(ZPlane), hipMemcpyHostToDevice,
                             c->stream));
    for (const auto &s : fresh) {
        const long long i0 = (long long)s.z0 * (long long)S->plane, cnt = (long long)s.H * (long long)S->plane;
        const dim3 grid = grid1(cnt, 256);
        hipLaunchKernelGGL((k_fill<float>), grid, dim3(256), 0, c->stream, g, (V4<float> *)c->ru[c->cur],
                           (float)s.n0, 0.f, 0.f, 0.f, i0, cnt);
        hipLaunchKernelGGL((k_init<float, float>), grid, dim3(256), 0, c->stream, g,
                           (const V4<float> *)c->ru[c->cur], (float *)c->h[c->cur], i0, cnt);
    }
    HIPCHK(c, hipGetLastError());
    // process the planes up to the highest resident slit's trailing gap: no
    // fluid stencil reaches beyond that gap
    int top = 1;
    for (int z = S->Z - 1; z >= 0; --z)
        if (S->used[z]) {
            top = z + 1;
            break;
        }
    c->nz_run = top;
    wdlb_status st = wdlb_step(c, S->sp.check_every);
    if (st != WDLB_OK) return st;
    st = pass<true>(c);
    if (st != WDLB_OK) return st;
    hipLaunchKernelGGL((k_planes<float>), dim3(top), dim3(256), 0, c->stream, g, c->pad, (const float *)c->rho_p,
                       (const float *)c->u_rd, c->planes);
    HIPCHK(c, hipGetLastError());
    sums.assign(3 * (size_t)g.nz, 0.0);
    HIPCHK(c, hipMemcpyAsync(sums.data(), c->planes, sums.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    flags.assign(1 + (size_t)g.nz, 0);
    HIPCHK(c, hipMemcpyAsync(flags.data(), c->flag, flags.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flags[0]) {
        HIPCHK(c, hipMemsetAsync(c->flag, 0, flags.size() * sizeof(int), c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return WDLB_OK;
}

void serve(wdlb_server *S)
{
    if (hipSetDevice(S->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(S->mu);
        fail_all(S, WDLB_E_HIP, "hipSetDevice failed in the server thread");
        return;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        if (S->stop) break;
        // admit
        std::vector<wdlb_server::Slot> fresh;
        for (auto it = S->queue.begin(); it != S->queue.end();) {
            const int z0 = find_run(S, it->req.H + S->gap);
            if (z0 < 0) {
                ++it;
                continue;
            }
            const wdlb_request &r = it->req;
            for (int z = z0; z < z0 + r.H + S->gap; ++z) S->used[z] = 1;
            for (int z = z0; z < z0 + r.H; ++z) {
                ZPlane &q = S->zp[z];
                q = ZPlane{};
                q.gx = r.gx;
                q.omega = 1.0 / r.tau;
                q.ksrc = 1.0 - 0.5 / r.tau;
                q.fluid = 1;
            }
            const double s3 = S->sp.sigma * S->sp.sigma * S->sp.sigma;
            fresh.push_back({it->id, z0, r.H, 6.0 * r.eta / (M_PI * s3), 0, 0.0, false});
            auto &e = S->entries[it->id];
            e.res.state = 1;
            e.res.t_admit = S->now();
            it = S->queue.erase(it);
        }
        if (S->active.empty() && fresh.empty()) {
            S->cv_work.wait(lk);
            continue;
        }
        lk.unlock();
        const double tb = S->now();
        std::vector<double> sums;
        std::vector<int> flags;
        const wdlb_status st = server_round(S, fresh, sums, flags);
        const double te = S->now();
        lk.lock();
        if (st != WDLB_OK) {
            for (auto &s : fresh) S->active.push_back(s);
            fail_all(S, st, S->ctx->err);
            break;
        }
        for (auto &s : fresh) S->active.push_back(s);
        int fluid = 0;
        for (auto &s : S->active) fluid += s.H;
        S->stats.chunks++;
        S->stats.steps += S->sp.check_every;
        S->stats.node_updates += (double)fluid * S->plane * S->sp.check_every;
        S->stats.busy_s += te - tb;
        S->stats.max_resident = std::max<int32_t>(S->stats.max_resident, (int32_t)S->active.size());
        // evaluate and retire
        const int nz = S->Z;
        std::vector<wdlb_server::Slot> keep;
        for (auto &s : S->active) {
            s.steps += S->sp.check_every;
            double M = 0, U = 0, J = 0;
            std::vector<double> ux(s.H);
            for (int k = 0; k < s.H; ++k) {
                const int z = s.z0 + k;
                M += sums[z];
                ux[k] = sums[nz + z] / S->plane;
                U += ux[k];
                J += sums[2 * nz + z];
            }
            J /= S->plane * s.H;
            U /= s.H;
            bool bad = !std::isfinite(J) || !std::isfinite(U) || !(M > 0);
            for (int k = 0; k < s.H; ++k) bad = bad || flags[1 + s.z0 + k] != 0;
            const bool conv = s.have_prev && std::fabs(J - s.Jprev) <= S->sp.tol * std::fabs(J);
            wdlb_status fst = WDLB_OK;
            bool done = false;
            if (bad) {
                fst = WDLB_E_UNSTABLE;
                done = true;
            } else if (conv) {
                done = true;
            } else if (s.steps >= S->sp.max_steps) {
                fst = WDLB_E_NOT_CONVERGED;
                done = true;
            }
            if (done) {
                finish(S, s.id, fst, s.steps, J, U, std::move(ux));
                for (int z = s.z0; z < s.z0 + s.H + S->gap; ++z) {
                    S->used[z] = 0;
                    S->zp[z] = ZPlane{};
                }
                S->to_clear.push_back({s.z0, s.H + S->gap});
            } else {
                s.Jprev = J;
                s.have_prev = true;
                keep.push_back(s);
            }
        }
        S->active.swap(keep);
        S->stats.resident = (int32_t)S->active.size();
        S->stats.queued = (int32_t)S->queue.size();
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

wdlb_status wdlb_server_workspace_size(const wdlb_lattice_desc *desc, const wdlb_server_params *sp, size_t *bytes)
{
    if (!server_params_ok(desc, sp) || !bytes) return WDLB_E_INVAL;
    *bytes = layout(desc).total;
    return WDLB_OK;
}

wdlb_status wdlb_server_create(const wdlb_lattice_desc *desc, const wdlb_server_params *sp, void *d_pool,
                               size_t bytes, wdlb_server **out)
{
    if (!out) return WDLB_E_INVAL;
    *out = nullptr;
    if (!server_params_ok(desc, sp) || !d_pool) return WDLB_E_INVAL;
    wdlb_server *S = new (std::nothrow) wdlb_server();
    if (!S) return WDLB_E_NOMEM;
    S->desc = *desc;
    S->sp = *sp;
    if (hipGetDevice(&S->device) != hipSuccess || hipStreamCreate(&S->stream) != hipSuccess) {
        delete S;
        return WDLB_E_HIP;
    }
    wdlb_lattice_desc d = *desc;
    d.stream = S->stream;
    wdlb_params p = server_lattice_params(sp);
    wdlb_status st = wdlb_create(&d, &p, d_pool, bytes, &S->ctx);
    if (st != WDLB_OK) {
        (void)hipStreamDestroy(S->stream);
        delete S;
        return st;
    }
    wdlb_ctx *c = S->ctx;
    S->Z = desc->nz;
    S->gap = c->reach;
    S->plane = (double)desc->nx * desc->ny;
    S->zp.assign(S->Z, ZPlane{});
    S->used.assign(S->Z, 0);
    c->g.zp = c->zp_dev;
    c->inited = true;
    c->cur = 0;
    c->step = 0;
    if (hipMemcpyAsync(c->zp_dev, S->zp.data(), S->zp.size() * sizeof(ZPlane), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipMemsetAsync(c->flag, 0, sizeof(int) * (1 + (size_t)S->Z), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        wdlb_destroy(c);
        (void)hipStreamDestroy(S->stream);
        delete S;
        return WDLB_E_HIP;
    }
    S->t0 = std::chrono::steady_clock::now();
    S->worker = std::thread(serve, S);
    *out = S;
    return WDLB_OK;
}

wdlb_status wdlb_server_submit(wdlb_server *S, const wdlb_request *r, uint64_t *id)
{
    if (!S || !r || !id) return WDLB_E_INVAL;
    if (r->H < 1 || r->H + S->gap > S->Z || !(r->eta > 0 && r->eta < 1) || !(r->tau > 0.5) ||
        !std::isfinite(r->gx))
        return WDLB_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->dead || S->stop) return WDLB_E_STATE;
    const uint64_t k = S->next_id++;
    auto &e = S->entries[k];
    e.res = wdlb_result{};
    e.res.state = 0;
    e.res.H = r->H;
    e.res.t_submit = S->now();
    S->queue.push_back({k, *r});
    S->pending++;
    S->stats.queued = (int32_t)S->queue.size();
    *id = k;
    S->cv_work.notify_one();
    return WDLB_OK;
}

wdlb_status wdlb_server_poll(wdlb_server *S, uint64_t id, wdlb_result *res, double *h_ux_z, int32_t n_ux)
{
    if (!S || !res) return WDLB_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->entries.find(id);
    if (it == S->entries.end()) return WDLB_E_INVAL;
    *res = it->second.res;
    if (h_ux_z && res->state == 2) {
        // the profile has the request's own H values: refuse a smaller buffer
        if (n_ux < 0 || (size_t)n_ux < it->second.ux.size()) return WDLB_E_INVAL;
        std::copy(it->second.ux.begin(), it->second.ux.end(), h_ux_z);
    }
    return WDLB_OK;
}

wdlb_status wdlb_server_drain(wdlb_server *S)
{
    if (!S) return WDLB_E_INVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->pending == 0 || S->dead; });
    return S->dead ? WDLB_E_HIP : WDLB_OK;
}

wdlb_status wdlb_server_stats_get(wdlb_server *S, wdlb_server_stats *st)
{
    if (!S || !st) return WDLB_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *st = S->stats;
    return WDLB_OK;
}

const char *wdlb_server_last_error(wdlb_server *S)
{
    if (!S) return "null server";
    std::lock_guard<std::mutex> lk(S->mu);
    return S->err.c_str();
}

void wdlb_server_destroy(wdlb_server *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    if (S->ctx) {
        (void)hipStreamSynchronize(S->stream);
        wdlb_destroy(S->ctx);
    }
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
}

}  // extern "C"
