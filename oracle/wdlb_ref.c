/*
 * wdlb_ref.c -- plain FP64 CPU oracle of the weighted-density lattice
 * Boltzmann (WDLB) time step for the isothermal hard-sphere fluid
 * (Marini Bettolo Marconi & Melchionna, "Weighted density Lattice Boltzmann
 * approach to fluids under confinement", arXiv:1304.7880).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference for
 * the GPU library.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source, header, table or
 * helper with the GPU path, and the GPU path never calls it.
 *
 * What it computes, one time step t -> t+1 on a D3Q19 lattice (Sec. 5, the
 * five-step LB algorithm; steps 2-4 below, step 1 is wdlb_ref_init):
 *   O1  rho = sum_a f_a, j = sum_a c_a f_a              (Sec. 2, moments (colonna))
 *   O2  nbar(r) = ball mean of rho over |e| <= sigma/2  (Sec. 3, Fischer-Methfessel
 *       smoothed density; normalised by the lattice ball size)
 *   O3  shell sums over |e| ~ sigma, with the contact value g_CS evaluated at
 *       the weighted density of the midpoint r + e/2:
 *     a   F^mf  (Sec. 3, mean-field force), then u1 = j/rho + (g + F^mf)/2
 *     b   F^v   (Sec. 3, viscous force; the velocity part of eq. campoc)
 *         A_ij  (Sec. 3, eq. campod), both with du = u1(r+e) - u1(r)
 *   O4  F = rho (g + F^mf + F^v); A0 = traceless symmetric part of A;
 *       u = (j + F/2)/rho
 *   O5  forced BGK collision with the SMDB source (Sec. 2, eq. eq:dufty2 and
 *       eq. SMDB, isothermal so B_i = Q = 0):
 *         f*_a = f_a - (f_a - feq_a)/tau
 *                + (1 - 1/(2 tau)) [ w_a (3(c_a - u) + 9 (c_a.u) c_a).F
 *                                    + (9/2) w_a (c_ai c_aj - delta_ij/3) A0_ij ]
 *   O6  streaming f_a(r + c_a) <- f*_a(r), half-way bounce-back at the walls
 *
 * Readings of the paper where it is silent or ambiguous (all fixed here once;
 * the GPU library follows the same readings):
 *   - textbook D3Q19, weights 1/3, 1/18, 1/36; m = a = dt = 1; kT = c_s^2 = 1/3
 *   - "explicit trapezoidal rule" (Sec. 5, step 3) = the He-Shan-Doolen change
 *     of variables: u = (j + F/2)/rho and a factor (1 - 1/(2 tau)) on all
 *     sources (force and A-term)
 *   - g_2 at contact = Carnahan-Starling (1 - eta/2)/(1 - eta)^3, eta = pi
 *     sigma^3 nbar / 6, nbar taken at the midpoint r + sigma k/2; off-lattice
 *     midpoints take the mean of nbar over the surrounding lattice nodes
 *   - the unit-sphere integral is the lattice shell (sigma-1/2)^2 <= |e|^2 <
 *     (sigma+1/2)^2 with uniform weight 4 pi/|S| and direction e/|e|
 *   - the ball is |e|^2 <= sigma^2/4, divided by its own size
 *   - the velocity with which F^v and A_ij are formed (Sec. 5, step 2: "using
 *     the fields u and n") is u1 = j/rho + (g + F^mf)/2, the velocity of the
 *     current populations with the half-step forcing of every force except
 *     F^v itself.  One velocity field on both ends of every pair keeps the
 *     pair force antisymmetric (momentum is conserved), is exact at rest
 *     (F^v = A = 0 when u1 = 0), and damps the z-checkerboard momentum mode,
 *     which streaming flips every step; a velocity lagged by one step makes
 *     that mode grow by about (1 + kappa) per step.  rho is the current one.
 *   - the A-source is the second-order Hermite term about u = 0, built from
 *     the traceless symmetric part of A_ij, with the 1/2 A_ij of eq. eq:dufty2
 *     taken literally (it injects exactly A0 into the second moment)
 *   - walls: no-slip half-way bounce-back; outside the slit rho = u = 0 for
 *     every stencil; x, y (and z when there are no walls) are periodic and
 *     offsets wrap onto periodic images, self-images included
 *   - B_i, Q and F^T vanish (isothermal, Sec. 5)
 *
 * Layout: populations are structure-of-arrays f[a][z][y][x] (x fastest), node
 * index i = (z*ny + y)*nx + x; vectors are u[c][i]; tensors A[c][i] with
 * c = 3*row + col.  Every array is FP64.  Node loops run under OpenMP; every
 * node's arithmetic is independent of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19
#define REF_OK 0
#define REF_EINVAL 1
#define REF_EUNSTABLE 2
#define REF_ENOMEM 3

typedef struct {
    int32_t nx, ny, nz;   /* fluid nodes per axis */
    int32_t walls_z;      /* 1: walls at z = -1/2 and nz - 1/2; 0: periodic in z */
    double sigma;         /* hard-sphere diameter in lattice units */
    double tau;           /* BGK relaxation time (omega_0 = 1/tau) */
    double g[3];          /* body acceleration (external force per unit mass) */
    int32_t nonlocal;     /* 0: plain forced BGK, no hard-sphere fields */
    int32_t smdb;         /* 1: include the A_ij relaxation term (SMDB); 0: DSB */
} wdlb_ref_cfg;

/* D3Q19 velocity set: rest, 6 axis, 12 face diagonals. */
static const int CV[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static const double KT = 1.0 / 3.0;

static double weight(int a)
{
    int n2 = CV[a][0] * CV[a][0] + CV[a][1] * CV[a][1] + CV[a][2] * CV[a][2];
    return n2 == 0 ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

static int opposite(int a)
{
    for (int b = 0; b < NQ; ++b)
        if (CV[b][0] == -CV[a][0] && CV[b][1] == -CV[a][1] && CV[b][2] == -CV[a][2]) return b;
    return -1;
}

static int cfg_ok(const wdlb_ref_cfg *c)
{
    return c && c->nx > 0 && c->ny > 0 && c->nz > 0 && c->tau > 0.5 &&
           (c->nonlocal == 0 || c->sigma >= 1.0);
}

static long nnodes(const wdlb_ref_cfg *c) { return (long)c->nx * c->ny * c->nz; }

static int wrapi(int a, int n)
{
    int m = a % n;
    return m < 0 ? m + n : m;
}

/* Fluid node index of lattice point (x, y, z), or -1 outside the slit. */
static long site(const wdlb_ref_cfg *c, int x, int y, int z)
{
    x = wrapi(x, c->nx);
    y = wrapi(y, c->ny);
    if (c->walls_z) {
        if (z < 0 || z >= c->nz) return -1;
    } else {
        z = wrapi(z, c->nz);
    }
    return ((long)z * c->ny + y) * c->nx + x;
}

/* ------------------------------------------------------------------ */
/* Stencils                                                             */
/* ------------------------------------------------------------------ */

/* Ball of diameter sigma: integer e with |e|^2 <= sigma^2/4 (Sec. 3,
 * smoothed density nbar).  Writes up to cap triples, returns the count. */
int wdlb_ref_ball(double sigma, int32_t *e, int32_t cap)
{
    int R = (int)ceil(sigma / 2.0) + 1, n = 0;
    for (int z = -R; z <= R; ++z)
        for (int y = -R; y <= R; ++y)
            for (int x = -R; x <= R; ++x)
                if (4.0 * (x * x + y * y + z * z) <= sigma * sigma) {
                    if (e && n < cap) { e[3 * n] = x; e[3 * n + 1] = y; e[3 * n + 2] = z; }
                    ++n;
                }
    return n;
}

/* Contact shell of radius sigma: (sigma-1/2)^2 <= |e|^2 < (sigma+1/2)^2
 * (discrete stand-in for the integral over the unit vector k in Sec. 3). */
int wdlb_ref_shell(double sigma, int32_t *e, int32_t cap)
{
    int R = (int)ceil(sigma + 0.5) + 1, n = 0;
    double lo = (sigma - 0.5) * (sigma - 0.5), hi = (sigma + 0.5) * (sigma + 0.5);
    for (int z = -R; z <= R; ++z)
        for (int y = -R; y <= R; ++y)
            for (int x = -R; x <= R; ++x) {
                double r2 = (double)(x * x + y * y + z * z);
                if (r2 >= lo && r2 < hi) {
                    if (e && n < cap) { e[3 * n] = x; e[3 * n + 1] = y; e[3 * n + 2] = z; }
                    ++n;
                }
            }
    return n;
}

/* Carnahan-Starling contact value of the pair correlation. */
double wdlb_ref_gcs(double eta) { return (1.0 - 0.5 * eta) / ((1.0 - eta) * (1.0 - eta) * (1.0 - eta)); }

/* ------------------------------------------------------------------ */
/* Equilibrium and collision (one node)                                 */
/* ------------------------------------------------------------------ */

/* Second-order Hermite expansion of n phi_M on D3Q19, isothermal. */
void wdlb_ref_equilibrium(double rho, const double u[3], double feq[NQ])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int a = 0; a < NQ; ++a) {
        double cu = CV[a][0] * u[0] + CV[a][1] * u[1] + CV[a][2] * u[2];
        feq[a] = weight(a) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* O5: forced BGK relaxation plus the SMDB A-source, trapezoidal weighting.
 * A0 is the traceless symmetric tensor (row-major 3x3). */
void wdlb_ref_collide_node(const double f[NQ], double rho, const double u[3], const double F[3],
                           const double A0[9], double tau, double fout[NQ])
{
    double feq[NQ];
    wdlb_ref_equilibrium(rho, u, feq);
    double k = 1.0 - 0.5 / tau;
    for (int a = 0; a < NQ; ++a) {
        double w = weight(a);
        double c[3] = {CV[a][0], CV[a][1], CV[a][2]};
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double guo = 0.0;
        for (int i = 0; i < 3; ++i) guo += (3.0 * (c[i] - u[i]) + 9.0 * cu * c[i]) * F[i];
        guo *= w;
        double sa = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) sa += (c[i] * c[j] - (i == j ? 1.0 / 3.0 : 0.0)) * A0[3 * i + j];
        sa *= 4.5 * w;
        fout[a] = f[a] - (f[a] - feq[a]) / tau + k * (guo + sa);
    }
}

/* ------------------------------------------------------------------ */
/* O1-O4                                                                */
/* ------------------------------------------------------------------ */

/* O1: density and momentum of the current populations. */
int wdlb_ref_moments(const wdlb_ref_cfg *c, const double *f, double *rho, double *j)
{
    if (!cfg_ok(c)) return REF_EINVAL;
    long N = nnodes(c);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        double r = 0, jx = 0, jy = 0, jz = 0;
        for (int a = 0; a < NQ; ++a) {
            double fa = f[(long)a * N + i];
            r += fa;
            jx += CV[a][0] * fa;
            jy += CV[a][1] * fa;
            jz += CV[a][2] * fa;
        }
        rho[i] = r;
        j[i] = jx;
        j[N + i] = jy;
        j[2 * N + i] = jz;
    }
    return REF_OK;
}

/* O2: smoothed density, ball mean with rho = 0 outside the slit. */
int wdlb_ref_nbar(const wdlb_ref_cfg *c, const double *rho, double *nbar)
{
    if (!cfg_ok(c) || c->sigma < 1.0) return REF_EINVAL;
    int nb = wdlb_ref_ball(c->sigma, NULL, 0);
    int32_t *b = (int32_t *)malloc(sizeof(int32_t) * 3 * nb);
    if (!b) return REF_ENOMEM;
    wdlb_ref_ball(c->sigma, b, nb);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                double s = 0.0;
                for (int q = 0; q < nb; ++q) {
                    long t = site(c, x + b[3 * q], y + b[3 * q + 1], z + b[3 * q + 2]);
                    if (t >= 0) s += rho[t];
                }
                nbar[site(c, x, y, z)] = s / nb;
            }
    free(b);
    return REF_OK;
}

/* G(r, e) = (4 pi/|S|) g_CS(eta_mid) rho(r+e): the weight with which the
 * shell point r+e enters every shell sum (Sec. 3, contact value at the
 * weighted density of the midpoint r + e/2).  Returns 0 when r+e lies
 * outside the slit (no contribution), 1 on success, -1 when the midpoint
 * packing fraction reaches 1 (g_CS diverges). */
static int shell_weight(const wdlb_ref_cfg *c, const double *rho, const double *nbar, double wS, int x,
                        int y, int z, const int32_t e[3], long *s_out, double *G)
{
    long s = site(c, x + e[0], y + e[1], z + e[2]);
    *s_out = s;
    *G = 0.0;
    if (s < 0) return 0;
    /* midpoint p = r + e/2: average nbar over the lattice nodes around p */
    int lo[3], np[3], rr[3] = {x, y, z};
    for (int d = 0; d < 3; ++d) {
        if (e[d] % 2 == 0) { lo[d] = rr[d] + e[d] / 2; np[d] = 1; }
        else { lo[d] = rr[d] + (e[d] - 1) / 2; np[d] = 2; }
    }
    double nsum = 0.0;
    int cnt = 0;
    for (int kz = 0; kz < np[2]; ++kz)
        for (int ky = 0; ky < np[1]; ++ky)
            for (int kx = 0; kx < np[0]; ++kx) {
                long t = site(c, lo[0] + kx, lo[1] + ky, lo[2] + kz);
                nsum += (t >= 0) ? nbar[t] : 0.0;
                ++cnt;
            }
    double nmid = nsum / cnt;
    double eta = M_PI * c->sigma * c->sigma * c->sigma * nmid / 6.0;
    if (!(eta < 1.0)) return -1;
    *G = wS * wdlb_ref_gcs(eta) * rho[s];
    return 1;
}

static int32_t *shell_table(const wdlb_ref_cfg *c, int *ns)
{
    *ns = wdlb_ref_shell(c->sigma, NULL, 0);
    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * 3 * (*ns));
    if (e) wdlb_ref_shell(c->sigma, e, *ns);
    return e;
}

/* the member of each {e, -e} pair from which the pair is visited */
static int positive(const int32_t *e)
{
    return e[2] > 0 || (e[2] == 0 && (e[1] > 0 || (e[1] == 0 && e[0] > 0)));
}

/* O3a: mean-field force F^mf(r) = -kT sigma^2 sum_e (e/|e|) G(r, e)
 * (Sec. 3, F^mf).  Each offset is added together with its partner -e before
 * it enters the running sum, so a uniform density gives exactly zero. */
int wdlb_ref_meanfield(const wdlb_ref_cfg *c, const double *rho, const double *nbar, double *Fmf)
{
    if (!cfg_ok(c) || c->sigma < 1.0) return REF_EINVAL;
    long N = nnodes(c);
    int ns;
    int32_t *e = shell_table(c, &ns);
    if (!e) return REF_ENOMEM;
    double wS = 4.0 * M_PI / ns, cmf = -KT * c->sigma * c->sigma;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                double acc[3] = {0, 0, 0};
                for (int q = 0; q < ns; ++q) {
                    const int32_t *ep = e + 3 * q;
                    if (!positive(ep)) continue;
                    int32_t em[3] = {-ep[0], -ep[1], -ep[2]};
                    long sp, sm;
                    double Gp, Gm;
                    int a = shell_weight(c, rho, nbar, wS, x, y, z, ep, &sp, &Gp);
                    int b = shell_weight(c, rho, nbar, wS, x, y, z, em, &sm, &Gm);
                    if (a < 0 || b < 0) { bad = 1; continue; }
                    double len = sqrt((double)(ep[0] * ep[0] + ep[1] * ep[1] + ep[2] * ep[2]));
                    for (int i = 0; i < 3; ++i) {
                        double k = ep[i] / len;
                        acc[i] += cmf * k * Gp + cmf * (-k) * Gm;
                    }
                }
                long r = site(c, x, y, z);
                for (int i = 0; i < 3; ++i) Fmf[(long)i * N + r] = acc[i];
            }
    free(e);
    return bad ? REF_EUNSTABLE : REF_OK;
}

/* O3b: viscous force and the SMDB field with du = v(r+e) - v(r) for a given
 * velocity field v:
 *   F^v(r)  =  2 sigma^2 sqrt(kT/pi) sum_e k (k.du) G(r,e)       (Sec. 3, F^v)
 *   A_ij(r) = -(kT/5) sigma^2 rho(r) sum_e G(r,e) (k_j du_i + k_i du_j)
 *                                                            (Sec. 3, eq. campod)
 * with k = e/|e|; A is 9 per node (row-major).  Pairs {e, -e} are summed
 * first, as in O3a. */
int wdlb_ref_viscous(const wdlb_ref_cfg *c, const double *rho, const double *nbar, const double *v,
                     double *Fv, double *A)
{
    if (!cfg_ok(c) || c->sigma < 1.0) return REF_EINVAL;
    long N = nnodes(c);
    int ns;
    int32_t *e = shell_table(c, &ns);
    if (!e) return REF_ENOMEM;
    double wS = 4.0 * M_PI / ns, s2 = c->sigma * c->sigma;
    double cv = 2.0 * s2 * sqrt(KT / M_PI);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long r = site(c, x, y, z);
                double ca = -(KT / 5.0) * s2 * rho[r];
                double acc[12] = {0};
                for (int q = 0; q < ns; ++q) {
                    const int32_t *ep = e + 3 * q;
                    if (!positive(ep)) continue;
                    double term[2][12];
                    for (int side = 0; side < 2; ++side) {
                        int32_t ee[3] = {side ? -ep[0] : ep[0], side ? -ep[1] : ep[1], side ? -ep[2] : ep[2]};
                        long s;
                        double G;
                        int ok = shell_weight(c, rho, nbar, wS, x, y, z, ee, &s, &G);
                        for (int t = 0; t < 12; ++t) term[side][t] = 0.0;
                        if (ok < 0) { bad = 1; continue; }
                        if (ok == 0) continue;
                        double len = sqrt((double)(ee[0] * ee[0] + ee[1] * ee[1] + ee[2] * ee[2]));
                        double k[3] = {ee[0] / len, ee[1] / len, ee[2] / len}, du[3];
                        for (int d = 0; d < 3; ++d) du[d] = v[(long)d * N + s] - v[(long)d * N + r];
                        double kdu = k[0] * du[0] + k[1] * du[1] + k[2] * du[2];
                        for (int i = 0; i < 3; ++i) term[side][i] = cv * k[i] * kdu * G;
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) term[side][3 + 3 * i + j] = ca * G * (k[j] * du[i] + k[i] * du[j]);
                    }
                    for (int t = 0; t < 12; ++t) acc[t] += term[0][t] + term[1][t];
                }
                for (int i = 0; i < 3; ++i) Fv[(long)i * N + r] = acc[i];
                for (int t = 0; t < 9; ++t) A[(long)t * N + r] = acc[3 + t];
            }
    free(e);
    return bad ? REF_EUNSTABLE : REF_OK;
}

/* Thermal fields (Sec. 3; the isothermal step of Sec. 5 uses none of them),
 * for given fields n (rho), v and T with k_B = m = 1, at each node r:
 *   Q(r)   = n(r) sigma^2 sum_e G(r,e) [ -T(r) (k.dv)/2 + sqrt(T(r)/pi) dT ]
 *                                                          (eq. campob1)
 *   B_i(r) = -2 T(r) n(r) sigma^2 sum_e k_i G(r,e) dT        (eq. campos)
 *   F^T_i(r) = -(sigma^2/2) sum_e k_i G(r,e) dT              (eq. thermalforce)
 * with k = e/|e|, dv = v(r+e) - v(r), dT = T(r+e) - T(r) and G the shell
 * weight of O3 (contact value at the midpoint, rho(r+e)), the k_B T factor
 * of eq. campob1 cancelling the 1/T of its temperature term.  Pairs {e, -e}
 * are summed first, as in O3a, so uniform v and T give exactly zero.
 * Outputs Q (N), B (3N), FT (3N); nbar from wdlb_ref_nbar. */
int wdlb_ref_thermal(const wdlb_ref_cfg *c, const double *rho, const double *nbar, const double *v,
                     const double *T, double *Q, double *B, double *FT)
{
    if (!cfg_ok(c) || c->sigma < 1.0) return REF_EINVAL;
    long N = nnodes(c);
    int ns;
    int32_t *e = shell_table(c, &ns);
    if (!e) return REF_ENOMEM;
    double wS = 4.0 * M_PI / ns, s2 = c->sigma * c->sigma;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long r = site(c, x, y, z);
                double Tr = T[r];
                double acc[5] = {0};   /* sum G k dT (3), sum G dT, sum G k.dv */
                for (int q = 0; q < ns; ++q) {
                    const int32_t *ep = e + 3 * q;
                    if (!positive(ep)) continue;
                    double term[2][5];
                    for (int side = 0; side < 2; ++side) {
                        int32_t ee[3] = {side ? -ep[0] : ep[0], side ? -ep[1] : ep[1], side ? -ep[2] : ep[2]};
                        long s;
                        double G;
                        int ok = shell_weight(c, rho, nbar, wS, x, y, z, ee, &s, &G);
                        for (int t = 0; t < 5; ++t) term[side][t] = 0.0;
                        if (ok < 0) { bad = 1; continue; }
                        if (ok == 0) continue;
                        double len = sqrt((double)(ee[0] * ee[0] + ee[1] * ee[1] + ee[2] * ee[2]));
                        double k[3] = {ee[0] / len, ee[1] / len, ee[2] / len};
                        double dT = T[s] - Tr, kdv = 0.0;
                        for (int d = 0; d < 3; ++d) kdv += k[d] * (v[(long)d * N + s] - v[(long)d * N + r]);
                        for (int i = 0; i < 3; ++i) term[side][i] = k[i] * G * dT;
                        term[side][3] = G * dT;
                        term[side][4] = G * kdv;
                    }
                    for (int t = 0; t < 5; ++t) acc[t] += term[0][t] + term[1][t];
                }
                double nr = rho[r];
                Q[r] = nr * s2 * (-0.5 * Tr * acc[4] + sqrt(Tr / M_PI) * acc[3]);
                for (int i = 0; i < 3; ++i) {
                    B[(long)i * N + r] = -2.0 * Tr * nr * s2 * acc[i];
                    FT[(long)i * N + r] = -0.5 * s2 * acc[i];
                }
            }
    free(e);
    return bad ? REF_EUNSTABLE : REF_OK;
}

/* O1-O4: the fields at the current time (Sec. 5, steps 2 and 4).
 *   u1 = j/rho + (g + F^mf)/2   velocity of the current populations with the
 *                               half-step forcing of every force but F^v;
 *                               it is the u with which F^v and A_ij are formed
 *   F  = rho (g + F^mf + F^v),  u = (j + F/2)/rho,  A0 = traceless sym(A)
 * Outputs rho, u, F and A0 (9 per node); any output pointer may be NULL;
 * u1_o (3 per node) may be NULL. */
int wdlb_ref_fields(const wdlb_ref_cfg *c, const double *f, double *rho_o, double *u_o, double *F_o,
                    double *A0_o, double *u1_o)
{
    if (!cfg_ok(c)) return REF_EINVAL;
    long N = nnodes(c);
    double *rho = (double *)malloc(sizeof(double) * N);
    double *j = (double *)malloc(sizeof(double) * 3 * N);
    double *nb = (double *)malloc(sizeof(double) * N);
    double *u1 = (double *)malloc(sizeof(double) * 3 * N);
    double *fmf = (double *)calloc(3 * N, sizeof(double));
    double *fv = (double *)calloc(3 * N, sizeof(double));
    double *A = (double *)calloc(9 * N, sizeof(double));
    int rc = REF_OK, bad = 0;
    if (!rho || !j || !nb || !u1 || !fmf || !fv || !A) { rc = REF_ENOMEM; goto out; }
    wdlb_ref_moments(c, f, rho, j);
    for (long i = 0; i < N; ++i)
        if (!(rho[i] > 0.0) || !isfinite(rho[i])) bad = 1;
    if (bad) { rc = REF_EUNSTABLE; goto out; }
    if (c->nonlocal) {
        rc = wdlb_ref_nbar(c, rho, nb);
        if (rc == REF_OK) rc = wdlb_ref_meanfield(c, rho, nb, fmf);
        if (rc != REF_OK) goto out;
    }
    for (long i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d)
            u1[(long)d * N + i] = j[(long)d * N + i] / rho[i] + 0.5 * (c->g[d] + fmf[(long)d * N + i]);
    if (c->nonlocal) {
        rc = wdlb_ref_viscous(c, rho, nb, u1, fv, A);
        if (rc != REF_OK) goto out;
    }
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long i = 0; i < N; ++i) {
        double r = rho[i], F[3], u[3], A0[9];
        for (int d = 0; d < 3; ++d) {
            F[d] = r * (c->g[d] + fmf[(long)d * N + i] + fv[(long)d * N + i]);
            u[d] = (j[(long)d * N + i] + 0.5 * F[d]) / r;
            if (!isfinite(u[d]) || !isfinite(F[d])) bad = 1;
        }
        double tr = A[0 * N + i] + A[4 * N + i] + A[8 * N + i];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                A0[3 * a + b] = (c->smdb && c->nonlocal)
                                    ? 0.5 * (A[(long)(3 * a + b) * N + i] + A[(long)(3 * b + a) * N + i]) -
                                          (a == b ? tr / 3.0 : 0.0)
                                    : 0.0;
        if (rho_o) rho_o[i] = r;
        for (int d = 0; d < 3; ++d) {
            if (u_o) u_o[(long)d * N + i] = u[d];
            if (F_o) F_o[(long)d * N + i] = F[d];
            if (u1_o) u1_o[(long)d * N + i] = u1[(long)d * N + i];
        }
        if (A0_o)
            for (int k = 0; k < 9; ++k) A0_o[(long)k * N + i] = A0[k];
    }
    if (bad) rc = REF_EUNSTABLE;
out:
    free(rho); free(j); free(nb); free(u1); free(fmf); free(fv); free(A);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Step 1 (init), O5-O7 (step) and O8 (reductions)                      */
/* ------------------------------------------------------------------ */

/* Sec. 5, step 1: f = feq(n, u) at every node. */
int wdlb_ref_init(const wdlb_ref_cfg *c, const double *n, const double *u, double *f)
{
    if (!cfg_ok(c)) return REF_EINVAL;
    long N = nnodes(c);
    for (long i = 0; i < N; ++i) {
        double ui[3] = {u[i], u[N + i], u[2 * N + i]}, feq[NQ];
        wdlb_ref_equilibrium(n[i], ui, feq);
        for (int a = 0; a < NQ; ++a) f[(long)a * N + i] = feq[a];
    }
    return REF_OK;
}

/* nsteps full steps in place on f (Sec. 5, steps 2-5). */
int wdlb_ref_step(const wdlb_ref_cfg *c, double *f, int64_t nsteps)
{
    if (!cfg_ok(c) || nsteps < 0) return REF_EINVAL;
    long N = nnodes(c);
    double *rho = (double *)malloc(sizeof(double) * N);
    double *u = (double *)malloc(sizeof(double) * 3 * N);
    double *F = (double *)malloc(sizeof(double) * 3 * N);
    double *A0 = (double *)malloc(sizeof(double) * 9 * N);
    double *fs = (double *)malloc(sizeof(double) * NQ * N);
    int rc = REF_OK;
    if (!rho || !u || !F || !A0 || !fs) { rc = REF_ENOMEM; goto out; }
    for (int64_t t = 0; t < nsteps; ++t) {
        rc = wdlb_ref_fields(c, f, rho, u, F, A0, NULL);
        if (rc != REF_OK) break;
        /* O5: collide every node into fs */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            double fi[NQ], fo[NQ], ui[3], Fi[3], Ai[9];
            for (int a = 0; a < NQ; ++a) fi[a] = f[(long)a * N + i];
            for (int d = 0; d < 3; ++d) { ui[d] = u[(long)d * N + i]; Fi[d] = F[(long)d * N + i]; }
            for (int k = 0; k < 9; ++k) Ai[k] = A0[(long)k * N + i];
            wdlb_ref_collide_node(fi, rho[i], ui, Fi, Ai, c->tau, fo);
            for (int a = 0; a < NQ; ++a) fs[(long)a * N + i] = fo[a];
        }
        /* O6: stream (pull form) with half-way bounce-back */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < c->nz; ++z)
            for (int y = 0; y < c->ny; ++y)
                for (int x = 0; x < c->nx; ++x) {
                    long r = site(c, x, y, z);
                    for (int a = 0; a < NQ; ++a) {
                        long src = site(c, x - CV[a][0], y - CV[a][1], z - CV[a][2]);
                        f[(long)a * N + r] = src >= 0 ? fs[(long)a * N + src] : fs[(long)opposite(a) * N + r];
                    }
                }
    }
out:
    free(rho); free(u); free(F); free(A0); free(fs);
    return rc;
}

/* O8: plane means n(z), u_x(z); out3 = {J_pore, u_pore, mass} with
 * J_pore = sum(rho u_x)/N, u_pore = mean over z of u_x(z), mass = sum(rho). */
int wdlb_ref_reduce(const wdlb_ref_cfg *c, const double *rho, const double *u, double *n_z,
                    double *ux_z, double *out3)
{
    if (!cfg_ok(c)) return REF_EINVAL;
    long N = nnodes(c), plane = (long)c->nx * c->ny;
    double J = 0.0, M = 0.0, up = 0.0;
    for (int z = 0; z < c->nz; ++z) {
        double sn = 0.0, su = 0.0;
        for (long k = 0; k < plane; ++k) {
            long i = (long)z * plane + k;
            sn += rho[i];
            su += u[i];
            J += rho[i] * u[i];
        }
        M += sn;
        if (n_z) n_z[z] = sn / plane;
        if (ux_z) ux_z[z] = su / plane;
        up += su / plane;
    }
    out3[0] = J / N;
    out3[1] = up / c->nz;
    out3[2] = M;
    return REF_OK;
}

int wdlb_ref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void wdlb_ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* The coupled thermal flow (a hybrid reading of this project: the     */
/* paper's LB scheme is isothermal, Sec. 5)                             */
/* ------------------------------------------------------------------ */

/* The temperature term of the second-order Hermite equilibrium at
 * theta = T / kT: w_a rho (3/2) (theta - 1) (|c_a|^2 - 1). */
static double theta_term(int a, double rho, double theta)
{
    double c2 = (double)(CV[a][0] * CV[a][0] + CV[a][1] * CV[a][1] + CV[a][2] * CV[a][2]);
    return weight(a) * rho * 1.5 * (theta - 1.0) * (c2 - 1.0);
}

/* f = feq(n, u) plus the temperature term at T (N values). */
int wdlb_ref_init_thermal(const wdlb_ref_cfg *c, const double *n, const double *u, const double *T, double *f)
{
    int rc = wdlb_ref_init(c, n, u, f);
    if (rc != REF_OK) return rc;
    long N = nnodes(c);
    for (long i = 0; i < N; ++i)
        for (int a = 0; a < NQ; ++a) f[(long)a * N + i] += theta_term(a, n[i], T[i] / KT);
    return REF_OK;
}

/* The energy balance with flow (Sec. 2 eq. energyequation, k_B = m = 1):
 *   dT/dt = -u.grad T + (2 / (3 n)) ( -div q - P:grad u + Q ),
 *   q = -(5/2)(n T / omega0) grad T + B / (2 omega0)            (eq. qexplicit)
 *   P_ij = n T d_ij - (n T / omega0)(d_i u_j + d_j u_i - (2/3) d_ij div u)
 *          + (2 / omega0) A0_ij                                 (eqs. pexplicit, extrapressure)
 * Gradients by central differences (beyond a wall: u mirrored to -u, the
 * no-slip wall half-way; T mirrored, adiabatic); div q by face fluxes as in
 * the conduction at rest (no flux through a wall).  One LB step dt = 1 in
 * nsub sub-steps: the advection, work, B and Q terms at the step's start,
 * the kinetic conduction re-evaluated every sub-step. */
static void energy_update(const wdlb_ref_cfg *c, const double *rho, const double *u, const double *A0,
                          const double *Q, const double *B, double *T, int nsub, double *Rfix, double *Tw)
{
    long N = nnodes(c);
    double omega0 = 1.0 / c->tau;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                long r = site(c, x, y, z);
                double n = rho[r], Tr = T[r], gu[3][3], gT[3], divdq = 0.0;
                for (int i = 0; i < 3; ++i) {
                    int dx = i == 0, dy = i == 1, dz = i == 2;
                    long sp = site(c, x + dx, y + dy, z + dz), sm = site(c, x - dx, y - dy, z - dz);
                    for (int j = 0; j < 3; ++j) {
                        double up = sp >= 0 ? u[(long)j * N + sp] : -u[(long)j * N + r];
                        double um = sm >= 0 ? u[(long)j * N + sm] : -u[(long)j * N + r];
                        gu[i][j] = 0.5 * (up - um);
                    }
                    double Tp = sp >= 0 ? T[sp] : Tr, Tm = sm >= 0 ? T[sm] : Tr;
                    gT[i] = 0.5 * (Tp - Tm);
                    double q0 = B[(long)i * N + r] / (2.0 * omega0);
                    double fp = sp >= 0 ? 0.5 * (q0 + B[(long)i * N + sp] / (2.0 * omega0)) : 0.0;
                    double fm = sm >= 0 ? 0.5 * (B[(long)i * N + sm] / (2.0 * omega0) + q0) : 0.0;
                    divdq += fp - fm;
                }
                double divu = gu[0][0] + gu[1][1] + gu[2][2], work = 0.0, adv = 0.0;
                for (int i = 0; i < 3; ++i) {
                    adv += u[(long)i * N + r] * gT[i];
                    for (int j = 0; j < 3; ++j) {
                        double P = (i == j ? n * Tr : 0.0) -
                                   n * Tr / omega0 * (gu[i][j] + gu[j][i] - (i == j ? 2.0 / 3.0 * divu : 0.0)) +
                                   2.0 / omega0 * A0[(long)(3 * i + j) * N + r];
                        work += P * gu[i][j];
                    }
                }
                Rfix[r] = -adv + 2.0 / (3.0 * n) * (-divdq - work + Q[r]);
            }
    for (int s = 0; s < nsub; ++s) {
#pragma omp parallel for schedule(static)
        for (int z = 0; z < c->nz; ++z)
            for (int y = 0; y < c->ny; ++y)
                for (int x = 0; x < c->nx; ++x) {
                    long r = site(c, x, y, z);
                    double n = rho[r], Tr = T[r], div = 0.0;
                    for (int i = 0; i < 3; ++i) {
                        int dx = i == 0, dy = i == 1, dz = i == 2;
                        long sp = site(c, x + dx, y + dy, z + dz), sm = site(c, x - dx, y - dy, z - dz);
                        double fp = 0.0, fm = 0.0;
                        if (sp >= 0) fp = -2.5 / omega0 * 0.5 * (n * Tr + rho[sp] * T[sp]) * (T[sp] - Tr);
                        if (sm >= 0) fm = -2.5 / omega0 * 0.5 * (rho[sm] * T[sm] + n * Tr) * (Tr - T[sm]);
                        div += fp - fm;
                    }
                    Tw[r] = Tr + (Rfix[r] + 2.0 / (3.0 * n) * (-div)) / nsub;
                }
        memcpy(T, Tw, sizeof(double) * N);
    }
}

/* nsteps steps of the coupled thermal flow in place on f and T:
 *   fields as in O1-O4 with theta = T / kT: F^mf scaled by theta, F^v by
 *   sqrt(theta), A by theta (Sec. 3: the mean-field force carries k_B T,
 *   the viscous force sqrt(k_B T), A_ij k_B T), plus the thermal force F^T
 *   (eq. thermalforce, from n and T alone); u1 = j/rho + (g + theta F^mf +
 *   F^T)/2 carries every force known before the viscous sums, and F^v, A
 *   and Q are formed with it;
 *   O5 with the temperature term of the equilibrium (theta_term, relaxed
 *   at 1/tau; the forcing and A-source as in the isothermal step);
 *   O6 stream; then the energy balance (energy_update) with the step's u,
 *   A0, Q and B.  At T = kT everywhere the populations take the isothermal
 *   step exactly. */
int wdlb_ref_step_thermal(const wdlb_ref_cfg *c, double *f, double *T, int64_t nsteps, int32_t nsub)
{
    if (!cfg_ok(c) || nsteps < 0 || nsub < 1) return REF_EINVAL;
    long N = nnodes(c);
    double *rho = malloc(sizeof(double) * N), *j = malloc(sizeof(double) * 3 * N);
    double *nb = malloc(sizeof(double) * N), *u1 = malloc(sizeof(double) * 3 * N);
    double *fmf = calloc(3 * N, sizeof(double)), *fv = calloc(3 * N, sizeof(double));
    double *A = calloc(9 * N, sizeof(double)), *Q = calloc(N, sizeof(double));
    double *B = calloc(3 * N, sizeof(double)), *FT = calloc(3 * N, sizeof(double));
    double *u = malloc(sizeof(double) * 3 * N), *F = malloc(sizeof(double) * 3 * N);
    double *A0 = malloc(sizeof(double) * 9 * N), *fs = malloc(sizeof(double) * NQ * N);
    double *Rfix = malloc(sizeof(double) * N), *Tw = malloc(sizeof(double) * N);
    int rc = REF_OK, bad = 0;
    if (!rho || !j || !nb || !u1 || !fmf || !fv || !A || !Q || !B || !FT || !u || !F || !A0 || !fs || !Rfix || !Tw) {
        rc = REF_ENOMEM;
        goto out;
    }
    for (int64_t t = 0; t < nsteps && rc == REF_OK; ++t) {
        wdlb_ref_moments(c, f, rho, j);
        for (long i = 0; i < N; ++i)
            if (!(rho[i] > 0.0) || !isfinite(rho[i]) || !(T[i] > 0.0) || !isfinite(T[i])) bad = 1;
        if (bad) { rc = REF_EUNSTABLE; break; }
        if (c->nonlocal) {
            rc = wdlb_ref_nbar(c, rho, nb);
            if (rc == REF_OK) rc = wdlb_ref_meanfield(c, rho, nb, fmf);
            if (rc != REF_OK) break;
        }
        /* F^T depends on n and T alone (eq. thermalforce): formed first (the
         * velocity argument only enters Q), so that u1 carries every force
         * known before the viscous sums, F^T with the others */
        if (c->nonlocal) {
            for (long i = 0; i < 3 * N; ++i) u1[i] = 0.0;
            rc = wdlb_ref_thermal(c, rho, nb, u1, T, Q, B, FT);
            if (rc != REF_OK) break;
        }
        for (long i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d)
                u1[(long)d * N + i] = j[(long)d * N + i] / rho[i] +
                                      0.5 * (c->g[d] + T[i] / KT * fmf[(long)d * N + i] + FT[(long)d * N + i]);
        if (c->nonlocal) {
            rc = wdlb_ref_viscous(c, rho, nb, u1, fv, A);
            if (rc == REF_OK) rc = wdlb_ref_thermal(c, rho, nb, u1, T, Q, B, FT);
            if (rc != REF_OK) break;
        }
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (long i = 0; i < N; ++i) {
            double r = rho[i], th = T[i] / KT, sq = sqrt(th);
            double fi[NQ], fo[NQ], ui[3], Fi[3], Ai[9];
            for (int d = 0; d < 3; ++d) {
                Fi[d] = r * (c->g[d] + th * fmf[(long)d * N + i] + sq * fv[(long)d * N + i] + FT[(long)d * N + i]);
                ui[d] = (j[(long)d * N + i] + 0.5 * Fi[d]) / r;
                if (!isfinite(ui[d]) || !isfinite(Fi[d])) bad = 1;
                u[(long)d * N + i] = ui[d];
            }
            double tr = A[0 * N + i] + A[4 * N + i] + A[8 * N + i];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    Ai[3 * a + b] = (c->smdb && c->nonlocal)
                                        ? th * (0.5 * (A[(long)(3 * a + b) * N + i] + A[(long)(3 * b + a) * N + i]) -
                                                (a == b ? tr / 3.0 : 0.0))
                                        : 0.0;
                    A0[(long)(3 * a + b) * N + i] = Ai[3 * a + b];
                }
            for (int a = 0; a < NQ; ++a) fi[a] = f[(long)a * N + i];
            wdlb_ref_collide_node(fi, r, ui, Fi, Ai, c->tau, fo);
            for (int a = 0; a < NQ; ++a) fs[(long)a * N + i] = fo[a] + theta_term(a, r, th) / c->tau;
        }
        if (bad) { rc = REF_EUNSTABLE; break; }
#pragma omp parallel for schedule(static)
        for (int z = 0; z < c->nz; ++z)
            for (int y = 0; y < c->ny; ++y)
                for (int x = 0; x < c->nx; ++x) {
                    long r = site(c, x, y, z);
                    for (int a = 0; a < NQ; ++a) {
                        long src = site(c, x - CV[a][0], y - CV[a][1], z - CV[a][2]);
                        f[(long)a * N + r] = src >= 0 ? fs[(long)a * N + src] : fs[(long)opposite(a) * N + r];
                    }
                }
        energy_update(c, rho, u, A0, Q, B, T, nsub, Rfix, Tw);
    }
out:
    free(rho); free(j); free(nb); free(u1); free(fmf); free(fv); free(A); free(Q); free(B); free(FT);
    free(u); free(F); free(A0); free(fs); free(Rfix); free(Tw);
    return rc;
}
