/*
 * wdlb.h -- C ABI of the MI355X (gfx950) weighted-density lattice Boltzmann
 * (WDLB) library, libwdlb.so.
 *
 * The method is the isothermal SMDB/WDA lattice Boltzmann scheme for a
 * hard-sphere fluid of Marini Bettolo Marconi & Melchionna (arXiv:1304.7880):
 * a D3Q19 lattice whose collision carries the mean-field and viscous forces
 * of the hard-sphere contact shell and the SMDB relaxation field A_ij
 * (Sec. 3), evaluated with the Carnahan-Starling contact value at the
 * Fischer-Methfessel weighted density (Sec. 3), and advanced by the
 * five-step algorithm of Sec. 5 (initialise; fields; collide and stream;
 * new moments; repeat).  Geometry: a slit pore between two smooth parallel
 * walls normal to z (half-way bounce-back), periodic in x and y; or a fully
 * periodic box.
 *
 * Conventions for every call:
 *   - Every function returns a wdlb_status; no C++ exception crosses the ABI.
 *   - Host pointers (h_*) are borrowed for the duration of the call only.
 *   - Device memory is owned by the caller: the library carves its arrays out
 *     of one caller-allocated device workspace that must outlive the context.
 *     The library never frees caller memory and allocates no device memory.
 *   - All GPU work is enqueued on the caller's HIP stream (desc.stream;
 *     NULL = the default stream).  Calls that return host data synchronise
 *     that stream.
 *   - One host thread per context; contexts are independent.
 *   - Node order is x fastest: i = (z*ny + y)*nx + x, z = 0 the first fluid
 *     plane next to the lower wall.  Vector fields are component-major
 *     (u[c*N + i]).  Populations use the D3Q19 order
 *       0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1)
 *       6:(0,0,-1) 7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0) 11:(1,0,1)
 *       12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1) 15:(0,1,1) 16:(0,-1,-1)
 *       17:(0,1,-1) 18:(0,-1,1).
 *   - Lattice units: spacing, time step and particle mass are 1; kT = 1/3.
 */
#ifndef WDLB_H
#define WDLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WDLB_OK = 0,
    WDLB_E_INVAL = 1,          /* bad argument: shape, sigma outside [1, 16], tau <= 1/2, eta outside (0,1), size */
    WDLB_E_NOMEM = 2,          /* workspace smaller than wdlb_workspace_size reports */
    WDLB_E_HIP = 3,            /* a HIP call failed; wdlb_last_error has its message */
    WDLB_E_UNSTABLE = 4,       /* non-finite or non-positive density (or temperature), or a midpoint packing fraction >= 1 */
    WDLB_E_STATE = 5,          /* call out of order (e.g. step before init) or state buffer mismatch */
    WDLB_E_NOT_CONVERGED = 6   /* a serving request hit its step cap */
} wdlb_status;

/* Precision modes.  Storage is that of the populations and the per-step
 * fields; the stencil sums (weighted density, contact values, shell sums)
 * run in the storage's arithmetic (FP32 for the BF16 mode); the local
 * kernels (pull, moments, collision) in the arithmetic named; reductions
 * (plane means, pore averages, the serving convergence test) in FP64. */
typedef enum {
    WDLB_FP64 = 0,             /* FP64 storage and arithmetic */
    WDLB_FP32 = 1,             /* FP32 storage and arithmetic */
    WDLB_BF16_NEQ = 2,         /* BF16 storage of f - f_eq (FP32 closure populations), FP32 arithmetic */
    WDLB_FP32_LOCAL64 = 3,     /* FP32 storage, FP64 arithmetic in the local kernels */
    WDLB_BF16_NEQ_LOCAL64 = 4  /* BF16 f - f_eq storage, FP64 arithmetic in the local kernels */
} wdlb_precision;

typedef struct wdlb_ctx wdlb_ctx;  /* opaque */

/* Lattice: fluid nodes nx * ny * nz.  walls_z = 1: walls at z = -1/2 and
 * nz - 1/2 (the slit width H = nz); walls_z = 0: periodic in z. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t walls_z;
    int32_t precision;         /* wdlb_precision */
    void *stream;              /* hipStream_t, or NULL */
} wdlb_lattice_desc;

/* Physical parameters (Sec. 5: sigma a multiple of the lattice spacing;
 * eta = pi sigma^3 n / 6 the packing fraction of the uniform initial state;
 * omega_0 = 1/tau; g the external force per unit mass of eq. (1)).
 * nonlocal = 0 drops the hard-sphere fields (plain forced BGK); smdb = 0
 * drops the A_ij relaxation term (the DSB form of Sec. 2). */
typedef struct {
    double sigma;
    double eta;
    double tau;
    double g[3];
    int32_t nonlocal;
    int32_t smdb;
} wdlb_params;

/* Bytes of device workspace a context with this lattice needs (the same for
 * every sigma the library accepts, 1 <= sigma <= 16).  *bytes receives the
 * size. */
wdlb_status wdlb_workspace_size(const wdlb_lattice_desc *desc, const wdlb_params *params, size_t *bytes);

/* Create a context on the current HIP device.  d_workspace: device memory of
 * at least wdlb_workspace_size bytes, 256-byte aligned, owned by the caller.
 * On success *out receives the context; nothing is initialised until one of
 * the wdlb_init_* calls. */
wdlb_status wdlb_create(const wdlb_lattice_desc *desc, const wdlb_params *params, void *d_workspace,
                        size_t bytes, wdlb_ctx **out);

/* Create a context without allocating device memory, for callers that
 * cannot allocate (code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc).  The same context as wdlb_create, whose
 * workspace is instead a device array of WDLB_STATIC_WORKSPACE_BYTES that
 * the library holds on every device it runs on until the process ends.  No
 * device memory is allocated by this call or by stepping the context: it
 * steps launch by launch (graph replay, whose capture allocates, starts off;
 * wdlb_set_graphs can turn it on).  Limits and errors: WDLB_E_NOMEM when the
 * lattice's wdlb_workspace_size exceeds the array (a 64^3 FP32 lattice needs
 * about 120 MB); WDLB_E_STATE while another such context is alive on the
 * current device (both would use the one array: calls that overlap on a
 * device would race); WDLB_E_HIP if the array cannot be located.  The array
 * keeps the contents of the last context that used it; creation clears what
 * must start at zero and init writes the state.  wdlb_destroy (after the
 * stream has drained) frees the array for the next context. */
#define WDLB_STATIC_WORKSPACE_BYTES ((size_t)256 << 20)
wdlb_status wdlb_create_static(const wdlb_lattice_desc *desc, const wdlb_params *params, wdlb_ctx **out);

/* Replace sigma, tau, g, nonlocal, smdb (eta only matters for init). */
wdlb_status wdlb_set_params(wdlb_ctx *ctx, const wdlb_params *params);

/* Sec. 5, step 1: f = f_eq(n0, u0) at every node, n0 = 6 eta/(pi sigma^3). */
wdlb_status wdlb_init_uniform(wdlb_ctx *ctx, const double u0[3]);

/* Sec. 5, step 1 from given fields: h_n[N] density, h_u[3N] velocity (FP64,
 * host).  f = f_eq(n, u) at every node. */
wdlb_status wdlb_init_fields(wdlb_ctx *ctx, const double *h_n, const double *h_u);

/* Sec. 5, steps 2-5 repeated nsteps times: fields, collide + stream with
 * bounce-back, new moments.  Asynchronous on the stream; instability is
 * flagged on the device and reported by the next synchronising call. */
wdlb_status wdlb_step(wdlb_ctx *ctx, int64_t nsteps);

/* Block until the stream has drained; WDLB_E_UNSTABLE if any step so far
 * met a non-finite or non-positive density (or temperature, in
 * wdlb_step_thermal) or a packing fraction >= 1. */
wdlb_status wdlb_sync(wdlb_ctx *ctx);

/* Fields at the current time (Sec. 5, step 4: the new density and velocity
 * computed from the evolved populations): density h_n[N] = sum_a f_a and
 * velocity h_u[3N] = (j + F/2)/rho, the velocity of the trapezoidal forcing
 * of Sec. 5, step 3.  FP64 host arrays.  Either pointer may be NULL.
 * Synchronises. */
wdlb_status wdlb_read_fields(wdlb_ctx *ctx, double *h_n, double *h_u);

/* As wdlb_read_fields plus the fields of Sec. 5, step 2 at the current time:
 * the total force density h_F[3N] = n (g + F^mf + F^v), the external force of
 * eq. (1) plus the hydrodynamic collision term C_i = n (F^mf + F^v) of the
 * decomposition in Sec. 3 (mean-field force and the velocity-dependent part
 * of eq. campoc), and the traceless symmetric SMDB field h_A0[9N] of
 * eq. campod (row-major 3x3 per node).  Any pointer may be NULL. */
wdlb_status wdlb_read_fields_ex(wdlb_ctx *ctx, double *h_n, double *h_u, double *h_F, double *h_A0);

/* Plane means at the current time of the fields of Sec. 5, step 4 (density
 * and velocity recomputed from the evolved populations), reduced on the
 * device in FP64: h_n_z[nz] = <rho>_xy and h_ux_z[nz] = <u_x>_xy, the
 * density and flow profiles across the slit of the confinement experiments
 * of Sec. 5.  Either may be NULL. */
wdlb_status wdlb_read_profiles(wdlb_ctx *ctx, double *h_n_z, double *h_ux_z);

/* Pore-averaged properties at the current time (the pore-averaged transport
 * quantities of the abstract and introduction, from which the effective
 * viscosity of the slit experiment of Sec. 5 follows), FP64 device
 * reductions of the Sec. 5, step 4 fields: j_pore = sum(rho u_x)/N (mass
 * flux per node), u_pore = mean over z of <u_x>_xy, mass = sum(rho) (the
 * particle number conserved by the collision operator, Sec. 2).  Any pointer
 * may be NULL. */
wdlb_status wdlb_read_flux(wdlb_ctx *ctx, double *j_pore, double *u_pore, double *mass);

/* Thermal fields of Sec. 3 at given fields (k_B = m = 1), with the
 * context's sigma and shell (the contact value g_CS at the Fischer-Methfessel
 * weighted density of the given n at each pair midpoint, as in the step):
 *   h_Q[N]   energy source Q of eq. campob1,
 *   h_B[3N]  heat-flux correction B_i of eq. campos,
 *   h_FT[3N] thermal-gradient force F^T_i of eq. thermalforce,
 * from h_n[N] density (>= 0), h_u[3N] velocity and h_T[N] temperature
 * (> 0), all FP64 host arrays in the node order above (vectors
 * component-major).  The isothermal step does not use these fields; this
 * call evaluates them on request.  The fields are computed in the storage
 * arithmetic (FP64 or FP32), the inputs rounded to it first; the outputs may
 * be NULL.  The context's state is left as it was (the call may come before
 * init or between steps; it reuses per-step arrays that the next step
 * rewrites).  Errors: WDLB_E_INVAL for a null input, a negative or
 * non-finite density, a non-positive temperature or a non-finite velocity;
 * WDLB_E_UNSTABLE when a midpoint packing fraction of n reaches 1 (the
 * fields are then not written).  The nonlocal and smdb switches of the step
 * do not apply.  Synchronises. */
wdlb_status wdlb_thermal_fields(wdlb_ctx *ctx, const double *h_n, const double *h_u, const double *h_T, double *h_Q,
                                double *h_B, double *h_FT);

/* The same fields from device arrays, without host transfers: d_n[N],
 * d_u[3N], d_T[N] in, d_Q[N], d_B[3N], d_FT[3N] out, all device memory of
 * the storage real (double for WDLB_FP64, float in every other mode), in
 * the node order above; owned by the caller.  Asynchronous on the
 * context's stream (the inputs must stay valid, and the outputs are ready,
 * when the stream reaches the call); outputs may alias inputs.  The values
 * are not checked: a non-positive temperature gives non-finite fields, and
 * a midpoint packing fraction >= 1 of n is reported as WDLB_E_UNSTABLE by
 * the next synchronising call, as for a step.  WDLB_E_INVAL for a null
 * pointer, WDLB_E_STATE for a stacked lattice. */
wdlb_status wdlb_thermal_fields_device(wdlb_ctx *ctx, const void *d_n, const void *d_u, const void *d_T, void *d_Q,
                                       void *d_B, void *d_FT);

/* The energy balance of Sec. 2 (eq. energyequation) for the fluid at rest
 * (u = 0) with a fixed density, the setting in which Sec. 4 derives the
 * thermal conductivity (eq. thermalcond), k_B = m = 1:
 *   (3/2) n dT/dt = -div q + Q,  q = -(5/2)(n T / omega0) grad T + B / (2 omega0)
 * (eq. qexplicit; B and Q of Sec. 3 at u = 0 with the context's sigma and
 * shell).  Discretised by the flux through the six faces of each node (the
 * kinetic conductivity at the mean of n T of the two nodes, the mean of
 * B / (2 omega0)), no flux through a wall, and nsteps forward-Euler steps of
 * length dt.  h_n[N] (> 0) and h_T[N] (> 0, updated in place) are FP64 host
 * arrays in the node order above; omega0 > 0 the BGK rate of eq. qexplicit.
 * Computed in the storage arithmetic.  The context's state is untouched.
 * Errors: WDLB_E_INVAL for a bad argument or field, WDLB_E_UNSTABLE when a
 * midpoint packing fraction of n reaches 1 (h_T is then not written).
 * Explicit steps are stable for dt (5/3) T / omega0 <= 1/6 (the kinetic
 * part).  Synchronises. */
wdlb_status wdlb_conduction_at_rest(wdlb_ctx *ctx, const double *h_n, double *h_T, double omega0, double dt,
                                    int64_t nsteps);

/* The coupled thermal flow: the step with a local temperature T(r), a
 * hybrid of the paper's isothermal scheme (Sec. 5) and its non-isothermal
 * fields (Sec. 3) and energy balance (Sec. 2, eq. energyequation).  With
 * theta = T / kT at each node the step's mean-field force is scaled by
 * theta, the viscous force by sqrt(theta), A_ij by theta (Sec. 3 gives them
 * as k_B T, sqrt(k_B T) and k_B T times the isothermal sums), the thermal
 * force F^T (eq. thermalforce, from n and T alone) is added to the force,
 * the velocity u1 = j/rho + (g + theta F^mf + F^T)/2 of the viscous and
 * thermal sums carries every force known before them, and the collision
 * relaxes towards the equilibrium plus w_a rho (3/2)(theta - 1)(|c_a|^2 -
 * 1).  After the
 * stream T advances by one step of
 *   dT/dt = -u.grad T + (2/(3n)) (-div q - P:grad u + Q)
 * with q of eq. qexplicit (omega0 = 1/tau), P of eqs. pexplicit and
 * extrapressure (with the step's A), Q of eq. campob1; central differences
 * (beyond a wall u mirrored to -u and T to T), div q through the six faces
 * (none through a wall), the kinetic conduction in nsub sub-steps.
 *
 * FP64 or FP32 storage (WDLB_FP64, WDLB_FP32, WDLB_FP32_LOCAL64: T and
 * every field in the storage real, the local kernels in the mode's
 * arithmetic), the nonlocal fields on (smdb as set), one slit (not a
 * stacked lattice); otherwise WDLB_E_INVAL (the BF16 modes, the local
 * model) or WDLB_E_STATE (a stacked lattice).
 *
 * wdlb_init_thermal: the state as wdlb_init_fields(h_n, h_u) plus the
 * temperature term at h_T (N host doubles, each > 0 and finite, else
 * WDLB_E_INVAL); h_T is rounded to the storage real and copied to d_T, N
 * reals of device memory (double in WDLB_FP64, float otherwise) owned by
 * the caller, which holds T from then on.  Synchronises.
 *
 * wdlb_step_thermal: nsteps (>= 0) coupled steps; T in d_T is updated in
 * place, nsub >= 1 sub-steps of the conduction per step (WDLB_E_INVAL
 * otherwise; the explicit sub-steps are stable for (5/3) T tau / nsub <=
 * 1/6 at the largest T, the kinetic part).  Asynchronous on the context's
 * stream like wdlb_step: a density or temperature that is not positive and
 * finite at a step's start is reported as WDLB_E_UNSTABLE by the next
 * synchronising call (and the state is then not meaningful).  Pairs of
 * steps replay a captured graph as in wdlb_step (not while kernels are
 * timed, nor once wdlb_set_graphs has turned replay off); a call with
 * another d_T or nsub captures anew.  The state can be read, saved and
 * stepped isothermally as any other; the field reads give the isothermal
 * forces. */
wdlb_status wdlb_init_thermal(wdlb_ctx *ctx, const double *h_n, const double *h_u, const double *h_T, void *d_T);
wdlb_status wdlb_step_thermal(wdlb_ctx *ctx, void *d_T, int64_t nsteps, int32_t nsub);

/* Current post-stream populations f_a (19N, FP64, order above). */
wdlb_status wdlb_read_populations(wdlb_ctx *ctx, double *h_f);

/* Checkpoint: the complete state (populations in their stored encoding and
 * the step count) in wdlb_state_size bytes, copied to / from a host buffer.
 * A state can only be loaded into a context with the same lattice and
 * precision (WDLB_E_STATE otherwise). */
wdlb_status wdlb_state_size(const wdlb_ctx *ctx, size_t *bytes);
wdlb_status wdlb_save_state(wdlb_ctx *ctx, void *h_buf, size_t bytes);
wdlb_status wdlb_load_state(wdlb_ctx *ctx, const void *h_buf, size_t bytes);

/* Steps taken since the last init or load. */
wdlb_status wdlb_get_step(const wdlb_ctx *ctx, int64_t *step);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * the kernel launches of wdlb_step (off by default; each timed launch costs
 * a few microseconds of event overhead).  wdlb_profile(ctx, mask) times the
 * kernels whose id k has bit k set in mask (-1: all) and resets the totals;
 * mask 0 disables.  wdlb_profile_read synchronises and returns, for kernel
 * id k (0 .. WDLB_NKERNELS-1), the summed device time in milliseconds and
 * the number of launches timed.  wdlb_kernel_name(k) names the kernel (""
 * for an unknown id): 0 moments, 1 density, 2 meanfield, 3 shell,
 * 4 collide (the step's), 5 thermal (the thermal-field kernel of
 * wdlb_thermal_fields, wdlb_thermal_fields_device and wdlb_conduction_at_rest). */
#define WDLB_NKERNELS 6
wdlb_status wdlb_profile(wdlb_ctx *ctx, int32_t mask);
wdlb_status wdlb_profile_read(wdlb_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches);
const char *wdlb_kernel_name(int32_t kernel);

/* Contact-shell kernel choice (a tuning and testing knob: every choice sums
 * the same terms in the same order of mirror groups, so all of them give
 * the same result).  The two shell kernels (mean-field force; viscous force
 * and SMDB field) run on tiles of one of WDLB_NTILES variants:
 *   0..2  32 x 8 x 2 nodes, contact values and (rho, u1) staged in LDS, for
 *         growing shell reach;
 *   3     32 x 16 x 1 nodes, both staged in LDS;
 *   4     16 x 16 x 1 nodes, contact values read through the caches;
 *   5     16 x 16 x 2 nodes, both staged in LDS (lattices at most 16 wide);
 *   6     32 x 8 x 2 nodes, (rho, u1) staged in LDS, contact values read
 *         through the caches.
 * wdlb_set_tile(ctx, -1) (the default) picks variant 5 for lattices at most
 * 16 nodes wide in x when it fits, else the first of 0..4 whose LDS rings
 * fit the shell reach of sigma.  For sigma = 3, 4, 6, 8 or 10 it runs
 * kernels compiled for that shell (offsets and weights fixed at compile
 * time): on the chosen one of 0..3, or of 5 at sigma = 4 in FP32; at
 * sigma = 8 or 10 in FP32 the viscous/SMDB kernel moves to variant 6 (the
 * variant reported); in FP64 at sigma = 10, where no tile holds both LDS
 * rings of the viscous/SMDB kernel, it runs compiled on variant 6 (the
 * variant reported) and the mean-field kernel compiled on variant 1.
 * Variant 6 needs a padded sub-lattice below 2e9 bytes.  A variant >= 0 forces that tile with the
 * table-driven kernels and fails with WDLB_E_INVAL, leaving the previous
 * choice, when it does not fit.  wdlb_set_params re-applies the request for
 * the new sigma.  wdlb_get_tile returns the variant in use and (if
 * specialised is not NULL) 1 when compiled-shell kernels run, else 0.
 * wdlb_thermal_fields follows the same request: its compiled-shell kernel
 * (FP32, sigma = 3, 4, 6, 8 or 10) runs only under the automatic choice,
 * its table-driven kernels (same result, bit for bit) under a forced one. */
#define WDLB_NTILES 7
wdlb_status wdlb_set_tile(wdlb_ctx *ctx, int32_t variant);
wdlb_status wdlb_get_tile(wdlb_ctx *ctx, int32_t *variant, int32_t *specialised);

/* wdlb_step and wdlb_step_thermal replay pairs of steps as HIP graphs
 * (captured on first use on a private stream, launched on the context's
 * stream) unless kernel timing is on or the mode is WDLB_BF16_NEQ; the
 * result is the same as stepping launch by launch.  wdlb_set_graphs(ctx, 0)
 * turns replay off (1: on, the default). */
wdlb_status wdlb_set_graphs(wdlb_ctx *ctx, int32_t enable);

/* Message of the last failed call on this context ("" if none).  The
 * pointer stays valid until the next call on the context. */
const char *wdlb_last_error(const wdlb_ctx *ctx);

/* Release the context (host memory only; the workspace stays the caller's). */
void wdlb_destroy(wdlb_ctx *ctx);

/* ------------------------------------------------------------------------
 * Serving: batched solves of slit pores over resident requests (a project
 * addition on top of the paper's step).  A server owns one lattice of
 * nx x ny x nz planes (desc; walls_z must be 1, precision WDLB_FP32) and a
 * worker thread.  A request is a slit of height H (fluid planes) with its own
 * packing fraction eta (uniform start n0 = 6 eta / (pi sigma^3), u = 0),
 * body force g_x and relaxation time tau; sigma and the x,y extent are the
 * server's.  Resident requests are stacked along z, each followed by R gap
 * planes (R = the shell reach of sigma) that no stencil crosses, and are
 * stepped together, one launch chain per step.  A request is admitted
 * (arrival order, skipping those that do not fit yet) when a run of H + R
 * free planes exists, and retired when its pore flux changed by less than
 * tol (relative) over the last check_every steps, or after max_steps
 * (status WDLB_E_NOT_CONVERGED).  Its planes are then reused.  A request's
 * result does not depend on the other residents.
 *
 * The caller owns the device pool (size from wdlb_server_workspace_size,
 * 256-byte aligned); it must outlive the server.  The server runs its GPU
 * work on a stream of its own on the device current at create.
 * submit, poll, drain and stats may be called from any thread. */
typedef struct wdlb_server wdlb_server;

typedef struct {
    double sigma;        /* hard-sphere diameter of every request */
    double tol;          /* steady-state test |J(t) - J(t - check_every)| <= tol |J(t)| */
    int32_t check_every; /* steps between flux checks (and admissions) */
    int32_t pad;
    int64_t max_steps;   /* cap per request */
} wdlb_server_params;

typedef struct {
    int32_t H;           /* fluid planes of the slit (walls at z = -1/2 and H - 1/2) */
    int32_t pad;
    double eta, gx, tau;
} wdlb_request;

/* state: 0 queued, 1 running, 2 finished.  Times are seconds since the
 * server was created: submitted, admitted, finished. */
typedef struct {
    int32_t state;
    int32_t status;      /* wdlb_status of a finished request */
    int32_t H;
    int32_t pad;
    int64_t steps;       /* steps taken */
    double j_pore, u_pore;
    double t_submit, t_admit, t_done;
} wdlb_result;

typedef struct {
    int64_t chunks;        /* launch chains of check_every steps */
    int64_t steps;         /* steps of the server lattice */
    double node_updates;   /* fluid-node updates summed over steps */
    int32_t resident, max_resident, queued, finished;
    double busy_s;         /* wall time spent stepping */
} wdlb_server_stats;

wdlb_status wdlb_server_workspace_size(const wdlb_lattice_desc *desc, const wdlb_server_params *sp, size_t *bytes);
wdlb_status wdlb_server_create(const wdlb_lattice_desc *desc, const wdlb_server_params *sp, void *d_pool,
                               size_t bytes, wdlb_server **out);
/* Queue a request; *id identifies it.  WDLB_E_INVAL if it can never fit or
 * its parameters are invalid. */
wdlb_status wdlb_server_submit(wdlb_server *srv, const wdlb_request *req, uint64_t *id);
/* The request's state into *res.  When the request has finished and h_ux_z
 * is not NULL, also its plane means <u_x>_xy: res->H values (FP64) written
 * to h_ux_z, a host buffer of n_ux doubles; WDLB_E_INVAL (and nothing
 * written to h_ux_z) when n_ux < res->H.  *res is filled in either case, so
 * a first call with h_ux_z = NULL tells the size. */
wdlb_status wdlb_server_poll(wdlb_server *srv, uint64_t id, wdlb_result *res, double *h_ux_z, int32_t n_ux);
/* Block until every submitted request has finished. */
wdlb_status wdlb_server_drain(wdlb_server *srv);
wdlb_status wdlb_server_stats_get(wdlb_server *srv, wdlb_server_stats *st);
const char *wdlb_server_last_error(wdlb_server *srv);
/* Stop the worker (requests not finished are abandoned) and release the
 * server (host memory; the pool stays the caller's). */
void wdlb_server_destroy(wdlb_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* WDLB_H */
