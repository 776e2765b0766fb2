/*
 * vlbm.h -- C ABI of the MI355X (gfx950) vielbein lattice Boltzmann library.
 *
 * The library advances the D2Q16 populations f_k(theta, phi) of the vielbein
 * lattice Boltzmann method on a sphere (arXiv:2504.15574, Sec. III): BGK
 * collision toward the order-3 Hermite equilibrium, the Hermite-projected
 * inertial force, WENO-5 flux-form advection in theta and phi with periodic and
 * pole ghosts, and SSP-RK3 time stepping (Sec. III.G, eq. (Lf)).
 *
 * Conventions shared by every entry point
 *  - Grid (Sec. III.D, eq. (discrete_coord_sphere), 0-based): theta_s =
 *    (s + 1/2) pi / n_theta, phi_q = (q + 1/2) 2 pi / n_phi.
 *  - Fields are FP64, row-major [n_theta][n_phi] (phi fastest).  Velocities are
 *    the orthonormal (vielbein) components u^theta, u^phi.
 *  - Populations exchanged through the ABI are FP64 [Q*Q][n_theta][n_phi] with
 *    k = Q*k_theta + k_phi over the ascending nodes: Q = 4 (D2Q16, App. A.2)
 *    -sqrt(3+sqrt6), -sqrt(3-sqrt6), +sqrt(3-sqrt6), +sqrt(3+sqrt6); Q = 3
 *    (D2Q9, App. A.1) -sqrt3, 0, +sqrt3.  The equilibrium is eq. (feq_Q=4)
 *    or eq. (feq_Q=3).
 *  - "ptr_on_device" = 1: the pointer is HIP device memory and the call is
 *    asynchronous on the context stream; 0: host memory and the call
 *    synchronises the context stream before returning.
 *  - Every function returns a vlbm_status; no C++ exception crosses the ABI.
 *    On failure vlbm_last_error() (thread-local) describes the cause.
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Memory: the caller owns the device workspace (size from
 *    vlbm_workspace_bytes) and every field buffer; the library owns only the
 *    context object.  The workspace must outlive the context.
 */
#ifndef VLBM_H
#define VLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VLBM_ABI_VERSION 1u

typedef struct vlbm_ctx vlbm_ctx;

typedef enum {
    VLBM_OK = 0,
    VLBM_ERR_ARG = 1,          /* invalid argument; nothing was changed        */
    VLBM_ERR_UNSUPPORTED = 2,  /* valid but not implemented (Q != 4, scheme)   */
    VLBM_ERR_ALLOC = 3,        /* workspace too small / host allocation failed */
    VLBM_ERR_DEVICE = 4,       /* a HIP call failed                            */
    VLBM_ERR_UNSTABLE = 5      /* diagnostics found non-finite populations     */
} vlbm_status;

typedef enum {
    VLBM_STORE_F64 = 0,      /* f_k - w_k rho0 stored in FP64, FP64 arithmetic          */
    VLBM_STORE_F32_DEV = 1,  /* f_k - w_k rho0 stored in FP32, FP32 arithmetic          */
    VLBM_STORE_F16_DEV = 2   /* (f_k - w_k rho0) * 2^e_k stored in FP16, FP32 arithmetic */
} vlbm_storage;

/* Advection scheme (Sec. III.E): the interface flux in the low bits, optionally
 * OR-ed with VLBM_ADV_KOMISSAROV for the theta derivative of eq.
 * (Komissarov_scheme): flux function v f (no sin theta), interface flux times
 * sin theta_{s+-1/2} (exactly 0 at the poles), divided by
 * R (cos theta_{s-1/2} - cos theta_{s+1/2}); exactly well-balanced at rest and
 * at most second order. */
typedef enum {
    VLBM_ADV_WENO5 = 0,          /* WENO-5 fluxes, eqs. (fluxes_W5)-(WENO5_sigma) */
    VLBM_ADV_U1 = 1,             /* first-order upwind, eq. (fluxes_U1-3)          */
    VLBM_ADV_U2 = 2,             /* second-order upwind                            */
    VLBM_ADV_U3 = 3,             /* third-order upwind                             */
    VLBM_ADV_SCHEME_MASK = 0xff,
    VLBM_ADV_KOMISSAROV = 0x100
} vlbm_advection;

/* Problem statement (Sec. III, Sec. IV): grid, quadrature, tau, dt, scheme. */
typedef struct {
    uint32_t abi_version;  /* must equal VLBM_ABI_VERSION                            */
    int32_t n_theta;       /* >= 3 (pole ghosts mirror rows 0..2)                    */
    int32_t n_phi;         /* 1 (axisymmetric) or even (phi + pi must be a column)   */
    int32_t q;             /* Gauss-Hermite points per axis: 4 (D2Q16) or 3 (D2Q9)   */
    double radius;         /* R > 0                                                  */
    double tau;            /* BGK relaxation time > 0 (nu = tau at T0 = 1)           */
    double dt;             /* time step > 0; not clamped (see vlbm_suggest_dt)       */
    double rho0;           /* reference density of the stored deviations (> 0)       */
    double weno_eps;       /* > 0; nonlinear weights delta_j / (eps + sigma_j)^2     */
    int32_t storage;       /* vlbm_storage                                           */
    int32_t advection;     /* vlbm_advection: scheme | optional VLBM_ADV_KOMISSAROV  */
} vlbm_params;

/* Bytes of device workspace a context with these parameters needs (0 when the
 * parameters are invalid).  Holds the three population buffers of SSP-RK3
 * (f_n and two stages), FP64 metric tables, FP64 field staging and reduction
 * partials. */
size_t vlbm_workspace_bytes(const vlbm_params* params);

/* Create a context on the current HIP device.  hip_stream: a hipStream_t (NULL:
 * the default stream) on which every kernel of the context is launched.
 * workspace: device memory of at least vlbm_workspace_bytes(params) bytes,
 * 256-byte aligned.  Builds the FP64 tables (nodes, weights, K^H and K~^H of
 * eqs. (kernels), sin/cot tables of Sec. III.E) and uploads them; synchronises
 * the stream once.  Errors: VLBM_ERR_ARG (bad params / NULL pointers),
 * VLBM_ERR_UNSUPPORTED (q != 4, unknown storage or scheme), VLBM_ERR_ALLOC
 * (workspace too small), VLBM_ERR_DEVICE. */
vlbm_status vlbm_create(const vlbm_params* params, void* hip_stream, void* workspace,
                        size_t workspace_bytes, vlbm_ctx** out);

/* Set f_n = f^eq(rho, u, T) cell by cell (order-3 Hermite projection of a
 * Maxwellian at temperature T; T NULL means T = 1 everywhere), then encode it
 * in the storage format.  Fields as described above. */
vlbm_status vlbm_init_fields(vlbm_ctx* ctx, const double* rho, const double* u_theta,
                             const double* u_phi, const double* T, int ptr_on_device);

/* Advance n_steps >= 0 SSP-RK3 steps (Sec. III.G): three fused stage kernels per
 * step on the context stream, asynchronous.  Validates only its arguments. */
vlbm_status vlbm_step(vlbm_ctx* ctx, int64_t n_steps);

/* Macroscopic fields (eq. (f_moments_sum)): rho = sum f, u = sum f v / rho and
 * T = sum f |v - u|^2 / (2 rho).  T may be NULL. */
vlbm_status vlbm_moments(vlbm_ctx* ctx, double* rho, double* u_theta, double* u_phi,
                         double* T, int ptr_on_device);

/* Release the context (not the workspace, which belongs to the caller). */
vlbm_status vlbm_destroy(vlbm_ctx* ctx);

/* ---- support entry points (tests, checkpoints, diagnostics) ---- */

/* FP64 global reductions over the sphere with area element R^2 sin th dth dph:
 * out[0] mass, out[1] sum f|v|^2/2, out[2] kinetic energy rho|u|^2/2,
 * out[3] angular momentum rho u_phi R sin th, out[4] count of non-finite
 * populations, out[5] max |u|, out[6] min rho, out[7] max rho.  Host output;
 * synchronises the stream.  Returns VLBM_ERR_UNSTABLE when out[4] > 0. */
vlbm_status vlbm_diagnostics(vlbm_ctx* ctx, double out[8]);

/* Vorticity [d_th(u_phi sin th) - d_ph u_th] / (R sin th) (Sec. IV.D) of the
 * current state, fourth-order central differences, pole continuation by
 * velocity inversion at phi + pi.  Output field as above. */
vlbm_status vlbm_vorticity(vlbm_ctx* ctx, double* omega, int ptr_on_device);

/* Decode the current populations f_n to FP64 [Q*Q][n_theta][n_phi]. */
vlbm_status vlbm_get_populations(vlbm_ctx* ctx, double* f, int ptr_on_device);

/* Encode FP64 populations [Q*Q][n_theta][n_phi] into f_n (checkpoint resume). */
vlbm_status vlbm_set_populations(vlbm_ctx* ctx, const double* f, int ptr_on_device);

/* Moment correction (used by the learned closure): in every cell, with rho, u
 * the current moments, f_k += f^eq_k(rho + d_rho, u + d_u) - f^eq_k(rho, u)
 * (isothermal order-3 equilibrium, eq. (feq_Q=4)); the non-equilibrium part of
 * f is kept.  Fields as described above. */
vlbm_status vlbm_correct_moments(vlbm_ctx* ctx, const double* d_rho, const double* d_u_theta,
                                 const double* d_u_phi, int ptr_on_device);

/* Largest stable time step suggested for these parameters: the smallest of
 * 0.2 dth, tau (explicit BGK needs dt < tau, Sec. V) and half the phi-CFL limit
 * of the row next to the pole, 0.5 R sin(dth/2) dph / v_max (dropped when
 * n_phi = 1).  Returns 0 for invalid parameters. */
double vlbm_suggest_dt(const vlbm_params* params);

/* The FP32 nodes v[4] (ascending) and product weights w[16] (k = 4 k_theta +
 * k_phi) that the FP32 and FP16 storage formats compute with.  They are the
 * D2Q16 Gauss-Hermite rule (App. A) moved by at most 10 ulps (nodes) and 40
 * ulps (weights) so that, evaluated on these FP32 values, sum w - 1
 * (residual[0]) is 0 and the fourth moments sum w v_theta^4 - 3 (residual[2])
 * and sum w v_theta^2 v_phi^2 - 1 (residual[3]) nearly vanish; residual[1] =
 * sum w v_theta^2 - 1 is absorbed by the equilibrium's coefficients, which the
 * float kernels derive from these moments so that BGK conserves mass and
 * momentum on the FP32 rule.  Plain rounding of the FP64 rule misses the
 * fourth moment by 2e-7.  residual[0] and residual[1] are exact, residual[2]
 * and residual[3] accurate to 1e-18.  Host only; needs no device.  Errors:
 * VLBM_ERR_ARG (NULL pointer). */
vlbm_status vlbm_quadrature_f32(float v[4], float w[16], double residual[4]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the eight
 * diagnostics of vlbm_diagnostics (same order) of FP64 populations
 * f [q*q][n_theta][n_phi] in device memory (full f, as vlbm_get_populations
 * returns them), without a context or workspace.  out: device memory for 8
 * FP64 values.  Asynchronous on hip_stream (NULL: the default stream); it
 * neither synchronises nor allocates (no hipMalloc, no memset), so it can be
 * recorded into a HIP graph.  Its partial sums and sin(theta) table live in a
 * 1 MiB static device array of the library, one per device, held until the
 * process ends and shared by every call on that device: calls that overlap in
 * time on one device race (serialise them on one stream).  Grids up to
 * n_theta = 122 874 rows (the table's reach) and 2^31 - 1 cells.  Unlike
 * vlbm_diagnostics it does not report VLBM_ERR_UNSTABLE: out[4] counts the
 * non-finite populations.  Errors: VLBM_ERR_ARG (NULL pointer, bad grid or
 * radius, n_theta beyond the scratch), VLBM_ERR_UNSUPPORTED (q not 3 or 4),
 * VLBM_ERR_DEVICE. */
vlbm_status vlbm_diagnostics_static(int n_theta, int n_phi, int q, double radius, const double* f,
                                    double* out, void* hip_stream);

/* ---- ensembles (many independent runs per launch) ---- */

typedef struct vlbm_graph vlbm_graph;

/* Advance n_ctx independent contexts by n_steps SSP-RK3 steps with one stage
 * launch per RK stage covering the tiles of all of them (64 contexts per
 * launch; more are split into several launches).  The contexts may differ in
 * grid, tau and dt but must share the storage format, the device and the
 * stream, and appear once each.  Every cell runs the same arithmetic as in
 * vlbm_step, so the result equals stepping each context alone, bit for bit.
 * Asynchronous on the shared stream.  Errors: VLBM_ERR_ARG. */
vlbm_status vlbm_step_batch(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps);

/* The same steps as vlbm_step_batch in one persistent launch per 64
 * contexts: a cooperative kernel whose co-resident workgroups take the tiles
 * of every RK stage in turn and meet at a grid-wide barrier between stages
 * (SSP-RK3, Sec. III.G: stage s+1 reads stage s over every halo).  Results
 * equal vlbm_step_batch and vlbm_step bit for bit.  The contexts must use
 * D2Q16 and the standard WENO-5 form (VLBM_ADV_WENO5), besides sharing what
 * vlbm_step_batch requires; the barrier count lives in the first context's
 * workspace, so two persistent calls on the same first context must not
 * overlap.  Synchronous: returns after the launch has finished.  Each
 * barrier wait is bounded (vlbm_set_barrier_spin_limit); a wait that gives up
 * (a grid that was not co-resident) leaves the runs' state undefined and
 * returns VLBM_ERR_DEVICE.  Errors: VLBM_ERR_ARG, VLBM_ERR_DEVICE. */
vlbm_status vlbm_step_batch_persistent(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps);

/* Polls of one grid-barrier wait before vlbm_step_batch_persistent gives up
 * (default 2^20, about a second; one stage takes milliseconds).  Process-wide.
 * A tiny limit makes the waits give up, which tests use to check the error
 * path without stalling the device. */
vlbm_status vlbm_set_barrier_spin_limit(uint32_t polls);

/* Record n_steps >= 1 of vlbm_step_batch(ctxs, n_ctx, .) into a HIP graph
 * (captured on a private stream; nothing runs now).  The graph refers to the
 * contexts (launch and check read them) and their workspaces: destroy it
 * before either.  Errors: VLBM_ERR_ARG,
 * VLBM_ERR_DEVICE (capture or instantiation failed), VLBM_ERR_ALLOC. */
vlbm_status vlbm_graph_create(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps,
                              vlbm_graph** out);

/* Record n_steps >= 1 of vlbm_step_batch_persistent(ctxs, n_ctx, .) into a HIP
 * graph: per 64 contexts a kernel that clears the barrier state and the
 * persistent stage kernel, as ordinary kernel nodes (no memset nodes).  In
 * the graph the persistent launch is not cooperative: its grid is what the
 * CUs hold at once, so it is co-resident while nothing else runs on the
 * device, and a barrier wait that gives up is reported by vlbm_graph_check.
 * The contexts' constraints are those of vlbm_step_batch_persistent.  Errors:
 * as vlbm_graph_create. */
vlbm_status vlbm_graph_create_persistent(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps,
                                         vlbm_graph** out);

/* Replay the recorded steps on the contexts' stream (asynchronous). */
vlbm_status vlbm_graph_launch(vlbm_graph* graph);

/* Wait for the graph's last replay and report whether a persistent launch in
 * it gave up at a grid barrier (VLBM_ERR_DEVICE; the runs' state is then
 * undefined).  Synchronises the contexts' stream.  VLBM_OK for graphs of
 * vlbm_graph_create once their work has finished.  Errors: VLBM_ERR_ARG. */
vlbm_status vlbm_graph_check(vlbm_graph* graph);

/* Release the graph (not the contexts). */
vlbm_status vlbm_graph_destroy(vlbm_graph* graph);

/* Tile shape (theta rows x phi columns) of the context's stage launches: 15 x 16
 * (the default) or 7 x 32.  The shape never changes a cell's arithmetic, so
 * every choice gives the same bits; contexts of one batch must share it.
 * Errors: VLBM_ERR_ARG (NULL), VLBM_ERR_UNSUPPORTED (other shapes). */
vlbm_status vlbm_set_tile_shape(vlbm_ctx* ctx, int rows, int cols);

/* Number of stage-kernel launches issued so far by this context (a batched
 * launch counts once for every context it covers). */
int64_t vlbm_stage_launches(const vlbm_ctx* ctx);

/* Text of the last error on this thread ("" if none). */
const char* vlbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VLBM_H */
