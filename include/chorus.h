/*
 * chorus.h -- C ABI of the MI355X spectral-difference (SD) library.
 *
 * The library evaluates the SD residual and the explicit SSP-RK3 update of
 * the compressible Navier-Stokes equations in a rotating frame with radial
 * 1/r^2 gravity (Wang, Liang & Miesch, "A Compressible High-Order
 * Unstructured Spectral Difference Code for Stratified Convection in
 * Rotating Spherical Shells": Section 2, Eqs. 1-9; Section 3, the SD
 * discretisation on 20-node hexahedra; Section 5, wall conditions) on GPU
 * (gfx950, HIP).  Every call below that touches device memory is
 * asynchronous on the given stream unless stated otherwise.
 *
 * Conventions
 *   Status: every function returns 0 (CHORUS_OK) or a negative CHORUS_E*
 *   code; chorus_last_error() gives the detail text of the calling thread's
 *   last failure.  No C++ exception crosses this boundary.
 *
 *   Ownership: the caller owns every device buffer (state, residual,
 *   workspace, geometry image, network weights); the library never
 *   allocates or frees device memory.  A mesh handle owns host arrays only
 *   and remembers the device geometry image registered by
 *   chorus_mesh_upload, which must stay alive while the handle is used.
 *   Handles are not thread-safe: use one handle from one thread at a time.
 *
 *   State layout: Q is the physical conserved vector (rho, rho u, rho v,
 *   rho w, E) at the N^3 solution points of each element, structure of
 *   arrays [5][E][N^3] in float64, solution point index i + N (j + N k)
 *   with i along the element's local xi axis (Section 3: DOFs = E N^3).
 *
 *   Hex20 node order (local reference cube [0,1]^3): corners (i,j,k) in
 *   {0,1}^3 at index i + 2j + 4k; xi-edge midpoints (1/2,j,k) at 8 + j + 2k;
 *   eta-edge midpoints (i,1/2,k) at 12 + i + 2k; zeta-edge midpoints
 *   (i,j,1/2) at 16 + i + 2j.  Local faces 0..5 = xi=0, xi=1, eta=0, eta=1,
 *   zeta=0, zeta=1.  Face tags: -1 interior, 1 inner wall, 2 outer wall,
 *   3 far-field state.
 *
 *   stream: a hipStream_t passed as void* (NULL = default stream).
 */
#ifndef CHORUS_H
#define CHORUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CHORUS_OK = 0,
    CHORUS_EINVAL = -1,      /* bad argument: null pointer, size, order   */
    CHORUS_EMESH = -2,       /* non-conforming mesh, unmatched face, |J|<=0 */
    CHORUS_ENOTSUP = -3,     /* valid but unsupported combination         */
    CHORUS_EHIP = -4,        /* HIP runtime error                         */
    CHORUS_ENONFINITE = -5,  /* NaN/Inf or non-positive rho/p found        */
    CHORUS_ESTATE = -6       /* call order: e.g. no geometry uploaded      */
};

enum { CHORUS_FP64 = 0, CHORUS_MIXED = 1 };            /* chorus_physics.precision */
enum { CHORUS_CLOSURE_NONE = 0, CHORUS_CLOSURE_MLP = 1 }; /* chorus_physics.closure */
enum { CHORUS_SSPRK3 = 0, CHORUS_SSPRK54 = 1 };         /* chorus_physics.integrator */
enum { CHORUS_CHECK_FINITE = 1,                       /* chorus_physics.flags     */
       CHORUS_BALANCED = 2 };                          /* see chorus_set_background */
enum { CHORUS_BC_INTERIOR = -1, CHORUS_BC_INNER = 1, CHORUS_BC_OUTER = 2,
       CHORUS_BC_STATE = 3 };

typedef struct chorus_mesh_s *chorus_mesh_t;

/* Cubed-sphere shell: 6 equiangular panels of panel_n x panel_n columns and
 * radial_n uniform layers between r_inner and r_outer (the paper's shells
 * are all-hex with uniform radial spacing, Section 3 mesh figure). */
typedef struct {
    int32_t panel_n, radial_n, order;
    double r_inner, r_outer;
} chorus_shell_desc;

/* Explicit hex20 mesh (arrays are copied; caller keeps ownership). */
typedef struct {
    int64_t n_nodes;
    const double *xyz;        /* [n_nodes][3]                                 */
    int64_t n_elems;
    const int64_t *elem20;    /* [n_elems][20] node indices, order above      */
    const int32_t *face_bc;   /* [n_elems][6] face tags                       */
    const int64_t *match_id;  /* [n_nodes] topological ids (periodic images
                                 share one) or NULL for the node index         */
    int32_t order;            /* N, 2..6                                      */
} chorus_hex20_desc;

/* Physics (Section 2).  g_vec = -GM x / r^3; rotation Omega about z; mu =
 * rho nu; diffusive energy flux f = -kappa rho T grad S - kappa_r rho c_p
 * grad T; walls impermeable and stress-free (Section 5) with f.r_hat =
 * F_bottom at the inner wall and T = T_top at the outer wall (T_top <= 0:
 * interior temperature kept).  The radiative diffusivity may vary with
 * radius as in the solar benchmark (Section 7.4, a quadratic in r):
 * kappa_r(r) = kappa_r + kappa_r1 r + kappa_r2 r^2, evaluated at the radius
 * of each flux point (kappa_r1 = kappa_r2 = 0: constant).  It must not be
 * negative anywhere on the mesh (CHORUS_EINVAL). */
typedef struct {
    double gamma, R_gas, GM, omega, nu, kappa, kappa_r, T_top, F_bottom;
    double bc_state[5];       /* state for CHORUS_BC_STATE faces              */
    int32_t precision;        /* CHORUS_FP64 or CHORUS_MIXED                  */
    int32_t closure;          /* CHORUS_CLOSURE_NONE, or CHORUS_CLOSURE_MLP:
                                 add the learned subgrid flux (order 3, FP64
                                 precision only; see the closure section)     */
    int32_t flags;            /* CHORUS_CHECK_FINITE                          */
    int32_t integrator;       /* chorus_rk_step: CHORUS_SSPRK3 or
                                 CHORUS_SSPRK54                               */
    const void *closure_model;/* device image from chorus_closure_pack when
                                 closure == CHORUS_CLOSURE_MLP, else ignored   */
    double kappa_r1, kappa_r2;/* radial terms of kappa_r(r) (see above)      */
} chorus_physics;

/* Build a cubed-sphere shell mesh (host only). */
int chorus_mesh_create(const chorus_shell_desc *desc, chorus_mesh_t *out);
/* Build a mesh from explicit hex20 arrays (host only). */
int chorus_mesh_create_hex20(const chorus_hex20_desc *desc, chorus_mesh_t *out);
int chorus_mesh_destroy(chorus_mesh_t mesh);

/* Sizes: elements, order, solution points (E N^3), faces (interior + wall),
 * wall faces and the byte size of the device geometry image. */
int chorus_mesh_query(chorus_mesh_t mesh, int64_t *n_elems, int32_t *order,
                      int64_t *n_solpts, int64_t *n_faces, int64_t *n_wall_faces,
                      size_t *device_bytes);
/* Hex20 arrays of the mesh (host buffers of n_nodes*3, n_elems*20,
 * n_elems*6); n_nodes is returned first when xyz == NULL. */
int chorus_mesh_nodes(chorus_mesh_t mesh, int64_t *n_nodes, double *xyz, int64_t *elem20,
                      int32_t *face_bc);
/* Solution-point coordinates [3][E N^3] and quadrature weights
 * w_i w_j w_k |J| [E N^3] (host buffers). */
int chorus_mesh_solpts(chorus_mesh_t mesh, double *xyz_host, double *wJ_host);
/* Geometry as used by the kernels (host buffers, any may be NULL):
 * |J| [E N^3]; |J| grad xi_d at solution points [E N^3][3 d][3 c];
 * |J| grad xi_d at the d-flux points [E][3 d][(N+1) N^2][3 c] (flux point
 * index a + (N+1)(t1 + N t2), a along d, t1 < t2 the other axes). */
int chorus_mesh_geometry(chorus_mesh_t mesh, double *jac, double *met_sol, double *met_flux);
/* Face table: neighbour element, neighbour face and orientation code
 * (swap*4 + flip1*2 + flip2) per element face, -1 on boundaries. */
int chorus_mesh_face_table(chorus_mesh_t mesh, int32_t *nbr_elem, int32_t *nbr_face,
                           int32_t *orient);
/* Copy the geometry image into the caller-owned device buffer dev_buf of
 * at least device_bytes bytes and register it with the handle.
 * Synchronises the stream. */
int chorus_mesh_upload(chorus_mesh_t mesh, void *dev_buf, size_t bytes, void *stream);

/* Workspace bytes for every residual, step, background and closure call on
 * this mesh: one layout serves all precisions, closures and integrators
 * (phys, if given, is only validated). */
int chorus_workspace_bytes(chorus_mesh_t mesh, const chorus_physics *phys, size_t *bytes);

/* Polytropic adiabatic initial state (Section 4.2) at the solution points:
 * depth 1, rho = p = 1 at mid-layer, given aspect ratio beta, density scale
 * heights n_rho and index poly_n; optional entropy perturbation
 * S' = amp c_p noise[i] at fixed pressure (noise: host [E N^3] or NULL).
 * Q_host [5][E N^3]; pars (may be NULL) receives chi_o, c, alpha, GM. */
int chorus_init_polytrope(chorus_mesh_t mesh, double beta, double n_rho, double poly_n,
                          double gamma, double R_gas, const double *noise, double amp,
                          double *Q_host, double pars[4]);

/* Almost-flux-balance background (Section 4.3): the polytrope of Section
 * 4.2 (same units as chorus_init_polytrope) gives the target entropy
 * gradient Gamma = -(L / (4 pi r^2) + rho_a c_p kappa_r dT_a/dr) /
 * (rho_a T_a kappa) at which the diffusive flux of Section 2 carries L
 * outward; the hydrostatic state with that entropy gradient,
 * d p0/dr = -rho0 g and d rho0/dr = -rho0 (Gamma / c_p + g rho0 /
 * (gamma p0)), is integrated from the polytrope's mid-layer point (rho0 =
 * p0 = 1) to both walls.  Q_host [5][E N^3] receives the state at rest;
 * pars (may be NULL) receives (chi_o, c, alpha, GM, T0 at the outer wall,
 * bottom flux L / (4 pi R_i^2)) for chorus_physics (GM, T_top, F_bottom).
 * kappa is the solver's constant entropy diffusivity; kappa_r(r) =
 * kappa_r + kappa_r1 r + kappa_r2 r^2 its radiative diffusivity (as in
 * chorus_physics). */
typedef struct {
    double beta, n_rho, poly_n, gamma, R_gas;
    double luminosity;        /* L in the units of depth 1, rho_c = p_c = 1 */
    double kappa, kappa_r;
    double kappa_r1, kappa_r2;
    const double *noise;      /* host [E N^3] or NULL: entropy perturbation
                                 S' = amp c_p noise at fixed pressure, as in
                                 chorus_init_polytrope                         */
    double amp;
} chorus_afb_desc;
int chorus_init_afb(chorus_mesh_t mesh, const chorus_afb_desc *desc, double *Q_host, double pars[6]);

/* Radiative diffusivity of the solar benchmark (Section 7.4, Table 2) in
 * the units of chorus_init_polytrope (depth 1, rho = p = 1 at mid-layer):
 * the printed quadratic lambda (c0 + c1 w + c2 w^2) in w = r / 1e10 cm,
 * with r = r_unit * depth_cm (depth_cm <= 0: Table 2's shell depth,
 * 1.74e10 cm), written as kappa_r(r) = out[0] + out[1] r + out[2] r^2 for
 * chorus_physics (kappa_r, kappa_r1, kappa_r2).  lambda is set so that the
 * polytrope's radiative flux -kappa_r rho c_p dT/dr carries L / (4 pi R_i^2)
 * through the inner wall, which makes the almost-flux-balance entropy
 * gradient (Section 4.3) vanish there, as the section describes for the
 * solar run.  Host only; CHORUS_EINVAL for beta outside (0, 1), poly_n,
 * R_gas <= 0, gamma <= 1, a negative luminosity or out == NULL. */
int chorus_solar_kappa_r(double beta, double n_rho, double poly_n, double gamma, double R_gas,
                         double luminosity, double depth_cm, double out[3]);

/* Mixed mode: register the background state Q0 (device, [5][E N^3] FP64)
 * and compute, once, its complete FP64 residual R(Q0) and the background
 * arrays into the workspace.  Synchronises.  Q0 must be at rest (zero
 * momentum; CHORUS_EINVAL otherwise); CHORUS_BC_STATE faces are not
 * supported (CHORUS_ENOTSUP).  A failed call leaves no background
 * registered: chorus_rk_step and chorus_sd_residual in mixed precision
 * then return CHORUS_ESTATE until a call succeeds.
 * Balanced mode (phys->flags & CHORUS_BALANCED, set here and in every call
 * that uses it): the residual becomes R(Q) - R(Q0) in both precisions, so
 * the background is a discrete steady state (to rounding) and only its
 * departure from one evolves.  The subtracted term is the discretisation's
 * own imbalance of Q0, of the order of the truncation error (h^N); it lets
 * a background built from the continuous equations, such as the
 * almost-flux-balance state of Section 4.3, start convection from a seeded
 * perturbation instead of adjustment flows.  FP64 calls with the flag need
 * a background registered with this workspace and the same physics
 * (CHORUS_ESTATE otherwise); mixed calls need a background registered with
 * the flag. */
int chorus_set_background(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q0_dev,
                          void *ws, void *stream);

/* SD residual dQ/dt = -(div F~)/|J| - M at the solution points (Section 3:
 * transformed equations, Rusanov + BR1 interface treatment).
 * Q_dev, dQdt_dev: device [5][E N^3] float64. */
int chorus_sd_residual(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q_dev,
                       double *dQdt_dev, void *ws, void *stream);

/* n_steps explicit Runge-Kutta steps of size dt, in place on Q_dev:
 * phys->integrator = CHORUS_SSPRK3, the three-stage third-order SSP method
 * (Shu-Osher), or CHORUS_SSPRK54, the five-stage fourth-order SSP method of
 * Spiteri & Ruuth (2002) that the paper uses (Section 7.5), in Shu-Osher
 * form with one extra accumulation register (the workspace grows by two
 * state copies).  The state stays FP64 in both precisions. */
int chorus_rk_step(chorus_mesh_t mesh, const chorus_physics *phys, double *Q_dev, double dt,
                   int32_t n_steps, void *ws, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * FP64 steps as chorus_rk_step (SSP-RK3 or SSPRK(5,4), in place on Q_dev,
 * bitwise equal results) without a workspace argument.  The stage registers,
 * mailboxes and flag live in a fixed device array of
 * CHORUS_NOALLOC_SCRATCH_BYTES inside the library: one copy per GPU, held
 * until the process ends, its address looked up on the first call on each
 * device (the current device must be the stream's).  No allocator is
 * called.  Limits: CHORUS_FP64 precision without the learned closure or
 * CHORUS_BALANCED (CHORUS_ENOTSUP otherwise); the mesh must fit the array (about 6,500
 * hexes at N = 4 with SSP-RK3, 4,300 with SSPRK(5,4)), else CHORUS_EINVAL
 * before anything runs, with the bytes needed in chorus_last_error.  Every
 * call on one GPU shares the array and leaves its contents behind (no
 * kernel reads a value it did not write in the same call): calls that
 * overlap on one GPU, from other streams or threads, race and must be
 * serialised by the caller.  CHORUS_CHECK_FINITE synchronises, as in
 * chorus_rk_step. */
#define CHORUS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int chorus_rk_step_noalloc(chorus_mesh_t mesh, const chorus_physics *phys, double *Q_dev, double dt,
                           int32_t n_steps, void *stream);

/* Conserved totals (Section 6: the conservative form with interface fluxes
 * shared by both sides conserves them discretely): the sum over solution
 * points of w_i w_j w_k |J| Q_v for the 5 conserved variables, in a fixed
 * reduction order (bitwise reproducible).  Q_dev: device [5][E N^3] FP64;
 * the workspace holds the partial sums; the 5 sums are returned on the host
 * (synchronises).  CHORUS_EINVAL for null pointers, CHORUS_ESTATE before
 * chorus_mesh_upload. */
int chorus_conserved_sums(chorus_mesh_t mesh, const double *Q_dev, double out_host[5], void *ws,
                          void *stream);

/* Angular momentum over the shell (Section 6): out_host = (L_x, L_y, L_z,
 * I_x, I_y, I_z) with L = integral of rho r x u and I_x = integral of
 * rho (y^2 + z^2) (likewise I_y, I_z), by the solution-point quadrature in a
 * fixed reduction order.  Synchronises. */
int chorus_angular_momentum(chorus_mesh_t mesh, const double *Q_dev, double out_host[6], void *ws, void *stream);
/* Angular-momentum correction (Section 6): dOmega_c = L_c / I_c and, at
 * every solution point, u <- u - dOmega x r (the paper's velocity update;
 * its atan2 forms are the components of dOmega x r), keeping density and
 * pressure (the total energy takes the kinetic-energy change).  The paper
 * applies it every 5000 steps.  dOmega_host (may be NULL) receives the
 * rates.  Synchronises for the reduction; the update is queued on stream. */
int chorus_am_correct(chorus_mesh_t mesh, double *Q_dev, double dOmega_host[3], void *ws, void *stream);

/* Explicit time step from the host state Q_host [5][E N^3] (host only):
 * dt = cfl / (N max_points sum_d (|u . grad xi_d| + c |grad xi_d|)), the
 * acoustic CFL condition dt < delta / c_s of Section 7 measured in
 * reference-element units and summed over the three directions. */
int chorus_stable_dt(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q_host,
                     double cfl, double *dt);

/* Opt-in kernel timing for benchmarks: while enabled, every kernel launch of
 * chorus_sd_residual / chorus_rk_step is bracketed by a pair of HIP events
 * recorded on the launch stream (no extra work is launched).
 * chorus_kernel_times waits for the recorded events and returns, per kernel
 * kind, the summed milliseconds and launch counts, then clears the record.
 * Kinds: 0 the face traces that start a call (FP64: trace push; mixed:
 * perturbation set-up and its traces); 1 the first pass of a stage, the flux
 * pass (common values, gradients, fluxes, divergence, source, stage
 * combination); 2 the second pass, the lift pass (the neighbours' viscous
 * halves added in place, the next face traces pushed).  Both precisions
 * have the same two passes.  Not thread-safe; process-wide. */
int chorus_kernel_timing(int enable);
int chorus_kernel_times(double ms[3], int64_t counts[3]);

/* ------------------------------------------------------------------------
 * Learned subgrid closure.  The paper names large-eddy simulation with
 * subgrid modelling as the code's next step (Summary) and treats entropy
 * diffusion as a parameterisation of unresolved motion (Section 2).  Here a
 * pointwise network 20 -> 64 -> 64 -> 15 with GELU (x Phi(x)) activations
 * maps the features of a solution point -- the conserved state Q (5) and
 * its BR1 gradients dQ_v/dx_c (15, index 5 + 3 v + c) -- to a Cartesian
 * subgrid flux tau[3 v + c] that is added to the total flux: interpolated
 * to the flux points like the gradients, averaged between the two sides of
 * an interior interface, and left out at wall and far-field faces.
 *
 * Parameter vector (FP32, CHORUS_MLP_NPARAM values, z_j = sum_i W[j][i]
 * x_i + b_j): W1[64][20], b1[64], W2[64][64], b2[64], W3[15][64], b3[15].
 * Normalisation (FP32, CHORUS_MLP_NNORM values): x_mean[20], x_inv_std[20],
 * y_mean[15], y_std[15]; network input x = (feature - x_mean) x_inv_std,
 * output tau = y_mean + y_std y.
 * Inference runs on bfloat16 matrix cores with FP32 accumulation (inputs,
 * weights and hidden activations rounded to bfloat16, nearest-even), inside
 * the order-3 flux pass of a solve; training runs in FP32.
 * ---------------------------------------------------------------------- */
enum { CHORUS_MLP_IN = 20, CHORUS_MLP_HIDDEN = 64, CHORUS_MLP_OUT = 15, CHORUS_MLP_NPARAM = 6479,
       CHORUS_MLP_NNORM = 70 };

/* Byte size of the packed inference image. */
int chorus_closure_model_bytes(size_t *bytes);
/* Pack FP32 parameters and normalisation (device) into the inference image
 * model_dev (device, chorus_closure_model_bytes, 256-byte aligned).
 * Synchronises; returns CHORUS_ENONFINITE (image marked unusable) if any
 * value is NaN or infinite, so a caller can fall back to the plain solve. */
int chorus_closure_pack(const float *params_dev, const float *norm_dev, void *model_dev, void *stream);
/* Raw features at every solution point: X_dev [E N^3][20] FP32 (Q, then
 * the BR1 gradients), from Q_dev [5][E N^3] (FP64 precision, any order). */
int chorus_closure_features(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q_dev, float *X_dev,
                            void *ws, void *stream);
/* Subgrid flux of the network phys->closure_model at every solution point:
 * sgs_dev [15][E N^3] FP32 (order 3, FP64 precision). */
int chorus_closure_infer(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q_dev, float *sgs_dev,
                         void *ws, void *stream);
/* Training workspace bytes for mini-batches of up to `batch` samples. */
int chorus_closure_train_workspace_bytes(int64_t batch, size_t *bytes);
/* Mean-squared-error loss over n samples (X_dev [n][20] normalised inputs,
 * Y_dev [n][15] normalised targets) and its gradient with respect to the
 * parameter vector: grad_dev [CHORUS_MLP_NPARAM], loss_dev [1] (device,
 * FP32, fixed summation order).  n <= the workspace's batch. */
int chorus_closure_grad(const float *X_dev, const float *Y_dev, int64_t n, const float *params_dev,
                        float *grad_dev, float *loss_dev, void *ws, size_t ws_bytes, void *stream);
/* `iters` Adam steps (Kingma & Ba 2015) on mini-batches: iteration i uses
 * the samples idx_dev[i batch .. (i+1) batch - 1] (int32, device; the
 * caller draws them).  params/adam_m/adam_v [CHORUS_MLP_NPARAM] FP32 are
 * updated in place; the bias correction uses step step0 + i + 1;
 * hyper = (lr, beta1, beta2, eps); loss_dev [iters] receives the loss of
 * each mini-batch before its update.  Every index is checked on the device
 * first: one outside [0, n) returns CHORUS_EINVAL with the parameters
 * untouched (the call waits for the stream once, to read that check). */
int chorus_closure_train(const float *X_dev, const float *Y_dev, int64_t n, const int32_t *idx_dev,
                         int32_t batch, int32_t iters, float *params_dev, float *adam_m_dev, float *adam_v_dev,
                         int64_t step0, const double hyper[4], float *loss_dev, void *ws, size_t ws_bytes,
                         void *stream);
/* Training targets from a higher-order solution on the same hex mesh:
 * per element the L2 projection of |J| U onto tensor polynomials of
 * degree N_c - 1, divided by |J| at the coarse solution points (G U;
 * preserves element integrals).  Qbar_dev [5][E N_c^3] = G Q and
 * tau_dev [15][E N_c^3] = G F(Q) - F(G Q), F the Cartesian inviscid flux
 * (Section 2), both FP64.  fine and coarse: the same hex mesh at orders
 * N_f > N_c, both uploaded; gamma: ratio of specific heats. */
int chorus_closure_filter(chorus_mesh_t fine, chorus_mesh_t coarse, double gamma, const double *Qfine_dev,
                          double *Qbar_dev, double *tau_dev, void *stream);

const char *chorus_strerror(int status);
int chorus_last_error(char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* CHORUS_H */
