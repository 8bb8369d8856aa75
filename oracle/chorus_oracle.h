/*
 * CPU FP64 oracle of the spectral-difference (SD) residual and SSP-RK3 update
 * of "A Compressible High-Order Unstructured Spectral Difference Code for
 * Stratified Convection in Rotating Spherical Shells" (Wang, Liang, Miesch).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, loop-by-loop statement of
 * the method used to check the GPU library.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.  It shares no code with the GPU library.
 *
 * Conventions (shared with the library only through documentation):
 *   state Q     [5][E][N^3]  (rho, rho u, rho v, rho w, E), solution point
 *               index i + N (j + N k), i along xi;
 *   hex20 nodes as documented in chorus_inputs (corners i+2j+4k, then the
 *               xi-, eta- and zeta-edge midpoints);
 *   faces 0..5  = xi=0, xi=1, eta=0, eta=1, zeta=0, zeta=1;
 *   face_bc     -1 interior, 1 inner wall, 2 outer wall, 3 far-field state.
 */
#ifndef CHORUS_ORACLE_H
#define CHORUS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAXN 8

typedef struct {
    double gamma, R_gas, GM, omega, nu, kappa, kappa_r;
    double T_top;     /* outer-wall temperature; <= 0 keeps the interior p */
    double F_bottom;  /* prescribed f . r_hat at the inner wall            */
    double bc_state[5];
    /* radius-dependent radiative diffusivity (Section 7.4, solar case):
     * kappa_r(r) = kappa_r + kappa_r1 r + kappa_r2 r^2 at each flux point */
    double kappa_r1, kappa_r2;
} ora_phys;

typedef struct ora_mesh ora_mesh;

/* 1D SD operators (Section 3): solution points xs[N], flux points xf[N+1],
 * interpolation I[(N+1)][N] (I[m][s] = h_s(xf[m])), derivative
 * D[N][N+1] (D[s][m] = l'_m(xs[s])), weights w[N] = int_0^1 h_s. */
int ora_basis(int N, double *xs, double *xf, double *I, double *D, double *w);

ora_mesh *ora_mesh_new(int N, long n_nodes, const double *xyz, long n_elems,
                       const long *elem20, const int *face_bc,
                       const long *match_id);
void ora_mesh_free(ora_mesh *m);
/* last error text of ora_mesh_new (static buffer) */
const char *ora_error(void);

/* solution-point coordinates [3][E N^3] and quadrature weights w w w |J| */
void ora_solpts(const ora_mesh *m, double *xyz, double *wJ);
/* geometry export: |J| [E N^3], exact metrics at solution points
 * [E N^3][3 (direction d)][3 (component)], flux-point metrics
 * [E][3 d][(N+1) N^2][3] (curl form) */
void ora_geometry(const ora_mesh *m, double *jac, double *met_sol, double *met_flux);
/* face table export: nbr_e[E*6], nbr_f[E*6], nbr_p[E*6*N^2] (-1 on boundaries) */
void ora_faces(const ora_mesh *m, long *nbr_e, int *nbr_f, int *nbr_p);

void ora_residual(const ora_mesh *m, const ora_phys *ph, const double *Q, double *dQdt);
/* residual with an additional Cartesian flux sgs[v*3+c][E][N^3] at the
 * solution points (NULL: none), see the definition */
void ora_residual_sgs(const ora_mesh *m, const ora_phys *ph, const double *Q, const double *sgs,
                      double *dQdt);
/* BR1 gradients of the conserved variables at the solution points,
 * out[v*3+c][E][N^3] */
void ora_gradients(const ora_mesh *m, const ora_phys *ph, const double *Q, double *out);
void ora_rk3(const ora_mesh *m, const ora_phys *ph, double *Q, double dt, int nsteps);
/* five-stage fourth-order SSP Runge-Kutta (Spiteri & Ruuth 2002), Shu-Osher
 * form; ora_ssp54_table exports its alpha[5][5], beta[5][5] (row = stage) */
void ora_ssp54(const ora_mesh *m, const ora_phys *ph, double *Q, double dt, int nsteps);
void ora_ssp54_table(double alpha[25], double beta[25]);
/* angular momentum L (3) and diagonal moments of inertia I (3) over the
 * shell (Section 6), and the rigid-rotation correction u -= (L_i/I_i) x r */
void ora_angular_momentum(const ora_mesh *m, const double *Q, double out[6]);
void ora_am_correct(const ora_mesh *m, double *Q, double dOmega[3]);
/* sum over all solution points of w w w |J| Q_v, fixed serial order */
void ora_sums(const ora_mesh *m, const double *Q, double out[5]);

/* Polytropic adiabatic reference state (Section 4.2) with depth d = 1,
 * rho_c = p_c = 1 at mid-layer and the given gas constant; pars[4] receives
 * (chi_o, c, alpha, GM).  If noise != NULL an entropy perturbation
 * S' = amp * c_p * noise is applied at constant pressure. */
void ora_polytrope(const ora_mesh *m, double beta, double n_rho, double poly_n,
                   double gamma, double R_gas, const double *noise, double amp,
                   double *Q, double pars[4]);

#ifdef __cplusplus
}
#endif
#endif
