// Kernel launchers shared by the ABI layer and the kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "chorus_internal.hpp"
#include "physics.hpp"

namespace chorus {

// device geometry image views
struct Geo {
    const double *solgeo;   // [E][13][NP]
    const double *fluxgeo;  // [E][3][3][NFL]
    const int32_t *link;    // [E][6]
    const int32_t *info;    // [E][6]
    int64_t E;
    const double *rflux;    // [E][3][NFL] radius at the d-flux points
};

// stage combination of a Shu-Osher Runge-Kutta stage (mode 1):
//   Qout = c0 A + c1 (Q + c2 R)              (A read only when c0 != 0)
//   Tout = d0 B + d1 (Q + d2 R)  if Tout     (B read only when d0 != 0)
// with Q the stage input and R = dQ/dt(Q); c2, d2 include dt.  Each output
// may alias the array combined into it (A or B).  Mode 0 writes R to Qout.
struct StageArgs {
    const double *A;
    double *Qout;
    double *TQout;     // face traces of Qout (RK mode) or null
    double c0, c1, c2;
    const double *B;
    double *Tout;
    double d0, d1, d2;
    int mode;          // 0 residual, 1 RK stage
    const double *R0;  // background residual subtracted from R (balanced
                       // mode, added by the lift pass) or null
};

// learned subgrid closure (FP64 path, N = 3): model == null switches it off
struct ClosureArgs {
    const unsigned char *model;  // packed BF16 network image
    float *tau;                  // [15][E][NP] subgrid flux at the solution points (written by
                                 // the network-only flux pass, read by the flux pass)
};

hipError_t launch_trace(const Mesh &m, const Geo &G, const double *Q, double *TQ, hipStream_t s);
// learned subgrid flux at the solution points -> C.tau (order 3; traces from
// launch_trace_push in TQ)
hipError_t launch_closure_tau(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q, const double *TQ,
                              const ClosureArgs &C, hipStream_t s);
hipError_t launch_features(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q, const double *TQ,
                           float *X, hipStream_t s);
// FP64 stage split used by the solver (mailboxes indexed by the receiving
// element, face and point): the face traces of Q pushed to the neighbours;
// the flux pass (gradients, fluxes, divergence with the own-side face
// fluxes, source, [subgrid flux], the stage combination with this partial
// residual into sa.Qout / sa.Tout, own viscous face flux -> neighbour
// mailbox TV); the lift pass (neighbours' viscous halves added in place with
// the stage weights, traces of the new state -> sa.TQout)
hipError_t launch_trace_push(const Mesh &m, const Geo &G, const double *Q, double *TQ, hipStream_t s);
hipError_t launch_flux64(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q, const double *TQ,
                         double *TV, const StageArgs &sa, const ClosureArgs &C, hipStream_t s);
// closure: the flux pass ran with the learned subgrid flux (five mailbox
// components per point instead of four)
hipError_t launch_lift64(const Mesh &m, const Geo &G, const double *TV, const StageArgs &sa, bool closure,
                         hipStream_t s);

// closure training buffers for a mini-batch of nb samples (rows of 64 or 16)
struct TrainBufs {
    float *H1, *H2, *dZ1, *dZ2;  // [nb][64]: activations and pre-activation gradients
    float *dY;                   // [nb][16]
    float *lossv;                // [nb]
    float *part;                 // [ceil(nb/64)][6480] chunk partial gradients and losses
    int64_t n_mean;              // samples the loss is averaged over
};

struct AdamArgs {
    float lr, b1, b2, eps, inv_bc1, inv_bc2;  // inv_bc = 1 / (1 - beta^t)
};

// filter from order nf to order nc (nc <= 3, nf <= 6) on one hex mesh
struct FilterArgs {
    const double *Qf;        // [5][E][nf^3]
    const double *solgeo_f;  // fine geometry image: 1/|J| at index 9 of [E][13][nf^3]
    const double *solgeo_c;  // coarse geometry image
    double *Qbar;            // [5][E][nc^3]
    double *tau;             // [15][E][nc^3]
    int64_t E;
    int nf, nc;
    double gamma;
    double P[3][6];          // 1D projection: coarse point a <- fine point i
};

hipError_t launch_pack(const float *W, const float *norm, unsigned char *model, hipStream_t s);
hipError_t launch_train_grad(const float *X, const float *Y, const int32_t *idx, int64_t base, int nb,
                             const float *W, const TrainBufs &T, float *grad, float *loss, hipStream_t s);
// one training iteration: gradient of the mini-batch (as launch_train_grad)
// and the Adam update of the parameters
hipError_t launch_train_step(const float *X, const float *Y, const int32_t *idx, int64_t base, int nb, float *W,
                             float *m, float *v, const TrainBufs &T, const AdamArgs &a, float *loss, hipStream_t s);
hipError_t launch_filter(const FilterArgs &A, hipStream_t s);
// flag[0] = 1 if any of idx[0 .. count) lies outside [0, n)
hipError_t launch_check_idx(const int32_t *idx, int64_t count, int64_t n, int *flag, hipStream_t s);

hipError_t launch_sums(const double *Q, const double *solw, int64_t n, double *part, int nblocks, double *out,
                       hipStream_t s);
hipError_t launch_check(const double *Q, int64_t n, double gm1, int *flag, hipStream_t s);
// angular momentum and diagonal moments of inertia (6 rows of nblocks
// partials in part, results in out[6]); rigid-rotation removal
hipError_t launch_am_sums(const double *Q, const double *solw, const double *xsol, int64_t E, int NP, double *part,
                          int nblocks, double *out, hipStream_t s);
hipError_t launch_am_apply(double *Q, const double *xsol, int64_t E, int NP, const double dO[3], hipStream_t s);
hipError_t launch_clear_flag(int *flag, hipStream_t s);

// mixed-precision path: FP32 geometry, background arrays and FP64 Q0 copy
struct GeoM {
    const float *solgeo32;   // [E][13][NP]
    const float *fluxgeo32;  // [E][3][3][NFL]
    const int32_t *link;     // [E][6]
    const int32_t *info;     // [E][6]
    int64_t E;
    const float *bg;         // [E][2][NP]  rho0, E0
    const float *dbg;        // [E][6][2][NF2] neighbour minus own background face trace
    const float *gS0;        // [E][3][NFL] background entropy gradient along the flux metric
    const float *R0;         // [5][E][NP]  background residual
    const float *gbg;        // [E][3][NP]  grad rho0 at the solution points
    const double *Q0;        // [5][E][NP]  background state
    const float *rflux32;    // [E][3][NFL] radius at the d-flux points
};

// as StageArgs, on the perturbation P (mode 0 writes dQ/dt to Pout)
struct MixedStageArgs {
    const double *A;
    double *Pout;
    float *TQout;      // FP32 face traces of Pout (RK mode) or null
    double c0, c1, c2;
    const double *B;
    double *Tout;
    double d0, d1, d2;
    int mode;
};

hipError_t launch_pert_begin(const Mesh &m, const GeoM &g, const double *Q, double *Pq, float *TQ, hipStream_t s);
// stage split used by the solver: flux pass (gradients, fluxes, divergence
// with the own-side face fluxes, source; the stage combination with this
// partial residual into a.Pout / a.Tout; own viscous face flux -> neighbour
// mailbox TV), then lift pass (neighbours' viscous halves added in place to
// a.Pout / a.Tout with their stage weights; traces -> a.TQout)
hipError_t launch_flux_mixed(const Mesh &m, const GeoM &g, const PhysParams &P, const double *Pq, const float *TQ,
                             float *TV, const MixedStageArgs &a, hipStream_t s);
hipError_t launch_lift_mixed(const Mesh &m, const GeoM &g, const float *TV, const MixedStageArgs &a, hipStream_t s);
hipError_t launch_bg_setup(const Mesh &m, const Geo &G, const double *Q0, const double *TQ0, float *bg, float *dbg,
                           int *flag, hipStream_t s);
// background entropy gradient along the flux-point metric (out) and the
// gradient of rho0 at the solution points (gout [E][3][NP])
hipError_t launch_bg_entropy(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q0, const double *TQ,
                             float *out, float *gout, hipStream_t s);
hipError_t launch_pert_end(const double *Q0, const double *Pq, double *Q, int64_t n, hipStream_t s);
hipError_t launch_to_float(const double *a, float *b, int64_t n, hipStream_t s);

}  // namespace chorus
