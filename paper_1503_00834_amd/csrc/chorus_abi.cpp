// extern "C" entry points of the SD library (declared in include/chorus.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "launch.hpp"
#include "mlp_bf16.hpp"

namespace chorus {



static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

static int hip_fail(hipError_t e, const char *where) {
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return CHORUS_EHIP;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// workspace layout
struct WsLayout {
    size_t Qs, TQ0, TQ1, TV, part, sums, flag;
    size_t Q2, Q4;  // SSPRK(5,4): extra stage registers (FP64 path), 0 otherwise
    size_t tau;  // learned closure: subgrid flux [15][E][NP] FP32 (0 when off)
    // mixed-precision path
    size_t P0, P1, TQm, TVm, bg, dbg, gS0, R0, Q0, gbg;
    size_t P2, P4;  // SSPRK(5,4) on the perturbation
    size_t R64;     // FP64 background residual R(Q0) (balanced mode)
    bool mixed;
    size_t total;
};
static constexpr int kSumBlocks = 512;

// One layout for every mode (precision, closure, integrator), so that a
// workspace sized by chorus_workspace_bytes serves any call on the mesh.
static WsLayout ws_layout(const Mesh &m) {
    const int N = m.N, NP = N * N * N, NF2 = N * N;
    const int64_t E = m.E;
    WsLayout w;
    w.mixed = true;
    size_t off = 0;
    const size_t state = sizeof(double) * 5 * E * NP;
    w.Qs = off;   off = align256(off + state);
    w.TQ0 = off;  off = align256(off + sizeof(double) * E * 6 * 5 * NF2);
    w.TQ1 = off;  off = align256(off + sizeof(double) * E * 6 * 5 * NF2);
    w.TV = off;   off = align256(off + sizeof(double) * E * 6 * 5 * NF2);
    w.part = off; off = align256(off + sizeof(double) * 6 * kSumBlocks);
    w.sums = off; off = align256(off + sizeof(double) * 8);
    w.flag = off; off = align256(off + sizeof(int) * 4);
    w.tau = off;  off = align256(off + sizeof(float) * 15 * E * NP);
    w.Q2 = off;   off = align256(off + state);
    w.Q4 = off;   off = align256(off + state);
    w.P0 = off;   off = align256(off + state);
    w.P1 = off;   off = align256(off + state);
    w.P2 = off;   off = align256(off + state);
    w.P4 = off;   off = align256(off + state);
    w.TQm = off;  off = align256(off + sizeof(float) * E * 6 * 5 * NF2);
    w.TVm = off;  off = align256(off + sizeof(float) * E * 6 * 4 * NF2);  // momentum and energy only
    w.bg = off;   off = align256(off + sizeof(float) * E * 2 * NP);
    w.dbg = off;  off = align256(off + sizeof(float) * E * 6 * 2 * NF2);
    w.gS0 = off;  off = align256(off + sizeof(float) * E * 3 * (N + 1) * NF2);
    w.gbg = off;  off = align256(off + sizeof(float) * E * 3 * NP);
    w.R0 = off;   off = align256(off + sizeof(float) * 5 * E * NP);
    w.Q0 = off;   off = align256(off + state);
    w.R64 = off;  off = align256(off + state);
    w.total = off;
    return w;
}

static GeoM geom_of(const Mesh &m, const WsLayout &w, unsigned char *W) {
    const unsigned char *b = (const unsigned char *)m.dev_image;
    GeoM g;
    g.solgeo32 = (const float *)(b + m.layout.solgeo32);
    g.fluxgeo32 = (const float *)(b + m.layout.fluxgeo32);
    g.link = (const int32_t *)(b + m.layout.link);
    g.info = (const int32_t *)(b + m.layout.info);
    g.E = m.E;
    g.bg = (const float *)(W + w.bg);
    g.dbg = (const float *)(W + w.dbg);
    g.gS0 = (const float *)(W + w.gS0);
    g.gbg = (const float *)(W + w.gbg);
    g.R0 = (const float *)(W + w.R0);
    g.Q0 = (const double *)(W + w.Q0);
    g.rflux32 = (const float *)(b + m.layout.rflux32);
    return g;
}

static Geo geo_of(const Mesh &m, unsigned char *W) {
    const unsigned char *b = (const unsigned char *)m.dev_image;
    Geo g;
    g.solgeo = (const double *)(b + m.layout.solgeo);
    g.fluxgeo = (const double *)(b + m.layout.fluxgeo);
    g.link = (const int32_t *)(b + m.layout.link);
    g.info = (const int32_t *)(b + m.layout.info);
    g.E = m.E;
    g.rflux = (const double *)(b + m.layout.rflux);
    return g;
}

static int check_phys(const chorus_physics *p) {
    if (!p) {
        set_error("physics is null");
        return CHORUS_EINVAL;
    }
    if (!(p->gamma > 1.0) || !(p->R_gas > 0.0) || p->nu < 0.0 || p->kappa < 0.0 || p->kappa_r < 0.0) {
        set_error("physics: need gamma > 1, R_gas > 0 and non-negative diffusivities");
        return CHORUS_EINVAL;
    }
    if (p->precision != CHORUS_FP64 && p->precision != CHORUS_MIXED) {
        set_error("physics: unknown precision");
        return CHORUS_EINVAL;
    }
    if (p->integrator != CHORUS_SSPRK3 && p->integrator != CHORUS_SSPRK54) {
        set_error("physics: unknown integrator");
        return CHORUS_EINVAL;
    }
    if (p->closure != CHORUS_CLOSURE_NONE && p->closure != CHORUS_CLOSURE_MLP) {
        set_error("physics: unknown closure");
        return CHORUS_EINVAL;
    }
    if (p->closure == CHORUS_CLOSURE_MLP) {
        if (!p->closure_model) {
            set_error("closure: no network image (closure_model is null)");
            return CHORUS_EINVAL;
        }
        if (p->precision != CHORUS_FP64) {
            set_error("closure: only the FP64 precision path carries the learned closure");
            return CHORUS_ENOTSUP;
        }
    }
    return CHORUS_OK;
}

static int check_closure_order(const Mesh &m, const chorus_physics *p) {
    if (p->closure == CHORUS_CLOSURE_MLP && m.N != 3) {
        set_error("closure: the learned closure runs at order 3 only");
        return CHORUS_ENOTSUP;
    }
    return CHORUS_OK;
}

static ClosureArgs closure_of(const chorus_physics *p, const WsLayout &w, unsigned char *W) {
    ClosureArgs C{nullptr, nullptr};
    if (p->closure == CHORUS_CLOSURE_MLP) {
        C.model = (const unsigned char *)p->closure_model;
        C.tau = (float *)(W + w.tau);
    }
    return C;
}

// the mixed path needs a registered background computed with the same
// inviscid physics, in the same workspace, on a mesh without state faces
static int check_mixed(const Mesh &m, const chorus_physics *p, const void *ws) {
    if (!m.bg_ready || m.bg_ws != ws) {
        set_error("mixed precision needs chorus_set_background with this workspace first");
        return CHORUS_ESTATE;
    }
    const chorus_physics &b = m.bg_phys;
    if (b.gamma != p->gamma || b.R_gas != p->R_gas || b.GM != p->GM || b.omega != p->omega || b.nu != p->nu ||
        b.kappa != p->kappa || b.kappa_r != p->kappa_r || b.kappa_r1 != p->kappa_r1 ||
        b.kappa_r2 != p->kappa_r2 || b.T_top != p->T_top || b.F_bottom != p->F_bottom ||
        (b.flags & CHORUS_BALANCED) != (p->flags & CHORUS_BALANCED)) {
        set_error("the physics (and the balanced flag) must match the one passed to chorus_set_background");
        return CHORUS_ESTATE;
    }
    return CHORUS_OK;
}

static PhysParams params_of(const chorus_physics *p) {
    PhysParams P;
    P.gamma = p->gamma;
    P.R_gas = p->R_gas;
    P.GM = p->GM;
    P.omega = p->omega;
    P.nu = p->nu;
    P.kappa = p->kappa;
    P.kappa_r = p->kappa_r;
    P.T_top = p->T_top;
    P.F_bottom = p->F_bottom;
    for (int v = 0; v < 5; ++v) P.bc_state[v] = p->bc_state[v];
    P.cp = p->gamma * p->R_gas / (p->gamma - 1.0);
    P.kappa_r1 = p->kappa_r1;
    P.kappa_r2 = p->kappa_r2;
    return P;
}

// the radiative diffusivity kappa_r(r) (a quadratic) must not be negative
// at any flux-point radius of the mesh: checked at both ends of the radius
// range and at the vertex when it lies inside
static int check_kappa_r(const Mesh &m, const chorus_physics *p) {
    if (!std::isfinite(p->kappa_r1) || !std::isfinite(p->kappa_r2)) {
        set_error("physics: kappa_r1 and kappa_r2 must be finite");
        return CHORUS_EINVAL;
    }
    if (p->kappa_r1 == 0.0 && p->kappa_r2 == 0.0) return CHORUS_OK;
    const PhysParams P = params_of(p);
    double lo = std::min(kappa_r_at(P, m.rflux_min), kappa_r_at(P, m.rflux_max));
    if (p->kappa_r2 != 0.0) {
        const double rv = -p->kappa_r1 / (2.0 * p->kappa_r2);
        if (rv > m.rflux_min && rv < m.rflux_max) lo = std::min(lo, kappa_r_at(P, rv));
    }
    if (!(lo >= 0.0)) {
        set_error("physics: kappa_r(r) = kappa_r + kappa_r1 r + kappa_r2 r^2 is negative on the mesh");
        return CHORUS_EINVAL;
    }
    return CHORUS_OK;
}

static int check_ready(const Mesh *m) {
    if (!m) {
        set_error("mesh is null");
        return CHORUS_EINVAL;
    }
    if (!m->dev_image) {
        set_error("no geometry uploaded (chorus_mesh_upload)");
        return CHORUS_ESTATE;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
        set_error("current device differs from the device of the uploaded geometry");
        return CHORUS_ESTATE;
    }
    return CHORUS_OK;
}

static int finite_check_flag(const Mesh &m, const PhysParams &P, const double *Q, int *flag, hipStream_t s) {
    hipError_t e = launch_check(Q, m.E * m.N * m.N * m.N, P.gamma - 1.0, flag, s);
    if (e != hipSuccess) return hip_fail(e, "finite check");
    int h = 0;
    e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "finite check");
    if (h) {
        set_error("non-finite or non-positive density/pressure in the state");
        return CHORUS_ENONFINITE;
    }
    return CHORUS_OK;
}

static int finite_check(const Mesh &m, const PhysParams &P, const double *Q, const WsLayout &w,
                        unsigned char *ws, hipStream_t s) {
    return finite_check_flag(m, P, Q, (int *)(ws + w.flag), s);
}

// ---------------------------------------------------------------------------
// opt-in kernel timing: event pairs recorded on the launch stream
// ---------------------------------------------------------------------------
struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
};
static bool g_timing = false;
static std::vector<TimedLaunch> g_launches;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t pooled_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t ev = g_event_pool.back();
        g_event_pool.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    return ev;
}

template <typename F>
static hipError_t timed(int kind, hipStream_t s, F &&launch) {
    if (!g_timing) return launch();
    TimedLaunch t{kind, pooled_event(), pooled_event()};
    if (!t.start || !t.stop) return launch();
    hipError_t e = hipEventRecord(t.start, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(t.stop, s);
    g_launches.push_back(t);
    return e;
}

}  // namespace chorus

using namespace chorus;

extern "C" {

const char *chorus_strerror(int status) {
    switch (status) {
        case CHORUS_OK: return "ok";
        case CHORUS_EINVAL: return "invalid argument";
        case CHORUS_EMESH: return "invalid mesh";
        case CHORUS_ENOTSUP: return "not supported";
        case CHORUS_EHIP: return "HIP runtime error";
        case CHORUS_ENONFINITE: return "non-finite state";
        case CHORUS_ESTATE: return "invalid call order";
        default: return "unknown status";
    }
}

int chorus_last_error(char *buf, size_t len) {
    if (!buf || len == 0) return CHORUS_EINVAL;
    std::strncpy(buf, g_last_error.c_str(), len - 1);
    buf[len - 1] = 0;
    return CHORUS_OK;
}

static int create_common(Mesh *m, chorus_mesh_t *out) {
    int rc = finish_mesh(*m);
    if (rc) {
        delete m;
        return rc;
    }
    *out = reinterpret_cast<chorus_mesh_t>(m);
    return CHORUS_OK;
}

int chorus_mesh_create(const chorus_shell_desc *desc, chorus_mesh_t *out) {
    if (!desc || !out) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    if (desc->order < 2 || desc->order > kMaxOrder) {
        set_error("order must be in [2, 6]");
        return CHORUS_EINVAL;
    }
    Mesh *m = new (std::nothrow) Mesh();
    if (!m) return CHORUS_EINVAL;
    try {
        int rc = build_shell(*desc, *m);
        if (rc) {
            delete m;
            return rc;
        }
        return create_common(m, out);
    } catch (const std::exception &ex) {
        set_error(std::string("mesh create: ") + ex.what());
        delete m;
        return CHORUS_EINVAL;
    }
}

int chorus_mesh_create_hex20(const chorus_hex20_desc *desc, chorus_mesh_t *out) {
    if (!desc || !out) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    if (desc->order < 2 || desc->order > kMaxOrder) {
        set_error("order must be in [2, 6]");
        return CHORUS_EINVAL;
    }
    Mesh *m = new (std::nothrow) Mesh();
    if (!m) return CHORUS_EINVAL;
    try {
        int rc = build_from_hex20(*desc, *m);
        if (rc) {
            delete m;
            return rc;
        }
        return create_common(m, out);
    } catch (const std::exception &ex) {
        set_error(std::string("mesh create: ") + ex.what());
        delete m;
        return CHORUS_EINVAL;
    }
}

int chorus_mesh_destroy(chorus_mesh_t mesh) {
    delete reinterpret_cast<Mesh *>(mesh);
    return CHORUS_OK;
}

int chorus_mesh_query(chorus_mesh_t mesh, int64_t *n_elems, int32_t *order, int64_t *n_solpts,
                      int64_t *n_faces, int64_t *n_wall_faces, size_t *device_bytes) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m) {
        set_error("mesh is null");
        return CHORUS_EINVAL;
    }
    if (n_elems) *n_elems = m->E;
    if (order) *order = m->N;
    if (n_solpts) *n_solpts = m->E * m->N * m->N * m->N;
    if (n_faces) *n_faces = m->n_faces;
    if (n_wall_faces) *n_wall_faces = m->n_wall_faces;
    if (device_bytes) *device_bytes = m->layout.total;
    return CHORUS_OK;
}

int chorus_mesh_nodes(chorus_mesh_t mesh, int64_t *n_nodes, double *xyz, int64_t *elem20, int32_t *face_bc) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m) {
        set_error("mesh is null");
        return CHORUS_EINVAL;
    }
    if (n_nodes) *n_nodes = m->n_nodes();
    if (xyz) std::memcpy(xyz, m->xyz.data(), sizeof(double) * m->xyz.size());
    if (elem20) std::memcpy(elem20, m->elem20.data(), sizeof(int64_t) * m->elem20.size());
    if (face_bc) std::memcpy(face_bc, m->face_bc.data(), sizeof(int32_t) * m->face_bc.size());
    return CHORUS_OK;
}

int chorus_mesh_solpts(chorus_mesh_t mesh, double *xyz_host, double *wJ_host) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m) {
        set_error("mesh is null");
        return CHORUS_EINVAL;
    }
    const int N = m->N, NP = N * N * N;
    const int64_t n = m->E * NP;
    for (int64_t e = 0; e < m->E; ++e)
        for (int p = 0; p < NP; ++p) {
            const int64_t g = e * NP + p;
            if (xyz_host)
                for (int c = 0; c < 3; ++c) xyz_host[c * n + g] = m->xsol[g * 3 + c];
            if (wJ_host) {
                const int i = p % N, j = (p / N) % N, k = p / (N * N);
                wJ_host[g] = m->basis.w[i] * m->basis.w[j] * m->basis.w[k] * m->jac[g];
            }
        }
    return CHORUS_OK;
}

int chorus_mesh_geometry(chorus_mesh_t mesh, double *jac, double *met_sol, double *met_flux) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m) {
        set_error("mesh is null");
        return CHORUS_EINVAL;
    }
    if (jac) std::memcpy(jac, m->jac.data(), sizeof(double) * m->jac.size());
    if (met_sol) std::memcpy(met_sol, m->met.data(), sizeof(double) * m->met.size());
    if (met_flux) std::memcpy(met_flux, m->metf.data(), sizeof(double) * m->metf.size());
    return CHORUS_OK;
}

int chorus_mesh_face_table(chorus_mesh_t mesh, int32_t *nbr_elem, int32_t *nbr_face, int32_t *orient) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m) {
        set_error("mesh is null");
        return CHORUS_EINVAL;
    }
    for (int64_t i = 0; i < m->E * 6; ++i) {
        if (nbr_elem) nbr_elem[i] = m->links[i].nbr_elem;
        if (nbr_face) nbr_face[i] = m->links[i].nbr_face;
        if (orient) orient[i] = m->links[i].orient;
    }
    return CHORUS_OK;
}

int chorus_mesh_upload(chorus_mesh_t mesh, void *dev_buf, size_t bytes, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m || !dev_buf) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    if (bytes < m->layout.total) {
        set_error("device buffer smaller than the geometry image");
        return CHORUS_EINVAL;
    }
    if (((uintptr_t)dev_buf) & 255) {
        set_error("device buffer must be 256-byte aligned");
        return CHORUS_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(dev_buf, m->image.data(), m->layout.total, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "upload");
    int dev = -1;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "upload");
    m->dev_image = dev_buf;
    m->device = dev;
    return CHORUS_OK;
}

int chorus_workspace_bytes(chorus_mesh_t mesh, const chorus_physics *phys, size_t *bytes) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m || !bytes) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    *bytes = ws_layout(*m).total;
    return CHORUS_OK;
}

int chorus_init_polytrope(chorus_mesh_t mesh, double beta, double n_rho, double poly_n, double gamma,
                          double R_gas, const double *noise, double amp, double *Q_host, double pars[4]) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m || !Q_host) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    if (!(beta > 0.0 && beta < 1.0) || !(poly_n > 0.0) || !(gamma > 1.0) || !(R_gas > 0.0)) {
        set_error("polytrope: need 0 < beta < 1, poly_n > 0, gamma > 1, R_gas > 0");
        return CHORUS_EINVAL;
    }
    // Section 4.2 with d = 1, rho_c = p_c = 1: chi = c + alpha d / r
    const double ebn = std::exp(n_rho / poly_n);
    const double chi_o = (beta + 1.0) / (beta * ebn + 1.0);
    const double om = 1.0 - beta;
    const double c = (2.0 * chi_o - beta - 1.0) / om;
    const double alpha = (1.0 + beta) * (1.0 - chi_o) / (om * om);
    const double GM = (poly_n + 1.0) * alpha;  // p_c/rho_c = GM / ((n+1) alpha d)
    const int64_t n = m->E * m->N * m->N * m->N;
    for (int64_t g = 0; g < n; ++g) {
        const double *x = &m->xsol[g * 3];
        const double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double chi = c + alpha / r;
        double rho = std::pow(chi, poly_n);
        const double p = rho * chi;
        if (noise) rho = rho * std::exp(-amp * noise[g]);
        Q_host[g] = rho;
        Q_host[n + g] = 0.0;
        Q_host[2 * n + g] = 0.0;
        Q_host[3 * n + g] = 0.0;
        Q_host[4 * n + g] = p / (gamma - 1.0);
    }
    if (pars) {
        pars[0] = chi_o;
        pars[1] = c;
        pars[2] = alpha;
        pars[3] = GM;
    }
    return CHORUS_OK;
}

// Almost-flux-balance background (Section 4.3): from the polytrope
// (rho_a, p_a, T_a = p_a / (R rho_a)) the target entropy gradient
//   Gamma(r) = -(L / (4 pi r^2) + rho_a c_p kappa_r(r) dT_a/dr) / (rho_a T_a kappa),
// the gradient at which the diffusive flux f = -kappa rho T grad S -
// kappa_r rho c_p grad T (Section 2) carries the luminosity L outward (the
// printed equation lacks this overall sign; with it L > 0 gives the
// superadiabatic dS/dr < 0 the section asks for)
// and then the state equations
//   dp0/dr = -rho0 g,  d rho0/dr = -rho0 (Gamma / c_p + g rho0 / (gamma p0)),
// g = GM / r^2, integrated from the polytrope's mid-layer point (chi = 1,
// rho0 = p0 = 1) out to both walls with classical RK4 on a fine uniform
// grid; values at the solution points by cubic Hermite interpolation with
// the ODE's own derivatives.
namespace {
struct AfbModel {
    double c, alpha, n, gamma, R, cp, GM, L, kappa, kappa_r, kappa_r1, kappa_r2;
    double chi(double r) const { return c + alpha / r; }
    double gamma_target(double r) const {
        const double ch = chi(r);
        const double rho_a = std::pow(ch, n), T_a = ch / R;
        const double dTa = -alpha / (r * r) / R;
        const double kr = kappa_r + r * (kappa_r1 + r * kappa_r2);
        return -(L / (4.0 * M_PI * r * r) + rho_a * cp * kr * dTa) / (rho_a * T_a * kappa);
    }
    // d(rho, p)/dr
    void rhs(double r, const double y[2], double dy[2]) const {
        const double g = GM / (r * r);
        dy[1] = -y[0] * g;
        dy[0] = -y[0] * (gamma_target(r) / cp + g * y[0] / (gamma * y[1]));
    }
};

static void rk4_table(const AfbModel &M, double r0, double r1, int steps, std::vector<double> &rr,
                      std::vector<double> &yy) {
    const double h = (r1 - r0) / steps;
    double y[2] = {1.0, 1.0};
    rr.assign(steps + 1, 0.0);
    yy.assign(2 * (steps + 1), 0.0);
    rr[0] = r0;
    yy[0] = y[0];
    yy[1] = y[1];
    for (int k = 0; k < steps; ++k) {
        const double r = r0 + k * h;
        double k1[2], k2[2], k3[2], k4[2], t[2];
        M.rhs(r, y, k1);
        for (int i = 0; i < 2; ++i) t[i] = y[i] + 0.5 * h * k1[i];
        M.rhs(r + 0.5 * h, t, k2);
        for (int i = 0; i < 2; ++i) t[i] = y[i] + 0.5 * h * k2[i];
        M.rhs(r + 0.5 * h, t, k3);
        for (int i = 0; i < 2; ++i) t[i] = y[i] + h * k3[i];
        M.rhs(r + h, t, k4);
        for (int i = 0; i < 2; ++i) y[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        rr[k + 1] = r0 + (k + 1) * h;
        yy[2 * (k + 1)] = y[0];
        yy[2 * (k + 1) + 1] = y[1];
    }
}

// cubic Hermite interpolation of the table at r (r within the table; the
// table step may be negative)
static void hermite(const AfbModel &M, const std::vector<double> &rr, const std::vector<double> &yy, double r,
                    double out[2]) {
    const int n = (int)rr.size() - 1;
    const double h = rr[1] - rr[0];
    int k = (int)std::floor((r - rr[0]) / h);
    if (k < 0) k = 0;
    if (k >= n) k = n - 1;
    const double s = (r - rr[k]) / h;
    double d0[2], d1[2];
    M.rhs(rr[k], &yy[2 * k], d0);
    M.rhs(rr[k + 1], &yy[2 * (k + 1)], d1);
    const double h00 = (1 + 2 * s) * (1 - s) * (1 - s), h10 = s * (1 - s) * (1 - s);
    const double h01 = s * s * (3 - 2 * s), h11 = s * s * (s - 1);
    for (int i = 0; i < 2; ++i)
        out[i] = h00 * yy[2 * k + i] + h10 * h * d0[i] + h01 * yy[2 * (k + 1) + i] + h11 * h * d1[i];
}
}  // namespace

int chorus_init_afb(chorus_mesh_t mesh, const chorus_afb_desc *desc, double *Q_host, double pars[6]) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m || !desc || !Q_host) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    const chorus_afb_desc &d = *desc;
    if (!(d.beta > 0.0 && d.beta < 1.0) || !(d.poly_n > 0.0) || !(d.gamma > 1.0) || !(d.R_gas > 0.0) ||
        !(d.kappa > 0.0) || d.kappa_r < 0.0 || d.luminosity < 0.0 || !std::isfinite(d.kappa_r1) ||
        !std::isfinite(d.kappa_r2)) {
        set_error("afb: need 0 < beta < 1, poly_n > 0, gamma > 1, R_gas > 0, kappa > 0, kappa_r >= 0, L >= 0");
        return CHORUS_EINVAL;
    }
    // the polytrope of Section 4.2 with depth 1 and rho_c = p_c = 1
    const double ebn = std::exp(d.n_rho / d.poly_n);
    const double chi_o = (d.beta + 1.0) / (d.beta * ebn + 1.0);
    const double om = 1.0 - d.beta;
    AfbModel M;
    M.c = (2.0 * chi_o - d.beta - 1.0) / om;
    M.alpha = (1.0 + d.beta) * (1.0 - chi_o) / (om * om);
    M.n = d.poly_n;
    M.gamma = d.gamma;
    M.R = d.R_gas;
    M.cp = d.gamma * d.R_gas / (d.gamma - 1.0);
    M.GM = (d.poly_n + 1.0) * M.alpha;  // p_c / rho_c = 1 = GM / ((n+1) alpha d)
    M.L = d.luminosity;
    M.kappa = d.kappa;
    M.kappa_r = d.kappa_r;
    M.kappa_r1 = d.kappa_r1;
    M.kappa_r2 = d.kappa_r2;
    const double ri = d.beta / om, ro = 1.0 / om, rc = M.alpha / (1.0 - M.c);
    const int steps = 20000;
    std::vector<double> r_out, y_out, r_in, y_in;
    rk4_table(M, rc, ro, steps, r_out, y_out);
    rk4_table(M, rc, ri, steps, r_in, y_in);
    const int64_t n = m->E * m->N * m->N * m->N;
    for (int64_t g = 0; g < n; ++g) {
        const double *x = &m->xsol[g * 3];
        const double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        double y[2];
        // both tables interpolate with a signed step (the inward one runs
        // from rc down to ri)
        if (r >= rc) hermite(M, r_out, y_out, r, y);
        else hermite(M, r_in, y_in, r, y);
        // rho at fixed p for the entropy perturbation S' = amp c_p noise
        Q_host[g] = d.noise ? y[0] * std::exp(-d.amp * d.noise[g]) : y[0];
        Q_host[n + g] = 0.0;
        Q_host[2 * n + g] = 0.0;
        Q_host[3 * n + g] = 0.0;
        Q_host[4 * n + g] = y[1] / (d.gamma - 1.0);
    }
    if (pars) {
        double yo[2];
        hermite(M, r_out, y_out, ro, yo);
        pars[0] = chi_o;
        pars[1] = M.c;
        pars[2] = M.alpha;
        pars[3] = M.GM;
        pars[4] = yo[1] / (yo[0] * d.R_gas);                  // T0 at the outer wall
        pars[5] = d.luminosity / (4.0 * M_PI * ri * ri);       // bottom flux L / (4 pi R_i^2)
    }
    return CHORUS_OK;
}

// the printed radiative-diffusivity polynomial of the solar benchmark
// (Section 7.4): coefficients of w = r / 1e10 cm, and Table 2's shell depth
static const double kSolarKr[3] = {1.5600975e8, -4.5631718e7, 3.3370368e6};
static const double kSolarDepthCm = 1.74e10;

int chorus_solar_kappa_r(double beta, double n_rho, double poly_n, double gamma, double R_gas, double luminosity,
                         double depth_cm, double out[3]) {
    if (!out || !(beta > 0.0 && beta < 1.0) || !(poly_n > 0.0) || !(gamma > 1.0) || !(R_gas > 0.0) ||
        !(luminosity >= 0.0) || !std::isfinite(n_rho) || !std::isfinite(depth_cm)) {
        set_error("solar_kappa_r: need 0 < beta < 1, poly_n > 0, gamma > 1, R_gas > 0, L >= 0, out");
        return CHORUS_EINVAL;
    }
    const double s = (depth_cm > 0.0 ? depth_cm : kSolarDepthCm) * 1e-10;  // w per unit r
    // the polytrope of Section 4.2 with depth 1, rho_c = p_c = 1
    const double om = 1.0 - beta;
    const double chi_o = (beta + 1.0) / (beta * std::exp(n_rho / poly_n) + 1.0);
    const double c = (2.0 * chi_o - beta - 1.0) / om;
    const double alpha = (1.0 + beta) * (1.0 - chi_o) / (om * om);
    const double ri = beta / om, w = ri * s;
    const double rho_i = std::pow(c + alpha / ri, poly_n);
    const double cp = gamma * R_gas / (gamma - 1.0);
    // -lambda poly(w_i) rho_a c_p dT_a/dr = L / (4 pi R_i^2) at the inner
    // wall, with dT_a/dr = -alpha / (R_gas r^2)
    const double poly = kSolarKr[0] + kSolarKr[1] * w + kSolarKr[2] * w * w;
    const double lam = luminosity * R_gas / (4.0 * M_PI * poly * rho_i * cp * alpha);
    out[0] = lam * kSolarKr[0];
    out[1] = lam * kSolarKr[1] * s;
    out[2] = lam * kSolarKr[2] * s * s;
    return CHORUS_OK;
}

int chorus_set_background(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q0_dev, void *ws,
                          void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    rc = check_phys(phys);
    if (rc) return rc;
    rc = check_kappa_r(*m, phys);
    if (rc) return rc;
    if (!Q0_dev || !ws) {
        set_error("null device pointer");
        return CHORUS_EINVAL;
    }
    for (int32_t b : m->face_bc)
        if (b == CHORUS_BC_STATE) {
            set_error("mixed precision supports interior and wall faces only");
            return CHORUS_ENOTSUP;
        }
    // the workspace's background arrays are rewritten from here on: until
    // this call succeeds no background is registered (a failed call leaves
    // none, not the previous one half overwritten)
    m->bg_ready = false;
    m->bg_ws = nullptr;
    const WsLayout w = ws_layout(*m);
    unsigned char *W = (unsigned char *)ws;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = m->E * m->N * m->N * m->N;
    double *Q0 = (double *)(W + w.Q0);
    int *flag = (int *)(W + w.flag);
    hipError_t e = hipMemcpyAsync(Q0, Q0_dev, sizeof(double) * 5 * n, hipMemcpyDeviceToDevice, s);
    chorus_physics p64 = *phys;
    p64.precision = CHORUS_FP64;
    const PhysParams P = params_of(&p64);
    const Geo G = geo_of(*m, (unsigned char *)ws);
    double *R0d = (double *)(W + w.Qs), *TQ = (double *)(W + w.TQ0), *TV = (double *)(W + w.TV);
    if (e == hipSuccess) e = launch_clear_flag(flag, s);
    if (e == hipSuccess) e = launch_trace(*m, G, Q0, TQ, s);
    if (e == hipSuccess) e = launch_bg_setup(*m, G, Q0, TQ, (float *)(W + w.bg), (float *)(W + w.dbg), flag, s);
    if (e == hipSuccess) e = launch_bg_entropy(*m, G, P, Q0, TQ, (float *)(W + w.gS0), (float *)(W + w.gbg), s);
    // R0 = R(Q0), the complete FP64 residual of the background (the flux and
    // lift passes read receiver-indexed traces: a second trace buffer)
    const ClosureArgs C0{nullptr, nullptr};
    double *TQp = (double *)(W + w.TQ1);
    StageArgs sa{nullptr, R0d, nullptr, 0.0, 1.0, 0.0, nullptr, nullptr, 0.0, 0.0, 0.0, 0};
    if (e == hipSuccess) e = launch_trace_push(*m, G, Q0, TQp, s);
    if (e == hipSuccess) e = launch_flux64(*m, G, P, Q0, TQp, TV, sa, C0, s);
    if (e == hipSuccess) e = launch_lift64(*m, G, TV, sa, false, s);
    if (e == hipSuccess) e = hipMemcpyAsync(W + w.R64, R0d, sizeof(double) * 5 * n, hipMemcpyDeviceToDevice, s);
    // the mixed path adds R0 to its FP32 perturbation residual; in balanced
    // mode R(Q) - R(Q0) is the perturbation residual alone
    if (e == hipSuccess) {
        if (phys->flags & CHORUS_BALANCED) e = hipMemsetAsync(W + w.R0, 0, sizeof(float) * 5 * n, s);
        else e = launch_to_float(R0d, (float *)(W + w.R0), 5 * n, s);
    }
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "set_background");
    if (h) {
        set_error("background state must be at rest (zero momentum)");
        return CHORUS_EINVAL;
    }
    m->bg_ready = true;
    m->bg_ws = ws;
    m->bg_phys = *phys;
    return CHORUS_OK;
}

int chorus_sd_residual(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q_dev, double *dQdt_dev,
                       void *ws, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    rc = check_phys(phys);
    if (rc) return rc;
    rc = check_kappa_r(*m, phys);
    if (rc) return rc;
    if (!Q_dev || !dQdt_dev || !ws) {
        set_error("null device pointer");
        return CHORUS_EINVAL;
    }
    rc = check_closure_order(*m, phys);
    if (rc) return rc;
    const bool mixed = phys->precision == CHORUS_MIXED;
    const WsLayout w = ws_layout(*m);
    unsigned char *W = (unsigned char *)ws;
    const PhysParams P = params_of(phys);
    const ClosureArgs C = closure_of(phys, w, W);
    hipStream_t s = (hipStream_t)stream;
    if (mixed) {
        rc = check_mixed(*m, phys, ws);
        if (rc) return rc;
        const GeoM g = geom_of(*m, w, W);
        double *P0 = (double *)(W + w.P0);
        float *TQm = (float *)(W + w.TQm), *TVm = (float *)(W + w.TVm);
        hipError_t e = timed(0, s, [&] { return launch_pert_begin(*m, g, Q_dev, P0, TQm, s); });
        MixedStageArgs a{nullptr, dQdt_dev, nullptr, 0.0, 1.0, 0.0, nullptr, nullptr, 0.0, 0.0, 0.0, 0};
        if (e == hipSuccess) e = timed(1, s, [&] { return launch_flux_mixed(*m, g, P, P0, TQm, TVm, a, s); });
        if (e == hipSuccess) e = timed(2, s, [&] { return launch_lift_mixed(*m, g, TVm, a, s); });
        if (e != hipSuccess) return hip_fail(e, "sd_residual (mixed)");
        if (phys->flags & CHORUS_CHECK_FINITE) return finite_check(*m, P, Q_dev, w, W, s);
        return CHORUS_OK;
    }
    double *TQ = (double *)(W + w.TQ0), *TV = (double *)(W + w.TV);
    const Geo G = geo_of(*m, (unsigned char *)ws);
    StageArgs sa{nullptr, dQdt_dev, nullptr, 0.0, 1.0, 0.0, nullptr, nullptr, 0.0, 0.0, 0.0, 0, nullptr};
    if (phys->flags & CHORUS_BALANCED) {
        rc = check_mixed(*m, phys, ws);
        if (rc) return rc;
        sa.R0 = (const double *)(W + w.R64);
    }
    hipError_t e = timed(0, s, [&] { return launch_trace_push(*m, G, Q_dev, TQ, s); });
    if (e == hipSuccess) e = timed(1, s, [&] { return launch_flux64(*m, G, P, Q_dev, TQ, TV, sa, C, s); });
    if (e == hipSuccess) e = timed(2, s, [&] { return launch_lift64(*m, G, TV, sa, C.model != nullptr, s); });
    if (e != hipSuccess) return hip_fail(e, "sd_residual");
    if (phys->flags & CHORUS_CHECK_FINITE) return finite_check(*m, P, Q_dev, w, W, s);
    return CHORUS_OK;
}

// One Runge-Kutta stage in Shu-Osher form on the stage registers
// (0: the step-start state, updated in place by the last stage; 1: the
// running stage; 2, 3: extra registers of SSPRK(5,4)): reads register `in`,
// writes `out` = c0 [a] + c1 (in + c2 dt R(in)) and, if tout >= 0,
// [tout] = d0 [b] + d1 (in + d2 dt R(in)).
struct StagePlan {
    int in, out, a, b, tout;
    double c0, c1, c2, d0, d1, d2;
};

// Shu-Osher SSP-RK3
static const StagePlan kSSPRK3[3] = {
    {0, 1, -1, -1, -1, 0.0, 1.0, 1.0, 0, 0, 0},
    {1, 1, 0, -1, -1, 0.75, 0.25, 1.0, 0, 0, 0},
    {1, 0, 0, -1, -1, 1.0 / 3.0, 2.0 / 3.0, 1.0, 0, 0, 0},
};

// SSPRK(5,4) of Spiteri & Ruuth (2002): u_i = sum_k alpha_ik u_k + beta_ik dt
// L(u_k) with the published coefficients; the last stage needs u2, u3 and
// L(u3), which stage 4 folds into register 2 (T = a52 u2 + a53 u3 + b53 dt
// L(u3)), so u^{n+1} = T + a54 u4 + b54 dt L(u4)
static const double kA10 = 1.0, kB10 = 0.391752226571890;
static const double kA20 = 0.444370493651235, kA21 = 0.555629506348765, kB21 = 0.368410593050371;
static const double kA30 = 0.620101851488403, kA32 = 0.379898148511597, kB32 = 0.251891774271694;
static const double kA40 = 0.178079954393132, kA43 = 0.821920045606868, kB43 = 0.544974750228521;
static const double kA52 = 0.517231671970585, kA53 = 0.096059710526147, kB53 = 0.063692468666290;
static const double kA54 = 0.386708617503269, kB54 = 0.226007483236906;
static const StagePlan kSSPRK54[5] = {
    {0, 1, -1, -1, -1, 0.0, kA10, kB10 / kA10, 0, 0, 0},
    {1, 2, 0, -1, -1, kA20, kA21, kB21 / kA21, 0, 0, 0},
    {2, 1, 0, -1, -1, kA30, kA32, kB32 / kA32, 0, 0, 0},
    {1, 3, 0, 2, 2, kA40, kA43, kB43 / kA43, kA52, kA53, kB53 / kA53},
    {3, 0, 2, -1, -1, 1.0, kA54, kB54 / kA54, 0, 0, 0},
};

// buffers of the FP64 step: stage registers (Q itself is register 0),
// the receiver-indexed trace and viscous mailboxes and the finite-check flag
struct Fp64Bufs {
    double *Qs, *Q2, *Q4;  // Q2, Q4: SSPRK(5,4) only
    double *TQ, *TV;       // [E][6][5][N^2]
    int *flag;
    const double *R0;      // subtracted background residual (balanced) or null
};

// n steps of the FP64 path on explicit buffers (no allocation); kernel
// timing only when allowed and switched on
static int rk_fp64(const Mesh &m, const chorus_physics *phys, const ClosureArgs &C, double *Q_dev, double dt,
                   int32_t n_steps, const Fp64Bufs &b, hipStream_t s, bool allow_timing) {
    const bool rk54 = phys->integrator == CHORUS_SSPRK54;
    const StagePlan *plan = rk54 ? kSSPRK54 : kSSPRK3;
    const int nst = rk54 ? 5 : 3;
    const PhysParams P = params_of(phys);
    double *reg[4] = {Q_dev, b.Qs, b.Q2, b.Q4};
    // the flux pass reads the trace mailbox and writes the viscous one; the
    // lift pass reads the viscous mailbox and rewrites the traces (kernel
    // order separates every read from the next write)
    const Geo G = geo_of(m, nullptr);
    auto run = [&](int kind, auto &&launch) { return allow_timing ? timed(kind, s, launch) : launch(); };
    hipError_t e = run(0, [&] { return launch_trace_push(m, G, Q_dev, b.TQ, s); });
    for (int st = 0; st < n_steps && e == hipSuccess; ++st) {
        for (int k = 0; k < nst && e == hipSuccess; ++k) {
            const StagePlan &sp = plan[k];
            const double *qin = reg[sp.in];
            StageArgs sa{sp.a >= 0 ? reg[sp.a] : nullptr, reg[sp.out], b.TQ, sp.c0, sp.c1, sp.c2 * dt,
                         sp.b >= 0 ? reg[sp.b] : nullptr, sp.tout >= 0 ? reg[sp.tout] : nullptr, sp.d0, sp.d1,
                         sp.d2 * dt, 1, b.R0};
            e = run(1, [&] { return launch_flux64(m, G, P, qin, b.TQ, b.TV, sa, C, s); });
            if (e == hipSuccess) e = run(2, [&] { return launch_lift64(m, G, b.TV, sa, C.model != nullptr, s); });
        }
    }
    if (e != hipSuccess) return hip_fail(e, "rk_step");
    if (phys->flags & CHORUS_CHECK_FINITE) return finite_check_flag(m, P, Q_dev, b.flag, s);
    return CHORUS_OK;
}

int chorus_rk_step(chorus_mesh_t mesh, const chorus_physics *phys, double *Q_dev, double dt, int32_t n_steps,
                   void *ws, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    rc = check_phys(phys);
    if (rc) return rc;
    rc = check_kappa_r(*m, phys);
    if (rc) return rc;
    if (!Q_dev || !ws || n_steps < 0 || !std::isfinite(dt)) {
        set_error("rk_step: null pointer, negative step count or non-finite dt");
        return CHORUS_EINVAL;
    }
    if (n_steps == 0) return CHORUS_OK;
    rc = check_closure_order(*m, phys);
    if (rc) return rc;
    const bool mixed = phys->precision == CHORUS_MIXED;
    const bool rk54 = phys->integrator == CHORUS_SSPRK54;
    const StagePlan *plan = rk54 ? kSSPRK54 : kSSPRK3;
    const int nst = rk54 ? 5 : 3;
    const WsLayout w = ws_layout(*m);
    unsigned char *W = (unsigned char *)ws;
    const ClosureArgs C = closure_of(phys, w, W);
    const PhysParams P = params_of(phys);
    hipStream_t s = (hipStream_t)stream;
    if (mixed) {
        rc = check_mixed(*m, phys, ws);
        if (rc) return rc;
        const GeoM g = geom_of(*m, w, W);
        double *reg[4] = {(double *)(W + w.P0), (double *)(W + w.P1), rk54 ? (double *)(W + w.P2) : nullptr,
                          rk54 ? (double *)(W + w.P4) : nullptr};
        // the flux pass reads the Q-trace mailbox and writes the viscous one;
        // the lift pass reads the viscous mailbox and rewrites the Q traces
        // (kernel order separates every read from the next write)
        float *TQm = (float *)(W + w.TQm), *TVm = (float *)(W + w.TVm);
        hipError_t e = timed(0, s, [&] { return launch_pert_begin(*m, g, Q_dev, reg[0], TQm, s); });
        for (int st = 0; st < n_steps && e == hipSuccess; ++st) {
            for (int k = 0; k < nst && e == hipSuccess; ++k) {
                const StagePlan &sp = plan[k];
                const double *pin = reg[sp.in];
                MixedStageArgs a{sp.a >= 0 ? reg[sp.a] : nullptr, reg[sp.out], TQm, sp.c0, sp.c1,
                                 sp.c2 * dt, sp.b >= 0 ? reg[sp.b] : nullptr, sp.tout >= 0 ? reg[sp.tout] : nullptr,
                                 sp.d0, sp.d1, sp.d2 * dt, 1};
                e = timed(1, s, [&] { return launch_flux_mixed(*m, g, P, pin, TQm, TVm, a, s); });
                if (e == hipSuccess) e = timed(2, s, [&] { return launch_lift_mixed(*m, g, TVm, a, s); });
            }
        }
        if (e == hipSuccess) e = launch_pert_end(g.Q0, reg[0], Q_dev, 5 * m->E * m->N * m->N * m->N, s);
        if (e != hipSuccess) return hip_fail(e, "rk_step (mixed)");
        if (phys->flags & CHORUS_CHECK_FINITE) return finite_check(*m, P, Q_dev, w, W, s);
        return CHORUS_OK;
    }
    const double *R0 = nullptr;
    if (phys->flags & CHORUS_BALANCED) {
        rc = check_mixed(*m, phys, ws);
        if (rc) return rc;
        R0 = (const double *)(W + w.R64);
    }
    const Fp64Bufs b{(double *)(W + w.Qs), rk54 ? (double *)(W + w.Q2) : nullptr,
                     rk54 ? (double *)(W + w.Q4) : nullptr, (double *)(W + w.TQ0), (double *)(W + w.TV),
                     (int *)(W + w.flag), R0};
    return rk_fp64(*m, phys, C, Q_dev, dt, n_steps, b, s, true);
}

// ---------------------------------------------------------------------------
// FP64 steps without a caller workspace: the stage registers, mailboxes and
// flag live in a fixed device array (one copy per GPU, held until the
// process ends).  Host code uses the address hipGetSymbolAddress returns on
// each device, never the array's name (a host-side stand-in).
// ---------------------------------------------------------------------------
static constexpr size_t kStaticScratchBytes = CHORUS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices];

// the scratch address on the current device, looked up once per device
static int scratch_address(unsigned char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "rk_step_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("rk_step_noalloc: device index beyond the supported count");
        return CHORUS_ENOTSUP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "rk_step_noalloc: hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return CHORUS_OK;
}

int chorus_rk_step_noalloc(chorus_mesh_t mesh, const chorus_physics *phys, double *Q_dev, double dt,
                           int32_t n_steps, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    rc = check_phys(phys);
    if (rc) return rc;
    rc = check_kappa_r(*m, phys);
    if (rc) return rc;
    if (!Q_dev || n_steps < 0 || !std::isfinite(dt)) {
        set_error("rk_step_noalloc: null pointer, negative step count or non-finite dt");
        return CHORUS_EINVAL;
    }
    if (phys->precision != CHORUS_FP64 || phys->closure != CHORUS_CLOSURE_NONE || (phys->flags & CHORUS_BALANCED)) {
        set_error("rk_step_noalloc: FP64 precision without the learned closure or the balanced mode only");
        return CHORUS_ENOTSUP;
    }
    // compact layout: stage register, [two SSPRK(5,4) registers], trace and
    // viscous mailboxes, flag
    const int N = m->N, NP = N * N * N, NF2 = N * N;
    const bool rk54 = phys->integrator == CHORUS_SSPRK54;
    const size_t state = sizeof(double) * 5 * (size_t)m->E * NP;
    const size_t mbox = sizeof(double) * (size_t)m->E * 6 * 5 * NF2;
    size_t off = 0;
    const size_t oQs = off;  off = align256(off + state);
    const size_t oQ2 = off;  off = rk54 ? align256(off + state) : off;
    const size_t oQ4 = off;  off = rk54 ? align256(off + state) : off;
    const size_t oTQ = off;  off = align256(off + mbox);
    const size_t oTV = off;  off = align256(off + mbox);
    const size_t oFl = off;  off = align256(off + sizeof(int) * 4);
    if (off > kStaticScratchBytes) {
        set_error("rk_step_noalloc: this mesh and integrator need " + std::to_string(off) +
                  " bytes of scratch; the fixed maximum is " + std::to_string(kStaticScratchBytes) +
                  " (use chorus_rk_step with a workspace)");
        return CHORUS_EINVAL;
    }
    if (n_steps == 0) return CHORUS_OK;
    unsigned char *S = nullptr;
    rc = scratch_address(&S);
    if (rc) return rc;
    const Fp64Bufs b{(double *)(S + oQs), rk54 ? (double *)(S + oQ2) : nullptr, rk54 ? (double *)(S + oQ4) : nullptr,
                     (double *)(S + oTQ), (double *)(S + oTV), (int *)(S + oFl), nullptr};
    const ClosureArgs C{nullptr, nullptr};
    return rk_fp64(*m, phys, C, Q_dev, dt, n_steps, b, (hipStream_t)stream, false);
}

int chorus_conserved_sums(chorus_mesh_t mesh, const double *Q_dev, double out_host[5], void *ws, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    if (!Q_dev || !ws || !out_host) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    const WsLayout w = ws_layout(*m);
    unsigned char *W = (unsigned char *)ws;
    const double *solw = (const double *)((const unsigned char *)m->dev_image + m->layout.solw);
    hipStream_t s = (hipStream_t)stream;
    double *out = (double *)(W + w.sums);
    hipError_t e = launch_sums(Q_dev, solw, m->E * m->N * m->N * m->N, (double *)(W + w.part), kSumBlocks, out, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, out, 5 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "conserved_sums");
    return CHORUS_OK;
}

int chorus_angular_momentum(chorus_mesh_t mesh, const double *Q_dev, double out_host[6], void *ws, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    if (!Q_dev || !ws || !out_host) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    const WsLayout w = ws_layout(*m);
    unsigned char *W = (unsigned char *)ws;
    const unsigned char *img = (const unsigned char *)m->dev_image;
    hipStream_t s = (hipStream_t)stream;
    double *out = (double *)(W + w.sums);
    hipError_t e = launch_am_sums(Q_dev, (const double *)(img + m->layout.solw), (const double *)(img + m->layout.xsol),
                                  m->E, m->N * m->N * m->N, (double *)(W + w.part), kSumBlocks, out, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, out, 6 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "angular_momentum");
    return CHORUS_OK;
}

int chorus_am_correct(chorus_mesh_t mesh, double *Q_dev, double dOmega_host[3], void *ws, void *stream) {
    double LI[6];
    int rc = chorus_angular_momentum(mesh, Q_dev, LI, ws, stream);
    if (rc) return rc;
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    double dO[3];
    for (int c = 0; c < 3; ++c) {
        if (!(LI[3 + c] > 0.0)) {
            set_error("am_correct: non-positive moment of inertia");
            return CHORUS_ENONFINITE;
        }
        dO[c] = LI[c] / LI[3 + c];
        if (!std::isfinite(dO[c])) {
            set_error("am_correct: non-finite angular momentum");
            return CHORUS_ENONFINITE;
        }
    }
    const unsigned char *img = (const unsigned char *)m->dev_image;
    hipError_t e = launch_am_apply(Q_dev, (const double *)(img + m->layout.xsol), m->E, m->N * m->N * m->N, dO,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "am_correct");
    if (dOmega_host)
        for (int c = 0; c < 3; ++c) dOmega_host[c] = dO[c];
    return CHORUS_OK;
}

int chorus_stable_dt(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q_host, double cfl,
                     double *dt) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    if (!m || !phys || !Q_host || !dt || !(cfl > 0.0)) {
        set_error("null argument or non-positive cfl");
        return CHORUS_EINVAL;
    }
    // multi-dimensional signal speed in reference units at every solution
    // point: sum_d (|u . grad xi_d| + c |grad xi_d|)
    const int N = m->N, NP = N * N * N;
    const int64_t n = m->E * NP;
    double smax = 0.0;
    for (int64_t g = 0; g < n; ++g) {
        const double r = Q_host[g], mx = Q_host[n + g], my = Q_host[2 * n + g], mz = Q_host[3 * n + g];
        const double E = Q_host[4 * n + g];
        const double u[3] = {mx / r, my / r, mz / r};
        const double p = (phys->gamma - 1.0) * (E - 0.5 * (mx * u[0] + my * u[1] + mz * u[2]));
        const double c = std::sqrt(phys->gamma * p / r);
        const double J = m->jac[g];
        double sum = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double *a = &m->met[(g * 3 + d) * 3];
            const double un = (u[0] * a[0] + u[1] * a[1] + u[2] * a[2]) / J;
            sum += std::fabs(un) + c * std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) / J;
        }
        if (!(sum == sum)) smax = NAN;
        else smax = std::fmax(smax, sum);
    }
    if (!(smax > 0.0) || !std::isfinite(smax)) {
        set_error("stable_dt: state has no finite positive signal speed");
        return CHORUS_ENONFINITE;
    }
    *dt = cfl / (N * smax);
    return CHORUS_OK;
}

int chorus_kernel_timing(int enable) {
    g_timing = enable != 0;
    return CHORUS_OK;
}

int chorus_kernel_times(double ms[3], int64_t counts[3]) {
    if (!ms || !counts) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    for (int k = 0; k < 3; ++k) {
        ms[k] = 0.0;
        counts[k] = 0;
    }
    int rc = CHORUS_OK;
    for (TimedLaunch &t : g_launches) {
        float el = 0.0f;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&el, t.start, t.stop);
        if (e != hipSuccess) rc = hip_fail(e, "kernel_times");
        if (t.kind >= 0 && t.kind < 3) {
            ms[t.kind] += el;
            counts[t.kind] += 1;
        }
        g_event_pool.push_back(t.start);
        g_event_pool.push_back(t.stop);
    }
    g_launches.clear();
    return rc;
}


// ---------------------------------------------------------------------------
// learned subgrid closure
// ---------------------------------------------------------------------------
int chorus_closure_model_bytes(size_t *bytes) {
    if (!bytes) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    *bytes = kMlpModelBytes;
    return CHORUS_OK;
}

int chorus_closure_pack(const float *params_dev, const float *norm_dev, void *model_dev, void *stream) {
    if (!params_dev || !norm_dev || !model_dev) {
        set_error("null device pointer");
        return CHORUS_EINVAL;
    }
    if (((uintptr_t)model_dev) & 255) {
        set_error("model image must be 256-byte aligned");
        return CHORUS_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned char *M = (unsigned char *)model_dev;
    hipError_t e = launch_pack(params_dev, norm_dev, M, s);
    int ok = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&ok, M + kMlpFlagOff, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "closure_pack");
    if (ok != 1) {
        set_error("closure_pack: non-finite parameter or normalisation value");
        return CHORUS_ENONFINITE;
    }
    return CHORUS_OK;
}

int chorus_closure_features(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q_dev, float *X_dev,
                            void *ws, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    rc = check_phys(phys);
    if (rc) return rc;
    if (!Q_dev || !X_dev || !ws) {
        set_error("null device pointer");
        return CHORUS_EINVAL;
    }
    if (phys->precision != CHORUS_FP64) {
        set_error("closure_features: FP64 precision only");
        return CHORUS_ENOTSUP;
    }
    const WsLayout w = ws_layout(*m);
    unsigned char *W = (unsigned char *)ws;
    const Geo G = geo_of(*m, (unsigned char *)ws);
    const PhysParams P = params_of(phys);
    hipStream_t s = (hipStream_t)stream;
    double *TQ = (double *)(W + w.TQ0);
    hipError_t e = launch_trace(*m, G, Q_dev, TQ, s);
    if (e == hipSuccess) e = launch_features(*m, G, P, Q_dev, TQ, X_dev, s);
    if (e != hipSuccess) return hip_fail(e, "closure_features");
    return CHORUS_OK;
}

int chorus_closure_infer(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q_dev, float *sgs_dev,
                         void *ws, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    rc = check_phys(phys);
    if (rc) return rc;
    if (phys->closure != CHORUS_CLOSURE_MLP) {
        set_error("closure_infer: physics has no closure (closure != CHORUS_CLOSURE_MLP)");
        return CHORUS_EINVAL;
    }
    rc = check_closure_order(*m, phys);
    if (rc) return rc;
    if (!Q_dev || !sgs_dev || !ws) {
        set_error("null device pointer");
        return CHORUS_EINVAL;
    }
    const WsLayout w = ws_layout(*m);
    unsigned char *W = (unsigned char *)ws;
    const Geo G = geo_of(*m, (unsigned char *)ws);
    const PhysParams P = params_of(phys);
    hipStream_t s = (hipStream_t)stream;
    double *TQ = (double *)(W + w.TQ0), *TV = (double *)(W + w.TV);
    const ClosureArgs C{(const unsigned char *)phys->closure_model, sgs_dev};
    hipError_t e = launch_trace_push(*m, G, Q_dev, TQ, s);
    if (e == hipSuccess) e = launch_closure_tau(*m, G, P, Q_dev, TQ, C, s);
    if (e != hipSuccess) return hip_fail(e, "closure_infer");
    return CHORUS_OK;
}

struct TrainLayout {
    size_t H1, H2, dZ1, dZ2, dY, lossv, part, flag, total;
};

static TrainLayout train_layout(int64_t B) {
    TrainLayout L;
    size_t off = 0;
    const size_t row = sizeof(float) * 64 * (size_t)B;
    L.H1 = off;  off = align256(off + row);
    L.H2 = off;  off = align256(off + row);
    L.dZ1 = off; off = align256(off + row);
    L.dZ2 = off; off = align256(off + row);
    L.dY = off;  off = align256(off + sizeof(float) * 16 * (size_t)B);
    L.lossv = off; off = align256(off + sizeof(float) * (size_t)B);
    L.part = off;  off = align256(off + sizeof(float) * (kMlpParams + 1) * (size_t)((B + 63) / 64));
    L.flag = off;  off = align256(off + sizeof(int));
    L.total = off;
    return L;
}

static TrainBufs train_bufs(const TrainLayout &L, unsigned char *W, int64_t n_mean) {
    TrainBufs T;
    T.H1 = (float *)(W + L.H1);
    T.H2 = (float *)(W + L.H2);
    T.dZ1 = (float *)(W + L.dZ1);
    T.dZ2 = (float *)(W + L.dZ2);
    T.dY = (float *)(W + L.dY);
    T.lossv = (float *)(W + L.lossv);
    T.part = (float *)(W + L.part);
    T.n_mean = n_mean;
    return T;
}

static constexpr int64_t kMaxBatch = 1 << 20;

int chorus_closure_train_workspace_bytes(int64_t batch, size_t *bytes) {
    if (!bytes || batch < 1 || batch > kMaxBatch) {
        set_error("closure workspace: need 1 <= batch <= 2^20");
        return CHORUS_EINVAL;
    }
    *bytes = train_layout(batch).total;
    return CHORUS_OK;
}

int chorus_closure_grad(const float *X_dev, const float *Y_dev, int64_t n, const float *params_dev,
                        float *grad_dev, float *loss_dev, void *ws, size_t ws_bytes, void *stream) {
    if (!X_dev || !Y_dev || !params_dev || !grad_dev || !loss_dev || !ws) {
        set_error("null device pointer");
        return CHORUS_EINVAL;
    }
    if (n < 1 || n > kMaxBatch || train_layout(n).total > ws_bytes) {
        set_error("closure_grad: need 1 <= n <= 2^20 and a workspace for n samples");
        return CHORUS_EINVAL;
    }
    const TrainLayout L = train_layout(n);
    unsigned char *W = (unsigned char *)ws;
    const TrainBufs T = train_bufs(L, W, n);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_train_grad(X_dev, Y_dev, nullptr, 0, (int)n, params_dev, T, grad_dev, loss_dev, s);
    if (e != hipSuccess) return hip_fail(e, "closure_grad");
    return CHORUS_OK;
}

int chorus_closure_train(const float *X_dev, const float *Y_dev, int64_t n, const int32_t *idx_dev, int32_t batch,
                         int32_t iters, float *params_dev, float *adam_m_dev, float *adam_v_dev, int64_t step0,
                         const double hyper[4], float *loss_dev, void *ws, size_t ws_bytes, void *stream) {
    if (!X_dev || !Y_dev || !idx_dev || !params_dev || !adam_m_dev || !adam_v_dev || !hyper || !loss_dev || !ws) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    if (n < 1 || n > INT32_MAX || batch < 1 || batch > kMaxBatch || iters < 0 || step0 < 0 ||
        train_layout(batch).total > ws_bytes) {
        set_error("closure_train: need 1 <= n < 2^31, 1 <= batch <= 2^20, iters >= 0, step0 >= 0 and a "
                  "workspace for the batch");
        return CHORUS_EINVAL;
    }
    const double lr = hyper[0], b1 = hyper[1], b2 = hyper[2], eps = hyper[3];
    if (!(lr > 0.0) || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) || !(eps > 0.0)) {
        set_error("closure_train: need lr > 0, 0 <= beta < 1, eps > 0");
        return CHORUS_EINVAL;
    }
    if (iters == 0) return CHORUS_OK;
    hipStream_t s = (hipStream_t)stream;
    const TrainLayout L = train_layout(batch);
    unsigned char *W = (unsigned char *)ws;
    const TrainBufs T = train_bufs(L, W, batch);
    // every sample index must address a row of X and Y (checked on the
    // device, before any training kernel reads through the indices)
    int *flag = (int *)(W + L.flag), bad = 0;
    hipError_t e = launch_check_idx(idx_dev, (int64_t)iters * batch, n, flag, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "closure_train");
    if (bad) {
        set_error("closure_train: sample index out of range");
        return CHORUS_EINVAL;
    }
    for (int32_t it = 0; it < iters && e == hipSuccess; ++it) {
        const double t = (double)(step0 + it + 1);
        AdamArgs a;
        a.lr = (float)lr;
        a.b1 = (float)b1;
        a.b2 = (float)b2;
        a.eps = (float)eps;
        a.inv_bc1 = (float)(1.0 / (1.0 - std::pow(b1, t)));
        a.inv_bc2 = (float)(1.0 / (1.0 - std::pow(b2, t)));
        e = launch_train_step(X_dev, Y_dev, idx_dev, (int64_t)it * batch, batch, params_dev, adam_m_dev, adam_v_dev,
                              T, a, loss_dev + it, s);
    }
    if (e != hipSuccess) return hip_fail(e, "closure_train");
    return CHORUS_OK;
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton on the three-term
// recurrence)
static void gauss01(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) p0 = 1.0;
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[i] = 0.5 * (1.0 - t);
        w[i] = 1.0 / ((1.0 - t * t) * dp * dp);  // (2 / ((1-t^2) P'^2)) / 2
    }
}

// shifted Legendre polynomial of degree k on [0, 1]
static double legendre01(int k, double x) {
    const double t = 2.0 * x - 1.0;
    double p0 = 1.0, p1 = t;
    if (k == 0) return 1.0;
    for (int j = 2; j <= k; ++j) {
        const double p2 = ((2 * j - 1) * t * p1 - (j - 1) * p0) / j;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

int chorus_closure_filter(chorus_mesh_t fine, chorus_mesh_t coarse, double gamma, const double *Qfine_dev,
                          double *Qbar_dev, double *tau_dev, void *stream) {
    Mesh *mf = reinterpret_cast<Mesh *>(fine);
    Mesh *mc = reinterpret_cast<Mesh *>(coarse);
    int rc = check_ready(mf);
    if (rc) return rc;
    rc = check_ready(mc);
    if (rc) return rc;
    if (!Qfine_dev || !Qbar_dev || !tau_dev || !(gamma > 1.0)) {
        set_error("null device pointer or gamma <= 1");
        return CHORUS_EINVAL;
    }
    if (mf->E != mc->E || mf->elem20 != mc->elem20 || mf->xyz != mc->xyz) {
        set_error("closure_filter: fine and coarse must be the same hex mesh");
        return CHORUS_EINVAL;
    }
    if (mf->N > 6 || mc->N > 3 || mc->N < 1 || mf->N <= mc->N) {
        set_error("closure_filter: need coarse order <= 3, fine order <= 6 and fine order > coarse order");
        return CHORUS_ENOTSUP;
    }
    FilterArgs A;
    A.Qf = Qfine_dev;
    A.solgeo_f = (const double *)((const unsigned char *)mf->dev_image + mf->layout.solgeo);
    A.solgeo_c = (const double *)((const unsigned char *)mc->dev_image + mc->layout.solgeo);
    A.Qbar = Qbar_dev;
    A.tau = tau_dev;
    A.E = mf->E;
    A.nf = mf->N;
    A.nc = mc->N;
    A.gamma = gamma;
    // P[a][i] = sum_k (2k+1) L_k(xc_a) int_0^1 L_k h_i, h_i the Lagrange basis
    // on the fine solution points (quadrature exact for degree nf + nc)
    const int nq = mf->N + mc->N;
    double xq[16], wq[16];
    gauss01(nq, xq, wq);
    const double *xf = mf->basis.xs, *xc = mc->basis.xs;
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 6; ++i) A.P[a][i] = 0.0;
    for (int i = 0; i < mf->N; ++i) {
        for (int k = 0; k < mc->N; ++k) {
            double integ = 0.0;
            for (int q = 0; q < nq; ++q) {
                double h = 1.0;
                for (int j = 0; j < mf->N; ++j)
                    if (j != i) h *= (xq[q] - xf[j]) / (xf[i] - xf[j]);
                integ += wq[q] * legendre01(k, xq[q]) * h;
            }
            for (int a = 0; a < mc->N; ++a) A.P[a][i] += (2 * k + 1) * legendre01(k, xc[a]) * integ;
        }
    }
    hipError_t e = launch_filter(A, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "closure_filter");
    return CHORUS_OK;
}

}  // extern "C"
