// extern "C" entry points of the SD library (declared in include/chorus.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "launch.hpp"

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
    // mixed-precision path
    size_t P0, P1, TQm0, TQm1, TVm, bg, dbg, gS0, R0, Q0;
    bool mixed;
    size_t total;
};
static constexpr int kSumBlocks = 512;

static WsLayout ws_layout(const Mesh &m, bool mixed) {
    const int N = m.N, NP = N * N * N, NF2 = N * N;
    const int64_t E = m.E;
    WsLayout w;
    w.mixed = mixed;
    size_t off = 0;
    w.Qs = off;   off = align256(off + sizeof(double) * 5 * E * NP);
    w.TQ0 = off;  off = align256(off + sizeof(double) * E * 6 * 5 * NF2);
    w.TQ1 = off;  off = align256(off + sizeof(double) * E * 6 * 5 * NF2);
    w.TV = off;   off = align256(off + sizeof(double) * E * 6 * 5 * NF2);
    w.part = off; off = align256(off + sizeof(double) * 5 * kSumBlocks);
    w.sums = off; off = align256(off + sizeof(double) * 8);
    w.flag = off; off = align256(off + sizeof(int) * 4);
    w.P0 = w.P1 = w.TQm0 = w.TQm1 = w.TVm = w.bg = w.dbg = w.gS0 = w.R0 = w.Q0 = 0;
    if (mixed) {
        w.P0 = off;   off = align256(off + sizeof(double) * 5 * E * NP);
        w.P1 = off;   off = align256(off + sizeof(double) * 5 * E * NP);
        w.TQm0 = off; off = align256(off + sizeof(float) * E * 6 * 5 * NF2);
        w.TQm1 = off; off = align256(off + sizeof(float) * E * 6 * 5 * NF2);
        w.TVm = off;  off = align256(off + sizeof(float) * E * 6 * 5 * NF2);
        w.bg = off;   off = align256(off + sizeof(float) * E * 2 * NP);
        w.dbg = off;  off = align256(off + sizeof(float) * E * 6 * 2 * NF2);
        w.gS0 = off;  off = align256(off + sizeof(float) * E * 3 * (N + 1) * NF2);
        w.R0 = off;   off = align256(off + sizeof(float) * 5 * E * NP);
        w.Q0 = off;   off = align256(off + sizeof(double) * 5 * E * NP);
    }
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
    g.R0 = (const float *)(W + w.R0);
    g.Q0 = (const double *)(W + w.Q0);
    return g;
}

static Geo geo_of(const Mesh &m) {
    const unsigned char *b = (const unsigned char *)m.dev_image;
    Geo g;
    g.solgeo = (const double *)(b + m.layout.solgeo);
    g.fluxgeo = (const double *)(b + m.layout.fluxgeo);
    g.link = (const int32_t *)(b + m.layout.link);
    g.info = (const int32_t *)(b + m.layout.info);
    g.E = m.E;
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
    if (p->closure != 0) {
        set_error("learned closure is not available in this build");
        return CHORUS_ENOTSUP;
    }
    return CHORUS_OK;
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
        b.kappa != p->kappa || b.kappa_r != p->kappa_r || b.T_top != p->T_top || b.F_bottom != p->F_bottom) {
        set_error("mixed precision: the physics must match the one passed to chorus_set_background");
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
    return P;
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

static int finite_check(const Mesh &m, const PhysParams &P, const double *Q, const WsLayout &w,
                        unsigned char *ws, hipStream_t s) {
    int *flag = (int *)(ws + w.flag);
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
    (void)phys;
    *bytes = ws_layout(*m, phys && phys->precision == CHORUS_MIXED).total;
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

int chorus_set_background(chorus_mesh_t mesh, const chorus_physics *phys, const double *Q0_dev, void *ws,
                          void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    rc = check_phys(phys);
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
    const WsLayout w = ws_layout(*m, true);
    unsigned char *W = (unsigned char *)ws;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = m->E * m->N * m->N * m->N;
    double *Q0 = (double *)(W + w.Q0);
    int *flag = (int *)(W + w.flag);
    hipError_t e = hipMemcpyAsync(Q0, Q0_dev, sizeof(double) * 5 * n, hipMemcpyDeviceToDevice, s);
    chorus_physics p64 = *phys;
    p64.precision = CHORUS_FP64;
    const PhysParams P = params_of(&p64);
    const Geo G = geo_of(*m);
    double *R0d = (double *)(W + w.Qs), *TQ = (double *)(W + w.TQ0), *TV = (double *)(W + w.TV);
    if (e == hipSuccess) e = launch_clear_flag(flag, s);
    if (e == hipSuccess) e = launch_trace(*m, G, Q0, TQ, s);
    if (e == hipSuccess) e = launch_bg_setup(*m, G, Q0, TQ, (float *)(W + w.bg), (float *)(W + w.dbg), flag, s);
    if (e == hipSuccess) e = launch_bg_entropy(*m, G, P, Q0, TQ, (float *)(W + w.gS0), s);
    // R0 = R(Q0), the complete FP64 residual of the background
    if (e == hipSuccess) e = launch_grad(*m, G, P, Q0, TQ, TV, s);
    StageArgs sa{nullptr, R0d, nullptr, 0.0, 1.0, 0.0, 0};
    if (e == hipSuccess) e = launch_resid(*m, G, P, Q0, TQ, TV, sa, s);
    if (e == hipSuccess) e = launch_to_float(R0d, (float *)(W + w.R0), 5 * n, s);
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
    if (!Q_dev || !dQdt_dev || !ws) {
        set_error("null device pointer");
        return CHORUS_EINVAL;
    }
    const bool mixed = phys->precision == CHORUS_MIXED;
    const WsLayout w = ws_layout(*m, mixed);
    unsigned char *W = (unsigned char *)ws;
    const PhysParams P = params_of(phys);
    hipStream_t s = (hipStream_t)stream;
    if (mixed) {
        rc = check_mixed(*m, phys, ws);
        if (rc) return rc;
        const GeoM g = geom_of(*m, w, W);
        double *P0 = (double *)(W + w.P0);
        float *TQm = (float *)(W + w.TQm0), *TVm = (float *)(W + w.TVm);
        hipError_t e = timed(0, s, [&] { return launch_pert_begin(*m, g, Q_dev, P0, TQm, s); });
        if (e == hipSuccess) e = timed(1, s, [&] { return launch_grad_mixed(*m, g, P, P0, TQm, TVm, s); });
        MixedStageArgs a{nullptr, dQdt_dev, nullptr, 0.0, 1.0, 0.0, 0};
        if (e == hipSuccess) e = timed(2, s, [&] { return launch_resid_mixed(*m, g, P, P0, TQm, TVm, a, s); });
        if (e != hipSuccess) return hip_fail(e, "sd_residual (mixed)");
        if (phys->flags & CHORUS_CHECK_FINITE) return finite_check(*m, P, Q_dev, w, W, s);
        return CHORUS_OK;
    }
    double *TQ = (double *)(W + w.TQ0), *TV = (double *)(W + w.TV);
    const Geo G = geo_of(*m);
    hipError_t e = timed(0, s, [&] { return launch_trace(*m, G, Q_dev, TQ, s); });
    if (e == hipSuccess) e = timed(1, s, [&] { return launch_grad(*m, G, P, Q_dev, TQ, TV, s); });
    StageArgs sa{nullptr, dQdt_dev, nullptr, 0.0, 1.0, 0.0, 0};
    if (e == hipSuccess) e = timed(2, s, [&] { return launch_resid(*m, G, P, Q_dev, TQ, TV, sa, s); });
    if (e != hipSuccess) return hip_fail(e, "sd_residual");
    if (phys->flags & CHORUS_CHECK_FINITE) return finite_check(*m, P, Q_dev, w, W, s);
    return CHORUS_OK;
}

int chorus_rk_step(chorus_mesh_t mesh, const chorus_physics *phys, double *Q_dev, double dt, int32_t n_steps,
                   void *ws, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    rc = check_phys(phys);
    if (rc) return rc;
    if (!Q_dev || !ws || n_steps < 0 || !std::isfinite(dt)) {
        set_error("rk_step: null pointer, negative step count or non-finite dt");
        return CHORUS_EINVAL;
    }
    if (n_steps == 0) return CHORUS_OK;
    const bool mixed = phys->precision == CHORUS_MIXED;
    const WsLayout w = ws_layout(*m, mixed);
    unsigned char *W = (unsigned char *)ws;
    if (mixed) {
        rc = check_mixed(*m, phys, ws);
        if (rc) return rc;
        const GeoM g = geom_of(*m, w, W);
        const PhysParams P = params_of(phys);
        hipStream_t s = (hipStream_t)stream;
        double *Pb[2] = {(double *)(W + w.P0), (double *)(W + w.P1)};
        float *TQb[2] = {(float *)(W + w.TQm0), (float *)(W + w.TQm1)};
        float *TVm = (float *)(W + w.TVm);
        int cur = 0;
        hipError_t e = timed(0, s, [&] { return launch_pert_begin(*m, g, Q_dev, Pb[0], TQb[cur], s); });
        const double ca[3] = {0.0, 0.75, 1.0 / 3.0}, cb[3] = {1.0, 0.25, 2.0 / 3.0};
        for (int st = 0; st < n_steps && e == hipSuccess; ++st) {
            for (int k = 0; k < 3 && e == hipSuccess; ++k) {
                const double *pin = (k == 0) ? Pb[0] : Pb[1];
                double *pout = (k == 2) ? Pb[0] : Pb[1];
                e = timed(1, s, [&] { return launch_grad_mixed(*m, g, P, pin, TQb[cur], TVm, s); });
                if (e != hipSuccess) break;
                MixedStageArgs a{Pb[0], pout, TQb[cur ^ 1], ca[k], cb[k], dt, 1};
                e = timed(2, s, [&] { return launch_resid_mixed(*m, g, P, pin, TQb[cur], TVm, a, s); });
                cur ^= 1;
            }
        }
        if (e == hipSuccess) e = launch_pert_end(g.Q0, Pb[0], Q_dev, 5 * m->E * m->N * m->N * m->N, s);
        if (e != hipSuccess) return hip_fail(e, "rk_step (mixed)");
        if (phys->flags & CHORUS_CHECK_FINITE) return finite_check(*m, P, Q_dev, w, W, s);
        return CHORUS_OK;
    }
    double *Qs = (double *)(W + w.Qs), *TV = (double *)(W + w.TV);
    double *TQb[2] = {(double *)(W + w.TQ0), (double *)(W + w.TQ1)};
    const Geo G = geo_of(*m);
    const PhysParams P = params_of(phys);
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    hipError_t e = timed(0, s, [&] { return launch_trace(*m, G, Q_dev, TQb[cur], s); });
    // SSP-RK3: Q1 = Q + dt R(Q); Q2 = 3/4 Q + 1/4 (Q1 + dt R(Q1));
    //          Q  = 1/3 Q + 2/3 (Q2 + dt R(Q2))
    const double ca[3] = {0.0, 0.75, 1.0 / 3.0}, cb[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int st = 0; st < n_steps && e == hipSuccess; ++st) {
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            const double *qin = (k == 0) ? Q_dev : Qs;
            double *qout = (k == 2) ? Q_dev : Qs;
            e = timed(1, s, [&] { return launch_grad(*m, G, P, qin, TQb[cur], TV, s); });
            if (e != hipSuccess) break;
            StageArgs sa{Q_dev, qout, TQb[cur ^ 1], ca[k], cb[k], dt, 1};
            e = timed(2, s, [&] { return launch_resid(*m, G, P, qin, TQb[cur], TV, sa, s); });
            cur ^= 1;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "rk_step");
    if (phys->flags & CHORUS_CHECK_FINITE) return finite_check(*m, P, Q_dev, w, W, s);
    return CHORUS_OK;
}

int chorus_conserved_sums(chorus_mesh_t mesh, const double *Q_dev, double out_host[5], void *ws, void *stream) {
    Mesh *m = reinterpret_cast<Mesh *>(mesh);
    int rc = check_ready(m);
    if (rc) return rc;
    if (!Q_dev || !ws || !out_host) {
        set_error("null argument");
        return CHORUS_EINVAL;
    }
    const WsLayout w = ws_layout(*m, false);
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

}  // extern "C"
